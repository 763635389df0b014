"""Pins of the oracle's bead double sum (paper section 2, first equation)
against closed forms, finite differences, Newton's third law and symmetry."""
import os

import numpy as np
import pytest

from oracle import beads, frames
from synth import configs, sampling

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lj_points.txt")


def test_lj_golden_points():
    for r, u, f in np.loadtxt(GOLD):
        e, fr = beads.lj(r)
        assert e == pytest.approx(u, abs=1e-12)
        assert fr * r == pytest.approx(f, abs=1e-9)


def test_single_bead_bodies_reduce_to_lj():
    one = np.zeros((1, 3))
    qi = sampling.uniform_quaternions(sampling.rng(1), 1)[0]
    qj = sampling.uniform_quaternions(sampling.rng(2), 1)[0]
    for r in (0.9, 1.0, 1.3, 2.0, 2.49):
        d = np.array([0.3, -0.4, 0.5])
        d = d / np.linalg.norm(d) * r
        out = beads.bead_pair(one, one, np.zeros(3), qi, d, qj)
        e, fr = beads.lj(r)
        assert out["E"] == pytest.approx(e, rel=1e-14)
        np.testing.assert_allclose(out["Fj"], fr * d, rtol=1e-13)     # repulsive pushes j along d
        np.testing.assert_allclose(out["taui"], 0, atol=1e-13)
        np.testing.assert_allclose(out["tauj"], 0, atol=1e-13)
        assert out["rmin"] == pytest.approx(r, rel=1e-14)


def test_parallel_dumbbells_closed_form():
    a, D = 1.2, 1.7
    dumb = np.array([[-a / 2, 0, 0], [a / 2, 0, 0]])
    ident = np.array([1.0, 0, 0, 0])
    out = beads.bead_pair(dumb, dumb, np.zeros(3), ident, np.array([0, D, 0.0]), ident)
    e_near, _ = beads.lj(D)
    e_diag, _ = beads.lj(np.hypot(D, a))
    assert out["E"] == pytest.approx(2 * e_near + 2 * e_diag, rel=1e-14)
    # by symmetry the force on j is along +y and there is no torque
    assert abs(out["Fj"][0]) < 1e-12 and abs(out["Fj"][2]) < 1e-12
    np.testing.assert_allclose(out["tauj"], 0, atol=1e-12)


def test_crossed_dumbbells_closed_form():
    # dumbbell i along x, dumbbell j along y, centres separated by D along z:
    # all four bead distances are sqrt(D^2 + a^2/2)
    a, D = 1.0, 1.4
    dumb = np.array([[-a / 2, 0, 0], [a / 2, 0, 0]])
    ident = np.array([1.0, 0, 0, 0])
    qz90 = np.array([np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)])
    out = beads.bead_pair(dumb, dumb, np.zeros(3), ident, np.array([0, 0, D]), qz90)
    e, _ = beads.lj(np.sqrt(D * D + a * a / 2))
    assert out["E"] == pytest.approx(4 * e, rel=1e-13)


def _random_close_pair(seed, body):
    g = sampling.rng(seed)
    q = sampling.uniform_quaternions(g, 2)
    while True:
        xj = sampling.uniform_directions(g, 1)[0] * g.uniform(body.r_in * 2 + 0.5, body.r_in * 2 + 3)
        out = beads.bead_pair(body.beads, body.beads, np.zeros(3), q[0], xj, q[1])
        if out["rmin"] > 0.85 and abs(out["E"]) > 1e-3:
            return np.zeros(3), q[0], xj, q[1], out


@pytest.mark.parametrize("shape", ["cube5", "cyl134"])
def test_forces_are_minus_energy_gradient(shape):
    body = getattr(configs, shape)()
    xi, qi, xj, qj, out = _random_close_pair(7, body)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        ep = beads.bead_pair(body.beads, body.beads, xi, qi, xj + e, qj)["E"]
        em = beads.bead_pair(body.beads, body.beads, xi, qi, xj - e, qj)["E"]
        assert -(ep - em) / (2 * h) == pytest.approx(out["Fj"][a], rel=2e-5, abs=1e-6)
        ep = beads.bead_pair(body.beads, body.beads, xi + e, qi, xj, qj)["E"]
        em = beads.bead_pair(body.beads, body.beads, xi - e, qi, xj, qj)["E"]
        assert -(ep - em) / (2 * h) == pytest.approx(out["Fi"][a], rel=2e-5, abs=1e-6)


@pytest.mark.parametrize("shape", ["cube6", "cyl134"])
def test_torques_are_minus_rotation_derivative(shape):
    # supplementary section 6: tau_eta = -dE/dtheta_eta; rotate each body about
    # its own centre by a small lab-frame angle
    body = getattr(configs, shape)()
    xi, qi, xj, qj, out = _random_close_pair(11, body)
    h = 1e-6
    for a in range(3):
        n = np.zeros(3)
        n[a] = h
        rp, rm = frames.qexp(n), frames.qexp(-n)
        ep = beads.bead_pair(body.beads, body.beads, xi, qi, xj, frames.qmul(rp, qj))["E"]
        em = beads.bead_pair(body.beads, body.beads, xi, qi, xj, frames.qmul(rm, qj))["E"]
        assert -(ep - em) / (2 * h) == pytest.approx(out["tauj"][a], rel=2e-5, abs=1e-6)
        ep = beads.bead_pair(body.beads, body.beads, xi, frames.qmul(rp, qi), xj, qj)["E"]
        em = beads.bead_pair(body.beads, body.beads, xi, frames.qmul(rm, qi), xj, qj)["E"]
        assert -(ep - em) / (2 * h) == pytest.approx(out["taui"][a], rel=2e-5, abs=1e-6)


def test_newton_third_law_and_angular_identity():
    body = configs.cube6()
    for seed in range(5):
        xi, qi, xj, qj, out = _random_close_pair(100 + seed, body)
        scale = np.abs(out["Fi"]).max()
        np.testing.assert_allclose(out["Fi"] + out["Fj"], 0, atol=1e-12 * scale)
        d = xj - xi
        resid = out["taui"] + out["tauj"] + np.cross(d, out["Fj"])
        np.testing.assert_allclose(resid, 0, atol=1e-11 * max(scale, 1))


def test_invariance_translation_rotation_image():
    body = configs.cyl134()
    xi, qi, xj, qj, ref = _random_close_pair(5, body)
    shift = np.array([3.3, -7.1, 12.0])
    t = beads.bead_pair(body.beads, body.beads, xi + shift, qi, xj + shift, qj)
    assert t["E"] == pytest.approx(ref["E"], rel=1e-12)
    np.testing.assert_allclose(t["Fj"], ref["Fj"], rtol=1e-10, atol=1e-10)
    # global rotation: positions and orientations rotated, vectors co-rotate
    g = frames.qexp(np.array([0.4, -1.1, 0.7]))
    r = beads.bead_pair(body.beads, body.beads, frames.qrotate(g, xi), frames.qmul(g, qi),
                        frames.qrotate(g, xj), frames.qmul(g, qj))
    assert r["E"] == pytest.approx(ref["E"], rel=1e-12)
    np.testing.assert_allclose(r["Fj"], frames.qrotate(g, ref["Fj"]), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(r["taui"], frames.qrotate(g, ref["taui"]), rtol=1e-9, atol=1e-9)
    # periodic image of j
    box = 40.0
    p = beads.bead_pair(body.beads, body.beads, xi, qi, xj + np.array([box, -box, 2 * box]), qj,
                        box=box)
    assert p["E"] == pytest.approx(ref["E"], rel=1e-12)
    np.testing.assert_allclose(p["tauj"], ref["tauj"], rtol=1e-10, atol=1e-10)


def test_system_sum_equals_all_pairs_double_loop():
    # the centre-distance prefilter of the system sum must not drop any pair
    body = configs.cube5()
    g = sampling.rng(3)
    box = 20.0
    x, q = sampling.place_bodies(g, 10, body, box)
    sysres = beads.bead_system(x, q, np.zeros(10, np.int32), [body.beads], box)
    E = 0.0
    F = np.zeros((10, 3))
    T = np.zeros((10, 3))
    for i in range(10):
        for j in range(i + 1, 10):
            o = beads.bead_pair(body.beads, body.beads, x[i], q[i], x[j], q[j], box=box)
            E += o["E"]
            F[i] += o["Fi"]
            F[j] += o["Fj"]
            T[i] += o["taui"]
            T[j] += o["tauj"]
    assert sysres["E"] == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(sysres["F"], F, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(sysres["tau"], T, rtol=1e-10, atol=1e-10)
    # total force vanishes; total torque about the origin vanishes up to the
    # periodic wrap, so check it with minimum-image arms in a pair sum instead
    np.testing.assert_allclose(sysres["F"].sum(axis=0), 0, atol=1e-9)


def test_pairs_within_small_hand_case():
    box = 10.0
    x = np.array([[0.5, 0.5, 0.5], [9.7, 0.5, 0.5], [5.0, 5.0, 5.0], [5.0, 5.0, 7.9]])
    # 0-1 are 0.8 apart through the boundary, 2-3 are 2.9 apart
    got = {tuple(p) for p in beads.pairs_within(x, box, 1.0)}
    assert got == {(0, 1)}
    got = {tuple(p) for p in beads.pairs_within(x, box, 3.0)}
    assert got == {(0, 1), (2, 3)}
