"""Pins of the oracle's half-power half-cosine bead potential (paper section
3; the attractive branch read as -A (1 + cos(c (r - b))), see oracle/bead.c)
and of the bead sums taken with it."""
import math

import numpy as np
import pytest

from oracle import beads, frames
from synth import configs, sampling

P = beads.HPHC_PAPER
A, B, CC, PP = P["A"], P["b"], P["c"], P["p"]
RC = B + math.pi / CC


def test_paper_parameters_and_closed_forms():
    assert (A, B, CC, PP) == (0.00035, 1.46375, 3.3833, 2.5)
    assert RC == pytest.approx(2.3923087, abs=1e-6)
    assert beads.hphc(B, **P)[0] == pytest.approx(-2 * A, abs=1e-18)           # bottom of the well
    e, fr = beads.hphc(B + math.pi / (2 * CC), **P)                            # half-way up the cosine
    assert e == pytest.approx(-A, rel=1e-14)
    assert fr * (B + math.pi / (2 * CC)) == pytest.approx(-A * CC, rel=1e-14)
    e, fr = beads.hphc(0.5, **P)                                               # soft core
    assert e == pytest.approx((B - 0.5) ** 2.5 - 2 * A, rel=1e-14)
    assert fr * 0.5 == pytest.approx(2.5 * (B - 0.5) ** 1.5, rel=1e-14)
    for r in (RC, RC + 1e-9, 3.0, 10.0):
        assert beads.hphc(r, **P) == (0.0, 0.0)


def test_continuous_with_zero_slope_at_b_and_cutoff():
    for r0 in (B, RC - 1e-12):
        lo, hi = beads.hphc(r0 - 1e-7, **P), beads.hphc(r0 + 1e-7, **P)
        assert lo[0] == pytest.approx(hi[0], abs=1e-12)
        assert abs(lo[1]) < 1e-9 and abs(hi[1]) < 1e-9


@pytest.mark.parametrize("r", [0.3, 0.9, 1.2, 1.5, 1.8, 2.1, 2.35])
def test_force_is_minus_derivative(r):
    h = 1e-6
    d = -(beads.hphc(r + h, **P)[0] - beads.hphc(r - h, **P)[0]) / (2 * h)
    assert beads.hphc(r, **P)[1] * r == pytest.approx(d, rel=1e-6, abs=1e-12)


def test_single_bead_bodies_reduce_to_the_potential():
    one = np.zeros((1, 3))
    qi = sampling.uniform_quaternions(sampling.rng(1), 1)[0]
    qj = sampling.uniform_quaternions(sampling.rng(2), 1)[0]
    with beads.use_hphc(**P):
        for r in (0.7, 1.2, B, 1.9, 2.3, 2.5):
            d = np.array([0.3, -0.4, 0.5]) / np.linalg.norm([0.3, -0.4, 0.5]) * r
            out = beads.bead_pair(one, one, np.zeros(3), qi, d, qj)
            e, fr = beads.hphc(r, **P)
            assert out["E"] == pytest.approx(e, rel=1e-13, abs=1e-18)
            np.testing.assert_allclose(out["Fj"], fr * d, rtol=1e-12, atol=1e-18)
    # back to Lennard-Jones outside the context
    out = beads.bead_pair(one, one, np.zeros(3), qi, np.array([1.1, 0, 0]), qj)
    assert out["E"] == pytest.approx(beads.lj(1.1)[0], rel=1e-14)


def _close_pair(seed, body):
    g = sampling.rng(seed)
    qi, qj = sampling.uniform_quaternions(g, 2)
    xi = g.normal(size=3)
    n = sampling.uniform_directions(g, 1)[0]
    # scan inwards until some bead pair is inside the well or the core
    for dist in np.linspace(2 * body.r_max + RC, 0.5 * body.r_max, 400):
        out = beads.bead_pair(body.beads, body.beads, xi, qi, xi + dist * n, qj)
        if out["rmin"] < 1.2:
            return xi, qi, xi + dist * n, qj, out
    raise AssertionError("no close configuration")


@pytest.mark.parametrize("shape", ["cube5", "cyl134"])
def test_bead_sum_forces_torques_from_energy(shape):
    body = getattr(configs, shape)()
    with beads.use_hphc(**P):
        xi, qi, xj, qj, out = _close_pair(21, body)
        assert out["E"] != 0.0
        h = 1e-6
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            ep = beads.bead_pair(body.beads, body.beads, xi, qi, xj + e, qj)["E"]
            em = beads.bead_pair(body.beads, body.beads, xi, qi, xj - e, qj)["E"]
            assert -(ep - em) / (2 * h) == pytest.approx(out["Fj"][a], rel=1e-5, abs=1e-9)
            rp, rm = frames.qexp(e), frames.qexp(-e)
            ep = beads.bead_pair(body.beads, body.beads, xi, qi, xj, frames.qmul(rp, qj))["E"]
            em = beads.bead_pair(body.beads, body.beads, xi, qi, xj, frames.qmul(rm, qj))["E"]
            assert -(ep - em) / (2 * h) == pytest.approx(out["tauj"][a], rel=1e-5, abs=1e-9)
        np.testing.assert_allclose(out["Fi"] + out["Fj"], 0, atol=1e-14)
        resid = out["taui"] + out["tauj"] + np.cross(xj - xi, out["Fj"])
        np.testing.assert_allclose(resid, 0, atol=1e-12)


def test_system_sum_uses_the_potential_cutoff():
    # two bodies farther apart than 2 r_max + 2.5 (no LJ pair) but closer than
    # 2 r_max + r_c(HPHC) are not summed under LJ; under HPHC the system sum
    # equals the pair sum
    body = configs.cube5()
    x = np.array([[0.0, 0, 0], [2 * body.r_max + 2.0, 0, 0]])
    q = np.tile([1.0, 0, 0, 0], (2, 1))
    with beads.use_hphc(**P):
        s = beads.bead_system(x, q, np.zeros(2, np.int32), [body.beads], None)
        p = beads.bead_pair(body.beads, body.beads, x[0], q[0], x[1], q[1])
    assert s["E"] == pytest.approx(p["E"], rel=1e-13)
    np.testing.assert_allclose(s["F"][1], p["Fj"], rtol=1e-12, atol=1e-18)
