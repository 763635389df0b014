"""Pins of the oracle's rigid-body integrator (velocity Verlet with the
NO_SQUISH free-rotation splitting of Miller et al. 2002; the paper fixes
only dt = 0.005 tau, section 3) against closed forms and invariants."""
import numpy as np
import pytest

from oracle import beads, frames
from synth import configs, sampling


def _free_run(q0, L0, inertia, t_end, dt):
    n = int(round(t_end / dt))
    x = np.zeros((1, 3))
    P = np.zeros((1, 3))
    q = q0.copy()[None, :]
    L = L0.copy()[None, :]
    zero = np.zeros((1, 3))
    for _ in range(n):
        beads.rigid_phase1(dt, x, P, q, L, 1.0, inertia, zero, zero)
        beads.rigid_phase2(dt, P, q, L, 1.0, inertia, zero, zero)
    return q[0], L[0]


def _qdist(a, b):
    return min(np.linalg.norm(a - b), np.linalg.norm(a + b))


def test_free_translation_is_exact():
    x = np.array([[1.0, 2.0, 3.0]])
    P = np.array([[0.3, -0.2, 0.1]])
    q = np.array([[1.0, 0, 0, 0]])
    L = np.zeros((1, 3))
    zero = np.zeros((1, 3))
    for _ in range(100):
        beads.rigid_phase1(0.01, x, P, q, L, 2.0, [1.0, 1.0, 1.0], zero, zero)
        beads.rigid_phase2(0.01, P, q, L, 2.0, [1.0, 1.0, 1.0], zero, zero)
    np.testing.assert_allclose(x[0], [1.0 + 0.15, 2.0 - 0.1, 3.0 + 0.05], rtol=1e-13)


def test_spherical_top_closed_form_and_second_order():
    # isotropic inertia: the body turns at constant lab angular velocity
    # omega = R(q0) L0 / I, so q(t) = exp(t omega / 2) q0
    I = 1100.0
    q0 = sampling.uniform_quaternions(sampling.rng(4), 1)[0]
    L0 = np.array([30.0, -50.0, 20.0])
    omega = frames.qrotate(q0, L0) / I
    t = 2.0
    exact = frames.qmul(frames.qexp(t * omega), q0)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        q, L = _free_run(q0, L0, [I, I, I], t, dt)
        errs.append(_qdist(q, exact))
        # lab-frame angular momentum is conserved by every sub-rotation
        np.testing.assert_allclose(frames.qrotate(q, L), frames.qrotate(q0, L0), rtol=1e-12)
    assert errs[-1] < 1e-5
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.15)


def test_symmetric_top_precession_rate():
    # I1 = I2: in the body frame L_perp rotates about the symmetry axis at
    # Omega = (I3 - I1) / I1 * omega_3 (Euler's equations), L_3 constant
    body = configs.cyl134()
    I1, I3 = body.inertia[0], body.inertia[2]
    L0 = np.array([40.0, 0.0, 60.0])
    q0 = np.array([1.0, 0, 0, 0])
    Om = (I3 - I1) / I1 * (L0[2] / I3)
    t = 3.0
    q, L = _free_run(q0, L0, body.inertia, t, 0.0025)
    want = np.array([40.0 * np.cos(Om * t), 40.0 * np.sin(Om * t), 60.0])
    np.testing.assert_allclose(L, want, atol=2e-3)


def _two_cubes():
    # two cube shells brought together along a fixed direction until the
    # closest bead pair is 1.05 sigma apart, so they start inside the well
    body = configs.cube5()
    q = np.ascontiguousarray(sampling.uniform_quaternions(sampling.rng(31), 2))
    u = np.array([0.9, 0.15, -0.1])
    u /= np.linalg.norm(u)
    r = 9.0
    while beads.bead_pair(body.beads, body.beads, np.zeros(3), q[0], r * u, q[1])["rmin"] > 1.05:
        r -= 0.01
    x = np.array([[0.0, 0.0, 0.0], r * u])
    P = np.array([[0.2, 0.1, -0.1], [-0.2, -0.1, 0.1]]) * body.mass
    L = np.array([[5.0, -3.0, 2.0], [-4.0, 1.0, 6.0]])
    return body, x, P, q, L


def test_time_reversibility():
    body, x, P, q, L = _two_cubes()
    x0, q0 = x.copy(), q.copy()
    kw = dict(types=[0, 0], templates=[body.beads], masses=[body.mass],
              inertias=[body.inertia], box=None, dt=0.005)
    beads.nve(x, P, q, L, steps=200, **kw)
    P *= -1
    L *= -1
    beads.nve(x, P, q, L, steps=200, **kw)
    # exact in exact arithmetic; rounding grows along the 400 steps
    np.testing.assert_allclose(x, x0, atol=1e-7)
    assert max(_qdist(q[i], q0[i]) for i in range(2)) < 1e-7


def test_energy_conservation_two_bodies():
    body, x, P, q, L = _two_cubes()
    r = beads.nve(x, P, q, L, [0, 0], [body.beads], [body.mass], [body.inertia], None, 400, 0.005)
    tot = r["pe"] + r["ke"]
    assert abs(r["pe"][0]) > 1.0             # the pair interacts
    assert np.max(np.abs(tot - tot[0])) < 2e-3 * (np.abs(r["pe"]).max() + r["ke"][0])
    # halving dt cuts the energy error about four-fold (second order)
    body, x, P, q, L = _two_cubes()
    r2 = beads.nve(x, P, q, L, [0, 0], [body.beads], [body.mass], [body.inertia], None, 800, 0.0025)
    tot2 = r2["pe"] + r2["ke"]
    e1 = np.max(np.abs(tot - tot[0]))
    e2 = np.max(np.abs(tot2 - tot2[0]))
    assert 2.5 < e1 / e2 < 6.0
