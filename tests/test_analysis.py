"""Observables used to compare trajectories (host-side numpy)."""
import numpy as np
from scipy.spatial.transform import Rotation

from paper_2402_12199_amd import analysis


def test_rotate_matches_rotation_matrices():
    g = np.random.default_rng(1)
    q = g.normal(size=(40, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    v = g.normal(size=(40, 3))
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()     # scipy: scalar last
    np.testing.assert_allclose(analysis.rotate(q, v), np.einsum("nij,nj->ni", R, v), atol=1e-12)


def test_rdf_of_ideal_gas_is_one():
    g = np.random.default_rng(2)
    box = 40.0
    x = g.random((12000, 3)) * box + box * g.integers(-2, 3, (12000, 3))   # any periodic image
    r, gr = analysis.rdf(x, box, 6.0, 40)
    assert np.all(np.abs(gr[10:] - 1.0) < 0.05)
    assert abs(gr[10:].mean() - 1.0) < 0.01


def test_rdf_of_a_lattice_peaks_at_the_spacing():
    a, m = 2.0, 10
    c = np.arange(m) * a
    x = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    r, gr = analysis.rdf(x, m * a, 3.0, 60)
    hit = r[gr > 0]
    # neighbours only at a (6) and a sqrt(2) (12) below 3
    assert abs(hit[0] - a) <= 3.0 / 60 and abs(hit[1] - a * np.sqrt(2)) <= 3.0 / 60 and len(hit) == 2
    # the shells hold 6 and 12 neighbours per body
    dr = r[1] - r[0]
    rho = len(x) / (m * a) ** 3
    counts = gr * rho * 4 * np.pi * r ** 2 * dr
    np.testing.assert_allclose(counts[gr > 0], [6, 12], rtol=0.05)


def test_p2_limits():
    n = 2000
    aligned = np.tile([1.0, 0, 0, 0], (n, 1))
    assert abs(analysis.p2(aligned) - 1.0) < 1e-12
    # axis z spread uniformly in the xy plane: Q has eigenvalue 1/4 twice and -1/2 once
    t = np.linspace(0, np.pi, n, endpoint=False)
    q = np.stack([np.cos(np.pi / 4) * np.ones(n), np.sin(np.pi / 4) * np.cos(t), np.sin(np.pi / 4) * np.sin(t),
                  np.zeros(n)], 1)        # rotations by 90 degrees about in-plane axes
    assert abs(analysis.p2(q) - 0.25) < 1e-3
    g = np.random.default_rng(3)
    r = g.normal(size=(200000, 4))
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    assert analysis.p2(r) < 0.01


def test_msd_and_rdf_distance():
    x0 = np.zeros((5, 3))
    x = np.tile([1.0, 2.0, 2.0], (5, 1))
    assert analysis.msd(x0, x) == 9.0
    r = np.linspace(0.05, 5, 50)
    g1 = np.ones(50)
    assert analysis.rdf_distance(r, g1, g1) == 0.0
    assert abs(analysis.rdf_distance(r, g1, 2 * g1) - 1.0) < 1e-12


def test_msr_closed_forms():
    g = np.random.default_rng(5)
    n = 20000
    q0 = g.normal(size=(n, 4))
    q0 /= np.linalg.norm(q0, axis=1, keepdims=True)
    assert abs(analysis.msr(q0, q0)) < 1e-14
    assert abs(analysis.msr(q0, -q0)) < 1e-14            # q and -q are the same orientation
    # a turn by theta about any body axis: distance sin^2(theta / 2)
    theta = 0.7
    axis = g.normal(size=(n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    r = Rotation.from_quat(q0[:, [1, 2, 3, 0]]) * Rotation.from_rotvec(theta * axis)
    q1 = r.as_quat()[:, [3, 0, 1, 2]]
    assert abs(analysis.msr(q0, q1) - np.sin(theta / 2) ** 2) < 1e-12
    # independent uniform orientations: <q0, q>^2 averages 1/4 on S^3, so 3/4
    q2 = g.normal(size=(n, 4))
    q2 /= np.linalg.norm(q2, axis=1, keepdims=True)
    assert abs(analysis.msr(q0, q2) - 0.75) < 0.01
