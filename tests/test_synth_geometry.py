"""Bead templates and box sizes of the workloads, against hand arithmetic."""
import numpy as np
import pytest

from synth import configs, sampling


def test_bead_counts_com_inertia():
    c5, c6, cy = configs.cube5(), configs.cube6(), configs.cyl134()
    assert (c5.n, c6.n, cy.n) == (98, 152, 134)          # n^3 - (n-2)^3; 8*12 + 2*19
    for b in (c5, c6, cy):
        np.testing.assert_allclose(b.beads.mean(axis=0), 0, atol=1e-12)
    # cube shell: I = 2 * (sum of y^2 over the full lattice minus the interior)
    np.testing.assert_allclose(c5.inertia, 2 * (25 * 10 - 9 * 2), rtol=1e-12)        # 464
    np.testing.assert_allclose(c6.inertia, 2 * (36 * 17.5 - 16 * 5), rtol=1e-12)     # 1100
    # cylinder: I_zz = 96 * 1.5^2 + 2 * (6 * 0.75^2 + 12 * 1.5^2)
    izz = 96 * 2.25 + 2 * (6 * 0.5625 + 12 * 2.25)
    szz = 12 * 0.81 * 42 + 38 * 4.05 ** 2
    np.testing.assert_allclose(cy.inertia, [izz / 2 + szz, izz / 2 + szz, izz], rtol=1e-12)
    assert cy.r_max == pytest.approx(np.hypot(1.5, 4.05))
    assert c6.r_max == pytest.approx(2.5 * np.sqrt(3))


def test_box_lengths():
    assert configs.config1().box == pytest.approx((64 * 125 / 0.1) ** (1 / 3))
    assert configs.config2().box == pytest.approx((4096 * 216 / 0.2) ** (1 / 3))
    assert configs.config5().box == pytest.approx((32768 * np.pi * 4 * 9.1 / 0.15) ** (1 / 3))


def test_placement_respects_bead_gap():
    from scipy.spatial import cKDTree
    from scipy.spatial.transform import Rotation
    cfg = configs.config1()
    x, q = sampling.place_bodies(sampling.rng(cfg.seed), cfg.n_bodies, cfg.body, cfg.box)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    pts = (x[:, None, :] + np.einsum("nab,kb->nka", R, cfg.body.beads)) % cfg.box
    owner = np.repeat(np.arange(len(x)), cfg.body.n)
    tree = cKDTree(pts.reshape(-1, 3), boxsize=cfg.box)
    for a, b in tree.query_pairs(1.0 - 1e-9):
        assert owner[a] == owner[b]


def test_quaternions_unit_and_uniform_moments():
    q = sampling.uniform_quaternions(sampling.rng(0), 200000)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1, rtol=1e-12)
    # uniform on S^3: E[q_c^2] = 1/4, E[q_c] = 0
    np.testing.assert_allclose((q * q).mean(axis=0), 0.25, atol=3e-3)
    np.testing.assert_allclose(q.mean(axis=0), 0, atol=5e-3)
