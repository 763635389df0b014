"""Pins of the oracle's symmetry-reduced cube-pair descriptor (supplementary
section 1): invariance under the cube's symmetries, completeness (the bead
energy is a function of the descriptor), ranges, and forces/torques of an
energy written in it by the chain rule through its Jacobian."""
import itertools

import numpy as np
import pytest

from oracle import beads, frames, mlp, symmetry
from synth import configs, sampling


def _signed_perms():
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1.0, -1.0], repeat=3):
            g = np.zeros((3, 3))
            for r, c in enumerate(perm):
                g[r, c] = signs[r]
            out.append(g)
    return out


def _quat(M):
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(M).as_quat()
    return np.array([w, x, y, z])


def _pairs(n, seed):
    return sampling.pair_batch(sampling.rng(seed), n, 6.0, 11.2)


def test_ranges():
    s = symmetry.cube_angles(_pairs(400, 1))
    assert np.all(s[:, 0] >= s[:, 1]) and np.all(s[:, 1] >= s[:, 2]) and np.all(s[:, 2] >= 0)
    assert np.all(s[:, 3] >= 0) and np.all(s[:, 3] <= np.arccos(1 / np.sqrt(3)) + 1e-12)
    assert np.all(s[:, 4] > -np.pi) and np.all(s[:, 4] <= np.pi)
    assert np.all(s[:, 5] >= 0) and np.all(s[:, 5] < np.pi / 2)


def test_invariant_under_the_cube_symmetries():
    # relabelling body 1's axes (48 signed permutations, reflections
    # included) and turning body 2 by any of its 24 self-rotations leave the
    # descriptor unchanged
    desc = _pairs(30, 2)
    s = symmetry.cube_angles(desc)
    G = _signed_perms()
    H = [g for g in G if np.linalg.det(g) > 0]
    assert len(G) == 48 and len(H) == 24
    R = symmetry.rotation_matrices(desc[:, 3:7])
    rng = np.random.default_rng(3)
    for g in G:
        h = H[rng.integers(len(H))]
        moved = np.array([np.concatenate([g @ d, _quat(g @ Rn @ g.T @ h)]) for d, Rn in zip(desc[:, :3], R)])
        np.testing.assert_allclose(symmetry.cube_angles(moved), s, atol=1e-10)


def test_bead_energy_is_a_function_of_the_descriptor():
    # the configuration rebuilt from s has the same bead energy, force and
    # torque magnitudes, and the same descriptor
    body = configs.cube6()
    T = body.beads.astype(np.float32).astype(np.float64)
    desc = _pairs(120, 4)
    s = symmetry.cube_descriptor(desc)
    rec = symmetry.cube_configuration(s)
    np.testing.assert_allclose(symmetry.cube_descriptor(rec), s, atol=1e-12)
    a, b = beads.bead_pair_desc(T, T, desc), beads.bead_pair_desc(T, T, rec)
    np.testing.assert_allclose(b[:, 0], a[:, 0], rtol=1e-11, atol=1e-12)
    for lo in (1, 4, 7):
        np.testing.assert_allclose(np.linalg.norm(b[:, lo:lo + 3], axis=1), np.linalg.norm(a[:, lo:lo + 3], axis=1),
                                   rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_chain_rule_forces_of_an_energy_in_the_descriptor(seed):
    # E = net(s(d, q)): F_j, tau_j from g_u = J^T g_s and the closed form
    # against central differences of the whole chain in the lab frame
    p = sampling.xavier_params(60 + seed)
    nrm = mlp.Norm(in_scale=np.array([0.2, 0.2, 0.2, 2.0, 2.0, 1.0, 1.0]))
    g = sampling.rng(70 + seed)
    qi, qj = sampling.uniform_quaternions(g, 2)
    xi = np.zeros(3)
    xj = sampling.uniform_directions(g, 1)[0] * 8.0

    def E(xj_, qj_):
        u = frames.descriptors(xi, qi, xj_, qj_)[None, :]
        return mlp.forward(p, symmetry.cube_descriptor(u), nrm)[0]

    u = frames.descriptors(xi, qi, xj, qj)[None, :]
    _, gs = mlp.input_grad(p, symmetry.cube_descriptor(u), nrm)
    gu = np.einsum("pk,pkm->pm", gs, symmetry.cube_descriptor_jacobian(u))
    lab = frames.to_lab(qi[None, :], frames.forces_from_grad(u, gu))[0]
    h = 1e-5
    sc = max(np.abs(lab).max(), 1e-3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd_F = -(E(xj + e, qj) - E(xj - e, qj)) / (2 * h)
        fd_t = -(E(xj, frames.qmul(frames.qexp(e), qj)) - E(xj, frames.qmul(frames.qexp(-e), qj))) / (2 * h)
        assert lab[a] == pytest.approx(fd_F, abs=1e-6 * sc)
        assert lab[6 + a] == pytest.approx(fd_t, abs=1e-6 * sc)


def test_smooth_form_carries_the_angles():
    # the network's seven numbers give the paper's six back, and stay smooth
    # where the angles are not: w on the x axis (alpha_2 undefined) and
    # alpha_3 at its cut
    desc = _pairs(300, 6)
    a = symmetry.cube_angles(desc)
    np.testing.assert_allclose(symmetry.angles_of(symmetry.cube_descriptor(desc)), a, atol=1e-12)
    s = symmetry.cube_descriptor(symmetry.cube_configuration(np.array([[8.0, 2.0, 1.0, 0.0, 0.0, 1.0, 0.0]])))
    np.testing.assert_allclose(s, [[8.0, 2.0, 1.0, 0.0, 0.0, 1.0, 0.0]], atol=1e-12)
    eps = 1e-7
    lo = symmetry.cube_descriptor(symmetry.cube_configuration(
        np.array([[8.0, 2.0, 1.0, 0.1, 0.2, np.cos(4 * eps), np.sin(4 * eps)]])))
    hi = symmetry.cube_descriptor(symmetry.cube_configuration(
        np.array([[8.0, 2.0, 1.0, 0.1, 0.2, np.cos(-4 * eps), np.sin(-4 * eps)]])))
    assert np.abs(lo - hi).max() < 1e-5
