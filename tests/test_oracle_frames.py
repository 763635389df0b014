"""Pins of the oracle's descriptors and of forces/torques from an energy's
gradient in those descriptors (supplementary section 6 defines
f = -dE/dx and tau = -dE/dtheta)."""
import numpy as np
import pytest

from oracle import beads, frames, mlp
from synth import configs, sampling


def _state(seed):
    g = sampling.rng(seed)
    q = sampling.uniform_quaternions(g, 2)
    xi = g.normal(size=3) * 3
    xj = xi + sampling.uniform_directions(g, 1)[0] * g.uniform(5, 9)
    return xi, q[0], xj, q[1]


def test_quaternion_rotation_matches_matrix_convention():
    # a quarter turn about z maps x to y
    q = frames.qexp(np.array([0, 0, np.pi / 2]))
    np.testing.assert_allclose(frames.qrotate(q, np.array([1.0, 0, 0])), [0, 1, 0], atol=1e-15)
    # composition: R(a b) = R(a) R(b)
    a, b = sampling.uniform_quaternions(sampling.rng(1), 2)
    v = np.array([0.3, -1.2, 2.0])
    np.testing.assert_allclose(frames.qrotate(frames.qmul(a, b), v),
                               frames.qrotate(a, frames.qrotate(b, v)), atol=1e-14)


def test_descriptor_definition_and_invariance():
    xi, qi, xj, qj = _state(3)
    u = frames.descriptors(xi, qi, xj, qj)
    # body j's frame seen from body i: R(q_rel) = R_i^T R_j
    v = np.array([0.7, 0.1, -0.5])
    np.testing.assert_allclose(frames.qrotate(u[3:], v),
                               frames.qrotate(frames.qconj(qi), frames.qrotate(qj, v)), atol=1e-14)
    np.testing.assert_allclose(frames.qrotate(qi, u[:3]), xj - xi, atol=1e-13)
    # unchanged by a global rotation and translation of the pair
    g = frames.qexp(np.array([1.0, 0.2, -0.3]))
    s = np.array([5.0, 6.0, -7.0])
    u2 = frames.descriptors(frames.qrotate(g, xi) + s, frames.qmul(g, qi),
                            frames.qrotate(g, xj) + s, frames.qmul(g, qj))
    np.testing.assert_allclose(u2, u, atol=1e-13)
    # periodic image
    u3 = frames.descriptors(xi, qi, xj + np.array([30.0, 0, -30.0]), qj, box=30.0)
    np.testing.assert_allclose(u3, u, atol=1e-12)


def _chain_energy(p, nrm):
    def E(xi, qi, xj, qj):
        return mlp.forward(p, frames.descriptors(xi, qi, xj, qj)[None, :], nrm)[0]
    return E


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_closed_form_torques_match_full_chain_differences(seed):
    p = sampling.xavier_params(40 + seed)
    nrm = mlp.Norm(in_scale=np.array([1 / 11.0] * 3 + [1.0] * 4))
    E = _chain_energy(p, nrm)
    xi, qi, xj, qj = _state(seed)
    u = frames.descriptors(xi, qi, xj, qj)[None, :]
    _, g = mlp.input_grad(p, u, nrm)
    lab = frames.to_lab(qi[None, :], frames.forces_from_grad(u, g))[0]
    Fj, taui, tauj = lab[:3], lab[3:6], lab[6:]
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd_Fj = -(E(xi, qi, xj + e, qj) - E(xi, qi, xj - e, qj)) / (2 * h)
        fd_Fi = -(E(xi + e, qi, xj, qj) - E(xi - e, qi, xj, qj)) / (2 * h)
        rp, rm = frames.qexp(e), frames.qexp(-e)
        fd_tj = -(E(xi, qi, xj, frames.qmul(rp, qj)) - E(xi, qi, xj, frames.qmul(rm, qj))) / (2 * h)
        fd_ti = -(E(xi, frames.qmul(rp, qi), xj, qj) - E(xi, frames.qmul(rm, qi), xj, qj)) / (2 * h)
        sc = max(np.abs(lab).max(), 1e-3)
        assert Fj[a] == pytest.approx(fd_Fj, abs=1e-7 * sc)
        assert -Fj[a] == pytest.approx(fd_Fi, abs=1e-7 * sc)
        assert tauj[a] == pytest.approx(fd_tj, abs=1e-7 * sc)
        assert taui[a] == pytest.approx(fd_ti, abs=1e-7 * sc)


def test_closed_form_matches_bead_sum_forces():
    # An independent pin: take the bead double sum itself as E(d, q/|q|),
    # differentiate it numerically in the 7 descriptor numbers and push the
    # gradient through the closed form; it must reproduce the bead sum's own
    # directly accumulated forces and torques.
    body = configs.cube5()
    g = sampling.rng(21)
    for _ in range(3):
        while True:
            u = sampling.pair_batch(g, 1, 5.2, 6.5)
            ref = beads.bead_pair_desc(body.beads, body.beads, u)[0]
            if ref[10] > 0.9 and abs(ref[0]) > 1e-2:
                break
        h = 1e-6
        gr = np.zeros((1, 7))
        for k in range(7):
            up, um = u.copy(), u.copy()
            up[0, k] += h
            um[0, k] -= h
            gr[0, k] = (beads.bead_pair_desc(body.beads, body.beads, up)[0, 0]
                        - beads.bead_pair_desc(body.beads, body.beads, um)[0, 0]) / (2 * h)
        ft = frames.forces_from_grad(u, gr)[0]
        np.testing.assert_allclose(ft, ref[1:10], rtol=1e-5, atol=1e-6 * np.abs(ref[1:10]).max())


def test_orientation_only_columns_zero_gives_no_torque_on_j():
    p = sampling.xavier_params(5)
    layers = mlp.unpack(p)
    W1, b1 = layers[0]
    W1 = W1.copy()
    W1[:, 3:] = 0.0
    layers[0] = (W1, b1)
    p = mlp.pack(layers)
    u = sampling.pair_batch(sampling.rng(6), 8, 4, 11)
    _, g = mlp.input_grad(p, u)
    ft = frames.forces_from_grad(u, g)
    np.testing.assert_allclose(ft[:, 6:], 0, atol=1e-15)
    np.testing.assert_allclose(ft[:, 3:6], np.cross(u[:, :3], g[:, :3]), rtol=1e-12)


def test_identities_and_quaternion_sign():
    u = sampling.pair_batch(sampling.rng(7), 50, 4, 11)
    g = sampling.rng(8).normal(size=(50, 7))
    ft = frames.forces_from_grad(u, g)
    # torque balance about x_i: tau_i + tau_j + d x F_j = 0
    np.testing.assert_allclose(ft[:, 3:6] + ft[:, 6:] + np.cross(u[:, :3], ft[:, :3]), 0, atol=1e-12)
    # q and -q are the same orientation; the gradient flips sign with q
    u2, g2 = u.copy(), g.copy()
    u2[:, 3:] *= -1
    g2[:, 3:] *= -1
    np.testing.assert_allclose(frames.forces_from_grad(u2, g2), ft, atol=1e-13)
    # a purely radial quaternion gradient (g_q parallel to q) gives no torque
    g3 = np.zeros_like(g)
    g3[:, 3:] = u[:, 3:] * 2.5
    np.testing.assert_allclose(frames.forces_from_grad(u, g3)[:, 6:], 0, atol=1e-13)
