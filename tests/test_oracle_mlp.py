"""Pins of the oracle network (paper section 2: g_NN_U maps the pair
configuration to the energy) against closed forms and finite differences."""
import numpy as np
import pytest

from oracle import frames, mlp
from synth import sampling


def _norm():
    return mlp.Norm(in_shift=np.array([0.1, -0.2, 0.3, 0, 0, 0, 0.05]),
                    in_scale=np.array([1 / 11.0] * 3 + [1.0] * 4),
                    out_shift=-3.0, out_scale=7.5)


def _inputs(n, seed=5):
    return sampling.pair_batch(sampling.rng(seed), n, 4.2, 11.1)


def test_silu_values():
    # SiLU(z) = z * sigmoid(z): SiLU(0) = 0, slope 1/2 at 0, SiLU(1) = 1/(1+1/e)
    z = np.array([0.0, 1.0, -1.0, 40.0, -40.0])
    np.testing.assert_allclose(mlp.act(z), [0.0, 0.7310585786300049, -0.2689414213699951, 40.0,
                                             -40.0 * np.exp(-40.0)], rtol=1e-12, atol=1e-300)
    assert mlp.act_grad(np.array([0.0]))[0] == pytest.approx(0.5)


def test_identity_activation_collapses_to_one_affine_map():
    p = sampling.xavier_params(3)
    layers = mlp.unpack(p)
    rng = sampling.rng(9)
    # non-zero biases so the folded bias is exercised
    p = mlp.pack([(W, rng.normal(size=b.shape)) for W, b in layers])
    layers = mlp.unpack(p)
    M = np.eye(7)
    c = np.zeros(7)
    for W, b in layers:
        c = W @ c + b
        M = W @ M
    nrm = _norm()
    u = _inputs(64)
    un = (u - nrm.in_shift) * nrm.in_scale
    want = (un @ M.T + c)[:, 0] * nrm.out_scale + nrm.out_shift
    np.testing.assert_allclose(mlp.forward(p, u, nrm, kind="identity"), want, rtol=1e-12)
    # and the input gradient of an affine map is its matrix row
    _, g = mlp.input_grad(p, u, nrm, kind="identity")
    np.testing.assert_allclose(g, np.broadcast_to(M[0] * nrm.in_scale * nrm.out_scale, g.shape),
                               rtol=1e-12)


def test_input_gradient_central_differences_h1e4():
    # the workload checks the network gradient by central differences, h = 1e-4
    p = sampling.xavier_params(1003)
    nrm = _norm()
    u = _inputs(32)
    E, g = mlp.input_grad(p, u, nrm)
    h = 1e-4
    for k in range(7):
        up, um = u.copy(), u.copy()
        up[:, k] += h
        um[:, k] -= h
        fd = (mlp.forward(p, up, nrm) - mlp.forward(p, um, nrm)) / (2 * h)
        np.testing.assert_allclose(g[:, k], fd, rtol=1e-6, atol=1e-7 * np.abs(g).max())
    np.testing.assert_allclose(E, mlp.forward(p, u, nrm), rtol=0, atol=0)


def test_parameter_gradient_central_differences():
    p = sampling.xavier_params(7)
    rng = sampling.rng(8)
    p = p + 0.05 * rng.normal(size=p.size)       # non-zero biases
    nrm = _norm()
    u = _inputs(16)
    y = rng.normal(size=16) * 5
    loss, g = mlp.loss_and_grad(p, u, y, nrm)
    idx = np.concatenate([rng.choice(p.size, 60, replace=False),
                          [0, 895, 896, 1023, p.size - 129, p.size - 1]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss_and_grad(pp, u, y, nrm)[0] - mlp.loss_and_grad(pm, u, y, nrm)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adam_first_step_closed_form():
    # with m = v = 0 and t = 1 the bias-corrected step is -lr g / (|g| + eps)
    rng = sampling.rng(2)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    g[3] = 0.0
    new, m, v = mlp.adam_step(p, np.zeros(100), np.zeros(100), 1, g, lr=1e-3)
    np.testing.assert_allclose(new - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_overfits_small_set():
    p = sampling.xavier_params(11)
    u = _inputs(16, seed=12)
    y = sampling.rng(13).normal(size=16)
    nrm = mlp.Norm(in_scale=np.array([1 / 11.0] * 3 + [1.0] * 4))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    loss0 = mlp.loss_and_grad(p, u, y, nrm)[0]
    for t in range(1, 1001):
        loss, g = mlp.loss_and_grad(p, u, y, nrm)
        p, m, v = mlp.adam_step(p, m, v, t, g, lr=1e-3)
    assert loss < 1e-3 * loss0


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1);
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: rounds to 1 + 2^-6
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -3.0e-5, 65504.0], np.float32)
    want = [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, None, 65536.0]
    got = mlp.round_bf16(x)
    for g, w in zip(got, want):
        if w is not None:
            assert g == w
    assert abs(got[4] / -3.0e-5 - 1) < 2 ** -8


def _fm_case(seed, P=10):
    rng = np.random.default_rng(seed)
    p = sampling.xavier_params(seed)
    u = sampling.pair_batch(rng, P, 4.0, 11.0)
    y = rng.normal(size=P)
    ft = rng.normal(size=(P, 6))
    norm = mlp.Norm(in_shift=rng.normal(size=7) * 0.1, in_scale=rng.uniform(0.2, 0.5, size=7), out_shift=0.2,
                    out_scale=1.7)
    return p, u, y, ft, norm, rng


def test_force_matching_gradient_central_differences():
    # the exact (forward-over-reverse) parameter gradient of energy + force
    # + torque matching against central differences of the loss, on
    # parameters of every layer
    p, u, y, ft, norm, rng = _fm_case(11)
    lam_f, lam_t = 0.7, 1.3
    _, _, grad = mlp.fm_loss_and_grad(p, u, y, ft, lam_f, lam_t, norm)

    def loss(pp):
        a, b, _ = mlp.fm_loss_and_grad(pp, u, y, ft, lam_f, lam_t, norm)
        return a + b

    bounds = np.cumsum([0] + [fo * fi + fo for fi, fo in zip(mlp.DIMS[:-1], mlp.DIMS[1:])])
    idx = [int(rng.integers(lo, hi)) for lo, hi in zip(bounds[:-1], bounds[1:]) for _ in range(3)]
    idx += [int(bounds[-1] - 1), 0]
    h = 1e-5
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-5 * max(abs(fd), 1e-3), (k, grad[k], fd)


def test_force_matching_reduces_to_energy_loss_and_matches_its_forces():
    p, u, y, ft, norm, _ = _fm_case(12)
    e_loss, fm0, g0 = mlp.fm_loss_and_grad(p, u, y, ft, 0.0, 0.0, norm)
    ref_loss, ref_grad = mlp.loss_and_grad(p, u, y, norm)
    assert fm0 == 0.0 and e_loss == ref_loss
    np.testing.assert_array_equal(g0, ref_grad)
    # labels equal to the network's own forces and torques: zero matching
    # loss and no gradient beyond the energy term's
    _, g = mlp.input_grad(p, u, norm)
    own = frames.forces_from_grad(u, g)
    _, fm, g1 = mlp.fm_loss_and_grad(p, u, y, np.concatenate([own[:, :3], own[:, 6:9]], 1), 2.0, 3.0, norm)
    assert fm < 1e-25
    np.testing.assert_allclose(g1, ref_grad, rtol=0, atol=1e-12)


def test_bf16_network_rounds_exactly_the_hidden_to_hidden_weights():
    # A hand-built net of widths 7 -> 4 -> 4 -> 4 -> 4 -> 1 in which every
    # parameter is 1 + 3 * 2^-10 or, in a second pass, 1 + 5 * 2^-9.  BF16
    # keeps 7 fraction bits, so the BF16 neighbours are 1 and 1 + 2^-7: the
    # first value (3 * 2^-10 below the midpoint 2^-8) rounds to 1, the second
    # (5 * 2^-9 above it) to 1 + 2^-7.  Only W2, W3 and W4 may change, each
    # element to that hand-computed value; W1, W5 and every bias must come
    # back unchanged.
    dims = (7, 4, 4, 4, 4, 1)
    n = sum(fi * fo + fo for fi, fo in zip(dims[:-1], dims[1:]))
    for val, rounded in ((1 + 3 * 2 ** -10, 1.0), (1 + 5 * 2 ** -9, 1 + 2 ** -7)):
        p = np.full(n, val, np.float32)
        assert float(p[0]) == val                      # exact in FP32
        out = mlp.unpack(mlp.bf16_network(p, dims), dims)
        assert len(out) == 5
        for li, (W, b) in enumerate(out):
            want_W = rounded if li in (1, 2, 3) else val
            np.testing.assert_array_equal(W, np.full(W.shape, want_W), err_msg=f"W{li + 1}")
            np.testing.assert_array_equal(b, np.full(b.shape, val), err_msg=f"b{li + 1}")
    # the full-size network: the same rule on the Xavier parameters, compared
    # with the element-wise rounding of each block
    p = sampling.xavier_params(3).astype(np.float32)
    p = p + np.float32(1e-3) * np.arange(p.size, dtype=np.float32) / p.size   # non-zero biases
    got = mlp.unpack(mlp.bf16_network(p))
    ref = mlp.unpack(p.astype(np.float64))
    for li, ((Wg, bg), (Wr, br)) in enumerate(zip(got, ref)):
        if li in (1, 2, 3):
            assert np.any(Wg != Wr)
            np.testing.assert_array_equal(Wg, mlp.round_bf16(Wr.astype(np.float32)))
        else:
            np.testing.assert_array_equal(Wg, Wr)
        np.testing.assert_array_equal(bg, br)
