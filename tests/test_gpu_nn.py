"""GPU parity of the network kernels (forward, hand-written input gradient,
forces/torques from it, descriptors, per-body accumulation) against the
FP64 oracle network with the same (FP32-rounded) weights."""
import numpy as np
import pytest

from oracle import beads as obeads
from oracle import frames as oframes
from oracle import mlp as omlp
from synth import configs, sampling, state
from tests.tolerances import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = {0: (2e-2, 2e-2), 1: (1e-5, 1e-4)}    # precision -> (energy, gradient)


def _net(params, prec):
    """FP64 oracle parameters of the network a precision mode implements:
    BF16 mode holds W2..W4 in BF16 (round to nearest even of the FP32 master),
    every other parameter in FP32."""
    return omlp.bf16_network(params) if prec == 0 else params.astype(np.float64)


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12199_amd import abi as _abi
    return _abi


def _setup(n, seed=1003, d_lo=4.2, d_hi=11.138):
    params = sampling.xavier_params(seed).astype(np.float32)
    # non-zero biases so every parameter block is exercised
    g = sampling.rng(seed + 1)
    layers = omlp.unpack(params.astype(np.float64))
    params = omlp.pack([(W, g.normal(size=b.shape) * 0.1) for W, b in layers]).astype(np.float32)
    norm = omlp.Norm(in_shift=np.array([0.1, -0.1, 0.05, 0, 0, 0, 0]),
                     in_scale=np.array([1 / 11.138] * 3 + [1.0] * 4), out_shift=-1.5, out_scale=6.0)
    desc = sampling.pair_batch(sampling.rng(seed + 2), n, d_lo, d_hi).astype(np.float32)
    return params, norm, desc


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [1, 37, 4099])
def test_eval_matches_oracle(abi, prec, n):
    params, norm, desc = _setup(n)
    E = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    abi.rb_nn_pair_eval(_dev(params), norm.as_array(), prec, _dev(desc.T), E)
    ref = omlp.forward(_net(params, prec), desc.astype(np.float64), norm)
    assert_close(E.cpu().numpy(), ref, RTOL[prec][0], "E")


@pytest.mark.parametrize("prec", [0, 1])
def test_grad_and_pair_forces_match_oracle(abi, prec):
    n = 3001
    params, norm, desc = _setup(n, seed=7)
    gE = sampling.rng(3).uniform(0.5, 1.5, size=n).astype(np.float32)
    E = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.zeros((7, n), dtype=torch.float32, device="cuda")
    ft = torch.zeros((9, n), dtype=torch.float32, device="cuda")
    abi.rb_nn_pair_grad(_dev(params), norm.as_array(), prec, _dev(desc.T), _dev(gE), E, g, ft)
    Er, gr = omlp.input_grad(_net(params, prec), desc.astype(np.float64), norm)
    gr = gr * gE[:, None]
    ftr = oframes.forces_from_grad(desc.astype(np.float64), gr)
    etol, gtol = RTOL[prec]
    assert_close(E.cpu().numpy(), Er, etol, "E")
    assert_close(g.cpu().numpy().T[:, :3], gr[:, :3], gtol, "dE/dd")
    assert_close(g.cpu().numpy().T[:, 3:], gr[:, 3:], gtol, "dE/dq")
    got = ft.cpu().numpy().T
    for s, name in ((0, "F_j"), (3, "tau_i"), (6, "tau_j")):
        assert_close(got[:, s:s + 3], ftr[:, s:s + 3], gtol, name)


def test_bf16_mode_against_unrounded_master_weights(abi):
    # The BF16 kernels hold W2..W4 in BF16; the trainer's FP32 master weights
    # are what dynamics and training mean by "the network".  Energy and input
    # gradient of the BF16 mode against the FP64 network on those unrounded
    # weights, at the same 2e-2 bound (weight rounding and BF16 activations
    # together).
    n = 4099
    params, norm, desc = _setup(n, seed=13)
    E = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.zeros((7, n), dtype=torch.float32, device="cuda")
    abi.rb_nn_pair_grad(_dev(params), norm.as_array(), 0, _dev(desc.T), None, E, g, None)
    Er, gr = omlp.input_grad(params.astype(np.float64), desc.astype(np.float64), norm)
    assert_close(E.cpu().numpy(), Er, 2e-2, "E vs FP32 master weights")
    assert_close(g.cpu().numpy().T, gr, 2e-2, "dE/du vs FP32 master weights")


def test_config3_full_batch_sampled_rows(abi):
    # 2^20 rows in the launch configuration of the benchmark; every output is
    # compared on a random sample of rows the oracle evaluates one by one
    cfg = configs.config3()
    params = sampling.xavier_params(cfg.seed).astype(np.float32)
    desc = sampling.pair_batch(sampling.rng(cfg.seed), cfg.n_pairs, cfg.d_lo, cfg.d_cut).astype(np.float32)
    norm = omlp.Norm(in_scale=np.array([1 / cfg.d_cut] * 3 + [1.0] * 4))
    d = _dev(desc.T)
    pick = np.sort(sampling.rng(9).choice(cfg.n_pairs, 2048, replace=False))
    pick = np.concatenate([[0, 1], pick, [cfg.n_pairs - 1]])
    for prec in (0, 1):
        E = torch.zeros(cfg.n_pairs, dtype=torch.float32, device="cuda")
        ft = torch.zeros((9, cfg.n_pairs), dtype=torch.float32, device="cuda")
        abi.rb_nn_pair_grad(_dev(params), norm.as_array(), prec, d, None, E, None, ft)
        Er, gr = omlp.input_grad(_net(params, prec), desc[pick].astype(np.float64), norm)
        ftr = oframes.forces_from_grad(desc[pick].astype(np.float64), gr)
        etol, gtol = RTOL[prec]
        assert_close(E.cpu().numpy()[pick], Er, etol, f"E prec={prec}")
        assert_close(ft.cpu().numpy().T[pick][:, :3], ftr[:, :3], gtol, f"F_j prec={prec}")
        assert_close(ft.cpu().numpy().T[pick][:, 6:], ftr[:, 6:], gtol, f"tau_j prec={prec}")
        assert torch.isfinite(E).all()


def test_autograd_function_matches_kernel_gradient(abi):
    from paper_2402_12199_amd.nn import nn_pair_energy
    params, norm, desc = _setup(513)
    d = _dev(desc.T).requires_grad_(True)
    E = nn_pair_energy(d, _dev(params), norm.as_array(), 1)
    w = torch.linspace(0.5, 2.0, 513, device="cuda")
    (E * w).sum().backward()
    _, gr = omlp.input_grad(params.astype(np.float64), desc.astype(np.float64), norm)
    assert_close(d.grad.cpu().numpy().T, gr * w.cpu().numpy()[:, None], 1e-4, "autograd grad")


def test_descriptors_match_oracle(abi):
    cfg = configs.config1()
    st = state.initial_state(cfg)
    from paper_2402_12199_amd.md import NNModel, RigidSystem
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    sysm.set_nn(NNModel(params=torch.zeros(abi.RB_MLP_NPARAMS, device="cuda"), norm=np.zeros(16, np.float32),
                        d_min=cfg.d_min))
    sysm.build_pairs(always=True)
    abi.rb_pair_descriptors(sysm.x, sysm.q, sysm.box, sysm.pair_i, sysm.pair_j, cfg.d_min, sysm.desc,
                            sysm.idx_nn, sysm.idx_bead, sysm.flags)
    f = sysm.flags_host()
    pairs = sysm.pairs_host()
    ref = oframes.descriptors(st["x"][pairs[:, 0]], st["q"][pairs[:, 0]], st["x"][pairs[:, 1]],
                              st["q"][pairs[:, 1]], cfg.box)
    got = sysm.desc.cpu().numpy()[:, :len(pairs)].T
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6 * cfg.box)
    far = np.linalg.norm(ref[:, :3], axis=1) >= cfg.d_min
    assert f[abi.RB_FLAG_NNN] == far.sum() and f[abi.RB_FLAG_NBEAD] == (~far).sum()
    nn = np.sort(sysm.idx_nn.cpu().numpy()[:f[abi.RB_FLAG_NNN]])
    np.testing.assert_array_equal(nn, np.nonzero(far)[0])


def test_routing_window_and_pair_configurations(abi):
    # pairs below d_lo go to the bead list, d_lo <= |d| < d_hi to the network
    # list, the rest to neither; pair_configurations returns the network
    # window's descriptors in list order
    cfg = configs.config1()
    st = state.initial_state(cfg)
    from paper_2402_12199_amd.md import RigidSystem
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    sysm.build_pairs(always=True)
    pairs = sysm.pairs_host()
    ref = oframes.descriptors(st["x"][pairs[:, 0]], st["q"][pairs[:, 0]], st["x"][pairs[:, 1]],
                              st["q"][pairs[:, 1]], cfg.box)
    r = np.linalg.norm(ref[:, :3], axis=1)
    d_lo, d_hi = (float(v) for v in np.quantile(r, [0.3, 0.7]))
    got = sysm.pair_configurations(d_lo, d_hi).cpu().numpy().T
    win = (r >= d_lo) & (r < d_hi)
    assert got.shape == (win.sum(), 7)
    np.testing.assert_allclose(got, ref[win], rtol=0, atol=2e-6 * cfg.box)
    f = sysm.flags_host()
    assert f[abi.RB_FLAG_NNN] == win.sum() and f[abi.RB_FLAG_NBEAD] == (r < d_lo).sum()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("cfgname", ["config1", "config2"])
def test_md_forces_nn_plus_bead_fallback_match_oracle(abi, prec, cfgname):
    # per-body forces of the mixed path: network for |d| >= d_min (with the
    # energy switch), bead sum below, against the oracle doing the same; the
    # 4096-cube system is the launch the benchmark times (about 9.5k network
    # pairs, 600 tiles)
    from paper_2402_12199_amd.md import NNModel, RigidSystem
    cfg = getattr(configs, cfgname)()
    st = state.initial_state(cfg)
    b = cfg.body
    params, norm, _ = _setup(1)
    sw_lo, sw_hi = cfg.d_cut - 1.0, cfg.d_cut
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    sysm.set_nn(NNModel(params=_dev(params), norm=norm.as_array(), precision=prec, d_min=cfg.d_min,
                        sw_lo=sw_lo, sw_hi=sw_hi))
    sysm.build_pairs(always=True)
    sysm.compute_forces("nn")
    f = sysm.check_capacity()
    pairs = obeads.pairs_within(st["x"], cfg.box, cfg.r_list)
    n = cfg.n_bodies
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    E = 0.0
    x, q = st["x"], st["q"]
    u = oframes.descriptors(x[pairs[:, 0]], q[pairs[:, 0]], x[pairs[:, 1]], q[pairs[:, 1]], cfg.box)
    # the kernels see FP32 descriptors
    u = u.astype(np.float32).astype(np.float64)
    r = np.linalg.norm(u[:, :3], axis=1)
    nnm = r >= cfg.d_min
    Ep, g = omlp.input_grad(_net(params, prec), u, norm)
    t = np.clip((r - sw_lo) / (sw_hi - sw_lo), 0, 1)
    S = 1 - t * t * (3 - 2 * t)
    dS = np.where((r > sw_lo) & (r < sw_hi), -6 * t * (1 - t) / (sw_hi - sw_lo), 0.0)
    g = g * S[:, None]
    g[:, :3] += (Ep * dS / r)[:, None] * u[:, :3]
    ft = oframes.to_lab(q[pairs[:, 0]], oframes.forces_from_grad(u, g))
    pi, pj = pairs[nnm, 0], pairs[nnm, 1]
    E += np.sum(S[nnm] * Ep[nnm])
    np.add.at(F, pi, -ft[nnm, :3])
    np.add.at(F, pj, ft[nnm, :3])
    np.add.at(T, pi, ft[nnm, 3:6])
    np.add.at(T, pj, ft[nnm, 6:])
    for k, (i, j) in enumerate(pairs):
        if not nnm[k]:
            o = obeads.bead_pair(b.beads, b.beads, x[i], q[i], x[j], q[j], box=cfg.box)
            E += o["E"]
            F[i] += o["Fi"]
            F[j] += o["Fj"]
            T[i] += o["taui"]
            T[j] += o["tauj"]
    assert f[abi.RB_FLAG_NNN] == (nnm & (r < sw_hi)).sum()
    etol, gtol = RTOL[prec]
    assert sysm.energy() == pytest.approx(E, rel=max(etol, 1e-5))
    assert_close(sysm.force.cpu().numpy().T, F, max(gtol, 1e-4), "force")
    assert_close(sysm.torque.cpu().numpy().T, T, max(gtol, 1e-4), "torque")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("count", [0, 1, 17, 48, 49, 130])
def test_nn_pair_forces_ragged_counts_match_oracle(abi, prec, count):
    # the dynamics forces kernel at tile- and block-ragged list lengths (16
    # pairs per tile, three tiles per block in BF16), through an index list,
    # with the count read on the device and clipped at the capacity (120)
    g = sampling.rng(2024)
    n, P, cap = 40, 160, 120
    params, norm, _ = _setup(1, seed=11)
    q = g.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    pi = g.integers(0, n, P).astype(np.int32)
    pj = ((pi + 1 + g.integers(0, n - 1, P)) % n).astype(np.int32)
    desc = sampling.pair_batch(g, P, 4.2, 11.138).astype(np.float32)
    idx = g.permutation(P)[:cap].astype(np.int32)
    sw_lo, sw_hi = 10.0, 11.138
    acc = torch.zeros(abi.acc_len(n), dtype=torch.int64, device="cuda")
    flags = torch.zeros(abi.RB_NFLAGS, dtype=torch.int32, device="cuda")
    cnt = torch.tensor([count], dtype=torch.int32, device="cuda")
    abi.rb_nn_pair_forces(_dev(params), norm.as_array(), prec, _dev(q.T), _dev(pi), _dev(pj), _dev(desc.T),
                          _dev(idx), cnt, cap, sw_lo, sw_hi, acc, flags)
    force = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    torque = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    ev = torch.zeros(10, dtype=torch.float64, device="cuda")
    abi.rb_accum_finalize(n, acc, force, torque, ev)
    m = min(count, cap)
    assert int(flags[abi.RB_FLAG_NEVAL].item()) == m
    rows = idx[:m]
    u = desc[rows].astype(np.float64)
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    W = np.zeros((3, 3))
    E = 0.0
    if m:
        r = np.linalg.norm(u[:, :3], axis=1)
        Ep, gr = omlp.input_grad(_net(params, prec), u, norm)
        t = np.clip((r - sw_lo) / (sw_hi - sw_lo), 0, 1)
        S = 1 - t * t * (3 - 2 * t)
        dS = np.where((r > sw_lo) & (r < sw_hi), -6 * t * (1 - t) / (sw_hi - sw_lo), 0.0)
        gr = gr * S[:, None]
        gr[:, :3] += (Ep * dS / r)[:, None] * u[:, :3]
        qi = q[pi[rows]]
        ft = oframes.to_lab(qi, oframes.forces_from_grad(u, gr))
        np.add.at(F, pi[rows], -ft[:, :3])
        np.add.at(F, pj[rows], ft[:, :3])
        np.add.at(T, pi[rows], ft[:, 3:6])
        np.add.at(T, pj[rows], ft[:, 6:])
        E = float(np.sum(S * Ep))
        dl = oframes.qrotate(qi, u[:, :3])
        W = dl.T @ ft[:, :3]
    etol, gtol = RTOL[prec]
    got_ev = ev.cpu().numpy()
    if m == 0:
        assert not acc.any() and not force.any() and not torque.any() and not got_ev.any()
        return
    assert got_ev[0] == pytest.approx(E, rel=max(etol, 1e-5))
    assert_close(force.cpu().numpy().T, F, max(gtol, 1e-4), "force")
    assert_close(torque.cpu().numpy().T, T, max(gtol, 1e-4), "torque")
    assert_close(got_ev[1:].reshape(3, 3), W, max(gtol, 1e-4), "virial")
