"""GPU parity at the sizes the benchmark workloads run, against the FP64
oracle: the 32768-cylinder system at t = 0 (bead forces over a list that
spans several rounds of the persistent bead kernel; network forces over
about ten rounds of the four-wave network kernel), the network gradient at
65536 rows (the persistent loop of the four-wave kernel) and the training
step at batch 8192 (32 weight-gradient chunks summed in order by Adam)."""
import numpy as np
import pytest

from oracle import beads as obeads
from oracle import frames as oframes
from oracle import mlp as omlp
from synth import sampling
from tests.tolerances import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = {0: (2e-2, 2e-2), 1: (1e-5, 1e-4)}    # precision -> (energy, gradient)
LAYER_SLICES = [(0, 896, "W1"), (896, 1024, "b1"), (1024, 17408, "W2"), (17408, 17536, "b2"),
                (17536, 33920, "W3"), (33920, 34048, "b3"), (34048, 50432, "W4"), (50432, 50560, "b4"),
                (50560, 50688, "W5"), (50688, 50689, "b5")]


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12199_amd import abi as _abi
    return _abi


@pytest.fixture(scope="module")
def cyl(cyl_workload):
    return cyl_workload


def _net(params, prec):
    return omlp.bf16_network(params) if prec == 0 else params.astype(np.float64)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _system(cfg, st, margin=None):
    from paper_2402_12199_amd.md import RigidSystem
    b = cfg.body
    return RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin, margin=margin)


def _params(seed):
    params = sampling.xavier_params(seed).astype(np.float32)
    g = sampling.rng(seed + 1)
    layers = omlp.unpack(params.astype(np.float64))
    return omlp.pack([(W, g.normal(size=b.shape) * 0.1) for W, b in layers]).astype(np.float32)


def test_config5_bead_forces_match_oracle(abi, cyl):
    # 148k listed pairs: about 4.5 rounds of 64 pairs for each of the
    # persistent kernel's blocks (at most 2 blocks per CU x 256 CUs), so the
    # alternating queues run over several rounds; the two-level form must
    # give the same sums bit for bit
    cfg, st, pairs = cyl
    assert len(pairs) >= 3 * 2 * 256 * 64
    one = _system(cfg, st)
    one.init_forces("bead")
    f = one.check_capacity()
    assert f[abi.RB_FLAG_NPAIRS] == len(pairs)
    two = _system(cfg, st, margin=cfg.bead_margin)
    two.init_forces("bead")
    two.check_capacity()
    for name in ("force", "torque", "ev"):
        assert torch.equal(getattr(one, name), getattr(two, name)), name
    ref = obeads.bead_system(st["x"], st["q"], st["types"], [cfg.body.beads], cfg.box)
    assert one.energy() == pytest.approx(ref["E"], rel=1e-5)
    assert_close(one.force.cpu().numpy().T, ref["F"], 1e-4, "force")
    assert_close(one.torque.cpu().numpy().T, ref["tau"], 1e-4, "torque")
    W = one.ev[1:].cpu().numpy().reshape(3, 3)
    np.testing.assert_allclose(W, ref["virial"], rtol=1e-4, atol=1e-4 * np.abs(ref["virial"]).max())


def _mixed_oracle(cfg, st, pairs, params, prec, norm, sw_lo, sw_hi):
    """Per-body F, tau and total E of the mixed path in FP64: the network
    (switched energy) for d_min <= |d|, the bead sum below."""
    b = cfg.body
    n = cfg.n_bodies
    x, q = st["x"], st["q"]
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    u = oframes.descriptors(x[pairs[:, 0]], q[pairs[:, 0]], x[pairs[:, 1]], q[pairs[:, 1]], cfg.box)
    u = u.astype(np.float32).astype(np.float64)      # the kernels see FP32 descriptors
    r = np.linalg.norm(u[:, :3], axis=1)
    nnm = r >= cfg.d_min
    Ep, g = omlp.input_grad(_net(params, prec), u[nnm], norm)
    rn, un = r[nnm], u[nnm]
    t = np.clip((rn - sw_lo) / (sw_hi - sw_lo), 0, 1)
    S = 1 - t * t * (3 - 2 * t)
    dS = np.where((rn > sw_lo) & (rn < sw_hi), -6 * t * (1 - t) / (sw_hi - sw_lo), 0.0)
    g = g * S[:, None]
    g[:, :3] += (Ep * dS / rn)[:, None] * un[:, :3]
    pn = pairs[nnm]
    ft = oframes.to_lab(q[pn[:, 0]], oframes.forces_from_grad(un, g))
    E = float(np.sum(S * Ep))
    np.add.at(F, pn[:, 0], -ft[:, :3])
    np.add.at(F, pn[:, 1], ft[:, :3])
    np.add.at(T, pn[:, 0], ft[:, 3:6])
    np.add.at(T, pn[:, 1], ft[:, 6:])
    for i, j in pairs[~nnm]:
        o = obeads.bead_pair(b.beads, b.beads, x[i], q[i], x[j], q[j], box=cfg.box)
        E += o["E"]
        F[i] += o["Fi"]
        F[j] += o["Fj"]
        T[i] += o["taui"]
        T[j] += o["tauj"]
    return E, F, T, int((nnm & (r < sw_hi)).sum()), int((~nnm).sum())


@pytest.mark.parametrize("prec", [0, 1])
def test_config5_network_forces_match_oracle(abi, cyl, prec):
    # about 1.1e5 network pairs: the persistent loop of the four-wave forces
    # kernel (256 blocks x 3 tiles of 16 pairs per round) runs about nine
    # rounds; bead fallback below d_min
    from paper_2402_12199_amd.md import NNModel
    cfg, st, pairs = cyl
    params = _params(1)
    norm = omlp.Norm(in_shift=np.array([0.1, -0.1, 0.05, 0, 0, 0, 0]),
                     in_scale=np.array([1 / cfg.d_cut] * 3 + [1.0] * 4), out_shift=-1.5, out_scale=6.0)
    sw_lo, sw_hi = cfg.d_cut - 1.0, cfg.d_cut
    sysm = _system(cfg, st)
    sysm.set_nn(NNModel(params=_dev(params), norm=norm.as_array(), precision=prec, d_min=cfg.d_min,
                        sw_lo=sw_lo, sw_hi=sw_hi))
    sysm.build_pairs(always=True)
    sysm.compute_forces("nn")
    f = sysm.check_capacity()
    E, F, T, n_nn, n_bead = _mixed_oracle(cfg, st, pairs, params, prec, norm, sw_lo, sw_hi)
    assert n_nn > 6 * 256 * 3 * 16
    assert f[abi.RB_FLAG_NNN] == n_nn and f[abi.RB_FLAG_NBEAD] == n_bead
    etol, gtol = RTOL[prec]
    assert sysm.energy() == pytest.approx(E, rel=max(etol, 1e-5))
    assert_close(sysm.force.cpu().numpy().T, F, max(gtol, 1e-4), "force")
    assert_close(sysm.torque.cpu().numpy().T, T, max(gtol, 1e-4), "torque")


@pytest.mark.parametrize("prec", [0, 1])
def test_network_gradient_65536_rows_matches_oracle(abi, prec):
    # 4096 tiles: the four-wave kernel's persistent loop (768 tiles per
    # round on 256 CUs) runs six rounds
    n = 1 << 16
    params = _params(21)
    norm = omlp.Norm(in_shift=np.array([0.1, -0.1, 0.05, 0, 0, 0, 0]),
                     in_scale=np.array([1 / 11.138] * 3 + [1.0] * 4), out_shift=-1.5, out_scale=6.0)
    desc = sampling.pair_batch(sampling.rng(23), n, 4.2, 11.138).astype(np.float32)
    gE = sampling.rng(24).uniform(0.5, 1.5, size=n).astype(np.float32)
    E = torch.full((n,), float("nan"), device="cuda")
    g = torch.full((7, n), float("nan"), device="cuda")
    ft = torch.full((9, n), float("nan"), device="cuda")
    abi.rb_nn_pair_grad(_dev(params), norm.as_array(), prec, _dev(desc.T), _dev(gE), E, g, ft)
    Er, gr = omlp.input_grad(_net(params, prec), desc.astype(np.float64), norm)
    gr = gr * gE[:, None]
    ftr = oframes.forces_from_grad(desc.astype(np.float64), gr)
    etol, gtol = RTOL[prec]
    assert_close(E.cpu().numpy(), Er, etol, "E")
    assert_close(g.cpu().numpy().T, gr, gtol, "dE/du")
    got = ft.cpu().numpy().T
    for s, name in ((0, "F_j"), (3, "tau_i"), (6, "tau_j")):
        assert_close(got[:, s:s + 3], ftr[:, s:s + 3], gtol, name)


def _train_problem(n_data, seed=5):
    g = sampling.rng(seed)
    params = sampling.xavier_params(seed)
    layers = omlp.unpack(params)
    params = omlp.pack([(W, g.normal(size=b.shape) * 0.05) for W, b in layers]).astype(np.float32)
    desc = sampling.pair_batch(g, n_data, 4.0, 11.138).astype(np.float32)
    labels = (g.normal(size=n_data) * 3.0 + 1.0).astype(np.float32)
    norm = omlp.Norm(in_scale=np.array([1 / 11.138] * 3 + [1.0] * 4), out_shift=0.5, out_scale=2.5)
    return params, desc, labels, norm


@pytest.mark.parametrize("prec", [0, 1])
def test_training_step_batch_8192_matches_oracle(abi, prec):
    # the batch size of the training workload: 32 chunks of 256 rows, whose
    # partial gradients Adam sums in order (the 32-wide load loop)
    batch = 8192
    params, desc, labels, norm = _train_problem(12000)
    idx = sampling.rng(11).choice(len(labels), batch, replace=False).astype(np.int32)
    p = _dev(params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros_like(p)
    ws = torch.zeros(abi.rb_nn_train_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
    abi.rb_nn_train_step(p, m, v, 1, norm.as_array(), prec, batch, _dev(desc.T), _dev(labels), _dev(idx),
                         1e-3, 0.9, 0.999, 1e-8, loss, grad, ws)
    lref, gref = omlp.loss_and_grad(_net(params, prec), desc[idx].astype(np.float64),
                                    labels[idx].astype(np.float64), norm)
    tol = 2e-2 if prec == 0 else 1e-4
    assert loss.item() == pytest.approx(lref, rel=tol)
    gg = grad.cpu().numpy()
    for a, b, name in LAYER_SLICES:
        assert_close(gg[a:b], gref[a:b], tol, f"grad {name}")
    pref, mref, _ = omlp.adam_step(params.astype(np.float64), 0.0, 0.0, 1, gg.astype(np.float64))
    np.testing.assert_allclose(p.cpu().numpy(), pref, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(m.cpu().numpy(), mref, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("prec", [0, 1])
def test_force_matching_step_batch_8192_matches_oracle(abi, prec):
    # the workload's batch with force/torque matching: 8192 primal and 8192
    # tangent rows through the four-wave kernel's persistent loop and 64
    # weight-gradient chunks (biases from the first 32 only)
    from tests.test_gpu_train import fm_step_vs_oracle
    fm_step_vs_oracle(abi, prec, 8192, 12000, lam=30.0)
