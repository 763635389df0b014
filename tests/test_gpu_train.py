"""GPU parity of the training step (hand-written reverse pass, weight
gradients, Adam) against the FP64 oracle, and a short training run on
bead-sum labels that must beat the untrained network."""
import numpy as np
import pytest

from oracle import mlp as omlp
from synth import configs, sampling
from tests.tolerances import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAYER_SLICES = [(0, 896, "W1"), (896, 1024, "b1"), (1024, 17408, "W2"), (17408, 17536, "b2"),
                (17536, 33920, "W3"), (33920, 34048, "b3"), (34048, 50432, "W4"), (50432, 50560, "b4"),
                (50560, 50688, "W5"), (50688, 50689, "b5")]


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12199_amd import abi as _abi
    return _abi


def _net(params, prec):
    return omlp.bf16_network(params) if prec == 0 else params.astype(np.float64)


def _problem(n_data=700, seed=5):
    g = sampling.rng(seed)
    params = sampling.xavier_params(seed)
    layers = omlp.unpack(params)
    params = omlp.pack([(W, g.normal(size=b.shape) * 0.05) for W, b in layers]).astype(np.float32)
    desc = sampling.pair_batch(g, n_data, 4.0, 11.138).astype(np.float32)
    labels = (g.normal(size=n_data) * 3.0 + 1.0).astype(np.float32)
    norm = omlp.Norm(in_scale=np.array([1 / 11.138] * 3 + [1.0] * 4), out_shift=0.5, out_scale=2.5)
    return params, desc, labels, norm


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("batch", [64, 544])
def test_gradient_and_adam_match_oracle(abi, prec, batch):
    params, desc, labels, norm = _problem()
    idx = sampling.rng(11).choice(len(labels), batch, replace=False).astype(np.int32)
    dev = "cuda"
    p = torch.tensor(params, device=dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.zeros(1, device=dev)
    grad = torch.zeros_like(p)
    ws = torch.zeros(abi.rb_nn_train_workspace_bytes(batch), dtype=torch.uint8, device=dev)
    abi.rb_nn_train_step(p, m, v, 1, norm.as_array(), prec, batch, torch.tensor(np.ascontiguousarray(desc.T),
                         device=dev), torch.tensor(labels, device=dev), torch.tensor(idx, device=dev),
                         1e-3, 0.9, 0.999, 1e-8, loss, grad, ws)
    lref, gref = omlp.loss_and_grad(_net(params, prec), desc[idx].astype(np.float64),
                                    labels[idx].astype(np.float64), norm)
    tol = 2e-2 if prec == 0 else 1e-4
    assert loss.item() == pytest.approx(lref, rel=tol)
    gg = grad.cpu().numpy()
    for a, b, name in LAYER_SLICES:
        assert_close(gg[a:b], gref[a:b], tol, f"grad {name}")
    # Adam from the kernel's own gradient: FP32 arithmetic against FP64
    pref, mref, vref = omlp.adam_step(params.astype(np.float64), 0.0, 0.0, 1, gg.astype(np.float64))
    np.testing.assert_allclose(p.cpu().numpy(), pref, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(m.cpu().numpy(), mref, rtol=1e-6, atol=1e-12)


def fm_step_vs_oracle(abi, prec, batch, n_data, seed=5, lam=3.0):
    """One force/torque-matching step on the GPU against the oracle's exact
    loss and gradient (tangents forward, reverse through both chains); lam
    weights both matching terms."""
    params, desc, labels, norm = _problem(n_data, seed)
    ft = (sampling.rng(21).normal(size=(len(labels), 6)) * 0.5).astype(np.float32)
    idx = sampling.rng(11).choice(len(labels), batch, replace=False).astype(np.int32)
    dev = "cuda"
    p = torch.tensor(params, device=dev)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    loss = torch.zeros(2, device=dev)
    grad = torch.zeros_like(p)
    ws = torch.zeros(abi.rb_nn_train_fm_workspace_bytes(batch), dtype=torch.uint8, device=dev)
    abi.rb_nn_train_step_fm(p, m, v, 1, norm.as_array(), prec, batch, torch.tensor(np.ascontiguousarray(desc.T),
                            device=dev), torch.tensor(labels, device=dev), torch.tensor(np.ascontiguousarray(ft.T),
                            device=dev), torch.tensor(idx, device=dev), lam, lam, 1e-3, 0.9, 0.999, 1e-8, loss,
                            grad, ws)
    u, y, f = desc[idx].astype(np.float64), labels[idx].astype(np.float64), ft[idx].astype(np.float64)
    el, fl, gref = omlp.fm_loss_and_grad(_net(params, prec), u, y, f, lam, lam, norm)
    _, g_energy = omlp.loss_and_grad(_net(params, prec), u, y, norm)
    assert np.linalg.norm(gref - g_energy) > 0.2 * np.linalg.norm(g_energy)   # the matching term matters
    tol = 2e-2 if prec == 0 else 1e-4
    assert loss[0].item() == pytest.approx(el, rel=tol) and loss[1].item() == pytest.approx(fl, rel=tol)
    gg = grad.cpu().numpy().astype(np.float64)
    for a, b, name in LAYER_SLICES:
        assert_close(gg[a:b], gref[a:b], tol, f"grad {name}")
    pref, _, _ = omlp.adam_step(params.astype(np.float64), 0.0, 0.0, 1, gg)
    np.testing.assert_allclose(p.cpu().numpy(), pref, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("batch", [32, 256])
def test_force_matching_gradient_matches_oracle(abi, prec, batch):
    # energy + force/torque matching: the step's losses and its exact
    # gradient against the oracle's, at 2e-2 (BF16) and 1e-4 (FP32)
    fm_step_vs_oracle(abi, prec, batch, 700)


def test_training_on_bead_labels_beats_untrained(abi):
    # the learned part: fit bead-sum energies of a rigid dumbbell (two beads
    # 1.2 sigma apart), labelled by the GPU bead kernel, then compare the
    # held-out error of the trained and the untrained network
    from paper_2402_12199_amd import nn
    beads = np.array([[-0.6, 0.0, 0.0], [0.6, 0.0, 0.0]])
    inertia = np.array([0.01, 0.72, 0.72])
    ctx = abi.Ctx([beads], [2.0], [inertia])
    d_lo, d_cut = 1.0, 1.2 + 2.5
    g = sampling.rng(4)
    raw = sampling.pair_batch(g, 1 << 15, d_lo, d_cut)
    lab = nn.label_pairs(ctx, raw)
    # attractive and contact configurations; the steep repulsive wall below
    # 1 sigma dominates a squared loss and needs far longer training
    keep = lab[:, 10] >= 1.0
    raw, lab = raw[keep], lab[keep]
    ntr = (len(raw) * 7 // 8) // 1024 * 1024
    e = lab[:, 0].astype(np.float64)
    norm = nn.make_norm(d_cut, float(e[:ntr].mean()), float(e[:ntr].std()))
    tr = nn.Trainer(sampling.xavier_params(3), norm, precision=abi.RB_PREC_BF16, batch=1024, lr=1e-3)
    desc_tr = torch.tensor(np.ascontiguousarray(raw[:ntr].T, dtype=np.float32), device="cuda")
    y_tr = torch.tensor(lab[:ntr, 0], device="cuda")
    test = torch.tensor(np.ascontiguousarray(raw[ntr:].T, dtype=np.float32), device="cuda")
    E0 = torch.zeros(test.shape[1], device="cuda")
    abi.rb_nn_pair_eval(tr.params, norm, abi.RB_PREC_BF16, test, E0)
    first = tr.epoch(desc_tr, y_tr, g)
    for _ in range(39):
        last = tr.epoch(desc_tr, y_tr, g)
    E1 = torch.zeros(test.shape[1], device="cuda")
    abi.rb_nn_pair_eval(tr.params, norm, abi.RB_PREC_BF16, test, E1)
    ref = lab[ntr:, 0]
    rmse0 = float(np.sqrt(np.mean((E0.cpu().numpy() - ref) ** 2)))
    rmse1 = float(np.sqrt(np.mean((E1.cpu().numpy() - ref) ** 2)))
    assert last < 0.3 * first, (first, last)
    assert rmse1 < 0.5 * rmse0, (rmse0, rmse1)


def test_network_path_is_faster_than_bead_sum(abi):
    # what the network gains over the method without it: per-pair energy,
    # force and torque of 2^16 cylinder pairs, bead double sum vs network
    # forward + input gradient on the same GPU
    from paper_2402_12199_amd import nn
    cy = configs.cyl134()
    ctx = abi.Ctx([cy.beads], [cy.mass], [cy.inertia])
    P = 1 << 16
    desc = torch.tensor(np.ascontiguousarray(
        sampling.pair_batch(sampling.rng(8), P, 4.0, 11.138).T.astype(np.float32)), device="cuda")
    out = torch.empty((11, P), device="cuda")
    E = torch.empty(P, device="cuda")
    ft = torch.empty((9, P), device="cuda")
    params = torch.tensor(sampling.xavier_params(2).astype(np.float32), device="cuda")
    norm = nn.make_norm(11.138)

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 5

    t_bead = timeit(lambda: abi.rb_bead_pair_eval(ctx, desc, 0, 0, out))
    t_nn = timeit(lambda: abi.rb_nn_pair_grad(params, norm, abi.RB_PREC_BF16, desc, None, E, None, ft))
    print(f"bead {t_bead:.3f} ms, network {t_nn:.3f} ms, ratio {t_bead / t_nn:.1f}")
    assert t_nn * 2 < t_bead


def test_labelled_sets_reject_overlaps_and_match_the_oracle(abi):
    # uniform pair configurations labelled by the GPU bead kernel: the count
    # asked for, none closer than r_rej, labels equal to the oracle's
    from oracle import beads as obeads
    from paper_2402_12199_amd.surrogate import make_dataset
    body = configs.cube5()
    ctx = abi.Ctx([body.beads], [body.mass], [body.inertia])
    d_min = 2 * body.r_in + 1.0
    d_cut = 2 * body.r_max + 2.5
    desc, lab, rej, _, drawn = make_dataset(ctx, 300, 17, d_min, d_cut, r_rej=0.8)
    assert desc.shape == (300, 7) and lab.shape == (300, 11) and 0 < rej < 1 and drawn >= 300
    assert lab[:, 10].min() >= 0.8
    ref = obeads.bead_pair_desc(body.beads.astype(np.float32).astype(np.float64),
                                body.beads.astype(np.float32).astype(np.float64), desc.astype(np.float64))
    assert_close(lab[:, 0], ref[:, 0], 1e-5, "E")
    assert_close(lab[:, 1:10], ref[:, 1:10], 1e-4, "F, tau")


def test_hphc_surrogate_dynamics_follow_the_bead_path(abi):
    # With the paper's half-power half-cosine bead potential the pair energy
    # is smooth enough for the surrogate to drive the dynamics: trained on
    # the pairs the bead dynamics visits, its trajectory from the same start
    # stays finite, conserves energy and diffuses like the bead trajectory.
    import dataclasses
    from paper_2402_12199_amd.compare import compare
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.surrogate import train_surrogate_md
    from synth import state
    cfg = dataclasses.replace(configs.config_hphc(), name="cubes512_hphc", body=configs.cube5(), n_bodies=512,
                              seed=77)
    st = state.initial_state(cfg)
    sur = train_surrogate_md(cfg, st, 1 << 17, 1 << 13, 60, r_rej=0.0, batch=2048)
    h = sur["trained"]
    assert h["rmse_E"] < 0.5 * h["std_E"] and h["rmse_F"] < h["std_F"]
    model = NNModel(params=sur["params"], norm=sur["norm"], precision=abi.RB_PREC_BF16, d_min=cfg.d_min,
                    sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut)
    out = compare(cfg, st, {"nn": model}, chunks=3, replays=10)
    bead, nn = out["bead"], out["nn"]
    assert bead["error"] is None and nn["error"] is None and nn["steps"] == bead["steps"] == 303
    assert abs(nn["drift_per_body"]) < 5e-3 and abs(bead["drift_per_body"]) < 1e-5
    assert 0.7 < nn["msd_ratio_vs_bead"] < 1.3
    assert nn["rdf_l1_vs_bead"] < 0.2
    assert 0.5 < nn["msr_ratio_vs_bead"] < 2.0
    # the same at constant temperature (Nose-Hoover): both paths stay near
    # the target and the network path still moves like the bead path
    out = compare(cfg, st, {"nn": model}, chunks=3, replays=10, nvt=dict(kT=cfg.kT, tau=0.5))
    bead, nn = out["bead"], out["nn"]
    assert bead["error"] is None and nn["error"] is None and nn["steps"] == bead["steps"] == 303
    for r in (bead, nn):
        assert 0.6 * cfg.kT < r["temperature_last"] < 1.4 * cfg.kT
    assert abs(bead["drift_per_body"]) < 1e-4 and abs(nn["drift_per_body"]) < 5e-3
    assert 0.7 < nn["msd_ratio_vs_bead"] < 1.3
