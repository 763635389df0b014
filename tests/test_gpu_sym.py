"""GPU parity of the symmetry-reduced cube-pair descriptor (supplementary
section 1): descriptor and Jacobian kernel, network gradient through it, and
network forces of a system through it, against the FP64 oracle."""
import numpy as np
import pytest

from oracle import frames as oframes
from oracle import mlp as omlp
from oracle import symmetry as osym
from synth import configs, sampling, state
from tests.tolerances import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12199_amd import abi as _abi
    return _abi


def _away_from_cuts(desc, margin=2e-3):
    """Rows whose descriptor does not sit near a switch of its choices (sort
    ties, face-normal ties), where FP32 input rounding could take the other
    branch."""
    a = np.sort(np.abs(desc[:, :3]), axis=1)
    R = osym.rotation_matrices(desc[:, 3:7])
    ok = (a[:, 2] - a[:, 1] > margin) & (a[:, 1] - a[:, 0] > margin)
    for n in np.nonzero(ok)[0]:
        g = np.zeros((3, 3))
        for r, k in enumerate(sorted(range(3), key=lambda k: (-abs(desc[n, k]), k))):
            g[r, k] = 1.0
        m = np.sort(np.abs((g @ R[n] @ g.T)[0]))
        ok[n] = m[2] - m[1] > margin
    return ok


def test_descriptor_and_jacobian_match_oracle(abi):
    P = 3000
    desc = sampling.pair_batch(sampling.rng(31), P, 6.0, 11.2).astype(np.float32)
    d = torch.tensor(np.ascontiguousarray(desc.T), device="cuda")
    sym = torch.full((7, P), float("nan"), device="cuda")
    jac = torch.full((49, P), float("nan"), device="cuda")
    abi.rb_cube_sym_descriptors(d, sym, jac)
    got_s = sym.cpu().numpy().T
    got_j = jac.cpu().numpy().T.reshape(P, 7, 7)
    u = desc.astype(np.float64)
    ref_s = osym.cube_descriptor(u)
    ok = _away_from_cuts(u)
    assert ok.sum() > 0.8 * P
    err = np.abs(got_s[ok] - ref_s[ok]) / np.abs(ref_s).max(axis=0)
    assert err.max() < 2e-5, (err.max(axis=0), np.argmax(err, axis=0))
    ref_j = osym.cube_descriptor_jacobian(u[ok])
    assert_close(got_j[ok].reshape(-1, 49), ref_j.reshape(-1, 49), 1e-4, "jacobian")
    # compacted form: pairs idx[0 .. count) into rows 0 .. count
    idx = np.sort(sampling.rng(32).choice(P, 700, replace=False)).astype(np.int32)
    m = 1024
    cnt = torch.tensor([len(idx)], dtype=torch.int32, device="cuda")
    sym2 = torch.zeros((7, m), device="cuda")
    jac2 = torch.zeros((49, m), device="cuda")
    abi.rb_cube_sym_descriptors(d, sym2, jac2, torch.tensor(idx, device="cuda"), cnt, m)
    assert torch.equal(sym2[:, :len(idx)], sym[:, idx]) and torch.equal(jac2[:, :len(idx)], jac[:, idx])
    assert torch.all(sym2[:, len(idx):] == 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_network_gradient_through_the_descriptor_matches_oracle(abi, prec):
    P = 1500
    desc = sampling.pair_batch(sampling.rng(33), P, 6.0, 11.2).astype(np.float32)
    u = desc.astype(np.float64)
    ok = _away_from_cuts(u)
    params = sampling.xavier_params(34)
    from paper_2402_12199_amd.nn import make_norm_sym
    norm = make_norm_sym(11.2)
    d = torch.tensor(np.ascontiguousarray(desc.T), device="cuda")
    sym = torch.empty((7, P), device="cuda")
    jac = torch.empty((49, P), device="cuda")
    abi.rb_cube_sym_descriptors(d, sym, jac)
    e = torch.empty(P, device="cuda")
    g = torch.empty((7, P), device="cuda")
    ft = torch.empty((9, P), device="cuda")
    p_dev = torch.tensor(params.astype(np.float32), device="cuda")
    abi.rb_nn_pair_grad_sym(p_dev, norm, prec, d, sym, jac, None, e, g, ft)
    net = omlp.bf16_network(params) if prec == 0 else params.astype(np.float32).astype(np.float64)
    on = omlp.Norm(in_shift=norm[:7].astype(np.float64), in_scale=norm[7:14].astype(np.float64),
                   out_shift=float(norm[14]), out_scale=float(norm[15]))
    E_ref, gs = omlp.input_grad(net, osym.cube_descriptor(u[ok]), on)
    gu = np.einsum("pk,pkm->pm", gs, osym.cube_descriptor_jacobian(u[ok]))
    ft_ref = oframes.forces_from_grad(u[ok], gu)
    tol = 2e-2 if prec == 0 else 1e-4
    assert_close(e.cpu().numpy()[ok], E_ref, tol, "E")
    assert_close(g.cpu().numpy().T[ok], gu, tol, "dE/du")
    for lo, name in ((0, "F_j"), (3, "tau_i"), (6, "tau_j")):
        assert_close(ft.cpu().numpy().T[ok, lo:lo + 3], ft_ref[:, lo:lo + 3], tol, name)


def test_system_forces_through_the_descriptor_match_oracle(abi):
    # every listed pair on the network (no switch, no fallback): per-body
    # forces and torques against the oracle's sum over the same pairs
    from paper_2402_12199_amd.md import NNModel, RigidSystem
    from paper_2402_12199_amd.nn import make_norm_sym
    cfg = configs.config1()
    st = state.initial_state(cfg)
    b = cfg.body
    params = sampling.xavier_params(35)
    norm = make_norm_sym(cfg.d_cut)
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    sysm.set_nn(NNModel(params=torch.tensor(params.astype(np.float32), device="cuda"), norm=norm, sym=True))
    sysm.init_forces("nn")
    sysm.check_capacity()
    pairs = sysm.pairs_host()
    assert len(pairs) > 20
    u = oframes.descriptors(st["x"][pairs[:, 0]], st["q"][pairs[:, 0]], st["x"][pairs[:, 1]], st["q"][pairs[:, 1]],
                            box=cfg.box)
    on = omlp.Norm(in_shift=norm[:7].astype(np.float64), in_scale=norm[7:14].astype(np.float64),
                   out_shift=float(norm[14]), out_scale=float(norm[15]))
    E, gs = omlp.input_grad(omlp.bf16_network(params), osym.cube_descriptor(u), on)
    gu = np.einsum("pk,pkm->pm", gs, osym.cube_descriptor_jacobian(u))
    lab = oframes.to_lab(st["q"][pairs[:, 0]], oframes.forces_from_grad(u, gu))
    F = np.zeros((cfg.n_bodies, 3))
    T = np.zeros((cfg.n_bodies, 3))
    np.add.at(F, pairs[:, 1], lab[:, :3])
    np.add.at(F, pairs[:, 0], -lab[:, :3])
    np.add.at(T, pairs[:, 0], lab[:, 3:6])
    np.add.at(T, pairs[:, 1], lab[:, 6:9])
    assert sysm.energy() == pytest.approx(E.sum(), rel=2e-2)
    assert_close(sysm.force.cpu().numpy().T, F, 2e-2, "force")
    assert_close(sysm.torque.cpu().numpy().T, T, 2e-2, "torque")


def test_surrogate_on_the_descriptor_drives_dynamics(abi):
    # half-power half-cosine cube-5 shells: a surrogate trained on the
    # symmetry-reduced descriptor of bead-MD pairs runs the dynamics from the
    # same start as the bead path and follows it
    import dataclasses
    from paper_2402_12199_amd.compare import compare
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.surrogate import train_surrogate_md
    cfg = dataclasses.replace(configs.config_hphc(), name="cubes512_hphc", body=configs.cube5(), n_bodies=512,
                              seed=78)
    st = state.initial_state(cfg)
    sur = train_surrogate_md(cfg, st, 1 << 17, 1 << 13, 60, r_rej=0.0, batch=2048, sym=True)
    h = sur["trained"]
    assert h["rmse_E"] < 0.5 * h["std_E"] and h["rmse_F"] < 0.8 * h["std_F"] and h["rmse_tau_j"] < h["std_tau_j"]
    model = NNModel(params=sur["params"], norm=sur["norm"], precision=abi.RB_PREC_BF16, d_min=cfg.d_min,
                    sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut, sym=True)
    out = compare(cfg, st, {"nn": model}, chunks=3, replays=10)
    bead, nn = out["bead"], out["nn"]
    assert bead["error"] is None and nn["error"] is None and nn["steps"] == bead["steps"] == 303
    assert abs(nn["drift_per_body"]) < 5e-3
    assert 0.7 < nn["msd_ratio_vs_bead"] < 1.3 and nn["rdf_l1_vs_bead"] < 0.2
