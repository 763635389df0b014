"""GPU parity of the cylinder-pair four-number descriptor (supplementary
section 2), of the network gradient and the dynamics forces through it, and
of the routing by the shells' lower bound on the closest bead distance,
against the oracle."""
import numpy as np
import pytest

from oracle import beads as obeads
from oracle import cylinder as ocyl
from oracle import domain as odom
from oracle import frames as oframes
from oracle import mlp as omlp
from synth import configs, sampling
from tests.tolerances import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = {0: (2e-2, 2e-2), 1: (1e-5, 1e-4)}


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12199_amd import abi as _abi
    return _abi


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _net(params, prec):
    return omlp.bf16_network(params) if prec == 0 else params.astype(np.float64)


def _configs(n, seed):
    u = sampling.pair_batch(sampling.rng(seed), n, 1.0, 11.2)
    # the frame choice's special places: on body 1's axis, in its mid plane
    u[:8, 0:2] *= 1e-9
    u[8:16, 2] = 0.0
    u[16:24, :2] = 0.0
    u[16:24, 2] = 0.0
    return u.astype(np.float32)


def test_descriptor_and_jacobian_match_oracle(abi):
    n = 3000
    u = _configs(n, 31)
    sym = torch.full((7, n), float("nan"), device="cuda")
    jac = torch.full((49, n), float("nan"), device="cuda")
    abi.rb_cyl_sym_descriptors(_dev(u.T), sym, jac)
    ud = u.astype(np.float64)
    s_ref = ocyl.cyl_descriptor(ud)
    J_ref = ocyl.cyl_descriptor_jacobian(ud)
    got = sym.cpu().numpy().T
    for r in range(7):
        assert_close(got[:, r], s_ref[:, r], 1e-5, f"s[{r}]")
    J = jac.cpu().numpy().T.reshape(n, 7, 7)
    for r in range(5):
        assert_close(J[:, r, :], J_ref[:, r, :], 1e-5, f"J[{r}]")
    assert not J[:, 5:, :].any()
    # compacted form: rows idx[0 .. count) with row stride max_count
    g = sampling.rng(32)
    idx = g.permutation(n)[:500].astype(np.int32)
    m = 600
    sym2 = torch.zeros((7, m), device="cuda")
    jac2 = torch.zeros((49, m), device="cuda")
    cnt = torch.tensor([450], dtype=torch.int32, device="cuda")
    abi.rb_cyl_sym_descriptors(_dev(u.T), sym2, jac2, _dev(idx), cnt, m)
    np.testing.assert_array_equal(sym2.cpu().numpy()[:, :450], sym.cpu().numpy()[:, idx[:450]])
    np.testing.assert_array_equal(jac2.cpu().numpy()[:, :450], jac.cpu().numpy()[:, idx[:450]])
    assert not sym2[:, 450:].any()


def _params(seed):
    params = sampling.xavier_params(seed).astype(np.float32)
    g = sampling.rng(seed + 1)
    layers = omlp.unpack(params.astype(np.float64))
    return omlp.pack([(W, g.normal(size=b.shape) * 0.1) for W, b in layers]).astype(np.float32)


def _norm():
    return omlp.Norm(in_shift=np.array([30.0, 30.0, 0.3, 20.0, 0.0, 0.0, 0.0]),
                     in_scale=np.array([0.03, 0.03, 3.0, 0.04, 0.05, 0.0, 0.0]), out_shift=-0.5, out_scale=3.0)


@pytest.mark.parametrize("prec", [0, 1])
def test_network_gradient_through_the_descriptor_matches_oracle(abi, prec):
    n = 2049
    u = _configs(n, 33)
    params, norm = _params(3), _norm()
    sym = torch.zeros((7, n), device="cuda")
    jac = torch.zeros((49, n), device="cuda")
    d = _dev(u.T)
    abi.rb_cyl_sym_descriptors(d, sym, jac)
    E = torch.zeros(n, device="cuda")
    g = torch.zeros((7, n), device="cuda")
    ft = torch.zeros((9, n), device="cuda")
    abi.rb_nn_pair_grad_sym(_dev(params), norm.as_array(), prec, d, sym, jac, None, E, g, ft)
    ud = u.astype(np.float64)
    s = ocyl.cyl_descriptor(ud)
    Er, gs = omlp.input_grad(_net(params, prec), s, norm)
    gu = np.einsum("pr,prm->pm", gs, ocyl.cyl_descriptor_jacobian(ud))
    ftr = oframes.forces_from_grad(ud, gu)
    etol, gtol = RTOL[prec]
    assert_close(E.cpu().numpy(), Er, etol, "E")
    assert_close(g.cpu().numpy().T, gu, gtol, "dE/du")
    got = ft.cpu().numpy().T
    for k, name in ((0, "F_j"), (3, "tau_i"), (6, "tau_j")):
        assert_close(got[:, k:k + 3], ftr[:, k:k + 3], gtol, name)
    # no torque about either cylinder's own axis
    aj = oframes.qrotate(ud[:, 3:] / np.linalg.norm(ud[:, 3:], axis=1, keepdims=True),
                         np.broadcast_to([0.0, 0, 1], (n, 3)))
    assert np.abs(got[:, 5]).max() <= 1e-4 * np.abs(got[:, 3:6]).max()
    assert np.abs(np.sum(got[:, 6:9] * aj, 1)).max() <= 1e-4 * np.abs(got[:, 6:9]).max()


def _oracle_routes(cfg, st, pairs, gap_min, gap_max):
    """Oracle routing of the listed pairs (network / bead / neither) by the
    shells' bound."""
    x, q = st["x"], st["q"]
    u = oframes.descriptors(x[pairs[:, 0]], q[pairs[:, 0]], x[pairs[:, 1]], q[pairs[:, 1]], cfg.box)
    r = np.linalg.norm(u[:, :3], axis=1)
    inr = r < cfg.d_cut
    G = np.full(len(u), np.inf)
    G[inr] = odom.gap(cfg.body.beads, cfg.body.beads, u[inr])
    bead = inr & ((r < cfg.d_min) | (G < gap_min))
    net = inr & ~bead & (G < gap_max)
    return u, r, G, net, bead


def _check_routes(abi, cfg, st, lp, gnet, gbead, gap_min, gap_max):
    """The GPU's routing of the list pairs lp against the oracle's.  The
    bound is a lower bound found by an iteration, and either side's bound is
    valid: where the two straddle a threshold (at most 0.1 % of the pairs)
    the GPU's choice must still be valid, i.e. a network pair has no bead
    pair closer than gap_min and a skipped pair none closer than gap_max
    (the oracle's bead sum decides).  A sample of all network and skipped
    pairs is checked the same way.  Returns the oracle's descriptors."""
    b = cfg.body
    u, r, G, net, bead = _oracle_routes(cfg, st, lp, gap_min, gap_max)
    inr = r < cfg.d_cut
    skip = inr & ~gnet & ~gbead
    assert not (gnet & gbead).any() and not (gnet & ~inr).any() and not (gbead & ~inr).any()
    diff = (gnet != net) | (gbead != bead)
    assert diff.sum() <= 1e-3 * inr.sum(), (int(diff.sum()), int(inr.sum()))
    assert net.sum() > 10000 and bead.sum() > 0 and inr.sum() > 2 * net.sum()
    g = sampling.rng(34)
    for sel, lo in ((gnet, gap_min), (skip, gap_max)):
        ids = np.nonzero(sel)[0]
        pick = np.union1d(g.choice(ids, min(1500, len(ids)), replace=False), np.nonzero(sel & diff)[0])
        rmin = obeads.bead_pair_desc(b.beads, b.beads, u[pick], rc=1e3)[:, 10]
        assert (rmin >= lo - 1e-9).all()
    return u, r


def test_shell_routing_matches_oracle_and_keeps_the_network_in_its_domain(abi, cyl_workload):
    # On the 32768-cylinder system at t = 0: the GPU routes the pairs as the
    # oracle's bound does (see _check_routes), every network pair has its
    # closest bead pair at least gap_min apart and every skipped pair inside
    # d_cut none within gap_max
    from paper_2402_12199_amd.md import RigidSystem
    cfg, st, pairs = cyl_workload
    gap_min, gap_max = 0.8, 2.5
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    sysm.desc = torch.zeros((7, sysm.max_pairs), dtype=torch.float32, device="cuda")
    sysm.idx_nn = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
    sysm.idx_bead = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
    sysm.build_pairs(always=True)
    sysm.route(cfg.d_min, cfg.d_cut, gap_min, gap_max)
    f = sysm.check_capacity()
    got_pairs = sysm.pairs_host()
    key = got_pairs[:, 0].astype(np.int64) * cfg.n_bodies + got_pairs[:, 1]
    order = np.argsort(key)
    ref_key = pairs[:, 0].astype(np.int64) * cfg.n_bodies + pairs[:, 1]
    np.testing.assert_array_equal(key[order], np.sort(ref_key))
    nn_ids = np.zeros(len(key), bool)
    nn_ids[sysm.idx_nn[:f[abi.RB_FLAG_NNN]].cpu().numpy()] = True
    bd_ids = np.zeros(len(key), bool)
    bd_ids[sysm.idx_bead[:f[abi.RB_FLAG_NBEAD]].cpu().numpy()] = True
    _check_routes(abi, cfg, st, got_pairs[order], nn_ids[order], bd_ids[order], gap_min, gap_max)


def test_routing_with_two_identical_templates_equals_the_single_template_routing(abi, cyl_workload):
    # The routing kernel, the bead kernel's screen and the fallback of the
    # one-launch network forces have a form for single-template contexts
    # (uniform shell sizes, no type loads) and the general one (per-pair
    # type lookups); the same cylinders under a context with the template
    # given twice (types alternating) must get the same descriptors, the
    # same routes and, bit for bit, the same bead-path and network-path
    # forces, torques and energy, and the same states after fused steps
    from paper_2402_12199_amd.md import NNModel, RigidSystem
    cfg, st, pairs = cyl_workload
    b = cfg.body
    params, norm = _params(5), _norm()
    out, sums = [], []
    for ntypes in (1, 2):
        types = (np.arange(cfg.n_bodies) % ntypes).astype(np.int32)
        sysm = RigidSystem([b.beads] * ntypes, [b.mass] * ntypes, [b.inertia] * ntypes, types, st["x"], st["q"],
                           st["P"], st["L"], cfg.box, cfg.r_list, cfg.skin)
        sysm.desc = torch.zeros((7, sysm.max_pairs), dtype=torch.float32, device="cuda")
        sysm.idx_nn = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
        sysm.idx_bead = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
        sysm.build_pairs(always=True)
        sysm.route(cfg.d_min, cfg.d_cut, 1.0, 2.5)
        f = sysm.check_capacity()
        p = sysm.pairs_host()
        key = p[:, 0].astype(np.int64) * cfg.n_bodies + p[:, 1]
        nn = np.sort(key[sysm.idx_nn[:f[abi.RB_FLAG_NNN]].cpu().numpy()])
        bd = np.sort(key[sysm.idx_bead[:f[abi.RB_FLAG_NBEAD]].cpu().numpy()])
        order = np.argsort(key)
        out.append((nn, bd, sysm.desc[:, :len(key)].cpu().numpy()[:, order]))
        res = []
        sysm.set_nn(NNModel(params=_dev(params), norm=norm.as_array(), precision=abi.RB_PREC_BF16,
                            d_min=cfg.d_min, sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut, form="cyl", gap_min=1.0,
                            gap_max=2.5))
        for path in ("bead", "nn"):
            sysm.compute_forces(path)
            sysm.check_capacity()
            res += [sysm.force.cpu().numpy(), sysm.torque.cpu().numpy(), sysm.ev.cpu().numpy()]
        # and three fused integrator steps (per-type masses and inertias)
        sysm.begin_fused(cfg.dt)
        for _ in range(3):
            sysm.fused_step(cfg.dt, "bead")
        sysm.end_fused(cfg.dt, "bead")
        sysm.check_capacity()
        res += [t.cpu().numpy() for t in (sysm.x, sysm.q, sysm.P, sysm.L, sysm.kinetic)]
        sums.append(res)
    assert len(out[0][0]) > 10000 and len(out[0][1]) > 500
    for a0, a1 in zip(out[0], out[1]):
        np.testing.assert_array_equal(a1, a0)
    for a0, a1 in zip(sums[0], sums[1]):
        np.testing.assert_array_equal(a1, a0)


def test_routing_over_several_rounds_per_block_matches_one_round(abi, cyl_workload):
    # 18 copies of the 32768-cylinder pair list (~610k entries, more than the
    # routing grid's 512 blocks of 1024 threads take in one round): the whole
    # list and its two halves (each taken in one round) give the same
    # descriptors and route the same entries, and the launch leaves its
    # working word zero
    from paper_2402_12199_amd.md import RigidSystem
    cfg, st, pairs = cyl_workload
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    pi = np.tile(pairs[:, 0].astype(np.int32), 18)
    pj = np.tile(pairs[:, 1].astype(np.int32), 18)
    M = len(pi)
    assert M > 512 * 1024

    def route(lo, hi):
        m = hi - lo
        desc = torch.zeros((7, m), dtype=torch.float32, device="cuda")
        inn = torch.zeros(m, dtype=torch.int32, device="cuda")
        ibd = torch.zeros(m, dtype=torch.int32, device="cuda")
        flags = torch.zeros(abi.RB_NFLAGS, dtype=torch.int32, device="cuda")
        flags[abi.RB_FLAG_NPAIRS] = m
        abi.rb_pair_descriptors(sysm.x, sysm.q, sysm.box, _dev(pi[lo:hi]), _dev(pj[lo:hi]), cfg.d_min, desc, inn,
                                ibd, flags, d_max=cfg.d_cut, ctx=sysm.ctx, types=sysm.types, gap_min=0.8,
                                gap_max=2.5)
        f = flags.cpu().numpy()
        assert (f[abi.RB_FLAG_ROUTE_WORK:abi.RB_FLAG_ROUTE_WORK + 2] == 0).all()
        return (desc.cpu().numpy(), np.sort(inn[:f[abi.RB_FLAG_NNN]].cpu().numpy()) + lo,
                np.sort(ibd[:f[abi.RB_FLAG_NBEAD]].cpu().numpy()) + lo)

    dw, nw, bw = route(0, M)
    h = M // 2
    d1, n1, b1 = route(0, h)
    d2, n2, b2 = route(h, M)
    np.testing.assert_array_equal(dw, np.concatenate([d1, d2], axis=1))
    np.testing.assert_array_equal(nw, np.concatenate([n1, n2]))
    np.testing.assert_array_equal(bw, np.concatenate([b1, b2]))
    assert len(nw) > 0 and len(bw) > 0 and len(np.unique(nw)) == len(nw)


def test_two_level_routing_routes_its_candidates_as_the_full_routing(abi, cyl_workload):
    # 32768 cylinders with the bead path's margin.  A screening call routes
    # as the full routing does; after moves that keep every bead within
    # margin / 2 the candidates alone are routed, each exactly as the full
    # routing routes it, and a pair only the full routing sends somewhere has
    # no bead pair within gap_max (the oracle's closest bead distance); a
    # rescreen matches the full routing again
    from paper_2402_12199_amd.md import RigidSystem
    cfg, st, pairs = cyl_workload
    b = cfg.body
    gap_min, gap_max, margin = 1.0, 2.5, cfg.bead_margin
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin, margin=margin)
    sysm.desc = torch.zeros((7, sysm.max_pairs), dtype=torch.float32, device="cuda")
    sysm.idx_nn = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
    sysm.idx_bead = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
    sysm.build_pairs(always=True)

    def routed(two_level):
        sysm.route(cfg.d_min, cfg.d_cut, gap_min, gap_max, two_level=two_level)
        f = sysm.flags_host()
        nn = np.sort(sysm.idx_nn[:f[abi.RB_FLAG_NNN]].cpu().numpy())
        bd = np.sort(sysm.idx_bead[:f[abi.RB_FLAG_NBEAD]].cpu().numpy())
        return nn, bd, sysm.desc.clone(), f

    nn2, bd2, desc2, f = routed(True)      # a screening call (the pair-list build set the flag)
    assert f[abi.RB_FLAG_RESCREEN] == 0 and f[abi.RB_FLAG_NRESCREENS] == 1
    ncand = int(f[abi.RB_FLAG_NSCREEN])
    assert len(nn2) + len(bd2) < ncand < f[abi.RB_FLAG_NPAIRS]
    assert (sysm.x_sref == sysm.x).all() and (sysm.q_sref == sysm.q).all()
    cand = np.sort(sysm.cand_list[:ncand].cpu().numpy())
    assert len(np.unique(cand)) == ncand
    nn1, bd1, desc1, _ = routed(False)
    np.testing.assert_array_equal(nn2, nn1)
    np.testing.assert_array_equal(bd2, bd1)

    # moves: |dx| <= 0.03 per axis, turns of 0.005 rad (beads move < 0.08 < margin / 2)
    g = sampling.rng(41)
    n = sysm.n
    sysm.x += torch.tensor(g.uniform(-0.03, 0.03, (3, n)), device="cuda")
    ax = g.normal(size=(n, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    dq = np.concatenate([np.full((n, 1), np.cos(0.0025)), np.sin(0.0025) * ax], axis=1)
    qn = oframes.qmul(sysm.q.cpu().numpy().T, dq)
    sysm.q.copy_(torch.tensor((qn / np.linalg.norm(qn, axis=1, keepdims=True)).T.copy(), device="cuda"))
    nn2, bd2, desc2, f = routed(True)
    assert f[abi.RB_FLAG_NRESCREENS] == 1 and f[abi.RB_FLAG_NSCREEN] == ncand
    nn1, bd1, desc1, _ = routed(False)
    np.testing.assert_array_equal(nn2, np.intersect1d(nn1, cand))
    np.testing.assert_array_equal(bd2, np.intersect1d(bd1, cand))
    both = np.concatenate([nn2, bd2]).astype(np.int64)
    assert torch.equal(desc2[:, both], desc1[:, both])
    extra = np.setdiff1d(np.concatenate([nn1, bd1]), cand)
    if len(extra):
        pl = sysm.pairs_host()[extra[:500]]
        xh, qh = sysm.x.cpu().numpy().T, sysm.q.cpu().numpy().T
        u = oframes.descriptors(xh[pl[:, 0]], qh[pl[:, 0]], xh[pl[:, 1]], qh[pl[:, 1]], cfg.box)
        assert (obeads.bead_pair_desc(b.beads, b.beads, u, rc=1e3)[:, 10] >= gap_max - 1e-9).all()

    sysm.flags[abi.RB_FLAG_RESCREEN] = 1
    nn2, bd2, _, f = routed(True)
    assert f[abi.RB_FLAG_NRESCREENS] == 2
    np.testing.assert_array_equal(nn2, nn1)
    np.testing.assert_array_equal(bd2, bd1)


def test_pair_with_overlapping_bead_boxes_goes_to_the_bead_sum(abi):
    # Body j turned so that its axis lies along x, centre 1.5 + 0.6 + 4.05
    # from body i's axis: its end cap sits 0.6 sigma from body i's side (the
    # closest bead pair is 0.75 apart, inside the training data's rejected
    # range) while the centres are 6.15 apart, beyond d_min = 4.  The
    # shells' bound (0.6) is below gap_min, so the pair must go to the bead
    # sum.  Side by side and parallel at 4.5 (bound 1.5) it goes to the
    # network; parallel at 6.15 (bound 3.15 >= gap_max) to neither.
    from paper_2402_12199_amd.md import RigidSystem
    cyl = configs.cyl134()
    turn = [np.cos(np.pi / 4), 0.0, -np.sin(np.pi / 4), 0.0]          # body axis e_z -> -e_x
    ident = [1.0, 0.0, 0.0, 0.0]
    zero = np.zeros((2, 3))
    for dx, qj, want in ((6.15, turn, "bead"), (4.5, ident, "nn"), (6.15, ident, "none")):
        x = np.array([[20.0, 20.0, 20.0], [20.0 + dx, 20.0, 20.0]])
        qq = np.array([ident, qj])
        sysm = RigidSystem([cyl.beads], [cyl.mass], [cyl.inertia], np.zeros(2, np.int32), x, qq, zero, zero, 60.0,
                           2 * cyl.r_max + 3.5, 1.0)
        sysm.desc = torch.zeros((7, sysm.max_pairs), dtype=torch.float32, device="cuda")
        sysm.idx_nn = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
        sysm.idx_bead = torch.zeros(sysm.max_pairs, dtype=torch.int32, device="cuda")
        sysm.build_pairs(always=True)
        sysm.route(4.0, 2 * cyl.r_max + 2.5, 0.8, 2.5)
        f = sysm.flags_host()
        assert f[abi.RB_FLAG_NPAIRS] == 1
        u = oframes.descriptors(x[:1], qq[:1], x[1:], qq[1:])
        G = odom.gap(cyl.beads, cyl.beads, u)[0]
        rmin = obeads.bead_pair_desc(cyl.beads, cyl.beads, u, rc=1e3)[0, 10]
        assert G <= rmin
        got = "bead" if f[abi.RB_FLAG_NBEAD] else ("nn" if f[abi.RB_FLAG_NNN] else "none")
        assert got == want, (dx, G, rmin, got)
        if want == "bead":
            assert abs(G - 0.6) < 1e-9 and rmin < 0.8


@pytest.mark.parametrize("prec", [0, 1])
def test_cylinder_dynamics_forces_match_oracle(abi, cyl_workload, prec):
    # rb_nn_pair_forces_cyl on the 32768-cylinder system at t = 0 with the
    # shells' routing: the network (features and Jacobian formed inside the
    # kernel, switched energy) for the routed pairs, the bead sum for the
    # fallback pairs, against the oracle doing the same
    from paper_2402_12199_amd.md import NNModel, RigidSystem
    cfg, st, pairs = cyl_workload
    gap_min, gap_max = 0.8, 2.5
    sw_lo, sw_hi = cfg.d_cut - 1.0, cfg.d_cut
    params, norm = _params(5), _norm()
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    sysm.set_nn(NNModel(params=_dev(params), norm=norm.as_array(), precision=prec, d_min=cfg.d_min, sw_lo=sw_lo,
                        sw_hi=sw_hi, form="cyl", gap_min=gap_min, gap_max=gap_max))
    sysm.build_pairs(always=True)
    sysm.compute_forces("nn")
    f = sysm.check_capacity()
    lp = sysm.pairs_host()
    nn_ids = np.zeros(len(lp), bool)
    nn_ids[sysm.idx_nn[:f[abi.RB_FLAG_NNN]].cpu().numpy()] = True
    bd_ids = np.zeros(len(lp), bool)
    bd_ids[sysm.idx_bead[:f[abi.RB_FLAG_NBEAD]].cpu().numpy()] = True
    # the routing checked as in the routing test; the sums then follow it
    u, r = _check_routes(abi, cfg, st, lp, nn_ids, bd_ids, gap_min, gap_max)
    net, bead = nn_ids, bd_ids
    x, q = st["x"], st["q"]
    n = cfg.n_bodies
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    un = u[net].astype(np.float32).astype(np.float64)
    rn = np.linalg.norm(un[:, :3], axis=1)
    s = ocyl.cyl_descriptor(un)
    Ep, gs = omlp.input_grad(_net(params, prec), s, norm)
    gu = np.einsum("pr,prm->pm", gs, ocyl.cyl_descriptor_jacobian(un))
    t = np.clip((rn - sw_lo) / (sw_hi - sw_lo), 0, 1)
    S = 1 - t * t * (3 - 2 * t)
    dS = np.where((rn > sw_lo) & (rn < sw_hi), -6 * t * (1 - t) / (sw_hi - sw_lo), 0.0)
    gu = gu * S[:, None]
    gu[:, :3] += (Ep * dS / rn)[:, None] * un[:, :3]
    pn = lp[net]
    ft = oframes.to_lab(q[pn[:, 0]], oframes.forces_from_grad(un, gu))
    E = float(np.sum(S * Ep))
    np.add.at(F, pn[:, 0], -ft[:, :3])
    np.add.at(F, pn[:, 1], ft[:, :3])
    np.add.at(T, pn[:, 0], ft[:, 3:6])
    np.add.at(T, pn[:, 1], ft[:, 6:])
    for i, j in lp[bead]:
        o = obeads.bead_pair(b.beads, b.beads, x[i], q[i], x[j], q[j], box=cfg.box)
        E += o["E"]
        F[i] += o["Fi"]
        F[j] += o["Fj"]
        T[i] += o["taui"]
        T[j] += o["tauj"]
    etol, gtol = RTOL[prec]
    assert sysm.energy() == pytest.approx(E, rel=max(etol, 1e-5))
    assert_close(sysm.force.cpu().numpy().T, F, max(gtol, 1e-4), "force")
    assert_close(sysm.torque.cpu().numpy().T, T, max(gtol, 1e-4), "torque")


@pytest.mark.parametrize("case", ["both", "no_network_pairs", "no_bead_pairs"])
def test_routed_forces_in_one_launch_equal_the_two_calls(abi, cyl_workload, case):
    # rb_nn_pair_forces_routed (BF16: the network tiles, then the bead sums of
    # the fallback pairs in the same launch) against rb_nn_pair_forces_cyl
    # followed by rb_bead_pair_forces on the same routing, with empty lists
    # as edge cases: the same per-pair arithmetic, so the same fixed-point
    # sums, forces, torques, energy and virial
    from paper_2402_12199_amd.md import NNModel, RigidSystem
    cfg, st, pairs = cyl_workload
    b = cfg.body
    params, norm = _params(5), _norm()
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin)
    m = NNModel(params=_dev(params), norm=norm.as_array(), precision=abi.RB_PREC_BF16, d_min=cfg.d_min,
                sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut, form="cyl", gap_min=1.0, gap_max=2.5)
    sysm.set_nn(m)
    sysm.build_pairs(always=True)
    sysm.route(m.d_min, m.sw_hi, m.gap_min, m.gap_max)
    f = sysm.check_capacity()
    assert f[abi.RB_FLAG_NNN] > 12288 and f[abi.RB_FLAG_NBEAD] > 500   # several network rounds, a real fallback
    zero = torch.zeros(1, dtype=torch.int32, device="cuda")
    nn_cnt = zero if case == "no_network_pairs" else sysm.flags[abi.RB_FLAG_NNN:]
    bd_cnt = zero if case == "no_bead_pairs" else sysm.flags[abi.RB_FLAG_NBEAD:]
    results = []
    for one_launch in (False, True):
        flags = sysm.flags.clone()
        abi.rb_accum_zero(sysm.n, sysm.acc)
        if one_launch:
            abi.rb_nn_pair_forces_routed(sysm.ctx, m.params, m.norm, m.precision, 1, sysm.x, sysm.q, sysm.types,
                                         sysm.box, sysm.pair_i, sysm.pair_j, sysm.desc, sysm.idx_nn, nn_cnt,
                                         sysm.idx_bead, bd_cnt, sysm.max_pairs, m.sw_lo, m.sw_hi, sysm.acc, flags)
        else:
            abi.rb_nn_pair_forces_cyl(m.params, m.norm, m.precision, sysm.q, sysm.pair_i, sysm.pair_j, sysm.desc,
                                      sysm.idx_nn, nn_cnt, sysm.max_pairs, m.sw_lo, m.sw_hi, sysm.acc, flags)
            abi.rb_bead_pair_forces(sysm.ctx, sysm.x, sysm.q, sysm.types, sysm.box, sysm.pair_i, sysm.pair_j,
                                    sysm.idx_bead, bd_cnt, sysm.max_pairs, sysm.acc, flags)
        force = torch.zeros_like(sysm.force)
        torque = torch.zeros_like(sysm.torque)
        ev = torch.zeros_like(sysm.ev)
        abi.rb_accum_finalize(sysm.n, sysm.acc, force, torque, ev, flags)
        torch.cuda.synchronize()
        fh = flags.cpu().numpy()
        assert abi.rb_flags_check(fh)[0] == abi.RB_OK
        assert (fh[abi.RB_FLAG_FB_WORK:abi.RB_FLAG_FB_WORK + 2] == 0).all()   # working words left zero
        results.append((force.cpu().numpy(), torque.cpu().numpy(), ev.cpu().numpy(), int(fh[abi.RB_FLAG_NEVAL])))
    (f0, t0, e0, n0), (f1, t1, e1, n1) = results
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(t1, t0)
    np.testing.assert_array_equal(e1, e0)
    assert n1 == n0
    if case != "both":
        assert np.abs(f0).max() > 0
