"""Benchmark of the rigid-body pair path on one MI355X.

Workload of the headline: 32768 cylinders (8 rings of 12 beads, radius 1.5,
ring spacing 0.9, two end-cap discs of 19 beads: 134 beads) at volume
fraction 0.15, Lennard-Jones beads (rc = 2.5), NVE velocity Verlet at
kT = 1, dt = 0.005, cell-list pair list with skin 1.0.  A step is one MD
step: half kick + drift + free rotation, conditional list rebuild, the pair
forces and torques, the second half kick (the kinetic energy is reduced once
per graph of 10 steps).  Two paths from the same start:

  bead    the FP32 bead double sum over the listed pairs (two-level list),
  nn      the BF16 network surrogate on the cylinder four-number descriptor
          for the pairs whose shells' bound on the closest bead distance lies
          in [1.0, 2.5), the bead sum for the pairs below 1.0, nothing for
          the pairs at or above 2.5 (no bead pair within the cutoff); the
          routing visits the candidates of a two-level list (same margin as
          the bead path's), re-screened when a bead may have moved margin/2.

The surrogate is trained here, on the GPU, by the library's own training
step, on pairs visited by bead-path runs of the same system at
kT = 1, 2, 4 (energy loss, Adam, batch 8192, cosine decay); its held-out
errors are reported.  value = the network path's rigid-pair F+tau
evaluations per second: pairs whose centre distance is below the interaction
range 2 r_max + rc (the same count for both paths; measured at the start and
end of the timed steps) x steps per second.

Also reported: the bead path's rate and the ratio of the two, the roofline
of the network path's dominant kernel (network forces, timed with HIP events
on its stream), the other kernels of both paths, the network kernels on 2^20
random pairs, the training step at batch 8192, the bead-vs-network dynamics
over 2008 steps (energy drift, g(r), P2, MSD, MSR), and the FP64 oracle on
the host as the CPU baseline.  Inputs are synthetic and seeded.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 78.6e12     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, packed FP32 math not used
BF16_MFMA_PEAK = 2.5e15        # dense
FP32_MFMA_PEAK = 157.3e12
HBM_PEAK = 8.0e12
FLOP_PER_TEST = 8              # bead-bead distance test: 3 sub + 1 mul + 2 fma
NN_FLOP_PER_ROW = 100352       # 2 x (7 x 128 + 3 x 128 x 128 + 128) multiply-adds
GRAPH_STEPS = 10               # MD steps recorded per HIP graph

# Gap window of the network path (shells' lower bound on the closest bead
# distance, sigma units) and that of the pairs its training data is drawn from.
GAP_MIN, GAP_MAX, SAMPLE_GAP_MIN = 1.0, 2.5, 0.8

# HBM bytes per launch of the network path's forces kernel on the headline
# workload at its start (31.3k network pairs, 2.5k fallback pairs), from two
# rocprofv3 counter runs (FETCH_SIZE 8204.81 KiB x 2.000, WRITE_SIZE
# 12726.69 KiB x 1.000; the factors are what the counters read for a 256 MiB
# copy), see profiles/k_nn_wide_cyl32768_hbm_traffic.txt.  Valid only for the
# kernel sources they were taken on (hash below); otherwise reported as null.
NN_TRAFFIC_BYTES = 29835581
NN_TRAFFIC_SOURCES = ("paper_2402_12199_amd/csrc/nn.hip", "paper_2402_12199_amd/csrc/nn_tile.hpp",
                      "paper_2402_12199_amd/csrc/nn_common.hpp", "paper_2402_12199_amd/csrc/cyl_form.hpp",
                      "paper_2402_12199_amd/csrc/rb_common.hpp", "paper_2402_12199_amd/csrc/bead_pair.hpp")
NN_TRAFFIC_HASH = "45f80cbe9c57f728"


def sources_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def nn_traffic():
    if NN_TRAFFIC_BYTES is None or sources_hash(NN_TRAFFIC_SOURCES) != NN_TRAFFIC_HASH:
        return None
    return NN_TRAFFIC_BYTES


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_system(cfg, st, path, model=None):
    from paper_2402_12199_amd.md import RigidSystem
    b = cfg.body
    s = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                    cfg.r_list, cfg.skin, hphc=cfg.hphc, margin=cfg.bead_margin)
    if model is not None:
        s.set_nn(model)
    return s


def count_within(sysm, r, torch, abi):
    """Listed pairs whose minimum-image centre distance is below r (counted
    on the device from the list and the positions)."""
    m = int(sysm.flags[abi.RB_FLAG_NPAIRS].item())
    i = sysm.pair_i[:m].long()
    j = sysm.pair_j[:m].long()
    d = sysm.x[:, j] - sysm.x[:, i]
    box = torch.as_tensor(np.broadcast_to(np.asarray(sysm.box, np.float64), (3,)).copy(), device=d.device)[:, None]
    d = d - box * torch.round(d / box)
    return int(((d * d).sum(0) < r * r).sum().item())


def run_md(sysm, steps, warmup, dt, path, d_cut, torch, abi):
    """Warm up eagerly, record GRAPH_STEPS fused steps into a HIP graph (and
    the remainder of `steps` into a second one), and time exactly `steps`
    steps as graph replays between a synchronisation on each side."""
    for _ in range(warmup):
        sysm.step(dt, path)
    torch.cuda.synchronize()
    sysm.check_capacity()
    sysm.begin_fused(dt)
    g = sysm.capture(dt, path, GRAPH_STEPS, fused=True)
    rem = steps % GRAPH_STEPS
    g_rem = sysm.capture(dt, path, rem, fused=True) if rem else None
    g.replay()                      # one untimed replay
    torch.cuda.synchronize()
    f0 = sysm.check_capacity()
    within0 = count_within(sysm, d_cut, torch, abi)
    st = torch.cuda.current_stream()
    e_start = torch.cuda.Event(enable_timing=True)
    e_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record(st)
    for _ in range(steps // GRAPH_STEPS):
        g.replay()
    if g_rem is not None:
        g_rem.replay()
    e_end.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f1 = sysm.check_capacity()
    within1 = count_within(sysm, d_cut, torch, abi)
    gpu_ms = e_start.elapsed_time(e_end)
    sysm.end_fused(dt, path)
    torch.cuda.synchronize()
    sysm.check_capacity()
    return dict(wall_s=wall, steps=steps, gpu_ms=gpu_ms, pairs_within=[within0, within1],
                pairs_within_mean=0.5 * (within0 + within1),
                listed_pairs_evaluated=(int(f1[abi.RB_FLAG_NEVAL]) - int(f0[abi.RB_FLAG_NEVAL])) % (1 << 32),
                rebuilds=int(f1[abi.RB_FLAG_NREBUILDS] - f0[abi.RB_FLAG_NREBUILDS]),
                rescreens=int(f1[abi.RB_FLAG_NRESCREENS] - f0[abi.RB_FLAG_NRESCREENS]),
                n_candidates=int(f1[abi.RB_FLAG_NSCREEN]),
                n_listed=int(f1[abi.RB_FLAG_NPAIRS]), n_nn=int(f1[abi.RB_FLAG_NNN]), n_bead=int(f1[abi.RB_FLAG_NBEAD]))


def time_launches(fn, reps, torch):
    """Mean device duration of `fn` (kernel launches on the current stream):
    `reps` calls recorded once into a HIP graph, the graph replayed on the
    current stream between HIP events recorded on that stream."""
    fn()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for _ in range(reps):
            fn()
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(st)
    g.replay()
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def roof(ms, work, peak, unit, bound, what):
    rate = work / (ms * 1e-3)
    scale = 1e9 if unit == "GB/s" else 1e12
    return {"ms": ms, "bound": bound, "achieved": rate / scale, "unit": unit, "peak": peak / scale,
            "frac": rate / peak, "algorithmic_work": what}


def ntests(sysm, abi):
    f = sysm.flags_host()
    return int(f[abi.RB_FLAG_NTESTS:abi.RB_FLAG_NTESTS + 2].view(np.int64)[0])


def nn_forces_launch(sysm, abi):
    """The network path's pair forces of one step: one launch that evaluates
    the network pairs and then the bead sums of the fallback pairs."""
    m = sysm.nn
    return lambda: abi.rb_nn_pair_forces_routed(sysm.ctx, m.params, m.norm, m.precision, 1, sysm.x, sysm.q,
                                                sysm.types, sysm.box, sysm.pair_i, sysm.pair_j, sysm.desc,
                                                sysm.idx_nn, sysm.flags[abi.RB_FLAG_NNN:], sysm.idx_bead,
                                                sysm.flags[abi.RB_FLAG_NBEAD:], sysm.max_pairs, m.sw_lo, m.sw_hi,
                                                sysm.acc, sysm.flags)


def nn_forces_roofline(sysm, torch, abi, reps=20):
    """The network path's dominant kernel alone on the current routing: mean
    duration over `reps` launches.  achieved = the network's FLOP per launch
    (2 x 100352 per network pair: forward and input-gradient pass) over that
    duration, against the dense BF16 MFMA peak; the bead sums of the fallback
    pairs in the same launch are FP32 vector work, reported beside it (tests
    x 8 FLOP against the FP32 vector peak) and in frac_combined, the sum of
    both parts' times at their peaks over the launch's duration."""
    launch = nn_forces_launch(sysm, abi)
    t0 = ntests(sysm, abi)
    ms = time_launches(launch, reps, torch)
    tests = (ntests(sysm, abi) - t0) / (reps + 1)    # one eager call + one replay of reps
    abi.rb_accum_zero(sysm.n, sysm.acc)
    f = sysm.flags_host()
    nnn, nbead = int(f[abi.RB_FLAG_NNN]), int(f[abi.RB_FLAG_NBEAD])
    flop = 2.0 * NN_FLOP_PER_ROW * nnn
    r = roof(ms, flop, BF16_MFMA_PEAK, "TFLOP/s", "mfma",
             f"2 x {NN_FLOP_PER_ROW} FLOP per network pair (forward + input-gradient pass) x {nnn} pairs "
             f"per launch; the same launch's bead sums of {nbead} fallback pairs are not counted here")
    bead_flop = tests * FLOP_PER_TEST
    r["pairs_per_launch"] = nnn
    r["fallback"] = {"pairs_per_launch": nbead, "bead_tests_per_launch": tests, "flop": bead_flop,
                     "peak_tflops": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s"}
    r["frac_combined"] = (flop / BF16_MFMA_PEAK + bead_flop / FP32_VECTOR_PEAK) / (ms * 1e-3)
    return r


def path_kernels(sysn, sysb, cfg, torch, abi):
    """The per-step kernels of both paths, each timed alone on the current
    state of its system (after the timed steps)."""
    out = {}
    n = sysn.n
    npairs = int(sysn.flags_host()[abi.RB_FLAG_NPAIRS])
    ms = time_launches(lambda: sysn.build_pairs(always=True), 10, torch)
    out["pair_list_rebuild"] = roof(ms, 32.0 * n + 8.0 * npairs, HBM_PEAK, "GB/s", "hbm",
                                    f"32 B per body + 8 B per listed pair ({n} bodies, {npairs} pairs)")
    m = sysn.nn
    ms = time_launches(lambda: sysn.route(m.d_min, m.sw_hi, m.gap_min, m.gap_max, two_level=False), 20, torch)
    f = sysn.flags_host()
    nnn, nbead = int(f[abi.RB_FLAG_NNN]), int(f[abi.RB_FLAG_NBEAD])
    out["pair_descriptors_routing_full"] = roof(ms, 128.0 * npairs + 32.0 * (nnn + nbead), HBM_PEAK, "GB/s", "hbm",
                                                f"128 B read per listed pair (FP64 state of both bodies, indices, "
                                                f"types) + 32 B written per routed pair ({npairs} listed, {nnn} "
                                                f"network, {nbead} bead)")
    out["pair_descriptors_routing_full"]["note"] = "every listed pair (a screening step's work, less its list)"
    ms = time_launches(lambda: sysn.route(m.d_min, m.sw_hi, m.gap_min, m.gap_max), 20, torch)
    f = sysn.flags_host()
    ncand = int(f[abi.RB_FLAG_NSCREEN])
    nnn, nbead = int(f[abi.RB_FLAG_NNN]), int(f[abi.RB_FLAG_NBEAD])
    out["pair_descriptors_routing"] = roof(ms, 132.0 * ncand + 32.0 * (nnn + nbead), HBM_PEAK, "GB/s", "hbm",
                                           f"132 B read per candidate pair (its index, FP64 state of both "
                                           f"bodies, indices, types) + 32 B written per routed pair ({ncand} "
                                           f"candidates of {npairs} listed, {nnn} network, {nbead} bead)")
    out["pair_descriptors_routing"]["note"] = ("two-level routing between screenings; bound by the shells' "
                                               "arithmetic and the load latency, not by HBM")
    ms = time_launches(lambda: abi.rb_nn_pair_forces_cyl(m.params, m.norm, m.precision, sysn.q, sysn.pair_i,
                                                         sysn.pair_j, sysn.desc, sysn.idx_nn,
                                                         sysn.flags[abi.RB_FLAG_NNN:], sysn.max_pairs, m.sw_lo,
                                                         m.sw_hi, sysn.acc, sysn.flags), 20, torch)
    abi.rb_accum_zero(n, sysn.acc)
    out["network_pairs_only"] = roof(ms, 2.0 * NN_FLOP_PER_ROW * nnn, BF16_MFMA_PEAK, "TFLOP/s", "mfma",
                                     f"2 x {NN_FLOP_PER_ROW} FLOP per network pair x {nnn} pairs per launch "
                                     f"(the network part of the step's forces launch, alone)")
    t0 = ntests(sysn, abi)
    ms = time_launches(lambda: abi.rb_bead_pair_forces(sysn.ctx, sysn.x, sysn.q, sysn.types, sysn.box, sysn.pair_i,
                                                       sysn.pair_j, sysn.idx_bead, sysn.flags[abi.RB_FLAG_NBEAD:],
                                                       sysn.max_pairs, sysn.acc, sysn.flags), 10, torch)
    tests = (ntests(sysn, abi) - t0) / 21            # one eager call + two replays of 10
    abi.rb_accum_zero(n, sysn.acc)
    out["bead_fallback"] = roof(ms, tests * FLOP_PER_TEST, FP32_VECTOR_PEAK, "TFLOP/s", "alu",
                                f"{tests:.0f} bead-bead tests x {FLOP_PER_TEST} FLOP per launch ({nbead} pairs)")
    t0 = ntests(sysb, abi)
    ms = time_launches(sysb.bead_forces, 10, torch)
    tests = (ntests(sysb, abi) - t0) / 21
    abi.rb_accum_zero(sysb.n, sysb.acc)
    out["bead_path_forces"] = roof(ms, tests * FLOP_PER_TEST, FP32_VECTOR_PEAK, "TFLOP/s", "alu",
                                   f"{tests:.0f} bead-bead tests x {FLOP_PER_TEST} FLOP per launch (the tests "
                                   f"left after culling; two-level list)")
    ms = time_launches(lambda: abi.rb_accum_finalize(n, sysn.acc, sysn.force, sysn.torque, sysn.ev, sysn.flags), 20,
                       torch)
    out["accum_finalize"] = roof(ms, 120.0 * n, HBM_PEAK, "GB/s", "hbm",
                                 "120 B per body (6 int64 read and cleared, 6 FP32 written)")
    saved = {k: getattr(sysn, k).clone() for k in ("x", "P", "q", "L")}
    ms = time_launches(lambda: abi.rb_rigid_step_fused(sysn.ctx, cfg.dt, sysn.x, sysn.P, sysn.q, sysn.L, sysn.types,
                                                       sysn.acc, sysn.force, sysn.torque, sysn.ev, sysn.x_ref,
                                                       sysn.half_skin, None, sysn.flags, sysn.ws_rig), 20, torch)
    for k, v in saved.items():
        getattr(sysn, k).copy_(v)
    out["rigid_step_fused"] = roof(ms, 248.0 * n, HBM_PEAK, "GB/s", "hbm",
                                   "248 B per body (FP64 state read and written, accumulator, forces)")
    return out


def builder_4m(box_per_body, r_list, torch, abi):
    """The pair builder in its bandwidth regime: 2^22 point bodies at the
    headline system's number density, uniform positions."""
    from paper_2402_12199_amd.md import RigidSystem
    from synth import sampling
    nb = 1 << 22
    boxb = box_per_body * nb ** (1.0 / 3.0)
    zero = np.zeros((nb, 3))
    big = RigidSystem([np.zeros((1, 3))], [1.0], [[1.0, 1.0, 1.0]], np.zeros(nb, np.int32),
                      sampling.rng(31).random((nb, 3)) * boxb, np.tile([1.0, 0, 0, 0], (nb, 1)), zero, zero, boxb,
                      r_list, 0.0)
    ms = time_launches(lambda: big.build_pairs(always=True), 5, torch)
    npb = int(big.check_capacity()[abi.RB_FLAG_NPAIRS])
    del big
    torch.cuda.empty_cache()
    return roof(ms, 32.0 * nb + 8.0 * npb, HBM_PEAK, "GB/s", "hbm",
                f"32 B per body + 8 B per listed pair ({nb} bodies, {npb} pairs)")


def nn_kernels(torch, abi):
    """Network kernels on 2^20 random cylinder pair configurations (forward,
    forward + input gradient; BF16 and FP32)."""
    from paper_2402_12199_amd.nn import make_norm
    from synth import configs, sampling
    cfg = configs.config3()
    desc = sampling.pair_batch(sampling.rng(cfg.seed), cfg.n_pairs, cfg.d_lo, cfg.d_cut).astype(np.float32)
    d = torch.tensor(np.ascontiguousarray(desc.T), device="cuda")
    params = torch.tensor(sampling.xavier_params(cfg.seed).astype(np.float32), device="cuda")
    norm = make_norm(cfg.d_cut)
    P = cfg.n_pairs
    E = torch.empty(P, dtype=torch.float32, device="cuda")
    ft = torch.empty((9, P), dtype=torch.float32, device="cuda")
    out = {}
    for prec, name in ((abi.RB_PREC_BF16, "bf16"), (abi.RB_PREC_FP32, "fp32")):
        for kind in ("fwd", "fwd_grad"):
            def call():
                if kind == "fwd":
                    abi.rb_nn_pair_eval(params, norm, prec, d, E)
                else:
                    abi.rb_nn_pair_grad(params, norm, prec, d, None, E, None, ft)
            ms = time_launches(call, 5, torch)
            flop = (1 if kind == "fwd" else 2) * NN_FLOP_PER_ROW * P
            peak = BF16_MFMA_PEAK if prec == abi.RB_PREC_BF16 else FP32_MFMA_PEAK
            out[f"{name}_{kind}"] = dict(ms=ms, pairs_per_s=P / (ms * 1e-3), tflops=flop / (ms * 1e-3) / 1e12,
                                         mfma_frac=flop / (ms * 1e-3) / peak)
    return out


def train_kernels(body, d_min, d_cut, torch, abi):
    """One training step at batch 8192 (energy loss; energy + force/torque
    matching), and the bead labelling of 2^16 cylinder pairs."""
    from paper_2402_12199_amd.nn import Trainer, make_norm
    from synth import sampling
    g = sampling.rng(9)
    n = 1 << 16
    desc = sampling.pair_batch(g, n, d_min, d_cut).astype(np.float32)
    dd = torch.tensor(np.ascontiguousarray(desc.T), device="cuda")
    yy = torch.tensor(g.standard_normal(n).astype(np.float32), device="cuda")
    ft = torch.tensor(g.standard_normal((6, n)).astype(np.float32), device="cuda")
    idx = torch.arange(8192, dtype=torch.int32, device="cuda")
    norm = make_norm(d_cut)
    out = {}
    tr = Trainer(sampling.xavier_params(6), norm, batch=8192)
    ms = time_launches(lambda: tr.step(dd, yy, idx), 20, torch)
    out["train_step_8192"] = roof(ms, 3.0 * NN_FLOP_PER_ROW * 8192, BF16_MFMA_PEAK, "TFLOP/s", "mfma",
                                  "3 x 100352 FLOP per sample (forward, reverse pass, weight gradients), "
                                  "batch 8192")
    trf = Trainer(sampling.xavier_params(6), norm, batch=8192, fm=dict(lam_f=1e-3, lam_t=1e-3))
    ms = time_launches(lambda: trf.step(dd, yy, idx, ft=ft), 20, torch)
    out["train_step_fm_8192"] = roof(ms, 9.0 * NN_FLOP_PER_ROW * 8192, BF16_MFMA_PEAK, "TFLOP/s", "mfma",
                                     "9 x 100352 FLOP per sample (forward and tangent rows, their reverse "
                                     "passes, weight gradients over both), batch 8192")
    ctx = abi.Ctx([body.beads], [body.mass], [body.inertia])
    flags = torch.zeros(abi.RB_NFLAGS, dtype=torch.int32, device="cuda")
    lab = torch.empty((11, n), dtype=torch.float32, device="cuda")
    ms = time_launches(lambda: abi.rb_bead_pair_eval(ctx, dd, 0, 0, lab, flags), 5, torch)
    f = flags.cpu().numpy()
    tests = int(f[abi.RB_FLAG_NTESTS:abi.RB_FLAG_NTESTS + 2].view(np.int64)[0]) / 11
    out["bead_labels_2^16"] = roof(ms, tests * FLOP_PER_TEST, FP32_VECTOR_PEAK, "TFLOP/s", "alu",
                                   f"{tests:.0f} culled bead tests x {FLOP_PER_TEST} FLOP per launch "
                                   f"(2^16 uniformly drawn cylinder pairs)")
    out["bead_labels_2^16"]["pairs_per_s"] = n / (ms * 1e-3)
    return out


def cpu_baseline(cfg, st, target_s=12.0):
    """The FP64 oracle on the host: NVE steps of the headline system (full
    force evaluation + integration per step), the oracle network's forward
    and input gradient on 2^16 rows, the oracle bead sum on 2^14 cylinder
    pairs."""
    from oracle import beads as ob
    from oracle import mlp as om
    from synth import sampling
    x = np.ascontiguousarray(st["x"].copy())
    P = np.ascontiguousarray(st["P"].copy())
    q = np.ascontiguousarray(st["q"].copy())
    L = np.ascontiguousarray(st["L"].copy())
    b = cfg.body
    t0 = time.perf_counter()
    r = ob.bead_system(x, q, st["types"], [b.beads], cfg.box)
    per_eval = time.perf_counter() - t0
    steps = max(1, int(target_s / max(per_eval, 1e-3)) - 1)
    t0 = time.perf_counter()
    ob.nve(x, P, q, L, st["types"], [b.beads], [b.mass], [b.inertia], cfg.box, steps, cfg.dt)
    wall = time.perf_counter() - t0
    evals = steps + 1
    out = dict(value=r["n_pairs"] * evals / wall, unit="rigid-pair F+tau evals/s", cores=ob.num_threads(),
               kind="oracle",
               sample=f"{steps} NVE steps (+1 initial force evaluation) of the same {cfg.n_bodies}-cylinder system "
                      f"from the same start, {r['n_pairs']} pairs within 2 r_max + rc per evaluation, FP64 C "
                      f"oracle (all-pairs search, OpenMP over pairs), wall {wall:.1f} s",
               md_steps_per_s=evals / wall)
    params = sampling.xavier_params(5)
    d = sampling.pair_batch(sampling.rng(3), 1 << 16, cfg.d_min, cfg.d_cut)
    norm = om.Norm(in_scale=np.array([1 / cfg.d_cut] * 3 + [1.0] * 4))
    t0 = time.perf_counter()
    om.input_grad(params, d, norm)
    t_mlp = time.perf_counter() - t0
    out["mlp_fwd_grad"] = dict(rows=1 << 16, s=t_mlp, pairs_per_s=(1 << 16) / t_mlp,
                               kind="oracle (numpy FP64 forward + input gradient)")
    t0 = time.perf_counter()
    ob.bead_pair_desc(b.beads, b.beads, d[:1 << 14])
    t_bead = time.perf_counter() - t0
    out["bead_pairs"] = dict(pairs=1 << 14, s=t_bead, pairs_per_s=(1 << 14) / t_bead,
                             kind="oracle (C FP64 bead double sum, uniformly drawn cylinder pairs)")
    return out


def kernels_only(args, torch, abi):
    """The dominant kernels of both paths on the headline system at its start
    (network with Xavier weights: routing and cost do not depend on the
    weights), for counter runs."""
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.nn import make_norm_features, sym_descriptors
    from synth import configs, sampling, state
    c5 = configs.config5()
    st = state.initial_state(c5)
    sysb = make_system(c5, st, "bead")
    sysb.init_forces("bead")
    sysn = make_system(c5, st, "nn")
    desc = sysn.pair_configurations(c5.d_min, c5.d_cut, GAP_MIN, GAP_MAX)
    s = sym_descriptors(desc.contiguous(), with_jac=False, form="cyl")[0].cpu().numpy().T
    model = NNModel(params=torch.tensor(sampling.xavier_params(7).astype(np.float32), device="cuda"),
                    norm=make_norm_features(s), d_min=c5.d_min, sw_lo=c5.d_cut - 1.0, sw_hi=c5.d_cut, form="cyl",
                    gap_min=GAP_MIN, gap_max=GAP_MAX)
    sysn.set_nn(model)
    sysn.init_forces("nn")
    torch.cuda.synchronize()
    r = {"nn_forces": nn_forces_roofline(sysn, torch, abi, reps=args.steps)}
    ms = time_launches(sysb.bead_forces, args.steps, torch)
    r["bead_path_forces_ms"] = ms
    print(json.dumps(r), flush=True)


def cubes_part(args, torch, abi):
    """The bead path on 4096 cube shells (152 beads, volume fraction 0.20)."""
    from synth import configs, state
    cfg = configs.config2()
    st = state.initial_state(cfg)
    sysm = make_system(cfg, st, "bead")
    sysm.init_forces("bead")
    r = run_md(sysm, args.steps, args.warmup, cfg.dt, "bead", cfg.d_cut, torch, abi)
    return {"workload": f"{cfg.name}: {cfg.n_bodies} cube shells ({cfg.body.n} beads), LJ, NVE kT={cfg.kT} "
                        f"dt={cfg.dt}, bead path",
            "pair_evals_per_s": r["pairs_within_mean"] * r["steps"] / r["wall_s"],
            "md_steps_per_s": r["steps"] / r["wall_s"], "pairs_within": r["pairs_within"],
            "listed_pairs": r["n_listed"]}


def hphc_part(args, torch, abi):
    """The paper's half-power half-cosine bead potential on 4096 cube shells
    (volume fraction 0.16, kT=1): surrogates trained on the pairs the bead
    dynamics visits (energy; energy with force and torque matching; the
    symmetry-reduced cube-pair descriptor), then 2008 steps of the bead path
    and of each network path from the same start, at constant energy and at
    constant temperature (Nose-Hoover)."""
    from paper_2402_12199_amd.compare import compare
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.surrogate import train_surrogate_md
    from synth import configs, state
    cfg = configs.config_hphc()
    st = state.initial_state(cfg)
    kw = dict(precision=abi.RB_PREC_BF16, d_min=cfg.d_min, sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut)
    ep = args.hphc_epochs
    sur = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, ep, r_rej=0.0, log=log)
    fm = dict(weight=10.0)
    surf = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, ep, r_rej=0.0, log=log, fm=fm)
    surs = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, ep, r_rej=0.0, log=log, sym=True)
    models = {"nn_md": NNModel(params=sur["params"], norm=sur["norm"], **kw),
              "nn_md_fm": NNModel(params=surf["params"], norm=surf["norm"], **kw),
              "nn_md_sym": NNModel(params=surs["params"], norm=surs["norm"], sym=True, **kw)}
    out = {"workload": f"{cfg.name}: {cfg.n_bodies} cube shells ({cfg.body.n} beads), half-power half-cosine "
                       f"A={cfg.hphc['A']} b={cfg.hphc['b']} c={cfg.hphc['c']} p={cfg.hphc['p']}, "
                       f"kT={cfg.kT} dt={cfg.dt}",
           "held_out": {"energy": sur["trained"], "force_matching": surf["trained"], "symmetry_reduced":
                        surs["trained"]}}
    out["dynamics"] = compare(cfg, st, models, chunks=8, replays=25, log=log)
    out["dynamics_nvt"] = compare(cfg, st, models, chunks=8, replays=25, log=log, nvt=dict(kT=cfg.kT, tau=0.5))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=600, help="surrogate training epochs (2^21 pairs each)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-dynamics", action="store_true", help="skip the 2008-step bead-vs-network comparison")
    ap.add_argument("--no-kernels", action="store_true", help="skip the per-kernel table")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch the dominant kernels of both paths on the headline system (counter runs)")
    ap.add_argument("--extras", action="store_true",
                    help="also the bead path on 4096 cubes and the half-power half-cosine cube surrogates")
    ap.add_argument("--hphc-epochs", type=int, default=300)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path is single-GPU (--gpus {args.gpus} is not supported)",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be at least 1 and --warmup at least 0", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2402_12199_amd import abi
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.surrogate import train_surrogate_md
    from synth import configs, state

    if args.kernels_only:
        kernels_only(args, torch, abi)
        return

    c5 = configs.config5()
    log(f"[bench] generating {c5.name}")
    st = state.initial_state(c5)

    log(f"[bench] surrogate: bead-MD pairs of {c5.name} at kT = 1, 2, 4, {args.epochs} epochs")
    t0 = time.perf_counter()
    sur = train_surrogate_md(c5, st, 1 << 21, 1 << 16, args.epochs, every=25, gap_min=SAMPLE_GAP_MIN,
                             gap_max=GAP_MAX, form="cyl", kTs=[1.0, 2.0, 4.0], lr_end=1e-5, log=log)
    t_sur = time.perf_counter() - t0
    model = NNModel(params=sur["params"], norm=sur["norm"], precision=abi.RB_PREC_BF16, d_min=c5.d_min,
                    sw_lo=c5.d_cut - 1.0, sw_hi=c5.d_cut, form="cyl", gap_min=GAP_MIN, gap_max=GAP_MAX)
    surrogate = {k: sur[k] for k in ("sampling", "epochs", "steps", "batch", "n_train", "n_test", "label_s",
                                     "train_s", "samples_per_s")}
    surrogate.update(form="cylinder four-number descriptor", total_s=t_sur, held_out=sur["trained"],
                     held_out_untrained=sur["untrained"], loss_first_last=[sur["loss_history"][0],
                                                                           sur["loss_history"][-1]])

    legs = {}
    systems = {}
    for path in ("bead", "nn"):
        sysm = make_system(c5, st, path, model if path == "nn" else None)
        sysm.init_forces(path)
        torch.cuda.synchronize()
        ke0 = float((st["P"] ** 2).sum() / (2 * c5.body.mass) + (st["L"] ** 2 / (2 * c5.body.inertia)).sum())
        e0 = sysm.energy() + ke0
        log(f"[bench] {path} path: {args.warmup} warmup + {args.steps} timed steps")
        r = run_md(sysm, args.steps, args.warmup, c5.dt, path, c5.d_cut, torch, abi)
        e1 = sysm.energy() + float(sysm.kinetic_host().sum())
        r.update(md_steps_per_s=r["steps"] / r["wall_s"], ms_per_step=1e3 * r["wall_s"] / r["steps"],
                 gpu_ms_per_step=r["gpu_ms"] / r["steps"],
                 pair_evals_per_s=r["pairs_within_mean"] * r["steps"] / r["wall_s"],
                 total_energy_start_end=[e0, e1],
                 energy_change_per_body=(e1 - e0) / c5.n_bodies,
                 steps_in_energy_change=1 + args.warmup + GRAPH_STEPS + args.steps)
        legs[path] = r
        systems[path] = sysm
    nn, bead = legs["nn"], legs["bead"]
    nn["pairs_skipped_by_bound"] = nn["n_listed"] - nn["n_nn"] - nn["n_bead"]

    log("[bench] dominant kernel of the network path")
    rl = nn_forces_roofline(systems["nn"], torch, abi)
    roofline = {"kernel": "k_nn_wide<2, true, 1> (rb_nn_pair_forces_routed: network pairs, then the fallback "
                          "pairs' bead sums)", "bound": "mfma", "achieved": rl["achieved"],
                "peak": rl["peak"], "unit": "TFLOP/s", "frac": rl["frac"], "traffic": nn_traffic(),
                "traffic_unit": "bytes per launch", "kernel_ms": rl["ms"], "algorithmic_work": rl["algorithmic_work"],
                "fallback": rl["fallback"], "frac_combined": rl["frac_combined"]}

    value = nn["pair_evals_per_s"]
    result = {
        "metric": "rigid-pair F+tau evals/sec and MD steps/sec, NN(BF16) vs bead-sum(FP32), 1 GPU",
        "value": value,
        "unit": "rigid-pair F+tau evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": nn["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded random placement and orientations, Maxwell-Boltzmann momenta; surrogate "
                "trained in this run on pairs of seeded bead-path runs)",
        "config": {"workload": f"{c5.name}: {c5.n_bodies} cylinders ({c5.body.n} beads), LJ rc={c5.rc}, NVE "
                               f"kT={c5.kT} dt={c5.dt}, network path (BF16 surrogate on the cylinder "
                               f"four-number descriptor, bead sum below a shells' bound of {GAP_MIN})",
                   "n_bodies": c5.n_bodies, "beads_per_body": c5.body.n, "box": c5.box,
                   "pair_range": c5.d_cut, "pairs_within_range": nn["pairs_within"]},
        "md_steps_per_s": nn["md_steps_per_s"],
        "nn_path": nn,
        "bead_path": bead,
        "nn_vs_bead": {"md_steps_per_s": nn["md_steps_per_s"] / bead["md_steps_per_s"],
                       "pair_evals_per_s": nn["pair_evals_per_s"] / bead["pair_evals_per_s"]},
        "surrogate": surrogate,
        "roofline": roofline,
    }

    if not args.no_kernels:
        log("[bench] per-kernel table")
        kt = path_kernels(systems["nn"], systems["bead"], c5, torch, abi)
        kt["nn_pair_forces"] = rl
        box_per_body = float(c5.box) / c5.n_bodies ** (1.0 / 3.0)
        for k in list(systems):
            del systems[k]
        torch.cuda.empty_cache()
        kt["pair_list_rebuild_4M"] = builder_4m(box_per_body, c5.r_list, torch, abi)
        kt.update(train_kernels(c5.body, c5.d_min, c5.d_cut, torch, abi))
        result["kernels"] = kt
        log("[bench] network kernels on 2^20 pairs")
        result["nn_kernels_2^20"] = nn_kernels(torch, abi)
    systems.clear()

    if not args.no_dynamics:
        from paper_2402_12199_amd.compare import compare
        log("[bench] bead vs network dynamics, 2008 steps each")
        result["dynamics"] = compare(c5, st, {"nn": model}, chunks=8, replays=25, log=log)

    if args.extras:
        result["cubes4096"] = cubes_part(args, torch, abi)
        result["hphc_cubes"] = hphc_part(args, torch, abi)

    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(c5, st)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
