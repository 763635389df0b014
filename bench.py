"""Benchmark of the rigid-body pair path on one MI355X.

Workload of the headline number: 4096 cube shells of 152 beads (6x6x6
surface lattice) at volume fraction 0.20, kT = 1, NVE velocity Verlet at
dt = 0.005, cell-list pair list with skin 1.0.  A step is one MD step of the
plain bead path: half kick + drift + free rotation, conditional list
rebuild, the FP32 bead double sum over every listed pair with per-body
accumulation, the second half kick.  value = rigid-pair F+tau evaluations
per second over the timed steps.

Also reported (same run): a cube-6 surrogate trained on bead-labelled
pairs (held-out errors), the network path on the same system with it (BF16
MLP with bead fallback below d_min), the network kernels on 2^20 random
cylinder pairs (forward, forward + input gradient; BF16 and FP32), the
per-kernel roofline of the bead kernel, cylinder surrogates with the
bead-vs-network dynamics of 32768 cylinders, the same comparison on cube
shells with the paper's half-power half-cosine bead potential, and the FP64
oracle on the host as a CPU baseline.  Inputs are synthetic and seeded.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
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
FLOP_PER_TEST = 8              # 3 sub + 1 mul + 2 fma

# HBM bytes per launch of the bead kernel on this workload, from two rocprofv3
# counter runs (FETCH_SIZE, WRITE_SIZE; profiles/k_bead_md_cubes4096_hbm_traffic.txt),
# each scaled by what the counter reads for a copy kernel of known size.  Valid
# only for the kernel sources they were taken on (hash below); otherwise null.
BEAD_TRAFFIC_BYTES = 4.89e6
BEAD_TRAFFIC_SOURCES = ("paper_2402_12199_amd/csrc/bead.hip", "paper_2402_12199_amd/csrc/rb_common.hpp")
BEAD_TRAFFIC_HASH = "4365cb67d1289c21"


def bead_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in BEAD_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return BEAD_TRAFFIC_BYTES if h.hexdigest()[:16] == BEAD_TRAFFIC_HASH else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_system(cfg, st, torch):
    from paper_2402_12199_amd.md import RigidSystem
    b = cfg.body
    return RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin, hphc=cfg.hphc, margin=cfg.bead_margin)


GRAPH_STEPS = 10   # MD steps recorded per HIP graph


def run_md(sysm, steps, warmup, dt, path, torch, abi):
    """Warm up eagerly, record GRAPH_STEPS steps into a HIP graph, and time
    `steps` steps as graph replays (steps is rounded up to a multiple of
    GRAPH_STEPS).  Returns timing and device counters."""
    for _ in range(warmup):
        sysm.step(dt, path)
    torch.cuda.synchronize()
    sysm.check_capacity()
    # fused stepping: each step is pair list (skipped unless flagged), forces
    # into the accumulator, and one integrator launch that ends this step and
    # starts the next
    sysm.begin_fused(dt)
    g = sysm.capture(dt, path, GRAPH_STEPS, fused=True)
    g.replay()                      # one untimed replay
    torch.cuda.synchronize()
    f0 = sysm.check_capacity()
    st = torch.cuda.current_stream()
    reps = (steps + GRAPH_STEPS - 1) // GRAPH_STEPS
    e_start = torch.cuda.Event(enable_timing=True)
    e_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record(st)
    for _ in range(reps):
        g.replay()
    e_end.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f1 = sysm.check_capacity()
    gpu_ms = e_start.elapsed_time(e_end)
    neval = (int(f1[abi.RB_FLAG_NEVAL]) - int(f0[abi.RB_FLAG_NEVAL])) % (1 << 32)
    sysm.end_fused(dt, path)
    # eager steps, timed separately (host launch overhead included)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(GRAPH_STEPS * 5):
        sysm.step(dt, path)
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t1) / (GRAPH_STEPS * 5)
    return dict(wall_s=wall, steps=reps * GRAPH_STEPS, gpu_ms=gpu_ms, pairs_evaluated=neval,
                rebuilds=int(f1[abi.RB_FLAG_NREBUILDS] - f0[abi.RB_FLAG_NREBUILDS]),
                n_pairs=int(f1[abi.RB_FLAG_NPAIRS]), n_nn=int(f1[abi.RB_FLAG_NNN]),
                n_bead=int(f1[abi.RB_FLAG_NBEAD]), eager_ms_per_step=eager_ms)


def ntests(flags_np, abi):
    return int(flags_np[abi.RB_FLAG_NTESTS:abi.RB_FLAG_NTESTS + 2].view(np.int64)[0])


def bead_kernel_time(sysm, reps, torch, abi):
    """Mean duration of the bead-sum kernel alone on the current list (HIP
    events on the launch stream around `reps` back-to-back launches), and the
    bead-bead distance tests it performs per launch (after culling)."""
    st = torch.cuda.current_stream()
    abi.rb_accum_zero(sysm.n, sysm.acc)

    def launch():
        abi.rb_bead_pair_forces(sysm.ctx, sysm.x, sysm.q, sysm.types, sysm.box, sysm.pair_i, sysm.pair_j, None,
                                sysm.flags[abi.RB_FLAG_NPAIRS:], sysm.max_pairs, sysm.acc, sysm.flags)
    launch()
    torch.cuda.synchronize()
    t0 = ntests(sysm.flags_host(), abi)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        launch()
    b.record(st)
    torch.cuda.synchronize()
    tests = (ntests(sysm.flags_host(), abi) - t0) / reps
    abi.rb_accum_zero(sysm.n, sysm.acc)
    return a.elapsed_time(b) / reps, tests


def time_launches(fn, reps, torch):
    """Mean device duration of `fn` (one or more kernel launches on the
    current stream): `reps` calls recorded once into a HIP graph, the graph
    replayed between HIP events (so host launch overhead does not count)."""
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
    return {"ms": ms, "bound": bound, "achieved": rate / (1e9 if unit == "GB/s" else 1e12), "unit": unit,
            "peak": peak / (1e9 if unit == "GB/s" else 1e12), "frac": rate / peak, "algorithmic_work": what}


def kernel_table(sysm, cfg, torch, abi):
    """Roofline of the hot-path kernels other than the bead sum, each timed
    alone on the cube system's current state (after the timed run)."""
    from paper_2402_12199_amd.nn import Trainer, make_norm
    from synth import sampling
    n, out = sysm.n, {}
    f = sysm.flags_host()
    npairs = int(f[abi.RB_FLAG_NPAIRS])
    ms = time_launches(lambda: sysm.build_pairs(always=True), 10, torch)
    out["pair_list_rebuild"] = roof(ms, 32.0 * n + 8.0 * npairs, HBM_PEAK, "GB/s", "hbm",
                                    f"32 B per body + 8 B per listed pair ({n} bodies, {npairs} pairs)")
    # the builder in its bandwidth regime: 2^22 point bodies at the same
    # number density, uniform positions (multi-kernel path, list sorted by i)
    from paper_2402_12199_amd.md import RigidSystem
    nb = 1 << 22
    boxb = float(sysm.box[0]) * (nb / n) ** (1.0 / 3.0)
    gb = sampling.rng(31)
    zero = np.zeros((nb, 3))
    big = RigidSystem([np.zeros((1, 3))], [1.0], [[1.0, 1.0, 1.0]], np.zeros(nb, np.int32), gb.random((nb, 3)) * boxb,
                      np.tile([1.0, 0, 0, 0], (nb, 1)), zero, zero, boxb, sysm.r_list, 0.0)
    msb = time_launches(lambda: big.build_pairs(always=True), 5, torch)
    npb = int(big.check_capacity()[abi.RB_FLAG_NPAIRS])
    out["pair_list_rebuild_4M"] = roof(msb, 32.0 * nb + 8.0 * npb, HBM_PEAK, "GB/s", "hbm",
                                       f"32 B per body + 8 B per listed pair ({nb} bodies at the cube system's "
                                       f"number density, {npb} pairs)")
    del big
    torch.cuda.empty_cache()
    ms = time_launches(lambda: abi.rb_accum_finalize(n, sysm.acc, sysm.force, sysm.torque, sysm.ev, sysm.flags), 20,
                       torch)
    out["accum_finalize"] = roof(ms, 120.0 * n, HBM_PEAK, "GB/s", "hbm",
                                 "120 B per body (6 int64 read and cleared, 6 FP32 written)")
    st = {k: v.clone() for k, v in (("x", sysm.x), ("P", sysm.P), ("q", sysm.q), ("L", sysm.L))}
    ms = time_launches(lambda: abi.rb_rigid_step_fused(sysm.ctx, cfg.dt, sysm.x, sysm.P, sysm.q, sysm.L, sysm.types,
                                                       sysm.acc, sysm.force, sysm.torque, sysm.ev, sysm.x_ref,
                                                       sysm.half_skin, None, sysm.flags, sysm.ws_rig), 20, torch)
    for k, v in st.items():
        getattr(sysm, k).copy_(v)
    out["rigid_step_fused"] = roof(ms, 248.0 * n, HBM_PEAK, "GB/s", "hbm",
                                   "248 B per body (FP64 state read and written, accumulator, forces)")
    desc = sysm.pair_configurations(cfg.d_min, cfg.d_cut)      # allocates the routing buffers
    ms = time_launches(lambda: abi.rb_pair_descriptors(sysm.x, sysm.q, sysm.box, sysm.pair_i, sysm.pair_j, cfg.d_min,
                                                       sysm.desc, sysm.idx_nn, sysm.idx_bead, sysm.flags,
                                                       d_max=cfg.d_cut), 20, torch)
    out["pair_descriptors"] = roof(ms, 100.0 * npairs, HBM_PEAK, "GB/s", "hbm",
                                   f"100 B per listed pair ({npairs}): two bodies' FP64 state, 7 FP32 out")
    nnn = desc.shape[1]
    params = torch.tensor(sampling.xavier_params(5).astype(np.float32), device="cuda")
    norm = make_norm(cfg.d_cut)
    ms = time_launches(lambda: abi.rb_nn_pair_forces(params, norm, abi.RB_PREC_BF16, sysm.q, sysm.pair_i, sysm.pair_j,
                                                     sysm.desc, sysm.idx_nn, sysm.flags[abi.RB_FLAG_NNN:],
                                                     sysm.max_pairs, cfg.d_cut - 1.0, cfg.d_cut, sysm.acc,
                                                     sysm.flags), 20, torch)
    abi.rb_accum_zero(n, sysm.acc)
    out["nn_pair_forces_md"] = roof(ms, 2 * 100352.0 * nnn, BF16_MFMA_PEAK, "TFLOP/s", "mfma",
                                    f"2 x 100352 FLOP per network pair ({nnn} pairs of the list)")
    tr = Trainer(sampling.xavier_params(6), norm, batch=8192)
    g = sampling.rng(9)
    dd = torch.tensor(np.ascontiguousarray(sampling.pair_batch(g, 1 << 16, cfg.d_min, cfg.d_cut)
                                           .astype(np.float32).T), device="cuda")
    yy = torch.tensor(g.standard_normal(1 << 16).astype(np.float32), device="cuda")
    idx = torch.arange(8192, dtype=torch.int32, device="cuda")
    ms = time_launches(lambda: tr.step(dd, yy, idx), 20, torch)
    out["nn_train_step_8192"] = roof(ms, 3.0e5 * 8192, BF16_MFMA_PEAK, "TFLOP/s", "mfma",
                                     "3.0e5 FLOP per sample (forward, input-to-weight reverse pass, weight "
                                     "gradients), batch 8192")
    lab = torch.empty((11, 1 << 16), dtype=torch.float32, device="cuda")
    t0 = ntests(sysm.flags_host(), abi)
    ms = time_launches(lambda: abi.rb_bead_pair_eval(sysm.ctx, dd, 0, 0, lab, sysm.flags), 5, torch)
    tests = (ntests(sysm.flags_host(), abi) - t0) / 11          # 1 eager call + 2 replays of 5
    out["bead_pair_eval_labels"] = roof(ms, tests * FLOP_PER_TEST, FP32_VECTOR_PEAK, "TFLOP/s", "alu",
                                        f"{tests:.0f} culled bead tests x {FLOP_PER_TEST} FLOP per launch "
                                        f"(2^16 cube-6 configurations)")
    return out


def nn_kernels(torch, abi):
    """Network kernels on 2^20 random cylinder pair configurations."""
    from synth import configs, sampling
    from paper_2402_12199_amd.nn import make_norm
    cfg = configs.config3()
    desc = sampling.pair_batch(sampling.rng(cfg.seed), cfg.n_pairs, cfg.d_lo, cfg.d_cut).astype(np.float32)
    d = torch.tensor(np.ascontiguousarray(desc.T), device="cuda")
    params = torch.tensor(sampling.xavier_params(cfg.seed).astype(np.float32), device="cuda")
    norm = make_norm(cfg.d_cut)
    P = cfg.n_pairs
    E = torch.empty(P, dtype=torch.float32, device="cuda")
    ft = torch.empty((9, P), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    out = {}
    for prec, name in ((abi.RB_PREC_BF16, "bf16"), (abi.RB_PREC_FP32, "fp32")):
        for kind in ("fwd", "fwd_grad"):
            def call():
                if kind == "fwd":
                    abi.rb_nn_pair_eval(params, norm, prec, d, E)
                else:
                    abi.rb_nn_pair_grad(params, norm, prec, d, None, E, None, ft)
            for _ in range(3):
                call()
            reps = 10
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(st)
            for _ in range(reps):
                call()
            b.record(st)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            flop = (100352 if kind == "fwd" else 2 * 100352) * P
            peak = BF16_MFMA_PEAK if prec == abi.RB_PREC_BF16 else FP32_MFMA_PEAK
            out[f"{name}_{kind}"] = dict(ms=ms, pairs_per_s=P / (ms * 1e-3), tflops=flop / (ms * 1e-3) / 1e12,
                                         mfma_frac=flop / (ms * 1e-3) / peak)
    return out


def learned_part(args, torch, abi, log):
    """Cylinder surrogate trained on uniformly drawn pair configurations
    labelled by the bead kernel (2^21, held out 2^16 from another seed), then
    2008 NVE steps of 32768 cylinders with the bead path and with the
    network path (bead fallback below d_min) from the same start."""
    from paper_2402_12199_amd.compare import compare
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.surrogate import train_surrogate, train_surrogate_md
    from synth import configs, state
    c5 = configs.config5()
    log(f"[bench] cylinder surrogate: 2^21 uniform pairs, {args.cyl_epochs} epochs")
    cyl = train_surrogate(c5.body, 1 << 21, 1 << 16, args.cyl_epochs, log=log)
    out = {"surrogate": {k: cyl[k] for k in ("shape", "sampling", "epochs", "steps", "batch", "n_train", "n_test",
                                             "reject_rate", "label_s", "train_s", "samples_per_s", "d_min",
                                             "d_cut")},
           "held_out": cyl["trained"], "held_out_untrained": cyl["untrained"],
           "label_pairs_per_s_with_host_copies": cyl["label_kernel_pairs_per_s"]}
    log(f"[bench] generating {c5.name}")
    st5 = state.initial_state(c5)
    # a second surrogate trained on the pairs the bead dynamics of this
    # workload visits (the paper's data source), held out from later steps
    log(f"[bench] cylinder surrogate on bead-MD pairs of {c5.name}")
    cmd = train_surrogate_md(c5, st5, 1 << 21, 1 << 16, args.cyl_epochs, log=log)
    out["surrogate_md"] = {k: cmd[k] for k in ("sampling", "epochs", "n_train", "n_test", "train_s")}
    out["held_out_md"] = cmd["trained"]

    def model(r):
        return NNModel(params=r["params"], norm=r["norm"], precision=abi.RB_PREC_BF16, d_min=c5.d_min,
                       sw_lo=c5.d_cut - 1.0, sw_hi=c5.d_cut)
    out["dynamics"] = compare(c5, st5, {"nn_uniform": model(cyl), "nn_md": model(cmd)}, chunks=8, replays=25,
                              log=log)
    out["workload"] = f"{c5.name}: {c5.n_bodies} cylinders ({c5.body.n} beads), NVE kT={c5.kT} dt={c5.dt}"
    return out


def hphc_part(args, torch, abi, log):
    """The paper's half-power half-cosine bead potential on 4096 cube shells
    (volume fraction 0.16, NVE kT=1): a surrogate trained on the pairs the
    bead dynamics visits, then 2008 steps of the bead path and of the network
    path from the same start, compared through g(r), P2, MSD, MSR and energy;
    the same again at constant temperature (Nose-Hoover)."""
    from paper_2402_12199_amd.compare import compare
    from paper_2402_12199_amd.md import NNModel
    from paper_2402_12199_amd.surrogate import train_surrogate_md
    from synth import configs, state
    cfg = configs.config_hphc()
    log(f"[bench] generating {cfg.name}")
    st = state.initial_state(cfg)
    log(f"[bench] {cfg.body.name} half-power half-cosine surrogate on bead-MD pairs, {args.hphc_epochs} epochs")
    sur = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, args.hphc_epochs, r_rej=0.0, log=log)
    model = NNModel(params=sur["params"], norm=sur["norm"], precision=abi.RB_PREC_BF16, d_min=cfg.d_min,
                    sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut)
    # the same data with force and torque matching (weights 10 / mean squared label)
    log(f"[bench] {cfg.body.name} surrogate with force and torque matching, {args.hphc_epochs} epochs")
    fm = dict(weight=10.0)
    surf = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, args.hphc_epochs, r_rej=0.0, log=log, fm=fm)
    model_fm = NNModel(params=surf["params"], norm=surf["norm"], precision=abi.RB_PREC_BF16, d_min=cfg.d_min,
                       sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut)
    out = {"workload": f"{cfg.name}: {cfg.n_bodies} cube shells ({cfg.body.n} beads), half-power half-cosine "
                       f"A={cfg.hphc['A']} b={cfg.hphc['b']} c={cfg.hphc['c']} p={cfg.hphc['p']}, "
                       f"NVE kT={cfg.kT} dt={cfg.dt}",
           "surrogate": {k: sur[k] for k in ("sampling", "epochs", "n_train", "n_test", "train_s", "samples_per_s")},
           "held_out": sur["trained"], "held_out_untrained": sur["untrained"],
           "force_matching": {"weights": fm, "lam_f": surf["fm"]["lam_f"], "lam_t": surf["fm"]["lam_t"],
                              "train_s": surf["train_s"], "samples_per_s": surf["samples_per_s"],
                              "held_out": surf["trained"]}}
    # the paper's symmetry-reduced cube-pair descriptor (supplementary section 1)
    log(f"[bench] {cfg.body.name} surrogate on the symmetry-reduced descriptor, {args.hphc_epochs} epochs")
    surs = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, args.hphc_epochs, r_rej=0.0, log=log, sym=True)
    model_sym = NNModel(params=surs["params"], norm=surs["norm"], precision=abi.RB_PREC_BF16, d_min=cfg.d_min,
                        sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut, sym=True)
    out["symmetry_reduced"] = {"descriptor": "(p_x, p_y, p_z, w_y, w_z, cos 4 a3, sin 4 a3)", "train_s": surs["train_s"],
                               "held_out": surs["trained"]}
    models = {"nn_md": model, "nn_md_fm": model_fm, "nn_md_sym": model_sym}
    out["dynamics"] = compare(cfg, st, models, chunks=8, replays=25, log=log)
    # the paper's ensemble: Nose-Hoover NVT at the same temperature
    nvt = dict(kT=cfg.kT, tau=0.5)
    out["dynamics_nvt"] = compare(cfg, st, models, chunks=8, replays=25, log=log, nvt=nvt)
    out["dynamics_nvt"]["thermostat"] = dict(nvt, scheme="Nose-Hoover, one thermostat on all momenta, "
                                                       "g = 6 n - 3, Q = g kT tau^2")
    return out


def cpu_baseline(cfg, st, target_s=12.0):
    """The FP64 oracle (plain C, OpenMP over pairs) doing the same MD steps on
    the host: full force evaluation + integration per step."""
    from oracle import beads as ob
    n = cfg.n_bodies
    x = np.ascontiguousarray(st["x"].copy())
    P = np.ascontiguousarray(st["P"].copy())
    q = np.ascontiguousarray(st["q"].copy())
    L = np.ascontiguousarray(st["L"].copy())
    b = cfg.body
    t0 = time.perf_counter()
    r = ob.bead_system(x, q, st["types"], [b.beads], cfg.box)
    t1 = time.perf_counter()
    per_eval = t1 - t0
    steps = max(1, int(target_s / max(per_eval, 1e-3)))
    t0 = time.perf_counter()
    ob.nve(x, P, q, L, st["types"], [b.beads], [b.mass], [b.inertia], cfg.box, steps, cfg.dt)
    wall = time.perf_counter() - t0
    pairs = r["n_pairs"] * (steps + 1)
    return dict(value=pairs / wall, unit="rigid-pair F+tau evals/s", cores=ob.num_threads(), kind="oracle",
                sample=f"{steps} NVE steps (+1 initial force evaluation) of the same 4096-cube system, "
                       f"{r['n_pairs']} pairs per evaluation, FP64 C oracle, wall {wall:.1f} s",
                md_steps_per_s=(steps + 1) / wall)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-nn", action="store_true", help="skip the network measurements")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the cylinder and half-power half-cosine surrogates and their network-vs-bead "
                         "dynamics")
    ap.add_argument("--cyl-epochs", type=int, default=100, help="cylinder surrogate epochs (2^21 pairs each)")
    ap.add_argument("--hphc-epochs", type=int, default=300,
                    help="half-power half-cosine cube surrogate epochs (2^20 pairs each)")
    ap.add_argument("--nn-steps", type=int, default=100,
                    help="timed steps of the network path (its trajectory stays sound for a limited time)")
    ap.add_argument("--nn-epochs", type=int, default=100, help="surrogate training epochs (2^20 pairs each)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the path is single-GPU; --gpus {args.gpus} is not supported)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2402_12199_amd import abi
    from paper_2402_12199_amd.md import NNModel
    from synth import configs, sampling, state

    cfg = configs.config2()
    log(f"[bench] generating {cfg.name}")
    st = state.initial_state(cfg)
    sysm = make_system(cfg, st, torch)
    sysm.init_forces("bead")
    # one eager step first: its integrator pass yields the kinetic energy, so
    # the total energy is known at the start of the measured trajectory
    sysm.step(cfg.dt, "bead")
    e_start = sysm.energy() + float(sysm.kinetic_host().sum())
    torch.cuda.synchronize()
    log(f"[bench] bead path: {args.warmup} warmup + {args.steps} timed steps")
    bead = run_md(sysm, args.steps, args.warmup, cfg.dt, "bead", torch, abi)
    kin = sysm.kinetic_host()
    e_tot = sysm.energy() + float(kin.sum())
    kern_ms, tests_done = bead_kernel_time(sysm, 20, torch, abi)
    npairs_now = int(sysm.flags_host()[abi.RB_FLAG_NPAIRS])
    tests_brute = npairs_now * cfg.body.n * cfg.body.n
    achieved = tests_done * FLOP_PER_TEST / (kern_ms * 1e-3)
    nsteps = bead["steps"]
    steps_per_s = nsteps / bead["wall_s"]
    value = bead["pairs_evaluated"] / bead["wall_s"]

    result = {
        "metric": "rigid-pair F+tau evals/sec (bead sum FP32, MD step on 4096 cubes); MD steps/sec; "
                  "NN(BF16) vs bead-sum(FP32), 1 GPU",
        "value": value,
        "unit": "rigid-pair F+tau evals/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * bead["wall_s"] / nsteps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random placement, orientations, Maxwell-Boltzmann momenta)",
        "config": {"workload": "cubes4096_phi0.20: 4096 cube shells (152 beads), LJ rc=2.5, NVE dt=0.005, "
                               "kT=1, bead path",
                   "n_bodies": cfg.n_bodies, "beads_per_body": cfg.body.n, "box": cfg.box,
                   "pairs_per_step": npairs_now},
        "md_steps_per_s": steps_per_s,
        "bead_path": {"pairs_evaluated": bead["pairs_evaluated"], "rebuilds": bead["rebuilds"],
                      "gpu_ms_per_step": bead["gpu_ms"] / nsteps, "graph_steps": GRAPH_STEPS,
                      "eager_ms_per_step": bead["eager_ms_per_step"],
                      "total_energy_start": e_start, "total_energy_end": e_tot,
                      "energy_drift_per_body": (e_tot - e_start) / sysm.n,
                      # the first eager step, the warm-up, one untimed graph replay, the
                      # timed steps and the eager steps timed after them
                      "drift_over_steps": 1 + args.warmup + GRAPH_STEPS + nsteps + 5 * GRAPH_STEPS},
        "roofline": {"kernel": "k_bead_md (rb_bead_pair_forces)", "bound": "alu", "achieved": achieved / 1e12,
                     "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
                     "traffic": bead_traffic(), "traffic_unit": "bytes per launch", "kernel_ms": kern_ms,
                     "algorithmic_work": f"{tests_done:.0f} bead-bead distance tests x {FLOP_PER_TEST} FLOP per "
                                         f"launch (the tests that survive exact box culling; the brute-force "
                                         f"double sum would do {npairs_now} pairs x {cfg.body.n}^2 = "
                                         f"{tests_brute} tests)",
                     "brute_force_equivalent_tflops": tests_brute * FLOP_PER_TEST / (kern_ms * 1e-3) / 1e12},
    }

    log("[bench] per-kernel rooflines")
    result["kernels"] = kernel_table(sysm, cfg, torch, abi)

    if not args.no_nn:
        # network path on the same system, with a cube-6 surrogate trained
        # here on pairs visited by the bead dynamics from the same start,
        # labelled by the bead kernel (its held-out errors are reported)
        from paper_2402_12199_amd.surrogate import train_surrogate_md
        log(f"[bench] training a {cfg.body.name} surrogate ({args.nn_epochs} epochs)")
        sur = train_surrogate_md(cfg, st, 1 << 20, 1 << 16, args.nn_epochs, log=log)
        log(f"[bench] surrogate: label {sur['label_s']:.1f} s, train {sur['train_s']:.1f} s, "
            f"held-out E rmse {sur['trained']['rmse_E']:.3f} (std {sur['trained']['std_E']:.3f})")
        summary = {k: sur[k] for k in ("shape", "sampling", "epochs", "steps", "batch", "n_train", "n_test",
                                       "label_s", "train_s", "samples_per_s", "d_min", "d_cut")}
        summary["held_out"] = sur["trained"]
        summary["loss_first_last"] = [sur["loss_history"][0], sur["loss_history"][-1]]
        log("[bench] network path on the same system")
        st2 = state.initial_state(cfg)
        sysn = make_system(cfg, st2, torch)
        sysn.set_nn(NNModel(params=sur["params"], norm=sur["norm"], precision=abi.RB_PREC_BF16,
                            d_min=cfg.d_min, sw_lo=cfg.d_cut - 1.0, sw_hi=cfg.d_cut))
        sysn.init_forces("nn")
        ke0 = float((st2["P"] ** 2).sum() / (2 * cfg.body.mass) + (st2["L"] ** 2 / (2 * cfg.body.inertia)).sum())
        e_nn0 = sysn.energy() + ke0
        nn_steps = min(args.steps, args.nn_steps)
        nn_warm = min(args.warmup, 20)
        try:
            nnr = run_md(sysn, nn_steps, nn_warm, cfg.dt, "nn", torch, abi)
        except RuntimeError as e:       # a surrogate that lets bodies overlap
            result["nn_path"] = {"error": str(e), "surrogate": summary}
        else:
            kin_n = sysn.kinetic_host()
            e_end = sysn.energy() + float(kin_n.sum())
            # how long the surrogate trajectory stays sound: continue eagerly
            # to the bead run's length, checking the routing and the finite flag
            done = nn_warm + nnr["steps"] + GRAPH_STEPS * 6
            horizon, first_fallback = None, None
            while done < args.warmup + args.steps:
                for _ in range(50):
                    sysn.step(cfg.dt, "nn")
                done += 50
                f = sysn.flags_host()
                if first_fallback is None and f[abi.RB_FLAG_NBEAD] > 0:
                    first_fallback = done
                if f[abi.RB_FLAG_NONFINITE]:
                    horizon = done
                    break
            result["nn_path"] = {
                "pairs_per_s": nnr["pairs_evaluated"] / nnr["wall_s"],
                "md_steps_per_s": nnr["steps"] / nnr["wall_s"],
                "ms_per_step": 1e3 * nnr["wall_s"] / nnr["steps"],
                "timed_steps": nnr["steps"], "warmup": nn_warm,
                "eager_ms_per_step": nnr["eager_ms_per_step"],
                "pairs_nn": nnr["n_nn"], "pairs_bead_fallback": nnr["n_bead"],
                "speedup_steps_vs_bead": (nnr["steps"] / nnr["wall_s"]) / steps_per_s,
                "speedup_pairs_vs_bead": (nnr["pairs_evaluated"] / nnr["wall_s"]) / value,
                "total_energy_start_end_of_timed": [e_nn0, e_end],
                "first_bead_fallback_step": first_fallback,
                "nonfinite_at_step": horizon,
                "steps_checked": done,
                "surrogate": summary,
            }
        log("[bench] network kernels on 2^20 pairs")
        result["nn_kernels_2^20"] = nn_kernels(torch, abi)

    if not args.no_learned:
        result["cylinders"] = learned_part(args, torch, abi, log)
        result["hphc_cubes"] = hphc_part(args, torch, abi, log)

    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(cfg, st)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
