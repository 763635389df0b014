"""Network-accelerated dynamics against the plain bead path from the same
start (paper section 3: the trajectories are compared through g(r), the
orientational order, the mean-squared displacement and energy conservation,
and the two paths' time steps per second are reported).

Each path runs in chunks: an eager first half step, HIP-graph replays of
fused steps (timed with events), and an eager closing step, after which the
state is copied out for the observables.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import abi, analysis
from .md import NNModel, RigidSystem

GRAPH_STEPS = 10


def run_dynamics(cfg, st, path: str, nn: NNModel | None = None, chunks: int = 8, replays: int = 25,
                 log=None, nvt: dict | None = None) -> dict:
    """chunks x (replays x GRAPH_STEPS + 1) steps of NVE (or of Nose-Hoover
    NVT with nvt = dict(kT, tau), through graphs of plain steps); stops early
    when a force or energy turns non-finite."""
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], st["P"], st["L"], cfg.box,
                       cfg.r_list, cfg.skin, hphc=cfg.hphc, margin=cfg.bead_margin if path == "bead" else None,
                       nvt=nvt)
    if nn is not None:
        sysm.set_nn(nn)
    sysm.init_forces(path)
    ke0 = float((st["P"] ** 2).sum() / (2 * b.mass) + (st["L"] ** 2 / (2 * b.inertia)).sum())
    e0 = sysm.energy() + ke0
    x0, q0 = st["x"].copy(), st["q"].copy()
    stream = torch.cuda.current_stream()
    snaps, energies, times, steps_done, graph = [], [e0], [], 0, None
    f_prev = sysm.flags_host()
    eval0 = int(f_prev[abi.RB_FLAG_NEVAL])
    timed_steps, fallback_max, error, first = 0, 0, None, None
    for c in range(chunks):
        if nvt is None:
            sysm.begin_fused(cfg.dt)
        if graph is None:
            graph = sysm.capture(cfg.dt, path, GRAPH_STEPS, fused=nvt is None)
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(replays):
            graph.replay()
        e.record(stream)
        if nvt is None:
            sysm.end_fused(cfg.dt, path)
        else:
            sysm.step(cfg.dt, path)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(e))
        timed_steps += replays * GRAPH_STEPS
        steps_done += replays * GRAPH_STEPS + 1
        f = sysm.flags_host()
        fallback_max = max(fallback_max, int(f[abi.RB_FLAG_NBEAD])) if path == "nn" else 0
        if c == 0:
            # the first chunk alone: the path's speed before a learned
            # trajectory can drift into rebuild-heavy or unphysical states
            first = dict(steps=replays * GRAPH_STEPS, steps_per_s=replays * GRAPH_STEPS / (1e-3 * times[0]),
                         rebuilds=int(f[abi.RB_FLAG_NREBUILDS] - f_prev[abi.RB_FLAG_NREBUILDS]),
                         fallback=fallback_max, finite=abi.rb_flags_check(f)[0] == abi.RB_OK)
        rc, msg = abi.rb_flags_check(f)
        if rc != abi.RB_OK:
            error = msg
            break
        s = sysm.state_host()
        snaps.append((steps_done, s["x"], s["q"]))
        energies.append(sysm.extended_energy())
        if log:
            log(f"[{path}] step {steps_done}: E_total {energies[-1]:.3f}")
    f = sysm.flags_host()
    n_eval = (int(f[abi.RB_FLAG_NEVAL]) - eval0) % (1 << 32)
    gpu_s = 1e-3 * float(np.sum(times))
    temperature = None
    if nvt is not None:
        temperature = 2.0 * float(sysm.kinetic_host().sum()) / (6.0 * sysm.n - 3.0)
    return dict(path=path, temperature_last=temperature, steps=steps_done, timed_steps=timed_steps, timed_gpu_s=gpu_s,
                steps_per_s=timed_steps / gpu_s if gpu_s > 0 else None,
                pair_evals_per_step=n_eval / max(steps_done, 1), energies=energies, x0=x0, q0=q0, snaps=snaps,
                rebuilds=int(f[abi.RB_FLAG_NREBUILDS]), fallback_max=fallback_max, error=error, first_chunk=first)


def observables(cfg, run: dict, rdf_bins: int = 80) -> dict:
    """g(r) of the last snapshot, P2 of the body z axis, MSD and MSR per
    snapshot, energy drift per body."""
    if not run["snaps"]:
        return {}
    steps, x, q = run["snaps"][-1]
    r, g = analysis.rdf(x, cfg.box, min(0.5 * cfg.box, 2.0 * cfg.d_cut), rdf_bins)
    e = np.asarray(run["energies"])
    return dict(step=steps, r=r, g=g, p2=analysis.p2(q, axis=2),
                msd=[(s, analysis.msd(run["x0"], xs)) for s, xs, _ in run["snaps"]],
                msr=[(s, analysis.msr(run["q0"], qs)) for s, _, qs in run["snaps"]],
                drift_per_body=float((e[-1] - e[0]) / cfg.n_bodies),
                max_dev_per_body=float(np.abs(e - e[0]).max() / cfg.n_bodies))


def compare(cfg, st, models: dict, chunks: int = 8, replays: int = 25, log=None, nvt: dict | None = None) -> dict:
    """Bead path and one network path per model (name -> NNModel), all from
    the same start; summary for a report."""
    out = {}
    runs = {"bead": run_dynamics(cfg, st, "bead", None, chunks, replays, log, nvt)}
    for name, nn in models.items():
        runs[name] = run_dynamics(cfg, st, "nn", nn, chunks, replays, log, nvt)
    obs = {p: observables(cfg, runs[p]) for p in runs}
    for p in runs:
        r, o = runs[p], obs[p]
        out[p] = {k: r[k] for k in ("path", "steps", "timed_steps", "steps_per_s", "pair_evals_per_step", "rebuilds",
                                    "fallback_max", "error", "temperature_last", "first_chunk")}
        if o:
            out[p].update(p2=o["p2"], msd_last=o["msd"][-1][1], msr_last=o["msr"][-1][1],
                          drift_per_body=o["drift_per_body"],
                          max_dev_per_body=o["max_dev_per_body"],
                          rdf_peak=[float(o["r"][np.argmax(o["g"])]), float(o["g"].max())])
        if p == "bead" or not o or not obs["bead"]:
            continue
        if obs["bead"]["step"] == o["step"]:
            out[p]["rdf_l1_vs_bead"] = analysis.rdf_distance(obs["bead"]["r"], obs["bead"]["g"], o["g"])
            mb = obs["bead"]["msd"][-1][1]
            out[p]["msd_ratio_vs_bead"] = o["msd"][-1][1] / mb if mb > 0 else None
            rb = obs["bead"]["msr"][-1][1]
            out[p]["msr_ratio_vs_bead"] = o["msr"][-1][1] / rb if rb > 0 else None
        if out["bead"]["steps_per_s"] and out[p]["steps_per_s"]:
            out[p]["speedup_steps_vs_bead"] = out[p]["steps_per_s"] / out["bead"]["steps_per_s"]
        fb, fp = out["bead"].get("first_chunk"), out[p].get("first_chunk")
        if fb and fp:
            out[p]["first_chunk_speedup_vs_bead"] = fp["steps_per_s"] / fb["steps_per_s"]
    return out
