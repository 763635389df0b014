"""Surrogate pair energy: data from the bead path, training, held-out errors.

Paper section 2: the network is trained on pair configurations whose
energies, forces and torques come from the composite-bead method.  Two
sources of configurations: uniform draws (uniform direction, distance
uniform in [d_lo, d_hi], uniform relative orientation), or the pairs that
the bead-path dynamics of a workload visits (as in the paper, whose data
come from composite-body simulations).  They are labelled on the GPU by the
bead kernel (rb_bead_pair_eval); configurations whose closest bead pair is
below r_rej are rejected (deep overlaps, absent from dynamics at the
workloads' temperature).  Training runs rb_nn_train_step (BF16 MFMA, FP32
master weights, Adam) on the energy.  Errors are reported on a held-out set
from another seed: energy, force and torque RMSE, and the fraction of
force components outside a +-10 % band of the bead value (the paper's parity
statistic, section 3).

python -m paper_2402_12199_amd.surrogate --shape cyl134 --epochs 200
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import abi
from .nn import Trainer, label_pairs, make_norm, make_norm_features, make_norm_sym, sym_descriptors


def make_dataset(ctx: abi.Ctx, n: int, seed: int, d_lo: float, d_hi: float, r_rej: float = 0.8,
                 type_i: int = 0, type_j: int = 0):
    """n accepted configurations (desc (n, 7) FP32, labels (n, 11) FP32),
    the rejection rate, and the seconds and count of bead-kernel labelling."""
    from synth import sampling
    g = sampling.rng(seed)
    descs, labs = [], []
    have = drawn = 0
    t_lab = 0.0
    while have < n:
        m = int((n - have) * 1.5) + 1024
        d = sampling.pair_batch(g, m, d_lo, d_hi).astype(np.float32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lab = label_pairs(ctx, d, type_i, type_j)
        t_lab += time.perf_counter() - t0
        keep = lab[:, 10] >= r_rej
        drawn += m
        descs.append(d[keep])
        labs.append(lab[keep])
        have += int(keep.sum())
    desc = np.concatenate(descs)[:n]
    lab = np.concatenate(labs)[:n]
    return desc, lab, 1.0 - have / drawn, t_lab, drawn


def evaluate(params, norm, precision, desc: np.ndarray, lab: np.ndarray, chunk: int = 1 << 18,
             sym: bool = False, form: str | None = None) -> dict:
    """Held-out errors of the network against bead labels (body i frame);
    form: the network's input, "dq" (the pair descriptor), "cube" (the
    symmetry-reduced cube-pair descriptor; sym=True) or "cyl" (the
    four-number cylinder-pair form)."""
    form = form or ("cube" if sym else "dq")
    P = len(desc)
    E = np.empty(P, np.float32)
    ft = np.empty((P, 9), np.float32)
    for s in range(0, P, chunk):
        d = torch.tensor(np.ascontiguousarray(desc[s:s + chunk].T), device="cuda")
        e = torch.empty(d.shape[1], device="cuda")
        f = torch.empty((9, d.shape[1]), device="cuda")
        if form != "dq":
            sy, jc = sym_descriptors(d, form=form)
            abi.rb_nn_pair_grad_sym(params, norm, precision, d, sy, jc, None, e, None, f)
        else:
            abi.rb_nn_pair_grad(params, norm, precision, d, None, e, None, f)
        E[s:s + chunk] = e.cpu().numpy()
        ft[s:s + chunk] = f.cpu().numpy().T
    ref_e, ref_ft = lab[:, 0].astype(np.float64), lab[:, 1:10].astype(np.float64)
    rmse = lambda a, b: float(np.sqrt(np.mean((np.asarray(a, np.float64) - b) ** 2)))
    fx, rfx = ft[:, 0].astype(np.float64), ref_ft[:, 0]
    sig = np.abs(rfx) > 1e-3
    outside = float(np.mean(np.abs(fx[sig] - rfx[sig]) > 0.1 * np.abs(rfx[sig]))) if sig.any() else float("nan")
    return {
        "n": int(P),
        "rmse_E": rmse(E, ref_e), "std_E": float(ref_e.std()),
        "rmse_F": rmse(ft[:, :3], ref_ft[:, :3]), "std_F": float(ref_ft[:, :3].std()),
        "rmse_tau_i": rmse(ft[:, 3:6], ref_ft[:, 3:6]), "std_tau_i": float(ref_ft[:, 3:6].std()),
        "rmse_tau_j": rmse(ft[:, 6:9], ref_ft[:, 6:9]), "std_tau_j": float(ref_ft[:, 6:9].std()),
        "frac_fx_outside_10pct": outside,
    }


def label_set(ctx: abi.Ctx, desc: np.ndarray, r_rej: float = 0.8, type_i: int = 0, type_j: int = 0):
    """Bead labels of given configurations, rejecting r_min < r_rej."""
    lab = label_pairs(ctx, desc.astype(np.float32), type_i, type_j)
    keep = lab[:, 10] >= r_rej
    return desc[keep].astype(np.float32), lab[keep]


def fit(desc: np.ndarray, lab: np.ndarray, tdesc: np.ndarray, tlab: np.ndarray, d_cut: float, epochs: int,
        seed: int, batch: int = 8192, lr: float = 1e-3, precision: int = abi.RB_PREC_BF16, init_seed: int = 1003,
        log=None, name: str = "", fm: dict | None = None, sym: bool = False, form: str | None = None,
        lr_end: float | None = None) -> dict:
    """Train a fresh network (Xavier init) on energies (and, with fm =
    dict(lam_f, lam_t) or dict(weight), on the bead
    forces and torques too; `weight` sets lam_f, lam_t to weight over the
    mean squared label), return it with the held-out errors before and
    after.  lr_end: the learning rate decays from lr to lr_end over the
    epochs (half a cosine period); None keeps lr.  sym: train on the
    symmetry-reduced cube-pair descriptor
    (supplementary section 1; energy loss only)."""
    from synth import sampling
    form = form or ("cube" if sym else "dq")
    if form != "dq" and fm is not None:
        raise ValueError("force matching takes the (d, q) descriptor")
    e = lab[:, 0].astype(np.float64)
    d_dev = torch.tensor(np.ascontiguousarray(desc.T), device="cuda")
    if form == "cyl":
        d_dev = sym_descriptors(d_dev, with_jac=False, form="cyl")[0]
        norm = make_norm_features(d_dev.cpu().numpy().T, float(e.mean()), float(e.std()))
    else:
        norm = (make_norm_sym if form == "cube" else make_norm)(d_cut, float(e.mean()), float(e.std()))
        if form == "cube":
            d_dev = sym_descriptors(d_dev, with_jac=False)[0]
    y_dev = torch.tensor(lab[:, 0].copy(), device="cuda")
    ft_dev = None
    if fm is not None:   # F_j and tau_j columns of the bead labels
        ft = lab[:, [1, 2, 3, 7, 8, 9]].astype(np.float64)
        if "weight" in fm:   # weights from the label spread: each term ~ weight x (relative error)^2
            fm = dict(fm, lam_f=fm["weight"] / max(float((ft[:, :3] ** 2).sum(1).mean()), 1e-30),
                      lam_t=fm["weight"] / max(float((ft[:, 3:] ** 2).sum(1).mean()), 1e-30))
        ft_dev = torch.tensor(np.ascontiguousarray(ft.T.astype(np.float32)), device="cuda")
    tr = Trainer(sampling.xavier_params(init_seed), norm, precision=precision, batch=batch, lr=lr, fm=fm)
    g = sampling.rng(seed + 7)
    before = evaluate(tr.params, norm, precision, tdesc, tlab, form=form)
    hist = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for ep in range(epochs):
        if lr_end is not None:      # cosine decay from lr to lr_end over the epochs
            tr.lr = lr_end + 0.5 * (lr - lr_end) * (1.0 + np.cos(np.pi * ep / max(epochs - 1, 1)))
        hist.append(tr.epoch(d_dev, y_dev, g, ft_dev))
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(f"[surrogate {name}] epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}" +
                (f" matching {tr.fm_loss:.4f}" if fm is not None else ""))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    after = evaluate(tr.params, norm, precision, tdesc, tlab, form=form)
    return dict(shape=name, params=tr.params, norm=norm, precision=precision, d_cut=d_cut, epochs=epochs, fm=fm,
                sym=form == "cube", form=form,
                steps=tr.t, batch=batch, n_train=int(len(desc)), n_test=int(len(tdesc)), train_s=t_train,
                samples_per_s=tr.t * batch / max(t_train, 1e-9), loss_history=hist, untrained=before,
                trained=after)


def train_surrogate(body, n_train: int, n_test: int, epochs: int, seed: int = 1004, test_seed: int = 2004,
                    r_rej: float = 0.8, rc: float = 2.5, sigma: float = 1.0, log=None, **kw) -> dict:
    """Surrogate for pairs of one body type from uniformly drawn
    configurations (distance uniform in [d_min, d_cut], orientation uniform)."""
    t0 = time.perf_counter()
    ctx = abi.Ctx([body.beads], [body.mass], [body.inertia])
    d_min = 2.0 * body.r_in + sigma
    d_cut = 2.0 * body.r_max + rc
    desc, lab, rej, tl1, n1 = make_dataset(ctx, n_train, seed, d_min, d_cut, r_rej)
    tdesc, tlab, _, tl2, n2 = make_dataset(ctx, n_test, test_seed, d_min, d_cut, r_rej)
    t_label = time.perf_counter() - t0
    r = fit(desc, lab, tdesc, tlab, d_cut, epochs, seed, log=log, name=body.name, **kw)
    r.update(sampling="uniform", d_min=d_min, reject_rate=rej, label_s=t_label,
             label_kernel_pairs_per_s=(n1 + n2) / max(tl1 + tl2, 1e-9))
    return r


def md_pair_samples(sysm, dt: float, n: int, every: int, d_min: float, d_max: float, path: str = "bead",
                    gap_min=None, gap_max=None):
    """Pair configurations visited by the dynamics: every `every` steps, the
    descriptors of all listed pairs the router sends to the network
    (d_min <= |d| < d_max; with gap_min, a shells' bound on the closest bead
    distance in [gap_min, gap_max)), until n are collected (the system must
    have current forces)."""
    out, have, steps = [], 0, 0
    while have < n:
        for _ in range(every):
            sysm.step(dt, path)
        steps += every
        d = sysm.pair_configurations(d_min, d_max, gap_min, gap_max).cpu().numpy().T
        out.append(d)
        have += len(d)
    sysm.check_capacity()
    return np.concatenate(out)[:n], steps


def train_surrogate_md(cfg, st, n_train: int, n_test: int, epochs: int, every: int = 10, seed: int = 1006,
                       r_rej: float = 0.8, log=None, gap_min=None, gap_max=None, kTs=None, **kw) -> dict:
    """Surrogate trained on configurations drawn from the bead-path dynamics
    of a workload (paper section 2: training pairs come from composite-body
    simulations).  The held-out set comes from the later part of the same
    trajectory, after the training snapshots.  With gap_min the pairs are
    those the shells' routing gives the network (see rb_pair_descriptors).
    kTs: temperatures of constant-temperature (Nose-Hoover) bead runs that
    share the training set equally, as the paper samples over a range of
    temperatures so that touching and slightly overlapping pairs are covered
    (section 2); the held-out set then comes from the later part of the run
    at kTs[0] (the workload's own temperature, normally).  None: the
    workload's constant-energy run alone."""
    from .md import RigidSystem
    t0 = time.perf_counter()
    b = cfg.body

    def system(kT):
        nvt = None if kT is None else dict(kT=kT, tau=0.5)
        P, L = st["P"], st["L"]
        if kT is not None:      # momenta drawn at cfg.kT, rescaled to kT
            P, L = P * np.sqrt(kT / cfg.kT), L * np.sqrt(kT / cfg.kT)
        s = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"], st["x"], st["q"], P, L, cfg.box, cfg.r_list,
                        cfg.skin, hphc=cfg.hphc, margin=cfg.bead_margin if kT is None else None, nvt=nvt)
        s.init_forces("bead")
        return s

    route = dict(gap_min=gap_min, gap_max=gap_max)
    if kTs is None:
        sysm = system(None)
        desc, s_train = md_pair_samples(sysm, cfg.dt, n_train, every, cfg.d_min, cfg.d_cut, **route)
        tdesc, s_test = md_pair_samples(sysm, cfg.dt, n_test, max(1, every // 2), cfg.d_min, cfg.d_cut, **route)
    else:
        parts, s_train, first = [], 0, None
        for k, kT in enumerate(kTs):
            m = n_train // len(kTs) + (n_train % len(kTs) if k == 0 else 0)
            sk = system(kT)
            first = first or sk
            d, s_k = md_pair_samples(sk, cfg.dt, m, every, cfg.d_min, cfg.d_cut, **route)
            parts.append(d)
            s_train += s_k
            if log:
                log(f"[surrogate {b.name}] {len(d)} pairs from a bead run at kT={kT} ({s_k} steps)")
        desc = np.concatenate(parts)
        # held out: the later part of the first temperature's run
        sysm = first
        tdesc, s_test = md_pair_samples(sysm, cfg.dt, n_test, max(1, every // 2), cfg.d_min, cfg.d_cut, **route)
    desc, lab = label_set(sysm.ctx, desc, r_rej)
    tdesc, tlab = label_set(sysm.ctx, tdesc, r_rej)
    t_label = time.perf_counter() - t0
    r = fit(desc, lab, tdesc, tlab, cfg.d_cut, epochs, seed, log=log, name=b.name, **kw)
    where = "" if kTs is None else f" at kT = {', '.join(str(v) for v in kTs)} (constant temperature)"
    r.update(sampling=f"bead MD of {cfg.name}{where}: {s_train} steps, every {every} (train), then {s_test} steps "
                      f"(held out)", d_min=cfg.d_min, label_s=t_label)
    return r


def main():
    from synth import configs
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", default="cyl134", choices=["cyl134", "cube6", "cube5"])
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--n-train", type=int, default=1 << 21)
    ap.add_argument("--n-test", type=int, default=1 << 16)
    ap.add_argument("--out", default=None, help="write params/norm to this .npz")
    a = ap.parse_args()
    body = getattr(configs, a.shape)()
    r = train_surrogate(body, a.n_train, a.n_test, a.epochs, log=lambda m: print(m, file=sys.stderr, flush=True))
    if a.out:
        np.savez(a.out, params=r["params"].cpu().numpy(), norm=r["norm"], d_min=r["d_min"], d_cut=r["d_cut"])
    r = {k: v for k, v in r.items() if k not in ("params", "norm")}
    print(json.dumps(r))


if __name__ == "__main__":
    main()
