"""Thin Python binding of the C ABI in include/rigidnn.h.

Every function has the C entry point's name and only marshals arguments:
it checks tensor device, dtype, shape and contiguity, passes device
pointers and the current HIP stream, and raises on a non-zero status.  All
arithmetic runs in the HIP kernels.  torch tensors are used for device
memory and streams only.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from ._lib import check, lib

RB_FLAG_REBUILD, RB_FLAG_NPAIRS, RB_FLAG_OVERFLOW, RB_FLAG_NREBUILDS = 0, 1, 2, 3
RB_FLAG_NBEAD, RB_FLAG_NNN, RB_FLAG_NONFINITE, RB_FLAG_NEVAL, RB_FLAG_NTESTS, RB_NFLAGS = 4, 5, 6, 7, 8, 24
RB_FLAG_NSCREEN, RB_FLAG_RESCREEN, RB_FLAG_NRESCREENS = 10, 11, 12
RB_FLAG_FIXOVF, RB_FLAG_QDRIFT, RB_FLAG_ROUTE_WORK, RB_FLAG_WAIT_TIMEOUT, RB_FLAG_FB_WORK = 13, 14, 16, 19, 20
RB_OK, RB_ERR_INVALID_ARG, RB_ERR_CAPACITY, RB_ERR_HIP, RB_ERR_UNSUPPORTED, RB_ERR_NONFINITE = 0, -1, -2, -3, -4, -5
RB_PREC_BF16, RB_PREC_FP32 = 0, 1
RB_BUILD_ALWAYS, RB_BUILD_IF_FLAGGED = 0, 1
RB_MLP_NPARAMS = 50689
RB_ACC_SCALE = 4294967296.0


RB_ACC_SLOTS = 64


def acc_len(n: int) -> int:
    return 6 * n + 10 * RB_ACC_SLOTS


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor", optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _box(box):
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    return b, b.ctypes.data_as(C.POINTER(C.c_double))


def _norm(norm):
    a = np.ascontiguousarray(np.asarray(norm, dtype=np.float32).reshape(16))
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


class Ctx:
    """Owner of an rb_ctx (bead templates, potential, per-type mass/inertia)."""

    def __init__(self, templates, masses, inertias, eps=1.0, sigma=1.0, rc=2.5):
        nb = np.array([len(t) for t in templates], dtype=np.int32)
        beads = np.ascontiguousarray(np.concatenate([np.asarray(t, np.float32) for t in templates]))
        m = np.ascontiguousarray(np.asarray(masses, np.float64))
        inert = np.ascontiguousarray(np.asarray(inertias, np.float64).reshape(-1))
        h = C.c_void_p()
        check(lib().rb_ctx_create(C.byref(h), len(templates), nb.ctypes.data_as(C.POINTER(C.c_int32)),
                                  beads.ctypes.data_as(C.POINTER(C.c_float)),
                                  m.ctypes.data_as(C.POINTER(C.c_double)),
                                  inert.ctypes.data_as(C.POINTER(C.c_double)), eps, sigma, rc),
              "rb_ctx_create")
        self.handle = h
        self.n_beads = nb

    def set_hphc(self, A, b, c, p):
        """Half-power half-cosine bead potential (rb_ctx_set_hphc)."""
        check(lib().rb_ctx_set_hphc(self.handle, float(A), float(b), float(c), float(p)), "rb_ctx_set_hphc")
        self.rc = float(b) + math.pi / float(c)

    def close(self):
        if self.handle:
            lib().rb_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rb_ctx_create(templates, masses, inertias, eps=1.0, sigma=1.0, rc=2.5) -> Ctx:
    return Ctx(templates, masses, inertias, eps, sigma, rc)


def rb_pairlist_workspace_bytes(n: int, box, r_list: float) -> int:
    _, bp = _box(box)
    return int(lib().rb_pairlist_workspace_bytes(n, bp, r_list))


def rb_pairlist_build(x, box, r_list, pair_i, pair_j, x_ref, flags, mode, ws):
    n = x.shape[1]
    _, bp = _box(box)
    check(lib().rb_pairlist_build(n, _ptr(x, torch.float64, (3, n), "x"), bp, float(r_list),
                                  _ptr(pair_i, torch.int32, name="pair_i"),
                                  _ptr(pair_j, torch.int32, name="pair_j"), pair_i.numel(),
                                  _ptr(x_ref, torch.float64, (3, n), "x_ref", optional=True),
                                  _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), mode,
                                  _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()),
          "rb_pairlist_build")


def rb_pair_descriptors(x, q, box, pair_i, pair_j, d_min, desc, idx_nn, idx_bead, flags, d_max=0.0, ctx=None,
                        types=None, gap_min=0.0, gap_max=0.0):
    """ctx (Ctx) and types (n int32) switch on the routing by the shells'
    lower bound on the closest bead distance (gap_min, gap_max)."""
    n = x.shape[1]
    maxp = pair_i.numel()
    _, bp = _box(box)
    if (ctx is None) != (types is None):
        raise ValueError("ctx and types go together")
    check(lib().rb_pair_descriptors(n, _ptr(x, torch.float64, (3, n), "x"),
                                    _ptr(q, torch.float64, (4, n), "q"), bp,
                                    _ptr(pair_i, torch.int32, name="pair_i"),
                                    _ptr(pair_j, torch.int32, name="pair_j"), maxp, float(d_min), float(d_max),
                                    _ptr(desc, torch.float32, (7, maxp), "desc"),
                                    _ptr(idx_nn, torch.int32, (maxp,), "idx_nn"),
                                    _ptr(idx_bead, torch.int32, (maxp,), "idx_bead"),
                                    _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"),
                                    None if ctx is None else ctx.handle,
                                    _ptr(types, torch.int32, (n,), "types", optional=True), float(gap_min),
                                    float(gap_max), _stream()),
          "rb_pair_descriptors")


def rb_pair_descriptors_screened(x, q, box, pair_i, pair_j, d_min, desc, idx_nn, idx_bead, flags, d_max, ctx,
                                 types, gap_min, gap_max, margin, cand_list, x_sref, q_sref):
    """Two-level routing: the full routing (and a new candidate list) when
    flags[RESCREEN] is set, the candidates only otherwise."""
    n = x.shape[1]
    maxp = pair_i.numel()
    _, bp = _box(box)
    check(lib().rb_pair_descriptors_screened(n, _ptr(x, torch.float64, (3, n), "x"),
                                             _ptr(q, torch.float64, (4, n), "q"), bp,
                                             _ptr(pair_i, torch.int32, name="pair_i"),
                                             _ptr(pair_j, torch.int32, name="pair_j"), maxp, float(d_min),
                                             float(d_max), _ptr(desc, torch.float32, (7, maxp), "desc"),
                                             _ptr(idx_nn, torch.int32, (maxp,), "idx_nn"),
                                             _ptr(idx_bead, torch.int32, (maxp,), "idx_bead"),
                                             _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), ctx.handle,
                                             _ptr(types, torch.int32, (n,), "types"), float(gap_min),
                                             float(gap_max), float(margin),
                                             _ptr(cand_list, torch.int32, (maxp,), "cand_list"),
                                             _ptr(x_sref, torch.float64, (3, n), "x_sref"),
                                             _ptr(q_sref, torch.float64, (4, n), "q_sref"), _stream()),
          "rb_pair_descriptors_screened")


def rb_bead_pair_eval(ctx: Ctx, desc, type_i: int, type_j: int, out, flags=None):
    P = desc.shape[1]
    check(lib().rb_bead_pair_eval(ctx.handle, P, _ptr(desc, torch.float32, (7, P), "desc"), type_i, type_j,
                                  _ptr(out, torch.float32, (11, P), "out"),
                                  _ptr(flags, torch.int32, (RB_NFLAGS,), "flags", optional=True), _stream()),
          "rb_bead_pair_eval")


def rb_bead_pair_forces(ctx: Ctx, x, q, types, box, pair_i, pair_j, idx, count_dev, max_count, acc, flags):
    n = x.shape[1]
    _, bp = _box(box)
    check(lib().rb_bead_pair_forces(ctx.handle, n, _ptr(x, torch.float64, (3, n), "x"),
                                    _ptr(q, torch.float64, (4, n), "q"), _ptr(types, torch.int32, (n,), "type"),
                                    bp, _ptr(pair_i, torch.int32, name="pair_i"),
                                    _ptr(pair_j, torch.int32, name="pair_j"),
                                    _ptr(idx, torch.int32, name="idx", optional=True),
                                    _ptr(count_dev, torch.int32, name="count_dev"), int(max_count),
                                    _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                    _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_bead_pair_forces")


def rb_bead_pair_forces_screened(ctx: Ctx, x, q, types, box, pair_i, pair_j, count_dev, max_count, margin,
                                 screen_list, x_sref, q_sref, tmp, acc, flags):
    n = x.shape[1]
    _, bp = _box(box)
    if screen_list.numel() < max_count:
        raise ValueError("screen_list must hold max_count entries")
    check(lib().rb_bead_pair_forces_screened(ctx.handle, n, _ptr(x, torch.float64, (3, n), "x"),
                                             _ptr(q, torch.float64, (4, n), "q"),
                                             _ptr(types, torch.int32, (n,), "type"), bp,
                                             _ptr(pair_i, torch.int32, name="pair_i"),
                                             _ptr(pair_j, torch.int32, name="pair_j"),
                                             _ptr(count_dev, torch.int32, name="count_dev"), int(max_count),
                                             float(margin), _ptr(screen_list, torch.int32, name="screen_list"),
                                             _ptr(x_sref, torch.float64, (3, n), "x_sref"),
                                             _ptr(q_sref, torch.float64, (4, n), "q_sref"),
                                             _ptr(tmp, torch.int32, (4,), "tmp"),
                                             _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                             _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_bead_pair_forces_screened")


def rb_bead_screen(ctx: Ctx, x, q, types, box, pair_i, pair_j, idx, count_dev, max_count, idx_out, count_out, tmp,
                   flags=None):
    n = x.shape[1]
    _, bp = _box(box)
    check(lib().rb_bead_screen(ctx.handle, n, _ptr(x, torch.float64, (3, n), "x"),
                               _ptr(q, torch.float64, (4, n), "q"), _ptr(types, torch.int32, (n,), "type"),
                               bp, _ptr(pair_i, torch.int32, name="pair_i"),
                               _ptr(pair_j, torch.int32, name="pair_j"),
                               _ptr(idx, torch.int32, name="idx", optional=True),
                               _ptr(count_dev, torch.int32, name="count_dev"), int(max_count),
                               _ptr(idx_out, torch.int32, name="idx_out"),
                               _ptr(count_out, torch.int32, name="count_out"),
                               _ptr(tmp, torch.int32, (2,), "tmp"),
                               _ptr(flags, torch.int32, (RB_NFLAGS,), "flags", optional=True), _stream()),
          "rb_bead_screen")


def rb_accum_zero(n: int, acc):
    check(lib().rb_accum_zero(n, _ptr(acc, torch.int64, (acc_len(n),), "acc"), _stream()), "rb_accum_zero")


def rb_accum_finalize(n: int, acc, force, torque, energy_virial=None, flags=None):
    check(lib().rb_accum_finalize(n, _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                  _ptr(force, torch.float32, (3, n), "force"),
                                  _ptr(torque, torch.float32, (3, n), "torque"),
                                  _ptr(energy_virial, torch.float64, (10,), "energy_virial", optional=True),
                                  _ptr(flags, torch.int32, (RB_NFLAGS,), "flags", optional=True),
                                  _stream()),
          "rb_accum_finalize")


def rb_flags_check(flags_host) -> tuple[int, str]:
    """Status of a host copy of the flag array (RB_OK, RB_ERR_CAPACITY or
    RB_ERR_NONFINITE) and the library's message for it."""
    f = np.ascontiguousarray(np.asarray(flags_host, dtype=np.int32).reshape(RB_NFLAGS))
    rc = lib().rb_flags_check(f.ctypes.data_as(C.POINTER(C.c_int32)))
    return int(rc), (lib().rb_last_error().decode(errors="replace") if rc else "")


def rb_nn_pair_eval(params, norm, precision: int, desc, energy):
    P = desc.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_pair_eval(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn, precision, P,
                                _ptr(desc, torch.float32, (7, P), "desc"),
                                _ptr(energy, torch.float32, (P,), "energy"), _stream()),
          "rb_nn_pair_eval")


def rb_nn_pair_grad(params, norm, precision: int, desc, gE=None, energy=None, dE_ddesc=None, pair_ft=None):
    P = desc.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_pair_grad(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn, precision, P,
                                _ptr(desc, torch.float32, (7, P), "desc"),
                                _ptr(gE, torch.float32, (P,), "gE", optional=True),
                                _ptr(energy, torch.float32, (P,), "energy", optional=True),
                                _ptr(dE_ddesc, torch.float32, (7, P), "dE_ddesc", optional=True),
                                _ptr(pair_ft, torch.float32, (9, P), "pair_ft", optional=True), _stream()),
          "rb_nn_pair_grad")


def rb_nn_pair_forces(params, norm, precision, q, pair_i, pair_j, desc, idx, count_dev, max_count,
                      sw_lo, sw_hi, acc, flags):
    n = q.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_pair_forces(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn, precision, n,
                                  _ptr(q, torch.float64, (4, n), "q"),
                                  _ptr(pair_i, torch.int32, name="pair_i"),
                                  _ptr(pair_j, torch.int32, name="pair_j"),
                                  _ptr(desc, torch.float32, name="desc"), desc.shape[1],
                                  _ptr(idx, torch.int32, name="idx", optional=True),
                                  _ptr(count_dev, torch.int32, name="count_dev"), int(max_count),
                                  float(sw_lo), float(sw_hi), _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                  _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_nn_pair_forces")


def _sym_descriptors(fn, name, desc, sym, jac, idx, count_dev, max_count):
    stride = desc.shape[1]
    m = int(max_count if count_dev is not None else stride)
    if sym.shape != (7, m) or jac.shape != (49, m):
        raise ValueError(f"sym must be (7, {m}) and jac (49, {m})")
    check(fn(stride if count_dev is None else 0, _ptr(desc, torch.float32, name="desc"), stride,
             _ptr(idx, torch.int32, name="idx", optional=True),
             _ptr(count_dev, torch.int32, name="count_dev", optional=True), m,
             _ptr(sym, torch.float32, (7, m), "sym"), _ptr(jac, torch.float32, (49, m), "jac"), _stream()), name)


def rb_cube_sym_descriptors(desc, sym, jac, idx=None, count_dev=None, max_count=None):
    """Symmetry-reduced cube-pair descriptors of desc's pairs (all of them,
    or idx[0 .. *count_dev) compacted to rows 0 .. count with row stride
    max_count)."""
    _sym_descriptors(lib().rb_cube_sym_descriptors, "rb_cube_sym_descriptors", desc, sym, jac, idx, count_dev,
                     max_count)


def rb_cyl_sym_descriptors(desc, sym, jac, idx=None, count_dev=None, max_count=None):
    """Four-number cylinder-pair descriptors of desc's pairs, laid out as
    rb_cube_sym_descriptors."""
    _sym_descriptors(lib().rb_cyl_sym_descriptors, "rb_cyl_sym_descriptors", desc, sym, jac, idx, count_dev,
                     max_count)


def rb_nn_pair_forces_cyl(params, norm, precision, q, pair_i, pair_j, desc, idx, count_dev, max_count,
                          sw_lo, sw_hi, acc, flags):
    n = q.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_pair_forces_cyl(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn, precision, n,
                                      _ptr(q, torch.float64, (4, n), "q"),
                                      _ptr(pair_i, torch.int32, name="pair_i"),
                                      _ptr(pair_j, torch.int32, name="pair_j"),
                                      _ptr(desc, torch.float32, name="desc"), desc.shape[1],
                                      _ptr(idx, torch.int32, name="idx", optional=True),
                                      _ptr(count_dev, torch.int32, name="count_dev"), int(max_count),
                                      float(sw_lo), float(sw_hi), _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                      _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_nn_pair_forces_cyl")


def rb_nn_pair_forces_routed(ctx: Ctx, params, norm, precision, form: int, x, q, types, box, pair_i, pair_j, desc,
                             idx_nn, nn_count_dev, idx_bead, bead_count_dev, max_count, sw_lo, sw_hi, acc, flags):
    n = q.shape[1]
    _, npn = _norm(norm)
    boxa, bp = _box(box)
    check(lib().rb_nn_pair_forces_routed(ctx.handle, _ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn,
                                         precision, int(form), n, _ptr(x, torch.float64, (3, n), "x"),
                                         _ptr(q, torch.float64, (4, n), "q"), _ptr(types, torch.int32, (n,), "type"),
                                         bp,
                                         _ptr(pair_i, torch.int32, name="pair_i"),
                                         _ptr(pair_j, torch.int32, name="pair_j"),
                                         _ptr(desc, torch.float32, name="desc"), desc.shape[1],
                                         _ptr(idx_nn, torch.int32, name="idx_nn"),
                                         _ptr(nn_count_dev, torch.int32, name="nn_count_dev"),
                                         _ptr(idx_bead, torch.int32, name="idx_bead"),
                                         _ptr(bead_count_dev, torch.int32, name="bead_count_dev"), int(max_count),
                                         float(sw_lo), float(sw_hi), _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                         _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_nn_pair_forces_routed")


def rb_nn_pair_grad_sym(params, norm, precision: int, desc, sym, jac, gE=None, energy=None, dE_ddesc=None,
                        pair_ft=None):
    P = desc.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_pair_grad_sym(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn, precision, P,
                                    _ptr(desc, torch.float32, (7, P), "desc"), _ptr(sym, torch.float32, (7, P), "sym"),
                                    _ptr(jac, torch.float32, (49, P), "jac"),
                                    _ptr(gE, torch.float32, (P,), "gE", optional=True),
                                    _ptr(energy, torch.float32, (P,), "energy", optional=True),
                                    _ptr(dE_ddesc, torch.float32, (7, P), "dE_ddesc", optional=True),
                                    _ptr(pair_ft, torch.float32, (9, P), "pair_ft", optional=True), _stream()),
          "rb_nn_pair_grad_sym")


def rb_nn_pair_forces_sym(params, norm, precision, q, pair_i, pair_j, desc, sym, jac, idx, count_dev, max_count,
                          sw_lo, sw_hi, acc, flags):
    n = q.shape[1]
    _, npn = _norm(norm)
    m = int(max_count)
    check(lib().rb_nn_pair_forces_sym(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"), npn, precision, n,
                                      _ptr(q, torch.float64, (4, n), "q"),
                                      _ptr(pair_i, torch.int32, name="pair_i"),
                                      _ptr(pair_j, torch.int32, name="pair_j"),
                                      _ptr(desc, torch.float32, name="desc"), desc.shape[1],
                                      _ptr(sym, torch.float32, (7, m), "sym"), _ptr(jac, torch.float32, (49, m), "jac"),
                                      _ptr(idx, torch.int32, name="idx", optional=True),
                                      _ptr(count_dev, torch.int32, name="count_dev"), m,
                                      float(sw_lo), float(sw_hi), _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                      _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_nn_pair_forces_sym")


def rb_rigid_workspace_bytes(n: int) -> int:
    return int(lib().rb_rigid_workspace_bytes(n))


def rb_rigid_step(ctx: Ctx, phase: int, dt: float, x, P, q, L, types, force, torque, x_ref=None,
                  half_skin=0.0, kinetic=None, flags=None, ws=None, x_sref=None, q_sref=None, half_margin=0.0,
                  nh=None):
    n = P.shape[1]
    check(lib().rb_rigid_step(ctx.handle, phase, n, float(dt),
                              _ptr(x, torch.float64, (3, n), "x", optional=True),
                              _ptr(P, torch.float64, (3, n), "P"), _ptr(q, torch.float64, (4, n), "q"),
                              _ptr(L, torch.float64, (3, n), "L"), _ptr(types, torch.int32, (n,), "type"),
                              _ptr(force, torch.float32, (3, n), "force"),
                              _ptr(torque, torch.float32, (3, n), "torque"),
                              _ptr(x_ref, torch.float64, (3, n), "x_ref", optional=True), float(half_skin),
                              _ptr(x_sref, torch.float64, (3, n), "x_sref", optional=True),
                              _ptr(q_sref, torch.float64, (4, n), "q_sref", optional=True), float(half_margin),
                              _ptr(kinetic, torch.float64, (2,), "kinetic", optional=True),
                              _ptr(nh, torch.float64, (5,), "nh", optional=True),
                              _ptr(flags, torch.int32, (RB_NFLAGS,), "flags", optional=True),
                              _ptr(ws, torch.uint8, name="ws", optional=True), 0 if ws is None else ws.numel(),
                              _stream()),
          "rb_rigid_step")


def rb_rigid_step_fused(ctx: Ctx, dt: float, x, P, q, L, types, acc, force, torque, energy_virial, x_ref,
                        half_skin, kinetic, flags, ws, x_sref=None, q_sref=None, half_margin=0.0):
    n = P.shape[1]
    check(lib().rb_rigid_step_fused(ctx.handle, n, float(dt), _ptr(x, torch.float64, (3, n), "x"),
                                    _ptr(P, torch.float64, (3, n), "P"), _ptr(q, torch.float64, (4, n), "q"),
                                    _ptr(L, torch.float64, (3, n), "L"), _ptr(types, torch.int32, (n,), "type"),
                                    _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                    _ptr(force, torch.float32, (3, n), "force"),
                                    _ptr(torque, torch.float32, (3, n), "torque"),
                                    _ptr(energy_virial, torch.float64, (10,), "energy_virial", optional=True),
                                    _ptr(x_ref, torch.float64, (3, n), "x_ref", optional=True), float(half_skin),
                                    _ptr(x_sref, torch.float64, (3, n), "x_sref", optional=True),
                                    _ptr(q_sref, torch.float64, (4, n), "q_sref", optional=True), float(half_margin),
                                    _ptr(kinetic, torch.float64, (2,), "kinetic", optional=True),
                                    _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"),
                                    _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()),
          "rb_rigid_step_fused")


def rb_rigid_step_fused_noalloc(ctx: Ctx, dt: float, x, P, q, L, types, acc, force, torque, energy_virial, x_ref,
                                half_skin, kinetic, flags, x_sref=None, q_sref=None, half_margin=0.0):
    n = P.shape[1]
    check(lib().rb_rigid_step_fused_noalloc(ctx.handle, n, float(dt), _ptr(x, torch.float64, (3, n), "x"),
                                            _ptr(P, torch.float64, (3, n), "P"),
                                            _ptr(q, torch.float64, (4, n), "q"),
                                            _ptr(L, torch.float64, (3, n), "L"),
                                            _ptr(types, torch.int32, (n,), "type"),
                                            _ptr(acc, torch.int64, (acc_len(n),), "acc"),
                                            _ptr(force, torch.float32, (3, n), "force"),
                                            _ptr(torque, torch.float32, (3, n), "torque"),
                                            _ptr(energy_virial, torch.float64, (10,), "energy_virial",
                                                 optional=True),
                                            _ptr(x_ref, torch.float64, (3, n), "x_ref", optional=True),
                                            float(half_skin),
                                            _ptr(x_sref, torch.float64, (3, n), "x_sref", optional=True),
                                            _ptr(q_sref, torch.float64, (4, n), "q_sref", optional=True),
                                            float(half_margin),
                                            _ptr(kinetic, torch.float64, (2,), "kinetic", optional=True),
                                            _ptr(flags, torch.int32, (RB_NFLAGS,), "flags"), _stream()),
          "rb_rigid_step_fused_noalloc")


def rb_rigid_step_fused_noalloc_max_bodies() -> int:
    return int(lib().rb_rigid_step_fused_noalloc_max_bodies())


def rb_nn_train_step_fm(params, adam_m, adam_v, t: int, norm, precision: int, batch: int, desc, labels, ft_labels,
                        idx, lam_f, lam_t, lr, beta1, beta2, eps, loss, grad_out=None, ws=None):
    nd = desc.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_train_step_fm(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"),
                                    _ptr(adam_m, torch.float32, (RB_MLP_NPARAMS,), "adam_m"),
                                    _ptr(adam_v, torch.float32, (RB_MLP_NPARAMS,), "adam_v"), int(t), npn,
                                    precision, int(batch), _ptr(desc, torch.float32, (7, nd), "desc"), nd,
                                    _ptr(labels, torch.float32, (nd,), "labels"),
                                    _ptr(ft_labels, torch.float32, (6, nd), "ft_labels"),
                                    _ptr(idx, torch.int32, name="idx"), float(lam_f), float(lam_t), float(lr), float(beta1), float(beta2), float(eps),
                                    _ptr(loss, torch.float32, (2,), "loss"),
                                    _ptr(grad_out, torch.float32, (RB_MLP_NPARAMS,), "grad_out", optional=True),
                                    _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()),
          "rb_nn_train_step_fm")


def rb_nn_train_fm_workspace_bytes(batch: int) -> int:
    return int(lib().rb_nn_train_fm_workspace_bytes(batch))


def rb_nn_train_workspace_bytes(batch: int) -> int:
    return int(lib().rb_nn_train_workspace_bytes(batch))


def rb_nn_train_step(params, adam_m, adam_v, t: int, norm, precision: int, batch: int, desc, labels, idx,
                     lr, beta1, beta2, eps, loss, grad_out=None, ws=None):
    nd = desc.shape[1]
    _, npn = _norm(norm)
    check(lib().rb_nn_train_step(_ptr(params, torch.float32, (RB_MLP_NPARAMS,), "params"),
                                 _ptr(adam_m, torch.float32, (RB_MLP_NPARAMS,), "adam_m"),
                                 _ptr(adam_v, torch.float32, (RB_MLP_NPARAMS,), "adam_v"), int(t), npn,
                                 precision, int(batch), _ptr(desc, torch.float32, (7, nd), "desc"), nd,
                                 _ptr(labels, torch.float32, (nd,), "labels"),
                                 _ptr(idx, torch.int32, name="idx"), float(lr), float(beta1), float(beta2),
                                 float(eps), _ptr(loss, torch.float32, name="loss"),
                                 _ptr(grad_out, torch.float32, (RB_MLP_NPARAMS,), "grad_out", optional=True),
                                 _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()),
          "rb_nn_train_step")
