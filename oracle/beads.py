"""ORACLE (test infrastructure only): ctypes front end of oracle/bead.c.

Functions follow the paper's statement of the composite-bead method
(section 2, first equation: the body-body energy is the double sum of the
bead potential over the beads of the two bodies) with the bead potential of
the workloads (Lennard-Jones 12-6, energy-shifted at r_c), and the
rigid-body velocity Verlet of Miller et al. (J. Chem. Phys. 116, 8649, 2002)
for the time integration (the paper states only dt = 0.005 tau, section 3).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        L.oracle_num_threads.restype = C.c_int
        L.oracle_lj.restype = C.c_double
        L.oracle_lj.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.oracle_hphc.restype = C.c_double
        L.oracle_hphc.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.oracle_set_hphc.restype = None
        L.oracle_set_hphc.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_set_lj.restype = None
        L.oracle_set_lj.argtypes = []
        L.oracle_bead_pair.restype = None
        L.oracle_bead_pair.argtypes = [C.c_int, _D, C.c_int, _D, _D, _D, _D, _D, _D,
                                       C.c_double, C.c_double, C.c_double, _D]
        L.oracle_pairs_within.restype = C.c_long
        L.oracle_pairs_within.argtypes = [C.c_int, _D, _D, C.c_double, C.c_long, _I, _I]
        L.oracle_bead_system.restype = C.c_long
        L.oracle_bead_system.argtypes = [C.c_int, _D, _D, _I, C.c_int, _I, _I, _D, _D,
                                         C.c_double, C.c_double, C.c_double, _D, _D, _D, _D]
        L.oracle_rigid_phase1.restype = None
        L.oracle_rigid_phase1.argtypes = [C.c_int, C.c_double, _D, _D, _D, _D, _D, _D, _D, _D]
        L.oracle_rigid_phase2.restype = C.c_double
        L.oracle_rigid_phase2.argtypes = [C.c_int, C.c_double, _D, _D, _D, _D, _D, _D, _D]
        L.oracle_nve.restype = None
        L.oracle_nve.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D, _D, _D, _I, _D, _D,
                                 C.c_int, _I, _I, _D, _D, C.c_double, C.c_double, C.c_double,
                                 _D, _D]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _i(a: np.ndarray):
    return a.ctypes.data_as(_I)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def lj(r, eps=1.0, sigma=1.0, rc=2.5):
    """Energy-shifted LJ 12-6 and -(du/dr)/r at distance r (scalar)."""
    fr = C.c_double()
    e = lib().oracle_lj(float(r) ** 2, eps, sigma, rc, C.byref(fr))
    return e, fr.value


# Half-power half-cosine parameters of the paper (section 3), epsilon and sigma units.
HPHC_PAPER = dict(A=0.00035, b=1.46375, c=3.3833, p=2.5)


def hphc(r, A, b, c, p):
    """Half-power half-cosine energy and -(du/dr)/r at distance r (scalar)."""
    fr = C.c_double()
    e = lib().oracle_hphc(float(r) ** 2, A, b, c, p, C.byref(fr))
    return e, fr.value


class use_hphc:
    """Context in which every bead sum of the oracle uses the half-power
    half-cosine potential (the Lennard-Jones arguments are then ignored)."""

    def __init__(self, A, b, c, p):
        self.args = (A, b, c, p)

    def __enter__(self):
        lib().oracle_set_hphc(*self.args)
        return self

    def __exit__(self, *exc):
        lib().oracle_set_lj()
        return False


def bead_pair(bi, bj, xi, qi, xj, qj, box=None, eps=1.0, sigma=1.0, rc=2.5) -> dict:
    """Bead double sum between two bodies; all outputs in the lab frame."""
    bi, bj = _f64(bi), _f64(bj)
    xi, qi, xj, qj = _f64(xi), _f64(qi), _f64(xj), _f64(qj)
    boxa = None if box is None else _f64(np.broadcast_to(box, (3,)))
    out = np.zeros(14)
    lib().oracle_bead_pair(len(bi), _d(bi), len(bj), _d(bj), _d(xi), _d(qi), _d(xj), _d(qj),
                           None if boxa is None else _d(boxa), eps, sigma, rc, _d(out))
    return dict(E=out[0], Fi=out[1:4].copy(), Fj=out[4:7].copy(), taui=out[7:10].copy(),
                tauj=out[10:13].copy(), rmin=out[13])


def bead_pair_desc(bi, bj, desc, eps=1.0, sigma=1.0, rc=2.5) -> np.ndarray:
    """Per-pair outputs for pair configurations desc (P,7) = (d, q).

    Body i sits at the origin with identity orientation, body j at d with
    orientation q / |q|.  Returns (P, 11): E, F_j (3), tau_i (3), tau_j (3),
    r_min, all in body i's frame.
    """
    desc = _f64(desc)
    out = np.zeros((len(desc), 11))
    zero = np.zeros(3)
    ident = np.array([1.0, 0.0, 0.0, 0.0])
    for p in range(len(desc)):
        q = desc[p, 3:7] / np.linalg.norm(desc[p, 3:7])
        r = bead_pair(bi, bj, zero, ident, desc[p, :3], q, None, eps, sigma, rc)
        out[p] = np.concatenate([[r["E"]], r["Fj"], r["taui"], r["tauj"], [r["rmin"]]])
    return out


def pairs_within(x, box, r) -> np.ndarray:
    """All pairs i < j with minimum-image centre distance < r, shape (P, 2)."""
    x = _f64(x)
    n = len(x)
    boxa = None if box is None else _f64(np.broadcast_to(box, (3,)))
    cap = max(16, n * 64)
    while True:
        pi = np.zeros(cap, dtype=np.int32)
        pj = np.zeros(cap, dtype=np.int32)
        cnt = lib().oracle_pairs_within(n, _d(x), None if boxa is None else _d(boxa), r, cap,
                                        _i(pi), _i(pj))
        if cnt <= cap:
            return np.stack([pi[:cnt], pj[:cnt]], axis=1)
        cap = int(cnt)


def _types(templates):
    nb = np.array([len(t) for t in templates], dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(nb)[:-1]]).astype(np.int32)
    tmpl = _f64(np.concatenate([np.asarray(t, dtype=np.float64) for t in templates], axis=0))
    return nb, off, tmpl


def bead_system(x, q, types, templates, box, eps=1.0, sigma=1.0, rc=2.5) -> dict:
    """Energy, per-body force/torque and virial of a periodic system."""
    x, q = _f64(x), _f64(q)
    types = np.ascontiguousarray(types, dtype=np.int32)
    nb, off, tmpl = _types(templates)
    boxa = None if box is None else _f64(np.broadcast_to(box, (3,)))
    n = len(x)
    E = np.zeros(1)
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    W = np.zeros(9)
    npairs = lib().oracle_bead_system(n, _d(x), _d(q), _i(types), len(templates), _i(nb), _i(off),
                                      _d(tmpl), None if boxa is None else _d(boxa), eps, sigma, rc,
                                      _d(E), _d(F), _d(T), _d(W))
    return dict(E=E[0], F=F, tau=T, virial=W.reshape(3, 3), n_pairs=int(npairs))


def rigid_phase1(dt, x, P, q, L, mass, inertia, F, tau):
    """In place: half kick, drift, NO_SQUISH free rotation, renormalise."""
    n = len(x)
    for a in (x, P, q, L):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    m = _f64(np.broadcast_to(mass, (n,)))
    I = _f64(np.broadcast_to(inertia, (n, 3)))
    lib().oracle_rigid_phase1(n, dt, _d(x), _d(P), _d(q), _d(L), _d(m), _d(I), _d(_f64(F)),
                              _d(_f64(tau)))


def rigid_phase2(dt, P, q, L, mass, inertia, F, tau) -> float:
    """In place: second half kick; returns the kinetic energy."""
    n = len(P)
    for a in (P, q, L):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    m = _f64(np.broadcast_to(mass, (n,)))
    I = _f64(np.broadcast_to(inertia, (n, 3)))
    return float(lib().oracle_rigid_phase2(n, dt, _d(P), _d(q), _d(L), _d(m), _d(I),
                                           _d(_f64(F)), _d(_f64(tau))))


def nve(x, P, q, L, types, templates, masses, inertias, box, steps, dt,
        eps=1.0, sigma=1.0, rc=2.5) -> dict:
    """NVE run; state arrays are advanced in place.  Returns pe, ke series."""
    for a in (x, P, q, L):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    types = np.ascontiguousarray(types, dtype=np.int32)
    nb, off, tmpl = _types(templates)
    m = _f64(masses)
    I = _f64(inertias).reshape(-1)
    boxa = None if box is None else _f64(np.broadcast_to(box, (3,)))
    pe = np.zeros(steps + 1)
    ke = np.zeros(steps + 1)
    lib().oracle_nve(len(x), steps, dt, _d(x), _d(P), _d(q), _d(L), _i(types), _d(m), _d(I),
                     len(templates), _i(nb), _i(off), _d(tmpl),
                     None if boxa is None else _d(boxa), eps, sigma, rc, _d(pe), _d(ke))
    return dict(pe=pe, ke=ke)
