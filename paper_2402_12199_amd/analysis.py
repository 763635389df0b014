"""Structural and dynamic observables used to compare two trajectories
(paper section 3: centre-of-mass pair correlation g(r), orientational order,
mean-squared displacement, energy conservation).

Host-side numpy on snapshots copied out of the dynamics; none of this is on
the simulation's hot path.
"""
from __future__ import annotations

import numpy as np


def rotate(q: np.ndarray, v: np.ndarray) -> np.ndarray:
    """R(q) v for unit quaternions q (n, 4) = (w, x, y, z) and vectors v (3,) or (n, 3)."""
    w, u = q[:, :1], q[:, 1:]
    v = np.broadcast_to(v, u.shape)
    t = 2.0 * np.cross(u, v)
    return v + w * t + np.cross(u, t)


def rdf(x: np.ndarray, box: float, r_max: float, nbins: int = 100) -> tuple[np.ndarray, np.ndarray]:
    """Centre-of-mass g(r) of one periodic snapshot (cubic box), bins on [0, r_max)."""
    from scipy.spatial import cKDTree
    n = len(x)
    xw = np.mod(x, box)
    pairs = cKDTree(xw, boxsize=box).query_pairs(r_max, output_type="ndarray")
    d = xw[pairs[:, 1]] - xw[pairs[:, 0]]
    d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(axis=1))
    edges = np.linspace(0.0, r_max, nbins + 1)
    h, _ = np.histogram(r, edges)
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    ideal = 0.5 * n * (n - 1) / box ** 3 * shell
    return 0.5 * (edges[1:] + edges[:-1]), h / ideal


def p2(q: np.ndarray, axis: int = 2) -> float:
    """Nematic order parameter of the body axis `axis`: the largest eigenvalue
    of Q = < (3 u u^T - I) / 2 >."""
    e = np.zeros(3)
    e[axis] = 1.0
    u = rotate(q, e)
    Q = 1.5 * (u[:, :, None] * u[:, None, :]).mean(axis=0) - 0.5 * np.eye(3)
    return float(np.linalg.eigvalsh(Q)[-1])


def msd(x0: np.ndarray, x: np.ndarray) -> float:
    """Mean-squared displacement of unwrapped centres."""
    d = x - x0
    return float((d * d).sum(axis=1).mean())


def msr(q0: np.ndarray, q: np.ndarray) -> float:
    """Mean-squared rotation (supplementary section 5): the mean over bodies
    of the orientational distance 1 - <q0, q>^2 between each body's starting
    and current unit quaternions (0 for the same orientation, q and -q
    included; 1 for orientations a half turn apart)."""
    dot = (np.asarray(q0, np.float64) * np.asarray(q, np.float64)).sum(axis=1)
    return float((1.0 - dot * dot).mean())


def rdf_distance(r: np.ndarray, g1: np.ndarray, g2: np.ndarray) -> float:
    """Integrated absolute difference of two g(r) on the same bins, divided by
    the integral of the first."""
    dr = r[1] - r[0]
    return float(np.abs(g1 - g2).sum() * dr / max(np.abs(g1).sum() * dr, 1e-300))
