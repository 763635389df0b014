"""Seeded random inputs: orientations, placements, momenta, pair batches, weights.

Quaternions are (w, x, y, z), Hamilton convention, unit norm, mapping body
frame to lab frame.  All generators take a numpy Generator (PCG64) so every
input is reproducible from its seed.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

from .geometry import BodyType

MLP_DIMS = (7, 128, 128, 128, 128, 1)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_quaternions(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions on S^3 (Shoemake's subgroup method)."""
    u1, u2, u3 = g.random(n), g.random(n), g.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    t2, t3 = 2.0 * np.pi * u2, 2.0 * np.pi * u3
    # (w, x, y, z)
    return np.stack([b * np.cos(t3), a * np.sin(t2), a * np.cos(t2), b * np.sin(t3)], axis=1)


def uniform_directions(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rotate(q: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Rotate body-frame points v (M,3) by each quaternion q (K,4) -> (K,M,3)."""
    rot = Rotation.from_quat(np.stack([q[:, 1], q[:, 2], q[:, 3], q[:, 0]], axis=1))
    return np.einsum("kab,mb->kma", rot.as_matrix(), v)


def place_bodies(g: np.random.Generator, n: int, body: BodyType, box: float,
                 min_bead_gap: float = 1.0, max_tries: int = 1000) -> tuple[np.ndarray, np.ndarray]:
    """Random sequential addition of n bodies in a periodic cubic box.

    Each trial body gets a uniform position and a uniform orientation; it is
    rejected if any of its beads is closer than `min_bead_gap` to a bead of an
    already placed body (minimum image).  Trials are drawn in chunks from g,
    so the result depends only on the seed.  Returns x (n,3) in [0, box) and
    q (n,4).
    """
    reach = 2.0 * body.r_max + min_bead_gap
    nc = max(1, int(box // reach))
    cell_w = box / nc
    cells: dict[int, list[int]] = {}
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    x = np.zeros((n, 3))
    q = np.zeros((n, 4))
    beads = np.zeros((n, body.n, 3))
    gap2 = min_bead_gap * min_bead_gap
    placed = 0
    tries = 0
    chunk = 1024
    while placed < n:
        xs = g.random((chunk, 3)) * box
        qs = uniform_quaternions(g, chunk)
        bs = _rotate(qs, body.beads)
        for t in range(chunk):
            if placed == n:
                break
            tries += 1
            if tries > max_tries * n:
                raise RuntimeError(f"placement stalled at {placed}/{n} bodies")
            xt = xs[t]
            c = (xt // cell_w).astype(int) % nc
            cand = []
            for o in offs:
                key = (((c[0] + o[0]) % nc) * nc + (c[1] + o[1]) % nc) * nc + (c[2] + o[2]) % nc
                lst = cells.get(key)
                if lst:
                    cand.extend(lst)
            ok = True
            if cand:
                cand = np.unique(np.asarray(cand))
                d = x[cand] - xt
                d -= box * np.round(d / box)
                near = np.einsum("ka,ka->k", d, d) < reach * reach
                # only beads within r_max + gap of the other body's centre
                # can be closer than gap to one of its beads
                shell2 = (body.r_max + min_bead_gap) ** 2
                bt = bs[t]
                for j, dj in zip(cand[near], d[near]):
                    other = beads[j] + dj
                    o = other[np.einsum("ma,ma->m", other, other) < shell2]
                    tt = bt[np.einsum("ma,ma->m", bt - dj, bt - dj) < shell2]
                    if len(o) and len(tt):
                        diff = tt[:, None, :] - o[None, :, :]
                        if np.min(np.einsum("abc,abc->ab", diff, diff)) < gap2:
                            ok = False
                            break
            if not ok:
                continue
            x[placed], q[placed], beads[placed] = xt, qs[t], bs[t]
            key = (c[0] * nc + c[1]) * nc + c[2]
            cells.setdefault(key, []).append(placed)
            placed += 1
    return x, q


def maxwell_boltzmann(g: np.random.Generator, n: int, body: BodyType, kT: float
                      ) -> tuple[np.ndarray, np.ndarray]:
    """Linear momenta P (n,3) and body-frame angular momenta L (n,3).

    P ~ N(0, M kT) per component with the total momentum removed;
    L_a ~ N(0, I_a kT) per principal axis.
    """
    p = g.standard_normal((n, 3)) * np.sqrt(body.mass * kT)
    p -= p.mean(axis=0, keepdims=True)
    lb = g.standard_normal((n, 3)) * np.sqrt(body.inertia[None, :] * kT)
    return p, lb


def pair_batch(g: np.random.Generator, n: int, d_lo: float, d_hi: float) -> np.ndarray:
    """Random pair configurations (n, 7) = (d_x, d_y, d_z, q_w, q_x, q_y, q_z).

    d is the separation of body j from body i in body i's frame: a uniform
    direction on S^2 times a distance uniform in [d_lo, d_hi].  q is the
    orientation of body j relative to body i, uniform on S^3 (the relative
    orientation of two independent uniform orientations is itself uniform).
    """
    d = uniform_directions(g, n) * g.uniform(d_lo, d_hi, size=(n, 1))
    return np.concatenate([d, uniform_quaternions(g, n)], axis=1)


def xavier_params(seed: int, dims=MLP_DIMS) -> np.ndarray:
    """Glorot-uniform weights, zero biases, as one float64 vector.

    Layout, layer by layer: W_l (out x in, row major) then b_l (out).
    """
    g = rng(seed)
    parts = []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(g.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def n_params(dims=MLP_DIMS) -> int:
    return int(sum(o * i + o for i, o in zip(dims[:-1], dims[1:])))
