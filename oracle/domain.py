"""ORACLE (test infrastructure only): a lower bound on the closest bead-bead
distance of a body pair, from two convex shells around each body's bead
centres, and the routing it implies.

The learned pair energy is fitted on configurations whose closest bead pair
is at least r_rej apart (deeper overlaps are absent from dynamics at the
workloads' temperatures and are rejected from the training data).  A pair
may be handed to the network only when it provably lies in that domain;
every other pair goes to the bead sum, which is exact everywhere (paper
section 2: the bead path is the reference the network approximates).

Shells, in the body frame (centre of mass at the origin):
* the bead-centre box: |x| <= h_x, |y| <= h_y, |z| <= h_z (largest
  coordinate magnitudes);
* a capsule along the body axis k with the largest h_k: the points within
  R of the segment from -H e_k to +H e_k, with R the largest distance of a
  bead from that axis and H the smallest half-length that keeps every bead
  inside;
* the solid cylinder around the same axis with radius R and half-height h_k.
The round shells (capsule, cylinder) are formed only for bodies whose
cylinder is narrower than their box (pi R^2 < 4 h_a h_b across the axis):
cylinders, not cubes.

For convex sets, the gap between the projections onto any unit axis is a
lower bound on their distance (separating-axis theorem); for the boxes the
15 candidate axes of two boxes are tried (each box's face normals and the
cross products of their edges).  The capsule distance is the distance of the
two segments minus both radii.  For the cylinders, the projected gap along
trial directions: starting from the direction between the capsules' closest
points, and again from the direction between the centres, each next
direction is that of the difference of the two support points along the
current one (six directions from each start).  gap = the largest of these
bounds the closest bead-centre distance from below.
"""
from __future__ import annotations

import numpy as np

from . import frames


def shells(beads: np.ndarray):
    """Box half extents h (3), capsule axis k, radius R and half-length H."""
    b = np.asarray(beads, np.float64)
    h = np.abs(b).max(axis=0)
    k = int(np.argmax(h))
    perp = np.sqrt(np.sum(np.delete(b, k, axis=1) ** 2, axis=1))
    R = float(perp.max())
    H = float(max(0.0, np.max(np.abs(b[:, k]) - np.sqrt(np.maximum(R * R - perp * perp, 0.0)))))
    return h, k, R, H


def _corners(h: np.ndarray) -> np.ndarray:
    s = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], np.float64)
    return s * h


def box_gap(ha: np.ndarray, hb: np.ndarray, d: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Largest projected gap between box A (origin, frame axes, half extents
    ha) and box B (centre d, axes the columns of R, half extents hb) over
    the 15 separating-axis candidates, each box projected through its 8
    corners; d (P, 3), R (P, 3, 3) -> (P,).  Negative when no candidate axis
    separates them."""
    d = np.atleast_2d(np.asarray(d, np.float64))
    R = np.asarray(R, np.float64).reshape(-1, 3, 3)
    P = len(d)
    ca = _corners(np.asarray(ha, np.float64))                          # (8, 3)
    cb = d[:, None, :] + np.einsum("ck,pjk->pcj", _corners(np.asarray(hb, np.float64)), R)   # (P, 8, 3)
    E = np.broadcast_to(np.eye(3), (P, 3, 3))
    axes = [E[:, i] for i in range(3)] + [R[:, :, j] for j in range(3)]
    axes += [np.cross(E[:, i], R[:, :, j]) for i in range(3) for j in range(3)]
    best = np.full(P, -np.inf)
    for L in axes:
        n = np.linalg.norm(L, axis=1)
        use = n >= 1e-6                     # (near-)parallel edges: no usable axis
        L = L / np.where(use, n, 1.0)[:, None]
        pa = np.einsum("ck,pk->pc", ca, L)
        pb = np.einsum("pck,pk->pc", cb, L)
        g = np.maximum(pb.min(1) - pa.max(1), pa.min(1) - pb.max(1))
        best = np.where(use, np.maximum(best, g), best)
    return best


def segment_distance(p0, p1, q0, q1) -> np.ndarray:
    """Distance between the segments [p0, p1] and [q0, q1] (each (3,) or
    (P, 3)): the smallest of the distances of each end point to the other
    segment and, when the segments' lines meet the interior of both, the
    distance of the lines' closest points."""
    p0, p1, q0, q1 = (np.atleast_2d(np.asarray(v, np.float64)) for v in (p0, p1, q0, q1))

    def point_seg(x, a, b):
        ab = b - a
        den = np.sum(ab * ab, 1)
        t = np.clip(np.sum((x - a) * ab, 1) / np.where(den > 0, den, 1.0), 0.0, 1.0)
        t = np.where(den > 0, t, 0.0)
        return np.linalg.norm(x - (a + t[:, None] * ab), axis=1)

    best = np.minimum.reduce([point_seg(p0, q0, q1), point_seg(p1, q0, q1), point_seg(q0, p0, p1),
                              point_seg(q1, p0, p1)])
    u, v, w = p1 - p0, q1 - q0, p0 - q0
    a, b, c = np.sum(u * u, 1), np.sum(u * v, 1), np.sum(v * v, 1)
    dd, e = np.sum(u * w, 1), np.sum(v * w, 1)
    den = a * c - b * b
    ok = den > 1e-12 * a * c
    dsafe = np.where(ok, den, 1.0)
    s = (b * e - c * dd) / dsafe
    t = (a * e - b * dd) / dsafe
    ok &= (s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)
    inner = np.linalg.norm(w + s[:, None] * u - t[:, None] * v, axis=1)
    out = np.where(ok, np.minimum(best, inner), best)
    return out if out.size > 1 else float(out[0])


def cylinder_support(c, a, H, R, n):
    """Support points (P, 3) of solid cylinders (centres c, unit axes a,
    half-height H, radius R) in the unit directions n: the cap centre on the
    side n faces plus R along n's component perpendicular to the axis."""
    na = np.sum(n * a, 1, keepdims=True)
    perp = n - na * a
    pn = np.linalg.norm(perp, axis=1, keepdims=True)
    radial = np.where(pn > 1e-12, R * perp / np.where(pn > 1e-12, pn, 1.0), 0.0)
    return c + np.where(na >= 0, H, -H) * a + radial


def cylinder_gap(ca, aa, Ha, Ra, cb, ab, Hb, Rb, n0, iters=6):
    """Largest projected gap between cylinders A and B over the trial
    directions of the support-point iteration started from n0 (P, 3)."""
    n = n0 / np.linalg.norm(n0, axis=1, keepdims=True)
    best = np.full(len(n), -np.inf)
    for _ in range(iters):
        diff = cylinder_support(cb, ab, Hb, Rb, -n) - cylinder_support(ca, aa, Ha, Ra, n)
        best = np.maximum(best, np.sum(n * diff, 1))
        dn = np.linalg.norm(diff, axis=1, keepdims=True)
        n = np.where(dn > 1e-12, diff / np.where(dn > 1e-12, dn, 1.0), n)
    return best


def _closest_direction(p0, p1, q0, q1):
    """Unit vectors from the closest point of [p0, p1] to that of [q0, q1]
    (dense parameter search around the exact distance is not needed: the
    direction only seeds the cylinder iteration)."""
    u, v, w = p1 - p0, q1 - q0, p0 - q0
    a, b, c = np.sum(u * u, 1), np.sum(u * v, 1), np.sum(v * v, 1)
    dd, e = np.sum(u * w, 1), np.sum(v * w, 1)
    den = a * c - b * b
    s = np.where(den > 1e-12 * a * c, np.clip((b * e - c * dd) / np.where(den > 0, den, 1.0), 0, 1), 0.5)
    t = np.clip((b * s + e) / np.where(c > 0, c, 1.0), 0, 1)
    s = np.clip((b * t - dd) / np.where(a > 0, a, 1.0), 0, 1)
    diff = (q0 + t[:, None] * v) - (p0 + s[:, None] * u)
    return diff


def _round(h, k, R) -> bool:
    """Whether the round shells (capsule, cylinder) are formed for a body:
    its cylinder's cross-section pi R^2 is smaller than its box's across the
    axis (cylinders yes, cubes no)."""
    return np.pi * R * R < 4.0 * h[(k + 1) % 3] * h[(k + 2) % 3]


def gap(beads_i: np.ndarray, beads_j: np.ndarray, desc: np.ndarray) -> np.ndarray:
    """Lower bound (P,) on the closest bead-centre distance of each pair
    configuration desc (P, 7) = (d, q) (body j at d with orientation q in
    body i's frame)."""
    hi, ki, Ri, Hi = shells(beads_i)
    hj, kj, Rj, Hj = shells(beads_j)
    desc = np.atleast_2d(np.asarray(desc, np.float64))
    d = desc[:, :3]
    q = desc[:, 3:] / np.linalg.norm(desc[:, 3:], axis=1, keepdims=True)
    R = np.stack([frames.qrotate(q, np.broadcast_to(e, (len(q), 3))) for e in np.eye(3)], axis=2)
    gb = box_gap(hi, hj, d, R)
    ei = np.broadcast_to(np.eye(3)[ki], d.shape)
    ej = R[:, :, kj]
    if not (_round(hi, ki, Ri) and _round(hj, kj, Rj)):
        return gb
    gc = np.atleast_1d(segment_distance(-Hi * ei, Hi * ei, d - Hj * ej, d + Hj * ej)) - Ri - Rj
    G = np.maximum(gb, gc)
    zero = np.zeros_like(d)
    for n0 in (_closest_direction(-Hi * ei, Hi * ei, d - Hj * ej, d + Hj * ej), d):
        ok = np.linalg.norm(n0, axis=1) > 1e-9
        n0 = np.where(ok[:, None], n0, 1.0)
        gcyl = cylinder_gap(zero, ei, hi[ki], Ri, d, ej, hj[kj], Rj, n0)
        G = np.where(ok, np.maximum(G, gcyl), G)
    return G
