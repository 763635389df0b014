"""ORACLE (test infrastructure only): the symmetry-reduced pair descriptor
of two identical cubes (supplementary section 1).

A cube pair has six degrees of freedom; the cube's symmetry group (48
signed permutations of the axes, rotations and reflections) acting on body
1's frame, and the 24 rotations that map body 2 onto itself, leave the bead
energy unchanged.  The descriptor picks one representative:

* position: body 1's axes are relabelled and their signs chosen (a signed
  permutation g, reflections allowed) so that body 2's centre p = g d has
  p_x >= p_y >= p_z >= 0 -- non-negative coordinates, the largest along x
  (body 1's interacting face normal is (1, 0, 0)), and p_y >= p_z (the
  reflection across the y = z plane);
* orientation, M = g R g^T with R body 2's orientation in body 1's frame:
  w is the face normal of body 2 with the largest x component (the normal
  opposite the face nearest to body 1), alpha_1 = arccos(w_x),
  alpha_2 = atan2(w_z, w_y); after the smallest rotation Q that takes w to
  (1, 0, 0), the remaining turn of body 2 about x is the angle of Q v in the
  y-z plane for a second face normal v of body 2, alpha_3 = that angle
  modulo pi/2 (the four face normals perpendicular to w give the same value).

Readings (the supplement is silent on them): ties in the sort and in the
choice of w go to the lower axis index; alpha_2 in (-pi, pi], alpha_3 in
[0, pi/2).  The descriptor is s = (p_x, p_y, p_z, alpha_1, alpha_2,
alpha_3).
"""
from __future__ import annotations

import numpy as np

from . import frames

HALF_PI = 0.5 * np.pi


def rotation_matrices(q: np.ndarray) -> np.ndarray:
    """R(q) (P, 3, 3), body to frame, columns R e_k, for unit quaternions."""
    q = np.asarray(q, np.float64)
    cols = [frames.qrotate(q, np.broadcast_to(e, q.shape[:-1] + (3,))) for e in np.eye(3)]
    return np.stack(cols, axis=-1)


def cube_descriptor(desc: np.ndarray) -> np.ndarray:
    """s (P, 6) from pair descriptors desc (P, 7) = (d, q), d body 2's centre
    in body 1's frame and q its orientation relative to body 1."""
    desc = np.asarray(desc, np.float64)
    d, R = desc[:, :3], rotation_matrices(desc[:, 3:7])
    out = np.empty((len(desc), 6))
    for n in range(len(desc)):
        a = np.abs(d[n])
        order = sorted(range(3), key=lambda k: (-a[k], k))          # largest first, ties by index
        g = np.zeros((3, 3))
        for row, k in enumerate(order):
            g[row, k] = 1.0 if d[n, k] >= 0 else -1.0
        p = g @ d[n]
        M = g @ R[n] @ g.T
        k = max(range(3), key=lambda c: (abs(M[0, c]), -c))        # face normal with the largest |x|
        w = np.sign(M[0, k]) * M[:, k] if M[0, k] != 0 else M[:, k]
        v = M[:, (k + 1) % 3]
        c = v[0] / (1.0 + w[0])                                     # Q v = v - (w + e_x) v_x / (1 + w_x)
        beta = np.arctan2(v[2] - w[2] * c, v[1] - w[1] * c)
        out[n] = (p[0], p[1], p[2], np.arccos(np.clip(w[0], -1.0, 1.0)), np.arctan2(w[2], w[1]),
                  beta - HALF_PI * np.floor(beta / HALF_PI))
    return out


def cube_configuration(s: np.ndarray) -> np.ndarray:
    """A pair configuration (P, 7) = (d, q) with descriptor s: body 2 at p
    with w = (cos a1, sin a1 cos a2, sin a1 sin a2) and the turn a3 about it."""
    from scipy.spatial.transform import Rotation
    s = np.asarray(s, np.float64)
    out = np.empty((len(s), 7))
    for n, (px, py, pz, a1, a2, a3) in enumerate(s):
        w = np.array([np.cos(a1), np.sin(a1) * np.cos(a2), np.sin(a1) * np.sin(a2)])
        axis = np.cross(w, [1.0, 0.0, 0.0])
        nrm = np.linalg.norm(axis)
        Q = Rotation.from_rotvec(axis / nrm * a1).as_matrix() if nrm > 0 else np.eye(3)
        Rx = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(a3), -np.sin(a3)], [0.0, np.sin(a3), np.cos(a3)]])
        M = Q.T @ Rx                                                # M e_x = w; Q M e_y at angle a3
        x, y, z, qw = Rotation.from_matrix(M).as_quat()             # scipy: scalar last
        out[n] = (px, py, pz, qw, x, y, z)
    return out


def cube_descriptor_jacobian(desc: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """d s / d (d, q) (P, 6, 7) by central differences of cube_descriptor
    (q treated as four free components; alpha_3 unwrapped across its cut)."""
    desc = np.asarray(desc, np.float64)
    J = np.empty((len(desc), 6, 7))
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        sp, sm = cube_descriptor(desc + e), cube_descriptor(desc - e)
        diff = sp - sm
        diff[:, 5] -= HALF_PI * np.round(diff[:, 5] / HALF_PI)
        diff[:, 4] -= 2 * np.pi * np.round(diff[:, 4] / (2 * np.pi))
        J[:, :, k] = diff / (2 * h)
    return J
