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
[0, pi/2).  The network takes the angles through smooth functions of them,
s = (p_x, p_y, p_z, sin a1 cos a2, sin a1 sin a2, cos 4 a3, sin 4 a3) =
(p, w_y, w_z, cos 4 a3, sin 4 a3): the same information (w_x >= 1/sqrt 3 is
fixed by w_y, w_z; alpha_3 is taken modulo pi/2) without the polar
singularity of (alpha_1, alpha_2) at w = (1, 0, 0), where the chain rule of
the angles divides by sin alpha_1, and without the cut of alpha_3 between 0
and pi/2.  cube_angles gives the paper's six numbers.
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


def _canonical(desc: np.ndarray):
    """Per pair: p (3), the face normal w (3) and the turn beta about it
    (not yet reduced modulo pi/2)."""
    desc = np.asarray(desc, np.float64)
    d, R = desc[:, :3], rotation_matrices(desc[:, 3:7])
    out = np.empty((len(desc), 7))
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
        out[n] = (p[0], p[1], p[2], w[0], w[1], w[2], beta)
    return out


def cube_angles(desc: np.ndarray) -> np.ndarray:
    """The paper's six numbers (p_x, p_y, p_z, alpha_1, alpha_2, alpha_3)
    (P, 6) from pair descriptors desc (P, 7) = (d, q), d body 2's centre in
    body 1's frame and q its orientation relative to body 1."""
    c = _canonical(desc)
    beta = c[:, 6]
    return np.stack([c[:, 0], c[:, 1], c[:, 2], np.arccos(np.clip(c[:, 3], -1.0, 1.0)), np.arctan2(c[:, 5], c[:, 4]),
                     beta - HALF_PI * np.floor(beta / HALF_PI)], axis=1)


def cube_descriptor(desc: np.ndarray) -> np.ndarray:
    """The network's input s (P, 7) = (p, w_y, w_z, cos 4 a3, sin 4 a3) =
    (p, sin a1 cos a2, sin a1 sin a2, cos 4 a3, sin 4 a3) from pair
    descriptors desc (P, 7) = (d, q)."""
    c = _canonical(desc)
    return np.stack([c[:, 0], c[:, 1], c[:, 2], c[:, 4], c[:, 5], np.cos(4 * c[:, 6]), np.sin(4 * c[:, 6])], axis=1)


def angles_of(s: np.ndarray) -> np.ndarray:
    """The six angles' form of descriptors s (P, 7)."""
    s = np.asarray(s, np.float64)
    a3 = 0.25 * np.arctan2(s[:, 6], s[:, 5])
    return np.stack([s[:, 0], s[:, 1], s[:, 2], np.arcsin(np.clip(np.hypot(s[:, 3], s[:, 4]), 0.0, 1.0)),
                     np.arctan2(s[:, 4], s[:, 3]), a3 - HALF_PI * np.floor(a3 / HALF_PI)], axis=1)


def cube_configuration(s: np.ndarray) -> np.ndarray:
    """A pair configuration (P, 7) = (d, q) with descriptor s (P, 7): body 2
    at p with w = (cos a1, sin a1 cos a2, sin a1 sin a2) and the turn a3
    about it."""
    from scipy.spatial.transform import Rotation
    out = np.empty((len(s), 7))
    for n, (px, py, pz, a1, a2, a3) in enumerate(angles_of(s)):
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
    """d s / d (d, q) (P, 7, 7) by central differences of cube_descriptor
    (q treated as four free components)."""
    desc = np.asarray(desc, np.float64)
    J = np.empty((len(desc), 7, 7))
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        J[:, :, k] = (cube_descriptor(desc + e) - cube_descriptor(desc - e)) / (2 * h)
    return J
