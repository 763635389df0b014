"""ORACLE (test infrastructure only): pair descriptors and forces/torques from
the gradient of a pair energy expressed in those descriptors.

Paper section 2: a pair configuration is fixed by the position and the
orientation of body j in the frame of body i, so the pair energy is a
function U = g(x, Omega) of those numbers.  Here x = d = R_i^T (x_j - x_i)
(minimum image) and Omega is the relative unit quaternion q = q_i^* q_j, so
R(q) = R_i^T R_j.  Forces and torques are minus the derivatives of that
energy with respect to translations and rotations (supplementary section 6:
f = -dE/dx, tau_eta = -dE/dtheta_eta).  The paper obtains them by central
finite differences plus a chain rule through its angle descriptors; with a
quaternion descriptor the derivatives have a closed form, derived here from
the same definitions:

  rotating body j by a small angle theta about a lab axis n maps
  q -> exp(theta n'/2) q with n' = R_i^T n, so
  dE/dtheta = (1/2) n' . (w g_v - g_w v + v x g_v) for q = (w, v) and
  g = dE/dq, giving tau_j = -(1/2)(w g_v - g_w v + v x g_v) in body i's frame;
  F_j = -dE/dd, F_i = -F_j;
  rotating the whole pair rigidly about x_i leaves E unchanged, so
  tau_i = -tau_j - d x F_j.
"""
from __future__ import annotations

import numpy as np


def qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of quaternion arrays (..., 4), scalar first."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def qconj(q: np.ndarray) -> np.ndarray:
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def qrotate(q: np.ndarray, v: np.ndarray) -> np.ndarray:
    """R(q) v computed as the vector part of q (0, v) q^* (q unit)."""
    v4 = np.concatenate([np.zeros(v.shape[:-1] + (1,)), v], axis=-1)
    return qmul(qmul(q, v4), qconj(q))[..., 1:]


def qexp(axis_angle: np.ndarray) -> np.ndarray:
    """exp of the pure quaternion (0, a/2): rotation by |a| about a/|a|."""
    a = np.asarray(axis_angle, dtype=np.float64)
    th = np.linalg.norm(a, axis=-1, keepdims=True)
    half = 0.5 * th
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(th > 0, np.sin(half) / np.where(th > 0, th, 1.0), 0.5)
    return np.concatenate([np.cos(half), s * a], axis=-1)


def min_image(d: np.ndarray, box) -> np.ndarray:
    if box is None:
        return d
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    return d - b * np.round(d / b)


def descriptors(xi, qi, xj, qj, box=None) -> np.ndarray:
    """(P, 7) = (d, q_rel): d = R_i^T minimg(x_j - x_i), q_rel = q_i^* q_j."""
    xi, qi, xj, qj = (np.asarray(a, dtype=np.float64) for a in (xi, qi, xj, qj))
    dl = min_image(xj - xi, box)
    d = qrotate(qconj(qi), dl)
    return np.concatenate([d, qmul(qconj(qi), qj)], axis=-1)


def forces_from_grad(desc: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Per-pair (P, 9) = F_j, tau_i, tau_j in body i's frame from g = dE/du."""
    desc = np.asarray(desc, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    d, w, v = desc[:, :3], desc[:, 3:4], desc[:, 4:7]
    gd, gw, gv = g[:, :3], g[:, 3:4], g[:, 4:7]
    Fj = -gd
    tauj = -0.5 * (w * gv - gw * v + np.cross(v, gv))
    taui = -tauj - np.cross(d, Fj)
    return np.concatenate([Fj, taui, tauj], axis=1)


def to_lab(qi: np.ndarray, ft: np.ndarray) -> np.ndarray:
    """Rotate per-pair (P, 9) body-i-frame vectors into the lab frame."""
    out = np.empty_like(ft)
    for s in range(3):
        out[:, 3 * s:3 * s + 3] = qrotate(qi, ft[:, 3 * s:3 * s + 3])
    return out
