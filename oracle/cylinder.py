"""ORACLE (test infrastructure only): the four-number pair descriptor of two
identical cylinders (paper section 2: a cylinder pair is a function of four
numbers thanks to the cylindrical symmetry; supplementary section 2: how the
four numbers are formed).

Steps of the supplement, for body 1's frame (its axis is the body z axis):
* the frame's z axis is body 1's axis, pointing so that body 2's centre has
  p_z >= 0;
* the frame's x axis is chosen so that body 2's centre has p_y = 0 and
  p_x >= 0, so (p_r, p_z) = (p_x, p_z) fixes the position (a third number
  would be redundant under the assumed cylindrical symmetry of body 1);
* body 2's axis, a unit vector in that frame, in spherical coordinates
  (theta, phi) gives the two remaining numbers.

Readings (the supplement is silent on them): the frame's y axis completes a
right-handed frame (z cross x); at p_r = 0 the x axis is body 1's own x axis;
theta = arccos(a_z) in [0, pi], phi = atan2(a_y, a_x) in (-pi, pi].  The
network takes the four numbers through smooth functions that are also
unchanged under the two symmetries the supplement leaves to the data -- body
2 turned end over end (a -> -a; the bead cylinder is symmetric under it)
and the mirror y -> -y of the canonical frame (both cylinders and the bead
potential are mirror symmetric):

  s = (p_r^2, p_z^2, a_z^2, (p_r a_x)^2, p_r a_x a_z p_z, 0, 0)

with a = (sin theta cos phi, sin theta sin phi, cos theta).  Written in the
pair descriptor (d, q) these are polynomials: with t = d_x A_x + d_y A_y and
A = R(q) e_z, s = (d_x^2 + d_y^2, d_z^2, A_z^2, t^2, t A_z d_z, 0, 0), so the
squares keep s smooth where the frame choice is not (p_r = 0, p_z = 0).
R(q) is taken in the homogeneous form v -> q v q^* for the Jacobian (q as
four free components), as for the cube descriptor.
"""
from __future__ import annotations

import numpy as np

from . import frames

EZ = np.array([0.0, 0.0, 1.0])


def _axis(q: np.ndarray) -> np.ndarray:
    """Body 2's axis R(q) e_z (homogeneous form: |q|^2 times the unit axis)."""
    q = np.asarray(q, np.float64)
    return frames.qrotate(q, np.broadcast_to(EZ, q.shape[:-1] + (3,)))


def _canonical(desc: np.ndarray):
    """Per pair, following the supplement's steps: (p_r, p_z) and body 2's
    axis components (a_x, a_y, a_z) in the canonical frame."""
    desc = np.asarray(desc, np.float64)
    d = desc[:, :3]
    A = _axis(desc[:, 3:7])
    out = np.empty((len(desc), 5))
    for n in range(len(desc)):
        ez = EZ if d[n, 2] >= 0 else -EZ
        rho = np.hypot(d[n, 0], d[n, 1])
        ex = np.array([d[n, 0] / rho, d[n, 1] / rho, 0.0]) if rho > 0 else np.array([1.0, 0.0, 0.0])
        ey = np.cross(ez, ex)
        p = np.array([d[n] @ ex, d[n] @ ey, d[n] @ ez])
        assert abs(p[1]) <= 1e-12 * max(1.0, rho) and p[0] >= 0 and p[2] >= 0
        out[n] = (p[0], p[2], A[n] @ ex, A[n] @ ey, A[n] @ ez)
    return out


def cyl_numbers(desc: np.ndarray) -> np.ndarray:
    """The supplement's four numbers (p_r, p_z, theta, phi) (P, 4) of pair
    descriptors desc (P, 7) = (d, q) (q unit)."""
    c = _canonical(desc)
    a = c[:, 2:5] / np.linalg.norm(c[:, 2:5], axis=1, keepdims=True)
    return np.stack([c[:, 0], c[:, 1], np.arccos(np.clip(a[:, 2], -1.0, 1.0)), np.arctan2(a[:, 1], a[:, 0])], axis=1)


def cyl_descriptor(desc: np.ndarray) -> np.ndarray:
    """The network's input s (P, 7) = (p_r^2, p_z^2, a_z^2, (p_r a_x)^2,
    p_r a_x a_z p_z, 0, 0) from pair descriptors desc (P, 7) = (d, q)."""
    c = _canonical(desc)
    pr, pz, ax, az = c[:, 0], c[:, 1], c[:, 2], c[:, 4]
    z = np.zeros_like(pr)
    return np.stack([pr * pr, pz * pz, az * az, (pr * ax) ** 2, pr * ax * az * pz, z, z], axis=1)


def descriptor_of_numbers(num: np.ndarray) -> np.ndarray:
    """s (P, 7) from the four numbers (p_r, p_z, theta, phi) (P, 4)."""
    num = np.asarray(num, np.float64)
    pr, pz, th, ph = num.T
    ax, az = np.sin(th) * np.cos(ph), np.cos(th)
    z = np.zeros_like(pr)
    return np.stack([pr * pr, pz * pz, az * az, (pr * ax) ** 2, pr * ax * az * pz, z, z], axis=1)


def cyl_configuration(num: np.ndarray) -> np.ndarray:
    """A pair configuration (P, 7) = (d, q) with the four numbers num (P, 4):
    body 2 at (p_r, 0, p_z), its axis turned from e_z to
    (sin th cos ph, sin th sin ph, cos th) by the smallest rotation."""
    num = np.asarray(num, np.float64)
    out = np.empty((len(num), 7))
    for n, (pr, pz, th, ph) in enumerate(num):
        a = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        axis = np.cross(EZ, a)
        s = np.linalg.norm(axis)
        q = frames.qexp(axis / s * th) if s > 1e-15 else (np.array([1.0, 0, 0, 0]) if a[2] > 0 else
                                                          np.array([0.0, 1.0, 0, 0]))
        out[n, :3] = (pr, 0.0, pz)
        out[n, 3:] = q
    return out


def cyl_descriptor_jacobian(desc: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """d s / d (d, q) (P, 7, 7) by central differences of cyl_descriptor
    (q treated as four free components)."""
    desc = np.asarray(desc, np.float64)
    J = np.empty((len(desc), 7, 7))
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        J[:, :, k] = (cyl_descriptor(desc + e) - cyl_descriptor(desc - e)) / (2 * h)
    return J
