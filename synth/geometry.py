"""Bead templates of the composite rigid bodies used by the workloads.

A composite rigid body is a rigid set of spherical beads (paper section 2,
first equation: the body-body energy is the double sum over bead pairs).  The
paper does not give bead counts for its shapes, so the workloads define their
own: the surface shell of an n x n x n cubic lattice, and a ring-stacked
cylinder with two filled end-cap discs.

Every template is returned in its body frame: centre of mass at the origin,
principal axes along x, y, z (both shapes are symmetric enough for this to
hold exactly), unit bead mass.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class BodyType:
    name: str
    beads: np.ndarray        # (N, 3) float64, body frame
    mass: float              # = number of beads (unit bead mass)
    inertia: np.ndarray      # (3,) principal moments, body frame
    r_max: float             # circumradius of bead centres
    r_in: float              # inscribed radius of bead centres (see d_min)
    volume: float            # body volume used for the volume fraction

    @property
    def n(self) -> int:
        return int(self.beads.shape[0])


def cube_shell(n: int, a: float = 1.0) -> np.ndarray:
    """Surface points of an n^3 cubic lattice with spacing a, centred at 0.

    A lattice point is on the surface when at least one integer coordinate is
    0 or n-1.  Count n^3 - (n-2)^3 (98 for n=5, 152 for n=6).  Ordered
    lexicographically in (x, y, z) so neighbouring indices are close in space.
    """
    c = (np.arange(n) - (n - 1) / 2.0) * a
    pts = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                if min(i, j, k) == 0 or max(i, j, k) == n - 1:
                    pts.append((c[i], c[j], c[k]))
    return np.asarray(pts, dtype=np.float64)


def cylinder_rings_caps(rings: int = 8, per_ring: int = 12, radius: float = 1.5,
                        spacing: float = 0.9) -> np.ndarray:
    """Cylinder of `rings` rings of `per_ring` beads plus two filled end caps.

    Rings: angles 2*pi*k/per_ring, z = (r - (rings-1)/2) * spacing.
    Caps: a 19-bead disc (centre, 6 beads at radius/2 at 60 degree steps,
    12 beads at `radius` at 30 degree steps) one `spacing` beyond each end
    ring, i.e. at z = +-((rings-1)/2 + 1) * spacing.
    """
    pts = []
    for r in range(rings):
        z = (r - (rings - 1) / 2.0) * spacing
        for k in range(per_ring):
            t = 2.0 * math.pi * k / per_ring
            pts.append((radius * math.cos(t), radius * math.sin(t), z))
    zc = ((rings - 1) / 2.0 + 1.0) * spacing
    for z in (-zc, zc):
        pts.append((0.0, 0.0, z))
        for k in range(6):
            t = 2.0 * math.pi * k / 6
            pts.append((0.5 * radius * math.cos(t), 0.5 * radius * math.sin(t), z))
        for k in range(12):
            t = 2.0 * math.pi * k / 12
            pts.append((radius * math.cos(t), radius * math.sin(t), z))
    return np.asarray(pts, dtype=np.float64)


def principal_inertia(beads: np.ndarray) -> np.ndarray:
    """Diagonal of the unit-mass inertia tensor sum(|r|^2 I - r r^T)."""
    r2 = np.sum(beads * beads, axis=1)
    full = np.eye(3) * r2.sum() - beads.T @ beads
    off = full - np.diag(np.diag(full))
    if np.max(np.abs(off)) > 1e-9 * max(1.0, np.max(np.abs(full))):
        raise ValueError("template is not in its principal frame")
    return np.diag(full).copy()


def make_cube(n: int, a: float = 1.0, sigma: float = 1.0) -> BodyType:
    b = cube_shell(n, a)
    half = (n - 1) * a / 2.0
    return BodyType(
        name=f"cube{n}", beads=b, mass=float(len(b)), inertia=principal_inertia(b),
        r_max=float(np.sqrt(3.0) * half), r_in=half,
        volume=((n - 1) * a + sigma) ** 3)


def make_cylinder(rings: int = 8, per_ring: int = 12, radius: float = 1.5,
                  spacing: float = 0.9, sigma: float = 1.0) -> BodyType:
    b = cylinder_rings_caps(rings, per_ring, radius, spacing)
    length = float(b[:, 2].max() - b[:, 2].min())
    return BodyType(
        name="cyl134", beads=b, mass=float(len(b)), inertia=principal_inertia(b),
        r_max=float(np.sqrt(np.max(np.sum(b * b, axis=1)))), r_in=radius,
        volume=math.pi * (radius + sigma / 2.0) ** 2 * (length + sigma))


def box_length(n_bodies: int, body: BodyType, phi: float) -> float:
    """Cubic box edge for volume fraction phi = N * V_body / V_box."""
    return (n_bodies * body.volume / phi) ** (1.0 / 3.0)
