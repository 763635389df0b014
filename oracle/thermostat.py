"""ORACLE (test infrastructure only): constant-temperature dynamics.

The paper runs its simulations in the canonical ensemble with a Nose-Hoover
thermostat (section 3); it does not give the scheme.  This oracle uses the
textbook single-thermostat Nose-Hoover equations (Nose, Mol. Phys. 52, 255,
1984; Hoover, Phys. Rev. A 31, 1695, 1985) on every momentum of the rigid
bodies, translational and angular:

    dP/dt = F - xi P,   dL/dt = tau - xi L,   dxi/dt = (2K - g kT) / Q,
    deta/dt = xi,

with K the total kinetic energy and g the number of degrees of freedom; the
conserved quantity is K + U + Q xi^2 / 2 + g kT eta.  The time step is the
constant-energy velocity Verlet of `beads` followed by the thermostat flow
over dt taken as two half steps; each half step h moves xi by (h/2) G(K),
scales the momenta by exp(-xi h) (the exact solution of dP/dt = -xi P at
fixed xi), moves eta by xi h, and moves xi by (h/2) G(K') with the scaled
K', where G(K) = (2K - g kT) / Q.  The scale factor of a step is applied to
the momenta at the start of the next step, before its half kick.
"""
from __future__ import annotations

import math

import numpy as np

from . import beads


def nh_flow(K: float, xi: float, eta: float, Q: float, gkT: float, dt: float):
    """Thermostat flow over dt at kinetic energy K: returns the new xi, eta,
    the momentum scale factor and the scaled kinetic energy."""
    h = 0.5 * dt
    scale = 1.0
    for _ in range(2):
        xi += 0.5 * h * (2.0 * K - gkT) / Q
        s = math.exp(-xi * h)
        eta += xi * h
        K *= s * s
        scale *= s
        xi += 0.5 * h * (2.0 * K - gkT) / Q
    return xi, eta, scale, K


def nvt(x, P, q, L, types, templates, masses, inertias, box, steps, dt, Q, gkT, eps=1.0, sigma=1.0,
        rc=2.5) -> dict:
    """`steps` thermostatted steps; x, P, q, L (n x 3 / n x 4, FP64) are
    advanced in place and left with the last step's scale factor still
    unapplied (as the GPU leaves them).  Returns per-step series of the
    potential and kinetic energy (before the thermostat), xi, eta, the scale
    factor and the conserved quantity."""
    types = np.asarray(types)
    m = np.asarray(masses, np.float64)[types]
    I = np.asarray(inertias, np.float64).reshape(-1, 3)[types]
    r = beads.bead_system(x, q, types, templates, box, eps, sigma, rc)
    F, T = r["F"], r["tau"]
    xi, eta, scale = 0.0, 0.0, 1.0
    out = {k: [] for k in ("pe", "ke", "xi", "eta", "scale", "conserved")}
    for _ in range(steps):
        P *= scale
        L *= scale
        beads.rigid_phase1(dt, x, P, q, L, m, I, F, T)
        r = beads.bead_system(x, q, types, templates, box, eps, sigma, rc)
        F, T = r["F"], r["tau"]
        K = beads.rigid_phase2(dt, P, q, L, m, I, F, T)
        pe = r["E"]
        xi, eta, scale, Ks = nh_flow(K, xi, eta, Q, gkT, dt)
        out["pe"].append(pe)
        out["ke"].append(K)
        out["xi"].append(xi)
        out["eta"].append(eta)
        out["scale"].append(scale)
        # conserved quantity after the thermostat flow (Ks: kinetic energy of
        # the scaled momenta)
        out["conserved"].append(Ks + pe + 0.5 * Q * xi * xi + gkT * eta)
    return {k: np.asarray(v) for k, v in out.items()}
