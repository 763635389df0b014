"""Initial states of the dynamics workloads (positions, orientations, momenta)."""
from __future__ import annotations

import numpy as np

from .configs import SystemConfig
from .sampling import maxwell_boltzmann, place_bodies, rng


def initial_state(cfg: SystemConfig) -> dict:
    """Seeded random placement (overlaps rejected), uniform orientations and
    Maxwell-Boltzmann momenta at cfg.kT.  Arrays are (n, k) float64."""
    g = rng(cfg.seed)
    x, q = place_bodies(g, cfg.n_bodies, cfg.body, cfg.box)
    P, L = maxwell_boltzmann(g, cfg.n_bodies, cfg.body, cfg.kT)
    return dict(x=x, q=q, P=P, L=L, types=np.zeros(cfg.n_bodies, np.int32))
