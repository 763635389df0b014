"""The five workloads, as concrete seeded parameter sets.

Distances in units of the bead size sigma, energies in epsilon.  Readings of
points the workload statements leave open are explicit fields here:

* lj cut-and-shift shifts the energy only (the force is not shifted);
* the body diameter in the pair cutoff is 2 * r_max (bead-centre
  circumradius), so d_cut = 2 r_max + r_c bounds every interacting pair;
* the body volume for the volume fraction is the bead-centre hull dilated
  by sigma/2;
* overlap rejection at placement is any inter-body bead distance < 1 sigma;
* the network's training minimum is d_min = 2 r_in + sigma.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

from .geometry import BodyType, box_length, make_cube, make_cylinder

LJ_EPS = 1.0
LJ_SIGMA = 1.0
LJ_RC = 2.5


@dataclass
class SystemConfig:
    name: str
    body: BodyType
    n_bodies: int
    phi: float
    seed: int
    kT: float = 1.0
    dt: float = 0.005
    n_steps: int = 0
    skin: float = 1.0
    rc: float = LJ_RC
    eps: float = LJ_EPS
    sigma: float = LJ_SIGMA
    hphc: dict | None = None     # half-power half-cosine parameters (A, b, c, p) instead of LJ
    bead_margin: float | None = None   # two-level list margin for the bead path (None: one level)

    @property
    def box(self) -> float:
        return box_length(self.n_bodies, self.body, self.phi)

    @property
    def d_cut(self) -> float:
        return 2.0 * self.body.r_max + self.rc

    @property
    def r_list(self) -> float:
        return self.d_cut + self.skin

    @property
    def d_min(self) -> float:
        return 2.0 * self.body.r_in + self.sigma


@dataclass
class PairBatchConfig:
    name: str
    body: BodyType
    n_pairs: int
    seed: int
    d_lo_factor: float = 1.0     # d_lo = d_lo_factor * d_min
    rc: float = LJ_RC
    sigma: float = LJ_SIGMA
    dims: tuple = field(default=(7, 128, 128, 128, 128, 1))

    @property
    def d_cut(self) -> float:
        return 2.0 * self.body.r_max + self.rc

    @property
    def d_min(self) -> float:
        return 2.0 * self.body.r_in + self.sigma

    @property
    def d_lo(self) -> float:
        return self.d_lo_factor * self.d_min


def cube5() -> BodyType:
    return make_cube(5)


def cube6() -> BodyType:
    return make_cube(6)


def cyl134() -> BodyType:
    return make_cylinder()


def config1() -> SystemConfig:
    """64 cube shells of 98 beads, volume fraction 0.10, FP64 oracle case."""
    return SystemConfig("cubes64_phi0.10", cube5(), 64, 0.10, seed=1001)


def config2() -> SystemConfig:
    """4096 cube shells of 152 beads, volume fraction 0.20, NVE at kT=1."""
    return SystemConfig("cubes4096_phi0.20", cube6(), 4096, 0.20, seed=1002, n_steps=1000)


def config3() -> PairBatchConfig:
    """2^20 random cylinder pair configurations for the network kernels."""
    return PairBatchConfig("nn_pairs_2^20", cyl134(), 1 << 20, seed=1003, d_lo_factor=1.05)


def config4(n_train: int = 1 << 21, n_test: int = 1 << 16) -> tuple[PairBatchConfig, PairBatchConfig]:
    """Cylinder surrogate training set and a held-out set from another seed."""
    return (PairBatchConfig("cyl_train", cyl134(), n_train, seed=1004),
            PairBatchConfig("cyl_test", cyl134(), n_test, seed=2004))


def config5() -> SystemConfig:
    """32768 cylinders, volume fraction 0.15, NVE at kT=1."""
    return SystemConfig("cyl32768_phi0.15", cyl134(), 32768, 0.15, seed=1005, n_steps=2000, bead_margin=0.4)


# Half-power half-cosine parameters of the paper (section 3), epsilon and sigma units.
HPHC_PAPER = dict(A=0.00035, b=1.46375, c=3.3833, p=2.5)


def config_hphc() -> SystemConfig:
    """4096 cube shells of 152 beads with the paper's half-power half-cosine
    bead potential (its parameters), volume fraction 0.16 (the paper's), NVE
    at kT=1: the surrogate's dynamics against the bead path on a smooth pair
    interaction."""
    return SystemConfig("cubes4096_phi0.16_hphc", cube6(), 4096, 0.16, seed=1006, n_steps=2000,
                        rc=HPHC_PAPER["b"] + math.pi / HPHC_PAPER["c"], hphc=dict(HPHC_PAPER))
