"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *generates inputs*: bead templates of the workload shapes,
random body placements, random orientations, random momenta, random pair
configurations and random network weights.  It holds none of the method's
arithmetic (no bead-pair energy, no descriptor, no network evaluation, no
integration step), so the oracle and the HIP path can both draw from it
without sharing any computation.
"""
from . import geometry, sampling, configs  # noqa: F401
