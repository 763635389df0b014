"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct FP64 CPU implementation of everything the
rigid-body pair path computes, written from the paper's statement of the
method and from textbook definitions.  It shares no code with the HIP
library: only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it, and the product path must never route through it.

Modules
  beads   ctypes front end of bead.c: bead double sum, brute-force pair
          search, rigid-body integrator, NVE driver
  frames  pair descriptors (separation in body i's frame, relative
          quaternion) and forces/torques from the gradient of a pair energy
          written in those descriptors
  mlp     the energy network: forward pass, input gradient, parameter
          gradient of the training loss, Adam
  thermostat  Nose-Hoover constant-temperature steps around the integrator
  symmetry    the symmetry-reduced descriptor of a cube pair, its inverse
              and its Jacobian
"""
from . import beads, frames, mlp, symmetry, thermostat  # noqa: F401
