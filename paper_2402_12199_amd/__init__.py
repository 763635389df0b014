"""MI355X-native rigid-body pair path: composite-bead sums and a learned pair
energy for molecular dynamics of anisotropic rigid bodies.

The compute path is the HIP library librigidnn.so (C ABI in
include/rigidnn.h); `abi` is its thin Python binding, `md` composes the
entry points into dynamics steps, `nn` drives the network kernels
(autograd wrapper, training loop, data labelling).
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
