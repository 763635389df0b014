"""The C-ABI library loads and exports every entry point the header declares,
and argument checks that run before any device work report errors.  No
compute call is made here (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rigidnn.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for want in ("rb_pairlist_build", "rb_bead_pair_eval", "rb_nn_pair_eval", "rb_nn_pair_grad",
                 "rb_rigid_step", "rb_nn_train_step", "rb_pair_descriptors", "rb_bead_pair_forces",
                 "rb_nn_pair_forces", "rb_accum_finalize"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2402_12199_amd import _lib
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) <= set(_lib.SIGNATURES)


def test_host_side_argument_errors():
    from paper_2402_12199_amd import _lib
    L = _lib.lib()
    h = C.c_void_p()
    nb = (C.c_int32 * 1)(0)
    rc = L.rb_ctx_create(C.byref(h), 1, nb, None, None, None, 1.0, 1.0, 2.5)
    assert rc == -1
    assert b"null" in L.rb_last_error() or b"beads" in L.rb_last_error()
    box = (C.c_double * 3)(10.0, 10.0, 10.0)
    # box smaller than 2 r_list: no valid cell grid
    assert L.rb_pairlist_workspace_bytes(100, box, 6.0) == 0
    assert L.rb_pairlist_workspace_bytes(100, box, 4.0) > 0
    assert L.rb_rigid_workspace_bytes(1000) >= 16 * 4


def test_flags_check_reports_device_conditions():
    # rb_flags_check is a host function over a host copy of the flag array:
    # each device-reported condition maps to its status code and message
    from paper_2402_12199_amd import abi
    f = np.zeros(abi.RB_NFLAGS, np.int32)
    f[abi.RB_FLAG_NPAIRS] = 123
    f[abi.RB_FLAG_NEVAL] = 99
    assert abi.rb_flags_check(f) == (abi.RB_OK, "")
    cases = [(abi.RB_FLAG_OVERFLOW, 5000, abi.RB_ERR_CAPACITY, "overflow"),
             (abi.RB_FLAG_NONFINITE, 1, abi.RB_ERR_NONFINITE, "non-finite"),
             (abi.RB_FLAG_FIXOVF, 1, abi.RB_ERR_NONFINITE, "fixed-point"),
             (abi.RB_FLAG_QDRIFT, 3, abi.RB_ERR_NONFINITE, "quaternion")]
    for k, v, rc, word in cases:
        g = f.copy()
        g[k] = v
        got, msg = abi.rb_flags_check(g)
        assert got == rc and word in msg, (k, got, msg)
    assert abi.RB_ERR_NONFINITE == -5
