"""Comparison rules of the parity tests.

Per element, a value v (scalar or 3-vector) passes when
    |v_gpu - v_ref| <= rtol * max(|v_ref|, rms(v_ref over the batch))
so entries near zero are judged against the batch's typical size rather
than against themselves; the relative error of the whole batch
(Frobenius norm) must pass the same rtol.  rtol: 1e-5 for FP32 bead energies,
1e-4 for FP32 bead forces/torques, 2e-2 for the BF16 network against the
FP64 network with the same weights.
"""
import numpy as np


def _norms(a):
    a = np.asarray(a, dtype=np.float64)
    return np.abs(a) if a.ndim == 1 else np.linalg.norm(a, axis=-1)


def assert_close(got, ref, rtol, what="value"):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, f"{what}: shape {got.shape} vs {ref.shape}"
    err = _norms(got - ref)
    rn = _norms(ref)
    rms = np.sqrt(np.mean(rn ** 2)) if rn.size else 0.0
    bound = rtol * np.maximum(rn, rms)
    bad = err > bound
    if bad.any():
        k = int(np.argmax(err / np.maximum(bound, 1e-300)))
        raise AssertionError(
            f"{what}: {int(bad.sum())}/{bad.size} outside rtol={rtol}; worst index {k}: "
            f"got {got[k]} ref {ref[k]} err {err[k]:.3e} bound {bound[k]:.3e}")
    tot = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert tot <= rtol, f"{what}: batch relative error {tot:.3e} > {rtol}"


def max_rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rn = _norms(ref)
    rms = np.sqrt(np.mean(rn ** 2)) if rn.size else 1.0
    return float(np.max(_norms(got - ref) / np.maximum(rn, rms)))
