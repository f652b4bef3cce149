"""Per-element parity measures shared by the GPU tests.

The norm checks (relative L2 of phi, relative RMS of the force vectors) can
hide one bad atom among thousands; these bound every element. An element's
error is taken relative to the RMS magnitude of the reference (a potential or
force near zero makes its own relative error meaningless):
  max_i |a_i - b_i| / rms(b)        for per-atom scalars,
  max_i ||a_i - b_i|| / rms(||b||)  for per-atom vectors.
"""
import numpy as np


def elem_err(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.ndim == 1:
        return float(np.abs(a - b).max() / np.sqrt(np.mean(b * b)))
    d = np.sqrt(np.sum((a - b) ** 2, axis=1))
    return float(d.max() / np.sqrt(np.mean(np.sum(b * b, axis=1))))
