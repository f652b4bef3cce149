"""Per-element parity measures shared by the GPU tests, and the ELLPACK rows of a pair list.

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


def ell_from_pairs(pairs, n):
    """ELLPACK rows built on the host from a pair list: (i, j, v) is the
    neighbour (j, v) of row i and (i, -v) of row j; rows in ascending
    (j, v0, v1, v2) order."""
    fwd = np.concatenate([pairs[:, :2], pairs[:, 2:]], 1)
    bwd = np.concatenate([pairs[:, 1:2], pairs[:, 0:1], -pairs[:, 2:]], 1)
    e = np.concatenate([fwd, bwd], 0)
    e = e[np.lexsort((e[:, 4], e[:, 3], e[:, 2], e[:, 1], e[:, 0]))]
    cnt = np.bincount(e[:, 0], minlength=n)
    K = int(cnt.max()) if len(e) else 0
    nbr = -np.ones((n, K), np.int64)
    img = np.zeros((n, K, 3), np.int64)
    start = np.concatenate([[0], np.cumsum(cnt)])
    col = np.arange(len(e)) - start[e[:, 0]]
    nbr[e[:, 0], col] = e[:, 1]
    img[e[:, 0], col] = e[:, 2:]
    return nbr, img, cnt
