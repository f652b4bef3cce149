"""Canonical neighbour pair set by brute force (oracle; test infrastructure only).

Section "Cell based Neighbor List" of the paper builds, with cells, the set of
atom pairs closer than a cutoff under periodic boundaries; the set itself has a
plain definition, which is what this computes:

  (i, j, n) is a pair iff  d = (w_j - w_i) + n*L  has  d.d < cut^2,
  (triclinic cells: n*L becomes the lattice vector n H, summed as image_offsets
  states)
  w = canonical wrap of the FP64 positions, d.d = dx*dx + dy*dy + dz*dz
  evaluated left to right in FP64 without fused multiply-add, and
  (i, j, n) != (i, i, 0).

Every unordered pair is listed once: (i < j, n), or (i, i, n) with n
lexicographically positive for an atom and its own image. All periodic images
with |n_d| <= ceil(cut/w_d) are considered (w_d the distance between opposite
faces of the cell), so boxes smaller than twice the
cutoff are covered.
"""
from __future__ import annotations

import numpy as np

from .ewald import image_offsets, image_shifts, wrap


def neighbor_pairs(pos, box, cut, chunk_elems=4_000_000) -> np.ndarray:
    """Sorted int64 array (npairs, 5) of rows (i, j, n0, n1, n2)."""
    w = wrap(np.asarray(pos, np.float64), box)
    n = len(w)
    shifts = image_shifts(box, cut)
    sL = image_offsets(shifts, box)
    cut2 = cut * cut
    pos_shift = (shifts[:, 0] > 0) | ((shifts[:, 0] == 0) & (shifts[:, 1] > 0)) | \
                ((shifts[:, 0] == 0) & (shifts[:, 1] == 0) & (shifts[:, 2] > 0))
    out = []
    step = max(1, chunk_elems // max(1, n * len(shifts)))
    jj = np.arange(n)
    for s in range(0, n, step):
        I = np.arange(s, min(n, s + step))
        dd = (w[None, :, :] - w[I][:, None, :])[:, :, None, :] + sL[None, None, :, :]
        r2 = dd[..., 0] * dd[..., 0] + dd[..., 1] * dd[..., 1] + dd[..., 2] * dd[..., 2]
        keep = r2 < cut2
        keep &= (I[:, None, None] < jj[None, :, None]) | \
                ((I[:, None, None] == jj[None, :, None]) & pos_shift[None, None, :])
        b, j, si = np.nonzero(keep)
        if len(b):
            out.append(np.concatenate([I[b][:, None], j[:, None], shifts[si]], 1))
    if not out:
        return np.zeros((0, 5), np.int64)
    P = np.concatenate(out, 0).astype(np.int64)
    order = np.lexsort((P[:, 4], P[:, 3], P[:, 2], P[:, 1], P[:, 0]))
    return P[order]
