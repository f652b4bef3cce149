"""Pins of the brute-force canonical neighbour set (no GPU)."""
import itertools
import math

import numpy as np

import oracle as O
import workloads as W


def _loops(pos, box, cut):
    """Pure-Python definition on tiny inputs: every (i, j, n), canonical orientation."""
    w = O.wrap(pos, box)
    m = [int(math.ceil(cut / L)) for L in box]
    out = []
    for i in range(len(w)):
        for j in range(i, len(w)):
            for n in itertools.product(*(range(-k, k + 1) for k in m)):
                if i == j and not (n > (0, 0, 0)):
                    continue
                d = [(w[j][a] - w[i][a]) + n[a] * box[a] for a in range(3)]
                if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < cut * cut:
                    out.append((i, j) + tuple(n))
    return sorted(out)


def test_pairs_match_python_loops_tiny_and_multi_image():
    for (n, L, cut, seed) in [(7, 6.0, 2.5, 1), (9, 5.0, 6.2, 2), (5, 3.0, 4.0, 3)]:
        s = W.small_random(n, L, seed=seed, dmin=0.3)
        P = O.neighbor_pairs(s.pos, s.box, cut)
        assert [tuple(r) for r in P] == _loops(s.pos, s.box, cut)


def test_pairs_match_kdtree_minimum_image():
    from scipy.spatial import cKDTree
    s = W.small_random(600, 20.0, seed=4)
    cut = 6.0
    P = O.neighbor_pairs(s.pos, s.box, cut)
    w = O.wrap(s.pos, s.box)
    ref = cKDTree(w, boxsize=20.0).query_pairs(cut, output_type="ndarray")
    got = {(int(a), int(b)) for a, b in P[:, :2]}
    want = {(min(a, b), max(a, b)) for a, b in ref}
    assert got == want
    assert len(P) == len(got)        # one image per pair when cut < L/2


def test_pair_count_matches_density_estimate():
    s = W.random_ionic(n=2000, seed=5, grid=None)
    P = O.neighbor_pairs(s.pos, s.box, 10.0)
    # half pairs ~ N/2 * rho * 4/3 pi rc^3 (uniform density), within sampling noise
    est = 0.5 * 2000 * 0.1 * 4.0 / 3.0 * math.pi * 1000.0
    assert abs(len(P) / est - 1) < 0.03
