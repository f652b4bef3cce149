"""Pins of the oracle's triclinic cells (lattice vectors the rows of a lower
triangular H), against facts that do not come from the oracle's own formulas:
a crystal's Madelung constant, invariance under a change of lattice basis, an
independent pair enumeration, the orthorhombic special case, SPME converging
to the direct sum, and forces as the negative gradient of the energy."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import ewald as EW
from oracle import pairs as PR
from oracle import spme as SP

MADELUNG_NACL = 1.747564594633182   # rock salt, energy per ion pair -M KE / r0


def lower_triangular(A, B, C):
    """Rotate lattice vectors A, B, C into rows of a lower triangular matrix."""
    A, B, C = (np.asarray(v, np.float64) for v in (A, B, C))
    ax = np.linalg.norm(A)
    ah = A / ax
    bx = B @ ah
    by = np.linalg.norm(np.cross(ah, B))
    cx = C @ ah
    cy = (B @ C - bx * cx) / by
    cz = math.sqrt(C @ C - cx * cx - cy * cy)
    return np.array([[ax, 0, 0], [bx, by, 0], [cx, cy, cz]])


def tric_system(n=24, seed=3, H=None):
    rng = np.random.default_rng(seed)
    if H is None:
        H = np.array([[11.0, 0, 0], [3.1, 10.0, 0], [-2.4, 2.9, 12.0]])
    s = rng.random((n, 3))
    pos = s @ H + rng.normal(0, 3.0, (n, 3))      # some atoms outside the cell
    q = rng.normal(0, 1, n)
    q -= q.mean()
    return pos, q, H


def test_zero_tilt_is_the_orthorhombic_case_bit_for_bit():
    rng = np.random.default_rng(0)
    L = np.array([9.3, 11.7, 10.1])
    pos = rng.normal(0, 20, (60, 3))
    H = np.diag(L)
    assert np.array_equal(EW.wrap(pos, H), EW.wrap(pos, L))
    assert np.array_equal(PR.neighbor_pairs(pos, H, 5.5), PR.neighbor_pairs(pos, L, 5.5))
    q = rng.normal(0, 1, 60)
    a, b = EW.ewald_direct(pos, q, H, 0.4, 5.5, 6), EW.ewald_direct(pos, q, L, 0.4, 5.5, 6)
    assert a["E"] == pytest.approx(b["E"], rel=1e-13)
    assert np.allclose(a["F"], b["F"], rtol=0, atol=1e-11)
    a, b = SP.spme_full(pos, q, H, 0.4, 5.5, 20, 5), SP.spme_full(pos, q, L, 0.4, 5.5, 20, 5)
    assert a["E"] == pytest.approx(b["E"], rel=1e-13)
    assert np.allclose(a["F"], b["F"], rtol=0, atol=1e-11)


def test_wrap_lands_in_the_cell_by_a_lattice_vector():
    pos, _, H = tric_system(200, 5)
    w = EW.wrap(pos, H)
    s = EW.fractional(w, H)
    assert np.all(s > -1e-12) and np.all(s < 1 + 1e-12)
    n = (pos - w) @ np.linalg.inv(H)
    assert np.allclose(n, np.round(n), atol=1e-9)


def test_pairs_match_an_independent_kd_tree_enumeration():
    pos, _, H = tric_system(80, 7)
    cut = 6.5
    P = PR.neighbor_pairs(pos, H, cut)
    # independent: every atom's images over a block of cells, found by a k-d tree
    w = EW.wrap(pos, H)
    R = 2
    shifts = np.array([(a, b, c) for a in range(-R, R + 1) for b in range(-R, R + 1) for c in range(-R, R + 1)])
    img = (w[None, :, :] + (shifts @ H)[:, None, :]).reshape(-1, 3)
    tree = cKDTree(img)
    ref = set()
    for i in range(len(w)):
        for k in tree.query_ball_point(w[i], cut):
            si, j = divmod(k, len(w))
            n = tuple(shifts[si])
            if j == i and n == (0, 0, 0):
                continue
            if i < j or (i == j and n > (0, 0, 0)):
                ref.add((i, j) + n)
            elif j < i:
                ref.add((j, i) + tuple(-np.array(n)))
            elif i == j:
                ref.add((i, j) + tuple(-np.array(n)))
    assert set(map(tuple, P.tolist())) == ref


def nacl_primitive(a0=5.64):
    H = lower_triangular(np.array([0, 0.5, 0.5]) * a0, np.array([0.5, 0, 0.5]) * a0,
                         np.array([0.5, 0.5, 0]) * a0)
    pos = np.array([[0.0, 0.0, 0.0], 0.5 * (H[0] + H[1] + H[2])])
    return pos, np.array([1.0, -1.0]), H, a0 / 2


def test_nacl_primitive_cell_madelung_constant():
    pos, q, H, r0 = nacl_primitive()
    E = EW.ewald_direct(pos, q, H, 0.6, 9.0, 14)["E"]
    assert E == pytest.approx(-MADELUNG_NACL * EW.KE / r0, rel=1e-9)
    Es = SP.spme_full(pos, q, H, 0.6, 9.0, 32, 8)["E"]
    assert Es == pytest.approx(-MADELUNG_NACL * EW.KE / r0, rel=1e-6)


def test_change_of_lattice_basis_changes_nothing():
    pos, q, H = tric_system(20, 11)
    H2 = np.array([H[0], H[1] + H[0], H[2] + H[1]])    # same lattice, other basis
    a = EW.ewald_direct(pos, q, H, 0.35, 9.5, 12)
    b = EW.ewald_direct(pos, q, H2, 0.35, 9.5, 16)
    assert a["E"] == pytest.approx(b["E"], rel=1e-10)
    assert np.allclose(a["phi"], b["phi"], rtol=0, atol=1e-9)
    assert np.allclose(a["F"], b["F"], rtol=0, atol=1e-9)


def test_spme_converges_to_the_direct_sum():
    pos, q, H = tric_system(30, 13)
    ref = EW.ewald_direct(pos, q, H, 0.38, 5.5, 14)
    got = SP.spme_full(pos, q, H, 0.38, 5.5, 48, 8)
    assert got["E"] == pytest.approx(ref["E"], rel=1e-7)
    assert np.abs(got["phi"] - ref["phi"]).max() < 1e-6 * np.abs(ref["phi"]).max()
    assert np.abs(got["F"] - ref["F"]).max() < 1e-5 * np.abs(ref["F"]).max()


@pytest.mark.parametrize("method", ["ewald", "pme"])
def test_forces_are_minus_the_energy_gradient(method):
    pos, q, H = tric_system(12, 17)
    h = 1e-5

    def run(p):
        if method == "ewald":
            return EW.ewald_direct(p, q, H, 0.4, 5.0, 9)
        return SP.spme_full(p, q, H, 0.4, 5.0, 24, 6)

    F = run(pos)["F"]
    for i, k in [(0, 0), (3, 1), (7, 2), (11, 0)]:
        pp, pm = pos.copy(), pos.copy()
        pp[i, k] += h
        pm[i, k] -= h
        fd = -(run(pp)["E"] - run(pm)["E"]) / (2 * h)
        assert fd == pytest.approx(F[i, k], rel=1e-5, abs=1e-6)
