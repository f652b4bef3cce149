"""Pins of the FP64 smooth-PME oracle (no GPU)."""
import math

import numpy as np

import oracle as O
import workloads as W
from oracle import spme as S


def test_bspline_integer_values_are_eulerian_numbers():
    # M_p(k) for k = 1..p-1 equals the Eulerian numbers A(p-1, k-1) / (p-1)!
    eul = {4: [1, 4, 1], 5: [1, 11, 11, 1], 6: [1, 26, 66, 26, 1]}
    for p, e in eul.items():
        vals = S.bspline(p, np.arange(1, p, dtype=float))
        assert np.allclose(vals, np.array(e) / math.factorial(p - 1), rtol=0, atol=1e-15)


def test_bspline_partition_of_unity_support_and_derivative():
    x = np.linspace(0.0, 1.0, 37)
    for p in (3, 4, 5, 6, 8):
        tot = sum(S.bspline(p, x + t) for t in range(p))
        assert np.abs(tot - 1.0).max() < 1e-14
        assert S.bspline(p, np.array([-0.3, p + 0.2])).max() == 0.0
        h = 1e-6
        xs = np.linspace(0.1, p - 0.1, 29) + 0.0137   # off the integer knots
        fd = (S.bspline(p, xs + h) - S.bspline(p, xs - h)) / (2 * h)
        assert np.abs(fd - S.bspline_deriv(p, xs)).max() < 1e-8
    # integral of M_p over its support is 1
    xs = np.linspace(0, 6, 600001)
    assert abs(np.trapezoid(S.bspline(6, xs), xs) - 1.0) < 1e-9


def test_euler_factor_odd_order_even_grid():
    # p = 5, even K: the m = K/2 denominator vanishes and is replaced by the
    # mean of its neighbours, which are equal by symmetry
    b = S.euler_factors(16, 5)
    assert np.isfinite(b).all()
    assert abs(b[8] - b[7]) < 1e-12 and abs(b[7] - b[9]) < 1e-12


def test_pme_converges_to_ewald():
    s = W.small_random(40, 12.0, seed=21)
    a, rc = 0.45, 6.0
    ref = O.ewald_direct(s.pos, s.q, s.box, a, rc, 14)
    errs = []
    for K in (12, 16, 24, 32):
        p = O.spme_full(s.pos, s.q, s.box, a, rc, K, 6)
        errs.append(np.abs(p["phi_rec"] - ref["phi_rec"]).max())
        assert abs(p["E_rec"] - 0.5 * s.q @ p["phi_rec"]) < 1e-10 * abs(p["E_rec"]) + 1e-12
    assert all(errs[i + 1] < errs[i] for i in range(3))
    assert errs[-1] < 1e-6 * np.abs(ref["phi_rec"]).max()
    # higher order at a fixed grid is more accurate too
    e4 = np.abs(O.spme_reciprocal(s.pos, s.q, s.box, a, 16, 4)[0] - ref["phi_rec"]).max()
    e8 = np.abs(O.spme_reciprocal(s.pos, s.q, s.box, a, 16, 8)[0] - ref["phi_rec"]).max()
    assert e8 < e4


def test_pme_nacl_matches_madelung():
    s = W.nacl()
    p = O.spme_full(s.pos, s.q, s.box, 0.35, 8.0, 32, 4)
    M = -float(np.mean(s.q * p["phi"])) * 2.82 / O.KE
    assert abs(M / 1.747564594633 - 1) < 1.5e-4


def test_pme_force_is_minus_gradient_of_rec_energy():
    s = W.small_random(16, 9.0, seed=22)
    a, K, p = 0.4, 20, 5
    _, F, _ = O.spme_reciprocal(s.pos, s.q, s.box, a, K, p)
    h = 1e-6
    for k in (0, 7, 20, 47):
        pp = s.pos.reshape(-1).copy()
        pm = pp.copy()
        pp[k] += h
        pm[k] -= h
        g = (O.spme_reciprocal(pp.reshape(-1, 3), s.q, s.box, a, K, p)[2]
             - O.spme_reciprocal(pm.reshape(-1, 3), s.q, s.box, a, K, p)[2]) / (2 * h)
        assert abs(-g - F.reshape(-1)[k]) < 1e-6 * max(1.0, abs(g))


def test_pme_potential_is_charge_gradient():
    s = W.small_random(16, 9.0, seed=23)
    a, K, p = 0.4, 20, 6
    phi, _, _ = O.spme_reciprocal(s.pos, s.q, s.box, a, K, p)
    h = 1e-6
    for i in (0, 9, 15):
        qp, qm = s.q.copy(), s.q.copy()
        qp[i] += h
        qm[i] -= h
        g = (O.spme_reciprocal(s.pos, qp, s.box, a, K, p)[2]
             - O.spme_reciprocal(s.pos, qm, s.box, a, K, p)[2]) / (2 * h)
        assert abs(g - phi[i]) < 1e-7 * max(1.0, abs(g))


def test_pme_translation_by_grid_vector_is_exact():
    s = W.small_random(20, 10.0, seed=24)
    K = 20
    shift = np.array([3, -7, 11]) * (10.0 / K)   # whole grid cells
    a = O.spme_reciprocal(s.pos, s.q, s.box, 0.4, K, 5)
    b = O.spme_reciprocal(s.pos + shift, s.q, s.box, 0.4, K, 5)
    assert np.abs(a[0] - b[0]).max() < 1e-10
    assert np.abs(a[1] - b[1]).max() < 1e-10
