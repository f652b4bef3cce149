"""Pins of the dense QEQ / shadow-step / gradient oracle (no GPU)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import grad as G
from oracle import qeq as Q

COUL = dict(method="ewald", alpha=0.5, rc=9.0, kmax=11)


@pytest.fixture(scope="module")
def small():
    s = W.small_random(14, 8.0, seed=31)
    A = Q.coulomb_matrix(s.pos, s.box, COUL)
    return s, A


def test_matrix_matches_matrix_free_product(small):
    s, A = small
    v = np.random.default_rng(1).normal(size=s.n)
    assert np.abs(A @ v - Q.potential(s.pos, v, s.box, COUL)).max() < 1e-10 * np.abs(A @ v).max()
    # the diagonal carries the periodic self-interaction: for one charge alone
    # in a cubic box it is KE * (-2.837297479 / L)
    one = Q.coulomb_matrix(s.pos[:1], s.box, COUL)
    assert abs(one[0, 0] / (O.KE * -2.837297479 / 8.0) - 1) < 1e-8


def test_qeq_dense_solution_properties(small):
    s, A = small
    q, lam = Q.qeq_dense(A, s.chi, s.eta, 0.7)
    assert abs(q.sum() - 0.7) < 1e-12
    assert Q.bordered_residual(A, s.chi, s.eta, 0.7, q, lam) < 1e-13
    # stationarity: chi + u q + A q + lambda = 0 (electronegativity equalisation)
    assert np.abs(s.chi + s.eta * q + A @ q + lam).max() < 1e-11


def test_qeq_two_atom_closed_form():
    s = W.small_random(2, 7.0, seed=32)
    A = Q.coulomb_matrix(s.pos, s.box, COUL)
    q, _ = Q.qeq_dense(A, s.chi, s.eta, 0.0)
    C = A + np.diag(s.eta)
    q1 = (s.chi[1] - s.chi[0]) / (C[0, 0] + C[1, 1] - 2 * C[0, 1])
    assert abs(q[0] - q1) < 1e-12 and abs(q[1] + q1) < 1e-12


def test_shadow_fixed_point_and_energy(small):
    s, A = small
    qstar, lam = Q.qeq_dense(A, s.chi, s.eta, 0.0)
    qn, lamn = Q.shadow_charges(A @ qstar, s.chi, s.eta, 0.0)
    assert np.abs(qn - qstar).max() < 1e-12 and abs(lamn - lam) < 1e-10
    # the shadow energy equals the regular energy at n = q*
    assert abs(Q.shadow_energy(A, s.chi, s.eta, qn, qstar) - Q.qeq_energy(A, s.chi, s.eta, qstar)) < 1e-10
    # q[n] is always neutral and minimises the shadow energy on sum q = 0
    n = qstar + np.random.default_rng(2).normal(0, 0.05, s.n)
    qn, _ = Q.shadow_charges(A @ n, s.chi, s.eta, 0.0)
    assert abs(qn.sum()) < 1e-12
    d = np.random.default_rng(3).normal(size=s.n)
    d -= d.mean()
    e0 = Q.shadow_energy(A, s.chi, s.eta, qn, n)
    assert Q.shadow_energy(A, s.chi, s.eta, qn + 1e-3 * d, n) > e0
    assert Q.shadow_energy(A, s.chi, s.eta, qn - 1e-3 * d, n) > e0


def test_jacobian_matches_finite_difference(small):
    s, A = small
    J = Q.jacobian(A, s.eta)
    n0 = np.random.default_rng(4).normal(0, 0.3, s.n)
    h = 1e-6

    def resid(n):
        return Q.shadow_charges(A @ n, s.chi, s.eta, 0.0)[0] - n
    for j in (0, 5, 13):
        e = np.zeros(s.n)
        e[j] = h
        fd = (resid(n0 + e) - resid(n0 - e)) / (2 * h)
        assert np.abs(fd - J[:, j]).max() < 1e-7


def test_gmres_iterate_definition(small):
    s, A = small
    J = Q.jacobian(A, s.eta)
    b = np.random.default_rng(5).normal(size=s.n)
    # full Krylov dimension: the exact solution
    x = Q.gmres_iterate(lambda y: J @ y, b, s.n)
    assert np.abs(J @ x - b).max() < 1e-9 * np.abs(b).max()
    # m < N: least squares over an explicit (power) Krylov basis gives the same iterate
    m = 5
    Kr = np.stack([np.linalg.matrix_power(J, i) @ b for i in range(m)], 1)
    c, *_ = np.linalg.lstsq(J @ Kr, b, rcond=None)
    assert np.abs(Q.gmres_iterate(lambda y: J @ y, b, m) - Kr @ c).max() < 1e-8 * np.abs(Kr @ c).max()


def test_energy_gradient_envelope_vs_finite_differences():
    # separations >= 3 A keep C = diag(u) + A well conditioned (KE/r < min u)
    s = W.small_random(6, 9.0, seed=33, dmin=3.0)
    E, q, dR, dchi, deta = G.qeq_energy_and_grad(s.pos, s.box, COUL, s.chi, s.eta)

    def e_of_pos(p):
        return G.qeq_energy_and_grad(p, s.box, COUL, s.chi, s.eta)[0]

    def e_of_chi(c):
        return G.qeq_energy_and_grad(s.pos, s.box, COUL, c, s.eta)[0]

    def e_of_eta(u):
        return G.qeq_energy_and_grad(s.pos, s.box, COUL, s.chi, u)[0]
    idx = [0, 4, 8, 17]
    assert np.abs(G.central_difference(e_of_pos, s.pos, 1e-4, idx) - dR.reshape(-1)[idx]).max() < 1e-6
    assert np.abs(G.central_difference(e_of_chi, s.chi, 1e-4, [0, 3]) - dchi[[0, 3]]).max() < 1e-8
    assert np.abs(G.central_difference(e_of_eta, s.eta, 1e-4, [1, 5]) - deta[[1, 5]]).max() < 1e-8


def test_vjp_vs_finite_differences():
    s = W.small_random(6, 9.0, seed=34, dmin=3.0)
    g = np.random.default_rng(6).normal(size=s.n)

    def loss(pos=s.pos, chi=s.chi, eta=s.eta):
        A = Q.coulomb_matrix(pos, s.box, COUL)
        return float(g @ Q.qeq_dense(A, chi, eta, 0.0)[0])
    dR, dchi, deta = G.qeq_vjp(s.pos, s.box, COUL, s.chi, s.eta, g)
    idx = [1, 6, 11]
    fdR = G.central_difference(lambda p: loss(pos=p), s.pos, 1e-4, idx)
    assert np.abs(fdR - dR.reshape(-1)[idx]).max() < 1e-6 * max(1, np.abs(fdR).max())
    assert np.abs(G.central_difference(lambda c: loss(chi=c), s.chi, 1e-5, [0, 2]) - dchi[[0, 2]]).max() < 1e-8
    assert np.abs(G.central_difference(lambda u: loss(eta=u), s.eta, 1e-5, [3, 4]) - deta[[3, 4]]).max() < 1e-8


def test_blocked_matrix_equals_column_by_column():
    s = W.small_random(37, 7.5, seed=35)
    for coul in (COUL, dict(method="pme", alpha=0.45, rc=7.0, grid=15, order=5)):
        A1 = Q.coulomb_matrix(s.pos, s.box, coul)
        A2 = Q.coulomb_matrix_blocked(s.pos, s.box, coul, chunk=8)
        assert np.abs(A1 - A2).max() < 1e-10 * np.abs(A1).max()
