"""Pins of the FP64 shadow-MD oracle (oracle/md.py): the V_short stand-in
against closed forms and finite differences, the dissipation coefficients,
uniform motion, and the second order of the velocity-Verlet energy error."""
import numpy as np
import pytest

import workloads as W
from oracle import md as M

COUL = dict(method="ewald", alpha=0.35, rc=6.0, kmax=5)


def test_short_range_two_atoms_closed_form():
    box = np.array([50.0, 50.0, 50.0])
    pos = np.array([[10.0, 10.0, 10.0], [11.3, 10.4, 9.8]])
    A, rho, rc = 300.0, 0.3, 6.0
    F, E = M.short_range(pos, box, rc, A, rho)
    d = pos[1] - pos[0]
    r = np.linalg.norm(d)
    assert abs(E - A * np.exp(-r / rho)) < 1e-13 * E
    f1 = A / rho * np.exp(-r / rho) * d / r      # pushes atom 1 away from atom 0
    assert np.allclose(F[1], f1, rtol=1e-12) and np.allclose(F[0], -f1, rtol=1e-12)


def test_short_range_force_is_minus_gradient():
    s = W.small_random(20, (20 / 0.1) ** (1 / 3), seed=3)   # L = 5.85 A < 2 rc: own images count
    A, rho, rc = 200.0, 0.4, 4.0
    F, _ = M.short_range(s.pos, s.box, rc, A, rho)
    h = 1e-5
    for i, d in [(0, 0), (3, 1), (7, 2), (11, 0)]:
        p1, p2 = s.pos.copy(), s.pos.copy()
        p1[i, d] += h
        p2[i, d] -= h
        fd = -(M.short_range(p1, s.box, rc, A, rho)[1] - M.short_range(p2, s.box, rc, A, rho)[1]) / (2 * h)
        assert abs(fd - F[i, d]) < 1e-6 * (1 + abs(F[i, d]))


def test_dissipation_coefficients_keep_constant_and_linear_histories():
    kappa, alpha, c = M.XL5
    k = np.arange(len(c))
    assert sum(c) == 0.0 and float(np.dot(k, c)) == 0.0


def test_uniform_motion_without_forces():
    # no charges and no repulsion: every force vanishes and R advances by dt v
    s = W.small_random(16, (16 / 0.1) ** (1 / 3), seed=4)
    n = s.n
    rng = np.random.default_rng(0)
    vel = rng.normal(0, 3e-3, (n, 3))
    hist = np.zeros((2, n))
    pos, vel2, _, e = M.md_run(s.pos, vel, np.full(n, 20.0), s.box, COUL, np.zeros(n), np.full(n, 20.0), hist, 4,
                               dt=0.5, dissipation=0, kappa=1.9)
    assert np.allclose(pos, s.pos + 4 * 0.5 * vel, rtol=0, atol=1e-13)
    assert np.array_equal(vel2, vel)
    assert np.allclose(e[:, 3], e[0, 3], rtol=1e-14)


def test_verlet_energy_error_is_second_order():
    # repulsion only (no charges): E_tot fluctuates as dt^2
    s = W.small_random(24, (24 / 0.1) ** (1 / 3), seed=6)
    n = s.n
    rng = np.random.default_rng(1)
    vel = rng.normal(0, 2e-2, (n, 3))
    mass = np.full(n, 20.0)
    dev = []
    for dt, steps in ((1.0, 40), (0.5, 80)):
        *_, e = M.md_run(s.pos, vel, mass, s.box, COUL, np.zeros(n), np.full(n, 20.0), np.zeros((2, n)), steps,
                         dt=dt, dissipation=0, kappa=1.9, rep_a=100.0, rep_rho=0.4)
        dev.append(np.max(np.abs(e[:, 3] - e[0, 3])))
    ratio = dev[0] / dev[1]
    assert 3.0 < ratio < 5.0, ratio


def test_shadow_step_at_the_ground_state_is_regular_bo():
    # n = q*: q[n] = q*, the shadow force is F[q*] and the shadow energy the QEQ energy
    s = W.small_random(24, (24 / 0.1) ** (1 / 3), seed=8)
    eta = np.random.default_rng(2).uniform(20.0, 25.0, s.n)
    F, E, _, q = M.regular_state(s.pos, s.box, COUL, s.chi, eta, 0.0)
    Fs, x, Es, _, qs = M.shadow_state(s.pos, s.box, COUL, s.chi, eta, 0.0, q, 4)
    assert np.allclose(qs, q, rtol=0, atol=1e-12)
    assert np.allclose(Fs, F, rtol=1e-10, atol=1e-12)
    assert abs(Es - E) < 1e-10 * abs(E)
    assert np.abs(x).max() < 1e-9


def test_shadow_force_is_minus_gradient_of_shadow_energy_at_fixed_n():
    # Away from the ground state (n != q*) the shadow force at fixed n is
    # -dU/dR of the shadow energy U(R, n) = E(R, q[n](R), n) (eq. qeq_energy
    # with the linearised Coulomb term); q[n] is recomputed at every probe, so
    # this also checks that its R-dependence drops out (the stationarity of
    # q[n] under the charge constraint). Central differences, h = 1e-5 A.
    s = W.small_random(12, (12 / 0.1) ** (1 / 3), seed=21)
    rng = np.random.default_rng(5)
    eta = rng.uniform(20.0, 25.0, s.n)
    _, _, _, qstar = M.regular_state(s.pos, s.box, COUL, s.chi, eta, 0.0)
    n_vec = qstar + rng.normal(0.0, 0.15, s.n)
    n_vec -= n_vec.mean()

    def energy(p):
        return M.shadow_state(p, s.box, COUL, s.chi, eta, 0.0, n_vec, 1)[2]

    F, _, _, _, q = M.shadow_state(s.pos, s.box, COUL, s.chi, eta, 0.0, n_vec, 1)
    assert np.abs(q - n_vec).max() > 0.05          # genuinely off the ground state
    h = 1e-5
    fd = np.zeros((s.n, 3))
    for i in range(s.n):
        for d in range(3):
            p1, p2 = s.pos.copy(), s.pos.copy()
            p1[i, d] += h
            p2[i, d] -= h
            fd[i, d] = -(energy(p1) - energy(p2)) / (2 * h)
    scale = np.abs(F).max()
    assert np.abs(fd - F).max() < 1e-6 * scale, (np.abs(fd - F).max(), scale)


def test_charged_shadow_md_conserves_energy_to_second_order():
    # Charged NVE run of the full shadow loop (velocity Verlet on the shadow
    # potential, extended-charge Verlet step with K = 5 dissipation): the
    # total shadow energy fluctuates as dt^2, and the extended charges n stay
    # close to q[n] (eq. Jnddot drives n towards the ground state).
    s = W.small_random(16, (16 / 0.1) ** (1 / 3), seed=23)
    n = s.n
    rng = np.random.default_rng(7)
    eta = rng.uniform(20.0, 25.0, n)
    vel = rng.normal(0, 1e-2, (n, 3))
    mass = np.full(n, 20.0)
    _, _, _, q0 = M.regular_state(s.pos, s.box, COUL, s.chi, eta, 0.0)
    hist = np.tile(q0, (M.history_length(5), 1))
    dev = []
    for dt, steps in ((1.0, 30), (0.5, 60)):
        pos, _, h, e = M.md_run(s.pos, vel, mass, s.box, COUL, s.chi, eta, hist, steps, dt=dt, n_krylov=4,
                                dissipation=5, rep_a=100.0, rep_rho=0.4)
        dev.append(np.max(np.abs(e[:, 3] - e[0, 3])))
        _, _, _, qs = M.regular_state(pos, s.box, COUL, s.chi, eta, 0.0)
        assert np.abs(h[0] - qs).max() < 2e-3, np.abs(h[0] - qs).max()
    ratio = dev[0] / dev[1]
    assert 3.0 < ratio < 5.0, (ratio, dev)
