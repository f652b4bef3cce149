"""Shadow Born-Oppenheimer (XL-BOMD) molecular dynamics in FP64 (oracle; test
infrastructure only).

Section "Shadow Born-Oppenheimer MD for a Charge Equilibration Model": the
atoms move on the shadow potential U(R, n) = V_short(R) + E(R, q[n], n) with
the force taken at fixed n, and the extended charges follow
n'' = -omega^2 K (q[n] - n), whose right-hand side is x, the m-step GMRES
iterate for J x = -(q[n] - n) (eq. Jnddot, omega^2 = 1).

Step, in the order the library takes it (units A, fs, amu, eV):
  v += dt/2 F/m;  R += dt v;
  n(t+dt) = 2 n(t) - n(t-dt) + kappa x(t) + alpha sum_k c_k n(t - k dt);
  at (R, n)(t+dt): F, x and the shadow energy;  v += dt/2 F/m.
The n step is the Verlet step of extended-Lagrangian BOMD; with dissipation
it is the K = 5 scheme of Niklasson et al. (J. Chem. Phys. 130, 214109,
2009): kappa = 1.82, alpha = 0.018, c = (-6, 14, -8, -3, 4, -1).

V_short, the paper's trained short-range model, is replaced by a repulsive
pair term A exp(-r/rho) over every pair and periodic image closer than the
cutoff (the library uses the same stand-in).

The Coulomb operator is applied matrix-free through the oracle's potential
and force functions: v = A n, the products J y = -y - P D^-1 A y inside the
GMRES iterate, and F[q] - F[q - n].
"""
from __future__ import annotations

import numpy as np

from . import qeq as Q
from .ewald import wrap

ACC = 9.648533212331e-3          # (eV/A)/amu in A/fs^2
XL5 = (1.82, 0.018, (-6.0, 14.0, -8.0, -3.0, 4.0, -1.0))


def history_length(dissipation: int) -> int:
    return 6 if dissipation == 5 else 2


def short_range(pos, box, rc: float, A: float, rho: float):
    """Repulsion A exp(-r/rho) summed over every pair and image with
    0 < r < rc (an atom with its own images included); returns (F, E)."""
    w = wrap(np.asarray(pos, np.float64), box)
    box = np.asarray(box, np.float64)
    n = len(w)
    F = np.zeros((n, 3))
    E = 0.0
    m = np.ceil(rc / box).astype(int) + 1
    for s0 in range(-m[0], m[0] + 1):
        for s1 in range(-m[1], m[1] + 1):
            for s2 in range(-m[2], m[2] + 1):
                d = w[None, :, :] - w[:, None, :] + np.array([s0, s1, s2]) * box   # d[i, j] = r_j' - r_i
                r2 = np.sum(d * d, axis=2)
                ok = (r2 < rc * rc) & (r2 > 0.0)
                r = np.sqrt(np.where(ok, r2, 1.0))
                v = np.where(ok, A * np.exp(-r / rho), 0.0)
                E += 0.5 * v.sum()
                g = v / (rho * r)
                F -= np.sum(g[:, :, None] * d, axis=1)
    return F, float(E)


def shadow_state(pos, box, coul, chi, eta, q_tot, n_vec, n_krylov, rep_a=0.0, rep_rho=0.3):
    """Force, GMRES iterate x, shadow energy, V_short and q[n] at (R, n)."""
    chi = np.asarray(chi, np.float64)
    eta = np.asarray(eta, np.float64)
    v = Q.potential(pos, n_vec, box, coul)
    q, _ = Q.shadow_charges(v, chi, eta, q_tot)
    F = Q.force(pos, q, box, coul) - Q.force(pos, q - n_vec, box, coul)
    dinv = 1.0 / eta

    def J(y):
        t = dinv * Q.potential(pos, y, box, coul)
        return -y - (t - dinv * t.sum() / dinv.sum())

    b = -(q - n_vec)
    x = Q.gmres_iterate(J, b, n_krylov) if np.any(b) else np.zeros_like(b)
    E = float(q @ chi + 0.5 * np.sum(eta * q * q) + 0.5 * (2 * q - n_vec) @ v)
    Es = 0.0
    if rep_a > 0.0:
        Fs, Es = short_range(pos, box, coul["rc"], rep_a, rep_rho)
        F = F + Fs
    return F, x, E, Es, q


def regular_state(pos, box, coul, chi, eta, q_tot, rep_a=0.0, rep_rho=0.3):
    """Regular Born-Oppenheimer force and QEQ energy (Section "Regular
    Born-Oppenheimer MD for a Charge Equilibration Model") at the exact QEQ
    charges (dense LU of the bordered system): (F, E, V_short, q)."""
    A = Q.coulomb_matrix(pos, box, coul)
    q, _ = Q.qeq_dense(A, chi, eta, q_tot)
    F = Q.force(pos, q, box, coul)
    E = Q.qeq_energy(A, chi, eta, q)
    Es = 0.0
    if rep_a > 0.0:
        Fs, Es = short_range(pos, box, coul["rc"], rep_a, rep_rho)
        F = F + Fs
    return F, float(E), Es, q


def kinetic(vel, mass) -> float:
    return float(0.5 * np.sum(np.asarray(mass)[:, None] * vel * vel) / ACC)


def md_run(pos, vel, mass, box, coul, chi, eta, n_hist, steps, dt=0.5, n_krylov=8, dissipation=5, kappa=1.82,
           rep_a=0.0, rep_rho=0.3, q_tot=0.0, regular=False):
    """Returns (pos, vel, n_hist, energies) after `steps` steps; n_hist is
    newest first; energies[t] = (kinetic, potential, V_short, total).
    regular: Born-Oppenheimer MD on the exact QEQ charges instead (n_hist is
    returned unchanged)."""
    if regular:
        pos = np.array(pos, np.float64)
        vel = np.array(vel, np.float64)
        mass = np.asarray(mass, np.float64)
        F, E, Es, _ = regular_state(pos, box, coul, chi, eta, q_tot, rep_a, rep_rho)
        rows = [(kinetic(vel, mass), E, Es, kinetic(vel, mass) + E + Es)]
        for _ in range(steps):
            vel = vel + 0.5 * dt * ACC * F / mass[:, None]
            pos = pos + dt * vel
            F, E, Es, _ = regular_state(pos, box, coul, chi, eta, q_tot, rep_a, rep_rho)
            vel = vel + 0.5 * dt * ACC * F / mass[:, None]
            ke = kinetic(vel, mass)
            rows.append((ke, E, Es, ke + E + Es))
        return pos, vel, np.array(n_hist, np.float64), np.array(rows)
    pos = np.array(pos, np.float64)
    vel = np.array(vel, np.float64)
    mass = np.asarray(mass, np.float64)
    hist = [np.array(h, np.float64) for h in n_hist]
    if dissipation == 5:
        kappa, alpha, c = XL5
    else:
        alpha, c = 0.0, ()
    F, x, E, Es, _ = shadow_state(pos, box, coul, chi, eta, q_tot, hist[0], n_krylov, rep_a, rep_rho)
    rows = [(kinetic(vel, mass), E, Es, kinetic(vel, mass) + E + Es)]
    for _ in range(steps):
        vel = vel + 0.5 * dt * ACC * F / mass[:, None]
        pos = pos + dt * vel
        new = 2.0 * hist[0] - hist[1] + kappa * x
        if alpha != 0.0:
            new = new + alpha * sum(ck * hk for ck, hk in zip(c, hist))
        hist = [new] + hist[:-1]
        F, x, E, Es, _ = shadow_state(pos, box, coul, chi, eta, q_tot, hist[0], n_krylov, rep_a, rep_rho)
        vel = vel + 0.5 * dt * ACC * F / mass[:, None]
        ke = kinetic(vel, mass)
        rows.append((ke, E, Es, ke + E + Es))
    return pos, vel, np.stack(hist), np.array(rows)
