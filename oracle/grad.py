"""Gradients through the QEQ solve in FP64 (oracle; test infrastructure only).

The paper trains chi and u through the QEQ solve (Section "Validation and
Performance") and integrates forces -grad U_BO (Section "Regular
Born-Oppenheimer MD"); it prints no gradient formulas. What this computes is
the plain calculus of the bordered system M(R,u) z = b(chi):

* energy at the constrained minimum q*: by stationarity (envelope theorem)
  dE/dR = -F[q*], dE/dchi = q*, dE/du = q*^2 / 2;
* a general loss L(q*) with upstream g = dL/dq*: adjoint solve
  M [a; mu] = [g; 0], then dL/dchi = -a, dL/du_i = -a_i q*_i and
  dL/dR = -d/dR (a^T A(R) q*) = F[a + q*] - F[a] - F[q*],
  where F[x] = -d/dR (1/2 x^T A x);
* central finite differences, used by the tests to pin the formulas.
"""
from __future__ import annotations

import numpy as np

from .qeq import bordered, coulomb_matrix, force, qeq_dense


def qeq_energy_and_grad(pos, box, coul, chi, eta, q_tot=0.0):
    """Returns (E, q*, dE/dR, dE/dchi, dE/du) for the regular QEQ energy."""
    A = coulomb_matrix(pos, box, coul)
    q, _ = qeq_dense(A, chi, eta, q_tot)
    E = float(q @ chi + 0.5 * np.sum(eta * q * q) + 0.5 * q @ (A @ q))
    return E, q, -force(pos, q, box, coul), q.copy(), 0.5 * q * q


def qeq_vjp(pos, box, coul, chi, eta, gbar, q_tot=0.0):
    """Vector-Jacobian product of q*(R, chi, u) with upstream gbar.
    Returns (dL/dR, dL/dchi, dL/du)."""
    A = coulomb_matrix(pos, box, coul)
    q, _ = qeq_dense(A, chi, eta, q_tot)
    n = len(q)
    z = np.linalg.solve(bordered(A, eta), np.concatenate([gbar, [0.0]]))
    a = z[:n]
    dR = force(pos, a + q, box, coul) - force(pos, a, box, coul) - force(pos, q, box, coul)
    return dR, -a, -a * q


def central_difference(f, x: np.ndarray, h: float, idx) -> np.ndarray:
    """(f(x + h e_k) - f(x - h e_k)) / 2h for the flat indices in idx."""
    x = np.array(x, np.float64)
    flat = x.reshape(-1)
    out = []
    for k in idx:
        xp = flat.copy()
        xp[k] += h
        xm = flat.copy()
        xm[k] -= h
        out.append((f(xp.reshape(x.shape)) - f(xm.reshape(x.shape))) / (2.0 * h))
    return np.array(out)
