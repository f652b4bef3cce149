"""Charge equilibration in FP64 (oracle; test infrastructure only).

Follows the paper's Sections "Regular Born-Oppenheimer MD for a Charge
Equilibration Model" and "Shadow Born-Oppenheimer MD":

* QEQ energy  E(R,q) = sum q_i chi_i + 1/2 sum q_i^2 u_i + E_Coul(R,q)
  (eq. qeq_energy_func), minimised under sum q = Q_tot via the bordered
  system [[C, 1], [1^T, 0]] [q; lambda] = [-chi; Q_tot] (eq. linear_qeq).
* Matrix-free product  C v = u o v + dE_Coul/dv  (the Cv identity of the
  same section).
* Shadow charges q[n] from the quasi-diagonal system (eq. diag_linear_qeq):
  v = A n,  lambda = -(Q_tot + sum (chi_i + v_i)/u_i) / sum 1/u_i,
  q_i[n] = -(chi_i + v_i + lambda)/u_i.
* Jacobian J = d(q[n] - n)/dn and the Krylov (GMRES) approximation of
  J x = -(q[n] - n) (eq. Jnddot, omega^2 = 1).

Readings: C = diag(u) + A with A the Hessian of E_Coul in the charges, i.e.
A v = phi[v] including every periodic-image, self and background term. The
paper's printed off-diagonal sign (delta_ij - 1) is read as +phi_ij, which is
what the Cv identity implies, and the diagonal carries the periodic self
interaction (A_ii != 0). A is built column by column from the oracle's own
potential functions, so it is exactly the operator whose action those
functions define.
"""
from __future__ import annotations

import numpy as np

from .ewald import KE, ewald_direct, real_space, reciprocal_direct, self_background  # noqa: F401
from .spme import spme_reciprocal


# --------------------------------------------------------------------------
# the Coulomb operator A (phi = A q)
# --------------------------------------------------------------------------
def potential(pos, q, box, coul: dict) -> np.ndarray:
    """phi[q] = dE_Coul/dq for the operator described by ``coul``:
    dict(method='ewald'|'pme', alpha, rc, kmax | grid+order)."""
    a, rc = coul["alpha"], coul["rc"]
    pr, _ = real_space(pos, q, box, a, rc, force=False)
    if coul["method"] == "ewald":
        pk, _, _ = reciprocal_direct(pos, q, box, a, coul["kmax"])
    else:
        pk, _, _ = spme_reciprocal(pos, q, box, a, coul["grid"], coul["order"])
    return pr + pk + self_background(q, box, a)


def force(pos, q, box, coul: dict) -> np.ndarray:
    """F[q] = -d(1/2 q^T A(R) q)/dR for the same operator."""
    a, rc = coul["alpha"], coul["rc"]
    _, fr = real_space(pos, q, box, a, rc)
    if coul["method"] == "ewald":
        _, fk, _ = reciprocal_direct(pos, q, box, a, coul["kmax"])
    else:
        _, fk, _ = spme_reciprocal(pos, q, box, a, coul["grid"], coul["order"])
    return fr + fk


def coulomb_matrix(pos, box, coul: dict) -> np.ndarray:
    """Dense A with A[:, j] = phi[e_j] (symmetric up to rounding)."""
    n = len(pos)
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = potential(pos, e, box, coul)
    return 0.5 * (A + A.T)


def coulomb_matrix_blocked(pos, box, coul: dict, chunk: int = 32) -> np.ndarray:
    """The same A as coulomb_matrix, assembled term by term for larger N:
    the real-space pair potentials erfc(a|d|)/|d| summed over images (the
    terms of eq. ewald_real), the smooth-PME reciprocal potential of unit
    charges computed for a block of columns at once (same steps as
    spme_reciprocal), and the self and background terms on every entry."""
    from .ewald import image_offsets, image_shifts, volume, wrap
    from .spme import _stencil, influence
    from scipy.special import erfc
    n = len(pos)
    a, rc = coul["alpha"], coul["rc"]
    w = wrap(np.asarray(pos, np.float64), box)
    shifts = image_shifts(box, rc)
    sL = image_offsets(shifts, box)
    zero = np.all(shifts == 0, axis=1)
    A = np.zeros((n, n))
    step = max(1, 2_000_000 // max(1, n * len(shifts)))
    for s in range(0, n, step):
        I = np.arange(s, min(n, s + step))
        dd = (w[None, :, :] - w[I][:, None, :])[:, :, None, :] + sL[None, None, :, :]
        r2 = dd[..., 0] * dd[..., 0] + dd[..., 1] * dd[..., 1] + dd[..., 2] * dd[..., 2]
        mask = (r2 < rc * rc) & ~((I[:, None] == np.arange(n)[None, :])[:, :, None] & zero[None, None, :])
        r = np.sqrt(np.where(mask, r2, 1.0))
        A[I] = KE * np.where(mask, erfc(a * r) / r, 0.0).sum(2)
    if coul["method"] == "ewald":
        from .ewald import kvectors
        _, k = kvectors(box, coul["kmax"])
        k2 = np.sum(k * k, 1)
        V = volume(box)
        ck = 4.0 * np.pi / V * np.exp(-k2 / (4 * a * a)) / k2
        ph = w @ k.T
        C, S = np.cos(ph), np.sin(ph)
        A += KE * ((C * ck) @ C.T + (S * ck) @ S.T)
    else:
        K = np.broadcast_to(np.asarray(coul["grid"]), (3,)).astype(int)
        idx, W, _ = _stencil(pos, box, K, coul["order"])
        flat = ((idx[:, 0, :, None, None] * K[1] + idx[:, 1, None, :, None]) * K[2]
                + idx[:, 2, None, None, :]).reshape(n, -1)
        wt = (W[:, 0, :, None, None] * W[:, 1, None, :, None] * W[:, 2, None, None, :]).reshape(n, -1)
        G = influence(box, a, K, coul["order"])
        nk = int(np.prod(K))
        for j0 in range(0, n, chunk):
            J = np.arange(j0, min(n, j0 + chunk))
            Q = np.zeros((len(J), nk))
            for t, j in enumerate(J):
                Q[t] = np.bincount(flat[j], weights=wt[j], minlength=nk)
            FQ = np.fft.fftn(Q.reshape(len(J), *K), axes=(1, 2, 3))
            psi = np.real(np.fft.ifftn(G[None] * FQ, axes=(1, 2, 3))).reshape(len(J), nk) * nk
            A[:, J] += np.einsum("ip,jip->ij", wt, psi[:, flat])   # G carries KE
    V = volume(box)
    A += -KE * np.pi / (V * a * a)
    A[np.diag_indices(n)] += -KE * 2.0 * a / np.sqrt(np.pi)
    return 0.5 * (A + A.T)


# --------------------------------------------------------------------------
# regular QEQ
# --------------------------------------------------------------------------
def bordered(A: np.ndarray, eta) -> np.ndarray:
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A + np.diag(eta)
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    return M


def qeq_dense(A: np.ndarray, chi, eta, q_tot: float = 0.0):
    """Solve the bordered system by LU; returns (q, lambda)."""
    n = A.shape[0]
    rhs = np.concatenate([-np.asarray(chi, np.float64), [q_tot]])
    z = np.linalg.solve(bordered(A, eta), rhs)
    return z[:n], float(z[n])


def qeq_energy(A, chi, eta, q):
    """E(q) = q.chi + 1/2 sum u q^2 + 1/2 q^T A q."""
    return float(q @ chi + 0.5 * np.sum(eta * q * q) + 0.5 * q @ (A @ q))


def bordered_residual(A, chi, eta, q_tot, q, lam) -> float:
    """Relative residual ||b - M z|| / ||b|| of the bordered system."""
    rhs = np.concatenate([-np.asarray(chi, np.float64), [q_tot]])
    z = np.concatenate([q, [lam]])
    return float(np.linalg.norm(rhs - bordered(A, eta) @ z) / np.linalg.norm(rhs))


# --------------------------------------------------------------------------
# shadow step
# --------------------------------------------------------------------------
def shadow_charges(v, chi, eta, q_tot: float = 0.0):
    """q[n] from v = A n (eq. diag_linear_qeq); returns (q, lambda)."""
    chi = np.asarray(chi, np.float64)
    inv = 1.0 / np.asarray(eta, np.float64)
    lam = -(q_tot + np.sum((chi + v) * inv)) / np.sum(inv)
    return -(chi + v + lam) * inv, float(lam)


def jacobian(A, eta) -> np.ndarray:
    """J = d(q[n] - n)/dn = -I - P D^-1 A with P = I - D^-1 1 1^T / (1^T D^-1 1)."""
    n = A.shape[0]
    dinv = 1.0 / np.asarray(eta, np.float64)
    P = np.eye(n) - np.outer(dinv, np.ones(n)) / dinv.sum()
    return -np.eye(n) - P @ (dinv[:, None] * A)


def gmres_iterate(apply, b, m: int) -> np.ndarray:
    """m-th GMRES iterate from x0 = 0: the x in the Krylov space
    K_m = span{b, Jb, ..., J^{m-1} b} that minimises ||b - J x||.
    Plain definition: orthonormal basis V of K_m (modified Gram-Schmidt),
    then the least-squares problem min_y ||b - (J V) y||."""
    n = len(b)
    V = np.zeros((n, m))
    v = b / np.linalg.norm(b)
    k = 0
    for k in range(m):
        V[:, k] = v
        w = apply(v)
        for i in range(k + 1):
            w = w - (V[:, i] @ w) * V[:, i]
        nw = np.linalg.norm(w)
        if nw < 1e-300:
            V = V[:, :k + 1]
            break
        v = w / nw
    JV = np.stack([apply(V[:, i]) for i in range(V.shape[1])], 1)
    y, *_ = np.linalg.lstsq(JV, b, rcond=None)
    return V @ y


def shadow_step_dense(A, chi, eta, n_vec, q_tot: float = 0.0, n_krylov: int = 8):
    """Shadow step with a dense operator: (q[n], lambda, x) where x is the
    n_krylov-step GMRES iterate for J x = -(q[n] - n)."""
    v = A @ n_vec
    q, lam = shadow_charges(v, chi, eta, q_tot)
    J = jacobian(A, eta)
    x = gmres_iterate(lambda y: J @ y, -(q - n_vec), n_krylov)
    return q, lam, x


def shadow_energy(A, chi, eta, q, n_vec) -> float:
    """Shadow energy (eq. qeq_energy) without V_short:
    sum q chi + 1/2 sum u q^2 + 1/2 (2q - n)^T A n."""
    return float(q @ chi + 0.5 * np.sum(eta * q * q) + 0.5 * (2 * q - n_vec) @ (A @ n_vec))
