"""Direct Ewald summation in FP64 (oracle; test infrastructure only).

Follows the paper's Section "Regular Ewald Summation":
  E_Coul = 1/2 sum_i sum_{j != i} q_i q_j phi(r_ij)            (eq. ewald_general)
         = E_real + E_rec + E_self                              (Ewald split)
  E_real = 1/2 sum_i sum_j q_i q_j sum_n' erfc(a|r_ij+nL|)/|r_ij+nL|   (eq. ewald_real)
  E_rec  = 1/(2V) sum_{k!=0} 4 pi/k^2 exp(-k^2/4a^2) |sum_j q_j exp(i k.r_j)|^2 (eq. ewald_rec)
  E_self = -a/sqrt(pi) sum_i q_i^2                               (eq. ewald_self)

Readings taken where the paper is silent:
* energies carry the Coulomb constant KE (eV, Angstrom, e);
* a neutralising background -pi Q^2/(2 V a^2) (Q = sum q) is added, so the
  potential of a non-neutral charge vector (a Krylov vector) is well defined
  and independent of a; it vanishes for neutral charges;
* the real-space sum is truncated at |d| < rc (strict, unshifted) and runs
  over every periodic image with |d| < rc, including an atom's own images
  when rc exceeds half the box;
* the k-sum runs over the cube |n_d| <= kmax, k = 2 pi n / L, n != 0;
* triclinic cells (which the paper mentions for the Ewald sum without
  formulas) replace n*L by the lattice vector n H and 2 pi n / L by the
  reciprocal vector 2 pi H^-1 n; everything else is unchanged.

The per-atom potential is phi_i = dE_Coul/dq_i, so E_Coul = 1/2 sum_i q_i phi_i,
and the force is F_i = -dE_Coul/dr_i.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import erfc

KE = 14.3996454784  # e^2/(4 pi eps0) in eV*Angstrom


def is_triclinic(box) -> bool:
    """A box is either the three edges of an orthorhombic cell or a 3x3 lower
    triangular matrix whose rows are the lattice vectors a = (L0, 0, 0),
    b = (t_xy, L1, 0), c = (t_xz, t_yz, L2)."""
    return np.asarray(box).shape == (3, 3)


def cell_matrix(box) -> np.ndarray:
    """The lattice vectors as rows of a 3x3 matrix (diagonal for an orthorhombic box)."""
    b = np.asarray(box, np.float64)
    if b.shape == (3, 3):
        if b[0, 1] != 0 or b[0, 2] != 0 or b[1, 2] != 0 or np.any(np.diag(b) <= 0):
            raise ValueError("triclinic box must be lower triangular with a positive diagonal")
        return b
    return np.diag(b)


def volume(box) -> float:
    return float(np.prod(np.diag(cell_matrix(box))))


def wrap(pos: np.ndarray, box) -> np.ndarray:
    """Canonical wrap into the cell (the neighbour predicate depends on it; every
    step is a separately rounded FP64 operation).

    Orthorhombic: w = x - L*floor(x*(1/L)) per axis.
    Triclinic (rows a, b, c as in is_triclinic): the c, b and a components are
    removed in turn, each by the floor of the current fractional coordinate:
      f2 = floor(z*(1/L2));                 (x, y, z) -= f2 * c
      f1 = floor((y - z*r_yz)*(1/L1));      (x, y)    -= f1 * (t_xy, L1)
      f0 = floor(((x - y*c_xy) - z*c_xz)*(1/L0));  x  -= f0 * L0
    with r_yz = t_yz/L2, c_xy = t_xy/L1, c_xz = (t_xz - t_yz*c_xy)/L2 (each
    product and difference rounded once). With zero tilts every tilt term is an
    exact zero and this is the orthorhombic wrap bit for bit.
    """
    if not is_triclinic(box):
        box = np.asarray(box, dtype=np.float64)
        inv = 1.0 / box
        return pos - box * np.floor(pos * inv)
    H = cell_matrix(box)
    L0, L1, L2 = H[0, 0], H[1, 1], H[2, 2]
    txy, txz, tyz = H[1, 0], H[2, 0], H[2, 1]
    i0, i1, i2 = 1.0 / L0, 1.0 / L1, 1.0 / L2
    ryz = tyz * i2
    cxy = txy * i1
    cxz = (txz - tyz * cxy) * i2
    pos = np.asarray(pos, np.float64)
    x, y, z = pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy()
    f2 = np.floor(z * i2)
    z = z - f2 * L2
    y = y - f2 * tyz
    x = x - f2 * txz
    f1 = np.floor((y - z * ryz) * i1)
    y = y - f1 * L1
    x = x - f1 * txy
    f0 = np.floor(((x - y * cxy) - z * cxz) * i0)
    x = x - f0 * L0
    return np.stack([x, y, z], 1)


def fractional(w: np.ndarray, box) -> np.ndarray:
    """Fractional coordinates s with r = s . H (rows of H the lattice vectors)."""
    if not is_triclinic(box):
        return w / np.asarray(box, np.float64)[None, :]
    return w @ np.linalg.inv(cell_matrix(box))


def plane_widths(box) -> np.ndarray:
    """Distances between opposite faces of the cell, V / |b x c|, V / |c x a|, V / |a x b|."""
    H = cell_matrix(box)
    V = volume(box)
    a, b, c = H
    return np.array([V / np.linalg.norm(np.cross(b, c)), V / np.linalg.norm(np.cross(c, a)),
                     V / np.linalg.norm(np.cross(a, b))])


def image_shifts(box, rc: float) -> np.ndarray:
    """All integer image vectors n with |n_d| <= ceil(rc/w_d), w_d the plane
    widths (the edges L_d for an orthorhombic box): enough for every
    |w_j - w_i + n H| < rc when w is wrapped into the cell."""
    wd = np.asarray(box, np.float64) if not is_triclinic(box) else plane_widths(box)
    r = [int(math.ceil(rc / float(L))) for L in wd]
    return np.array(list(itertools.product(*(range(-m, m + 1) for m in r))), dtype=np.int64)


def image_offsets(shifts: np.ndarray, box) -> np.ndarray:
    """Cartesian offsets n H of integer image vectors, each component summed left
    to right with separately rounded products:
      x = (n0*L0 + n1*t_xy) + n2*t_xz,  y = n1*L1 + n2*t_yz,  z = n2*L2
    (orthorhombic: n*L; the same values, as the tilt terms are exact zeros)."""
    if not is_triclinic(box):
        return shifts * np.asarray(box, np.float64)
    H = cell_matrix(box)
    n = shifts.astype(np.float64)
    x = (n[:, 0] * H[0, 0] + n[:, 1] * H[1, 0]) + n[:, 2] * H[2, 0]
    y = n[:, 1] * H[1, 1] + n[:, 2] * H[2, 1]
    z = n[:, 2] * H[2, 2]
    return np.stack([x, y, z], 1)


def real_space(pos, q, box, alpha, rc, rows=None, force=True, chunk_elems=4_000_000):
    """Real-space part (eq. ewald_real), brute force over all pairs and images.

    Returns (phi, F) for the atoms in ``rows`` (all atoms by default); phi_i
    includes KE. The pair (i, j, n) contributes iff d = (w_j - w_i) + n*L has
    d.d < rc^2 (d.d summed left to right) and not (j == i and n == 0).
    """
    w = wrap(np.asarray(pos, np.float64), box)
    q = np.asarray(q, np.float64)
    n = len(q)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    shifts = image_shifts(box, rc)
    sL = image_offsets(shifts, box)                # (ns, 3) FP64 image offsets
    zero = np.all(shifts == 0, axis=1)
    rc2 = rc * rc
    phi = np.zeros(len(rows))
    F = np.zeros((len(rows), 3))
    step = max(1, chunk_elems // max(1, n * len(shifts)))
    c = 2.0 * alpha / math.sqrt(math.pi)
    for s in range(0, len(rows), step):
        I = rows[s:s + step]
        dd = (w[None, :, :] - w[I][:, None, :])[:, :, None, :] + sL[None, None, :, :]   # (b, n, ns, 3)
        r2 = dd[..., 0] * dd[..., 0] + dd[..., 1] * dd[..., 1] + dd[..., 2] * dd[..., 2]
        mask = r2 < rc2
        selfm = (I[:, None] == np.arange(n)[None, :])[:, :, None] & zero[None, None, :]
        mask &= ~selfm
        r = np.sqrt(np.where(mask, r2, 1.0))
        e = np.where(mask, erfc(alpha * r) / r, 0.0)
        phi[s:s + step] = KE * np.einsum("bjs,j->b", e, q)
        if force:
            # d points from i to the image of j; the force on i is
            # KE q_i q_j [erfc(ar)/r + c exp(-a^2 r^2)] (r_i - r_j')/r^2 = -(...) d / r^2
            g = np.where(mask, (e + c * np.exp(-(alpha * r) ** 2)) / (r * r), 0.0)
            F[s:s + step] = -KE * q[I][:, None] * np.einsum("bjs,j,bjsx->bx", g, q, dd)
    return phi, F


def kvectors(box, kmax):
    """Integer vectors n of the cube |n_d| <= kmax without 0, and the wave
    vectors k = 2 pi n / L (triclinic: k = 2 pi H^-1 n, the reciprocal lattice,
    so that k . r = 2 pi n . s with s the fractional coordinates)."""
    km = np.broadcast_to(np.asarray(kmax), (3,))
    nv = np.array([v for v in itertools.product(*(range(-m, m + 1) for m in km)) if any(v)],
                  dtype=np.float64)
    if is_triclinic(box):
        return nv, 2.0 * math.pi * nv @ np.linalg.inv(cell_matrix(box)).T
    return nv, 2.0 * math.pi * nv / np.asarray(box, np.float64)[None, :]


def reciprocal_direct(pos, q, box, alpha, kmax, rows=None, chunk=512):
    """Reciprocal part (eq. ewald_rec) by the plain k-sum.

    S(k) = sum_j q_j exp(i k.r_j);  c_k = (4 pi/V) exp(-k^2/4a^2)/k^2
    E_rec = KE/2 sum_k c_k |S(k)|^2
    phi_i = dE_rec/dq_i = KE sum_k c_k Re(exp(-i k.r_i) S(k))
    F_i  = -dE_rec/dr_i = KE q_i sum_k c_k k Im(conj(S(k)) exp(i k.r_i))
    Returns (phi, F, E_rec).
    """
    w = wrap(np.asarray(pos, np.float64), box)
    q = np.asarray(q, np.float64)
    V = volume(box)
    rows = np.arange(len(q)) if rows is None else np.asarray(rows)
    _, k = kvectors(box, kmax)
    k2 = np.sum(k * k, axis=1)
    ck = 4.0 * math.pi / V * np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    phi = np.zeros(len(rows))
    F = np.zeros((len(rows), 3))
    E = 0.0
    for s in range(0, len(k), chunk):
        kk = k[s:s + chunk]
        cc = ck[s:s + chunk]
        ph = w @ kk.T                                  # (N, nk)
        S = (q[:, None] * np.exp(1j * ph)).sum(0)      # (nk,)
        E += 0.5 * KE * float(np.sum(cc * np.abs(S) ** 2))
        e = np.exp(1j * ph[rows])                      # (nr, nk)
        phi += KE * (np.real(np.conj(e) * S[None, :]) * cc[None, :]).sum(1)
        F += KE * q[rows][:, None] * ((np.imag(np.conj(S)[None, :] * e) * cc[None, :]) @ kk)
    return phi, F, E


def self_background(q, box, alpha):
    """Self term (eq. ewald_self) and neutralising background, as potentials.

    phi_self,i = -KE 2a/sqrt(pi) q_i ; phi_bg = -KE pi Q/(V a^2), Q = sum q.
    Their energies are 1/2 sum q_i phi_i: -KE a/sqrt(pi) sum q^2 and
    -KE pi Q^2/(2 V a^2).
    """
    q = np.asarray(q, np.float64)
    V = volume(box)
    Q = float(q.sum())
    return -KE * 2.0 * alpha / math.sqrt(math.pi) * q - KE * math.pi * Q / (V * alpha * alpha)


def ewald_direct(pos, q, box, alpha, rc, kmax, rows=None):
    """Full periodic Coulomb potential, force and energy by direct Ewald.

    Returns a dict with phi, F (rows only), and the energy split
    E, E_real, E_rec, E_selfbg (energies need all rows).
    """
    q = np.asarray(q, np.float64)
    allrows = rows is None
    rows = np.arange(len(q)) if allrows else np.asarray(rows)
    pr, fr = real_space(pos, q, box, alpha, rc, rows=rows)
    pk, fk, Erec = reciprocal_direct(pos, q, box, alpha, kmax, rows=rows)
    ps = self_background(q, box, alpha)[rows]
    out = dict(phi=pr + pk + ps, F=fr + fk, phi_real=pr, phi_rec=pk, phi_selfbg=ps,
               F_real=fr, F_rec=fk)
    if allrows:
        out.update(E_real=0.5 * float(q @ pr), E_rec=Erec, E_selfbg=0.5 * float(q @ ps))
        out["E"] = out["E_real"] + out["E_rec"] + out["E_selfbg"]
    return out
