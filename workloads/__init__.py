"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests.

This module holds no arithmetic of the method (no Ewald, PME, QEQ or
neighbour logic): it only draws positions, charges and QEQ parameters, and
states the run parameters of each workload as plain numbers.

Workloads (units: Angstrom, elementary charge, eV):

* ``nacl``            rock-salt crystal, 4x4x4 conventional cells (512 ions).
* ``water_box``       3000 rigid 3-site molecules on a jittered cubic lattice.
* ``random_ionic``    uniform random +-1 ions at a fixed number density with a
                      minimum pair separation (the 300k-atom workload and the
                      per-request systems of the serving stream).
* ``serving_stream``  512 QEQ requests with log-uniform sizes and Poisson
                      arrival times.
* ``diff_batch``      64 independent 2000-atom systems for the gradient checks.
* ``triclinic_random`` random charges in a triclinic cell (box = the 3x3
                      lattice matrix), for the triclinic parity cases.

The Ewald splitting parameter for the workloads that do not state one follows
``alpha = sqrt(-ln(2*delta)) / rc`` with delta = 5e-4 (the paper's default
Ewald accuracy); the numbers below are that formula evaluated once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ALPHA_RC10 = 0.2628260884878466   # sqrt(-ln(1e-3)) / 10
ALPHA_RC9 = 0.29202898720871845  # sqrt(-ln(1e-3)) / 9


@dataclass
class System:
    """One periodic system: positions (N,3) float64, charges (N,) float64,
    orthorhombic box (3,) or triclinic lattice matrix (3,3), and the run
    parameters of its workload."""
    name: str
    pos: np.ndarray
    q: np.ndarray
    box: np.ndarray
    params: dict = field(default_factory=dict)
    chi: np.ndarray | None = None
    eta: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


# --------------------------------------------------------------------------
# rock-salt
# --------------------------------------------------------------------------
def nacl(ncell: int = 4, a: float = 5.64, shuffle_seed: int | None = None) -> System:
    """NaCl rock salt: sites (i,j,k)*a/2 for i,j,k in [0, 2*ncell), charge
    (-1)^(i+j+k). Cubic box of side ncell*a. Optional seeded atom shuffle."""
    m = 2 * ncell
    idx = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    pos = idx.astype(np.float64) * (a / 2.0)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    if shuffle_seed is not None:
        perm = np.random.default_rng(shuffle_seed).permutation(len(q))
        pos, q = pos[perm], q[perm]
    L = ncell * a
    return System("nacl", pos, q, np.array([L, L, L]),
                  dict(cutoff=8.0, alpha=0.35, kmax=8, grid=32, order=4, nn_dist=a / 2.0))


# --------------------------------------------------------------------------
# water-like box
# --------------------------------------------------------------------------
def water_box(n_mol: int = 3000, L: float = 31.0, seed: int = 2, sites_per_dim: int = 15,
              jitter: float = 0.2, min_inter: float = 0.8) -> System:
    """Rigid 3-site molecules (O-H 0.9572 A, H-O-H 104.52 deg), O on the
    first ``n_mol`` sites of a seeded permutation of a simple-cubic lattice;
    every molecule has the same orientation (bisector along (1,1,1), H-H along
    (1,-1,0)). Each molecule is rigidly translated by N(0, jitter^2); a
    molecule that comes within ``min_inter`` of another molecule is redrawn.
    Charges O -0.82, H +0.41."""
    rng = np.random.default_rng(seed)
    s = L / sites_per_dim
    g = np.stack(np.meshgrid(*(np.arange(sites_per_dim),) * 3, indexing="ij"), -1).reshape(-1, 3)
    sites = g[rng.permutation(len(g))[:n_mol]].astype(np.float64) * s
    d_oh = 0.9572
    half = math.radians(104.52) / 2.0
    b = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    h = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
    o_h1 = d_oh * (math.cos(half) * b + math.sin(half) * h)
    o_h2 = d_oh * (math.cos(half) * b - math.sin(half) * h)
    shift = rng.normal(0.0, jitter, size=(n_mol, 3))
    for _ in range(100):
        o = sites + shift
        mol = np.stack([o, o + o_h1, o + o_h2], 1)           # (n_mol, 3, 3)
        bad = _close_molecules(mol, L, min_inter)
        if not bad.any():
            break
        shift[bad] = rng.normal(0.0, jitter, size=(int(bad.sum()), 3))
    else:  # pragma: no cover
        raise RuntimeError("water_box: could not place molecules")
    pos = mol.reshape(-1, 3)
    q = np.tile(np.array([-0.82, 0.41, 0.41]), n_mol)
    return System("water", pos, q, np.array([L, L, L]),
                  dict(cutoff=10.0, alpha=ALPHA_RC10, grid=64, order=6, kmax=10))


def _close_molecules(mol: np.ndarray, L: float, dmin: float) -> np.ndarray:
    """Boolean mask of molecules with an atom within dmin of another molecule."""
    from scipy.spatial import cKDTree
    n_mol = mol.shape[0]
    flat = np.mod(mol.reshape(-1, 3), L)
    tree = cKDTree(flat, boxsize=L)
    pairs = tree.query_pairs(dmin, output_type="ndarray")
    bad = np.zeros(n_mol, bool)
    if len(pairs):
        mi, mj = pairs[:, 0] // 3, pairs[:, 1] // 3
        inter = mi != mj
        # redraw the later molecule of each clashing pair
        bad[np.maximum(mi[inter], mj[inter])] = True
    return bad


# --------------------------------------------------------------------------
# uniform random ions with a minimum separation
# --------------------------------------------------------------------------
def random_positions(n: int, L: float, rng: np.random.Generator, dmin: float = 1.0) -> np.ndarray:
    """Uniform positions in [0,L)^3; any atom closer than dmin (periodic) to an
    atom of lower index is redrawn until no such pair remains."""
    from scipy.spatial import cKDTree
    pos = rng.uniform(0.0, L, size=(n, 3))
    for _ in range(1000):
        tree = cKDTree(pos, boxsize=L)
        pairs = tree.query_pairs(dmin, output_type="ndarray")
        if len(pairs) == 0:
            return pos
        redo = np.unique(np.maximum(pairs[:, 0], pairs[:, 1]))
        pos[redo] = rng.uniform(0.0, L, size=(len(redo), 3))
        pos = np.mod(pos, L)  # uniform() may return L after rounding in float; keep [0,L)
        pos[pos >= L] = 0.0
    raise RuntimeError("random_positions: did not converge")


def balanced_charges(n: int, rng: np.random.Generator) -> np.ndarray:
    """+1/-1 charges, as balanced as n allows, in a seeded random order."""
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    if n % 2:
        q[-1] = 0.0
    return q[rng.permutation(n)]


def qeq_parameters(n: int, rng: np.random.Generator):
    """Electronegativity chi ~ N(0,1) eV and hardness eta ~ U(5,10) eV."""
    chi = rng.normal(0.0, 1.0, size=n)
    eta = rng.uniform(5.0, 10.0, size=n)
    return chi, eta


def random_ionic(n: int = 300_000, density: float = 0.1, seed: int = 3, cutoff: float = 10.0,
                 alpha: float = ALPHA_RC10, grid: int | None = 144, order: int = 6,
                 dmin: float = 1.0) -> System:
    """Neutral random ionic system at the given number density."""
    rng = np.random.default_rng(seed)
    L = (n / density) ** (1.0 / 3.0)
    pos = random_positions(n, L, rng, dmin)
    q = balanced_charges(n, rng)
    chi, eta = qeq_parameters(n, rng)
    if grid is None:
        grid = smooth_grid(L, 1.0, order)
    return System("random_ionic", pos, q, np.array([L, L, L]),
                  dict(cutoff=cutoff, alpha=alpha, grid=grid, order=order), chi=chi, eta=eta)


def smooth_grid(L: float, spacing: float, order: int) -> int:
    """Smallest 2^a 3^b 5^c that is >= ceil(L/spacing) and >= 2*order."""
    need = max(int(math.ceil(L / spacing)), 2 * order)
    k = need
    while True:
        m = k
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return k
        k += 1


# --------------------------------------------------------------------------
# serving stream and differentiation batch
# --------------------------------------------------------------------------
def serving_stream(n_req: int = 512, qps: float = 100.0, seed_sizes: int = 4, seed_arrivals: int = 40,
                   nmin: int = 64, nmax: int = 20000, density: float = 0.1):
    """List of (arrival_time_s, System) for the QEQ serving stream.

    Sizes are floor(exp(U(ln nmin, ln nmax))); each request is a random ionic
    system (cutoff 9, PME spacing 1 A, order 5) with chi, eta as above and a
    random neutral starting charge vector q0 = N(0, 0.5) minus its mean,
    solved to relative residual 1e-5 within 200 products without restarts.
    Arrivals are a Poisson process at ``qps`` requests per second."""
    rs = np.random.default_rng(seed_sizes)
    sizes = np.floor(np.exp(rs.uniform(math.log(nmin), math.log(nmax), size=n_req))).astype(int)
    ra = np.random.default_rng(seed_arrivals)
    t = np.cumsum(ra.exponential(1.0 / qps, size=n_req))
    out = []
    for r, (n, ta) in enumerate(zip(sizes, t)):
        out.append((float(ta), serving_request(int(n), 40_000 + r, density)))
    return out


def serving_request(n: int, seed: int, density: float = 0.1) -> System:
    rng = np.random.default_rng(seed)
    L = (n / density) ** (1.0 / 3.0)
    pos = random_positions(n, L, rng, 1.0)
    chi, eta = qeq_parameters(n, rng)
    q0 = rng.normal(0.0, 0.5, size=n)
    q0 -= q0.mean()
    order = 5
    K = smooth_grid(L, 1.0, order)
    return System("serving", pos, q0, np.array([L, L, L]),
                  dict(cutoff=9.0, alpha=ALPHA_RC9, grid=K, order=order, tol=1e-5,
                       max_it=200, restart=200), chi=chi, eta=eta)


def diff_batch(n_sys: int = 64, n: int = 2000, density: float = 0.1, seed0: int = 5000):
    """Independent systems for the gradient checks (cutoff 9, PME 48^3 order 5)."""
    out = []
    for s in range(n_sys):
        rng = np.random.default_rng(seed0 + s)
        L = (n / density) ** (1.0 / 3.0)
        pos = random_positions(n, L, rng, 1.0)
        q = balanced_charges(n, rng)
        chi, eta = qeq_parameters(n, rng)
        out.append(System("diff", pos, q, np.array([L, L, L]),
                          dict(cutoff=9.0, alpha=ALPHA_RC9, grid=48, order=5), chi=chi, eta=eta))
    return out


def triclinic_random(n: int, edges, tilts, seed: int, dmin: float = 1.0, neutral: bool = True) -> System:
    """Random system in a triclinic cell whose lattice vectors are the rows of
    H = [[L0, 0, 0], [t_xy, L1, 0], [t_xz, t_yz, L2]] (``box`` is H): uniform
    fractional coordinates (minimum separation dmin scaled to fractional units
    by 0.7 of the shortest edge), mapped through H, and every atom moved by a
    random lattice vector with components in {-1, 0, 1} so that positions lie
    outside the cell too."""
    rng = np.random.default_rng(seed)
    L0, L1, L2 = (float(x) for x in edges)
    txy, txz, tyz = (float(x) for x in tilts)
    H = np.array([[L0, 0.0, 0.0], [txy, L1, 0.0], [txz, tyz, L2]])
    s = random_positions(n, 1.0, rng, dmin / (0.7 * min(L0, L1, L2)))
    s = s + rng.integers(-1, 2, size=(n, 3))
    pos = s @ H
    q = rng.normal(0.0, 1.0, size=n)
    if neutral:
        q -= q.mean()
    chi, eta = qeq_parameters(n, rng)
    return System("triclinic", pos, q, H, {}, chi=chi, eta=eta)


def small_random(n: int, L: float, seed: int, dmin: float = 1.0, neutral: bool = True) -> System:
    """Small random system for oracle pins and parity cases."""
    rng = np.random.default_rng(seed)
    pos = random_positions(n, L, rng, dmin)
    q = rng.normal(0.0, 1.0, size=n)
    if neutral:
        q -= q.mean()
    chi, eta = qeq_parameters(n, rng)
    return System("small", pos, q, np.array([L, L, L]), {}, chi=chi, eta=eta)
