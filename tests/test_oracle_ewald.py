"""Pins of the direct-Ewald oracle against values and identities that the
paper and textbook electrostatics fix (no GPU)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

# NaCl rock-salt Madelung constant (textbook value, the workload's target 1.747565)
MADELUNG_NACL = 1.747564594633
# Lattice sum of a simple cubic Wigner lattice of unit charges in a neutralising
# background, in units of 1/L (textbook value).
WIGNER_SC = -2.837297479


def madelung(sys_, res):
    return -float(np.mean(sys_.q * res["phi"])) * sys_.params["nn_dist"] / O.KE


@pytest.fixture(scope="module")
def nacl_cfg():
    s = W.nacl()
    return s, O.ewald_direct(s.pos, s.q, s.box, 0.35, 8.0, 8)


def test_madelung_tight_parameters():
    # rc 11 A, alpha 0.5/A, kmax 12: both Ewald truncations below 1e-12
    s = W.nacl(ncell=2)          # 64 ions, 11.28 A box, multi-image real space
    r = O.ewald_direct(s.pos, s.q, s.box, 0.5, 11.0, 12)
    assert abs(madelung(s, r) - MADELUNG_NACL) < 1e-9


def test_madelung_workload_parameters(nacl_cfg):
    s, r = nacl_cfg
    M = madelung(s, r)
    # at rc 8 A, alpha 0.35 the real-space tail is a 1.3e-4 relative truncation
    assert abs(M / MADELUNG_NACL - 1.0) < 1.5e-4
    # every ion of the perfect crystal sees the same |phi|
    assert np.ptp(s.q * r["phi"]) < 1e-9
    # energy split consistency: E = 1/2 sum q phi
    assert abs(r["E"] - 0.5 * s.q @ r["phi"]) < 1e-9 * abs(r["E"])


def test_wigner_single_charge_alpha_independent():
    L = 10.0
    for a, rc, km in [(0.3, 12.0, 10), (0.45, 8.0, 12), (0.6, 6.0, 16)]:
        r = O.ewald_direct(np.array([[1.0, 2.0, 3.0]]), np.array([1.0]), [L, L, L], a, rc, km)
        assert abs(r["E"] / (0.5 * O.KE * WIGNER_SC / L) - 1.0) < 1e-8


def test_alpha_independence_and_force_sum():
    s = W.small_random(12, 7.0, seed=11)
    outs = []
    for a, rc, km in [(0.4, 13.5, 8), (0.55, 9.8, 10), (0.7, 7.7, 12)]:
        outs.append(O.ewald_direct(s.pos, s.q, s.box, a, rc, km))
    for r in outs[1:]:
        assert np.abs(r["phi"] - outs[0]["phi"]).max() < 1e-8 * np.abs(outs[0]["phi"]).max()
        assert np.abs(r["F"] - outs[0]["F"]).max() < 1e-8 * np.abs(outs[0]["F"]).max()
    for r in outs:
        assert np.abs(r["F"].sum(0)).max() < 1e-10 * np.abs(r["F"]).max()


def test_translation_and_scale_invariance():
    s = W.small_random(10, 8.0, seed=12)
    a, rc, km = 0.5, 7.0, 10
    r0 = O.ewald_direct(s.pos, s.q, s.box, a, rc, km)
    r1 = O.ewald_direct(s.pos + np.array([3.3, -17.1, 41.7]), s.q, s.box, a, rc, km)
    assert np.abs(r1["phi"] - r0["phi"]).max() < 1e-9
    assert np.abs(r1["F"] - r0["F"]).max() < 1e-9
    sc = 1.7
    r2 = O.ewald_direct(s.pos * sc, s.q, s.box * sc, a / sc, rc * sc, km)
    assert np.abs(r2["phi"] * sc - r0["phi"]).max() < 1e-9
    assert np.abs(r2["F"] * sc * sc - r0["F"]).max() < 1e-9


def test_force_is_minus_energy_gradient():
    s = W.small_random(8, 7.0, seed=13)
    a, rc, km = 0.5, 9.0, 11           # erfc(a rc) ~ 1e-10: no cutoff crossing matters
    r = O.ewald_direct(s.pos, s.q, s.box, a, rc, km)
    h = 1e-5

    def energy(p):
        return O.ewald_direct(p, s.q, s.box, a, rc, km)["E"]
    for k in [0, 4, 10, 23]:
        pp = s.pos.copy().reshape(-1)
        pm = pp.copy()
        pp[k] += h
        pm[k] -= h
        g = (energy(pp.reshape(-1, 3)) - energy(pm.reshape(-1, 3))) / (2 * h)
        assert abs(-g - r["F"].reshape(-1)[k]) < 1e-6 * max(1.0, abs(g))


def test_potential_is_charge_derivative_and_symmetric_operator():
    s = W.small_random(9, 7.0, seed=14)
    a, rc, km = 0.5, 9.0, 11
    rng = np.random.default_rng(0)
    v, w = rng.normal(size=9), rng.normal(size=9)   # non-neutral on purpose
    pv = O.ewald_direct(s.pos, v, s.box, a, rc, km)["phi"]
    pw = O.ewald_direct(s.pos, w, s.box, a, rc, km)["phi"]
    assert abs(w @ pv - v @ pw) < 1e-10 * abs(w @ pv)
    # linearity in the charges
    pvw = O.ewald_direct(s.pos, v + 2 * w, s.box, a, rc, km)["phi"]
    assert np.abs(pvw - pv - 2 * pw).max() < 1e-10 * np.abs(pvw).max()


def _spherical_sum(pos, q, L, nshell):
    """Plain Coulomb sum over whole-box images inside a sphere of radius nshell*L."""
    rng_ = np.arange(-nshell, nshell + 1)
    n = np.stack(np.meshgrid(rng_, rng_, rng_, indexing="ij"), -1).reshape(-1, 3)
    n = n[np.sum(n * n, 1) <= nshell * nshell]
    E = 0.0
    for i in range(len(q)):
        d = pos[None, :, :] - pos[i][None, None, :] + n[:, None, :] * L   # (nimg, N, 3)
        r = np.linalg.norm(d, axis=2)
        self_ = (np.all(n == 0, 1)[:, None]) & (np.arange(len(q))[None, :] == i)
        E += 0.5 * q[i] * np.sum(np.where(self_, 0.0, q[None, :] / np.where(self_, 1.0, r)))
    return O.KE * E


def test_brute_force_spherical_lattice_sum():
    """de Leeuw-Perram-Smith: the sum over images in growing spheres tends to
    E_Ewald + (2 pi KE / 3V) |sum q_i r_i|^2."""
    L = 6.0
    pos = np.array([[0.5, 0.7, 0.9], [2.9, 1.1, 3.5], [4.2, 4.6, 1.3], [1.7, 5.1, 4.4]])
    q = np.array([1.0, -0.6, 0.9, -1.3])
    r = O.ewald_direct(pos, q, [L, L, L], 0.6, 8.0, 12)
    dip = q @ pos
    target = r["E"] + 2 * math.pi * O.KE / (3 * L ** 3) * dip @ dip
    errs = [abs(_spherical_sum(pos, q, L, m) - target) for m in (8, 16, 24)]
    assert errs[0] > errs[1] > errs[2]
    # the dipole term is about half of the energy here, so a wrong reciprocal
    # normalisation or sign could not reach this agreement
    assert errs[2] < 5e-6 * abs(target)


# Madelung constants of two more binary crystals (textbook values, per ion pair,
# referred to the nearest-neighbour distance): their geometries differ from
# rock salt, so a wrong image set, k-vector set or self term would not match
# all three.
MADELUNG_CSCL = 1.762674773
MADELUNG_ZINCBLENDE = 1.638055053


def _crystal(basis, charges, ncell, a):
    cells = np.stack(np.meshgrid(*[np.arange(ncell)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = (cells[:, None, :] + np.asarray(basis)[None, :, :]).reshape(-1, 3) * a
    q = np.tile(np.asarray(charges, dtype=np.float64), len(cells))
    return pos, q, [ncell * a] * 3


@pytest.mark.parametrize("name", ["cscl", "zincblende"])
def test_madelung_constants_of_other_lattices(name):
    a = 4.0
    if name == "cscl":
        basis, charges, r0, M = [[0, 0, 0], [0.5, 0.5, 0.5]], [1, -1], a * math.sqrt(3) / 2, MADELUNG_CSCL
    else:
        fcc = [[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]]
        basis = fcc + [[x + 0.25, y + 0.25, z + 0.25] for x, y, z in fcc]
        charges, r0, M = [1] * 4 + [-1] * 4, a * math.sqrt(3) / 4, MADELUNG_ZINCBLENDE
    pos, q, box = _crystal(basis, charges, 3, a)
    # rc 11 A, alpha 0.5/A, kmax 12: both truncations far below the tolerance
    r = O.ewald_direct(pos, q, box, 0.5, 11.0, 12)
    qphi = q * r["phi"]
    assert np.ptp(qphi) < 1e-9                  # all ions equivalent
    assert abs(-qphi.mean() * r0 / O.KE - M) < 1e-9
