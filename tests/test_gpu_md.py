"""Shadow XL-BOMD on the GPU (pq_md_run): trajectory parity with the FP64
oracle integrator over a few steps, and energy conservation of a longer NVE
run (the paper's validation criterion for shadow MD, Section "Validation and
Performance": the total energy's fluctuation)."""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import md as M
from oracle import qeq as Q

pytestmark = pytest.mark.gpu

COUL = dict(method="pme", alpha=0.35, rc=6.0, grid=16, order=6)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2503_21176_amd as P
    P.load()
    return P


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def initial_state(n, seed, L=None):
    L = L or (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=seed)
    rng = np.random.default_rng(seed + 1)
    eta = rng.uniform(20.0, 25.0, n)           # well-posed hardness (positive-definite C)
    mass = rng.choice([16.0, 23.0, 35.5], n)
    vel = rng.normal(0.0, 1.0, (n, 3)) * np.sqrt(0.02585 * M.ACC / mass)[:, None]   # ~300 K
    return s, eta, mass, vel


@pytest.mark.parametrize("dissipation", [5, 0])
def test_md_matches_oracle(P, dissipation):
    n, steps = 64, 4
    s, eta, mass, vel = initial_state(n, 21)
    A = Q.coulomb_matrix(s.pos, s.box, COUL)
    qstar, _ = Q.qeq_dense(A, s.chi, eta, 0.0)
    H = P.md_history(dissipation)
    hist = np.tile(qstar, (H, 1))
    kw = dict(dt=0.5, n_krylov=6, dissipation=dissipation, kappa=1.9, rep_a=400.0, rep_rho=0.25)
    po, vo, ho, eo = M.md_run(s.pos, vel, mass, s.box, COUL, s.chi, eta, hist, steps, **kw)
    say(f"[md] n={n} steps={steps} dissipation={dissipation} L={s.box[0]:.3f}")
    ctx = P.Context(0)
    prm = P.make_params(s.box, COUL["rc"], COUL["alpha"], grid=COUL["grid"], order=COUL["order"])
    pos, v, h = gpu(s.pos), gpu(vel), gpu(hist)
    ctx.set_system(pos, prm)
    e = ctx.md_run(pos, v, gpu(mass), gpu(s.chi), gpu(eta), h, steps, dt_fs=0.5, n_krylov=6,
                   dissipation=dissipation, kappa=1.9, rep_a=400.0, rep_rho=0.25)
    pos, v, h = pos.cpu().numpy(), v.cpu().numpy(), h.cpu().numpy()
    ctx.close()
    dpos = np.abs((pos - s.pos) - (po - s.pos)).max() / np.abs(po - s.pos).max()
    dvel = np.abs(v - vo).max() / np.abs(vo).max()
    dn = np.abs(h - ho).max() / np.abs(ho).max()
    de = np.abs(e[:, :4] - eo).max() / np.abs(eo[:, 1]).max()
    say(f"[md] displacement {dpos:.2e} velocity {dvel:.2e} n {dn:.2e} energies {de:.2e}; "
        f"E_tot {e[0, 3]:.8f} -> {e[-1, 3]:.8f} (oracle {eo[-1, 3]:.8f})")
    assert dpos < 1e-5 and dvel < 1e-5
    assert dn < 1e-4
    assert de < 1e-5


def test_md_nve_energy_conservation(P):
    n, steps = 300, 400
    s, eta, mass, vel = initial_state(n, 31)
    prm = P.make_params(s.box, 7.0, 0.4, grid=24, order=6)
    ctx = P.Context(0)
    pos = gpu(s.pos)
    ctx.set_system(pos, prm)
    r = ctx.qeq_solve(gpu(s.chi), gpu(eta), tol=1e-10, max_it=400, restart=400)
    H = P.md_history(5)
    hist = r.q.reshape(1, n).repeat(H, 1).contiguous()
    e = ctx.md_run(pos, gpu(vel), gpu(mass), gpu(s.chi), gpu(eta), hist, steps, dt_fs=0.5, n_krylov=6,
                   dissipation=5, rep_a=400.0, rep_rho=0.25)
    ctx.close()
    tot, ke = e[:, 3], e[:, 0]
    t = np.arange(len(tot)) * 0.5e-3   # ps
    slope = np.polyfit(t, tot, 1)[0]
    say(f"[md-nve] n={n} {steps} steps of 0.5 fs: E_tot std {tot.std():.3e} eV, drift {slope:.3e} eV/ps, "
        f"KE std {ke.std():.3e} eV, KE mean {ke.mean():.4f} eV")
    assert np.all(np.isfinite(e))
    # the total energy is conserved far better than its parts exchange energy
    assert tot.std() < 0.02 * ke.std()
    assert abs(slope) * t[-1] < 0.05 * ke.std()


def test_regular_bo_md_matches_oracle(P):
    # tight solves (1e-7: FP32-bulk products reach residuals of a few 1e-8):
    # the trajectory follows the oracle's exact-charge BO-MD
    n, steps = 64, 3
    s, eta, mass, vel = initial_state(n, 23)
    po, vo, _, eo = M.md_run(s.pos, vel, mass, s.box, COUL, s.chi, eta, np.zeros((2, n)), steps, dt=0.5,
                             rep_a=400.0, rep_rho=0.25, regular=True)
    ctx = P.Context(0)
    prm = P.make_params(s.box, COUL["rc"], COUL["alpha"], grid=COUL["grid"], order=COUL["order"])
    pos, v = gpu(s.pos), gpu(vel)
    ctx.set_system(pos, prm)
    h = gpu(np.zeros((P.md_history(0), n)))
    e = ctx.md_run(pos, v, gpu(mass), gpu(s.chi), gpu(eta), h, steps, dt_fs=0.5, dissipation=0, rep_a=400.0,
                   rep_rho=0.25, regular=True, tol=1e-7, max_it=300, restart=80)
    pos, v, h = pos.cpu().numpy(), v.cpu().numpy(), h.cpu().numpy()
    ctx.close()
    dpos = np.abs((pos - s.pos) - (po - s.pos)).max() / np.abs(po - s.pos).max()
    dvel = np.abs(v - vo).max() / np.abs(vo).max()
    de = np.abs(e[:, :4] - eo).max() / np.abs(eo[:, 1]).max()
    say(f"[md-regular] displacement {dpos:.2e} velocity {dvel:.2e} energies {de:.2e}; "
        f"Coulomb evaluations per step {e[1:, 4].tolist()}")
    assert dpos < 1e-5 and dvel < 1e-5 and de < 1e-5
    assert np.all(e[1:, 4] >= 2) and np.all(e[1:, 4] < 300)   # every solve converged
    assert abs(h[0].sum()) < 1e-6   # the last charges come back in n_hist[0], neutral to the tolerance
