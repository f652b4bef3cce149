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


@pytest.mark.parametrize("dissipation,skin", [(5, 0.0), (0, 0.0), (5, 1.0)])
def test_md_matches_oracle(P, dissipation, skin):
    n, steps = 64, 4
    s, eta, mass, vel = initial_state(n, 21)
    A = Q.coulomb_matrix(s.pos, s.box, COUL)
    qstar, _ = Q.qeq_dense(A, s.chi, eta, 0.0)
    H = P.md_history(dissipation)
    hist = np.tile(qstar, (H, 1))
    kw = dict(dt=0.5, n_krylov=6, dissipation=dissipation, kappa=1.9, rep_a=400.0, rep_rho=0.25)
    po, vo, ho, eo = M.md_run(s.pos, vel, mass, s.box, COUL, s.chi, eta, hist, steps, **kw)
    say(f"[md] n={n} steps={steps} dissipation={dissipation} skin={skin} L={s.box[0]:.3f}")
    ctx = P.Context(0)
    prm = P.make_params(s.box, COUL["rc"], COUL["alpha"], skin=skin, grid=COUL["grid"], order=COUL["order"])
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
    if skin > 0:
        assert e[1:, 5].sum() == 0      # the moves stay within skin/2: the list is kept


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


@pytest.mark.parametrize("fp64", [False, True])
def test_update_positions_keeps_the_list_and_the_pair_set(P, fp64):
    """Moves within skin/2 keep the list (no cluster-pair search); the pair
    set is then exactly the oracle's at rc on the new positions, including
    atoms that crossed a face of the cell, and the evaluation matches the
    oracle there (FP32 form to 1e-5, FP64 form to 1e-10). A move beyond
    skin/2 rebuilds."""
    import oracle as O
    from _parity import elem_err
    n, rc, skin = 2000, 8.0, 1.0
    s = W.small_random(n, (n / 0.1) ** (1 / 3), seed=41)
    L = s.box[0]
    a = 0.35
    prm = P.make_params(s.box, rc, a, skin=skin, grid=32, order=5, fp64=fp64)
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), prm)
    rng = np.random.default_rng(42)
    d = rng.normal(size=(n, 3))
    d *= (0.45 * skin / 2) / np.linalg.norm(d, axis=1).max()
    w = np.mod(s.pos, L)
    near = np.where(w[:, 0] > L - 0.3)[0]          # these cross the x face
    d[near] = [0.24, 0.0, 0.0]
    new = s.pos + d
    rebuilt = ctx.update_positions(gpu(new))
    got = ctx.neighbor_pairs().cpu().numpy().astype(np.int64)
    got = got[np.lexsort((got[:, 4], got[:, 3], got[:, 2], got[:, 1], got[:, 0]))]
    want = O.neighbor_pairs(new, s.box, rc)
    say(f"[update] kept={not rebuilt} pairs {len(got)} vs {len(want)}, {len(near)} atoms crossed the x face")
    assert not rebuilt and len(near) > 0
    assert np.array_equal(got, want)
    # the ELLPACK form of the kept list: rows at rc with the current images
    from _parity import ell_from_pairs
    nbr, img, cnt = ctx.neighbor_ell()
    e_nbr, e_img, e_cnt = ell_from_pairs(want, n)
    assert np.array_equal(cnt.cpu().numpy(), e_cnt)
    assert np.array_equal(nbr.cpu().numpy(), e_nbr) and np.array_equal(img.cpu().numpy(), e_img)
    phi, F, E = ctx.coulomb(gpu(s.q))
    ref = O.spme_full(new, s.q, s.box, a, rc, 32, 5)
    ephi = np.linalg.norm(phi.cpu().numpy() - ref["phi"]) / np.linalg.norm(ref["phi"])
    mf = elem_err(F.cpu().numpy(), ref["F"])
    say(f"[update fp64={fp64}] phi rel {ephi:.2e}, per-atom F {mf:.2e}")
    tol = 1e-10 if fp64 else 1e-5
    assert ephi < tol and mf < tol
    # one atom beyond skin/2: a full build
    far = new.copy()
    far[7] += [0.6 * skin, 0.0, 0.0]
    assert ctx.update_positions(gpu(far))
    got = ctx.neighbor_pairs().cpu().numpy().astype(np.int64)
    assert len(got) == len(O.neighbor_pairs(far, s.box, rc + skin))
    ctx.close()


def test_md_skin_reuse_pairs_exact_every_step(P):
    """Shadow MD with a 1 A skin: the list is rebuilt on fewer steps than it
    is used, and after every step the pair set is the oracle's at rc."""
    import oracle as O
    n, steps = 300, 24
    s, eta, mass, vel = initial_state(n, 51)
    vel *= 3.0                                     # hot: atoms cross skin/2 within the run
    prm = P.make_params(s.box, 7.0, 0.4, skin=1.0, grid=24, order=6)
    ctx = P.Context(0)
    pos = gpu(s.pos)
    ctx.set_system(pos, prm)
    r = ctx.qeq_solve(gpu(s.chi), gpu(eta), tol=1e-8, max_it=400, restart=400)
    hist = r.q.reshape(1, n).repeat(P.md_history(5), 1).contiguous()
    v, ref = gpu(vel), pos.clone()
    rebuilt = []
    for t in range(steps):
        e = ctx.md_run(pos, v, gpu(mass), gpu(s.chi), gpu(eta), hist, 1, dt_fs=1.0, n_krylov=4, dissipation=5,
                       rep_a=400.0, rep_rho=0.25, pos_ref=ref)
        rebuilt.append(int(e[1, 5]))
        got = ctx.neighbor_pairs().cpu().numpy().astype(np.int64)
        got = got[np.lexsort((got[:, 4], got[:, 3], got[:, 2], got[:, 1], got[:, 0]))]
        cut = 7.0 + (1.0 if rebuilt[-1] else 0.0)   # a fresh build exports rc + skin
        want = O.neighbor_pairs(pos.cpu().numpy(), s.box, cut)
        assert np.array_equal(got, want), (t, len(got), len(want))
    ctx.close()
    say(f"[md-skin] rebuilt on {sum(rebuilt)} of {steps} steps: {rebuilt}")
    assert 0 < sum(rebuilt) < steps


def test_md_checkpoint_resume_is_bit_identical(P, tmp_path):
    n, steps = 200, 16
    s, eta, mass, vel = initial_state(n, 61)
    vel *= 3.0
    prm = P.make_params(s.box, 7.0, 0.4, skin=1.0, grid=24, order=6)
    H = P.md_history(5)

    def fresh():
        ctx = P.Context(0)
        pos = gpu(s.pos)
        ctx.set_system(pos, prm)
        r = ctx.qeq_solve(gpu(s.chi), gpu(eta), tol=1e-8, max_it=400, restart=400)
        return ctx, pos, gpu(vel), r.q.reshape(1, n).repeat(H, 1).contiguous(), pos.clone()

    kw = dict(dt_fs=1.0, n_krylov=4, dissipation=5, rep_a=400.0, rep_rho=0.25)
    ctx, pos, v, h, ref = fresh()
    eA = ctx.md_run(pos, v, gpu(mass), gpu(s.chi), gpu(eta), h, steps, pos_ref=ref, **kw)
    A = (pos.clone(), v.clone(), h.clone(), ref.clone())
    ctx.close()
    ctx, pos, v, h, ref = fresh()
    eB1 = ctx.md_run(pos, v, gpu(mass), gpu(s.chi), gpu(eta), h, steps // 2, pos_ref=ref, **kw)
    P.md_state_save(tmp_path / "md.npz", pos, v, h, ref)
    ctx.close()
    ctx = P.Context(0)
    pos, v, h, ref = P.md_state_load(tmp_path / "md.npz")
    ctx.set_system(pos, prm)
    eB2 = ctx.md_run(pos, v, gpu(mass), gpu(s.chi), gpu(eta), h, steps - steps // 2, pos_ref=ref, **kw)
    ctx.close()
    say(f"[md-checkpoint] rebuilds {int(eA[1:, 5].sum())} of {steps}; "
        f"E_tot {eA[-1, 3]:.10f} vs {eB2[-1, 3]:.10f}")
    assert 0 < eA[1:, 5].sum() < steps
    for a, b in zip(A, (pos, v, h, ref)):
        assert torch.equal(a, b)
    assert np.array_equal(eA[:steps // 2 + 1], eB1)
    assert np.array_equal(eA[steps // 2 + 1:, :5], eB2[1:, :5])
