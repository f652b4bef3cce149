"""Parity of the device QEQ solver, shadow step and adjoint with the FP64
dense oracle built from the same Coulomb operator (same alpha, cutoff, grid,
order).

The operator products are FP32-bulk Coulomb evaluations with a relative
error of ~3e-7, so a solution differs from the dense FP64 solution by up to
cond(M) times that. The tests therefore check (a) the backward error: the
residual of the GPU solution in the oracle's FP64 bordered system, which does
not depend on the conditioning, and (b) the forward error against a bound of
30 * cond(M) * 1e-6 (relative).
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import grad as G
from oracle import qeq as Q

pytestmark = pytest.mark.gpu

EPS_OP = 1e-6   # bound on the relative error of one FP32-bulk operator product


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


def host(t):
    return t.detach().cpu().numpy()


COUL = dict(method="pme", alpha=0.5, rc=5.0, grid=16, order=5)


@pytest.fixture(scope="module")
def system():
    """Well-posed QEQ: hardness U(20, 25) eV exceeds the largest pair Coulomb
    coupling (KE/1 A = 14.4 eV plus the self-image term), so C is positive
    definite (cond(M) ~ 14)."""
    n = 120
    L = (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=321)
    s.eta = np.random.default_rng(1).uniform(20.0, 25.0, n)
    A = Q.coulomb_matrix(s.pos, s.box, COUL)
    return s, COUL, A


@pytest.fixture(scope="module")
def system_workload():
    """The workloads' hardness U(5, 10) eV with 1 A minimum separations: C is
    indefinite (about half the eigenvalues negative); restarted GMRES
    stagnates on it, full GMRES converges."""
    n = 120
    L = (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=321)
    A = Q.coulomb_matrix(s.pos, s.box, COUL)
    return s, COUL, A


def make_ctx(P, s, coul):
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), P.make_params(s.box, coul["rc"], coul["alpha"], grid=coul["grid"],
                                             order=coul["order"]))
    return ctx


@pytest.mark.parametrize("which,restart,q0,tol", [("posdef", 50, False, 1e-7), ("posdef", 6, True, 1e-7),
                                                  ("workload", 128, False, 1e-6)])
def test_qeq_solve_matches_dense(P, system, system_workload, which, restart, q0, tol):
    s, coul, A = system if which == "posdef" else system_workload
    say(f"[qeq-{which}] n={s.n} restart={restart} q0={q0} tol={tol}")
    ctx = make_ctx(P, s, coul)
    q0v = gpu(np.random.default_rng(3).normal(0, 0.2, s.n)) if q0 else None
    r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta), q_tot=0.0, tol=tol, max_it=400, restart=restart, q0=q0v,
                      force=True)
    torch.cuda.synchronize()
    q = host(r.q)
    qd, lam = Q.qeq_dense(A, s.chi, s.eta, 0.0)
    M = Q.bordered(A, s.eta)
    kappa = np.linalg.cond(M)
    back = Q.bordered_residual(A, s.chi, s.eta, 0.0, q, r.lam)
    fwd = np.linalg.norm(q - qd) / np.linalg.norm(qd)
    say(f"[qeq] its={r.iterations} restarts={r.restarts} gpu relres={r.rel_residual:.2e} "
        f"oracle backward err={back:.2e} forward err={fwd:.2e} cond={kappa:.1f}")
    assert r.status == 0
    # the charge constraint is the last row of the bordered system: it holds
    # to the solve's residual, |sum q - Q_tot| <= back * ||b||
    assert abs(q.sum()) <= back * np.linalg.norm(np.concatenate([s.chi, [0.0]])) + 1e-12
    assert back < 5e-6
    assert fwd < 30 * kappa * EPS_OP
    assert abs(r.lam - lam) < 30 * kappa * EPS_OP * max(1.0, abs(lam))
    if restart < 20:
        assert r.restarts >= 1
    # energy and force at the solution
    E = float(host(r.energy)[0])
    Ed = Q.qeq_energy(A, s.chi, s.eta, qd)
    assert abs(E - Ed) < 1e-5 * abs(Ed)
    Fd = Q.force(s.pos, qd, s.box, coul)
    F = host(r.force)
    assert np.linalg.norm(F - Fd) / np.linalg.norm(Fd) < 30 * kappa * EPS_OP
    ctx.close()


def test_qeq_not_converged_returns_warning(P, system, system_workload):
    s, coul, A = system
    ctx = make_ctx(P, s, coul)
    r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta), tol=1e-12, max_it=3, restart=50)
    assert r.status == P.PQ_WARN_NOT_CONVERGED
    assert r.iterations <= 4 and r.rel_residual > 1e-12
    ctx.close()
    # indefinite workload system, restarted GMRES(20): stagnates; the reported
    # residual is the true residual of the returned iterate
    s, coul, A = system_workload
    ctx = make_ctx(P, s, coul)
    r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta), tol=1e-6, max_it=60, restart=20)
    torch.cuda.synchronize()
    back = Q.bordered_residual(A, s.chi, s.eta, 0.0, host(r.q), r.lam)
    say(f"[qeq-stagnation] status={r.status} its={r.iterations} relres={r.rel_residual:.3e} oracle={back:.3e}")
    assert r.status == P.PQ_WARN_NOT_CONVERGED
    assert abs(r.rel_residual - back) < 1e-3 * back + 1e-6
    ctx.close()


def test_shadow_step_matches_dense(P, system):
    s, coul, A = system
    qstar, _ = Q.qeq_dense(A, s.chi, s.eta, 0.0)
    n_vec = qstar + np.random.default_rng(4).normal(0, 0.05, s.n)
    say(f"[shadow] n={s.n} n_krylov=8")
    ctx = make_ctx(P, s, coul)
    q, F, x, e = ctx.shadow_step(gpu(s.chi), gpu(s.eta), gpu(n_vec), q_tot=0.0, n_krylov=8)
    torch.cuda.synchronize()
    qo, lamo, xo = Q.shadow_step_dense(A, s.chi, s.eta, n_vec, 0.0, 8)
    Fo = Q.force(s.pos, qo, s.box, coul) - Q.force(s.pos, qo - n_vec, s.box, coul)
    Eo = Q.shadow_energy(A, s.chi, s.eta, qo, n_vec)
    eq = np.linalg.norm(host(q) - qo) / np.linalg.norm(qo)
    ex = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    eF = np.linalg.norm(host(F) - Fo) / np.linalg.norm(Fo)
    ee = host(e)
    say(f"[shadow] q err {eq:.2e}  x err {ex:.2e}  F err {eF:.2e}  E {ee[0]:.9g} vs {Eo:.9g}  "
        f"lambda {ee[1]:.9g} vs {lamo:.9g}")
    assert eq < 1e-5
    assert eF < 1e-5
    assert ex < 1e-4
    assert abs(ee[0] - Eo) < 1e-5 * abs(Eo)
    assert abs(ee[1] - lamo) < 1e-5 * max(1.0, abs(lamo))
    assert abs(host(q).sum()) < 1e-10
    ctx.close()


def test_shadow_fixed_point(P, system):
    """At n = q* the shadow charges reproduce q* and the shadow force is the
    regular Born-Oppenheimer force."""
    s, coul, A = system
    qstar, _ = Q.qeq_dense(A, s.chi, s.eta, 0.0)
    ctx = make_ctx(P, s, coul)
    q, F, x, e = ctx.shadow_step(gpu(s.chi), gpu(s.eta), gpu(qstar), n_krylov=4)
    torch.cuda.synchronize()
    assert np.linalg.norm(host(q) - qstar) / np.linalg.norm(qstar) < 1e-5
    Fbo = Q.force(s.pos, qstar, s.box, coul)
    assert np.linalg.norm(host(F) - Fbo) / np.linalg.norm(Fbo) < 1e-5
    # the Krylov right-hand side is ~0, so is the solution
    assert np.abs(host(x)).max() < 1e-3 * np.abs(qstar).max()
    ctx.close()


def test_vjp_energy_envelope(P, system):
    s, coul, A = system
    ctx = make_ctx(P, s, coul)
    r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta), tol=1e-9, max_it=400)
    dpos, dchi, deta = ctx.qeq_vjp(gpu(s.chi), gpu(s.eta), r.q)
    torch.cuda.synchronize()
    _, qd, dR, dc, de = G.qeq_energy_and_grad(s.pos, s.box, coul, s.chi, s.eta)
    kappa = np.linalg.cond(Q.bordered(A, s.eta))
    tol = 30 * kappa * EPS_OP
    say(f"[vjp-energy] dR err {np.linalg.norm(host(dpos) - dR) / np.linalg.norm(dR):.2e} tol {tol:.1e}")
    assert np.linalg.norm(host(dpos) - dR) / np.linalg.norm(dR) < tol
    assert np.linalg.norm(host(dchi) - dc) / np.linalg.norm(dc) < tol
    assert np.linalg.norm(host(deta) - de) / np.linalg.norm(de) < 2 * tol
    ctx.close()


def test_vjp_general_upstream(P, system):
    s, coul, A = system
    g = np.random.default_rng(8).normal(size=s.n)
    ctx = make_ctx(P, s, coul)
    r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta), tol=1e-9, max_it=400)
    dpos, dchi, deta = ctx.qeq_vjp(gpu(s.chi), gpu(s.eta), r.q, gpu(g), tol=1e-9)
    torch.cuda.synchronize()
    dR, dc, de = G.qeq_vjp(s.pos, s.box, coul, s.chi, s.eta, g)
    kappa = np.linalg.cond(Q.bordered(A, s.eta))
    tol = 30 * kappa * EPS_OP
    errs = [np.linalg.norm(host(a) - b) / np.linalg.norm(b) for a, b in ((dpos, dR), (dchi, dc), (deta, de))]
    say(f"[vjp-general] errs {errs} tol {tol:.1e}")
    assert max(errs) < 3 * tol
    ctx.close()


def test_autograd_function(P, system):
    s, coul, A = system
    ctx = make_ctx(P, s, coul)
    pos = gpu(s.pos).requires_grad_(True)
    chi = gpu(s.chi).requires_grad_(True)
    eta = gpu(s.eta).requires_grad_(True)
    E = P.QEQEnergy.apply(pos, chi, eta, ctx, 0.0, 1e-9)
    E.backward()
    _, qd, dR, dc, de = G.qeq_energy_and_grad(s.pos, s.box, coul, s.chi, s.eta)
    kappa = np.linalg.cond(Q.bordered(A, s.eta))
    assert np.linalg.norm(host(pos.grad) - dR) / np.linalg.norm(dR) < 30 * kappa * EPS_OP
    assert np.linalg.norm(host(chi.grad) - dc) / np.linalg.norm(dc) < 30 * kappa * EPS_OP
    # charges function: gradient of sum(w * q*) equals the general VJP
    w = np.random.default_rng(9).normal(size=s.n)
    chi2 = gpu(s.chi).requires_grad_(True)
    qs = P.QEQCharges.apply(gpu(s.pos), chi2, gpu(s.eta), ctx, 0.0, 1e-9)
    (qs * gpu(w)).sum().backward()
    _, dcw, _ = G.qeq_vjp(s.pos, s.box, coul, s.chi, s.eta, w)
    assert np.linalg.norm(host(chi2.grad) - dcw) / np.linalg.norm(dcw) < 90 * kappa * EPS_OP
    ctx.close()


def test_graph_replays_match_direct_launches(P, system):
    """Each Arnoldi step is one replay of a captured HIP graph, with the
    solver's own eager kernels, copies and host synchronisations between the
    replays; phase-timing mode launches the same kernels directly. Solves with
    several restart cycles (graph reused across cycles and calls) and the
    fixed-length shadow Krylov solve must agree bit for bit with the direct
    launches, on every call."""
    s, coul, A = system
    ctx = make_ctx(P, s, coul)
    n_vec = gpu(Q.qeq_dense(A, s.chi, s.eta, 0.0)[0] + np.random.default_rng(5).normal(0, 0.05, s.n))
    runs = {}
    for mode in (0, 1, 0, 1, 0):
        ctx.set_timing(mode)
        r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta), tol=1e-7, max_it=400, restart=6)
        q, F, x, e = ctx.shadow_step(gpu(s.chi), gpu(s.eta), n_vec, n_krylov=8)
        torch.cuda.synchronize()
        runs.setdefault(mode, []).append((host(r.q), r.iterations, r.restarts, host(x), host(q)))
        if mode:
            ctx.timings()
    ctx.close()
    ref = runs[1][0]
    say(f"[graph] its {ref[1]} restarts {ref[2]}, {len(runs[0])} graph runs, {len(runs[1])} direct runs")
    assert ref[2] >= 2
    for run in runs[0] + runs[1]:
        assert np.array_equal(run[0], ref[0])
        assert run[1:3] == ref[1:3]
        assert np.array_equal(run[3], ref[3])
        assert np.array_equal(run[4], ref[4])
