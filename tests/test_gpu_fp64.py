"""Parity of the FP64 form (PQ_FLAG_FP64: every bulk operation in double
precision, as in the paper's timed runs) with the FP64 oracle.

Both sides compute the same smooth-PME / Ewald approximation in FP64 and
differ only in rounding order: sums of at most ~10^4 terms and 3-D FFTs of a
few thousand points lose at most a few hundred ulps, so
  ||dphi||_2 / ||phi||_2 <= 1e-11,  ||dF||_rms / ||F||_rms <= 1e-11,
  |dE| <= 1e-12 (|E_real| + |E_rec| + |E_self+bg|).
The QEQ solve in this form converges to a relative residual of 1e-12; its
charges then agree with the dense FP64 solution to cond(M) * 1e-11.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from _parity import elem_err
from oracle import qeq as Q

pytestmark = pytest.mark.gpu

TOL = 1e-11
TOL_E = 1e-12


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


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rms_rel(a, b):
    return float(np.sqrt(np.mean(np.sum((a - b) ** 2, 1))) / np.sqrt(np.mean(np.sum(b ** 2, 1))))


def run(P, s, params):
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), params)
    phi, F, E = ctx.coulomb(gpu(s.q))
    torch.cuda.synchronize()
    out = phi.cpu().numpy(), F.cpu().numpy(), E.cpu().numpy()
    ctx.close()
    return out


def check(name, phi, F, E, ref, rows=None, energies=True, forces=True):
    if rows is not None:
        phi, F = phi[rows], F[rows]
    ephi, ef = rel2(phi, ref["phi"]), rms_rel(F, ref["F"])
    mphi, mf = elem_err(phi, ref["phi"]), elem_err(F, ref["F"])
    say(f"[fp64 {name}] phi rel {ephi:.2e}  F rms rel {ef:.2e}  per atom: phi {mphi:.2e} F {mf:.2e}")
    assert ephi <= TOL and mphi <= 10 * TOL
    if forces:
        assert ef <= TOL and mf <= 10 * TOL
    if energies:
        scale = abs(ref["E_real"]) + abs(ref["E_rec"]) + abs(ref["E_selfbg"])
        eE = abs(E[0] - ref["E"]) / scale
        say(f"[fp64 {name}] E {E[0]:.15g} vs {ref['E']:.15g} rel(parts) {eE:.2e}")
        assert eE <= TOL_E
        for k, key in ((1, "E_real"), (2, "E_rec"), (3, "E_selfbg")):
            assert abs(E[k] - ref[key]) <= TOL_E * scale


def test_nacl_madelung_fp64(P):
    # at alpha = 0.35, rc = 8, kmax = 8 the Ewald sum of the rock-salt crystal
    # is converged well below 1e-9, so the Madelung constant comes out to
    # the accuracy of the tabulated value
    s = W.nacl()
    prm = P.make_params(s.box, 8.0, 0.35, kmax=8, method="ewald", fp64=True)
    phi, F, E = run(P, s, prm)
    ref = O.ewald_direct(s.pos, s.q, s.box, 0.35, 8.0, 8)
    # every force vanishes by symmetry: both sides hold rounding noise only
    check("nacl-ewald", phi, F, E, ref, forces=False)
    M = -float(np.mean(s.q * phi)) * 2.82 / O.KE
    say(f"[fp64 nacl] Madelung {M:.12f}")
    assert abs(M / 1.747564594633 - 1) < 1.5e-4
    assert np.abs(F).max() < 1e-9


@pytest.mark.parametrize("name", ["cscl", "zincblende"])
def test_madelung_other_lattices_fp64(P, name):
    """CsCl and zinc blende (3x3x3 cubic cells of 4 A, box 12 A, rc 11 A: the
    real-space sum reaches past the nearest image) with the direct Ewald
    method at truncations far below 1e-9: the oracle to 1e-11 and the
    textbook Madelung constants to 1e-9."""
    import math
    a = 4.0
    if name == "cscl":
        basis, charges, r0, M_ref = [[0, 0, 0], [0.5, 0.5, 0.5]], [1, -1], a * math.sqrt(3) / 2, 1.762674773
    else:
        fcc = [[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]]
        basis = fcc + [[x + 0.25, y + 0.25, z + 0.25] for x, y, z in fcc]
        charges, r0, M_ref = [1] * 4 + [-1] * 4, a * math.sqrt(3) / 4, 1.638055053
    cells = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = (cells[:, None, :] + np.asarray(basis, dtype=np.float64)[None]).reshape(-1, 3) * a
    q = np.tile(np.asarray(charges, dtype=np.float64), len(cells))
    box = np.array([3 * a] * 3)
    s = W.System(name, pos, q, box, {})
    prm = P.make_params(box, 11.0, 0.5, kmax=12, method="ewald", fp64=True)
    phi, F, E = run(P, s, prm)
    ref = O.ewald_direct(pos, q, box, 0.5, 11.0, 12)
    check(name, phi, F, E, ref, forces=False)
    M = -float(np.mean(q * phi)) * r0 / O.KE
    say(f"[fp64 {name}] Madelung {M:.12f} (textbook {M_ref})")
    assert abs(M - M_ref) < 1e-9
    assert np.abs(F).max() < 1e-9


@pytest.mark.parametrize("n,order,K", [(64, 5, 10), (300, 6, 16), (300, 4, 15)])
def test_small_boxes_pme_fp64(P, n, order, K):
    L = (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=100 + n)
    a, rc = W.ALPHA_RC9, 9.0
    say(f"[fp64 small-pme] n={n} L={L:.3f} K={K} p={order}")
    phi, F, E = run(P, s, P.make_params(s.box, rc, a, grid=K, order=order, fp64=True))
    check(f"small-pme n={n}", phi, F, E, O.spme_full(s.pos, s.q, s.box, a, rc, K, order))


def test_small_box_ewald_fp64(P):
    n, kmax = 200, 7
    L = (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=200 + n)
    phi, F, E = run(P, s, P.make_params(s.box, 9.0, 0.35, kmax=kmax, method="ewald", fp64=True))
    check("small-ewald", phi, F, E, O.ewald_direct(s.pos, s.q, s.box, 0.35, 9.0, kmax))


def test_anisotropic_non_neutral_fp64(P):
    rng = np.random.default_rng(7)
    box = np.array([17.0, 21.0, 25.0])
    n = 700
    pos = rng.uniform(-30, 60, size=(n, 3))
    q = rng.normal(0.3, 1.0, size=n)
    s = W.System("aniso", pos, q, box)
    phi, F, E = run(P, s, P.make_params(box, 7.5, 0.4, grid=(20, 24, 30), order=6, fp64=True))
    check("aniso", phi, F, E, O.spme_full(pos, q, box, 0.4, 7.5, (20, 24, 30), 6))


def test_random_ionic_3000_fp64(P):
    s = W.random_ionic(n=3000, seed=9, grid=None, order=6)
    phi, F, E = run(P, s, P.make_params(s.box, 10.0, W.ALPHA_RC10, grid=32, order=6, fp64=True))
    check("ionic-3000", phi, F, E, O.spme_full(s.pos, s.q, s.box, W.ALPHA_RC10, 10.0, 32, 6))


def test_fp64_and_fp32_forms_agree_and_repeat(P):
    # the two forms of one system differ by the FP32 rounding only, and each
    # form is bitwise reproducible
    s = W.random_ionic(n=3000, seed=12, grid=None, order=6)
    p32 = P.make_params(s.box, 10.0, W.ALPHA_RC10, grid=32, order=6)
    p64 = P.make_params(s.box, 10.0, W.ALPHA_RC10, grid=32, order=6, fp64=True)
    a = run(P, s, p64)
    b = run(P, s, p64)
    c = run(P, s, p32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    say(f"[fp64 vs fp32] phi {rel2(c[0], a[0]):.2e} F {rms_rel(c[1], a[1]):.2e}")
    assert rel2(c[0], a[0]) < 1e-5
    assert rms_rel(c[1], a[1]) < 1e-5


def test_switch_precision_on_one_context(P):
    # one context, FP32 then FP64 then FP32 again: buffers are re-typed
    s = W.small_random(300, (300 / 0.1) ** (1 / 3), seed=400)
    a, rc, K, p = W.ALPHA_RC9, 9.0, 16, 6
    ref = O.spme_full(s.pos, s.q, s.box, a, rc, K, p)
    ctx = P.Context(0)
    errs = []
    for fp64 in (False, True, False):
        ctx.set_system(gpu(s.pos), P.make_params(s.box, rc, a, grid=K, order=p, fp64=fp64))
        phi, F, E = ctx.coulomb(gpu(s.q))
        errs.append(rel2(phi.cpu().numpy(), ref["phi"]))
    ctx.close()
    say(f"[fp64 switch] phi rel {errs}")
    assert errs[0] < 1e-5 and errs[2] < 1e-5 and errs[1] < TOL


def test_qeq_solve_fp64(P):
    coul = dict(method="pme", alpha=0.5, rc=5.0, grid=16, order=5)
    n = 120
    L = (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=321)
    eta = np.random.default_rng(1).uniform(20.0, 25.0, n)
    A = Q.coulomb_matrix(s.pos, s.box, coul)
    qd, lam = Q.qeq_dense(A, s.chi, eta, 0.0)
    kappa = np.linalg.cond(Q.bordered(A, eta))
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), P.make_params(s.box, coul["rc"], coul["alpha"], grid=16, order=5, fp64=True))
    r = ctx.qeq_solve(gpu(s.chi), gpu(eta), tol=1e-12, max_it=300, restart=50)
    q = r.q.cpu().numpy()
    back = Q.bordered_residual(A, s.chi, eta, 0.0, q, r.lam)
    say(f"[fp64 qeq] its {r.iterations} relres {r.rel_residual:.2e} oracle residual {back:.2e} "
        f"q err {rel2(q, qd):.2e} cond {kappa:.1f}")
    assert r.status == 0
    assert back < 1e-11
    assert rel2(q, qd) < kappa * 1e-11
    assert abs(r.lam - lam) <= kappa * 1e-11 * abs(lam)
    ctx.close()
