"""Edge cases on the GPU against the FP64 oracle: every FFT path (grid sizes
with two register radices and sizes that take the Stockham passes, mixed in
one box), a single charge and a pair in boxes shorter than the cutoff (only
periodic images interact), the rejected empty system, zero and doubled
charges (exact zeros; exact linear and quadratic scaling), and every subset
of the outputs (bitwise the full call's values)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from _parity import elem_err

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def run(P, pos, q, box, prm):
    ctx = P.Context(0)
    ctx.set_system(gpu(pos), prm)
    phi, F, E = ctx.coulomb(gpu(q))
    torch.cuda.synchronize()
    out = phi.cpu().numpy(), F.cpu().numpy(), E.cpu().numpy()
    ctx.close()
    return out


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rms_rel(a, b):
    return float(np.sqrt(np.mean(np.sum((a - b) ** 2, 1))) / np.sqrt(np.mean(np.sum(b ** 2, 1))))


# Two register radices: 20 = 5*4, 27 = 9*3, 45 = 9*5, 81 = 9*9, 48 = 16*3, and
# with the composite radices 30 = 6*5, 50 = 10*5, 54 = 9*6, 60 = 10*6, 90 = 10*9,
# 96 = 12*8, 100 = 10*10, 120 = 12*10; 75 and 108 take the Stockham passes.
# The mixed cases take different paths per axis.
@pytest.mark.parametrize("grid", [(20, 20, 20), (27, 27, 27), (30, 30, 30), (45, 45, 45), (50, 50, 50),
                                  (54, 54, 54), (60, 60, 60), (81, 81, 81), (30, 48, 27), (90, 96, 100),
                                  (120, 75, 108)])
def test_fft_paths(P, grid):
    n = 400
    L = (n / 0.1) ** (1 / 3)
    s = W.small_random(n, L, seed=900 + sum(grid))
    box = np.array([L, L * 1.05, L * 0.95])
    a, rc, p = 0.35, 7.0, 5
    phi, F, E = run(P, s.pos, s.q, box, P.make_params(box, rc, a, grid=grid, order=p))
    ref = O.spme_full(s.pos, s.q, box, a, rc, grid, p)
    ep, ef = rel2(phi, ref["phi"]), rms_rel(F, ref["F"])
    mp, mf = elem_err(phi, ref["phi"]), elem_err(F, ref["F"])
    scale = abs(ref["E_real"]) + abs(ref["E_rec"]) + abs(ref["E_selfbg"])
    ee = abs(E[0] - ref["E"]) / scale
    say(f"[fft {grid}] phi {ep:.2e} F {ef:.2e} E {ee:.2e} per atom: phi {mp:.2e} F {mf:.2e}")
    assert ep < TOL and ef < TOL and ee < 1e-6
    assert mp < TOL and mf < TOL
    assert abs(E[2] - ref["E_rec"]) < 1e-6 * scale


@pytest.mark.parametrize("method", ["pme", "ewald"])
def test_single_charge_sees_only_its_images(P, method):
    # one charge in a 6 A box with rc 5 A: the real-space sum runs over its own
    # images only, and the charge is not neutral (background term)
    box = np.array([6.0, 6.0, 6.0])
    pos, q = np.array([[1.2, 3.4, 5.1]]), np.array([1.0])
    a, rc = 0.45, 5.0
    if method == "pme":
        prm, ref = (P.make_params(box, rc, a, grid=16, order=6), O.spme_full(pos, q, box, a, rc, 16, 6))
    else:
        prm, ref = (P.make_params(box, rc, a, kmax=8, method="ewald"), O.ewald_direct(pos, q, box, a, rc, 8))
    phi, F, E = run(P, pos, q, box, prm)
    say(f"[one charge {method}] phi {phi[0]:.9f} vs {ref['phi'][0]:.9f}  |F| {np.abs(F).max():.2e}")
    assert abs(phi[0] - ref["phi"][0]) < TOL * abs(ref["phi"][0])
    # a lone charge feels no net force (its images are symmetric about it)
    assert np.abs(F).max() < 1e-4


def test_two_charges_in_a_short_box(P):
    box = np.array([7.0, 5.5, 6.5])
    pos = np.array([[0.3, 0.2, 0.1], [2.9, 4.7, 5.8]])
    q = np.array([0.7, -0.7])
    a, rc = 0.4, 6.0
    phi, F, E = run(P, pos, q, box, P.make_params(box, rc, a, grid=(16, 12, 15), order=5))
    ref = O.spme_full(pos, q, box, a, rc, (16, 12, 15), 5)
    say(f"[two charges] phi {rel2(phi, ref['phi']):.2e} F {rms_rel(F, ref['F']):.2e}")
    assert rel2(phi, ref["phi"]) < TOL and rms_rel(F, ref["F"]) < TOL
    assert np.allclose(F[0], -F[1], rtol=1e-4, atol=1e-6)   # action and reaction


def test_empty_system_is_rejected(P):
    ctx = P.Context(0)
    with pytest.raises((P.PQError, ValueError)):
        ctx.set_system(torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                       P.make_params(10.0, 4.0, 0.5, grid=16, order=4))
    ctx.close()


@pytest.mark.parametrize("method,fp64", [("pme", False), ("pme", True), ("ewald", False)])
def test_zero_and_scaled_charges(P, method, fp64):
    """The potential is linear and the forces and energy quadratic in the
    charges (eqs. ewald_real/rec/self): zero charges give exact zeros, and
    doubling the charges, which every floating-point step carries exactly,
    doubles phi and quadruples F and E bit for bit, on a 3000-atom system."""
    s = W.random_ionic(n=3000, seed=17)
    if method == "pme":
        prm = P.make_params(s.box, 9.0, W.ALPHA_RC9, grid=32, order=6, fp64=fp64)
    else:
        prm = P.make_params(s.box, 9.0, W.ALPHA_RC9, kmax=6, method="ewald", fp64=fp64)
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), prm)
    outs = []
    for scale in (0.0, 1.0, 2.0):
        phi, F, E = ctx.coulomb(gpu(scale * s.q))
        torch.cuda.synchronize()
        outs.append((phi.cpu().numpy(), F.cpu().numpy(), E.cpu().numpy()))
    ctx.close()
    (p0, f0, e0), (p1, f1, e1), (p2, f2, e2) = outs
    say(f"[scaling {method} fp64={fp64}] max|phi0| {np.abs(p0).max():.1e}, phi x2 exact "
        f"{np.array_equal(p2, 2 * p1)}, F x4 exact {np.array_equal(f2, 4 * f1)}")
    assert not np.any(p0) and not np.any(f0) and not np.any(e0)
    assert np.array_equal(p2, 2 * p1)
    assert np.array_equal(f2, 4 * f1)
    assert np.array_equal(e2, 4 * e1)


@pytest.mark.parametrize("method", ["pme", "ewald"])
def test_output_subsets(P, method):
    """pq_coulomb with any of phi, force and energy left out gives the full
    call's values bit for bit: the potential-only kernels that run without
    forces sum the potentials in the same order."""
    s = W.random_ionic(n=3000, seed=19, grid=None)
    if method == "pme":
        prm = P.make_params(s.box, 9.0, W.ALPHA_RC9, grid=32, order=6)
    else:
        prm = P.make_params(s.box, 9.0, W.ALPHA_RC9, kmax=6, method="ewald")
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), prm)
    q = gpu(s.q)
    full = [x.cpu().numpy() for x in ctx.coulomb(q)]
    p_e = ctx.coulomb(q, force=False)
    f_only = ctx.coulomb(q, phi=False, energy=False)
    e_only = ctx.coulomb(q, phi=False, force=False)
    p_only = ctx.coulomb(q, force=False, energy=False)
    torch.cuda.synchronize()
    assert p_e[1] is None and f_only[0] is None and f_only[2] is None and e_only[0] is None and p_only[2] is None
    assert np.array_equal(f_only[1].cpu().numpy(), full[1])
    ephi = rel2(p_e[0].cpu().numpy(), full[0])
    say(f"[subsets {method}] phi without forces: rel {ephi:.2e}, bitwise {np.array_equal(p_e[0].cpu().numpy(), full[0])}")
    assert np.array_equal(p_e[0].cpu().numpy(), full[0])
    assert np.array_equal(p_only[0].cpu().numpy(), full[0])
    assert np.array_equal(p_e[2].cpu().numpy(), full[2])
    assert np.array_equal(e_only[2].cpu().numpy(), full[2])
    ctx.close()
