"""Parity of the HIP path with the FP64 oracle in triclinic cells (lattice
vectors the rows of a lower triangular H: pq_params.tilt).

Tolerances as for orthorhombic boxes (FP32 bulk arithmetic, FP64 reductions,
the oracle run with the same alpha, cutoff, grid and order):
  ||dphi||_2 / ||phi||_2 <= 1e-5,  ||dF||_rms / ||F||_rms <= 1e-5,  |dE| <= 1e-6 of the parts;
the FP64 form to 1e-11. Neighbour pair sets must match exactly.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from _parity import elem_err, ell_from_pairs

pytestmark = pytest.mark.gpu

TOL_PHI, TOL_F, TOL_E = 1e-5, 1e-5, 1e-6
TOL64 = 1e-11


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


def check(name, got, ref, tol_phi=TOL_PHI, tol_f=TOL_F, tol_e=TOL_E):
    phi, F, E = got
    ephi, ef = rel2(phi, ref["phi"]), rms_rel(F, ref["F"])
    mphi, mf = elem_err(phi, ref["phi"]), elem_err(F, ref["F"])
    scale = abs(ref["E_real"]) + abs(ref["E_rec"]) + abs(ref["E_selfbg"])
    eE = abs(E[0] - ref["E"]) / scale
    say(f"[{name}] phi rel {ephi:.2e}  F rms rel {ef:.2e}  per atom: phi {mphi:.2e} F {mf:.2e}  "
        f"E {E[0]:.12g} vs {ref['E']:.12g} rel(parts) {eE:.2e}")
    assert ephi <= tol_phi and ef <= tol_f and eE <= tol_e
    assert mphi <= 10 * tol_phi and mf <= 10 * tol_f
    for k, key in ((1, "E_real"), (2, "E_rec"), (3, "E_selfbg")):
        assert abs(E[k] - ref[key]) <= tol_e * scale


CELLS = {
    "cell-300": (300, (15.0, 16.0, 17.0), (4.0, -3.5, 5.0), 6.0, 0.5),
    "multi-image-40": (40, (8.6, 9.1, 9.5), (2.1, -1.7, 3.0), 9.0, 0.0),
    "ionic-2000": (2000, (27.0, 27.5, 28.0), (8.0, -6.0, 9.0), 10.0, 1.0),
}


@pytest.mark.parametrize("case", list(CELLS))
def test_triclinic_pairs_exact(P, case):
    n, edges, tilts, rc, skin = CELLS[case]
    s = W.triclinic_random(n, edges, tilts, seed=21)
    say(f"[tric-pairs-{case}] n={n} edges={edges} tilts={tilts} cut={rc + skin}")
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), P.make_params(s.box, rc, 0.3, skin=skin, kmax=1, method="ewald"))
    got = ctx.neighbor_pairs().cpu().numpy().astype(np.int64)
    nbr, img, cnt = ctx.neighbor_ell()
    ctx.close()
    got = got[np.lexsort((got[:, 4], got[:, 3], got[:, 2], got[:, 1], got[:, 0]))]
    want = O.neighbor_pairs(s.pos, s.box, rc + skin)
    say(f"[tric-pairs-{case}] gpu {len(got)} oracle {len(want)}")
    assert got.shape == want.shape and np.array_equal(got, want)
    # the ELLPACK form: both directions of every pair, lattice image vectors
    e_nbr, e_img, e_cnt = ell_from_pairs(want, n)
    assert np.array_equal(cnt.cpu().numpy(), e_cnt)
    assert np.array_equal(nbr.cpu().numpy(), e_nbr) and np.array_equal(img.cpu().numpy(), e_img)


@pytest.mark.parametrize("fp64", [False, True])
def test_triclinic_pme_parity(P, fp64):
    s = W.triclinic_random(500, (18.0, 19.0, 20.0), (5.0, -4.0, 6.0), seed=22)
    a, rc, K, p = 0.35, 7.0, 32, 6
    say(f"[tric-pme fp64={fp64}] n={s.n} grid {K} order {p}")
    got = run(P, s, P.make_params(s.box, rc, a, grid=K, order=p, fp64=fp64))
    ref = O.spme_full(s.pos, s.q, s.box, a, rc, K, p)
    if fp64:
        check("tric-pme-fp64", got, ref, TOL64, TOL64, 1e-12)
    else:
        check("tric-pme", got, ref)


@pytest.mark.parametrize("fp64", [False, True])
def test_triclinic_ewald_parity(P, fp64):
    s = W.triclinic_random(200, (12.0, 13.0, 14.0), (3.0, -2.5, 4.0), seed=23)
    a, rc, km = 0.4, 6.0, 7
    say(f"[tric-ewald fp64={fp64}] n={s.n} kmax {km}")
    got = run(P, s, P.make_params(s.box, rc, a, kmax=km, method="ewald", fp64=fp64))
    ref = O.ewald_direct(s.pos, s.q, s.box, a, rc, km)
    if fp64:
        check("tric-ewald-fp64", got, ref, TOL64, TOL64, 1e-12)
    else:
        check("tric-ewald", got, ref)


def test_triclinic_multi_image_pme(P):
    # cell narrower than twice the cutoff: atoms see their own images
    s = W.triclinic_random(40, (8.6, 9.1, 9.5), (2.1, -1.7, 3.0), seed=24)
    a, rc, K, p = 0.33, 9.0, 24, 6
    got = run(P, s, P.make_params(s.box, rc, a, grid=K, order=p))
    check("tric-multi-image", got, O.spme_full(s.pos, s.q, s.box, a, rc, K, p))


def test_nacl_primitive_cell_on_the_gpu(P):
    # rock salt as its 2-atom rhombohedral primitive cell, in the FP64 form:
    # E = -M KE / r0 with the Madelung constant M of rock salt
    a0 = 5.64
    A, B, C = np.array([0, .5, .5]) * a0, np.array([.5, 0, .5]) * a0, np.array([.5, .5, 0]) * a0
    ax = np.linalg.norm(A)
    ah = A / ax
    bx, by = B @ ah, np.linalg.norm(np.cross(ah, B))
    cx = C @ ah
    cy = (B @ C - bx * cx) / by
    H = np.array([[ax, 0, 0], [bx, by, 0], [cx, cy, np.sqrt(C @ C - cx * cx - cy * cy)]])
    # reduce the tilts into |t| <= half the edge (same lattice)
    H[2] -= np.round(H[2, 1] / H[1, 1]) * H[1]
    H[1] -= np.round(H[1, 0] / H[0, 0]) * H[0]
    H[2] -= np.round(H[2, 0] / H[0, 0]) * H[0]
    pos = np.array([[0.0, 0.0, 0.0], 0.5 * (H[0] + H[1] + H[2])])
    s = W.System("nacl-primitive", pos, np.array([1.0, -1.0]), H)
    _, _, E = run(P, s, P.make_params(H, 8.0, 0.6, kmax=14, method="ewald", fp64=True))
    want = -1.747564594633182 * O.KE / (a0 / 2)
    say(f"[nacl-primitive] E {E[0]:.12f} vs {want:.12f}")
    assert abs(E[0] - want) <= 1e-9 * abs(want)


def test_zero_tilt_matrix_takes_the_orthorhombic_path(P):
    s = W.small_random(300, 14.0, seed=25)
    a, rc, K, p = 0.35, 6.0, 24, 5
    got_box = run(P, s, P.make_params(s.box, rc, a, grid=K, order=p))
    got_mat = run(P, s, P.make_params(np.diag(s.box), rc, a, grid=K, order=p))
    for x, y in zip(got_box, got_mat):
        assert np.array_equal(x, y)


def test_tilts_beyond_half_an_edge_are_rejected(P):
    s = W.triclinic_random(64, (12.0, 12.0, 12.0), (2.0, 1.0, -2.0), seed=27)
    ctx = P.Context(0)
    for H in ([[12.0, 0, 0], [6.5, 12.0, 0], [0, 0, 12.0]], [[12.0, 0, 0], [0, 12.0, 0], [0, -6.1, 12.0]]):
        with pytest.raises(P.PQError):
            ctx.set_system(gpu(s.pos), P.make_params(H, 5.0, 0.4, grid=24, order=5))
    ctx.close()


def test_md_driver_rejects_tilted_cells(P):
    s = W.triclinic_random(64, (12.0, 12.0, 12.0), (2.0, 1.0, -2.0), seed=26)
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), P.make_params(s.box, 5.0, 0.4, grid=24, order=5))
    h = gpu(np.zeros((P.md_history(0), s.n)))
    with pytest.raises(P.PQError):
        ctx.md_run(gpu(s.pos), gpu(np.zeros((s.n, 3))), gpu(np.full(s.n, 20.0)), gpu(s.chi), gpu(s.eta), h, 1,
                   dt_fs=0.5, dissipation=0)
    ctx.close()


@pytest.mark.slow
def test_triclinic_300k_sampled(P):
    # the 300k-atom workload's fractional coordinates in a sheared cell of the
    # same volume, at the benchmark's parameters; 48 sampled atoms
    s0 = W.random_ionic()
    L = float(s0.box[0])
    H = np.array([[L, 0, 0], [0.25 * L, L, 0], [-0.2 * L, 0.3 * L, L]])
    s = W.System("ionic-300k-triclinic", (s0.pos / L) @ H, s0.q, H)
    a = W.ALPHA_RC10
    say("[tric-300k] n=300000 rc=10 grid 144 order 6, tilts (0.25, -0.2, 0.3) L (48 sampled atoms)")
    phi, F, E = run(P, s, P.make_params(H, 10.0, a, grid=144, order=6))
    rows = np.random.default_rng(2).choice(s.n, 48, replace=False)
    ref = O.spme_full(s.pos, s.q, s.box, a, 10.0, 144, 6, rows=rows)
    ephi, ef = rel2(phi[rows], ref["phi"]), rms_rel(F[rows], ref["F"])
    mphi, mf = elem_err(phi[rows], ref["phi"]), elem_err(F[rows], ref["F"])
    say(f"[tric-300k] phi rel {ephi:.2e}  F rms rel {ef:.2e}  per atom: phi {mphi:.2e} F {mf:.2e}  "
        f"E_rec {E[2]:.10g} vs {ref['E_rec']:.10g}")
    assert ephi <= TOL_PHI and ef <= TOL_F
    assert mphi <= 10 * TOL_PHI and mf <= 10 * TOL_F
    assert abs(E[2] - ref["E_rec"]) <= 1e-5 * abs(ref["E_rec"])
    assert abs(E[0] - E[1:].sum()) <= 1e-12 * abs(E[0])
