"""pq_coulomb_noalloc (the evaluation without device allocation) against
pq_coulomb, through the C ABI.

Both run the same kernels in the same order on the same inputs, so the
outputs must agree bit for bit (phi, forces, the four energies). Two calls in
a row on each method, the second with a smaller system, so the static scratch
array is reused with the previous call's contents still in it. The
no-allocation context never runs pq_coulomb, so its reduction buffers are
never allocated; free device memory must not drop across its calls.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


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


def cases(P):
    a, rc = W.ALPHA_RC9, 9.0
    big = W.small_random(3000, (3000 / 0.1) ** (1 / 3), seed=71)
    small = W.small_random(700, (700 / 0.1) ** (1 / 3), seed=72)
    return [
        ("pme", big, P.make_params(big.box, rc, a, grid=32, order=5)),
        ("pme", small, P.make_params(small.box, rc, a, grid=20, order=5)),
        ("ewald", big, P.make_params(big.box, rc, a, kmax=7, method="ewald")),
        ("ewald", small, P.make_params(small.box, rc, a, kmax=5, method="ewald")),
    ]


@pytest.mark.parametrize("method", ["pme", "ewald"])
def test_noalloc_matches_coulomb_twice(P, method):
    ref_ctx, na_ctx = P.Context(0), P.Context(0)
    for name, s, prm in [c for c in cases(P) if c[0] == method]:
        say(f"[noalloc] {method} n={s.n}")
        pos, q = gpu(s.pos), gpu(s.q)
        ref_ctx.set_system(pos, prm)
        phi0, F0, E0 = ref_ctx.coulomb(q)
        na_ctx.set_system(pos, prm)
        phi1 = torch.full((s.n,), float("nan"), dtype=torch.float64, device="cuda")
        F1 = torch.full((s.n, 3), float("nan"), dtype=torch.float64, device="cuda")
        E1 = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        na_ctx.coulomb_noalloc(q, phi1, F1, E1)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free0 - free1 < (2 << 20), (free0, free1)
        assert torch.equal(phi0, phi1)
        assert torch.equal(F0, F1)
        assert torch.equal(E0, E1)
        # outputs may be omitted, as with pq_coulomb
        na_ctx.coulomb_noalloc(q, phi1, None, None)
        torch.cuda.synchronize()
        assert torch.equal(phi0, phi1)
    ref_ctx.close()
    na_ctx.close()


def test_noalloc_rejects_too_large_grid_and_missing_system(P):
    ctx = P.Context(0)
    s = W.small_random(64, (64 / 0.1) ** (1 / 3), seed=73)
    q = gpu(s.q)
    with pytest.raises(P.PQError) as e:
        ctx.coulomb_noalloc(q, None, None, None)
    assert e.value.code == -8          # PQ_ERR_STATE: no system yet
    out = torch.empty(s.n, dtype=torch.float64, device="cuda")
    ctx.set_system(gpu(s.pos), P.make_params(s.box, 4.0, 0.6, grid=(512, 512, 16), order=4))
    with pytest.raises(P.PQError) as e:
        ctx.coulomb_noalloc(q, out, None, None)
    assert e.value.code == -6          # PQ_ERR_TOO_LARGE
    ctx.close()
