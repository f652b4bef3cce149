"""Workspaces through the caller's allocator (pq_create's pq_allocator): the
binding passes torch's caching allocator, so the library's device memory is
torch's, and the results equal those of a context on hipMalloc bit for bit."""
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


def test_workspaces_from_torch_allocator(P):
    s = W.small_random(3000, (3000 / 0.1) ** (1 / 3), seed=91)
    prm = P.make_params(s.box, 9.0, W.ALPHA_RC9, grid=32, order=5)
    pos, q = gpu(s.pos), gpu(s.q)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = P.Context(0)                      # torch's caching allocator
    ctx.set_system(pos, prm)
    phi, F, E = ctx.coulomb(q)
    r = ctx.qeq_solve(gpu(s.chi), gpu(s.eta + 15.0), tol=1e-6, max_it=200)
    torch.cuda.synchronize()
    # torch rounds each block up to a multiple of 512 bytes
    outputs = sum((t.numel() * t.element_size() + 511) // 512 * 512 for t in (phi, F, E, r.q, r.energy))
    grown = torch.cuda.memory_allocated() - base - outputs
    say(f"[alloc] library workspaces in torch's allocator: {grown / 2**20:.1f} MiB")
    assert grown > 4 << 20                   # lists, grids, partials and the Krylov basis
    ref = P.Context(0, allocator=None)       # hipMalloc
    ref.set_system(pos, prm)
    phi0, F0, E0 = ref.coulomb(q)
    r0 = ref.qeq_solve(gpu(s.chi), gpu(s.eta + 15.0), tol=1e-6, max_it=200)
    torch.cuda.synchronize()
    assert torch.equal(phi, phi0) and torch.equal(F, F0) and torch.equal(E, E0)
    assert torch.equal(r.q, r0.q) and r.iterations == r0.iterations
    ref.close()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated()
    ctx.close()
    torch.cuda.synchronize()
    assert held - torch.cuda.memory_allocated() == grown     # every workspace handed back
