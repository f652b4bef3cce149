"""The accuracy-driven parameters on the GPU: an evaluation at the parameters
pq_choose_params returns for a target accuracy delta reaches it against a
converged Ewald sum, and matches the oracle at the same parameters."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import params as OP

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


def rms_rel(a, b):
    return float(np.sqrt(np.mean(np.sum((a - b) ** 2, 1))) / np.sqrt(np.mean(np.sum(b ** 2, 1))))


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,delta,method", [(300, 5e-4, "auto"), (300, 1e-5, "pme"), (300, 1e-5, "ewald"),
                                            (1000, 5e-4, "pme")])
def test_chosen_parameters_on_gpu(P, n, delta, method):
    s = W.random_ionic(n=n, seed=11 + n, grid=None, order=6)
    prm = P.choose_params(s.box, n, 10.0, delta, 6, method)
    ch = OP.choose(s.box, n, 10.0, delta, 6, method, P.auto_pme_min_atoms())
    say(f"[params] n={n} delta={delta} method={ch['method']} grid={ch['grid']} kmax={ch['kmax']}")
    ctx = P.Context(0)
    ctx.set_system(gpu(s.pos), prm)
    phi, F, E = ctx.coulomb(gpu(s.q))
    torch.cuda.synchronize()
    phi, F = phi.cpu().numpy(), F.cpu().numpy()
    ctx.close()
    a = ch["alpha"]
    same = (O.spme_full(s.pos, s.q, s.box, a, 10.0, ch["grid"], 6) if ch["method"] == "pme"
            else O.ewald_direct(s.pos, s.q, s.box, a, 10.0, ch["kmax"]))
    conv = O.ewald_direct(s.pos, s.q, s.box, 0.3, 14.0, 10)
    say(f"[params] vs oracle at the same parameters: phi {rel2(phi, same['phi']):.2e} F {rms_rel(F, same['F']):.2e}; "
        f"vs converged: phi {rel2(phi, conv['phi']):.2e} F {rms_rel(F, conv['F']):.2e}")
    # FP32 bulk arithmetic against the FP64 oracle at identical parameters
    assert rel2(phi, same["phi"]) < 1e-5 and rms_rel(F, same["F"]) < 1e-5
    # the accuracy the parameters were chosen for
    assert rel2(phi, conv["phi"]) < delta and rms_rel(F, conv["F"]) < delta
