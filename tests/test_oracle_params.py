"""Accuracy-driven parameters: the oracle's heuristics pinned by their own
definitions and by the accuracy they promise, and the library's host-side
choice (pq_choose_params, no device work) checked against the oracle."""
import ctypes
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import params as OP

CASES = [  # box edges, atoms, cutoff, delta, order
    ((144.225, 144.225, 144.225), 300_000, 10.0, 5e-4, 6),
    ((31.0, 31.0, 31.0), 9000, 10.0, 5e-4, 6),
    ((22.56, 22.56, 22.56), 512, 8.0, 5e-4, 4),
    ((8.62, 8.62, 8.62), 64, 9.0, 5e-4, 5),
    ((17.0, 21.0, 25.0), 700, 7.5, 1e-5, 6),
    ((58.5, 58.5, 58.5), 20_000, 9.0, 1e-6, 5),
    ((40.0, 30.0, 20.0), 2400, 12.0, 3e-3, 3),
]


@pytest.mark.parametrize("delta,rc", [(5e-4, 10.0), (5e-4, 9.0), (1e-5, 8.0), (3e-3, 12.0)])
def test_alpha_closed_form(delta, rc):
    a = OP.alpha_for(delta, rc)
    assert abs(math.exp(-(a * rc) ** 2) / (2 * delta) - 1) < 1e-13
    # the complementary error function at the cutoff is of the order of delta
    assert 0.2 * delta < math.erfc(a * rc) < 2 * delta


def test_alpha_values():
    # the splitting parameters the workloads use at delta = 5e-4
    assert abs(OP.alpha_for(5e-4, 10.0) - W.ALPHA_RC10) < 5e-6
    assert abs(OP.alpha_for(5e-4, 9.0) - W.ALPHA_RC9) < 5e-6


@pytest.mark.parametrize("L,delta", [(8.62, 5e-4), (14.4, 5e-4), (31.0, 5e-4), (144.225, 5e-4), (21.5, 1e-6),
                                     (60.0, 3e-3)])
def test_kmax_is_first_k_past_the_peak_within_delta(L, delta):
    a = OP.alpha_for(delta, 10.0)
    k = OP.ewald_kmax(L, a, delta)
    kpeak = max(1, math.ceil(L * a / (math.pi * math.sqrt(2.0))))
    assert k >= kpeak
    assert OP.ewald_error(L, a, k) <= delta
    for j in range(kpeak, k):
        assert OP.ewald_error(L, a, j) > delta
    # the estimate decreases past the peak, so every larger range is as accurate
    for j in range(k, k + 20):
        e0, e1 = OP.ewald_error(L, a, j), OP.ewald_error(L, a, j + 1)
        assert e1 < e0 or e0 == 0.0


@pytest.mark.parametrize("L,delta,p", [(144.225, 5e-4, 6), (31.0, 5e-4, 6), (8.62, 5e-4, 5), (58.5, 1e-6, 5),
                                       (17.0, 1e-5, 4)])
def test_pme_grid_is_smallest_smooth_size(L, delta, p):
    a = OP.alpha_for(delta, 10.0)
    lo = max(math.ceil(2 * a * L / (3 * delta ** 0.2)), 2 * p)
    K = OP.pme_grid(L, a, delta, p)
    assert K >= lo
    smooth = lambda m: all(f in (2, 3, 5) for f in _factors(m))
    assert smooth(K)
    assert not any(smooth(m) for m in range(lo, K))


def _factors(m):
    out, d = [], 2
    while d * d <= m:
        while m % d == 0:
            out.append(d)
            m //= d
        d += 1
    if m > 1:
        out.append(m)
    return out


def test_auto_switch():
    assert OP.choose(20.0, 999, 9.0, 5e-4, 6, "auto", 1000)["method"] == "ewald"
    assert OP.choose(20.0, 1000, 9.0, 5e-4, 6, "auto", 1000)["method"] == "pme"
    # a range beyond kmax 64 falls back to PME
    assert OP.choose(400.0, 10, 9.0, 1e-8, 6, "auto", 1000)["method"] == "pme"


@pytest.mark.parametrize("delta", [5e-4, 1e-5])
def test_chosen_parameters_reach_the_accuracy(delta):
    # both reciprocal-space methods at the chosen parameters against a
    # converged Ewald sum (alpha 0.3, rc 14, kmax 10: every neglected term
    # below 1e-9): relative RMS force and potential errors below delta
    s = W.random_ionic(n=300, seed=11, grid=None, order=6)
    ref = O.ewald_direct(s.pos, s.q, s.box, 0.3, 14.0, 10)
    ch = OP.choose(s.box, s.n, 10.0, delta, 6, "auto", 5000)
    a = ch["alpha"]
    for res in (O.spme_full(s.pos, s.q, s.box, a, 10.0, ch["grid"], 6),
                O.ewald_direct(s.pos, s.q, s.box, a, 10.0, ch["kmax"])):
        ef = np.sqrt(np.mean(np.sum((res["F"] - ref["F"]) ** 2, 1)) / np.mean(np.sum(ref["F"] ** 2, 1)))
        ep = np.linalg.norm(res["phi"] - ref["phi"]) / np.linalg.norm(ref["phi"])
        assert ef < delta and ep < delta


def _lib():
    import paper_2503_21176_amd as P
    P.load()
    return P


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("method", ["pme", "ewald", "auto"])
def test_library_choice_matches_oracle(case, method):
    P = _lib()
    box, n, rc, delta, p = case
    ref = OP.choose(box, n, rc, delta, p, method, P.auto_pme_min_atoms())
    if method == "ewald" and max(ref["kmax"]) > 64 or method != "ewald" and ref["method"] == "pme" and max(ref["grid"]) > 1024:
        with pytest.raises(P.PQError):
            P.choose_params(box, n, rc, delta, p, method)
        return
    got = P.choose_params(box, n, rc, delta, p, method)
    assert abs(got.alpha - ref["alpha"]) <= 2e-16 * ref["alpha"]
    assert list(got.grid) == ref["grid"]
    assert list(got.kmax) == [min(k, 65) for k in ref["kmax"]]
    assert got.method == {"pme": P.METHOD_PME, "ewald": P.METHOD_EWALD}[ref["method"]]
    assert got.order == p and got.cutoff == rc and got.skin == 0.0 and got.flags == 0
    assert list(got.box) == list(box)


def test_library_rejects_bad_inputs():
    P = _lib()
    for args in [((10.0, 10.0, 10.0), 100, 9.0, 0.0, 6, "pme"),
                 ((10.0, 10.0, 10.0), 100, 9.0, 0.7, 6, "pme"),
                 ((10.0, -1.0, 10.0), 100, 9.0, 5e-4, 6, "pme"),
                 ((10.0, 10.0, 10.0), 0, 9.0, 5e-4, 6, "pme"),
                 ((10.0, 10.0, 10.0), 100, 9.0, 5e-4, 9, "pme")]:
        with pytest.raises(P.PQError) as e:
            P.choose_params(*args)
        assert e.value.code == -1
    # a grid beyond 1024 points per edge
    with pytest.raises(P.PQError) as e:
        P.choose_params((2000.0, 20.0, 20.0), 1000, 9.0, 1e-8, 6, "pme")
    assert e.value.code == -2
