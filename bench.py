"""Benchmark: PME potential+force atom-evaluations per second at 300k atoms on
one MI355X, plus the shadow-MD QEQ step and the batched QEQ serving stream.

A timed step is one full periodic Coulomb potential + force evaluation
(real-space pair sum, PME spread / FFT / convolution / inverse FFT / gather,
self and background terms, FP64 energies) of the 300,000-atom random ionic
system, with the cluster-pair neighbour list resident, as inside the Krylov
loop. value = atoms / seconds per step. The same JSON line also reports the
cold evaluation (neighbour build included), one shadow-MD QEQ step (rebuild,
potential of n, shadow force, 8 Krylov products), the serving stream
(solves/s, p50/p99 latency), the pair kernel's roofline and the FP64 oracle
timed on the host.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--serve-requests R]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PAIR_FLOPS = 50          # algorithmic FLOPs per in-cutoff half pair (phi + force), see the design notes
PEAK_FP32 = 157.3e12     # MI355X FP32 vector peak, FLOP/s
PEAK_HBM = 8.0e12        # MI355X HBM3E, B/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per pair-kernel launch from the committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2503_21176_amd", "csrc", "pair.hip")
    summ = os.path.join(ROOT, "profiles", "coulomb_300k_hbm_counters.md")
    if not os.path.exists(summ):
        return None
    m = re.search(r"TRAFFIC k_pair<true, false, false, float> pair_hip_sha256_16=(\w+) bytes_per_launch=(\d+)", open(summ).read())
    if not m:
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return int(m.group(2)) if sha == m.group(1) else None


def crossover(sizes=(250, 500, 1000, 2000, 3000, 4000, 5000, 6000, 8000, 12000, 20000), delta=5e-4, rc=10.0,
              order=6, reps=30):
    """Direct Ewald vs PME at the accuracy-driven parameters of the same
    target accuracy (pq_choose_params), phi + force + energy per evaluation,
    random ionic systems at 0.1 atoms/A^3. One JSON line per size, then the
    crossover (first size at which PME is the faster, interpolated in log N)."""
    import torch

    import paper_2503_21176_amd as P
    import workloads as W
    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for n in sizes:
        s = W.random_ionic(n=n, seed=7000 + n, grid=None, order=order)
        pos, q = t(s.pos), t(s.q)
        ms = {}
        for method in ("ewald", "pme"):
            prm = P.choose_params(s.box, n, rc, delta, order, method)
            ctx = P.Context(0)
            ctx.set_system(pos, prm)
            for _ in range(5):
                ctx.coulomb(q)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                ctx.coulomb(q)
            e1.record()
            torch.cuda.synchronize()
            ms[method] = e0.elapsed_time(e1) / reps
            ms[method + "_params"] = list(prm.grid) if method == "pme" else list(prm.kmax)
            ctx.close()
        row = {"n": n, "L": round(float(s.box[0]), 3), "ewald_ms": round(ms["ewald"], 4), "pme_ms": round(ms["pme"], 4),
               "kmax": ms["ewald_params"], "grid": ms["pme_params"]}
        rows.append(row)
        print(json.dumps(row), flush=True)
    cross = None
    for a, b in zip(rows, rows[1:]):
        if a["pme_ms"] > a["ewald_ms"] and b["pme_ms"] <= b["ewald_ms"]:
            # log-linear interpolation of the time ratio
            ra, rb = math.log(a["pme_ms"] / a["ewald_ms"]), math.log(b["pme_ms"] / b["ewald_ms"])
            la, lb = math.log(a["n"]), math.log(b["n"])
            cross = int(round(math.exp(la + (lb - la) * ra / (ra - rb))))
            break
    print(json.dumps({"crossover_atoms": cross, "delta": delta, "cutoff": rc, "order": order,
                      "library_auto_pme_min_atoms": P.auto_pme_min_atoms()}), flush=True)


def triclinic_bench(steps=20, warmup=3, tilts=(0.25, -0.2, 0.3)):
    """The 300k-atom phi+F evaluation in a triclinic cell against the same
    atoms in the cubic box: the cubic system's fractional coordinates mapped
    through H = [[L, 0, 0], [t_xy, L, 0], [t_xz, t_yz, L]] with tilts given as
    fractions of L (same volume and density). Rebuild time, step time
    (production configuration, autotuned), serialised phases and the pair
    kernel's FP32 rate. One JSON line."""
    import torch

    import paper_2503_21176_amd as P
    import workloads as W

    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731
    s = W.random_ionic()
    L = float(s.box[0])
    H = np.array([[L, 0, 0], [tilts[0] * L, L, 0], [tilts[1] * L, tilts[2] * L, L]])
    cells = {"cubic": (s.pos, s.box), "triclinic": ((s.pos / L) @ H, H)}
    q = t(s.q)
    out = {"workload": "random ionic 300k, rc 10, PME 144^3 order 6", "tilts_over_L": list(tilts)}
    for name, (pos_np, box) in cells.items():
        prm = P.make_params(box, 10.0, W.ALPHA_RC10, grid=144, order=6)
        pos = t(pos_np)
        ctx = P.Context(0)
        ctx.set_system(pos, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ctx.set_system(pos, prm)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3 / 3
        ctx.autotune(q, reps=5)
        for _ in range(warmup):
            ctx.coulomb(q)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ctx.coulomb(q)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ctx.set_timing(2)
        ctx.timings()
        for _ in range(steps):
            ctx.coulomb(q)
        phases, cnt = ctx.timings()
        ctx.set_timing(0)
        ph = {k: round(v / max(1, cnt), 4) for k, v in phases.items()}
        npairs = ctx.neighbor_count()
        ctx.close()
        out[name] = {"ms_per_step": round(ms, 4), "atom_evals_per_s": s.n / (ms / 1e3),
                     "neighbor_build_ms": round(build_ms, 3), "half_pairs": int(npairs),
                     "serialised_phases_ms": ph,
                     "pair_tflops": npairs * PAIR_FLOPS / (ph["pair"] / 1e3) / 1e12}
        log(f"[triclinic] {name}: {ms:.3f} ms/step, rebuild {build_ms:.2f} ms, {npairs} half pairs, phases {ph}")
    print(json.dumps(out), flush=True)


def md_bench(n=3000, steps=200, dt=0.5, n_krylov=6, seed=41):
    """Shadow XL-BOMD (pq_md_run) on a random ionic system at 0.1 atoms/A^3:
    masses 16/23/35.5 amu, hardness U(20, 25) eV, 300 K start, the repulsive
    V_short stand-in (400 exp(-r/0.25 A) eV), K = 5 dissipation, PME at the
    parameters for delta = 5e-4 and rc = 9 A; once with a rebuild every step
    (skin 0) and once with the paper's 1 A skin (list kept while every atom is
    within 0.5 A of its build position). One JSON line per run: ms per MD
    step, rebuilt steps and the total-energy statistics."""
    import torch

    import paper_2503_21176_amd as P
    import workloads as W
    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731
    s = W.small_random(n, (n / 0.1) ** (1 / 3), seed=seed)
    rng = np.random.default_rng(seed + 1)
    eta = rng.uniform(20.0, 25.0, n)
    mass = rng.choice([16.0, 23.0, 35.5], n)
    vel = rng.normal(0.0, 1.0, (n, 3)) * np.sqrt(0.02585 * 9.648533212331e-3 / mass)[:, None]
    for skin in (0.0, 1.0):
        prm = P.choose_params(s.box, n, 9.0, 5e-4, 6, "pme")
        prm.skin = skin
        ctx = P.Context(0)
        pos = t(s.pos)
        ctx.set_system(pos, prm)
        r = ctx.qeq_solve(t(s.chi), t(eta), tol=1e-10, max_it=400, restart=100)
        H = P.md_history(5)
        hist = r.q.reshape(1, n).repeat(H, 1).contiguous()
        v, m, chi, et = t(vel), t(mass), t(s.chi), t(eta)
        ref = pos.clone()
        kw = dict(dt_fs=dt, n_krylov=n_krylov, dissipation=5, rep_a=400.0, rep_rho=0.25, pos_ref=ref)
        ctx.md_run(pos, v, m, chi, et, hist, 5, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = ctx.md_run(pos, v, m, chi, et, hist, steps, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ctx.close()
        tot, ke = e[:, 3], e[:, 0]
        slope = float(np.polyfit(np.arange(len(tot)) * dt * 1e-3, tot, 1)[0])
        print(json.dumps({"md": "shadow XL-BOMD", "n_atoms": n, "steps": steps, "dt_fs": dt, "n_krylov": n_krylov,
                          "skin_A": skin, "rebuilt_steps": int(e[1:, 5].sum()),
                          "grid": list(prm.grid), "ms_per_md_step": round(ms, 4),
                          "md_steps_per_s": round(1e3 / ms, 1), "e_tot_std_eV": float(tot.std()),
                          "e_tot_drift_eV_per_ps": slope, "ke_std_eV": float(ke.std()),
                          "ke_mean_eV": float(ke.mean())}), flush=True)


def md_sweep(n=300, steps=1000, dt=0.5, seed=51):
    """Energy conservation against cost: regular Born-Oppenheimer MD with QEQ
    solves to tolerance tol (Jacobi GMRES, warm start) against shadow MD with
    m Krylov steps for n'' (K = 5 dissipation), from the same relaxed state
    and 300 K velocities, NVE, rebuild every step. System: N random atoms at
    0.1 atoms/A^3, masses 16 / 23 / 35.5 amu, chi ~ N(0, 1) eV, hardness
    U(20, 25) eV, the repulsive V_short stand-in, PME at the parameters for
    delta = 5e-4, rc = 7 A. One JSON line per run."""
    import torch

    import paper_2503_21176_amd as P
    import workloads as W
    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731
    s = W.small_random(n, (n / 0.1) ** (1 / 3), seed=seed)
    rng = np.random.default_rng(seed + 1)
    eta = rng.uniform(20.0, 25.0, n)
    mass = rng.choice([16.0, 23.0, 35.5], n)
    prm = P.choose_params(s.box, n, 7.0, 5e-4, 6, "pme")
    chi, et, m = t(s.chi), t(eta), t(mass)
    rep = dict(rep_a=400.0, rep_rho=0.25)
    ctx = P.Context(0)
    pos = t(s.pos)
    ctx.set_system(pos, prm)
    r = ctx.qeq_solve(chi, et, tol=1e-12, max_it=600, restart=n + 1)
    H = P.md_history(5)
    hist = r.q.reshape(1, n).repeat(H, 1).contiguous()
    # relax the random packing: short shadow runs with the velocities zeroed in between
    v = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    for _ in range(8):
        v.zero_()
        ctx.md_run(pos, v, m, chi, et, hist, 40, dt_fs=dt, n_krylov=8, dissipation=5, **rep)
    pos0 = pos.clone()
    ctx.set_system(pos0, prm)
    q0 = ctx.qeq_solve(chi, et, tol=1e-12, max_it=600, restart=n + 1).q
    vel0 = t(rng.normal(0.0, 1.0, (n, 3)) * np.sqrt(0.02585 * 9.648533212331e-3 / mass)[:, None])
    runs = [("regular", tol) for tol in (1e-2, 1e-3, 1e-4, 1e-6, 1e-8)] + [("shadow", k) for k in (1, 2, 4, 8)]
    for kind, val in runs:
        p, vv = pos0.clone(), vel0.clone()
        ctx.set_system(p, prm)
        h = q0.reshape(1, n).repeat(H, 1).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "regular":
            e = ctx.md_run(p, vv, m, chi, et, h, steps, dt_fs=dt, dissipation=5, regular=True, tol=val, max_it=400,
                           restart=50, **rep)
        else:
            e = ctx.md_run(p, vv, m, chi, et, h, steps, dt_fs=dt, n_krylov=val, dissipation=5, **rep)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        tot = e[:, 3]
        drift = float(np.polyfit(np.arange(len(tot)) * dt * 1e-3, tot, 1)[0])
        print(json.dumps({"md": kind, ("tol" if kind == "regular" else "n_krylov"): val, "n_atoms": n,
                          "steps": steps, "dt_fs": dt, "coulomb_evals_per_step": round(float(e[1:, 4].mean()), 2),
                          "e_tot_std_eV": float(tot.std()), "e_tot_drift_eV_per_ps": drift,
                          "ke_mean_eV": float(e[:, 0].mean()), "ms_per_md_step": round(ms, 4)}), flush=True)
    ctx.close()


def grad_batch(stated_systems=64, quiet=False):
    """The gradient batch: 64 periodic systems of 2000 atoms (rho 0.1/A^3,
    chi ~ N(0,1) eV, eta ~ U(5,10) eV, rc 9 A, PME 48^3 order 5). For each
    system the QEQ solve and dE/d(positions, chi, eta) at its solution (the
    envelope-theorem adjoint: -F[q*], q*, q*^2/2): at the stated hardness in
    the FP64 form with full GMRES to relative residual 1e-6 (the FP32 form
    stalls near 5e-5 on these systems, cond ~3e5), on the first
    `stated_systems` systems, and with the hardness raised by 15 eV in the
    FP32 form with GMRES(50) to 1e-6, on all 64. Returns one dict per form
    (and prints them as JSON lines unless quiet)."""
    import torch

    import paper_2503_21176_amd as P
    import workloads as W

    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731
    systems = W.diff_batch()
    out = []
    for label, fp64, shift, restart in (("stated", True, 0.0, 3000), ("well_posed", False, 15.0, 50)):
        batch = systems[:stated_systems] if label == "stated" else systems
        ctx = P.Context(0)
        its, conv = [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in batch:
            prm = P.make_params(s.box, 9.0, W.ALPHA_RC9, grid=48, order=5, fp64=fp64)
            ctx.set_system(t(s.pos), prm)
            chi, eta = t(s.chi), t(s.eta + shift)
            r = ctx.qeq_solve(chi, eta, tol=1e-6, max_it=3000, restart=restart, energy=True)
            ctx.qeq_vjp(chi, eta, r.q)
            its.append(r.iterations)
            conv += int(r.status == 0)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ctx.close()
        rec = {"grad_batch": label, "systems": len(batch), "n_atoms": 2000, "form": "fp64" if fp64 else "fp32",
               "hardness_shift_eV": shift, "converged": conv, "mean_products": float(np.mean(its)),
               "max_products": int(np.max(its)), "seconds": round(sec, 3),
               "gradients_per_s": round(len(batch) / sec, 2)}
        out.append(rec)
        if not quiet:
            print(json.dumps(rec), flush=True)
    return out


def krylov_study():
    """Operator products that each Krylov method needs to reach the serving
    tolerance (relative residual 1e-5) on requests of the serving stream,
    against the atom count: restarted GMRES(50), full GMRES (restart = the
    product budget) and preconditioned MINRES, at the stream's own hardness
    U(5, 10) eV (indefinite C) and shifted by +15 eV (positive definite C)."""
    import torch

    import paper_2503_21176_amd as P
    import workloads as W

    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731
    sizes = (64, 128, 256, 512, 1024, 2048, 4000)
    ctx = P.Context(0)
    for k, n in enumerate(sizes):
        r = W.serving_request(n, 90_000 + k)
        prm = P.make_params(r.box, r.params["cutoff"], r.params["alpha"], grid=r.params["grid"],
                            order=r.params["order"])
        ctx.set_system(t(r.pos), prm)
        for shift in (0.0, 15.0):
            eta = t(r.eta + shift)
            budget = min(3 * n + 100, 12000)
            for name, solver, restart in (("gmres50", "gmres", 50), ("gmres_full", "gmres", min(budget, 4096)),
                                          ("minres", "minres", 1)):
                ctx.set_solver(solver)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = ctx.qeq_solve(t(r.chi), eta, tol=1e-5, max_it=budget, restart=restart, q0=t(r.q),
                                    energy=False)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                print(json.dumps({"krylov": name, "n": n, "grid": r.params["grid"], "hardness_shift_eV": shift,
                                  "budget": budget, "converged": res.status == 0, "products": res.iterations,
                                  "rel_residual": res.rel_residual, "ms": round(ms, 2)}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad-batch", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=8, help="oracle real-space rows per host core")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--serve-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--crossover", action="store_true",
                    help="time direct Ewald against PME at equal accuracy over system sizes and exit")
    ap.add_argument("--md", action="store_true",
                    help="time shadow XL-BOMD steps (pq_md_run) on a 3000-atom system and exit")
    ap.add_argument("--md-sweep", action="store_true",
                    help="regular BO-MD over solver tolerances against shadow MD over Krylov steps and exit")
    ap.add_argument("--triclinic", action="store_true",
                    help="time the 300k-atom evaluation in a triclinic cell against the cubic box and exit")
    ap.add_argument("--grad-batch", action="store_true",
                    help="QEQ energies and gradients of the 64-system gradient batch (2000 atoms each) at the "
                         "stated hardness (FP64 form, full GMRES) and +15 eV (FP32, GMRES(50)), and exit")
    ap.add_argument("--krylov-study", action="store_true",
                    help="products to tol 1e-5 against system size on serving-stream requests (GMRES(50), "
                         "full GMRES, MINRES; stated and +15 eV hardness) and exit")
    args = ap.parse_args()
    if args.krylov_study:
        krylov_study()
        return
    if args.grad_batch:
        grad_batch()
        return
    if args.triclinic:
        triclinic_bench()
        return
    if args.crossover:
        crossover()
        return
    if args.md:
        md_bench()
        return
    if args.md_sweep:
        md_sweep()
        return
    if args.serve_only:
        import paper_2503_21176_amd as P
        import workloads as W
        print(json.dumps(serve(P, W, args)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library computes one system on one GPU; --gpus must be 1 (the multi-GPU decomposition is not built)"}))
        sys.exit(2)

    import torch

    import paper_2503_21176_amd as P
    import workloads as W

    dev = torch.device("cuda", 0)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)  # noqa: E731

    log("[bench] generating the 300k-atom random ionic system")
    s = W.random_ionic()
    N = s.n
    a, rc, K, p = W.ALPHA_RC10, 10.0, 144, 6
    prm = P.make_params(s.box, rc, a, grid=K, order=p)
    pos, q, chi, eta = t(s.pos), t(s.q), t(s.chi), t(s.eta)

    if args.calib_copy:
        # a plain copy of known size: 256 MiB read + 256 MiB written
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = P.Context(0)
    # cold: neighbour build + one evaluation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_system(pos, prm)
    ctx.coulomb(q)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] cold (build + eval) {cold_ms:.2f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_system(pos, prm)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3

    # launch shape of the pair kernel chosen by the library's autotuner
    tune = ctx.autotune(q, reps=5)
    log(f"[bench] autotune: {tune}")

    # warmup + timed steps (production configuration: no timing events, the
    # pair kernel overlaps the reciprocal chain on a second stream)
    for _ in range(args.warmup):
        ctx.coulomb(q)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        phi, F, E = ctx.coulomb(q)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = N / (ms_step / 1e3)
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f}), "
        f"{value:.4e} atom-evals/s")
    # per-phase device time, phases serialised so each kernel is timed alone
    ctx.set_timing(2)
    ctx.timings()
    for _ in range(args.steps):
        ctx.coulomb(q)
    phases, cnt = ctx.timings()
    ctx.set_timing(0)
    phase_ms = {k: v / max(1, cnt) for k, v in phases.items()}
    log(f"[bench] serialised phases (ms): {json.dumps({k: round(v, 4) for k, v in phase_ms.items()})}")

    # roofline of the dominant kernel (real-space pair sum)
    npairs = ctx.neighbor_count()          # half pairs with r < rc (skin 0)
    pair_s = phase_ms["pair"] / 1e3
    achieved = npairs * PAIR_FLOPS / pair_s
    roof = {"kernel": "k_pair<force>", "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": measured_traffic(),
            "algorithmic_flops_per_launch": npairs * PAIR_FLOPS, "half_pairs": int(npairs),
            "avg_launch_ms": phase_ms["pair"]}
    log(f"[bench] pair kernel {phase_ms['pair']:.3f} ms, {npairs} half pairs, "
        f"{achieved / 1e12:.2f} TFLOP/s ({100 * achieved / PEAK_FP32:.1f}% of FP32 peak)")

    # the neighbour list's two output formats (Section "Cell based Neighbor
    # List"): COO rows (i, j, image) of the half pairs and the n x K ELLPACK
    # matrix of both directions, exported from the resident list
    nl_out = {}
    for name, fn in (("coo", ctx.neighbor_pairs), ("ellpack", ctx.neighbor_ell)):
        r = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        nl_out[name + "_ms"] = (time.perf_counter() - t0) * 1e3
    nl_out["ellpack_K"] = int(r[0].shape[1])
    nl_out["coo_pairs"] = int(npairs)
    del r
    log(f"[bench] neighbour-list export: {nl_out}")

    # PME phases against HBM: algorithmic bytes (grid read/write per pass, atoms in/out)
    ng = K ** 3
    nspec = (K // 2 + 1) * K * K
    # (the FFT's algorithmic bytes: one read and one write of the grid per
    # direction, real grid in and half spectrum out, then back)
    pme_bytes = {
        "spread": 4 * ng + N * (16 + 4 + 8),            # grid write, atom frac+idx+q read
        "fft": 2 * (4 * ng + 8 * nspec),
        "gather": 4 * ng + N * (16 + 4 + 8 + 4 + 16),
    }
    pme_roof = {k: {"ms": phase_ms[k], "GB/s": pme_bytes[k] / (phase_ms[k] / 1e3) / 1e9,
                    "frac_hbm": pme_bytes[k] / (phase_ms[k] / 1e3) / PEAK_HBM} for k in pme_bytes}
    # the implementation's five passes (x, y, z, y, x) move the spectrum three more times
    pme_roof["fft"]["pass_bytes"] = 2 * (4 * ng + 8 * nspec) + 6 * 8 * nspec

    # shadow-MD QEQ step: rebuild + v = phi[n] + the shadow force (one bilinear evaluation) + 8 Krylov products
    n_vec = q
    for _ in range(2):
        ctx.shadow_step(chi, eta, n_vec, n_krylov=8)
    torch.cuda.synchronize()
    reps = 5
    e0.record()
    for _ in range(reps):
        ctx.set_system(pos, prm)
        ctx.shadow_step(chi, eta, n_vec, n_krylov=8)
    e1.record()
    torch.cuda.synchronize()
    shadow_ms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        ctx.shadow_step(chi, eta, n_vec, n_krylov=8)
    e1.record()
    torch.cuda.synchronize()
    shadow_res_ms = e0.elapsed_time(e1) / reps
    log(f"[bench] shadow step {shadow_ms:.3f} ms with rebuild, {shadow_res_ms:.3f} ms resident")

    # the same evaluation in the FP64 form (every bulk operation in FP64): at
    # equal (alpha, rc, K, p) both forms carry the same PME discretisation
    # error; they differ by the FP32 rounding, reported here
    phi32, F32 = phi.double().clone(), F.double().clone()
    prm64 = P.make_params(s.box, rc, a, grid=K, order=p, fp64=True)
    ctx.set_system(pos, prm64)
    for _ in range(2):
        ctx.coulomb(q)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        phi64, F64, E64 = ctx.coulomb(q)
    e1.record()
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1) / args.steps
    dphi = float(torch.linalg.norm(phi32 - phi64) / torch.linalg.norm(phi64))
    dF = float(torch.sqrt(((F32 - F64) ** 2).sum(1).mean()) / torch.sqrt((F64 ** 2).sum(1).mean()))
    fp64_form = {"ms_per_eval": ms64, "atom_evals_per_s": N / (ms64 / 1e3), "fp32_speedup": ms64 / ms_step,
                 "fp32_vs_fp64_phi_rel": dphi, "fp32_vs_fp64_F_rms_rel": dF}
    log(f"[bench] FP64 form {ms64:.3f} ms/eval ({ms64 / ms_step:.2f}x the FP32 form); FP32 vs FP64: "
        f"phi {dphi:.2e}, F {dF:.2e}")
    # the FP32 form with compensated pair sums (PQ_FLAG_COMPENSATED): its
    # cost in the pair kernel and the step, and its distance from the FP64 form
    prmc = P.make_params(s.box, rc, a, grid=K, order=p, compensated=True)
    ctx.set_system(pos, prmc)
    ctx.set_tuning(tune["pair_wg_per_cu"], tune["fft_lds_bytes"], tune["pair_fork"])
    for _ in range(2):
        ctx.coulomb(q)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        phic, Fc, _ = ctx.coulomb(q)
    e1.record()
    torch.cuda.synchronize()
    msc = e0.elapsed_time(e1) / args.steps
    ctx.set_timing(2)
    ctx.timings()
    for _ in range(args.steps):
        ctx.coulomb(q)
    ph_c, cnt_c = ctx.timings()
    ctx.set_timing(0)
    dphic = float(torch.linalg.norm(phic - phi64) / torch.linalg.norm(phi64))
    dFc = float(torch.sqrt(((Fc - F64) ** 2).sum(1).mean()) / torch.sqrt((F64 ** 2).sum(1).mean()))
    compensated = {"ms_per_eval": msc, "pair_ms": ph_c["pair"] / max(1, cnt_c), "pair_ms_plain": phase_ms["pair"],
                   "vs_fp64_phi_rel": dphic, "vs_fp64_F_rms_rel": dFc}
    log(f"[bench] compensated pair sums: {msc:.3f} ms/eval, pair {compensated['pair_ms']:.4f} ms "
        f"(plain {phase_ms['pair']:.4f}); vs FP64: phi {dphic:.2e}, F {dFc:.2e}")
    ctx.close()

    out = {
        "metric": "PME phi+force atom-evals/s @300k atoms; batched QEQ solves/s + p50/p99 ms",
        "value": value, "unit": "atom-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "random ionic, 300000 atoms, rho 0.1/A^3, L 144.225 A, +-1 charges, rc 10 A, "
                               "alpha 0.26283/A, PME 144^3 order 6, neighbours resident",
                   "n_atoms": N, "reductions": "f64"},
        "roofline": roof,
        "pme_phases": pme_roof,
        "phase_ms": phase_ms,
        "cold_eval_ms": cold_ms,
        "neighbor_build_ms": build_ms,
        "neighbor_export": nl_out,
        "shadow_step_ms": shadow_ms,
        "shadow_step_resident_ms": shadow_res_ms,
        "energy_eV": float(E[0]),
        "fp64_form": fp64_form,
        "compensated_form": compensated,
        "autotune": tune,
    }

    if not args.no_serving:
        out["serving"] = serve_child(args)
    # the gradient batch: all 64 systems well-posed; 8 at the stated hardness
    # (FP64 full GMRES, ~0.6 s each; all 64 with --grad-batch)
    if not args.no_grad_batch:
        gb = grad_batch(stated_systems=8, quiet=True)
        out["grad_batch"] = {g["grad_batch"]: g for g in gb}
        log(f"[grad] {gb}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, a, rc, K, p, args.cpu_rows)
    print(json.dumps(out), flush=True)


def serve_child(args):
    """The serving measurement in a child process (its own GPU context), so
    that a failure there cannot lose the evaluation results above."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--serve-only",
           "--serve-requests", str(args.serve_requests), "--serve-slots", str(args.serve_slots)]
    log(f"[serve] child: {' '.join(cmd)}")
    try:
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=None, timeout=600, text=True)
    except subprocess.TimeoutExpired:
        return {"error": "serving child timed out after 600 s"}
    lines = [x for x in p.stdout.splitlines() if x.startswith("{")]
    if p.returncode != 0 or not lines:
        return {"error": f"serving child exited with status {p.returncode}"}
    return json.loads(lines[-1])


def serve_run(P, reqs, slots, fp64=False, eta_shift=0.0, poisson=True, restart=None):
    """One pass of the served stream: saturation throughput (all requests
    submitted at t = 0) and, if asked, latency under Poisson arrivals at 80 %
    of that rate."""
    srv = P.Server(0, slots=slots, hbm_budget_bytes=100e9)

    def submit(sys_):
        pr = P.make_params(sys_.box, sys_.params["cutoff"], sys_.params["alpha"], grid=sys_.params["grid"],
                           order=sys_.params["order"], fp64=fp64)
        return srv.submit(sys_.pos, sys_.chi, sys_.eta + eta_shift, pr, q0=sys_.q, tol=sys_.params["tol"],
                          max_it=sys_.params["max_it"], restart=restart or sys_.params["restart"])

    # warm the slots (buffers grow to the largest request once)
    big = sorted(reqs, key=lambda r: -r.n)[:slots]
    for tk in [submit(r) for r in big]:
        srv.poll(tk)
    t0 = time.perf_counter()
    tickets = [submit(r) for r in reqs]
    res = [srv.poll(tk) for tk in tickets]
    sat_s = time.perf_counter() - t0
    statuses = {}
    for r in res:
        statuses[str(r["status"])] = statuses.get(str(r["status"]), 0) + 1
    errors = sorted({r["message"] for r in res if r["status"] < 0})[:3]
    conv = [r["status"] == 0 for r in res]
    sizes = np.array([x.n for x in reqs])
    out = {"slots": slots, "form": "fp64" if fp64 else "fp32", "hardness_shift_eV": eta_shift,
           "status_counts": statuses, "errors": errors,
           "saturation_solves_per_s": len(reqs) / sat_s,
           "converged": int(sum(conv)), "converged_fraction": float(np.mean(conv)),
           "converged_solves_per_s": float(sum(conv)) / sat_s,
           "largest_converged_n": int(sizes[np.array(conv)].max()) if any(conv) else 0,
           "median_iterations": float(np.median([r["iterations"] for r in res])),
           "mean_iterations": float(np.mean([r["iterations"] for r in res]))}
    if poisson:
        qps = 0.8 * out["saturation_solves_per_s"]
        gaps = np.random.default_rng(40).exponential(1.0 / qps, size=len(reqs))
        arr = np.cumsum(gaps)
        t0 = time.perf_counter()
        tickets = []
        for r, ta in zip(reqs, arr):
            while time.perf_counter() - t0 < ta:
                time.sleep(min(0.0005, max(0.0, ta - (time.perf_counter() - t0))))
            tickets.append(submit(r))
        done = [srv.poll(tk) for tk in tickets]
        lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in done])
        ok = np.array([r["status"] == 0 for r in done])
        out.update({"poisson_qps": qps, "p50_ms": float(np.percentile(lat, 50)),
                    "p99_ms": float(np.percentile(lat, 99))})
        if ok.any() and not ok.all():
            out.update({"p50_ms_converged": float(np.percentile(lat[ok], 50)),
                        "p99_ms_converged": float(np.percentile(lat[ok], 99))})
    srv.close()
    log(f"[serve] {out}")
    return out


def serve(P, W, args):
    """Served QEQ stream (log-uniform 64..20000 atoms, PME 1 A spacing order 5,
    rc 9 A, tol 1e-5, 200 products at most).
      main: the stream as stated, hardness U(5, 10) eV, FP32 bulk,
            `serve_slots` concurrent requests, full GMRES (restart = the
            200-product budget). C is indefinite there and Krylov methods need
            about n products (profiles/qeq_krylov_products_vs_size.md), so only
            the smallest requests converge; the converged fraction is reported
            beside the throughput of all requests;
      well_posed: the same requests with hardness shifted by +15 eV (positive
            definite C, every solve converges), GMRES(50);
      fp64_one_at_a_time: the well-posed stream in the FP64 form, one slot."""
    log(f"[serve] generating {args.serve_requests} requests")
    stream = W.serving_stream(n_req=args.serve_requests)
    reqs = [x[1] for x in stream]
    main = serve_run(P, reqs, args.serve_slots)
    well = serve_run(P, reqs, args.serve_slots, eta_shift=15.0, restart=50)
    f64 = serve_run(P, reqs, 1, fp64=True, eta_shift=15.0, poisson=False, restart=50)
    out = {"requests": len(reqs), "slots": args.serve_slots, "tol": 1e-5, "max_it": 200,
           "restart": reqs[0].params["restart"],
           "saturation_solves_per_s": main["saturation_solves_per_s"], "poisson_qps": main["poisson_qps"],
           "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"], "converged": main["converged"],
           "converged_fraction": main["converged_fraction"],
           "converged_solves_per_s": main["converged_solves_per_s"],
           "largest_converged_n": main["largest_converged_n"],
           "median_iterations": main["median_iterations"],
           "note": "hardness U(5,10) eV with 1 A separations makes C indefinite: Krylov solves need about n "
                   "products, so requests above ~200 atoms stop at max_it 200 (PQ_WARN_NOT_CONVERGED); "
                   "solves/s counts every request, converged_solves_per_s only the converged ones",
           "well_posed": well, "fp64_one_at_a_time": f64}
    for k in ("p50_ms_converged", "p99_ms_converged"):
        if k in main:
            out[k] = main[k]
    return out


def _oracle_rows(args):
    """Worker of cpu_baseline: the oracle's real-space sum for some rows."""
    import oracle as O
    pos, q, box, a, rc, rows = args
    O.real_space(pos, q, box, a, rc, rows=rows)
    return len(rows)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, a, rc, K, p, rows_per_core):
    """The FP64 oracle on the host's cores: the SPME grid steps of all atoms
    measured in full (NumPy, one core), and the brute-force real-space sum of
    `rows_per_core` atoms per worker on a pool of one worker per available
    core (at most 16), scaled to all atoms by the pool's wall time."""
    import multiprocessing as mp

    import oracle as O
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    nrows = cores * rows_per_core
    log(f"[cpu] oracle: SPME grid in full + real space for {nrows} atoms on {cores} processes")
    rows = np.random.default_rng(2).choice(s.n, nrows, replace=False)
    t0 = time.perf_counter()
    O.spme_reciprocal(s.pos, s.q, s.box, a, K, p, rows=rows[:8])
    t_rec = time.perf_counter() - t0
    parts = [(s.pos, s.q, s.box, a, rc, rows[k::cores]) for k in range(cores)]
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_rows, [(s.pos[:64], s.q[:64], s.box, a, rc, np.arange(1))] * cores)   # start-up
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_rows, parts))
        t_real = time.perf_counter() - t0
    t_eval = t_rec + t_real * s.n / done
    log(f"[cpu] spme {t_rec:.2f} s, real space {t_real:.2f} s wall for {done} rows on {cores} processes "
        f"-> {t_eval:.1f} s per evaluation")
    return {"value": s.n / t_eval, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "numpy": np.__version__,
            "sample": f"SPME spread/FFT/convolution of all {s.n} atoms timed in full on one core ({t_rec:.2f} s); "
                      f"brute-force real-space sum for {done} atoms on {cores} processes ({t_real:.2f} s wall) "
                      f"scaled by {s.n}/{done}",
            "seconds_per_eval": t_eval}


if __name__ == "__main__":
    main()
