// Charge equilibration on the device: restarted GMRES or preconditioned
// MINRES on the bordered QEQ system (eq. linear_qeq, matrix-free through the
// Cv identity; the paper names GMRES, CG and related approaches), the shadow
// step (eqs. diag_linear_qeq and Jnddot) and vector-Jacobian products through
// the QEQ solve. Krylov vectors, inner products and orthogonalisation are
// FP64 on the device; each operator product is one FP32-bulk Coulomb
// potential evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <functional>
#include <string>

#include "pmeqeq.h"
#include "pq_internal.h"
#include "vec.h"

namespace pq {

void set_error(const std::string& m);

namespace {

size_t round_ld(int64_t n) { return (size_t)((n + 63) / 64 * 64); }

// Work vectors of the solvers (each ld doubles).
enum { W_B = 0, W_X, W_R, W_W, W_T, W_PHI, W_PHI2, W_D, W_VJ, W_M1, W_M2, W_M3, W_M4, W_N };

struct Work {
    Ctx& c;
    size_t ld;
    int m;
    double* V;
    double* st;
    double* up = nullptr;   // chunk sums of long-basis combinations (m + 1 > 32)
    double* w(int k) { return c.kw.p + (size_t)k * ld; }
    double* sc(int k) { return c.scal.p + 16 + k; }   // device scalars 16..63
    Work(Ctx& cc, int mm) : c(cc), ld(round_ld(cc.n + 1)), m(mm) {
        c.kw.ensure(ld * W_N);
        c.kv.ensure(ld * (size_t)(m + 1));
        c.kh.ensure(gs_size(m) + 8);
        if (m + 1 > 32) {
            c.kup.ensure(vcomb_chunks(m + 1) * ld);
            up = c.kup.p;
        }
        ensure_red(c);
        V = c.kv.p;
        st = c.kh.p;
    }
};

using OpFn = std::function<void(const double* x, double* y)>;

struct GmresOut {
    int products = 0;
    int restarts = 0;
    double relres = 0.0;
    bool converged = false;
};

double read_scalar(Ctx& c, const double* dev, hipStream_t s) {
    PQ_HIP(hipMemcpyAsync(c.pinned, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    return c.pinned[0];
}

// One Arnoldi step at the device step index j = *kj: w = A V_j, CGS2 against
// V_0..V_j, V_{j+1} = w / |w|, Givens update of Hessenberg column j (|g[j+1]|
// into hist[j]), then j + 1. The kernels take j from device memory, so one
// captured step serves every iteration of a cycle.
void arnoldi_step(Work& W, const OpFn& op, int64_t nv) {
    Ctx& c = W.c;
    hipStream_t s = c.stream;
    const int m = W.m;
    double* xj = W.w(W_VJ);
    double* w = W.w(W_W);
    copy_j(nv, W.V, W.ld, c.kj.p, xj, s);
    op(xj, w);
    orthogonalize_j(c, nv, W.V, W.ld, m, c.kj.p, w, W.st, W.st + gs_t(m), W.up, s);
    dot_vector(c, w, w, nv, W.sc(2), s);
    normalize_j(nv, w, W.sc(2), W.st, m, W.V, W.ld, c.kj.p, s);
    givens_j(W.st, m, c.kj.p, W.st + gs_hist(m), s);
}

// One solver step (an Arnoldi step, or a MINRES step) as an instantiated HIP
// graph, built once per operator, system and workspace by recording the
// step's launches (cached in the context; pq_set_system invalidates it).
// Returns nullptr when graphs are off or the build fails (the caller then
// launches the step's kernels directly). A cached graph of another key is
// destroyed only after the context's stream has drained, so no launch of it
// can still be in flight.
hipGraphExec_t step_graph(Work& W, const std::function<void()>& body, int64_t nv, uintptr_t kind,
                          const void* opkey) {
    Ctx& c = W.c;
    if (!c.graphs || c.timing) return nullptr;
    std::vector<uintptr_t> key = {kind, (uintptr_t)opkey, (uintptr_t)nv, (uintptr_t)W.m, (uintptr_t)W.ld,
                                  (uintptr_t)c.kv.p, (uintptr_t)c.kw.p, (uintptr_t)c.kh.p, (uintptr_t)W.up,
                                  (uintptr_t)c.scal.p,
                                  (uintptr_t)c.part.p, (uintptr_t)c.kj.p, (uintptr_t)c.gen, (uintptr_t)c.pair_grid,
                                  (uintptr_t)c.fft_budget, (uintptr_t)c.fork_at};
    if (c.kgraph && key == c.kgraph_key) return c.kgraph;
    if (c.kgraph) {
        PQ_HIP(hipStreamSynchronize(c.stream));
        (void)hipGraphExecDestroy(c.kgraph);
        c.kgraph = nullptr;
        c.kgraph_key.clear();
    }
    ensure_side(c);
    GraphRec rec;
    hipGraphExec_t ex = nullptr;
    bool ok = hipGraphCreate(&rec.g, 0) == hipSuccess;
    if (ok) {
        graph_rec() = &rec;
        try {
            body();
        } catch (...) {
            ok = false;
        }
        graph_rec() = nullptr;
    }
    if (ok) ok = hipGraphInstantiate(&ex, rec.g, nullptr, nullptr, 0) == hipSuccess && ex;
    if (rec.g) (void)hipGraphDestroy(rec.g);
    if (!ok) {
        (void)hipGetLastError();
        c.graphs = false;   // launch the kernels directly from now on
        return nullptr;
    }
    c.kgraph = ex;
    c.kgraph_key = key;
    return ex;
}

// Host buffer of residual estimates with room for m values.
void ensure_pinned_hist(Ctx& c, int m) {
    if (c.pinned_hist && c.pinned_hist_n >= m) return;
    std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
    if (c.pinned_hist) {
        PQ_HIP(hipStreamSynchronize(c.stream));
        (void)hipHostFree(c.pinned_hist);
        c.pinned_hist = nullptr;
        c.pinned_hist_n = 0;
    }
    const int cap = std::max(m, 520);
    PQ_HIP(hipHostMalloc((void**)&c.pinned_hist, (size_t)cap * sizeof(double), hipHostMallocDefault));
    c.pinned_hist_n = cap;
}

// GMRES(m) for A x = b with vectors of length nv, x in/out (x_zero: x = 0 on
// entry). fixed: exactly m products from x = 0, no host synchronisation.
// Each Arnoldi step is one graph launch; the host reads the residual estimate
// of step j - 1 while step j runs, so a converged cycle has run at most one
// step more than it uses (its product is counted).
GmresOut gmres(Work& W, const OpFn& op, int64_t nv, const double* b, double* x, bool x_zero, double tol, int max_it,
               bool fixed, uintptr_t kind, const void* opkey) {
    Ctx& c = W.c;
    hipStream_t s = c.stream;
    const int m = W.m;
    double* r = W.w(W_R);
    double* w = W.w(W_W);
    GmresOut out;
    double bnorm = 1.0;
    c.kj.ensure(4);
    ensure_pinned_hist(c, m);
    for (auto& ev : c.kev)
        if (!ev) PQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (!fixed) {
        dot_vector(c, b, b, nv, W.sc(0), s);
        bnorm = std::sqrt(read_scalar(c, W.sc(0), s));
        if (bnorm == 0.0) {
            axpby(nv, 0.0, b, 0.0, nullptr, x, s);
            out.converged = true;
            return out;
        }
    }
    if (x_zero) {
        axpby(nv, 0.0, b, 0.0, nullptr, x, s);
        axpby(nv, 1.0, b, 0.0, nullptr, r, s);
    } else {
        op(x, w);
        out.products++;
        axpby(nv, 1.0, b, -1.0, w, r, s);
    }
    dot_vector(c, r, r, nv, W.sc(1), s);
    if (!fixed) {
        out.relres = std::sqrt(read_scalar(c, W.sc(1), s)) / bnorm;
        if (out.relres <= tol) {
            out.converged = true;
            return out;
        }
    }
    hipGraphExec_t step = step_graph(W, [&] { arnoldi_step(W, op, nv); }, nv, kind, opkey);
    const double* hist = W.st + gs_hist(m);
    for (;;) {
        gmres_start(W.st, m, W.sc(1), s);
        normalize(nv, r, W.sc(1), nullptr, W.V, s);
        set_int(c.kj.p, 0, s);
        int launched = 0, jdone = -1;
        for (int j = 0; j < m; ++j) {
            if (!fixed && out.products >= max_it) break;
            if (step)
                PQ_HIP(hipGraphLaunch(step, s));
            else
                arnoldi_step(W, op, nv);
            out.products++;
            ++launched;
            if (fixed) continue;
            PQ_HIP(hipMemcpyAsync(c.pinned_hist + j, hist + j, sizeof(double), hipMemcpyDeviceToHost, s));
            PQ_HIP(hipEventRecord(c.kev[j & 1], s));
            if (j >= 1) {
                PQ_HIP(hipEventSynchronize(c.kev[(j - 1) & 1]));
                if (c.pinned_hist[j - 1] / bnorm <= tol) {
                    jdone = j;
                    break;
                }
            }
        }
        if (jdone < 0) {
            jdone = launched;
            if (!fixed && launched > 0) PQ_HIP(hipEventSynchronize(c.kev[(launched - 1) & 1]));
        }
        backsolve(W.st, m, jdone, s);
        xupdate(nv, W.V, W.ld, jdone, W.st + gs_y(m), x, W.up, s);
        if (fixed) return out;
        // true residual
        op(x, w);
        out.products++;
        axpby(nv, 1.0, b, -1.0, w, r, s);
        dot_vector(c, r, r, nv, W.sc(1), s);
        out.relres = std::sqrt(read_scalar(c, W.sc(1), s)) / bnorm;
        if (out.relres <= tol) {
            out.converged = true;
            return out;
        }
        if (out.products >= max_it) return out;
        out.restarts++;
    }
}

// Preconditioned MINRES for the symmetric bordered system M z = b (n + 1
// unknowns) with D = diag(u, 1); z in/out in x (x_zero: z = 0 on entry). One
// step (v = y / beta, the product y = M v, the Lanczos and Givens updates and
// the solution update) is one graph launch; the host reads the estimate of
// step k - 1 while step k runs. The estimate phibar is the D^-1-norm of the
// residual: a cycle ends when it falls to target * ||b||_{D^-1}, and then the
// true relative residual ||b - M z||_2 / ||b||_2 decides; if it is still above
// tol, a new cycle starts from z with the target lowered by their ratio.
GmresOut minres(Work& W, const OpFn& op, const double* eta, int64_t n, const double* b, double* x, bool x_zero,
                double tol, int max_it) {
    Ctx& c = W.c;
    hipStream_t s = c.stream;
    const int64_t nv = n + 1;
    double* r1 = W.w(W_R);
    double* r2 = W.w(W_M1);
    double* y = W.w(W_W);
    double* v = W.w(W_VJ);
    double* wa = W.w(W_M2);
    double* wb = W.w(W_M3);
    double* t = W.w(W_M4);
    double* ms = W.sc(20);   // MR_N scalars
    static_assert(16 + 20 + MR_N <= 64, "MINRES scalars exceed the device scalar block");
    GmresOut out;
    ensure_pinned_hist(c, 2);
    for (auto& ev : c.kev)
        if (!ev) PQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    dot_vector(c, b, b, nv, W.sc(0), s);
    const double bnorm = std::sqrt(read_scalar(c, W.sc(0), s));
    if (bnorm == 0.0) {
        axpby(nv, 0.0, b, 0.0, nullptr, x, s);
        out.converged = true;
        return out;
    }
    minres_start(c, n, b, eta, y, ms, s);
    const double bnorm_d = read_scalar(c, ms + MR_BETA1, s);
    if (x_zero) axpby(nv, 0.0, b, 0.0, nullptr, x, s);
    auto body = [&] {
        minres_v(nv, y, ms, v, s);
        op(v, y);
        minres_update(c, n, y, r1, r2, v, eta, wa, wb, x, ms, s);
    };
    hipGraphExec_t step = nullptr;
    bool have_step = false;
    double target = tol;
    // r1 = b - M z
    if (x_zero) {
        axpby(nv, 1.0, b, 0.0, nullptr, r1, s);
    } else {
        op(x, t);
        out.products++;
        axpby(nv, 1.0, b, -1.0, t, r1, s);
    }
    dot_vector(c, r1, r1, nv, W.sc(1), s);
    out.relres = std::sqrt(read_scalar(c, W.sc(1), s)) / bnorm;
    if (out.relres <= tol) {
        out.converged = true;
        return out;
    }
    for (;;) {
        if (out.products >= max_it) return out;
        minres_start(c, n, r1, eta, y, ms, s);
        axpby(nv, 1.0, r1, 0.0, nullptr, r2, s);
        axpby(nv, 0.0, r1, 0.0, nullptr, wa, s);
        axpby(nv, 0.0, r1, 0.0, nullptr, wb, s);
        if (!have_step) {
            step = step_graph(W, body, nv, 3, eta);
            have_step = true;
        }
        const double stop = target * bnorm_d;
        int launched = 0;
        bool hit = false;
        for (int k = 0;; ++k) {
            if (out.products >= max_it) break;
            if (step)
                PQ_HIP(hipGraphLaunch(step, s));
            else
                body();
            out.products++;
            ++launched;
            PQ_HIP(hipMemcpyAsync(c.pinned_hist + (k & 1), ms + MR_PHIBAR, sizeof(double), hipMemcpyDeviceToHost, s));
            PQ_HIP(hipEventRecord(c.kev[k & 1], s));
            if (k >= 1) {
                PQ_HIP(hipEventSynchronize(c.kev[(k - 1) & 1]));
                if (c.pinned_hist[(k - 1) & 1] <= stop) {
                    hit = true;
                    break;
                }
            }
        }
        if (!hit && launched > 0) PQ_HIP(hipEventSynchronize(c.kev[(launched - 1) & 1]));
        // true residual (also the next cycle's start)
        op(x, t);
        out.products++;
        axpby(nv, 1.0, b, -1.0, t, r1, s);
        dot_vector(c, r1, r1, nv, W.sc(1), s);
        out.relres = std::sqrt(read_scalar(c, W.sc(1), s)) / bnorm;
        if (out.relres <= tol) {
            out.converged = true;
            return out;
        }
        if (out.products >= max_it) return out;
        target *= std::max(0.01, 0.5 * tol / out.relres);
        out.restarts++;
    }
}

void check_finite_host(double v, const char* what) {
    PQ_REQUIRE(std::isfinite(v), PQ_ERR_INVALID, std::string(what) + " must be finite");
}

// bordered QEQ product with right Jacobi preconditioning diag(u, 1):
//   out = [y_q + phi[y_q/u] + y_l ; sum y_q/u]
OpFn bordered_op(Work& W, const double* eta) {
    return [&W, eta](const double* y, double* out) {
        Ctx& c = W.c;
        hipStream_t s = c.stream;
        const int64_t n = c.n;
        double* t = W.w(W_T);
        double* phi = W.w(W_PHI2);
        vdiv(n, y, eta, t, s);
        coulomb_eval(c, t, phi, nullptr, nullptr, s);
        reduce(c, t, nullptr, n, 0, 1.0, W.sc(4), s);
        bordered_out(n, y, phi, W.sc(4), out, s);
    };
}

// bordered QEQ product without preconditioning (MINRES):
//   out = [u o v_q + phi[v_q] + v_l ; sum v_q]
OpFn plain_op(Work& W, const double* eta) {
    return [&W, eta](const double* v, double* out) {
        Ctx& c = W.c;
        hipStream_t s = c.stream;
        const int64_t n = c.n;
        double* phi = W.w(W_PHI2);
        coulomb_eval(c, v, phi, nullptr, nullptr, s);
        reduce(c, v, nullptr, n, 0, 1.0, W.sc(4), s);
        bordered_plain(n, v, eta, phi, W.sc(4), out, s);
    };
}

// bordered solve for right-hand side [rhs_q; rhs_l] by the context's Krylov
// method. GMRES: the solution z = P^-1 x is left as q = x_q/u in qout;
// MINRES: z = x, q = x_q. lambda is x[n] in both.
GmresOut bordered_solve(Work& W, const double* eta, const double* rhs_q, double rhs_l, bool negate_rhs,
                        const double* q0, double tol, int max_it, double* qout) {
    Ctx& c = W.c;
    hipStream_t s = c.stream;
    const int64_t n = c.n;
    double* b = W.w(W_B);
    double* x = W.w(W_X);
    axpby(n, negate_rhs ? -1.0 : 1.0, rhs_q, 0.0, nullptr, b, s);
    set_scalar(b + n, rhs_l, s);
    bool xz = true;
    if (q0) {
        vmul(n, q0, eta, 1.0, x, s);
        set_scalar(x + n, 0.0, s);
        xz = false;
    }
    if (c.solver == PQ_SOLVER_MINRES) {
        if (q0) {
            axpby(n, 1.0, q0, 0.0, nullptr, x, s);
            set_scalar(x + n, 0.0, s);
        }
        GmresOut o = minres(W, plain_op(W, eta), eta, n, b, x, !q0, tol, max_it);
        axpby(n, 1.0, x, 0.0, nullptr, qout, s);
        return o;
    }
    OpFn op = bordered_op(W, eta);
    GmresOut o = gmres(W, op, n + 1, b, x, xz, tol, max_it, false, 1, eta);
    vdiv(n, x, eta, qout, s);
    return o;
}

}  // namespace
}  // namespace pq

using namespace pq;

#define PQ_API_BEGIN try {
#define PQ_API_END                    \
    }                                 \
    catch (const pq::Error& e) {      \
        pq::set_error(e.what());      \
        return e.code;                \
    }                                 \
    catch (const std::exception& e) { \
        pq::set_error(e.what());      \
        return PQ_ERR_INVALID;        \
    }                                 \
    catch (...) {                     \
        pq::set_error("unknown error"); \
        return PQ_ERR_INVALID;        \
    }

extern "C" {

pq_status pq_set_solver(pq_ctx* ctx, int32_t solver, int32_t vjp_restart) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr, PQ_ERR_INVALID, "ctx is NULL");
    PQ_REQUIRE(solver == PQ_SOLVER_GMRES || solver == PQ_SOLVER_MINRES, PQ_ERR_INVALID, "unknown solver");
    PQ_REQUIRE(vjp_restart >= 1 && vjp_restart <= PQ_MAX_RESTART, PQ_ERR_INVALID, "vjp_restart must be in 1..4096");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    c.solver = solver;
    c.vjp_restart = vjp_restart;
    return PQ_OK;
    PQ_API_END
}

pq_status pq_qeq_solve(pq_ctx* ctx, const double* chi, const double* eta, double q_tot, double tol, int max_it,
                       int restart, const double* q0, double* q, double* force, double* energy, pq_solve_info* info) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx && chi && eta && q, PQ_ERR_INVALID, "ctx, chi, eta and q must not be NULL");
    PQ_REQUIRE(tol > 0.0 && max_it >= 1 && restart >= 1 && restart <= PQ_MAX_RESTART, PQ_ERR_INVALID,
               "need tol > 0, max_it >= 1, 1 <= restart <= 4096");
    check_finite_host(q_tot, "q_tot");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_HIP(hipSetDevice(c.device));
    hipStream_t s = c.stream;
    Work W(c, c.solver == PQ_SOLVER_MINRES ? 1 : restart);
    GmresOut o = bordered_solve(W, eta, chi, q_tot, true, q0, tol, max_it, q);
    double lam = read_scalar(c, W.w(W_X) + c.n, s);
    if (force || energy) {
        double* phi = W.w(W_PHI);
        coulomb_eval(c, q, phi, force, nullptr, s);
        if (energy) qeq_energy(c, c.n, q, chi, eta, q, phi, energy, s);
    }
    if (info) {
        info->iterations = o.products;
        info->restarts = o.restarts;
        info->rel_residual = o.relres;
        info->lambda = lam;
    }
    PQ_HIP(hipStreamSynchronize(s));
    return o.converged ? PQ_OK : PQ_WARN_NOT_CONVERGED;
    PQ_API_END
}

pq_status pq_shadow_step(pq_ctx* ctx, const double* chi, const double* eta, double q_tot, const double* n_vec,
                         int n_krylov, double* q_n, double* force, double* nddot, double* energy) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx && chi && eta && n_vec && q_n, PQ_ERR_INVALID, "ctx, chi, eta, n_vec and q_n must not be NULL");
    PQ_REQUIRE(n_krylov >= 1 && n_krylov <= 512, PQ_ERR_INVALID, "n_krylov must be in 1..512");
    check_finite_host(q_tot, "q_tot");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_HIP(hipSetDevice(c.device));
    hipStream_t s = c.stream;
    const int64_t n = c.n;
    Work W(c, n_krylov);
    c.kf.ensure((size_t)n * 3);
    // v = A n ; q[n] and lambda in closed form. With PME and a force to
    // compute, the evaluation keeps its convolved grid of n for the bilinear
    // force below.
    const bool bil = force && c.prm.method == PQ_METHOD_PME;
    if (bil) ensure_bilinear(c);
    double* phin = W.w(W_PHI);
    c.save_psi = bil;
    try {
        coulomb_eval(c, n_vec, phin, nullptr, nullptr, s);
    } catch (...) {
        c.save_psi = false;
        throw;
    }
    c.save_psi = false;
    shadow_sums(c, n, chi, phin, eta, W.sc(5), s);
    shadow_q(n, chi, phin, eta, W.sc(5), q_tot, q_n, W.sc(7), s);
    // shadow force F[q] - F[q - n] = -d/dR 1/2 (2q - n)^T A n
    if (force) {
        double* d = W.w(W_D);
        if (bil) {
            axpby(n, 2.0, q_n, -1.0, n_vec, d, s);
            coulomb_bilinear_force(c, d, n_vec, true, force, s);
        } else {
            coulomb_eval(c, q_n, nullptr, force, nullptr, s);
            axpby(n, 1.0, q_n, -1.0, n_vec, d, s);
            coulomb_eval(c, d, nullptr, c.kf.p, nullptr, s);
            axpby(3 * n, 1.0, force, -1.0, c.kf.p, force, s);
        }
    }
    if (energy) {
        double* a = W.w(W_D);
        axpby(n, 2.0, q_n, -1.0, n_vec, a, s);
        qeq_energy(c, n, q_n, chi, eta, a, phin, energy, s);
        copy_scalar(W.sc(7), energy + 1, s);
    }
    if (nddot) {
        // J x = -x - P D^-1 A x,  P y = y - D^-1 1 (1^T y) / (1^T D^-1 1)
        OpFn op = [&W, eta](const double* x, double* out) {
            Ctx& cc = W.c;
            hipStream_t ss = cc.stream;
            const int64_t nn = cc.n;
            double* phi = W.w(W_PHI2);
            double* t = W.w(W_T);
            coulomb_eval(cc, x, phi, nullptr, nullptr, ss);
            vdiv(nn, phi, eta, t, ss);
            shadow_sums(cc, nn, nullptr, phi, eta, W.sc(8), ss);
            jac_out(nn, x, t, eta, W.sc(8), out, ss);
        };
        double* b = W.w(W_B);
        axpby(n, 1.0, n_vec, -1.0, q_n, b, s);   // -(q[n] - n)
        gmres(W, op, n, b, nddot, true, 0.0, n_krylov, true, 2, eta);
    }
    return PQ_OK;
    PQ_API_END
}

pq_status pq_qeq_vjp(pq_ctx* ctx, const double* chi, const double* eta, const double* q_star, const double* gbar,
                     double tol, int max_it, double* d_pos, double* d_chi, double* d_eta) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx && chi && eta && q_star, PQ_ERR_INVALID, "ctx, chi, eta and q_star must not be NULL");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_HIP(hipSetDevice(c.device));
    hipStream_t s = c.stream;
    const int64_t n = c.n;
    if (!gbar) {
        // envelope theorem: dE/dR = -F[q*], dE/dchi = q*, dE/du = q*^2 / 2
        if (d_pos) {
            coulomb_eval(c, q_star, nullptr, d_pos, nullptr, s);
            axpby(3 * n, -1.0, d_pos, 0.0, nullptr, d_pos, s);
        }
        if (d_chi) axpby(n, 1.0, q_star, 0.0, nullptr, d_chi, s);
        if (d_eta) vmul(n, q_star, q_star, 0.5, d_eta, s);
        return PQ_OK;
    }
    PQ_REQUIRE(tol > 0.0 && max_it >= 1, PQ_ERR_INVALID, "need tol > 0 and max_it >= 1");
    Work W(c, c.solver == PQ_SOLVER_MINRES ? 1 : c.vjp_restart);
    c.kf.ensure((size_t)n * 3);
    double* a = W.w(W_D);
    GmresOut o = bordered_solve(W, eta, gbar, 0.0, false, nullptr, tol, max_it, a);
    if (d_chi) axpby(n, -1.0, a, 0.0, nullptr, d_chi, s);
    if (d_eta) vmul(n, a, q_star, -1.0, d_eta, s);
    if (d_pos) {
        // dL/dR = F[a + q] - F[a] - F[q] = -d/dR (a^T A q)
        double* aq = W.w(W_PHI);
        if (c.prm.method == PQ_METHOD_PME) {
            axpby(n, 2.0, a, 0.0, nullptr, aq, s);
            coulomb_bilinear_force(c, aq, q_star, false, d_pos, s);
        } else {
            axpby(n, 1.0, a, 1.0, q_star, aq, s);
            coulomb_eval(c, aq, nullptr, d_pos, nullptr, s);
            coulomb_eval(c, a, nullptr, c.kf.p, nullptr, s);
            axpby(3 * n, 1.0, d_pos, -1.0, c.kf.p, d_pos, s);
            coulomb_eval(c, q_star, nullptr, c.kf.p, nullptr, s);
            axpby(3 * n, 1.0, d_pos, -1.0, c.kf.p, d_pos, s);
        }
    }
    PQ_HIP(hipStreamSynchronize(s));
    return o.converged ? PQ_OK : PQ_WARN_NOT_CONVERGED;
    PQ_API_END
}

}  // extern "C"
