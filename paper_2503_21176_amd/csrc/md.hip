// Shadow Born-Oppenheimer MD driver (Section "Shadow Born-Oppenheimer MD for
// a Charge Equilibration Model"): the atoms move on the shadow potential
// U(R, n) = V_short(R) + E(R, q[n], n) with the force at fixed n, and the
// extended charges n(t) follow n'' = -omega^2 K (q[n] - n), whose right-hand
// side J x = -(q[n] - n) the shadow step approximates by a few Krylov steps.
//
// Integration (units A, fs, amu, eV):
//   v += dt/2 F/m ;  R += dt v                      (velocity Verlet)
//   n(t+dt) = 2 n(t) - n(t-dt) + kappa x(t) + alpha sum_k c_k n(t-k dt)
//                                                   (kappa = dt^2 omega^2)
//   move the system to R(t+dt) (neighbour list kept within the skin rule);
//   shadow step at (R, n)(t+dt) -> F, x, E_shadow
//   v += dt/2 F/m
// The n update is the time-reversible Verlet step of extended-Lagrangian
// BOMD with the weak dissipation of Niklasson et al. (J. Chem. Phys. 130,
// 214109, 2009), K = 5: kappa = 1.82, alpha = 0.018,
// c = (-6, 14, -8, -3, 4, -1); or, without dissipation, alpha = 0 and a
// caller-chosen kappa.
// Regular Born-Oppenheimer mode (Section "Regular Born-Oppenheimer MD for a
// Charge Equilibration Model"): each force evaluation instead solves the QEQ
// system to a relative residual tol by the Jacobi-preconditioned GMRES of
// pq_qeq_solve, started from the previous step's charges, and takes the force
// and energy at those charges (exact only at convergence).
// V_short: the paper's short-range model is a trained network that is not
// part of this library; a repulsive pair term A exp(-r/rho) summed over every
// pair (and periodic image) closer than the cutoff stands in for it, in FP64,
// by brute force over all pairs (sized for MD test systems of up to a few
// thousand atoms).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dev.h"
#include "pmeqeq.h"
#include "pq_internal.h"

namespace pq {

constexpr double ACC_PER_EV_A_AMU = 9.648533212331e-3;   // (eV/A)/amu in A/fs^2
constexpr int MD_TILE = 256;
constexpr int MD_COLS = 6;   // kinetic, potential, V_short, total, Coulomb evaluations, list rebuilt

__global__ void k_md_kick(int64_t n3, double* __restrict__ v, const double* __restrict__ f,
                          const double* __restrict__ m, double c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) v[i] += c * f[i] / m[i / 3];
}

__global__ void k_md_drift(int64_t n3, double* __restrict__ x, const double* __restrict__ v, double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) x[i] += dt * v[i];
}

struct XlCoef {
    double c[8];
};

// hist holds H vectors of n; slot (head + k) % H is n(t - k dt). Writes
// n(t + dt) into slot (head + H - 1) % H, the oldest, after reading it.
__global__ void k_md_nupdate(int64_t n, double* __restrict__ hist, int H, int head, const double* __restrict__ x,
                             double kappa, double alpha, XlCoef cf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double n0 = hist[(size_t)head * n + i];
    const double n1 = hist[(size_t)((head + 1) % H) * n + i];
    double d = 0.0;
    if (alpha != 0.0)
        for (int k = 0; k < H; ++k) d += cf.c[k] * hist[(size_t)((head + k) % H) * n + i];
    hist[(size_t)((head + H - 1) % H) * n + i] = 2.0 * n0 - n1 + kappa * x[i] + alpha * d;
}

// out slot k = in slot (head + k) % H (newest first)
__global__ void k_md_unroll(int64_t n, const double* __restrict__ hist, int H, int head, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * H) return;
    const int k = (int)(t / n);
    const int64_t i = t - (int64_t)k * n;
    out[t] = hist[(size_t)((head + k) % H) * n + i];
}

__global__ void k_md_kinetic(int64_t n, const double* __restrict__ v, const double* __restrict__ m,
                             double* __restrict__ part) {
    __shared__ double red[MD_TILE / 64];
    double e = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * MD_TILE + threadIdx.x; i < n; i += (int64_t)gridDim.x * MD_TILE)
        e += 0.5 * m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
    e = block_sum<MD_TILE>(e, red);
    if (threadIdx.x == 0) part[blockIdx.x] = e / ACC_PER_EV_A_AMU;
}

// Repulsive stand-in for V_short: per pair (j, image) with 0 < r < rc,
// E = A exp(-r/rho); atom i gets F_i = sum (A/rho) exp(-r/rho) (r_i - r_j')/r and
// E_i = 1/2 sum E. Positions: the wrapped FP64 coordinates. One wavefront per
// atom i, its lanes taking every 64th partner j; the lane sums are combined by
// a fixed butterfly, and part[block] holds the block's energy.
constexpr int MD_SHORT_WAVES = MD_TILE / 64;   // atoms per block
__global__ __launch_bounds__(MD_TILE) void k_md_short(int n, const double* __restrict__ w, double L0, double L1,
                                                      double L2, double rc, double A, double rho,
                                                      double* __restrict__ f, double* __restrict__ part) {
    __shared__ double red[MD_SHORT_WAVES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * MD_SHORT_WAVES + wv;
    const double rc2 = rc * rc, inv_rho = 1.0 / rho;
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    if (i < n) {
        const double xi = w[3 * (size_t)i], yi = w[3 * (size_t)i + 1], zi = w[3 * (size_t)i + 2];
        for (int j = lane; j < n; j += 64) {
            // minimum image, then every image within the cutoff
            double d0 = w[3 * (size_t)j] - xi, d1 = w[3 * (size_t)j + 1] - yi, d2 = w[3 * (size_t)j + 2] - zi;
            d0 -= L0 * rint(d0 / L0);
            d1 -= L1 * rint(d1 / L1);
            d2 -= L2 * rint(d2 / L2);
            const int a0 = (int)ceil((-rc - d0) / L0), b0 = (int)floor((rc - d0) / L0);
            const int a1 = (int)ceil((-rc - d1) / L1), b1 = (int)floor((rc - d1) / L1);
            const int a2 = (int)ceil((-rc - d2) / L2), b2 = (int)floor((rc - d2) / L2);
            for (int p = a0; p <= b0; ++p)
                for (int q = a1; q <= b1; ++q)
                    for (int r = a2; r <= b2; ++r) {
                        const double ex = d0 + p * L0, ey = d1 + q * L1, ez = d2 + r * L2;
                        const double r2 = ex * ex + ey * ey + ez * ez;
                        if (r2 >= rc2 || r2 == 0.0) continue;
                        const double rr = sqrt(r2);
                        const double v = A * exp(-rr * inv_rho);
                        const double g = v * inv_rho / rr;   // -dE/dr / r
                        fx -= g * ex;
                        fy -= g * ey;
                        fz -= g * ez;
                        e += 0.5 * v;
                    }
        }
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    fz = wave_sum(fz);
    e = wave_sum(e);
    if (lane == 0) {
        if (i < n) {
            f[3 * (size_t)i] += fx;
            f[3 * (size_t)i + 1] += fy;
            f[3 * (size_t)i + 2] += fz;
        }
        red[wv] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < MD_SHORT_WAVES; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

__global__ void k_md_record(const double* __restrict__ kin_part, int nk, const double* __restrict__ sr_part, int ns,
                            const double* __restrict__ e_pot, double evals, double rebuilt, double* __restrict__ row) {
    // one wavefront: lane-strided partial sums, then a fixed butterfly
    if (blockIdx.x != 0 || threadIdx.x >= 64) return;
    double ke = 0.0, es = 0.0;
    for (int k = threadIdx.x; k < nk; k += 64) ke += kin_part[k];
    for (int k = threadIdx.x; k < ns; k += 64) es += sr_part[k];
    ke = wave_sum(ke);
    es = wave_sum(es);
    if (threadIdx.x != 0) return;
    row[0] = ke;
    row[1] = e_pot[0];
    row[2] = es;
    row[3] = (ke + e_pot[0]) + es;
    row[4] = evals;
    row[5] = rebuilt;
}

void set_error(const std::string& m);

static void check(pq_status st) {
    if (st != PQ_OK) throw Error(st, pq_last_error());
}

// vectors of n kept in the history: n(t), ..., n(t - K dt)
static int md_history(int dissipation) { return dissipation == 5 ? 6 : 2; }

void md_run(Ctx& c, double* pos, double* vel, const double* mass, const double* chi, const double* eta,
            double q_tot, double* n_hist, double* pos_ref, int steps, const pq_md_cfg& cfg, double* energies) {
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_REQUIRE(!is_tric(c.prm), PQ_ERR_BOX, "the MD driver takes orthorhombic boxes (zero tilts)");
    PQ_REQUIRE(std::isfinite(cfg.dt_fs) && cfg.dt_fs > 0.0, PQ_ERR_INVALID, "dt_fs must be > 0");
    PQ_REQUIRE(cfg.n_krylov >= 1 && cfg.n_krylov <= 512, PQ_ERR_INVALID, "n_krylov must be in 1..512");
    PQ_REQUIRE(cfg.dissipation == 0 || cfg.dissipation == 5, PQ_ERR_INVALID, "dissipation must be 0 or 5");
    PQ_REQUIRE(std::isfinite(cfg.kappa) && cfg.rep_a >= 0.0 && (cfg.rep_a == 0.0 || cfg.rep_rho > 0.0),
               PQ_ERR_INVALID, "bad kappa or repulsion parameters");
    PQ_REQUIRE(steps >= 0, PQ_ERR_INVALID, "steps must be >= 0");
    PQ_REQUIRE(cfg.mode == PQ_MD_SHADOW || cfg.mode == PQ_MD_REGULAR, PQ_ERR_INVALID, "unknown MD mode");
    const bool regular = cfg.mode == PQ_MD_REGULAR;
    if (regular)
        PQ_REQUIRE(std::isfinite(cfg.tol) && cfg.tol > 0.0 && cfg.max_it >= 1 && cfg.restart >= 1, PQ_ERR_INVALID,
                   "regular mode needs tol > 0, max_it >= 1, restart >= 1");
    const int64_t n = c.n;
    const int H = md_history(cfg.dissipation);
    XlCoef cf{};
    double kappa = cfg.kappa, alpha = 0.0;
    if (cfg.dissipation == 5) {
        const double c5[6] = {-6.0, 14.0, -8.0, -3.0, 4.0, -1.0};
        for (int k = 0; k < 6; ++k) cf.c[k] = c5[k];
        kappa = 1.82;
        alpha = 0.018;
    }
    const pq_params prm = c.prm;
    hipStream_t s = c.stream;
    // every step rebuilds the system: no Arnoldi-step graphs
    const bool graphs_was = c.graphs;
    c.graphs = false;
    DBuf<double> f, x, qn, esh, kin, srp, hist2, rows;
    const int nb3 = (int)cdiv(3 * n, 256), nb1 = (int)cdiv(n, 256);
    const int kb = std::min<int>(256, std::max(1, nb1));
    const int sb = (int)cdiv(n, MD_SHORT_WAVES);
    f.ensure(3 * n);
    x.ensure(n);
    qn.ensure(n);
    esh.ensure(2);
    kin.ensure(kb);
    srp.ensure(std::max(1, sb));
    rows.ensure((size_t)MD_COLS * (steps + 1));
    DBuf<double> qprev;
    if (regular) {
        // charges of the previous step (start vector of each solve): n_hist[0] on entry
        qprev.ensure(n);
        PQ_HIP(hipMemcpyAsync(qprev.p, n_hist, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    double evals = 0.0;   // Coulomb evaluations of the current force evaluation
    double rebuilt = 0.0;
    int head = 0;   // n_hist is newest first on entry
    pq_ctx* h = reinterpret_cast<pq_ctx*>(&c);
    auto forces = [&](int row) {
        int32_t rb = 1;
        if (row == 0 && pos_ref) {
            // the list of the interrupted run: built at pos_ref, moved to pos
            check(pq_set_system(h, n, pos_ref, &prm));
            check(pq_update_positions(h, pos, &rb));
        } else if (row == 0) {
            check(pq_set_system(h, n, pos, &prm));
        } else {
            check(pq_update_positions(h, pos, &rb));
        }
        rebuilt = rb ? 1.0 : 0.0;
        if (regular) {
            pq_solve_info info{};
            const pq_status st = pq_qeq_solve(reinterpret_cast<pq_ctx*>(&c), chi, eta, q_tot, cfg.tol, cfg.max_it,
                                              cfg.restart, qprev.p, qn.p, f.p, esh.p, &info);
            if (st != PQ_WARN_NOT_CONVERGED) check(st);
            PQ_HIP(hipMemcpyAsync(qprev.p, qn.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            evals = info.iterations + 1.0;   // products + the force evaluation
        } else {
            check(pq_shadow_step(reinterpret_cast<pq_ctx*>(&c), chi, eta, q_tot, n_hist + (size_t)head * n,
                                 cfg.n_krylov, qn.p, f.p, x.p, esh.p));
            // potential of n, the shadow force (PME: one bilinear evaluation,
            // counted as two), Krylov products
            evals = 3.0 + cfg.n_krylov;
        }
        if (cfg.rep_a > 0.0)
            PQ_LAUNCH(k_md_short, sb, MD_TILE, 0, s, (int)n, c.w64.p, prm.box[0], prm.box[1], prm.box[2],
                      prm.cutoff, cfg.rep_a, cfg.rep_rho, f.p, srp.p);
        (void)row;
    };
    auto record = [&](int row) {
        PQ_LAUNCH(k_md_kinetic, kb, MD_TILE, 0, s, n, (const double*)vel, mass, kin.p);
        PQ_LAUNCH(k_md_record, 1, 64, 0, s, (const double*)kin.p, kb, (const double*)srp.p,
                  cfg.rep_a > 0.0 ? sb : 0, (const double*)esh.p, evals, rebuilt, rows.p + (size_t)MD_COLS * row);
    };
    try {
        forces(0);
        record(0);
        const double hdt = 0.5 * cfg.dt_fs * ACC_PER_EV_A_AMU;
        for (int t = 0; t < steps; ++t) {
            PQ_LAUNCH(k_md_kick, nb3, 256, 0, s, 3 * n, vel, (const double*)f.p, mass, hdt);
            PQ_LAUNCH(k_md_drift, nb3, 256, 0, s, 3 * n, pos, (const double*)vel, cfg.dt_fs);
            if (!regular) {
                PQ_LAUNCH(k_md_nupdate, nb1, 256, 0, s, n, n_hist, H, head, (const double*)x.p, kappa, alpha, cf);
                head = (head + H - 1) % H;
            }
            forces(t + 1);
            PQ_LAUNCH(k_md_kick, nb3, 256, 0, s, 3 * n, vel, (const double*)f.p, mass, hdt);
            record(t + 1);
        }
        // history back in newest-first order
        if (head != 0) {
            hist2.ensure((size_t)H * n);
            PQ_LAUNCH(k_md_unroll, (unsigned)cdiv((int64_t)H * n, 256), 256, 0, s, n, (const double*)n_hist, H, head,
                      hist2.p);
            PQ_HIP(hipMemcpyAsync(n_hist, hist2.p, sizeof(double) * H * n, hipMemcpyDeviceToDevice, s));
        }
        if (regular) PQ_HIP(hipMemcpyAsync(n_hist, qprev.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        // positions of the last full build (with skin 0 every step rebuilt)
        if (pos_ref) {
            const double* last = (prm.skin > 0.0 && c.pos_build.n >= (size_t)n * 3) ? c.pos_build.p : pos;
            PQ_HIP(hipMemcpyAsync(pos_ref, last, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
        }
        if (energies)
            PQ_HIP(hipMemcpyAsync(energies, rows.p, sizeof(double) * MD_COLS * (steps + 1), hipMemcpyDeviceToHost, s));
        PQ_HIP(hipStreamSynchronize(s));
    } catch (...) {
        c.graphs = graphs_was;
        throw;
    }
    c.graphs = graphs_was;
}

}  // namespace pq

using namespace pq;

extern "C" pq_status pq_md_run(pq_ctx* ctx, double* pos, double* vel, const double* mass, const double* chi,
                               const double* eta, double q_tot, double* n_hist, double* pos_ref, int32_t steps,
                               const pq_md_cfg* cfg, double* energies) {
    pq::CtxErrScope err_scope(ctx);
    try {
        PQ_REQUIRE(ctx && pos && vel && mass && chi && eta && n_hist && cfg, PQ_ERR_INVALID,
                   "ctx, pos, vel, mass, chi, eta, n_hist and cfg must not be NULL");
        Ctx& c = *reinterpret_cast<Ctx*>(ctx);
        AllocScope alloc_scope(c);
        PQ_HIP(hipSetDevice(c.device));
        md_run(c, pos, vel, mass, chi, eta, q_tot, n_hist, pos_ref, steps, *cfg, energies);
        return PQ_OK;
    } catch (const Error& e) {
        set_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return PQ_ERR_INVALID;
    }
}

extern "C" int32_t pq_md_history(int32_t dissipation) { return md_history(dissipation); }
