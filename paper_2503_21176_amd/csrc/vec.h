// FP64 vector and small-dense helpers of the Krylov solvers (vec.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pq_internal.h"

namespace pq {

// Layout of the small GMRES state for restart length m (all FP64):
// H (m+1) x m column-major, then g[m+1], cs[m], sn[m], y[m], h2[m+1],
// hist[m] (|g[j+1]| after step j).
__host__ __device__ inline size_t gs_g(int m) { return (size_t)(m + 1) * m; }
__host__ __device__ inline size_t gs_c(int m) { return gs_g(m) + m + 1; }
__host__ __device__ inline size_t gs_s(int m) { return gs_c(m) + m; }
__host__ __device__ inline size_t gs_y(int m) { return gs_s(m) + m; }
__host__ __device__ inline size_t gs_t(int m) { return gs_y(m) + m; }
__host__ __device__ inline size_t gs_hist(int m) { return gs_t(m) + m + 2; }   // residual estimates, m
__host__ __device__ inline size_t gs_size(int m) { return gs_hist(m) + m + 1; }

// Device scalar state of the preconditioned MINRES solver (FP64, MR_N words).
enum { MR_BETA = 0, MR_BETA1, MR_OLDB, MR_ALFA, MR_BETA2, MR_DBAR, MR_EPS, MR_PHIBAR, MR_CS, MR_SN, MR_PHI,
       MR_DELTA, MR_OLDEPS, MR_DENOM, MR_N };

// mode 0: sum x; 1: sum x*y; 2: sum x/y. out = alpha * result (device scalar)
void reduce(Ctx& c, const double* x, const double* y, int64_t n, int mode, double alpha, double* out, hipStream_t s);
void axpby(int64_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s);
void vdiv(int64_t n, const double* x, const double* u, double* z, hipStream_t s);
void vmul(int64_t n, const double* x, const double* u, double sc, double* z, hipStream_t s);
void bordered_out(int64_t n, const double* y, const double* phi, const double* tsum, double* out, hipStream_t s);
void jac_out(int64_t n, const double* x, const double* t, const double* u, const double* sums, double* out,
             hipStream_t s);
void shadow_sums(Ctx& c, int64_t n, const double* chi, const double* v, const double* u, double* out2, hipStream_t s);
void shadow_q(int64_t n, const double* chi, const double* v, const double* u, const double* sums, double qtot,
              double* q, double* lam, hipStream_t s);
void normalize(int64_t n, const double* w, const double* nrm2, double* hsub, double* out, hipStream_t s);
void gmres_start(double* st, int m, const double* nrm2, hipStream_t s);
void backsolve(double* st, int m, int k, hipStream_t s);
// x += sum_{k < nk} y[k] V_k; up: chunk sums (vcomb_chunks(nk) x ld) when nk > 32
void xupdate(int64_t n, const double* V, size_t ld, int nk, const double* y, double* x, double* up, hipStream_t s);
size_t vcomb_chunks(int nk);
void qeq_energy(Ctx& c, int64_t n, const double* q, const double* chi, const double* u, const double* a,
                const double* phi, double* out, hipStream_t s);
void copy_scalar(const double* a, double* b, hipStream_t s);
// device-indexed forms: the step index j is *jdev (graph-captured steps)
void copy_j(int64_t n, const double* V, size_t ld, const int* jdev, double* out, hipStream_t s);
// CGS2 of w against V_0..V_{*jdev} into column *jdev of H; up: chunk sums
// (vcomb_chunks(m + 1) x ld) when m + 1 > 32
void orthogonalize_j(Ctx& c, int64_t n, const double* V, size_t ld, int m, const int* jdev, double* w, double* st,
                     double* tmp2, double* up, hipStream_t s);
void normalize_j(int64_t n, const double* w, const double* nrm2, double* st, int m, double* V, size_t ld,
                 const int* jdev, hipStream_t s);
void givens_j(double* st, int m, int* jdev, double* hist, hipStream_t s);
void set_int(int* p, int v, hipStream_t s);
void set_scalar(double* b, double v, hipStream_t s);
// preconditioned MINRES on the bordered system (n + 1 unknowns, D = diag(u, 1)):
// cycle start from the residual r (y = D^-1 r, beta1 = sqrt(r . y)), the
// vector v = y / beta that the step applies the operator to, and the rest of
// the step after y = M v (the estimate phibar lands in ms[MR_PHIBAR])
void minres_start(Ctx& c, int64_t n, const double* r, const double* u, double* y, double* ms, hipStream_t s);
void minres_v(int64_t nv, const double* y, const double* ms, double* v, hipStream_t s);
void minres_update(Ctx& c, int64_t n, double* y, double* r1, double* r2, const double* v, const double* u, double* wa,
                   double* wb, double* x, double* ms, hipStream_t s);
// out = [u o v + phi + v_n ; *vsum] (the bordered product without preconditioning)
void bordered_plain(int64_t n, const double* v, const double* u, const double* phi, const double* vsum, double* out,
                    hipStream_t s);

}  // namespace pq
