// FP64 reductions and vector kernels: energy assembly (self and background
// terms, the paper's eq. ewald_self plus the neutralising background), and the
// building blocks of the Krylov solvers (dot products, classical Gram-Schmidt
// with one re-orthogonalisation, Givens rotations of the Hessenberg matrix).
// Every reduction uses fixed block partials summed in a fixed order, so the
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dev.h"
#include "pq_internal.h"
#include "vec.h"

namespace pq {

constexpr int VB = 256;   // threads per block of the vector kernels

// ---- reductions -----------------------------------------------------------
// MK sums over the VB threads of a block, reduced together (the same tree per
// sum as block_sum); the totals land in thread 0's v[].
template <int MK>
__device__ __forceinline__ void block_sum_n(double (&v)[MK], double* lds /* (VB/64) * MK */) {
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < MK; ++k) v[k] += __shfl_xor(v[k], o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < MK; ++k) lds[w * MK + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            double t = 0.0;
            for (int ww = 0; ww < VB / 64; ++ww) t += lds[ww * MK + k];
            v[k] = t;
        }
    }
    __syncthreads();
}
constexpr int MD_K = 8;   // dot products (or columns) reduced together

// Partial sums of x (mode 0), x.y (mode 1) or x/y (mode 2) per block.
__global__ __launch_bounds__(VB) void k_part_sum(const double* __restrict__ x, const double* __restrict__ y,
                                                 int64_t n, int mode, double* __restrict__ part) {
    __shared__ double red[VB / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const double a = x[i];
        v += (mode == 0) ? a : (mode == 1 ? a * y[i] : a / y[i]);
    }
    v = block_sum<VB>(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// Step index of a graph-captured Arnoldi step: *jdev when given, else j.
__device__ __forceinline__ int step_of(const int* jdev, int j) { return jdev ? *jdev : j; }

// out[k] = alpha * sum of part[k*nb .. k*nb+nb-1], k < nk; with jdev:
// nk = *jdev + 1 and out advanced by *jdev * ostride
// With acc, also acc[k] += out[k] (acc advanced by *jdev * astride with jdev).
__global__ __launch_bounds__(VB) void k_part_final(const double* __restrict__ part, int nb, int nk, double alpha,
                                                   double* __restrict__ out, const int* __restrict__ jdev,
                                                   size_t ostride, double* __restrict__ acc, size_t astride) {
    __shared__ double red[(VB / 64) * MD_K];
    if (jdev) {
        nk = *jdev + 1;
        out += (size_t)(*jdev) * ostride;
        if (acc) acc += (size_t)(*jdev) * astride;
    }
    for (int k0 = 0; k0 < nk; k0 += MD_K) {
        double v[MD_K];
#pragma unroll
        for (int k = 0; k < MD_K; ++k) {
            v[k] = 0.0;
            if (k0 + k < nk)
                for (int i = threadIdx.x; i < nb; i += VB) v[k] += part[(size_t)(k0 + k) * nb + i];
        }
        block_sum_n<MD_K>(v, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < MD_K; ++k) {
                if (k0 + k >= nk) break;
                const double r = alpha * v[k];
                out[k0 + k] = r;
                if (acc) acc[k0 + k] = acc[k0 + k] + r;
            }
        }
    }
}

static int red_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + VB - 1) / VB)); }

void reduce(Ctx& c, const double* x, const double* y, int64_t n, int mode, double alpha, double* out, hipStream_t s) {
    const int nb = red_blocks(n);
    c.part.ensure(nb + 16);
    PQ_LAUNCH(k_part_sum, nb, VB, 0, s, x, y, n, mode, c.part.p);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, c.part.p, nb, 1, alpha, out, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
}

void sum_vector(Ctx& c, const double* x, int64_t n, double* out, hipStream_t s) { reduce(c, x, nullptr, n, 0, 1.0, out, s); }
void sum_vector_into(const double* x, int64_t n, double* out, double* part, hipStream_t s) {
    const int nb = red_blocks(n);
    PQ_LAUNCH(k_part_sum, nb, VB, 0, s, x, (const double*)nullptr, n, 0, part);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, part, nb, 1, 1.0, out, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
}
void dot_vector(Ctx& c, const double* x, const double* y, int64_t n, double* out, hipStream_t s) {
    reduce(c, x, y, n, 1, 1.0, out, s);
}

// ---- energy assembly --------------------------------------------------------
// phi_i = KE (phi_real + phi_rec + self_i + background), F_i = KE (F_real + F_rec)
// part: 3 partial sums per block of q_i * (real, rec, self+bg) potentials.
template <class T>
__global__ __launch_bounds__(VB) void k_combine(int64_t n, const double* __restrict__ q, const double* __restrict__ Q,
                                                const T* __restrict__ pr, const V4<T>* __restrict__ fr,
                                                const T* __restrict__ pk, const V4<T>* __restrict__ fk,
                                                double cself, double cbg, double* __restrict__ phi,
                                                double* __restrict__ force, double* __restrict__ part) {
    __shared__ double red[VB / 64];
    const double Qs = *Q;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const double qi = q[i];
        const double a = KE * (double)pr[i];
        const double b = KE * (double)pk[i];
        const double sb = KE * (cself * qi + cbg * Qs);
        if (phi) phi[i] = (a + b) + sb;
        if (force) {
            const V4<T> x = fr[i], y = fk[i];
            force[3 * i + 0] = KE * ((double)x.x + (double)y.x);
            force[3 * i + 1] = KE * ((double)x.y + (double)y.y);
            force[3 * i + 2] = KE * ((double)x.z + (double)y.z);
        }
        e0 += qi * a;
        e1 += qi * b;
        e2 += qi * sb;
    }
    e0 = block_sum<VB>(e0, red);
    e1 = block_sum<VB>(e1, red);
    e2 = block_sum<VB>(e2, red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = e0;
        part[3 * blockIdx.x + 1] = e1;
        part[3 * blockIdx.x + 2] = e2;
    }
}

// energy = {total, real, rec, self+bg}; rec from the spectral sum (erec, no KE)
__global__ void k_energy_final(const double* __restrict__ part, int nb, const double* __restrict__ erec,
                               double* __restrict__ energy) {
    __shared__ double red[VB / 64];
    double v[3];
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int i = threadIdx.x; i < nb; i += VB) t += part[3 * i + k];
        v[k] = block_sum<VB>(t, red);
    }
    if (threadIdx.x == 0) {
        const double er = 0.5 * v[0], ek = KE * (*erec), es = 0.5 * v[2];
        energy[0] = er + ek + es;
        energy[1] = er;
        energy[2] = ek;
        energy[3] = es;
    }
}

void combine(Ctx& c, const double* q, double* phi, double* force, double* energy, hipStream_t s) {
    const int64_t n = c.n;
    const int nb = red_blocks(n);
    PQ_REQUIRE(c.ews.part_n >= (size_t)(3 * nb + 16), PQ_ERR_STATE, "energy partials not sized");
    const double a = c.prm.alpha;
    const double V = c.prm.box[0] * c.prm.box[1] * c.prm.box[2];
    const double cself = -2.0 * a / std::sqrt(PI);
    const double cbg = -PI / (V * a * a);
    if (c.fp64)
        PQ_LAUNCH(k_combine<double>, nb, VB, 0, s, n, q, c.ews.scal + 0, as<double>(c.phi_r), as<double4>(c.f_r),
                  as<double>(c.phi_k), as<double4>(c.f_k), cself, cbg, phi, force, c.ews.part);
    else
        PQ_LAUNCH(k_combine<float>, nb, VB, 0, s, n, q, c.ews.scal + 0, as<float>(c.phi_r), as<float4>(c.f_r),
                  as<float>(c.phi_k),
                  as<float4>(c.f_k), cself, cbg, phi, force, c.ews.part);
    if (energy) PQ_LAUNCH(k_energy_final, 1, VB, 0, s, c.ews.part, nb, c.ews.scal + 1, energy);
}

template <class T>
__global__ void k_combine_force(int64_t n, const V4<T>* __restrict__ fr, const V4<T>* __restrict__ fk,
                                double* __restrict__ force) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const V4<T> x = fr[i], y = fk[i];
        force[3 * i + 0] = KE * ((double)x.x + (double)y.x);
        force[3 * i + 1] = KE * ((double)x.y + (double)y.y);
        force[3 * i + 2] = KE * ((double)x.z + (double)y.z);
    }
}
void combine_force(Ctx& c, double* force, hipStream_t s) {
    const int64_t n = c.n;
    const unsigned g = std::min<int64_t>(cdiv(n, VB), 4096);
    if (c.fp64)
        PQ_LAUNCH(k_combine_force<double>, g, VB, 0, s, n, as<double4>(c.f_r), as<double4>(c.f_k), force);
    else
        PQ_LAUNCH(k_combine_force<float>, g, VB, 0, s, n, as<float4>(c.f_r), as<float4>(c.f_k), force);
}

// ---- elementwise kernels ----------------------------------------------------
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        z[i] = a * x[i] + (y ? b * y[i] : 0.0);
}
void axpby(int64_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s) {
    PQ_LAUNCH(k_axpby, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, a, x, b, y, z);
}

__global__ void k_div(int64_t n, const double* __restrict__ x, const double* __restrict__ u, double* __restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) z[i] = x[i] / u[i];
}
void vdiv(int64_t n, const double* x, const double* u, double* z, hipStream_t s) {
    PQ_LAUNCH(k_div, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, x, u, z);
}

__global__ void k_mul(int64_t n, const double* __restrict__ x, const double* __restrict__ u, double sc,
                      double* __restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) z[i] = sc * x[i] * u[i];
}
void vmul(int64_t n, const double* x, const double* u, double sc, double* z, hipStream_t s) {
    PQ_LAUNCH(k_mul, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, x, u, sc, z);
}

// bordered product (right-preconditioned): out_q = y_q + phi + y_l, out_l = t_sum
__global__ void k_bordered_out(int64_t n, const double* __restrict__ y, const double* __restrict__ phi,
                               const double* __restrict__ tsum, double* __restrict__ out) {
    const double yl = y[n];
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        out[i] = y[i] + phi[i] + yl;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *tsum;
}
void bordered_out(int64_t n, const double* y, const double* phi, const double* tsum, double* out, hipStream_t s) {
    PQ_LAUNCH(k_bordered_out, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, y, phi, tsum, out);
}

// shadow Jacobian product: out = -x - (t - dinv * c),  t = phi/u, c = sum(t)/sum(1/u)
__global__ void k_jac_out(int64_t n, const double* __restrict__ x, const double* __restrict__ t,
                          const double* __restrict__ u, const double* __restrict__ sums, double* __restrict__ out) {
    const double c = sums[0] / sums[1];
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        out[i] = -x[i] - (t[i] - c / u[i]);
}
void jac_out(int64_t n, const double* x, const double* t, const double* u, const double* sums, double* out,
             hipStream_t s) {
    PQ_LAUNCH(k_jac_out, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, x, t, u, sums, out);
}

// shadow charges: lambda = -(Qtot + sum (chi+v)/u) / sum(1/u);  q = -(chi + v + lambda)/u
__global__ void k_shadow_q(int64_t n, const double* __restrict__ chi, const double* __restrict__ v,
                           const double* __restrict__ u, const double* __restrict__ sums, double qtot,
                           double* __restrict__ q, double* __restrict__ lam_out) {
    const double lam = -(qtot + sums[0]) / sums[1];
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        q[i] = -(chi[i] + v[i] + lam) / u[i];
    if (blockIdx.x == 0 && threadIdx.x == 0 && lam_out) *lam_out = lam;
}
void shadow_q(int64_t n, const double* chi, const double* v, const double* u, const double* sums, double qtot,
              double* q, double* lam, hipStream_t s) {
    PQ_LAUNCH(k_shadow_q, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, chi, v, u, sums, qtot, q, lam);
}

// (chi + v)/u and 1/u summed in one pass: part[0..nb) and part[nb..2nb)
__global__ __launch_bounds__(VB) void k_part_shadow(int64_t n, const double* __restrict__ chi,
                                                    const double* __restrict__ v, const double* __restrict__ u,
                                                    double* __restrict__ part) {
    __shared__ double red[VB / 64];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const double iu = 1.0 / u[i];
        a += ((chi ? chi[i] : 0.0) + v[i]) * iu;
        b += iu;
    }
    a = block_sum<VB>(a, red);
    b = block_sum<VB>(b, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
    }
}
void shadow_sums(Ctx& c, int64_t n, const double* chi, const double* v, const double* u, double* out2,
                 hipStream_t s) {
    const int nb = red_blocks(n);
    c.part.ensure(2 * nb + 16);
    PQ_LAUNCH(k_part_shadow, nb, VB, 0, s, n, chi, v, u, c.part.p);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, c.part.p, nb, 2, 1.0, out2, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
}

// ---- Gram-Schmidt -----------------------------------------------------------
// part[k*nb + b] = partial of V_k . w, nk = *jdev + 1 basis vectors with jdev.
// Grid (nb, ceil(nk_max / MD_K)): workgroup (b, c) takes MD_K dot products of
// chunk c over the b-th slice of the rows (the same slices and the same tree
// for every dot product), so long bases keep the whole device busy.
__global__ __launch_bounds__(VB) void k_mdot(int64_t n, const double* __restrict__ V, size_t ld, int nk,
                                             const int* __restrict__ jdev, const double* __restrict__ w,
                                             double* __restrict__ part) {
    __shared__ double red[(VB / 64) * MD_K];
    if (jdev) nk = *jdev + 1;
    const int k0 = blockIdx.y * MD_K;
    if (k0 >= nk) return;
    double v[MD_K];
#pragma unroll
    for (int k = 0; k < MD_K; ++k) v[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const double wi = w[i];
#pragma unroll
        for (int k = 0; k < MD_K; ++k)
            if (k0 + k < nk) v[k] += V[(size_t)(k0 + k) * ld + i] * wi;
    }
    block_sum_n<MD_K>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < MD_K; ++k)
            if (k0 + k < nk) part[(size_t)(k0 + k) * gridDim.x + blockIdx.x] = v[k];
    }
}
// The final sums of k_mdot's partials, one workgroup per chunk of MD_K:
// out[k] = sum of part[k*nb .. k*nb+nb-1] (with jdev: nk = *jdev + 1 and out
// advanced by *jdev * ostride); with acc also acc[k] += out[k].
__global__ __launch_bounds__(VB) void k_mdot_final(const double* __restrict__ part, int nb, int nk,
                                                   double* __restrict__ out, const int* __restrict__ jdev,
                                                   size_t ostride, double* __restrict__ acc, size_t astride) {
    __shared__ double red[(VB / 64) * MD_K];
    if (jdev) {
        nk = *jdev + 1;
        out += (size_t)(*jdev) * ostride;
        if (acc) acc += (size_t)(*jdev) * astride;
    }
    const int k0 = blockIdx.x * MD_K;
    if (k0 >= nk) return;
    double v[MD_K];
#pragma unroll
    for (int k = 0; k < MD_K; ++k) {
        v[k] = 0.0;
        if (k0 + k < nk)
            for (int i = threadIdx.x; i < nb; i += VB) v[k] += part[(size_t)(k0 + k) * nb + i];
    }
    block_sum_n<MD_K>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < MD_K; ++k) {
            if (k0 + k >= nk) break;
            out[k0 + k] = v[k];
            if (acc) acc[k0 + k] = acc[k0 + k] + v[k];
        }
    }
}
// w -= sum_k h[k] V_k, k < nk (with jdev: nk = *jdev + 1, h advanced by
// *jdev * hstride); one pass for bases of at most KU vectors
__global__ void k_mupdate(int64_t n, const double* __restrict__ V, size_t ld, int nk, const int* __restrict__ jdev,
                          size_t hstride, const double* __restrict__ h, double* __restrict__ w) {
    if (jdev) {
        nk = *jdev + 1;
        h += (size_t)(*jdev) * hstride;
    }
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        double acc = w[i];
        for (int k = 0; k < nk; ++k) acc -= h[k] * V[(size_t)k * ld + i];
        w[i] = acc;
    }
}
// Longer bases in two passes: grid (rows, chunks of KU vectors) writes
// up[c*ld + i] = sum over chunk c of h[k] V_k[i]; then every row adds its
// chunk sums in chunk order: w += sign * sum_c up[c*ld + i].
constexpr int KU = 32;
__global__ void k_vcomb_part(int64_t n, const double* __restrict__ V, size_t ld, int nk, const int* __restrict__ jdev,
                             size_t hstride, const double* __restrict__ h, double* __restrict__ up) {
    if (jdev) {
        nk = *jdev + 1;
        h += (size_t)(*jdev) * hstride;
    }
    const int k0 = blockIdx.y * KU;
    if (k0 >= nk) return;
    const int k1 = min(nk, k0 + KU);
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        double acc = 0.0;
        for (int k = k0; k < k1; ++k) acc += h[k] * V[(size_t)k * ld + i];
        up[(size_t)blockIdx.y * ld + i] = acc;
    }
}
__global__ void k_vcomb_apply(int64_t n, int nk, const int* __restrict__ jdev, const double* __restrict__ up, size_t ld,
                              double sign, double* __restrict__ w) {
    if (jdev) nk = *jdev + 1;
    const int nc = (nk + KU - 1) / KU;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        double t = 0.0;
        for (int c = 0; c < nc; ++c) t += up[(size_t)c * ld + i];
        w[i] = w[i] + sign * t;
    }
}
size_t vcomb_chunks(int nk) { return (size_t)((nk + KU - 1) / KU); }

// w += sign * sum_{k < nk} h[k] V_k (nk_max bounds the device count with jdev)
static void vcomb(int64_t n, const double* V, size_t ld, int nk_max, const int* jdev, size_t hstride, const double* h,
                  double sign, double* up, double* w, hipStream_t s) {
    const unsigned g = std::min<int64_t>(cdiv(n, VB), 4096);
    const unsigned nc = (unsigned)vcomb_chunks(nk_max);
    PQ_LAUNCH(k_vcomb_part, dim3(g, nc), VB, 0, s, n, V, ld, nk_max, jdev, hstride, h, up);
    PQ_LAUNCH(k_vcomb_apply, g, VB, 0, s, n, nk_max, jdev, (const double*)up, ld, sign, w);
}

// CGS2 of w against V_0..V_{nk-1} (nk = *jdev + 1, at most m + 1); the
// coefficients of step *jdev go to column *jdev of H (stride m + 1), the
// re-orthogonalisation's into tmp2 and added to the column; up: chunk sums
// (vcomb_chunks(m + 1) x ld) when m + 1 > KU.
void orthogonalize_j(Ctx& c, int64_t n, const double* V, size_t ld, int m, const int* jdev, double* w, double* st,
                     double* tmp2, double* up, hipStream_t s) {
    const int nk = m + 1;
    const size_t hstride = (size_t)(m + 1);
    const int nb = red_blocks(n);
    const unsigned kc = cdiv(nk, MD_K);
    c.part.ensure((size_t)(nk + 1) * nb + 16);
    const unsigned g = std::min<int64_t>(cdiv(n, VB), 4096);
    auto mdot = [&](double* dst, size_t ostride, double* acc, size_t astride) {
        PQ_LAUNCH(k_mdot, dim3(nb, kc), VB, 0, s, n, V, ld, nk, jdev, w, c.part.p);
        PQ_LAUNCH(k_mdot_final, kc, VB, 0, s, (const double*)c.part.p, nb, nk, dst, jdev, ostride, acc, astride);
    };
    auto update = [&](size_t hs, const double* h) {
        if (nk <= KU)
            PQ_LAUNCH(k_mupdate, g, VB, 0, s, n, V, ld, nk, jdev, hs, h, w);
        else
            vcomb(n, V, ld, nk, jdev, hs, h, -1.0, up, w, s);
    };
    // pass 1
    mdot(st, hstride, (double*)nullptr, (size_t)0);
    update(hstride, st);
    // pass 2 (re-orthogonalisation); its coefficients are also added to the column
    mdot(tmp2, (size_t)0, st, hstride);
    update((size_t)0, tmp2);
}

// V_{j+1} = w / h, h = sqrt(nrm2) stored into H(j+1, j); zero vector if h == 0
__global__ void k_normalize(int64_t n, const double* __restrict__ w, const double* __restrict__ nrm2,
                            double* __restrict__ hsub, double* __restrict__ out) {
    const double h = sqrt(fmax(*nrm2, 0.0));
    const double inv = h > 0.0 ? 1.0 / h : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) out[i] = w[i] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0 && hsub) *hsub = h;
}
void normalize(int64_t n, const double* w, const double* nrm2, double* hsub, double* out, hipStream_t s) {
    PQ_LAUNCH(k_normalize, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, w, nrm2, hsub, out);
}

// ---- small dense GMRES state ---------------------------------------------------
// Layout of st (m = restart length): H (m+1) x m column-major at 0,
// g[m+1] at GS_G, cs[m] at GS_C, sn[m] at GS_S, y[m] at GS_Y, scalars at GS_X.
// start of a cycle: g = (beta, 0, ...), beta = sqrt(nrm2)
__global__ void k_gmres_start(double* __restrict__ st, int m, const double* __restrict__ nrm2) {
    if (threadIdx.x != 0) return;
    double* g = st + gs_g(m);
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = sqrt(fmax(*nrm2, 0.0));
}
void gmres_start(double* st, int m, const double* nrm2, hipStream_t s) { PQ_LAUNCH(k_gmres_start, 1, 64, 0, s, st, m, nrm2); }

// y = R^-1 g for the first k columns, column by column: y_i = t_i / R_ii,
// then t_r -= R_ri y_i for every r < i at once (column i of H is contiguous)
constexpr int BS_T = 1024;
__global__ __launch_bounds__(BS_T) void k_backsolve(double* __restrict__ st, int m, int k) {
    extern __shared__ double t[];
    __shared__ double yi;
    const double* H = st;
    const double* g = st + gs_g(m);
    double* y = st + gs_y(m);
    for (int r = threadIdx.x; r < k; r += BS_T) t[r] = g[r];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double* col = H + (size_t)i * (m + 1);
        if (threadIdx.x == 0) {
            const double d = col[i];
            yi = d != 0.0 ? t[i] / d : 0.0;
            y[i] = yi;
        }
        __syncthreads();
        const double v = yi;
        for (int r = threadIdx.x; r < i; r += BS_T) t[r] -= col[r] * v;
        __syncthreads();
    }
}
void backsolve(double* st, int m, int k, hipStream_t s) {
    if (k > 0) PQ_LAUNCH(k_backsolve, 1, BS_T, (size_t)k * sizeof(double), s, st, m, k);
}

// x += sum_k y[k] V_k
__global__ void k_xupdate(int64_t n, const double* __restrict__ V, size_t ld, int nk, const double* __restrict__ y,
                          double* __restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        double acc = x[i];
        for (int k = 0; k < nk; ++k) acc += y[k] * V[(size_t)k * ld + i];
        x[i] = acc;
    }
}
void xupdate(int64_t n, const double* V, size_t ld, int nk, const double* y, double* x, double* up, hipStream_t s) {
    if (nk <= KU)
        PQ_LAUNCH(k_xupdate, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, V, ld, nk, y, x);
    else
        vcomb(n, V, ld, nk, (const int*)nullptr, (size_t)0, y, 1.0, up, x, s);
}

// QEQ energy: E = sum q chi + 1/2 sum u q^2 + 1/2 sum q phi  (shadow: 1/2 sum (2q - n) phi_n)
__global__ __launch_bounds__(VB) void k_part_energy(int64_t n, const double* __restrict__ q,
                                                    const double* __restrict__ chi, const double* __restrict__ u,
                                                    const double* __restrict__ a, const double* __restrict__ phi,
                                                    double* __restrict__ part) {
    __shared__ double red[VB / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        const double qi = q[i];
        v += qi * chi[i] + 0.5 * u[i] * qi * qi + 0.5 * a[i] * phi[i];
    }
    v = block_sum<VB>(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}
void qeq_energy(Ctx& c, int64_t n, const double* q, const double* chi, const double* u, const double* a,
                const double* phi, double* out, hipStream_t s) {
    const int nb = red_blocks(n);
    c.part.ensure(nb + 16);
    PQ_LAUNCH(k_part_energy, nb, VB, 0, s, n, q, chi, u, a, phi, c.part.p);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, c.part.p, nb, 1, 1.0, out, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
}

// ---- device-indexed steps (graph-captured Arnoldi iterations) --------------
// out = V_{*jdev}
__global__ void k_copy_j(int64_t n, const double* __restrict__ V, size_t ld, const int* __restrict__ jdev,
                         double* __restrict__ out) {
    const double* v = V + (size_t)(*jdev) * ld;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) out[i] = v[i];
}
void copy_j(int64_t n, const double* V, size_t ld, const int* jdev, double* out, hipStream_t s) {
    PQ_LAUNCH(k_copy_j, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, V, ld, jdev, out);
}
// V_{j+1} = w / h and H(j+1, j) = h = sqrt(nrm2), j = *jdev
__global__ void k_normalize_j(int64_t n, const double* __restrict__ w, const double* __restrict__ nrm2,
                              double* __restrict__ st, int m, double* __restrict__ V, size_t ld,
                              const int* __restrict__ jdev) {
    const int j = *jdev;
    const double h = sqrt(fmax(*nrm2, 0.0));
    const double inv = h > 0.0 ? 1.0 / h : 0.0;
    double* out = V + (size_t)(j + 1) * ld;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) out[i] = w[i] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) st[(size_t)j * (m + 1) + j + 1] = h;
}
void normalize_j(int64_t n, const double* w, const double* nrm2, double* st, int m, double* V, size_t ld,
                 const int* jdev, hipStream_t s) {
    PQ_LAUNCH(k_normalize_j, std::min<int64_t>(cdiv(n, VB), 4096), VB, 0, s, n, w, nrm2, st, m, V, ld, jdev);
}
// Givens update of column j = *jdev; |g[j+1]| into hist[j]; then *jdev = j + 1.
// The earlier rotations apply in sequence (each one mixes the rows the next
// one reads); the column and the rotations are staged in LDS first, so the
// sequential part runs from LDS. Bases too long for LDS read them in place.
constexpr int GV_T = 256;
__device__ __forceinline__ void givens_tail(double* __restrict__ col, double* __restrict__ g, double* __restrict__ cs,
                                            double* __restrict__ sn, int j, double* __restrict__ hist) {
    const double a = col[j], b = col[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
    cs[j] = c;
    sn[j] = s;
    col[j] = r;
    col[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    hist[j] = fabs(g[j + 1]);
}
__global__ __launch_bounds__(GV_T) void k_givens_j(double* __restrict__ st, int m, int* __restrict__ jdev,
                                                   double* __restrict__ hist, int staged) {
    extern __shared__ double sh[];
    const int j = *jdev;
    double* g = st + gs_g(m);
    double* cs = st + gs_c(m);
    double* sn = st + gs_s(m);
    double* col = st + (size_t)j * (m + 1);
    if (!staged) {
        if (threadIdx.x == 0) {
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            givens_tail(col, g, cs, sn, j, hist);
            *jdev = j + 1;
        }
        return;
    }
    double* lc = sh;              // rows 0..j+1 of the column
    double* lcs = sh + (m + 1);   // cs[0..j-1]
    double* lsn = lcs + m;        // sn[0..j-1]
    for (int i = threadIdx.x; i <= j + 1; i += GV_T) lc[i] = col[i];
    for (int i = threadIdx.x; i < j; i += GV_T) {
        lcs[i] = cs[i];
        lsn[i] = sn[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < j; ++i) {
            const double t = lcs[i] * lc[i] + lsn[i] * lc[i + 1];
            lc[i + 1] = -lsn[i] * lc[i] + lcs[i] * lc[i + 1];
            lc[i] = t;
        }
        givens_tail(lc, g, cs, sn, j, hist);
        *jdev = j + 1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += GV_T) col[i] = lc[i];
}
void givens_j(double* st, int m, int* jdev, double* hist, hipStream_t s) {
    const size_t lds = (size_t)(3 * m + 1) * sizeof(double);
    const int staged = lds <= 65536 ? 1 : 0;
    PQ_LAUNCH(k_givens_j, 1, GV_T, staged ? lds : 0, s, st, m, jdev, hist, staged);
}
__global__ void k_set_int(int* __restrict__ p, int v) {
    if (threadIdx.x == 0) *p = v;
}
void set_int(int* p, int v, hipStream_t s) { PQ_LAUNCH(k_set_int, 1, 64, 0, s, p, v); }

__global__ void k_copy_scalar(const double* __restrict__ a, double* __restrict__ b) {
    if (threadIdx.x == 0) *b = *a;
}
void copy_scalar(const double* a, double* b, hipStream_t s) { PQ_LAUNCH(k_copy_scalar, 1, 64, 0, s, a, b); }

__global__ void k_set_scalar(double* __restrict__ b, double v) {
    if (threadIdx.x == 0) *b = v;
}
void set_scalar(double* b, double v, hipStream_t s) { PQ_LAUNCH(k_set_scalar, 1, 64, 0, s, b, v); }

// ---- preconditioned MINRES (Paige and Saunders) -------------------------------
// For the symmetric bordered system M z = b with the SPD preconditioner
// D = diag(u, 1): a Lanczos recurrence in the D^-1 inner product, the QR
// factorisation of its tridiagonal matrix by Givens rotations, and the
// solution update by the three-term direction recurrence. The scalars live in
// ms[MR_*] on the device, so a whole step (product included) is recordable
// into a graph. nv = n + 1; d_i = u_i for i < n, d_n = 1.
__device__ __forceinline__ double mr_d(const double* __restrict__ u, int64_t n, int64_t i) { return i < n ? u[i] : 1.0; }

// y = r / d, partials of r . y (start of a cycle: beta1^2)
__global__ __launch_bounds__(VB) void k_mr_prec(int64_t n, const double* __restrict__ r, const double* __restrict__ u,
                                                double* __restrict__ y, double* __restrict__ part) {
    __shared__ double red[VB / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i <= n; i += (int64_t)gridDim.x * VB) {
        const double t = r[i] / mr_d(u, n, i);
        y[i] = t;
        v += r[i] * t;
    }
    v = block_sum<VB>(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void k_mr_init(double* __restrict__ ms) {
    if (threadIdx.x != 0) return;
    const double b = sqrt(fmax(ms[MR_BETA2], 0.0));
    ms[MR_BETA] = b;
    ms[MR_BETA1] = b;
    ms[MR_OLDB] = 0.0;
    ms[MR_DBAR] = 0.0;
    ms[MR_EPS] = 0.0;
    ms[MR_PHIBAR] = b;
    ms[MR_CS] = -1.0;
    ms[MR_SN] = 0.0;
    ms[MR_PHI] = 0.0;
    ms[MR_DELTA] = 0.0;
    ms[MR_OLDEPS] = 0.0;
    ms[MR_DENOM] = 0.0;
}

// v = y / beta
__global__ void k_mr_v(int64_t nv, const double* __restrict__ y, const double* __restrict__ ms, double* __restrict__ v) {
    const double b = ms[MR_BETA];
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < nv; i += (int64_t)gridDim.x * VB) v[i] = y[i] * inv;
}

// y -= (beta / oldb) r1 (no term at the first step, oldb = 0); partials of v . y
__global__ __launch_bounds__(VB) void k_mr_a(int64_t nv, double* __restrict__ y, const double* __restrict__ r1,
                                             const double* __restrict__ v, const double* __restrict__ ms,
                                             double* __restrict__ part) {
    __shared__ double red[VB / 64];
    const double ob = ms[MR_OLDB];
    const double c1 = ob > 0.0 ? ms[MR_BETA] / ob : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < nv; i += (int64_t)gridDim.x * VB) {
        const double t = y[i] - c1 * r1[i];
        y[i] = t;
        acc += v[i] * t;
    }
    acc = block_sum<VB>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// t = y - (alfa / beta) r2; r1 = r2; r2 = t; y = t / d; partials of t . y
__global__ __launch_bounds__(VB) void k_mr_b(int64_t n, double* __restrict__ y, double* __restrict__ r1,
                                             double* __restrict__ r2, const double* __restrict__ u,
                                             const double* __restrict__ ms, double* __restrict__ part) {
    __shared__ double red[VB / 64];
    const double b = ms[MR_BETA];
    const double c2 = b > 0.0 ? ms[MR_ALFA] / b : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i <= n; i += (int64_t)gridDim.x * VB) {
        const double t = y[i] - c2 * r2[i];
        r1[i] = r2[i];
        r2[i] = t;
        const double z = t / mr_d(u, n, i);
        y[i] = z;
        acc += t * z;
    }
    acc = block_sum<VB>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Givens step on the tridiagonal column (alfa, beta) and the residual
// estimate phibar (the D^-1 norm of the residual)
__global__ void k_mr_givens(double* __restrict__ ms) {
    if (threadIdx.x != 0) return;
    const double alfa = ms[MR_ALFA];
    const double oldb = ms[MR_BETA];
    const double beta = sqrt(fmax(ms[MR_BETA2], 0.0));
    const double cs = ms[MR_CS], sn = ms[MR_SN], dbar = ms[MR_DBAR];
    const double oldeps = ms[MR_EPS];
    const double delta = cs * dbar + sn * alfa;
    const double gbar = sn * dbar - cs * alfa;
    const double eps = sn * beta;
    const double dbar2 = -cs * beta;
    const double gamma = fmax(hypot(gbar, beta), 1e-300);
    const double c = gbar / gamma, s = beta / gamma;
    const double phibar = ms[MR_PHIBAR];
    ms[MR_OLDB] = oldb;
    ms[MR_BETA] = beta;
    ms[MR_OLDEPS] = oldeps;
    ms[MR_DELTA] = delta;
    ms[MR_EPS] = eps;
    ms[MR_DBAR] = dbar2;
    ms[MR_CS] = c;
    ms[MR_SN] = s;
    ms[MR_PHI] = c * phibar;
    ms[MR_PHIBAR] = s * phibar;
    ms[MR_DENOM] = 1.0 / gamma;
}

// wn = (v - oldeps wb - delta wa) / gamma; wb = wa; wa = wn; x += phi wn
__global__ void k_mr_x(int64_t nv, const double* __restrict__ v, double* __restrict__ wa, double* __restrict__ wb,
                       double* __restrict__ x, const double* __restrict__ ms) {
    const double oe = ms[MR_OLDEPS], de = ms[MR_DELTA], dn = ms[MR_DENOM], ph = ms[MR_PHI];
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < nv; i += (int64_t)gridDim.x * VB) {
        const double a = wa[i];
        const double wn = (v[i] - oe * wb[i] - de * a) * dn;
        wb[i] = a;
        wa[i] = wn;
        x[i] = x[i] + ph * wn;
    }
}

static unsigned vgrid(int64_t nv) { return (unsigned)std::min<int64_t>(cdiv(nv, VB), 4096); }

void minres_start(Ctx& c, int64_t n, const double* r, const double* u, double* y, double* ms, hipStream_t s) {
    const int nb = red_blocks(n + 1);
    c.part.ensure(nb + 16);
    PQ_LAUNCH(k_mr_prec, nb, VB, 0, s, n, r, u, y, c.part.p);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, c.part.p, nb, 1, 1.0, ms + MR_BETA2, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
    PQ_LAUNCH(k_mr_init, 1, 64, 0, s, ms);
}
void minres_v(int64_t nv, const double* y, const double* ms, double* v, hipStream_t s) {
    PQ_LAUNCH(k_mr_v, vgrid(nv), VB, 0, s, nv, y, ms, v);
}
void minres_update(Ctx& c, int64_t n, double* y, double* r1, double* r2, const double* v, const double* u, double* wa,
                   double* wb, double* x, double* ms, hipStream_t s) {
    const int64_t nv = n + 1;
    const int nb = red_blocks(nv);
    c.part.ensure(nb + 16);
    PQ_LAUNCH(k_mr_a, nb, VB, 0, s, nv, y, r1, v, ms, c.part.p);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, c.part.p, nb, 1, 1.0, ms + MR_ALFA, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
    PQ_LAUNCH(k_mr_b, nb, VB, 0, s, n, y, r1, r2, u, ms, c.part.p);
    PQ_LAUNCH(k_part_final, 1, VB, 0, s, c.part.p, nb, 1, 1.0, ms + MR_BETA2, (const int*)nullptr, (size_t)0,
              (double*)nullptr, (size_t)0);
    PQ_LAUNCH(k_mr_givens, 1, 64, 0, s, ms);
    PQ_LAUNCH(k_mr_x, vgrid(nv), VB, 0, s, nv, v, wa, wb, x, ms);
}

// unpreconditioned bordered product: out = [u o v + phi + v_n ; *vsum]
__global__ void k_bordered_plain(int64_t n, const double* __restrict__ v, const double* __restrict__ u,
                                 const double* __restrict__ phi, const double* __restrict__ vsum,
                                 double* __restrict__ out) {
    const double vl = v[n];
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        out[i] = u[i] * v[i] + phi[i] + vl;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *vsum;
}
void bordered_plain(int64_t n, const double* v, const double* u, const double* phi, const double* vsum, double* out,
                    hipStream_t s) {
    PQ_LAUNCH(k_bordered_plain, vgrid(n), VB, 0, s, n, v, u, phi, vsum, out);
}

}  // namespace pq
