// Direct reciprocal Ewald sum (the paper's eq. ewald_rec and its derivatives),
// computed blockwise without materialising the N x k phase matrix, as the
// paper's blockwise variant does.
//
// Half space of k = 2 pi n / L (n != 0, |n_d| <= kmax_d, first nonzero
// component positive); the other half follows from S(-k) = conj S(k).
//   S(k)  = sum_j q_j exp(i k.r_j)                       (FP64 sums of FP32 phases)
//   E_rec = sum_half c_k |S(k)|^2,  c_k = (4 pi/V) exp(-k^2/4a^2)/k^2
//   phi_i = 2 sum_half c_k Re(exp(-i k.r_i) S(k))
//   F_i   = 2 q_i sum_half c_k k Im(conj(S(k)) exp(i k.r_i))
// Phases: k.r = 2 pi (n . s), s = r/L; the fractional part of n . s is taken
// in FP64, then sin/cos of 2 pi f in the bulk precision T (FP32: phase error
// ~2e-7 rad; FP64).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "dev.h"
#include "pq_internal.h"

namespace pq {

constexpr int EW_TILE = 256;
constexpr int EW_BLOCKS = 2048;   // target workgroups per direct-Ewald sum

__device__ __forceinline__ void phase(const int4 nk, double s0, double s1, double s2, float& sn, float& cs) {
    double t = (double)nk.x * s0 + (double)nk.y * s1 + (double)nk.z * s2;
    t -= rint(t);
    sincospif(2.0f * (float)t, &sn, &cs);
}
__device__ __forceinline__ void phase(const int4 nk, double s0, double s1, double s2, double& sn, double& cs) {
    double t = (double)nk.x * s0 + (double)nk.y * s1 + (double)nk.z * s2;
    t -= rint(t);
    sincospi(2.0 * t, &sn, &cs);
}

// Both sums run over a second grid dimension so that small systems still
// fill the device: the structure factors over chunks of atoms, the
// potentials and forces over chunks of k vectors; the chunk partials are then
// added in chunk order (deterministic, independent of the launch).

// Fractional coordinates s = r H^-1 of a wrapped position (orthorhombic:
// s_d = r_d / L_d), and the rows of R = H^-1 that turn the fractional
// gradient into the Cartesian force.
struct EwFrac {
    double inv[3];
    int tric;
    Tric t;
    double r10, r20, r21;
};
__device__ __forceinline__ void ew_frac(const double* __restrict__ w, const EwFrac& f, double& s0, double& s1,
                                        double& s2) {
    if (f.tric) {
        frac_tric(w[0], w[1], w[2], f.inv, f.t, s0, s1, s2);
    } else {
        s0 = w[0] * f.inv[0];
        s1 = w[1] * f.inv[1];
        s2 = w[2] * f.inv[2];
    }
}

// Structure-factor partials: one thread per k vector, blockIdx.y = atom chunk
// [y cs, (y+1) cs), atoms staged through LDS.
template <class T>
__global__ __launch_bounds__(EW_TILE) void k_sfac(int n, int nk, int cs, const int4* __restrict__ kn,
                                                 const double* __restrict__ w64, EwFrac fr,
                                                 const double* __restrict__ q, double2* __restrict__ spart) {
    __shared__ double s_s[EW_TILE * 3];
    __shared__ double s_q[EW_TILE];
    const int kidx = blockIdx.x * EW_TILE + threadIdx.x;
    const bool valid = kidx < nk;
    const int4 nv = valid ? kn[kidx] : make_int4(0, 0, 0, 0);
    const int jb = blockIdx.y * cs, je = min(n, jb + cs);
    double re = 0.0, im = 0.0;
    for (int j0 = jb; j0 < je; j0 += EW_TILE) {
        const int j = j0 + threadIdx.x;
        if (j < je) {
            ew_frac(w64 + 3 * (size_t)j, fr, s_s[3 * threadIdx.x + 0], s_s[3 * threadIdx.x + 1],
                    s_s[3 * threadIdx.x + 2]);
            s_q[threadIdx.x] = q[j];
        }
        __syncthreads();
        const int m = min(EW_TILE, je - j0);
        if (valid)
            for (int t = 0; t < m; ++t) {
                T sn, cs_;
                phase(nv, s_s[3 * t], s_s[3 * t + 1], s_s[3 * t + 2], sn, cs_);
                re += s_q[t] * (double)cs_;
                im += s_q[t] * (double)sn;
            }
        __syncthreads();
    }
    if (valid) spart[(size_t)blockIdx.y * nk + kidx] = make_double2(re, im);
}

// S(k) = sum of the chunk partials in chunk order; energy partial per block.
__global__ __launch_bounds__(EW_TILE) void k_sfac_sum(int nk, int nch, const double* __restrict__ kc,
                                                     const double2* __restrict__ spart,
                                                     double2* __restrict__ sfac, double* __restrict__ epart) {
    __shared__ double red[EW_TILE / 64];
    const int kidx = blockIdx.x * EW_TILE + threadIdx.x;
    double e = 0.0;
    if (kidx < nk) {
        double re = 0.0, im = 0.0;
        for (int c = 0; c < nch; ++c) {
            const double2 v = spart[(size_t)c * nk + kidx];
            re += v.x;
            im += v.y;
        }
        sfac[kidx] = make_double2(re, im);
        e = kc[kidx] * (re * re + im * im);
    }
    e = block_sum<EW_TILE>(e, red);
    if (threadIdx.x == 0) epart[blockIdx.x] = e;
}

// Potential / force partials: one thread per atom, blockIdx.y = k chunk
// [y kcs, (y+1) kcs), k vectors staged through LDS.
template <bool FORCE, class T>
__global__ __launch_bounds__(EW_TILE) void k_kgather(int n, int nk, int kcs, const int4* __restrict__ kn,
                                                    const double* __restrict__ kc,
                                                    const double2* __restrict__ sfac, const double* __restrict__ w64,
                                                    EwFrac fr, double4* __restrict__ gpart) {
    __shared__ int4 s_n[EW_TILE];
    __shared__ double s_c[EW_TILE];
    __shared__ double2 s_S[EW_TILE];
    const int i = blockIdx.x * EW_TILE + threadIdx.x;
    const bool valid = i < n;
    double s0 = 0, s1 = 0, s2 = 0;
    if (valid) ew_frac(w64 + 3 * (size_t)i, fr, s0, s1, s2);
    const int kb = blockIdx.y * kcs, ke = min(nk, kb + kcs);
    double phi = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int k0 = kb; k0 < ke; k0 += EW_TILE) {
        const int k = k0 + threadIdx.x;
        if (k < ke) {
            s_n[threadIdx.x] = kn[k];
            s_c[threadIdx.x] = kc[k];
            s_S[threadIdx.x] = sfac[k];
        }
        __syncthreads();
        const int m = min(EW_TILE, ke - k0);
        if (valid)
            for (int t = 0; t < m; ++t) {
                T sn, cs;
                const int4 nv = s_n[t];
                phase(nv, s0, s1, s2, sn, cs);
                const double2 S = s_S[t];
                const double c = s_c[t];
                phi += c * ((double)cs * S.x + (double)sn * S.y);
                if (FORCE) {
                    const double im = c * (S.x * (double)sn - S.y * (double)cs);
                    g0 += im * nv.x;
                    g1 += im * nv.y;
                    g2 += im * nv.z;
                }
            }
        __syncthreads();
    }
    if (valid) gpart[(size_t)blockIdx.y * n + i] = make_double4(phi, g0, g1, g2);
}

// Per atom: the k-chunk partials in chunk order, then phi and F.
template <bool FORCE, class T>
__global__ __launch_bounds__(EW_TILE) void k_kgather_sum(int n, int nkch, const double4* __restrict__ gpart,
                                                        EwFrac fr, const double* __restrict__ q,
                                                        T* __restrict__ phi_out, V4<T>* __restrict__ f_out) {
    const int i = blockIdx.x * EW_TILE + threadIdx.x;
    if (i >= n) return;
    double phi = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int c = 0; c < nkch; ++c) {
        const double4 v = gpart[(size_t)c * n + i];
        phi += v.x;
        g0 += v.y;
        g1 += v.z;
        g2 += v.w;
    }
    phi_out[i] = (T)(2.0 * phi);
    if (FORCE) {
        const double f = 2.0 * q[i] * 2.0 * PI;
        if (fr.tric)
            f_out[i] = mk4<T>((T)(f * (g0 * fr.inv[0])), (T)(f * (g1 * fr.inv[1] + g0 * fr.r10)),
                              (T)(f * ((g2 * fr.inv[2] + g1 * fr.r21) + g0 * fr.r20)), T(0));
        else
            f_out[i] = mk4<T>((T)(f * g0 * fr.inv[0]), (T)(f * g1 * fr.inv[1]), (T)(f * g2 * fr.inv[2]), T(0));
    }
}

__global__ void k_sum_part_e(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    v = block_sum<256>(v, red);
    if (threadIdx.x == 0) *out = v;
}

void ewald_setup(Ctx& c) {
    const int* km = c.prm.kmax;
    const double V = c.prm.box[0] * c.prm.box[1] * c.prm.box[2];
    const double a = c.prm.alpha;
    std::vector<int4> nv;
    std::vector<double> cv;
    const bool tric = is_tric(c.prm);
    const double L0 = c.prm.box[0], L1 = c.prm.box[1], L2 = c.prm.box[2];
    const double txy = c.prm.tilt[0], txz = c.prm.tilt[1], tyz = c.prm.tilt[2];
    const double r00 = 1.0 / L0, r11 = 1.0 / L1, r22 = 1.0 / L2, r10 = -txy / (L0 * L1),
                 r21 = -tyz / (L1 * L2), r20 = (txy * tyz - L1 * txz) / (L0 * L1 * L2);
    for (int x = 0; x <= km[0]; ++x)
        for (int y = -km[1]; y <= km[1]; ++y)
            for (int z = -km[2]; z <= km[2]; ++z) {
                if (!(x > 0 || (x == 0 && (y > 0 || (y == 0 && z > 0))))) continue;
                double k2;
                if (tric) {
                    // k = 2 pi R n with R = H^-1 lower triangular
                    const double kx = 2.0 * PI * (r00 * x), ky = 2.0 * PI * (r10 * x + r11 * y),
                                 kz = 2.0 * PI * ((r20 * x + r21 * y) + r22 * z);
                    k2 = kx * kx + ky * ky + kz * kz;
                } else {
                    const double kx = 2.0 * PI * x / c.prm.box[0], ky = 2.0 * PI * y / c.prm.box[1],
                                 kz = 2.0 * PI * z / c.prm.box[2];
                    k2 = kx * kx + ky * ky + kz * kz;
                }
                nv.push_back(make_int4(x, y, z, 0));
                cv.push_back(4.0 * PI / V * std::exp(-k2 / (4.0 * a * a)) / k2);
            }
    c.nk = (int)nv.size();
    c.kn.ensure(std::max(1, c.nk));
    c.kc.ensure(std::max(1, c.nk));
    c.sfac.ensure(std::max(1, c.nk));
    // chunking: about EW_BLOCKS workgroups per sum, chunks of at least 32
    const int n = (int)c.n, nk = std::max(1, c.nk);
    const int kblk = (int)cdiv(nk, EW_TILE), ablk = (int)cdiv(std::max(1, n), EW_TILE);
    c.ew_nch = std::max(1, std::min((int)cdiv(std::max(1, n), 32), (int)cdiv(EW_BLOCKS, kblk)));
    c.ew_cs = (int)cdiv(std::max(1, n), c.ew_nch);
    c.ew_nch = (int)cdiv(std::max(1, n), c.ew_cs);
    c.ew_nkch = std::max(1, std::min((int)cdiv(nk, 32), (int)cdiv(EW_BLOCKS, ablk)));
    c.ew_kcs = (int)cdiv(nk, c.ew_nkch);
    c.ew_nkch = (int)cdiv(nk, c.ew_kcs);
    c.spart.ensure((size_t)c.ew_nch * nk);
    c.gpart.ensure((size_t)c.ew_nkch * std::max(1, n));
    if (c.nk) {
        PQ_HIP(hipMemcpy(c.kn.p, nv.data(), nv.size() * sizeof(int4), hipMemcpyHostToDevice));
        PQ_HIP(hipMemcpy(c.kc.p, cv.data(), cv.size() * sizeof(double), hipMemcpyHostToDevice));
    }
}

__global__ void k_zero_bytes(unsigned char* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

template <class T>
static void ewald_eval_t(Ctx& c, const double* q, bool force, hipStream_t s) {
    const int n = (int)c.n;
    EwFrac fr;
    for (int d = 0; d < 3; ++d) fr.inv[d] = 1.0 / c.prm.box[d];
    fr.tric = is_tric(c.prm) ? 1 : 0;
    fr.t = make_tric(c.prm);
    {
        const double L0 = c.prm.box[0], L1 = c.prm.box[1], L2 = c.prm.box[2];
        const double txy = c.prm.tilt[0], txz = c.prm.tilt[1], tyz = c.prm.tilt[2];
        fr.r10 = -txy / (L0 * L1);
        fr.r21 = -tyz / (L1 * L2);
        fr.r20 = (txy * tyz - L1 * txz) / (L0 * L1 * L2);
    }
    T* phi = as<T>(c.phi_k);
    V4<T>* f = as<V4<T>>(c.f_k);
    if (c.nk == 0) {
        // no k vectors: the reciprocal part vanishes (fill kernels, no memsets,
        // so the evaluation stays capturable in a graph)
        const size_t nb = (size_t)n * sizeof(T);
        PQ_LAUNCH(k_zero_bytes, std::max(1u, std::min(cdiv(nb, 256), 4096u)), 256, 0, s, c.phi_k.p, nb);
        if (force) {
            const size_t fb = (size_t)n * sizeof(V4<T>);
            PQ_LAUNCH(k_zero_bytes, std::max(1u, std::min(cdiv(fb, 256), 4096u)), 256, 0, s, c.f_k.p, fb);
        }
        PQ_LAUNCH(k_zero_bytes, 1, 64, 0, s, reinterpret_cast<unsigned char*>(c.ews.scal + 1), sizeof(double));
        return;
    }
    const int nb = cdiv(c.nk, EW_TILE);
    PQ_REQUIRE(c.ews.part_n >= (size_t)nb + 16 && c.spart.n >= (size_t)c.ew_nch * c.nk &&
                   c.gpart.n >= (size_t)c.ew_nkch * n,
               PQ_ERR_STATE, "direct-Ewald workspaces not sized");
    PQ_LAUNCH(k_sfac<T>, dim3(nb, c.ew_nch), EW_TILE, 0, s, n, c.nk, c.ew_cs, c.kn.p, c.w64.p, fr, q, c.spart.p);
    PQ_LAUNCH(k_sfac_sum, nb, EW_TILE, 0, s, c.nk, c.ew_nch, c.kc.p, c.spart.p, c.sfac.p, c.ews.part);
    PQ_LAUNCH(k_sum_part_e, 1, 256, 0, s, c.ews.part, nb, c.ews.scal + 1);
    if (n == 0) return;
    const dim3 g(cdiv(n, EW_TILE), c.ew_nkch);
    if (force) {
        PQ_LAUNCH((k_kgather<true, T>), g, EW_TILE, 0, s, n, c.nk, c.ew_kcs, c.kn.p, c.kc.p, c.sfac.p, c.w64.p, fr,
                  c.gpart.p);
        PQ_LAUNCH((k_kgather_sum<true, T>), cdiv(n, EW_TILE), EW_TILE, 0, s, n, c.ew_nkch, c.gpart.p, fr, q, phi, f);
    } else {
        PQ_LAUNCH((k_kgather<false, T>), g, EW_TILE, 0, s, n, c.nk, c.ew_kcs, c.kn.p, c.kc.p, c.sfac.p, c.w64.p, fr,
                  c.gpart.p);
        PQ_LAUNCH((k_kgather_sum<false, T>), cdiv(n, EW_TILE), EW_TILE, 0, s, n, c.ew_nkch, c.gpart.p, fr, q, phi, f);
    }
}

// phi, f (original order, without KE) into c.phi_k, c.f_k; E_rec (without KE) into c.ews.scal[1]
void ewald_eval(Ctx& c, const double* q, bool force, hipStream_t s) {
    if (c.fp64)
        ewald_eval_t<double>(c, q, force, s);
    else
        ewald_eval_t<float>(c, q, force, s);
}

}  // namespace pq
