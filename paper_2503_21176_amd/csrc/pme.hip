// Smooth PME charge spreading and potential/force gathering
// (Algorithm "Smooth PME", steps 1 and 5), FP32 bulk arithmetic.
//
// Atoms are sorted by the "brick" (B x B x B block of grid points) that holds
// their base grid point floor(u). One workgroup owns one brick:
//  * spreading accumulates q_i M_p(u_x - k_x) M_p(u_y - k_y) M_p(u_z - k_z)
//    into an LDS copy of the brick plus its (p-1)-point halo with LDS atomics,
//    then flushes the non-zero points to the global grid with FP32 atomics
//    (one global atomic per brick point instead of one per atom and point);
//  * gathering stages the same region of the convolved grid in LDS and
//    reads each atom's p^3 stencil from there.
// Eight lanes serve one atom; lane y < p walks the (z, x) plane of stencil row y.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dev.h"
#include "pq_internal.h"

namespace pq {

constexpr int PME_B = 8;

// Cardinal B-spline weights M_p(f + t), t = 0..P-1 (grid point base - t), and
// their derivatives, by the Cox-de Boor recursion, f in [0, 1).
template <int P>
__device__ __forceinline__ void bspline(float f, float* w, float* dw) {
    float m[P];
#pragma unroll
    for (int t = 0; t < P; ++t) m[t] = 0.0f;
    m[0] = f;
    m[1] = 1.0f - f;
#pragma unroll
    for (int k = 3; k <= P; ++k) {
        if (k == P) {
#pragma unroll
            for (int t = 0; t < P; ++t) dw[t] = m[t] - (t > 0 ? m[t - 1] : 0.0f);
        }
        const float inv = 1.0f / (float)(k - 1);
        m[k - 1] = (1.0f - f) * m[k - 2] * inv;
#pragma unroll
        for (int t = k - 2; t >= 1; --t) m[t] = ((f + t) * m[t] + ((float)k - f - t) * m[t - 1]) * inv;
        m[0] = f * m[0] * inv;
    }
#pragma unroll
    for (int t = 0; t < P; ++t) w[t] = m[t];
}

template <int P>
__device__ __forceinline__ float pick(const float* v, int i) {
    float r = 0.0f;
#pragma unroll
    for (int t = 0; t < P; ++t) r = (t == i) ? v[t] : r;
    return r;
}

struct PmeGeo {
    int K0, K1, K2;
    int nb0, nb1, nb2;
    double L[3], invL[3];
};

__global__ void k_pme_setup(int n, const double* __restrict__ w64, PmeGeo G, int* __restrict__ brick_of,
                            float4* __restrict__ frac_tmp, int* __restrict__ brick_cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int K[3] = {G.K0, G.K1, G.K2};
    int base[3];
    float fr[3];
    for (int d = 0; d < 3; ++d) {
        double u = (double)K[d] * (w64[3 * (size_t)i + d] * G.invL[d]);
        double fl = floor(u);
        int b = (int)fl;
        double f = u - fl;
        if (b >= K[d]) b -= K[d];
        if (b < 0) b += K[d];
        base[d] = b;
        fr[d] = (float)f;
        if (fr[d] >= 1.0f) fr[d] = 0.99999994f;
    }
    int br = base[0] / PME_B + G.nb0 * (base[1] / PME_B + G.nb1 * (base[2] / PME_B));
    brick_of[i] = br;
    frac_tmp[i] = make_float4(fr[0], fr[1], fr[2], __int_as_float(base[0] | (base[1] << 10) | (base[2] << 20)));
    atomicAdd(&brick_cnt[br], 1);
}

__global__ void k_pme_scatter(int n, const int* __restrict__ brick_of, const float4* __restrict__ frac_tmp,
                              const int* __restrict__ brick_start, int* __restrict__ brick_fill,
                              int* __restrict__ pme_idx, float4* __restrict__ pme_frac) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int br = brick_of[i];
    int pos = brick_start[br] + atomicAdd(&brick_fill[br], 1);
    pme_idx[pos] = i;
    pme_frac[pos] = frac_tmp[i];
}

__global__ void k_zero_f(float* __restrict__ a, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) a[i] = 0.0f;
}

template <int P>
__global__ __launch_bounds__(256) void k_spread(PmeGeo G, const int* __restrict__ brick_start,
                                                const int* __restrict__ pme_idx, const float4* __restrict__ pme_frac,
                                                const double* __restrict__ q, float* __restrict__ grid) {
    constexpr int R = PME_B + P - 1;
    __shared__ float lds[R * R * R];
    const int bid = blockIdx.x;
    const int bx = bid % G.nb0, by = (bid / G.nb0) % G.nb1, bz = bid / (G.nb0 * G.nb1);
    const int s0 = brick_start[bid], s1 = brick_start[bid + 1];
    if (s0 == s1) return;
    for (int t = threadIdx.x; t < R * R * R; t += 256) lds[t] = 0.0f;
    __syncthreads();
    const int x0 = bx * PME_B - (P - 1), y0 = by * PME_B - (P - 1), z0 = bz * PME_B - (P - 1);
    const int sub = threadIdx.x & 7, grp = threadIdx.x >> 3;
    for (int k = s0 + grp; k < s1; k += 32) {
        const float4 f4 = pme_frac[k];
        const float qq = (float)q[pme_idx[k]];
        const int pk = __float_as_int(f4.w);
        const int gx = pk & 1023, gy = (pk >> 10) & 1023, gz = (pk >> 20) & 1023;
        float wx[P], wy[P], wz[P], dd[P];
        bspline<P>(f4.x, wx, dd);
        bspline<P>(f4.y, wy, dd);
        bspline<P>(f4.z, wz, dd);
        if (sub < P) {
            const int ly = gy - sub - y0;
            const float qy = qq * pick<P>(wy, sub);
#pragma unroll
            for (int tz = 0; tz < P; ++tz) {
                const int lz = gz - tz - z0;
                const float qyz = qy * wz[tz];
                float* row = lds + (lz * R + ly) * R + (gx - x0);
#pragma unroll
                for (int tx = 0; tx < P; ++tx) atomicAdd(row - tx, qyz * wx[tx]);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < R * R * R; t += 256) {
        const float v = lds[t];
        if (v == 0.0f) continue;
        const int lx = t % R, ly = (t / R) % R, lz = t / (R * R);
        int X = x0 + lx, Y = y0 + ly, Z = z0 + lz;
        X += (X < 0) ? G.K0 : 0;
        X -= (X >= G.K0) ? G.K0 : 0;
        Y += (Y < 0) ? G.K1 : 0;
        Y -= (Y >= G.K1) ? G.K1 : 0;
        Z += (Z < 0) ? G.K2 : 0;
        Z -= (Z >= G.K2) ? G.K2 : 0;
        atomicAdd(&grid[((size_t)Z * G.K1 + Y) * G.K0 + X], v);
    }
}

template <int P, bool FORCE>
__global__ __launch_bounds__(256) void k_gather(PmeGeo G, const int* __restrict__ brick_start,
                                                const int* __restrict__ pme_idx, const float4* __restrict__ pme_frac,
                                                const double* __restrict__ q, const float* __restrict__ grid,
                                                float* __restrict__ phi_out, float4* __restrict__ f_out) {
    constexpr int R = PME_B + P - 1;
    __shared__ float lds[R * R * R];
    const int bid = blockIdx.x;
    const int bx = bid % G.nb0, by = (bid / G.nb0) % G.nb1, bz = bid / (G.nb0 * G.nb1);
    const int s0 = brick_start[bid], s1 = brick_start[bid + 1];
    if (s0 == s1) return;
    const int x0 = bx * PME_B - (P - 1), y0 = by * PME_B - (P - 1), z0 = bz * PME_B - (P - 1);
    for (int t = threadIdx.x; t < R * R * R; t += 256) {
        const int lx = t % R, ly = (t / R) % R, lz = t / (R * R);
        int X = x0 + lx, Y = y0 + ly, Z = z0 + lz;
        X += (X < 0) ? G.K0 : 0;
        X -= (X >= G.K0) ? G.K0 : 0;
        Y += (Y < 0) ? G.K1 : 0;
        Y -= (Y >= G.K1) ? G.K1 : 0;
        Z += (Z < 0) ? G.K2 : 0;
        Z -= (Z >= G.K2) ? G.K2 : 0;
        lds[t] = grid[((size_t)Z * G.K1 + Y) * G.K0 + X];
    }
    __syncthreads();
    const int sub = threadIdx.x & 7, grp = threadIdx.x >> 3;
    const float kx = (float)(G.K0 * G.invL[0]), ky = (float)(G.K1 * G.invL[1]), kz = (float)(G.K2 * G.invL[2]);
    // every group runs the same number of iterations so the shuffles see full groups
    const int iters = (s1 - s0 + 31) / 32;
    for (int it = 0; it < iters; ++it) {
        const int k = s0 + grp + 32 * it;
        const bool valid = k < s1;
        float phi = 0.0f, gxs = 0.0f, gys = 0.0f, gzs = 0.0f;
        int i = -1;
        if (valid) {
            const float4 f4 = pme_frac[k];
            i = pme_idx[k];
            const int pk = __float_as_int(f4.w);
            const int gx = pk & 1023, gy = (pk >> 10) & 1023, gz = (pk >> 20) & 1023;
            float wx[P], wy[P], wz[P], dx[P], dy[P], dz[P];
            bspline<P>(f4.x, wx, dx);
            bspline<P>(f4.y, wy, dy);
            bspline<P>(f4.z, wz, dz);
            if (sub < P) {
                const int ly = gy - sub - y0;
                const float wys = pick<P>(wy, sub), dys = pick<P>(dy, sub);
#pragma unroll
                for (int tz = 0; tz < P; ++tz) {
                    const float* row = lds + ((gz - tz - z0) * R + ly) * R + (gx - x0);
                    float s = 0.0f, sdx = 0.0f;
#pragma unroll
                    for (int tx = 0; tx < P; ++tx) {
                        const float v = row[-tx];
                        s = fmaf(wx[tx], v, s);
                        if (FORCE) sdx = fmaf(dx[tx], v, sdx);
                    }
                    phi = fmaf(wys * wz[tz], s, phi);
                    if (FORCE) {
                        gxs = fmaf(wys * wz[tz], sdx, gxs);
                        gys = fmaf(dys * wz[tz], s, gys);
                        gzs = fmaf(wys * dz[tz], s, gzs);
                    }
                }
            }
        }
        for (int o = 1; o < 8; o <<= 1) {
            phi += __shfl_xor(phi, o, 64);
            if (FORCE) {
                gxs += __shfl_xor(gxs, o, 64);
                gys += __shfl_xor(gys, o, 64);
                gzs += __shfl_xor(gzs, o, 64);
            }
        }
        if (valid && sub == 0) {
            phi_out[i] = phi;
            if (FORCE) {
                const float qq = (float)q[i];
                f_out[i] = make_float4(-qq * kx * gxs, -qq * ky * gys, -qq * kz * gzs, 0.0f);
            }
        }
    }
}

static PmeGeo geo(const Ctx& c) {
    PmeGeo G;
    G.K0 = c.K[0];
    G.K1 = c.K[1];
    G.K2 = c.K[2];
    G.nb0 = c.nb[0];
    G.nb1 = c.nb[1];
    G.nb2 = c.nb[2];
    for (int d = 0; d < 3; ++d) {
        G.L[d] = c.prm.box[d];
        G.invL[d] = 1.0 / c.prm.box[d];
    }
    return G;
}

void pme_setup(Ctx& c) {
    const int n = (int)c.n;
    hipStream_t s = c.stream;
    for (int d = 0; d < 3; ++d) {
        c.K[d] = c.prm.grid[d];
        c.nb[d] = (c.K[d] + PME_B - 1) / PME_B;
    }
    c.P = c.prm.order;
    c.nbrick = c.nb[0] * c.nb[1] * c.nb[2];
    c.brick_of.ensure(n);
    c.brick_cnt.ensure(c.nbrick);
    c.brick_fill.ensure(c.nbrick);
    c.brick_start.ensure(c.nbrick + 1);
    c.pme_idx.ensure(n);
    c.pme_frac.ensure(n);
    c.f_k.ensure(n);   // temporary for the unsorted fractional parts
    const size_t ng = (size_t)c.K[0] * c.K[1] * c.K[2];
    c.grid.ensure(ng);
    c.spec.ensure((size_t)(c.K[0] / 2 + 1) * c.K[1] * c.K[2]);
    PmeGeo G = geo(c);
    PQ_HIP(hipMemsetAsync(c.brick_cnt.p, 0, sizeof(int) * c.nbrick, s));
    PQ_HIP(hipMemsetAsync(c.brick_fill.p, 0, sizeof(int) * c.nbrick, s));
    PQ_LAUNCH(k_pme_setup, cdiv(n, 256), 256, 0, s, n, c.w64.p, G, c.brick_of.p, c.f_k.p, c.brick_cnt.p);
    scan_ints(c.brick_cnt.p, c.brick_start.p, c.nbrick, false, s);
    PQ_LAUNCH(k_pme_scatter, cdiv(n, 256), 256, 0, s, n, c.brick_of.p, c.f_k.p, c.brick_start.p, c.brick_fill.p,
              c.pme_idx.p, c.pme_frac.p);
    fft_setup(c);
}

template <int P>
static void pme_eval_p(Ctx& c, const double* q, bool force, float* phi, float4* f, hipEvent_t* ev, hipStream_t s) {
    PmeGeo G = geo(c);
    const size_t ng = (size_t)c.K[0] * c.K[1] * c.K[2];
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_SPREAD], s));
    PQ_LAUNCH(k_zero_f, std::min<size_t>(cdiv(ng, 256), 4096), 256, 0, s, c.grid.p, ng);
    PQ_LAUNCH(k_spread<P>, c.nbrick, 256, 0, s, G, c.brick_start.p, c.pme_idx.p, c.pme_frac.p, q, c.grid.p);
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_SPREAD + 1], s));
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_FFT], s));
    fft_convolve(c, s);
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_FFT + 1], s));
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_GATHER], s));
    if (force)
        PQ_LAUNCH((k_gather<P, true>), c.nbrick, 256, 0, s, G, c.brick_start.p, c.pme_idx.p, c.pme_frac.p, q,
                  c.grid.p, phi, f);
    else
        PQ_LAUNCH((k_gather<P, false>), c.nbrick, 256, 0, s, G, c.brick_start.p, c.pme_idx.p, c.pme_frac.p, q,
                  c.grid.p, phi, f);
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_GATHER + 1], s));
}

void pme_eval(Ctx& c, const double* q, bool force, float* phi, float4* f, hipEvent_t* ev, hipStream_t s) {
    switch (c.P) {
        case 3: pme_eval_p<3>(c, q, force, phi, f, ev, s); break;
        case 4: pme_eval_p<4>(c, q, force, phi, f, ev, s); break;
        case 5: pme_eval_p<5>(c, q, force, phi, f, ev, s); break;
        case 6: pme_eval_p<6>(c, q, force, phi, f, ev, s); break;
        case 7: pme_eval_p<7>(c, q, force, phi, f, ev, s); break;
        case 8: pme_eval_p<8>(c, q, force, phi, f, ev, s); break;
        default: throw Error(PQ_ERR_INVALID, "spline order must be in 3..8");
    }
}

}  // namespace pq
