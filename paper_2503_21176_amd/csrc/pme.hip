// Smooth PME charge spreading and potential/force gathering
// (Algorithm "Smooth PME", steps 1 and 5). Bulk precision T: FP32 (the
// production form) or FP64 (the same kernels instantiated in double).
//
// Atoms are sorted by the "brick" (B x B x B block of grid points) that holds
// their base grid point floor(u), in atom-index order inside each brick.
//  * spreading accumulates each brick's atoms into LDS copies of the brick
//    plus its (p-1)-point halo (one atom per wavefront step, one stencil row
//    per lane: conflict-free plain updates, no atomics), stores that region to
//    a staging buffer, and a second pass sums, per grid point, the (at most 8)
//    regions that overlap it: deterministic, no clearing pass;
//  * gathering stages the same region of the convolved grid in LDS and
//    reads each atom's p^3 stencil from there.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>

#include "dev.h"
#include "pq_internal.h"

namespace pq {

constexpr int PME_B = 8;
constexpr int PME_WSTRIDE = 48;   // stored B-spline values per atom (weights, derivatives)

// Cardinal B-spline weights M_p(f + t), t = 0..P-1 (grid point base - t), and
// their derivatives, by the Cox-de Boor recursion, f in [0, 1).
template <int P, class T>
__device__ __forceinline__ void bspline(T f, T* w, T* dw) {
    T m[P];
#pragma unroll
    for (int t = 0; t < P; ++t) m[t] = T(0);
    m[0] = f;
    m[1] = T(1) - f;
#pragma unroll
    for (int k = 3; k <= P; ++k) {
        if (k == P) {
#pragma unroll
            for (int t = 0; t < P; ++t) dw[t] = m[t] - (t > 0 ? m[t - 1] : T(0));
        }
        const T inv = T(1) / (T)(k - 1);
        m[k - 1] = (T(1) - f) * m[k - 2] * inv;
#pragma unroll
        for (int t = k - 2; t >= 1; --t) m[t] = ((f + t) * m[t] + ((T)k - f - t) * m[t - 1]) * inv;
        m[0] = f * m[0] * inv;
    }
#pragma unroll
    for (int t = 0; t < P; ++t) w[t] = m[t];
}

template <int P, class T>
__device__ __forceinline__ T pick(const T* v, int i) {
    T r = T(0);
#pragma unroll
    for (int t = 0; t < P; ++t) r = (t == i) ? v[t] : r;
    return r;
}

struct PmeGeo {
    int K0, K1, K2;
    int nb0, nb1, nb2;
    double L[3], invL[3];
    int tric;              // triclinic cell: fractional coordinates from t
    Tric t;
    double jyx, jzx, jzy;  // off-diagonal du/dr factors K0 R10, K0 R20, K1 R21 (R = H^-1)
};

// Base grid point, fractional offsets and brick of atom i.
template <class T>
__device__ __forceinline__ int pme_atom_setup(int i, const double* __restrict__ w64, const PmeGeo& G,
                                              int* __restrict__ brick_of, V4<T>* __restrict__ frac_tmp) {
    const int K[3] = {G.K0, G.K1, G.K2};
    int base[3];
    T fr[3];
    double s[3];
    if (G.tric) {
        frac_tric(w64[3 * (size_t)i], w64[3 * (size_t)i + 1], w64[3 * (size_t)i + 2], G.invL, G.t, s[0], s[1], s[2]);
    } else {
        for (int d = 0; d < 3; ++d) s[d] = w64[3 * (size_t)i + d] * G.invL[d];
    }
    for (int d = 0; d < 3; ++d) {
        double u = (double)K[d] * s[d];
        double fl = floor(u);
        int b = (int)fl;
        double f = u - fl;
        if (b >= K[d]) b -= K[d];
        if (b < 0) b += K[d];
        base[d] = b;
        fr[d] = (T)f;
        if (fr[d] >= T(1)) fr[d] = T(1) - T(1e-7);
    }
    const int br = base[0] / PME_B + G.nb0 * (base[1] / PME_B + G.nb1 * (base[2] / PME_B));
    brick_of[i] = br;
    frac_tmp[i] = mk4<T>(fr[0], fr[1], fr[2], pack_int(base[0] | (base[1] << 10) | (base[2] << 20), T(0)));
    return br;
}

template <class T>
__global__ void k_pme_setup(int n, const double* __restrict__ w64, PmeGeo G, int* __restrict__ brick_of,
                            V4<T>* __restrict__ frac_tmp, int* __restrict__ brick_cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicAdd(&brick_cnt[pme_atom_setup<T>(i, w64, G, brick_of, frac_tmp)], 1);
}

__global__ void k_pme_scatter(int n, const int* __restrict__ brick_of, const int* __restrict__ brick_start,
                              int* __restrict__ brick_fill, int* __restrict__ unordered) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int br = brick_of[i];
    unordered[brick_start[br] + atomicAdd(&brick_fill[br], 1)] = i;
}

// The same binning without global atomics (bricks that fit the LDS counters):
// workgroup w takes atoms [w per, (w + 1) per), counts them per brick in LDS
// and stores the counts brick-major, hist[b nwg + w]; the exclusive scan of
// hist gives each workgroup its first slot in every brick, where
// k_pme_scatter_hist places its atoms with LDS cursors. The order inside a
// brick is settled by k_pme_order.
constexpr int BRICK_LDS_MAX = 16384;
template <class T>
__global__ __launch_bounds__(256) void k_pme_setup_hist(int n, int per, int nbrick, const double* __restrict__ w64,
                                                        PmeGeo G, int* __restrict__ brick_of,
                                                        V4<T>* __restrict__ frac_tmp, int* __restrict__ hist) {
    extern __shared__ int cntl[];
    for (int b = threadIdx.x; b < nbrick; b += blockDim.x) cntl[b] = 0;
    __syncthreads();
    const int a0 = blockIdx.x * per, a1 = min(n, a0 + per);
    for (int i = a0 + threadIdx.x; i < a1; i += blockDim.x) atomicAdd(&cntl[pme_atom_setup<T>(i, w64, G, brick_of, frac_tmp)], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < nbrick; b += blockDim.x) hist[(size_t)b * gridDim.x + blockIdx.x] = cntl[b];
}
__global__ void k_brick_starts(int nbrick, int nwg, const int* __restrict__ hscan, int* __restrict__ brick_start) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= nbrick) brick_start[b] = hscan[(size_t)b * nwg];
}
__global__ __launch_bounds__(256) void k_pme_scatter_hist(int n, int per, int nbrick, const int* __restrict__ brick_of,
                                                          const int* __restrict__ hscan, int* __restrict__ unordered) {
    extern __shared__ int cur[];
    for (int b = threadIdx.x; b < nbrick; b += blockDim.x) cur[b] = hscan[(size_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const int a0 = blockIdx.x * per, a1 = min(n, a0 + per);
    for (int i = a0 + threadIdx.x; i < a1; i += blockDim.x) unordered[atomicAdd(&cur[brick_of[i]], 1)] = i;
}

// Deterministic order inside each brick (by atom index), so every
// accumulation order, and hence every result, is reproducible bit for bit.
// One wavefront per brick: each lane holds one of the brick's atoms and counts
// the smaller indices among all of the brick's atoms, 64 at a time from lane
// registers.
template <class T>
__global__ __launch_bounds__(256) void k_pme_order(int nbrick, const int* __restrict__ brick_start,
                                                   const int* __restrict__ unordered,
                                                   const V4<T>* __restrict__ frac_tmp, int* __restrict__ pme_idx,
                                                   V4<T>* __restrict__ pme_frac) {
    const int lane = threadIdx.x & 63;
    const int br = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (br >= nbrick) return;
    const int s0 = brick_start[br], m = brick_start[br + 1] - s0;
    for (int ab = 0; ab < m; ab += 64) {
        const int t = ab + lane;
        const int ki = t < m ? unordered[s0 + t] : 0x7fffffff;
        int r = 0;
        for (int kb = 0; kb < m; kb += 64) {
            const int kv = (kb + lane < m) ? unordered[s0 + kb + lane] : 0x7fffffff;
            const int lim = min(64, m - kb);
            for (int u = 0; u < lim; ++u) r += __builtin_amdgcn_readlane(kv, u) < ki;
        }
        if (t < m) {
            pme_idx[s0 + r] = ki;
            pme_frac[s0 + r] = frac_tmp[ki];
        }
    }
}

// B-spline weights and derivatives of every atom (brick order), computed once
// per set of positions: pme_w[48 k ...] = {M_p(f_x + t)}_t, {M_p(f_y + t)}_t,
// {M_p(f_z + t)}_t, then the three derivative rows, each padded to 8 entries.
template <int P, class T>
__global__ void k_pme_weights(int n, const V4<T>* __restrict__ pme_frac, T* __restrict__ pme_w) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const V4<T> f4 = pme_frac[k];
    T w[P], dd[P];
    T* out = pme_w + (size_t)k * PME_WSTRIDE;
    const T fr[3] = {f4.x, f4.y, f4.z};
    for (int d = 0; d < 3; ++d) {
        bspline<P, T>(fr[d], w, dd);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            out[8 * d + t] = (t < P) ? w[t] : T(0);
            out[24 + 8 * d + t] = (t < P) ? dd[t] : T(0);
        }
    }
}

// Spreading, pass 1: the workgroup of brick b accumulates
// q_i M_p(u_x - k_x) M_p(u_y - k_y) M_p(u_z - k_z) of its own atoms over the
// region [b*B - (p-1), b*B + B - 1]^3 (the brick plus its halo on the low
// side) and stores the region to a per-brick staging slot with plain
// coalesced stores. Each wavefront keeps a private LDS copy of the region and
// takes one atom per step, lane (y, z) updating stencil row (y, z): the
// updates of one step hit distinct addresses, so plain read-modify-writes
// replace atomics; the copies are summed at the end. No atomics at all.
// A wavefront first loads a batch of up to SPREAD_BATCH of its atoms (weights,
// base index, charge; one atom per lane) into an LDS table, so its update
// steps wait on LDS only.
constexpr int SPREAD_BATCH = 16;
// value v of lane i (i wave-uniform), through the scalar unit
__device__ __forceinline__ float lane_value(float v, int i) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}
__device__ __forceinline__ double lane_value(double v, int i) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), i);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
#ifndef SPREAD_WAVES
#define SPREAD_WAVES 2
#endif
constexpr int SW = SPREAD_WAVES;   // wavefronts (and private region copies) per brick
template <int P, class T>
__global__ __launch_bounds__(64 * SW) void k_spread_stage(PmeGeo G, const int* __restrict__ brick_start,
                                                      const V4<T>* __restrict__ pme_frac,
                                                      const T* __restrict__ pme_w, const T* __restrict__ qbrick,
                                                      T* __restrict__ stage) {
    chain_priority();
    constexpr int R = PME_B + P - 1;
    constexpr int R3 = R * R * R;
    constexpr int R3P = (R3 + 3) & ~3;          // region copies padded to 4 values (vector clears)
    __shared__ __align__(32) T lds[SW][R3P];
    __shared__ __align__(32) T tab[SW][SPREAD_BATCH][32];   // per atom: weights x, y, z (8 each), base, charge
    const int bid = blockIdx.x;
    const int bx = bid % G.nb0, by = (bid / G.nb0) % G.nb1, bz = bid / (G.nb0 * G.nb1);
    const int s0 = brick_start[bid], s1 = brick_start[bid + 1];
    {
        V4<T>* l4 = reinterpret_cast<V4<T>*>(&lds[0][0]);
        for (int t = threadIdx.x; t < SW * R3P / 4; t += 64 * SW) l4[t] = mk4<T>(T(0), T(0), T(0), T(0));
    }
    __syncthreads();
    const int x0 = bx * PME_B - (P - 1), y0 = by * PME_B - (P - 1), z0 = bz * PME_B - (P - 1);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ty = lane & 7, tz = lane >> 3;
    const bool active = (ty < P) && (tz < P);
    T* my = lds[wv];
    T(*tb)[32] = tab[wv];
    // the wave's atoms are s0 + wv, s0 + wv + SW, ...
    for (int k0 = s0 + wv; k0 < s1; k0 += SW * SPREAD_BATCH) {
        const int nb = min(SPREAD_BATCH, (s1 - k0 + SW - 1) / SW);
        // lane l < nb holds atom l's x weights, base index and charge in
        // registers (read by every lane through readlane) and puts its y and z
        // weights in the LDS table (each lane reads its own row's)
        V4<T> wxa = mk4<T>(T(0), T(0), T(0), T(0)), wxb = wxa;
        T base = T(0), qa = T(0);
        if (lane < nb) {
            const int k = k0 + SW * lane;
            const V4<T>* wk = reinterpret_cast<const V4<T>*>(pme_w + (size_t)k * PME_WSTRIDE);
            T* row = tb[lane];
            wxa = wk[0];
            wxb = wk[1];
#pragma unroll
            for (int u = 2; u < 6; ++u) {
                const V4<T> w4 = wk[u];
                row[4 * u + 0] = w4.x;
                row[4 * u + 1] = w4.y;
                row[4 * u + 2] = w4.z;
                row[4 * u + 3] = w4.w;
            }
            base = pme_frac[k].w;
            qa = qbrick[k];
        }
        // the table is written and read by different lanes
        __builtin_amdgcn_wave_barrier();
        for (int i = 0; i < nb; ++i) {
            const T* at = tb[i];
            const T wxs[8] = {lane_value(wxa.x, i), lane_value(wxa.y, i), lane_value(wxa.z, i), lane_value(wxa.w, i),
                              P > 4 ? lane_value(wxb.x, i) : T(0), P > 5 ? lane_value(wxb.y, i) : T(0),
                              P > 6 ? lane_value(wxb.z, i) : T(0), P > 7 ? lane_value(wxb.w, i) : T(0)};
            const int pk = unpack_int(lane_value(base, i));
            const T qi = lane_value(qa, i);
            const int gx = pk & 1023, gy = (pk >> 10) & 1023, gz = (pk >> 20) & 1023;
            if (active) {
                const T c = qi * at[8 + ty] * at[16 + tz];
                T* rowp = my + ((gz - tz - z0) * R + (gy - ty - y0)) * R + (gx - x0);
                T v[P];
#pragma unroll
                for (int tx = 0; tx < P; ++tx) v[tx] = rowp[-tx];
#pragma unroll
                for (int tx = 0; tx < P; ++tx) rowp[-tx] = fma(c, wxs[tx], v[tx]);
            }
            // the next atom may update the same rows
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    T* out = stage + (size_t)bid * R3;
    for (int t = threadIdx.x; t < R3; t += 64 * SW) {
        T v = lds[0][t];
#pragma unroll
        for (int w = 1; w < SW; ++w) v += lds[w][t];
        out[t] = v;
    }
}

// Bricks b (and local coordinates l in [0, R)) whose region holds grid
// coordinate g along one axis: b*B - (p-1) + l == g (mod K).
template <int P>
__device__ __forceinline__ int region_hits(int g, int K, int nb, int* bb, int* ll) {
    constexpr int R = PME_B + P - 1;
    int cnt = 0;
    for (int m = -1; m <= 1; ++m) {
        const int gp = g + m * K;
        // b*B - (P-1) <= gp <= b*B + B - 1
        int blo = gp - PME_B + 1;
        blo = (blo >= 0) ? (blo + PME_B - 1) / PME_B : -((-blo) / PME_B);
        const int bhi_num = gp + P - 1;
        const int bhi = (bhi_num >= 0) ? bhi_num / PME_B : -((-bhi_num + PME_B - 1) / PME_B);
        for (int b = max(blo, 0); b <= min(bhi, nb - 1); ++b) {
            const int l = gp - b * PME_B + (P - 1);
            if (l >= 0 && l < R && cnt < 6) {
                bb[cnt] = b;
                ll[cnt] = l;
                ++cnt;
            }
        }
    }
    return cnt;
}

// Spreading, pass 2: each grid point sums the staged regions that hold it,
// in a fixed order (z hit, then y, then x: deterministic). One wavefront per
// grid row (y, z), so the regions along y and z are found once per row; lanes
// walk x. On grids of at least 2 bricks per axis a point lies in at most two
// regions per axis, and its (at most 8) loads are issued together; smaller
// grids take the general loop.
constexpr int REDUCE_ROWS = 4;   // grid rows (wavefronts) per workgroup
template <int P, class T>
__global__ __launch_bounds__(64 * REDUCE_ROWS) void k_spread_reduce(PmeGeo G, const T* __restrict__ stage,
                                                                    T* __restrict__ grid) {
    chain_priority();
    constexpr int R = PME_B + P - 1;
    constexpr int R3 = R * R * R;
    const int row = __builtin_amdgcn_readfirstlane(blockIdx.x * REDUCE_ROWS + (threadIdx.x >> 6));
    if (row >= G.K1 * G.K2) return;
    const int gy = row % G.K1, gz = row / G.K1;
    int by[6], ly[6], bz[6], lz[6];
    const int ny = region_hits<P>(gy, G.K1, G.nb1, by, ly);
    const int nz = region_hits<P>(gz, G.K2, G.nb2, bz, lz);
    // offsets of the (y, z) hits: plane[iz][iy]
    size_t plane[2][2];
#pragma unroll
    for (int iz = 0; iz < 2; ++iz)
#pragma unroll
        for (int iy = 0; iy < 2; ++iy) {
            const int z = min(iz, nz - 1), y = min(iy, ny - 1);
            plane[iz][iy] = (size_t)R3 * (G.nb0 * (by[y] + G.nb1 * bz[z])) + (lz[z] * R + ly[y]) * R;
        }
    T* out = grid + (size_t)row * G.K0;
    for (int gx = threadIdx.x & 63; gx < G.K0; gx += 64) {
        int bx[6], lx[6];
        const int nx = region_hits<P>(gx, G.K0, G.nb0, bx, lx);
        T v = T(0);
        if (nx <= 2 && ny <= 2 && nz <= 2) {
            size_t xo[2];
            xo[0] = (size_t)R3 * bx[0] + lx[0];
            xo[1] = (size_t)R3 * bx[min(1, nx - 1)] + lx[min(1, nx - 1)];
            T t[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int ix = q & 1, iy = (q >> 1) & 1, iz = q >> 2;
                t[q] = (ix < nx && iy < ny && iz < nz) ? stage[plane[iz][iy] + xo[ix]] : T(0);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int ix = q & 1, iy = (q >> 1) & 1, iz = q >> 2;
                if (ix < nx && iy < ny && iz < nz) v += t[q];
            }
        } else {
            for (int iz = 0; iz < nz; ++iz)
                for (int iy = 0; iy < ny; ++iy) {
                    const T* base =
                        stage + (size_t)R3 * (G.nb0 * (by[iy] + G.nb1 * bz[iz])) + (lz[iz] * R + ly[iy]) * R;
                    for (int ix = 0; ix < nx; ++ix) v += base[(size_t)R3 * bx[ix] + lx[ix]];
                }
        }
        out[gx] = v;
    }
}

// Gathering (step 5): phi_rec,i = sum_k W_i(k) psi(k) and
// F_rec,i = -q_i sum_k grad W_i(k) psi(k), from an LDS copy of the brick's
// region of the convolved grid (staged row by row); eight lanes per atom,
// lane y < p walks the (z, x) plane of stencil row y with the atom's stored
// B-spline weights and derivatives.
// BIL: the two-charge (bilinear) reciprocal force of u (qbrick, convolved
// grid psi_u in `grid`) and v (qbrick2, psi_v in `grid2`):
//   F_i = -1/2 (u_i grad_i(theta . psi_v) + v_i grad_i(theta . psi_u)), no potential.
constexpr int GATHER_THREADS = 256;   // per workgroup: 8 lanes per atom, 16 lanes per staged region row
template <int P, bool FORCE, bool BIL, class T>
__global__ __launch_bounds__(GATHER_THREADS) void k_gather(PmeGeo G, const int* __restrict__ brick_start,
                                                const int* __restrict__ pme_idx, const V4<T>* __restrict__ pme_frac,
                                                const T* __restrict__ pme_w, const T* __restrict__ qbrick,
                                                const T* __restrict__ grid, const T* __restrict__ qbrick2,
                                                const T* __restrict__ grid2, T* __restrict__ phi_out,
                                                V4<T>* __restrict__ f_out) {
    chain_priority();
    constexpr int R = PME_B + P - 1;
    static_assert(R <= 16, "a region row must fit 16 lanes");
    __shared__ T lds[R * R * R];
    __shared__ T lds2[BIL ? R * R * R : 1];
    const int bid = blockIdx.x;
    const int bx = bid % G.nb0, by = (bid / G.nb0) % G.nb1, bz = bid / (G.nb0 * G.nb1);
    const int s0 = brick_start[bid], s1 = brick_start[bid + 1];
    if (s0 == s1) return;
    const int x0 = bx * PME_B - (P - 1), y0 = by * PME_B - (P - 1), z0 = bz * PME_B - (P - 1);
    {
        // 16 lanes per region row, GATHER_THREADS / 16 rows per pass
        const int lx = threadIdx.x & 15;
        int X = x0 + lx;
        X += (X < 0) ? G.K0 : 0;
        X -= (X >= G.K0) ? G.K0 : 0;
        for (int r = threadIdx.x >> 4; r < R * R; r += GATHER_THREADS / 16) {
            const int ly = r % R, lz = r / R;
            int Y = y0 + ly, Z = z0 + lz;
            Y += (Y < 0) ? G.K1 : 0;
            Y -= (Y >= G.K1) ? G.K1 : 0;
            Z += (Z < 0) ? G.K2 : 0;
            Z -= (Z >= G.K2) ? G.K2 : 0;
            if (lx < R) {
                const size_t gi = ((size_t)Z * G.K1 + Y) * G.K0 + X;
                lds[r * R + lx] = grid[gi];
                if (BIL) lds2[r * R + lx] = grid2[gi];
            }
        }
    }
    __syncthreads();
    const int sub = threadIdx.x & 7, grp = threadIdx.x >> 3;
    const T kx = (T)(G.K0 * G.invL[0]), ky = (T)(G.K1 * G.invL[1]), kz = (T)(G.K2 * G.invL[2]);
    // every group runs the same number of iterations so the shuffles see full groups
    constexpr int APW = GATHER_THREADS / 8;   // atoms per pass
    const int iters = (s1 - s0 + APW - 1) / APW;
    for (int it = 0; it < iters; ++it) {
        const int k = s0 + grp + APW * it;
        const bool valid = k < s1;
        T phi = 0, gxs = 0, gys = 0, gzs = 0;
        T hxs = 0, hys = 0, hzs = 0;   // BIL: gradient sums on psi_v
        int i = -1;
        T qq = 0, qv = 0;
        if (valid) {
            qq = qbrick[k];
            if (BIL) qv = qbrick2[k];
            i = pme_idx[k];
            const int pk = unpack_int(pme_frac[k].w);
            const int gx = pk & 1023, gy = (pk >> 10) & 1023, gz = (pk >> 20) & 1023;
            if (sub < P) {
                const T* wk = pme_w + (size_t)k * PME_WSTRIDE;
                T wx[P], wz[P], dx[P], dz[P];
#pragma unroll
                for (int t = 0; t < P; ++t) {
                    wx[t] = wk[t];
                    wz[t] = wk[16 + t];
                    dx[t] = wk[24 + t];
                    dz[t] = wk[40 + t];
                }
                const T wys = wk[8 + sub], dys = wk[32 + sub];
                const int ly = gy - sub - y0;
#pragma unroll
                for (int tz = 0; tz < P; ++tz) {
                    const int off = ((gz - tz - z0) * R + ly) * R + (gx - x0);
                    const T* row = lds + off;
                    T s = 0, sdx = 0;
#pragma unroll
                    for (int tx = 0; tx < P; ++tx) {
                        const T v = row[-tx];
                        s = fma(wx[tx], v, s);
                        if (FORCE) sdx = fma(dx[tx], v, sdx);
                    }
                    if (!BIL) phi = fma(wys * wz[tz], s, phi);
                    if (FORCE) {
                        gxs = fma(wys * wz[tz], sdx, gxs);
                        gys = fma(dys * wz[tz], s, gys);
                        gzs = fma(wys * dz[tz], s, gzs);
                    }
                    if (BIL) {
                        const T* row2 = lds2 + off;
                        T s2 = 0, sdx2 = 0;
#pragma unroll
                        for (int tx = 0; tx < P; ++tx) {
                            const T v = row2[-tx];
                            s2 = fma(wx[tx], v, s2);
                            sdx2 = fma(dx[tx], v, sdx2);
                        }
                        hxs = fma(wys * wz[tz], sdx2, hxs);
                        hys = fma(dys * wz[tz], s2, hys);
                        hzs = fma(wys * dz[tz], s2, hzs);
                    }
                }
            }
        }
        for (int o = 1; o < 8; o <<= 1) {
            if (!BIL) phi += __shfl_xor(phi, o, 64);
            if (FORCE) {
                gxs += __shfl_xor(gxs, o, 64);
                gys += __shfl_xor(gys, o, 64);
                gzs += __shfl_xor(gzs, o, 64);
            }
            if (BIL) {
                hxs += __shfl_xor(hxs, o, 64);
                hys += __shfl_xor(hys, o, 64);
                hzs += __shfl_xor(hzs, o, 64);
            }
        }
        if (BIL && valid && sub == 0) {
            // u_i (grad on psi_v) + v_i (grad on psi_u), then the chain factors
            const T cx = T(0.5) * fma(qq, hxs, qv * gxs);
            const T cy = T(0.5) * fma(qq, hys, qv * gys);
            const T cz = T(0.5) * fma(qq, hzs, qv * gzs);
            if (G.tric) {
                const T jyx = (T)G.jyx, jzx = (T)G.jzx, jzy = (T)G.jzy;
                f_out[i] = mk4<T>(-(kx * cx), -(ky * cy + jyx * cx), -((kz * cz + jzy * cy) + jzx * cx), T(0));
            } else {
                f_out[i] = mk4<T>(-kx * cx, -ky * cy, -kz * cz, T(0));
            }
        }
        if (!BIL && valid && sub == 0) {
            phi_out[i] = phi;
            if (FORCE) {
                if (G.tric) {
                    // F = -q J^T g with J[d][k] = du_d/dr_k (lower triangular R = H^-1)
                    const T jyx = (T)G.jyx, jzx = (T)G.jzx, jzy = (T)G.jzy;
                    f_out[i] = mk4<T>(-qq * (kx * gxs), -qq * (ky * gys + jyx * gxs),
                                      -qq * ((kz * gzs + jzy * gys) + jzx * gxs), T(0));
                } else {
                    f_out[i] = mk4<T>(-qq * kx * gxs, -qq * ky * gys, -qq * kz * gzs, T(0));
                }
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
    G.tric = is_tric(c.prm) ? 1 : 0;
    G.t = make_tric(c.prm);
    // R = H^-1 below the diagonal: R10 = -txy/(L0 L1), R21 = -tyz/(L1 L2),
    // R20 = (txy tyz - L1 txz)/(L0 L1 L2)
    const double L0 = c.prm.box[0], L1 = c.prm.box[1], L2 = c.prm.box[2];
    const double txy = c.prm.tilt[0], txz = c.prm.tilt[1], tyz = c.prm.tilt[2];
    G.jyx = c.K[0] * (-txy / (L0 * L1));
    G.jzx = c.K[0] * ((txy * tyz - L1 * txz) / (L0 * L1 * L2));
    G.jzy = c.K[1] * (-tyz / (L1 * L2));
    return G;
}

template <class T>
static void pme_setup_t(Ctx& c) {
    const int n = (int)c.n;
    hipStream_t s = c.stream;
    using v4 = V4<T>;
    PmeGeo G = geo(c);
    c.f_k.ensure((size_t)n * sizeof(v4));   // temporary for the unsorted fractional parts
    c.pme_frac.ensure((size_t)n * sizeof(v4));
    c.pme_w.ensure((size_t)n * PME_WSTRIDE * sizeof(T));
    c.tmp_atoms.ensure(n);
    if (c.nbrick <= BRICK_LDS_MAX) {
        const int nwg = std::max(1, std::min(256, (int)cdiv(n, 1024)));
        const int per = (int)cdiv(n, nwg);
        const size_t nh = (size_t)c.nbrick * nwg;
        c.bin_hist.ensure(nh + 1);
        c.bin_scan.ensure(nh + 1);
        PQ_LAUNCH(k_pme_setup_hist<T>, nwg, 256, sizeof(int) * c.nbrick, s, n, per, c.nbrick, c.w64.p, G,
                  c.brick_of.p, as<v4>(c.f_k), c.bin_hist.p);
        scan_ints(c, c.bin_hist.p, c.bin_scan.p, (int)nh, false, s);
        PQ_LAUNCH(k_brick_starts, cdiv(c.nbrick + 1, 256), 256, 0, s, c.nbrick, nwg, c.bin_scan.p, c.brick_start.p);
        PQ_LAUNCH(k_pme_scatter_hist, nwg, 256, sizeof(int) * c.nbrick, s, n, per, c.nbrick, c.brick_of.p,
                  c.bin_scan.p, c.tmp_atoms.p);
    } else {
        PQ_HIP(hipMemsetAsync(c.brick_cnt.p, 0, sizeof(int) * c.nbrick, s));
        PQ_HIP(hipMemsetAsync(c.brick_fill.p, 0, sizeof(int) * c.nbrick, s));
        PQ_LAUNCH(k_pme_setup<T>, cdiv(n, 256), 256, 0, s, n, c.w64.p, G, c.brick_of.p, as<v4>(c.f_k),
                  c.brick_cnt.p);
        scan_ints(c, c.brick_cnt.p, c.brick_start.p, c.nbrick, false, s);
        PQ_LAUNCH(k_pme_scatter, cdiv(n, 256), 256, 0, s, n, c.brick_of.p, c.brick_start.p, c.brick_fill.p,
                  c.tmp_atoms.p);
    }
    PQ_LAUNCH(k_pme_order<T>, cdiv(c.nbrick, 4), 256, 0, s, c.nbrick, c.brick_start.p, c.tmp_atoms.p,
              as<v4>(c.f_k), c.pme_idx.p, as<v4>(c.pme_frac));
    switch (c.P) {
        case 3: PQ_LAUNCH((k_pme_weights<3, T>), cdiv(n, 256), 256, 0, s, n, as<v4>(c.pme_frac), as<T>(c.pme_w)); break;
        case 4: PQ_LAUNCH((k_pme_weights<4, T>), cdiv(n, 256), 256, 0, s, n, as<v4>(c.pme_frac), as<T>(c.pme_w)); break;
        case 5: PQ_LAUNCH((k_pme_weights<5, T>), cdiv(n, 256), 256, 0, s, n, as<v4>(c.pme_frac), as<T>(c.pme_w)); break;
        case 6: PQ_LAUNCH((k_pme_weights<6, T>), cdiv(n, 256), 256, 0, s, n, as<v4>(c.pme_frac), as<T>(c.pme_w)); break;
        case 7: PQ_LAUNCH((k_pme_weights<7, T>), cdiv(n, 256), 256, 0, s, n, as<v4>(c.pme_frac), as<T>(c.pme_w)); break;
        case 8: PQ_LAUNCH((k_pme_weights<8, T>), cdiv(n, 256), 256, 0, s, n, as<v4>(c.pme_frac), as<T>(c.pme_w)); break;
        default: throw Error(PQ_ERR_INVALID, "spline order must be in 3..8");
    }
}

void pme_setup(Ctx& c) {
    const int n = (int)c.n;
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
    c.qbrick.ensure((size_t)n * rsz(c));
    const size_t ng = (size_t)c.K[0] * c.K[1] * c.K[2];
    c.grid.ensure(ng * rsz(c));
    const int R = PME_B + c.P - 1;
    c.stage.ensure((size_t)c.nbrick * R * R * R * rsz(c));
    c.spec.ensure((size_t)(c.K[0] / 2 + 1) * c.K[1] * c.K[2] * 2 * rsz(c));
    if (c.fp64)
        pme_setup_t<double>(c);
    else
        pme_setup_t<float>(c);
    fft_setup(c);
}

template <class T>
__global__ void k_copy_grid(size_t n, const T* __restrict__ a, T* __restrict__ b) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <int P, class T>
static void pme_eval_p(Ctx& c, const double* q, bool force, hipEvent_t* ev, hipStream_t s,
                       const std::function<void()>& at_fork) {
    using v4 = V4<T>;
    PmeGeo G = geo(c);
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_SPREAD], s));
    PQ_LAUNCH((k_spread_stage<P, T>), c.nbrick, 64 * SW, 0, s, G, c.brick_start.p, as<v4>(c.pme_frac), as<T>(c.pme_w),
              as<T>(c.qbrick), as<T>(c.stage));
    if (at_fork && c.fork_at == 1) at_fork();
    PQ_LAUNCH((k_spread_reduce<P, T>), cdiv(c.K[1] * c.K[2], REDUCE_ROWS), 64 * REDUCE_ROWS, 0, s, G,
              as<T>(c.stage), as<T>(c.grid));
    if (at_fork && c.fork_at == 2) at_fork();
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_SPREAD + 1], s));
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_FFT], s));
    fft_convolve(c, s);
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_FFT + 1], s));
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_GATHER], s));
    if (c.save_psi) {
        // keep the convolved grid for a bilinear force evaluation that follows
        const size_t ng = (size_t)c.K[0] * c.K[1] * c.K[2];
        PQ_LAUNCH((k_copy_grid<T>), std::min<size_t>(cdiv(ng, 256), 8192), 256, 0, s, ng, as<T>(c.grid),
                  as<T>(c.grid2));
    }
    if (force)
        PQ_LAUNCH((k_gather<P, true, false, T>), c.nbrick, GATHER_THREADS, 0, s, G, c.brick_start.p, c.pme_idx.p,
                  as<v4>(c.pme_frac), as<T>(c.pme_w), as<T>(c.qbrick), as<T>(c.grid), (const T*)nullptr,
                  (const T*)nullptr, as<T>(c.phi_k), as<v4>(c.f_k));
    else
        PQ_LAUNCH((k_gather<P, false, false, T>), c.nbrick, GATHER_THREADS, 0, s, G, c.brick_start.p, c.pme_idx.p,
                  as<v4>(c.pme_frac), as<T>(c.pme_w), as<T>(c.qbrick), as<T>(c.grid), (const T*)nullptr,
                  (const T*)nullptr, as<T>(c.phi_k), as<v4>(c.f_k));
    if (ev) PQ_HIP(hipEventRecord(ev[2 * PQ_PHASE_GATHER + 1], s));
}

// Bilinear reciprocal force of u (qbrick) and v (qbrick2) into c.f_k: the
// convolved grid of v from grid2 (have_psi_v: kept by the last potential
// evaluation of v, c.save_psi) or computed here, that of u into grid.
template <int P, class T>
static void pme_bilinear_p(Ctx& c, bool have_psi_v, hipStream_t s) {
    using v4 = V4<T>;
    PmeGeo G = geo(c);
    const size_t ng = (size_t)c.K[0] * c.K[1] * c.K[2];
    auto chain = [&](const T* q) {
        PQ_LAUNCH((k_spread_stage<P, T>), c.nbrick, 64 * SW, 0, s, G, c.brick_start.p, as<v4>(c.pme_frac),
                  as<T>(c.pme_w), q, as<T>(c.stage));
        PQ_LAUNCH((k_spread_reduce<P, T>), cdiv(c.K[1] * c.K[2], REDUCE_ROWS), 64 * REDUCE_ROWS, 0, s, G,
                  as<T>(c.stage), as<T>(c.grid));
        fft_convolve(c, s);
    };
    if (!have_psi_v) {
        chain(as<T>(c.qbrick2));
        PQ_LAUNCH((k_copy_grid<T>), std::min<size_t>(cdiv(ng, 256), 8192), 256, 0, s, ng, as<T>(c.grid),
                  as<T>(c.grid2));
    }
    chain(as<T>(c.qbrick));
    PQ_LAUNCH((k_gather<P, true, true, T>), c.nbrick, GATHER_THREADS, 0, s, G, c.brick_start.p, c.pme_idx.p, as<v4>(c.pme_frac),
              as<T>(c.pme_w), as<T>(c.qbrick), as<T>(c.grid), as<T>(c.qbrick2), as<T>(c.grid2), as<T>(c.phi_k),
              as<v4>(c.f_k));
}

template <class T>
static void pme_bilinear_t(Ctx& c, bool have_psi_v, hipStream_t s) {
    switch (c.P) {
        case 3: pme_bilinear_p<3, T>(c, have_psi_v, s); break;
        case 4: pme_bilinear_p<4, T>(c, have_psi_v, s); break;
        case 5: pme_bilinear_p<5, T>(c, have_psi_v, s); break;
        case 6: pme_bilinear_p<6, T>(c, have_psi_v, s); break;
        case 7: pme_bilinear_p<7, T>(c, have_psi_v, s); break;
        case 8: pme_bilinear_p<8, T>(c, have_psi_v, s); break;
        default: throw Error(PQ_ERR_INVALID, "spline order must be in 3..8");
    }
}

void pme_bilinear(Ctx& c, bool have_psi_v, hipStream_t s) {
    const bool we = c.want_energy;
    c.want_energy = false;   // no reciprocal energy for these chains
    if (c.fp64)
        pme_bilinear_t<double>(c, have_psi_v, s);
    else
        pme_bilinear_t<float>(c, have_psi_v, s);
    c.want_energy = we;
}

template <class T>
static void pme_eval_t(Ctx& c, const double* q, bool force, hipEvent_t* ev, hipStream_t s,
                       const std::function<void()>& at_fork) {
    switch (c.P) {
        case 3: pme_eval_p<3, T>(c, q, force, ev, s, at_fork); break;
        case 4: pme_eval_p<4, T>(c, q, force, ev, s, at_fork); break;
        case 5: pme_eval_p<5, T>(c, q, force, ev, s, at_fork); break;
        case 6: pme_eval_p<6, T>(c, q, force, ev, s, at_fork); break;
        case 7: pme_eval_p<7, T>(c, q, force, ev, s, at_fork); break;
        case 8: pme_eval_p<8, T>(c, q, force, ev, s, at_fork); break;
        default: throw Error(PQ_ERR_INVALID, "spline order must be in 3..8");
    }
}

void pme_eval(Ctx& c, const double* q, bool force, hipEvent_t* ev, hipStream_t s,
              const std::function<void()>& at_fork) {
    if (c.fp64)
        pme_eval_t<double>(c, q, force, ev, s, at_fork);
    else
        pme_eval_t<float>(c, q, force, ev, s, at_fork);
}

}  // namespace pq
