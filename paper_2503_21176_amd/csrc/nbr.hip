// Cell (column) sort, cluster build and cluster-pair neighbour list.
//
// Section "Cell based Neighbor List" of the paper bins atoms into cells of
// about the cutoff size and searches neighbouring cells under periodic
// boundaries. Here the cells are x-y columns sized so that 8 consecutive
// z-sorted atoms of a column form a compact cluster; the list holds pairs of
// clusters (i-cluster, j-cluster, image vector n) whose bounding boxes are
// closer than the list radius, which is what the wave64 pair kernel consumes
// (8 i-atoms x 8 j-atoms per wavefront step). Every periodic image is
// enumerated, so boxes shorter than twice the cutoff are handled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dev.h"
#include "pq_internal.h"

namespace pq {

__global__ void k_fill_int(int* __restrict__ a, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Canonical wrap of atom i into the cell (stored in w64) and its column: x-y
// columns of the box, or of the fractional coordinates (s0, s1) of a
// triclinic cell. A non-finite position raises the flag and is placed at 0.
__device__ __forceinline__ int wrap_column(int i, const double* __restrict__ pos, const Geom& g,
                                           double* __restrict__ w64, int* __restrict__ flag) {
    double w[3];
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
        w[d] = pos[3 * (size_t)i + d];
        ok = ok && isfinite(w[d]);
    }
    if (!ok) {
        atomicOr(flag, 1);
        w[0] = w[1] = w[2] = 0.0;
    }
    int cx, cy;
    if (g.tric) {
        canon_wrap_tric(w[0], w[1], w[2], g.L, g.invL, g.t);
        double s0, s1, s2;
        frac_tric(w[0], w[1], w[2], g.invL, g.t, s0, s1, s2);
        cx = (int)floor(s0 * (double)g.ncx);
        cy = (int)floor(s1 * (double)g.ncy);
    } else {
        for (int d = 0; d < 3; ++d) w[d] = canon_wrap(w[d], g.L[d], g.invL[d]);
        cx = (int)floor(w[0] * ((double)g.ncx * g.invL[0]));
        cy = (int)floor(w[1] * ((double)g.ncy * g.invL[1]));
    }
    for (int d = 0; d < 3; ++d) w64[3 * (size_t)i + d] = w[d];
    cx = min(max(cx, 0), g.ncx - 1);
    cy = min(max(cy, 0), g.ncy - 1);
    return cx + g.ncx * cy;
}

// Wrap positions into the box, pick each atom's column, count per column.
__global__ void k_wrap_count(int n, const double* __restrict__ pos, Geom g, double* __restrict__ w64,
                             int* __restrict__ col_of, int* __restrict__ col_cnt, int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = wrap_column(i, pos, g, w64, flag);
    col_of[i] = c;
    atomicAdd(&col_cnt[c], 1);
}

// Exclusive scan of a small integer array by one workgroup (OP 1: scan of
// ceil(x/8)). out[n] receives the total.
template <int OP>
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ in, int* __restrict__ out, int n) {
    __shared__ int buf[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        int i = base + t;
        int v = 0;
        if (i < n) v = (OP == 1) ? (in[i] + CL - 1) / CL : in[i];
        buf[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int x = (t >= off) ? buf[t - off] : 0;
            __syncthreads();
            buf[t] += x;
            __syncthreads();
        }
        if (i < n) out[i] = carry + buf[t] - v;
        __syncthreads();
        if (t == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (t == 0) out[n] = carry;
}

// Wavefront-wide inclusive prefix sum.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan over several workgroups for long arrays: SCAN_BLOCK values
// per workgroup; k_scan_part sums each block, k_scan_apply adds the sums of the
// blocks before its own (read directly, they are few) to a scan of its block.
constexpr int SCAN_BLOCK = 4096;   // 1024 threads x 4 consecutive values
template <int OP>
__device__ __forceinline__ int scan_val(const int* __restrict__ in, int i, int n) {
    if (i >= n) return 0;
    return (OP == 1) ? (in[i] + CL - 1) / CL : in[i];
}
__device__ __forceinline__ int block_sum_int(int v, int* lds /* 16 */) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < 16; ++w) t += lds[w];
    __syncthreads();
    return t;
}
template <int OP>
__global__ __launch_bounds__(1024) void k_scan_part(const int* __restrict__ in, int n, int* __restrict__ part) {
    __shared__ int lds[16];
    const int b0 = blockIdx.x * SCAN_BLOCK + 4 * threadIdx.x;
    int v = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) v += scan_val<OP>(in, b0 + r, n);
    v = block_sum_int(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}
template <int OP>
__global__ __launch_bounds__(1024) void k_scan_apply(const int* __restrict__ in, int* __restrict__ out, int n,
                                                     const int* __restrict__ part) {
    __shared__ int lds[16];
    __shared__ int wtot[16];
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    int off = 0;
    for (int k = t; k < (int)blockIdx.x; k += 1024) off += part[k];
    off = block_sum_int(off, lds);
    const int b0 = blockIdx.x * SCAN_BLOCK + 4 * t;
    int v[4], sum = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v[r] = scan_val<OP>(in, b0 + r, n);
        sum += v[r];
    }
    const int incl = wave_incl_scan(sum);
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int before = off;
    for (int k = 0; k < w; ++k) before += wtot[k];
    int run = before + incl - sum;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (b0 + r < n) out[b0 + r] = run;
        run += v[r];
    }
    if (blockIdx.x == gridDim.x - 1 && t == 1023) out[n] = run;
}

__global__ void k_bin(int n, const int* __restrict__ col_of, const int* __restrict__ col_start,
                      int* __restrict__ col_fill, int* __restrict__ tmp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = col_of[i];
    tmp[col_start[c] + atomicAdd(&col_fill[c], 1)] = i;
}

// Column binning without global atomics: workgroup w takes atoms
// [w per, (w + 1) per), counts them per column in LDS and stores its counts
// column-major, hist[c nwg + w]; an exclusive scan of hist then gives each
// workgroup its first slot in every column, where k_bin_hist places its atoms
// (LDS cursors). The order inside a column is settled by k_rank_col.
constexpr int BIN_LDS_COLS = 16384;   // columns that fit the LDS counters
__global__ __launch_bounds__(256) void k_wrap_hist(int n, int per, const double* __restrict__ pos, Geom g,
                                                   double* __restrict__ w64, int* __restrict__ col_of,
                                                   int* __restrict__ hist, int* __restrict__ flag) {
    extern __shared__ int cntl[];
    const int ncol = g.ncx * g.ncy;
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) cntl[c] = 0;
    __syncthreads();
    const int a0 = blockIdx.x * per, a1 = min(n, a0 + per);
    for (int i = a0 + threadIdx.x; i < a1; i += blockDim.x) {
        const int c = wrap_column(i, pos, g, w64, flag);
        col_of[i] = c;
        atomicAdd(&cntl[c], 1);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) hist[(size_t)c * gridDim.x + blockIdx.x] = cntl[c];
}

// Column starts and counts from the scanned per-workgroup histogram.
__global__ void k_col_from_hist(int ncol, int nwg, const int* __restrict__ hscan, int* __restrict__ col_start,
                                int* __restrict__ col_cnt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncol) return;
    const int a = hscan[(size_t)c * nwg];
    col_start[c] = a;
    if (c < ncol) col_cnt[c] = hscan[(size_t)(c + 1) * nwg] - a;
}

__global__ __launch_bounds__(256) void k_bin_hist(int n, int per, int ncol, const int* __restrict__ col_of,
                                                  const int* __restrict__ hscan, int* __restrict__ tmp) {
    extern __shared__ int cur[];
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) cur[c] = hscan[(size_t)c * gridDim.x + blockIdx.x];
    __syncthreads();
    const int a0 = blockIdx.x * per, a1 = min(n, a0 + per);
    for (int i = a0 + threadIdx.x; i < a1; i += blockDim.x) tmp[atomicAdd(&cur[col_of[i]], 1)] = i;
}

// Rank of each atom inside its column by (z, index), a deterministic sort:
// one workgroup per column stages the column's (z, index) keys in LDS (padded
// to a multiple of 8 with keys that rank below nobody) and every atom counts
// the keys below its own there, 8 keys per step (512 threads: one pass for
// columns of up to 512 atoms). Columns longer than RANK_CAP atoms count from
// global memory instead.
constexpr int RANK_CAP = 2048;   // a multiple of 8
__global__ __launch_bounds__(512) void k_rank_col(int ncol, const int* __restrict__ col_start,
                                                  const int* __restrict__ col_cl, const int* __restrict__ tmp,
                                                  const double* __restrict__ w64, int* __restrict__ orig) {
    __shared__ double sz[RANK_CAP];
    __shared__ int si[RANK_CAP];
    const int c = blockIdx.x;
    if (c >= ncol) return;
    const int k0 = col_start[c], m = col_start[c + 1] - k0;
    int* __restrict__ dst = orig + (size_t)col_cl[c] * CL;
    if (m > RANK_CAP) {
        for (int t = threadIdx.x; t < m; t += blockDim.x) {
            const int i = tmp[k0 + t];
            const double zi = w64[3 * (size_t)i + 2];
            int r = 0;
            for (int u = 0; u < m; ++u) {
                const int j = tmp[k0 + u];
                const double zj = w64[3 * (size_t)j + 2];
                r += (zj < zi) || (zj == zi && j < i);
            }
            dst[r] = i;
        }
        return;
    }
    const int m8 = (m + 7) & ~7;
    for (int t = threadIdx.x; t < m8; t += blockDim.x) {
        int j = 0x7fffffff;
        double z = __builtin_inf();
        if (t < m) {
            j = tmp[k0 + t];
            z = w64[3 * (size_t)j + 2];
        }
        si[t] = j;
        sz[t] = z;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int i = si[t];
        const double zi = sz[t];
        int r = 0;
        for (int u = 0; u < m8; u += 8) {
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const double zj = sz[u + v];
                const int j = si[u + v];
                r += (zj < zi) || (zj == zi && j < i);
            }
        }
        dst[r] = i;
    }
}

__global__ void k_cluster_col(int ncol, const int* __restrict__ col_cl, int* __restrict__ cl_col) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    for (int k = col_cl[c]; k < col_cl[c + 1]; ++k) cl_col[k] = c;
}

// Bounding box, reference point and offsets (bulk precision T) of each cluster;
// cpos: the wrapped FP64 positions in slot order (w = 1, padding w = 0).
template <class T>
__global__ void k_cluster(int ncl, const int* __restrict__ orig, const double* __restrict__ w64,
                          double* __restrict__ ref, double* __restrict__ lo, double* __restrict__ hi,
                          V4<T>* __restrict__ xyzq, double4* __restrict__ cpos) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncl) return;
    double l[3] = {1e300, 1e300, 1e300}, h[3] = {-1e300, -1e300, -1e300};
    for (int a = 0; a < CL; ++a) {
        int i = orig[(size_t)c * CL + a];
        if (i < 0) continue;
        for (int d = 0; d < 3; ++d) {
            double w = w64[3 * (size_t)i + d];
            l[d] = fmin(l[d], w);
            h[d] = fmax(h[d], w);
        }
    }
    double r[3];
    for (int d = 0; d < 3; ++d) {
        r[d] = 0.5 * (l[d] + h[d]);
        ref[3 * (size_t)c + d] = r[d];
        lo[3 * (size_t)c + d] = l[d];
        hi[3 * (size_t)c + d] = h[d];
    }
    for (int a = 0; a < CL; ++a) {
        size_t s = (size_t)c * CL + a;
        int i = orig[s];
        V4<T> v;
        double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
        if (i >= 0) {
            p = make_double4(w64[3 * (size_t)i + 0], w64[3 * (size_t)i + 1], w64[3 * (size_t)i + 2], 1.0);
            v.x = (T)(p.x - r[0]);
            v.y = (T)(p.y - r[1]);
            v.z = (T)(p.z - r[2]);
        } else {
            // padding: far from everything, zero charge
            v.x = v.y = v.z = (T)1.0e4;
        }
        v.w = (T)0;
        xyzq[s] = v;
        cpos[s] = p;
    }
}

__device__ __forceinline__ double gap1(double lo_j, double hi_j, double lo_i, double hi_i) {
    return fmax(0.0, fmax(lo_j - hi_i, lo_i - hi_j));
}

// z window of the clusters of each column. Within a column both the lowest
// and the highest z of a cluster grow with the cluster index (clusters are
// runs of 8 atoms in z order), so for bin edges z_t = t bw, t = 0..nbin:
//   zta[c][t] = first cluster j of column c with hi_z(j) > z_t (t = 0: the first),
//   ztb[c][t] = first cluster j with lo_z(j) >= z_t (t = nbin: one past the last).
// Clusters that reach into a window (zlo, zhi) then lie in
// [zta[c][t0], ztb[c][t1]) for any t0 with z_t0 < zlo and t1 with z_t1 > zhi.
__global__ void k_ztab(int ncol, int nbin, double bw, const int* __restrict__ col_cl, const double* __restrict__ lo,
                       const double* __restrict__ hi, int* __restrict__ zta, int* __restrict__ ztb) {
    const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (idx >= (size_t)ncol * (nbin + 1)) return;
    const int c = (int)(idx / (nbin + 1)), t = (int)(idx % (nbin + 1));
    const int j0 = col_cl[c], j1 = col_cl[c + 1];
    const double z = (double)t * bw;
    int a = j0;
    if (t > 0) {
        int l = j0, h = j1;
        while (l < h) {
            const int m = (l + h) >> 1;
            if (hi[3 * (size_t)m + 2] > z) h = m; else l = m + 1;
        }
        a = l;
    }
    int b = j1;
    if (t < nbin) {
        int l = j0, h = j1;
        while (l < h) {
            const int m = (l + h) >> 1;
            if (lo[3 * (size_t)m + 2] >= z) h = m; else l = m + 1;
        }
        b = l;
    }
    zta[idx] = a;
    ztb[idx] = b;
}

// Cluster-pair list: one wavefront per i-cluster. For each z image whose
// window (the i-cluster's z range widened by the list radius) can hold
// clusters, the candidate columns (the periodic (2Rx+1) x (2Ry+1)
// neighbourhood, dy-major) are taken 64 at a time, one per lane: a column
// whose x-y strip lies beyond the list radius drops out, the others look up
// their clusters in the window (k_ztab) and put them into one flat sequence
// that the wavefront walks 64 clusters per step with the bounding-box test.
// Every cluster the test accepts lies in its column's window, so the list is
// the same as from testing whole columns. LIST_UNROLL steps load their
// cluster bounds before any is tested, so that their latencies overlap. The
// entries of i-cluster ic go to lj[ic * cap + k] in a deterministic order
// (z image, flat position); those with k >= cap are counted but not written
// (cap = 0: count only).
constexpr int LIST_UNROLL = 4;
__global__ __launch_bounds__(256) void k_list(int ncl, Geom g, const int* __restrict__ cl_col,
                                              const int* __restrict__ zta, const int* __restrict__ ztb, int nbin,
                                              double bw, const double* __restrict__ lo,
                                              const double* __restrict__ hi, int* __restrict__ lcount, int cap,
                                              int2* __restrict__ lj) {
    const int lane = lane_id();
    const int ic = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ic >= ncl) return;
    const double rl2 = g.rlist * g.rlist * (1.0 + 1e-9) + 1e-12;
    const double zr = sqrt(rl2) * (1.0 + 1e-9) + 1e-9;   // above every z gap the box test accepts
    const double eps = 1e-6;
    const int coli = cl_col[ic];
    const int cxi = coli % g.ncx, cyi = coli / g.ncx;
    const double loi0 = lo[3 * ic], loi1 = lo[3 * ic + 1], loi2 = lo[3 * ic + 2];
    const double hii0 = hi[3 * ic], hii1 = hi[3 * ic + 1], hii2 = hi[3 * ic + 2];
    const int nxc = 2 * g.Rx + 1, ncand = nxc * (2 * g.Ry + 1);
    int cnt = 0;
    int2* __restrict__ out = lj + (size_t)ic * cap;
    for (int nz = -g.Rz; nz <= g.Rz; ++nz) {
        const double sz = (double)nz * g.L[2];
        const double zlo = loi2 - zr - sz, zhi = hii2 + zr - sz;
        // wrapped z lies within a rounding error of [0, L]
        if (zhi <= -bw || zlo >= g.L[2] + bw) continue;
        const int t0 = (int)fmin(fmax(floor(zlo / bw) - 1.0, 0.0), (double)nbin);
        const int t1 = (int)fmin(fmax(floor(zhi / bw) + 2.0, 0.0), (double)nbin);
        for (int cb = 0; cb < ncand; cb += 64) {
            // this lane's candidate column: clusters [ja, ja + nc) and image (nx, ny, nz)
            const int k = cb + lane;
            int ja = 0, nc = 0, img = 0;
            if (k < ncand) {
                const int dy = k / nxc - g.Ry, dx = k % nxc - g.Rx;
                const int cy = cyi + dy;
                const int ny = (cy >= 0) ? cy / g.ncy : -((-cy + g.ncy - 1) / g.ncy);
                const int cyw = cy - ny * g.ncy;
                const int cx = cxi + dx;
                const int nx = (cx >= 0) ? cx / g.ncx : -((-cx + g.ncx - 1) / g.ncx);
                const int cxw = cx - nx * g.ncx;
                // strip test of the column's x and y extent (orthorhombic; a
                // triclinic column is a slanted prism and takes the box test only)
                bool near = true;
                if (!g.tric) {
                    const double sy = (double)ny * g.L[1];
                    const double gy = gap1(cyw * g.wy + sy, (cyw + 1) * g.wy + sy, loi1, hii1) - eps;
                    const double sx = (double)nx * g.L[0];
                    const double gx = gap1(cxw * g.wx + sx, (cxw + 1) * g.wx + sx, loi0, hii0) - eps;
                    near = !(gy > 0.0 && gy * gy >= rl2) && !(gx > 0.0 && gx * gx >= rl2);
                }
                if (near) {
                    const size_t row = (size_t)(cxw + g.ncx * cyw) * (nbin + 1);
                    ja = zta[row + t0];
                    nc = max(0, ztb[row + t1] - ja);
                    img = pack_img(nx, ny, nz);
                }
            }
            const int incl = wave_incl_scan(nc);
            const int total = __shfl(incl, 63, 64);
            const int jofs = ja - (incl - nc);   // cluster = flat position + jofs of the owning lane
            for (int fb = 0; fb < total; fb += 64 * LIST_UNROLL) {
                int jc[LIST_UNROLL], im[LIST_UNROLL];
                double l0[LIST_UNROLL], l1[LIST_UNROLL], l2[LIST_UNROLL];
                double h0[LIST_UNROLL], h1[LIST_UNROLL], h2[LIST_UNROLL];
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    const int f = fb + 64 * u + lane;
                    // owner: the first lane whose inclusive count exceeds f
                    int o = 0;
#pragma unroll
                    for (int st = 32; st >= 1; st >>= 1)
                        if (__shfl(incl, o + st - 1, 64) <= f) o += st;
                    jc[u] = f + __shfl(jofs, o, 64);
                    im[u] = __shfl(img, o, 64);
                    l0[u] = l1[u] = l2[u] = h0[u] = h1[u] = h2[u] = 0.0;
                    if (f < total) {
                        l0[u] = lo[3 * jc[u]];
                        l1[u] = lo[3 * jc[u] + 1];
                        l2[u] = lo[3 * jc[u] + 2];
                        h0[u] = hi[3 * jc[u]];
                        h1[u] = hi[3 * jc[u] + 1];
                        h2[u] = hi[3 * jc[u] + 2];
                    }
                }
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    if (fb + 64 * u >= total) break;
                    const bool valid = fb + 64 * u + lane < total;
                    int nx, ny, nzz;
                    unpack_img(im[u], nx, ny, nzz);
                    double sx, sy, szz;
                    lattice_vec(nx, ny, nzz, g.L, g.t, sx, sy, szz);
                    const double gxx = gap1(l0[u] + sx, h0[u] + sx, loi0, hii0);
                    const double gyy = gap1(l1[u] + sy, h1[u] + sy, loi1, hii1);
                    const double gz = gap1(l2[u] + sz, h2[u] + sz, loi2, hii2);
                    const bool pass = valid && (gxx * gxx + gyy * gyy + gz * gz < rl2);
                    const unsigned long long m = __ballot(pass);
                    const int kk = cnt + lanes_below(m);
                    if (pass && kk < cap) out[kk] = make_int2(jc[u], im[u]);
                    cnt += __popcll(m);
                }
            }
        }
    }
    if (lane == 0) lcount[ic] = cnt;
}

// Largest of n integers (n >= 0; 0 for n == 0), one workgroup.
__global__ __launch_bounds__(1024) void k_max_int(const int* __restrict__ a, int n, int* __restrict__ out) {
    __shared__ int lds[16];
    int v = 0;
    for (int i = threadIdx.x; i < n; i += 1024) v = max(v, a[i]);
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) v = max(v, lds[w]);
        out[0] = v;
    }
}

// Atom-level j list of each i-cluster, derived from its cluster-pair list: the
// atoms of the listed j-clusters, at the entry's periodic image, that are
// within the cutoff of at least one atom of the i-cluster, decided pair by
// pair with the canonical FP64 predicate (d^2 < rc^2, d^2 > 0). Entries are
// V4<T>: x, y, z of the image relative to the i-cluster's reference point
// (rounded once from FP64) and a packed word, j slot | colmask << JL_SLOT_BITS,
// where bit a of colmask says that i-atom a and this entry are a pair. Entries
// are grouped in rows of 8; the last row is padded with atoms far outside any
// cutoff (mask 0). About 60 % of the 8 x 8 candidates of a row are pairs at
// liquid-like densities (~50 % with a bounding-box test, ~29 % for whole
// cluster pairs).
// Order: the list order is spatial (column by column), so taken as it is one
// i-atom collects its pairs faster than another for long stretches, and the
// pair kernel's compute rounds run part-empty. The R rows of a cluster (runs
// of 8 consecutive list entries, which keeps the charge loads of a row on few
// cache lines) are therefore stored in a golden-ratio stride permutation
// (position p holds row (p S) mod R, S ~ 0.618 R, gcd(S, R) = 1), which
// spreads every stretch of the list over the whole walk: with it ~92 % of the
// compute lanes are busy against ~79 % in list order.
// FILL = false decides every candidate, stores its colmask (one byte per
// cluster-pair entry and j atom, at jmask[8 e + b]) and counts rows; FILL =
// true reads those bytes back and writes the entries.
__device__ __forceinline__ long long gcd_ll(long long a, long long b) {
    while (b != 0) {
        const long long t = a % b;
        a = b;
        b = t;
    }
    return a;
}
// x with (s x) mod n == 1, for gcd(s, n) == 1 and n >= 2
__device__ __forceinline__ long long inv_mod(long long s, long long n) {
    long long r0 = n, r1 = s % n, t0 = 0, t1 = 1;
    while (r1 != 0) {
        const long long qq = r0 / r1;
        long long t = r0 - qq * r1;
        r0 = r1;
        r1 = t;
        t = t0 - qq * t1;
        t0 = t1;
        t1 = t;
    }
    return t0 < 0 ? t0 + n : t0;
}

// cw, kimg (both NULL after a full build): a list kept across moves
// (nbr_refresh). Then cpos holds the continuous positions x = w + k L since
// the build (entry positions), cw the canonical wrap w of the current
// positions and kimg the lattice steps k between the two, and the pair
// (i, j) of a cluster pair with image n has the canonical image
// n + k_j - k_i, on which the FP64 predicate decides.
template <bool FILL, class T>
__global__ __launch_bounds__(256) void k_jlist(int ncl, Geom g, const int* __restrict__ lcount, int lcap,
                                               const int2* __restrict__ lj, const double4* __restrict__ cpos,
                                               const double4* __restrict__ cw, const int4* __restrict__ kimg,
                                               const double* __restrict__ ref, unsigned char* __restrict__ jmask,
                                               int* __restrict__ jcount, const int* __restrict__ jstart,
                                               V4<T>* __restrict__ jl) {
    const int lane = lane_id();
    const int ic = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (ic >= ncl) return;
    const double rc2 = g.rc * g.rc;
    const bool moved = kimg != nullptr;
    // the i-cluster's atoms (the same in every lane)
    bool ireal[CL];
    double wi[CL][3];
    int ki[CL][3];
    if (!FILL) {
#pragma unroll
        for (int a = 0; a < CL; ++a) {
            const double4 p = (moved ? cw : cpos)[(size_t)ic * CL + a];
            ireal[a] = p.w != 0.0;
            wi[a][0] = p.x;
            wi[a][1] = p.y;
            wi[a][2] = p.z;
            const int4 k = moved ? kimg[(size_t)ic * CL + a] : make_int4(0, 0, 0, 0);
            ki[a][0] = k.x;
            ki[a][1] = k.y;
            ki[a][2] = k.z;
        }
    }
    const double r0 = ref[3 * ic], r1 = ref[3 * ic + 1], r2 = ref[3 * ic + 2];
    const size_t e0 = (size_t)ic * lcap, e1 = e0 + min(lcount[ic], lcap);
    const int eo = lane >> 3, b = lane & 7;
    const size_t base = FILL ? (size_t)jstart[ic] * CL : 0;
    // row r of list order is stored at row (r * sinv) mod nrow
    long long nrow = 1, sinv = 1;
    if (FILL) {
        nrow = jcount[ic];
        if (nrow > 2) {
            long long st = (long long)((double)nrow * 0.6180339887498949 + 0.5);
            while (gcd_ll(st, nrow) != 1) ++st;
            sinv = inv_mod(st, nrow);
        }
    }
    auto dest = [&](long long k) -> size_t { return base + (size_t)(((k >> 3) * sinv) % nrow) * CL + (k & 7); };
    // two-stage load pipeline: the list entry (and stored mask) of step s + 2
    // and the j position of step s + 1 are in flight while step s is handled;
    // the fill pass loads positions only where the mask is not empty
    auto entry = [&](size_t eb, int& msk) -> int2 {
        const size_t e = eb + eo;
        msk = 0;
        if (e >= e1) return make_int2(-1, 0);
        if (FILL) msk = jmask[8 * e + b];
        return lj[e];
    };
    auto jpos = [&](int2 je, int msk) -> double4 {
        return (je.x >= 0 && (!FILL || msk != 0)) ? cpos[(size_t)je.x * CL + b] : make_double4(0.0, 0.0, 0.0, 0.0);
    };
    int m1, m2;
    int2 je1 = entry(e0, m1);
    double4 p1 = jpos(je1, m1);
    int2 je2 = entry(e0 + 8, m2);
    int cnt = 0;
    for (size_t eb = e0; eb < e1; eb += 8) {
        const int2 je = je1;
        const double4 pj = p1;
        int col = m1;
        je1 = je2;
        m1 = m2;
        p1 = jpos(je1, m1);
        je2 = entry(eb + 16, m2);
        double p0 = 0.0, pp1 = 0.0, p2 = 0.0;
        if (pj.w != 0.0) {
            int n0, n1, n2;
            unpack_img(je.y, n0, n1, n2);
            double sx, sy, sz;
            lattice_vec(n0, n1, n2, g.L, g.t, sx, sy, sz);
            if (!FILL) {
                if (moved) {
                    const size_t js = (size_t)je.x * CL + b;
                    const double4 w4 = cw[js];
                    const int4 kj = kimg[js];
                    const double wj[3] = {w4.x, w4.y, w4.z};
#pragma unroll
                    for (int a = 0; a < CL; ++a) {
                        double tx, ty, tz;
                        lattice_vec(n0 + kj.x - ki[a][0], n1 + kj.y - ki[a][1], n2 + kj.z - ki[a][2], g.L, g.t, tx,
                                    ty, tz);
                        const double d2 = canon_d2s(wi[a], wj, tx, ty, tz);
                        if (ireal[a] && d2 > 0.0 && d2 < rc2) col |= 1 << a;
                    }
                } else {
                    const double wj[3] = {pj.x, pj.y, pj.z};
#pragma unroll
                    for (int a = 0; a < CL; ++a) {
                        const double d2 = canon_d2s(wi[a], wj, sx, sy, sz);
                        if (ireal[a] && d2 > 0.0 && d2 < rc2) col |= 1 << a;
                    }
                }
            }
            p0 = pj.x + sx;
            pp1 = pj.y + sy;
            p2 = pj.z + sz;
        }
        if (!FILL && eb + eo < e1) jmask[8 * (eb + eo) + b] = (unsigned char)col;
        const bool pass = col != 0;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(pass);
        if (FILL && pass) {
            jl[dest(cnt + lanes_below(m))] = mk4<T>((T)(p0 - r0), (T)(pp1 - r1), (T)(p2 - r2),
                                                    pack_int((je.x * CL + b) | (col << JL_SLOT_BITS), T(0)));
        }
        cnt += __popcll(m);
    }
    const int rows = (cnt + CL - 1) / CL;
    if (!FILL) {
        if (lane == 0) jcount[ic] = rows;
    } else {
        for (int k = cnt + lane; k < rows * CL; k += 64)
            jl[dest(k)] = mk4<T>((T)-1.0e4, (T)-1.0e4, (T)-1.0e4, pack_int(0, T(0)));
    }
}

template <class T>
__global__ void k_far_entries(V4<T>* __restrict__ out, int n) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) out[k] = mk4<T>((T)-1.0e4, (T)-1.0e4, (T)-1.0e4, pack_int(0, T(0)));
}

// Entry e of an i-cluster's list seen from lane (a, b): the pair (i, j, n) of
// i-atom i (canonical position wi, lattice steps ki) and the entry's atom b.
// True when it is a pair closer than sqrt(rl2) by the canonical FP64
// predicate; with half, only if listed once (i < j, or i == j with n
// lexicographically positive), else for every (j, n) != (i, 0) (each i-atom's
// list holds all its neighbours). With kimg (a list kept across moves, see
// k_jlist) the positions are the canonical wraps and the image of a pair is
// n + k_j - k_i.
__device__ __forceinline__ bool export_pair(const Geom& g, const int2* __restrict__ lj, const int* __restrict__ orig,
                                            const double4* __restrict__ cpos, const int4* __restrict__ kimg, int i,
                                            const double wi[3], int4 ki, double rl2, int b, size_t e, int& j, int& n0,
                                            int& n1, int& n2, bool half = true) {
    const int2 je = lj[e];
    const size_t slot = (size_t)je.x * CL + b;
    j = orig[slot];
    const double4 pj = cpos[slot];
    unpack_img(je.y, n0, n1, n2);
    if (kimg) {
        const int4 kj = kimg[slot];
        n0 += kj.x - ki.x;
        n1 += kj.y - ki.y;
        n2 += kj.z - ki.z;
    }
    bool ok = (i >= 0) && (j >= 0) &&
              (half ? ((i < j) || (i == j && lex_positive(n0, n1, n2))) : (i != j || n0 != 0 || n1 != 0 || n2 != 0));
    if (ok) {
        const double wj[3] = {pj.x, pj.y, pj.z};
        double sx, sy, sz;
        lattice_vec(n0, n1, n2, g.L, g.t, sx, sy, sz);
        ok = canon_d2s(wi, wj, sx, sy, sz) < rl2;
    }
    return ok;
}

// Export of the atom pairs closer than the list radius, by the canonical FP64
// predicate; each unordered pair once. A wavefront counts its i-cluster's
// pairs, reserves that many rows with one atomic on the global counter and,
// when `out` is given, walks the list again to write them; rows beyond `cap`
// are not written but still counted. With kimg the radius is the cutoff (the
// kept list covers the pairs closer than rc, not rc + skin).
__global__ __launch_bounds__(256) void k_export(int ncl, Geom g, const int* __restrict__ lcount, int lcap,
                                                const int2* __restrict__ lj, const int* __restrict__ orig,
                                                const double4* __restrict__ cpos, const int4* __restrict__ kimg,
                                                int64_t cap, int32_t* __restrict__ out,
                                                unsigned long long* __restrict__ counter) {
    const int lane = lane_id();
    const int ic = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ic >= ncl) return;
    const int a = lane >> 3, b = lane & 7;
    const int i = orig[(size_t)ic * CL + a];
    const double4 pi4 = cpos[(size_t)ic * CL + a];
    const int4 ki = kimg ? kimg[(size_t)ic * CL + a] : make_int4(0, 0, 0, 0);
    const double wi[3] = {pi4.x, pi4.y, pi4.z};
    const double rl = kimg ? g.rc : g.rlist;
    const double rl2 = rl * rl;
    const size_t e0 = (size_t)ic * lcap, e1 = e0 + min(lcount[ic], lcap);
    unsigned long long cnt = 0;
    for (size_t e = e0; e < e1; ++e) {
        int j, n0, n1, n2;
        cnt += __popcll(__ballot(export_pair(g, lj, orig, cpos, kimg, i, wi, ki, rl2, b, e, j, n0, n1, n2)));
    }
    if (cnt == 0) return;
    unsigned long long pos = 0;
    if (lane == 0) pos = atomicAdd(counter, cnt);
    pos = __shfl(pos, 0, 64);
    if (!out) return;
    for (size_t e = e0; e < e1; ++e) {
        int j, n0, n1, n2;
        const bool ok = export_pair(g, lj, orig, cpos, kimg, i, wi, ki, rl2, b, e, j, n0, n1, n2);
        const unsigned long long m = __ballot(ok);
        if (ok) {
            const unsigned long long k = pos + lanes_below(m);
            if ((int64_t)k < cap) {
                int32_t* r = out + 5 * k;
                r[0] = i;
                r[1] = j;
                r[2] = n0;
                r[3] = n1;
                r[4] = n2;
            }
        }
        pos += __popcll(m);
    }
}

// ELLPACK key of neighbour (j, n) in a row: j in the high word, the image
// components biased by 512 in three 10-bit fields below, so that ascending
// keys are ascending (j, n0, n1, n2).
__device__ __forceinline__ unsigned long long ell_key(int j, int n0, int n1, int n2) {
    return ((unsigned long long)(unsigned)j << 32) |
           (unsigned long long)(((unsigned)(n0 + 512) << 20) | ((unsigned)(n1 + 512) << 10) | (unsigned)(n2 + 512));
}

// ELLPACK rows from each i-cluster's own list, which holds every neighbour
// (j, n) of each of its atoms, so rows are counted and filled without
// atomics: FILL = false stores each atom's row count, FILL = true its keys in
// list order at row-major n x K (a lane's place from the ballot of its
// i-atom's eight lanes; the caller has checked K against the counts);
// k_ell_sort orders each row afterwards.
template <bool FILL>
__global__ __launch_bounds__(256) void k_ell(int ncl, Geom g, const int* __restrict__ lcount, int lcap,
                                             const int2* __restrict__ lj, const int* __restrict__ orig,
                                             const double4* __restrict__ cpos, const int4* __restrict__ kimg,
                                             int* __restrict__ rowcnt, int K, unsigned long long* __restrict__ keys) {
    const int lane = lane_id();
    const int ic = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ic >= ncl) return;
    const int a = lane >> 3, b = lane & 7;
    const int i = orig[(size_t)ic * CL + a];
    const double4 pi4 = cpos[(size_t)ic * CL + a];
    const int4 ki = kimg ? kimg[(size_t)ic * CL + a] : make_int4(0, 0, 0, 0);
    const double wi[3] = {pi4.x, pi4.y, pi4.z};
    const double rl = kimg ? g.rc : g.rlist;
    const double rl2 = rl * rl;
    const size_t e0 = (size_t)ic * lcap, e1 = e0 + min(lcount[ic], lcap);
    const unsigned below = (1u << b) - 1u;
    int pos = 0;   // entries of i-atom a so far (the same in its eight lanes)
    for (size_t e = e0; e < e1; ++e) {
        int j, n0, n1, n2;
        const bool ok = export_pair(g, lj, orig, cpos, kimg, i, wi, ki, rl2, b, e, j, n0, n1, n2, false);
        const unsigned seg = (unsigned)(__ballot(ok) >> (8 * a)) & 0xffu;
        if (FILL && ok) keys[(size_t)i * K + pos + __popc(seg & below)] = ell_key(j, n0, n1, n2);
        pos += __popc(seg);
    }
    if (!FILL && b == 0 && i >= 0) rowcnt[i] = pos;
}

// One workgroup per row: the row's cnt keys are sorted ascending in LDS
// (bitonic network over the next power of two >= cnt, padded with the
// largest key) and written out as neighbour indices and image vectors, then
// -1 (index) and 0 (image) up to K.
__global__ __launch_bounds__(256) void k_ell_sort(int n, int K, const int* __restrict__ rowcnt,
                                                  const unsigned long long* __restrict__ keys,
                                                  int32_t* __restrict__ nbr, int32_t* __restrict__ img) {
    extern __shared__ unsigned long long sk[];
    const int row = blockIdx.x;
    const int cnt = rowcnt[row];
    int kp = 1;
    while (kp < cnt) kp <<= 1;
    const unsigned long long* src = keys + (size_t)row * K;
    for (int t = threadIdx.x; t < kp; t += blockDim.x) sk[t] = t < cnt ? src[t] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= kp; k <<= 1) {
        for (int h = k >> 1; h > 0; h >>= 1) {
            for (int t = threadIdx.x; t < kp; t += blockDim.x) {
                const int u = t ^ h;
                if (u > t) {
                    const unsigned long long x = sk[t], y = sk[u];
                    if (((t & k) == 0) == (x > y)) {
                        sk[t] = y;
                        sk[u] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < K; t += blockDim.x) {
        const size_t o = (size_t)row * K + t;
        int j = -1, n0 = 0, n1 = 0, n2 = 0;
        if (t < cnt) {
            const unsigned long long key = sk[t];
            j = (int)(key >> 32);
            const unsigned lo = (unsigned)key;
            n0 = (int)((lo >> 20) & 1023u) - 512;
            n1 = (int)((lo >> 10) & 1023u) - 512;
            n2 = (int)(lo & 1023u) - 512;
        }
        if (nbr) nbr[o] = j;
        if (img) {
            img[3 * o] = n0;
            img[3 * o + 1] = n1;
            img[3 * o + 2] = n2;
        }
    }
}

void scan_ints(Ctx& c, const int* in, int* out, int n, bool ceil8, hipStream_t s) {
    if (n <= SCAN_BLOCK) {
        if (ceil8)
            PQ_LAUNCH(k_scan<1>, 1, 1024, 0, s, in, out, n);
        else
            PQ_LAUNCH(k_scan<0>, 1, 1024, 0, s, in, out, n);
        return;
    }
    const int nb = cdiv(n, SCAN_BLOCK);
    c.scan_part.ensure(nb);
    if (ceil8) {
        PQ_LAUNCH(k_scan_part<1>, nb, 1024, 0, s, in, n, c.scan_part.p);
        PQ_LAUNCH(k_scan_apply<1>, nb, 1024, 0, s, in, out, n, c.scan_part.p);
    } else {
        PQ_LAUNCH(k_scan_part<0>, nb, 1024, 0, s, in, n, c.scan_part.p);
        PQ_LAUNCH(k_scan_apply<0>, nb, 1024, 0, s, in, out, n, c.scan_part.p);
    }
}

// ---------------------------------------------------------------------------
void nbr_build(Ctx& c, const double* pos) {
    const int n = (int)c.n;
    hipStream_t s = c.stream;
    Geom& g = c.g;
    const pq_params& p = c.prm;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = p.box[d];
        g.invL[d] = 1.0 / p.box[d];
    }
    g.rc = p.cutoff;
    g.rlist = p.cutoff + p.skin;
    g.tric = is_tric(p) ? 1 : 0;
    g.t = make_tric(p);
    // columns sized for ~8 atoms per cubic cluster
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double rho = (double)n / V;
    const double a = std::cbrt((double)CL / rho);
    // extent of the cell across its a and b faces: the edges, or for a
    // triclinic cell the distances V/|b x c| and V/|c x a| between opposite
    // faces (a pair within rlist differs by at most rlist/width in s_d)
    double wid0 = p.box[0], wid1 = p.box[1];
    if (g.tric) {
        const double bx = p.tilt[0], cx = p.tilt[1], cy = p.tilt[2];
        const double L0 = p.box[0], L1 = p.box[1], L2 = p.box[2];
        wid0 = V / std::sqrt((L1 * L2) * (L1 * L2) + (bx * L2) * (bx * L2) + (bx * cy - L1 * cx) * (bx * cy - L1 * cx));
        wid1 = V / (L0 * std::sqrt(L2 * L2 + cy * cy));
    }
    g.ncx = std::max(1, (int)std::lround(wid0 / a));
    g.ncy = std::max(1, (int)std::lround(wid1 / a));
    g.wx = wid0 / g.ncx;
    g.wy = wid1 / g.ncy;
    g.Rx = (int)std::floor((g.rlist + 1e-6) / g.wx) + 1;
    g.Ry = (int)std::floor((g.rlist + 1e-6) / g.wy) + 1;
    g.Rz = (int)std::floor(g.rlist / p.box[2]) + 1;
    c.ncol = g.ncx * g.ncy;
    PQ_REQUIRE(2 * g.Rx + 1 <= 511 && 2 * g.Ry + 1 <= 511 && g.Rz <= 255, PQ_ERR_BOX,
               "cutoff too large for the box (more than 255 periodic images)");

    c.w64.ensure((size_t)n * 3);
    c.col_of.ensure(n);
    c.col_cnt.ensure(c.ncol);
    c.col_fill.ensure(c.ncol);
    c.col_start.ensure(c.ncol + 1);
    c.col_cl.ensure(c.ncol + 1);
    c.tmp_atoms.ensure(n);
    c.flag.ensure(4);
    c.counter.ensure(1);

    PQ_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int) * 4, s));
    // binning by per-workgroup LDS histograms (global counters when the
    // columns do not fit in LDS)
    const bool hist = c.ncol <= BIN_LDS_COLS;
    const int nwg = std::max(1, std::min(256, (int)cdiv(n, 1024)));
    const int per = (int)cdiv(n, nwg);
    if (hist) {
        const size_t nh = (size_t)c.ncol * nwg;
        c.bin_hist.ensure(nh + 1);
        c.bin_scan.ensure(nh + 1);
        PQ_LAUNCH(k_wrap_hist, nwg, 256, sizeof(int) * c.ncol, s, n, per, pos, g, c.w64.p, c.col_of.p,
                  c.bin_hist.p, c.flag.p);
        scan_ints(c, c.bin_hist.p, c.bin_scan.p, (int)nh, false, s);
        PQ_LAUNCH(k_col_from_hist, cdiv(c.ncol + 1, 256), 256, 0, s, c.ncol, nwg, c.bin_scan.p, c.col_start.p,
                  c.col_cnt.p);
    } else {
        PQ_HIP(hipMemsetAsync(c.col_cnt.p, 0, sizeof(int) * c.ncol, s));
        PQ_HIP(hipMemsetAsync(c.col_fill.p, 0, sizeof(int) * c.ncol, s));
        PQ_LAUNCH(k_wrap_count, cdiv(n, 256), 256, 0, s, n, pos, g, c.w64.p, c.col_of.p, c.col_cnt.p, c.flag.p);
        scan_ints(c, c.col_cnt.p, c.col_start.p, c.ncol, false, s);
    }
    scan_ints(c, c.col_cnt.p, c.col_cl.p, c.ncol, true, s);
    // small read-backs go through the context's pinned host words
    int* hv = reinterpret_cast<int*>(c.pinned + 48);
    PQ_HIP(hipMemcpyAsync(&hv[0], c.col_cl.p + c.ncol, sizeof(int), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipMemcpyAsync(&hv[1], c.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    PQ_REQUIRE(hv[1] == 0, PQ_ERR_NAN, "non-finite position");
    c.ncl = hv[0];
    const int ncl = c.ncl;
    const size_t nslot = (size_t)ncl * CL;
    PQ_REQUIRE(nslot < ((size_t)1 << JL_SLOT_BITS), PQ_ERR_TOO_LARGE,
               "too many atoms for the packed j-list slot index (2^24 cluster slots)");
    c.orig.ensure(nslot);
    c.xyzq.ensure(nslot * 4 * rsz(c));
    c.cl_ref.ensure((size_t)ncl * 3);
    c.cl_pos.ensure(nslot);
    c.cl_lo.ensure((size_t)ncl * 3);
    c.cl_hi.ensure((size_t)ncl * 3);
    c.cl_col.ensure(ncl);
    c.lcount.ensure(ncl + 1);

    if (hist)
        PQ_LAUNCH(k_bin_hist, nwg, 256, sizeof(int) * c.ncol, s, n, per, c.ncol, c.col_of.p, c.bin_scan.p,
                  c.tmp_atoms.p);
    else
        PQ_LAUNCH(k_bin, cdiv(n, 256), 256, 0, s, n, c.col_of.p, c.col_start.p, c.col_fill.p, c.tmp_atoms.p);
    PQ_LAUNCH(k_fill_int, cdiv(nslot, 256), 256, 0, s, c.orig.p, (int)nslot, -1);
    PQ_LAUNCH(k_rank_col, c.ncol, 512, 0, s, c.ncol, c.col_start.p, c.col_cl.p, c.tmp_atoms.p, c.w64.p, c.orig.p);
    PQ_LAUNCH(k_cluster_col, cdiv(c.ncol, 256), 256, 0, s, c.ncol, c.col_cl.p, c.cl_col.p);
    if (c.fp64)
        PQ_LAUNCH(k_cluster<double>, cdiv(ncl, 256), 256, 0, s, ncl, c.orig.p, c.w64.p, c.cl_ref.p, c.cl_lo.p,
                  c.cl_hi.p, as<double4>(c.xyzq), c.cl_pos.p);
    else
        PQ_LAUNCH(k_cluster<float>, cdiv(ncl, 256), 256, 0, s, ncl, c.orig.p, c.w64.p, c.cl_ref.p, c.cl_lo.p,
                  c.cl_hi.p, as<float4>(c.xyzq), c.cl_pos.p);
    // cluster-pair list, one segment of lcap entries per i-cluster; lcap is
    // kept across builds and raised when a cluster has more entries (the pass
    // then runs again)
    // per-column z windows: bins of rlist/8 (at most 4096 over the box)
    const double bw = std::max(g.rlist / 8.0, p.box[2] / 4096.0);
    const int nbin = (int)std::ceil(p.box[2] / bw) + 1;
    const size_t nzt = (size_t)c.ncol * (nbin + 1);
    c.zta.ensure(nzt);
    c.ztb.ensure(nzt);
    PQ_LAUNCH(k_ztab, cdiv(nzt, 256), 256, 0, s, c.ncol, nbin, bw, c.col_cl.p, c.cl_lo.p, c.cl_hi.p, c.zta.p,
              c.ztb.p);
    // The capacity check rides on the read-back of the atom-list row count:
    // the atom-list count pass takes at most lcap entries per cluster, so an
    // overflowing build stays in bounds and is then repeated with the larger
    // capacity (a context's first build, or a denser system).
    c.jcount.ensure(ncl + 1);
    c.jstart.ensure(ncl + 1);
    for (int pass = 0;; ++pass) {
        c.lj.ensure(std::max<size_t>(1, (size_t)ncl * c.lcap));
        c.jmask.ensure(std::max<size_t>(1, (size_t)ncl * c.lcap * CL));
        PQ_LAUNCH(k_list, cdiv(ncl, 4), 256, 0, s, ncl, g, c.cl_col.p, c.zta.p, c.ztb.p, nbin, bw, c.cl_lo.p,
                  c.cl_hi.p, c.lcount.p, c.lcap, c.lj.p);
        PQ_LAUNCH(k_max_int, 1, 1024, 0, s, c.lcount.p, ncl, c.flag.p + 2);
        // atom-level j lists for the pair kernel: count pass
        if (c.fp64)
            PQ_LAUNCH((k_jlist<false, double>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lcount.p, c.lcap, c.lj.p,
                      c.cl_pos.p, (const double4*)nullptr, (const int4*)nullptr, c.cl_ref.p, c.jmask.p, c.jcount.p,
                      (const int*)nullptr, (double4*)nullptr);
        else
            PQ_LAUNCH((k_jlist<false, float>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lcount.p, c.lcap, c.lj.p,
                      c.cl_pos.p, (const double4*)nullptr, (const int4*)nullptr, c.cl_ref.p, c.jmask.p, c.jcount.p,
                      (const int*)nullptr, (float4*)nullptr);
        scan_ints(c, c.jcount.p, c.jstart.p, ncl, false, s);
        PQ_HIP(hipMemcpyAsync(&hv[2], c.flag.p + 2, sizeof(int), hipMemcpyDeviceToHost, s));
        PQ_HIP(hipMemcpyAsync(&hv[3], c.jstart.p + ncl, sizeof(int), hipMemcpyDeviceToHost, s));
        PQ_HIP(hipStreamSynchronize(s));
        const int mx = hv[2];
        if (mx <= c.lcap) break;
        PQ_REQUIRE(pass == 0, PQ_ERR_BOX, "cluster-pair list overflow");
        c.lcap = mx + mx / 8 + 8;
    }
    const int rows = hv[3];
    c.moved = false;
    jlist_fill(c, rows);
    // positions of this build, for the moves that keep the list
    if (p.skin > 0.0) {
        c.pos_build.ensure((size_t)n * 3);
        c.cl_pos0.ensure(nslot);
        PQ_HIP(hipMemcpyAsync(c.pos_build.p, pos, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
        PQ_HIP(hipMemcpyAsync(c.cl_pos0.p, c.cl_pos.p, sizeof(double4) * nslot, hipMemcpyDeviceToDevice, s));
    }
}

// The atom-level j lists from the counted rows: the far-away tail, then the
// fill pass (canonical images of a kept list when c.moved).
void jlist_fill(Ctx& c, int rows) {
    hipStream_t s = c.stream;
    const int ncl = c.ncl;
    const Geom& g = c.g;
    PQ_REQUIRE(rows >= 0, PQ_ERR_BOX, "atom list overflow");
    c.njrows = rows;
    // JL_TAIL far-away entries after the last row keep the pair kernel's
    // look-ahead loads in bounds
    c.jl.ensure(((size_t)rows * CL + JL_TAIL) * 4 * rsz(c));
    const double4* cw = c.moved ? c.cl_w.p : nullptr;
    const int4* kimg = c.moved ? c.cl_k.p : nullptr;
    if (c.fp64)
        PQ_LAUNCH(k_far_entries<double>, 1, 256, 0, s, as<double4>(c.jl) + (size_t)rows * CL, JL_TAIL);
    else
        PQ_LAUNCH(k_far_entries<float>, 1, 256, 0, s, as<float4>(c.jl) + (size_t)rows * CL, JL_TAIL);
    if (c.fp64)
        PQ_LAUNCH((k_jlist<true, double>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lcount.p, c.lcap, c.lj.p, c.cl_pos.p,
                  cw, kimg, c.cl_ref.p, c.jmask.p, c.jcount.p, c.jstart.p, as<double4>(c.jl));
    else
        PQ_LAUNCH((k_jlist<true, float>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lcount.p, c.lcap, c.lj.p, c.cl_pos.p,
                  cw, kimg, c.cl_ref.p, c.jmask.p, c.jcount.p, c.jstart.p, as<float4>(c.jl));
}

// ---- moves that keep the list ------------------------------------------------
// Largest squared displacement of an atom since the build (block partials).
__global__ __launch_bounds__(256) void k_disp2(int n, const double* __restrict__ pos, const double* __restrict__ pos0,
                                               double* __restrict__ part) {
    __shared__ double red[4];
    double m = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double dx = pos[3 * (size_t)i] - pos0[3 * (size_t)i];
        const double dy = pos[3 * (size_t)i + 1] - pos0[3 * (size_t)i + 1];
        const double dz = pos[3 * (size_t)i + 2] - pos0[3 * (size_t)i + 2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        m = (d2 > m || d2 != d2) ? d2 : m;   // a NaN displacement wins (forces a rebuild)
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(m, o, 64);
        m = (t > m || t != t) ? t : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int k = 1; k < 4; ++k) r = (red[k] > r || red[k] != red[k]) ? red[k] : r;
        part[blockIdx.x] = r;
    }
}
__global__ void k_max_part(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double r = 0.0;
    for (int k = 0; k < nb; ++k) r = (part[k] > r || part[k] != part[k]) ? part[k] : r;
    *out = r;
}

// Per slot: continuous position x = (build wrap) + (pos - pos at build), the
// canonical wrap w of pos, the lattice steps k = (x - w)/L, the pair kernel's
// position x - ref, and w into w64 (original order). Orthorhombic cells.
template <class T>
__global__ void k_refresh(int nslot, const int* __restrict__ orig, const double* __restrict__ pos,
                          const double* __restrict__ pos0, const double4* __restrict__ cpos0, Geom g,
                          const double* __restrict__ ref, double4* __restrict__ cpos, double4* __restrict__ cw,
                          int4* __restrict__ kimg, V4<T>* __restrict__ xyzq, double* __restrict__ w64) {
    const int sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslot) return;
    const int i = orig[sl];
    if (i < 0) {
        cw[sl] = make_double4(0.0, 0.0, 0.0, 0.0);
        kimg[sl] = make_int4(0, 0, 0, 0);
        return;
    }
    const double4 p0 = cpos0[sl];
    double x[3], w[3];
    int k[3];
    const double b0[3] = {p0.x, p0.y, p0.z};
    for (int d = 0; d < 3; ++d) {
        const double pd = pos[3 * (size_t)i + d];
        x[d] = b0[d] + (pd - pos0[3 * (size_t)i + d]);
        w[d] = canon_wrap(pd, g.L[d], g.invL[d]);
        k[d] = (int)rint((x[d] - w[d]) * g.invL[d]);
        w64[3 * (size_t)i + d] = w[d];
    }
    const int c = sl / CL;
    cpos[sl] = make_double4(x[0], x[1], x[2], 1.0);
    cw[sl] = make_double4(w[0], w[1], w[2], 1.0);
    kimg[sl] = make_int4(k[0], k[1], k[2], 0);
    V4<T> v = xyzq[sl];
    v.x = (T)(x[0] - ref[3 * (size_t)c + 0]);
    v.y = (T)(x[1] - ref[3 * (size_t)c + 1]);
    v.z = (T)(x[2] - ref[3 * (size_t)c + 2]);
    xyzq[sl] = v;
}

double nbr_max_disp2(Ctx& c, const double* pos) {
    hipStream_t s = c.stream;
    const int n = (int)c.n;
    const int nb = std::max(1, std::min(256, (int)cdiv(n, 256)));
    c.disp_part.ensure(nb + 1);
    PQ_LAUNCH(k_disp2, nb, 256, 0, s, n, pos, (const double*)c.pos_build.p, c.disp_part.p);
    PQ_LAUNCH(k_max_part, 1, 64, 0, s, (const double*)c.disp_part.p, nb, c.disp_part.p + nb);
    double* h = c.pinned + 40;
    PQ_HIP(hipMemcpyAsync(h, c.disp_part.p + nb, sizeof(double), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    return *h;
}

void nbr_refresh(Ctx& c, const double* pos) {
    hipStream_t s = c.stream;
    const int ncl = c.ncl;
    const int nslot = ncl * CL;
    Geom& g = c.g;
    c.cl_w.ensure(nslot);
    c.cl_k.ensure(nslot);
    c.moved = true;
    if (c.fp64)
        PQ_LAUNCH(k_refresh<double>, cdiv(nslot, 256), 256, 0, s, nslot, c.orig.p, pos, (const double*)c.pos_build.p,
                  (const double4*)c.cl_pos0.p, g, (const double*)c.cl_ref.p, c.cl_pos.p, c.cl_w.p, c.cl_k.p,
                  as<double4>(c.xyzq), c.w64.p);
    else
        PQ_LAUNCH(k_refresh<float>, cdiv(nslot, 256), 256, 0, s, nslot, c.orig.p, pos, (const double*)c.pos_build.p,
                  (const double4*)c.cl_pos0.p, g, (const double*)c.cl_ref.p, c.cl_pos.p, c.cl_w.p, c.cl_k.p,
                  as<float4>(c.xyzq), c.w64.p);
    // count pass with the canonical images, then the fill pass
    if (c.fp64)
        PQ_LAUNCH((k_jlist<false, double>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lcount.p, c.lcap, c.lj.p, c.cl_pos.p,
                  (const double4*)c.cl_w.p, (const int4*)c.cl_k.p, c.cl_ref.p, c.jmask.p, c.jcount.p,
                  (const int*)nullptr, (double4*)nullptr);
    else
        PQ_LAUNCH((k_jlist<false, float>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lcount.p, c.lcap, c.lj.p, c.cl_pos.p,
                  (const double4*)c.cl_w.p, (const int4*)c.cl_k.p, c.cl_ref.p, c.jmask.p, c.jcount.p,
                  (const int*)nullptr, (float4*)nullptr);
    scan_ints(c, c.jcount.p, c.jstart.p, ncl, false, s);
    int* hv = reinterpret_cast<int*>(c.pinned + 48);
    PQ_HIP(hipMemcpyAsync(&hv[3], c.jstart.p + ncl, sizeof(int), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    jlist_fill(c, hv[3]);
}

int nbr_export_ell(Ctx& c, int K, int32_t* nbr, int32_t* img, int32_t* count) {
    hipStream_t s = c.stream;
    const int n = (int)c.n;
    const double4* cpos = (const double4*)(c.moved ? c.cl_w.p : c.cl_pos.p);
    const int4* kimg = (const int4*)(c.moved ? c.cl_k.p : nullptr);
    DBuf<int> rowcnt, mx;
    rowcnt.ensure((size_t)n);
    mx.ensure(1);
    PQ_HIP(hipMemsetAsync(rowcnt.p, 0, sizeof(int) * (size_t)n, s));
    PQ_LAUNCH(k_ell<false>, cdiv(c.ncl, 4), 256, 0, s, c.ncl, c.g, c.lcount.p, c.lcap, c.lj.p, c.orig.p, cpos, kimg,
              rowcnt.p, 0, (unsigned long long*)nullptr);
    PQ_LAUNCH(k_max_int, 1, 1024, 0, s, rowcnt.p, n, mx.p);
    if (count) PQ_HIP(hipMemcpyAsync(count, rowcnt.p, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s));
    int kmax = 0;
    PQ_HIP(hipMemcpyAsync(&kmax, mx.p, sizeof(int), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    if (!(nbr || img) || kmax > K || K == 0) return kmax;
    if (kmax > PQ_ELL_MAX_K)
        throw Error(PQ_ERR_TOO_LARGE, "ELLPACK rows of " + std::to_string(kmax) + " neighbours exceed the limit of " +
                                          std::to_string(PQ_ELL_MAX_K));
    DBuf<unsigned long long> keys;
    if (kmax > 0) {
        keys.ensure((size_t)n * K);
        PQ_LAUNCH(k_ell<true>, cdiv(c.ncl, 4), 256, 0, s, c.ncl, c.g, c.lcount.p, c.lcap, c.lj.p, c.orig.p, cpos,
                  kimg, (int*)nullptr, K, keys.p);
    }
    int kp = 1;
    while (kp < kmax) kp <<= 1;
    PQ_LAUNCH(k_ell_sort, n, 256, (size_t)kp * sizeof(unsigned long long), s, n, K, rowcnt.p, keys.p, nbr, img);
    PQ_HIP(hipStreamSynchronize(s));
    return kmax;
}

int64_t nbr_export_pairs(Ctx& c, int64_t cap, int32_t* pairs) {
    hipStream_t s = c.stream;
    PQ_HIP(hipMemsetAsync(c.counter.p, 0, sizeof(unsigned long long), s));
    PQ_LAUNCH(k_export, cdiv(c.ncl, 4), 256, 0, s, c.ncl, c.g, c.lcount.p, c.lcap, c.lj.p, c.orig.p,
              (const double4*)(c.moved ? c.cl_w.p : c.cl_pos.p), (const int4*)(c.moved ? c.cl_k.p : nullptr),
              pairs ? cap : (int64_t)0, pairs, c.counter.p);
    unsigned long long tot = 0;
    PQ_HIP(hipMemcpyAsync(&tot, c.counter.p, sizeof(tot), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    return (int64_t)tot;
}

}  // namespace pq
