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

// Wrap positions into the box, pick each atom's column, count per column.
__global__ void k_wrap_count(int n, const double* __restrict__ pos, Geom g, double* __restrict__ w64,
                             int* __restrict__ col_of, int* __restrict__ col_cnt, int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w[3];
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
        double x = pos[3 * (size_t)i + d];
        ok = ok && isfinite(x);
        w[d] = canon_wrap(x, g.L[d], g.invL[d]);
        w64[3 * (size_t)i + d] = w[d];
    }
    if (!ok) {
        atomicOr(flag, 1);
        w[0] = w[1] = w[2] = 0.0;
    }
    int cx = (int)floor(w[0] * ((double)g.ncx * g.invL[0]));
    int cy = (int)floor(w[1] * ((double)g.ncy * g.invL[1]));
    cx = min(max(cx, 0), g.ncx - 1);
    cy = min(max(cy, 0), g.ncy - 1);
    int c = cx + g.ncx * cy;
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

__global__ void k_bin(int n, const int* __restrict__ col_of, const int* __restrict__ col_start,
                      int* __restrict__ col_fill, int* __restrict__ tmp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = col_of[i];
    tmp[col_start[c] + atomicAdd(&col_fill[c], 1)] = i;
}

// Rank of each atom inside its column by (z, index): a deterministic sort.
__global__ void k_rank(int n, const int* __restrict__ col_of, const int* __restrict__ col_start,
                       const int* __restrict__ col_cl, const int* __restrict__ tmp,
                       const double* __restrict__ w64, int* __restrict__ orig) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = col_of[i];
    double zi = w64[3 * (size_t)i + 2];
    int r = 0;
    for (int k = col_start[c]; k < col_start[c + 1]; ++k) {
        int j = tmp[k];
        double zj = w64[3 * (size_t)j + 2];
        r += (zj < zi) || (zj == zi && j < i);
    }
    orig[(size_t)col_cl[c] * CL + r] = i;
}

__global__ void k_cluster_col(int ncol, const int* __restrict__ col_cl, int* __restrict__ cl_col) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    for (int k = col_cl[c]; k < col_cl[c + 1]; ++k) cl_col[k] = c;
}

// Bounding box, reference point and offsets (bulk precision T) of each cluster.
template <class T>
__global__ void k_cluster(int ncl, const int* __restrict__ orig, const double* __restrict__ w64,
                          double* __restrict__ ref, double* __restrict__ lo, double* __restrict__ hi,
                          V4<T>* __restrict__ xyzq) {
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
        if (i >= 0) {
            v.x = (T)(w64[3 * (size_t)i + 0] - r[0]);
            v.y = (T)(w64[3 * (size_t)i + 1] - r[1]);
            v.z = (T)(w64[3 * (size_t)i + 2] - r[2]);
        } else {
            // padding: far from everything, zero charge
            v.x = v.y = v.z = (T)1.0e4;
        }
        v.w = (T)0;
        xyzq[s] = v;
    }
}

__device__ __forceinline__ double gap1(double lo_j, double hi_j, double lo_i, double hi_i) {
    return fmax(0.0, fmax(lo_j - hi_i, lo_i - hi_j));
}

// Cluster-pair list: one wavefront per i-cluster; lanes scan the clusters of
// each candidate column and every z image. FILL = false counts, FILL = true
// writes at lstart[ic] in the same deterministic order.
template <bool FILL>
__global__ __launch_bounds__(256) void k_list(int ncl, Geom g, const int* __restrict__ cl_col,
                                              const int* __restrict__ col_cl, const double* __restrict__ lo,
                                              const double* __restrict__ hi, int* __restrict__ lcount,
                                              const int* __restrict__ lstart, int2* __restrict__ lj) {
    const int lane = lane_id();
    const int ic = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ic >= ncl) return;
    const double rl2 = g.rlist * g.rlist * (1.0 + 1e-9) + 1e-12;
    const double eps = 1e-6;
    const int coli = cl_col[ic];
    const int cxi = coli % g.ncx, cyi = coli / g.ncx;
    const double loi0 = lo[3 * ic], loi1 = lo[3 * ic + 1], loi2 = lo[3 * ic + 2];
    const double hii0 = hi[3 * ic], hii1 = hi[3 * ic + 1], hii2 = hi[3 * ic + 2];
    int cnt = 0;
    const int base = FILL ? lstart[ic] : 0;
    for (int dy = -g.Ry; dy <= g.Ry; ++dy) {
        int cy = cyi + dy;
        int ny = (cy >= 0) ? cy / g.ncy : -((-cy + g.ncy - 1) / g.ncy);
        int cyw = cy - ny * g.ncy;
        double sy = (double)ny * g.L[1];
        double gy = gap1(cyw * g.wy + sy, (cyw + 1) * g.wy + sy, loi1, hii1) - eps;
        if (gy > 0.0 && gy * gy >= rl2) continue;
        for (int dx = -g.Rx; dx <= g.Rx; ++dx) {
            int cx = cxi + dx;
            int nx = (cx >= 0) ? cx / g.ncx : -((-cx + g.ncx - 1) / g.ncx);
            int cxw = cx - nx * g.ncx;
            double sx = (double)nx * g.L[0];
            double gx = gap1(cxw * g.wx + sx, (cxw + 1) * g.wx + sx, loi0, hii0) - eps;
            if (gx > 0.0 && gx * gx >= rl2) continue;
            const int col = cxw + g.ncx * cyw;
            const int j0 = col_cl[col], j1 = col_cl[col + 1];
            for (int jb = j0; jb < j1; jb += 64) {
                const int jc = jb + lane;
                const bool valid = jc < j1;
                double dxy2 = 0.0, loj2 = 0.0, hij2 = 0.0;
                if (valid) {
                    double gxx = gap1(lo[3 * jc] + sx, hi[3 * jc] + sx, loi0, hii0);
                    double gyy = gap1(lo[3 * jc + 1] + sy, hi[3 * jc + 1] + sy, loi1, hii1);
                    dxy2 = gxx * gxx + gyy * gyy;
                    loj2 = lo[3 * jc + 2];
                    hij2 = hi[3 * jc + 2];
                }
                for (int nz = -g.Rz; nz <= g.Rz; ++nz) {
                    double sz = (double)nz * g.L[2];
                    double gz = gap1(loj2 + sz, hij2 + sz, loi2, hii2);
                    bool pass = valid && (dxy2 + gz * gz < rl2);
                    unsigned long long m = __ballot(pass);
                    if (FILL && pass) lj[base + cnt + lanes_below(m)] = make_int2(jc, pack_img(nx, ny, nz));
                    cnt += __popcll(m);
                }
            }
        }
    }
    if (!FILL && lane == 0) lcount[ic] = cnt;
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
// FILL = false counts entries and rows, FILL = true writes.
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

template <bool FILL, class T>
__global__ __launch_bounds__(256) void k_jlist(int ncl, Geom g, const int* __restrict__ lstart,
                                               const int2* __restrict__ lj, const int* __restrict__ orig,
                                               const double* __restrict__ w64, const double* __restrict__ ref,
                                               int* __restrict__ jcount, const int* __restrict__ jstart,
                                               V4<T>* __restrict__ jl) {
    const int lane = lane_id();
    const int ic = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (ic >= ncl) return;
    const double rc2 = g.rc * g.rc;
    // the i-cluster's atoms (the same in every lane)
    int ii[CL];
    double wi[CL][3];
#pragma unroll
    for (int a = 0; a < CL; ++a) {
        ii[a] = orig[(size_t)ic * CL + a];
        const int k = ii[a] >= 0 ? ii[a] : 0;
        wi[a][0] = w64[3 * (size_t)k + 0];
        wi[a][1] = w64[3 * (size_t)k + 1];
        wi[a][2] = w64[3 * (size_t)k + 2];
    }
    const double r0 = ref[3 * ic], r1 = ref[3 * ic + 1], r2 = ref[3 * ic + 2];
    const int e0 = lstart[ic], e1 = lstart[ic + 1];
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
    int cnt = 0;
    for (int eb = e0; eb < e1; eb += 8) {
        const int e = eb + eo;
        int col = 0, slot = 0;
        double p0 = 0.0, p1 = 0.0, p2 = 0.0;
        if (e < e1) {
            const int2 je = lj[e];
            slot = je.x * CL + b;
            const int j = orig[slot];
            if (j >= 0) {
                int n0, n1, n2;
                unpack_img(je.y, n0, n1, n2);
                const double* wj = w64 + 3 * (size_t)j;
#pragma unroll
                for (int a = 0; a < CL; ++a) {
                    const double d2 = canon_d2(wi[a], wj, n0, n1, n2, g.L[0], g.L[1], g.L[2]);
                    if (ii[a] >= 0 && d2 > 0.0 && d2 < rc2) col |= 1 << a;
                }
                p0 = wj[0] + (double)n0 * g.L[0];
                p1 = wj[1] + (double)n1 * g.L[1];
                p2 = wj[2] + (double)n2 * g.L[2];
            }
        }
        const bool pass = col != 0;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(pass);
        if (FILL && pass) {
            jl[dest(cnt + lanes_below(m))] =
                mk4<T>((T)(p0 - r0), (T)(p1 - r1), (T)(p2 - r2), pack_int(slot | (col << JL_SLOT_BITS), T(0)));
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

// Export of the atom pairs closer than the list radius, by the canonical FP64
// predicate; each unordered pair once. Rows are reserved with a global
// counter; rows beyond `cap` are not written but still counted.
__global__ __launch_bounds__(256) void k_export(int ncl, Geom g, const int* __restrict__ lstart,
                                                const int2* __restrict__ lj, const int* __restrict__ orig,
                                                const double* __restrict__ w64, int64_t cap,
                                                int32_t* __restrict__ out, unsigned long long* __restrict__ counter) {
    const int lane = lane_id();
    const int ic = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ic >= ncl) return;
    const int a = lane >> 3, b = lane & 7;
    const int i = orig[(size_t)ic * CL + a];
    const double rl2 = g.rlist * g.rlist;
    for (int e = lstart[ic]; e < lstart[ic + 1]; ++e) {
        const int2 je = lj[e];
        const int j = orig[(size_t)je.x * CL + b];
        int n0, n1, n2;
        unpack_img(je.y, n0, n1, n2);
        bool ok = (i >= 0) && (j >= 0) && ((i < j) || (i == j && lex_positive(n0, n1, n2)));
        if (ok) ok = canon_d2(w64 + 3 * (size_t)i, w64 + 3 * (size_t)j, n0, n1, n2, g.L[0], g.L[1], g.L[2]) < rl2;
        unsigned long long m = __ballot(ok);
        if (m == 0ull) continue;
        unsigned long long basepos = 0;
        if (lane == 0) basepos = atomicAdd(counter, (unsigned long long)__popcll(m));
        basepos = __shfl(basepos, 0, 64);
        if (ok) {
            unsigned long long pos = basepos + lanes_below(m);
            if ((int64_t)pos < cap && out) {
                int32_t* r = out + 5 * pos;
                r[0] = i;
                r[1] = j;
                r[2] = n0;
                r[3] = n1;
                r[4] = n2;
            }
        }
    }
}

void scan_ints(const int* in, int* out, int n, bool ceil8, hipStream_t s) {
    if (ceil8)
        PQ_LAUNCH(k_scan<1>, 1, 1024, 0, s, in, out, n);
    else
        PQ_LAUNCH(k_scan<0>, 1, 1024, 0, s, in, out, n);
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
    // columns sized for ~8 atoms per cubic cluster
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double rho = (double)n / V;
    const double a = std::cbrt((double)CL / rho);
    g.ncx = std::max(1, (int)std::lround(p.box[0] / a));
    g.ncy = std::max(1, (int)std::lround(p.box[1] / a));
    g.wx = p.box[0] / g.ncx;
    g.wy = p.box[1] / g.ncy;
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

    PQ_HIP(hipMemsetAsync(c.col_cnt.p, 0, sizeof(int) * c.ncol, s));
    PQ_HIP(hipMemsetAsync(c.col_fill.p, 0, sizeof(int) * c.ncol, s));
    PQ_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int) * 4, s));
    PQ_LAUNCH(k_wrap_count, cdiv(n, 256), 256, 0, s, n, pos, g, c.w64.p, c.col_of.p, c.col_cnt.p, c.flag.p);
    PQ_LAUNCH(k_scan<0>, 1, 1024, 0, s, c.col_cnt.p, c.col_start.p, c.ncol);
    PQ_LAUNCH(k_scan<1>, 1, 1024, 0, s, c.col_cnt.p, c.col_cl.p, c.ncol);
    int hv[2];
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
    c.cl_lo.ensure((size_t)ncl * 3);
    c.cl_hi.ensure((size_t)ncl * 3);
    c.cl_col.ensure(ncl);
    c.lcount.ensure(ncl + 1);
    c.lstart.ensure(ncl + 1);

    PQ_LAUNCH(k_bin, cdiv(n, 256), 256, 0, s, n, c.col_of.p, c.col_start.p, c.col_fill.p, c.tmp_atoms.p);
    PQ_LAUNCH(k_fill_int, cdiv(nslot, 256), 256, 0, s, c.orig.p, (int)nslot, -1);
    PQ_LAUNCH(k_rank, cdiv(n, 256), 256, 0, s, n, c.col_of.p, c.col_start.p, c.col_cl.p, c.tmp_atoms.p,
              c.w64.p, c.orig.p);
    PQ_LAUNCH(k_cluster_col, cdiv(c.ncol, 256), 256, 0, s, c.ncol, c.col_cl.p, c.cl_col.p);
    if (c.fp64)
        PQ_LAUNCH(k_cluster<double>, cdiv(ncl, 256), 256, 0, s, ncl, c.orig.p, c.w64.p, c.cl_ref.p, c.cl_lo.p,
                  c.cl_hi.p, as<double4>(c.xyzq));
    else
        PQ_LAUNCH(k_cluster<float>, cdiv(ncl, 256), 256, 0, s, ncl, c.orig.p, c.w64.p, c.cl_ref.p, c.cl_lo.p,
                  c.cl_hi.p, as<float4>(c.xyzq));
    PQ_LAUNCH((k_list<false>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.cl_col.p, c.col_cl.p, c.cl_lo.p, c.cl_hi.p,
              c.lcount.p, (const int*)nullptr, (int2*)nullptr);
    PQ_LAUNCH(k_scan<0>, 1, 1024, 0, s, c.lcount.p, c.lstart.p, ncl);
    int tot = 0;
    PQ_HIP(hipMemcpyAsync(&tot, c.lstart.p + ncl, sizeof(int), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    PQ_REQUIRE(tot >= 0, PQ_ERR_BOX, "cluster-pair list overflow");
    c.nlist = tot;
    c.lj.ensure(std::max(1, tot));
    PQ_LAUNCH((k_list<true>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.cl_col.p, c.col_cl.p, c.cl_lo.p, c.cl_hi.p,
              c.lcount.p, c.lstart.p, c.lj.p);
    // atom-level j lists for the pair kernel
    c.jcount.ensure(ncl + 1);
    c.jstart.ensure(ncl + 1);
    if (c.fp64)
        PQ_LAUNCH((k_jlist<false, double>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lstart.p, c.lj.p, c.orig.p, c.w64.p,
                  c.cl_ref.p, c.jcount.p, (const int*)nullptr, (double4*)nullptr);
    else
        PQ_LAUNCH((k_jlist<false, float>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lstart.p, c.lj.p, c.orig.p, c.w64.p,
                  c.cl_ref.p, c.jcount.p, (const int*)nullptr, (float4*)nullptr);
    PQ_LAUNCH(k_scan<0>, 1, 1024, 0, s, c.jcount.p, c.jstart.p, ncl);
    int rows = 0;
    PQ_HIP(hipMemcpyAsync(&rows, c.jstart.p + ncl, sizeof(int), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    PQ_REQUIRE(rows >= 0, PQ_ERR_BOX, "atom list overflow");
    c.njrows = rows;
    // JL_TAIL far-away entries after the last row keep the pair kernel's
    // look-ahead loads in bounds
    c.jl.ensure(((size_t)rows * CL + JL_TAIL) * 4 * rsz(c));
    if (c.fp64)
        PQ_LAUNCH(k_far_entries<double>, 1, 256, 0, s, as<double4>(c.jl) + (size_t)rows * CL, JL_TAIL);
    else
        PQ_LAUNCH(k_far_entries<float>, 1, 256, 0, s, as<float4>(c.jl) + (size_t)rows * CL, JL_TAIL);
    if (c.fp64)
        PQ_LAUNCH((k_jlist<true, double>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lstart.p, c.lj.p, c.orig.p, c.w64.p,
                  c.cl_ref.p, c.jcount.p, c.jstart.p, as<double4>(c.jl));
    else
        PQ_LAUNCH((k_jlist<true, float>), cdiv(ncl, 4), 256, 0, s, ncl, g, c.lstart.p, c.lj.p, c.orig.p, c.w64.p,
                  c.cl_ref.p, c.jcount.p, c.jstart.p, as<float4>(c.jl));
}

int64_t nbr_export_pairs(Ctx& c, int64_t cap, int32_t* pairs) {
    hipStream_t s = c.stream;
    PQ_HIP(hipMemsetAsync(c.counter.p, 0, sizeof(unsigned long long), s));
    PQ_LAUNCH(k_export, cdiv(c.ncl, 4), 256, 0, s, c.ncl, c.g, c.lstart.p, c.lj.p, c.orig.p, c.w64.p,
              pairs ? cap : (int64_t)0, pairs, c.counter.p);
    unsigned long long tot = 0;
    PQ_HIP(hipMemcpyAsync(&tot, c.counter.p, sizeof(tot), hipMemcpyDeviceToHost, s));
    PQ_HIP(hipStreamSynchronize(s));
    return (int64_t)tot;
}

}  // namespace pq
