// Device helpers shared by the kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "pq_internal.h"

namespace pq {

// Canonical wrap into [0, L): w = x - L*floor(x*(1/L)), three separately
// rounded FP64 operations (no contraction), so the host-side definition of
// the neighbour predicate can be reproduced bit for bit.
__device__ __forceinline__ double canon_wrap(double x, double L, double invL) {
#pragma clang fp contract(off)
    double t = x * invL;
    double f = floor(t);
    double m = L * f;
    return x - m;
}

// Canonical wrap into the triclinic cell: the c, b and a components are
// removed in turn by the floor of the current fractional coordinate, every
// product and difference rounded once (with zero tilts: canon_wrap per axis).
__device__ __forceinline__ void canon_wrap_tric(double& x, double& y, double& z, const double* L, const double* inv,
                                                const Tric& t) {
#pragma clang fp contract(off)
    const double f2 = floor(z * inv[2]);
    z = z - f2 * L[2];
    y = y - f2 * t.tyz;
    x = x - f2 * t.txz;
    const double f1 = floor((y - z * t.ryz) * inv[1]);
    y = y - f1 * L[1];
    x = x - f1 * t.txy;
    const double f0 = floor(((x - y * t.cxy) - z * t.cxz) * inv[0]);
    x = x - f0 * L[0];
}

// Fractional coordinates of a wrapped position.
__device__ __forceinline__ void frac_tric(double x, double y, double z, const double* inv, const Tric& t, double& s0,
                                          double& s1, double& s2) {
#pragma clang fp contract(off)
    s2 = z * inv[2];
    s1 = (y - z * t.ryz) * inv[1];
    s0 = ((x - y * t.cxy) - z * t.cxz) * inv[0];
}

// Lattice vector n0 a + n1 b + n2 c, each component summed left to right from
// separately rounded products: x = (n0 L0 + n1 txy) + n2 txz, y = n1 L1 + n2 tyz,
// z = n2 L2 (with zero tilts exactly n*L).
__device__ __forceinline__ void lattice_vec(int n0, int n1, int n2, const double* L, const Tric& t, double& sx,
                                            double& sy, double& sz) {
#pragma clang fp contract(off)
    sx = ((double)n0 * L[0] + (double)n1 * t.txy) + (double)n2 * t.txz;
    sy = (double)n1 * L[1] + (double)n2 * t.tyz;
    sz = (double)n2 * L[2];
}

// Canonical squared distance between w_i and w_j + s (s a lattice vector):
// d = (w_j - w_i) + s per axis, d.d = (dx*dx + dy*dy) + dz*dz, no contraction.
__device__ __forceinline__ double canon_d2s(const double* __restrict__ wi, const double* __restrict__ wj, double sx,
                                            double sy, double sz) {
#pragma clang fp contract(off)
    double dx = (wj[0] - wi[0]) + sx;
    double dy = (wj[1] - wi[1]) + sy;
    double dz = (wj[2] - wi[2]) + sz;
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    return (a + b) + c;
}

// Image vector packed as three signed 10-bit fields.
__host__ __device__ __forceinline__ int pack_img(int n0, int n1, int n2) {
    return (n0 & 1023) | ((n1 & 1023) << 10) | ((n2 & 1023) << 20);
}
__host__ __device__ __forceinline__ void unpack_img(int p, int& n0, int& n1, int& n2) {
    n0 = (p << 22) >> 22;
    n1 = (p << 12) >> 22;
    n2 = (p << 2) >> 22;
}
__host__ __device__ __forceinline__ bool lex_positive(int n0, int n1, int n2) {
    return n0 > 0 || (n0 == 0 && (n1 > 0 || (n1 == 0 && n2 > 0)));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Waves of the reciprocal-space chain (the evaluation's critical path while the
// pair kernel runs beside it) raise their instruction-issue priority, so that on
// a SIMD shared with pair-kernel waves their few instructions go first.
__device__ __forceinline__ void chain_priority() { __builtin_amdgcn_s_setprio(3); }

// Vector types of the bulk precision T (float: the production form, double:
// the same kernels in FP64).
template <class T>
struct VecT;
template <>
struct VecT<float> {
    using v2 = float2;
    using v4 = float4;
};
template <>
struct VecT<double> {
    using v2 = double2;
    using v4 = double4;
};
template <class T>
using V2 = typename VecT<T>::v2;
template <class T>
using V4 = typename VecT<T>::v4;

template <class T>
__host__ __device__ __forceinline__ V4<T> mk4(T x, T y, T z, T w) {
    V4<T> r;
    r.x = x;
    r.y = y;
    r.z = z;
    r.w = w;
    return r;
}
template <class T>
__host__ __device__ __forceinline__ V2<T> mk2(T x, T y) {
    V2<T> r;
    r.x = x;
    r.y = y;
    return r;
}

// An integer (packed grid base index, atom slot) stored in the 4th component
// of a V4<T>: the bit pattern in FP32, the value in FP64 (exact below 2^53).
__device__ __forceinline__ float pack_int(int b, float) { return __int_as_float(b); }
__device__ __forceinline__ double pack_int(int b, double) { return (double)b; }
__device__ __forceinline__ int unpack_int(float w) { return __float_as_int(w); }
__device__ __forceinline__ int unpack_int(double w) { return (int)w; }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// FP64 sum over the 64 lanes of a wavefront (result in every lane).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// FP64 sum over a block of NT threads; returns the total in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds /* NT/64 */) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) t += lds[k];
    __syncthreads();
    return t;
}

}  // namespace pq
