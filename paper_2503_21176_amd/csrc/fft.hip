// Hand-written 3-D real-to-complex FFT, influence-function convolution and
// complex-to-real FFT for smooth PME (Algorithm "Smooth PME", steps 2-4).
//
// Grid layout: real Q[z][y][x] (x fastest); half spectrum H[z][y][mx],
// mx < K0/2 + 1. Five kernels, each one read and one write of the grid:
//   x: pairs of real rows packed as one complex sequence (a + i b), one
//      complex FFT, split into the two half spectra;
//   y: complex FFT along y for a tile of mx columns of one z plane;
//   z: complex FFT along z, multiply by G(m) = T0 T1 T2 / (pi V |m|^2),
//      accumulate E_rec = 1/2 sum_m w(mx) G |FQ|^2 in FP64, inverse FFT along z
//      (one read and one write for the three steps);
//   y inverse; x: two Hermitian half spectra combined into one complex
//      sequence, inverse FFT, real and imaginary parts are the two rows.
// Each 1-D transform runs in LDS as mixed-radix Stockham passes (self-sorting,
// ping-pong buffers) with radices 16, 8, 9, 4, 2, 3, 5: the composite ones
// (16 = 4 x 4, 8 = 2 x 4, 9 = 3 x 3) are done in registers, so 144 = 16 x 9
// takes two passes. Twiddles come from FP64 tables rounded to the bulk
// precision and are staged in LDS with the data.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <vector>

#include "dev.h"
#include "pq_internal.h"

namespace pq {

struct FftDev {
    int n, nst, ntw;
    int radix[FFT_MAX_STAGES];
    int ns[FFT_MAX_STAGES];
    int twoff[FFT_MAX_STAGES];
};

template <class C>
__device__ __forceinline__ C cmk(decltype(C::x) x, decltype(C::x) y) {
    C r;
    r.x = x;
    r.y = y;
    return r;
}
template <class C>
__device__ __forceinline__ C cmul(C a, C b) {
    return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class C>
__device__ __forceinline__ C cadd(C a, C b) {
    return cmk<C>(a.x + b.x, a.y + b.y);
}
template <class C>
__device__ __forceinline__ C csub(C a, C b) {
    return cmk<C>(a.x - b.x, a.y - b.y);
}
// multiply by sign*i
template <int SIGN, class C>
__device__ __forceinline__ C mul_i(C a) {
    return SIGN > 0 ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}

// cos and sin of 2 pi j / N for the composite radices
template <int N>
__device__ __forceinline__ constexpr double twc(int j) {
    if constexpr (N == 6) {
        constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
        return c[j];
    } else if constexpr (N == 10) {
        constexpr double c[10] = {1.0, 0.80901699437494742410, 0.30901699437494742410, -0.30901699437494742410,
                                   -0.80901699437494742410, -1.0, -0.80901699437494742410, -0.30901699437494742410,
                                   0.30901699437494742410, 0.80901699437494742410};
        return c[j];
    } else if constexpr (N == 12) {
        constexpr double c[12] = {1.0, 0.86602540378443864676, 0.5, 0.0, -0.5, -0.86602540378443864676, -1.0,
                                   -0.86602540378443864676, -0.5, 0.0, 0.5, 0.86602540378443864676};
        return c[j];
    } else if constexpr (N == 8) {
        constexpr double c[8] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                                 -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440};
        return c[j];
    } else if constexpr (N == 9) {
        constexpr double c[9] = {1.0, 0.76604444311897803520, 0.17364817766693034885, -0.5, -0.93969262078590838405,
                                 -0.93969262078590838405, -0.5, 0.17364817766693034885, 0.76604444311897803520};
        return c[j];
    } else {
        static_assert(N == 16, "no twiddle table for this length");
        constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                  0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                  -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                                  0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
        return c[j];
    }
}
template <int N>
__device__ __forceinline__ constexpr double tws(int j) {
    if constexpr (N == 6) {
        constexpr double s[6] = {0.0, 0.86602540378443864676, 0.86602540378443864676, 0.0, -0.86602540378443864676,
                                  -0.86602540378443864676};
        return s[j];
    } else if constexpr (N == 10) {
        constexpr double s[10] = {0.0, 0.58778525229247312917, 0.95105651629515357212, 0.95105651629515357212,
                                   0.58778525229247312917, 0.0, -0.58778525229247312917, -0.95105651629515357212,
                                   -0.95105651629515357212, -0.58778525229247312917};
        return s[j];
    } else if constexpr (N == 12) {
        constexpr double s[12] = {0.0, 0.5, 0.86602540378443864676, 1.0, 0.86602540378443864676, 0.5, 0.0, -0.5,
                                   -0.86602540378443864676, -1.0, -0.86602540378443864676, -0.5};
        return s[j];
    } else if constexpr (N == 8) {
        constexpr double s[8] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440,
                                 0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440};
        return s[j];
    } else if constexpr (N == 9) {
        constexpr double s[9] = {0.0, 0.64278760968653932632, 0.98480775301220805936, 0.86602540378443864676,
                                 0.34202014332566873304, -0.34202014332566873304, -0.86602540378443864676,
                                 -0.98480775301220805936, -0.64278760968653932632};
        return s[j];
    } else {
        static_assert(N == 16, "no twiddle table for this length");
        constexpr double s[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                  1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                  0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                  -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};
        return s[j];
    }
}

template <int R, int SIGN, class C>
__device__ __forceinline__ void dft(C* v);

// In-register DFT of length N = P Q by Cooley-Tukey: P-point DFTs over the
// inputs q + Q p, twiddles W_N^(q k1), Q-point DFTs, output k1 + P k2.
template <int P, int Q, int SIGN, class C>
__device__ __forceinline__ void dft_pq(C* v) {
    using T = decltype(C::x);
    constexpr int N = P * Q;
    C y[N];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        C t[P];
#pragma unroll
        for (int p = 0; p < P; ++p) t[p] = v[q + Q * p];
        dft<P, SIGN>(t);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            const int e = (q * k1) % N;
            if (e == 0) {
                y[k1 * Q + q] = t[k1];
            } else {
                const C w = cmk<C>(T(twc<N>(e)), T(SIGN * tws<N>(e)));
                y[k1 * Q + q] = cmul(t[k1], w);
            }
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
        C u[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) u[q] = y[k1 * Q + q];
        dft<Q, SIGN>(u);
#pragma unroll
        for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = u[k2];
    }
}

// In-register DFT of length R with kernel exp(SIGN 2 pi i r s / R).
template <int R, int SIGN, class C>
__device__ __forceinline__ void dft(C* v) {
    using T = decltype(C::x);
    if constexpr (R == 8) {
        dft_pq<2, 4, SIGN>(v);
    } else if constexpr (R == 6) {
        dft_pq<2, 3, SIGN>(v);
    } else if constexpr (R == 10) {
        dft_pq<2, 5, SIGN>(v);
    } else if constexpr (R == 12) {
        dft_pq<4, 3, SIGN>(v);
    } else if constexpr (R == 9) {
        dft_pq<3, 3, SIGN>(v);
    } else if constexpr (R == 16) {
        dft_pq<4, 4, SIGN>(v);
    } else if constexpr (R == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T c = T(-0.5), s = T(0.86602540378443864676);
        C t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        C a = cmk<C>(v[0].x + c * t1.x, v[0].y + c * t1.y);
        C b = mul_i<SIGN>(cmk<C>(s * t2.x, s * t2.y));
        v[0] = cadd(v[0], t1);
        v[1] = cadd(a, b);
        v[2] = csub(a, b);
    } else if constexpr (R == 4) {
        C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        C s13 = cadd(v[1], v[3]), d13 = mul_i<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if constexpr (R == 5) {
        const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
        const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
        C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        C a1 = cmk<C>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
        C a2 = cmk<C>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
        C b1 = mul_i<SIGN>(cmk<C>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
        C b2 = mul_i<SIGN>(cmk<C>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
}

template <int R, int SIGN, class C>
__device__ __forceinline__ void butterfly(const C* __restrict__ a, C* __restrict__ b, const C* __restrict__ tw, int j,
                                          int m, int Ns, int s, int es, int ss) {
    const int k = j % Ns;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[(j + r * m) * es + s * ss];
    if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C w = tw[k * (R - 1) + (r - 1)];
            if (SIGN > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
    }
    dft<R, SIGN>(v);
    const int o = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) b[(o + r * Ns) * es + s * ss] = v[r];
}

// All Stockham passes for nseq sequences held in LDS (element k of sequence
// s at k*es + s*ss). Returns the buffer holding the result.
// SFAST: consecutive threads take consecutive sequences (use when ss == 1).
template <int SIGN, bool SFAST, class C>
__device__ C* fft_lds(C* a, C* b, const FftDev& pl, const C* __restrict__ tw, int nseq, int es, int ss) {
    const int n = pl.n;
    for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.radix[st], Ns = pl.ns[st], m = n / R;
        const C* twst = tw + pl.twoff[st];
        const int total = nseq * m;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            int s, j;
            if (SFAST) {
                s = t % nseq;
                j = t / nseq;
            } else {
                j = t % m;
                s = t / m;
            }
            switch (R) {
                case 2: butterfly<2, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
                case 3: butterfly<3, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
                case 4: butterfly<4, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
                case 5: butterfly<5, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
                case 8: butterfly<8, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
                case 9: butterfly<9, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
                default: butterfly<16, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
            }
        }
        __syncthreads();
        C* t = a;
        a = b;
        b = t;
    }
    return a;
}

// ---- x: real rows -> half spectra ----------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_fft_x_r2c(FftDev pl, const V2<T>* __restrict__ tw, int nrows, int np,
                                                   const T* __restrict__ grid, V2<T>* __restrict__ spec) {
    chain_priority();
    using C = V2<T>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C* sm = reinterpret_cast<C*>(smraw);
    const int n = pl.n, X = n / 2 + 1;
    C* a = sm;
    C* b = sm + np * n;
    C* tl = sm + 2 * np * n;   // twiddles of this axis
    for (int i = threadIdx.x; i < pl.ntw; i += blockDim.x) tl[i] = tw[i];
    const int p0 = blockIdx.x * np;
    for (int idx = threadIdx.x; idx < np * n; idx += blockDim.x) {
        const int s = idx / n, k = idx % n;
        const int r0 = 2 * (p0 + s), r1 = r0 + 1;
        const T re = (r0 < nrows) ? grid[(size_t)r0 * n + k] : T(0);
        const T im = (r1 < nrows) ? grid[(size_t)r1 * n + k] : T(0);
        a[s * n + k] = cmk<C>(re, im);
    }
    __syncthreads();
    const C* o = fft_lds<-1, false>(a, b, pl, tl, np, 1, n);
    const T h = T(0.5);
    for (int idx = threadIdx.x; idx < np * X; idx += blockDim.x) {
        const int s = idx / X, m = idx % X;
        const int r0 = 2 * (p0 + s), r1 = r0 + 1;
        if (r0 >= nrows) continue;
        const C z = o[s * n + m];
        const C zr = o[s * n + (n - m) % n];
        spec[(size_t)r0 * X + m] = cmk<C>(h * (z.x + zr.x), h * (z.y - zr.y));
        if (r1 < nrows) spec[(size_t)r1 * X + m] = cmk<C>(h * (z.y + zr.y), -h * (z.x - zr.x));
    }
}

// ---- x: half spectra -> real rows ----------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_fft_x_c2r(FftDev pl, const V2<T>* __restrict__ tw, int nrows, int np,
                                                   const V2<T>* __restrict__ spec, T* __restrict__ grid) {
    chain_priority();
    using C = V2<T>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C* sm = reinterpret_cast<C*>(smraw);
    const int n = pl.n, X = n / 2 + 1;
    C* a = sm;
    C* b = sm + np * n;
    C* tl = sm + 2 * np * n;   // twiddles of this axis
    for (int i = threadIdx.x; i < pl.ntw; i += blockDim.x) tl[i] = tw[i];
    const int p0 = blockIdx.x * np;
    for (int idx = threadIdx.x; idx < np * n; idx += blockDim.x) {
        const int s = idx / n, m = idx % n;
        const int r0 = 2 * (p0 + s), r1 = r0 + 1;
        C A = cmk<C>(T(0), T(0)), B = cmk<C>(T(0), T(0));
        if (m < X) {
            if (r0 < nrows) A = spec[(size_t)r0 * X + m];
            if (r1 < nrows) B = spec[(size_t)r1 * X + m];
        } else {
            if (r0 < nrows) A = spec[(size_t)r0 * X + (n - m)];
            if (r1 < nrows) B = spec[(size_t)r1 * X + (n - m)];
            A.y = -A.y;
            B.y = -B.y;
        }
        a[s * n + m] = cmk<C>(A.x - B.y, A.y + B.x);
    }
    __syncthreads();
    const C* o = fft_lds<1, false>(a, b, pl, tl, np, 1, n);
    for (int idx = threadIdx.x; idx < np * n; idx += blockDim.x) {
        const int s = idx / n, k = idx % n;
        const int r0 = 2 * (p0 + s), r1 = r0 + 1;
        const C z = o[s * n + k];
        if (r0 < nrows) grid[(size_t)r0 * n + k] = z.x;
        if (r1 < nrows) grid[(size_t)r1 * n + k] = z.y;
    }
}

// ---- strided column transforms (y pass, and z pass with the convolution) --
struct ConvArgs {
    const double* T0;
    const double* T1;
    const double* T2;
    const double* S0;
    const double* S1;
    const double* S2;
    double scale;
    int K0;
    int tric;
    const double *B0, *B1, *B2, *M0, *M1, *M2;
    double r00, r10, r11, r20, r21, r22, pa2;
};

// G(m) of a triclinic cell: scale B0 B1 B2 exp(-pi^2 |k|^2 / alpha^2) / |k|^2
// with k = R m' (R = H^-1 lower triangular, m' the signed frequencies).
__device__ __forceinline__ double conv_g_tric(const ConvArgs& cv, int mx, int my, int mz) {
    const double m0 = cv.M0[mx], m1 = cv.M1[my], m2 = cv.M2[mz];
    const double kx = cv.r00 * m0, ky = cv.r10 * m0 + cv.r11 * m1, kz = (cv.r20 * m0 + cv.r21 * m1) + cv.r22 * m2;
    const double k2 = kx * kx + ky * ky + kz * kz;
    return cv.scale * cv.B0[mx] * cv.B1[my] * cv.B2[mz] * exp(-cv.pa2 * k2) / k2;
}

template <int SIGN, bool CONV, class T>
__global__ __launch_bounds__(256) void k_fft_col(FftDev pl, const V2<T>* __restrict__ tw, int X, int tx,
                                                 size_t estride, size_t ostride, V2<T>* __restrict__ spec,
                                                 ConvArgs cv, double* __restrict__ epart) {
    chain_priority();
    // CONV: epart == NULL skips the energy
    using C = V2<T>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C* sm = reinterpret_cast<C*>(smraw);
    const int n = pl.n;
    C* a = sm;
    C* b = sm + n * tx;
    C* tl = sm + 2 * n * tx;   // twiddles of this axis
    for (int i = threadIdx.x; i < pl.ntw; i += blockDim.x) tl[i] = tw[i];
    const int mx0 = blockIdx.x * tx;
    const int o = blockIdx.y;
    C* base = spec + (size_t)o * ostride;
    for (int idx = threadIdx.x; idx < n * tx; idx += blockDim.x) {
        const int k = idx / tx, s = idx % tx;
        const int mx = mx0 + s;
        a[idx] = (mx < X) ? base[(size_t)k * estride + mx] : cmk<C>(T(0), T(0));
    }
    __syncthreads();
    C* r = fft_lds<SIGN, true>(a, b, pl, tl, tx, tx, 1);
    if (CONV) {
        // r holds F(mx, my = o, mz = k). Energy: one partial per column
        // (mx, my) from 16 threads (thread u sums mz = u, u + 16, ... in
        // order, then a fixed xor tree over the 16), so E_rec does not depend
        // on the tiling (tx <= 16); then multiply by G.
        const int my = o;
        if (epart) {
            const int s = threadIdx.x >> 4, u = threadIdx.x & 15;
            const int mx = mx0 + s;
            double e = 0.0;
            if (s < tx && mx < X) {
                const double wgt = (mx == 0 || (2 * mx == cv.K0)) ? 1.0 : 2.0;
                const double tx0 = cv.scale * cv.T0[mx] * cv.T1[my], sx0 = cv.S0[mx] + cv.S1[my];
                for (int mz = u; mz < n; mz += 16) {
                    if ((mx | my | mz) == 0) continue;
                    const double g = cv.tric ? conv_g_tric(cv, mx, my, mz) : tx0 * cv.T2[mz] / (sx0 + cv.S2[mz]);
                    const C v = r[mz * tx + s];
                    e += wgt * g * ((double)v.x * v.x + (double)v.y * v.y);
                }
            }
#pragma unroll
            for (int w = 8; w > 0; w >>= 1) e += __shfl_xor(e, w, 16);
            if (u == 0 && s < tx && mx < X) epart[(size_t)my * X + mx] = 0.5 * e;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < n * tx; idx += blockDim.x) {
            const int mz = idx / tx, s = idx % tx;
            const int mx = mx0 + s;
            T gk = T(0);
            if (mx < X && (mx | my | mz) != 0)
                gk = (T)(cv.tric ? conv_g_tric(cv, mx, my, mz)
                                 : cv.scale * cv.T0[mx] * cv.T1[my] * cv.T2[mz] / (cv.S0[mx] + cv.S1[my] + cv.S2[mz]));
            r[idx] = cmk<C>(r[idx].x * gk, r[idx].y * gk);
        }
        __syncthreads();
        C* other = (r == a) ? b : a;
        r = fft_lds<-SIGN, true>(r, other, pl, tl, tx, tx, 1);
    }
    for (int idx = threadIdx.x; idx < n * tx; idx += blockDim.x) {
        const int k = idx / tx, s = idx % tx;
        const int mx = mx0 + s;
        if (mx < X) base[(size_t)k * estride + mx] = r[idx];
    }
}

// ---- strided column transforms, two register radices ----------------------
// For n = R1 R2 with both factors register radices, a column transform takes
// one LDS exchange. With j = R2 n1 + n2 and k = k1 + R1 k2,
//   X[k1 + R1 k2] = sum_n2 w_R2^(n2 k2) w_n^(n2 k1) sum_n1 x[R2 n1 + n2] w_R1^(n1 k1),
// w_m = exp(SIGN 2 pi i / m):
//   stage A: thread (n2, column) loads its R1 points straight from the grid
//            (CT consecutive columns: coalesced rows), R1-point DFT, twiddles,
//            into LDS;
//   stage B: thread (k1, column) reads its R2 values, R2-point DFT, holding
//            X[k1 + R1 k2] for k2 < R2.
// In the z pass (CONV) the thread multiplies its outputs by G, accumulates
// the energy and runs the inverse transform back the same way:
//   x[j2 + R2 j1] = sum_k1 w_R1^(-j1 k1) w_n^(-j2 k1) sum_k2 Y[k1 + R1 k2] w_R2^(-j2 k2).
constexpr int CT = 16;   // columns per workgroup

template <int R1, int R2, int SIGN, bool CONV, class T>
__global__ __launch_bounds__(CT*(R1 > R2 ? R1 : R2)) void k_fft_col2(const V2<T>* __restrict__ wn, int X,
                                                                     size_t estride, size_t ostride,
                                                                     V2<T>* __restrict__ spec, ConvArgs cv,
                                                                     double* __restrict__ epart) {
    chain_priority();
    using C = V2<T>;
    constexpr int N = R1 * R2;
    __shared__ C sm[N * CT];   // element (a, b) of a column at (a * R2 + b) * CT + column
    __shared__ double se[CONV ? R1 * CT : 1];
    const int mx0 = blockIdx.x * CT;
    const int o = blockIdx.y;
    C* base = spec + (size_t)o * ostride;
    const int s = threadIdx.x % CT, g = threadIdx.x / CT;
    const int mx = mx0 + s;
    const bool col = mx < X;
    // w_n^e for the sign of the transform (wn holds exp(-2 pi i e / n))
    auto tw = [&](int e, int sign) {
        C w = wn[e % N];
        if (sign > 0) w.y = -w.y;
        return w;
    };
    if (g < R2) {
        C v[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1)
            v[n1] = col ? base[(size_t)(R2 * n1 + g) * estride + mx] : cmk<C>(T(0), T(0));
        dft<R1, SIGN>(v);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) sm[(k1 * R2 + g) * CT + s] = (k1 == 0 || g == 0) ? v[k1] : cmul(v[k1], tw(g * k1, SIGN));
    }
    __syncthreads();
    C u[R2];
    if (g < R1) {
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) u[n2] = sm[(g * R2 + n2) * CT + s];
        dft<R2, SIGN>(u);   // u[k2] = X[g + R1 k2]
    }
    if constexpr (!CONV) {
        if (g < R1 && col) {
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) base[(size_t)(g + R1 * k2) * estride + mx] = u[k2];
        }
    } else {
        // o = my; u[k2] holds mz = g + R1 k2. Energy: each thread sums its
        // modes in k2 order, then the R1 threads of a column in g order.
        const int my = o;
        if (g < R1) {
            double e = 0.0;
            const double wgt = (mx == 0 || (2 * mx == cv.K0)) ? 1.0 : 2.0;
            const double t01 = col ? cv.scale * cv.T0[mx] * cv.T1[my] : 0.0;
            const double s01 = col ? cv.S0[mx] + cv.S1[my] : 1.0;
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int mz = g + R1 * k2;
                double gk = 0.0;
                if (col && (mx | my | mz) != 0)
                    gk = cv.tric ? conv_g_tric(cv, mx, my, mz) : t01 * cv.T2[mz] / (s01 + cv.S2[mz]);
                if (epart) e += wgt * gk * ((double)u[k2].x * u[k2].x + (double)u[k2].y * u[k2].y);
                u[k2] = cmk<C>(u[k2].x * (T)gk, u[k2].y * (T)gk);
            }
            if (epart) se[g * CT + s] = 0.5 * e;
            // inverse: R2-point transforms in registers, conjugate twiddles
            dft<R2, -SIGN>(u);   // u[j2]
        }
        __syncthreads();   // stage B has read sm
        if (g < R1) {
#pragma unroll
            for (int j2 = 0; j2 < R2; ++j2) sm[(g * R2 + j2) * CT + s] = (g == 0 || j2 == 0) ? u[j2] : cmul(u[j2], tw(j2 * g, -SIGN));
        }
        __syncthreads();
        if (epart && g == 0 && col) {
            double e = 0.0;
            for (int k = 0; k < R1; ++k) e += se[k * CT + s];
            epart[(size_t)my * X + mx] = e;
        }
        if (g < R2) {
            C v[R1];
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) v[k1] = sm[(k1 * R2 + g) * CT + s];
            dft<R1, -SIGN>(v);   // v[j1] = x[g + R2 j1]
            if (col) {
#pragma unroll
                for (int j1 = 0; j1 < R1; ++j1) base[(size_t)(g + R2 * j1) * estride + mx] = v[j1];
            }
        }
    }
}

// ---- x passes, two register radices --------------------------------------
// The same decomposition along rows: a workgroup takes RP pairs of real rows,
// each pair the complex sequence z = row0 + i row1 of length n = R1 R2.
// Forward: thread (n2, pair) loads z[R2 n1 + n2] (R2 consecutive threads read
// consecutive points of a row), R1-point DFT, twiddles, LDS; thread (k1, pair)
// the R2-point DFT; the spectrum goes through LDS once more, where the two
// half spectra are split off: H0[m] = (Z[m] + conj Z[n-m]) / 2,
// H1[m] = (Z[m] - conj Z[n-m]) / 2i. Inverse: thread (n2, pair) builds
// z[m] = H0[m] + i H1[m] (Hermitian halves for m > n/2) from the spectra,
// R1-point DFT, twiddles, LDS; R2-point DFT; real and imaginary parts are the
// two rows, stored from registers.
// RP row pairs per workgroup (16, 8 or 4: from the LDS budget of the FFT
// tiles, which the autotuner chooses).

template <int R1, int R2, int RP, class T>
__global__ __launch_bounds__(RP*(R1 > R2 ? R1 : R2)) void k_fft_x2_r2c(const V2<T>* __restrict__ wn, int nrows,
                                                                       const T* __restrict__ grid,
                                                                       V2<T>* __restrict__ spec) {
    chain_priority();
    using C = V2<T>;
    constexpr int N = R1 * R2, X = N / 2 + 1;
    __shared__ C sm[N * RP];
    const int p0 = blockIdx.x * RP;
    {
        const int n2 = threadIdx.x % R2, pr = threadIdx.x / R2;
        const int r0 = 2 * (p0 + pr), r1 = r0 + 1;
        if (pr < RP) {
            C v[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) {
                const int k = R2 * n1 + n2;
                const T re = (r0 < nrows) ? grid[(size_t)r0 * N + k] : T(0);
                const T im = (r1 < nrows) ? grid[(size_t)r1 * N + k] : T(0);
                v[n1] = cmk<C>(re, im);
            }
            dft<R1, -1>(v);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1)
                sm[pr * N + k1 * R2 + n2] = (k1 == 0 || n2 == 0) ? v[k1] : cmul(v[k1], wn[(n2 * k1) % N]);
        }
    }
    __syncthreads();
    C u[R2];
    const int k1 = threadIdx.x % R1, pb = threadIdx.x / R1;
    if (pb < RP) {
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) u[n2] = sm[pb * N + k1 * R2 + n2];
        dft<R2, -1>(u);
    }
    __syncthreads();
    if (pb < RP) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) sm[pb * N + k1 + R1 * k2] = u[k2];
    }
    __syncthreads();
    const T h = T(0.5);
    for (int idx = threadIdx.x; idx < RP * X; idx += blockDim.x) {
        const int pr = idx / X, m = idx - pr * X;
        const int r0 = 2 * (p0 + pr), r1 = r0 + 1;
        if (r0 >= nrows) continue;
        const C z = sm[pr * N + m];
        const C zr = sm[pr * N + (m == 0 ? 0 : N - m)];
        spec[(size_t)r0 * X + m] = cmk<C>(h * (z.x + zr.x), h * (z.y - zr.y));
        if (r1 < nrows) spec[(size_t)r1 * X + m] = cmk<C>(h * (z.y + zr.y), -h * (z.x - zr.x));
    }
}

template <int R1, int R2, int RP, class T>
__global__ __launch_bounds__(RP*(R1 > R2 ? R1 : R2)) void k_fft_x2_c2r(const V2<T>* __restrict__ wn, int nrows,
                                                                       const V2<T>* __restrict__ spec,
                                                                       T* __restrict__ grid) {
    chain_priority();
    using C = V2<T>;
    constexpr int N = R1 * R2, X = N / 2 + 1;
    __shared__ C sm[N * RP];
    const int p0 = blockIdx.x * RP;
    {
        const int n2 = threadIdx.x % R2, pr = threadIdx.x / R2;
        const int r0 = 2 * (p0 + pr), r1 = r0 + 1;
        if (pr < RP) {
            C v[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) {
                const int m = R2 * n1 + n2;
                C A = cmk<C>(T(0), T(0)), B = cmk<C>(T(0), T(0));
                if (m < X) {
                    if (r0 < nrows) A = spec[(size_t)r0 * X + m];
                    if (r1 < nrows) B = spec[(size_t)r1 * X + m];
                } else {
                    if (r0 < nrows) A = spec[(size_t)r0 * X + (N - m)];
                    if (r1 < nrows) B = spec[(size_t)r1 * X + (N - m)];
                    A.y = -A.y;
                    B.y = -B.y;
                }
                v[n1] = cmk<C>(A.x - B.y, A.y + B.x);
            }
            dft<R1, 1>(v);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                C w = wn[(n2 * k1) % N];
                w.y = -w.y;
                sm[pr * N + k1 * R2 + n2] = (k1 == 0 || n2 == 0) ? v[k1] : cmul(v[k1], w);
            }
        }
    }
    __syncthreads();
    const int k1 = threadIdx.x % R1, pb = threadIdx.x / R1;
    if (pb < RP) {
        C u[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) u[n2] = sm[pb * N + k1 * R2 + n2];
        dft<R2, 1>(u);
        const int r0 = 2 * (p0 + pb), r1 = r0 + 1;
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            if (r0 < nrows) grid[(size_t)r0 * N + k1 + R1 * k2] = u[k2].x;
            if (r1 < nrows) grid[(size_t)r1 * N + k1 + R1 * k2] = u[k2].y;
        }
    }
}

// Sum of n partials in a fixed order: thread t adds t, t + 1024, ... with four
// independent accumulators (loads in flight together), then a block tree.
__global__ __launch_bounds__(1024) void k_sum_part(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[16];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
        a0 += part[i];
        a1 += part[i + 1024];
        a2 += part[i + 2 * 1024];
        a3 += part[i + 3 * 1024];
    }
    for (; i < n; i += 1024) a0 += part[i];
    const double v = block_sum<1024>((a0 + a1) + (a2 + a3), red);
    if (threadIdx.x == 0) *out = v;
}

// ---------------------------------------------------------------------------
// host side: plans, twiddles, influence tables
// ---------------------------------------------------------------------------
static void factorize(int n, std::vector<int>& r) {
    r.clear();
    while (n % 16 == 0) {
        r.push_back(16);
        n /= 16;
    }
    if (n % 8 == 0) {
        r.push_back(8);
        n /= 8;
    }
    while (n % 9 == 0) {
        r.push_back(9);
        n /= 9;
    }
    while (n % 4 == 0) {
        r.push_back(4);
        n /= 4;
    }
    while (n % 2 == 0) {
        r.push_back(2);
        n /= 2;
    }
    while (n % 3 == 0) {
        r.push_back(3);
        n /= 3;
    }
    while (n % 5 == 0) {
        r.push_back(5);
        n /= 5;
    }
    if (n != 1) throw Error(PQ_ERR_BOX, "PME grid sizes must have no prime factor other than 2, 3, 5");
}

// Cardinal B-spline M_p at x (FP64, host), Cox-de Boor recursion.
static double bspline_host(int p, double x) {
    if (p == 2) return (x >= 0.0 && x <= 2.0) ? 1.0 - std::fabs(x - 1.0) : 0.0;
    return (x * bspline_host(p - 1, x) + (p - x) * bspline_host(p - 1, x - 1.0)) / (p - 1);
}

// |b(m)|^2 of the smooth PME structure-factor approximation; a vanishing
// denominator (odd order, m = K/2) takes the mean of its neighbours.
static std::vector<double> euler_factors(int K, int p) {
    std::vector<double> out(K), den(K);
    for (int m = 0; m < K; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= p - 2; ++k) {
            const double Mk = bspline_host(p, k + 1.0);
            const double ang = 2.0 * PI * (double)m * k / K;
            re += Mk * std::cos(ang);
            im += Mk * std::sin(ang);
        }
        den[m] = re * re + im * im;
    }
    for (int m = 0; m < K; ++m) out[m] = den[m] < 1e-10 ? 0.0 : 1.0 / den[m];
    for (int m = 0; m < K; ++m)
        if (den[m] < 1e-10) out[m] = 0.5 * (out[(m + K - 1) % K] + out[(m + 1) % K]);
    return out;
}

static FftDev to_dev(const Fft1D& f) {
    FftDev d;
    d.n = f.n;
    d.nst = f.nst;
    d.ntw = f.ntw;
    for (int i = 0; i < FFT_MAX_STAGES; ++i) {
        d.radix[i] = f.radix[i];
        d.ns[i] = f.ns[i];
        d.twoff[i] = f.twoff[i];
    }
    return d;
}

template <class T>
static void upload_twiddles(Ctx& c, const std::vector<double>& tw, const int* off, const int* woff) {
    std::vector<V2<T>> h(tw.size() / 2);
    for (size_t i = 0; i < h.size(); ++i) h[i] = mk2<T>((T)tw[2 * i], (T)tw[2 * i + 1]);
    c.twid.ensure(std::max<size_t>(1, h.size()) * sizeof(V2<T>));
    PQ_HIP(hipMemcpy(c.twid.p, h.data(), h.size() * sizeof(V2<T>), hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) {
        c.fft[d].tw = as<V2<T>>(c.twid) + off[d];
        c.fft[d].wn = as<V2<T>>(c.twid) + woff[d];
    }
}

// Register radices (R1 >= R2, the smallest R1) with R1 R2 = n, or 0, 0. The
// composite radices 6, 10 and 12 are taken only for lengths with no pair of
// the others (30, 50, 54, 60, 90, 96, 100, 120).
static void col2_radices(int n, int& r1, int& r2) {
    static const int R[] = {2, 3, 4, 5, 8, 9, 16};
    static const int RX[] = {2, 3, 4, 5, 6, 8, 9, 10, 12, 16};
    r1 = r2 = 0;
    for (int a : R)
        for (int b : R)
            if (b <= a && a * b == n && (r1 == 0 || a < r1)) {
                r1 = a;
                r2 = b;
            }
    if (r1 != 0) return;
    for (int a : RX)
        for (int b : RX)
            if (b <= a && a * b == n && (r1 == 0 || a < r1)) {
                r1 = a;
                r2 = b;
            }
}

void fft_setup(Ctx& c) {
    // twiddle and influence tables depend only on the grid, the spline order,
    // alpha, the box and the precision: kept when none of them changed
    const double key[12] = {(double)c.K[0], (double)c.K[1], (double)c.K[2], (double)c.P, c.prm.alpha,
                            c.prm.box[0],   c.prm.box[1],   c.prm.box[2],   c.prm.tilt[0], c.prm.tilt[1],
                            c.prm.tilt[2],  c.fp64 ? 1.0 : 0.0};
    if (c.fft_key_valid && std::equal(key, key + 12, c.fft_key)) return;
    c.fft_key_valid = false;
    std::vector<double> tw;   // interleaved (cos, sin), rounded to the bulk precision on upload
    int off[3];
    for (int d = 0; d < 3; ++d) {
        Fft1D& f = c.fft[d];
        f.n = c.K[d];
        std::vector<int> rad;
        factorize(f.n, rad);
        PQ_REQUIRE((int)rad.size() <= FFT_MAX_STAGES, PQ_ERR_BOX, "PME grid too large");
        f.nst = (int)rad.size();
        off[d] = (int)tw.size() / 2;
        int ns = 1;
        for (int st = 0; st < f.nst; ++st) {
            const int R = rad[st];
            f.radix[st] = R;
            f.ns[st] = ns;
            f.twoff[st] = (int)tw.size() / 2 - off[d];
            for (int k = 0; k < ns; ++k)
                for (int r = 1; r < R; ++r) {
                    const double ang = -2.0 * PI * (double)k * r / ((double)ns * R);
                    tw.push_back(std::cos(ang));
                    tw.push_back(std::sin(ang));
                }
            ns *= R;
        }
        for (int st = f.nst; st < FFT_MAX_STAGES; ++st) f.radix[st] = f.ns[st] = f.twoff[st] = 0;
        f.ntw = (int)tw.size() / 2 - off[d];
    }
    int woff[3];
    for (int d = 0; d < 3; ++d) {
        Fft1D& f = c.fft[d];
        col2_radices(f.n, f.r1, f.r2);
        woff[d] = (int)tw.size() / 2;
        for (int e = 0; e < f.n; ++e) {
            const double ang = -2.0 * PI * (double)e / f.n;
            tw.push_back(std::cos(ang));
            tw.push_back(std::sin(ang));
        }
    }
    if (c.fp64)
        upload_twiddles<double>(c, tw, off, woff);
    else
        upload_twiddles<float>(c, tw, off, woff);

    // influence tables
    const double a = c.prm.alpha;
    std::vector<double> tab;
    int toff[3], soff[3], boff[3], moff[3];
    for (int d = 0; d < 3; ++d) {
        const int K = c.K[d];
        const double L = c.prm.box[d];
        std::vector<double> B = euler_factors(K, c.P);
        toff[d] = (int)tab.size();
        for (int m = 0; m < K; ++m) {
            const double mp = (m <= K / 2) ? m : m - K;
            const double S = (mp / L) * (mp / L);
            tab.push_back(B[m] * std::exp(-PI * PI * S / (a * a)));
        }
        soff[d] = (int)tab.size();
        for (int m = 0; m < K; ++m) {
            const double mp = (m <= K / 2) ? m : m - K;
            tab.push_back((mp / L) * (mp / L));
        }
        boff[d] = (int)tab.size();
        for (int m = 0; m < K; ++m) tab.push_back(B[m]);
        moff[d] = (int)tab.size();
        for (int m = 0; m < K; ++m) tab.push_back((m <= K / 2) ? (double)m : (double)(m - K));
    }
    c.inftab.ensure(tab.size());
    PQ_HIP(hipMemcpy(c.inftab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) {
        c.inf.T[d] = c.inftab.p + toff[d];
        c.inf.S[d] = c.inftab.p + soff[d];
        c.inf.B[d] = c.inftab.p + boff[d];
        c.inf.M[d] = c.inftab.p + moff[d];
    }
    const double V = c.prm.box[0] * c.prm.box[1] * c.prm.box[2];
    c.inf.scale = 1.0 / (PI * V);
    {
        const double L0 = c.prm.box[0], L1 = c.prm.box[1], L2 = c.prm.box[2];
        const double txy = c.prm.tilt[0], txz = c.prm.tilt[1], tyz = c.prm.tilt[2];
        c.inf.tric = is_tric(c.prm) ? 1 : 0;
        c.inf.r00 = 1.0 / L0;
        c.inf.r11 = 1.0 / L1;
        c.inf.r22 = 1.0 / L2;
        c.inf.r10 = -txy / (L0 * L1);
        c.inf.r21 = -tyz / (L1 * L2);
        c.inf.r20 = (txy * tyz - L1 * txz) / (L0 * L1 * L2);
        c.inf.pa2 = PI * PI / (a * a);
    }
    std::copy(key, key + 12, c.fft_key);
    c.fft_key_valid = true;
}

// LDS budget of one FFT workgroup: two ping-pong buffers of `budget` bytes
// each (a tuning choice: smaller tiles leave room for kernels running beside
// the FFT; every tile gives the same results).
static int col_tile(int n, size_t esz, int budget) { return std::max(1, std::min(16, (int)(budget / (n * esz)))); }
static int row_pairs(int n, size_t esz, int budget) { return std::max(1, (int)(budget / (n * esz))); }

// The two-radix column transform for (r1, r2) of one axis; false if that
// pair has no instance (the caller then takes the Stockham kernel).
template <int SIGN, bool CONV, class T>
static bool col2_launch(int r1, int r2, dim3 grid, hipStream_t s, const V2<T>* wn, int X, size_t es, size_t os,
                        V2<T>* spec, const ConvArgs& cv, double* epart) {
#define PQ_COL2(A, B)                                                                                       \
    if (r1 == A && r2 == B) {                                                                               \
        PQ_LAUNCH((k_fft_col2<A, B, SIGN, CONV, T>), grid, CT*(A > B ? A : B), 0, s, wn, X, es, os, spec, cv, \
                  epart);                                                                                   \
        return true;                                                                                        \
    }
    PQ_COL2(3, 2) PQ_COL2(4, 2) PQ_COL2(3, 3) PQ_COL2(5, 2) PQ_COL2(4, 3) PQ_COL2(5, 3) PQ_COL2(4, 4)
    PQ_COL2(9, 2) PQ_COL2(5, 4) PQ_COL2(8, 3) PQ_COL2(5, 5) PQ_COL2(9, 3) PQ_COL2(8, 4) PQ_COL2(9, 4)
    PQ_COL2(8, 5) PQ_COL2(9, 5) PQ_COL2(16, 3) PQ_COL2(8, 8) PQ_COL2(9, 8) PQ_COL2(16, 5) PQ_COL2(9, 9)
    PQ_COL2(16, 8) PQ_COL2(16, 9) PQ_COL2(16, 16)
    PQ_COL2(6, 5) PQ_COL2(10, 5) PQ_COL2(9, 6) PQ_COL2(10, 6) PQ_COL2(10, 9) PQ_COL2(12, 8) PQ_COL2(10, 10)
    PQ_COL2(12, 10)
#undef PQ_COL2
    return false;
}

// The two-radix x passes for (r1, r2); false if that pair has no instance.
template <bool FWD, int RP, class T>
static bool x2_launch_rp(int r1, int r2, int npairs, hipStream_t s, const V2<T>* wn, int nrows, T* grid,
                         V2<T>* spec) {
#define PQ_X2(A, B)                                                                                          \
    if (r1 == A && r2 == B) {                                                                                \
        if (FWD)                                                                                             \
            PQ_LAUNCH((k_fft_x2_r2c<A, B, RP, T>), cdiv(npairs, RP), RP*(A > B ? A : B), 0, s, wn, nrows,      \
                      (const T*)grid, spec);                                                                 \
        else                                                                                                 \
            PQ_LAUNCH((k_fft_x2_c2r<A, B, RP, T>), cdiv(npairs, RP), RP*(A > B ? A : B), 0, s, wn, nrows,      \
                      (const V2<T>*)spec, grid);                                                             \
        return true;                                                                                         \
    }
    PQ_X2(3, 2) PQ_X2(4, 2) PQ_X2(3, 3) PQ_X2(5, 2) PQ_X2(4, 3) PQ_X2(5, 3) PQ_X2(4, 4) PQ_X2(9, 2)
    PQ_X2(5, 4) PQ_X2(8, 3) PQ_X2(5, 5) PQ_X2(9, 3) PQ_X2(8, 4) PQ_X2(9, 4) PQ_X2(8, 5) PQ_X2(9, 5)
    PQ_X2(16, 3) PQ_X2(8, 8) PQ_X2(9, 8) PQ_X2(16, 5) PQ_X2(9, 9) PQ_X2(16, 8) PQ_X2(16, 9) PQ_X2(16, 16)
    PQ_X2(6, 5) PQ_X2(10, 5) PQ_X2(9, 6) PQ_X2(10, 6) PQ_X2(10, 9) PQ_X2(12, 8) PQ_X2(10, 10) PQ_X2(12, 10)
#undef PQ_X2
    return false;
}
// row pairs per workgroup from the LDS budget: RP n complex values
template <bool FWD, class T>
static bool x2_launch(int r1, int r2, int npairs, hipStream_t s, const V2<T>* wn, int nrows, T* grid, V2<T>* spec,
                      int budget) {
    const size_t row = (size_t)r1 * r2 * sizeof(V2<T>);
    if ((size_t)budget >= 16 * row) return x2_launch_rp<FWD, 16, T>(r1, r2, npairs, s, wn, nrows, grid, spec);
    if ((size_t)budget >= 8 * row) return x2_launch_rp<FWD, 8, T>(r1, r2, npairs, s, wn, nrows, grid, spec);
    return x2_launch_rp<FWD, 4, T>(r1, r2, npairs, s, wn, nrows, grid, spec);
}

template <class T>
static void fft_convolve_t(Ctx& c, hipStream_t s) {
    using C = V2<T>;
    const size_t esz = sizeof(C);
    const int K0 = c.K[0], K1 = c.K[1], K2 = c.K[2];
    const int X = K0 / 2 + 1;
    const int nrows = K1 * K2;
    const FftDev px = to_dev(c.fft[0]), py = to_dev(c.fft[1]), pz = to_dev(c.fft[2]);
    const C* tw0 = static_cast<const C*>(c.fft[0].tw);
    const C* tw1 = static_cast<const C*>(c.fft[1].tw);
    const C* tw2 = static_cast<const C*>(c.fft[2].tw);
    T* grid = as<T>(c.grid);
    C* spec = as<C>(c.spec);
    const InfTab& it = c.inf;
    ConvArgs cv{it.T[0], it.T[1], it.T[2], it.S[0], it.S[1], it.S[2], it.scale, K0,
                it.tric, it.B[0], it.B[1], it.B[2], it.M[0], it.M[1], it.M[2],
                it.r00, it.r10, it.r11, it.r20, it.r21, it.r22, it.pa2};
    const int np = row_pairs(K0, esz, c.fft_budget);
    const int npairs = (nrows + 1) / 2;
    const C* wn0 = static_cast<const C*>(c.fft[0].wn);
    const int x1 = c.fft[0].r1, x2 = c.fft[0].r2;
    // x forward
    if (!x2_launch<true, T>(x1, x2, npairs, s, wn0, nrows, grid, spec, c.fft_budget))
        PQ_LAUNCH(k_fft_x_r2c<T>, cdiv(npairs, np), 256, (2 * np * K0 + px.ntw) * esz, s, px, tw0, nrows, np, grid,
                  spec);
    const C* wn1 = static_cast<const C*>(c.fft[1].wn);
    const C* wn2 = static_cast<const C*>(c.fft[2].wn);
    const int y1 = c.fft[1].r1, y2 = c.fft[1].r2, z1 = c.fft[2].r1, z2 = c.fft[2].r2;
    // y forward: sequences over (z, mx), elements stride X
    const int ty = col_tile(K1, esz, c.fft_budget);
    if (!col2_launch<-1, false, T>(y1, y2, dim3(cdiv(X, CT), K2), s, wn1, X, (size_t)X, (size_t)X * K1, spec, cv,
                                   (double*)nullptr))
        PQ_LAUNCH((k_fft_col<-1, false, T>), dim3(cdiv(X, ty), K2), 256, (2 * K1 * ty + py.ntw) * esz, s, py, tw1, X,
                  ty, (size_t)X, (size_t)X * K1, spec, cv, (double*)nullptr);
    // z forward + convolution + z inverse: sequences over (y, mx), elements stride X*K1
    const int tz = col_tile(K2, esz, c.fft_budget);
    // one energy partial per spectral column (mx, my); sized by set_system
    PQ_REQUIRE(c.ews.part_n >= (size_t)X * K1 + 16, PQ_ERR_STATE, "energy partials not sized");
    double* ep = c.want_energy ? c.ews.part : nullptr;
    if (!col2_launch<-1, true, T>(z1, z2, dim3(cdiv(X, CT), K1), s, wn2, X, (size_t)X * K1, (size_t)X, spec, cv, ep))
        PQ_LAUNCH((k_fft_col<-1, true, T>), dim3(cdiv(X, tz), K1), 256, (2 * K2 * tz + pz.ntw) * esz, s, pz, tw2, X,
                  tz, (size_t)X * K1, (size_t)X, spec, cv, ep);
    if (c.want_energy) PQ_LAUNCH(k_sum_part, 1, 1024, 0, s, c.ews.part, X * K1, c.ews.scal + 1);
    // y inverse
    if (!col2_launch<1, false, T>(y1, y2, dim3(cdiv(X, CT), K2), s, wn1, X, (size_t)X, (size_t)X * K1, spec, cv,
                                  (double*)nullptr))
        PQ_LAUNCH((k_fft_col<1, false, T>), dim3(cdiv(X, ty), K2), 256, (2 * K1 * ty + py.ntw) * esz, s, py, tw1, X,
                  ty, (size_t)X, (size_t)X * K1, spec, cv, (double*)nullptr);
    // x inverse
    if (!x2_launch<false, T>(x1, x2, npairs, s, wn0, nrows, grid, spec, c.fft_budget))
        PQ_LAUNCH(k_fft_x_c2r<T>, cdiv(npairs, np), 256, (2 * np * K0 + px.ntw) * esz, s, px, tw0, nrows, np, spec,
                  grid);
}

// grid (real, Q) -> grid (real, psi = conv(Q)); E_rec (without KE) into c.ews.scal[1]
// when c.want_energy
void fft_convolve(Ctx& c, hipStream_t s) {
    if (c.fp64)
        fft_convolve_t<double>(c, s);
    else
        fft_convolve_t<float>(c, s);
}

}  // namespace pq
