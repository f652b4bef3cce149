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
// Each 1-D transform runs in LDS as mixed-radix (2, 3, 4, 5) Stockham passes
// (self-sorting, ping-pong buffers), twiddles from FP64 tables rounded to the
// bulk precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "dev.h"
#include "pq_internal.h"

namespace pq {

struct FftDev {
    int n, nst;
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

// In-register DFT of length R with kernel exp(SIGN 2 pi i r s / R).
template <int R, int SIGN, class C>
__device__ __forceinline__ void dft(C* v) {
    using T = decltype(C::x);
    if (R == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 3) {
        const T c = T(-0.5), s = T(0.86602540378443864676);
        C t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        C a = cmk<C>(v[0].x + c * t1.x, v[0].y + c * t1.y);
        C b = mul_i<SIGN>(cmk<C>(s * t2.x, s * t2.y));
        v[0] = cadd(v[0], t1);
        v[1] = cadd(a, b);
        v[2] = csub(a, b);
    } else if (R == 4) {
        C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        C s13 = cadd(v[1], v[3]), d13 = mul_i<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if (R == 5) {
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
                default: butterfly<5, SIGN>(a, b, twst, j, m, Ns, s, es, ss); break;
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
    using C = V2<T>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C* sm = reinterpret_cast<C*>(smraw);
    const int n = pl.n, X = n / 2 + 1;
    C* a = sm;
    C* b = sm + np * n;
    const int p0 = blockIdx.x * np;
    for (int idx = threadIdx.x; idx < np * n; idx += blockDim.x) {
        const int s = idx / n, k = idx % n;
        const int r0 = 2 * (p0 + s), r1 = r0 + 1;
        const T re = (r0 < nrows) ? grid[(size_t)r0 * n + k] : T(0);
        const T im = (r1 < nrows) ? grid[(size_t)r1 * n + k] : T(0);
        a[s * n + k] = cmk<C>(re, im);
    }
    __syncthreads();
    const C* o = fft_lds<-1, false>(a, b, pl, tw, np, 1, n);
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
    using C = V2<T>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C* sm = reinterpret_cast<C*>(smraw);
    const int n = pl.n, X = n / 2 + 1;
    C* a = sm;
    C* b = sm + np * n;
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
    const C* o = fft_lds<1, false>(a, b, pl, tw, np, 1, n);
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
};

template <int SIGN, bool CONV, class T>
__global__ __launch_bounds__(256) void k_fft_col(FftDev pl, const V2<T>* __restrict__ tw, int X, int tx,
                                                 size_t estride, size_t ostride, V2<T>* __restrict__ spec,
                                                 ConvArgs cv, double* __restrict__ epart) {
    using C = V2<T>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C* sm = reinterpret_cast<C*>(smraw);
    __shared__ double red[4];
    const int n = pl.n;
    C* a = sm;
    C* b = sm + n * tx;
    const int mx0 = blockIdx.x * tx;
    const int o = blockIdx.y;
    C* base = spec + (size_t)o * ostride;
    for (int idx = threadIdx.x; idx < n * tx; idx += blockDim.x) {
        const int k = idx / tx, s = idx % tx;
        const int mx = mx0 + s;
        a[idx] = (mx < X) ? base[(size_t)k * estride + mx] : cmk<C>(T(0), T(0));
    }
    __syncthreads();
    C* r = fft_lds<SIGN, true>(a, b, pl, tw, tx, tx, 1);
    if (CONV) {
        // r holds F(mx, my = o, mz = k); multiply by G and sum the energy
        double e = 0.0;
        const int my = o;
        for (int idx = threadIdx.x; idx < n * tx; idx += blockDim.x) {
            const int mz = idx / tx, s = idx % tx;
            const int mx = mx0 + s;
            T gk = T(0);
            if (mx < X && (mx | my | mz) != 0) {
                const double g = cv.scale * cv.T0[mx] * cv.T1[my] * cv.T2[mz] / (cv.S0[mx] + cv.S1[my] + cv.S2[mz]);
                gk = (T)g;
                const C v = r[idx];
                const double wgt = (mx == 0 || (2 * mx == cv.K0)) ? 1.0 : 2.0;
                e += wgt * g * ((double)v.x * v.x + (double)v.y * v.y);
            }
            r[idx] = cmk<C>(r[idx].x * gk, r[idx].y * gk);
        }
        e = block_sum<256>(e, red);
        if (threadIdx.x == 0) epart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = 0.5 * e;
        __syncthreads();
        C* other = (r == a) ? b : a;
        r = fft_lds<-SIGN, true>(r, other, pl, tw, tx, tx, 1);
    }
    for (int idx = threadIdx.x; idx < n * tx; idx += blockDim.x) {
        const int k = idx / tx, s = idx % tx;
        const int mx = mx0 + s;
        if (mx < X) base[(size_t)k * estride + mx] = r[idx];
    }
}

__global__ void k_sum_part(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    v = block_sum<256>(v, red);
    if (threadIdx.x == 0) *out = v;
}

// ---------------------------------------------------------------------------
// host side: plans, twiddles, influence tables
// ---------------------------------------------------------------------------
static void factorize(int n, std::vector<int>& r) {
    r.clear();
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
    for (int i = 0; i < FFT_MAX_STAGES; ++i) {
        d.radix[i] = f.radix[i];
        d.ns[i] = f.ns[i];
        d.twoff[i] = f.twoff[i];
    }
    return d;
}

template <class T>
static void upload_twiddles(Ctx& c, const std::vector<double>& tw, const int* off) {
    std::vector<V2<T>> h(tw.size() / 2);
    for (size_t i = 0; i < h.size(); ++i) h[i] = mk2<T>((T)tw[2 * i], (T)tw[2 * i + 1]);
    c.twid.ensure(std::max<size_t>(1, h.size()) * sizeof(V2<T>));
    PQ_HIP(hipMemcpy(c.twid.p, h.data(), h.size() * sizeof(V2<T>), hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) c.fft[d].tw = as<V2<T>>(c.twid) + off[d];
}

void fft_setup(Ctx& c) {
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
    }
    if (c.fp64)
        upload_twiddles<double>(c, tw, off);
    else
        upload_twiddles<float>(c, tw, off);

    // influence tables
    const double a = c.prm.alpha;
    std::vector<double> tab;
    int toff[3], soff[3];
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
    }
    c.inftab.ensure(tab.size());
    PQ_HIP(hipMemcpy(c.inftab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) {
        c.inf.T[d] = c.inftab.p + toff[d];
        c.inf.S[d] = c.inftab.p + soff[d];
    }
    const double V = c.prm.box[0] * c.prm.box[1] * c.prm.box[2];
    c.inf.scale = 1.0 / (PI * V);
}

// LDS budget of one FFT workgroup: two ping-pong buffers of 18 KiB.
static int col_tile(int n, size_t esz) { return std::max(1, std::min(16, (int)(18432 / (n * esz)))); }
static int row_pairs(int n, size_t esz) { return std::max(1, (int)(18432 / (n * esz))); }

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
    ConvArgs cv{c.inf.T[0], c.inf.T[1], c.inf.T[2], c.inf.S[0], c.inf.S[1], c.inf.S[2], c.inf.scale, K0};
    const int np = row_pairs(K0, esz);
    const int npairs = (nrows + 1) / 2;
    // x forward
    PQ_LAUNCH(k_fft_x_r2c<T>, cdiv(npairs, np), 256, 2 * np * K0 * esz, s, px, tw0, nrows, np, grid, spec);
    // y forward: sequences over (z, mx), elements stride X
    const int ty = col_tile(K1, esz);
    PQ_LAUNCH((k_fft_col<-1, false, T>), dim3(cdiv(X, ty), K2), 256, 2 * K1 * ty * esz, s, py, tw1, X, ty,
              (size_t)X, (size_t)X * K1, spec, cv, (double*)nullptr);
    // z forward + convolution + z inverse: sequences over (y, mx), elements stride X*K1
    const int tz = col_tile(K2, esz);
    const dim3 gz(cdiv(X, tz), K1);
    c.part.ensure((size_t)gz.x * gz.y + 16);
    PQ_LAUNCH((k_fft_col<-1, true, T>), gz, 256, 2 * K2 * tz * esz, s, pz, tw2, X, tz, (size_t)X * K1, (size_t)X,
              spec, cv, c.part.p);
    PQ_LAUNCH(k_sum_part, 1, 256, 0, s, c.part.p, (int)(gz.x * gz.y), c.scal.p + 1);
    // y inverse
    PQ_LAUNCH((k_fft_col<1, false, T>), dim3(cdiv(X, ty), K2), 256, 2 * K1 * ty * esz, s, py, tw1, X, ty, (size_t)X,
              (size_t)X * K1, spec, cv, (double*)nullptr);
    // x inverse
    PQ_LAUNCH(k_fft_x_c2r<T>, cdiv(npairs, np), 256, 2 * np * K0 * esz, s, px, tw0, nrows, np, spec, grid);
}

// grid (real, Q) -> grid (real, psi = conv(Q)); E_rec (without KE) into c.scal[1]
void fft_convolve(Ctx& c, hipStream_t s) {
    if (c.fp64)
        fft_convolve_t<double>(c, s);
    else
        fft_convolve_t<float>(c, s);
}

}  // namespace pq
