// Internal declarations of the pmeqeq HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "pmeqeq.h"

namespace pq {

constexpr double KE = 14.3996454784;   // e^2/(4 pi eps0), eV*A
constexpr double PI = 3.14159265358979323846;

struct Error : std::runtime_error {
    pq_status code;
    Error(pq_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PQ_HIP(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::pq::Error(PQ_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define PQ_REQUIRE(cond, code, msg)                    \
    do {                                               \
        if (!(cond)) throw ::pq::Error((code), (msg)); \
    } while (0)

#define PQ_LAUNCH(kern, grid, block, shmem, stream, ...)                               \
    do {                                                                               \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
        PQ_HIP(hipGetLastError());                                                     \
    } while (0)

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Device buffer owned by a context; grows on demand, never shrinks.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void ensure(size_t m) {
        if (m <= n) return;
        release();
        if (m == 0) return;
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, m * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(PQ_ERR_NOMEM, "hipMalloc of " + std::to_string(m * sizeof(T)) + " bytes failed");
        }
        p = static_cast<T*>(q);
        n = m;
    }
    void release() {
        // kernels queued on any stream may still use the old buffer
        if (p) (void)hipDeviceSynchronize();
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

constexpr int CL = 8;           // atoms per cluster
constexpr int RED_BLOCKS = 512; // blocks of the FP64 partial-sum reductions

// Geometry of the cluster (column) decomposition used by the neighbour list.
struct Geom {
    double L[3], invL[3];
    int ncx, ncy;     // column grid in x, y
    double wx, wy;    // column widths
    double rc, rlist; // cutoff and list radius
    int Rx, Ry, Rz;   // column and z-image search ranges
};

// 1-D FFT plan (mixed radix 2/3/4/5 Stockham), twiddles in a device table.
constexpr int FFT_MAX_STAGES = 12;
struct Fft1D {
    int n = 0;
    int nst = 0;
    int radix[FFT_MAX_STAGES];
    int ns[FFT_MAX_STAGES];     // product of the radices of earlier stages
    int twoff[FFT_MAX_STAGES];  // offset of the stage's twiddles in the table
    const void* tw = nullptr;   // V2<T> exp(-2 pi i k r / (ns*R)) for k < ns, 1 <= r < R
};

// Per-axis influence-function tables (without KE and 1/(pi V)):
//   T_d(m) = |b_d(m)|^2 exp(-pi^2 m'^2 / (a^2 L_d^2)),   S_d(m) = m'^2 / L_d^2.
struct InfTab {
    const double* T[3];
    const double* S[3];
    double scale;     // 1 / (pi V)
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool have_system = false;
    bool fp64 = false;       // bulk arithmetic in FP64 (PQ_FLAG_FP64) instead of FP32
    int64_t n = 0;
    pq_params prm{};
    Geom g{};

    // --- neighbour list (set_system) ---
    int ncol = 0, ncl = 0;
    int64_t nlist = 0;
    DBuf<double> w64;        // wrapped FP64 positions, original order, n*3
    DBuf<int> col_of;        // column of each atom
    DBuf<int> col_cnt;       // atoms per column
    DBuf<int> col_start;     // ncol+1, atom offsets per column (unpadded)
    DBuf<int> col_fill;      // fill counters
    DBuf<int> col_cl;        // ncol+1, cluster offsets per column
    DBuf<int> tmp_atoms;     // atoms grouped by column, unordered
    DBuf<int> orig;          // slot -> original atom (-1 padding), ncl*8
    DBuf<unsigned char> xyzq; // slot-ordered V4<T>: offset from the cluster reference + charge
    DBuf<double> cl_ref;     // ncl*3 reference points
    DBuf<double> cl_lo;      // ncl*3 bounding boxes
    DBuf<double> cl_hi;
    DBuf<int> cl_col;        // column of each cluster
    DBuf<int> lcount;        // ncl+1
    DBuf<int> lstart;        // ncl+1
    DBuf<int2> lj;           // list: (j cluster, packed image vector)
    DBuf<unsigned char> ls;   // list: V4<T> shift ref_j + nL - ref_i
    DBuf<int> flag;          // device error flags
    DBuf<unsigned long long> counter;

    // --- PME ---
    int K[3] = {0, 0, 0}, P = 0, B = 8;
    int nb[3] = {0, 0, 0}, nbrick = 0;
    DBuf<int> brick_of, brick_cnt, brick_start, brick_fill;
    DBuf<int> pme_idx;       // brick-ordered original indices
    DBuf<unsigned char> pme_frac; // V4<T>: fractional parts + packed base index
    DBuf<unsigned char> pme_w;    // T: B-spline weights per atom, 3 x 8 (brick order)
    DBuf<unsigned char> grid;     // T: real grid K1*K2*K3 (x fastest)
    DBuf<unsigned char> stage;    // T: per-brick spreading regions (B+p-1)^3
    DBuf<unsigned char> spec;     // V2<T>: half spectrum (K1/2+1)*K2*K3
    DBuf<unsigned char> twid;     // V2<T>: FFT twiddles of the three axes
    DBuf<double> inftab;     // T and S tables (FP64)
    Fft1D fft[3];
    InfTab inf{};

    // --- direct Ewald ---
    int nk = 0;
    DBuf<int4> kn;           // half-space integer k vectors
    DBuf<double> kc;         // c_k = (4 pi / V) exp(-k^2/4a^2)/k^2
    DBuf<double2> sfac;      // structure factors

    // --- per-evaluation scratch ---
    DBuf<unsigned char> phi_r, phi_k;   // T per atom (original order, without KE)
    DBuf<unsigned char> f_r, f_k;       // V4<T> per atom
    DBuf<double> part;       // reduction partials
    DBuf<double> scal;       // small device scalars
    double* pinned = nullptr;// pinned host scalars

    // --- second stream: the pair kernel overlaps the PME chain ---
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // --- phase timing ---
    bool timing = false;
    bool serial = false;     // run the pair kernel on the main stream (phase timing mode 2)
    std::vector<hipEvent_t> ev_pool;          // free events
    std::vector<std::vector<hipEvent_t>> ev_pending;   // PQ_NPHASE*2 events per timed evaluation

    // --- Krylov workspace ---
    DBuf<double> kv;         // basis vectors (m+1) x ld
    DBuf<double> kw;         // work vectors
    DBuf<double> kh;         // Hessenberg and small solver state
    DBuf<double> kf;         // force scratch n*3 (x2)
    size_t kld = 0;
    int km = 0;

    ~Ctx();
};

// Typed view of a precision-dependent byte buffer.
template <class X>
inline X* as(DBuf<unsigned char>& b) {
    return reinterpret_cast<X*>(b.p);
}
// Bytes of one bulk real number (4: FP32 form, 8: FP64 form).
inline size_t rsz(const Ctx& c) { return c.fp64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
// nbr.hip
void scan_ints(const int* in, int* out, int n, bool ceil8, hipStream_t s);  // exclusive; out[n] = total
void nbr_build(Ctx& c, const double* pos);
int64_t nbr_export_pairs(Ctx& c, int64_t cap, int32_t* pairs);
// pair.hip: outputs in original atom order, without KE; force includes q_i
void stage_charges(Ctx& c, const double* q, hipStream_t s);
void pair_sum(Ctx& c, bool force, hipStream_t s);   // into c.phi_r, c.f_r
// pme.hip
void pme_setup(Ctx& c);
// ev: 2*PQ_NPHASE timing events or NULL (spread, FFT and gather phases are recorded)
void pme_eval(Ctx& c, const double* q, bool force, hipEvent_t* ev, hipStream_t s);   // into c.phi_k, c.f_k
// fft.hip
void fft_setup(Ctx& c);
void fft_convolve(Ctx& c, hipStream_t s);   // grid -> psi in place; energy partials into c.part
// ewald.hip
void ewald_setup(Ctx& c);
void ewald_eval(Ctx& c, const double* q, bool force, hipStream_t s);   // into c.phi_k, c.f_k
// vec.hip
void sum_vector(Ctx& c, const double* x, int64_t n, double* out, hipStream_t s);
void dot_vector(Ctx& c, const double* x, const double* y, int64_t n, double* out, hipStream_t s);
void combine(Ctx& c, const double* q, const double* Q, double* phi, double* force,
             double* energy, hipStream_t s);

// high-level evaluation used by the ABI and the Krylov solvers (abi.cpp)
void coulomb_eval(Ctx& c, const double* q, double* phi, double* force, double* energy,
                  hipStream_t s);

}  // namespace pq
