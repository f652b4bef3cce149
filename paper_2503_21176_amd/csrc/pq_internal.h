// Internal declarations of the pmeqeq HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <tuple>
#include <utility>
#include <stdexcept>
#include <string>
#include <functional>
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

// ---------------------------------------------------------------------------
// Graph recorder: while one is active on the calling thread, kernel launches
// and the fork/join event operations of an evaluation become nodes and edges
// of a HIP graph instead of running. The graph is built node by node (no
// stream capture), so no stream of the process is ever in capture mode and
// other threads can allocate, free and synchronise freely meanwhile.
// ---------------------------------------------------------------------------
struct GraphRec {
    hipGraph_t g = nullptr;
    // per stream: the nodes its next node depends on
    std::vector<std::pair<hipStream_t, std::vector<hipGraphNode_t>>> deps;
    // per recorded event: the nodes it stands for
    std::vector<std::pair<hipEvent_t, std::vector<hipGraphNode_t>>> evs;
    std::vector<hipGraphNode_t>& deps_of(hipStream_t s) {
        for (auto& d : deps)
            if (d.first == s) return d.second;
        deps.emplace_back(s, std::vector<hipGraphNode_t>{});
        return deps.back().second;
    }
    void add_kernel(const void* f, dim3 grid, dim3 block, size_t shmem, hipStream_t s, void** args) {
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(f);
        p.gridDim = grid;
        p.blockDim = block;
        p.sharedMemBytes = (unsigned)shmem;
        p.kernelParams = args;
        p.extra = nullptr;
        std::vector<hipGraphNode_t>& d = deps_of(s);
        hipGraphNode_t node = nullptr;
        PQ_HIP(hipGraphAddKernelNode(&node, g, d.empty() ? nullptr : d.data(), d.size(), &p));
        d.assign(1, node);
    }
    void record(hipEvent_t e, hipStream_t s) {
        const std::vector<hipGraphNode_t> d = deps_of(s);
        for (auto& x : evs)
            if (x.first == e) {
                x.second = d;
                return;
            }
        evs.emplace_back(e, d);
    }
    void wait(hipStream_t s, hipEvent_t e) {
        std::vector<hipGraphNode_t>& d = deps_of(s);
        for (auto& x : evs)
            if (x.first == e)
                for (hipGraphNode_t n : x.second)
                    if (std::find(d.begin(), d.end(), n) == d.end()) d.push_back(n);
    }
};
inline GraphRec*& graph_rec() {
    thread_local GraphRec* r = nullptr;
    return r;
}

template <class Tup, size_t... I>
inline void arg_ptrs(Tup& t, void** out, std::index_sequence<I...>) {
    ((out[I] = (void*)&std::get<I>(t)), ...);
}

// Launches kernel k, or adds it to the active graph recorder. The arguments
// are converted to the kernel's parameter types first.
template <class... P, class... A>
inline void launch_kernel(void (*k)(P...), dim3 grid, dim3 block, size_t shmem, hipStream_t s, A&&... a) {
    static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
    std::tuple<std::decay_t<P>...> t(std::forward<A>(a)...);
    void* args[sizeof...(P) > 0 ? sizeof...(P) : 1];
    arg_ptrs(t, args, std::index_sequence_for<P...>{});
    if (GraphRec* r = graph_rec()) {
        r->add_kernel(reinterpret_cast<const void*>(k), grid, block, shmem, s, args);
        return;
    }
    PQ_HIP(hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, args, shmem, s));
}

#define PQ_LAUNCH(kern, grid, block, shmem, stream, ...) \
    ::pq::launch_kernel(kern, dim3(grid), dim3(block), (size_t)(shmem), stream, __VA_ARGS__)

// Event record / stream wait that a graph recorder turns into edges.
inline void ev_record(hipEvent_t e, hipStream_t s) {
    if (GraphRec* r = graph_rec())
        r->record(e, s);
    else
        PQ_HIP(hipEventRecord(e, s));
}
inline void stream_wait(hipStream_t s, hipEvent_t e) {
    if (GraphRec* r = graph_rec())
        r->wait(s, e);
    else
        PQ_HIP(hipStreamWaitEvent(s, e, 0));
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Process-wide lock ordering device allocation, free and device-wide
// synchronisation against stream captures in other threads (several contexts
// may be used from several threads, as in the server): a free or a device
// synchronise must never meet a stream that is being captured.
std::recursive_mutex& device_mem_lock();

// The allocator of the context whose entry point is running on this thread
// (AllocScope sets it); null: hipMalloc / hipFree.
inline const pq_allocator*& tl_alloc() {
    thread_local const pq_allocator* a = nullptr;
    return a;
}

// Device buffer owned by a context; grows on demand, never shrinks. It
// remembers the allocator that gave it its block and returns the block there.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    pq_allocator owner{};
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void ensure(size_t m) {
        if (m <= n) return;
        std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
        release();
        if (m == 0) return;
        const size_t bytes = m * sizeof(T);
        const pq_allocator* a = tl_alloc();
        void* q = nullptr;
        if (a && a->alloc && a->free) {
            q = a->alloc(bytes, a->user_data);
            if (!q) throw Error(PQ_ERR_NOMEM, "allocator callback failed for " + std::to_string(bytes) + " bytes");
            owner = *a;
        } else {
            hipError_t e = hipMalloc(&q, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Error(PQ_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
            }
            owner = pq_allocator{};
        }
        p = static_cast<T*>(q);
        n = m;
    }
    void release() {
        if (!p) return;
        std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
        // kernels queued on any stream may still use the old buffer
        (void)hipDeviceSynchronize();
        if (owner.free)
            owner.free(p, owner.user_data);
        else
            (void)hipFree(p);
        p = nullptr;
        n = 0;
        owner = pq_allocator{};
    }
    size_t bytes() const { return n * sizeof(T); }
};

constexpr int CL = 8;           // atoms per cluster
constexpr int JL_TAIL = 256;    // padding entries after the atom-level j lists
constexpr int JL_SLOT_BITS = 24; // j-list entry word: slot in the low bits, i-atom mask above
constexpr int RED_BLOCKS = 512; // blocks of the FP64 partial-sum reductions

// Geometry of the cluster (column) decomposition used by the neighbour list.
// Triclinic cells: lattice vectors a = (L0, 0, 0), b = (txy, L1, 0),
// c = (txz, tyz, L2). Derived coefficients (host, no contraction):
// ryz = tyz/L2, cxy = txy/L1, cxz = (txz - tyz*cxy)/L2, so that the fractional
// coordinates are s2 = z/L2, s1 = (y - z*ryz)/L1, s0 = ((x - y*cxy) - z*cxz)/L0.
struct Tric {
    double txy, txz, tyz;
    double ryz, cxy, cxz;
};

struct Geom {
    double L[3], invL[3];
    int ncx, ncy;     // column grid in x, y (fractional s0, s1 when triclinic)
    double wx, wy;    // column widths (orthorhombic)
    double rc, rlist; // cutoff and list radius
    int Rx, Ry, Rz;   // column and z-image search ranges
    int tric;         // nonzero: triclinic cell, tilts in t
    Tric t;
};

// Tilt factors and fractional-coordinate coefficients of the system's cell
// (all zero for an orthorhombic box), computed without contraction.
Tric make_tric(const pq_params& p);
inline bool is_tric(const pq_params& p) { return p.tilt[0] != 0.0 || p.tilt[1] != 0.0 || p.tilt[2] != 0.0; }

// 1-D FFT plan (mixed radix 2/3/4/5 Stockham), twiddles in a device table.
constexpr int FFT_MAX_STAGES = 12;
struct Fft1D {
    int n = 0;
    int nst = 0;
    int ntw = 0;                // twiddles of all stages
    int radix[FFT_MAX_STAGES];
    int ns[FFT_MAX_STAGES];     // product of the radices of earlier stages
    int twoff[FFT_MAX_STAGES];  // offset of the stage's twiddles in the table
    const void* tw = nullptr;   // V2<T> exp(-2 pi i k r / (ns*R)) for k < ns, 1 <= r < R
    int r1 = 0, r2 = 0;         // register radices of the two-radix column transform (0: none)
    const void* wn = nullptr;   // V2<T> exp(-2 pi i e / n) for e < n
};

// Per-axis influence-function tables (without KE and 1/(pi V)):
//   T_d(m) = |b_d(m)|^2 exp(-pi^2 m'^2 / (a^2 L_d^2)),   S_d(m) = m'^2 / L_d^2.
struct InfTab {
    const double* T[3];
    const double* S[3];
    double scale;     // 1 / (pi V)
    // triclinic cells: |m|^2 = |R m'|^2 (R = H^-1) is not separable; Euler
    // factors B[d] and signed frequencies M[d] per axis, and R below the
    // diagonal; pa2 = pi^2 / alpha^2
    int tric = 0;
    const double* B[3];
    const double* M[3];
    double r00, r10, r11, r20, r21, r22, pa2;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_err;    // message of the last failed call on this context
    pq_allocator alloc{};    // workspace allocator (pq_create); null members: hipMalloc
    bool have_system = false;
    bool fp64 = false;       // bulk arithmetic in FP64 (PQ_FLAG_FP64) instead of FP32
    int64_t n = 0;
    pq_params prm{};
    Geom g{};

    // --- neighbour list (set_system) ---
    int ncol = 0, ncl = 0;
    DBuf<double> w64;        // wrapped FP64 positions, original order, n*3
    DBuf<int> col_of;        // column of each atom
    DBuf<int> col_cnt;       // atoms per column
    DBuf<int> col_start;     // ncol+1, atom offsets per column (unpadded)
    DBuf<int> col_fill;      // fill counters
    DBuf<int> col_cl;        // ncol+1, cluster offsets per column
    DBuf<int> tmp_atoms;     // atoms grouped by column, unordered
    DBuf<int> bin_hist, bin_scan; // per-workgroup column counts (column-major) and their scan
    DBuf<int> orig;          // slot -> original atom (-1 padding), ncl*8
    DBuf<unsigned char> xyzq; // slot-ordered V4<T>: offset from the cluster reference + charge
    DBuf<double> cl_ref;     // ncl*3 reference points
    DBuf<double4> cl_pos;    // slot-ordered FP64 wrapped positions, w = 1 (0: padding)
    DBuf<double> cl_lo;      // ncl*3 bounding boxes
    DBuf<double> cl_hi;
    DBuf<int> cl_col;        // column of each cluster
    DBuf<int> zta, ztb;      // per-column z-window tables, ncol*(nbin+1) each
    DBuf<int> lcount;        // ncl+1: cluster-pair entries per i-cluster
    int lcap = 0;            // entries reserved per i-cluster (kept across builds)
    DBuf<int2> lj;           // cluster-pair list, ncl*lcap: (j cluster, packed image vector)
    DBuf<unsigned char> jmask; // ncl*lcap*8: colmask of each (entry, j atom)
    DBuf<int> jcount;        // ncl+1: rows of 8 j atoms per i-cluster
    DBuf<int> jstart;        // ncl+1: row offsets
    DBuf<unsigned char> jl;  // atom-level j lists: V4<T> (image position - ref_i, slot)
    int64_t njrows = 0;
    DBuf<int> flag;          // device error flags
    DBuf<unsigned long long> counter;
    DBuf<int> scan_part;     // block sums of the multi-workgroup scan
    // moves that keep the list (skin > 0, nbr_refresh)
    bool moved = false;      // the list was kept across a move: cl_w and cl_k are valid
    DBuf<double> pos_build;  // positions of the last full build, n*3
    DBuf<double4> cl_pos0;   // slot-ordered wrapped positions of that build
    DBuf<double4> cl_w;      // slot-ordered canonical wraps of the current positions
    DBuf<int4> cl_k;         // lattice steps between continuous and wrapped positions
    DBuf<double> disp_part;  // partial maxima of the displacement

    // --- PME ---
    int K[3] = {0, 0, 0}, P = 0, B = 8;
    int nb[3] = {0, 0, 0}, nbrick = 0;
    DBuf<int> brick_of, brick_cnt, brick_start, brick_fill;
    DBuf<int> pme_idx;       // brick-ordered original indices
    DBuf<unsigned char> qbrick;   // T: charges in brick order (staged per evaluation)
    DBuf<unsigned char> pme_frac; // V4<T>: fractional parts + packed base index
    DBuf<unsigned char> pme_w;    // T: B-spline weights per atom, 3 x 8 (brick order)
    DBuf<unsigned char> grid;     // T: real grid K1*K2*K3 (x fastest)
    DBuf<unsigned char> stage;    // T: per-brick spreading regions (B+p-1)^3
    DBuf<unsigned char> spec;     // V2<T>: half spectrum (K1/2+1)*K2*K3
    DBuf<unsigned char> twid;     // V2<T>: FFT twiddles of the three axes
    // bilinear (two-charge) force: the second charge vector per slot and in
    // brick order, and the second convolved grid
    DBuf<unsigned char> qv;       // T per slot
    DBuf<unsigned char> qbrick2;  // T in brick order
    DBuf<unsigned char> grid2;    // T, like grid
    bool save_psi = false;        // the next PME evaluation copies its convolved grid to grid2
    DBuf<double> inftab;     // T and S tables (FP64)
    Fft1D fft[3];
    InfTab inf{};
    double fft_key[12] = {}; // (K, p, alpha, box, tilts, precision) the tables above were made for
    bool fft_key_valid = false;

    // --- direct Ewald ---
    int nk = 0;
    DBuf<int4> kn;           // half-space integer k vectors
    DBuf<double> kc;         // c_k = (4 pi / V) exp(-k^2/4a^2)/k^2
    DBuf<double2> sfac;      // structure factors
    int ew_nch = 1, ew_cs = 1;     // atom chunks of the structure-factor sums (chunk size)
    int ew_nkch = 1, ew_kcs = 1;   // k-vector chunks of the potential / force sums (chunk size)
    DBuf<double2> spart;     // structure-factor partials, [atom chunk][k]
    DBuf<double4> gpart;     // potential / force partials, [k chunk][atom]

    // --- per-evaluation scratch ---
    DBuf<unsigned char> phi_r, phi_k;   // T per atom (original order, without KE)
    DBuf<unsigned char> f_r, f_k;       // V4<T> per atom
    DBuf<double> part;       // reduction partials
    DBuf<double> qpart;      // partials of the total-charge sum (on the pair kernel's stream)
    DBuf<double> scal;       // small device scalars
    double* pinned = nullptr;// pinned host scalars
    // Reduction workspace of the evaluation in progress: block partials
    // (part_n doubles), the partials of the total-charge sum and the
    // evaluation's device scalars (0: total charge, 1: reciprocal energy
    // without KE). coulomb_eval points it at part / qpart / scal above;
    // pq_coulomb_noalloc points it into the library's static scratch array.
    struct EvalWs {
        double* part = nullptr;
        size_t part_n = 0;
        double* qpart = nullptr;
        double* scal = nullptr;
    } ews;

    // --- tuned launch shapes (pq_autotune) ---
    bool want_energy = true; // the current evaluation reports energies (E_rec reduction)
    int pair_grid = 0;       // pair kernel workgroups (0: one wavefront per i-cluster)
    int fft_budget = 18432;  // bytes per FFT ping-pong buffer (sets the tile sizes)
    int fork_at = 0;         // PME: where the pair kernel's stream forks (0 start, 1 after the
                             // spreading pass 1, 2 after spreading)
    double tune_ms = 0.0;    // evaluation time of the chosen shape

    // --- second stream: the pair kernel overlaps the PME chain ---
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // --- phase timing ---
    bool timing = false;
    bool serial = false;     // pair kernel on the main stream (phase timing mode 2, server slots)
    std::vector<hipEvent_t> ev_pool;          // free events
    std::vector<std::vector<hipEvent_t>> ev_pending;   // PQ_NPHASE*2 events per timed evaluation

    // --- Krylov workspace ---
    DBuf<double> kv;         // basis vectors (m+1) x ld
    DBuf<double> kw;         // work vectors
    DBuf<double> kh;         // Hessenberg and small solver state
    DBuf<double> kf;         // force scratch n*3 (x2)
    DBuf<double> kup;        // chunk sums of the long-basis vector combinations
    size_t kld = 0;
    int km = 0;

    // --- Arnoldi step as a HIP graph (one step replayed every iteration) ---
    uint64_t gen = 0;                 // incremented by every pq_set_system
    bool graphs = true;               // off after a failed capture
    hipGraphExec_t kgraph = nullptr;
    std::vector<uintptr_t> kgraph_key;
    DBuf<int> kj;                     // device step index j
    double* pinned_hist = nullptr;    // host copy of the residual estimates
    int pinned_hist_n = 0;            // its capacity (doubles)
    int solver = PQ_SOLVER_GMRES;     // Krylov method of the QEQ solves (pq_set_solver)
    int vjp_restart = 50;             // GMRES restart length of the adjoint solve
    hipEvent_t kev[2] = {nullptr, nullptr};

    ~Ctx();
};

// Makes a context's allocator the current one of this thread for the
// duration of an entry point (restored on exit, also by an exception).
struct AllocScope {
    const pq_allocator* prev;
    explicit AllocScope(const Ctx& c) : prev(tl_alloc()) { tl_alloc() = c.alloc.alloc ? &c.alloc : nullptr; }
    ~AllocScope() { tl_alloc() = prev; }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
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
void scan_ints(Ctx& c, const int* in, int* out, int n, bool ceil8, hipStream_t s);  // exclusive; out[n] = total
void nbr_build(Ctx& c, const double* pos);
void jlist_fill(Ctx& c, int rows);
// largest squared displacement since the last build (host-synchronising)
double nbr_max_disp2(Ctx& c, const double* pos);
// moves the atoms to pos keeping the cluster-pair list (orthorhombic, skin > 0,
// every atom within skin/2 of its build position)
void nbr_refresh(Ctx& c, const double* pos);
int64_t nbr_export_pairs(Ctx& c, int64_t cap, int32_t* pairs);
// ELLPACK export (pq_neighbor_ell); returns the largest row count
int nbr_export_ell(Ctx& c, int K, int32_t* nbr, int32_t* img, int32_t* count);
// pair.hip: outputs in original atom order, without KE; force includes q_i
void stage_charges(Ctx& c, const double* q, hipStream_t s);
void pair_sum(Ctx& c, bool force, hipStream_t s);   // into c.phi_r, c.f_r
// two charge vectors u (slots, qbrick) and v (qv, qbrick2); the bilinear pair
// force 1/2 sum_j (u_i v_j + v_i u_j) f_ij into c.f_r
void stage_charges2(Ctx& c, const double* u, const double* v, hipStream_t s);
void pair_sum_bilinear(Ctx& c, hipStream_t s);
// pme.hip
void pme_setup(Ctx& c);
// ev: 2*PQ_NPHASE timing events or NULL (spread, FFT and gather phases are recorded)
// into c.phi_k, c.f_k; calls at_fork (if not empty) after the spreading
// kernel c.fork_at names (1: pass 1, 2: pass 2)
void pme_eval(Ctx& c, const double* q, bool force, hipEvent_t* ev, hipStream_t s,
              const std::function<void()>& at_fork = {});
// bilinear reciprocal force of the staged u and v into c.f_k (PME; psi_v
// from grid2 when have_psi_v, else computed)
void pme_bilinear(Ctx& c, bool have_psi_v, hipStream_t s);
// fft.hip
void fft_setup(Ctx& c);
void fft_convolve(Ctx& c, hipStream_t s);   // grid -> psi in place; energy partials into c.ews.part
// ewald.hip
void ewald_setup(Ctx& c);
void ewald_eval(Ctx& c, const double* q, bool force, hipStream_t s);   // into c.phi_k, c.f_k
// vec.hip
void sum_vector(Ctx& c, const double* x, int64_t n, double* out, hipStream_t s);
// the same with a caller-provided partial buffer (>= RED_BLOCKS + 16 doubles)
void sum_vector_into(const double* x, int64_t n, double* out, double* part, hipStream_t s);
void dot_vector(Ctx& c, const double* x, const double* y, int64_t n, double* out, hipStream_t s);
// after the total charge is in c.ews.scal[0]
void combine(Ctx& c, const double* q, double* phi, double* force, double* energy, hipStream_t s);
// force = KE (c.f_r + c.f_k), FP64 n x 3
void combine_force(Ctx& c, double* force, hipStream_t s);

// high-level evaluation used by the ABI and the Krylov solvers (abi.cpp)
void ensure_side(Ctx& c);   // creates the pair kernel's stream and fork/join events
void ensure_red(Ctx& c);    // reduction partials and device scalars (part, qpart, scal)
void coulomb_eval(Ctx& c, const double* q, double* phi, double* force, double* energy,
                  hipStream_t s);
// Bilinear force F = -d/dR (1/2 u^T A(R) v) into force (device n x 3 FP64),
// one pass of the pair list with both charge vectors and the PME chains of u
// (and of v unless have_psi_v: its convolved grid kept in grid2 by the last
// evaluation, which ran with c.save_psi). PME only.
void coulomb_bilinear_force(Ctx& c, const double* u, const double* v, bool have_psi_v, double* force,
                            hipStream_t s);
void ensure_bilinear(Ctx& c);   // qv, qbrick2, grid2
// the same on the reduction workspace c.ews as it stands (allocates nothing
// once pq_set_system has sized the per-atom buffers)
void coulomb_eval_ws(Ctx& c, const double* q, double* phi, double* force, double* energy,
                     hipStream_t s);

// While alive, errors reported on this thread (set_error) are also recorded
// as the context's last error; entry points that take a context hold one.
void set_error(const std::string& m);
struct CtxErrScope {
    explicit CtxErrScope(pq_ctx* c);
    ~CtxErrScope();
    CtxErrScope(const CtxErrScope&) = delete;
    CtxErrScope& operator=(const CtxErrScope&) = delete;
    Ctx* prev;
};

}  // namespace pq
