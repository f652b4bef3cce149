// C ABI of the pmeqeq library: contexts, systems and Coulomb evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pmeqeq.h"
#include "pq_internal.h"
#include "vec.h"

namespace pq {

thread_local std::string g_err;
thread_local Ctx* g_err_ctx = nullptr;   // context of the entry point running on this thread

std::recursive_mutex& device_mem_lock() {
    static std::recursive_mutex m;
    return m;
}

void set_error(const std::string& m) {
    g_err = m;
    if (g_err_ctx) g_err_ctx->last_err = m;
}

CtxErrScope::CtxErrScope(pq_ctx* c) : prev(g_err_ctx) {
    if (c) g_err_ctx = reinterpret_cast<Ctx*>(c);
}
CtxErrScope::~CtxErrScope() { g_err_ctx = prev; }

// ---------------------------------------------------------------------------
// Reduction scratch of pq_coulomb_noalloc: one file-scope device array (each
// device holds its own copy for the life of the process). Layout in doubles:
// [0, 64) device scalars, [64, 64 + RED_BLOCKS + 16) total-charge partials,
// the rest block partials. Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): pq_create
// resolves each device's copy with hipGetSymbolAddress, once per device, and
// the kernels receive that address.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_DOUBLES = PQ_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr size_t SCRATCH_QPART = 64;
constexpr size_t SCRATCH_PART = SCRATCH_QPART + RED_BLOCKS + 16;
static_assert(SCRATCH_PART + 4096 < SCRATCH_DOUBLES, "scratch too small");

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
bool g_scratch_done[MAX_DEVICES] = {};

// With `device` current: resolves this device's copy of the scratch array
// (first call per device); returns it, or nullptr if the lookup failed.
double* scratch_for_device(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) {
            g_scratch_ptr[device] = static_cast<double*>(p);
        } else {
            (void)hipGetLastError();
            g_scratch_ptr[device] = nullptr;
        }
        g_scratch_done[device] = true;
    }
    return g_scratch_ptr[device];
}

Ctx::~Ctx() {
    std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
    if (side) (void)hipStreamSynchronize(side);
    if (kgraph) (void)hipGraphExecDestroy(kgraph);
    for (auto e : kev)
        if (e) (void)hipEventDestroy(e);
    if (pinned_hist) (void)hipHostFree(pinned_hist);
    if (pinned) (void)hipHostFree(pinned);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    for (auto& v : ev_pending)
        for (auto e : v) (void)hipEventDestroy(e);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
}

Tric make_tric(const pq_params& p) {
#pragma clang fp contract(off)
    Tric t;
    t.txy = p.tilt[0];
    t.txz = p.tilt[1];
    t.tyz = p.tilt[2];
    const double i1 = 1.0 / p.box[1], i2 = 1.0 / p.box[2];
    t.ryz = t.tyz * i2;
    t.cxy = t.txy * i1;
    t.cxz = (t.txz - t.tyz * t.cxy) * i2;
    return t;
}

static bool smooth235(int k) {
    if (k <= 0) return false;
    for (int p : {2, 3, 5})
        while (k % p == 0) k /= p;
    return k == 1;
}

static void validate(int64_t n, const pq_params* p) {
    PQ_REQUIRE(p != nullptr, PQ_ERR_INVALID, "params is NULL");
    PQ_REQUIRE(n >= 1 && n <= (int64_t)1 << 27, PQ_ERR_INVALID, "n must be in [1, 2^27]");
    for (int d = 0; d < 3; ++d)
        PQ_REQUIRE(std::isfinite(p->box[d]) && p->box[d] > 0.0, PQ_ERR_INVALID, "box edges must be finite and > 0");
    PQ_REQUIRE(std::isfinite(p->cutoff) && p->cutoff > 0.0, PQ_ERR_INVALID, "cutoff must be > 0");
    PQ_REQUIRE(std::isfinite(p->skin) && p->skin >= 0.0, PQ_ERR_INVALID, "skin must be >= 0");
    PQ_REQUIRE(std::isfinite(p->alpha) && p->alpha > 0.0, PQ_ERR_INVALID, "alpha must be > 0");
    for (int d = 0; d < 3; ++d) PQ_REQUIRE(std::isfinite(p->tilt[d]), PQ_ERR_INVALID, "tilt factors must be finite");
    PQ_REQUIRE(std::fabs(p->tilt[0]) <= 0.5 * p->box[0] * (1 + 1e-12) &&
                   std::fabs(p->tilt[1]) <= 0.5 * p->box[0] * (1 + 1e-12) &&
                   std::fabs(p->tilt[2]) <= 0.5 * p->box[1] * (1 + 1e-12),
               PQ_ERR_BOX, "tilt factors must satisfy |t_xy|, |t_xz| <= L0/2 and |t_yz| <= L1/2");
    PQ_REQUIRE((p->flags & ~(PQ_FLAG_FP64 | PQ_FLAG_COMPENSATED)) == 0, PQ_ERR_INVALID, "unknown bits in flags");
    PQ_REQUIRE(p->method == PQ_METHOD_PME || p->method == PQ_METHOD_EWALD, PQ_ERR_INVALID, "unknown method");
    if (p->method == PQ_METHOD_PME) {
        PQ_REQUIRE(p->order >= 3 && p->order <= 8, PQ_ERR_INVALID, "order must be in 3..8");
        for (int d = 0; d < 3; ++d) {
            PQ_REQUIRE(p->grid[d] >= 2 * p->order && p->grid[d] <= 1024, PQ_ERR_BOX,
                       "grid must satisfy 2*order <= K <= 1024");
            PQ_REQUIRE(smooth235(p->grid[d]), PQ_ERR_BOX, "grid sizes must be 2^a 3^b 5^c");
        }
    } else {
        for (int d = 0; d < 3; ++d)
            PQ_REQUIRE(p->kmax[d] >= 0 && p->kmax[d] <= 64, PQ_ERR_INVALID, "kmax must be in 0..64");
    }
}

// Atom count from which the accuracy-driven choice takes PME (measured
// crossover of the two reciprocal-space methods on MI355X, random ionic
// systems at 0.1 atoms/A^3, delta 5e-4, rc 10 A, order 6).
constexpr int64_t AUTO_PME_MIN_ATOMS = 3500;

// OpenMM's estimate of the direct-Ewald error with |n_d| <= k on an edge L
static double ewald_err(double L, double alpha, int k) {
    const double t = M_PI * k / (L * alpha);
    return 0.05 * std::sqrt(L * alpha) * k * std::exp(-t * t);
}

static void choose_params(const double* box, int64_t n, double rc, double delta, int order, int method,
                          pq_params* out) {
    PQ_REQUIRE(box != nullptr && out != nullptr, PQ_ERR_INVALID, "box and out must not be NULL");
    for (int d = 0; d < 3; ++d)
        PQ_REQUIRE(std::isfinite(box[d]) && box[d] > 0.0, PQ_ERR_INVALID, "box edges must be finite and > 0");
    PQ_REQUIRE(n >= 1, PQ_ERR_INVALID, "n must be >= 1");
    PQ_REQUIRE(std::isfinite(rc) && rc > 0.0, PQ_ERR_INVALID, "cutoff must be > 0");
    PQ_REQUIRE(std::isfinite(delta) && delta > 0.0 && delta < 0.5, PQ_ERR_INVALID, "delta must be in (0, 0.5)");
    PQ_REQUIRE(order >= 3 && order <= 8, PQ_ERR_INVALID, "order must be in 3..8");
    PQ_REQUIRE(method == PQ_METHOD_PME || method == PQ_METHOD_EWALD || method == PQ_METHOD_AUTO, PQ_ERR_INVALID,
               "unknown method");
    pq_params p;
    std::memset(&p, 0, sizeof(p));
    const double alpha = std::sqrt(-std::log(2.0 * delta)) / rc;
    bool grid_ok = true, kmax_ok = true;
    for (int d = 0; d < 3; ++d) {
        p.box[d] = box[d];
        const double L = box[d];
        // PME grid
        const double want = std::ceil(2.0 * alpha * L / (3.0 * std::pow(delta, 0.2)));
        int K = (int)std::min(want, 4096.0);
        K = std::max(K, 2 * order);
        while (!smooth235(K)) ++K;
        p.grid[d] = K;
        grid_ok = grid_ok && K <= 1024;
        // direct Ewald range, searched from past the maximum of the estimate
        int k = std::max(1, (int)std::ceil(L * alpha / (M_PI * std::sqrt(2.0))));
        while (k <= 64 && ewald_err(L, alpha, k) > delta) ++k;
        p.kmax[d] = k;
        kmax_ok = kmax_ok && k <= 64;
    }
    p.cutoff = rc;
    p.skin = 0.0;
    p.alpha = alpha;
    p.order = order;
    p.flags = 0;
    if (method == PQ_METHOD_AUTO) method = (n < AUTO_PME_MIN_ATOMS && kmax_ok) ? PQ_METHOD_EWALD : PQ_METHOD_PME;
    p.method = method;
    if (method == PQ_METHOD_PME)
        PQ_REQUIRE(grid_ok, PQ_ERR_BOX, "PME grid for this accuracy exceeds 1024 points per axis");
    else
        PQ_REQUIRE(kmax_ok, PQ_ERR_BOX, "direct Ewald range for this accuracy exceeds kmax 64");
    *out = p;
}

void ensure_eval(Ctx& c) {
    const size_t n = (size_t)c.n;
    c.phi_r.ensure(n * rsz(c));
    c.phi_k.ensure(n * rsz(c));
    c.f_r.ensure(n * 4 * rsz(c));
    c.f_k.ensure(n * 4 * rsz(c));
}

// Reduction partials and device scalars of the evaluations and solvers: sized
// once for every reduction the solvers issue and the PME energy partials (one
// per spectral column), so nothing grows while an evaluation is being
// recorded into a graph. Allocated by the first evaluation or solve, not by
// pq_set_system (pq_coulomb_noalloc never needs them).
size_t red_part_need(const Ctx& c) {
    size_t need = (size_t)RED_BLOCKS * 520 + 4096;
    if (c.prm.method == PQ_METHOD_PME)
        need = std::max(need, (size_t)(c.prm.grid[0] / 2 + 1) * (size_t)c.prm.grid[1] + 16);
    return need;
}

void ensure_red(Ctx& c) {
    c.scal.ensure(64);
    c.part.ensure(red_part_need(c));
    c.qpart.ensure((size_t)RED_BLOCKS + 16);
}

// Phase events of one timed evaluation (null when timing is off).
struct PhaseEvents {
    Ctx& c;
    hipStream_t s;
    std::vector<hipEvent_t> ev;
    PhaseEvents(Ctx& cc, hipStream_t ss) : c(cc), s(ss) {
        if (!c.timing) return;
        ev.resize(2 * PQ_NPHASE);
        for (auto& e : ev) {
            if (!c.ev_pool.empty()) {
                e = c.ev_pool.back();
                c.ev_pool.pop_back();
            } else {
                PQ_HIP(hipEventCreate(&e));
            }
        }
    }
    void begin(int ph, hipStream_t on = nullptr) {
        if (!ev.empty()) PQ_HIP(hipEventRecord(ev[2 * ph], on ? on : s));
    }
    void end(int ph, hipStream_t on = nullptr) {
        if (!ev.empty()) PQ_HIP(hipEventRecord(ev[2 * ph + 1], on ? on : s));
    }
    void commit() {
        if (!ev.empty()) c.ev_pending.push_back(std::move(ev));
    }
};

void ensure_side(Ctx& c) {
    if (c.side) return;
    PQ_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    PQ_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
    PQ_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
}

void coulomb_eval(Ctx& c, const double* q, double* phi, double* force, double* energy, hipStream_t s) {
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    ensure_eval(c);
    ensure_red(c);
    c.ews.part = c.part.p;
    c.ews.part_n = c.part.n;
    c.ews.qpart = c.qpart.p;
    c.ews.scal = c.scal.p;
    coulomb_eval_ws(c, q, phi, force, energy, s);
}

void coulomb_eval_ws(Ctx& c, const double* q, double* phi, double* force, double* energy, hipStream_t s) {
    const bool fo = force != nullptr;
    c.want_energy = energy != nullptr;
    PhaseEvents E(c, s);
    E.begin(PQ_PHASE_TOTAL);
    E.begin(PQ_PHASE_STAGE);
    stage_charges(c, q, s);
    E.end(PQ_PHASE_STAGE);
    // the real-space pair kernel (ALU bound) runs on the context's second
    // stream, concurrently with the memory-bound reciprocal-space chain
    // (serial contexts: on the same stream, no fork and join). With PME it
    // forks before the chain, or (c.fork_at) after a spreading pass, so that
    // spreading runs with the device to itself.
    hipStream_t ps = s;
    auto fork_pair = [&]() {
        if (!c.serial) {
            ensure_side(c);
            ps = c.side;
            ev_record(c.ev_fork, s);
            stream_wait(ps, c.ev_fork);
        }
        E.begin(PQ_PHASE_PAIR, ps);
        pair_sum(c, fo, ps);
        E.end(PQ_PHASE_PAIR, ps);
        // the total charge (background term) is only needed by the final
        // combine: summed after the pair kernel, off the reciprocal-space chain
        sum_vector_into(q, c.n, c.ews.scal + 0, c.ews.qpart, ps);
        if (ps != s) ev_record(c.ev_join, ps);
    };
    if (c.prm.method == PQ_METHOD_PME) {
        const bool late = c.fork_at > 0 && !c.serial;
        if (!late) fork_pair();
        pme_eval(c, q, fo, E.ev.empty() ? nullptr : E.ev.data(), s, late ? std::function<void()>(fork_pair)
                                                                          : std::function<void()>());
    } else {
        fork_pair();
        E.begin(PQ_PHASE_SPREAD);
        E.end(PQ_PHASE_SPREAD);
        E.begin(PQ_PHASE_FFT);
        E.end(PQ_PHASE_FFT);
        E.begin(PQ_PHASE_GATHER);
        ewald_eval(c, q, fo, s);
        E.end(PQ_PHASE_GATHER);
    }
    if (ps != s) stream_wait(s, c.ev_join);
    E.begin(PQ_PHASE_COMBINE);
    combine(c, q, phi, force, energy, s);
    E.end(PQ_PHASE_COMBINE);
    E.end(PQ_PHASE_TOTAL);
    E.commit();
}

void ensure_bilinear(Ctx& c) {
    PQ_REQUIRE(c.prm.method == PQ_METHOD_PME, PQ_ERR_STATE, "the bilinear force path needs PME");
    c.qv.ensure((size_t)c.ncl * CL * rsz(c));
    c.qbrick2.ensure((size_t)c.n * rsz(c));
    c.grid2.ensure((size_t)c.K[0] * c.K[1] * c.K[2] * rsz(c));
}

void coulomb_bilinear_force(Ctx& c, const double* u, const double* v, bool have_psi_v, double* force,
                            hipStream_t s) {
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    ensure_eval(c);
    ensure_red(c);
    ensure_bilinear(c);
    stage_charges2(c, u, v, s);
    // the pair kernel beside the reciprocal chains, as in coulomb_eval
    hipStream_t ps = s;
    if (!c.serial) {
        ensure_side(c);
        ps = c.side;
        ev_record(c.ev_fork, s);
        stream_wait(ps, c.ev_fork);
    }
    pair_sum_bilinear(c, ps);
    if (ps != s) ev_record(c.ev_join, ps);
    pme_bilinear(c, have_psi_v, s);
    if (ps != s) stream_wait(s, c.ev_join);
    combine_force(c, force, s);
}

}  // namespace pq

using namespace pq;

#define PQ_API_BEGIN try {
#define PQ_API_END                              \
    }                                           \
    catch (const pq::Error& e) {                \
        pq::set_error(e.what());                \
        return e.code;                          \
    }                                           \
    catch (const std::exception& e) {           \
        pq::set_error(e.what());                \
        return PQ_ERR_INVALID;                  \
    }                                           \
    catch (...) {                               \
        pq::set_error("unknown error");         \
        return PQ_ERR_INVALID;                  \
    }

extern "C" {

int pq_abi_version(void) { return PQ_ABI_VERSION; }

pq_status pq_choose_params(const double* box, int64_t n, double cutoff, double delta, int32_t order, int32_t method,
                           pq_params* out) {
    PQ_API_BEGIN
    choose_params(box, n, cutoff, delta, order, method, out);
    return PQ_OK;
    PQ_API_END
}

int64_t pq_auto_pme_min_atoms(void) { return AUTO_PME_MIN_ATOMS; }

double pq_coulomb_constant(void) { return KE; }

const char* pq_last_error(void) { return pq::g_err.c_str(); }

const char* pq_ctx_last_error(const pq_ctx* ctx) {
    return ctx ? reinterpret_cast<const Ctx*>(ctx)->last_err.c_str() : "";
}

pq_status pq_create(pq_ctx** out, int device, void* stream, const pq_allocator* alloc) {
    PQ_API_BEGIN
    PQ_REQUIRE(out != nullptr, PQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    PQ_HIP(hipGetDeviceCount(&ndev));
    PQ_REQUIRE(device >= 0 && device < ndev, PQ_ERR_INVALID, "no such HIP device");
    PQ_HIP(hipSetDevice(device));
    // this device's copy of the no-allocation scratch (pq_coulomb_noalloc
    // reports a failed lookup)
    (void)scratch_for_device(device);
    PQ_REQUIRE(!alloc || (alloc->alloc == nullptr) == (alloc->free == nullptr), PQ_ERR_INVALID,
               "an allocator needs both alloc and free (or neither)");
    Ctx* c = new Ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    if (alloc) c->alloc = *alloc;
    std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
    if (hipHostMalloc((void**)&c->pinned, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete c;
        throw Error(PQ_ERR_NOMEM, "pinned host allocation failed");
    }
    *out = reinterpret_cast<pq_ctx*>(c);
    return PQ_OK;
    PQ_API_END
}

pq_status pq_set_stream(pq_ctx* ctx, void* stream) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr, PQ_ERR_INVALID, "ctx is NULL");
    reinterpret_cast<Ctx*>(ctx)->stream = static_cast<hipStream_t>(stream);
    return PQ_OK;
    PQ_API_END
}

pq_status pq_destroy(pq_ctx* ctx) {
    PQ_API_BEGIN
    if (!ctx) return PQ_OK;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    PQ_HIP(hipSetDevice(c->device));
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return PQ_OK;
    PQ_API_END
}

pq_status pq_set_system(pq_ctx* ctx, int64_t n, const double* pos, const pq_params* prm) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && pos != nullptr, PQ_ERR_INVALID, "ctx or pos is NULL");
    validate(n, prm);
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_HIP(hipSetDevice(c.device));
    c.have_system = false;
    ++c.gen;
    c.n = n;
    c.prm = *prm;
    c.fp64 = (prm->flags & PQ_FLAG_FP64) != 0;
    nbr_build(c, pos);
    if (prm->method == PQ_METHOD_PME)
        pme_setup(c);
    else
        ewald_setup(c);
    ensure_eval(c);
    c.have_system = true;
    return PQ_OK;
    PQ_API_END
}

pq_status pq_update_positions(pq_ctx* ctx, const double* pos, int32_t* rebuilt) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && pos != nullptr, PQ_ERR_INVALID, "ctx or pos is NULL");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_HIP(hipSetDevice(c.device));
    // the list radius rc + skin covers every pair closer than rc while no
    // atom has moved more than skin/2 since the build
    bool keep = c.prm.skin > 0.0 && !is_tric(c.prm) && c.pos_build.n >= (size_t)c.n * 3;
    if (keep) {
        const double d2 = nbr_max_disp2(c, pos);
        const double h = 0.5 * c.prm.skin;
        keep = d2 <= h * h;   // false for a NaN displacement
    }
    if (rebuilt) *rebuilt = keep ? 0 : 1;
    const pq_params prm = c.prm;
    if (!keep) return pq_set_system(ctx, c.n, pos, &prm);
    c.have_system = false;
    ++c.gen;
    nbr_refresh(c, pos);
    if (c.prm.method == PQ_METHOD_PME)
        pme_setup(c);
    else
        ewald_setup(c);
    ensure_eval(c);
    c.have_system = true;
    return PQ_OK;
    PQ_API_END
}

pq_status pq_neighbor_pairs(pq_ctx* ctx, int64_t cap, int32_t* pairs, int64_t* n_pairs) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && n_pairs != nullptr, PQ_ERR_INVALID, "ctx or n_pairs is NULL");
    PQ_REQUIRE(cap >= 0, PQ_ERR_INVALID, "cap must be >= 0");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_HIP(hipSetDevice(c.device));
    const int64_t tot = nbr_export_pairs(c, pairs ? cap : 0, pairs);
    *n_pairs = tot;
    if (pairs && tot > cap) {
        set_error("pair buffer too small: " + std::to_string(tot) + " pairs");
        return PQ_ERR_CAPACITY;
    }
    return PQ_OK;
    PQ_API_END
}

pq_status pq_neighbor_ell(pq_ctx* ctx, int32_t K, int32_t* nbr, int32_t* img, int32_t* count, int32_t* k_max) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && k_max != nullptr, PQ_ERR_INVALID, "ctx or k_max is NULL");
    PQ_REQUIRE(K >= 0, PQ_ERR_INVALID, "K must be >= 0");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_HIP(hipSetDevice(c.device));
    const int km = nbr_export_ell(c, K, nbr, img, count);
    *k_max = km;
    if ((nbr || img) && km > K) {
        set_error("ELLPACK width " + std::to_string(K) + " below the largest row count " + std::to_string(km));
        return PQ_ERR_CAPACITY;
    }
    return PQ_OK;
    PQ_API_END
}

pq_status pq_autotune(pq_ctx* ctx, const double* q, int32_t reps, pq_tune_result* out) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && q != nullptr, PQ_ERR_INVALID, "ctx and q must not be NULL");
    PQ_REQUIRE(reps >= 1 && reps <= 1000, PQ_ERR_INVALID, "reps must be in 1..1000");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_REQUIRE(!c.timing, PQ_ERR_STATE, "phase timing must be off while tuning");
    PQ_HIP(hipSetDevice(c.device));
    int ncu = 0;
    PQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device));
    hipStream_t s = c.stream;
    const size_t n = (size_t)c.n;
    DBuf<double> phi, f, e;
    phi.ensure(n);
    f.ensure(3 * n);
    e.ensure(4);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PQ_HIP(hipEventCreate(&e0));
    PQ_HIP(hipEventCreate(&e1));
    const int cand[] = {0, 1, 2, 3, 4, 6, 8};
    const int budgets[] = {18432, 9216, 4608};
    const int nfork = c.prm.method == PQ_METHOD_PME ? 3 : 1;
    int best = 0, best_b = 18432, best_f = 0, ntried = 0;
    double best_ms = 1e300, ms0 = 0.0;
    struct Cand {
        double ms;
        int k, b, f;
    };
    std::vector<Cand> tried;
    // the choice in force before tuning, kept if tuning fails
    const int old_grid = c.pair_grid, old_budget = c.fft_budget, old_fork = c.fork_at;
    // mean time of one evaluation over `r` evaluations after one warm-up
    auto time_config = [&](int k, int bgt, int fk, int r) {
        c.pair_grid = k * ncu;
        c.fft_budget = bgt;
        c.fork_at = fk;
        coulomb_eval(c, q, phi.p, f.p, e.p, s);
        PQ_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < r; ++i) coulomb_eval(c, q, phi.p, f.p, e.p, s);
        PQ_HIP(hipEventRecord(e1, s));
        PQ_HIP(hipEventSynchronize(e1));
        float el = 0.f;
        PQ_HIP(hipEventElapsedTime(&el, e0, e1));
        return (double)el / r;
    };
    try {
        for (int fk = 0; fk < nfork; ++fk)
        for (int bgt : budgets)
        for (int k : cand) {
            ++ntried;
            const double ms = time_config(k, bgt, fk, reps);
            if (k == 0 && bgt == 18432 && fk == 0) ms0 = ms;
            tried.push_back({ms, k, bgt, fk});
        }
        // the closest few are timed again, longer and interleaved, so that the
        // noise of one short measurement does not pick the configuration
        std::sort(tried.begin(), tried.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        const size_t top = std::min<size_t>(4, tried.size());
        std::vector<double> acc(top, 0.0);
        for (int pass = 0; pass < 2; ++pass)
            for (size_t i = 0; i < top; ++i) acc[i] += time_config(tried[i].k, tried[i].b, tried[i].f, 2 * reps);
        for (size_t i = 0; i < top; ++i) {
            const double ms = acc[i] / 2.0;
            if (ms < best_ms) {
                best_ms = ms;
                best = tried[i].k;
                best_b = tried[i].b;
                best_f = tried[i].f;
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        if (c.side) (void)hipStreamSynchronize(c.side);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c.pair_grid = old_grid;
        c.fft_budget = old_budget;
        c.fork_at = old_fork;
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.pair_grid = best * ncu;
    c.fft_budget = best_b;
    c.fork_at = best_f;
    c.tune_ms = best_ms;
    if (out) {
        out->pair_wg_per_cu = best;
        out->candidates = ntried;
        out->ms = best_ms;
        out->ms_default = ms0;
        out->fft_lds_bytes = best_b;
        out->pair_fork = best_f;
    }
    return PQ_OK;
    PQ_API_END
}

pq_status pq_set_tuning(pq_ctx* ctx, const pq_tune_result* t) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && t != nullptr, PQ_ERR_INVALID, "ctx and t must not be NULL");
    PQ_REQUIRE(t->pair_wg_per_cu >= 0 && t->pair_wg_per_cu <= 64, PQ_ERR_INVALID, "pair_wg_per_cu must be in 0..64");
    PQ_REQUIRE(t->fft_lds_bytes == 0 || (t->fft_lds_bytes >= 1024 && t->fft_lds_bytes <= 65536), PQ_ERR_INVALID,
               "fft_lds_bytes must be 0 or in 1024..65536");
    PQ_REQUIRE(t->pair_fork >= 0 && t->pair_fork <= 2, PQ_ERR_INVALID, "pair_fork must be in 0..2");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    c.fft_budget = t->fft_lds_bytes ? t->fft_lds_bytes : 18432;
    c.fork_at = t->pair_fork;
    PQ_HIP(hipSetDevice(c.device));
    int ncu = 0;
    PQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device));
    c.pair_grid = t->pair_wg_per_cu * ncu;
    return PQ_OK;
    PQ_API_END
}

pq_status pq_set_timing(pq_ctx* ctx, int on) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr, PQ_ERR_INVALID, "ctx is NULL");
    PQ_REQUIRE(on >= 0 && on <= 2, PQ_ERR_INVALID, "timing mode must be 0, 1 or 2");
    reinterpret_cast<Ctx*>(ctx)->timing = on != 0;
    reinterpret_cast<Ctx*>(ctx)->serial = on == 2;
    return PQ_OK;
    PQ_API_END
}

pq_status pq_timings(pq_ctx* ctx, double* ms, int64_t* count) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && ms != nullptr && count != nullptr, PQ_ERR_INVALID, "NULL argument");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_HIP(hipSetDevice(c.device));
    for (int k = 0; k < PQ_NPHASE; ++k) ms[k] = 0.0;
    *count = (int64_t)c.ev_pending.size();
    for (auto& v : c.ev_pending) {
        PQ_HIP(hipEventSynchronize(v[2 * PQ_PHASE_TOTAL + 1]));
        for (int k = 0; k < PQ_NPHASE; ++k) {
            float t = 0.0f;
            PQ_HIP(hipEventElapsedTime(&t, v[2 * k], v[2 * k + 1]));
            ms[k] += t;
        }
        for (auto e : v) c.ev_pool.push_back(e);
    }
    c.ev_pending.clear();
    return PQ_OK;
    PQ_API_END
}

pq_status pq_coulomb(pq_ctx* ctx, const double* q, double* phi, double* force, double* energy) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && q != nullptr, PQ_ERR_INVALID, "ctx or q is NULL");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_HIP(hipSetDevice(c.device));
    coulomb_eval(c, q, phi, force, energy, c.stream);
    return PQ_OK;
    PQ_API_END
}

pq_status pq_coulomb_noalloc(pq_ctx* ctx, const double* q, double* phi, double* force, double* energy) {
    pq::CtxErrScope err_scope(ctx);
    PQ_API_BEGIN
    PQ_REQUIRE(ctx != nullptr && q != nullptr, PQ_ERR_INVALID, "ctx or q is NULL");
    Ctx& c = *reinterpret_cast<Ctx*>(ctx);
    AllocScope alloc_scope(c);
    PQ_REQUIRE(c.have_system, PQ_ERR_STATE, "pq_set_system has not been called");
    PQ_REQUIRE(!c.timing, PQ_ERR_STATE, "phase timing must be off (it creates events)");
    PQ_HIP(hipSetDevice(c.device));
    double* base = scratch_for_device(c.device);
    PQ_REQUIRE(base != nullptr, PQ_ERR_STATE, "the scratch array of this device could not be resolved");
    // the per-atom buffers that pq_set_system sized
    const size_t n = (size_t)c.n;
    PQ_REQUIRE(c.phi_r.n >= n * rsz(c) && c.phi_k.n >= n * rsz(c) && c.f_r.n >= n * 4 * rsz(c) &&
                   c.f_k.n >= n * 4 * rsz(c),
               PQ_ERR_STATE, "per-atom buffers not sized");
    const size_t part_n = SCRATCH_DOUBLES - SCRATCH_PART;
    // partials: energy assembly (3 per reduction block), and one per spectral
    // column (PME) or per k-vector tile (direct Ewald)
    const size_t need = std::max<size_t>(3 * RED_BLOCKS + 16,
                                         c.prm.method == PQ_METHOD_PME
                                             ? (size_t)(c.prm.grid[0] / 2 + 1) * (size_t)c.prm.grid[1] + 16
                                             : (size_t)(c.nk + 255) / 256 + 16);
    if (need > part_n) {
        set_error("PME grid needs " + std::to_string(need) + " partial sums; the no-allocation scratch holds " +
                  std::to_string(part_n) + " ((grid[0]/2 + 1) * grid[1] + 16 must not exceed it)");
        return PQ_ERR_TOO_LARGE;
    }
    // every scratch word the evaluation reads is written by it first (the
    // scalars and partials are assigned, not accumulated), so nothing is
    // cleared; the pair kernel runs on the context's stream (no second stream)
    const bool serial = c.serial;
    c.serial = true;
    c.ews.part = base + SCRATCH_PART;
    c.ews.part_n = part_n;
    c.ews.qpart = base + SCRATCH_QPART;
    c.ews.scal = base;
    try {
        coulomb_eval_ws(c, q, phi, force, energy, c.stream);
    } catch (...) {
        c.serial = serial;
        c.ews = Ctx::EvalWs{};
        throw;
    }
    c.serial = serial;
    c.ews = Ctx::EvalWs{};
    return PQ_OK;
    PQ_API_END
}

}  // extern "C"
