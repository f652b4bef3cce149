// Continuous-batching QEQ server.
//
// Requests (host copies) wait in a FIFO. A scheduler admits the head request
// when a slot is free and its estimated device footprint fits the remaining
// budget; each slot owns a context and a HIP stream and runs its request on a
// worker thread, so admitted solves overlap on the device and new requests
// start as soon as earlier ones release a slot and memory. Results stay in the
// server until polled. The queue, admission and threads are in pq_sched.h; this
// file holds what runs on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pmeqeq.h"
#include "pq_internal.h"
#include "pq_sched.h"

namespace pq {

void set_error(const std::string& m);

// Estimated device bytes of one request: neighbour lists, per-atom arrays,
// PME grids and staging, Krylov basis. Bulk arrays take 4 or 8 bytes per real
// (FP32 or FP64 form). The list sizes follow from the volume within the list
// radius of a cluster's bounding box (edge a for 8 atoms at the system's
// density): a box of edge e grown by a ball of radius r has volume
// e^3 + 6 e^2 r + 3 pi e r^2 + 4/3 pi r^3.
double request_footprint(int64_t n, const pq_params& p, int restart) {
    const double rs = (p.flags & PQ_FLAG_FP64) ? 8.0 : 4.0;
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double rho = (double)n / V;
    const double a = std::cbrt(8.0 / rho);
    const double rl = p.cutoff + p.skin;
    auto grown = [&](double e) { return e * e * e + 6 * e * e * rl + 3 * PI * e * rl * rl + 4.0 / 3.0 * PI * rl * rl * rl; };
    const double ncl = std::ceil((double)n / 8.0) + 1.0;
    // cluster pairs: int2 and 8 mask bytes each, in per-cluster segments sized
    // for the fullest cluster
    const double pairs = ncl * grown(2.0 * a) * rho / 8.0 * 16.0 * 1.3;
    const double jatoms = ncl * (grown(a) * rho + 8.0) * 4.0 * rs;       // atom list, V4 each
    const double atoms = (double)n * (24 + 16 + 16 + 16 + 20 + 8 + 32 + 24 + 32) + (double)n * (4 + 4 + 16 + 24) * rs;
    double grid = 0;
    if (p.method == PQ_METHOD_PME) {
        const double K3 = (double)p.grid[0] * p.grid[1] * p.grid[2];
        const double R = 8 + p.order - 1;
        const double nbrick = std::ceil(p.grid[0] / 8.0) * std::ceil(p.grid[1] / 8.0) * std::ceil(p.grid[2] / 8.0);
        grid = K3 * rs + (p.grid[0] / 2 + 1) * (double)p.grid[1] * p.grid[2] * 2.0 * rs + nbrick * R * R * R * rs +
               (double)n * 48.0 * rs;
    } else {
        // k vectors, structure factors and the chunk partials of the direct sum
        const double nk = ((2.0 * p.kmax[0] + 1) * (2.0 * p.kmax[1] + 1) * (2.0 * p.kmax[2] + 1)) / 2.0 + 1.0;
        grid = nk * (16 + 8 + 16) + 2048.0 * 256.0 * (16 + 32);
    }
    const double kry = ((double)n + 64) * 8.0 * (13 + restart + 1);
    return 1.25 * (pairs + jatoms + atoms + grid + kry) + (1 << 20);
}

}  // namespace pq

struct pq_server {
    pq_server_cfg cfg{};
    // device resources of each slot
    struct Slot {
        pq_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        double* io = nullptr;      // device copies of a request's inputs and outputs; grows, never shrinks
        size_t io_bytes = 0;
    };
    std::vector<Slot> slots;
    // queue, admission and worker threads (declared last: stopped first)
    std::unique_ptr<pq::Sched> sched;
};

namespace pq {
namespace {

void run_request(const pq_server_cfg& cfg, pq_server::Slot* sl, Req& r) {
    (void)hipSetDevice(cfg.device);
    pq_ctx* ctx = sl->ctx;
    const int64_t n = r.n;
    r.q.assign(n, 0.0);
    pq_status st = PQ_OK;
    hipStream_t s = sl->stream;
    // pos, chi, eta, q0, q, energy in the slot's buffer; it is reallocated only
    // when a larger request arrives (a free synchronises the whole device)
    const size_t bytes = sizeof(double) * (size_t)(n * 3 + n * 4 + 1);
    if (bytes > sl->io_bytes) {
        std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
        (void)hipStreamSynchronize(s);
        if (sl->io) (void)hipFree(sl->io);
        sl->io = nullptr;
        sl->io_bytes = 0;
        const size_t want = bytes + bytes / 2;
        if (hipMalloc(&sl->io, want) != hipSuccess) {
            (void)hipGetLastError();
            sl->io = nullptr;
            r.status = PQ_ERR_NOMEM;
            return;
        }
        sl->io_bytes = want;
    }
    double* dpos = sl->io;
    double* dchi = dpos + 3 * n;
    double* deta = dchi + n;
    double* dq0 = deta + n;
    double* dq = dq0 + n;
    double* den = dq + n;
    bool ok = hipMemcpyAsync(dpos, r.pos.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(dchi, r.chi.data(), sizeof(double) * n, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(deta, r.eta.data(), sizeof(double) * n, hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok && r.has_q0)
        ok = hipMemcpyAsync(dq0, r.q0.data(), sizeof(double) * n, hipMemcpyHostToDevice, s) == hipSuccess;
    std::string copy_err;
    if (!ok) {
        st = PQ_ERR_HIP;
        copy_err = "copy of the request's inputs to the device failed";
    }
    if (st == PQ_OK) st = pq_set_solver(ctx, r.solver, 50);
    if (st == PQ_OK) st = pq_set_system(ctx, n, dpos, &r.params);
    if (st == PQ_OK)
        st = pq_qeq_solve(ctx, dchi, deta, r.q_tot, r.tol, r.max_it, r.restart, r.has_q0 ? dq0 : nullptr, dq,
                          nullptr, den, &r.info);
    if (st >= 0) {
        if (hipMemcpyAsync(r.q.data(), dq, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&r.energy, den, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = PQ_ERR_HIP;
            copy_err = "copy of the result to the host failed";
        }
    }
    (void)hipStreamSynchronize(s);
    r.status = st;
    if (st < 0) r.message = copy_err.empty() ? std::string(pq_ctx_last_error(ctx)) : copy_err;
}

// Contexts, streams and buffers of the slots (the worker threads have ended).
void release_slots(pq_server& S) {
    for (auto& sl : S.slots) {
        if (sl.ctx) pq_destroy(sl.ctx);
        sl.ctx = nullptr;
        std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
        if (sl.io) (void)hipFree(sl.io);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        sl.io = nullptr;
        sl.stream = nullptr;
    }
}

}  // namespace
}  // namespace pq

using namespace pq;

#define PQ_API_BEGIN try {
#define PQ_API_END                      \
    }                                   \
    catch (const pq::Error& e) {        \
        pq::set_error(e.what());        \
        return e.code;                  \
    }                                   \
    catch (const std::exception& e) {   \
        pq::set_error(e.what());        \
        return PQ_ERR_INVALID;          \
    }                                   \
    catch (...) {                       \
        pq::set_error("unknown error"); \
        return PQ_ERR_INVALID;          \
    }

extern "C" {

pq_status pq_server_create(pq_server** out, const pq_server_cfg* cfg) {
    PQ_API_BEGIN
    PQ_REQUIRE(out && cfg, PQ_ERR_INVALID, "out and cfg must not be NULL");
    PQ_REQUIRE(cfg->slots >= 1 && cfg->slots <= 64, PQ_ERR_INVALID, "slots must be in 1..64");
    PQ_REQUIRE(cfg->hbm_budget_bytes > 0, PQ_ERR_INVALID, "hbm_budget_bytes must be > 0");
    *out = nullptr;
    PQ_HIP(hipSetDevice(cfg->device));
    auto S = std::make_unique<pq_server>();
    S->cfg = *cfg;
    S->slots.resize(cfg->slots);
    try {
        for (auto& sl : S->slots) {
            PQ_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            pq_status st = pq_create(&sl.ctx, cfg->device, sl.stream, nullptr);
            if (st != PQ_OK) throw Error(st, pq_last_error());
            // slots launch their kernels directly; Arnoldi-step graphs are kept
            // for contexts driven from one thread (several slots replaying their
            // graphs concurrently crashed the process; the cause is not known)
            reinterpret_cast<Ctx*>(sl.ctx)->graphs = false;
            // requests overlap across slots, so a slot evaluates on its one
            // stream: no second stream and no fork/join events per evaluation
            reinterpret_cast<Ctx*>(sl.ctx)->serial = true;
        }
    } catch (...) {
        release_slots(*S);
        throw;
    }
    pq_server* raw = S.get();
    try {
        S->sched = std::make_unique<Sched>(cfg->slots, cfg->hbm_budget_bytes,
                                           [raw](int k, Req& r) { run_request(raw->cfg, &raw->slots[k], r); });
    } catch (...) {
        release_slots(*S);
        throw;
    }
    *out = S.release();
    return PQ_OK;
    PQ_API_END
}

pq_status pq_server_submit(pq_server* S, const pq_request* req, uint64_t* ticket) {
    PQ_API_BEGIN
    PQ_REQUIRE(S && req && ticket, PQ_ERR_INVALID, "server, request and ticket must not be NULL");
    PQ_REQUIRE(req->n >= 1 && req->pos && req->chi && req->eta, PQ_ERR_INVALID, "request needs n, pos, chi, eta");
    PQ_REQUIRE(req->tol > 0 && req->max_it >= 1 && req->restart >= 1 && req->restart <= PQ_MAX_RESTART &&
                   (req->solver == PQ_SOLVER_GMRES || req->solver == PQ_SOLVER_MINRES),
               PQ_ERR_INVALID, "bad solver settings");
    auto r = std::make_shared<Req>();
    const int64_t n = req->n;
    r->n = n;
    r->pos.assign(req->pos, req->pos + 3 * n);
    r->chi.assign(req->chi, req->chi + n);
    r->eta.assign(req->eta, req->eta + n);
    r->has_q0 = req->q0 != nullptr;
    if (r->has_q0) r->q0.assign(req->q0, req->q0 + n);
    r->q_tot = req->q_tot;
    r->tol = req->tol;
    r->max_it = req->max_it;
    r->restart = req->restart;
    r->solver = req->solver;
    r->params = req->params;
    r->footprint = request_footprint(n, req->params, req->solver == PQ_SOLVER_MINRES ? 1 : req->restart);
    std::string msg;
    const pq_status st = S->sched->submit(r, ticket, &msg);
    if (st != PQ_OK) set_error(msg);
    return st;
    PQ_API_END
}

pq_status pq_server_poll(pq_server* S, uint64_t ticket, pq_result* res, int64_t timeout_us) {
    PQ_API_BEGIN
    PQ_REQUIRE(S && res, PQ_ERR_INVALID, "server and result must not be NULL");
    std::shared_ptr<Req> r;
    std::string msg;
    const pq_status st = S->sched->poll(ticket, timeout_us, &r, &msg);
    if (st == PQ_ERR_TIMEOUT) return st;
    if (st != PQ_OK) {
        set_error(msg);
        return st;
    }
    if (res->q && !r->q.empty()) std::memcpy(res->q, r->q.data(), sizeof(double) * r->q.size());
    res->energy = r->energy;
    res->info = r->info;
    res->status = r->status;
    res->t_submit_s = r->t_submit;
    res->t_start_s = r->t_start;
    res->t_done_s = r->t_done;
    std::snprintf(res->message, sizeof(res->message), "%s", r->message.c_str());
    return PQ_OK;
    PQ_API_END
}

double pq_request_footprint(int64_t n, const pq_params* params, int32_t restart) {
    if (n < 1 || !params || restart < 1) return -1.0;
    return request_footprint(n, *params, restart);
}

pq_status pq_server_destroy(pq_server* S) {
    PQ_API_BEGIN
    if (!S) return PQ_OK;
    // queued requests still run; then the worker threads end
    if (S->sched) S->sched->stop();
    release_slots(*S);
    delete S;
    return PQ_OK;
    PQ_API_END
}

}  // extern "C"
