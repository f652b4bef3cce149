// Continuous-batching QEQ server.
//
// Requests (host copies) wait in a FIFO. A scheduler admits the head request
// when a slot is free and its estimated device footprint fits the remaining
// budget; each slot owns a context and a HIP stream and runs its request on a
// worker thread, so admitted solves overlap on the device and new requests
// start as soon as earlier ones release a slot and memory. Results stay in the
// server until polled.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pmeqeq.h"
#include "pq_internal.h"

namespace pq {

void set_error(const std::string& m);

namespace {

struct Req {
    uint64_t ticket;
    int64_t n;
    std::vector<double> pos, chi, eta, q0;
    bool has_q0;
    double q_tot, tol;
    int max_it, restart, solver;
    pq_params params;
    double footprint;
    double t_submit, t_start = 0, t_done = 0;
    // result
    std::vector<double> q;
    double energy = 0;
    pq_solve_info info{};
    int status = 0;
    std::string message;
    bool done = false;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

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
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<std::shared_ptr<pq::Req>> queue;
    std::map<uint64_t, std::shared_ptr<pq::Req>> all;
    uint64_t next_ticket = 1;
    double in_use = 0;
    bool stopping = false;
    // slots
    struct Slot {
        pq_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        double* io = nullptr;      // device copies of a request's inputs and outputs; grows, never shrinks
        size_t io_bytes = 0;
        std::shared_ptr<pq::Req> req;
        std::thread th;
        std::condition_variable cv;
        bool busy = false;
        bool quit = false;
    };
    std::vector<std::unique_ptr<Slot>> slots;
    std::thread sched;
};

namespace pq {
namespace {

void run_request(pq_server* S, pq_server::Slot* sl, Req& r) {
    (void)S;
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
    if (!ok) st = PQ_ERR_HIP;
    if (st == PQ_OK) st = pq_set_solver(ctx, r.solver, 50);
    if (st == PQ_OK) st = pq_set_system(ctx, n, dpos, &r.params);
    if (st == PQ_OK)
        st = pq_qeq_solve(ctx, dchi, deta, r.q_tot, r.tol, r.max_it, r.restart, r.has_q0 ? dq0 : nullptr, dq,
                          nullptr, den, &r.info);
    if (st >= 0) {
        if (hipMemcpyAsync(r.q.data(), dq, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&r.energy, den, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = PQ_ERR_HIP;
    }
    (void)hipStreamSynchronize(s);
    r.status = st;
    if (st < 0) r.message = pq_last_error();
}

void slot_main(pq_server* S, pq_server::Slot* sl) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        sl->cv.wait(lk, [&] { return sl->quit || sl->req != nullptr; });
        if (sl->req == nullptr && sl->quit) return;
        std::shared_ptr<Req> r = sl->req;
        lk.unlock();
        r->t_start = now_s(S->t0);
        run_request(S, sl, *r);
        r->t_done = now_s(S->t0);
        lk.lock();
        r->done = true;
        S->in_use -= r->footprint;
        sl->req = nullptr;
        sl->busy = false;
        S->cv_done.notify_all();
        S->cv_sched.notify_all();
    }
}

void sched_main(pq_server* S) {
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_sched.wait(lk, [&] {
            if (S->stopping && S->queue.empty()) return true;
            if (S->queue.empty()) return false;
            const auto& h = S->queue.front();
            bool free_slot = false;
            for (auto& sl : S->slots) free_slot = free_slot || !sl->busy;
            return free_slot && S->in_use + h->footprint <= S->cfg.hbm_budget_bytes;
        });
        if (S->queue.empty() && S->stopping) break;
        // admit as many head requests as fit
        while (!S->queue.empty()) {
            auto h = S->queue.front();
            if (S->in_use + h->footprint > S->cfg.hbm_budget_bytes) break;
            pq_server::Slot* free_sl = nullptr;
            for (auto& sl : S->slots)
                if (!sl->busy) {
                    free_sl = sl.get();
                    break;
                }
            if (!free_sl) break;
            S->queue.pop_front();
            S->in_use += h->footprint;
            free_sl->busy = true;
            free_sl->req = h;
            free_sl->cv.notify_one();
        }
    }
    for (auto& sl : S->slots) {
        sl->quit = true;
        sl->cv.notify_one();
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
    S->t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < cfg->slots; ++k) {
        auto sl = std::make_unique<pq_server::Slot>();
        PQ_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
        pq_status st = pq_create(&sl->ctx, cfg->device, sl->stream, nullptr);
        if (st != PQ_OK) throw Error(st, pq_last_error());
        // slots launch their kernels directly; Arnoldi-step graphs are kept
        // for contexts driven from one thread (several slots replaying their
        // graphs concurrently crashed the process; the cause is not known)
        reinterpret_cast<Ctx*>(sl->ctx)->graphs = false;
        // requests overlap across slots, so a slot evaluates on its one
        // stream: no second stream and no fork/join events per evaluation
        reinterpret_cast<Ctx*>(sl->ctx)->serial = true;
        S->slots.push_back(std::move(sl));
    }
    for (auto& sl : S->slots) sl->th = std::thread(slot_main, S.get(), sl.get());
    S->sched = std::thread(sched_main, S.get());
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
    if (r->footprint > S->cfg.hbm_budget_bytes) {
        set_error("request footprint " + std::to_string(r->footprint) + " B exceeds the server budget");
        return PQ_ERR_TOO_LARGE;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    PQ_REQUIRE(!S->stopping, PQ_ERR_STATE, "server is stopping");
    r->ticket = S->next_ticket++;
    r->t_submit = now_s(S->t0);
    S->all[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
    S->cv_sched.notify_all();
    return PQ_OK;
    PQ_API_END
}

pq_status pq_server_poll(pq_server* S, uint64_t ticket, pq_result* res, int64_t timeout_us) {
    PQ_API_BEGIN
    PQ_REQUIRE(S && res, PQ_ERR_INVALID, "server and result must not be NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    PQ_REQUIRE(it != S->all.end(), PQ_ERR_INVALID, "unknown ticket");
    std::shared_ptr<Req> r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_us < 0)
        S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
        return PQ_ERR_TIMEOUT;
    if (res->q && !r->q.empty()) std::memcpy(res->q, r->q.data(), sizeof(double) * r->q.size());
    res->energy = r->energy;
    res->info = r->info;
    res->status = r->status;
    res->t_submit_s = r->t_submit;
    res->t_start_s = r->t_start;
    res->t_done_s = r->t_done;
    std::snprintf(res->message, sizeof(res->message), "%s", r->message.c_str());
    S->all.erase(it);
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
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        S->cv_sched.notify_all();
    }
    if (S->sched.joinable()) S->sched.join();
    for (auto& sl : S->slots) {
        if (sl->th.joinable()) sl->th.join();
        pq_destroy(sl->ctx);
        std::lock_guard<std::recursive_mutex> lk(device_mem_lock());
        if (sl->io) (void)hipFree(sl->io);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
    }
    delete S;
    return PQ_OK;
    PQ_API_END
}

}  // extern "C"
