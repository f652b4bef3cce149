// Host side of the continuous-batching QEQ server: the FIFO of requests,
// admission by estimated device footprint against a budget, the worker slots
// and the tickets. Nothing here touches the device: the work of a request is
// an executor callback, so the scheduling logic builds and runs on the CPU
// alone (the tests drive it with a fake executor under ThreadSanitizer).
//
// Admission is strictly in submission order: the head request waits until a
// slot is free and its footprint fits what the running requests leave of the
// budget; requests behind it do not overtake it.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pmeqeq.h"

namespace pq {

struct Req {
    uint64_t ticket = 0;
    int64_t n = 0;
    std::vector<double> pos, chi, eta, q0;
    bool has_q0 = false;
    double q_tot = 0, tol = 0;
    int max_it = 0, restart = 0, solver = 0;
    pq_params params{};
    double footprint = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    uint64_t admit_seq = 0;   // 1, 2, ... in the order requests were admitted
    // result
    std::vector<double> q;
    double energy = 0;
    pq_solve_info info{};
    int status = 0;
    std::string message;
    bool done = false;
};

class Sched {
public:
    // exec(slot, r) runs request r on slot `slot` (0 <= slot < slots) and
    // fills its result fields; it runs on that slot's worker thread, one
    // request at a time per slot. An exception it throws becomes the
    // request's error status.
    using Exec = std::function<void(int slot, Req& r)>;

    Sched(int slots, double budget, Exec exec) : budget_(budget), exec_(std::move(exec)) {
        t0_ = std::chrono::steady_clock::now();
        for (int k = 0; k < slots; ++k) slots_.push_back(std::make_unique<Slot>());
        try {
            for (int k = 0; k < slots; ++k) slots_[k]->th = std::thread(&Sched::slot_main, this, k);
            sched_ = std::thread(&Sched::sched_main, this);
        } catch (...) {
            // a thread could not start: end the ones that did before unwinding
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (auto& sl : slots_) sl->quit = true;
            }
            for (auto& sl : slots_) {
                sl->cv.notify_all();
                if (sl->th.joinable()) sl->th.join();
            }
            throw;
        }
    }
    ~Sched() { stop(); }
    Sched(const Sched&) = delete;
    Sched& operator=(const Sched&) = delete;

    double clock() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count(); }

    // Queues r (its footprint set by the caller) and returns its ticket.
    // PQ_ERR_TOO_LARGE if the footprint exceeds the whole budget,
    // PQ_ERR_STATE once the server is stopping; *msg says why.
    pq_status submit(std::shared_ptr<Req> r, uint64_t* ticket, std::string* msg) {
        if (r->footprint > budget_) {
            *msg = "request footprint " + std::to_string(r->footprint) + " B exceeds the server budget";
            return PQ_ERR_TOO_LARGE;
        }
        std::lock_guard<std::mutex> lk(mu_);
        if (stopping_) {
            *msg = "server is stopping";
            return PQ_ERR_STATE;
        }
        r->ticket = next_ticket_++;
        r->t_submit = clock();
        all_[r->ticket] = r;
        queue_.push_back(r);
        *ticket = r->ticket;
        cv_sched_.notify_all();
        return PQ_OK;
    }

    // Waits for the request's result (timeout_us < 0: without limit). On
    // PQ_OK the request leaves the server and *out holds it; PQ_ERR_TIMEOUT
    // leaves it in place; an unknown (or already polled) ticket is
    // PQ_ERR_INVALID.
    pq_status poll(uint64_t ticket, int64_t timeout_us, std::shared_ptr<Req>* out, std::string* msg) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = all_.find(ticket);
        if (it == all_.end()) {
            *msg = "unknown ticket";
            return PQ_ERR_INVALID;
        }
        std::shared_ptr<Req> r = it->second;
        auto pred = [&] { return r->done; };
        if (timeout_us < 0)
            cv_done_.wait(lk, pred);
        else if (!cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
            return PQ_ERR_TIMEOUT;
        // another poll of the same ticket may have taken it meanwhile
        it = all_.find(ticket);
        if (it == all_.end()) {
            *msg = "ticket already polled";
            return PQ_ERR_INVALID;
        }
        all_.erase(it);
        *out = r;
        return PQ_OK;
    }

    // Runs the queued requests to completion, then joins every thread. After
    // it returns, submit fails and the executor is no longer called. Safe to
    // call again; not to be called concurrently with itself.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (joined_) return;
            stopping_ = true;
            cv_sched_.notify_all();
        }
        if (sched_.joinable()) sched_.join();
        for (auto& sl : slots_)
            if (sl->th.joinable()) sl->th.join();
        std::lock_guard<std::mutex> lk(mu_);
        joined_ = true;
    }

    // Largest sum of admitted footprints seen at any time (never above the
    // budget).
    double max_in_use() const {
        std::lock_guard<std::mutex> lk(mu_);
        return max_in_use_;
    }

private:
    struct Slot {
        std::shared_ptr<Req> req;
        std::thread th;
        std::condition_variable cv;
        bool busy = false;
        bool quit = false;
    };

    void slot_main(int k) {
        Slot* sl = slots_[k].get();
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            sl->cv.wait(lk, [&] { return sl->quit || sl->req != nullptr; });
            if (sl->req == nullptr) return;   // quit with nothing assigned
            std::shared_ptr<Req> r = sl->req;
            lk.unlock();
            r->t_start = clock();
            try {
                exec_(k, *r);
            } catch (const std::exception& e) {
                r->status = PQ_ERR_INVALID;
                r->message = e.what();
            } catch (...) {
                r->status = PQ_ERR_INVALID;
                r->message = "executor failed";
            }
            r->t_done = clock();
            lk.lock();
            r->done = true;
            in_use_ -= r->footprint;
            sl->req = nullptr;
            sl->busy = false;
            cv_done_.notify_all();
            cv_sched_.notify_all();
        }
    }

    Slot* free_slot() {
        for (auto& sl : slots_)
            if (!sl->busy) return sl.get();
        return nullptr;
    }

    void sched_main() {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_sched_.wait(lk, [&] {
                if (stopping_ && queue_.empty()) return true;
                if (queue_.empty()) return false;
                return free_slot() != nullptr && in_use_ + queue_.front()->footprint <= budget_;
            });
            if (queue_.empty() && stopping_) break;
            // admit as many head requests as fit
            while (!queue_.empty()) {
                std::shared_ptr<Req> h = queue_.front();
                if (in_use_ + h->footprint > budget_) break;
                Slot* sl = free_slot();
                if (!sl) break;
                queue_.pop_front();
                in_use_ += h->footprint;
                if (in_use_ > max_in_use_) max_in_use_ = in_use_;
                h->admit_seq = ++admitted_;
                sl->busy = true;
                sl->req = h;
                sl->cv.notify_one();
            }
        }
        for (auto& sl : slots_) {
            sl->quit = true;
            sl->cv.notify_one();
        }
    }

    const double budget_;
    const Exec exec_;
    std::chrono::steady_clock::time_point t0_;
    mutable std::mutex mu_;
    std::condition_variable cv_sched_, cv_done_;
    std::deque<std::shared_ptr<Req>> queue_;
    std::map<uint64_t, std::shared_ptr<Req>> all_;
    uint64_t next_ticket_ = 1, admitted_ = 0;
    double in_use_ = 0, max_in_use_ = 0;
    bool stopping_ = false, joined_ = false;
    std::vector<std::unique_ptr<Slot>> slots_;
    std::thread sched_;
};

}  // namespace pq
