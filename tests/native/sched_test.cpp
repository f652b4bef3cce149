// The QEQ server's scheduler (pq_sched.h) driven by a fake executor on the
// CPU: no device, the same queue, admission, slot threads and tickets as the
// library's server. Built with ThreadSanitizer, and with AddressSanitizer +
// UndefinedBehaviorSanitizer, by tests/test_sched_native.py; exits non-zero
// on the first failed check.
//
// The fake executor computes a deterministic function of the request (so a
// result computed in the mix can be compared bit for bit with the same
// request computed alone) and checks, as it starts, that the admitted
// footprints never exceed the budget and that no more requests run than
// there are slots.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <random>
#include <stdexcept>
#include <thread>
#include <vector>

#include "pq_sched.h"

using pq::Req;
using pq::Sched;

static int g_fails = 0;
#define CHECK(c)                                                                        \
    do {                                                                                \
        if (!(c)) {                                                                     \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);      \
            ++g_fails;                                                                  \
        }                                                                               \
    } while (0)

// markers carried in max_it
enum { PLAIN = 1, GATED = 2, THROWS = 3 };

struct Fake {
    int slots;
    double budget;
    std::atomic<int> running{0};
    std::atomic<long long> running_fp{0};   // footprints are whole numbers here
    std::atomic<int> violations{0};
    std::atomic<bool> gate{false};

    static void compute(Req& r) {
        double s = 0;
        for (int64_t i = 0; i < r.n; ++i) s += r.chi[i] * (double)(i + 1);
        r.q.assign(r.n, 0.0);
        double e = 0;
        for (int64_t i = 0; i < r.n; ++i) {
            r.q[i] = r.chi[i] / r.eta[i] - 1e-3 * s;
            e += r.q[i] * r.chi[i];
        }
        r.energy = e;
        r.info.iterations = (int32_t)r.n;
    }

    void operator()(int slot, Req& r) {
        if (slot < 0 || slot >= slots) violations++;
        const int now = ++running;
        const long long fp = running_fp += (long long)r.footprint;
        if (now > slots || (double)fp > budget) violations++;
        if (r.max_it == GATED)
            while (!gate.load()) std::this_thread::sleep_for(std::chrono::microseconds(100));
        std::this_thread::sleep_for(std::chrono::microseconds(20 * (r.n % 7)));
        struct Leave {
            Fake* f;
            long long fp;
            ~Leave() {
                f->running_fp -= fp;
                --f->running;
            }
        } leave{this, (long long)r.footprint};
        if (r.max_it == THROWS) throw std::runtime_error("fake executor failure");
        compute(r);
    }
};

static std::shared_ptr<Req> make_req(std::mt19937_64& rng, int64_t n, double fp, int marker = PLAIN) {
    auto r = std::make_shared<Req>();
    r->n = n;
    std::uniform_real_distribution<double> U(-1.0, 1.0), E(5.0, 10.0);
    r->chi.resize(n);
    r->eta.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        r->chi[i] = U(rng);
        r->eta[i] = E(rng);
    }
    r->footprint = fp;
    r->max_it = marker;
    return r;
}

// Many submitters and pollers against 4 slots and a budget that admits a few
// requests at a time: every result equals the request computed alone, the
// budget and slot limits hold at every start, and requests are admitted in
// ticket order.
static void mixed_stream() {
    const int slots = 4, per_thread = 150, submitters = 3, pollers = 2;
    const double budget = 40;
    Fake fake{slots, budget};
    Sched S(slots, budget, std::ref(fake));
    std::mutex mu;
    std::vector<std::pair<uint64_t, std::shared_ptr<Req>>> submitted;   // ticket, alone copy
    std::vector<std::shared_ptr<Req>> polled;
    std::atomic<int> n_submitted{0}, errors{0};
    const int total = per_thread * submitters;
    std::vector<std::thread> th;
    for (int t = 0; t < submitters; ++t)
        th.emplace_back([&, t] {
            std::mt19937_64 rng(1000 + t);
            for (int k = 0; k < per_thread; ++k) {
                const int64_t n = 1 + (int64_t)(rng() % 64);
                const double fp = (double)(1 + rng() % 20);
                auto r = make_req(rng, n, fp);
                auto alone = std::make_shared<Req>(*r);
                Fake::compute(*alone);
                uint64_t ticket = 0;
                std::string msg;
                if (S.submit(r, &ticket, &msg) != PQ_OK) {
                    errors++;
                    continue;
                }
                {
                    std::lock_guard<std::mutex> lk(mu);
                    submitted.emplace_back(ticket, alone);
                }
                n_submitted++;
            }
        });
    for (int p = 0; p < pollers; ++p)
        th.emplace_back([&] {
            for (;;) {
                std::pair<uint64_t, std::shared_ptr<Req>> job{0, nullptr};
                {
                    std::lock_guard<std::mutex> lk(mu);
                    if (!submitted.empty()) {
                        job = submitted.back();
                        submitted.pop_back();
                    } else if ((int)polled.size() + errors.load() >= total) {
                        return;
                    }
                }
                if (!job.second) {
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                    continue;
                }
                std::shared_ptr<Req> got;
                std::string msg;
                if (S.poll(job.first, -1, &got, &msg) != PQ_OK) {
                    errors++;
                    continue;
                }
                if (got->status != 0 || got->q != job.second->q || got->energy != job.second->energy) errors++;
                std::lock_guard<std::mutex> lk(mu);
                polled.push_back(got);
            }
        });
    for (auto& x : th) x.join();
    CHECK(errors.load() == 0);
    CHECK(n_submitted.load() == total);
    CHECK((int)polled.size() == total);
    CHECK(fake.violations.load() == 0);
    CHECK(S.max_in_use() <= budget);
    CHECK(S.max_in_use() > 20);   // several requests did run together
    // FIFO admission: admission order is ticket order
    std::vector<uint64_t> seq(total + 1, 0);
    for (auto& r : polled)
        if (r->ticket >= 1 && r->ticket <= (uint64_t)total) seq[r->ticket] = r->admit_seq;
    for (int k = 1; k <= total; ++k) CHECK(seq[k] == (uint64_t)k);
    for (auto& r : polled) CHECK(r->t_submit <= r->t_start && r->t_start <= r->t_done);
}

// The head request waits for room in the budget; a smaller request behind it
// that would fit does not overtake it.
static void head_of_line() {
    const int slots = 4;
    const double budget = 10;
    Fake fake{slots, budget};
    Sched S(slots, budget, std::ref(fake));
    std::mt19937_64 rng(7);
    uint64_t ta, tb, tc;
    std::string msg;
    CHECK(S.submit(make_req(rng, 5, 8, GATED), &ta, &msg) == PQ_OK);
    CHECK(S.submit(make_req(rng, 5, 5), &tb, &msg) == PQ_OK);
    CHECK(S.submit(make_req(rng, 5, 1), &tc, &msg) == PQ_OK);
    std::shared_ptr<Req> r;
    // A holds the budget: nothing finishes, polls time out
    CHECK(S.poll(ta, 2000, &r, &msg) == PQ_ERR_TIMEOUT);
    CHECK(S.poll(tc, 2000, &r, &msg) == PQ_ERR_TIMEOUT);
    fake.gate = true;
    std::shared_ptr<Req> ra, rb, rc;
    CHECK(S.poll(tc, -1, &rc, &msg) == PQ_OK);
    CHECK(S.poll(tb, -1, &rb, &msg) == PQ_OK);
    CHECK(S.poll(ta, -1, &ra, &msg) == PQ_OK);
    CHECK(ra && rb && rc);
    if (ra && rb && rc) {
        CHECK(ra->admit_seq == 1 && rb->admit_seq == 2 && rc->admit_seq == 3);
        CHECK(rb->t_start >= ra->t_done);   // B needed A's share of the budget
    }
    CHECK(fake.violations.load() == 0);
}

// Error paths: a request larger than the budget, an unknown ticket, a second
// poll of one ticket, an executor that throws, submit after stop, and stop
// with requests still queued (they all complete).
static void error_paths() {
    const int slots = 2;
    const double budget = 10;
    Fake fake{slots, budget};
    fake.gate = true;
    Sched S(slots, budget, std::ref(fake));
    std::mt19937_64 rng(9);
    uint64_t t;
    std::string msg;
    std::shared_ptr<Req> r;
    CHECK(S.submit(make_req(rng, 4, 11), &t, &msg) == PQ_ERR_TOO_LARGE);
    CHECK(!msg.empty());
    CHECK(S.poll(12345, 0, &r, &msg) == PQ_ERR_INVALID);
    CHECK(S.submit(make_req(rng, 4, 2, THROWS), &t, &msg) == PQ_OK);
    CHECK(S.poll(t, -1, &r, &msg) == PQ_OK);
    CHECK(r && r->status == PQ_ERR_INVALID && r->message == "fake executor failure");
    CHECK(S.poll(t, 0, &r, &msg) == PQ_ERR_INVALID);
    // queued work survives stop
    std::vector<uint64_t> ts;
    for (int k = 0; k < 40; ++k) {
        CHECK(S.submit(make_req(rng, 1 + k, 1 + k % 9), &t, &msg) == PQ_OK);
        ts.push_back(t);
    }
    S.stop();
    S.stop();   // again: no effect
    CHECK(S.submit(make_req(rng, 3, 1), &t, &msg) == PQ_ERR_STATE);
    for (uint64_t x : ts) {
        CHECK(S.poll(x, 0, &r, &msg) == PQ_OK);
        CHECK(r && r->done && r->status == 0 && (int64_t)r->q.size() == r->n);
    }
    CHECK(fake.violations.load() == 0);
}

// Destroying a scheduler with requests running and queued and nobody
// polling: the destructor drains the queue and joins the threads.
static void destroy_busy() {
    Fake fake{3, 100};
    fake.gate = true;
    std::mt19937_64 rng(11);
    {
        Sched S(3, 100, std::ref(fake));
        uint64_t t;
        std::string msg;
        for (int k = 0; k < 30; ++k) CHECK(S.submit(make_req(rng, 1 + k, 10), &t, &msg) == PQ_OK);
    }
    CHECK(fake.running.load() == 0 && fake.violations.load() == 0);
}

int main() {
    mixed_stream();
    head_of_line();
    error_paths();
    destroy_busy();
    if (g_fails) {
        std::fprintf(stderr, "%d checks failed\n", g_fails);
        return 1;
    }
    std::printf("scheduler checks passed\n");
    return 0;
}
