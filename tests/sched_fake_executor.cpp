// The served path's scheduler (paper_2404_01817_amd/csrc/scheduler.h) driven by a
// fake executor on the CPU, for a ThreadSanitizer build: several submitter
// threads, a fake device that finishes batches after random delays, launch
// errors, rejection by footprint, and shutdown with queued requests.  The
// fake executor checks the scheduler's promises at every launch: the slot is
// idle, at most `slots` batches run, the footprint (resident + running)
// stays under the cap, and every submitter's requests are admitted in the
// order it submitted them.  Exit status 0 when every check held.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "scheduler.h"

using neat::sched::Executor;
using neat::sched::Result;
using neat::sched::Scheduler;

namespace {

std::atomic<int> g_fail{0};

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            g_fail++;                                                          \
        }                                                                      \
    } while (0)

int64_t now_us() {
    return std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    int submitter = -1, seq = -1;
    uint64_t bytes = 0;
};

class FakeExec : public Executor<Req> {
  public:
    FakeExec(int slots, uint64_t cap, uint64_t resident, int min_us, int max_us, int fail_every)
        : cap_(cap), resident_(resident), min_us_(min_us), max_us_(max_us),
          fail_every_(fail_every), end_(slots, -1), bytes_(slots, 0), last_seq_(64, -1),
          rng_(12345) {}

    void thread_init() override {
        std::lock_guard<std::mutex> lk(m_);
        worker_ = std::this_thread::get_id();
    }
    int launch(int k, const std::vector<const Req *> &batch) override {
        {
            std::lock_guard<std::mutex> lk(m_);
            CHECK(launching_ == 0);  // launches never overlap
            launching_++;
            launching_slot_ = k;
            if (std::this_thread::get_id() != worker_) off_worker_++;
        }
        // a launch takes a while (as a real one does): nobody may poll the
        // slot or launch beside it meanwhile
        std::this_thread::sleep_for(std::chrono::microseconds(3));
        std::lock_guard<std::mutex> lk(m_);
        launching_--;
        launching_slot_ = -1;
        CHECK(k >= 0 && k < (int)end_.size());
        CHECK(end_[k] < 0);  // the slot is idle
        uint64_t b = 0;
        for (const Req *q : batch) {
            b += q->bytes;
            // per submitter, admission follows submission order
            CHECK(q->seq > last_seq_[q->submitter]);
            last_seq_[q->submitter] = q->seq;
        }
        uint64_t running = resident_ + b;
        int busy = 1;
        for (size_t j = 0; j < end_.size(); ++j)
            if ((int)j != k && end_[j] >= 0) running += bytes_[j], ++busy;
        CHECK(running <= cap_);
        CHECK(busy <= (int)end_.size());
        launches_++;
        max_batch_ = std::max<size_t>(max_batch_, batch.size());
        if (fail_every_ > 0 && launches_ % fail_every_ == 0) return NEAT_E_HIP;
        std::uniform_int_distribution<int> d(min_us_, max_us_);
        end_[k] = now_us() + d(rng_);
        bytes_[k] = b;
        return NEAT_OK;
    }
    bool finished(int k) override {
        std::lock_guard<std::mutex> lk(m_);
        CHECK(k != launching_slot_);  // never polled while its launch runs
        if (end_[k] >= 0 && now_us() >= end_[k]) {
            end_[k] = -1;
            bytes_[k] = 0;
            return true;
        }
        return false;
    }
    void drain(int k) override {
        std::lock_guard<std::mutex> lk(m_);
        end_[k] = -1;
        bytes_[k] = 0;
    }
    int launches() {
        std::lock_guard<std::mutex> lk(m_);
        return launches_;
    }
    // launches made by a thread other than the worker (direct admissions)
    int off_worker() {
        std::lock_guard<std::mutex> lk(m_);
        return off_worker_;
    }
    size_t max_batch() {
        std::lock_guard<std::mutex> lk(m_);
        return max_batch_;
    }

  private:
    std::mutex m_;
    const uint64_t cap_, resident_;
    const int min_us_, max_us_, fail_every_;
    std::vector<int64_t> end_;
    std::vector<uint64_t> bytes_;
    std::vector<int> last_seq_;
    std::mt19937 rng_;
    int launches_ = 0;
    size_t max_batch_ = 0;
    int launching_ = 0, launching_slot_ = -1;
    std::thread::id worker_;
    int off_worker_ = 0;
};

// Light load: one submitter waits for each result before the next request,
// so every request finds the scheduler idle.  With direct admission each is
// launched by the submitting thread; without, by the worker.
void light_test(bool direct) {
    FakeExec fx(2, 1000, 0, 20, 60, 0);
    Scheduler<Req> s(&fx, 2, 1000, 16, 5, 100, direct);
    for (int i = 0; i < 200; ++i) {
        Req q;
        q.submitter = 0;
        q.seq = i;
        q.bytes = 10;
        uint64_t tk = 0;
        CHECK(s.submit(q, q.bytes, 1, (uint64_t)i, false, &tk) == NEAT_OK);
        Result r;
        int rc;
        while ((rc = s.poll(tk, &r)) == NEAT_PENDING) std::this_thread::yield();
        CHECK(rc == NEAT_OK && r.status == NEAT_OK && r.tag == (uint64_t)i);
        CHECK(r.t_submit_ns <= r.t_admit_ns && r.t_admit_ns <= r.t_done_ns);
    }
    const neat::sched::Stats st = s.stats();
    CHECK(st.completed == 200 && st.batches == 200 && st.queued == 0);
    CHECK(fx.launches() == 200);
    CHECK(direct ? fx.off_worker() == 200 : fx.off_worker() == 0);
    std::printf("light load (direct %d): %d of 200 launches on the submitting thread, p50 %.3f ms\n",
                (int)direct, fx.off_worker(), st.p50_ms);
}

// spin: the scheduler's polling without sleeping (0: timed waits only);
// direct: requests admitted and launched by the submitting thread when
// nothing waits
void stream_test(int spin, bool direct) {
    const int slots = 4, threads = 6, per = 300;
    const uint64_t cap = 1000, resident = 200;
    FakeExec fx(slots, cap, resident, 20, 400, 41);
    Scheduler<Req> s(&fx, slots, cap, 16, 5, spin, direct);
    CHECK(s.add_resident(resident) == NEAT_OK);
    CHECK(s.add_resident(cap) == NEAT_E_TOO_LARGE);  // nothing held by the refusal
    std::atomic<int> rejected{0}, ok{0}, errored{0};
    std::vector<std::thread> th;
    for (int t = 0; t < threads; ++t)
        th.emplace_back([&, t] {
            std::mt19937 rng(1000 + t);
            std::uniform_int_distribution<int> bytes(1, 300), pause(0, 60);
            std::vector<uint64_t> tickets;
            for (int i = 0; i < per; ++i) {
                Req q;
                q.submitter = t;
                q.seq = i;
                // every 37th request could never fit beside the resident bytes
                q.bytes = (i % 37 == 36) ? 900 : (uint64_t)bytes(rng);
                uint64_t tk = 0;
                const int rc = s.submit(q, q.bytes, 10, (uint64_t)(t * per + i), false, &tk);
                if (q.bytes == 900) {
                    CHECK(rc == NEAT_E_TOO_LARGE);
                    rejected++;
                } else {
                    CHECK(rc == NEAT_OK);
                    tickets.push_back(tk);
                }
                std::this_thread::sleep_for(std::chrono::microseconds(pause(rng)));
            }
            for (uint64_t tk : tickets) {
                Result r;
                int rc;
                while ((rc = s.poll(tk, &r)) == NEAT_PENDING) std::this_thread::yield();
                CHECK(rc == NEAT_OK);
                CHECK(r.status == NEAT_OK || r.status == NEAT_E_HIP);
                CHECK(r.t_submit_ns <= r.t_admit_ns && r.t_admit_ns <= r.t_done_ns);
                (r.status == NEAT_OK ? ok : errored)++;
                CHECK(s.poll(tk, &r) == NEAT_E_UNKNOWN_TICKET);  // forgotten once reported
            }
        });
    for (auto &x : th) x.join();
    const neat::sched::Stats st = s.stats();
    const int accepted = threads * per - rejected.load();
    CHECK((int)st.submitted == accepted);
    CHECK((int)st.completed == accepted);
    CHECK((int)st.rejected == rejected.load());
    CHECK(st.admitted == st.batched_requests);
    CHECK(st.queued == 0);
    CHECK(st.peak_bytes <= cap);
    CHECK(st.resident_bytes == resident);
    CHECK(errored.load() > 0 && ok.load() > 0);
    CHECK(st.batches == (uint64_t)fx.launches());
    // continuous batching: under this load some batch held several requests
    CHECK(fx.max_batch() > 1);
    std::printf("stream (spin %d us, direct %d): %d requests, %d rejected, %llu batches (%.2f "
                "requests per batch, largest %zu), %d failed launches' requests, p50 %.3f ms p99 "
                "%.3f ms\n",
                spin, (int)direct, threads * per, rejected.load(), (unsigned long long)st.batches,
                (double)st.batched_requests / (double)st.batches, fx.max_batch(),
                errored.load(), st.p50_ms, st.p99_ms);
}

void shutdown_test(int spin, bool direct) {
    const int slots = 2;
    FakeExec fx(slots, 1u << 30, 0, 20000, 30000, 0);
    auto *s = new Scheduler<Req>(&fx, slots, 1u << 30, 4, 5, spin, direct);
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 100; ++i) {
        Req q;
        q.submitter = 0;
        q.seq = i;
        q.bytes = 1;
        uint64_t tk = 0;
        CHECK(s->submit(q, 1, 1, i, false, &tk) == NEAT_OK);
        tickets.push_back(tk);
    }
    // shut down once the first batches run (the rest is still queued)
    while (s->stats().admitted == 0) std::this_thread::yield();
    s->shutdown();
    int done = 0, cancelled = 0;
    for (uint64_t tk : tickets) {
        Result r;
        CHECK(s->poll(tk, &r) == NEAT_OK);
        (r.status == NEAT_E_SHUTDOWN ? cancelled : done)++;
    }
    CHECK(cancelled > 0 && done > 0 && done + cancelled == 100);
    uint64_t tk = 0;
    Req q;
    q.submitter = 0;
    q.seq = 1000;
    CHECK(s->submit(q, 1, 1, 0, false, &tk) == NEAT_E_SHUTDOWN);
    delete s;
    std::printf("shutdown (spin %d us, direct %d): %d finished, %d cancelled\n", spin, (int)direct,
                done, cancelled);
}

void empty_request_test() {
    FakeExec fx(1, 100, 0, 10, 20, 0);
    Scheduler<Req> s(&fx, 1, 100, 4, 5);
    Req q;
    q.submitter = 0;
    q.seq = 0;
    uint64_t tk = 0;
    CHECK(s.submit(q, 0, 0, 7, true, &tk) == NEAT_OK);
    Result r;
    CHECK(s.poll(tk, &r) == NEAT_OK && r.tag == 7 && r.status == NEAT_OK);
    CHECK(s.poll(tk + 99, &r) == NEAT_E_UNKNOWN_TICKET);
    CHECK(fx.launches() == 0);
}

}  // namespace

int main() {
    for (int spin : {0, 100})
        for (bool direct : {false, true}) {
            stream_test(spin, direct);
            shutdown_test(spin, direct);
        }
    for (bool direct : {false, true}) light_test(direct);
    empty_request_test();
    if (g_fail) {
        std::fprintf(stderr, "%d check(s) failed\n", g_fail.load());
        return 1;
    }
    std::printf("scheduler checks passed\n");
    return 0;
}
