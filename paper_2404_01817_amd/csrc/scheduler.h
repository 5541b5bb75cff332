// scheduler.h -- the continuous-batching scheduler of the served path, free of
// any HIP call so that it can be built and tested on the CPU.
//
// Requests carry a payload (for the server: the request and its resident
// population), the device bytes they touch while running, and their
// genome-inputs.  One worker thread admits queued requests in arrival order
// into a free slot while the device footprint stays under the cap: bytes of
// resident populations (registered once, held for good) plus the bytes of
// every running request.  Everything admitted together forms one batch,
// started on that slot by the executor; up to `slots` batches run at once,
// so requests that arrive while others run are admitted as slots and bytes
// free up and their work overlaps on the device.  Completions are polled
// through the executor without holding the scheduler's lock: while batches
// run, the worker polls without sleeping for up to spin_us (a timed wait
// wakes tens of microseconds after its deadline, which would add to every
// request's latency), then sleeps in poll_us steps.  With `direct`, a
// request that finds the scheduler idle (nothing queued, no slot busy, so
// the worker is asleep) is admitted and launched by the submitting thread
// itself (the worker would admit it alone anyway; this saves waking it),
// and the worker then polls its completion as any other.  Launches never
// overlap, so their order is the admission order.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "neat.h"

namespace neat {
namespace sched {

struct Result {
    int32_t status = NEAT_OK;
    uint64_t tag = 0;
    int64_t t_submit_ns = -1, t_admit_ns = -1, t_done_ns = -1;
};

struct Stats {
    uint64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, batches = 0, queued = 0;
    uint64_t genome_inputs = 0;       // of completed requests
    uint64_t batched_requests = 0;    // admitted requests over all batches
    double p50_ms = 0.0, p99_ms = 0.0;  // t_done - t_submit of completed requests
    double throughput = 0.0;          // genome_inputs / (last done - first submit) per s
    uint64_t resident_bytes = 0;
    uint64_t peak_bytes = 0;          // largest footprint (resident + running) admitted
};

// The device side of the scheduler.  Calls come from the worker thread
// (thread_init first) or, for a request admitted at submission, from the
// submitting thread; never with the scheduler's lock held, and a slot is
// never polled (finished) while its launch is in progress.
template <class Payload>
struct Executor {
    virtual ~Executor() = default;
    virtual void thread_init() {}
    // Start a batch (requests in admission order) on slot; 0 or an error
    // code, which then ends every request of the batch.
    virtual int launch(int slot, const std::vector<const Payload *> &batch) = 0;
    // True once the slot's batch has finished.
    virtual bool finished(int slot) = 0;
    // Wait for the slot's work (error paths).
    virtual void drain(int slot) = 0;
};

template <class Payload>
class Scheduler {
  public:
    // slots: batches running at once; cap: device footprint in bytes;
    // max_batch: requests per batch; poll_us: completion polling period
    // once spin_us of polling without sleeping found nothing; direct: admit
    // and launch a request on the submitting thread when nothing waits.
    Scheduler(Executor<Payload> *ex, int slots, uint64_t cap, int max_batch, int poll_us,
              int spin_us = 0, bool direct = false)
        : ex_(ex), cap_(cap), max_batch_(max_batch), poll_us_(poll_us), spin_us_(spin_us),
          direct_(direct), slots_(slots), t0_(std::chrono::steady_clock::now()) {
        worker_ = std::thread([this] { loop(); });
    }
    Scheduler(const Scheduler &) = delete;
    Scheduler &operator=(const Scheduler &) = delete;
    ~Scheduler() { shutdown(); }

    // Queued requests end with NEAT_E_SHUTDOWN; running batches finish; the
    // worker exits.  Idempotent.
    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(m_);
            if (!stop_) {
                for (uint64_t tk : queue_) {
                    Req &q = reqs_[tk];
                    q.state = DONE;
                    q.res.status = NEAT_E_SHUTDOWN;
                }
                queue_.clear();
                stop_ = true;
            }
        }
        cv_.notify_all();
        if (worker_.joinable()) worker_.join();
    }

    // Hold `bytes` of resident data against the cap for good; NEAT_E_TOO_LARGE
    // (nothing held) when it does not fit beside what is resident.
    int add_resident(uint64_t bytes) {
        std::lock_guard<std::mutex> lk(m_);
        if (resident_ + bytes > cap_) return NEAT_E_TOO_LARGE;
        resident_ += bytes;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return NEAT_OK;
    }

    // Queue a request.  `empty` requests (nothing to compute) finish at
    // once.  NEAT_E_TOO_LARGE when it could never fit beside the resident
    // bytes, NEAT_E_SHUTDOWN after shutdown.
    int submit(const Payload &p, uint64_t bytes, uint64_t genome_inputs, uint64_t tag,
               bool empty, uint64_t *ticket) {
        std::unique_lock<std::mutex> lk(m_);
        if (stop_) return NEAT_E_SHUTDOWN;
        if (resident_ + bytes > cap_) {
            rejected_++;
            return NEAT_E_TOO_LARGE;
        }
        const uint64_t tk = next_ticket_++;
        Req &q = reqs_[tk];
        q.payload = p;
        q.bytes = bytes;
        q.genome_inputs = genome_inputs;
        q.res.tag = tag;
        q.res.t_submit_ns = now_ns();
        if (first_submit_ < 0) first_submit_ = q.res.t_submit_ns;
        submitted_++;
        *ticket = tk;
        if (empty) {
            q.state = DONE;
            q.res.t_admit_ns = q.res.t_done_ns = q.res.t_submit_ns;
        } else if (direct_ && idle() && used_ + bytes <= cap_) {
            const int fs = free_slot();
            admit(fs, tk);
            run(lk, fs, {&q.payload});
            return NEAT_OK;
        } else {
            queue_.push_back(tk);
        }
        wake_.fetch_add(1, std::memory_order_release);
        lk.unlock();
        cv_.notify_one();
        return NEAT_OK;
    }

    // NEAT_OK (result filled, ticket forgotten), NEAT_PENDING, or
    // NEAT_E_UNKNOWN_TICKET.  Never blocks on the device.
    int poll(uint64_t ticket, Result *res) {
        std::lock_guard<std::mutex> lk(m_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return NEAT_E_UNKNOWN_TICKET;
        if (it->second.state != DONE) return NEAT_PENDING;
        if (res) *res = it->second.res;
        reqs_.erase(it);
        return NEAT_OK;
    }

    Stats stats() {
        std::lock_guard<std::mutex> lk(m_);
        Stats s;
        s.submitted = submitted_;
        s.admitted = admitted_;
        s.completed = completed_;
        s.rejected = rejected_;
        s.batches = batches_;
        s.batched_requests = batched_;
        s.queued = queue_.size();
        s.genome_inputs = genome_inputs_;
        s.p50_ms = (double)percentile(lat_ns_, 0.50) / 1e6;
        s.p99_ms = (double)percentile(lat_ns_, 0.99) / 1e6;
        const int64_t span = last_done_ - first_submit_;
        s.throughput = span > 0 ? (double)genome_inputs_ * 1e9 / (double)span : 0.0;
        s.resident_bytes = resident_;
        s.peak_bytes = peak_;
        return s;
    }

    void reset_stats() {
        std::lock_guard<std::mutex> lk(m_);
        lat_ns_.clear();
        submitted_ = admitted_ = completed_ = rejected_ = batches_ = batched_ = 0;
        genome_inputs_ = 0;
        first_submit_ = last_done_ = -1;
        peak_ = used_;
    }

  private:
    enum State { QUEUED = 0, ADMITTED = 1, DONE = 2 };
    struct Req {
        Payload payload{};
        Result res{};
        uint64_t bytes = 0, genome_inputs = 0;
        int state = QUEUED;
    };
    struct Slot {
        bool busy = false;
        bool launching = false;  // its launch is in progress (not polled meanwhile)
        std::vector<uint64_t> tickets;
        uint64_t bytes = 0, genome_inputs = 0;
    };

    int64_t now_ns() const {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now() - t0_)
            .count();
    }

    static int64_t percentile(std::vector<int64_t> v, double q) {
        if (v.empty()) return 0;
        const size_t k = (size_t)(q * (double)(v.size() - 1) + 0.5);
        std::nth_element(v.begin(), v.begin() + (long)k, v.end());
        return v[k];
    }

    // Caller holds the lock.
    void finish(int k, int status) {
        Slot &sl = slots_[k];
        const int64_t t = now_ns();
        for (uint64_t tk : sl.tickets) {
            auto it = reqs_.find(tk);
            if (it == reqs_.end()) continue;
            Req &q = it->second;
            q.state = DONE;
            if (status != NEAT_OK) q.res.status = status;
            q.res.t_done_ns = t;
            lat_ns_.push_back(t - q.res.t_submit_ns);
            completed_++;
        }
        genome_inputs_ += sl.genome_inputs;
        last_done_ = t;
        used_ -= sl.bytes;
        sl.tickets.clear();
        sl.bytes = sl.genome_inputs = 0;
        sl.busy = false;
    }

    // Caller holds the lock.  Nothing queued and no slot busy: the worker is
    // asleep, not polling (a launch on another thread beside its polling
    // would contend with it for the runtime).
    bool idle() const {
        if (!queue_.empty()) return false;
        for (const Slot &sl : slots_)
            if (sl.busy) return false;
        return true;
    }

    // Caller holds the lock.  A free slot (next in turn), or -1.
    int free_slot() const {
        for (int k = 0; k < (int)slots_.size(); ++k) {
            const int c = (next_slot_ + k) % (int)slots_.size();
            if (!slots_[c].busy) return c;
        }
        return -1;
    }

    // Caller holds the lock.  Admit queued-or-new request tk into slot fs.
    void admit(int fs, uint64_t tk) {
        Slot &sl = slots_[fs];
        Req &q = reqs_[tk];
        q.state = ADMITTED;
        q.res.t_admit_ns = now_ns();
        used_ += q.bytes;
        sl.bytes += q.bytes;
        sl.genome_inputs += q.genome_inputs;
        sl.tickets.push_back(tk);
        admitted_++;
    }

    // Caller holds the lock, which is released around the launch of slot fs
    // (its admitted requests' payloads in `batch`) and held again on return.
    // The slot is marked busy and launching first, so that nobody polls it
    // or launches beside it until the executor has started it.
    void run(std::unique_lock<std::mutex> &lk, int fs,
             const std::vector<const Payload *> &batch) {
        Slot &sl = slots_[fs];
        peak_ = std::max(peak_, used_);
        sl.busy = true;
        sl.launching = true;
        launching_++;
        next_slot_ = (fs + 1) % (int)slots_.size();
        batches_++;
        batched_ += sl.tickets.size();
        // payloads of admitted requests stay in place (the map keeps its
        // nodes; they are erased only once done)
        lk.unlock();
        const int rc = ex_->launch(fs, batch);
        if (rc != NEAT_OK) ex_->drain(fs);
        lk.lock();
        sl.launching = false;
        launching_--;
        if (rc != NEAT_OK) finish(fs, rc);
        // the worker polls the slot from now on
        wake_.fetch_add(1, std::memory_order_release);
        cv_.notify_one();
    }

    // Caller holds the lock.  Slots the worker may poll.
    void pollable(std::vector<int> &out) const {
        out.clear();
        for (int k = 0; k < (int)slots_.size(); ++k)
            if (slots_[k].busy && !slots_[k].launching) out.push_back(k);
    }

    // Caller holds the lock (released while polling, held again on return).
    // Poll the running slots without sleeping for up to spin_us, finishing
    // those that report completion (each report is acted on once); true once
    // one has finished, or a request was queued or a slot started meanwhile.
    bool spin(std::unique_lock<std::mutex> &lk) {
        std::vector<int> busy, done;
        pollable(busy);
        const uint64_t seen = wake_.load(std::memory_order_acquire);
        lk.unlock();
        const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(spin_us_);
        bool woken = false;
        while (done.empty() && !woken && std::chrono::steady_clock::now() < until) {
            for (int k : busy)
                if (ex_->finished(k)) done.push_back(k);
            woken = wake_.load(std::memory_order_acquire) != seen;
            if (done.empty() && !woken) std::this_thread::yield();
        }
        lk.lock();
        for (int k : done) finish(k, NEAT_OK);
        return !done.empty() || woken;
    }

    void loop() {
        ex_->thread_init();
        std::unique_lock<std::mutex> lk(m_);
        std::vector<int> busy, done;
        std::vector<const Payload *> batch;
        for (;;) {
            // completions, polled without the lock
            pollable(busy);
            if (!busy.empty()) {
                lk.unlock();
                done.clear();
                for (int k : busy)
                    if (ex_->finished(k)) done.push_back(k);
                lk.lock();
                for (int k : done) finish(k, NEAT_OK);
            }
            bool any_busy = false;
            for (const Slot &sl : slots_) any_busy = any_busy || sl.busy;
            if (stop_ && queue_.empty() && !any_busy) break;
            // admission into a free slot, in arrival order, while the
            // footprint fits (a request alone always fits beside the
            // resident bytes: submit refuses the others); one launch at a
            // time, so launches follow admission order
            const int fs = launching_ == 0 ? free_slot() : -1;
            if (fs >= 0 && !queue_.empty()) {
                Slot &sl = slots_[fs];
                batch.clear();
                while (!queue_.empty() && (int)sl.tickets.size() < max_batch_) {
                    Req &q = reqs_[queue_.front()];
                    if (used_ + q.bytes > cap_) break;
                    admit(fs, queue_.front());
                    batch.push_back(&q.payload);
                    queue_.pop_front();
                }
                if (!sl.tickets.empty()) {
                    run(lk, fs, batch);
                    continue;
                }
            }
            if (any_busy && spin_us_ > 0 && spin(lk)) continue;
            // (a system-clock deadline: pthread_cond_timedwait, which thread
            // checkers follow, unlike the clock-selecting wait)
            if (any_busy)
                cv_.wait_until(lk, std::chrono::system_clock::now() +
                                       std::chrono::microseconds(poll_us_));
            else
                // (a request admitted at submission starts a slot without
                // queueing anything: wake for a busy slot too)
                cv_.wait(lk, [this] {
                    if (stop_ || !queue_.empty()) return true;
                    for (const Slot &sl : slots_)
                        if (sl.busy) return true;
                    return false;
                });
        }
    }

    Executor<Payload> *ex_;
    const uint64_t cap_;
    const int max_batch_, poll_us_, spin_us_;
    const bool direct_;
    std::vector<Slot> slots_;
    const std::chrono::steady_clock::time_point t0_;
    std::mutex m_;
    std::condition_variable cv_;
    bool stop_ = false;
    std::unordered_map<uint64_t, Req> reqs_;
    std::deque<uint64_t> queue_;
    int next_slot_ = 0;
    uint64_t next_ticket_ = 1;
    int launching_ = 0;                // slots whose launch is in progress
    std::atomic<uint64_t> wake_{0};    // requests queued or slots started (read while spinning)
    uint64_t used_ = 0, resident_ = 0, peak_ = 0;
    std::vector<int64_t> lat_ns_;
    uint64_t submitted_ = 0, admitted_ = 0, completed_ = 0, rejected_ = 0, batches_ = 0;
    uint64_t batched_ = 0, genome_inputs_ = 0;
    int64_t first_submit_ = -1, last_done_ = -1;
    std::thread worker_;  // last: started once every member above exists
};

}  // namespace sched
}  // namespace neat
