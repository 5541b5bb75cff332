// server.hip -- the served path: resident populations and a continuous-
// batching request loop.
//
// Populations are registered once: the library copies their encoding into
// its own device memory and runs the transformation (Section 3.3) then, so
// every later request only runs the calculation.  Requests are queued by
// neat_submit; one scheduler thread admits them in arrival order while the
// bytes they touch (inputs, outputs, work-unit tables) fit under the
// configured cap and fewer than max_inflight batches are running, gathers
// everything admitted into one batch (forward_plan over all of its requests:
// one launch per value-store kernel), uploads the batch's work-unit tables
// and launches it on the next of max_inflight streams, so consecutive
// batches overlap on the device.  Completion is detected by polling each
// batch's event; the request is then done and its bytes are released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "abi.h"
#include "launch.h"
#include "neat.h"
#include "program.h"

using namespace neat::abi;

namespace {

constexpr int MAX_BATCH_REQUESTS = 1024;
constexpr size_t TABLE_ITEMS = 4 * MAX_BATCH_REQUESTS;  // items per batch table
// work-unit table bytes a request may add to its batch (one item per slot
// class)
constexpr size_t REQ_TABLE_BYTES = 4 * sizeof(neat::FwdItem);

int64_t now_ns(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now() - t0)
        .count();
}

struct Pop {
    neat_dims d{};
    float *nodes = nullptr, *conns = nullptr;
    int32_t *program = nullptr;
};

enum ReqState { Q_QUEUED = 0, Q_ADMITTED = 1, Q_DONE = 2 };

struct Req {
    neat_request r{};
    neat_result res{};
    size_t bytes = 0;
    int state = Q_QUEUED;
};

// Per in-flight slot: stream, event, pinned and device work-unit tables.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    neat::FwdItem *host = nullptr;  // pinned
    neat::FwdItem *dev = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
    size_t bytes = 0;
    int64_t genome_inputs = 0;
};

}  // namespace

struct neat_server {
    neat_server_cfg cfg{};
    std::chrono::steady_clock::time_point t0;
    std::mutex m;
    std::condition_variable cv;
    bool stop = false;
    std::thread worker;
    std::vector<std::unique_ptr<Pop>> pops;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;
    std::vector<Slot> slots;
    int next_slot = 0;
    uint64_t next_ticket = 1;
    size_t used = 0;
    // statistics since the last reset
    std::vector<int64_t> lat_ns;
    uint64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, batches = 0;
    int64_t genome_inputs = 0, first_submit = -1, last_done = -1;
};

namespace {

size_t request_bytes(const Pop &p, const neat_request &r) {
    const size_t P = (size_t)p.d.P, B = (size_t)r.B;
    size_t in = 0;
    if (r.input_mode == NEAT_INPUT_TENSOR)
        in = (r.input_genome_stride == 0 ? B : P * B) * (size_t)p.d.I * sizeof(float);
    const size_t out = P * B * (size_t)p.d.O * sizeof(float);
    return in + out + REQ_TABLE_BYTES;
}

void finish_slot(neat_server *s, Slot &sl) {
    const int64_t t = now_ns(s->t0);
    for (uint64_t tk : sl.tickets) {
        auto it = s->reqs.find(tk);
        if (it == s->reqs.end()) continue;
        Req &q = it->second;
        q.state = Q_DONE;
        q.res.t_done_ns = t;
        s->lat_ns.push_back(t - q.res.t_submit_ns);
        s->completed++;
    }
    s->genome_inputs += sl.genome_inputs;
    s->last_done = t;
    s->used -= sl.bytes;
    sl.tickets.clear();
    sl.bytes = 0;
    sl.genome_inputs = 0;
    sl.busy = false;
}

// Launch the calculation of the given admitted requests on slot sl (lock
// not held).  Returns NEAT_OK or an error code for all of them.
int launch_batch(neat_server *s, Slot &sl, const std::vector<neat::FwdJob> &jobs) {
    std::vector<neat::FwdKernelLaunch> fw;
    char err[256] = "";
    int rc = neat::forward_plan(jobs.data(), (int)jobs.size(), neat::FWD_AUTO, max_lds_bytes(),
                                fw, err, sizeof(err));
    if (rc != NEAT_OK) return rc;
    size_t n = 0;
    for (const neat::FwdKernelLaunch &k : fw) n += k.items.size();
    if (n > TABLE_ITEMS) return NEAT_E_TOO_LARGE;
    size_t at = 0;
    std::vector<size_t> off(fw.size());
    for (size_t k = 0; k < fw.size(); ++k) {
        off[k] = at;
        std::copy(fw[k].items.begin(), fw[k].items.end(), sl.host + at);
        at += fw[k].items.size();
    }
    hipError_t e = hipMemcpyAsync(sl.dev, sl.host, at * sizeof(neat::FwdItem),
                                  hipMemcpyHostToDevice, sl.stream);
    for (size_t k = 0; k < fw.size() && e == hipSuccess; ++k)
        e = neat::forward_launch(fw[k], sl.dev + off[k], sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    return e == hipSuccess ? NEAT_OK : NEAT_E_HIP;
}

void worker_loop(neat_server *s) {
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->m);
    for (;;) {
        // completions
        bool any_busy = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            if (hipEventQuery(sl.done) == hipSuccess) finish_slot(s, sl);
            else any_busy = true;
        }
        if (s->stop && s->queue.empty() && !any_busy) break;
        // admission into a free slot: requests in arrival order while they fit
        Slot *free_slot = nullptr;
        for (int k = 0; k < (int)s->slots.size(); ++k) {
            Slot &sl = s->slots[(s->next_slot + k) % s->slots.size()];
            if (!sl.busy) {
                free_slot = &sl;
                s->next_slot = (int)((&sl - s->slots.data()) + 1) % (int)s->slots.size();
                break;
            }
        }
        if (free_slot && !s->queue.empty()) {
            Slot &sl = *free_slot;
            std::vector<neat::FwdJob> jobs;
            const int64_t t = now_ns(s->t0);
            while (!s->queue.empty() && (int)sl.tickets.size() < MAX_BATCH_REQUESTS) {
                Req &q = s->reqs[s->queue.front()];
                // in arrival order: a request that does not fit waits for
                // running batches to release their bytes (alone it always
                // fits: neat_submit rejects larger ones)
                if (s->used + q.bytes > s->cfg.cap_bytes) break;
                const Pop &p = *s->pops[q.r.pop_id];
                const bool grid = q.r.input_mode == NEAT_INPUT_GRID;
                jobs.push_back(make_job(&p.d, p.program, q.r.inputs, q.r.input_genome_stride,
                                        q.r.B, q.r.outputs, grid ? q.r.grid_side : 0,
                                        q.r.grid_first));
                q.state = Q_ADMITTED;
                q.res.t_admit_ns = t;
                s->used += q.bytes;
                sl.bytes += q.bytes;
                sl.genome_inputs += (int64_t)p.d.P * q.r.B;
                sl.tickets.push_back(s->queue.front());
                s->queue.pop_front();
                s->admitted++;
            }
            if (!sl.tickets.empty()) {
                sl.busy = true;
                s->batches++;
                lk.unlock();
                const int rc = launch_batch(s, sl, jobs);
                lk.lock();
                if (rc != NEAT_OK) {
                    // the batch never ran: its requests end with the error
                    for (uint64_t tk : sl.tickets) s->reqs[tk].res.status = rc;
                    (void)hipStreamSynchronize(sl.stream);
                    finish_slot(s, sl);
                }
                continue;
            }
        }
        if (any_busy) {
            // poll the running batches again shortly
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        } else {
            s->cv.wait(lk, [s] { return s->stop || !s->queue.empty(); });
        }
    }
}

void free_server(neat_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
    }
    for (auto &p : s->pops) {
        if (p->nodes) (void)hipFree(p->nodes);
        if (p->conns) (void)hipFree(p->conns);
        if (p->program) (void)hipFree(p->program);
    }
    delete s;
}

int64_t percentile(std::vector<int64_t> v, double q) {
    if (v.empty()) return 0;
    const size_t k = (size_t)(q * (double)(v.size() - 1) + 0.5);
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
}

}  // namespace

extern "C" {

int neat_server_create(const neat_server_cfg *cfg, neat_server **out) {
    if (!cfg || !out) return fail(NEAT_E_INVALID, "cfg or out is NULL");
    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess) return hip_fail(e, "device count");
    if (cfg->device < 0 || cfg->device >= n_dev)
        return fail(NEAT_E_INVALID, "device %d outside [0, %d)", cfg->device, n_dev);
    if (cfg->max_inflight < 1 || cfg->max_inflight > 16)
        return fail(NEAT_E_INVALID, "max_inflight = %d outside [1, 16]", cfg->max_inflight);
    if (cfg->cap_bytes == 0) return fail(NEAT_E_INVALID, "cap_bytes is 0");
    neat_server *s = new (std::nothrow) neat_server;
    if (!s) return fail(NEAT_E_NOMEM, "out of host memory");
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    e = hipSetDevice(cfg->device);
    s->slots.resize(cfg->max_inflight);
    for (Slot &sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&sl.host, TABLE_ITEMS * sizeof(neat::FwdItem),
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dev, TABLE_ITEMS * sizeof(neat::FwdItem));
    }
    if (e != hipSuccess) {
        free_server(s);
        return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "server buffers: out of memory")
                                        : hip_fail(e, "server create");
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return NEAT_OK;
}

int neat_server_destroy(neat_server *s) {
    if (!s) return fail(NEAT_E_INVALID, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->m);
        // queued requests are cancelled; admitted ones finish
        for (uint64_t tk : s->queue) {
            Req &q = s->reqs[tk];
            q.state = Q_DONE;
            q.res.status = NEAT_E_SHUTDOWN;
        }
        s->queue.clear();
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->cfg.device);
    for (Slot &sl : s->slots)
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    free_server(s);
    return NEAT_OK;
}

int neat_server_register(neat_server *s, const neat_dims *d, const float *nodes,
                         const float *conns, int32_t *pop_id) {
    if (!s || !pop_id) return fail(NEAT_E_INVALID, "server or pop_id is NULL");
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    rc = check_topo_args(d, nodes, conns, nullptr);
    if (rc != NEAT_OK) return rc;
    std::unique_ptr<Pop> p(new (std::nothrow) Pop);
    if (!p) return fail(NEAT_E_NOMEM, "out of host memory");
    p->d = *d;
    const size_t nb = (size_t)d->P * d->N_max * 5 * sizeof(float);
    const size_t cb = (size_t)d->P * d->C_max * 4 * sizeof(float);
    hipError_t e = hipSetDevice(s->cfg.device);
    hipStream_t st = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void **)&p->nodes, std::max<size_t>(nb, 16));
    if (e == hipSuccess) e = hipMalloc((void **)&p->conns, std::max<size_t>(cb, 16));
    if (e == hipSuccess) e = hipMalloc((void **)&p->program, neat_program_bytes(d));
    if (e == hipSuccess && nb) e = hipMemcpyAsync(p->nodes, nodes, nb, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && cb) e = hipMemcpyAsync(p->conns, conns, cb, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && d->P > 0)
        e = neat::launch_topo(d->P, d->N_max, d->C_max, d->I, d->O, p->nodes, p->conns, nullptr,
                              nullptr, nullptr, p->program, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (st) (void)hipStreamDestroy(st);
    if (e != hipSuccess) {
        if (p->nodes) (void)hipFree(p->nodes);
        if (p->conns) (void)hipFree(p->conns);
        if (p->program) (void)hipFree(p->program);
        return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "register: out of device memory")
                                        : hip_fail(e, "register");
    }
    std::lock_guard<std::mutex> lk(s->m);
    *pop_id = (int32_t)s->pops.size();
    s->pops.push_back(std::move(p));
    return NEAT_OK;
}

int neat_submit(neat_server *s, const neat_request *r, uint64_t *ticket) {
    if (!s || !r || !ticket) return fail(NEAT_E_INVALID, "server, request or ticket is NULL");
    std::unique_lock<std::mutex> lk(s->m);
    if (s->stop) return fail(NEAT_E_SHUTDOWN, "server is shutting down");
    if (r->pop_id < 0 || r->pop_id >= (int32_t)s->pops.size())
        return fail(NEAT_E_INVALID, "unknown population %d", r->pop_id);
    const Pop &p = *s->pops[r->pop_id];
    const bool grid = r->input_mode == NEAT_INPUT_GRID;
    if (!grid && r->input_mode != NEAT_INPUT_TENSOR)
        return fail(NEAT_E_INVALID, "unknown input_mode %d", r->input_mode);
    lk.unlock();
    int rc = check_forward_args(&p.d, p.program, r->inputs, r->input_genome_stride, r->B,
                                r->outputs, grid, r->grid_side, r->grid_first);
    if (rc != NEAT_OK) return rc;
    const size_t bytes = request_bytes(p, *r);
    lk.lock();
    if (bytes > s->cfg.cap_bytes) {
        s->rejected++;
        return fail(NEAT_E_TOO_LARGE, "request needs %zu bytes, cap is %llu", bytes,
                    (unsigned long long)s->cfg.cap_bytes);
    }
    const uint64_t tk = s->next_ticket++;
    Req &q = s->reqs[tk];
    q.r = *r;
    q.bytes = bytes;
    q.res.status = NEAT_OK;
    q.res.tag = r->tag;
    q.res.t_submit_ns = now_ns(s->t0);
    q.res.t_admit_ns = q.res.t_done_ns = -1;
    if (s->first_submit < 0) s->first_submit = q.res.t_submit_ns;
    s->submitted++;
    if (r->B == 0 || p.d.P == 0) {
        // nothing to compute
        q.state = Q_DONE;
        q.res.t_admit_ns = q.res.t_done_ns = q.res.t_submit_ns;
    } else {
        s->queue.push_back(tk);
    }
    *ticket = tk;
    lk.unlock();
    s->cv.notify_one();
    return NEAT_OK;
}

int neat_poll(neat_server *s, uint64_t ticket, neat_result *res) {
    if (!s) return fail(NEAT_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(NEAT_E_UNKNOWN_TICKET, "unknown ticket %llu",
                                         (unsigned long long)ticket);
    if (it->second.state != Q_DONE) return NEAT_PENDING;
    if (res) *res = it->second.res;
    s->reqs.erase(it);
    return NEAT_OK;
}

int neat_server_stats(neat_server *s, neat_stats *st) {
    if (!s || !st) return fail(NEAT_E_INVALID, "server or stats is NULL");
    std::lock_guard<std::mutex> lk(s->m);
    neat_stats r{};
    r.submitted = s->submitted;
    r.admitted = s->admitted;
    r.completed = s->completed;
    r.rejected = s->rejected;
    r.batches = s->batches;
    r.queued = s->queue.size();
    r.genome_inputs = (uint64_t)s->genome_inputs;
    r.p50_ms = (double)percentile(s->lat_ns, 0.50) / 1e6;
    r.p99_ms = (double)percentile(s->lat_ns, 0.99) / 1e6;
    const int64_t span = s->last_done - s->first_submit;
    r.throughput = span > 0 ? (double)s->genome_inputs * 1e9 / (double)span : 0.0;
    *st = r;
    return NEAT_OK;
}

int neat_server_reset_stats(neat_server *s) {
    if (!s) return fail(NEAT_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->m);
    s->lat_ns.clear();
    s->submitted = s->admitted = s->completed = s->rejected = s->batches = 0;
    s->genome_inputs = 0;
    s->first_submit = s->last_done = -1;
    return NEAT_OK;
}

}  // extern "C"
