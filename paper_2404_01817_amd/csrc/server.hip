// server.hip -- the served path: resident populations and a continuous-
// batching request loop.
//
// Populations are registered once: the library copies their encoding into
// its own device memory and runs the transformation (Section 3.3) then, so
// every later request only runs the calculation.  The scheduler (scheduler.h)
// admits queued requests in arrival order while the device footprint --
// resident populations plus the bytes of running requests (inputs,
// outputs, work-unit tables) -- stays under the configured cap and fewer
// than max_inflight batches run; everything admitted together forms one
// batch.  The HIP executor below plans a batch (forward_plan over all of
// its requests: one launch per kernel kind, each request with the variant
// tuned for its bucket -- the latency winner when it runs alone, the
// throughput winner when it shares the batch), uploads the work-unit tables
// and launches the batch on its slot's stream, so consecutive batches
// overlap on the device; completion is an event per slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "abi.h"
#include "launch.h"
#include "neat.h"
#include "program.h"
#include "scheduler.h"
#include "tune.h"

using namespace neat::abi;

namespace {

constexpr int MAX_BATCH_REQUESTS = 1024;
constexpr size_t TABLE_ITEMS = 4 * MAX_BATCH_REQUESTS;  // items per batch table
// work-unit table bytes a request may add to its batch (one item per slot
// class)
constexpr size_t REQ_TABLE_BYTES = 4 * sizeof(neat::FwdItem);
// completion polling of the scheduler: without sleeping for up to SPIN_US
// after each admission or completion, then every POLL_US; a request that
// finds the server idle is launched by the submitting thread
constexpr int POLL_US = 20;
constexpr int SPIN_US = 250;
constexpr bool DIRECT = true;

struct Pop {
    neat_dims d{};
    float *nodes = nullptr, *conns = nullptr;
    int32_t *program = nullptr;
};

struct Payload {
    neat_request r{};
    const Pop *pop = nullptr;
};

// Per in-flight slot: stream, event, pinned and device work-unit tables.
struct SlotRes {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    neat::FwdItem *host = nullptr;  // pinned
    neat::FwdItem *dev = nullptr;
};

class HipExec : public neat::sched::Executor<Payload> {
  public:
    int device = 0;
    std::vector<SlotRes> slots;

    void thread_init() override { (void)hipSetDevice(device); }

    // A request admitted at submission is launched on the caller's thread:
    // the server's device for the launch, the caller's current device kept.
    int launch(int k, const std::vector<const Payload *> &batch) override {
        int prev = device;
        if (hipGetDevice(&prev) != hipSuccess) prev = device;
        if (prev != device && hipSetDevice(device) != hipSuccess) return NEAT_E_HIP;
        const int rc = launch_on(k, batch);
        if (prev != device) (void)hipSetDevice(prev);
        return rc;
    }

    int launch_on(int k, const std::vector<const Payload *> &batch) {
        SlotRes &sl = slots[k];
        std::vector<neat::FwdJob> jobs;
        jobs.reserve(batch.size());
        const int tp = batch.size() > 1 ? 1 : 0;
        for (const Payload *q : batch) {
            const neat_request &r = q->r;
            const bool grid = r.input_mode == NEAT_INPUT_GRID;
            neat::FwdJob j = make_job(&q->pop->d, q->pop->program, r.inputs,
                                      r.input_genome_stride, r.B, r.outputs,
                                      grid ? r.grid_side : 0, r.grid_first);
            j.variant = neat::tuned_variant(q->pop->d.N_max, q->pop->d.C_max, r.B, grid, tp);
            jobs.push_back(j);
        }
        std::vector<neat::FwdKernelLaunch> fw;
        char err[256] = "";
        int rc = neat::forward_plan(jobs.data(), (int)jobs.size(), neat::FWD_AUTO,
                                    max_lds_bytes(), fw, err, sizeof(err));
        if (rc != NEAT_OK) return rc;
        // only launches of several items read a table; a launch of one item
        // takes it inline in its arguments, so a batch of single-item
        // launches (a request alone, the common case at low rates) starts
        // without a copy ahead of it on the stream
        size_t n = 0;
        for (const neat::FwdKernelLaunch &f : fw)
            if (f.items.size() > 1) n += f.items.size();
        if (n > TABLE_ITEMS) return NEAT_E_TOO_LARGE;
        size_t at = 0;
        std::vector<long long> off(fw.size(), -1);
        for (size_t f = 0; f < fw.size(); ++f) {
            if (fw[f].items.size() <= 1) continue;
            off[f] = (long long)at;
            std::copy(fw[f].items.begin(), fw[f].items.end(), sl.host + at);
            at += fw[f].items.size();
        }
        hipError_t e = hipSuccess;
        if (at)
            e = hipMemcpyAsync(sl.dev, sl.host, at * sizeof(neat::FwdItem), hipMemcpyHostToDevice,
                               sl.stream);
        for (size_t f = 0; f < fw.size() && e == hipSuccess; ++f)
            e = neat::forward_launch(fw[f], off[f] >= 0 ? sl.dev + off[f] : nullptr, sl.stream);
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
        return e == hipSuccess ? NEAT_OK : NEAT_E_HIP;
    }

    bool finished(int k) override { return hipEventQuery(slots[k].done) == hipSuccess; }

    void drain(int k) override { (void)hipStreamSynchronize(slots[k].stream); }
};

size_t request_bytes(const Pop &p, const neat_request &r) {
    const size_t P = (size_t)p.d.P, B = (size_t)r.B;
    size_t in = 0;
    if (r.input_mode == NEAT_INPUT_TENSOR)
        in = (r.input_genome_stride == 0 ? B : P * B) * (size_t)p.d.I * sizeof(float);
    const size_t out = P * B * (size_t)p.d.O * sizeof(float);
    return in + out + REQ_TABLE_BYTES;
}

// device bytes a registered population holds for good
size_t resident_bytes(const neat_dims &d) {
    return (size_t)d.P * d.N_max * 5 * sizeof(float) + (size_t)d.P * d.C_max * 4 * sizeof(float) +
           neat_program_bytes(&d);
}

}  // namespace

struct neat_server {
    neat_server_cfg cfg{};
    HipExec exec;
    std::unique_ptr<neat::sched::Scheduler<Payload>> sched;
    std::mutex pm;  // guards pops
    std::vector<std::unique_ptr<Pop>> pops;
};

namespace {

void free_server(neat_server *s) {
    for (SlotRes &sl : s->exec.slots) {
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
    s->exec.device = cfg->device;
    neat::tune_cache_use(cfg->tune_cache_path);
    e = hipSetDevice(cfg->device);
    s->exec.slots.resize(cfg->max_inflight);
    for (SlotRes &sl : s->exec.slots) {
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
    s->sched.reset(new (std::nothrow) neat::sched::Scheduler<Payload>(
        &s->exec, cfg->max_inflight, cfg->cap_bytes, MAX_BATCH_REQUESTS, POLL_US, SPIN_US, DIRECT));
    if (!s->sched) {
        free_server(s);
        return fail(NEAT_E_NOMEM, "out of host memory");
    }
    *out = s;
    return NEAT_OK;
}

int neat_server_destroy(neat_server *s) {
    if (!s) return fail(NEAT_E_INVALID, "server is NULL");
    // queued requests are cancelled; admitted ones finish
    s->sched->shutdown();
    (void)hipSetDevice(s->cfg.device);
    for (SlotRes &sl : s->exec.slots)
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    s->sched.reset();
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
    const size_t held = resident_bytes(*d);
    if (s->sched->add_resident(held) != NEAT_OK)
        return fail(NEAT_E_TOO_LARGE,
                    "population needs %zu resident bytes beyond the cap of %llu", held,
                    (unsigned long long)s->cfg.cap_bytes);
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
        // the bytes stay counted: a failed registration leaves the
        // footprint as an upper bound (freed memory is not reused here)
        return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "register: out of device memory")
                                        : hip_fail(e, "register");
    }
    std::lock_guard<std::mutex> lk(s->pm);
    *pop_id = (int32_t)s->pops.size();
    s->pops.push_back(std::move(p));
    return NEAT_OK;
}

int neat_submit(neat_server *s, const neat_request *r, uint64_t *ticket) {
    if (!s || !r || !ticket) return fail(NEAT_E_INVALID, "server, request or ticket is NULL");
    Payload q;
    q.r = *r;
    {
        std::lock_guard<std::mutex> lk(s->pm);
        if (r->pop_id < 0 || r->pop_id >= (int32_t)s->pops.size())
            return fail(NEAT_E_INVALID, "unknown population %d", r->pop_id);
        q.pop = s->pops[r->pop_id].get();
    }
    const Pop &p = *q.pop;
    const bool grid = r->input_mode == NEAT_INPUT_GRID;
    if (!grid && r->input_mode != NEAT_INPUT_TENSOR)
        return fail(NEAT_E_INVALID, "unknown input_mode %d", r->input_mode);
    int rc = check_forward_args(&p.d, p.program, r->inputs, r->input_genome_stride, r->B,
                                r->outputs, grid, r->grid_side, r->grid_first);
    if (rc != NEAT_OK) return rc;
    const size_t bytes = request_bytes(p, *r);
    rc = s->sched->submit(q, bytes, (uint64_t)p.d.P * (uint64_t)r->B, r->tag,
                          r->B == 0 || p.d.P == 0, ticket);
    if (rc == NEAT_E_TOO_LARGE)
        return fail(rc, "request needs %zu bytes beyond the resident populations, cap is %llu",
                    bytes, (unsigned long long)s->cfg.cap_bytes);
    if (rc == NEAT_E_SHUTDOWN) return fail(rc, "server is shutting down");
    return rc;
}

int neat_submit_many(neat_server *s, const neat_request *reqs, int32_t n, uint64_t *tickets) {
    if (!s || n < 0 || (n > 0 && (!reqs || !tickets)))
        return fail(NEAT_E_INVALID, "server, requests or tickets is NULL, or n = %d", n);
    for (int32_t k = 0; k < n; ++k) {
        const int rc = neat_submit(s, &reqs[k], &tickets[k]);
        if (rc != NEAT_OK) {
            for (int32_t j = k; j < n; ++j) tickets[j] = 0;
            return fail(rc, "request %d of %d: %s", k, n, neat_last_error());
        }
    }
    return NEAT_OK;
}

int neat_poll(neat_server *s, uint64_t ticket, neat_result *res) {
    if (!s) return fail(NEAT_E_INVALID, "server is NULL");
    neat::sched::Result r;
    const int rc = s->sched->poll(ticket, &r);
    if (rc == NEAT_E_UNKNOWN_TICKET)
        return fail(rc, "unknown ticket %llu", (unsigned long long)ticket);
    if (rc == NEAT_OK && res) {
        res->status = r.status;
        res->tag = r.tag;
        res->t_submit_ns = r.t_submit_ns;
        res->t_admit_ns = r.t_admit_ns;
        res->t_done_ns = r.t_done_ns;
    }
    return rc;
}

int neat_server_stats(neat_server *s, neat_stats *st) {
    if (!s || !st) return fail(NEAT_E_INVALID, "server or stats is NULL");
    const neat::sched::Stats x = s->sched->stats();
    neat_stats r{};
    r.submitted = x.submitted;
    r.admitted = x.admitted;
    r.completed = x.completed;
    r.rejected = x.rejected;
    r.batches = x.batches;
    r.queued = x.queued;
    r.genome_inputs = x.genome_inputs;
    r.p50_ms = x.p50_ms;
    r.p99_ms = x.p99_ms;
    r.throughput = x.throughput;
    r.batched_requests = x.batched_requests;
    r.resident_bytes = x.resident_bytes;
    r.peak_bytes = x.peak_bytes;
    *st = r;
    return NEAT_OK;
}

int neat_server_reset_stats(neat_server *s) {
    if (!s) return fail(NEAT_E_INVALID, "server is NULL");
    s->sched->reset_stats();
    return NEAT_OK;
}

}  // extern "C"
