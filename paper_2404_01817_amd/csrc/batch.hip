// batch.hip -- the batched path: many populations in one call, recorded
// once into a HIP graph and replayed.
//
// The calculation of all items is planned together (forward_plan): one
// launch per value-store kernel whose work units span every population, so
// a batch of uneven populations costs a handful of launches rather than one
// (or four) per population, and small populations fill the GPU together.
// The work-unit tables of those launches live in device memory owned by the
// plan.  Transformations (items with nodes) are recorded before the
// calculations, batched the same way: one launch per workgroup size (64 to
// 1024 threads, in steps of 64) over the genomes of every population in
// it, then one launch listing the genomes of every population by class
// (populations of N_max <= 62 need no list: all their genomes are R64).
// The launches of each stage are independent and are recorded as parallel
// branches of the graph (the forward kernels after the class lists), so a
// long launch's tail overlaps the others.
//
// neat_forward_batch_noalloc plans the same launches and issues them
// directly on the caller's stream, with the work-unit tables in a static
// device array instead of allocated memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "abi.h"
#include "launch.h"
#include "tune.h"
#include "neat.h"
#include "program.h"

using namespace neat::abi;

struct neat_batch_plan {
    std::vector<neat_batch_item> items;
    int device = -1;
    void *tables = nullptr;  // FwdItem tables of the multi-item launches
    void *topo_tables = nullptr;  // TopoItem tables: buckets, then all items
    unsigned *counters = nullptr; // one unit counter per forward launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int launches = 0;
    unsigned tune_gen = 0;  // the tune table's generation the plan was built with
};

namespace {

void destroy(neat_batch_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->tables) (void)hipFree(p->tables);
    if (p->topo_tables) (void)hipFree(p->topo_tables);
    if (p->counters) (void)hipFree(p->counters);
    delete p;
}

int check_item(const neat_batch_item &it, int32_t k) {
    int rc = check_dims(&it.dims);
    if (rc != NEAT_OK) return fail(rc, "item %d: %s", k, neat_last_error());
    if (it.nodes) {
        rc = check_topo_args(&it.dims, it.nodes, it.conns, it.program);
        if (rc != NEAT_OK) return fail(rc, "item %d: %s", k, neat_last_error());
        if (it.dims.P > 0 && !it.program)
            return fail(NEAT_E_INVALID, "item %d: program is NULL", k);
    }
    rc = check_forward_args(&it.dims, it.program, it.inputs, it.input_genome_stride, it.B,
                            it.outputs, it.grid_side > 0, it.grid_side, it.grid_first);
    if (rc != NEAT_OK) return fail(rc, "item %d: %s", k, neat_last_error());
    return NEAT_OK;
}

// Transformation launches: one per workgroup-size bucket, then the class
// lists of every item.
struct TopoLaunch {
    int n;
    long long blocks;
    int threads;
    size_t lds;
    const neat::TopoItem *table;
};

// Capture streams: the launches of one stage (the transformation buckets,
// then the forward kernels) are independent, so they are recorded as
// parallel branches of the graph; the class lists wait for every bucket.
constexpr int N_BRANCH = 6;

// Streams 1 .. m-1 of cs join stream 0 (fork: 0 -> others; join: others ->
// 0); a stage of one launch stays on stream 0 with no fork at all.
hipError_t link(hipStream_t *cs, bool fork, hipEvent_t *ev, int m) {
    for (int i = 1; i < std::min(m, N_BRANCH); ++i) {
        hipStream_t from = fork ? cs[0] : cs[i], to = fork ? cs[i] : cs[0];
        hipError_t e = hipEventRecord(ev[i], from);
        if (e == hipSuccess) e = hipStreamWaitEvent(to, ev[i], 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Record every launch of the batch; cs[0] is capturing, the other streams
// are forked from it and joined back at the end.
int record(const std::vector<TopoLaunch> &topo, const neat::TopoItem *all_topo, int n_topo,
           const std::vector<neat::FwdKernelLaunch> &fw,
           const std::vector<const neat::FwdItem *> &tab, unsigned *counters, hipStream_t *cs,
           hipEvent_t *ev) {
    const int mt = (int)topo.size(), mf = (int)fw.size();
    hipError_t e = link(cs, true, ev, mt);
    for (size_t k = 0; e == hipSuccess && k < topo.size(); ++k) {
        const TopoLaunch &t = topo[k];
        e = neat::launch_topo_batch(t.table, t.n, t.blocks, t.threads, t.lds, cs[k % N_BRANCH]);
        if (e != hipSuccess) return hip_fail(e, "batch transformation launch");
    }
    if (e == hipSuccess) e = link(cs, false, ev, mt);
    if (e == hipSuccess && n_topo) {
        e = neat::launch_classify_batch(all_topo, n_topo, cs[0]);
        if (e != hipSuccess) return hip_fail(e, "batch class lists launch");
    }
    if (e == hipSuccess && counters) e = neat::launch_zero_counters(counters, (int)fw.size(), cs[0]);
    if (e == hipSuccess) e = link(cs, true, ev, mf);
    for (size_t k = 0; e == hipSuccess && k < fw.size(); ++k) {
        e = neat::forward_launch(fw[k], tab[k], cs[k % N_BRANCH], counters ? counters + k : nullptr);
        if (e != hipSuccess) return hip_fail(e, "batch forward launch");
    }
    if (e == hipSuccess) e = link(cs, false, ev, mf);
    return e == hipSuccess ? NEAT_OK : hip_fail(e, "batch stream fork or join");
}

// Everything one batch launches, planned on the host: the transformation
// launches (their table fields are offsets into topo_host until resolved),
// the class-list launch over topo_host[all_off ..], and the forward launches
// with the items of the multi-item ones gathered in fw_host (fw_off: each
// launch's first item there, -1 when its single item is passed inline).
struct HostPlan {
    std::vector<TopoLaunch> topo;
    std::vector<neat::TopoItem> topo_host;
    size_t all_off = 0;
    int n_topo = 0;
    std::vector<neat::FwdKernelLaunch> fw;
    std::vector<neat::FwdItem> fw_host;
    std::vector<long long> fw_off;
    int launches() const { return (int)topo.size() + (n_topo ? 1 : 0) + (int)fw.size(); }
};

int plan_host(const neat_batch_item *items, int32_t n, HostPlan &hp) {
    // transformations bucketed by workgroup size (64 x (b + 1) threads): each
    // genome runs with the waves its N_max needs, and a launch reserves the
    // LDS of its own genomes only
    constexpr int NB = 16;
    std::vector<neat::TopoItem> bucket[NB], all_topo;
    for (int32_t k = 0; k < n; ++k) {
        const neat_batch_item &it = items[k];
        if (!it.nodes || it.dims.P == 0) continue;
        const neat_dims &d = it.dims;
        neat::TopoItem ti{it.nodes, it.conns, nullptr, nullptr, it.status, (int32_t *)it.program,
                          d.P, d.N_max, d.C_max, d.I, d.O, neat::prog_words(d.N_max, d.C_max, d.O),
                          0};
        const int b = neat::topo_block_threads(d.N_max) / 64 - 1;
        bucket[b].push_back(ti);
        // class lists only where genomes can need more than 64 value slots
        if (neat::max_class(d.N_max) != neat::CLS_R64) all_topo.push_back(ti);
    }
    for (int b = 0; b < NB; ++b) {
        if (bucket[b].empty()) continue;
        TopoLaunch t{(int)bucket[b].size(), 0, 64, 0, nullptr};
        for (neat::TopoItem &ti : bucket[b]) {
            ti.block0 = t.blocks;
            t.blocks += ti.P;
            t.threads = std::max(t.threads, neat::topo_block_threads(ti.N));
            t.lds = std::max(t.lds, neat::topo_lds_bytes(ti.N, ti.C));
        }
        t.table = (const neat::TopoItem *)(uintptr_t)hp.topo_host.size();  // offset for now
        hp.topo_host.insert(hp.topo_host.end(), bucket[b].begin(), bucket[b].end());
        hp.topo.push_back(t);
    }
    hp.all_off = hp.topo_host.size();
    hp.topo_host.insert(hp.topo_host.end(), all_topo.begin(), all_topo.end());
    hp.n_topo = (int)all_topo.size();

    std::vector<neat::FwdJob> jobs;
    std::vector<int> job_variant;
    for (int32_t k = 0; k < n; ++k) {
        const neat_batch_item &it = items[k];
        if (it.dims.P == 0 || it.B == 0) continue;
        jobs.push_back(make_job(&it.dims, it.program, it.inputs, it.input_genome_stride, it.B,
                                it.outputs, it.grid_side, it.grid_first));
        job_variant.push_back(
            neat::tuned_variant(it.dims.N_max, it.dims.C_max, it.B, it.grid_side > 0, 1));
    }
    // every item with the variant tuned for its bucket's throughput (the
    // batch fills the GPU; FWD_AUTO while none is), one launch per kernel
    // kind over all of them
    for (size_t j = 0; j < jobs.size(); ++j) jobs[j].variant = job_variant[j];
    if (!jobs.empty()) {
        char err[256] = "";
        const int rc = neat::forward_plan(jobs.data(), (int)jobs.size(), neat::FWD_AUTO,
                                          max_lds_bytes(), hp.fw, err, sizeof(err));
        if (rc != NEAT_OK) return fail(rc, "%s", err);
    }
    // work-unit tables of the launches with more than one item
    hp.fw_off.assign(hp.fw.size(), -1);
    for (size_t k = 0; k < hp.fw.size(); ++k) {
        if (hp.fw[k].items.size() <= 1) continue;
        hp.fw_off[k] = (long long)hp.fw_host.size();
        hp.fw_host.insert(hp.fw_host.end(), hp.fw[k].items.begin(), hp.fw[k].items.end());
    }
    return NEAT_OK;
}

// Point the launches at their tables in device memory (topo_dev: a copy of
// topo_host, fw_dev: a copy of fw_host).
void resolve_tables(HostPlan &hp, const neat::TopoItem *topo_dev, const neat::FwdItem *fw_dev,
                    const neat::TopoItem **all_dev, std::vector<const neat::FwdItem *> &tab) {
    for (TopoLaunch &t : hp.topo) t.table = topo_dev + (uintptr_t)t.table;
    *all_dev = hp.n_topo ? topo_dev + hp.all_off : nullptr;
    tab.assign(hp.fw.size(), nullptr);
    for (size_t k = 0; k < hp.fw.size(); ++k)
        if (hp.fw_off[k] >= 0) tab[k] = fw_dev + hp.fw_off[k];
}

// Persistent forward launches of a batch deal their units to workgroups
// round robin.  NEAT_BATCH_DYNAMIC=1 makes every wave take its next unit
// from a counter instead (for comparison: on the uneven workload the
// tuned batch's calculation took 0.874 ms that way against 0.613 ms round
// robin, the atomics on one counter serializing over tens of thousands of
// units).
bool dynamic_units() {
    static const bool on = [] {
        const char *e = getenv("NEAT_BATCH_DYNAMIC");
        return e && e[0] == '1';
    }();
    return on;
}

int build(const neat_batch_item *items, int32_t n, neat_batch_plan **out) {
    neat_batch_plan *p = new (std::nothrow) neat_batch_plan;
    if (!p) return fail(NEAT_E_NOMEM, "out of host memory");
    p->items.assign(items, items + n);
    (void)hipGetDevice(&p->device);
    p->tune_gen = neat::tune_generation();
    HostPlan hp;
    int rc = plan_host(items, n, hp);
    if (rc != NEAT_OK) {
        destroy(p);
        return rc;
    }
    if (!hp.fw_host.empty()) {
        hipError_t e = hipMalloc(&p->tables, hp.fw_host.size() * sizeof(neat::FwdItem));
        if (e == hipSuccess)
            e = hipMemcpy(p->tables, hp.fw_host.data(), hp.fw_host.size() * sizeof(neat::FwdItem),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(p);
            return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "batch tables: out of memory")
                                            : hip_fail(e, "batch tables");
        }
    }
    if (!hp.topo_host.empty()) {
        hipError_t e = hipMalloc(&p->topo_tables, hp.topo_host.size() * sizeof(neat::TopoItem));
        if (e == hipSuccess)
            e = hipMemcpy(p->topo_tables, hp.topo_host.data(),
                          hp.topo_host.size() * sizeof(neat::TopoItem), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(p);
            return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "batch tables: out of memory")
                                            : hip_fail(e, "batch tables");
        }
    }
    if (dynamic_units() && !hp.fw.empty()) {
        hipError_t e = hipMalloc((void **)&p->counters, hp.fw.size() * sizeof(unsigned));
        if (e != hipSuccess) {
            destroy(p);
            return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "batch counters: out of memory")
                                            : hip_fail(e, "batch counters");
        }
    }
    const neat::TopoItem *all_dev = nullptr;
    std::vector<const neat::FwdItem *> tab;
    resolve_tables(hp, (const neat::TopoItem *)p->topo_tables, (const neat::FwdItem *)p->tables,
                   &all_dev, tab);

    // record the launches into a graph on private streams (default
    // priority), the branches of each stage on streams forked from cs[0]
    hipStream_t cs[N_BRANCH] = {};
    hipEvent_t ev[N_BRANCH] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < N_BRANCH && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&cs[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    }
    auto release = [&]() {
        for (int i = 0; i < N_BRANCH; ++i) {
            if (ev[i]) (void)hipEventDestroy(ev[i]);
            if (cs[i]) (void)hipStreamDestroy(cs[i]);
        }
    };
    if (e != hipSuccess) {
        release();
        destroy(p);
        return hip_fail(e, "capture streams");
    }
    e = hipStreamBeginCapture(cs[0], hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release();
        destroy(p);
        return hip_fail(e, "begin capture");
    }
    rc = record(hp.topo, all_dev, hp.n_topo, hp.fw, tab, p->counters, cs, ev);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs[0], &g);
    release();
    p->graph = g;
    if (rc != NEAT_OK || e != hipSuccess) {
        destroy(p);
        return rc != NEAT_OK ? rc : hip_fail(e, "end capture");
    }
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy(p);
        return hip_fail(e, "graph instantiate");
    }
    p->launches = hp.launches();
    *out = p;
    return NEAT_OK;
}

// ---- the batch without device allocation ---------------------------------
// The work-unit tables live in a file-scope device array (one copy per GPU,
// held until the process ends).  Host code never passes the array's name to
// a kernel or a copy: its device address comes from hipGetSymbolAddress,
// once per device, and only that address is used.
__device__ __align__(256) unsigned char scratch[NEAT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

int scratch_ptr(int dev, unsigned char **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(NEAT_E_INVALID, "device %d unsupported", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "address of the batch scratch area");
        if (!ptr) return fail(NEAT_E_HIP, "address of the batch scratch area is NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return NEAT_OK;
}

// Table words travel as kernel arguments (captured by value, no host buffer
// has to outlive the call) and a small kernel stores them.
constexpr int WR_WORDS = 896;
struct WriteChunk {
    uint32_t *dst;
    uint32_t n;
    uint32_t w[WR_WORDS];
};

__global__ __launch_bounds__(256) void write_words_kernel(WriteChunk c) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) c.dst[i] = c.w[i];
}

hipError_t write_words(unsigned char *dst, const void *src, size_t bytes, hipStream_t stream) {
    const uint32_t *s = (const uint32_t *)src;
    size_t words = bytes / 4;
    WriteChunk c;
    for (size_t off = 0; off < words; off += WR_WORDS) {
        c.dst = (uint32_t *)dst + off;
        c.n = (uint32_t)std::min<size_t>(WR_WORDS, words - off);
        memcpy(c.w, s + off, c.n * sizeof(uint32_t));
        hipLaunchKernelGGL(write_words_kernel, dim3(1), dim3(256), 0, stream, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }
// Field by field (struct padding may hold anything).
bool same_item(const neat_batch_item &a, const neat_batch_item &b) {
    return a.dims.P == b.dims.P && a.dims.N_max == b.dims.N_max && a.dims.C_max == b.dims.C_max &&
           a.dims.I == b.dims.I && a.dims.O == b.dims.O && a.nodes == b.nodes &&
           a.conns == b.conns && a.status == b.status && a.program == b.program &&
           a.inputs == b.inputs && a.input_genome_stride == b.input_genome_stride &&
           a.B == b.B && a.grid_side == b.grid_side && a.grid_first == b.grid_first &&
           a.outputs == b.outputs;
}

bool same_items(const neat_batch_plan *p, const neat_batch_item *items, int32_t n) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (p->device != dev || (size_t)n != p->items.size()) return false;
    if (p->tune_gen != neat::tune_generation()) return false;  // re-tuned since recorded
    for (int32_t k = 0; k < n; ++k)
        if (!same_item(p->items[k], items[k])) return false;
    return true;
}

}  // namespace

extern "C" {

int neat_forward_batch(const neat_batch_item *items, int32_t n, neat_batch_plan **plan,
                       void *stream) {
    if (!plan) return fail(NEAT_E_INVALID, "plan is NULL");
    if (n < 0 || (n > 0 && !items)) return fail(NEAT_E_INVALID, "bad item list (n = %d)", n);
    if (!*plan || !same_items(*plan, items, n)) {
        for (int32_t k = 0; k < n; ++k) {
            int rc = check_item(items[k], k);
            if (rc != NEAT_OK) return rc;
        }
        neat_batch_plan *p = nullptr;
        int rc = build(items, n, &p);
        if (rc != NEAT_OK) return rc;
        destroy(*plan);
        *plan = p;
    }
    hipError_t e = hipGraphLaunch((*plan)->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return NEAT_OK;
}

void neat_batch_plan_free(neat_batch_plan *plan) { destroy(plan); }

int neat_forward_batch_noalloc(const neat_batch_item *items, int32_t n, void *stream) {
    if (n < 0 || (n > 0 && !items)) return fail(NEAT_E_INVALID, "bad item list (n = %d)", n);
    for (int32_t k = 0; k < n; ++k) {
        const int rc = check_item(items[k], k);
        if (rc != NEAT_OK) return rc;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    unsigned char *base = nullptr;
    int rc = scratch_ptr(dev, &base);
    if (rc != NEAT_OK) return rc;
    HostPlan hp;
    rc = plan_host(items, n, hp);
    if (rc != NEAT_OK) return rc;
    const size_t topo_bytes = hp.topo_host.size() * sizeof(neat::TopoItem);
    const size_t fw_bytes = hp.fw_host.size() * sizeof(neat::FwdItem);
    const size_t cnt_bytes = dynamic_units() ? hp.fw.size() * sizeof(unsigned) : 0;
    const size_t need = align256(topo_bytes) + align256(fw_bytes) + cnt_bytes;
    if (need > NEAT_NOALLOC_SCRATCH_BYTES)
        return fail(NEAT_E_TOO_LARGE,
                    "the batch's work-unit tables need %zu B, the scratch area holds %d B",
                    need, NEAT_NOALLOC_SCRATCH_BYTES);
    hipStream_t s = (hipStream_t)stream;
    unsigned char *fw_base = base + align256(topo_bytes);
    if (topo_bytes) e = write_words(base, hp.topo_host.data(), topo_bytes, s);
    if (e == hipSuccess && fw_bytes) e = write_words(fw_base, hp.fw_host.data(), fw_bytes, s);
    if (e != hipSuccess) return hip_fail(e, "batch tables");
    const neat::TopoItem *all_dev = nullptr;
    std::vector<const neat::FwdItem *> tab;
    resolve_tables(hp, (const neat::TopoItem *)base, (const neat::FwdItem *)fw_base, &all_dev,
                   tab);
    for (const TopoLaunch &t : hp.topo) {
        e = neat::launch_topo_batch(t.table, t.n, t.blocks, t.threads, t.lds, s);
        if (e != hipSuccess) return hip_fail(e, "batch transformation launch");
    }
    if (hp.n_topo) {
        e = neat::launch_classify_batch(all_dev, hp.n_topo, s);
        if (e != hipSuccess) return hip_fail(e, "batch class lists launch");
    }
    // unit counters after the tables, zeroed by a kernel before the launches
    unsigned *cnt = cnt_bytes ? (unsigned *)(fw_base + align256(fw_bytes)) : nullptr;
    if (cnt) {
        e = neat::launch_zero_counters(cnt, (int)hp.fw.size(), s);
        if (e != hipSuccess) return hip_fail(e, "batch counters");
    }
    for (size_t k = 0; k < hp.fw.size(); ++k) {
        e = neat::forward_launch(hp.fw[k], tab[k], s, cnt ? cnt + k : nullptr);
        if (e != hipSuccess) return hip_fail(e, "batch forward launch");
    }
    return NEAT_OK;
}

int32_t neat_batch_plan_launches(const neat_batch_plan *plan) {
    return plan ? plan->launches : 0;
}

}  // extern "C"
