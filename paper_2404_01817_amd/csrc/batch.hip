// batch.hip -- the batched path: many populations in one call, recorded
// once into a HIP graph and replayed.
//
// The calculation of all items is planned together (forward_plan): one
// launch per value-store kernel whose work units span every population, so
// a batch of uneven populations costs a handful of launches rather than one
// (or four) per population, and small populations fill the GPU together.
// The work-unit tables of those launches live in device memory owned by the
// plan.  Transformations (items with nodes) are recorded before the
// calculations, batched the same way: one launch per workgroup-size bucket
// (64, 128, 256, 512, 1024 threads) over the genomes of every population in
// it, then one launch listing the genomes of every population by class.
// The launches of each stage are independent and are recorded as parallel
// branches of the graph (the forward kernels after the class lists), so a
// long launch's tail overlaps the others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
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
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int launches = 0;
};

namespace {

void destroy(neat_batch_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->tables) (void)hipFree(p->tables);
    if (p->topo_tables) (void)hipFree(p->topo_tables);
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

// Every stream of cs joins stream 0 (fork: 0 -> others; join: others -> 0).
hipError_t link(hipStream_t *cs, bool fork, hipEvent_t *ev) {
    for (int i = 1; i < N_BRANCH; ++i) {
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
           const std::vector<const neat::FwdItem *> &tab, hipStream_t *cs, hipEvent_t *ev) {
    hipError_t e = link(cs, true, ev);
    for (size_t k = 0; e == hipSuccess && k < topo.size(); ++k) {
        const TopoLaunch &t = topo[k];
        e = neat::launch_topo_batch(t.table, t.n, t.blocks, t.threads, t.lds, cs[k % N_BRANCH]);
        if (e != hipSuccess) return hip_fail(e, "batch transformation launch");
    }
    if (e == hipSuccess) e = link(cs, false, ev);
    if (e == hipSuccess && n_topo) {
        e = neat::launch_classify_batch(all_topo, n_topo, cs[0]);
        if (e != hipSuccess) return hip_fail(e, "batch class lists launch");
    }
    if (e == hipSuccess) e = link(cs, true, ev);
    for (size_t k = 0; e == hipSuccess && k < fw.size(); ++k) {
        e = neat::forward_launch(fw[k], tab[k], cs[k % N_BRANCH]);
        if (e != hipSuccess) return hip_fail(e, "batch forward launch");
    }
    if (e == hipSuccess) e = link(cs, false, ev);
    return e == hipSuccess ? NEAT_OK : hip_fail(e, "batch stream fork or join");
}

int build(const neat_batch_item *items, int32_t n, neat_batch_plan **out) {
    neat_batch_plan *p = new (std::nothrow) neat_batch_plan;
    if (!p) return fail(NEAT_E_NOMEM, "out of host memory");
    p->items.assign(items, items + n);
    (void)hipGetDevice(&p->device);

    std::vector<neat::FwdJob> jobs;
    // transformations bucketed by workgroup size
    static const int bucket_threads[] = {64, 128, 256, 512, 1024};
    std::vector<neat::TopoItem> bucket[5], all_topo;
    for (const neat_batch_item &it : p->items) {
        if (!it.nodes || it.dims.P == 0) continue;
        const neat_dims &d = it.dims;
        neat::TopoItem ti{it.nodes, it.conns, nullptr, nullptr, it.status, (int32_t *)it.program,
                          d.P, d.N_max, d.C_max, d.I, d.O, neat::prog_words(d.N_max, d.C_max, d.O),
                          0};
        int b = 0;
        while (bucket_threads[b] < neat::topo_block_threads(d.N_max)) ++b;
        bucket[b].push_back(ti);
        all_topo.push_back(ti);
    }
    std::vector<TopoLaunch> topo;
    std::vector<neat::TopoItem> topo_host;
    for (int b = 0; b < 5; ++b) {
        if (bucket[b].empty()) continue;
        TopoLaunch t{(int)bucket[b].size(), 0, 64, 0, nullptr};
        for (neat::TopoItem &ti : bucket[b]) {
            ti.block0 = t.blocks;
            t.blocks += ti.P;
            t.threads = std::max(t.threads, neat::topo_block_threads(ti.N));
            t.lds = std::max(t.lds, neat::topo_lds_bytes(ti.N, ti.C));
        }
        t.table = (const neat::TopoItem *)(uintptr_t)topo_host.size();  // offset for now
        topo_host.insert(topo_host.end(), bucket[b].begin(), bucket[b].end());
        topo.push_back(t);
    }
    const size_t all_off = topo_host.size();
    topo_host.insert(topo_host.end(), all_topo.begin(), all_topo.end());
    const int topo_launches = (int)topo.size() + (all_topo.empty() ? 0 : 1);
    std::vector<int> job_variant;
    for (const neat_batch_item &it : p->items) {
        if (it.dims.P == 0 || it.B == 0) continue;
        jobs.push_back(make_job(&it.dims, it.program, it.inputs, it.input_genome_stride, it.B,
                                it.outputs, it.grid_side, it.grid_first));
        job_variant.push_back(neat::tuned_variant(it.dims.N_max, it.dims.C_max, it.B));
    }
    // one plan per variant tuned for the items' buckets (all FWD_AUTO, one
    // plan, while nothing is tuned)
    std::vector<neat::FwdKernelLaunch> fw;
    char err[256] = "";
    int rc = NEAT_OK;
    for (int v = neat::FWD_AUTO; v <= neat::FWD_REG2 && rc == NEAT_OK; ++v) {
        std::vector<neat::FwdJob> group;
        for (size_t j = 0; j < jobs.size(); ++j)
            if (job_variant[j] == v) group.push_back(jobs[j]);
        if (group.empty()) continue;
        std::vector<neat::FwdKernelLaunch> part;
        rc = neat::forward_plan(group.data(), (int)group.size(), v, max_lds_bytes(), part, err,
                                sizeof(err));
        fw.insert(fw.end(), part.begin(), part.end());
    }
    if (rc != NEAT_OK) {
        destroy(p);
        return fail(rc, "%s", err);
    }

    // work-unit tables of the launches with more than one item
    size_t n_tab = 0;
    for (const neat::FwdKernelLaunch &k : fw)
        if (k.items.size() > 1) n_tab += k.items.size();
    std::vector<const neat::FwdItem *> tab(fw.size(), nullptr);
    if (n_tab) {
        hipError_t e = hipMalloc(&p->tables, n_tab * sizeof(neat::FwdItem));
        if (e != hipSuccess) {
            destroy(p);
            return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "batch tables: out of memory")
                                            : hip_fail(e, "batch tables");
        }
        std::vector<neat::FwdItem> host;
        host.reserve(n_tab);
        for (size_t k = 0; k < fw.size(); ++k) {
            if (fw[k].items.size() <= 1) continue;
            tab[k] = (const neat::FwdItem *)p->tables + host.size();
            host.insert(host.end(), fw[k].items.begin(), fw[k].items.end());
        }
        e = hipMemcpy(p->tables, host.data(), n_tab * sizeof(neat::FwdItem),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(p);
            return hip_fail(e, "batch tables upload");
        }
    }

    const neat::TopoItem *all_dev = nullptr;
    if (!topo_host.empty()) {
        hipError_t e = hipMalloc(&p->topo_tables, topo_host.size() * sizeof(neat::TopoItem));
        if (e == hipSuccess)
            e = hipMemcpy(p->topo_tables, topo_host.data(),
                          topo_host.size() * sizeof(neat::TopoItem), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(p);
            return e == hipErrorOutOfMemory ? fail(NEAT_E_NOMEM, "batch tables: out of memory")
                                            : hip_fail(e, "batch tables");
        }
        const neat::TopoItem *base = (const neat::TopoItem *)p->topo_tables;
        for (TopoLaunch &t : topo) t.table = base + (uintptr_t)t.table;
        all_dev = base + all_off;
    }

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
    rc = record(topo, all_dev, (int)all_topo.size(), fw, tab, cs, ev);
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
    p->launches = topo_launches + (int)fw.size();
    *out = p;
    return NEAT_OK;
}

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

int32_t neat_batch_plan_launches(const neat_batch_plan *plan) {
    return plan ? plan->launches : 0;
}

}  // extern "C"
