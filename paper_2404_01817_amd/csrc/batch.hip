// batch.hip -- the batched path: many populations in one call, recorded
// once into a HIP graph and replayed.
//
// The calculation of all items is planned together (forward_plan): one
// launch per value-store kernel whose work units span every population, so
// a batch of uneven populations costs a handful of launches rather than one
// (or four) per population, and small populations fill the GPU together.
// The work-unit tables of those launches live in device memory owned by the
// plan.  Transformations (items with nodes) are recorded before the
// calculations, one launch (plus the class listing) per population.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "abi.h"
#include "launch.h"
#include "neat.h"
#include "program.h"

using namespace neat::abi;

struct neat_batch_plan {
    std::vector<neat_batch_item> items;
    int device = -1;
    void *tables = nullptr;  // FwdItem tables of the multi-item launches
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

// Record every launch of the batch on stream s.
int record(const neat_batch_plan *p, const std::vector<neat::FwdKernelLaunch> &fw,
           const std::vector<const neat::FwdItem *> &tab, hipStream_t s) {
    for (const neat_batch_item &it : p->items) {
        if (!it.nodes || it.dims.P == 0) continue;
        const neat_dims &d = it.dims;
        hipError_t e = neat::launch_topo(d.P, d.N_max, d.C_max, d.I, d.O, it.nodes, it.conns,
                                         nullptr, nullptr, it.status, (int32_t *)it.program, s);
        if (e != hipSuccess) return hip_fail(e, "batch transformation launch");
    }
    for (size_t k = 0; k < fw.size(); ++k) {
        hipError_t e = neat::forward_launch(fw[k], tab[k], s);
        if (e != hipSuccess) return hip_fail(e, "batch forward launch");
    }
    return NEAT_OK;
}

int build(const neat_batch_item *items, int32_t n, neat_batch_plan **out) {
    neat_batch_plan *p = new (std::nothrow) neat_batch_plan;
    if (!p) return fail(NEAT_E_NOMEM, "out of host memory");
    p->items.assign(items, items + n);
    (void)hipGetDevice(&p->device);

    std::vector<neat::FwdJob> jobs;
    int topo_launches = 0;
    for (const neat_batch_item &it : p->items) {
        if (it.nodes && it.dims.P > 0)
            topo_launches += 1 + (neat::max_class(it.dims.N_max) != 0 ? 1 : 0);
        if (it.dims.P == 0 || it.B == 0) continue;
        jobs.push_back(make_job(&it.dims, it.program, it.inputs, it.input_genome_stride, it.B,
                                it.outputs, it.grid_side, it.grid_first));
    }
    std::vector<neat::FwdKernelLaunch> fw;
    char err[256] = "";
    int rc = neat::forward_plan(jobs.data(), (int)jobs.size(), neat::FWD_AUTO, max_lds_bytes(),
                                fw, err, sizeof(err));
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

    // record the launches into a graph on a private stream
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy(p);
        return hip_fail(e, "capture stream");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        destroy(p);
        return hip_fail(e, "begin capture");
    }
    rc = record(p, fw, tab, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
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
