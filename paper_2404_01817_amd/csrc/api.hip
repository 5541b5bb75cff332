// api.hip -- the C ABI declared in include/neat.h: argument checks, error
// reporting and kernel launches for the transformation and calculation
// stages.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "abi.h"
#include "genes.h"
#include "launch.h"
#include "tune.h"
#include "neat.h"
#include "program.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace neat {
namespace abi {

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(NEAT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Largest dynamic LDS allocation of one workgroup on the current device.
size_t max_lds_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
        return 65536;
    return (size_t)v;
}

int check_dims(const neat_dims *d) {
    if (!d) return fail(NEAT_E_INVALID, "dims is NULL");
    if (d->P < 0) return fail(NEAT_E_INVALID, "P = %d < 0", d->P);
    if (d->N_max < 1 || d->N_max > NEAT_MAX_NODES)
        return fail(NEAT_E_INVALID, "N_max = %d outside [1, %d]", d->N_max, NEAT_MAX_NODES);
    if (d->C_max < 0 || d->C_max > NEAT_MAX_CONNS)
        return fail(NEAT_E_INVALID, "C_max = %d outside [0, %d]", d->C_max, NEAT_MAX_CONNS);
    if (d->I < 1 || d->O < 1 || d->I + d->O > d->N_max)
        return fail(NEAT_E_INVALID, "need I >= 1, O >= 1, I + O <= N_max (I=%d O=%d N_max=%d)",
                    d->I, d->O, d->N_max);
    return NEAT_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_topo_args(const neat_dims *d, const float *nodes, const float *conns,
                    const void *program) {
    if (d->P > 0 && !nodes) return fail(NEAT_E_INVALID, "nodes is NULL");
    if (d->P > 0 && d->C_max > 0 && !conns) return fail(NEAT_E_INVALID, "conns is NULL");
    if (conns && !aligned(conns, 16)) return fail(NEAT_E_INVALID, "conns must be 16-byte aligned");
    if (program && !aligned(program, 16))
        return fail(NEAT_E_INVALID, "program must be 16-byte aligned");
    const size_t lds = topo_lds_bytes(d->N_max, d->C_max);
    if (lds > max_lds_bytes())
        return fail(NEAT_E_INVALID,
                    "N_max=%d, C_max=%d needs %zu B of LDS per genome, device allows %zu",
                    d->N_max, d->C_max, lds, max_lds_bytes());
    return NEAT_OK;
}

int check_forward_args(const neat_dims *d, const void *program, const float *inputs,
                       int64_t stride, int32_t B, float *outputs, bool grid, int32_t side,
                       int64_t first) {
    if (B < 0) return fail(NEAT_E_INVALID, "B = %d < 0", B);
    if (grid) {
        if (d->I != 5) return fail(NEAT_E_INVALID, "grid queries need I = 5, got %d", d->I);
        if (side < 2 || side > 256)
            return fail(NEAT_E_INVALID, "side = %d outside [2, 256]", side);
        const long long nq = (long long)side * side * side * side;
        if (first < 0 || first + B > nq)
            return fail(NEAT_E_INVALID, "queries [%lld, %lld) outside [0, %lld)",
                        (long long)first, (long long)first + B, nq);
    } else {
        if (stride < 0) return fail(NEAT_E_INVALID, "negative input_genome_stride");
        if (stride != 0 && stride < (int64_t)B * d->I)
            return fail(NEAT_E_INVALID, "input_genome_stride %lld < B * I = %lld",
                        (long long)stride, (long long)B * d->I);
    }
    if (d->P == 0 || B == 0) return NEAT_OK;
    if (!program || !outputs || (!grid && !inputs))
        return fail(NEAT_E_INVALID, "program, inputs or outputs is NULL");
    if (!aligned(program, 16)) return fail(NEAT_E_INVALID, "program must be 16-byte aligned");
    const long long tiles = (long long)d->P * ((B + 63) / 64);
    if (tiles >= (1ll << 31))
        return fail(NEAT_E_INVALID, "P * B too large for one launch (%lld tiles)", tiles);
    return NEAT_OK;
}

FwdJob make_job(const neat_dims *d, const void *program, const float *inputs, int64_t stride,
                int32_t B, float *outputs, int32_t side, int64_t first) {
    FwdJob job{};
    job.prog = (const int32_t *)program;
    job.inputs = inputs;
    job.outputs = outputs;
    job.gstride = stride;
    job.first = first;
    job.P = d->P, job.N = d->N_max, job.C = d->C_max, job.I = d->I, job.O = d->O, job.B = B;
    job.side = side;
    return job;
}

}  // namespace abi
}  // namespace neat

using namespace neat::abi;

// ---- autotuner: the fastest variant per (N_max, C_max, B, mode) bucket ---
// The table lives in process memory; with NEAT_TUNE_CACHE set (or a server
// created with a tune_cache_path) it is also read from and written to that
// text file, one "N_max C_max B grid variant" line per bucket (bucket
// values, powers of two), so tuning carries over between processes.
namespace {
std::mutex g_tune_mu;
// per bucket: the variant fastest alone (single calls) and the one with the
// most genome-inputs per second when the GPU is full (batches)
std::map<unsigned long long, int> g_tune, g_tune_tp;
std::string g_tune_path;
bool g_tune_env_read = false;
unsigned g_tune_gen = 0;

long long pow2_ceil(long long x) {
    long long p = 1;
    while (p < x) p <<= 1;
    return p;
}
unsigned long long tune_key(int N, int C, int B, int grid) {
    return ((unsigned long long)(grid ? 1 : 0) << 63) |
           ((unsigned long long)pow2_ceil(N) << 42) | ((unsigned long long)pow2_ceil(C) << 21) |
           (unsigned long long)std::min(pow2_ceil(B), 1024ll);
}
bool valid_tuned(int v) {
    return v == NEAT_FWD_AUTO || v == NEAT_FWD_REG || v == NEAT_FWD_LDS || v == NEAT_FWD_REG2 ||
           v == NEAT_FWD_LVL || v == NEAT_FWD_SEG;
}

// Merge the cache file's entries into the table (caller holds the lock).
void tune_read_locked(const std::string &path) {
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    long long N, C, B;
    int grid, v, vt;
    while (fscanf(f, "%lld %lld %lld %d %d %d", &N, &C, &B, &grid, &v, &vt) == 6)
        if (N > 0 && C >= 0 && B > 0 && valid_tuned(v) && valid_tuned(vt)) {
            g_tune[tune_key((int)N, (int)C, (int)B, grid)] = v;
            g_tune_tp[tune_key((int)N, (int)C, (int)B, grid)] = vt;
        }
    fclose(f);
    ++g_tune_gen;
}

void tune_env_locked() {
    if (g_tune_env_read) return;
    g_tune_env_read = true;
    const char *e = getenv("NEAT_TUNE_CACHE");
    if (e && *e) {
        g_tune_path = e;
        tune_read_locked(g_tune_path);
    }
}

// Rewrite the cache file from the table (caller holds the lock); a file
// that cannot be written leaves the in-memory table as it is.
void tune_write_locked() {
    if (g_tune_path.empty()) return;
    const std::string tmp = g_tune_path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : g_tune) {
        const unsigned long long k = kv.first;
        const auto tp = g_tune_tp.find(k);
        fprintf(f, "%llu %llu %llu %d %d %d\n", (k >> 42) & ((1ull << 21) - 1),
                (k >> 21) & ((1ull << 21) - 1), k & ((1ull << 21) - 1), (int)(k >> 63),
                kv.second, tp == g_tune_tp.end() ? kv.second : tp->second);
    }
    if (fclose(f) == 0) rename(tmp.c_str(), g_tune_path.c_str());
}
}  // namespace

namespace neat {
int tuned_variant(int N, int C, int B, int grid, int throughput) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_env_locked();
    const std::map<unsigned long long, int> &t = throughput ? g_tune_tp : g_tune;
    const auto it = t.find(tune_key(N, C, B, grid));
    return it == t.end() ? FWD_AUTO : it->second;
}
unsigned tune_generation() {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_env_locked();
    return g_tune_gen;
}
int tune_cache_use(const char *path) {
    if (!path || !*path) return NEAT_OK;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_env_locked();
    g_tune_path = path;
    tune_read_locked(g_tune_path);
    return NEAT_OK;
}
}  // namespace neat

extern "C" {

const char *neat_last_error(void) { return g_last_error.c_str(); }

const char *neat_strerror(int code) {
    switch (code) {
    case NEAT_OK: return "ok";
    case NEAT_PENDING: return "pending";
    case NEAT_E_INVALID: return "invalid argument";
    case NEAT_E_HIP: return "HIP runtime error";
    case NEAT_E_NOMEM: return "out of device memory";
    case NEAT_E_TOO_LARGE: return "request larger than the admission cap";
    case NEAT_E_UNKNOWN_TICKET: return "unknown ticket";
    case NEAT_E_SHUTDOWN: return "server shut down";
    }
    return "unknown code";
}

size_t neat_program_bytes(const neat_dims *d) {
    if (check_dims(d) != NEAT_OK) return 0;
    return (size_t)(neat::pop_off(d->P, d->N_max, d->C_max, d->O) + neat::pop_words(d->P)) *
           sizeof(int32_t);
}

size_t neat_program_stride(const neat_dims *d) {
    if (check_dims(d) != NEAT_OK) return 0;
    return (size_t)neat::prog_words(d->N_max, d->C_max, d->O) * sizeof(int32_t);
}

int neat_topo_sort(const neat_dims *d, const float *nodes, const float *conns, int32_t *order,
                   int32_t *level, uint32_t *status, void *program, void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (d->P == 0) return NEAT_OK;
    rc = check_topo_args(d, nodes, conns, program);
    if (rc != NEAT_OK) return rc;
    hipError_t e = neat::launch_topo(d->P, d->N_max, d->C_max, d->I, d->O, nodes, conns, order,
                                     level, status, (int32_t *)program, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "topo_sort launch");
    return NEAT_OK;
}

static int forward_common(const neat_dims *d, const void *program, const float *inputs,
                          int64_t stride, int32_t B, float *outputs, int variant, bool grid,
                          int32_t side, int64_t first, void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (variant < NEAT_FWD_AUTO || variant > NEAT_FWD_SEG)
        return fail(NEAT_E_INVALID, "unknown forward variant %d", variant);
    if (variant == NEAT_FWD_TUNED)
        variant = neat::tuned_variant(d->N_max, d->C_max, B, grid, 0);
    rc = check_forward_args(d, program, inputs, stride, B, outputs, grid, side, first);
    if (rc != NEAT_OK || d->P == 0 || B == 0) return rc;
    const neat::FwdJob job =
        make_job(d, program, inputs, stride, B, outputs, grid ? side : 0, first);
    std::vector<neat::FwdKernelLaunch> plan;
    char err[256] = "";
    rc = neat::forward_plan(&job, 1, variant, max_lds_bytes(), plan, err, sizeof(err));
    if (rc != NEAT_OK) return fail(rc, "%s", err);
    for (const neat::FwdKernelLaunch &k : plan) {
        hipError_t e = neat::forward_launch(k, nullptr, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "forward launch");
    }
    return NEAT_OK;
}

int neat_forward_ex(const neat_dims *d, const void *program, const float *inputs,
                    int64_t input_genome_stride, int32_t B, float *outputs, int32_t variant,
                    void *stream) {
    return forward_common(d, program, inputs, input_genome_stride, B, outputs, variant, false, 0,
                          0, stream);
}

int neat_forward(const neat_dims *d, const void *program, const float *inputs,
                 int64_t input_genome_stride, int32_t B, float *outputs, void *stream) {
    return neat_forward_ex(d, program, inputs, input_genome_stride, B, outputs, NEAT_FWD_AUTO,
                           stream);
}

// Launch `copies` copies of one population's calculation under one variant
// in a single plan (copies > 1 share a device table of items; every copy
// writes the same outputs with the same values).
static int launch_copies(const neat::FwdJob &job, int copies, int variant,
                         std::vector<void *> &tables, hipStream_t s) {
    std::vector<neat::FwdJob> jobs(copies, job);
    std::vector<neat::FwdKernelLaunch> plan;
    char err[256] = "";
    int rc = neat::forward_plan(jobs.data(), copies, variant, max_lds_bytes(), plan, err,
                                sizeof(err));
    if (rc != NEAT_OK) return fail(rc, "%s", err);
    for (const neat::FwdKernelLaunch &k : plan) {
        const neat::FwdItem *dev = nullptr;
        if (k.items.size() > 1) {
            void *t = nullptr;
            hipError_t e = hipMalloc(&t, k.items.size() * sizeof(neat::FwdItem));
            if (e == hipSuccess) {
                tables.push_back(t);
                e = hipMemcpy(t, k.items.data(), k.items.size() * sizeof(neat::FwdItem),
                              hipMemcpyHostToDevice);
            }
            if (e != hipSuccess) return hip_fail(e, "autotune item table");
            dev = (const neat::FwdItem *)t;
        }
        hipError_t e = neat::forward_launch(k, dev, s);
        if (e != hipSuccess) return hip_fail(e, "autotune launch");
    }
    return NEAT_OK;
}

// Mean ms per launch of `reps` launches of `copies` copies (after one
// warm-up), timed with events on s.
static int time_copies(const neat::FwdJob &job, int copies, int variant, int reps,
                       hipEvent_t e0, hipEvent_t e1, hipStream_t s, float *ms) {
    std::vector<void *> tables;
    int rc = launch_copies(job, copies, variant, tables, s);  // warm-up
    hipError_t e = hipSuccess;
    if (rc == NEAT_OK) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && rc == NEAT_OK && e == hipSuccess; ++r)
        rc = launch_copies(job, copies, variant, tables, s);
    if (rc == NEAT_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (rc == NEAT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (rc == NEAT_OK && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (rc == NEAT_OK && e != hipSuccess) rc = hip_fail(e, "autotune timing");
    (void)hipStreamSynchronize(s);
    for (void *t2 : tables) (void)hipFree(t2);
    *ms = t / (float)reps;
    return rc;
}

int neat_autotune_forward(const neat_dims *d, const void *program, const float *inputs,
                          int64_t input_genome_stride, int32_t B, float *outputs, int32_t reps,
                          int32_t *variant_out, float *ms_out, void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (!variant_out) return fail(NEAT_E_INVALID, "variant_out is NULL");
    if (reps < 1 || reps > 1000) return fail(NEAT_E_INVALID, "reps = %d outside [1, 1000]", reps);
    rc = check_forward_args(d, program, inputs, input_genome_stride, B, outputs, false, 0, 0);
    if (rc != NEAT_OK) return rc;
    constexpr int NC = NEAT_TUNE_CANDIDATES;
    const int cand[NC] = {NEAT_FWD_REG, NEAT_FWD_REG2, NEAT_FWD_LDS, NEAT_FWD_LVL,
                          NEAT_FWD_SEG};
    float ms[2 * NC];
    for (float &m : ms) m = -1.0f;
    int best = NEAT_FWD_AUTO, best_tp = NEAT_FWD_AUTO;
    if (d->P > 0 && B > 0) {
        // copies of the population that fill the GPU (about 16 waves per CU
        // of lane-per-sample tiles), for the throughput timing
        const long long waves = (long long)d->P * ((B + 63) / 64);
        const int copies = (int)std::max(1ll, std::min(64ll, (16384 + waves - 1) / waves));
        const neat::FwdJob job =
            make_job(d, program, inputs, input_genome_stride, B, outputs, 0, 0);
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return hip_fail(hipGetLastError(), "event");
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return hip_fail(hipGetLastError(), "event");
        }
        const hipStream_t s = (hipStream_t)stream;
        float best_ms = 0.0f, best_tp_ms = 0.0f;
        for (int i = 0; i < NC && rc == NEAT_OK; ++i) {
            rc = time_copies(job, 1, cand[i], reps, e0, e1, s, &ms[i]);
            if (rc == NEAT_OK) rc = time_copies(job, copies, cand[i], reps, e0, e1, s, &ms[NC + i]);
            if (rc != NEAT_OK) break;
            ms[NC + i] /= (float)copies;
            if (best == NEAT_FWD_AUTO || ms[i] < best_ms) best = cand[i], best_ms = ms[i];
            if (best_tp == NEAT_FWD_AUTO || ms[NC + i] < best_tp_ms)
                best_tp = cand[i], best_tp_ms = ms[NC + i];
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != NEAT_OK) return rc;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_env_locked();
        const unsigned long long key = tune_key(d->N_max, d->C_max, B, 0);
        int &slot = g_tune[key];
        int &slot_tp = g_tune_tp[key];
        if (slot != best || slot_tp != best_tp) ++g_tune_gen;
        slot = best;
        slot_tp = best_tp;
        tune_write_locked();
    }
    // the outputs end with the recorded latency winner's result
    if (d->P > 0 && B > 0) {
        rc = forward_common(d, program, inputs, input_genome_stride, B, outputs, best, false, 0, 0,
                            stream);
        if (rc != NEAT_OK) return rc;
    }
    *variant_out = best;
    if (ms_out)
        for (int i = 0; i < 2 * NC; ++i) ms_out[i] = ms[i];
    return NEAT_OK;
}

void neat_tune_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    g_tune_tp.clear();
    g_tune_path.clear();
    g_tune_env_read = true;  // NEAT_TUNE_CACHE is not read again
    ++g_tune_gen;
}

int32_t neat_tuned_variant(const neat_dims *d, int32_t B, int32_t grid, int32_t throughput) {
    if (check_dims(d) != NEAT_OK || B < 0) return NEAT_E_INVALID;
    return neat::tuned_variant(d->N_max, d->C_max, B, grid != 0, throughput != 0);
}

int neat_topo_sort_recurrent(const neat_dims *d, const float *nodes, const float *conns,
                             int32_t *order, int32_t *level, uint32_t *status, void *program,
                             void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (d->P == 0) return NEAT_OK;
    rc = check_topo_args(d, nodes, conns, program);
    if (rc != NEAT_OK) return rc;
    hipError_t e = neat::launch_topo(d->P, d->N_max, d->C_max, d->I, d->O, nodes, conns, order,
                                     level, status, (int32_t *)program, (hipStream_t)stream, 1);
    if (e != hipSuccess) return hip_fail(e, "topo_sort_recurrent launch");
    return NEAT_OK;
}

int neat_forward_recurrent(const neat_dims *d, const void *program, const float *inputs,
                           int64_t input_genome_stride, int32_t B, int32_t K, float *outputs,
                           void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (K < 0 || K > NEAT_MAX_SWEEPS)
        return fail(NEAT_E_INVALID, "K = %d outside [0, %d]", K, NEAT_MAX_SWEEPS);
    rc = check_forward_args(d, program, inputs, input_genome_stride, B, outputs, false, 0, 0);
    if (rc != NEAT_OK || d->P == 0 || B == 0) return rc;
    if (neat::max_class(d->N_max) == neat::CLS_R64) {
        // every genome fits the 64-slot register store
        neat::FwdJob job = make_job(d, program, inputs, input_genome_stride, B, outputs, 0, 0);
        job.recurrent = 1;
        job.sweeps = K;
        std::vector<neat::FwdKernelLaunch> plan;
        char err[256] = "";
        rc = neat::forward_plan(&job, 1, NEAT_FWD_AUTO, max_lds_bytes(), plan, err, sizeof(err));
        if (rc != NEAT_OK) return fail(rc, "%s", err);
        for (const neat::FwdKernelLaunch &k : plan) {
            hipError_t e = neat::forward_launch(k, nullptr, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "forward_recurrent launch");
        }
        return NEAT_OK;
    }
    const size_t lds = neat::recurrent_lds_bytes(d->N_max, d->I, 32);
    if (lds > max_lds_bytes())
        return fail(NEAT_E_TOO_LARGE,
                    "recurrent forward with N_max=%d, I=%d needs %zu B of LDS per wave, device "
                    "allows %zu",
                    d->N_max, d->I, lds, max_lds_bytes());
    neat::RecLaunch L{};
    L.prog = (const int32_t *)program;
    L.inputs = inputs;
    L.outputs = outputs;
    L.gstride = input_genome_stride;
    L.prog_words = neat::prog_words(d->N_max, d->C_max, d->O);
    L.P = d->P, L.N = d->N_max, L.I = d->I, L.O = d->O, L.B = B, L.K = K;
    L.rows = neat::class_slots(neat::max_class(d->N_max), d->N_max);
    L.vec4 = (aligned(inputs, 16) && input_genome_stride % 4 == 0) ? 1 : 0;
    hipError_t e = neat::recurrent_launch(L, max_lds_bytes(), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "forward_recurrent launch");
    return NEAT_OK;
}

int neat_distance(const neat_dims *d, const float *nodes, const float *conns, int32_t Q,
                  const float *rnodes, const float *rconns, float c_disjoint,
                  float c_homologous, float *out, void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (Q < 0) return fail(NEAT_E_INVALID, "Q = %d < 0", Q);
    if (d->P == 0 || Q == 0) return NEAT_OK;
    if (!nodes || !rnodes || !out || (d->C_max > 0 && (!conns || !rconns)))
        return fail(NEAT_E_INVALID, "nodes, conns, rnodes, rconns or out is NULL");
    const size_t lds = neat::distance_lds_bytes(d->N_max, d->C_max);
    if (lds > max_lds_bytes())
        return fail(NEAT_E_TOO_LARGE,
                    "distance with N_max=%d, C_max=%d needs %zu B of LDS, device allows %zu",
                    d->N_max, d->C_max, lds, max_lds_bytes());
    neat::DistLaunch L{};
    L.nodes = nodes, L.conns = conns, L.rnodes = rnodes, L.rconns = rconns, L.out = out;
    L.P = d->P, L.Q = Q, L.N = d->N_max, L.C = d->C_max;
    L.cd = c_disjoint, L.ch = c_homologous;
    hipError_t e = neat::distance_launch(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "distance launch");
    return NEAT_OK;
}

int neat_apply_edits(const neat_dims *d, float *nodes, float *conns, const neat_edit *edits,
                     int32_t n, int32_t *applied, void *stream) {
    static_assert(sizeof(neat_edit) == sizeof(neat::EditRec), "edit record layout");
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (n < 0) return fail(NEAT_E_INVALID, "n = %d < 0", n);
    if (n == 0) return NEAT_OK;
    if (!edits || !applied || (d->P > 0 && (!nodes || (d->C_max > 0 && !conns))))
        return fail(NEAT_E_INVALID, "a pointer argument is NULL");
    neat::EditLaunch L{};
    L.nodes = nodes, L.conns = conns, L.edits = (const neat::EditRec *)edits;
    L.applied = applied, L.n = n, L.P = d->P, L.N = d->N_max, L.C = d->C_max;
    hipError_t e = neat::edit_launch(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "edit launch");
    return NEAT_OK;
}

int neat_crossover(const neat_dims *d, const float *nodes, const float *conns, int32_t Pc,
                   const int32_t *pairs, const float *rn, const float *rc, float *child_nodes,
                   float *child_conns, void *stream) {
    int rc_ = check_dims(d);
    if (rc_ != NEAT_OK) return rc_;
    if (Pc < 0) return fail(NEAT_E_INVALID, "Pc = %d < 0", Pc);
    if (Pc == 0) return NEAT_OK;
    if (d->P == 0) return fail(NEAT_E_INVALID, "crossover needs parents (P = 0)");
    if (!nodes || !pairs || !rn || !child_nodes ||
        (d->C_max > 0 && (!conns || !rc || !child_conns)))
        return fail(NEAT_E_INVALID, "a pointer argument is NULL");
    if (child_conns && !aligned(child_conns, 16))
        return fail(NEAT_E_INVALID, "child_conns must be 16-byte aligned");
    const size_t lds = neat::gene_tables_lds_bytes(d->N_max, d->C_max);
    if (lds > max_lds_bytes())
        return fail(NEAT_E_TOO_LARGE,
                    "crossover with N_max=%d, C_max=%d needs %zu B of LDS, device allows %zu",
                    d->N_max, d->C_max, lds, max_lds_bytes());
    neat::CrossLaunch L{};
    L.nodes = nodes, L.conns = conns, L.pairs = pairs, L.rn = rn, L.rc = rc;
    L.cn = child_nodes, L.cc = child_conns;
    L.Pc = Pc, L.P = d->P, L.N = d->N_max, L.C = d->C_max;
    hipError_t e = neat::crossover_launch(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "crossover launch");
    return NEAT_OK;
}

int neat_substrate_forward(const neat_dims *d, const void *program, int32_t side,
                           float threshold, const float *x, int32_t B, float *weights,
                           float *outputs, void *stream) {
    int rc = check_dims(d);
    if (rc != NEAT_OK) return rc;
    if (d->I != 5 || d->O != 1)
        return fail(NEAT_E_INVALID, "substrate CPPNs need I = 5, O = 1 (got I=%d O=%d)", d->I,
                    d->O);
    if (side < 8 || side > 32 || (side * side) % 64 != 0)
        return fail(NEAT_E_INVALID, "substrate side %d: need 8 <= side <= 32, side^2 a multiple "
                                    "of 64", side);
    if (B < 0) return fail(NEAT_E_INVALID, "B = %d < 0", B);
    if (!(threshold >= 0.0f)) return fail(NEAT_E_INVALID, "threshold must be >= 0");
    if (d->P == 0) return NEAT_OK;
    if (!program || !weights || (B > 0 && (!x || !outputs)))
        return fail(NEAT_E_INVALID, "program, x, weights or outputs is NULL");
    if (!aligned(weights, 16) || (B > 0 && (!aligned(x, 16) || !aligned(outputs, 16))))
        return fail(NEAT_E_INVALID, "x, weights and outputs must be 16-byte aligned");
    const int S = side * side;
    if ((long long)d->P * ((B + 63) / 64) * (S / 64) >= (1ll << 31))
        return fail(NEAT_E_INVALID, "P * B too large for one launch");
    // the weights: the CPPN on all S x S pairs of the grid
    rc = neat_forward_grid(d, program, side, 0, S * S, weights, stream);
    if (rc != NEAT_OK || B == 0) return rc;
    neat::SubLaunch L{weights, x, outputs, threshold, d->P, S, B};
    hipError_t e = neat::substrate_launch(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "substrate launch");
    return NEAT_OK;
}

int neat_forward_grid(const neat_dims *d, const void *program, int32_t side, int64_t first,
                      int32_t Q, float *outputs, void *stream) {
    return forward_common(d, program, nullptr, 0, Q, outputs, NEAT_FWD_AUTO, true, side, first,
                          stream);
}

}  // extern "C"
