// launch.h -- host-side launchers of the kernels (internal to the library).
// Each returns a hipError_t from the launch; arguments are checked by the
// C-ABI layer before any launcher is called.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace neat {

// Dynamic LDS bytes the transformation kernel needs for one genome.
size_t topo_lds_bytes(int N, int C);
// Threads per block of the transformation kernel (one thread per node row).
int topo_block_threads(int N);

hipError_t launch_topo(int P, int N, int C, int I, int O, const float *nodes,
                       const float *conns, int32_t *order, int32_t *level,
                       uint32_t *status, int32_t *prog, hipStream_t stream,
                       int recurrent = 0);

// One population of a transformation launch; workgroups block0 ..
// block0 + P - 1 of a batched launch transform its genomes.  recurrent:
// cycles allowed, nodes in key order, one value slot per node.
struct TopoItem {
    const float *nodes;
    const float *conns;
    int32_t *order;
    int32_t *level;
    uint32_t *status;
    int32_t *prog;
    int P, N, C, I, O, prog_words;
    long long block0;
    int recurrent;
};

// Transformation of many populations in one launch (items in device memory,
// sorted by block0; threads >= topo_block_threads and lds >= topo_lds_bytes
// of every item), and the class lists of all of them (one workgroup each).
hipError_t launch_topo_batch(const TopoItem *dev_items, int n, long long blocks, int threads,
                             size_t lds, hipStream_t stream);
hipError_t launch_classify_batch(const TopoItem *dev_items, int n, hipStream_t stream);

// Forward variants (value stores of the lane-per-sample mapping).
constexpr int FWD_AUTO = 0;  // per slot class: registers, R64 with two samples per lane when B > 64
constexpr int FWD_REG = 1;   // registers, one sample per lane (LDS rows for the LDS class)
constexpr int FWD_LDS = 2;   // every genome in LDS rows
constexpr int FWD_REG2 = 3;  // as FWD_REG, R64 genomes two samples per lane
constexpr int FWD_LVL = 5;   // lanes over a level's nodes x a tile of samples (values in LDS)
constexpr int FWD_SEG = 6;   // lanes over a level's in-edges x a tile, segmented reduction

// Forward kernels, one per value store.
// KIND_R64REC: the recurrent calculation (K synchronous sweeps) with the
// 64-slot register store, for populations of N_max <= 62.  KIND_LDS32: the
// LDS-row store with half-wave tiles (32 samples), for genomes whose rows
// do not fit in LDS with 64 columns.
// KIND_LVL / KIND_SEG: the level and segment mappings (FWD_LVL, FWD_SEG),
// every genome of an item, tiles of 2^lvl_sh samples.
enum FwdKind {
    KIND_R64 = 0, KIND_R64X2, KIND_R128, KIND_R224, KIND_LDS, KIND_R64REC, KIND_LDS32, KIND_LVL,
    KIND_SEG, N_KINDS
};
constexpr int FWD_MAX_WAVES = 4;  // waves per workgroup

// One population of a forward call.
struct FwdJob {
    const int32_t *prog;  // programs of neat_topo_sort (+ population area)
    const float *inputs;  // [P or 1][B][I] with gstride floats between genomes
    float *outputs;       // [P][B][O]
    int64_t gstride;
    int64_t first;        // grid mode: first query
    int P, N, C, I, O, B;
    int side;             // > 0: grid mode (CPPN queries generated in the kernel)
    int recurrent;        // 1: a recurrent program, sweeps synchronous sweeps
    int sweeps;
    int variant = -1;     // FWD_*: this job's variant; -1: the plan's
};

// One population in one forward kernel (device-visible, read with scalar
// loads): the genomes of class cls (or all when cls < 0), P x chunks wave
// units starting at unit0 (unit (i, c): tiles c tpw .. c tpw + tpw - 1 of
// the i-th genome).
struct FwdItem {
    const int32_t *prog;
    const float *inputs;
    float *outputs;
    const int32_t *pop;  // population area (class lists)
    long long gstride, first, unit0;
    int P, N, I, O, B, side, vec4, cls;
    int tiles, tpw, chunks, prog_words;
    int sweeps;  // recurrent kernel: sweeps per sample
    int C;         // C_max (program layout)
    int lvl_sh;    // level and segment mappings: log2 of the samples per tile
    int lvl_rows;  // segment mapping: value rows before the edge offsets
};

// Kernel argument: one item inline, or a device table of items.
struct FwdLaunch {
    FwdItem one;
    const FwdItem *items;  // nullptr: the inline item
    long long units;   // wave units over all items
    int n_items;
    int wave_floats;   // LDS floats per wave: input staging, then value rows (LDS
                       // store) or the output staging (register stores)
    int stage_floats;
    int persistent;    // workgroups loop over units
    unsigned *counter; // persistent launches: next unit, taken by each wave in turn
                       // (device memory zeroed before the launch); nullptr: units
                       // dealt to workgroups round robin
};

struct FwdKernelLaunch {
    int kind;
    int grid_mode;  // items generate CPPN grid queries
    unsigned grid, block;
    size_t lds;
    FwdLaunch args;
    std::vector<FwdItem> items;
};

const char *kind_name(int kind);

// Plan the kernels of a forward over n populations: one launch per kernel
// kind in use, each covering its genomes of every population (jobs with
// their own variant join the same launches as the others of their kind).  Returns
// NEAT_OK or an error code with a message in err.
int forward_plan(const FwdJob *jobs, int n, int variant, size_t max_lds,
                 std::vector<FwdKernelLaunch> &out, char *err, size_t errlen);
// Launch one planned kernel.  dev_items: the launch's items in device memory
// (may be nullptr when the launch has a single item, passed inline).
hipError_t forward_launch(const FwdKernelLaunch &k, const FwdItem *dev_items, hipStream_t stream,
                          unsigned *counter = nullptr);
// Zero n unit counters (a kernel, so it can be recorded into a graph).
hipError_t launch_zero_counters(unsigned *c, int n, hipStream_t stream);

// Recurrent calculation: K synchronous sweeps, one wave per (genome, tile),
// rows = class_slots(max_class(N), N) LDS rows per value column; tiles of
// 64 samples, or 32 when recurrent_lds_bytes(N, I, 64) exceeds max_lds
// (recurrent_launch sets tiles and stage_floats).
struct RecLaunch {
    const int32_t *prog;
    const float *inputs;
    float *outputs;
    long long gstride;
    int prog_words, P, N, I, O, B, K, tiles, rows, stage_floats, vec4;
};
size_t recurrent_lds_bytes(int N, int I, int tile_samples);
hipError_t recurrent_launch(RecLaunch L, size_t max_lds, hipStream_t stream);

// HyperNEAT substrate layer: Y[g] = tanh(X W'[g]), W' = W with |w| < theta
// set to 0.  W [P][S][S], X [B][S], Y [P][B][S]; S a multiple of 64; X, W
// and the rows 16-byte aligned.
struct SubLaunch {
    const float *W;
    const float *X;
    float *Y;
    float theta;
    int P, S, B;
};
hipError_t substrate_launch(const SubLaunch &L, hipStream_t stream);

}  // namespace neat
