// program.h -- layout of the per-genome program that the transformation
// kernel writes and the calculation kernels read.
//
// The program replaces the paper's dense expanded-connection tensor C_exp
// (|N|max x |N|max cells, Section 3.3) by a compressed form in topological
// order.  Nodes are numbered by their position p in the (level, key) order,
// so the inputs, which have level 0 and the smallest keys, take positions
// 0..I-1, and every computed node p >= I has one record.
//
// Each position is stored in a value SLOT of the forward kernels' value
// vector.  For N_max <= 62 the slot is the position.  Otherwise slots are
// reused: the program build walks the positions in order
// and gives each value a free slot (a value's slot is freed after its last
// reader, so the reader's own result may take it), which keeps the number
// of slots at the largest number of simultaneously live values.  Inputs
// hold slots 0..I-1; outputs are never freed.  That number decides the
// genome's SLOT CLASS and where the two constant slots (0 and 1) sit:
//   R64   <= 62 values: 64 register slots, constants at 62 and 63;
//   R128  <= 126 values: 128 register slots, constants at 126 and 127;
//   R224  <= 222 values: 224 register slots, constants at 222 and 223;
//   LDS   otherwise: N_max + 2 LDS rows, constants at N_max and N_max + 1.
// A node's incoming edges are stored as (source slot, weight) in ascending
// source-key order, padded to an even count with one neutral edge, so the
// kernels consume edges in pairs without per-edge tests: for sum and mean a
// term 1 * v[zero slot], for product 1 * v[one slot], for max and min a copy
// of the node's first edge.  None of these changes any result.  The first
// three pairs live in the node's record (one scalar load brings a node and
// its usual in-edges); further pairs follow in the overflow edge array, node
// after node.
//
// After the P genome programs, a population area lists the genomes by slot
// class (written by the classification step for N_max > 62 only; smaller
// populations are all R64).
//
// All fields are 32-bit words; one genome's program is prog_words() words,
// a multiple of 64 (256 bytes), so every genome starts on its own lines.
#pragma once

#include <cstddef>
#include <cstdint>

namespace neat {

// header words
constexpr int HDR_NVALID = 0;   // node positions in use (0 when rejected)
constexpr int HDR_NEDGES = 1;   // stored edges, padding included
constexpr int HDR_STATUS = 2;   // status bit-mask (NEAT_ST_*)
constexpr int HDR_NLEVELS = 3;  // number of levels
constexpr int HDR_I = 4;
constexpr int HDR_O = 5;
constexpr int HDR_CLASS = 6;    // slot class
constexpr int HDR_NREAL = 7;    // enabled edges (without padding)
constexpr int HDR_SLOTS = 8;    // value slots in use (largest live set; nodes when N_max <= 62)
constexpr int HDR_WORDS = 16;

enum SlotClass { CLS_R64 = 0, CLS_R128 = 1, CLS_R224 = 2, CLS_LDS = 3 };
constexpr int N_CLASSES = 4;

__host__ __device__ constexpr int class_of(int live) {
    return live <= 62 ? CLS_R64 : (live <= 126 ? CLS_R128 : (live <= 222 ? CLS_R224 : CLS_LDS));
}
// the largest class a genome of N_max nodes can need (live <= N_max)
__host__ __device__ constexpr int max_class(int N) { return class_of(N); }
// number of value slots of a class (registers or LDS rows)
__host__ __device__ constexpr int class_slots(int cls, int N) {
    return cls == CLS_R64 ? 64 : (cls == CLS_R128 ? 128 : (cls == CLS_R224 ? 224 : N + 2));
}
// slot of the constant 0 (the constant 1 is the next slot)
__host__ __device__ constexpr int zero_slot(int cls, int N) { return class_slots(cls, N) - 2; }

// node record (16 words), record k describes position I + k:
//   code: dst slot | activation << 24 (the register kernels index with
//   the low 8 bits of the code word, and every register slot is below 256);
//   bias, response', pairs: pair count | aggregation entry << 24, then the
//   node's first three edge pairs.
// The register kernels jump on the fields at bit 24: each copy of their
// node loop has a table with one slot per activation code (0..6), the end
// of the loop (TAB_END) and one aggregation entry per (class, pair count):
// sum with 0..3 pairs or more (overflow), product and max with 1..3 pairs
// or more.  After the last node a sentinel record (code ACT_END, entry
// TAB_END, no pairs) ends the loop.
// Aggregation classes: SUM (sum, mean, and any node without incoming
// edges), PROD, MAX (max; min is stored as max over negated weights with
// the response negated, since min(t) = -max(-t) exactly);
// z = bias + response' * agg(terms), response' = response / in-degree for
// mean, -response for min, else response; y = act(z) with the activation
// code of the encoding (ACT_*).
constexpr int REC_CODE = 0;
constexpr int REC_BIAS = 1;   // float
constexpr int REC_RESP = 2;   // float, response'
constexpr int REC_NPAIRS = 3; // pair count (after padding to an even count) | entry << 24
constexpr int REC_PAIRS = 4;  // the node's first three edge pairs (12 words)
constexpr int REC_WORDS = 16;
constexpr int REC_INLINE_PAIRS = 3;
constexpr int REC_DST_MASK = 0x7ff;
constexpr int REC_FIELD_SHIFT = 24;
constexpr int REC_NPAIRS_MASK = 0x3fff;
constexpr int ACT_END = 7;    // sentinel activation code
enum AggClass { ACLS_SUM = 0, ACLS_PROD = 1, ACLS_MAX = 2 };
// table slots
constexpr int TAB_END = 7;
constexpr int TAB_AGG0 = 8;   // first aggregation entry: sum with 0 pairs
constexpr int TAB_SLOTS = TAB_AGG0 + 13;
__host__ __device__ constexpr int agg_slot(int acls, int pairs) {
    return TAB_AGG0 + (acls == ACLS_SUM ? (pairs < 4 ? pairs : 4)
                                        : 4 * acls + (pairs < 4 ? pairs : 4));
}
__host__ __device__ constexpr int slot_class(int slot) {
    return slot < TAB_AGG0 + 5 ? ACLS_SUM : (slot < TAB_AGG0 + 9 ? ACLS_PROD : ACLS_MAX);
}
__host__ __device__ constexpr uint32_t rec_code(int act, int dst) {
    return (uint32_t)dst | ((uint32_t)act << REC_FIELD_SHIFT);
}
__host__ __device__ constexpr uint32_t rec_npairs(int acls, int pairs) {
    return (uint32_t)pairs | ((uint32_t)agg_slot(acls, pairs) << REC_FIELD_SHIFT);
}
constexpr uint32_t REC_SENTINEL_CODE = (uint32_t)ACT_END << REC_FIELD_SHIFT;
constexpr uint32_t REC_SENTINEL_NPAIRS = (uint32_t)TAB_END << REC_FIELD_SHIFT;
// edge (2 words): source slot, weight
constexpr int EDGE_WORDS = 2;

__host__ __device__ constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }

// capacity of the overflow edge array: the connections plus one padding
// edge per node
__host__ __device__ constexpr int edge_cap(int N, int C) { return C + N; }

// output slots: O words (padded to 8)
__host__ __device__ constexpr int out_off() { return HDR_WORDS; }
__host__ __device__ constexpr int rec_off(int O) { return HDR_WORDS + round_up(O, 8); }
__host__ __device__ constexpr int edge_off(int N, int O) { return rec_off(O) + REC_WORDS * N; }
// first overflow edge of record k (N words)
__host__ __device__ constexpr int ebeg_off(int N, int C, int O) {
    return edge_off(N, O) + EDGE_WORDS * edge_cap(N, C);
}
// first position of level l, l = 0..n_levels (N + 1 words)
__host__ __device__ constexpr int lvl_off(int N, int C, int O) { return ebeg_off(N, C, O) + N; }
// 16 words of slack after the last array: the forward kernels read edges
// eight at a time (16 words) and may run past the last edge.
constexpr int PROG_SLACK = 16;
__host__ __device__ constexpr int prog_words(int N, int C, int O) {
    return round_up(lvl_off(N, C, O) + N + 1 + PROG_SLACK, 64);
}

// population area (after P programs): POP_COUNT + c genomes of class c,
// POP_BEGIN + c their first entry in the id list at POP_IDS
constexpr int POP_COUNT = 0;
constexpr int POP_BEGIN = 4;
constexpr int POP_IDS = 64;
__host__ __device__ constexpr long long pop_off(long long P, int N, int C, int O) {
    return P * prog_words(N, C, O);
}
__host__ __device__ constexpr long long pop_words(long long P) {
    return POP_IDS + (P + 63) / 64 * 64;
}

enum Act { ACT_IDENTITY = 0, ACT_TANH, ACT_SIGMOID, ACT_RELU, ACT_SIN, ACT_GAUSS, ACT_ABS };
enum Agg { AGG_SUM = 0, AGG_PRODUCT, AGG_MAX, AGG_MIN, AGG_MEAN };
constexpr int N_ACT = 7;
constexpr int N_AGG = 5;

}  // namespace neat
