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
// vector.  The slot numbering depends only on N_max (layout_of):
//   REG32  N_max <= 30: slot = position; slots 30, 31 hold the constants
//          0 and 1;
//   REG64  N_max <= 60: positions 0..29 -> slots 0..29, positions >= 30 ->
//          slot + 2; slots 30, 31 and 62, 63 hold 0 and 1 (one pair in each
//          32-slot half);
//   WIDE   otherwise: slot = position; slots N_max, N_max + 1 hold 0 and 1.
// A node's incoming edges are stored as (source slot, weight) in ascending
// source-key order, first those whose source lies in slots 0..31 ("low
// half"), then the others (REG64 only; the other layouts have one half).
// Each half is padded to an even count with one neutral edge, so kernels
// consume edges in pairs without per-edge tests: for sum and mean a term
// 1 * v[zero slot], for product 1 * v[one slot], for max and min a copy of
// the half's first edge.  None of these changes any result.
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
constexpr int HDR_LAYOUT = 6;
constexpr int HDR_NREAL = 7;    // enabled edges (without padding)
constexpr int HDR_WORDS = 16;

enum Layout { LAYOUT_REG32 = 0, LAYOUT_REG64 = 1, LAYOUT_WIDE = 2 };

__host__ __device__ constexpr int layout_of(int N) {
    return N <= 30 ? LAYOUT_REG32 : (N <= 60 ? LAYOUT_REG64 : LAYOUT_WIDE);
}
__host__ __device__ constexpr int slot_of(int layout, int p) {
    return (layout == LAYOUT_REG64 && p >= 30) ? p + 2 : p;
}
// number of value slots the forward kernels hold per sample
__host__ __device__ constexpr int n_slots(int layout, int N) {
    return layout == LAYOUT_REG32 ? 32 : (layout == LAYOUT_REG64 ? 64 : N + 2);
}
// slot of the constant 0 (the constant 1 is the next slot) in a half
__host__ __device__ constexpr int zero_slot(int layout, int N, int half) {
    return layout == LAYOUT_REG32 ? 30 : (layout == LAYOUT_REG64 ? (half ? 62 : 30) : N);
}
__host__ __device__ constexpr int half_of(int layout, int slot) {
    return (layout == LAYOUT_REG64 && slot >= 32) ? 1 : 0;
}

// node record (8 words), record k describes position I + k:
constexpr int REC_NLO = 0;    // edge pairs from the low half
constexpr int REC_NHI = 1;    // edge pairs from the high half
constexpr int REC_ACT = 2;
constexpr int REC_AGG = 3;
constexpr int REC_BIAS = 4;   // float
constexpr int REC_RESP = 5;   // float
constexpr int REC_SCALE = 6;  // float: 1 / in-degree for mean, else 1
constexpr int REC_DST = 7;    // slot of the node
constexpr int REC_WORDS = 8;
// edge (2 words): source slot, weight
constexpr int EDGE_WORDS = 2;

__host__ __device__ constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }

// capacity in edges: the connections plus one padding edge per half per node
__host__ __device__ constexpr int edge_cap(int N, int C) { return C + 2 * N; }

// output slots: O words (padded to 8)
__host__ __device__ constexpr int out_off() { return HDR_WORDS; }
__host__ __device__ constexpr int rec_off(int O) { return HDR_WORDS + round_up(O, 8); }
__host__ __device__ constexpr int edge_off(int N, int O) { return rec_off(O) + REC_WORDS * N; }
// first edge index of record k (N words)
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

enum Act { ACT_IDENTITY = 0, ACT_TANH, ACT_SIGMOID, ACT_RELU, ACT_SIN, ACT_GAUSS, ACT_ABS };
enum Agg { AGG_SUM = 0, AGG_PRODUCT, AGG_MAX, AGG_MIN, AGG_MEAN };
constexpr int N_ACT = 7;
constexpr int N_AGG = 5;

}  // namespace neat
