// node_loop_asm.h -- the calculation stage's node loop (Section 3.3: v[k] =
// act(bias + response * agg(w * v[src])) for every computed node in order),
// written in gfx950 assembly for one wave and one sample per lane.
//
// Register contract (the C++ caller binds the value vector with
// explicit-register constraints):
//   v0..v63    the value vector, slot s in v[s] (program.h layout REG: every
//              slot the program names is < 64, so an indexed access never
//              leaves v0..v63);
//   v64..v74   scratch;
//   s40..s55   record buffer A, s56..s71 record buffer B (16-word records
//              with the node's first two edge pairs; the next record is
//              prefetched while the current one runs);
//   s72..s79   two overflow edge pairs (slot, weight, slot, weight);
//   s80:81     record array, s82:83 overflow read pointer, s84:85 overflow
//              edges of the current node, s86 record byte offset, s87 pairs
//              left, s88 pairs of the node, s89 scratch, s90 saved M0,
//              s91 end offset.
// Reads of v[slot] and writes of v[dst] use the GPR-index mode with the
// program's uniform slot numbers; a run of indexed reads keeps the mode on
// and only changes the index (s_set_gpr_idx_idx), so a sum costs one scalar
// and one vector instruction per incoming edge.
//
// Classes (program.h): aggregation SUM / PROD / MAX (min is max of negated
// weights with negated response; mean is sum with response / degree);
// activation PL (identity, abs, relu), EXPO (sigmoid, tanh, gaussian), SIN,
// with the same arithmetic as act.h (exp2 / rcp based EXPO, Cody-Waite +
// Taylor sine).
//
// Hazards: one wait state after a transcendental before its result is read,
// two after a VALU write of VCC before a read of it.
#pragma once

// record field registers of buffer A (base 40) and B (base 56):
// code, bias, response, c, ea, eb, mask, then the inline pairs
#define NEAT_REC_A                                                                          \
    "s40", "s41", "s42", "s43", "s44", "s45", "s[46:47]", "s48", "s49", "s50", "s51", "s52", \
        "s53", "s54", "s55"
#define NEAT_REC_B                                                                          \
    "s56", "s57", "s58", "s59", "s60", "s61", "s[62:63]", "s64", "s65", "s66", "s67", "s68", \
        "s69", "s70", "s71"

// Combine one pair (slot S0 weight W0, slot S1 weight W1) into v64.
#define NEAT_SUM_PAIR(S0, W0, S1, W1)                                                      \
    "  s_set_gpr_idx_on " S0 ", gpr_idx(SRC0)\n"                                           \
    "  v_fmac_f32_e64 v64, v0, " W0 "\n"                                                   \
    "  s_set_gpr_idx_idx " S1 "\n"                                                         \
    "  v_fmac_f32_e64 v64, v0, " W1 "\n"                                                   \
    "  s_set_gpr_idx_off\n"
#define NEAT_PROD_TERM(S, W)                                                               \
    "  s_set_gpr_idx_on " S ", gpr_idx(SRC0)\n"                                            \
    "  v_mul_f32_e64 v65, v0, " W "\n"                                                     \
    "  s_set_gpr_idx_off\n"                                                                \
    "  v_mul_f32_e32 v64, v64, v65\n"
#define NEAT_PROD_PAIR(S0, W0, S1, W1) NEAT_PROD_TERM(S0, W0) NEAT_PROD_TERM(S1, W1)
#define NEAT_MAX_TERM(S, W)                                                                \
    "  s_set_gpr_idx_on " S ", gpr_idx(SRC0)\n"                                            \
    "  v_mul_f32_e64 v65, v0, " W "\n"                                                     \
    "  s_set_gpr_idx_off\n"                                                                \
    "  v_max_f32_e32 v64, v64, v65\n"                                                      \
    "  v_cmp_u_f32_e32 vcc, v65, v65\n"                                                    \
    "  s_nop 1\n"                                                                          \
    "  v_cndmask_b32_e32 v66, v66, v65, vcc\n"
#define NEAT_MAX_PAIR(S0, W0, S1, W1) NEAT_MAX_TERM(S0, W0) NEAT_MAX_TERM(S1, W1)

// One aggregation class: the record's inline pairs, then the overflow
// pairs (pairs - 2 of them) in chunks of two.  K: class tag; PAIR: combiner.
#define NEAT_AGG(X, K, PAIR, DONE, A0S, A0W, A1S, A1W, A2S, A2W, A3S, A3W)                   \
    "  s_cmp_eq_u32 s88, 0\n"                                                              \
    "  s_cbranch_scc1 " DONE X "%=\n"                                                      \
    PAIR(A0S, A0W, A1S, A1W)                                                               \
    "  s_cmp_eq_u32 s88, 1\n"                                                              \
    "  s_cbranch_scc1 " DONE X "%=\n"                                                      \
    PAIR(A2S, A2W, A3S, A3W)                                                               \
    "  s_cmp_le_u32 s88, 2\n"                                                              \
    "  s_cbranch_scc1 " DONE X "%=\n"                                                      \
    "  s_sub_u32 s87, s88, 2\n"                                                            \
    "  s_mov_b64 s[82:83], s[84:85]\n"                                                     \
    "  s_lshl_b32 s89, s87, 4\n"                                                           \
    "  s_add_u32 s84, s84, s89\n"                                                          \
    "  s_addc_u32 s85, s85, 0\n"                                                           \
    "Lo" K "_" X "%=:\n"                                                                   \
    "  s_load_dwordx8 s[72:79], s[82:83], 0x0\n"                                           \
    "  s_waitcnt lgkmcnt(0)\n"                                                             \
    PAIR("s72", "s73", "s74", "s75")                                                       \
    "  s_cmp_eq_u32 s87, 1\n"                                                              \
    "  s_cbranch_scc1 " DONE X "%=\n"                                                      \
    PAIR("s76", "s77", "s78", "s79")                                                       \
    "  s_sub_u32 s87, s87, 2\n"                                                            \
    "  s_add_u32 s82, s82, 32\n"                                                           \
    "  s_addc_u32 s83, s83, 0\n"                                                           \
    "  s_cmp_eq_u32 s87, 0\n"                                                              \
    "  s_cbranch_scc0 Lo" K "_" X "%=\n"                                                   \
    "  s_branch " DONE X "%=\n"

// One node.  X: label tag; CODE .. P3W: record fields of the buffer holding
// this node; PREF: the other buffer (receives the next record).
#define NEAT_NODE(X, CODE, BIAS, RESP, C, EA, EB, MASK, P0S, P0W, P1S, P1W, P2S, P2W, P3S,    \
                  P3W, PREF)                                                                \
    "Lnode_" X "%=:\n"                                                                      \
    "  s_waitcnt lgkmcnt(0)\n"                                                              \
    "  s_add_u32 s86, s86, 64\n"                                                            \
    "  s_load_dwordx16 " PREF ", s[80:81], s86\n"                                           \
    "  s_and_b32 s88, " CODE ", 0xffff\n"                                                   \
    "  s_bitcmp1_b32 " CODE ", 16\n"                                                        \
    "  s_cbranch_scc1 Lprod_" X "%=\n"                                                      \
    "  s_bitcmp1_b32 " CODE ", 17\n"                                                        \
    "  s_cbranch_scc1 Lmax_" X "%=\n"                                                       \
    "  v_mov_b32_e32 v64, 0\n"                                                              \
    NEAT_AGG(X, "s", NEAT_SUM_PAIR, "Lagg_", P0S, P0W, P1S, P1W, P2S, P2W, P3S, P3W)        \
    "Lprod_" X "%=:\n"                                                                      \
    "  v_mov_b32_e32 v64, 1.0\n"                                                            \
    NEAT_AGG(X, "p", NEAT_PROD_PAIR, "Lagg_", P0S, P0W, P1S, P1W, P2S, P2W, P3S, P3W)       \
    "Lmax_" X "%=:\n"                                                                       \
    "  v_mov_b32_e32 v64, 0xff800000\n"                                                     \
    "  v_mov_b32_e32 v66, 0\n"                                                              \
    NEAT_AGG(X, "m", NEAT_MAX_PAIR, "Lmaxe_", P0S, P0W, P1S, P1W, P2S, P2W, P3S, P3W)       \
    "Lmaxe_" X "%=:\n"                                                                      \
    "  v_cmp_u_f32_e32 vcc, v66, v66\n"                                                     \
    "  s_nop 1\n"                                                                           \
    "  v_cndmask_b32_e32 v64, v64, v66, vcc\n"                                              \
    /* ---- z = bias + response' * acc */                                                   \
    "Lagg_" X "%=:\n"                                                                       \
    "  v_mov_b32_e32 v67, " BIAS "\n"                                                       \
    "  v_fmac_f32_e64 v67, " RESP ", v64\n"                                                 \
    "  s_bitcmp1_b32 " CODE ", 18\n"                                                        \
    "  s_cbranch_scc1 Lexpo_" X "%=\n"                                                      \
    "  s_bitcmp1_b32 " CODE ", 19\n"                                                        \
    "  s_cbranch_scc1 Lsin_" X "%=\n"                                                       \
    /* ---- PL: z if !(z <= 0), else (mask ? 0 : c z) */                                    \
    "  v_mul_f32_e64 v68, v67, " C "\n"                                                     \
    "  v_cndmask_b32_e64 v68, v68, 0, " MASK "\n"                                           \
    "  v_cmp_ge_f32_e32 vcc, 0, v67\n"                                                      \
    "  s_nop 1\n"                                                                           \
    "  v_cndmask_b32_e32 v70, v67, v68, vcc\n"                                              \
    "  s_branch Lwr_" X "%=\n"                                                              \
    /* ---- EXPO: e = 2^(c u), u = mask ? z z : z; mask ? e : ea + eb / (1 + e) */          \
    "Lexpo_" X "%=:\n"                                                                      \
    "  v_mul_f32_e32 v68, v67, v67\n"                                                       \
    "  v_cndmask_b32_e64 v68, v67, v68, " MASK "\n"                                         \
    "  v_mul_f32_e64 v68, v68, " C "\n"                                                     \
    "  v_exp_f32_e32 v68, v68\n"                                                            \
    "  s_nop 0\n"                                                                           \
    "  v_add_f32_e32 v69, 1.0, v68\n"                                                       \
    "  v_rcp_f32_e32 v69, v69\n"                                                            \
    "  s_nop 0\n"                                                                           \
    "  v_mov_b32_e32 v70, " EA "\n"                                                         \
    "  v_fmac_f32_e64 v70, " EB ", v69\n"                                                   \
    "  v_cndmask_b32_e64 v70, v70, v68, " MASK "\n"                                         \
    "  s_branch Lwr_" X "%=\n"                                                              \
    /* ---- SIN: Cody-Waite by pi/2, Taylor sin / cos on [-pi/4, pi/4] */                   \
    "Lsin_" X "%=:\n"                                                                       \
    "  v_mul_f32_e32 v68, 0x3f22f983, v67\n"                                                \
    "  v_rndne_f32_e32 v68, v68\n"                                                          \
    "  v_fmamk_f32 v69, v68, 0xbfc90fdb, v67\n"                                             \
    "  v_fmac_f32_e32 v69, 0x333bbd2e, v68\n"                                               \
    "  v_cvt_i32_f32_e32 v72, v68\n"                                                        \
    "  v_mul_f32_e32 v71, v69, v69\n"                                                       \
    "  v_mov_b32_e32 v73, 0x3638ef1d\n"                                                     \
    "  v_fmaak_f32 v73, v71, v73, 0xb9500d01\n"                                             \
    "  v_fmaak_f32 v73, v71, v73, 0x3c088889\n"                                             \
    "  v_fmaak_f32 v73, v71, v73, 0xbe2aaaab\n"                                             \
    "  v_mul_f32_e32 v74, v69, v71\n"                                                       \
    "  v_fmac_f32_e32 v69, v74, v73\n"                                                      \
    "  v_mov_b32_e32 v73, 0xb493f27e\n"                                                     \
    "  v_fmaak_f32 v73, v71, v73, 0x37d00d01\n"                                             \
    "  v_fmaak_f32 v73, v71, v73, 0xbab60b61\n"                                             \
    "  v_fmaak_f32 v73, v71, v73, 0x3d2aaaab\n"                                             \
    "  v_fmaak_f32 v73, v71, v73, 0xbf000000\n"                                             \
    "  v_fma_f32 v73, v71, v73, 1.0\n"                                                      \
    "  v_and_b32_e32 v74, 1, v72\n"                                                         \
    "  v_cmp_eq_u32_e32 vcc, 0, v74\n"                                                      \
    "  s_nop 1\n"                                                                           \
    "  v_cndmask_b32_e32 v70, v73, v69, vcc\n"                                              \
    "  v_and_b32_e32 v74, 2, v72\n"                                                         \
    "  v_cmp_eq_u32_e32 vcc, 0, v74\n"                                                      \
    "  s_nop 1\n"                                                                           \
    "  v_cndmask_b32_e64 v70, -v70, v70, vcc\n"                                             \
    /* ---- v[dst] = y; next node */                                                        \
    "Lwr_" X "%=:\n"                                                                        \
    "  s_lshr_b32 s89, " CODE ", 20\n"                                                      \
    "  s_set_gpr_idx_on s89, gpr_idx(DST)\n"                                                \
    "  v_mov_b32_e32 v0, v70\n"                                                             \
    "  s_set_gpr_idx_off\n"                                                                 \
    "  s_cmp_eq_u32 s86, s91\n"                                                             \
    "  s_cbranch_scc1 Ldone%=\n"

#define NEAT_NODE_(X, ...) NEAT_NODE(X, __VA_ARGS__)

// The whole loop: %[rec] record 0, %[edg] overflow edge array, %[n] records.
#define NEAT_NODE_LOOP_ASM                                                                  \
    "  s_mov_b32 s90, m0\n"                                                                 \
    "  s_mov_b64 s[80:81], %[rec]\n"                                                        \
    "  s_mov_b64 s[84:85], %[edg]\n"                                                        \
    "  s_lshl_b32 s91, %[n], 6\n"                                                           \
    "  s_mov_b32 s86, 0\n"                                                                  \
    "  s_cmp_eq_u32 s91, 0\n"                                                               \
    "  s_cbranch_scc1 Ldone%=\n"                                                            \
    "  s_load_dwordx16 s[40:55], s[80:81], 0x0\n"                                           \
    NEAT_NODE_("A", NEAT_REC_A, "s[56:71]")                                                 \
    NEAT_NODE_("B", NEAT_REC_B, "s[40:55]")                                                 \
    "  s_branch Lnode_A%=\n"                                                                \
    "Ldone%=:\n"                                                                            \
    "  s_waitcnt lgkmcnt(0)\n"                                                              \
    "  s_mov_b32 m0, s90\n"

#define NEAT_NODE_LOOP_CLOBBERS                                                             \
    "v64", "v65", "v66", "v67", "v68", "v69", "v70", "v71", "v72", "v73", "v74", "s40", "s41", \
        "s42", "s43", "s44", "s45", "s46", "s47", "s48", "s49", "s50", "s51", "s52", "s53",    \
        "s54", "s55", "s56", "s57", "s58", "s59", "s60", "s61", "s62", "s63", "s64", "s65",    \
        "s66", "s67", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "s75", "s76", "s77",    \
        "s78", "s79", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87", "s88", "s89",    \
        "s90", "s91", "vcc", "scc"
