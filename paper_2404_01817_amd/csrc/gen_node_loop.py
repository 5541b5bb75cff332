#!/usr/bin/env python3
"""Generate node_loop_asm.h: the forward kernels' node loop in gfx950
assembly, one variant per value-vector shape.

The node loop evaluates, for every computed node of a genome in topological
order, v[dst] = act(bias + response * agg(w * v[src])) (the calculation
stage, Section 3.3), for one wave with one or two samples per lane.  The
value vector lives in VGPRs and is indexed with the program's uniform slot
numbers in GPR-index mode; records and edges are read with scalar loads.

Each variant is one tile of samples as a single assembly block: the
tile's inputs are moved from the LDS staging area into the value vectors,
the DMA of the next tile's inputs into that staging area is issued, the
node loop runs, and the outputs are written to an LDS output area.  No
value crosses from one block to the next, so the value vectors are plain
clobbers and the compiler never holds or copies them.

Variants (name: samples per lane, value slots, VGPRs of the value vectors):
  S1_64   1 sample,  64 slots,  v0..v63
  S2_64   2 samples, 64 slots,  v0..v63 (first) and v64..v127 (second)
  S1_128  1 sample, 128 slots,  v0..v127
  S1_224  1 sample, 224 slots,  v0..v223
  S1_64R  1 sample,  64 slots,  v0..v63 read and v64..v127 written: the
          recurrent calculation, %[nsw] synchronous sweeps of the node loop
Scratch VGPRs follow the value vectors.

Run as ``python gen_node_loop.py`` to rewrite node_loop_asm.h next to it;
the build does this before compiling, so the header always matches.
"""
from __future__ import annotations

import os
import sys

VARIANTS = [
    # name, samples per lane, value-vector bases, first scratch VGPR, and for
    # the recurrent variant the base of the vector the sweep writes
    ("S1_64", 1, (0,), 64, None),
    ("S2_64", 2, (0, 64), 128, None),
    ("S1_128", 1, (0,), 128, None),
    ("S1_224", 1, (0,), 224, None),
    ("S1_64R", 1, (0,), 128, (64,)),
]

# scalar register map (shared by all variants)
# record buffers: code, bias, response', pair count, three edge pairs
REC_A = tuple("s%d" % i for i in range(40, 56))
REC_B = tuple("s%d" % i for i in range(56, 72))
SGPR_CLOBBERS = ["s%d" % i for i in range(40, 96)]
INLINE_PAIRS = 3
# Record fields (program.h): the code word holds the destination slot in
# its low bits and the activation's table slot at bit 24; the pair-count
# word holds the pair count in its low 14 bits and the aggregation entry's
# table slot at bit 24.  Table (per copy of the node loop, one stride per
# slot): activation blocks 0..6, the end of the loop at 7, then the
# aggregation entries, one per (class, pairs): sum with 0..3 pairs and with
# overflow, product and max with 1..3 pairs and with overflow.
FIELD_SHIFT = 24
NP_MASK = "0x3fff"
TAB_END = 7
AGG_ENTRIES = [("sum", 0), ("sum", 1), ("sum", 2), ("sum", 3), ("sum", "ov"),
               ("prod", 1), ("prod", 2), ("prod", 3), ("prod", "ov"),
               ("max", 1), ("max", 2), ("max", 3), ("max", "ov")]
TAB_AGG0 = 8
NEG_LOG2E = "0xbfb8aa3b"    # -log2(e)
TWO_LOG2E = "0x4038aa3b"    # 2 log2(e)

# sine: k = rint(z / pi); r = z - k pi (pi split in two fp32 parts: fl(pi)
# and pi - fl(pi)); the Taylor polynomial of sin of degree 13 on [-pi/2, pi/2];
# the sign flips for odd k
ONE_OVER_PI = "0x3ea2f983"
NEG_PI_HI = "0xc0490fdb"
PI_HI_MINUS_PI = "0x33bbbd2e"
# 1/13!, -1/11!, 1/9!, -1/7!, 1/5!, -1/3! rounded to fp32
SIN_C = ("0x2f309231", "0xb2d7322b", "0x3638ef1d", "0xb9500d01", "0x3c088889", "0xbe2aaaab")


class Regs:
    """Scratch VGPR names of one variant (per sample h).

    The node loop uses five per sample (acc, ta, tb, z, p) and one shared
    constant (c13, the sine polynomial's leading coefficient); the input and
    output sections use G buffers per sample, an LDS address per sample and
    a 64-bit DMA address.  The two sets are never live together, so they
    share the same registers."""

    # Placement (in units of spl registers from the first scratch VGPR):
    # acc 0, ta 1, tb 2, z 3, then c13 (one register), then p.  Keep it:
    # on gfx950 a permutation of the same registers (c13, acc, z, ta, tb)
    # made the sine block's results vary from launch to launch under full
    # occupancy, while this placement gives repeatable bits (checked by the
    # full-size repeatability tests).  Both placements pass every static
    # check of check_node_loop.py (documented wait states, load completion,
    # GPR-index mode, clobbers) and assemble to the same table layout, so
    # the cause is not one of those rules and remains unknown.
    ROLES = ("acc", "ta", "tb", "z", "p")

    def __init__(self, spl, bases, scratch, wbases=None, group=8):
        self.spl = spl
        self.bases = ["v%d" % b for b in bases]
        # recurrent: reads from v[bases], writes to v[wbases]
        self.rec = wbases is not None
        self.wbases = ["v%d" % b for b in (wbases if self.rec else bases)]
        self.names = {}
        for k, role in enumerate(self.ROLES[:4]):
            self.names[role] = ["v%d" % (scratch + k * spl + h) for h in range(spl)]
        self.c13 = "v%d" % (scratch + 4 * spl)
        self.names["p"] = ["v%d" % (scratch + 4 * spl + 1 + h) for h in range(spl)]
        n = scratch + 5 * spl + 1
        # tile section registers: input buffers, staging addresses, DMA address
        self.group = group
        self.buf = [["v%d" % (scratch + group * h + k) for k in range(group)]
                    for h in range(spl)]
        self.addr = ["v%d" % (scratch + group * spl + h) for h in range(spl)]
        d = scratch + group * spl + spl
        d += d & 1  # 64-bit VGPR operands are even-aligned
        self.dma = "v[%d:%d]" % (d, d + 1)
        n = max(n, d + 2)
        self.last = n - 1
        assert self.last <= 255

    def __getattr__(self, role):
        return self.names[role]


def lines(*xs):
    return list(xs)


def per_sample(R, fmt):
    """One instruction per sample: fmt formatted with each sample's names."""
    out = []
    for h in range(R.spl):
        d = {k: v[h] for k, v in R.names.items()}
        d["val"] = R.bases[h]
        d["wval"] = R.wbases[h]
        out.append(fmt.format(**d))
    return out


def seq(R, *fmts):
    """Instructions for all samples, interleaved: fmt 1 for every sample,
    then fmt 2 ...  With two samples the other sample's instruction sits
    between a result and its use; with one, the caller adds wait states."""
    out = []
    for f in fmts:
        out += per_sample(R, f)
    return out


def nop_if_single(R, n=0):
    return ["s_nop %d" % n] if R.spl == 1 else []


# --------------------------------------------------------------- aggregation
def read_pair(R, s0, w0, s1, w1, op0, op1):
    """Indexed reads of one edge pair: op0 applied with (slot s0, weight w0),
    op1 with (s1, w1).  op formats get {val} (the indexed value register) and
    {w} (the weight SGPR)."""
    out = ["s_set_gpr_idx_on %s, gpr_idx(SRC0)" % s0]
    out += per_sample(R, op0.replace("{w}", w0))
    out += ["s_set_gpr_idx_idx %s" % s1]
    out += per_sample(R, op1.replace("{w}", w1))
    out += ["s_set_gpr_idx_off"]
    return out


def pair(R, cls, first, s0, w0, s1, w1):
    if cls == "sum":
        op0 = ("v_mul_f32_e64 {acc}, {val}, {w}" if first else
               "v_fmac_f32_e64 {acc}, {val}, {w}")
        return read_pair(R, s0, w0, s1, w1, op0, "v_fmac_f32_e64 {acc}, {val}, {w}")
    if cls == "prod":
        if first:
            return (read_pair(R, s0, w0, s1, w1, "v_mul_f32_e64 {acc}, {val}, {w}",
                              "v_mul_f32_e64 {tb}, {val}, {w}")
                    + seq(R, "v_mul_f32_e32 {acc}, {acc}, {tb}"))
        return (read_pair(R, s0, w0, s1, w1, "v_mul_f32_e64 {ta}, {val}, {w}",
                          "v_mul_f32_e64 {tb}, {val}, {w}")
                + seq(R, "v_mul_f32_e32 {acc}, {acc}, {ta}", "v_mul_f32_e32 {acc}, {acc}, {tb}"))
    assert cls == "max"
    comb = ("v_maximum3_f32 {acc}, {ta}, {tb}, {tb}" if first else
            "v_maximum3_f32 {acc}, {acc}, {ta}, {tb}")
    return (read_pair(R, s0, w0, s1, w1, "v_mul_f32_e64 {ta}, {val}, {w}",
                      "v_mul_f32_e64 {tb}, {val}, {w}")
            + seq(R, comb))


def inline_pairs(R, cls, rec, k):
    """The first k (<= 3) of the node's pairs, from its record."""
    p = rec[4:16]
    out = []
    for j in range(k):
        out += pair(R, cls, j == 0, *p[4 * j:4 * j + 4])
    return out


def overflow_loop(R, X, cls, rec):
    """Pairs after the third: s87 = pairs - 3 of them from the overflow
    array, two at a time (the first two were requested at the entry), then
    s[84:85] moves past them.  Ends where the aggregate is complete."""
    NP = rec[3]
    K = cls[0]
    done = "Lovd%s_%s%%=" % (K, X)
    out = ["s_and_b32 s87, %s, %s" % (NP, NP_MASK),
           "s_sub_u32 s87, s87, %d" % INLINE_PAIRS,
           "s_mov_b64 s[82:83], s[84:85]",
           "s_lshl_b32 s89, s87, 4",
           "s_add_u32 s84, s84, s89",
           "s_addc_u32 s85, s85, 0",
           "Lo%s_%s%%=:" % (K, X),
           "s_waitcnt lgkmcnt(0)"]
    out += pair(R, cls, False, "s72", "s73", "s74", "s75")
    out += ["s_cmp_eq_u32 s87, 1", "s_cbranch_scc1 " + done]
    out += pair(R, cls, False, "s76", "s77", "s78", "s79")
    out += ["s_sub_u32 s87, s87, 2",
            "s_cmp_eq_u32 s87, 0",
            "s_cbranch_scc1 " + done,
            "s_add_u32 s82, s82, 32",
            "s_addc_u32 s83, s83, 0",
            "s_load_dwordx8 s[72:79], s[82:83], 0x0",
            "s_branch Lo%s_%s%%=" % (K, X),
            done + ":"]
    return out


def jump(word, base, shift):
    """Computed jump to the table slot held at bit 24 of word."""
    lo, hi = base
    return ["s_lshr_b32 s88, %s, %d" % (word, shift),
            "s_add_u32 s88, s88, %s" % lo,
            "s_addc_u32 s89, %s, 0" % hi,
            "s_setpc_b64 s[88:89]"]


def to_activation(R, rec, base, shift):
    """z = bias (the activation block finishes z), then the jump to the
    node's activation block."""
    return seq(R, "v_mov_b32_e32 {z}, " + rec[1]) + jump(rec[0], base, shift)


def agg_entry(R, X, cls, k, rec, pref, base, shift):
    """Table entry for a node of class cls with k pairs (or "ov": three in
    the record, the rest in the overflow array): request the next node's
    record into pref, aggregate, and jump to the activation."""
    out = ["s_add_u32 s86, s86, 64",
           "s_load_dwordx16 %s, s[80:81], s86" % pref]
    if k == "ov":
        out += ["s_load_dwordx8 s[72:79], s[84:85], 0x0"]
        out += inline_pairs(R, cls, rec, INLINE_PAIRS)
        out += ["s_branch Lov%s_%s%%=" % (cls[0], X)]
        return out
    if k == 0:
        out += seq(R, "v_mov_b32_e32 {acc}, 0")
    out += inline_pairs(R, cls, rec, k)
    return out + to_activation(R, rec, base, shift)


# --------------------------------------------------------------- activation
# Activation blocks, one per code of the encoding (ACT_*).  On entry z holds
# the bias and acc the aggregate; every block returns (body, y): body
# computes y = act(z) into the scratch register named y, which a plain move
# with the destination indexed then writes to v[dst].  Only moves run with
# destination indexing; the arithmetic stays outside it, and two wait states
# separate a transcendental (v_exp, v_rcp, which completes after later
# instructions have issued) from the switch into indexed mode.
# z = fma(response', acc, bias) is the first step of every block.
TRANS_GAP = "s_nop 1"


def z_of(R):
    return seq(R, "v_fmac_f32_e64 {z}, " + "%(resp)s" + ", {acc}")


def act_identity(R):
    return z_of(R), "z"


def act_tanh(R):
    # 1 - 2 / (1 + 2^(2 log2(e) z))
    out = z_of(R) + seq(R, "v_mul_f32_e32 {ta}, " + TWO_LOG2E + ", {z}",
                        "v_exp_f32_e32 {ta}, {ta}")
    out += nop_if_single(R)
    out += seq(R, "v_add_f32_e32 {tb}, 1.0, {ta}", "v_rcp_f32_e32 {tb}, {tb}")
    out += nop_if_single(R)
    out += seq(R, "v_fma_f32 {ta}, {tb}, -2.0, 1.0")
    return out, "ta"


def act_sigmoid(R):
    # 1 / (1 + 2^(-log2(e) z))
    out = z_of(R) + seq(R, "v_mul_f32_e32 {ta}, " + NEG_LOG2E + ", {z}",
                        "v_exp_f32_e32 {ta}, {ta}")
    out += nop_if_single(R)
    out += seq(R, "v_add_f32_e32 {tb}, 1.0, {ta}", "v_rcp_f32_e32 {ta}, {tb}") + [TRANS_GAP]
    return out, "ta"


def act_relu(R):
    # maximum(z, 0), NaN-propagating
    return z_of(R) + seq(R, "v_maximum3_f32 {ta}, {z}, 0, 0"), "ta"


def act_gauss(R):
    # 2^(-log2(e) z z)
    out = z_of(R) + seq(R, "v_mul_f32_e32 {ta}, {z}, {z}",
                        "v_mul_f32_e32 {ta}, " + NEG_LOG2E + ", {ta}",
                        "v_exp_f32_e32 {tb}, {ta}") + [TRANS_GAP]
    return out, "tb"


def act_abs(R):
    # maximum(z, -z), NaN-propagating
    return z_of(R) + seq(R, "v_maximum3_f32 {ta}, {z}, -{z}, -{z}"), "ta"


def act_sin(R):
    # k = rint(z / pi) in tb, r = z - k pi in acc, then k -> int; r^2 in z;
    # p = -1/3! + r^2 (1/5! + ... + r^2 / 13!); sin r = r + (r r^2) p;
    # sin z = sin r with the sign flipped for odd k: adding k << 31 to the
    # bit pattern toggles its sign bit
    c13, c11, c9, c7, c5, c3 = SIN_C
    out = z_of(R) + seq(
        R,
        "v_mul_f32_e32 {tb}, " + ONE_OVER_PI + ", {z}",
        "v_rndne_f32_e32 {tb}, {tb}",
        "v_fmamk_f32 {acc}, {tb}, " + NEG_PI_HI + ", {z}",
        "v_fmac_f32_e32 {acc}, " + PI_HI_MINUS_PI + ", {tb}",
        "v_cvt_i32_f32_e32 {tb}, {tb}",
        "v_mul_f32_e32 {z}, {acc}, {acc}",
        "v_fmaak_f32 {p}, {z}, " + R.c13 + ", " + c11,
        "v_fmaak_f32 {p}, {z}, {p}, " + c9,
        "v_fmaak_f32 {p}, {z}, {p}, " + c7,
        "v_fmaak_f32 {p}, {z}, {p}, " + c5,
        "v_fmaak_f32 {p}, {z}, {p}, " + c3,
        "v_mul_f32_e32 {ta}, {acc}, {z}",
        "v_fmac_f32_e32 {acc}, {ta}, {p}",
        "v_lshl_add_u32 {ta}, {tb}, 31, {acc}")
    return out, "ta"


# in the order of the activation codes: identity, tanh, sigmoid, relu, sin,
# gaussian, abs
ACTS = (act_identity, act_tanh, act_sigmoid, act_relu, act_sin, act_gauss, act_abs)


# --------------------------------------------------------------- node, loop
INLINE_CONSTS = {"0", "1", "-1", "2", "4", "-2", "-4", "0.5", "-0.5", "1.0", "-1.0", "2.0",
                 "-2.0", "4.0", "-4.0"}


def encoded_bytes(line):
    """Upper bound of an instruction's encoding: 8 bytes for VOP3 forms,
    scalar memory loads and anything carrying a 32-bit literal, else 4."""
    op = line.split()[0]
    if op.startswith(".") or op.endswith(":"):
        return 0
    args = [a.strip() for a in line[len(op):].replace(",", " ").split()]
    literal = any(a.startswith("0x") or (a.lstrip("-").replace(".", "").isdigit() and
                                         a not in INLINE_CONSTS and not a.startswith("offset"))
                  for a in args)
    vop3 = op.endswith("_e64") or op in ("v_fma_f32", "v_maximum3_f32", "v_bfi_b32",
                                         "v_lshl_add_u64", "v_lshl_add_u32",
                                         "v_cmp_gt_u32_e64")
    smem = op.startswith("s_load") or op.startswith("s_buffer_load")
    return 8 if (vop3 or literal or smem or op in ("v_fmaak_f32", "v_fmamk_f32")) else 4


def act_blocks(R, rec, orec, obase, shift):
    """The activation blocks of the copy of the node loop with record buffer
    rec, each with the write of v[dst] and the jump into the next node's
    aggregation entry (record orec, the other copy's table at obase)."""
    CODE, RESP = rec[0], rec[2]
    blocks = []
    for fn in ACTS:
        body, y = fn(R)
        body = [l % {"resp": RESP} for l in body]
        # v[dst] = y (GPR-index mode uses the low 8 bits of the code word:
        # the destination slot); next node, once its record is in
        body += ["s_set_gpr_idx_on %s, gpr_idx(DST)" % CODE]
        body += per_sample(R, "v_mov_b32_e32 {wval}, {%s}" % y)
        body += ["s_set_gpr_idx_off", "s_waitcnt lgkmcnt(0)"]
        body += jump(orec[3], obase, shift)
        blocks.append(body)
    return blocks


def table(R, X, rec, pref, base, orec, obase, shift):
    """The slots of one copy's table, in order."""
    slots = act_blocks(R, rec, orec, obase, shift)
    slots.append(["s_branch Ldone%="])
    for cls, k in AGG_ENTRIES:
        slots.append(agg_entry(R, X, cls, k, rec, pref, base, shift))
    return slots


def table_stride(R):
    """Bytes per table slot: the smallest power of two (at least 64) that
    holds the largest slot."""
    size = max(sum(encoded_bytes(l) for l in b)
               for b in table(R, "A", REC_A, "s[56:71]", ("s92", "s93"), REC_B,
                              ("s94", "s95"), 16))
    stride = 64
    while stride < size:
        stride *= 2
    return stride


def copy(R, X, rec, pref, base, orec, obase):
    """One copy of the node loop: its table, then the overflow tails of its
    three aggregation classes (each ends with the jump to the activation)."""
    stride = table_stride(R)
    shift = FIELD_SHIFT - (stride.bit_length() - 1)
    align = stride.bit_length() - 1
    out = [".p2align %d" % align, "Ltab_%s%%=:" % X]
    for k, body in enumerate(table(R, X, rec, pref, base, orec, obase, shift)):
        size = sum(encoded_bytes(l) for l in body)
        assert size <= stride, "table slot %d needs %d > %d bytes" % (k, size, stride)
        if k:
            out += [".p2align %d" % align]
        out += body
    for cls in ("sum", "prod", "max"):
        out += ["Lov%s_%s%%=:" % (cls[0], X)] + overflow_loop(R, X, cls, rec)
        out += to_activation(R, rec, base, shift)
    return out


def node_loop(R):
    """All computed nodes: %[rec] record 0 (the records end with a sentinel
    whose entry is the end of the loop), %[edg] overflow edges.  Copy A runs
    the nodes at even positions (record buffer s40..s55), copy B the odd
    ones (s56..s71); each node's entry requests the next node's record into
    the other buffer, and its activation block waits for it and jumps into
    that node's entry.  M0 is saved in s90 by the caller."""
    stride = table_stride(R)
    shift = FIELD_SHIFT - (stride.bit_length() - 1)
    out = ["s_mov_b64 s[80:81], %[rec]",
           "s_mov_b64 s[84:85], %[edg]",
           "s_mov_b32 s86, 0",
           "v_mov_b32_e32 %s, %s" % (R.c13, SIN_C[0]),
           "s_load_dwordx16 s[40:55], s[80:81], 0x0",
           # addresses of the two copies' tables
           "s_getpc_b64 s[92:93]",
           "Lpc%=:",
           "s_add_u32 s94, s92, Ltab_B%= - Lpc%=",
           "s_addc_u32 s95, s93, 0",
           "s_add_u32 s92, s92, Ltab_A%= - Lpc%=",
           "s_addc_u32 s93, s93, 0",
           "s_waitcnt lgkmcnt(0)"]
    out += jump(REC_A[3], ("s92", "s93"), shift)
    out += copy(R, "A", REC_A, "s[56:71]", ("s92", "s93"), REC_B, ("s94", "s95"))
    out += copy(R, "B", REC_B, "s[40:55]", ("s94", "s95"), REC_A, ("s92", "s93"))
    out += ["Ldone%=:",
            "s_waitcnt lgkmcnt(0)"]
    return out


def place_inputs(R):
    """v[i] = staged input i of the lane's sample(s), i < %[ni], eight at a
    time (ds_read2 pairs, one index setting per eight moves).  The last
    group may write up to seven slots past the inputs: those belong to
    computed nodes (written before any read) or the constants (set after),
    and the reads past the lane's inputs stay inside the staging areas."""
    # lane l's first input: %[dm0] + 4 l ni (+ 256 ni for the second sample)
    out = ["s_lshl_b32 s41, %[ni], 2",
           "v_mul_u32_u24_e32 %s, s41, %%[lane]" % R.addr[0],
           "v_add_u32_e32 %s, %%[dm0], %s" % (R.addr[0], R.addr[0])]
    if R.spl == 2:
        out += ["s_lshl_b32 s41, %[ni], 8",
                "v_add_u32_e32 %s, s41, %s" % (R.addr[1], R.addr[0])]
    out += ["s_mov_b32 s40, 0",
            "s_cmp_eq_u32 %[ni], 0",
            "s_cbranch_scc1 Lpl_done%=",
            "Lpl%=:"]
    for h in range(R.spl):
        b = R.buf[h]
        for k in range(0, 8, 2):
            lo, hi = int(b[k][1:]), int(b[k + 1][1:])
            out.append("ds_read2_b32 v[%d:%d], %s offset0:%d offset1:%d"
                       % (lo, hi, R.addr[h], k, k + 1))
    for h in range(R.spl):
        out.append("v_add_u32_e32 %s, 32, %s" % (R.addr[h], R.addr[h]))
    out += ["s_waitcnt lgkmcnt(0)",
            "s_set_gpr_idx_on s40, gpr_idx(DST)"]
    for h in range(R.spl):
        for vb in sorted(set([R.bases[h], R.wbases[h]])):
            base = int(vb[1:])
            for k in range(8):
                out.append("v_mov_b32_e32 v%d, %s" % (base + k, R.buf[h][k]))
    out += ["s_set_gpr_idx_off",
            "s_add_u32 s40, s40, 8",
            "s_cmp_lt_u32 s40, %[ni]",
            "s_cbranch_scc1 Lpl%=",
            "Lpl_done%=:",
            # the constants 0 and 1 at the zero slot
            "s_set_gpr_idx_on %[zs], gpr_idx(DST)"]
    for h in range(R.spl):
        for vb in sorted(set([R.bases[h], R.wbases[h]])):
            base = int(vb[1:])
            out += ["v_mov_b32_e32 v%d, 0" % base, "v_mov_b32_e32 v%d, 1.0" % (base + 1)]
    out += ["s_set_gpr_idx_off"]
    return out


def dma_next(R):
    """Copy the next tile's inputs HBM -> LDS staging (the inputs just
    placed have been read): %[dn] pieces of 16 bytes (%[dvec] = 1) or 4
    bytes, lane l reading piece l of each round of 64 from %[dsrc] onward,
    to %[dm0] + piece offset.  Rounds mask off lanes past the last piece.
    The loads are non-temporal: every input is read exactly once."""
    d0 = R.dma[2:R.dma.index(":")]
    d1 = R.dma[R.dma.index(":") + 1:-1]
    out = ["s_cmp_eq_u32 %[dn], 0",
           "s_cbranch_scc1 Ldma_done%=",
           "s_mov_b64 s[42:43], exec",
           "s_cmp_eq_u32 %[dvec], 0",
           "s_cselect_b32 s41, 2, 4",
           "v_lshlrev_b32_e32 v%s, s41, %%[lane]" % d0,
           "v_mov_b32_e32 v%s, 0" % d1,
           "v_lshl_add_u64 %s, %s, 0, %%[dsrc]" % (R.dma, R.dma),
           "s_mov_b32 s40, 0",
           "s_mov_b32 m0, %[dm0]",
           "s_cmp_eq_u32 %[dvec], 0",
           "s_cbranch_scc1 Ldma1%="]
    for tag, op, step in (("4", "global_load_lds_dwordx4", 1024), ("1", "global_load_lds_dword", 256)):
        if tag == "1":
            out += ["Ldma1%=:"]
        out += ["s_mov_b64 s[46:47], %d" % step,
                "Ldl%s%%=:" % tag,
                "s_sub_u32 s41, %[dn], s40",
                "v_cmp_gt_u32_e64 s[44:45], s41, %[lane]",
                "s_and_b64 exec, s[42:43], s[44:45]",
                "s_nop 0",
                "%s %s, off nt" % (op, R.dma),
                "s_mov_b64 exec, s[42:43]",
                "v_lshl_add_u64 %s, %s, 0, s[46:47]" % (R.dma, R.dma),
                "s_add_u32 m0, m0, %d" % step,
                "s_add_u32 s40, s40, 64",
                "s_cmp_lt_u32 s40, %[dn]",
                "s_cbranch_scc1 Ldl%s%%=" % tag,
                "s_branch Ldma_done%="]
    out += ["Ldma_done%=:"]
    return out


def write_outputs(R):
    """Output j of the lane's sample(s) -> LDS output area %[om0] + 4 (l O
    + j) for lane l (+ 256 O for the second sample), slots from %[outs],
    O = %[no]."""
    out = ["s_mov_b64 s[44:45], %[outs]",
           "s_mov_b32 s40, 0",
           "s_lshl_b32 s41, %[no], 2",
           "v_mul_u32_u24_e32 %s, s41, %%[lane]" % R.addr[0],
           "v_add_u32_e32 %s, %%[om0], %s" % (R.addr[0], R.addr[0])]
    if R.spl == 2:
        out += ["s_lshl_b32 s41, %[no], 8",
                "v_add_u32_e32 %s, s41, %s" % (R.addr[1], R.addr[0])]
    out += ["Lout%=:",
            "s_load_dwordx8 s[48:55], s[44:45], 0x0",
            "s_waitcnt lgkmcnt(0)"]
    for k in range(8):
        out += ["s_set_gpr_idx_on s%d, gpr_idx(SRC0)" % (48 + k)]
        for h in range(R.spl):
            out += ["v_mov_b32_e32 %s, %s" % (R.buf[h][k], R.bases[h])]
        out += ["s_set_gpr_idx_off"]
        for h in range(R.spl):
            out += ["ds_write_b32 %s, %s offset:%d" % (R.addr[h], R.buf[h][k], 4 * k)]
        out += ["s_add_u32 s40, s40, 1",
                "s_cmp_ge_u32 s40, %[no]",
                "s_cbranch_scc1 Lout_done%="]
    for h in range(R.spl):
        out.append("v_add_u32_e32 %s, 32, %s" % (R.addr[h], R.addr[h]))
    out += ["s_add_u32 s44, s44, 32",
            "s_addc_u32 s45, s45, 0",
            "s_branch Lout%=",
            "Lout_done%=:"]
    return out


def zero_values(R):
    """Recurrent variant: v0 = 0 at every slot of the read vector (the inputs
    and constants are placed after)."""
    base = int(R.bases[0][1:])
    return ["v_mov_b32_e32 v%d, 0" % (base + k) for k in range(64)]


def sweeps(R):
    """Recurrent variant: %[nsw] sweeps of the node loop, each reading the
    previous sweep's values (read vector) and writing the write vector, then
    copying the write vector into the read vector (inputs and constants are
    in both, so the copy keeps them)."""
    rb, wb = int(R.bases[0][1:]), int(R.wbases[0][1:])
    out = ["s_mov_b32 s91, %[nsw]",
           "Lsw%=:",
           "s_cmp_eq_u32 s91, 0",
           "s_cbranch_scc1 Lsw_done%="]
    out += node_loop(R)
    out += ["v_mov_b32_e32 v%d, v%d" % (rb + k, wb + k) for k in range(64)]
    out += ["s_sub_u32 s91, s91, 1",
            "s_branch Lsw%=",
            "Lsw_done%=:"]
    return out


def clear_past_inputs(R):
    """Recurrent variant: place_inputs writes whole groups of eight, so the
    read vector's slots from %[ni] up to the next multiple of eight (below
    64) hold staging words; set them back to 0 (before the constants)."""
    base = int(R.bases[0][1:])
    return ["s_mov_b32 s41, %[ni]",
            "Lcl%=:",
            "s_and_b32 s40, s41, 7",
            "s_cbranch_scc0 Lcl_done%=",
            "s_set_gpr_idx_on s41, gpr_idx(DST)",
            "v_mov_b32_e32 v%d, 0" % base,
            "s_set_gpr_idx_off",
            "s_add_u32 s41, s41, 1",
            "s_branch Lcl%=",
            "Lcl_done%=:"]


def tile(R):
    if R.rec:
        pl = place_inputs(R)
        k = pl.index("Lpl_done%=:") + 1
        return (["s_mov_b32 s90, m0"] + zero_values(R) + pl[:k] + clear_past_inputs(R)
                + pl[k:] + dma_next(R) + sweeps(R) + write_outputs(R) + ["s_mov_b32 m0, s90"])
    return (["s_mov_b32 s90, m0"] + place_inputs(R) + dma_next(R) + node_loop(R)
            + write_outputs(R) + ["s_mov_b32 m0, s90"])


HEADER = """\
// node_loop_asm.h -- GENERATED by gen_node_loop.py; edit that script.
//
// One tile of the calculation stage (Section 3.3) in gfx950 assembly, for
// one wave with one or two samples per lane: for every computed node in
// topological order, v[dst] = act(bias + response * agg(w * v[src])).
//
// A tile block (NEAT_TILE_<variant>) does, in order:
//   1. v[i] = input i of the lane's sample(s), i < %[ni], from the LDS
//      staging area at byte address %[dm0] (sample s's inputs at + 4 s ni;
//      lane l holds samples l and, with two per lane, 64 + l); then the
//      constants 0 and 1 at slots %[zs], %[zs] + 1;
//   2. the DMA of the next tile's inputs into the staging area: %[dn]
//      pieces of 16 bytes (%[dvec] = 1) or 4 bytes (%[dvec] = 0) from the
//      global address %[dsrc] onward, lane l taking piece l of each round
//      of 64; %[lane] is the lane id (the only VGPR operand);
//   3. the node loop over the records from %[rec] up to the sentinel record
//      that follows the last node, overflow edges from %[edg];
//   4. output j of each sample s = v[slot j] (slots at %[outs], j < %[no])
//      to the LDS output area at %[om0] + 4 (s O + j).
// The value vectors (slot s of sample h in v[base_h + s]; every slot the
// program names is below the variant's slot count) live only inside the
// block and are listed as clobbers with the scratch VGPRs after them.
//
// Scalar registers: s40..s55 record buffer A, s56..s71 record buffer B
// (16-word records with the node's first three edge pairs; the next record
// is prefetched while the current one runs), s72..s79 two overflow pairs
// (the first two requested at the start of the node), s80:81 record array,
// s82:83 overflow read pointer, s84:85 overflow edges of the current node,
// s86 record byte offset, s87 pairs left, s88:89 jump target and scratch,
// s90 saved M0, s92:93 and s94:95 the two copies' activation blocks; steps
// 1, 2 and 4 use s40..s55 before and after the node loop.
// Reads of v[slot] and the write of v[dst] use GPR-index mode with the
// program's uniform slots; an indexed read of a pair keeps the mode on and
// only moves the index, and every sample of the lane shares it.
//
// Aggregation classes (program.h): sum (mean folds 1/degree into the
// response), product, max (min is max over negated weights with negated
// response), the first pair initialising the accumulator and an empty sum
// giving 0.  Max uses the NaN-propagating maximum.  Activations: one block
// per code, entered by a computed jump (blocks aligned to a fixed stride):
// identity; relu maximum(z, 0) and abs maximum(z, -z); sigmoid, tanh and
// gaussian on the hardware base-2 exponential and reciprocal; sin by
// Cody-Waite reduction and Taylor polynomials.  Each block ends with the
// write of v[dst] and the jump to the next node.  The C++ node loop of the
// LDS store performs the same operations in the same order.
//
// The recurrent block (NEAT_TILE_S1_64R) zeroes the read vector v0..v63,
// places the inputs and constants in it and in the write vector v64..v127,
// then runs the node loop %[nsw] times: every sweep reads v0.. and writes
// v64.., and 64 moves copy the write vector back (s91 counts the sweeps).
//
// Hazards: a transcendental's result is read no sooner than one instruction
// later (with two samples the other sample's instruction sits between); a
// write of M0 is followed by one wait state before the LDS DMA reads it.
#pragma once
"""


def c_string(lines_):
    return "\n".join('    "  %s\\n"' % l if not l.endswith(":") else '    "%s\\n"' % l
                     for l in lines_)


def generate():
    parts = [HEADER]
    for name, spl, bases, scratch, wbases in VARIANTS:
        R = Regs(spl, bases, scratch, wbases)
        body = tile(R)
        parts.append("// %s: %d sample(s) per lane, value vectors at %s, scratch v%d..v%d\n"
                     % (name, spl, ", ".join("v%d" % b for b in bases), scratch, R.last))
        parts.append("#define NEAT_TILE_%s \\\n%s\n" % (name, " \\\n".join(
            c_string([l]) for l in body)))
        vclob = ['"v%d"' % i for i in range(0, R.last + 1)]
        clob = vclob + ['"%s"' % s for s in SGPR_CLOBBERS] + ['"vcc"', '"scc"']
        rows = [", ".join(clob[i:i + 12]) for i in range(0, len(clob), 12)]
        parts.append("#define NEAT_CLOB_%s \\\n    %s\n" % (name, ", \\\n    ".join(rows)))
        parts.append("#define NEAT_SCRATCH_%s %d\n\n" % (name, scratch))
    return "\n".join(parts)


def main(argv):
    here = os.path.dirname(os.path.abspath(__file__))
    path = argv[1] if len(argv) > 1 else os.path.join(here, "node_loop_asm.h")
    text = generate()
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main(sys.argv)
