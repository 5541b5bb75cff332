#!/usr/bin/env python3
"""Static checks of the generated node-loop assembly (node_loop_asm.h).

The tile blocks are inline assembly, so the compiler's hazard recognizer
never sees the instructions inside them: every wait state and every wait
for an outstanding load is the generator's job.  This module rebuilds each
block's control-flow graph (fall-through, branches, and the computed jumps
of the node loop into its table slots) and checks, on every path:

Wait states (instructions or s_nop cycles between a producer and a
consumer), from the gfx9/CDNA hazard rules:
  TRANS    a transcendental VALU op (v_exp, v_log, v_rcp, v_rsq, v_sqrt,
           v_sin, v_cos) writes a VGPR -> a non-transcendental VALU op
           reads it: 1
  IDXTRANS a transcendental op -> s_set_gpr_idx_on (the generator's own
           rule: no transcendental result is still in flight when indexed
           mode starts): 2
  SGPRVMEM a VALU op writes an SGPR -> a VMEM op reads it: 5
  LANESEL  a VALU op writes an SGPR -> v_readlane / v_writelane selects a
           lane with it: 4
  M0LDS    an SALU op writes M0 (s_mov / s_add to m0, s_set_gpr_idx_on and
           s_set_gpr_idx_idx, which set M0's index bits) -> an LDS DMA load
           (global_load_lds_*), which takes its LDS address from M0: 1
  DPP      a VALU op writes a VGPR -> a DPP op reads it: 2; a VALU op
           writes EXEC -> a DPP op: 5
  EXECZ    a VALU op writes VCC or EXEC -> a VALU op reads VCCZ / EXECZ: 5

Outstanding loads (data flow to a fixed point over the graph):
  SMEM     the SGPRs a scalar load writes are neither read nor written
           until s_waitcnt lgkmcnt(0) (scalar loads return out of order, so
           only a zero count retires them)
  DS       the VGPRs an LDS read writes are neither read nor written until
           s_waitcnt lgkmcnt(0)

GPR-index mode (a state machine over the graph):
  IDXMODE  s_set_gpr_idx_on only with the mode off, _idx and _off only with
           it on; every join agrees on the mode; inside the mode only VALU
           moves and arithmetic (the instructions meant to be indexed) and
           s_set_gpr_idx_idx / _off; in SRC0 mode src0 is a VGPR of a value
           vector, in DST mode the instruction is a v_mov whose destination
           is a value vector's base; no transcendental op runs in the mode
  IDXRANGE every indexed base plus the largest slot index stays inside its
           value vector (below the first scratch register)

Registers:
  CLOBBER  every VGPR and SGPR the block writes is in its clobber list; the
           inline-asm operands (%[...]) are never written
  RESTORE  EXEC and M0, which are not clobbers, are restored on every path
           to the end of the block from the registers that saved them, and
           those registers are not overwritten in between

``check_text(header_text)`` returns the violations (empty when clean) for
every variant; ``main`` prints them for node_loop_asm.h and exits non-zero
when there are any.
"""
from __future__ import annotations

import os
import re
import sys
from collections import defaultdict

TRANS_OPS = ("v_exp_f32", "v_log_f32", "v_rcp_f32", "v_rcp_iflag_f32", "v_rsq_f32",
             "v_sqrt_f32", "v_sin_f32", "v_cos_f32", "v_exp_f16", "v_log_f16", "v_rcp_f16",
             "v_rsq_f16", "v_sqrt_f16", "v_sin_f16", "v_cos_f16", "v_rcp_f64", "v_rsq_f64",
             "v_sqrt_f64")

# Instructions whose first operand is read, not written.
NO_DST = ("s_cmp", "s_cbranch", "s_branch", "s_setpc", "s_waitcnt", "s_nop", "s_set_gpr_idx",
          "ds_write", "global_store", "global_load_lds", "buffer_store")


class Inst:
    def __init__(self, idx, text):
        self.idx = idx
        self.text = text
        parts = text.split(None, 1)
        self.op = parts[0]
        rest = parts[1] if len(parts) > 1 else ""
        self.args = [a.strip() for a in rest.split(",")] if rest else []
        self.label = text[:-1] if text.endswith(":") else None
        self.directive = text.startswith(".")

    # ---- classification
    @property
    def is_code(self):
        return not (self.label or self.directive)

    @property
    def base(self):
        return re.sub(r"_e(32|64)$", "", self.op)

    @property
    def is_valu(self):
        return self.is_code and self.op.startswith("v_")

    @property
    def is_trans(self):
        return self.is_valu and self.base in TRANS_OPS

    @property
    def is_smem(self):
        return self.is_code and (self.op.startswith("s_load") or
                                 self.op.startswith("s_buffer_load"))

    @property
    def is_ds(self):
        return self.is_code and self.op.startswith("ds_")

    @property
    def is_vmem(self):
        return self.is_code and self.op.split("_")[0] in ("global", "buffer", "flat", "scratch")

    @property
    def is_lds_dma(self):
        return self.is_code and self.op.startswith("global_load_lds")

    @property
    def is_salu(self):
        return self.is_code and self.op.startswith("s_") and not self.is_smem

    @property
    def is_dpp(self):
        return self.is_valu and ("row_" in self.text or "quad_perm" in self.text or
                                 "_dpp" in self.op)

    def wait_states(self):
        if not self.is_code:
            return 0
        if self.op == "s_nop":
            return int(self.args[0], 0) + 1
        return 1

    # ---- operands
    def dst_operands(self):
        if not self.is_code or not self.args or self.op.startswith(NO_DST):
            return []
        if self.op.startswith("v_cmp") and not self.op.startswith("v_cmpx"):
            # VOP3 compares write the SGPR pair named first; VOPC ones VCC
            return [self.args[0]] if self.op.endswith("_e64") else ["vcc"]
        return [self.args[0]]

    def src_operands(self):
        if not self.is_code:
            return []
        d = self.dst_operands()
        srcs = self.args[len(d):] if d else list(self.args)
        # accumulating forms also read their destination
        if self.base in ("v_fmac_f32", "v_mac_f32") or self.op.startswith("s_addc") or \
                self.op.startswith("s_subb"):
            srcs = srcs + d
        # drop modifiers after an operand ("s[46:47] nt", "v1 offset:4")
        srcs = [s.split()[0] for s in srcs if s]
        return [s for s in srcs if not s.startswith(("offset", "gpr_idx")) and s != "off"]


def regs_of(operand):
    """Architectural registers named by an operand: 'v12' -> {'v12'},
    'v[74:75]' -> {'v74', 'v75'}, 's[40:55]', 'exec' -> {'exec_lo',
    'exec_hi'}, 'vcc', 'm0'; modifiers (-, |..|) are ignored; constants and
    inline-asm operands give nothing."""
    o = operand.strip().lstrip("-").strip("|")
    m = re.fullmatch(r"([vs])(\d+)", o)
    if m:
        return {o}
    m = re.fullmatch(r"([vs])\[(\d+):(\d+)\]", o)
    if m:
        return {"%s%d" % (m.group(1), i) for i in range(int(m.group(2)), int(m.group(3)) + 1)}
    if o == "exec":
        return {"exec_lo", "exec_hi"}
    if o == "vcc":
        return {"vcc_lo", "vcc_hi"}
    if o in ("m0", "exec_lo", "exec_hi", "vcc_lo", "vcc_hi", "scc"):
        return {o}
    return set()


def defs(inst):
    out = set()
    for o in inst.dst_operands():
        out |= regs_of(o)
    if inst.op in ("s_set_gpr_idx_on", "s_set_gpr_idx_idx"):
        out.add("m0")
    if inst.op.startswith(("s_cmp", "s_add", "s_sub", "s_and", "s_or", "s_lshl", "s_lshr",
                           "s_cselect")) and not inst.op.startswith("s_cselect"):
        out.add("scc")
    return out


def uses(inst):
    out = set()
    for o in inst.src_operands():
        out |= regs_of(o)
    if inst.is_valu or inst.is_vmem or inst.is_ds:
        out |= {"exec_lo", "exec_hi"}
    if inst.is_lds_dma:
        out.add("m0")
    if inst.op.startswith(("s_cbranch_scc", "s_cselect", "s_addc", "s_subb")):
        out.add("scc")
    return out


# ------------------------------------------------------------------ parsing
def parse_header(text):
    """{variant: (instruction texts, clobber set, first scratch VGPR)}."""
    out = {}
    lines = text.splitlines()
    i = 0
    while i < len(lines):
        m = re.match(r"#define NEAT_TILE_(\w+) \\$", lines[i])
        if not m:
            i += 1
            continue
        name, body = m.group(1), []
        i += 1
        while i < len(lines) and lines[i].startswith('    "'):
            s = re.match(r'\s*"(.*)\\n"', lines[i]).group(1).strip()
            body.append(s.replace("%=", ""))
            i += 1
        out[name] = [body, None, None]
    for name in out:
        m = re.search(r"#define NEAT_CLOB_%s \\\n((?:    .*\n)+)" % name, text)
        out[name][1] = set(re.findall(r'"([^"]+)"', m.group(1)))
        m = re.search(r"#define NEAT_SCRATCH_%s (\d+)" % name, text)
        out[name][2] = int(m.group(1))
    return {k: tuple(v) for k, v in out.items()}


# Record words the node loop jumps on (program.h): the code word (field =
# activation slot 0..6, or 7 = end of the loop for the sentinel) and the
# pair-count word (field = aggregation entry 8..20, or 7 for the sentinel).
JUMP_WORDS = {"s40": "act", "s56": "act", "s43": "agg", "s59": "agg"}
TABLE_OF_BASE = {"s92": "A", "s94": "B"}
N_ACT_SLOTS, END_SLOT, N_SLOTS = 7, 7, 21


def build_cfg(insts):
    """Successors and predecessors of every instruction index; len(insts)
    is the exit.  A computed jump (s_lshr of a record word, s_add of a
    table base, s_setpc) reaches the slots of that table its word can
    select: activation slots and the end for the code word, the end and
    the aggregation entries for the pair-count word."""
    labels = {ins.label: ins.idx for ins in insts if ins.label}
    # table slot starts: the first instruction of each slot (slot 0 follows
    # the Ltab label, the others follow their alignment directive)
    tables = {}
    cur = None
    for k, ins in enumerate(insts):
        if ins.label and ins.label.startswith("Ltab_"):
            cur = ins.label[5]
            tables[cur] = [k]
        elif ins.label and ins.label.startswith(("Lov", "Ldone")):
            cur = None
        elif cur and ins.directive and ins.op == ".p2align" and \
                not (insts[k + 1].label or "").startswith("Ltab"):
            tables[cur].append(k)
    for t, sl in tables.items():
        assert len(sl) == N_SLOTS, "table %s has %d slots" % (t, len(sl))
    n = len(insts)
    succ = defaultdict(set)
    for k, ins in enumerate(insts):
        if ins.op == "s_branch":
            succ[k].add(labels[ins.args[0]])
        elif ins.op.startswith("s_cbranch"):
            succ[k].add(labels[ins.args[0]])
            succ[k].add(k + 1)
        elif ins.op == "s_setpc_b64":
            shr, add = insts[k - 3], insts[k - 2]
            assert shr.op == "s_lshr_b32" and add.op == "s_add_u32", ins.text
            kind = JUMP_WORDS[shr.args[1]]
            slots = tables[TABLE_OF_BASE[add.args[2]]]
            pick = (list(range(N_ACT_SLOTS)) + [END_SLOT] if kind == "act"
                    else [END_SLOT] + list(range(END_SLOT + 1, N_SLOTS)))
            succ[k].update(slots[j] for j in pick)
        else:
            succ[k].add(k + 1 if k + 1 <= n else n)
    pred = defaultdict(set)
    for k, ss in succ.items():
        for s in ss:
            pred[s].add(k)
    return succ, pred, labels


# ------------------------------------------------------------------ checks
def _back_hazard(insts, pred, k, need, is_def):
    """A producer p on some path before instruction k (is_def(p)) with
    fewer than `need` wait states between them; returns it or None."""
    seen = {}
    stack = [(q, 0) for q in pred[k]]
    while stack:
        q, ws = stack.pop()
        if q < 0 or q >= len(insts):
            continue
        ins = insts[q]
        if is_def(ins):
            return ins, ws
        ws2 = ws + ins.wait_states()
        if ws2 >= need:
            continue
        if seen.get(q, need + 1) <= ws:
            continue
        seen[q] = ws
        stack.extend((p, ws2) for p in pred[q])
    return None


def check_wait_states(insts, pred):
    out = []
    for ins in insts:
        if not ins.is_code:
            continue
        u = uses(ins)
        rules = []
        if ins.is_valu and not ins.is_trans:
            rules.append(("TRANS", 1, lambda p, u=u: p.is_trans and (defs(p) & u)))
        if ins.op == "s_set_gpr_idx_on":
            rules.append(("IDXTRANS", 2, lambda p: p.is_trans))
        if ins.is_vmem:
            rules.append(("SGPRVMEM", 5, lambda p, u=u: p.is_valu and any(
                r.startswith("s") for r in defs(p) & u)))
        if ins.op.startswith(("v_readlane", "v_writelane")):
            sel = regs_of(ins.args[-1])
            rules.append(("LANESEL", 4, lambda p, sel=sel: p.is_valu and (defs(p) & sel)))
        if ins.is_lds_dma:
            rules.append(("M0LDS", 1, lambda p: p.is_salu and "m0" in defs(p)))
        if ins.is_dpp:
            rules.append(("DPP", 2, lambda p, u=u: p.is_valu and (defs(p) & u)))
            rules.append(("DPP", 5, lambda p: p.is_valu and (defs(p) & {"exec_lo", "exec_hi"})))
        if ins.is_valu and ("vccz" in ins.text or "execz" in ins.text):
            rules.append(("EXECZ", 5, lambda p: p.is_valu and (defs(p) & {
                "vcc_lo", "vcc_hi", "exec_lo", "exec_hi"})))
        for name, need, fn in rules:
            hit = _back_hazard(insts, pred, ins.idx, need, fn)
            if hit:
                out.append("%s: '%s' -> '%s' with %d of %d wait states"
                           % (name, hit[0].text, ins.text, hit[1], need))
    return out


def _fixpoint(insts, succ, init, step, join):
    """Forward data flow: state at each instruction's entry."""
    state = {0: init}
    work = [0]
    while work:
        k = work.pop()
        if k >= len(insts):
            continue
        s_out = step(insts[k], state[k])
        for t in succ[k]:
            new = s_out if t not in state else join(state[t], s_out)
            if t not in state or new != state[t]:
                state[t] = new
                work.append(t)
    return state


def check_outstanding_loads(insts, succ):
    out = []

    def step(ins, pend):
        if not ins.is_code:
            return pend
        if ins.op == "s_waitcnt" and "lgkmcnt(0)" in ins.text:
            pend = frozenset()
        touched = (uses(ins) | defs(ins)) - {"exec_lo", "exec_hi", "scc", "m0"}
        if touched & pend:
            kind = {r[0] for r in touched & pend}
            out.append("%s: '%s' touches %s before its load completed"
                       % ("SMEM" if "s" in kind else "DS", ins.text,
                          ",".join(sorted(touched & pend))))
        if ins.is_smem or (ins.is_ds and ins.op.startswith("ds_read")):
            pend = pend | frozenset(defs(ins))
        return pend

    _fixpoint(insts, succ, frozenset(), step, lambda a, b: a | b)
    return sorted(set(out))


def check_index_mode(insts, succ, clob_first_scratch, value_bases):
    """Index-mode state machine; value_bases: {base VGPR number: slots}."""
    out = []
    conflict = "conflict"

    def step(ins, mode):
        if mode == conflict or not ins.is_code:
            return mode
        if ins.op == "s_set_gpr_idx_on":
            if mode:
                out.append("IDXMODE: '%s' with the mode already on" % ins.text)
            return "SRC0" if "SRC0" in ins.text else "DST"
        if ins.op == "s_set_gpr_idx_idx":
            if not mode:
                out.append("IDXMODE: '%s' with the mode off" % ins.text)
            return mode
        if ins.op == "s_set_gpr_idx_off":
            if not mode:
                out.append("IDXMODE: '%s' with the mode off" % ins.text)
            return None
        if not mode:
            return mode
        if not ins.is_valu:
            out.append("IDXMODE: '%s' inside %s mode" % (ins.text, mode))
            return mode
        if ins.is_trans:
            out.append("IDXMODE: transcendental '%s' inside %s mode" % (ins.text, mode))
        if mode == "SRC0":
            src0 = ins.src_operands()[0] if ins.src_operands() else ""
            r = regs_of(src0)
            if len(r) != 1 or not next(iter(r)).startswith("v") or \
                    int(next(iter(r))[1:]) not in value_bases:
                out.append("IDXMODE: src0 of '%s' is not a value-vector base" % ins.text)
        else:
            d = regs_of(ins.dst_operands()[0]) if ins.dst_operands() else set()
            r = int(next(iter(d))[1:]) if len(d) == 1 and next(iter(d))[0] == "v" else -1
            inside = any(b <= r < b + n for b, n in value_bases.items())
            if not ins.op.startswith("v_mov_b32") or not inside:
                out.append("IDXMODE: '%s' in DST mode is not a move into a value vector"
                           % ins.text)
        return mode

    def join(a, b):
        if a == b:
            return a
        out.append("IDXMODE: paths join with modes %s and %s" % (a, b))
        return conflict

    _fixpoint(insts, succ, None, step, join)
    for base, slots in value_bases.items():
        if base + slots > clob_first_scratch and not any(
                base < b for b in value_bases if b != base):
            out.append("IDXRANGE: value vector v%d + %d slots reaches the scratch registers"
                       % (base, slots))
    bases = sorted(value_bases)
    for a, b in zip(bases, bases[1:]):
        if a + value_bases[a] > b:
            out.append("IDXRANGE: value vectors v%d and v%d overlap" % (a, b))
    if bases and bases[-1] + value_bases[bases[-1]] > clob_first_scratch:
        out.append("IDXRANGE: the last value vector reaches the scratch registers")
    return sorted(set(out))


def check_registers(insts, succ, clobbers):
    out = []
    for ins in insts:
        if not ins.is_code:
            continue
        for o in ins.dst_operands():
            if o.startswith("%["):
                out.append("CLOBBER: '%s' writes the input operand %s" % (ins.text, o))
        for r in defs(ins):
            if r[0] in "vs" and r[1:].isdigit() and r not in clobbers:
                out.append("CLOBBER: '%s' writes %s, not a clobber" % (ins.text, r))

    # EXEC and M0: saved copies and restoration on every path to the exit
    def step(ins, st):
        saved_exec, saved_m0, dirty = st
        if not ins.is_code:
            return st
        d = defs(ins)
        srcs = [regs_of(s) for s in ins.src_operands()]
        if ins.op == "s_mov_b64" and regs_of(ins.args[1]) == {"exec_lo", "exec_hi"}:
            saved_exec = frozenset(regs_of(ins.args[0]))
        elif ins.op == "s_mov_b32" and ins.args[1] == "m0":
            saved_m0 = frozenset(regs_of(ins.args[0]))
        else:
            if saved_exec & d:
                saved_exec = frozenset()
            if saved_m0 & d:
                saved_m0 = frozenset()
        dirty = set(dirty)
        if d & {"exec_lo", "exec_hi"}:
            if ins.op == "s_mov_b64" and srcs and srcs[0] == saved_exec and saved_exec:
                dirty.discard("exec")
            else:
                dirty.add("exec")
        if "m0" in d:
            if ins.op == "s_mov_b32" and srcs and srcs[0] == saved_m0 and saved_m0:
                dirty.discard("m0")
            else:
                dirty.add("m0")
        return (saved_exec, saved_m0, frozenset(dirty))

    def join(a, b):
        return (a[0] & b[0], a[1] & b[1], a[2] | b[2])

    st = _fixpoint(insts, succ, (frozenset(), frozenset(), frozenset()), step, join)
    end = st.get(len(insts))
    if end is None:
        out.append("RESTORE: the block has no path to its end")
    else:
        for r in sorted(end[2]):
            out.append("RESTORE: %s is not restored on some path to the end" % r)
    return sorted(set(out))


VALUE_SLOTS = {"S1_64": {0: 64}, "S2_64": {0: 64, 64: 64}, "S1_128": {0: 128},
               "S1_224": {0: 224}, "S1_64R": {0: 64, 64: 64}}


def check_variant(name, body, clobbers, scratch):
    insts = [Inst(k, t) for k, t in enumerate(body)]
    succ, pred, _ = build_cfg(insts)
    out = []
    out += check_wait_states(insts, pred)
    out += check_outstanding_loads(insts, succ)
    out += check_index_mode(insts, succ, scratch, VALUE_SLOTS.get(name, {0: scratch}))
    out += check_registers(insts, succ, clobbers)
    return ["%s: %s" % (name, v) for v in out]


def check_text(text):
    out = []
    for name, (body, clobbers, scratch) in parse_header(text).items():
        out += check_variant(name, body, clobbers, scratch)
    return out


def main(argv):
    here = os.path.dirname(os.path.abspath(__file__))
    path = argv[1] if len(argv) > 1 else os.path.join(here, "node_loop_asm.h")
    v = check_text(open(path).read())
    for line in v:
        print(line)
    print("%d violation(s)" % len(v))
    return 1 if v else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
