"""CPU: static checks of the generated node-loop assembly.

The forward kernels' tile blocks are inline assembly, outside the
compiler's hazard recognizer.  csrc/check_node_loop.py rebuilds each
block's control flow (including the node loop's computed jumps into its
table slots) and checks the documented wait states, the completion of
scalar and LDS loads before their registers are touched, GPR-index mode,
clobbers and the restoration of EXEC and M0.  These tests run it on the
committed header, pin every rule with a planted mistake, and run it on the
register placement that was rejected after it gave unrepeatable sine
results on the GPU."""
from __future__ import annotations

import importlib.util
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_01817_amd", "csrc")
HEADER = os.path.join(CSRC, "node_loop_asm.h")


def _load(name):
    spec = importlib.util.spec_from_file_location(name, os.path.join(CSRC, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod
    spec.loader.exec_module(mod)
    return mod


check = _load("check_node_loop")
gen = _load("gen_node_loop")


def _text():
    return open(HEADER).read()


def _block(text, name):
    """(start, end) of one variant's tile block in the header text."""
    a = text.index("#define NEAT_TILE_%s \\" % name)
    b = text.index("#define NEAT_CLOB_%s" % name)
    return a, b


def _edit(text, name, old, new, count=1):
    a, b = _block(text, name)
    blk = text[a:b]
    assert old in blk, old
    return text[:a] + blk.replace(old, new, count) + text[b:]


def _rules(violations):
    return {v.split(": ")[1] for v in violations}


def test_generated_header_is_current_and_clean():
    assert gen.generate() == _text(), "node_loop_asm.h differs from gen_node_loop.py's output"
    v = check.check_text(_text())
    assert v == [], "\n".join(v)
    assert set(check.parse_header(_text())) == {"S1_64", "S2_64", "S1_128", "S1_224", "S1_64R"}


PLANTS = [
    # a transcendental's result read by the next instruction (tanh, one
    # sample per lane: the nop after v_exp removed)
    ("TRANS", "S1_64", '"  v_exp_f32_e32 v65, v65\\n" \\\n    "  s_nop 0\\n"',
     '"  v_exp_f32_e32 v65, v65\\n"'),
    # no wait states between v_rcp and the switch into indexed mode (sigmoid)
    ("IDXTRANS", "S1_64", '"  v_rcp_f32_e32 v65, v66\\n" \\\n    "  s_nop 1\\n"',
     '"  v_rcp_f32_e32 v65, v66\\n"'),
    # the next record read before its load completed: an activation block's
    # wait removed
    ("SMEM", "S1_64", '"  s_set_gpr_idx_off\\n" \\\n    "  s_waitcnt lgkmcnt(0)\\n" \\\n'
                      '    "  s_lshr_b32 s88, s59',
     '"  s_set_gpr_idx_off\\n" \\\n    "  s_lshr_b32 s88, s59'),
    # input buffers moved before their LDS reads completed
    ("DS", "S1_64", '"  v_add_u32_e32 v72, 32, v72\\n" \\\n    "  s_waitcnt lgkmcnt(0)\\n"',
     '"  v_add_u32_e32 v72, 32, v72\\n"'),
    # indexed mode left on after an edge pair
    ("IDXMODE", "S1_64", '"  v_fmac_f32_e64 v64, v0, s47\\n" \\\n    "  s_set_gpr_idx_off\\n"',
     '"  v_fmac_f32_e64 v64, v0, s47\\n"'),
    # EXEC not restored after the masked DMA rounds
    ("RESTORE", "S1_64", '"  s_mov_b64 exec, s[42:43]\\n"', '"  s_nop 0\\n"', 2),
    # M0 written right before the LDS DMA that reads it
    ("M0LDS", "S1_64", '"  s_nop 0\\n" \\\n    "  global_load_lds_dwordx4',
     '"  s_mov_b32 m0, %[dm0]\\n" \\\n    "  global_load_lds_dwordx4'),
    # a VALU write of an SGPR that the DMA load then reads
    ("SGPRVMEM", "S1_64", '"  s_nop 0\\n" \\\n    "  global_load_lds_dwordx4 v[74:75], off nt\\n"',
     '"  v_readfirstlane_b32 s46, v74\\n" \\\n'
     '    "  global_load_lds_dwordx4 v[74:75], s[46:47] nt\\n"'),
    # a register the block writes left out of its clobbers
    ("CLOBBER", None, None, None),
]


@pytest.mark.parametrize("rule,variant,old,new,count", [p if len(p) == 5 else p + (1,)
                                                        for p in PLANTS],
                         ids=[p[0] for p in PLANTS])
def test_planted_mistake_is_found(rule, variant, old, new, count):
    text = _text()
    if rule == "CLOBBER":
        a = text.index("#define NEAT_CLOB_S1_64 \\")
        b = text.index("#define NEAT_SCRATCH_S1_64")
        text = text[:a] + text[a:b].replace('"s87", ', "", 1) + text[b:]
    else:
        text = _edit(text, variant, old, new, count)
    v = check.check_text(text)
    assert any(x.split(": ")[1] == rule for x in v), (rule, v[:5])


def test_rejected_register_placement_is_clean_too():
    """The placement that gave unrepeatable sine results on the GPU (c13
    first, then acc, z, ta, tb, p) breaks none of the checked rules either:
    the two placements differ only in register numbers, so the cause is not
    one of the documented wait-state, load-completion, index-mode or
    clobber rules."""

    class Rejected(gen.Regs):
        def __init__(self, spl, bases, scratch, wbases=None, group=8):
            super().__init__(spl, bases, scratch, wbases, group)
            self.c13 = "v%d" % scratch
            for k, role in enumerate(("acc", "z", "ta", "tb")):
                self.names[role] = ["v%d" % (scratch + 1 + k * spl + h) for h in range(spl)]
            self.names["p"] = ["v%d" % (scratch + 1 + 4 * spl + h) for h in range(spl)]

    saved = gen.Regs
    try:
        gen.Regs = Rejected
        text = gen.generate()
    finally:
        gen.Regs = saved
    assert text != _text()
    assert check.check_text(text) == []
