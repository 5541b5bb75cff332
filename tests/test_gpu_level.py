"""GPU: the level mapping (NEAT_FWD_LVL, lanes over a level's nodes x a tile
of samples) against the lane-per-sample stores bit for bit, and the segment
mapping (NEAT_FWD_SEG, lanes over a level's in-edges, segmented reduction)
against the oracle; both within the parity rule, over every slot class,
aggregation and activation, tile widths from 1 to 64 samples, ragged tiles,
long in-edge lists and rejected genomes."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.parity import assert_parity
from workloads import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _neat():
    import paper_2404_01817_amd as neat
    return neat


def _same_bits(a, b):
    nan = np.isnan(a)
    return np.array_equal(nan, np.isnan(b)) and np.array_equal(a[~nan].view(np.uint32),
                                                                 b[~nan].view(np.uint32))


def _pop(seed, P, N, B):
    rng = np.random.default_rng(seed)
    return synth.uneven_population(rng, (P, P), (N, N), (B, B))


def _run(pop, variant):
    neat = _neat()
    dev = torch.device("cuda:0")
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    _, _, _, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    y = neat.forward(d, prog, tx, pop.B, variant=variant)
    torch.cuda.synchronize()
    return y.cpu().numpy()


# (P, N_max, B): N_max 12..62 are R64 genomes, 100..250 reach the 128- and
# 224-register classes, 400 and 600 the LDS-row class; B from 1 to 300
# covers tile widths 1..64 and ragged last tiles
SHAPES = [(40, 12, 1), (33, 30, 3), (50, 62, 17), (21, 100, 63), (17, 150, 64),
          (9, 250, 100), (6, 400, 5), (4, 600, 33), (30, 45, 300), (25, 80, 2)]


@pytest.mark.parametrize("P,N,B", SHAPES, ids=["P%dN%dB%d" % s for s in SHAPES])
def test_level_mapping_matches_stores_and_oracle(P, N, B):
    neat = _neat()
    pop = _pop(1000 + N + B, P, N, B)
    print("level mapping P=%d N_max=%d B=%d I=%d O=%d" % (P, N, B, pop.I, pop.O), flush=True)
    y = _run(pop, neat.FWD_LVL)
    ref = _run(pop, neat.FWD_REG)
    assert _same_bits(y, ref)
    y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
    assert_parity(y, y64, beta, "lvl P%d N%d B%d" % (P, N, B))
    ys = _run(pop, neat.FWD_SEG)
    assert_parity(ys, y64, beta, "seg P%d N%d B%d" % (P, N, B))
    # maxima and minima are exact in any order: those outputs' nodes aside,
    # the two mappings differ only by rounding
    assert np.array_equal(np.isnan(ys), np.isnan(y))


def test_level_mapping_every_activation_and_aggregation():
    """One population per (activation, aggregation) pair, so every node
    block and every aggregation class runs in the level mapping."""
    neat = _neat()
    rng = np.random.default_rng(7)
    for act in range(7):
        for agg in range(5):
            pop = synth.make_population(rng, 24, 40, 160, 5, 3, 30, synth._k_uniform(160),
                                        (act,), (agg,))
            pop.inputs = rng.standard_normal((24, 9, 5), dtype=np.float32)
            y = _run(pop, neat.FWD_LVL)
            assert _same_bits(y, _run(pop, neat.FWD_REG)), (act, agg)
            y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
            assert_parity(y, y64, beta, "act %d agg %d" % (act, agg))
            ys = _run(pop, neat.FWD_SEG)
            assert_parity(ys, y64, beta, "seg act %d agg %d" % (act, agg))
            if agg in (2, 3):  # max and min: exact in any order
                assert _same_bits(ys, y), (act, agg)


def test_level_mapping_rejected_genomes_and_shared_inputs():
    """Rejected genomes give NaN rows; shared inputs (stride 0) are read by
    every genome."""
    neat = _neat()
    pop = _pop(77, 30, 70, 11)
    pop.nodes[3, 0, 0] = 2.5          # a non-integer input key: BAD_VALUE
    pop.conns[5, :, :] = pop.conns[5, 0, :]  # duplicated enabled edges / refs
    y = _run(pop, neat.FWD_LVL)
    assert np.isnan(y[3]).all()
    assert _same_bits(y, _run(pop, neat.FWD_REG))
    ys = _run(pop, neat.FWD_SEG)
    assert np.isnan(ys[3]).all()
    y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
    assert_parity(y, y64, beta, "rejected")
    assert_parity(ys, y64, beta, "rejected, segment mapping")
    dev = torch.device("cuda:0")
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    x = pop.inputs[0]
    tx = torch.from_numpy(x).to(dev)
    _, _, _, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    ysh = neat.forward(d, prog, tx, pop.B, shared_inputs=True, variant=neat.FWD_LVL)
    yr = neat.forward(d, prog, tx, pop.B, shared_inputs=True, variant=neat.FWD_REG)
    yg = neat.forward(d, prog, tx, pop.B, shared_inputs=True, variant=neat.FWD_SEG)
    torch.cuda.synchronize()
    assert _same_bits(ysh.cpu().numpy(), yr.cpu().numpy())
    y64, beta = oracle.forward(pop.nodes, pop.conns, x, pop.I, pop.O, shared_inputs=True)
    assert_parity(yg.cpu().numpy(), y64, beta, "shared inputs, segment mapping")


def test_level_mapping_in_a_batch_after_tuning():
    """Autotuning a small-B bucket may record the level mapping; a recorded
    batch is rebuilt after the table changes and its outputs keep the same
    bits as the untuned single calls."""
    neat = _neat()
    dev = torch.device("cuda:0")
    pops = [_pop(200 + k, P, N, B) for k, (P, N, B) in enumerate(((300, 200, 2), (200, 60, 4),
                                                                   (100, 120, 90)))]
    bufs, refs = [], []
    for pop in pops:
        tn = torch.from_numpy(pop.nodes).to(dev)
        tc = torch.from_numpy(pop.conns).to(dev)
        tx = torch.from_numpy(pop.inputs).to(dev)
        _, _, _, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
        d = neat.dims_of(tn, tc, pop.I, pop.O)
        y = torch.full((pop.P, pop.B, pop.O), 7.0, device=dev)
        bufs.append((pop, d, prog, tx, y))
        refs.append(_run(pop, neat.FWD_AUTO))
    plan = neat.BatchPlan()
    items = [neat.batch_item(d, prog, y, inputs=tx, B=pop.B) for pop, d, prog, tx, y in bufs]
    plan.run(items)
    torch.cuda.synchronize()
    n0 = plan.launches
    tuned = []
    for pop, d, prog, tx, y in bufs[:2]:
        v, ms = neat.autotune_forward(d, prog, tx, pop.B, reps=3)
        tuned.append((v, ms))
    print("tuned", tuned, flush=True)
    for _ in range(2):
        for pop, d, prog, tx, y in bufs:
            y.fill_(7.0)
        plan.run(items)
        torch.cuda.synchronize()
        for (pop, d, prog, tx, y), r in zip(bufs, refs):
            if neat.tuned_variant(d, pop.B, throughput=True) == neat.FWD_SEG:
                y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
                assert_parity(y.cpu().numpy(), y64, beta, "batch item, segment mapping")
            else:
                assert _same_bits(y.cpu().numpy(), r)
    print("launches before and after tuning", n0, plan.launches, flush=True)
    plan.free()
    neat.tune_clear()  # later tests compare untuned bits


def test_segment_mapping_long_in_edge_lists():
    """Nodes with long in-edge lists (segments cut by the end of a step and
    continued through the carry, overflow edges past the record) and levels
    of more than 64 nodes, with one and with eight samples per tile."""
    neat = _neat()
    rng = np.random.default_rng(91)
    for B in (1, 8, 40):
        pop = synth.make_population(rng, 6, 300, 2400, 8, 4, 288,
                                    lambda r, na: min(2400, na), synth.CONTROL_ACTS,
                                    synth.ALL_AGGS)
        pop.inputs = rng.standard_normal((6, B, 8), dtype=np.float32)
        ys = _run(pop, neat.FWD_SEG)
        y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
        assert_parity(ys, y64, beta, "seg long lists B=%d" % B)
        assert _same_bits(_run(pop, neat.FWD_LVL), _run(pop, neat.FWD_REG))
    # wide levels: few connections among many nodes, so most of the 580
    # hidden nodes sit on levels 0 and 1 (more than 64 nodes per level)
    pop = synth.make_population(rng, 4, 600, 600, 8, 4, 580, lambda r, na: min(300, na),
                                synth.CONTROL_ACTS, synth.ALL_AGGS)
    pop.inputs = rng.standard_normal((4, 3, 8), dtype=np.float32)
    _, level, _ = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O)
    assert max(np.bincount(lv[lv >= 0]).max() for lv in level) > 64
    ys = _run(pop, neat.FWD_SEG)
    y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
    assert_parity(ys, y64, beta, "seg wide levels")
    assert_parity(_run(pop, neat.FWD_LVL), y64, beta, "lvl wide levels")
