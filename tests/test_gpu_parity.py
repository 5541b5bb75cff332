"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Topological orders, levels and status words must match bit for bit; fp32
outputs must satisfy the parity rule of ``oracle.within_tolerance``
(|y - y64| <= 1e-5 + 2 beta, NaN where the oracle is NaN)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.parity import assert_parity
from workloads import synth
from tests.helpers import genome, read_golden, stack

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _neat():
    import paper_2404_01817_amd as neat
    return neat


def _gpu(nodes, conns, I, O, x=None, shared=False, grid=None, variant=0):
    """Run transformation (+ calculation) on cuda:0; numpy results."""
    neat = _neat()
    dev = torch.device("cuda:0")
    tn = torch.from_numpy(np.ascontiguousarray(nodes)).to(dev)
    tc = torch.from_numpy(np.ascontiguousarray(conns)).to(dev)
    order, level, status, prog = neat.topo_sort(tn, tc, I, O)
    y = None
    d = neat.dims_of(tn, tc, I, O)
    if x is not None:
        tx = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        B = x.shape[0] if shared else x.shape[1]
        y = neat.forward(d, prog, tx, B, shared_inputs=shared, variant=variant)
    elif grid is not None:
        side, first, Q = grid
        y = neat.forward_grid(d, prog, side, first, Q)
    torch.cuda.synchronize()
    out = (order.cpu().numpy(), level.cpu().numpy(),
           status.cpu().numpy().astype(np.uint32))
    return out + ((y.cpu().numpy() if y is not None else None),)


def _assert_transform_exact(nodes, conns, I, O, g_order, g_level, g_status):
    o_order, o_level, o_status = oracle.transform(nodes, conns, I, O)
    bad = np.nonzero(o_status != g_status)[0]
    assert len(bad) == 0, "status differs at genomes %s: oracle %s gpu %s" % (
        bad[:5], o_status[bad[:5]], g_status[bad[:5]])
    assert np.array_equal(o_order, g_order)
    assert np.array_equal(o_level, g_level)


def _assert_outputs(y_gpu, y64, beta, label=""):
    stats = assert_parity(y_gpu, y64, beta, label)
    return stats


def test_golden_hand_network_exact():
    g = read_golden("hand_net.txt")
    order, level, status, y = _gpu(g["nodes_arr"], g["conns_arr"], g["I"], g["O"],
                                   g["x"][None])
    assert status[0] == 0
    assert oracle.order_keys(g["nodes_arr"], order)[0][:6].tolist() == g["order"]
    assert np.array_equal(y[0].astype(np.float64), g["y"])


def test_status_corpus_bit_exact():
    from tests.test_oracle_pins import CORPUS, _base
    gens = []
    for _, fn, _ in CORPUS:
        nodes, conns = _base()
        fn(nodes, conns)
        gens.append(genome(8, 10, nodes, conns))
    n, c = stack(gens)
    x = np.random.default_rng(0).standard_normal((len(gens), 5, 2)).astype(np.float32)
    order, level, status, y = _gpu(n, c, 2, 1, x)
    _assert_transform_exact(n, c, 2, 1, order, level, status)
    assert status.tolist() == [e for _, _, e in CORPUS]
    y64, beta = oracle.forward(n, c, x, 2, 1)
    _assert_outputs(y, y64, beta, "corpus")
    assert np.isnan(y[status != 0]).all()


def test_tiny_config():
    """P=16, N_max=8, C_max=16, sigmoid + sum, 32 shared inputs."""
    pop = synth.tiny()
    order, level, status, y = _gpu(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs, shared=True)
    _assert_transform_exact(pop.nodes, pop.conns, pop.I, pop.O, order, level, status)
    y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, shared_inputs=True)
    _assert_outputs(y, y64, beta, "tiny")


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("P,B", [(300, 130), (64, 64), (37, 1), (5, 191)])
def test_control_small_full_compare(P, B, variant):
    """Mixed activations/aggregations, several sample tiles and a ragged tail;
    both value stores (registers, LDS rows)."""
    pop = synth.control(seed=11 + P, P=P, B=B)
    order, level, status, y = _gpu(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs,
                                   variant=variant)
    _assert_transform_exact(pop.nodes, pop.conns, pop.I, pop.O, order, level, status)
    y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
    _assert_outputs(y, y64, beta, "control P=%d B=%d" % (P, B))


def test_control_full_size_sampled():
    """P=10000, B=1000 per-genome inputs in one launch: every genome's order,
    level and status, and all outputs of 150 sampled genomes."""
    pop = synth.control()
    order, level, status, y = _gpu(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs)
    _assert_transform_exact(pop.nodes, pop.conns, pop.I, pop.O, order, level, status)
    rng = np.random.default_rng(123)
    pick = np.sort(rng.choice(pop.P, 150, replace=False))
    pick = np.unique(np.concatenate([pick, [0, pop.P - 1]]))
    y64, beta = oracle.forward(pop.nodes[pick], pop.conns[pick], pop.inputs[pick], pop.I, pop.O)
    _assert_outputs(y[pick], y64, beta, "control full sampled")


def test_cppn_grid_queries():
    """CPPN genomes on 16x16 grid pairs, inputs generated in the kernel."""
    pop = synth.cppn(P=40)
    for first, Q in ((0, 65536), (1000, 777)):
        order, level, status, y = _gpu(pop.nodes, pop.conns, pop.I, pop.O, grid=(16, first, Q))
        _assert_transform_exact(pop.nodes, pop.conns, pop.I, pop.O, order, level, status)
        sub = slice(0, 8) if Q > 10000 else slice(None)
        x = synth.grid_queries(first, Q)
        y64, beta = oracle.forward(pop.nodes[sub], pop.conns[sub], x, pop.I, pop.O,
                                   shared_inputs=True)
        _assert_outputs(y[sub], y64, beta, "cppn first=%d Q=%d" % (first, Q))


def test_grid_inputs_match_generator():
    """A single identity network passes x1 through: the in-kernel grid
    coordinates equal the generator's fp32 values bit for bit."""
    for j in range(4):
        nodes = {i: (i, 0, 1, 0, 0) for i in range(5)}
        nodes[5] = (5, 0.0, 1.0, 0, 0)
        n, c = genome(6, 1, nodes, {0: (j, 5, 1, 1.0)})
        *_, y = _gpu(n, c, 5, 1, grid=(16, 0, 65536))
        assert np.array_equal(y[0, :, 0], synth.grid_queries()[:, j])


def _grid_reference(side, first, Q):
    """x1, y1, x2, y2 of queries first .. first+Q-1 (coordinates divided in
    fp32, as the definition rounds them)."""
    i = np.arange(side, dtype=np.float32)
    c = (np.float32(2) * i - np.float32(side - 1)) / np.float32(side - 1)
    q = np.arange(first, first + Q, dtype=np.int64)
    pts = side * side
    p1, p2 = q // pts, q % pts
    return np.stack([c[p1 % side], c[p1 // side], c[p2 % side], c[p2 // side]], axis=1)


@pytest.mark.parametrize("side,first,Q", [
    (2, 0, 16), (3, 0, 81), (5, 7, 600), (11, 0, 14641), (12, 100, 20000), (17, 0, 83521),
    (100, 0, 5000), (100, 10 ** 8 - 3000, 3000), (100, 12345678, 777),
    (256, 2 ** 32 - 1000, 1000), (256, 2 ** 31 + 5, 300), (256, 0, 70000)])
def test_grid_inputs_many_sides(side, first, Q):
    """Grid queries for small and large sides, partial tiles and the end of
    the query range: the four coordinates equal the definition bit for bit
    (identity networks pass each input through)."""
    gens = []
    for j in range(4):
        nodes = {i: (i, 0, 1, 0, 0) for i in range(5)}
        nodes[5] = (5, 0.0, 1.0, 0, 0)
        gens.append(genome(6, 1, nodes, {0: (j, 5, 1, 1.0)}))
    n, c = stack(gens)
    *_, y = _gpu(n, c, 5, 1, grid=(side, first, Q))
    ref = _grid_reference(side, first, Q)
    for j in range(4):
        assert np.array_equal(y[j, :, 0], ref[:, j]), (side, first, Q, j)


def test_uneven_populations():
    """Node counts up to 400 (multi-wave sort), I/O drawn per population."""
    pops = synth.uneven(seed=5, n_pops=6, P_range=(3, 40), N_range=(10, 400),
                        B_range=(1, 200))
    for pop in pops:
        order, level, status, y = _gpu(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs)
        _assert_transform_exact(pop.nodes, pop.conns, pop.I, pop.O, order, level, status)
        y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
        _assert_outputs(y, y64, beta, "uneven N=%d" % pop.N_max)


@pytest.mark.parametrize("N", [50, 300])
def test_planted_defects_status_bit_exact(N):
    """Duplicated keys, dangling references, edges into inputs and malformed
    values planted in every third genome, for node counts on both sides of
    the transformation's 256-row boundary: status, order and level match
    the oracle bit for bit."""
    rng = np.random.default_rng(N)
    pop = synth.make_population(rng, 60, N, 4 * N, 6, 3, N - 9, synth._k_density(4 * N),
                                synth.CONTROL_ACTS, synth.ALL_AGGS)
    nodes, conns = pop.nodes.copy(), pop.conns.copy()
    for g in range(0, 60, 3):
        rows = np.nonzero(~np.isnan(nodes[g, :, 0]))[0]
        kind = (g // 3) % 5
        if kind == 0:    # a hidden (or output) key repeated on another row
            nodes[g, rows[-1], 0] = nodes[g, rows[-2], 0]
        elif kind == 1:  # an input key repeated
            nodes[g, rows[-1], 0] = nodes[g, rows[0], 0]
        elif kind == 2:  # an enabled connection to a missing key
            c = np.nonzero(conns[g, :, 2] == 1.0)[0]
            if len(c):
                conns[g, c[0], 1] = 10 ** 6
        elif kind == 3:  # an edge into an input
            c = np.nonzero(~np.isnan(conns[g, :, 0]))[0]
            if len(c):
                conns[g, c[-1], 1] = 0.0
                conns[g, c[-1], 2] = 1.0
        else:            # a fractional key
            nodes[g, rows[-1], 0] = 7.5
    # every third genome from the second on: hidden keys moved to 2^22 and
    # above (valid keys; connections follow), the transformation's wide-key
    # ranking
    for g in range(1, 60, 3):
        hidden = nodes[g, :, 0] >= pop.I + pop.O
        nodes[g, hidden, 0] += 5000000.0
        for col in (0, 1):
            moved = conns[g, :, col] >= pop.I + pop.O
            conns[g, moved, col] += 5000000.0
    order, level, status, _ = _gpu(nodes, conns, pop.I, pop.O)
    _assert_transform_exact(nodes, conns, pop.I, pop.O, order, level, status)
    assert (status[0::3] != 0).all()
    assert (status[1::3] == 0).any()


def test_storage_invariants_bit_identical():
    """NaN padding rows, disabled junk rows and permuted storage give the
    same order (as keys) and bit-identical outputs on the GPU (N_max 50 -> 58
    keeps the value-slot layout, which fixes the summation order)."""
    pop = synth.control(seed=77, P=50, B=70)
    n, c, x, I, O = pop.nodes, pop.conns, pop.inputs, pop.I, pop.O
    o0, l0, s0, y0 = _gpu(n, c, I, O, x)
    rng = np.random.default_rng(3)
    n2 = np.full((50, 58, 5), np.nan, np.float32)
    c2 = np.full((50, 256, 4), np.nan, np.float32)
    n2[:, np.sort(rng.choice(58, 50, replace=False))] = n[:, rng.permutation(50)]
    c2[:, np.sort(rng.choice(256, 200, replace=False))] = c[:, rng.permutation(200)]
    junk = rng.standard_normal((50, 56, 4)).astype(np.float32) * 50
    junk[:, :, 2] = 0.0
    free = np.isnan(c2[:, :, 0])
    for p in range(50):
        rows = np.nonzero(free[p])[0][:56]
        c2[p, rows] = junk[p, :len(rows)]
    o2, l2, s2, y2 = _gpu(n2, c2, I, O, x)
    assert (s0 == 0).all() and (s2 == 0).all()
    assert np.array_equal(oracle.order_keys(n, o0)[:, :50], oracle.order_keys(n2, o2)[:, :50])
    assert np.array_equal(y0, y2)


def test_repeatable_bits():
    pop = synth.control(seed=8, P=200, B=100)
    a = _gpu(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs)
    b = _gpu(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("workload", ["control", "sine"])
def test_repeatable_bits_full_size(workload, variant):
    """Full-size populations (P=10000, B=1000), where thousands of waves
    share every compute unit: repeated launches give the same bits.  The
    sine workload makes every computed node a sine (the longest activation
    block)."""
    neat = _neat()
    if workload == "control":
        pop = synth.control()
    else:
        rng = np.random.default_rng(11)
        pop = synth.make_population(rng, 10000, 50, 200, 17, 6, 27, synth._k_uniform(200),
                                    (synth.ACT_SIN,), (synth.AGG_SUM,))
        pop.inputs = rng.standard_normal((10000, 1000, 17), dtype=np.float32)
    dev = torch.device("cuda:0")
    tn, tc = torch.from_numpy(pop.nodes).to(dev), torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    _, _, _, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    first = neat.forward(d, prog, tx, pop.inputs.shape[1], variant=variant).view(torch.int32)
    for rep in range(3):
        again = neat.forward(d, prog, tx, pop.inputs.shape[1], variant=variant)
        differ = int((again.view(torch.int32) != first).sum())
        print(workload, "variant", variant, "repeat", rep, "differing words", differ)
        assert differ == 0


def test_edge_cases():
    neat = _neat()
    dev = torch.device("cuda:0")
    # no hidden nodes, no connections: outputs are act(bias)
    nodes = {0: (0, 0, 1, 0, 0), 1: (1, 0.5, 1, 1, 0), 2: (2, -2.0, 1, 6, 3)}
    n, c = genome(3, 1, nodes, {})
    x = np.zeros((1, 3, 1), np.float32)
    order, level, status, y = _gpu(n, c, 1, 2, x)
    assert status[0] == 0 and order[0].tolist() == [0, 1, 2]
    assert np.allclose(y[0], [[np.tanh(0.5), 2.0]] * 3)
    # C_max = 0
    n0 = np.zeros((4, 3, 5), np.float32)
    n0[:] = n[0]
    c0 = np.zeros((4, 0, 4), np.float32)
    order, level, status, y = _gpu(n0, c0, 1, 2, np.zeros((4, 2, 1), np.float32))
    assert (status == 0).all() and np.allclose(y[:, :, 1], 2.0)
    # P = 0 and B = 0 are no-ops
    tn = torch.zeros((0, 8, 5), device=dev)
    tc = torch.zeros((0, 16, 4), device=dev)
    _, _, st_, prog = neat.topo_sort(tn, tc, 3, 1)
    pop = synth.tiny()
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    _, _, _, prog = neat.topo_sort(tn, tc, 3, 1)
    d = neat.dims_of(tn, tc, 3, 1)
    y = neat.forward(d, prog, torch.zeros((0, 3), device=dev), 0, shared_inputs=True)
    torch.cuda.synchronize()
    assert y.shape == (16, 0, 1)
    # invalid arguments are rejected before any launch
    with pytest.raises(neat.NeatError):
        neat.topo_sort(tn, tc, 8, 1)            # I + O > N_max
    with pytest.raises(neat.NeatError):
        neat._lib.check(neat.lib().neat_forward(None, None, None, 0, 4, None, None))


def test_all_genomes_rejected():
    pop = synth.control(seed=2, P=20, B=9)
    n = pop.nodes.copy()
    n[:, 0, 3] = 9.0      # bad activation code on every genome
    order, level, status, y = _gpu(n, pop.conns, pop.I, pop.O, pop.inputs)
    assert (status == 1).all() and (order == -1).all() and (level == -1).all()
    assert np.isnan(y).all()


# Shapes: inputs filling most of the 64-slot class, N_max around the class
# boundaries, and many outputs (live to the end) to force each slot class:
# O = 70 -> 128 register slots, O = 150 -> 224, O = 240 -> LDS rows.
SHAPES = [(30, 5, 2), (33, 5, 2), (60, 40, 3), (62, 20, 3), (63, 10, 4), (64, 10, 4),
          (48, 31, 1), (62, 45, 2), (8, 3, 1), (47, 29, 2), (100, 10, 70), (130, 60, 20),
          (200, 10, 150), (300, 20, 240)]


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("N,I,O", SHAPES)
def test_forward_kernel_shapes(N, I, O, variant):
    """Every value store and slot class: inputs spread over the value
    vector, the class boundaries, and outputs beyond one group of eight."""
    rng = np.random.default_rng(N * 100 + I)
    P, B, C = 40, 150, 4 * N
    nodes = np.full((P, N, 5), np.nan, np.float32)
    conns = np.full((P, C, 4), np.nan, np.float32)
    for p in range(P):
        h = int(rng.integers(0, N - I - O + 1))
        synth.make_genome(rng, N, C, I, O, h, lambda na: int(rng.integers(1, min(C, na) + 1)),
                          synth.CONTROL_ACTS, synth.ALL_AGGS, nodes_out=nodes[p],
                          conns_out=conns[p])
    x = rng.standard_normal((P, B, I)).astype(np.float32)
    order, level, status, y = _gpu(nodes, conns, I, O, x, variant=variant)
    _assert_transform_exact(nodes, conns, I, O, order, level, status)
    y64, beta = oracle.forward(nodes, conns, x, I, O)
    _assert_outputs(y, y64, beta, "shape N=%d I=%d O=%d variant=%d" % (N, I, O, variant))


@pytest.mark.parametrize("N", [50, 64])
def test_one_wave_genomes_with_long_connection_lists(N):
    """One-wave genomes (N_max <= 64) with C_max = 700 connection rows, more
    than the four rows per lane the transformation keeps in registers: rows
    256 and beyond go through LDS.  Duplicate edges are planted within the
    first 256 rows, within the rest and across the two ranges (a duplicate
    is the same source and destination keys on two enabled rows), and
    enabled rows are disabled at random; transformation bit-exact, outputs
    within the parity rule.  N_max = 64 also takes the liveness slots."""
    rng = np.random.default_rng(700 + N)
    P, B, C, I, O = 48, 70, 700, 9, 4
    nodes = np.full((P, N, 5), np.nan, np.float32)
    conns = np.full((P, C, 4), np.nan, np.float32)
    for p in range(P):
        synth.make_genome(rng, N, C, I, O, N - I - O,
                          lambda na: int(rng.integers(min(C, na) // 2, min(C, na) + 1)),
                          synth.CONTROL_ACTS, synth.ALL_AGGS, nodes_out=nodes[p],
                          conns_out=conns[p])
    # a few rows disabled first (their edges neither count nor duplicate)
    off = (rng.random((P, C)) < 0.05) & (conns[:, :, 2] == 1.0)
    conns[:, :, 2][off] = 0.0
    lo, hi = set(range(256)), list(range(256, C))
    for p in range(P):
        kind = p % 4
        if kind == 0:
            continue
        enabled = np.nonzero(conns[p, :, 2] == 1.0)[0]
        a = [r for r in enabled if (r in lo) == (kind in (1, 3))]
        dst_range = hi if kind in (1, 2) else sorted(lo)
        ra = a[0]
        rb = next(r for r in dst_range if r != ra)
        conns[p, rb, :3] = conns[p, ra, :3]
        conns[p, rb, 3] = conns[p, ra, 3] + 0.5
    x = rng.standard_normal((P, B, I)).astype(np.float32)
    order, level, status, y = _gpu(nodes, conns, I, O, x)
    _assert_transform_exact(nodes, conns, I, O, order, level, status)
    assert (status[0::4] == 0).all()
    assert all(status[k::4].astype(bool).all() for k in (1, 2, 3))
    assert all((status[k::4] & oracle.DUP_EDGE).all() for k in (1, 2, 3))
    y64, beta = oracle.forward(nodes, conns, x, I, O)
    _assert_outputs(y, y64, beta, "one-wave N=%d C=%d" % (N, C))


def test_wide_fan_in_every_aggregation():
    """Nodes with more incoming edges than the eight the forward keeps in
    registers (24 and 40 terms), for every aggregation."""
    for I in (24, 40):
        O = 5
        nodes = {i: (i, 0, 1, 0, 0) for i in range(I)}
        for j in range(O):
            nodes[I + j] = (I + j, 0.1 * j, 1.0, synth.ACT_TANH if j % 2 else 0, j)
        rng = np.random.default_rng(I)
        conns, r = {}, 0
        for j in range(O):
            for i in rng.permutation(I):
                conns[r] = (int(i), I + j, 1, float(rng.standard_normal() * 0.7))
                r += 1
        n, c = genome(I + O, r, nodes, conns)
        x = rng.uniform(0.5, 1.5, (1, 200, I)).astype(np.float32)
        order, level, status, y = _gpu(n, c, I, O, x)
        _assert_transform_exact(n, c, I, O, order, level, status)
        y64, beta = oracle.forward(n, c, x, I, O)
        _assert_outputs(y, y64, beta, "fan-in %d" % I)


def test_device_activations_accuracy():
    """Each activation on its own (one input -> one output, weight 1, bias 0)
    over a dense sweep: absolute error against the double-precision value
    stays within a few fp32 units in the last place (plus the rounding of
    the argument, which the bound beta carries)."""
    z = np.concatenate([np.linspace(-30, 30, 60001), np.linspace(-1e-3, 1e-3, 2001),
                        [0.0, -0.0, 1e-30, -1e-30, 88.0, -88.0, 100.0, -100.0, 1e4, -1e4,
                         np.inf, -np.inf, np.nan]]).astype(np.float32)
    gens = []
    for act in range(7):
        gens.append(genome(2, 1, {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, act, 0)},
                           {0: (0, 1, 1, 1.0)}))
    n, c = stack(gens)
    order, level, status, y = _gpu(n, c, 1, 1, z[:, None], shared=True)
    y64, beta = oracle.forward(n, c, z[:, None], 1, 1, shared_inputs=True)
    for act in range(7):
        fin = np.isfinite(y64[act, :, 0])
        err = np.abs(y[act, fin, 0].astype(np.float64) - y64[act, fin, 0])
        print("act", act, "max abs err", err.max())
        assert np.all(err <= beta[act, fin, 0]), act
        assert np.array_equal(np.isnan(y[act, :, 0]), np.isnan(y64[act, :, 0])), act


def _same_bits(a, b):
    """Equal bit patterns, except that any NaN matches any NaN."""
    nan = np.isnan(a)
    return np.array_equal(nan, np.isnan(b)) and np.array_equal(a[~nan].view(np.uint32),
                                                                 b[~nan].view(np.uint32))


@pytest.mark.parametrize("which", ["control", "classes"])
def test_value_stores_agree_bitwise(which):
    """All value stores run the same operations in the same order, so their
    outputs are identical bit for bit (registers with one or two samples per
    lane, any slot class, and LDS rows)."""
    neat = _neat()
    if which == "control":
        pop = synth.control(seed=31, P=200, B=150)
        nodes, conns, I, O, x = pop.nodes, pop.conns, pop.I, pop.O, pop.inputs
    else:
        pops = synth.uneven(seed=9, n_pops=3, P_range=(20, 40), N_range=(150, 400),
                            B_range=(70, 140))
        pop = max(pops, key=lambda q: q.N_max)
        nodes, conns, I, O, x = pop.nodes, pop.conns, pop.I, pop.O, pop.inputs
    ys = [_gpu(nodes, conns, I, O, x, variant=v)[3]
          for v in (neat.FWD_REG, neat.FWD_LDS, neat.FWD_REG2, neat.FWD_AUTO)]
    for k in range(1, len(ys)):
        assert _same_bits(ys[0], ys[k]), k


def _max_live(nodes, conns, I, O, order_rows):
    """Largest number of values held at once by a slot allocator that frees
    a value after its last reader (the reader may reuse the slot), keeps
    inputs from the start and outputs to the end."""
    valid = ~np.isnan(nodes[:, 0])
    key = {r: int(nodes[r, 0]) for r in np.nonzero(valid)[0]}
    rows = [r for r in order_rows if r >= 0]
    pos = {r: p for p, r in enumerate(rows)}
    row_of = {k: r for r, k in key.items()}
    n = len(rows)
    last = {r: pos[r] for r in rows}
    for c in conns:
        if np.isnan(c[0]) or c[2] != 1.0:
            continue
        s, d = row_of[int(c[0])], row_of[int(c[1])]
        last[s] = max(last[s], pos[d])
    for r in rows:
        if I <= key[r] < I + O:
            last[r] = n
    best = I
    for p in range(I, n):
        # values defined before p still needed after p, plus p itself;
        # unread inputs are dropped once the first computed node runs
        live = sum(1 for r in rows[:p] if last[r] > p) + 1
        best = max(best, live)
    return best


def test_slot_allocation_is_the_largest_live_set():
    """The program build's slot count equals the largest live set, and the
    slot class follows from it (program header words)."""
    neat = _neat()
    pops = synth.uneven(seed=13, n_pops=4, P_range=(4, 8), N_range=(20, 300), B_range=(1, 2))
    for pop in pops:
        dev = torch.device("cuda:0")
        tn = torch.from_numpy(pop.nodes).to(dev)
        tc = torch.from_numpy(pop.conns).to(dev)
        order, level, status, prog = neat.topo_sort(tn, tc, pop.I, pop.O)
        d = neat.dims_of(tn, tc, pop.I, pop.O)
        hdr = neat.program_headers(d, prog).cpu().numpy()
        order = order.cpu().numpy()
        for g in range(pop.P):
            if status[g].item() != 0:
                continue
            if pop.N_max <= 62:
                m = int((order[g] >= 0).sum())  # slot = position
            else:
                m = _max_live(pop.nodes[g], pop.conns[g], pop.I, pop.O, order[g])
            assert hdr[g, 8] == m, (pop.N_max, g, hdr[g, 8], m)
            cls = 0 if m <= 62 else 1 if m <= 126 else 2 if m <= 222 else 3
            assert hdr[g, 6] == cls


def test_retransformation_changes_only_slot_numbers():
    """Transforming the same populations of N_max > 64 again gives the same
    order, levels, status and program headers (slot count and class among
    them) and bit-identical outputs.  Only which free slot a value takes may
    change between calls (extra frees at one position are ranked by the
    order of LDS atomics across the group's waves), and every such program
    still computes the oracle's outputs."""
    neat = _neat()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    for lo, hi in ((65, 120), (260, 420)):
        pop = synth.uneven_population(rng, (40, 80), (lo, hi), (1, 2), with_inputs=False)
        print("case retransform N_max", pop.N_max, "P", pop.P, flush=True)
        tn = torch.from_numpy(pop.nodes).to(dev)
        tc = torch.from_numpy(pop.conns).to(dev)
        d = neat.dims_of(tn, tc, pop.I, pop.O)
        B = 40
        x = rng.standard_normal((pop.P, B, pop.I)).astype(np.float32)
        tx = torch.from_numpy(x).to(dev)
        runs = []
        for _ in range(4):
            order, level, status, prog = neat.topo_sort(tn, tc, pop.I, pop.O)
            # the defined header words (9..15 are not written)
            hdr = neat.program_headers(d, prog).cpu().numpy()[:, :9]
            y = neat.forward(d, prog, tx, B).cpu().numpy()
            runs.append((order.cpu().numpy(), level.cpu().numpy(), status.cpu().numpy(), hdr, y))
        for r in runs[1:]:
            for a, b in zip(runs[0][:4], r[:4]):
                assert np.array_equal(a, b)
            assert np.array_equal(runs[0][4].view(np.uint32), r[4].view(np.uint32))
        y64, beta = oracle.forward(pop.nodes, pop.conns, x, pop.I, pop.O)
        _assert_outputs(runs[0][4], y64, beta, "retransform N_max=%d" % pop.N_max)


@pytest.mark.parametrize("O", [4, 230])
def test_largest_supported_sizes(O):
    """N_max = 600 (I + N_max close to the LDS-row store's limit of 638) and
    C_max = 2400: the multi-wave transformation at its widest and, with 230
    outputs live to the end, genomes in the LDS-row store."""
    rng = np.random.default_rng(600 + O)
    P, N, C, I, B = 4, 600, 2400, 10, 70
    nodes = np.full((P, N, 5), np.nan, np.float32)
    conns = np.full((P, C, 4), np.nan, np.float32)
    for p in range(P):
        h = int(rng.integers(N // 2, N - I - O + 1))
        synth.make_genome(rng, N, C, I, O, h, lambda na: int(rng.integers(C // 2, min(C, na) + 1)),
                          synth.CONTROL_ACTS, synth.ALL_AGGS, nodes_out=nodes[p],
                          conns_out=conns[p])
    x = rng.standard_normal((P, B, I)).astype(np.float32)
    print("case largest sizes O", O, flush=True)
    order, level, status, y = _gpu(nodes, conns, I, O, x)
    _assert_transform_exact(nodes, conns, I, O, order, level, status)
    y64, beta = oracle.forward(nodes, conns, x, I, O)
    _assert_outputs(y, y64, beta, "largest sizes O=%d" % O)


def test_largest_nodes_in_half_wave_lds_tiles():
    """N_max = 1024, the ABI's largest, with 230 outputs live to the end:
    64 columns of 1026 rows exceed the LDS, so the LDS-row store runs tiles
    of 32 samples; every value store agrees with the oracle and with each
    other bit for bit."""
    neat = _neat()
    rng = np.random.default_rng(1024)
    P, N, C, I, O, B = 3, 1024, 2048, 6, 230, 45
    nodes = np.full((P, N, 5), np.nan, np.float32)
    conns = np.full((P, C, 4), np.nan, np.float32)
    for p in range(P):
        synth.make_genome(rng, N, C, I, O, int(rng.integers(300, 700)),
                          lambda na: int(rng.integers(C // 2, min(C, na) + 1)),
                          synth.CONTROL_ACTS, synth.ALL_AGGS, nodes_out=nodes[p],
                          conns_out=conns[p])
    x = rng.standard_normal((P, B, I)).astype(np.float32)
    print("case N_max 1024", flush=True)
    order, level, status, y = _gpu(nodes, conns, I, O, x)
    _assert_transform_exact(nodes, conns, I, O, order, level, status)
    y64, beta = oracle.forward(nodes, conns, x, I, O)
    _assert_outputs(y, y64, beta, "N_max 1024")
    _, _, _, y_lds = _gpu(nodes, conns, I, O, x, variant=neat.FWD_LDS)
    assert np.array_equal(y.view(np.uint32), y_lds.view(np.uint32))


def test_beyond_the_lds_row_store_is_refused():
    """I + N_max beyond the half-wave store's 1278 (N_max = 1024 with 300
    inputs) transforms but is refused by the forward with a clean
    NEAT_E_TOO_LARGE before any launch; N_max = 1024 with C_max = 16384 does
    not fit the transformation's LDS and is refused by it, while a one-wave
    genome with C_max = 16384 fits and transforms exactly."""
    neat = _neat()
    dev = torch.device("cuda:0")
    I = 300
    nodes = np.full((2, 1024, 5), np.nan, np.float32)
    nodes[:, :I + 1] = np.array([[k, 0.0, 1.0, 0, 0] for k in range(I + 1)], np.float32)
    conns = np.full((2, 64, 4), np.nan, np.float32)
    conns[:, 0] = (0, I, 1, 0.5)
    tn = torch.from_numpy(nodes).to(dev)
    tc = torch.from_numpy(conns).to(dev)
    order, level, status, prog = neat.topo_sort(tn, tc, I, 1)
    d = neat.dims_of(tn, tc, I, 1)
    with pytest.raises(neat.NeatError) as e:
        neat.forward(d, prog, torch.zeros((2, 4, I), device=dev), 4)
    assert e.value.code == -4
    torch.cuda.synchronize()
    o_order, o_level, o_status = oracle.transform(nodes, conns, I, 1)
    assert np.array_equal(o_order, order.cpu().numpy())
    assert np.array_equal(o_status, status.cpu().numpy().astype(np.uint32))
    big = torch.full((1, 1024, 5), float("nan"), device=dev)
    with pytest.raises(neat.NeatError) as e:
        neat.topo_sort(big, torch.full((1, 16384, 4), float("nan"), device=dev), 3, 1)
    assert e.value.code == -1  # NEAT_E_INVALID: the working set does not fit in LDS
    rng = np.random.default_rng(16384)
    nodes = np.full((3, 64, 5), np.nan, np.float32)
    conns = np.full((3, 16384, 4), np.nan, np.float32)
    for p in range(3):
        synth.make_genome(rng, 64, 16384, 7, 3, 54, lambda na: na, synth.CONTROL_ACTS,
                          synth.ALL_AGGS, nodes_out=nodes[p], conns_out=conns[p])
    order, level, status, _ = _gpu(nodes, conns, 7, 3)
    _assert_transform_exact(nodes, conns, 7, 3, order, level, status)
