"""Pins for the CPU oracle: every check here compares the oracle with something
other than itself -- closed forms, numpy/networkx routines, brute force on tiny
graphs, the paper's dense formulation, hand-computed fixtures, invariants."""
from __future__ import annotations

import itertools
import math

import networkx as nx
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from oracle import dense
from workloads import synth
from tests.helpers import genome, read_golden, stack

NAN = float("nan")
ACT_NUMPY = {
    0: lambda z: z,
    1: np.tanh,
    2: lambda z: 1.0 / (1.0 + np.exp(-z)),
    3: lambda z: np.maximum(z, 0.0),
    4: np.sin,
    5: lambda z: np.exp(-z * z),
    6: np.abs,
}


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("act", range(7))
def test_single_edge_closed_form(act):
    """y = act(b + r * w * x) for one input feeding one output (Section 3.3
    with f_c = w x and f_n = act(agg + b), response r)."""
    b, r, w = 0.375, 1.5, -0.8125
    n, c = genome(4, 3, {0: (0, 0, 1, 0, 0), 2: (1, b, r, act, 0)},
                  {1: (0, 1, 1, w)})
    x = np.linspace(-3, 3, 25, dtype=np.float32)[:, None]
    y, beta = oracle.forward(n, c, x[None], 1, 1)
    ref = ACT_NUMPY[act](b + r * w * x.astype(np.float64))
    np.testing.assert_allclose(y[0], ref, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("agg,fn", [
    (0, lambda t: t.sum(1)), (1, lambda t: t.prod(1)), (2, lambda t: t.max(1)),
    (3, lambda t: t.min(1)), (4, lambda t: t.mean(1))])
def test_single_node_aggregations(agg, fn):
    """Three inputs into one identity output node with each aggregation."""
    w = np.array([0.5, -2.0, 1.25])
    nodes = {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0), 2: (2, 0, 1, 0, 0),
             3: (3, 0.25, 1, 0, agg)}
    conns = {0: (2, 3, 1, w[2]), 1: (0, 3, 1, w[0]), 2: (1, 3, 1, w[1])}
    n, c = genome(4, 3, nodes, conns)
    x = np.random.default_rng(5).standard_normal((40, 3)).astype(np.float32)
    y, _ = oracle.forward(n, c, x[None], 3, 1)
    ref = 0.25 + fn(x.astype(np.float64) * w[None, :])
    np.testing.assert_allclose(y[0, :, 0], ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("agg", range(5))
@pytest.mark.parametrize("act", range(7))
def test_empty_aggregation_is_act_of_bias(agg, act):
    """A non-input node without enabled incoming edges evaluates act(bias)."""
    n, c = genome(3, 2, {0: (0, 0, 1, 0, 0), 1: (1, -0.7, 2.0, act, agg)},
                  {0: (0, 1, 0, 5.0)})   # disabled edge only
    y, _ = oracle.forward(n, c, np.ones((1, 3, 1), np.float32), 1, 1)
    ref = ACT_NUMPY[act](np.float64(np.float32(-0.7)))
    np.testing.assert_allclose(y, np.full(y.shape, ref), rtol=1e-15, atol=0)


def test_nan_propagates_through_max_min_relu():
    """NaN reaching a node through a weight propagates through max, min and
    relu (a reading: no NaN is silently dropped)."""
    for agg, act in ((2, 0), (3, 0), (0, 3)):
        n, c = genome(4, 3, {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0),
                             2: (2, 0, 1, act, agg)},
                      {0: (0, 2, 1, NAN), 1: (1, 2, 1, 1.0)})
        y, beta = oracle.forward(n, c, np.ones((1, 2, 2), np.float32), 2, 1)
        assert np.isnan(y).all() and (beta == 0).all()


def test_golden_hand_network():
    g = read_golden("hand_net.txt")
    I, O = g["I"], g["O"]
    order, level, status = oracle.transform(g["nodes_arr"], g["conns_arr"], I, O)
    assert status[0] == 0
    assert oracle.order_keys(g["nodes_arr"], order)[0][:6].tolist() == g["order"]
    for r in range(g["N_max"]):
        k = g["nodes_arr"][0, r, 0]
        assert level[0, r] == (g["level"][int(k)] if not np.isnan(k) else -1)
    y, _ = oracle.forward(g["nodes_arr"], g["conns_arr"], g["x"][None], I, O)
    assert np.array_equal(y[0], g["y"])
    y32 = oracle.forward(g["nodes_arr"], g["conns_arr"], g["x"][None], I, O,
                         precision="f32")
    assert np.array_equal(y32[0].astype(np.float64), g["y"])
    yd = dense.forward(g["nodes_arr"][0], g["conns_arr"][0], g["x"], I, O)
    assert np.array_equal(yd, g["y"])


# ------------------------------------------------------ linear nets: solve/paths
def _graph(nodes, conns):
    """networkx DiGraph over rows of one genome's enabled edges."""
    G = nx.DiGraph()
    key_row = {}
    for r in range(nodes.shape[0]):
        if not np.isnan(nodes[r, 0]):
            G.add_node(r)
            key_row[float(nodes[r, 0])] = r
    for cr in conns:
        if np.isnan(cr[0]) or cr[2] != 1:
            continue
        G.add_edge(key_row[float(cr[0])], key_row[float(cr[1])], w=float(cr[3]))
    return G, key_row


def _linear_genome(seed, n_hidden, I=2, O=2):
    rng = np.random.default_rng(seed)
    n, c = synth.make_genome(rng, I + O + n_hidden + 2, 24, I, O, n_hidden,
                             lambda na: min(na, 12), (synth.ACT_IDENTITY,),
                             (synth.AGG_SUM,))
    valid = ~np.isnan(n[:, 0])
    n[valid, 2] = rng.uniform(-1.5, 1.5, valid.sum()).astype(np.float32)  # response
    return n[None], c[None], I, O


@pytest.mark.parametrize("seed", range(12))
def test_linear_network_matches_linear_solve(seed):
    """identity + sum nets: v solves (1 - R W^T) v = b~ (unit triangular in
    topological order) -> numpy.linalg.solve."""
    n, c, I, O = _linear_genome(seed, n_hidden=seed % 5 + 1)
    G, key_row = _graph(n[0], c[0])
    rows = sorted(G.nodes)
    idx = {r: i for i, r in enumerate(rows)}
    x = np.random.default_rng(100 + seed).standard_normal((7, I)).astype(np.float32)
    y, _ = oracle.forward(n, c, x[None], I, O)
    for b in range(x.shape[0]):
        A = np.eye(len(rows))
        rhs = np.zeros(len(rows))
        for r in rows:
            key = n[0, r, 0]
            if key < I:
                rhs[idx[r]] = x[b, int(key)]
                continue
            rhs[idx[r]] = n[0, r, 1]
            for s in G.predecessors(r):
                A[idx[r], idx[s]] -= float(n[0, r, 2]) * G[s][r]["w"]
        v = np.linalg.solve(A, rhs)
        ref = [v[idx[key_row[float(I + j)]]] for j in range(O)]
        np.testing.assert_allclose(y[0, b], ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_linear_network_matches_path_enumeration(seed):
    """identity + sum: y_out = sum over all paths s -> ... -> out of
    prod(response_dst * w) * c(s), with c = x for inputs and bias otherwise."""
    n, c, I, O = _linear_genome(1000 + seed, n_hidden=seed % 4 + 1)
    G, key_row = _graph(n[0], c[0])
    x = np.random.default_rng(seed).standard_normal((3, I)).astype(np.float32)
    y, _ = oracle.forward(n, c, x[None], I, O)
    for b in range(3):
        for j in range(O):
            t = key_row[float(I + j)]
            total = float(n[0, t, 1])      # the trivial path: bias of t
            for s in G.nodes:
                if s == t:
                    continue
                for path in nx.all_simple_paths(G, s, t):
                    gain = 1.0
                    for a, bb in zip(path[:-1], path[1:]):
                        gain *= float(n[0, bb, 2]) * G[a][bb]["w"]
                    k = n[0, s, 0]
                    total += gain * (float(x[b, int(k)]) if k < I else float(n[0, s, 1]))
            assert math.isclose(y[0, b, j], total, rel_tol=1e-10, abs_tol=1e-12)


# ------------------------------------------------------------ levels and order
def _brute_levels(G):
    """Longest path into each node by enumerating every simple path."""
    lev = {v: 0 for v in G.nodes}
    for s in G.nodes:
        for t in G.nodes:
            if s == t:
                continue
            for p in nx.all_simple_paths(G, s, t):
                lev[t] = max(lev[t], len(p) - 1)
    return lev


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 32 - 1), hidden=st.integers(0, 4),
       I=st.integers(1, 2), O=st.integers(1, 2))
def test_levels_match_brute_force_and_networkx(seed, hidden, I, O):
    rng = np.random.default_rng(seed)
    N = I + O + hidden
    n, c = synth.make_genome(rng, N + 1, 20, I, O, hidden,
                             lambda na: int(rng.integers(0, na + 1)),
                             synth.CONTROL_ACTS, synth.ALL_AGGS)
    order, level, status = oracle.transform(n[None], c[None], I, O)
    assert status[0] == 0
    G, _ = _graph(n, c)
    brute = _brute_levels(G)
    gens = {v: i for i, gen in enumerate(nx.topological_generations(G)) for v in gen}
    for r in G.nodes:
        assert level[0, r] == brute[r] == gens[r]
    # order = valid rows sorted by (level, key); a valid topological order
    want = sorted(G.nodes, key=lambda r: (brute[r], n[r, 0]))
    assert order[0, :len(want)].tolist() == want
    assert (order[0, len(want):] == -1).all()
    pos = {r: i for i, r in enumerate(want)}
    assert all(pos[a] < pos[b] for a, b in G.edges)


def test_chain_and_star_levels():
    # chain 0 -> 5 -> 6 -> 7 -> 1 : levels 0,1,2,3,4
    keys = [0, 1, 5, 6, 7]
    nodes = {i: (k, 0, 1, 0, 0) for i, k in enumerate(keys)}
    chain = [(0, 5), (5, 6), (6, 7), (7, 1)]
    n, c = genome(5, 4, nodes, {i: (a, b, 1, 1.0) for i, (a, b) in enumerate(chain)})
    order, level, st_ = oracle.transform(n, c, 1, 1)
    assert st_[0] == 0
    assert [level[0, keys.index(k)] for k in (0, 5, 6, 7, 1)] == [0, 1, 2, 3, 4]
    # star: input 0 feeds 5 nodes directly: all leaves on level 1
    keys = [0, 1, 2, 3, 4, 5]
    n, c = genome(6, 5, {i: (k, 0, 1, 0, 0) for i, k in enumerate(keys)},
                  {i: (0, i + 1, 1, 1.0) for i in range(5)})
    order, level, st_ = oracle.transform(n, c, 1, 5)
    assert st_[0] == 0 and level[0].tolist() == [0, 1, 1, 1, 1, 1]


@settings(max_examples=80, deadline=None)
@given(seed=st.integers(0, 2 ** 32 - 1))
def test_cycle_detection_matches_networkx(seed):
    """Random digraphs (cycles allowed, no edges into inputs, no duplicates):
    CYCLE iff networkx finds the enabled graph is not a DAG."""
    rng = np.random.default_rng(seed)
    I, O, H = 1, 2, int(rng.integers(0, 4))
    keys = list(range(I + O)) + [10 + 3 * h for h in range(H)]
    N = len(keys)
    nodes = {r: (k, 0, 1, 0, 0) for r, k in enumerate(keys)}
    pairs = [(a, b) for a in keys for b in keys if b >= I]
    m = int(rng.integers(0, len(pairs) + 1))
    pick = rng.choice(len(pairs), size=m, replace=False)
    conns = {}
    for i, q in enumerate(pick):
        a, b = pairs[q]
        conns[i] = (a, b, float(rng.random() < 0.7), 1.0)
    n, c = genome(N, max(m, 1), nodes, conns)
    _, _, status = oracle.transform(n, c, I, O)
    G = nx.DiGraph()
    G.add_nodes_from(keys)
    G.add_edges_from((a, b) for (a, b, e, _) in conns.values() if e == 1)
    assert bool(status[0] & oracle.CYCLE) == (not nx.is_directed_acyclic_graph(G))
    assert status[0] & ~np.uint32(oracle.CYCLE) == 0


# ------------------------------------------------------------ status corpus
def _base():
    """A valid genome: I=2, O=1, hidden keys 5, 6."""
    nodes = {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0), 2: (2, 0.1, 1, 1, 0),
             4: (5, 0.2, 1, 2, 1), 6: (6, -0.3, 1, 3, 2)}
    conns = {0: (0, 5, 1, 0.5), 2: (1, 6, 1, -1.0), 3: (5, 2, 1, 2.0),
             5: (6, 2, 1, 1.5), 6: (5, 6, 0, 9.0)}
    return nodes, conns


def _status(nodes, conns, N=8, C=10, I=2, O=1):
    n, c = genome(N, C, nodes, conns)
    order, level, status = oracle.transform(n, c, I, O)
    if status[0] != 0:
        assert (order == -1).all() and (level == -1).all()
        y, beta = oracle.forward(n, c, np.zeros((1, 2, I), np.float32), I, O)
        assert np.isnan(y).all()
    return int(status[0])


def _mod(fn):
    nodes, conns = _base()
    fn(nodes, conns)
    return _status(nodes, conns)


CORPUS = [
    ("valid", lambda n, c: None, 0),
    ("non-integer key", lambda n, c: n.__setitem__(4, (5.5, 0.2, 1, 2, 1)), 1 | 8),
    ("negative key", lambda n, c: n.__setitem__(4, (-5, 0.2, 1, 2, 1)), 1 | 8),
    ("key too large", lambda n, c: n.__setitem__(4, (2.0 ** 24, 0.2, 1, 2, 1)), 1 | 8),
    ("act out of range", lambda n, c: n.__setitem__(4, (5, 0.2, 1, 7, 1)), 1),
    ("agg out of range", lambda n, c: n.__setitem__(4, (5, 0.2, 1, 2, 5)), 1),
    ("non-integer act", lambda n, c: n.__setitem__(4, (5, 0.2, 1, 1.5, 1)), 1),
    ("NaN agg", lambda n, c: n.__setitem__(4, (5, 0.2, 1, 2, NAN)), 1),
    ("enabled flag 0.5", lambda n, c: c.__setitem__(0, (0, 5, 0.5, 0.5)), 1),
    ("enabled flag NaN", lambda n, c: c.__setitem__(0, (0, 5, NAN, 0.5)), 1),
    ("duplicate key", lambda n, c: n.__setitem__(7, (6, 0, 1, 0, 0)), 2),
    ("missing output", lambda n, c: n.pop(2), 4 | 8),
    ("missing input", lambda n, c: (n.pop(1), c.pop(2)), 4),
    ("dangling in", lambda n, c: c.__setitem__(7, (42, 2, 1, 1.0)), 8),
    ("dangling out", lambda n, c: c.__setitem__(7, (5, 43, 1, 1.0)), 8),
    ("NaN out key", lambda n, c: c.__setitem__(7, (5, NAN, 1, 1.0)), 8),
    ("edge into input", lambda n, c: c.__setitem__(7, (5, 1, 1, 1.0)), 16),
    ("duplicate edge", lambda n, c: c.__setitem__(7, (0, 5, 1, -3.0)), 32),
    ("self loop", lambda n, c: c.__setitem__(7, (6, 6, 1, 1.0)), 64),
    ("two-cycle", lambda n, c: (c.__setitem__(6, (5, 6, 1, 1.0)),
                                c.__setitem__(7, (6, 5, 1, 1.0))), 64),
    ("three-cycle via output", lambda n, c: (c.__setitem__(7, (2, 5, 1, 1.0)),), 64),
    ("disabled junk ignored", lambda n, c: c.__setitem__(7, (77, 88, 0, NAN)), 0),
    ("disabled into input ignored", lambda n, c: c.__setitem__(7, (5, 0, 0, 1)), 0),
    ("disabled duplicate ignored", lambda n, c: c.__setitem__(7, (0, 5, 0, 1)), 0),
    ("padding with junk ignored", lambda n, c: c.__setitem__(7, (NAN, 5, 1, 1)), 0),
    ("node row with NaN key ignored", lambda n, c: n.__setitem__(7, (NAN, 1, 1, 99, 99)), 0),
    ("dup edge + into input", lambda n, c: (c.__setitem__(7, (5, 1, 1, 1.0)),
                                            c.__setitem__(8, (5, 1, 1, 2.0))), 16 | 32),
    ("bad ref hides cycle", lambda n, c: (c.__setitem__(6, (5, 6, 1, 1.0)),
                                          c.__setitem__(8, (6, 5, 1, 1.0)),
                                          c.__setitem__(7, (5, 99, 1, 1.0))), 8),
    ("bad value hides cycle", lambda n, c: (c.__setitem__(6, (5, 6, 1, 1.0)),
                                            c.__setitem__(8, (6, 5, 1, 1.0)),
                                            n.__setitem__(6, (6, 0, 1, 9, 0))), 1),
    ("cycle found without other flags", lambda n, c: (c.__setitem__(6, (5, 6, 1, 1.0)),
                                                      c.__setitem__(8, (6, 5, 1, 1.0))), 64),
    ("self loop kept with bad value", lambda n, c: (c.__setitem__(7, (6, 6, 1, 1.0)),
                                                    n.__setitem__(6, (6, 0, 1, 9, 0))), 1 | 64),
    ("missing io + bad value", lambda n, c: (n.pop(2), n.__setitem__(4, (5, 0, 1, 8, 0))),
     1 | 4 | 8),
]


@pytest.mark.parametrize("name,fn,expected", CORPUS, ids=[c[0] for c in CORPUS])
def test_status_corpus(name, fn, expected):
    assert _mod(fn) == expected


# ------------------------------------------------------------ invariants
def _eval(n, c, x, I, O):
    order, level, status = oracle.transform(n, c, I, O)
    y, beta = oracle.forward(n, c, x, I, O)
    return oracle.order_keys(n, order), status, y, beta


@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    pop = synth.control(seed=50 + seed, P=6, B=5)
    n, c, x, I, O = pop.nodes, pop.conns, pop.inputs, pop.I, pop.O
    ok, st0, y0, b0 = _eval(n, c, x, I, O)
    assert (st0 == 0).all()
    rng = np.random.default_rng(seed)
    # 1. more NaN padding rows, anywhere
    n2 = np.full((6, 70, 5), np.nan, np.float32)
    c2 = np.full((6, 260, 4), np.nan, np.float32)
    rn, rc = np.sort(rng.choice(70, 50, replace=False)), np.sort(rng.choice(260, 200, replace=False))
    n2[:, rn], c2[:, rc] = n, c
    ok2, st2, y2, _ = _eval(n2, c2, x, I, O)
    assert np.array_equal(y2, y0)
    assert np.array_equal(ok2[:, :50], ok0 := ok) and (ok2[:, 50:] == -1).all()
    # 2. disabled rows with arbitrary content (NaN, bad refs, into inputs)
    c3 = np.full((6, 240, 4), np.nan, np.float32)
    c3[:, :200] = c
    junk = rng.standard_normal((6, 40, 4)).astype(np.float32) * 100
    junk[:, :, 2] = 0.0
    junk[:, ::3, 3] = np.nan
    c3[:, 200:] = junk
    ok3, st3, y3, _ = _eval(n, c3, x, I, O)
    assert np.array_equal(y3, y0) and np.array_equal(ok3, ok0) and (st3 == 0).all()
    # 3. permuted node and connection storage: same keys in order, same bits
    pn, pc = rng.permutation(50), rng.permutation(200)
    ok4, st4, y4, _ = _eval(n[:, pn], c[:, pc], x, I, O)
    assert np.array_equal(y4, y0) and np.array_equal(ok4, ok0)
    # 4. an isolated hidden node changes nothing downstream
    n5 = n.copy()
    for p in range(6):
        free = np.nonzero(np.isnan(n5[p, :, 0]))[0]
        if len(free):
            n5[p, free[0]] = (5000, 3.0, 1.0, 1, 0)  # keys < 800 are taken
    _, st5, y5, _ = _eval(n5, c, x, I, O)
    assert np.array_equal(y5, y0) and (st5 == 0).all()
    # 5. response 0 on the outputs gives act(bias)
    n6 = n.copy()
    for p in range(6):
        for j in range(O):
            r = I + j
            n6[p, r, 2] = 0.0
    _, _, y6, _ = _eval(n6, c, x, I, O)
    for p in range(6):
        for j in range(O):
            r = I + j
            want = ACT_NUMPY[int(n6[p, r, 3])](np.float64(n6[p, r, 1]))
            np.testing.assert_allclose(y6[p, :, j], want, rtol=1e-15, atol=0)


# --------------------------------------------- dense paper formulation (O2)
@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 32 - 1))
def test_oracle_matches_dense_paper_formulation(seed):
    rng = np.random.default_rng(seed)
    I, O = int(rng.integers(1, 5)), int(rng.integers(1, 4))
    H = int(rng.integers(0, 10))
    N, C = I + O + H + int(rng.integers(0, 4)), 48
    n, c = synth.make_genome(rng, N, C, I, O, H, lambda na: int(rng.integers(1, min(na, C) + 1)),
                             tuple(range(7)), tuple(range(5)))
    x = rng.standard_normal((6, I)).astype(np.float32)
    y, _ = oracle.forward(n[None], c[None], x[None], I, O)
    yd = dense.forward(n, c, x, I, O)
    np.testing.assert_allclose(y[0], yd, rtol=1e-12, atol=1e-12, equal_nan=True)


def test_oracle_matches_dense_on_tiny_and_cppn():
    for pop, x in ((synth.tiny(), None), (synth.cppn(P=20), synth.grid_queries(0, 300))):
        shared = x if x is not None else pop.inputs
        y, _ = oracle.forward(pop.nodes, pop.conns, shared, pop.I, pop.O, shared_inputs=True)
        for p in range(pop.P):
            yd = dense.forward(pop.nodes[p], pop.conns[p], shared, pop.I, pop.O)
            np.testing.assert_allclose(y[p], yd, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------- fp32 error bound
def test_beta_bounds_an_fp32_evaluation():
    """The float instantiation of the oracle stays within the tolerance rule
    (|y32 - y64| <= 1e-5 + 2 beta); with atol = 0 it stays within 2 beta,
    which checks the bound itself."""
    for pop in (synth.control(seed=9, P=300, B=16), ):
        y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
        y32 = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, precision="f32")
        ok, stats = oracle.within_tolerance(y32, y64, beta, atol=0.0)
        assert stats["n_fail"] == 0, stats
    pop = synth.cppn(P=100)
    x = synth.grid_queries(0, 2000)
    y64, beta = oracle.forward(pop.nodes, pop.conns, x, pop.I, pop.O, shared_inputs=True)
    y32 = oracle.forward(pop.nodes, pop.conns, x, pop.I, pop.O, shared_inputs=True,
                         precision="f32")
    ok, stats = oracle.within_tolerance(y32, y64, beta, atol=0.0)
    assert stats["n_fail"] == 0, stats


def test_beta_covers_summation_rounding():
    """Wide identity + sum/mean nodes over large inputs, where the rounding
    of the additions (not of the products) dominates the fp32 error: the
    float evaluation must stay within beta itself (factor 1)."""
    I = 64
    rng = np.random.default_rng(21)
    for agg in (synth.AGG_SUM, synth.AGG_MEAN):
        nodes = {i: (i, 0, 1, 0, 0) for i in range(I)}
        nodes[I] = (I, 0.0, 1.0, 0, agg)
        conns = {i: (i, I, 1, float(rng.standard_normal())) for i in range(I)}
        n, c = genome(I + 1, I, nodes, conns)
        x = (rng.standard_normal((1, 4000, I)) * 1000).astype(np.float32)
        y64, beta = oracle.forward(n, c, x, I, 1)
        y32 = oracle.forward(n, c, x, I, 1, precision="f32")
        assert np.all(np.abs(y32 - y64) <= beta)
