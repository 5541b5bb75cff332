"""Pins for the oracle's recurrent calculation (synchronous update over K
sweeps; the paper names recurrent networks without defining them, so the
update rule is a reading).  Every check compares the oracle with something
other than itself: closed forms of a self-loop, numpy's linear solve at the
fixed point of a contracting linear net, the pinned feedforward oracle on
acyclic genomes, hand-made status cases, storage permutations and the fp32
error bound."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import synth
from tests.helpers import genome

NAN = float("nan")


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("w", [0.5, -0.8, 1.5, 1.0])
@pytest.mark.parametrize("K", [0, 1, 2, 5, 9])
def test_self_loop_geometric_series(w, K):
    """Input x -> output o (weight a), o -> o (weight w), identity + sum, bias
    b: v_t = b + a x + w v_{t-1}, v_0 = 0, so v_K = (b + a x) sum_{k<K} w^k."""
    a, b = 0.75, -0.3
    n, c = genome(2, 2, {0: (0, 0, 1, 0, 0), 1: (1, b, 1, 0, 0)},
                  {0: (0, 1, 1, a), 1: (1, 1, 1, w)})
    x = np.array([[[1.25], [-2.0], [0.0]]], np.float32)
    y, _ = oracle.forward_recurrent(n, c, x, 1, 1, K)
    b, w = float(np.float32(b)), float(np.float32(w))   # the values as stored
    for i, xv in enumerate(x[0, :, 0]):
        c0 = b + a * float(xv)
        ref = c0 * sum(w ** k for k in range(K))
        assert y[0, i, 0] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_two_node_oscillator():
    """Two identity nodes feeding each other with weight -1 and no bias,
    driven by x only through h: h_t = x - o_{t-1}, o_t = h_{t-1}; the output
    sequence is 0, x, x, 0, 0, x, x, 0, ... (period 4)."""
    n, c = genome(3, 3, {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0), 2: (7, 0, 1, 0, 0)},
                  {0: (0, 7, 1, 1.0), 1: (1, 7, 1, -1.0), 2: (7, 1, 1, 1.0)})
    x = np.array([[[3.0]]], np.float32)
    seq = [oracle.forward_recurrent(n, c, x, 1, 1, K)[0][0, 0, 0] for K in range(9)]
    assert seq == [0.0, 0.0, 3.0, 3.0, 0.0, 0.0, 3.0, 3.0, 0.0]


# ------------------------------------------------------------ fixed point
@pytest.mark.parametrize("seed", range(8))
def test_contracting_linear_net_reaches_linear_solve(seed):
    """Identity + sum with recurrent edges scaled so that sum |r w| into any
    node is below 1/2: the sweep v <- c + M v contracts, and after 200 sweeps
    the outputs equal the solution of (1 - M) v = c (numpy.linalg.solve),
    M[u, s] = r_u w_{s->u}, c_u = b_u + r_u sum_{inputs} w x."""
    rng = np.random.default_rng(seed)
    I, O, H = 3, 2, 4 + seed % 4
    N = I + O + H + 2
    n, c = synth.make_genome(rng, N, 40, I, O, H, 30, (synth.ACT_IDENTITY,),
                             (synth.AGG_SUM,), p_enabled=1.0, recurrent=True)
    valid = ~np.isnan(n[:, 0])
    n[valid, 2] = rng.uniform(-1.0, 1.0, valid.sum()).astype(np.float32)
    key_row = {float(n[r, 0]): r for r in range(N) if valid[r]}
    live = ~np.isnan(c[:, 0])
    # scale the weights into each node so that sum |r w| < 1/2
    for key in set(c[live, 1].tolist()):
        m = live & (c[:, 1] == key)
        tot = np.abs(c[m, 3]).sum() * abs(float(n[key_row[key], 2])) + 1e-9
        c[m, 3] = (c[m, 3] * (0.45 / max(tot, 0.45))).astype(np.float32)
    x = rng.standard_normal((5, I)).astype(np.float32)
    y, _ = oracle.forward_recurrent(n[None], c[None], x[None], I, O, 200)
    rows = [r for r in range(N) if valid[r]]
    idx = {r: i for i, r in enumerate(rows)}
    for b in range(x.shape[0]):
        A = np.eye(len(rows))
        rhs = np.zeros(len(rows))
        for r in rows:
            key = n[r, 0]
            if key < I:
                rhs[idx[r]] = x[b, int(key)]
            else:
                rhs[idx[r]] = n[r, 1]
        for cr in c[live]:
            d, s = key_row[float(cr[1])], key_row[float(cr[0])]
            A[idx[d], idx[s]] -= float(n[d, 2]) * float(cr[3])
        v = np.linalg.solve(A, rhs)
        ref = [v[idx[key_row[float(I + j)]]] for j in range(O)]
        np.testing.assert_allclose(y[0, b], ref, rtol=1e-9, atol=1e-11)


# ----------------------------------------------------- acyclic = feedforward
@pytest.mark.parametrize("seed", range(6))
def test_dag_after_depth_sweeps_equals_feedforward(seed):
    """On an acyclic genome a non-input node's value is final once the sweep
    count reaches its level plus one (a node without incoming edges takes
    act(bias) in the first sweep), so after max-level + 1 sweeps the outputs
    equal the feedforward oracle's bit for bit; further sweeps change
    nothing."""
    pop = synth.control(seed=40 + seed, P=40, B=6)
    _, level, status = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O)
    y_ff, _ = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
    for p in range(pop.P):
        if status[p]:
            continue
        depth = int(level[p].max())
        for K in (depth + 1, depth + 4):
            y, _ = oracle.forward_recurrent(pop.nodes[p:p + 1], pop.conns[p:p + 1],
                                            pop.inputs[p:p + 1], pop.I, pop.O, K)
            np.testing.assert_array_equal(y[0], y_ff[p])


def test_zero_sweeps_give_zero_outputs():
    pop = synth.recurrent_control(seed=3, P=20, B=4)
    y, beta = oracle.forward_recurrent(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, 0)
    _, _, status = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O, recurrent=True)
    assert np.all(y[status == 0] == 0.0) and np.all(beta[status == 0] == 0.0)
    assert np.all(np.isnan(y[status != 0]))


# ---------------------------------------------------------------- status
def _status(nodes, conns, I=2, O=1, recurrent=True):
    n, c = genome(6, 8, nodes, conns)
    return int(oracle.transform(n, c, I, O, recurrent=recurrent)[2][0])


def test_cycles_are_allowed_other_faults_are_not():
    base = {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0), 2: (2, 0, 1, 0, 0), 3: (9, 0, 1, 0, 0)}
    loop = {0: (0, 9, 1, 1.0), 1: (9, 2, 1, 1.0), 2: (2, 9, 1, 1.0), 3: (9, 9, 1, 0.5)}
    assert _status(base, loop) == 0
    assert _status(base, loop, recurrent=False) == oracle.CYCLE
    assert _status(base, {**loop, 4: (5, 9, 1, 1.0)}) == oracle.BAD_REF
    assert _status(base, {**loop, 4: (9, 1, 1, 1.0)}) == oracle.INTO_INPUT
    assert _status(base, {**loop, 4: (9, 9, 1, 2.0)}) == oracle.DUP_EDGE
    assert _status(base, {**loop, 4: (9, 2, 0.5, 1.0)}) == oracle.BAD_VALUE
    assert _status({**base, 4: (9, 0, 1, 0, 0)}, loop) == oracle.DUP_KEY
    del base[2]
    assert _status(base, {0: (0, 9, 1, 1.0)}) == oracle.MISSING_IO


def test_recurrent_order_is_key_order_with_level_zero():
    pop = synth.recurrent_control(seed=4, P=30, B=1)
    order, level, status = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O,
                                            recurrent=True)
    for p in range(pop.P):
        valid = np.flatnonzero(~np.isnan(pop.nodes[p, :, 0]))
        if status[p]:
            assert np.all(order[p] == -1) and np.all(level[p] == -1)
            continue
        keys = pop.nodes[p, valid, 0]
        np.testing.assert_array_equal(order[p, :len(valid)], valid[np.argsort(keys)])
        assert np.all(order[p, len(valid):] == -1)
        assert np.all(level[p, valid] == 0)


# ---------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(4))
def test_storage_permutation_and_padding_invariance(seed):
    """Shuffling node and connection rows, and adding NaN rows and disabled
    rows with arbitrary content, leaves the recurrent outputs bit-identical."""
    pop = synth.recurrent_control(seed=60 + seed, P=12, B=5)
    rng = np.random.default_rng(seed)
    K = 4
    y0, _ = oracle.forward_recurrent(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, K)
    N, C = pop.nodes.shape[1], pop.conns.shape[1]
    n2 = np.full((pop.P, N + 5, 5), np.nan, np.float32)
    c2 = np.full((pop.P, C + 7, 4), np.nan, np.float32)
    for p in range(pop.P):
        n2[p, rng.permutation(N + 5)[:N]] = pop.nodes[p]
        cp = np.concatenate([pop.conns[p], np.full((7, 4), np.nan, np.float32)])
        cp[C:C + 3] = [[1e9, NAN, 0.0, NAN]] * 3   # disabled junk rows
        c2[p] = cp[rng.permutation(C + 7)]
    y1, _ = oracle.forward_recurrent(n2, c2, pop.inputs, pop.I, pop.O, K)
    np.testing.assert_array_equal(y0, y1)


# ------------------------------------------------------ fp32 error bound
@pytest.mark.parametrize("K", [1, 3, 6])
def test_beta_bounds_an_fp32_recurrent_evaluation(K):
    pop = synth.recurrent_control(seed=8, P=200, B=8)
    y64, beta = oracle.forward_recurrent(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, K)
    y32 = oracle.forward_recurrent(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, K,
                                   precision="f32")
    ok, stats = oracle.within_tolerance(y32, y64, beta, atol=0.0)
    assert stats["n_fail"] == 0, stats
