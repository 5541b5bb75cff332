"""Pins for the HyperNEAT substrate oracle (``oracle/substrate.py``): brute
force on tiny substrates, closed forms for CPPNs whose weights are a constant
or a coordinate, the two ends of the threshold, and the fp32 bound against
an fp32 evaluation of the same definition."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import substrate
from workloads import synth
from tests.helpers import genome, stack


def _cppn_pop(seed, P):
    rng = np.random.default_rng(seed)
    return synth.make_population(rng, P, 12, 30, 5, 1, 6, synth._k_uniform(30),
                                 synth.CPPN_ACTS, (synth.AGG_SUM,))


@pytest.mark.parametrize("side", [4, 8])
def test_brute_force_loops(side):
    """Per output a plain loop over source points: sum of w' x, then tanh."""
    pop = _cppn_pop(side, 3)
    S = side * side
    X = synth.substrate_inputs(seed=side, B=4, side=side)
    Y, _ = substrate.forward(pop.nodes, pop.conns, side, X, theta=0.2)
    q = synth.grid_queries(0, S * S, side)
    w, _ = oracle.forward(pop.nodes, pop.conns, q, 5, 1, shared_inputs=True)
    for p in range(pop.P):
        for b in range(X.shape[0]):
            for p2 in range(0, S, 5):
                acc = 0.0
                for p1 in range(S):
                    wv = w[p, p1 * S + p2, 0]
                    if abs(wv) >= 0.2:
                        acc += wv * float(X[b, p1])
                assert Y[p, b, p2] == pytest.approx(np.tanh(acc), rel=1e-12, abs=1e-13)


def _const_cppn(bias, act=0):
    """Output node with no edges: w = act(bias) for every pair."""
    nodes = {k: (k, 0.0, 1.0, 0, 0) for k in range(6)}
    nodes[5] = (5, bias, 1.0, act, 0)
    return genome(6, 2, nodes, {})


@pytest.mark.parametrize("theta,kept", [(0.25, True), (0.5, True), (0.5000001, False),
                                        (0.0, True), (np.inf, False)])
def test_constant_weight_closed_form(theta, kept):
    """w = 0.5 everywhere: y_b = tanh(0.5 sum_p x_b[p]) when kept (|w| >=
    theta, equality kept), 0 when pruned."""
    n, c = _const_cppn(0.5)
    side = 4
    X = synth.substrate_inputs(seed=3, B=6, side=side)
    Y, _ = substrate.forward(n, c, side, X, theta=theta)
    ref = np.tanh(0.5 * X.astype(np.float64).sum(axis=1)) if kept else np.zeros(6)
    np.testing.assert_allclose(Y[0], np.repeat(ref[:, None], 16, axis=1), rtol=1e-13,
                               atol=1e-15)


def test_coordinate_weight_closed_form():
    """Output = identity(x1): w[p1, p2] = x coordinate of p1, so y_b[p2] =
    tanh(sum over p1 with |c(p1)| >= theta of c(p1) x_b[p1]) for every p2."""
    nodes = {k: (k, 0.0, 1.0, 0, 0) for k in range(6)}
    n, c = genome(6, 2, nodes, {0: (0, 5, 1, 1.0)})
    side = 8
    X = synth.substrate_inputs(seed=4, B=5, side=side)
    Y, _ = substrate.forward(n, c, side, X, theta=0.3)
    cx = synth.grid_coords(side)[np.arange(side * side) % side].astype(np.float64)
    w = np.where(np.abs(cx) >= 0.3, cx, 0.0)
    ref = np.tanh(X.astype(np.float64) @ w)
    np.testing.assert_allclose(Y[0], np.repeat(ref[:, None], side * side, axis=1),
                               rtol=1e-13, atol=1e-15)


def test_rejected_genome_gives_nan():
    good = _const_cppn(0.5)
    bad_nodes = {k: (k, 0.0, 1.0, 0, 0) for k in range(6)}
    bad_nodes[5] = (5, 0.5, 1.0, 9, 0)           # activation code 9: BAD_VALUE
    bad = genome(6, 2, bad_nodes, {})
    n, c = stack([good, bad])
    Y, bound = substrate.forward(n, c, 4, synth.substrate_inputs(B=3, side=4))
    assert np.all(np.isfinite(Y[0])) and np.all(np.isnan(Y[1]))


def test_bound_covers_an_fp32_evaluation():
    """fp32 weights from the oracle's float instantiation, thresholded in
    fp32, contracted by a float32 matmul, tanh in float32: within twice the
    bound (and within the bound itself away from uncertain thresholds)."""
    side = 8
    S = side * side
    pop = _cppn_pop(11, 20)
    X = synth.substrate_inputs(seed=12, B=16, side=side)
    Y, bound = substrate.forward(pop.nodes, pop.conns, side, X)
    q = synth.grid_queries(0, S * S, side)
    w32 = oracle.forward(pop.nodes, pop.conns, q, 5, 1, shared_inputs=True,
                         precision="f32").reshape(pop.P, S, S)
    w32 = np.where(np.abs(w32) < np.float32(substrate.THRESHOLD), np.float32(0), w32)
    for p in range(pop.P):
        y32 = np.tanh(X @ w32[p]).astype(np.float64)
        ok, stats = oracle.within_tolerance(y32, Y[p], bound[p], atol=0.0)
        assert stats["n_fail"] == 0, stats
