"""Pins for the oracle's crossover (key-aligned genes, fitter parent's
structure): the two ends of the random numbers, identical parents, a
hand-made pair, storage permutation of the second parent, and structural
invariants (keys, NaN rows and disjoint genes always from the first
parent)."""
from __future__ import annotations

import numpy as np

import oracle
from workloads import synth
from tests.helpers import stack
from tests.test_oracle_distance import _pair


def _pop(seed, P):
    return synth.make_population(np.random.default_rng(seed), P, 20, 40, 3, 2, 12,
                                 synth._k_uniform(40), synth.CONTROL_ACTS, synth.ALL_AGGS)


def _same(a, b):
    return np.array_equal(np.nan_to_num(a, nan=7.5e30), np.nan_to_num(b, nan=7.5e30))


def test_random_numbers_at_the_ends():
    pop = _pop(1, 8)
    pairs = np.array([[i, (i + 3) % 8] for i in range(8)], np.int32)
    ones = (np.ones((8, 20)), np.ones((8, 40)))
    cn, cc = oracle.crossover(pop.nodes, pop.conns, pairs, *ones)
    assert _same(cn, pop.nodes[pairs[:, 0]]) and _same(cc, pop.conns[pairs[:, 0]])
    cn2, cc2 = oracle.crossover(pop.nodes, pop.conns, pairs, np.zeros((8, 20)),
                                np.zeros((8, 40)))
    # keys and row layout are p1's in every case
    assert _same(cn2[:, :, 0], pop.nodes[pairs[:, 0], :, 0])
    assert _same(cc2[:, :, :2], pop.conns[pairs[:, 0], :, :2])


def test_identical_parents():
    pop = _pop(2, 5)
    pairs = np.array([[i, i] for i in range(5)], np.int32)
    rng = np.random.default_rng(0)
    cn, cc = oracle.crossover(pop.nodes, pop.conns, pairs, rng.random((5, 20)),
                              rng.random((5, 40)))
    assert _same(cn, pop.nodes) and _same(cc, pop.conns)


def test_hand_made_pair():
    """All numbers 0: A's node 1 takes B's (0.25, 1, sigmoid, product); node
    5 (not in B) stays; A's 0->1 takes B's (enabled, 1.5); A's 0->5 and
    5->1 stay."""
    (an, ac), (bn, bc) = _pair()
    n, c = stack([(an, ac), (bn, bc)])
    cn, cc = oracle.crossover(n, c, np.array([[0, 1]], np.int32), np.zeros((1, 4)),
                              np.zeros((1, 4)))
    assert cn[0, 1].tolist() == [1, 0.25, 1, 2, 1]
    assert cn[0, 3].tolist() == [5, -1, 1, 1, 0]
    assert cn[0, 0].tolist() == [0, 0, 1, 0, 0]
    assert cc[0, 3].tolist() == [0, 1, 1, 1.5]
    assert cc[0, 0].tolist() == [0, 5, 1, 0.5] and cc[0, 1].tolist() == [5, 1, 1, -1]
    assert np.all(np.isnan(cn[0, 2])) and np.all(np.isnan(cc[0, 2]))


def test_second_parent_storage_permutation():
    """Permuting the second parent's rows (keys unique) changes nothing."""
    pop = _pop(3, 6)
    rng = np.random.default_rng(4)
    n2, c2 = pop.nodes.copy(), pop.conns.copy()
    for p in range(3, 6):
        n2[p] = n2[p, rng.permutation(20)]
        c2[p] = c2[p, rng.permutation(40)]
    pairs = np.array([[0, 3], [1, 4], [2, 5]], np.int32)
    r = (rng.random((3, 20)), rng.random((3, 40)))
    a = oracle.crossover(pop.nodes, pop.conns, pairs, *r)
    b = oracle.crossover(n2, c2, pairs, *r)
    assert _same(a[0], b[0]) and _same(a[1], b[1])


def test_child_attributes_come_from_a_parent():
    """Every child gene equals the p1 gene or its p2 partner, the partner
    exactly where the gene is homologous and its number is below 0.5."""
    pop = _pop(5, 10)
    rng = np.random.default_rng(6)
    pairs = rng.integers(0, 10, (12, 2)).astype(np.int32)
    rn, rcn = rng.random((12, 20)), rng.random((12, 40))
    cn, cc = oracle.crossover(pop.nodes, pop.conns, pairs, rn, rcn)
    for k, (a, b) in enumerate(pairs):
        bkeys = {float(x[0]): x for x in pop.nodes[b][::-1] if not np.isnan(x[0])}
        for r in range(20):
            x = pop.nodes[a, r]
            if np.isnan(x[0]):
                assert np.all(np.isnan(cn[k, r]))
                continue
            want = bkeys[float(x[0])] if (float(x[0]) in bkeys and rn[k, r] < 0.5) else x
            assert cn[k, r, 0] == x[0] and _same(cn[k, r, 1:], want[1:])
