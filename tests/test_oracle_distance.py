"""Pins for the oracle's compatibility distance (NEAT's form; the paper names
the disjoint and homologous coefficients, Appendix A): a hand-computed
pair, identity, symmetry, storage invariance, and exact increments when one
gene is added or one attribute changed."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import synth
from tests.helpers import genome, stack


def _pair():
    """Two hand-made genomes (I = 1, O = 1).

    A: nodes 0 (0, 1, identity, sum), 1 (0.5, 1, sigmoid, sum), 5 (-1, 1,
       tanh, sum); conns 0->5 (on, 0.5), 5->1 (on, -1), 0->1 (off, 2).
    B: nodes 0 (0, 1, identity, sum), 1 (0.25, 1, sigmoid, product), 7;
       conns 0->1 (on, 1.5), 0->7 (on, 1), 7->1 (on, 1).
    Nodes: 3 and 3 genes, homologous 0 (distance 0) and 1 (|0.5 - 0.25| +
    [agg differs] = 1.25), 2 disjoint: (1 * 2 + 0.5 * 1.25) / 3 = 0.875.
    Connections: 3 and 3 genes, homologous 0->1 (|2 - 1.5| + [enabled
    differs] = 1.5), 4 disjoint: (1 * 4 + 0.5 * 1.5) / 3 = 19 / 12.
    Distance 0.875 + 19 / 12 = 59 / 24."""
    a = genome(4, 4, {0: (0, 0, 1, 0, 0), 1: (1, 0.5, 1, 2, 0), 3: (5, -1, 1, 1, 0)},
               {0: (0, 5, 1, 0.5), 1: (5, 1, 1, -1.0), 3: (0, 1, 0, 2.0)})
    b = genome(4, 4, {0: (0, 0, 1, 0, 0), 1: (1, 0.25, 1, 2, 1), 2: (7, 0, 1, 0, 0)},
               {1: (0, 1, 1, 1.5), 2: (0, 7, 1, 1.0), 3: (7, 1, 1, 1.0)})
    return a, b


def test_hand_computed_pair():
    (an, ac), (bn, bc) = _pair()
    d, bound = oracle.distance(an, ac, bn, bc)
    assert d[0, 0] == pytest.approx(59.0 / 24.0, rel=1e-15)
    d2, _ = oracle.distance(an, ac, bn, bc, c_disjoint=2.0, c_homologous=0.0)
    assert d2[0, 0] == pytest.approx(2 * 2 / 3 + 2 * 4 / 3, rel=1e-15)


def _unique(seed, P):
    return synth.make_population(np.random.default_rng(seed), P, 20, 40, 3, 2, 12,
                                 synth._k_uniform(40), synth.CONTROL_ACTS, synth.ALL_AGGS)


def test_identity_and_symmetry():
    pop = _unique(1, 12)
    d, _ = oracle.distance(pop.nodes, pop.conns, pop.nodes, pop.conns)
    assert np.all(np.diag(d) == 0.0)
    np.testing.assert_allclose(d, d.T, rtol=1e-14, atol=0)
    assert np.all(d[~np.eye(12, dtype=bool)] > 0)


def test_storage_permutation_invariance():
    pop = _unique(2, 6)
    rng = np.random.default_rng(3)
    n2, c2 = pop.nodes.copy(), pop.conns.copy()
    for p in range(pop.P):
        n2[p] = n2[p, rng.permutation(n2.shape[1])]
        c2[p] = c2[p, rng.permutation(c2.shape[1])]
    d0, _ = oracle.distance(pop.nodes, pop.conns, pop.nodes[:3], pop.conns[:3])
    d1, _ = oracle.distance(n2, c2, n2[:3], c2[:3])
    np.testing.assert_array_equal(d0, d1)


def test_exact_increments():
    """One extra disjoint connection gene in B raises the connection
    numerator by c_disjoint; one homologous weight moved by delta raises it
    by c_homologous |delta| (counts chosen so the denominators stay put)."""
    (an, ac), (bn, bc) = _pair()
    base, _ = oracle.distance(an, ac, bn, bc, 1.0, 0.5)
    bc2 = bc.copy()
    bc2[0, 0] = (1, 7, 1, 0.25)         # B gains a 4th connection gene: max 3 -> 4
    d, _ = oracle.distance(an, ac, bn, bc2, 1.0, 0.5)
    assert d[0, 0] == pytest.approx(0.875 + (5 + 0.75) / 4, rel=1e-15)
    bc3 = bc.copy()
    bc3[0, 1, 3] = 1.5 + 0.125          # homologous 0->1: |2 - 1.625| = 0.375
    d, _ = oracle.distance(an, ac, bn, bc3, 1.0, 0.5)
    assert d[0, 0] - base[0, 0] == pytest.approx(0.5 * (-0.125) / 3, abs=1e-15)


def test_bound_covers_an_fp32_evaluation():
    """The same sums evaluated in float32 (differences rounded, sums in
    gene order) stay within the bound."""
    pop = _unique(5, 30)
    d, bound = oracle.distance(pop.nodes, pop.conns, pop.nodes[:5], pop.conns[:5], 1.0, 0.5)
    f = np.float32
    for p in range(pop.P):
        for q in range(5):
            tot = f(0)
            for A, B, node in ((pop.nodes[p], pop.nodes[q], True),
                               (pop.conns[p], pop.conns[q], False)):
                a = A[~np.isnan(A[:, 0])]
                b = B[~np.isnan(B[:, 0])]
                h, s = 0, f(0)
                for x in a:
                    m = (b[:, 0] == x[0]) if node else ((b[:, 0] == x[0]) & (b[:, 1] == x[1]))
                    if m.any():
                        y = b[np.argmax(m)]
                        h += 1
                        if node:
                            t = (abs(f(x[1]) - f(y[1])) + abs(f(x[2]) - f(y[2]))
                                 + f(x[3] != y[3]) + f(x[4] != y[4]))
                        else:
                            t = abs(f(x[3]) - f(y[3])) + f(x[2] != y[2])
                        s = f(s + t)
                mx = max(len(a), len(b))
                if mx:
                    tot = f(tot + f(f(f(len(a) + len(b) - 2 * h) + f(0.5) * s) / f(mx)))
            assert abs(float(tot) - d[p, q]) <= bound[p, q] + 1e-12, (p, q)
