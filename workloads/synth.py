"""Seeded synthetic populations and inputs.

This module only draws random genomes and input vectors; it holds none of the
method's arithmetic, so both the GPU path and the CPU oracle can be fed from
it.  Everything is drawn from ``numpy.random.default_rng(seed)`` (PCG64).

Genome encoding (Section 3.1 of the paper): node rows
``(key, bias, response, act, agg)`` and connection rows
``(in key, out key, enabled, weight)``, padded with NaN rows up to N_max and
C_max.  Input nodes carry keys 0..I-1 and output nodes keys I..I+O-1 (the
paper's genome interface), stored at rows 0..I+O-1; hidden nodes get distinct
keys drawn from [I+O, 16 N_max) and sit at random free rows, so NaN gaps
appear anywhere, not only at the tail.  Connections are drawn without
replacement from the pairs allowed by a random topological permutation of the
non-input nodes (input -> non-input, or u -> v with u before v), each enabled
with probability 0.7, and written to random rows.  Weights and biases are
N(0, 1), response is 1 (the paper's experiment settings).

Workloads (stand-ins for the paper's Brax control tasks, whose observation
and action sizes they take):

* ``tiny``: P=16, I=3, O=1, N_max=8, C_max=16, sigmoid + sum, 32 shared
  inputs U[-1, 1], seed 0;
* ``control``: P=10000, I=17, O=6, N_max=50, C_max=200, 0..27 hidden nodes,
  mixed activations and aggregations, B=1000 N(0,1) inputs per genome, seed 1;
* ``uneven``: 64 populations, P, N_max and B log-uniform, C_max = 4 N_max,
  connection density U[0.1, 0.6], seed 2;
* ``served``: a pool of 128 populations for the request stream, seed 3;
* ``cppn``: P=1000, I=5 (x1, y1, x2, y2, 1), O=1, N_max=30, C_max=120, CPPN
  activations + sum, queried on all pairs of a 16x16 grid, seed 4;
* ``recurrent_control``: the control shapes with recurrent connections (any
  pair into a non-input node, self-loops and cycles included), seed 5.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# activation and aggregation codes of the node encoding
ACT_IDENTITY, ACT_TANH, ACT_SIGMOID, ACT_RELU, ACT_SIN, ACT_GAUSS, ACT_ABS = range(7)
AGG_SUM, AGG_PRODUCT, AGG_MAX, AGG_MIN, AGG_MEAN = range(5)

CONTROL_ACTS = (ACT_SIGMOID, ACT_TANH, ACT_RELU, ACT_IDENTITY, ACT_SIN)
ALL_AGGS = (AGG_SUM, AGG_PRODUCT, AGG_MAX, AGG_MIN, AGG_MEAN)
CPPN_ACTS = (ACT_SIN, ACT_GAUSS, ACT_ABS, ACT_TANH, ACT_SIGMOID)

P_ENABLED = 0.7


@dataclasses.dataclass
class Population:
    nodes: np.ndarray          # [P, N_max, 5] float32
    conns: np.ndarray          # [P, C_max, 4] float32
    I: int
    O: int
    inputs: Optional[np.ndarray] = None   # [P, B, I] or [B, I] (shared)
    shared_inputs: bool = False

    @property
    def P(self) -> int:
        return self.nodes.shape[0]

    @property
    def N_max(self) -> int:
        return self.nodes.shape[1]

    @property
    def C_max(self) -> int:
        return self.conns.shape[1]

    @property
    def B(self) -> int:
        if self.inputs is None:
            return 0
        return self.inputs.shape[0] if self.shared_inputs else self.inputs.shape[1]


_TRIU_CACHE = {}


def _triu(M: int):
    t = _TRIU_CACHE.get(M)
    if t is None:
        t = np.triu_indices(M, 1)
        _TRIU_CACHE[M] = t
    return t


def make_genome(rng, N_max: int, C_max: int, I: int, O: int, n_hidden: int,
                n_conns, acts: Sequence[int], aggs: Sequence[int],
                p_enabled: float = P_ENABLED, outputs_last: bool = False,
                nodes_out: Optional[np.ndarray] = None,
                conns_out: Optional[np.ndarray] = None, recurrent: bool = False):
    """Draw one genome into NaN-filled ``nodes_out`` [N_max,5] and
    ``conns_out`` [C_max,4] (allocated when None).

    ``n_conns`` is either an int or a callable mapping the number of allowed
    pairs to the number of connections to draw.  With ``outputs_last`` the
    topological permutation is hidden nodes first, then outputs (edges go
    from lower to higher generation index); otherwise it is random, so
    outputs may feed hidden nodes.  With ``recurrent`` every pair (input or
    non-input -> non-input) is allowed, self-loops and both directions
    included, so the enabled edges may form cycles."""
    assert I >= 1 and O >= 1 and I + O + n_hidden <= N_max
    nodes = nodes_out if nodes_out is not None else np.full((N_max, 5), np.nan, np.float32)
    conns = conns_out if conns_out is not None else np.full((C_max, 4), np.nan, np.float32)
    hidden_keys = (rng.choice(16 * N_max - (I + O), size=n_hidden, replace=False)
                   + (I + O)) if n_hidden else np.zeros(0, np.int64)
    hidden_rows = (rng.choice(N_max - (I + O), size=n_hidden, replace=False)
                   + (I + O)) if n_hidden else np.zeros(0, np.int64)
    rows = np.concatenate([np.arange(I + O), hidden_rows])
    keys = np.concatenate([np.arange(I + O), hidden_keys])
    n = I + O + n_hidden
    nodes[rows, 0] = keys
    nodes[rows, 1] = rng.standard_normal(n, dtype=np.float32)
    nodes[rows, 2] = 1.0
    nodes[rows, 3] = rng.choice(np.asarray(acts), n)
    nodes[rows, 4] = rng.choice(np.asarray(aggs), n)

    M = O + n_hidden
    nonin = np.concatenate([np.arange(I, I + O), hidden_keys])   # keys
    if outputs_last:
        topo = np.concatenate([hidden_keys[rng.permutation(n_hidden)],
                               np.arange(I, I + O)])
    else:
        topo = nonin[rng.permutation(M)]
    n_allowed = I * M + (M * M if recurrent else M * (M - 1) // 2)
    K = n_conns(n_allowed) if callable(n_conns) else int(n_conns)
    K = max(0, min(K, n_allowed, C_max))
    if K:
        q = rng.choice(n_allowed, size=K, replace=False)
        src = np.empty(K, np.int64)
        dst = np.empty(K, np.int64)
        a = q < I * M
        src[a] = q[a] // M
        dst[a] = topo[q[a] % M]
        qb = q[~a] - I * M
        if recurrent:
            src[~a] = nonin[qb // M]
            dst[~a] = nonin[qb % M]
        else:
            iu, ju = _triu(M)
            src[~a] = topo[iu[qb]]
            dst[~a] = topo[ju[qb]]
        crow = rng.choice(C_max, size=K, replace=False)
        conns[crow, 0] = src
        conns[crow, 1] = dst
        conns[crow, 2] = (rng.random(K) < p_enabled).astype(np.float32)
        conns[crow, 3] = rng.standard_normal(K, dtype=np.float32)
    return nodes, conns


def make_population(rng, P: int, N_max: int, C_max: int, I: int, O: int,
                    hidden_max: int, conns_fn, acts, aggs,
                    outputs_last: bool = False, recurrent: bool = False) -> Population:
    nodes = np.full((P, N_max, 5), np.nan, np.float32)
    conns = np.full((P, C_max, 4), np.nan, np.float32)
    hidden_max = min(hidden_max, N_max - I - O)
    for p in range(P):
        h = int(rng.integers(0, hidden_max + 1))
        make_genome(rng, N_max, C_max, I, O, h, lambda na: conns_fn(rng, na),
                    acts, aggs, outputs_last=outputs_last,
                    nodes_out=nodes[p], conns_out=conns[p], recurrent=recurrent)
    return Population(nodes, conns, I, O)


def _k_uniform(cap: int):
    """K ~ U{1 .. min(cap, allowed)}."""
    def fn(rng, n_allowed):
        hi = min(cap, n_allowed)
        return int(rng.integers(1, hi + 1)) if hi >= 1 else 0
    return fn


def _k_density(cap: int):
    """K = round(U[0.1, 0.6] * min(cap, allowed))."""
    def fn(rng, n_allowed):
        return int(round(rng.uniform(0.1, 0.6) * min(cap, n_allowed)))
    return fn


def tiny(seed: int = 0) -> Population:
    """P=16, I=3, O=1, N_max=8, C_max=16; sigmoid + sum; 32 shared inputs."""
    rng = np.random.default_rng(seed)
    pop = make_population(rng, 16, 8, 16, 3, 1, 4, _k_uniform(16),
                          (ACT_SIGMOID,), (AGG_SUM,), outputs_last=True)
    pop.inputs = rng.uniform(-1.0, 1.0, size=(32, 3)).astype(np.float32)
    pop.shared_inputs = True
    return pop


def control(seed: int = 1, P: int = 10000, B: int = 1000,
            with_inputs: bool = True) -> Population:
    """P=10000, I=17, O=6, N_max=50, C_max=200, B=1000 per-genome inputs."""
    rng = np.random.default_rng(seed)
    pop = make_population(rng, P, 50, 200, 17, 6, 27, _k_uniform(200),
                          CONTROL_ACTS, ALL_AGGS)
    if with_inputs:
        pop.inputs = rng.standard_normal((P, B, 17), dtype=np.float32)
    return pop


def recurrent_control(seed: int = 5, P: int = 10000, B: int = 1000,
                      with_inputs: bool = True) -> Population:
    """The control-policy shapes (P=10000, I=17, O=6, N_max=50, C_max=200,
    B=1000) with recurrent connections: any pair into a non-input node,
    self-loops and cycles included."""
    rng = np.random.default_rng(seed)
    pop = make_population(rng, P, 50, 200, 17, 6, 27, _k_uniform(200),
                          CONTROL_ACTS, ALL_AGGS, recurrent=True)
    if with_inputs:
        pop.inputs = rng.standard_normal((P, B, 17), dtype=np.float32)
    return pop


def _log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def uneven_population(rng, P_range, N_range, B_range, with_inputs=True) -> Population:
    """One population of the uneven workloads: C_max = 4 N_max, I and O
    drawn per population, hidden nodes U{0..N_max-I-O}, density U[0.1,0.6]."""
    P = _log_uniform_int(rng, *P_range)
    N = _log_uniform_int(rng, *N_range)
    B = _log_uniform_int(rng, *B_range)
    I = int(rng.integers(2, min(24, N // 2) + 1))
    O = int(rng.integers(1, min(8, N - I - 1) + 1))
    pop = make_population(rng, P, N, 4 * N, I, O, N - I - O, _k_density(4 * N),
                          CONTROL_ACTS, ALL_AGGS)
    if with_inputs:
        pop.inputs = rng.standard_normal((P, B, I), dtype=np.float32)
    return pop


def uneven(seed: int = 2, n_pops: int = 64, P_range=(100, 4096),
           N_range=(10, 400), B_range=(1, 512)) -> List[Population]:
    rng = np.random.default_rng(seed)
    return [uneven_population(rng, P_range, N_range, B_range) for _ in range(n_pops)]


def served_pool(seed: int = 3, n_pops: int = 128, P_range=(64, 8192),
                N_range=(8, 256)) -> List[Population]:
    """Resident populations for the request stream (inputs come per request)."""
    rng = np.random.default_rng(seed)
    return [uneven_population(rng, P_range, N_range, (1, 1), with_inputs=False)
            for _ in range(n_pops)]


GRID_SIDE = 16


def grid_coords(side: int = GRID_SIDE) -> np.ndarray:
    """The side substrate coordinates -1 + 2 i / (side - 1), rounded once to
    fp32."""
    i = np.arange(side, dtype=np.float64)
    return ((2.0 * i - (side - 1)) / (side - 1)).astype(np.float32)


def grid_queries(first: int = 0, count: int = None, side: int = GRID_SIDE) -> np.ndarray:
    """CPPN inputs [count, 5] for queries first .. first+count-1 (all
    side^4 of them by default).

    Grid point p has x = coord[p % side], y = coord[p // side]; query q pairs
    point q // side^2 (x1, y1) with point q % side^2 (x2, y2); the fifth
    input is the constant 1."""
    if count is None:
        count = side ** 4 - first
    c = grid_coords(side)
    S = side * side
    q = np.arange(first, first + count, dtype=np.int64)
    a, b = q // S, q % S
    out = np.empty((count, 5), np.float32)
    out[:, 0] = c[a % side]
    out[:, 1] = c[a // side]
    out[:, 2] = c[b % side]
    out[:, 3] = c[b // side]
    out[:, 4] = 1.0
    return out


def substrate_inputs(seed: int = 6, B: int = 256, side: int = GRID_SIDE) -> np.ndarray:
    """B input planes for a HyperNEAT substrate of side x side points
    ([B, side^2], U[-1, 1]), shared by every genome."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(B, side * side)).astype(np.float32)


def cppn(seed: int = 4, P: int = 1000) -> Population:
    """P=1000 CPPN genomes, I=5, O=1, N_max=30, C_max=120."""
    rng = np.random.default_rng(seed)
    return make_population(rng, P, 30, 120, 5, 1, 24, _k_uniform(120),
                           CPPN_ACTS, (AGG_SUM,))


def input_pool(seed: int, n_floats: int) -> np.ndarray:
    """A flat pool of N(0,1) fp32 values that request inputs are cut from."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n_floats, dtype=np.float32)
