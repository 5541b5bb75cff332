"""HyperNEAT substrate oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it.

The paper supports HyperNEAT (Section 1; Section 4.3, feature-rich
extensions) without defining it; the reading here follows the method it
cites: a CPPN genome, queried on pairs of substrate points, paints the
connection weights of a larger network, the substrate.

* Substrate: the side x side grid of the CPPN queries, S = side^2 points,
  point p at (c[p % side], c[p // side]) with c[i] = -1 + 2 i / (side - 1).
  The same points form the input plane and the output plane.
* Weights: w[p1, p2] = CPPN(x1, y1, x2, y2, 1) for source p1 (input plane)
  and target p2 (output plane), i.e. query q = p1 S + p2 of the grid.
* Expression threshold theta (HyperNEAT's pruning of weak connections, no
  rescaling): w'[p1, p2] = 0 where |w| < theta, else w (NaN stays NaN).
* Substrate forward for input planes x_b (b < B, shared by every genome):
  y_b[p2] = tanh(sum_p1 w'[p1, p2] x_b[p1]).
* Genomes that the transformation rejects give NaN outputs.

The reference arithmetic is float64: the CPPN comes from the C oracle (with
its fp32 error bound beta), the contraction is numpy's matmul.  ``forward``
also returns a first-order bound on the error of an fp32 evaluation of the
same definition, in which a threshold decision counts as uncertain when
|w| is within the weight's own fp32 allowance (1e-5 + 2 beta) of theta.
"""
from __future__ import annotations

import numpy as np

import oracle
from workloads import synth

THRESHOLD = 0.2
U32 = 2.0 ** -24


def weights(nodes, conns, side: int):
    """CPPN weights [P, S, S] (float64) and their fp32 error bounds."""
    S = side * side
    x = synth.grid_queries(0, S * S, side)
    y, beta = oracle.forward(nodes, conns, x, 5, 1, shared_inputs=True)
    P = y.shape[0]
    return y.reshape(P, S, S), beta.reshape(P, S, S)


def forward(nodes, conns, side: int, X, theta: float = THRESHOLD):
    """Substrate outputs [P, B, S] (float64) and an fp32 error bound of the
    same shape (inf where fp32 may overflow)."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    S = side * side
    if X.ndim != 2 or X.shape[1] != S:
        raise ValueError("X must be [B, side^2]")
    W, bw = weights(nodes, conns, side)
    with np.errstate(invalid="ignore"):
        keep = ~(np.abs(W) < theta)
        delta = 1e-5 + 2.0 * bw
        uncertain = np.abs(np.abs(W) - theta) <= delta
    Wp = np.where(keep, W, 0.0)
    # error of the fp32 weight as the kernel uses it
    ew = np.where(uncertain, np.abs(W) + delta, np.where(keep, delta, 0.0))
    ax = np.abs(X)
    gamma = S * U32 / (1.0 - S * U32)
    Y = np.empty((W.shape[0], X.shape[0], S))
    bound = np.empty_like(Y)
    with np.errstate(invalid="ignore", over="ignore"):
        for p in range(W.shape[0]):
            z = X @ Wp[p]
            ez = ax @ ew[p] + gamma * (ax @ np.abs(Wp[p])) + U32 * np.abs(z)
            y = np.tanh(z)
            Y[p] = y
            # tanh is 1-Lipschitz; its fp32 evaluation adds 8u|y| + 4u
            bound[p] = ez + 8.0 * U32 * np.abs(y) + 4.0 * U32
    bound = np.where(np.isnan(bound) & ~np.isnan(Y), np.inf, bound)
    bound = np.where(np.isnan(Y), 0.0, bound)
    return Y, bound
