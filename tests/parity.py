"""The fp32 parity assertion every GPU test uses against the fp64 oracle.

Rule (oracle.within_tolerance): an output passes when |y - y64| <= 1e-5 +
2 beta, where beta is the oracle's first-order bound on the error of an fp32
evaluation of the same graph; both NaN passes; beta = inf (fp32 may
overflow) is only counted.  On top of that, every output whose bound is
small (beta <= 1e-6, "well conditioned") must be within the flat 1e-5 the
outputs are held to: the beta relaxation is an exception for outputs
whose own rounding can exceed 1e-5, not a looser rule for all of them.
The share of outputs under the exception is printed with every check."""
from __future__ import annotations

import oracle

ATOL = 1e-5


def assert_parity(y, y64, beta, label=""):
    ok, stats = oracle.within_tolerance(y, y64, beta, atol=ATOL)
    n = max(stats["n"], 1)
    stats["ill_conditioned_fraction"] = stats["n_ill_conditioned"] / n
    print("parity", label, stats, flush=True)
    assert stats["n_fail"] == 0, (label, stats)
    assert stats["max_abs_err_well_conditioned"] <= ATOL, (label, stats)
    return stats
