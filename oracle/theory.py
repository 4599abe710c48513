"""Theorem 1 (Section 5): Guaranteed-Mode conditional recall lower bound.

With M subspaces, single-subspace collision probability p* of the true nearest
neighbour x*, and selection threshold tau < M p*, Hoeffding's inequality gives

    P(x* in C) >= 1 - exp(-2 (M p* - tau)^2 / M).

The proof bounds P(S <= tau) where S ~ Binomial(M, p*) and uses
P(S < tau) <= P(S <= tau).  The bound is vacuous (returned as 0 here) when
M p* <= tau, which is the case the candidate fallback covers.
"""
from __future__ import annotations

import math


def recall_lower_bound(m: int, p: float, tau: float) -> float:
    mu = m * p
    if mu <= tau:
        return 0.0
    return 1.0 - math.exp(-2.0 * (mu - tau) ** 2 / m)


def binomial_tail_ge(m: int, p: float, tau: int) -> float:
    """Exact P[Binomial(M, p) >= tau]."""
    tau = max(0, int(math.ceil(tau)))
    return sum(math.comb(m, s) * p ** s * (1.0 - p) ** (m - s) for s in range(tau, m + 1))
