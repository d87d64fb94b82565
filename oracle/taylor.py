"""Truncation order and step size for the Taylor propagator (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper says the CTQW state is psi(t) = exp(-iHt) psi(0) (Sec. 3.1) but not
how the exponential is evaluated.  The engine uses the order-K Taylor series
T_K(x) = sum_{k<=K} x^k / k! with x = -i H dt, applied `steps` times.  With
rho = dt * ||H|| the remainder of one step obeys

    || exp(-iH dt) - T_K(-iH dt) ||  <=  sum_{k>K} rho^k / k!
                                     <=  rho^(K+1)/(K+1)! * (K+2)/(K+2-rho),

(the tail of the exponential series bounded by a geometric series, valid
for rho < K+2), and since exp(-iH dt) is unitary the error after `steps`
steps is at most `steps` times that.  ||H|| is bounded by the largest
absolute row sum of H = -gamma A - sum_M |v><v|, i.e. max_v gamma*d(v) + [v in M].

The rule: K is the smallest order in [1, 64] for which
steps * bound(rho, K) <= tol.  When only the total time is fixed, the step
count is the smallest one keeping rho <= rho_max, and dt = t_total / steps.
"""
from __future__ import annotations

import math

import numpy as np

K_MAX = 64


def h_norm_bound(degrees, gamma: float, marked) -> float:
    """max_v gamma*d(v) + [v in M] (the infinity norm of H)."""
    d = np.asarray(degrees, dtype=np.float64)
    if d.size == 0:
        return 0.0
    row = gamma * d
    if marked is not None and len(marked):
        m = np.zeros(d.size, dtype=np.float64)
        m[np.asarray(marked, dtype=np.int64)] = 1.0
        row = row + m
    return float(row.max())


def tail_bound(rho: float, K: int) -> float:
    """Upper bound on sum_{k>K} rho^k/k!."""
    if rho <= 0.0:
        return 0.0
    if rho >= K + 2:
        return math.inf
    lead = math.exp((K + 1) * math.log(rho) - math.lgamma(K + 2))
    return lead * (K + 2) / (K + 2 - rho)


def taylor_order(rho: float, steps: int, tol: float) -> int:
    """Smallest K in [1, K_MAX] with steps * tail_bound(rho, K) <= tol; -1 if none."""
    for K in range(1, K_MAX + 1):
        if steps * tail_bound(rho, K) <= tol:
            return K
    return -1


def taylor_plan(h_bound: float, t_total: float, rho_max: float, tol: float):
    """(K, dt, steps) for a total time t_total with rho = dt*h_bound <= rho_max."""
    if t_total <= 0.0:
        return 1, 0.0, 0
    steps = max(1, math.ceil(t_total * h_bound / rho_max)) if h_bound > 0 else 1
    dt = t_total / steps
    return taylor_order(dt * h_bound, steps, tol), dt, steps
