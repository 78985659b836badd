"""Plain CPU oracle of the affine-invariant ensemble sampler (stretch move).

TEST INFRASTRUCTURE ONLY, under the same rules as ``excursion_set``: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
it shares no code with the GPU path.

What it computes.  Section 2.3 samples the parameter space with the affine
invariant ensemble sampler of Goodman & Weare (2010) in the parallel form of
its public implementations: the ensemble of W walkers is split into two
halves, and each half in turn moves every one of its walkers X_k by a stretch
move along the line through a walker X_j drawn uniformly from the other half:

    Y = X_j + z (X_k - X_j),  z drawn from g(z) ~ 1 / sqrt(z) on [1/a, a],

accepted with probability min(1, z^(d-1) p(Y) / p(X_k)) in d dimensions.  All
proposals of a half use the other half's positions from before that half
moves, so the walkers of a half are independent.  Here p is the likelihood of
21CMMC: ln p = -chi^2 / 2 summed over redshifts inside the prior box and -inf
outside it (uniform priors, Section 3.2), over the parameters with the virial
temperature as its decimal logarithm, as the paper quotes it.

Random numbers are inputs: for every half-step and active walker three
uniforms in [0, 1): u0 picks the partner, j = floor(u0 n_other); u1 gives
z = ((a - 1) u1 + 1)^2 / a (the inverse of the CDF of g); u2 accepts when
ln u2 < (d - 1) ln z + ln p(Y) - ln p(X_k).  The first half is walkers
[0, W/2), the second [W/2, W); a step moves the first half, then the second.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np

STRETCH_A = 2.0   # the scale parameter of g(z) used by Goodman & Weare and the public samplers


def stretch_factor(u: float, a: float = STRETCH_A) -> float:
    """z with CDF(z) = u for g(z) proportional to 1 / sqrt(z) on [1/a, a]."""
    return ((a - 1.0) * u + 1.0) ** 2 / a


def half_step(x: np.ndarray, lp: np.ndarray, first: bool, u: np.ndarray,
              log_prob: Callable[[np.ndarray], float], a: float = STRETCH_A):
    """Moves one half of the ensemble in place; returns the accept flags of its walkers.

    x: (W, d) positions, lp: (W,) their ln p, u: (W/2, 3) uniforms of this half.
    """
    w, d = x.shape
    h = w // 2
    active = range(0, h) if first else range(h, w)
    other = np.arange(h, w) if first else np.arange(0, h)
    start = x.copy()                  # the other half as it was before this half moves
    accepted = np.zeros(h, dtype=bool)
    for i, k in enumerate(active):
        j = other[min(int(u[i, 0] * len(other)), len(other) - 1)]
        z = stretch_factor(float(u[i, 1]), a)
        y = start[j] + z * (start[k] - start[j])
        lp_y = log_prob(y)
        log_r = (d - 1) * math.log(z) + lp_y - lp[k]
        log_u = math.log(u[i, 2]) if u[i, 2] > 0.0 else -math.inf
        if log_u < log_r:
            x[k] = y
            lp[k] = lp_y
            accepted[i] = True
    return accepted


def step(x: np.ndarray, lp: np.ndarray, u: np.ndarray, log_prob: Callable[[np.ndarray], float],
         a: float = STRETCH_A) -> np.ndarray:
    """One ensemble step (both halves, first then second); u: (2, W/2, 3).  Returns (W,) accept flags."""
    acc_a = half_step(x, lp, True, u[0], log_prob, a)
    acc_b = half_step(x, lp, False, u[1], log_prob, a)
    return np.concatenate([acc_a, acc_b])


def box_prior(lo: Sequence[float], hi: Sequence[float], log_like: Callable[[np.ndarray], float]):
    """ln p = log_like inside lo <= x <= hi (every coordinate), -inf outside."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)

    def log_prob(x):
        if np.all(x >= lo) and np.all(x <= hi):
            return float(log_like(x))
        return -math.inf
    return log_prob
