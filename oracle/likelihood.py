"""FP64 CPU oracle of the chi^2 likelihood epilogue.

TEST INFRASTRUCTURE ONLY, under the same rules as ``excursion_set``: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
it shares no code with the GPU path.

What it computes (Section 2.5 of Greig & Mesinger 2015, and the multi-epoch
combination of Section 3.4): the model 21 cm power spectrum of a walker is
compared with a mock observation through a chi^2 statistic restricted to
0.15 <= k <= 1.0 Mpc^-1.  The error of a mock bin is its observational noise
(thermal noise plus sample variance, here an input: the 21cmSense noise is
not available) with a constant multiplicative modelling error of 25 per cent
of the mock power added in quadrature.  The chi^2 of several redshifts are
added linearly.

Readings taken here (also listed in the design notes):
* the statistic compares Delta^2_21(k_b) = k_b^3 P_b / (2 pi^2) bin by bin on
  the model's own binning, with the mock given on the same bins;
* a bin takes part when it holds modes and its count-weighted mean |k|, k_b,
  lies in [k_lo, k_hi] (both edges included);
* a bin whose total variance is zero (no noise and zero mock power) is left
  out instead of dividing by zero.
"""
from __future__ import annotations

from typing import Iterable, Sequence

import numpy as np

MODEL_ERROR = 0.25   # multiplicative modelling error of the mock power (Section 2.5)
K_LO = 0.15          # Mpc^-1, lower end of the fitted k range (Section 2.5)
K_HI = 1.0           # Mpc^-1, upper end (the shot-noise cut of Section 2.5)


def likelihood_bins(k_mean: Sequence[float], counts: Sequence[float], k_lo: float = K_LO,
                    k_hi: float = K_HI) -> np.ndarray:
    """Boolean mask of the bins that enter the chi^2: modes present, k_lo <= k_b <= k_hi."""
    k = np.asarray(k_mean, dtype=np.float64)
    c = np.asarray(counts, dtype=np.float64)
    return (c > 0) & (k >= k_lo) & (k <= k_hi)


def bin_variance(delta2_mock: Sequence[float], noise_sigma: Sequence[float],
                 model_err: float = MODEL_ERROR) -> np.ndarray:
    """Total variance of each mock bin: noise^2 + (model_err * Delta^2_mock)^2."""
    m = np.asarray(delta2_mock, dtype=np.float64)
    s = np.asarray(noise_sigma, dtype=np.float64)
    return s * s + (model_err * m) ** 2


def chi2(delta2_model: Sequence[float], delta2_mock: Sequence[float], noise_sigma: Sequence[float],
         k_mean: Sequence[float], counts: Sequence[float], model_err: float = MODEL_ERROR,
         k_lo: float = K_LO, k_hi: float = K_HI) -> float:
    """chi^2 of one redshift: sum over the fitted bins of (model - mock)^2 / variance."""
    use = likelihood_bins(k_mean, counts, k_lo, k_hi)
    var = bin_variance(delta2_mock, noise_sigma, model_err)
    model = np.asarray(delta2_model, dtype=np.float64)
    mock = np.asarray(delta2_mock, dtype=np.float64)
    total = 0.0
    for b in range(len(model)):  # plain sum in bin order
        if use[b] and var[b] > 0.0:
            r = model[b] - mock[b]
            total += r * r / var[b]
    return total


def chi2_total(per_redshift: Iterable[float]) -> float:
    """Multi-epoch statistic: the chi^2 of the redshifts added linearly (Section 3.4)."""
    total = 0.0
    for c in per_redshift:
        total += float(c)
    return total
