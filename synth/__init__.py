"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only *generates inputs*: Gaussian random density boxes and walker
parameter draws.  It holds none of the excursion-set arithmetic (no filtering,
no collapse fractions, no thresholds, no power-spectrum estimator), so the GPU
path and the oracle stay independent while reading identical inputs.

Stand-ins.  The paper samples its parameter space on evolved 21CMFAST density
boxes built from a real cosmology (Section 2.5: 250 Mpc, 768^3 initial
conditions smoothed onto 128^3; the mock uses 500 Mpc, 1536^3 -> 256^3).  Those
boxes are not available, so a Gaussian random field with a fixed, smooth linear
power spectrum stands in for them:

    P(k, z) = D(z)^2 * A * k * (1 + (k / k0)^2)^-2,   k0 = 0.05 / Mpc,
    D(z)    = (1 + 9) / (1 + z)                       (growth normalised at z = 9),

with A fixed once so that the expected cell variance of the 64^3, 128 Mpc grid
at z = 9 is 0.6^2.  One realisation is drawn per (N, L) geometry and scaled by
D(z) to each redshift.  Values are Gaussian (no clamp at delta = -1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

PK_K0 = 0.05          # Mpc^-1, turnover scale of the synthetic spectrum
Z_REF = 9.0           # redshift at which A is normalised
CELL_STD_REF = 0.6    # target cell standard deviation on the reference grid
REF_GRID = (64, 128.0)  # (N, L / Mpc) of the reference grid

# Seeds: one density realisation per geometry, one walker draw per batch.
BOX_SEEDS = {(64, 128.0): 1, (128, 250.0): 2, (256, 250.0): 3, (256, 300.0): 4, (512, 400.0): 5}
WALKER_SEEDS = {"batched-256": 103, "uneven-mix": 104, "large-512": 105, "two-population-256": 106}

# Uniform priors (paper Section 2.1 ranges for zeta and R_mfp; log10 T_vir in [4, 6]).
PRIOR_LO = (5.0, 5.0, 4.0)
PRIOR_HI = (100.0, 20.0, 6.0)
# two-population walkers (zeta0, R_mfp, log10 T_feed, alpha, beta): the ranges
# of Section 2.1 for the first three and [-4/3, 10/3] for both indices (Section 4)
PRIOR2_LO = (5.0, 5.0, 4.0, -4.0 / 3.0, -4.0 / 3.0)
PRIOR2_HI = (100.0, 20.0, 5.301029995663981, 10.0 / 3.0, 10.0 / 3.0)


def growth(z: float) -> float:
    """Linear growth used to scale the synthetic box, normalised to 1 at z = 9."""
    return (1.0 + Z_REF) / (1.0 + z)


def _mode_k(n: int, box: float, half: bool) -> np.ndarray:
    kf = 2.0 * math.pi / box
    f = np.fft.fftfreq(n, d=1.0 / n)
    fl = np.fft.rfftfreq(n, d=1.0 / n) if half else f
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fl[None, None, :] ** 2
    return kf * np.sqrt(n2)


def _shape(k: np.ndarray, k0: float = PK_K0) -> np.ndarray:
    return k * (1.0 + (k / k0) ** 2) ** -2


def reference_amplitude(k0: float = PK_K0) -> float:
    """A such that the expected cell variance on the 64^3 / 128 Mpc grid at z = 9 is 0.36.

    Expected variance of a periodic Gaussian field = (1/V) * sum over all non-DC
    modes of the full grid of P(k).
    """
    n, box = REF_GRID
    k = _mode_k(n, box, half=False)
    s = _shape(k, k0)
    s[0, 0, 0] = 0.0
    return CELL_STD_REF ** 2 * box ** 3 / float(s.sum())


def make_box(n: int, box: float, z: float, seed: int | None = None,
             amp: float | None = None, dtype=np.float32) -> np.ndarray:
    """Gaussian random density box delta(x), shape (n, n, n), C order.

    White noise from numpy's PCG64(seed) is coloured in Fourier space by
    sqrt(P(k) / V_cell) (so the FFT estimator recovers P), the DC mode is set to
    zero, and the result is scaled by D(z).  The box is rounded to `dtype`.
    """
    if seed is None:
        seed = BOX_SEEDS[(n, float(box))]
    if amp is None:
        amp = reference_amplitude()
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    k = _mode_k(n, box, half=True)
    vcell = (box / n) ** 3
    colour = np.sqrt(amp * _shape(k) / vcell)
    colour[0, 0, 0] = 0.0
    field = np.fft.irfftn(wk * colour, s=(n, n, n), axes=(0, 1, 2))
    field *= growth(z)
    return np.ascontiguousarray(field.astype(dtype))


def draw_walkers(count: int, seed: int) -> np.ndarray:
    """(count, 3) float64 array of (zeta, R_mfp / Mpc, T_vir / K) from uniform priors.

    Each row draws zeta, R_mfp and log10 T_vir in that order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(low=PRIOR_LO, high=PRIOR_HI, size=(count, 3))
    out = u.copy()
    out[:, 2] = 10.0 ** u[:, 2]
    return out


def draw_walkers2(count: int, seed: int) -> np.ndarray:
    """(count, 5) float64 array of (zeta0, R_mfp / Mpc, T_feed / K, alpha, beta) from uniform priors.

    Each row draws zeta0, R_mfp, log10 T_feed, alpha and beta in that order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = rng.uniform(low=PRIOR2_LO, high=PRIOR2_HI, size=(count, 5))
    out[:, 2] = 10.0 ** out[:, 2]
    return out


def uniforms(shape, seed: int) -> np.ndarray:
    """float64 uniforms in [0, 1) of the given shape (the sampler's random inputs)."""
    return np.random.Generator(np.random.PCG64(seed)).random(shape)


@dataclasses.dataclass(frozen=True)
class BoxSpec:
    n: int
    box_mpc: float
    z: float
    n_bins: int


@dataclasses.dataclass(frozen=True)
class Workload:
    """One of the five synthetic workloads (geometry, redshifts, walkers, precision)."""
    name: str
    boxes: Tuple[BoxSpec, ...]
    walkers: Tuple[Tuple[float, float, float], ...] | None  # fixed walkers, or None
    walker_seed: int | None
    n_walkers: int
    dtype: str            # arithmetic type of FFTs and the per-cell pass
    storage: str          # storage type of the smoothed boxes
    batched: bool         # shared radius ladder (True) or each walker's own ladder


def _boxes(n, box, zs, nb):
    return tuple(BoxSpec(n, box, z, nb) for z in zs)


WORKLOADS = {
    "plain-f64-64": Workload("plain-f64-64", _boxes(64, 128.0, (9.0,), 12),
                             ((30.0, 15.0, 5e4),), None, 1, "f64", "f64", False),
    "plain-f32-128": Workload("plain-f32-128", _boxes(128, 250.0, (8.0, 9.0, 10.0), 15),
                              ((20.0, 15.0, 3e4),), None, 1, "f32", "f32", False),
    "batched-256": Workload("batched-256", _boxes(256, 250.0, (8.0, 9.0, 10.0), 15),
                            None, WALKER_SEEDS["batched-256"], 64, "f32", "f32", True),
    "uneven-mix": Workload("uneven-mix", _boxes(128, 250.0, (8.0, 9.0, 10.0), 15)
                           + _boxes(256, 300.0, (8.0, 9.0, 10.0), 15),
                           None, WALKER_SEEDS["uneven-mix"], 256, "f32", "bf16", True),
    "large-512": Workload("large-512", _boxes(512, 400.0, (8.0, 9.0, 10.0), 15),
                          None, WALKER_SEEDS["large-512"], 1024, "f32", "f32", True),
}


def workload_walkers(w: Workload) -> np.ndarray:
    if w.walkers is not None:
        return np.array(w.walkers, dtype=np.float64)
    return draw_walkers(w.n_walkers, w.walker_seed)


def workload_boxes(w: Workload, amp: float | None = None) -> List[np.ndarray]:
    """Density boxes of a workload (one realisation per geometry, scaled per z)."""
    dt = np.float64 if w.dtype == "f64" else np.float32
    cache = {}
    out = []
    if amp is None:
        amp = reference_amplitude()
    for b in w.boxes:
        key = (b.n, b.box_mpc)
        if key not in cache:
            cache[key] = make_box(b.n, b.box_mpc, 9.0, BOX_SEEDS[key], amp, np.float64)
        out.append(np.ascontiguousarray((cache[key] * (growth(b.z) / growth(9.0))).astype(dt)))
    return out
