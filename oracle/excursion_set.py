"""FP64 CPU oracle of the excursion-set ionisation -> 21 cm brightness -> P(k) path.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain, obviously correct
reference that the GPU path is checked against.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the product library
never calls it, and it shares no code with the GPU path (the two read the same
seeded inputs from ``synth`` and nothing else).

Every step follows the paper (Greig & Mesinger 2015, "21CMMC") in its own order,
written with NumPy/SciPy primitives in float64:

* Section 2.1 (eq. 1): a cell is tagged fully ionised if zeta * f_coll >= 1 for
  the density smoothed on a sphere of radius R, for R decreasing from the
  largest filtering scale R_mfp (Section 2.1.2) down to the cell scale.
* Section 2.1: cells not fully ionised receive the partial ionised fraction
  zeta * f_coll evaluated for the cell smoothed on the minimum scale R_cell.
* Section 2.1.3 (eq. 3): minimum halo mass from the virial temperature.
* Section 2.2 (eq. 4): 21 cm brightness temperature.
* Section 2.2: spherically averaged power spectrum Delta^2_21(k).

The paper leaves several choices open; the readings taken here (sharp-k filter
with k_c = (9 pi / 2)^(1/3) / R, EPS collapse fraction, radius ladder stepping
by a factor 1.1, logarithmic bins with an exact integer assignment, ...) are the
ones documented in the design notes and are stated again at each function.

Parity pinned by the tests under ``tests/test_oracle_*.py`` (brute-force DFTs,
closed forms, plane waves, uniform boxes, monotonicity, extremes).  The one part
that cannot be pinned to the paper itself is its printed neutral fractions,
which need the paper's own 21CMFAST boxes: that comparison is "parity unpinned".
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Sequence

import numpy as np
import scipy.fft
import scipy.integrate
import scipy.special

def _cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


FFT_WORKERS = _cores()  # threads the oracle's FFTs use (at most 16)


# ---------------------------------------------------------------------------
# Physical constants and parameters
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Physics:
    """Constants of the method.

    delta_c: linear collapse threshold (1.686).
    omega_m, omega_l, h: cosmology of the paper's Section 1 (0.27, 0.73, 0.7).
    tb0_mK: brightness prefactor of eq. (4) in its simplified form (27 mK).
    pk_amp, pk_k0, z_ref: linear spectrum A k (1 + (k/k0)^2)^-2 at z_ref, used
        for sigma^2(R); it is the spectrum the synthetic boxes are drawn from.
    radius_step: ratio between consecutive filter radii (1.1).
    ladder_top: top radius of the shared ladder used by batched walkers (20 Mpc,
        the upper bound of the paper's R_mfp prior).
    mmin_form: 0 = M_min = 1e8 (T/1e4)^1.5 ((1+z)/10)^-1.5 Msun; 1 = eq. (3).
    mu: mean molecular weight in eq. (3) (the paper does not fix it; 0.6).
    velocity: include the line-of-sight velocity-gradient factor H / (dv_r/dr + H)
        of eq. (4) in dT_b (off: the factor is 1).
    dvdr_max: limit on |dv_r/dr| / H in that factor (the paper gives none; 0.2).
    """
    delta_c: float = 1.686
    omega_m: float = 0.27
    omega_l: float = 0.73
    h: float = 0.7
    tb0_mK: float = 27.0
    pk_amp: float = 1.0
    pk_k0: float = 0.05
    z_ref: float = 9.0
    radius_step: float = 1.1
    ladder_top: float = 20.0
    mmin_form: int = 0
    mu: float = 0.6
    velocity: bool = False
    dvdr_max: float = 0.2


RHO_CRIT_H2 = 2.775e11  # critical density today in Msun Mpc^-3 h^-2


# ---------------------------------------------------------------------------
# Halo mass threshold and mass variance (host-side scalars)
# ---------------------------------------------------------------------------

def min_halo_mass(t_vir: float, z: float, phys: Physics) -> float:
    """M_min(T_vir, z) in Msun (Section 2.1.3).

    mmin_form 0 is the simplified scaling 1e8 Msun (T_vir / 1e4 K)^1.5
    ((1+z)/10)^-1.5; mmin_form 1 is the full eq. (3) with Omega_m^z and
    Delta_c = 18 pi^2 + 82 d - 39 d^2, d = Omega_m^z - 1.
    """
    if phys.mmin_form == 0:
        return 1e8 * (t_vir / 1e4) ** 1.5 * ((1.0 + z) / 10.0) ** -1.5
    a3 = phys.omega_m * (1.0 + z) ** 3
    om_z = a3 / (a3 + phys.omega_l)
    d = om_z - 1.0
    delta_vir = 18.0 * math.pi ** 2 + 82.0 * d - 39.0 * d ** 2
    return (1e8 / phys.h * (phys.mu / 0.6) ** -1.5
            * (phys.omega_m / om_z * delta_vir / (18.0 * math.pi ** 2)) ** -0.5
            * (t_vir / 1.98e4) ** 1.5 * ((1.0 + z) / 10.0) ** -1.5)


def mean_matter_density(phys: Physics) -> float:
    """Comoving mean matter density in Msun / Mpc^3."""
    return phys.omega_m * RHO_CRIT_H2 * phys.h ** 2


def radius_of_mass(mass: float, phys: Physics) -> float:
    """Lagrangian radius R with (4 pi / 3) R^3 rho_m = M."""
    return (3.0 * mass / (4.0 * math.pi * mean_matter_density(phys))) ** (1.0 / 3.0)


def sharpk_cutoff(radius: float) -> float:
    """Sharp-k cutoff k_c of a sphere of radius R (volume matching).

    The k-space ball |k| <= k_c holds k_c^3 / (6 pi^2) modes per unit volume,
    which equals 1 / (4 pi R^3 / 3) for k_c = (9 pi / 2)^(1/3) / R.
    """
    return (4.5 * math.pi) ** (1.0 / 3.0) / radius


def linear_growth(z: float, phys: Physics) -> float:
    """D(z) = (1 + z_ref) / (1 + z), the growth the synthetic boxes are scaled by."""
    return (1.0 + phys.z_ref) / (1.0 + z)


def linear_power(k, phys: Physics):
    """Linear power spectrum at z_ref, A k (1 + (k / k0)^2)^-2 (Mpc^3)."""
    return phys.pk_amp * k * (1.0 + (k / phys.pk_k0) ** 2) ** -2


def mass_variance(radius: float, z: float, phys: Physics) -> float:
    """sigma^2(R, z) for the sharp-k window, by direct quadrature.

    sigma^2 = D(z)^2 / (2 pi^2) * int_0^{k_c(R)} k^2 P(k) dk.  The paper cites
    the extended Press-Schechter collapse fraction (Section 2.1) without fixing a
    window; the sharp-k window is the one of the excursion-set filter itself.
    """
    kc = sharpk_cutoff(radius)
    val, _ = scipy.integrate.quad(lambda k: k * k * linear_power(k, phys), 0.0, kc,
                                  epsabs=0.0, epsrel=1e-13, limit=200)
    return linear_growth(z, phys) ** 2 * val / (2.0 * math.pi ** 2)


# ---------------------------------------------------------------------------
# Radius schedule
# ---------------------------------------------------------------------------

def radius_ladder(r_top: float, r_cell: float, step: float) -> List[float]:
    """Filter radii from r_top downwards by `step`, ending at the cell scale.

    R_i = r_top / step^i while R_i > r_cell, then r_cell itself (Section 2.1:
    decreasing radii from the maximum filtering scale; the last one is R_cell).
    If r_top <= r_cell the list is [r_cell].
    """
    out = []
    i = 0
    while True:
        r = r_top / step ** i
        if r > r_cell:
            out.append(r)
            i += 1
        else:
            break
    out.append(r_cell)
    return out


def walker_radii(shared: Sequence[float], r_mfp: float) -> List[float]:
    """Suffix of a shared ladder a walker with mean free path r_mfp uses.

    Radii above R_mfp are not filtered (Section 2.1.2: R_mfp is the largest
    filtering scale); the cell radius (the last entry) is always kept.
    """
    out = [r for r in shared[:-1] if r <= r_mfp]
    out.append(shared[-1])
    return out


# ---------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------

def mode_indices(n: int):
    """Integer mode indices (n0, n1, n2) of an rfftn half spectrum.

    n0, n1 in [-n/2, n/2) (numpy fftfreq * n), n2 in [0, n/2].
    """
    f = np.rint(np.fft.fftfreq(n, d=1.0 / n)).astype(np.int64)
    fl = np.arange(n // 2 + 1, dtype=np.int64)
    return f[:, None, None], f[None, :, None], fl[None, None, :]


def mode_n2(n: int) -> np.ndarray:
    a, b, c = mode_indices(n)
    return a * a + b * b + c * c


def tophat_k_mask(n: int, box: float, radius: float) -> np.ndarray:
    """Sharp-k mask |k| <= k_c(R) on the half spectrum (inclusive)."""
    kf = 2.0 * math.pi / box
    kmod = kf * np.sqrt(mode_n2(n).astype(np.float64))
    return kmod <= sharpk_cutoff(radius)


def smooth(delta_hat: np.ndarray, n: int, box: float, radius: float) -> np.ndarray:
    """delta_R: the box smoothed with the sharp-k top hat of radius R."""
    return scipy.fft.irfftn(delta_hat * tophat_k_mask(n, box, radius), s=(n, n, n),
                            workers=FFT_WORKERS)


def _elementwise(fn, x: np.ndarray) -> np.ndarray:
    """fn applied to every element of x, in contiguous chunks on FFT_WORKERS
    threads (NumPy/SciPy ufuncs release the GIL).  Each element is computed on
    its own, so the result does not depend on the split."""
    flat = np.ascontiguousarray(x).reshape(-1)
    out = np.empty_like(flat)
    if FFT_WORKERS <= 1 or flat.size < (1 << 20):
        out[:] = fn(flat)
        return out.reshape(x.shape)
    from concurrent.futures import ThreadPoolExecutor
    edges = np.linspace(0, flat.size, FFT_WORKERS + 1).astype(np.int64)

    def run(i):
        out[edges[i]:edges[i + 1]] = fn(flat[edges[i]:edges[i + 1]])

    with ThreadPoolExecutor(max_workers=FFT_WORKERS) as ex:
        list(ex.map(run, range(FFT_WORKERS)))
    return out.reshape(x.shape)


def collapse_fraction(delta_r: np.ndarray, dsig2: float, delta_c: float) -> np.ndarray:
    """Conditional collapse fraction erfc((delta_c - delta_R) / sqrt(2 (S_min - S_R))).

    Extended Press-Schechter form (Section 2.1 cites Bond et al. 1991, Lacey &
    Cole 1993).  When S_min <= S_R the sphere holds less than M_min of mass and
    no halo above M_min can form inside it: f_coll = 0.
    """
    if dsig2 <= 0.0:
        return np.zeros_like(delta_r)
    scale = math.sqrt(2.0 * dsig2)
    return _elementwise(lambda v: scipy.special.erfc((delta_c - v) / scale), delta_r)


def ionization_field(delta: np.ndarray, box: float, z: float, zeta: float, t_vir: float,
                     radii: Sequence[float], phys: Physics):
    """Excursion-set ionisation of one box for one walker (Section 2.1, eq. 1).

    For each radius from largest to smallest: smooth, evaluate f_coll, and tag
    the cell fully ionised where zeta * f_coll >= 1.  Cells never tagged get the
    partial ionised fraction zeta * f_coll at the last (cell) radius.
    Returns (flagged bool array, x_HI float64 array).
    """
    n = delta.shape[0]
    d64 = np.asarray(delta, dtype=np.float64)
    dhat = scipy.fft.rfftn(d64, workers=FFT_WORKERS)
    s_min = mass_variance(radius_of_mass(min_halo_mass(t_vir, z, phys), phys), z, phys)
    flagged = np.zeros(d64.shape, dtype=bool)
    f_cell = None
    for r in radii:
        d_r = smooth(dhat, n, box, r)
        f = collapse_fraction(d_r, s_min - mass_variance(r, z, phys), phys.delta_c)
        flagged |= zeta * f >= 1.0
        f_cell = f
    x_hi = np.where(flagged, 0.0, 1.0 - zeta * f_cell)
    return flagged, x_hi


def velocity_gradient(delta: np.ndarray, axis: int = 0) -> np.ndarray:
    """Line-of-sight gradient of the linear peculiar velocity, in units of -H.

    Linear continuity (Section 2.2 evaluates eq. 4 with the velocity field of
    the same density box): in Fourier space the gradient of the velocity
    component along the line of sight is -f H (k_r^2 / k^2) delta_hat, with the
    growth rate f = d ln D / d ln a = 1 for D proportional to 1 / (1 + z).
    Returns g(x) with dv_r/dr / H = -g; the k = 0 mode gives 0.  The line of
    sight is array axis `axis` (the first axis throughout this work).
    """
    d64 = np.asarray(delta, dtype=np.float64)
    n = d64.shape[0]
    dhat = scipy.fft.rfftn(d64, workers=FFT_WORKERS)
    idx = mode_indices(n)
    kk = idx[0] * idx[0] + idx[1] * idx[1] + idx[2] * idx[2]
    kr2 = idx[axis] * idx[axis]
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(kk > 0, kr2 / np.where(kk > 0, kk, 1), 0.0)
    return scipy.fft.irfftn(dhat * w, s=d64.shape, workers=FFT_WORKERS)


def velocity_factor(delta: np.ndarray, phys: Physics) -> np.ndarray:
    """H / (dv_r/dr + H) of eq. (4): 1 / (1 + t) with t = dv_r/dr / H = -g,
    t limited to [-dvdr_max, dvdr_max] (the paper states no limit; without one
    the factor diverges where the linear gradient reaches -H)."""
    t = np.clip(-velocity_gradient(delta), -phys.dvdr_max, phys.dvdr_max)
    return 1.0 / (1.0 + t)


def brightness_temperature(x_hi: np.ndarray, delta: np.ndarray, z: float,
                           phys: Physics) -> np.ndarray:
    """dT_b = tb0 x_HI (1 + delta) sqrt((1 + z) / 10) mK (eq. 4 with T_S >> T_gamma,
    without the cosmology factors), times H / (dv_r/dr + H) when phys.velocity."""
    dtb = phys.tb0_mK * x_hi * (1.0 + np.asarray(delta, dtype=np.float64)) * math.sqrt((1.0 + z) / 10.0)
    if phys.velocity:
        dtb = dtb * velocity_factor(delta, phys)
    return dtb


# ---------------------------------------------------------------------------
# Power spectrum
# ---------------------------------------------------------------------------

def bin_of_n2(n2: int, n: int, n_bins: int) -> int:
    """Log bin of a mode with integer |n|^2 = n2, or -1 if the mode is dropped.

    Edges e_b = k_f (n/2)^(b / n_bins), b = 0..n_bins, log spaced on [k_f, k_Ny].
    A mode is in bin b when e_b <= |k| < e_{b+1}; the top edge is closed.  The
    DC mode and corner modes with |n| > n/2 are dropped.  The comparison
    |k| >= e_b is decided exactly in integers: n2^n_bins >= (n/2)^(2 b).
    """
    half = n // 2
    if n2 <= 0 or n2 > half * half:
        return -1
    lhs = n2 ** n_bins
    b = 0
    for cand in range(1, n_bins + 1):
        if lhs >= half ** (2 * cand):
            b = cand
    return min(b, n_bins - 1)


def bin_table(n: int, n_bins: int) -> np.ndarray:
    """bin_of_n2 for every n2 in [0, 3 (n/2)^2]."""
    top = 3 * (n // 2) ** 2
    return np.array([bin_of_n2(v, n, n_bins) for v in range(top + 1)], dtype=np.int64)


def power_spectrum(field: np.ndarray, box: float, n_bins: int):
    """Spherically averaged power spectrum of a real field (Section 2.2).

    Per mode P(k) = |X(k)|^2 L^3 / N^6 with X the unnormalised forward DFT.  The
    half spectrum counts modes on the last-axis planes 0 and N/2 once and all
    others twice (they stand for their mirror too).  Returns
    (P_b, k_b, counts, Delta^2_b) with k_b the count-weighted mean |k| and
    Delta^2 = k^3 P / (2 pi^2).  Empty bins give P_b = k_b = 0.
    """
    n = field.shape[0]
    x = scipy.fft.rfftn(np.asarray(field, dtype=np.float64), workers=FFT_WORKERS)
    p = (x.real ** 2 + x.imag ** 2) * box ** 3 / float(n) ** 6
    n2 = mode_n2(n)
    w = np.full(x.shape, 2.0)
    w[:, :, 0] = 1.0
    w[:, :, n // 2] = 1.0
    bins = bin_table(n, n_bins)[n2]
    keep = bins >= 0
    kf = 2.0 * math.pi / box
    kmod = kf * np.sqrt(n2.astype(np.float64))
    b = bins[keep]
    counts = np.bincount(b, weights=w[keep], minlength=n_bins)
    psum = np.bincount(b, weights=(w * p)[keep], minlength=n_bins)
    ksum = np.bincount(b, weights=(w * kmod)[keep], minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        pb = np.where(counts > 0, psum / np.where(counts > 0, counts, 1.0), 0.0)
        kb = np.where(counts > 0, ksum / np.where(counts > 0, counts, 1.0), 0.0)
    delta2 = kb ** 3 * pb / (2.0 * math.pi ** 2)
    return pb, kb, counts, delta2


# ---------------------------------------------------------------------------
# One walker evaluation
# ---------------------------------------------------------------------------

@dataclass
class Evaluation:
    flagged: np.ndarray
    x_hi: np.ndarray
    dtb: np.ndarray
    pk: np.ndarray
    k_mean: np.ndarray
    counts: np.ndarray
    delta2: np.ndarray
    xhi_mean: float
    radii: List[float] = field(default_factory=list)


def evaluate(delta: np.ndarray, box: float, z: float, walker: Sequence[float],
             radii: Sequence[float], n_bins: int, phys: Physics) -> Evaluation:
    """Ionisation field, brightness temperature and binned P(k) for one walker."""
    zeta, _r_mfp, t_vir = (float(v) for v in walker)
    flagged, x_hi = ionization_field(delta, box, z, zeta, t_vir, radii, phys)
    dtb = brightness_temperature(x_hi, delta, z, phys)
    pb, kb, cnt, d2 = power_spectrum(dtb, box, n_bins)
    return Evaluation(flagged, x_hi, dtb, pb, kb, cnt, d2, float(np.mean(x_hi)), list(radii))


def plain_radii(r_mfp: float, n: int, box: float, phys: Physics) -> List[float]:
    """Radius list of the plain method: from R_mfp down to the cell size L/N."""
    return radius_ladder(r_mfp, box / n, phys.radius_step)


def shared_radii(n: int, box: float, phys: Physics) -> List[float]:
    """Radius ladder shared by batched walkers: from ladder_top down to L/N."""
    return radius_ladder(phys.ladder_top, box / n, phys.radius_step)
