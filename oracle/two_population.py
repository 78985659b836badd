"""FP64 CPU oracle of the two-population ionising efficiency (Section 4, eq. 9).

TEST INFRASTRUCTURE ONLY, under the same rules as ``excursion_set``: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
it shares no code with the GPU path.

What it computes.  Section 4 replaces the constant efficiency zeta of eq. (1)
by a function of the host halo's virial temperature (eq. 9): zeta0 (T/T_feed)^beta
above the feedback temperature T_feed, zeta0 (T/T_feed)^alpha between the
atomic-cooling limit 1e4 K and T_feed, and 0 below 1e4 K.  The ionisation
criterion of eq. (1) then weighs every collapsed halo by its own efficiency:

    F(delta_R, R) = int_{M_cool}^{M_R} zeta(M) dF_coll(>M | delta_R, R) / (-dM) dM

with the extended Press-Schechter conditional collapsed fraction
F_coll(>M | delta_R, R) = erfc(nu / sqrt(2 (S(M) - S_R))), nu = delta_c - delta_R,
S = sigma^2 of the sharp-k window, M_R the mass of the sphere of radius R and
M_cool the mass at 1e4 K.  A cell is fully ionised when F >= 1 at some radius;
otherwise its ionised fraction is F at the cell radius.  With zeta constant the
integral is zeta * erfc(nu / sqrt(2 (S(M_cool) - S_R))), the constant-efficiency
model of eq. (1).

Readings taken here (also listed in the design notes):
* T_vir and halo mass are tied by the same M_min(T_vir, z) relation as the
  constant model (M proportional to T^1.5 at fixed z), so T / T_feed =
  (M / M_feed)^(2/3);
* a sphere whose smoothed density reaches delta_c (nu <= 0) has all its mass in
  one halo of mass M_R: F = zeta(M_R);
* a sphere lighter than M_cool holds no ionising halo: F = 0;
* the integral is taken over the variance S of the halo mass, written in
  lambda = ln(S - S_R): dF_coll = p(S) dS with the first-crossing density
  p(S) = nu / sqrt(2 pi) (S - S_R)^-3/2 exp(-nu^2 / (2 (S - S_R))) (Lacey & Cole
  1993), from S_R up to S(M_cool), on composite Gauss-Legendre panels split at the
  feedback mass (where zeta has a kink).  Masses of variance S come from the
  sharp-k variance inverted in closed form (Lambert W function).  The panels
  start at S - S_R = S_R e^-30; below that zeta is zeta(M_R) to round-off and
  the head is added as zeta(M_R) erfc(nu / sqrt(2 (S - S_R))).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
import scipy.special

from . import excursion_set as es

T_COOL = 1e4          # K, atomic-cooling limit below which eq. (9) gives zero efficiency
_PANEL = 0.5          # width of a Gauss-Legendre panel in ln(S - S_R)
_NODES = 10           # nodes per panel
_HEAD = 30.0          # panels start at S - S_R = S_R exp(-_HEAD)
_CHUNK = 4096         # cells per vectorised block


def virial_temperature(mass, z: float, phys: es.Physics):
    """T_vir of a halo of mass M at redshift z, inverting M_min(T_vir, z) (M ~ T^1.5)."""
    return T_COOL * (np.asarray(mass, dtype=np.float64) / es.min_halo_mass(T_COOL, z, phys)) ** (2.0 / 3.0)


def efficiency(mass, z: float, walker: Sequence[float], phys: es.Physics):
    """zeta(M) of eq. (9) for walker (zeta0, R_mfp, T_feed, alpha, beta)."""
    zeta0, _r, t_feed, alpha, beta = (float(v) for v in walker)
    t = virial_temperature(mass, z, phys)
    ratio = t / t_feed
    with np.errstate(divide="ignore", over="ignore"):
        out = np.where(t >= t_feed, zeta0 * ratio ** beta, zeta0 * ratio ** alpha)
    return np.where(t >= T_COOL, out, 0.0)


def variance_scale(z: float, phys: es.Physics) -> float:
    """c with sigma^2 = c [ln(1 + y) + 1 / (1 + y) - 1], y = (k_c / k0)^2 (sharp-k window,
    spectrum A k (1 + (k/k0)^2)^-2): the integral of k^2 P(k) in closed form."""
    return es.linear_growth(z, phys) ** 2 * phys.pk_amp * phys.pk_k0 ** 4 / (4.0 * math.pi ** 2)


def radius_of_variance(s2, z: float, phys: es.Physics):
    """Radius R with sigma^2(R, z) = s2 (sharp-k window), in closed form.

    With t = 1 + y the variance reads c (ln t + 1/t - 1); putting w = 1/t gives
    w - ln w = s2 / c + 1, i.e. -w exp(-w) = -exp(-(s2/c + 1)), so
    w = -W0(-exp(-(s2/c + 1))) on the principal branch (w in (0, 1]).
    """
    s = np.asarray(s2, dtype=np.float64) / variance_scale(z, phys)
    w = -scipy.special.lambertw(-np.exp(-(s + 1.0)), 0).real
    y = 1.0 / w - 1.0
    kc = phys.pk_k0 * np.sqrt(y)
    return (4.5 * math.pi) ** (1.0 / 3.0) / kc


def sphere_mass(radius, phys: es.Physics):
    """Mass (4 pi / 3) R^3 rho_m of a sphere of radius R."""
    return 4.0 * math.pi / 3.0 * np.asarray(radius, dtype=np.float64) ** 3 * es.mean_matter_density(phys)


def _panels(a: float, b: float):
    """Gauss-Legendre nodes and weights of [a, b] cut into panels of width <= _PANEL."""
    if not b > a:
        return np.zeros(0), np.zeros(0)
    x, w = np.polynomial.legendre.leggauss(_NODES)
    count = max(1, int(math.ceil((b - a) / _PANEL)))
    h = (b - a) / count
    lo = a + h * np.arange(count)
    nodes = (lo[:, None] + 0.5 * h * (x[None, :] + 1.0)).reshape(-1)
    weights = np.tile(0.5 * h * w, count)
    return nodes, weights


def ionizing_fraction(delta_r, radius: float, z: float, walker: Sequence[float], phys: es.Physics):
    """F(delta_R, R): the efficiency-weighted collapsed fraction of Section 4 (per cell)."""
    d = np.asarray(delta_r, dtype=np.float64)
    s_r = es.mass_variance(radius, z, phys)
    m_cool = es.min_halo_mass(T_COOL, z, phys)
    s_cool = es.mass_variance(es.radius_of_mass(m_cool, phys), z, phys)
    if s_cool <= s_r:
        return np.zeros_like(d)
    m_r = float(sphere_mass(radius, phys))
    zeta_top = float(efficiency(m_r, z, walker, phys))
    lam_a = math.log(s_r) - _HEAD
    lam_b = math.log(s_cool - s_r)
    cuts = [lam_a, lam_b]
    m_feed = es.min_halo_mass(float(walker[2]), z, phys)
    if m_cool < m_feed < m_r:
        lam_f = math.log(es.mass_variance(es.radius_of_mass(m_feed, phys), z, phys) - s_r)
        if lam_a < lam_f < lam_b:
            cuts = [lam_a, lam_f, lam_b]
    parts = [_panels(cuts[i], cuts[i + 1]) for i in range(len(cuts) - 1)]
    lam = np.concatenate([p[0] for p in parts])
    wts = np.concatenate([p[1] for p in parts])
    ds = np.exp(lam)                                            # S - S_R at the nodes
    zeta = efficiency(sphere_mass(radius_of_variance(s_r + ds, z, phys), phys), z, walker, phys)
    # p(S) dS = nu / sqrt(2 pi) ds^-1/2 exp(-nu^2 / (2 ds)) dlambda
    coef = wts * zeta * ds ** -0.5 / math.sqrt(2.0 * math.pi)
    inv2 = 0.5 / ds
    head = 1.0 / math.sqrt(2.0 * math.exp(lam_a))
    out = np.empty(d.size)
    flat = d.reshape(-1)
    for c0 in range(0, flat.size, _CHUNK):
        nu = phys.delta_c - flat[c0:c0 + _CHUNK]
        res = np.full(nu.shape, zeta_top)           # nu <= 0: the sphere is one halo
        pos = nu > 0.0
        if np.any(pos):
            v = nu[pos]
            body = np.exp(-(v * v)[:, None] * inv2[None, :]) @ coef
            res[pos] = v * body + zeta_top * scipy.special.erfc(v * head)
        out[c0:c0 + _CHUNK] = res
    return out.reshape(d.shape)


def ionization_field(delta: np.ndarray, box: float, z: float, walker: Sequence[float],
                     radii: Sequence[float], phys: es.Physics):
    """Excursion-set ionisation of one box with the efficiency of eq. (9).

    Same steps as the constant-efficiency model: radii from largest to smallest,
    a cell is tagged fully ionised where F >= 1, untagged cells get the ionised
    fraction F at the last (cell) radius.  Returns (flagged, x_HI).
    """
    n = delta.shape[0]
    d64 = np.asarray(delta, dtype=np.float64)
    dhat = es.scipy.fft.rfftn(d64, workers=es.FFT_WORKERS)
    flagged = np.zeros(d64.shape, dtype=bool)
    f_cell = None
    for r in radii:
        f = ionizing_fraction(es.smooth(dhat, n, box, r), r, z, walker, phys)
        flagged |= f >= 1.0
        f_cell = f
    x_hi = np.where(flagged, 0.0, 1.0 - f_cell)
    return flagged, x_hi


def evaluate(delta: np.ndarray, box: float, z: float, walker: Sequence[float],
             radii: Sequence[float], n_bins: int, phys: es.Physics) -> es.Evaluation:
    """Ionisation, brightness temperature and binned P(k) for one five-parameter walker
    (zeta0, R_mfp, T_feed, alpha, beta)."""
    flagged, x_hi = ionization_field(delta, box, z, walker, radii, phys)
    dtb = es.brightness_temperature(x_hi, delta, z, phys)
    pb, kb, cnt, d2 = es.power_spectrum(dtb, box, n_bins)
    return es.Evaluation(flagged, x_hi, dtb, pb, kb, cnt, d2, float(np.mean(x_hi)), list(radii))
