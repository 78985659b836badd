"""Pins of the FP64 two-population oracle (Section 4, eq. 9).

The efficiency-weighted collapsed fraction F is fixed here through routes that
do not use the oracle's own quadrature: the closed-form erfc of the constant
efficiency model (eq. 1), an adaptive integration over the halo-mass variance S
with the masses found by root finding on the quadrature variance of the first
oracle, the limit of a sphere at the collapse threshold, linearity in zeta0,
and hand values of eq. (9).  No GPU.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize
import scipy.special

import oracle
import synth

es = oracle.excursion_set
tp = oracle.two_population
PHYS = oracle.Physics(pk_amp=synth.reference_amplitude())
FID = (70.0, 15.0, 10 ** 4.7, 4.0 / 3.0, -1.0 / 3.0)    # the fiducial of Section 4


def _variances(radius, z, walker=None):
    s_r = es.mass_variance(radius, z, PHYS)
    s_cool = es.mass_variance(es.radius_of_mass(es.min_halo_mass(1e4, z, PHYS), PHYS), z, PHYS)
    s_feed = None
    if walker is not None:
        s_feed = es.mass_variance(es.radius_of_mass(es.min_halo_mass(walker[2], z, PHYS), PHYS), z, PHYS)
    return s_r, s_cool, s_feed


def test_efficiency_hand_values():
    z = 9.0
    zeta0, t_feed, alpha, beta = 40.0, 2e5, 2.0, -0.5
    w = (zeta0, 10.0, t_feed, alpha, beta)
    m_at = lambda t: es.min_halo_mass(t, z, PHYS)      # mass of virial temperature t
    assert float(tp.efficiency(m_at(t_feed), z, w, PHYS)) == pytest.approx(zeta0, rel=1e-13)
    assert float(tp.efficiency(m_at(1e4), z, w, PHYS)) == pytest.approx(zeta0 * (1e4 / t_feed) ** alpha, rel=1e-12)
    assert float(tp.efficiency(m_at(4e4), z, w, PHYS)) == pytest.approx(zeta0 * 0.2 ** alpha, rel=1e-12)
    assert float(tp.efficiency(m_at(2e6), z, w, PHYS)) == pytest.approx(zeta0 * 10.0 ** beta, rel=1e-12)
    assert float(tp.efficiency(m_at(0.9e4), z, w, PHYS)) == 0.0


@pytest.mark.parametrize("z", [8.0, 10.0])
def test_radius_of_variance_inverts_the_quadrature_variance(z):
    for r in (0.5, 1.0, 3.7, 12.0, 20.0):
        s = es.mass_variance(r, z, PHYS)              # scipy quad of k^2 P(k)
        assert float(tp.radius_of_variance(s, z, PHYS)) == pytest.approx(r, rel=1e-11)


@pytest.mark.parametrize("z,radius", [(8.0, 1.0), (9.0, 4.0), (10.0, 20.0)])
def test_constant_efficiency_is_the_erfc_of_eq1(z, radius):
    # alpha = beta = 0: zeta = zeta0 for every halo above 1e4 K, so F must equal
    # zeta0 erfc(nu / sqrt(2 (S_cool - S_R))) -- the constant-efficiency form
    w = (25.0, 15.0, 3e5, 0.0, 0.0)
    s_r, s_cool, _ = _variances(radius, z)
    d = np.array([-2.0, -1.0, -0.3, 0.0, 0.5, 1.0, 1.5, 1.68, 1.6859, 1.686, 2.0])
    got = tp.ionizing_fraction(d, radius, z, w, PHYS)
    nu = PHYS.delta_c - d
    want = np.where(nu > 0, 25.0 * scipy.special.erfc(nu / math.sqrt(2 * (s_cool - s_r))), 25.0)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=0.0)


def _mass_of_variance(s2, z):
    """Mass of variance s2 by root finding on the quadrature variance (no closed form)."""
    f = lambda lr: es.mass_variance(math.exp(lr), z, PHYS) - s2
    lr = scipy.optimize.brentq(f, math.log(1e-3), math.log(1e3), xtol=1e-14, rtol=1e-14)
    return float(tp.sphere_mass(math.exp(lr), PHYS))


def _adaptive_f(delta, radius, z, w):
    """F by adaptive quadrature over S of zeta(M(S)) times the first-crossing density."""
    s_r, s_cool, s_feed = _variances(radius, z, w)
    nu = PHYS.delta_c - delta

    def dens(s):
        x = s - s_r
        m = _mass_of_variance(s, z)
        return float(tp.efficiency(m, z, w, PHYS)) * nu / math.sqrt(2 * math.pi) * x ** -1.5 * math.exp(-nu * nu / (2 * x))

    pts = [s_r]
    if s_r < s_feed < s_cool:
        pts.append(s_feed)
    pts.append(s_cool)
    return sum(scipy.integrate.quad(dens, pts[i], pts[i + 1], epsabs=0.0, epsrel=1e-10, limit=300)[0]
               for i in range(len(pts) - 1))


@pytest.mark.parametrize("w", [FID, (30.0, 15.0, 1e5, 10.0 / 3.0, -4.0 / 3.0), (12.0, 15.0, 3e4, -4.0 / 3.0, 2.0)])
@pytest.mark.parametrize("z,radius,delta", [(8.0, 20.0, 0.8), (9.0, 5.0, -0.7), (10.0, 1.2, 1.5), (8.0, 2.0, 1.65)])
def test_matches_adaptive_integration_over_mass_variance(w, z, radius, delta):
    got = float(tp.ionizing_fraction(np.array([delta]), radius, z, w, PHYS)[0])
    want = _adaptive_f(delta, radius, z, w)
    assert got == pytest.approx(want, rel=2e-9)


def test_threshold_limit_is_the_efficiency_of_the_sphere():
    # as delta_R -> delta_c all the sphere's mass ends up in one halo of mass M_R
    z, radius = 9.0, 6.0
    for w in (FID, (30.0, 15.0, 1e5, 10.0 / 3.0, -4.0 / 3.0)):
        top = float(tp.efficiency(tp.sphere_mass(radius, PHYS), z, w, PHYS))
        near = float(tp.ionizing_fraction(np.array([PHYS.delta_c - 1e-9]), radius, z, w, PHYS)[0])
        at = float(tp.ionizing_fraction(np.array([PHYS.delta_c]), radius, z, w, PHYS)[0])
        assert at == top
        assert near == pytest.approx(top, rel=1e-4)


def test_linear_in_zeta0_and_zero_below_cooling_mass():
    z, radius = 8.0, 3.0
    d = np.linspace(-1.5, 1.6, 9)
    a = tp.ionizing_fraction(d, radius, z, FID, PHYS)
    b = tp.ionizing_fraction(d, radius, z, (2 * FID[0],) + FID[1:], PHYS)
    np.testing.assert_allclose(b, 2 * a, rtol=1e-14)
    # a sphere lighter than the 1e4 K halo holds no ionising source
    r_small = 0.5 * es.radius_of_mass(es.min_halo_mass(1e4, z, PHYS), PHYS)
    assert np.all(tp.ionizing_fraction(d, r_small, z, FID, PHYS) == 0.0)


def test_step_limit_reduces_to_the_three_parameter_model():
    # beta = 0 and a very steep alpha switch haloes below T_feed off: the
    # criterion becomes zeta0 erfc(nu / sqrt(2 (S_feed - S_R)))
    z, radius, t_feed = 9.0, 4.0, 5e4
    w = (30.0, 15.0, t_feed, 1e6, 0.0)
    s_r, _, s_feed = _variances(radius, z, w)
    d = np.array([-1.0, 0.0, 0.9, 1.6])
    got = tp.ionizing_fraction(d, radius, z, w, PHYS)
    want = 30.0 * scipy.special.erfc((PHYS.delta_c - d) / math.sqrt(2 * (s_feed - s_r)))
    np.testing.assert_allclose(got, want, rtol=1e-9)


def test_whole_box_with_constant_efficiency_matches_eq1_oracle():
    n, box, z = 16, 32.0, 9.0
    d = synth.make_box(n, box, z, seed=7, amp=PHYS.pk_amp, dtype=np.float64)
    radii = oracle.plain_radii(10.0, n, box, PHYS)
    ev3 = oracle.evaluate(d, box, z, (20.0, 10.0, 1e4), radii, 6, PHYS)
    ev5 = tp.evaluate(d, box, z, (20.0, 10.0, 7e4, 0.0, 0.0), radii, 6, PHYS)
    assert np.array_equal(ev3.flagged, ev5.flagged)
    np.testing.assert_allclose(ev5.x_hi, ev3.x_hi, rtol=0, atol=1e-11)
    np.testing.assert_allclose(ev5.pk, ev3.pk, rtol=1e-10)


def test_unimodal_in_delta_over_the_prior():
    # the reading used by the device path: F rises with delta_R to one maximum
    # and then falls towards zeta(M_R); so {F >= 1} is one interval of delta_R
    rng = np.random.default_rng(11)
    d = np.linspace(-2.0, PHYS.delta_c - 1e-9, 80)
    for _ in range(24):
        z = float(rng.choice([8.0, 9.0, 10.0]))
        radius = float(rng.choice([0.8, 2.0, 6.0, 20.0]))
        w = (float(rng.uniform(5, 200)), 15.0, float(10 ** rng.uniform(4, 6)),
             float(rng.uniform(-4 / 3, 10 / 3)), float(rng.uniform(-4 / 3, 10 / 3)))
        f = tp.ionizing_fraction(d, radius, z, w, PHYS)
        steps = np.sign(np.diff(f))
        steps = steps[steps != 0]
        turns = int(np.sum(steps[1:] != steps[:-1]))
        assert turns == 0 or (turns == 1 and steps[0] > 0), (z, radius, w)
