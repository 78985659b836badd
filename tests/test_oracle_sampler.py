"""Pins of the stretch-move ensemble sampler oracle (Section 2.3; Goodman & Weare 2010).

Checked through properties that do not retype the oracle's update: the
inverse-CDF draw of z against the density 1/sqrt(z) and its symmetry
g(1/z) = z g(z) (the reason for the z^(d-1) factor), exact affine invariance
of whole chains, stationarity on a correlated Gaussian target, moves that
keep a walker where it is (z = 1), prior walls, and the independence of the
walkers of one half.  No GPU.
"""
import math

import numpy as np
import pytest
import scipy.integrate

import oracle

S = oracle.sampler


def _uniforms(rng, steps, w):
    return rng.random((steps, 2, w // 2, 3))


def test_stretch_draw_inverts_the_cdf_of_one_over_sqrt_z():
    a = 2.0
    norm = scipy.integrate.quad(lambda z: z ** -0.5, 1 / a, a)[0]
    for u in (0.0, 0.1, 0.37, 0.5, 0.9, 0.999999):
        z = S.stretch_factor(u, a)
        cdf = scipy.integrate.quad(lambda t: t ** -0.5, 1 / a, z)[0] / norm
        assert cdf == pytest.approx(u, abs=1e-12)
    assert S.stretch_factor(0.0, a) == pytest.approx(1 / a)
    assert S.stretch_factor(1.0, a) == pytest.approx(a)
    # g(1/z) = z g(z) on the support: the density in 1/z is z^(d-1)-compatible
    g = lambda z: z ** -0.5 / norm
    for z in (0.6, 1.0, 1.3, 1.9):
        assert g(1 / z) == pytest.approx(z * g(z), rel=1e-14)


def _gauss(mean, cov):
    icov = np.linalg.inv(cov)
    return lambda x: -0.5 * float((x - mean) @ icov @ (x - mean))


def test_affine_invariance_of_whole_chains():
    rng = np.random.default_rng(3)
    d, w, steps = 3, 12, 40
    mean = np.array([1.0, -2.0, 0.5])
    cov = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, -0.2], [0.1, -0.2, 0.5]])
    A = np.array([[3.0, 1.0, 0.0], [0.5, -2.0, 1.0], [0.0, 0.3, 4.0]])
    b = np.array([10.0, -1.0, 2.5])
    lp1 = _gauss(mean, cov)
    lp2 = _gauss(A @ mean + b, A @ cov @ A.T)
    x1 = rng.normal(size=(w, d))
    x2 = x1 @ A.T + b
    l1 = np.array([lp1(v) for v in x1])
    l2 = np.array([lp2(v) for v in x2])
    u = _uniforms(rng, steps, w)
    for s in range(steps):
        a1 = S.step(x1, l1, u[s], lp1)
        a2 = S.step(x2, l2, u[s], lp2)
        assert np.array_equal(a1, a2)
    np.testing.assert_allclose(x2, x1 @ A.T + b, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(l2, l1, rtol=1e-9, atol=1e-9)


def test_stationary_on_a_correlated_gaussian():
    rng = np.random.default_rng(5)
    d, w, steps, burn = 2, 32, 2500, 200
    mean = np.array([3.0, -1.0])
    cov = np.array([[1.0, 0.8], [0.8, 2.0]])
    lp = _gauss(mean, cov)
    x = rng.normal(size=(w, d)) * 0.1 + np.array([-3.0, 4.0])   # start far away and squeezed
    l = np.array([lp(v) for v in x])
    u = _uniforms(rng, steps, w)
    samples = []
    acc = 0
    for s in range(steps):
        acc += int(S.step(x, l, u[s], lp).sum())
        if s >= burn:
            samples.append(x.copy())
    xs = np.concatenate(samples)
    assert 0.2 < acc / (steps * w) < 0.9
    np.testing.assert_allclose(xs.mean(axis=0), mean, atol=0.1)
    np.testing.assert_allclose(np.cov(xs.T), cov, atol=0.15)


def test_unit_stretch_keeps_the_walker_and_is_accepted():
    # u1 = (sqrt(a) - 1) / (a - 1) gives z = 1, so Y = X_k and the ratio is 1
    a = 2.0
    u1 = (math.sqrt(a) - 1) / (a - 1)
    assert S.stretch_factor(u1, a) == pytest.approx(1.0, rel=1e-15)
    x = np.array([[0.0, 1.0], [2.0, 3.0], [4.0, -1.0], [5.0, 5.0]])
    lp = lambda v: -float(v @ v)
    l = np.array([lp(v) for v in x])
    u = np.array([[0.0, u1, 0.999999], [0.7, u1, 0.999999]])
    flags = S.half_step(x, l, True, u, lp)
    assert flags.all()
    np.testing.assert_allclose(x[:2], [[0.0, 1.0], [2.0, 3.0]], rtol=1e-15, atol=1e-15)


def test_prior_walls_reject_and_halves_use_the_other_halfs_start():
    rng = np.random.default_rng(8)
    lo, hi = [0.0, 0.0], [1.0, 1.0]
    lp = S.box_prior(lo, hi, lambda v: 0.0)
    x = rng.random((8, 2))
    l = np.zeros(8)
    for s in range(50):
        S.step(x, l, rng.random((2, 4, 3)), lp)
        assert np.all((x >= 0) & (x <= 1))
    # a far-out proposal (z = a stretching away from a partner) outside the box is never taken
    x = np.array([[0.9, 0.9], [0.9, 0.95], [0.05, 0.05], [0.1, 0.1]])
    l = np.zeros(4)
    flags = S.half_step(x, l, True, np.array([[0.0, 1.0 - 1e-12, 0.0], [0.5, 1.0 - 1e-12, 0.0]]), lp)
    assert not flags.any()
    # the moves of one half depend only on the other half: permuting the active
    # half permutes the outcome
    x = rng.random((6, 2))
    l = np.array([lp(v) for v in x])
    u = rng.random((3, 3))
    xa, la = x.copy(), l.copy()
    S.half_step(xa, la, True, u, lp)
    perm = [2, 0, 1]
    xb = x.copy()
    xb[:3] = x[perm]
    lb = l.copy()
    lb[:3] = l[perm]
    S.half_step(xb, lb, True, u[perm], lp)
    np.testing.assert_array_equal(xb[:3], xa[perm])
