"""Pins of the FP64 chi^2 likelihood oracle (Section 2.5, multi-epoch sum of Section 3.4).

Each test fixes the statistic through a route other than its own loop: exact
special cases (model equal to mock, a uniform fractional offset, noise only),
the fitted k range decided on hand-placed bin centres, linearity over
redshifts, scalings, and Delta^2 of a plane wave in closed form.  No GPU.
"""
import math

import numpy as np
import pytest

import oracle

L = oracle.likelihood


def _bins(k):
    return np.asarray(k, float), np.ones(len(k))


def test_model_equal_to_mock_gives_zero():
    k, c = _bins([0.1, 0.2, 0.5, 0.9, 1.5])
    mock = np.array([3.0, 10.0, 25.0, 40.0, 55.0])
    assert L.chi2(mock, mock, np.zeros(5), k, c) == 0.0


@pytest.mark.parametrize("eps", [0.01, -0.2, 0.5])
def test_uniform_fractional_offset_closed_form(eps):
    # noise 0: each fitted bin contributes (eps m)^2 / (0.25 m)^2 = (eps / 0.25)^2
    k, c = _bins([0.05, 0.15, 0.3, 0.6, 1.0, 1.01])
    mock = np.array([1.0, 2.0, 7.0, 11.0, 13.0, 17.0])
    got = L.chi2((1 + eps) * mock, mock, np.zeros(6), k, c)
    assert got == pytest.approx(4 * (eps / 0.25) ** 2, rel=1e-13)


def test_noise_only_hand_values():
    # model error switched off: sum of squared residuals over sigma
    k, c = _bins([0.2, 0.4, 0.8])
    model = np.array([2.0, 5.0, 9.0])
    mock = np.array([1.0, 1.0, 9.0])
    noise = np.array([1.0, 2.0, 3.0])
    assert L.chi2(model, mock, noise, k, c, model_err=0.0) == pytest.approx(1.0 + 4.0 + 0.0, rel=1e-15)


def test_noise_and_model_error_add_in_quadrature():
    # one fitted bin: residual 3, noise 4, mock 12 -> model error 3: variance 16 + 9 = 25
    k, c = _bins([0.5])
    assert L.chi2([15.0], [12.0], [4.0], k, c) == pytest.approx(9.0 / 25.0, rel=1e-15)


def test_fitted_range_is_inclusive_and_needs_modes():
    k = [0.1, 0.15, 0.5, 1.0, 1.2, 0.7]
    c = [4, 4, 4, 4, 4, 0]
    use = L.likelihood_bins(k, c)
    assert use.tolist() == [False, True, True, True, False, False]
    # only fitted bins count: a residual in an unfitted bin changes nothing
    mock = np.ones(6)
    model = np.array([50.0, 1.0, 1.0, 1.0, 50.0, 50.0])
    assert L.chi2(model, mock, np.zeros(6), k, c) == 0.0


def test_zero_variance_bin_is_left_out():
    k, c = _bins([0.2, 0.3])
    assert L.chi2([1.0, 2.0], [0.0, 1.0], [0.0, 0.0], k, c) == pytest.approx((1.0 / 0.25) ** 2)


def test_redshifts_add_linearly():
    k, c = _bins([0.2, 0.4, 0.8])
    rng = np.random.default_rng(5)
    parts = []
    for _ in range(3):
        mock = rng.uniform(1, 30, 3)
        model = rng.uniform(1, 30, 3)
        parts.append(L.chi2(model, mock, rng.uniform(0, 2, 3), k, c))
    assert L.chi2_total(parts) == pytest.approx(sum(parts), rel=1e-15)


def test_scaling_of_errors():
    # doubling the noise and the model error quarters the statistic
    k, c = _bins([0.2, 0.4, 0.8])
    model, mock, noise = np.array([3.0, 4.0, 5.0]), np.array([1.0, 6.0, 2.0]), np.array([0.5, 1.0, 2.0])
    a = L.chi2(model, mock, noise, k, c, model_err=0.25)
    b = L.chi2(model, mock, 2 * noise, k, c, model_err=0.5)
    assert b == pytest.approx(a / 4, rel=1e-14)


def test_delta2_of_a_plane_wave():
    # a single plane wave puts all power in one bin: P_b = A^2 L^3 / (2 c_b),
    # and Delta^2_b = k_b^3 P_b / (2 pi^2) with k_b the bin's mean |k|, found
    # here by enumerating the full (not half) grid of modes
    n, box, amp, nb = 16, 40.0, 2.0, 5
    m = (1, 2, 2)
    g = np.indices((n, n, n))
    f = amp * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)
    _, kb, c, d2 = oracle.power_spectrum(f, box, nb)
    b = oracle.bin_of_n2(9, n, nb)
    ks, cnt = 0.0, 0
    for i in range(n):
        for j in range(n):
            for l in range(n):
                v = [x if x < n // 2 else x - n for x in (i, j, l)]
                n2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
                if oracle.bin_of_n2(n2, n, nb) == b:
                    ks += 2 * math.pi / box * math.sqrt(n2)
                    cnt += 1
    assert c[b] == cnt
    k_b = ks / cnt
    assert kb[b] == pytest.approx(k_b, rel=1e-13)
    assert d2[b] == pytest.approx(k_b ** 3 * amp ** 2 * box ** 3 / (2 * cnt) / (2 * math.pi ** 2), rel=1e-11)
    assert np.all(np.abs(np.delete(d2, b)) <= 1e-12 * d2[b])  # FFT round-off only
