"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle through a route other than its own formula: exact
DFT sums, closed-form integrals, inverse functions, plane waves, hand-derived
tables and exact special cases.  None of these tests touch the GPU.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.special

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
PHYS = oracle.Physics(pk_amp=synth.reference_amplitude())


# ---------------------------------------------------------------- helpers

def brute_dft_full(f):
    """Unnormalised forward DFT by explicit sums (N^6 work), full grid."""
    n = f.shape[0]
    idx = np.arange(n)
    e = np.exp(-2j * np.pi * np.outer(idx, idx) / n)   # e[k, x]
    out = np.einsum("ax,by,cz,xyz->abc", e, e, e, f.astype(np.complex128))
    return out


def threshold_bins(n, n_bins):
    """Bin of each n2 from integer thresholds t_b = ceil((n/2)^(2b/n_bins)).

    A second route to the bin rule: derive the first integer n2 of each bin
    from the edge value instead of comparing powers.
    """
    half = n // 2
    t = []
    for b in range(n_bins + 1):
        num = 2 * b * int(math.log2(half))
        if num % n_bins == 0:
            t.append(2 ** (num // n_bins))
        else:
            v = half ** (2.0 * b / n_bins)
            assert abs(v - round(v)) > 1e-9
            t.append(math.ceil(v))
    out = {}
    for n2 in range(0, 3 * half * half + 1):
        if n2 == 0 or n2 > half * half:
            out[n2] = -1
            continue
        out[n2] = min(max(b for b in range(n_bins + 1) if n2 >= t[b]), n_bins - 1)
    return out


def sigma2_closed(radius, z, phys):
    """sigma^2 of the sharp-k window in closed form.

    With u = k^2 / k0^2: int_0^kc k^3 A (1 + k^2/k0^2)^-2 dk
      = A k0^4 / 2 [ln(1 + U) + 1 / (1 + U) - 1],  U = (kc / k0)^2.
    """
    kc = (4.5 * math.pi) ** (1 / 3) / radius
    u = (kc / phys.pk_k0) ** 2
    d = (1 + phys.z_ref) / (1 + z)
    return d * d * phys.pk_amp * phys.pk_k0 ** 4 / (4 * math.pi ** 2) * (math.log1p(u) + 1 / (1 + u) - 1)


# ---------------------------------------------------------------- FFT / P(k)

@pytest.mark.parametrize("n", [4, 8])
def test_power_spectrum_matches_brute_force_dft(n):
    rng = np.random.default_rng(11 + n)
    f = rng.standard_normal((n, n, n))
    box = 10.0
    nb = 3
    x = brute_dft_full(f)
    bins = threshold_bins(n, nb)
    a = np.rint(np.fft.fftfreq(n, 1.0 / n)).astype(int)
    psum = np.zeros(nb)
    ksum = np.zeros(nb)
    cnt = np.zeros(nb)
    kf = 2 * math.pi / box
    for i in range(n):
        for j in range(n):
            for k in range(n):
                n2 = a[i] ** 2 + a[j] ** 2 + a[k] ** 2
                b = bins[n2]
                if b < 0:
                    continue
                psum[b] += abs(x[i, j, k]) ** 2 * box ** 3 / n ** 6
                ksum[b] += kf * math.sqrt(n2)
                cnt[b] += 1
    pb, kb, c, d2 = oracle.power_spectrum(f, box, nb)
    np.testing.assert_array_equal(c, cnt)
    np.testing.assert_allclose(pb, psum / cnt, rtol=1e-12)
    np.testing.assert_allclose(kb, ksum / cnt, rtol=1e-13)
    np.testing.assert_allclose(d2, kb ** 3 * pb / (2 * math.pi ** 2), rtol=1e-13)


@pytest.mark.parametrize("m", [(1, 0, 0), (0, 0, 2), (1, 2, 3), (-3, 1, 1), (2, -2, 0)])
def test_plane_wave_power(m):
    n, box, amp, nb = 16, 50.0, 1.7, 6
    g = np.indices((n, n, n))
    f = amp * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)
    pb, kb, c, _ = oracle.power_spectrum(f, box, nb)
    b = oracle.bin_of_n2(sum(v * v for v in m), n, nb)
    expect = np.zeros(nb)
    expect[b] = amp ** 2 * box ** 3 / (2 * c[b])
    np.testing.assert_allclose(pb, expect, rtol=1e-11, atol=1e-9 * expect.max())


def test_parseval_band_limited():
    # a zero-mean field with no power beyond |n| = N/2: sum_b c_b P_b = V_cell sum f^2
    n, box = 16, 30.0
    rng = np.random.default_rng(5)
    f = rng.standard_normal((n, n, n))
    fh = np.fft.rfftn(f)
    fh *= (oracle.mode_n2(n) <= (n // 2) ** 2)
    fh[0, 0, 0] = 0
    f = np.fft.irfftn(fh, s=(n, n, n), axes=(0, 1, 2))
    pb, _, c, _ = oracle.power_spectrum(f, box, 5)
    np.testing.assert_allclose((c * pb).sum(), (box / n) ** 3 * (f ** 2).sum(), rtol=1e-12)


def test_bin_rule_golden():
    with open(os.path.join(HERE, "golden", "bin_edges_n8.json")) as fh:
        gold = json.load(fh)
    for case in gold["cases"]:
        for n2, b in case["bins"].items():
            assert oracle.bin_of_n2(int(n2), case["n"], case["n_bins"]) == b, (case["n_bins"], n2)


@pytest.mark.parametrize("n,nb", [(8, 12), (64, 12), (128, 15), (256, 15)])
def test_bin_rule_threshold_route(n, nb):
    tab = oracle.bin_table(n, nb)
    ref = threshold_bins(n, nb)
    assert all(tab[v] == ref[v] for v in range(len(tab)))


# ---------------------------------------------------------------- filter

def test_filter_constant_field_invariant():
    n, box = 16, 40.0
    d = np.full((n, n, n), 0.37)
    dh = np.fft.rfftn(d)
    for r in oracle.radius_ladder(20.0, box / n, 1.1):
        np.testing.assert_allclose(oracle.smooth(dh, n, box, r), 0.37, rtol=0, atol=1e-14)


def test_filter_plane_wave_cut_and_nesting():
    n, box = 16, 40.0
    kf = 2 * math.pi / box
    g = np.indices((n, n, n))
    m = (2, 1, 2)  # n2 = 9, |k| = 3 kf
    f = np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)
    fh = np.fft.rfftn(f)
    kc_of = lambda r: (4.5 * math.pi) ** (1 / 3) / r
    r_pass = (4.5 * math.pi) ** (1 / 3) / (3.01 * kf)   # k_c just above 3 kf
    r_stop = (4.5 * math.pi) ** (1 / 3) / (2.99 * kf)   # k_c just below
    assert kc_of(r_pass) > 3 * kf > kc_of(r_stop)
    np.testing.assert_allclose(oracle.smooth(fh, n, box, r_pass), f, atol=1e-13)
    np.testing.assert_allclose(oracle.smooth(fh, n, box, r_stop), 0.0, atol=1e-13)
    # idempotence and nesting of the sharp-k window
    rng = np.random.default_rng(3)
    x = rng.standard_normal((n, n, n))
    xh = np.fft.rfftn(x)
    a = oracle.smooth(xh, n, box, 5.0)
    np.testing.assert_allclose(oracle.smooth(np.fft.rfftn(a), n, box, 5.0), a, atol=1e-13)
    b = oracle.smooth(np.fft.rfftn(oracle.smooth(xh, n, box, 3.0)), n, box, 7.0)
    np.testing.assert_allclose(b, oracle.smooth(xh, n, box, 7.0), atol=1e-13)


def test_filter_matches_real_space_convolution():
    # N = 8: periodic convolution with K(x) = N^-3 sum_{|k| <= kc} exp(i k.x)
    n, box, r = 8, 16.0, 3.3
    kf = 2 * math.pi / box
    kc = (4.5 * math.pi) ** (1 / 3) / r
    a = np.rint(np.fft.fftfreq(n, 1.0 / n)).astype(int)
    kern = np.zeros((n, n, n), dtype=np.complex128)
    g = np.indices((n, n, n))
    for i in a:
        for j in a:
            for k in a:
                if kf * math.sqrt(i * i + j * j + k * k) <= kc:
                    kern += np.exp(2j * np.pi * (i * g[0] + j * g[1] + k * g[2]) / n)
    kern = kern.real / n ** 3
    rng = np.random.default_rng(8)
    f = rng.standard_normal((n, n, n))
    conv = np.zeros_like(f)
    for x0 in range(n):
        for x1 in range(n):
            for x2 in range(n):
                conv[x0, x1, x2] = (f * np.roll(np.roll(np.roll(kern[::-1, ::-1, ::-1], x0 + 1, 0),
                                                        x1 + 1, 1), x2 + 1, 2)).sum()
    got = oracle.smooth(np.fft.rfftn(f), n, box, r)
    np.testing.assert_allclose(got, conv, atol=1e-12)


# ---------------------------------------------------------------- scalars

@pytest.mark.parametrize("r,z", [(15.0, 9.0), (2.0, 9.0), (0.1937, 9.0), (20.0, 8.0), (0.78125, 10.0)])
def test_sigma2_quadrature_matches_closed_form(r, z):
    assert oracle.mass_variance(r, z, PHYS) == pytest.approx(sigma2_closed(r, z, PHYS), rel=1e-10)


def test_sigma2_is_variance_of_filtered_field():
    # expected variance of a sharp-k filtered Gaussian box = (1/V) sum_{0<|k|<=kc} P(k)
    # and approaches the continuous sigma^2 for R >> cell size
    n, box, r = 64, 128.0, 15.0
    kf = 2 * math.pi / box
    a = np.rint(np.fft.fftfreq(n, 1.0 / n))
    k = kf * np.sqrt(a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2)
    p = oracle.linear_power(k, PHYS)
    p[0, 0, 0] = 0
    keep = k <= oracle.sharpk_cutoff(r)
    expect = p[keep].sum() / box ** 3
    vals = []
    for seed in range(6):
        d = synth.make_box(n, box, 9.0, seed=100 + seed, amp=PHYS.pk_amp, dtype=np.float64)
        vals.append(oracle.smooth(np.fft.rfftn(d), n, box, r).var())
    assert np.mean(vals) == pytest.approx(expect, rel=0.25)
    assert expect == pytest.approx(oracle.mass_variance(r, 9.0, PHYS), rel=0.3)


def test_min_halo_mass_scalings():
    assert oracle.min_halo_mass(1e4, 9.0, PHYS) == pytest.approx(1e8, rel=1e-15)
    assert oracle.min_halo_mass(5e4, 9.0, PHYS) == pytest.approx(1e8 * 5 ** 1.5, rel=1e-15)
    assert oracle.min_halo_mass(1e4, 8.0, PHYS) == pytest.approx(1e8 * 0.9 ** -1.5, rel=1e-15)
    # eq. (3) in an Einstein-de Sitter universe: Omega_m^z = 1, Delta_c = 18 pi^2
    eds = oracle.Physics(omega_m=1.0, omega_l=0.0, h=1.0, mmin_form=1)
    assert oracle.min_halo_mass(1.98e4, 9.0, eds) == pytest.approx(1e8, rel=1e-14)
    assert oracle.min_halo_mass(1.98e4 * 4, 3.0, eds) == pytest.approx(8e8 * 0.4 ** -1.5, rel=1e-14)


def test_radius_of_mass_sphere():
    rho = 0.27 * 2.775e11 * 0.7 ** 2
    assert oracle.mean_matter_density(PHYS) == pytest.approx(rho, rel=1e-15)
    for m in (1e8, 1.1e9, 3e11):
        r = oracle.radius_of_mass(m, PHYS)
        assert 4 * math.pi / 3 * r ** 3 * rho == pytest.approx(m, rel=1e-13)


def test_sharpk_cutoff_volume_matching():
    # number of modes per unit volume inside |k| <= kc equals one per sphere volume
    for r in (0.5, 2.0, 15.0):
        kc = oracle.sharpk_cutoff(r)
        assert (4 * math.pi / 3 * kc ** 3) / (2 * math.pi) ** 3 == pytest.approx(1 / (4 * math.pi / 3 * r ** 3), rel=1e-14)


def test_radius_ladder():
    lad = oracle.radius_ladder(15.0, 2.0, 1.1)
    assert len(lad) == 23 and lad[0] == 15.0 and lad[-1] == 2.0
    assert all(a > b for a, b in zip(lad, lad[1:]))
    assert lad[-2] > 2.0 and lad[-2] / 1.1 <= 2.0
    assert oracle.radius_ladder(1.0, 2.0, 1.1) == [2.0]
    shared = oracle.radius_ladder(20.0, 250 / 256, 1.1)
    w = oracle.walker_radii(shared, 12.0)
    assert w[-1] == shared[-1] and max(w) <= 12.0 and max(w) * 1.1 > 12.0
    assert w == [r for r in shared if r <= 12.0]


# ---------------------------------------------------------------- ionisation

def _uniform_case(c, zeta, t_vir, n=8, box=16.0, z=9.0):
    d = np.full((n, n, n), c)
    radii = oracle.radius_ladder(10.0, box / n, 1.1)
    flagged, x_hi = oracle.ionization_field(d, box, z, zeta, t_vir, radii, PHYS)
    return radii, flagged, x_hi


def _dsig2(r, t_vir, z):
    smin = sigma2_closed(oracle.radius_of_mass(oracle.min_halo_mass(t_vir, z, PHYS), PHYS), z, PHYS)
    return smin - sigma2_closed(r, z, PHYS)


def test_uniform_box_flag_threshold_by_inverse_erfc():
    zeta, t_vir, z = 20.0, 3e4, 9.0
    radii = oracle.radius_ladder(10.0, 2.0, 1.1)
    # zeta erfc(u) >= 1  <=>  delta >= delta_c - sqrt(2 dsig2) erfcinv(1/zeta); the
    # largest radius has the largest dsig2 and so the lowest threshold
    thr = min(PHYS.delta_c - math.sqrt(2 * _dsig2(r, t_vir, z)) * scipy.special.erfcinv(1 / zeta)
              for r in radii)
    _, fl_hi, x_hi_hi = _uniform_case(thr + 1e-9, zeta, t_vir)
    _, fl_lo, x_hi_lo = _uniform_case(thr - 1e-9, zeta, t_vir)
    assert fl_hi.all() and not fl_lo.any()
    assert (x_hi_hi == 0).all() and (x_hi_lo > 0).all()


def test_uniform_box_partial_ionisation_at_cell_scale():
    # zeta = 1 never flags a box below delta_c; choose delta so that f_coll at the
    # cell radius is exactly y: x_HI must be 1 - zeta y
    t_vir, z = 2e4, 9.0
    for y in (0.25, 0.6, 0.9):
        c = PHYS.delta_c - math.sqrt(2 * _dsig2(2.0, t_vir, z)) * scipy.special.erfcinv(y)
        radii, flagged, x_hi = _uniform_case(c, 1.0, t_vir)
        assert radii[-1] == 2.0 and not flagged.any()
        np.testing.assert_allclose(x_hi, 1.0 - y, rtol=1e-12)


def test_uniform_box_power_is_zero_and_brightness_closed_form():
    n, box, z = 8, 16.0, 9.0
    c = 0.3
    radii, flagged, x_hi = _uniform_case(c, 5.0, 1e5)
    dtb = oracle.brightness_temperature(x_hi, np.full((n, n, n), c), z, PHYS)
    np.testing.assert_allclose(dtb, 27.0 * x_hi * 1.3, rtol=1e-15)
    # eq. (4) redshift factor sqrt((1 + z) / 10): 1.6 at z = 15, 0.9 at z = 8
    np.testing.assert_allclose(oracle.brightness_temperature(np.ones(3), np.zeros(3), 15.0, PHYS),
                               27.0 * math.sqrt(1.6), rtol=1e-15)
    np.testing.assert_allclose(oracle.brightness_temperature(np.full(3, 0.5), np.full(3, -0.5), 8.0, PHYS),
                               27.0 * 0.25 * math.sqrt(0.9), rtol=1e-15)
    pb, _, _, _ = oracle.power_spectrum(dtb, box, 3)
    assert np.all(np.abs(pb) < 1e-20)


def test_cells_below_minimum_mass_get_no_collapse():
    # T_vir high enough that the cell sphere holds less than M_min: f_coll = 0 there
    n, box, z = 8, 6.0, 9.0   # cell radius 0.75 Mpc
    t_vir = 1e6
    assert oracle.radius_of_mass(oracle.min_halo_mass(t_vir, z, PHYS), PHYS) > box / n
    d = np.full((n, n, n), 5.0)  # far above delta_c
    flagged, x_hi = oracle.ionization_field(d, box, z, 50.0, t_vir, [box / n], PHYS)
    assert not flagged.any() and (x_hi == 1.0).all()


def test_extremes():
    n, box = 16, 32.0
    d = synth.make_box(n, box, 9.0, seed=21, amp=PHYS.pk_amp, dtype=np.float64)
    radii = oracle.radius_ladder(15.0, box / n, 1.1)
    ev = oracle.evaluate(d, box, 9.0, (1e12, 15.0, 1e4), radii, 4, PHYS)
    assert ev.flagged.all() and ev.xhi_mean == 0.0 and np.all(ev.pk == 0.0)
    ev = oracle.evaluate(d, box, 9.0, (0.49, 15.0, 1e4), radii, 4, PHYS)
    assert not ev.flagged.any()


def test_monotonicity_in_parameters():
    n, box, z = 16, 32.0, 9.0
    d = synth.make_box(n, box, z, seed=22, amp=PHYS.pk_amp, dtype=np.float64)
    shared = oracle.radius_ladder(20.0, box / n, 1.1)

    def xh(zeta, rmfp, tv):
        return oracle.ionization_field(d, box, z, zeta, tv, oracle.walker_radii(shared, rmfp), PHYS)[1]

    base = xh(20.0, 10.0, 3e4)
    assert np.all(xh(40.0, 10.0, 3e4) <= base + 1e-15)          # more efficient -> more ionised
    assert np.all(xh(20.0, 18.0, 3e4) <= base + 1e-15)          # larger horizon -> more ionised
    assert np.all(xh(20.0, 10.0, 1e5) >= base - 1e-15)          # rarer sources -> less ionised
    assert xh(40.0, 10.0, 3e4).mean() < base.mean() < xh(20.0, 10.0, 1e5).mean()


def test_whole_path_brute_force_n8():
    """N = 8: the whole path with explicit DFT sums and math.erfc per cell."""
    n, box, z = 8, 16.0, 9.0
    zeta, t_vir = 25.0, 2e4
    d = synth.make_box(n, box, z, seed=31, amp=PHYS.pk_amp, dtype=np.float64)
    radii = oracle.radius_ladder(9.0, box / n, 1.1)
    kf = 2 * math.pi / box
    a = np.rint(np.fft.fftfreq(n, 1.0 / n)).astype(int)
    n2 = a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2
    dh = brute_dft_full(d)
    idx = np.arange(n)
    einv = np.exp(2j * np.pi * np.outer(idx, idx) / n) / n
    smin = sigma2_closed(oracle.radius_of_mass(oracle.min_halo_mass(t_vir, z, PHYS), PHYS), z, PHYS)
    flagged = np.zeros((n, n, n), dtype=bool)
    fcell = None
    for r in radii:
        kc = (4.5 * math.pi) ** (1 / 3) / r
        dr = np.einsum("xa,yb,zc,abc->xyz", einv, einv, einv, dh * (kf * np.sqrt(n2) <= kc)).real
        s2 = smin - sigma2_closed(r, z, PHYS)
        f = np.zeros_like(dr)
        if s2 > 0:
            f = np.vectorize(lambda v: math.erfc((PHYS.delta_c - v) / math.sqrt(2 * s2)))(dr)
        flagged |= zeta * f >= 1
        fcell = f
    x_hi = np.where(flagged, 0.0, 1 - zeta * fcell)
    dtb = 27.0 * x_hi * (1 + d) * math.sqrt((1 + z) / 10)
    ev = oracle.evaluate(d, box, z, (zeta, 9.0, t_vir), radii, 3, PHYS)
    assert 0 < flagged.mean() < 1
    np.testing.assert_array_equal(ev.flagged, flagged)
    np.testing.assert_allclose(ev.x_hi, x_hi, atol=1e-9)
    np.testing.assert_allclose(ev.dtb, dtb, atol=1e-8)
    x = brute_dft_full(dtb)
    bins = threshold_bins(n, 3)
    ps = np.zeros(3)
    cn = np.zeros(3)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                b = bins[int(n2[i, j, k])]
                if b >= 0:
                    ps[b] += abs(x[i, j, k]) ** 2 * box ** 3 / n ** 6
                    cn[b] += 1
    np.testing.assert_allclose(ev.pk, ps / cn, rtol=1e-9)
    assert ev.xhi_mean == pytest.approx(x_hi.mean(), rel=1e-12)


# ---------------------------------------------------------------- velocity-gradient factor (eq. 4)

def _wave(n, m, amp):
    g = np.indices((n, n, n))
    return amp * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)


@pytest.mark.parametrize("m,share", [((2, 0, 0), 1.0), ((0, 3, 0), 0.0), ((0, 0, 1), 0.0),
                                     ((1, 1, 0), 0.5), ((1, 1, 1), 1.0 / 3.0), ((-2, 1, 2), 4.0 / 9.0)])
def test_velocity_gradient_of_plane_waves(m, share):
    # a plane wave along k has gradient share (k_r / |k|)^2 of delta along the
    # line of sight (the first axis), from linear continuity with f = 1
    d = _wave(16, m, 0.3)
    np.testing.assert_allclose(oracle.velocity_gradient(d), share * d, atol=1e-14)


def test_velocity_gradients_of_three_sight_lines_sum_to_delta():
    # k_x^2 + k_y^2 + k_z^2 = k^2: the three line-of-sight gradients add up to
    # the density contrast minus its mean
    rng = np.random.default_rng(9)
    d = rng.standard_normal((16, 16, 16))
    total = sum(oracle.velocity_gradient(d, axis=a) for a in range(3))
    np.testing.assert_allclose(total, d - d.mean(), atol=1e-12)


def test_velocity_factor_limits_and_off_switch():
    d = _wave(16, (1, 0, 0), 1.0)        # gradient = delta, in [-1, 1]
    phys = oracle.Physics(pk_amp=PHYS.pk_amp, velocity=True, dvdr_max=0.2)
    f = oracle.velocity_factor(d, phys)
    assert f.min() == pytest.approx(1 / 1.2) and f.max() == pytest.approx(1 / 0.8)
    small = _wave(16, (1, 0, 0), 0.05)  # inside the limit: exactly 1 / (1 - delta)
    np.testing.assert_allclose(oracle.velocity_factor(small, phys), 1 / (1 - small), rtol=1e-13)
    x = np.full(d.shape, 0.7)
    on = oracle.brightness_temperature(x, small, 9.0, phys)
    off = oracle.brightness_temperature(x, small, 9.0, oracle.Physics(pk_amp=PHYS.pk_amp))
    np.testing.assert_allclose(on, off / (1 - small), rtol=1e-13)
    # a uniform box has no velocity gradient: the factor is 1
    u = np.full((8, 8, 8), 0.4)
    np.testing.assert_allclose(oracle.velocity_factor(u, phys), 1.0, atol=1e-15)
