"""Host planning of the library (FP64, no device) against the oracle and the header.

These call the C-ABI's pure host functions: radius ladders, sigma^2, the
per-walker flag thresholds (eq. 1 rewritten with erfc^-1), the exact k-bin
table, and argument validation.  No GPU is touched.
"""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.special

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
AMP = synth.reference_amplitude()
PHYS = oracle.Physics(pk_amp=AMP)


@pytest.fixture(scope="module")
def xs():
    import paper_1501_06576_amd as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1501_06576_amd import build
        build.build()
    mod.library()
    return mod


def test_header_symbols_exported(xs):
    header = open(os.path.join(ROOT, "include", "xs21.h")).read()
    declared = set(re.findall(r"^(?:xs21_status|const char\*)\s+(xs21_\w+)\s*\(", header, re.M))
    assert len(declared) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", xs.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (xs21_\w+)", out))
    assert declared <= exported, declared - exported
    for name in declared:
        assert hasattr(xs.library(), name)
    # the binding declares a signature for every exported entry point
    assert declared <= set(xs._SIGNATURES)


def test_physics_defaults(xs):
    p = xs.physics()
    assert (p.delta_c, p.omega_m, p.omega_l, p.h, p.tb0_mK) == (1.686, 0.27, 0.73, 0.7, 27.0)
    assert (p.pk_k0, p.z_ref, p.radius_step, p.ladder_top, p.mmin_form) == (0.05, 9.0, 1.1, 20.0, 0)


@pytest.mark.parametrize("top,cell", [(20.0, 250 / 256), (15.0, 2.0), (20.0, 400 / 512), (1.0, 2.0), (5.0, 128 / 64)])
def test_ladder_matches_oracle(xs, top, cell):
    assert xs.plan_ladder(top, cell, 1.1) == oracle.radius_ladder(top, cell, 1.1)


@pytest.mark.parametrize("r,z", [(20.0, 8.0), (15.0, 9.0), (2.0, 9.0), (0.976, 10.0), (0.19, 9.0), (0.05, 8.0)])
def test_sigma2_matches_quadrature(xs, r, z):
    p = xs.physics(pk_amp=AMP)
    assert xs.plan_sigma2(p, r, z) == pytest.approx(oracle.mass_variance(r, z, PHYS), rel=1e-10)


WALKERS = [(30.0, 15.0, 5e4), (5.0, 5.0, 1e6), (100.0, 20.0, 1e4), (0.7, 10.0, 2e4), (0.4, 12.0, 2e4),
           (50.0, 1.0, 3e4), (17.0, 7.7, 2.2e5)]


@pytest.mark.parametrize("w", WALKERS)
@pytest.mark.parametrize("mmin_form", [0, 1])
def test_walker_thresholds(xs, w, mmin_form):
    z, n, box = 8.5, 256, 250.0
    phys = oracle.Physics(pk_amp=AMP, mmin_form=mmin_form)
    radii = oracle.shared_radii(n, box, phys)
    got = xs.plan_walker(xs.physics(pk_amp=AMP, mmin_form=mmin_form), z, radii, w)
    zeta, r_mfp, t_vir = w
    m_min = oracle.min_halo_mass(t_vir, z, phys)
    assert got["m_min"] == pytest.approx(m_min, rel=1e-13)
    s_min = oracle.mass_variance(oracle.radius_of_mass(m_min, phys), z, phys)
    for j, r in enumerate(radii):
        ds = s_min - oracle.mass_variance(r, z, phys)
        assert got["dsig2"][j] == pytest.approx(ds, rel=1e-9, abs=1e-12)
        if ds > 0 and zeta > 0.5:
            thr = phys.delta_c - math.sqrt(2 * ds) * scipy.special.erfcinv(1 / zeta)
            assert got["thr"][j] == pytest.approx(thr, rel=1e-9, abs=1e-11)
            # the threshold is where zeta f_coll crosses 1
            f = lambda d: zeta * math.erfc((phys.delta_c - d) / math.sqrt(2 * ds))
            t = got["thr"][j]
            assert f(t + 1e-9 * max(1, abs(t))) >= 1.0 >= f(t - 1e-9 * max(1, abs(t)))
        else:
            assert math.isinf(got["thr"][j])
    first = next((j for j, r in enumerate(radii[:-1]) if r <= r_mfp), len(radii) - 1)
    assert got["first"] == first
    assert oracle.walker_radii(radii, r_mfp) == radii[first:]


@pytest.mark.parametrize("n,nb", [(8, 3), (8, 12), (16, 4), (64, 12), (128, 15), (256, 15), (512, 15), (64, 64)])
def test_bins_exact(xs, n, nb):
    np.testing.assert_array_equal(xs.plan_bins(n, nb), oracle.bin_table(n, nb))


def test_no_ladder_radius_on_a_mode_shell(xs):
    # the sharp-k mask is decided on integer |n|^2 <= floor((k_c L / 2 pi)^2); a
    # ladder radius whose cutoff lands within 1e-9 of a shell would make that
    # decision depend on rounding.  None of the workload geometries do.
    for (n, box) in synth.BOX_SEEDS:
        for r in oracle.shared_radii(n, box, PHYS) + oracle.plain_radii(15.0, n, box, PHYS):
            x = (oracle.sharpk_cutoff(r) * box / (2 * math.pi)) ** 2
            assert abs(x - round(x)) > 1e-9, (n, box, r)


def test_argument_validation(xs):
    p = xs.physics()
    with pytest.raises(xs.Xs21Error) as e:
        xs.plan_ladder(-1.0, 1.0, 1.1)
    assert e.value.status == -1
    with pytest.raises(xs.Xs21Error):
        xs.plan_ladder(10.0, 1.0, 1.0)
    with pytest.raises(xs.Xs21Error):
        xs.plan_bins(100, 10)
    with pytest.raises(xs.Xs21Error):
        xs.plan_bins(64, 0)
    with pytest.raises(xs.Xs21Error):
        xs.plan_walker(p, 9.0, [2.0], (float("nan"), 5.0, 1e4))
    with pytest.raises(xs.Xs21Error):
        xs.plan_walker(p, 9.0, [2.0], (10.0, -5.0, 1e4))
    with pytest.raises(xs.Xs21Error):
        xs.plan_sigma2(xs.physics(pk_amp=-1.0), 1.0, 9.0)
    bad = xs.physics(radius_step=0.9)
    with pytest.raises(xs.Xs21Error):
        xs.plan_sigma2(bad, 1.0, 9.0)


def test_context_needs_a_device(xs):
    # without a GPU the context cannot be created: the library reports it
    # instead of falling back to anything
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    p = xs.physics()
    st = xs.library().xs21_create(ctypes.byref(ctx), 0, None, ctypes.byref(p))
    assert st == -3 and not ctx.value
