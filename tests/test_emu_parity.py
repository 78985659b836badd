"""The library's own kernel and host sources, built for the CPU emulation of HIP
(tests/emu, AddressSanitizer on), against the FP64 oracle.

This is not the GPU path: it checks indexing, synchronisation structure, edge
cases and host logic of the same source files without a GPU.  The GPU parity
tests (test_gpu_parity.py) are the parity claim.
"""
import numpy as np
import pytest

import emu_harness as eh
import oracle
import synth

AMP = synth.reference_amplitude()
PHYS = oracle.Physics(pk_amp=AMP)
EDGE = [(30.0, 15.0, 5e4), (100.0, 20.0, 1e4), (5.0, 5.0, 1e6), (0.4, 12.0, 2e4), (60.0, 1.0, 3e4),
        (0.8, 9.0, 2e4)]


def _check(run, boxes, specs, walkers, tol_pk, flips_max, plain=True, tag="", fields=True, phys=PHYS):
    nbmax = max(s[3] for s in specs)
    pk = run.read(f"batch{tag}_pk.bin", np.float64, (len(walkers), len(specs), nbmax))
    xm = run.read(f"batch{tag}_xhi.bin", np.float64, (len(walkers), len(specs)))
    for bi, (n, box, z, nb) in enumerate(specs):
        dt = boxes[bi].dtype
        shared = oracle.shared_radii(n, box, phys)
        for wi, w in enumerate(walkers):
            ev = oracle.evaluate(boxes[bi], box, z, w, oracle.walker_radii(shared, w[1]), nb, phys)
            ok = ev.counts > 0
            scale = max(ev.pk[ok].max(), 1e-30)
            np.testing.assert_allclose(pk[wi, bi, :nb][ok], ev.pk[ok], rtol=tol_pk, atol=tol_pk * scale)
            assert np.all(pk[wi, bi, nb:] == 0)
            assert xm[wi, bi] == pytest.approx(ev.xhi_mean, abs=max(tol_pk, 1e-12))
            if wi == 1 and fields:
                x = run.read(f"mat_b{bi}_w1_xhi.bin", dt, (n, n, n))
                assert np.mean((x == 0) != ev.flagged) <= flips_max
        if plain:
            w = walkers[0]
            ev = oracle.evaluate(boxes[bi], box, z, w, oracle.plain_radii(w[1], n, box, phys), nb, phys)
            x = run.read(f"plain_b{bi}_w0_xhi.bin", dt, (n, n, n))
            d = run.read(f"plain_b{bi}_w0_dtb.bin", dt, (n, n, n))
            p = run.read(f"plain_b{bi}_w0_pk.bin", np.float64)[:nb]
            assert np.mean((x == 0) != ev.flagged) <= flips_max
            same = (x == 0) == ev.flagged
            assert np.abs(x.astype(np.float64) - ev.x_hi)[same].max() <= max(tol_pk, 1e-12) * 10
            assert np.abs(d.astype(np.float64) - ev.dtb)[same].max() <= max(tol_pk, 1e-12) * 300
            np.testing.assert_allclose(p, ev.pk, rtol=tol_pk)
            np.testing.assert_array_equal(run.read(f"plain_b{bi}_w0_cnt.bin", np.float64)[:nb], ev.counts)


def _run(storage, specs, walkers, max_walkers, dtype, extra=(), phys=None):
    run = eh.EmuRun(storage=storage, max_walkers=max_walkers, phys=phys or {"pk_amp": AMP})
    boxes = []
    for i, (n, box, z, nb) in enumerate(specs):
        d = synth.make_box(n, box, z, seed=60 + i, amp=AMP, dtype=dtype)
        boxes.append(d)
        run.box(d, box, z, nb)
    for w in walkers:
        run.walker(*w)
    run.cmd("prepare")
    run.cmd(f"batch {max(s[3] for s in specs)}")
    for bi in range(len(specs)):
        run.cmd(f"plain {bi} 0 -")
        run.cmd(f"materialize {bi} 1")
    for c in extra:
        run.cmd(c)
    run.run()
    return run, boxes


@pytest.mark.parametrize("radius_batch", [None, "3"])
def test_emu_f64_two_geometries_chunked(monkeypatch, radius_batch):
    # radius_batch: smoothed boxes per launch (default: all radii of a box at once)
    if radius_batch:
        monkeypatch.setenv("XS21_RADIUS_BATCH", radius_batch)
    specs = [(8, 6.0, 9.0, 3), (16, 12.0, 8.0, 4)]   # cell 0.75 Mpc: M_min can exceed the cell mass
    run, boxes = _run("f64", specs, EDGE, 2, np.float64, extra=("smoothed 1 3", "smoothed 1 0"))
    _check(run, boxes, specs, EDGE, 1e-11, 0.0)
    dh = np.fft.rfftn(boxes[1])
    shared = oracle.shared_radii(16, 12.0, PHYS)
    for j in (0, 3):
        got = run.read(f"sm_b1_j{j}.bin", np.float64, (16, 16, 16))
        np.testing.assert_allclose(got, oracle.smooth(dh, 16, 12.0, shared[j]), atol=1e-13)


def test_emu_f32_and_bf16():
    specs = [(16, 32.0, 9.0, 5)]
    run, boxes = _run("f32", specs, EDGE[:4], 8, np.float32)
    _check(run, boxes, specs, EDGE[:4], 2e-5, 1e-3)
    run, boxes = _run("bf16", specs, EDGE[:4], 8, np.float32)
    _check(run, boxes, specs, EDGE[:4], 5e-2, 3e-2, plain=False)


def test_emu_power_spectrum_plane_wave():
    n, box, nb, amp = 8, 20.0, 3, 0.9
    run = eh.EmuRun(storage="f64", max_walkers=1, phys={"pk_amp": AMP})
    run.box(np.zeros((n, n, n)), box, 9.0, nb)
    g = np.indices((n, n, n))
    m = (1, 1, 2)
    f = amp * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)
    path = run.write_array("field.bin", f)
    run.cmd("prepare")
    run.cmd(f"pk 0 {path}")
    run.run()
    pk = run.read("fpk_b0.bin", np.float64)[:nb]
    _, _, counts, _ = oracle.power_spectrum(f, box, nb)
    b = oracle.bin_of_n2(6, n, nb)
    expect = np.zeros(nb)
    expect[b] = amp ** 2 * box ** 3 / (2 * counts[b])
    np.testing.assert_allclose(pk, expect, rtol=1e-12, atol=1e-12 * expect.max())


def test_emu_rejects_bad_box():
    run = eh.EmuRun(storage="f32", max_walkers=1, phys={"pk_amp": AMP})
    run.box(np.zeros((12, 12, 12), dtype=np.float32), 10.0, 9.0, 3)
    with pytest.raises(RuntimeError, match="power of two"):
        run.run()


def test_emu_power_spectrum_n64_random_field():
    # N = 64: the y pass splits into full aligned tiles plus gathered Nyquist
    # columns, and the binning pass into main and rest tiles
    n, box, nb = 64, 100.0, 8
    rng = np.random.default_rng(64)
    f = rng.standard_normal((n, n, n))
    run = eh.EmuRun(storage="f64", max_walkers=1, phys={"pk_amp": AMP})
    run.box(np.zeros((n, n, n)), box, 9.0, nb)
    path = run.write_array("field.bin", f)
    run.cmd("prepare")
    run.cmd(f"pk 0 {path}")
    run.run(timeout=1800)
    pk = run.read("fpk_b0.bin", np.float64)[:nb]
    ref, _, _, _ = oracle.power_spectrum(f, box, nb)
    np.testing.assert_allclose(pk, ref, rtol=1e-12)


def test_emu_resmooth_between_batches():
    # A new density box re-smoothed between two batches (and an in-place
    # re-smoothing) must reach the next batch; with max_walkers = 2 a batch of
    # 5 walkers on 2 boxes runs as 6 (box, walker group) units through the
    # shared scratch.  The emulated runtime defers all device work until the
    # host synchronises, so reading results before the work is ordered fails.
    specs = [(8, 6.0, 9.0, 3), (16, 12.0, 8.0, 4)]
    walkers = EDGE[:5]
    run = eh.EmuRun(storage="f64", max_walkers=2, phys={"pk_amp": AMP})
    boxes = []
    for i, (n, box, z, nb) in enumerate(specs):
        d = synth.make_box(n, box, z, seed=70 + i, amp=AMP, dtype=np.float64)
        boxes.append(d)
        run.box(d, box, z, nb)
    for w in walkers:
        run.walker(*w)
    new1 = synth.make_box(16, 12.0, 8.0, seed=99, amp=AMP, dtype=np.float64)
    path = run.write_array("new1.bin", new1)
    nbmax = max(s[3] for s in specs)
    run.cmd("prepare")
    run.cmd(f"batch {nbmax} A")
    run.cmd(f"resmooth 1 {path}")
    run.cmd(f"batch {nbmax} B")
    run.cmd("resmooth 0 -")
    run.cmd("resmooth 1 -")
    run.cmd(f"batch {nbmax} C")
    run.cmd("smoothed 1 2")
    run.run()
    _check(run, boxes, specs, walkers, 1e-11, 0.0, plain=False, tag="A", fields=False)
    _check(run, [boxes[0], new1], specs, walkers, 1e-11, 0.0, plain=False, tag="B", fields=False)
    for name in ("pk", "xhi"):
        np.testing.assert_array_equal(run.read(f"batchB_{name}.bin", np.float64),
                                      run.read(f"batchC_{name}.bin", np.float64))
    shared = oracle.shared_radii(16, 12.0, PHYS)
    got = run.read("sm_b1_j2.bin", np.float64, (16, 16, 16))
    np.testing.assert_allclose(got, oracle.smooth(np.fft.rfftn(new1), 16, 12.0, shared[2]), atol=1e-13)


def test_emu_chi2_epilogue():
    # chi^2 against a mock (the fiducial walker's oracle Delta^2) over the
    # fitted bins of two boxes, one with noise and one without
    specs = [(16, 64.0, 9.0, 4), (8, 40.0, 8.0, 3)]
    walkers = EDGE[:3]
    run = eh.EmuRun(storage="f64", max_walkers=2, phys={"pk_amp": AMP})
    boxes, mocks, noises = [], [], []
    for i, (n, box, z, nb) in enumerate(specs):
        d = synth.make_box(n, box, z, seed=80 + i, amp=AMP, dtype=np.float64)
        boxes.append(d)
        run.box(d, box, z, nb)
        fid = oracle.evaluate(d, box, z, (30.0, 15.0, 5e4), oracle.walker_radii(oracle.shared_radii(n, box, PHYS), 15.0),
                              nb, PHYS)
        mocks.append(fid.delta2)
        noises.append(np.linspace(0.5, 2.0, nb) if i == 0 else None)
    for w in walkers:
        run.walker(*w)
    run.cmd("prepare")
    run.cmd(f"batch {max(s[3] for s in specs)} A")
    for i in range(len(specs)):
        mp = run.write_array(f"mock{i}.bin", mocks[i])
        npth = run.write_array(f"noise{i}.bin", noises[i]) if noises[i] is not None else "-"
        run.cmd(f"mock {i} {mp} {npth} 0.25 0.15 1.0")
    run.cmd("chi2 A")
    run.run()
    nbmax = max(s[3] for s in specs)
    pk = run.read("batchA_pk.bin", np.float64, (len(walkers), len(specs), nbmax))
    got = run.read("chi2A.bin", np.float64)
    for wi, w in enumerate(walkers):
        own, ref, scale = [], [], 0.0
        for bi, (n, box, z, nb) in enumerate(specs):
            shared = oracle.shared_radii(n, box, PHYS)
            ev = oracle.evaluate(boxes[bi], box, z, w, oracle.walker_radii(shared, w[1]), nb, PHYS)
            noise = noises[bi] if noises[bi] is not None else np.zeros(nb)
            d2_own = ev.k_mean ** 3 * pk[wi, bi, :nb] / (2 * np.pi ** 2)
            own.append(oracle.likelihood.chi2(d2_own, mocks[bi], noise, ev.k_mean, ev.counts))
            ref.append(oracle.likelihood.chi2(ev.delta2, mocks[bi], noise, ev.k_mean, ev.counts))
            # size of the statistic for a model of zero power: sets the absolute tolerance
            scale += oracle.likelihood.chi2(np.zeros(nb), mocks[bi], noise, ev.k_mean, ev.counts)
        assert scale > 0
        # the epilogue itself: the oracle's statistic on the library's own P(k)
        # (walker 0 is the fiducial walker itself: chi^2 ~ 0)
        assert got[wi] == pytest.approx(oracle.likelihood.chi2_total(own), rel=1e-12, abs=1e-14 * scale)
        # end to end against the oracle's P(k) (FP64 path)
        assert got[wi] == pytest.approx(oracle.likelihood.chi2_total(ref), rel=1e-9, abs=1e-11 * scale)


def test_emu_velocity_factor():
    # dT_b with the line-of-sight velocity-gradient factor of eq. (4)
    specs = [(16, 24.0, 9.0, 4)]
    phys = oracle.Physics(pk_amp=AMP, velocity=True, dvdr_max=0.2)
    run, boxes = _run("f64", specs, EDGE[:3], 2, np.float64, phys={"pk_amp": AMP, "velocity": 1, "dvdr_max": 0.2})
    _check(run, boxes, specs, EDGE[:3], 1e-11, 0.0, phys=phys)


# two-population walkers (zeta0, R_mfp, T_feed, alpha, beta) of Section 4
EDGE2 = [(70.0, 15.0, 10 ** 4.7, 4.0 / 3.0, -1.0 / 3.0),   # the fiducial of Section 4
         (30.0, 15.0, 1e5, 10.0 / 3.0, -4.0 / 3.0),        # falls below 1 towards delta_c: bounded intervals
         (12.0, 8.0, 3e4, -4.0 / 3.0, 2.0),
         (25.0, 10.0, 2e5, 0.0, 0.0),                      # constant efficiency above 1e4 K
         (0.4, 12.0, 2e4, 1.0, 0.0),                       # F < 1 everywhere
         (200.0, 3.0, 1e6, 2.0, 3.0),
         (60.0, 0.5, 3e4, 1.0, -1.0)]                      # R_mfp below every ladder radius


def test_emu_two_population():
    # one box, six walkers in chunks of 4 (ragged), two materialised; the cell
    # (0.75 Mpc) holds more than the 1e4 K halo mass
    specs = [(16, 12.0, 8.0, 4)]
    walkers = EDGE2[:5] + EDGE2[6:]
    run = eh.EmuRun(storage="f64", max_walkers=4, phys={"pk_amp": AMP})
    n, box, z, nb = specs[0]
    d = synth.make_box(n, box, z, seed=80, amp=AMP, dtype=np.float64)
    run.box(d, box, z, nb)
    for w in walkers:
        run.walker2(*w)
    run.cmd("prepare")
    run.cmd(f"batch2 {nb}")
    for wi in (0, 1):
        run.cmd(f"materialize2 0 {wi}")
    run.run()
    pk = run.read("batch2_pk.bin", np.float64, (len(walkers), 1, nb))
    xm = run.read("batch2_xhi.bin", np.float64, (len(walkers), 1))
    shared = oracle.shared_radii(n, box, PHYS)
    for wi, w in enumerate(walkers):
        ev = oracle.two_population.evaluate(d, box, z, w, oracle.walker_radii(shared, w[1]), nb, PHYS)
        ok = ev.counts > 0
        np.testing.assert_allclose(pk[wi, 0][ok], ev.pk[ok], rtol=1e-6, atol=1e-6 * ev.pk[ok].max())
        assert xm[wi, 0] == pytest.approx(ev.xhi_mean, abs=2e-7)
        if wi in (0, 1):
            x = run.read(f"mat2_b0_w{wi}_xhi.bin", np.float64, (n, n, n))
            same = (x == 0) == ev.flagged
            assert np.mean(~same) == 0.0
            assert np.abs(x - ev.x_hi)[same].max() <= 2e-7


# Two-population walkers with narrow flag intervals: on the 16^3, 32 Mpc box
# below, 3 and 6 cells skip over the interval between radii, so that only the
# upper ends keep them unflagged (by the oracle's per-radius fractions).
NARROW2 = [(15.0, 15.0, 1e5, 10.0 / 3.0, -4.0 / 3.0), (20.0, 15.0, 3e5, 10.0 / 3.0, -10.0 / 3.0)]


def test_emu_two_population_f32():
    """FP32 two-population walkers take the sorted interval test of the team
    ionisation pass (two searches per slot: lower ends, raised upper ends);
    P(k) and the mean x_HI against the oracle, FP32 bounds (one cell of 16^3
    moves the mean by 2.4e-4), walkers whose upper ends decide cells included."""
    specs = [(16, 32.0, 8.5, 4)]
    walkers = EDGE2[:5] + EDGE2[6:] + NARROW2
    run = eh.EmuRun(storage="f32", max_walkers=8, phys={"pk_amp": AMP})
    n, box, z, nb = specs[0]
    d = synth.make_box(n, box, z, seed=80, amp=AMP, dtype=np.float32)
    run.box(d, box, z, nb)
    for w in walkers:
        run.walker2(*w)
    run.cmd("prepare")
    run.cmd(f"batch2 {nb}")
    run.run()
    pk = run.read("batch2_pk.bin", np.float64, (len(walkers), 1, nb))
    xm = run.read("batch2_xhi.bin", np.float64, (len(walkers), 1))
    shared = oracle.shared_radii(n, box, PHYS)
    for wi, w in enumerate(walkers):
        ev = oracle.two_population.evaluate(d, box, z, w, oracle.walker_radii(shared, w[1]), nb, PHYS)
        ok = ev.counts > 0
        np.testing.assert_allclose(pk[wi, 0][ok], ev.pk[ok], rtol=1e-3, atol=1e-3 * ev.pk[ok].max())
        assert xm[wi, 0] == pytest.approx(ev.xhi_mean, abs=1e-4)


def _oracle_chain(boxes, specs, mocks, dim, lo, hi, x0, u, a=2.0):
    """The oracle sampler's chain with ln p = -chi^2 / 2 from full oracle evaluations."""
    def loglike(p):
        tot = 0.0
        for bi, (n, box, z, nb) in enumerate(specs):
            radii = oracle.walker_radii(oracle.shared_radii(n, box, PHYS), p[1])
            if dim == 3:
                ev = oracle.evaluate(boxes[bi], box, z, (p[0], p[1], 10 ** p[2]), radii, nb, PHYS)
            else:
                ev = oracle.two_population.evaluate(boxes[bi], box, z, (p[0], p[1], 10 ** p[2], p[3], p[4]),
                                                    radii, nb, PHYS)
            tot += oracle.likelihood.chi2(ev.delta2, mocks[bi], np.zeros(nb), ev.k_mean, ev.counts)
        return -0.5 * tot
    lp_fn = oracle.sampler.box_prior(lo, hi, loglike)
    x = x0.copy()
    lp = np.array([lp_fn(v) for v in x])
    xs, lps, accs = [x.copy()], [lp.copy()], []
    for t in range(u.shape[0]):
        accs.append(oracle.sampler.step(x, lp, u[t], lp_fn, a))
        xs.append(x.copy())
        lps.append(lp.copy())
    return np.array(xs), np.array(lps), np.array(accs)


@pytest.mark.parametrize("dim", [3, 5])
def test_emu_mcmc_chain(dim):
    # steps of a small ensemble in walker chunks of 2 (a half of 3 walkers is
    # ragged), against the oracle sampler fed with the same uniforms
    if dim == 3:
        specs = [(16, 32.0, 9.0, 5)]
        lo, hi = [5.0, 5.0, 4.0], [100.0, 20.0, 5.3]
        fid = (30.0, 15.0, np.log10(5e4))
        nw, steps = 6, 2
    else:
        specs = [(8, 24.0, 10.0, 3)]   # the fiducial leaves x_HI ~ 0.5 here
        lo, hi = [5.0, 5.0, 4.0, -4 / 3, -4 / 3], [100.0, 20.0, 5.3, 10 / 3, 10 / 3]
        fid = (70.0, 15.0, 4.7, 4 / 3, -1 / 3)
        nw, steps = 4, 1
    # walkers around the fiducial (within 10 % of the prior range), inside the prior
    x0 = np.asarray(fid) + (np.asarray(hi) - np.asarray(lo)) * 0.1 * (synth.uniforms((nw, dim), 200 + dim) - 0.5)
    u = synth.uniforms((steps, 2, nw // 2, 3), 300 + dim)
    run = eh.EmuRun(storage="f64", max_walkers=2, phys={"pk_amp": AMP})
    boxes, mocks = [], []
    for i, (n, box, z, nb) in enumerate(specs):
        d = synth.make_box(n, box, z, seed=90 + i, amp=AMP, dtype=np.float64)
        boxes.append(d)
        run.box(d, box, z, nb)
        radii = oracle.walker_radii(oracle.shared_radii(n, box, PHYS), fid[1])
        if dim == 3:
            ev = oracle.evaluate(d, box, z, (fid[0], fid[1], 10 ** fid[2]), radii, nb, PHYS)
        else:
            ev = oracle.two_population.evaluate(d, box, z, (fid[0], fid[1], 10 ** fid[2], fid[3], fid[4]), radii,
                                                nb, PHYS)
        mocks.append(ev.delta2)
    run.cmd("prepare")
    for i in range(len(specs)):
        run.cmd(f"mock {i} {run.write_array(f'mock{i}.bin', mocks[i])} - 0.25 0.15 1.0")
    bpath = run.write_array("bounds.bin", np.concatenate([lo, hi]).astype(np.float64))
    xpath = run.write_array("x0.bin", x0.astype(np.float64))
    upath = run.write_array("u.bin", u.astype(np.float64))
    run.cmd(f"mcmc {dim} 2.0 {nw} {steps} {bpath} {xpath} {upath} A")
    run.run()
    gx = run.read("mcmcA_x.bin", np.float64, (steps + 1, nw, dim))
    glp = run.read("mcmcA_lp.bin", np.float64, (steps + 1, nw))
    gacc = run.read("mcmcA_acc.bin", np.int32, (steps, nw))
    ox, olp, oacc = _oracle_chain(boxes, specs, mocks, dim, lo, hi, x0, u)
    assert np.ptp(olp[0]) > 0.1   # a likelihood that tells the walkers apart
    np.testing.assert_array_equal(gacc.astype(bool), oacc)
    np.testing.assert_allclose(gx, ox, rtol=1e-12)
    tol = 1e-9 if dim == 3 else 1e-5
    np.testing.assert_allclose(glp, olp, rtol=tol, atol=0 if dim == 3 else 1e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_emu_batch_fields_mid_group(dtype):
    """Fields written by the batched ionisation launch for a walker in the middle
    of a later walker group, on the second of two boxes, against the oracle cell by
    cell; the same call's P(k) equals the plain batch's bit for bit."""
    npd = np.float64 if dtype == "f64" else np.float32
    specs = [(16, 24.0, 8.0, 4), (16, 32.0, 9.0, 5)]
    walkers = [(30.0, 15.0, 5e4), (12.0, 8.0, 2e5), (80.0, 19.0, 1.2e4), (45.0, 6.0, 3e4), (9.0, 14.0, 7e4),
               (0.7, 10.0, 2e4)]
    run = eh.EmuRun(storage=dtype, max_walkers=4, phys={"pk_amp": AMP})
    boxes = []
    for i, (n, box, z, nb) in enumerate(specs):
        d = synth.make_box(n, box, z, seed=70 + i, amp=AMP, dtype=npd)
        boxes.append(d)
        run.box(d, box, z, nb)
    for w in walkers:
        run.walker(*w)
    run.cmd("prepare")
    run.cmd("batch 5")
    run.cmd("batch_fields 5 4 1")     # walker 4 = second slot of the second group of 4
    run.run()
    pk = run.read("batch_pk.bin", np.float64)
    np.testing.assert_array_equal(run.read("batchf_pk.bin", np.float64), pk)
    np.testing.assert_array_equal(run.read("batchf_xhi.bin", np.float64), run.read("batch_xhi.bin", np.float64))
    n, box, z, nb = specs[1]
    w = walkers[4]
    ev = oracle.evaluate(boxes[1], box, z, w, oracle.walker_radii(oracle.shared_radii(n, box, PHYS), w[1]), nb, PHYS)
    x = run.read("batchf_fx.bin", npd, (n, n, n)).astype(np.float64)
    d = run.read("batchf_fd.bin", npd, (n, n, n)).astype(np.float64)
    assert np.array_equal(x == 0, ev.flagged)
    same = (x == 0) == ev.flagged
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert np.abs(x - ev.x_hi)[same].max() <= tol
    assert np.abs(d - ev.dtb)[same].max() <= tol * np.abs(ev.dtb).max()


def test_emu_erfc_f32():
    """The FP32 erfc of the ionisation pass (Numerical Recipes' Chebyshev fit,
    fractional error < 1.2e-7) against math.erfc at the same float inputs, over
    [-3, 8] and densely over [0, 4], where the partial ionisation evaluates it.
    Besides the fit's own error, single precision rounds the exponent
    -z^2 + P(t) once (relative error of the result up to about (z^2 + 2) ulp),
    and t, P and the product a few times; the bound allows 1.2e-7 plus
    (2 z^2 + 8) units of 2^-24."""
    import math
    xs = np.concatenate([np.linspace(-3.0, 8.0, 4001), np.linspace(0.0, 4.0, 4001)]).astype(np.float32)
    run = eh.EmuRun(storage="f32", max_walkers=1, phys={"pk_amp": AMP})
    path = run.write_array("erfc_x.bin", xs)
    run.cmd(f"erfc {path} {xs.size}")
    run.run()
    y = run.read("erfc.bin", np.float32).astype(np.float64)
    ref = np.array([math.erfc(float(v)) for v in xs])
    z = np.abs(xs.astype(np.float64))
    rel = np.abs(y / ref - 1.0)
    bound = 1.2e-7 + (2.0 * z * z + 8.0) * 2.0 ** -24
    worst = int(np.argmax(rel / bound))
    assert np.all(rel <= bound), f"x = {xs[worst]}: relative error {rel[worst]:.3e} > {bound[worst]:.3e}"


def test_emu_launch_shapes_and_autotune_cache(tmp_path):
    """Explicit launch shapes (per-walker flag test, small ionisation grid, walker
    groups of 3, other pass grids) give the default shapes' results: P(k) up to
    the order of FP64 sums, mean x_HI up to the FP32 first level of its sums
    (the two flag tests run different ionisation kernels, which group the
    cells of a partial sum differently: relative error of each at most 4
    units of FP32 rounding); the autotuner writes its choice to a JSON cache under the
    device / size / dtype / ladder / group key and a second context reads it back
    without timing (the emulation's event timer reads 0 ms, so the defaults win)."""
    import json
    specs = [(16, 32.0, 9.0, 5)]
    walkers = [(30.0, 15.0, 5e4), (12.0, 8.0, 2e5), (80.0, 19.0, 1.2e4), (45.0, 6.0, 3e4), (0.7, 10.0, 2e4)]
    cache = str(tmp_path / "tune.json")
    run = eh.EmuRun(storage="f32", max_walkers=8, phys={"pk_amp": AMP})
    d = synth.make_box(16, 32.0, 9.0, seed=80, amp=AMP, dtype=np.float32)
    run.box(d, 32.0, 9.0, 5)
    for w in walkers:
        run.walker(*w)
    run.cmd("prepare")
    run.cmd("batch 5 a")
    run.cmd("tuning 16 2 1 1 0 3")
    run.cmd("batch 5 b")
    run.cmd(f"autotune 1 {cache} 1")
    run.run()
    pa = run.read("batcha_pk.bin", np.float64)
    pb = run.read("batchb_pk.bin", np.float64)
    np.testing.assert_allclose(pb, pa, rtol=1e-12, atol=0)
    np.testing.assert_allclose(run.read("batchb_xhi.bin", np.float64), run.read("batcha_xhi.bin", np.float64),
                               rtol=8 * 2.0 ** -24)
    t1 = run.read("tune1.bin", np.int32)
    assert t1[5] == 0 and t1[3] == 1 and t1[4] == 8   # timed; sorted flag test; groups up to max_walkers
    entries = json.load(open(cache))
    (key, val), = entries.items()
    assert key == "emu|n=16|f32|f32|nr=%d|g=5" % len(oracle.shared_radii(16, 32.0, PHYS))
    assert [val[k] for k in ("ion_blocks", "pipe_blocks", "bins_blocks", "flag_test", "group")] == list(t1[:5])
    run2 = eh.EmuRun(storage="f32", max_walkers=8, phys={"pk_amp": AMP})
    run2.box(d, 32.0, 9.0, 5)
    for w in walkers:
        run2.walker(*w)
    run2.cmd("prepare")
    run2.cmd(f"autotune 1 {cache} 2")
    run2.run()
    t2 = run2.read("tune2.bin", np.int32)
    assert t2[5] == 1 and list(t2[:5]) == list(t1[:5])
