"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances: flipped-cell fraction <= 1e-4 and per-bin P(k) relative error
<= 1e-3 for the FP32 path; the FP64 path is held to 1e-9.  Integer outputs
(bin counts) must match exactly.  Every input is seeded and synthetic.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

AMP = synth.reference_amplitude()
PHYS = oracle.Physics(pk_amp=AMP)


@pytest.fixture(scope="module")
def xs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1501_06576_amd as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1501_06576_amd import build
        build.build()
    mod.library()
    return mod


def _ctx(xs, **phys):
    return xs.Context(0, phys=xs.physics(pk_amp=AMP, **phys))


# Full-size oracle evaluations, started in worker processes when the module's
# first test runs so that they overlap the GPU tests before the ones that use
# them: (workload, sampled walker indices, boxes with per-cell fields).
B256_SAMPLE = (3, 11, 17, 26, 33, 40, 52, 63)
B256_FIELDS = ((40, 1), (17, 0))            # (walker, box) checked cell by cell
UNEVEN_SAMPLE = (2, 77, 130, 201)
UNEVEN_FIELDS = ((77, 4), (201, 0))


def _large_walker():
    """The 512^3 check's walker: the one of the first 64-walker launch (not at its ends)
    with the fewest radii, which keeps the 512^3 oracle to tens of seconds."""
    w = synth.draw_walkers(64, synth.WALKER_SEEDS["large-512"])
    return 1 + int(np.argmin(w[1:63, 1])), w


@pytest.fixture(scope="module", autouse=True)
def ojobs(request):
    names = {it.name.split("[")[0] for it in request.session.items}
    wanted = {"test_batched_256_full_size", "test_uneven_bf16_storage", "test_large_512_box"} & names
    try:
        import torch
        gpu = torch.cuda.is_available()
    except ImportError:
        gpu = False
    if not wanted or not gpu:
        yield {}
        return
    import oracle_jobs
    ex = oracle_jobs.pool()
    jobs = {}
    kw = {"pk_amp": AMP}
    if "test_large_512_box" in wanted:
        i, w = _large_walker()
        radii = oracle.walker_radii(oracle.shared_radii(512, 400.0, PHYS), w[i][1])
        jobs["large"] = oracle_jobs.submit(ex, "large-512", AMP, 1, w[i], radii, kw, fields=True)
    if "test_batched_256_full_size" in wanted:
        ws = synth.workload_walkers(synth.WORKLOADS["batched-256"])
        shared = oracle.shared_radii(256, 250.0, PHYS)
        for i in B256_SAMPLE:
            for bi in range(3):
                f = (i, bi) in B256_FIELDS
                jobs[("b256", i, bi)] = oracle_jobs.submit(ex, "batched-256", AMP, bi, ws[i],
                                                           oracle.walker_radii(shared, ws[i][1]), kw, fields=f)
    if "test_uneven_bf16_storage" in wanted:
        wl = synth.WORKLOADS["uneven-mix"]
        ws = synth.workload_walkers(wl)
        for bi, sp in enumerate(wl.boxes):
            shared = oracle.shared_radii(sp.n, sp.box_mpc, PHYS)
            for i in UNEVEN_SAMPLE:
                f = (i, bi) in UNEVEN_FIELDS
                jobs[("uneven", i, bi)] = oracle_jobs.submit(ex, "uneven-mix", AMP, bi, ws[i],
                                                             oracle.walker_radii(shared, ws[i][1]), kw, fields=f)
    yield jobs
    ex.shutdown(wait=True, cancel_futures=True)


def report(tag, x_gpu, ev, pk_gpu, xm_gpu):
    flips = float(np.mean((np.asarray(x_gpu) == 0) != ev.flagged)) if x_gpu is not None else 0.0
    ok = ev.counts > 0
    rel = np.abs(pk_gpu[ok] / ev.pk[ok] - 1.0)
    line = (f"[{tag}] flips={flips:.2e} pk_rel_max={rel.max():.2e} xhi_mean gpu={xm_gpu:.8f} "
            f"orc={ev.xhi_mean:.8f}")
    if x_gpu is not None:
        same = (np.asarray(x_gpu) == 0) == ev.flagged
        line += f" max|dx_HI|={np.abs(np.asarray(x_gpu, dtype=np.float64) - ev.x_hi)[same].max():.2e}"
    print(line, flush=True)
    return flips, rel.max()


# ------------------------------------------------------------------ plain path

def test_plain_f64_64(xs):
    """64^3, 128 Mpc, z = 9, FP64 on both sides."""
    n, box, z, nb = 64, 128.0, 9.0, 12
    w = (30.0, 15.0, 5e4)
    d = synth.make_box(n, box, z, seed=synth.BOX_SEEDS[(64, 128.0)], amp=AMP, dtype=np.float64)
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare("f64", max_walkers=1, max_plain_radii=30)
    radii = oracle.plain_radii(w[1], n, box, PHYS)
    out = ctx.eval(b, w, radii=radii)
    ev = oracle.evaluate(d, box, z, w, radii, nb, PHYS)
    flips, rel = report("plain-f64-64", out["x_hi"], ev, out["pk"], out["xhi_mean"])
    assert flips == 0.0
    assert rel <= 1e-9
    same = (out["x_hi"] == 0) == ev.flagged
    assert np.abs(out["x_hi"] - ev.x_hi)[same].max() <= 1e-10
    assert np.abs(out["dtb"] - ev.dtb)[same].max() <= 1e-8
    assert abs(out["xhi_mean"] - ev.xhi_mean) <= 1e-10
    np.testing.assert_array_equal(out["counts"], ev.counts)
    np.testing.assert_allclose(out["k_mean"], ev.k_mean, rtol=1e-12)
    # default radius list = the plain ladder from R_mfp
    out2 = ctx.eval(b, w, fields=False)
    np.testing.assert_array_equal(out2["pk"], out["pk"])
    ctx.close()


def test_plain_f32_128_three_redshifts(xs):
    """128^3, 250 Mpc, z = 8, 9, 10, FP32 path, one parameter set."""
    wl = synth.WORKLOADS["plain-f32-128"]
    boxes = synth.workload_boxes(wl, AMP)
    w = wl.walkers[0]
    ctx = _ctx(xs)
    hs = [ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(boxes, wl.boxes)]
    ctx.prepare("f32", max_walkers=1, max_plain_radii=30)
    for h, d, s in zip(hs, boxes, wl.boxes):
        radii = oracle.plain_radii(w[1], s.n, s.box_mpc, PHYS)
        out = ctx.eval(h, w, radii=radii)
        ev = oracle.evaluate(d, s.box_mpc, s.z, w, radii, s.n_bins, PHYS)
        flips, rel = report(f"plain-f32-128 z={s.z}", out["x_hi"], ev, out["pk"], out["xhi_mean"])
        assert flips <= 1e-4
        assert rel <= 1e-3
        assert abs(out["xhi_mean"] - ev.xhi_mean) <= 1e-4
        same = (out["x_hi"] == 0) == ev.flagged
        assert np.abs(out["x_hi"].astype(np.float64) - ev.x_hi)[same].max() <= 2e-5
        assert np.abs(out["dtb"].astype(np.float64) - ev.dtb)[same].max() <= 2e-5 * np.abs(ev.dtb).max()
        np.testing.assert_array_equal(out["counts"], ev.counts)
    ctx.close()


# ------------------------------------------------------------------ batched path

EDGE_WALKERS = [
    (30.0, 15.0, 5e4),      # fiducial-like
    (100.0, 20.0, 1e4),     # nearly fully ionised
    (5.0, 5.0, 1e6),        # nearly neutral
    (0.4, 12.0, 2e4),       # zeta < 1/2: no cell can be flagged
    (60.0, 1.0, 3e4),       # R_mfp below every ladder radius: cell radius only
    (17.3, 7.7, 2.2e5),
    (45.0, 19.9, 1.5e4),
    (8.0, 11.0, 6e5),
    (25.0, 20.0, 8e4),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_small_vs_oracle(xs, dtype):
    """N = 64 (several tiles, ragged walker groups) against the oracle for each walker."""
    n, box, z, nb = 64, 128.0, 8.5, 12
    npd = np.float64 if dtype == "f64" else np.float32
    d = synth.make_box(n, box, z, seed=41, amp=AMP, dtype=npd)
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare(dtype, max_walkers=4, max_plain_radii=30)   # 9 walkers -> 3 chunks, ragged last
    pk, xhi = ctx.eval_batch([b], EDGE_WALKERS)
    pk = pk.cpu().numpy()
    xhi = xhi.cpu().numpy()
    shared = ctx.radii(b)
    assert shared == pytest.approx(oracle.shared_radii(n, box, PHYS), rel=1e-15)
    for i, w in enumerate(EDGE_WALKERS):
        ev = oracle.evaluate(d, box, z, w, oracle.walker_radii(shared, w[1]), nb, PHYS)
        x, _ = ctx.materialize(b, w)
        flips, rel = report(f"batched-{dtype} w{i}", x.cpu().numpy(), ev, pk[i, 0], xhi[i, 0])
        same = (x.cpu().numpy() == 0) == ev.flagged
        dx = np.abs(x.cpu().numpy().astype(np.float64) - ev.x_hi)[same].max()
        if dtype == "f64":
            assert flips == 0.0 and rel <= 1e-9
            assert abs(xhi[i, 0] - ev.xhi_mean) <= 1e-10
            assert dx <= 1e-10
        else:
            assert flips <= 1e-4 and rel <= 1e-3
            assert abs(xhi[i, 0] - ev.xhi_mean) <= 1e-4
            assert dx <= 2e-5
        if w[0] < 0.5:
            assert not (x.cpu().numpy() == 0).any()
    ctx.close()


def test_smoothed_boxes(xs):
    """delta_R for every ladder radius against the oracle's sharp-k smoothing."""
    for dtype, n, box, tol in (("f64", 32, 64.0, 1e-12), ("f32", 64, 128.0, 2e-6)):
        npd = np.float64 if dtype == "f64" else np.float32
        d = synth.make_box(n, box, 9.0, seed=43, amp=AMP, dtype=npd)
        ctx = _ctx(xs)
        b = ctx.add_box(d, box, 9.0, 6)
        ctx.prepare(dtype, max_walkers=1, max_plain_radii=30)
        dh = np.fft.rfftn(d.astype(np.float64))
        scale = float(np.abs(d).max())
        worst = 0.0
        for j, r in enumerate(ctx.radii(b)):
            got = ctx.smoothed(b, j).cpu().numpy().astype(np.float64)
            ref = oracle.smooth(dh, n, box, r)
            worst = max(worst, float(np.abs(got - ref).max()) / scale)
        print(f"[smoothed {dtype} n={n}] max |err| / max|delta| = {worst:.2e}", flush=True)
        assert worst <= tol
        ctx.close()


@pytest.mark.parametrize("dtype,n", [("f64", 32), ("f32", 64), ("f32", 16), ("f64", 256)])
def test_power_spectrum_plane_wave(xs, dtype, n):
    """A single plane wave puts a^2 L^3 / (2 c_b) into its own bin and nothing elsewhere
    (FP64 at 256^3: the binning pass's 16 x 16 plan with FP64 tiles and slots)."""
    import torch
    box, nb, amp = (50.0 if n <= 64 else 250.0), 6, 1.7   # 250 Mpc keeps the 256^3 ladder within 40 radii
    m = (1, 2, 3) if n > 16 else (1, 0, 2)
    g = np.indices((n, n, n))
    f = amp * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)
    npd = np.float64 if dtype == "f64" else np.float32
    ctx = _ctx(xs)
    b = ctx.add_box(np.zeros((n, n, n), dtype=npd), box, 9.0, nb)
    ctx.prepare(dtype, max_walkers=1, max_plain_radii=30)
    pk = ctx.power_spectrum(b, torch.from_numpy(f.astype(npd)).cuda())
    _, counts = ctx.bins(b)
    bi = oracle.bin_of_n2(sum(v * v for v in m), n, nb)
    expect = np.zeros(nb)
    expect[bi] = amp ** 2 * box ** 3 / (2 * counts[bi])
    tol = 1e-10 if dtype == "f64" else 2e-5
    np.testing.assert_allclose(pk, expect, rtol=tol, atol=tol * expect.max())
    ctx.close()


def test_erfc_f32_device(xs):
    """The FP32 erfc of the ionisation pass, on the device (hardware reciprocal and
    exponential), against math.erfc at the same float inputs over [-3, 8] and densely
    over [0, 4]: the fit's 1.2e-7 plus single-precision rounding of the exponent and
    of a few products, at most (2 z^2 + 8) units of 2^-24, as on the CPU build, plus
    2 ulp for the approximate reciprocal and exponential."""
    import math
    import torch
    xv = np.concatenate([np.linspace(-3.0, 8.0, 40001), np.linspace(0.0, 4.0, 40001)]).astype(np.float32)
    ctx = _ctx(xs)
    y = ctx.erfc_f32(torch.from_numpy(xv).cuda()).cpu().numpy().astype(np.float64)
    ctx.close()
    ref = np.array([math.erfc(float(v)) for v in xv])
    z = np.abs(xv.astype(np.float64))
    rel = np.abs(y / ref - 1.0)
    bound = 1.2e-7 + (2.0 * z * z + 10.0) * 2.0 ** -24
    worst = int(np.argmax(rel / bound))
    print(f"[erfc_f32 device] worst relative error {rel[worst]:.3e} at x = {xv[worst]} (bound {bound[worst]:.3e}); "
          f"max over [0, 4]: {rel[z <= 4].max():.3e}", flush=True)
    assert np.all(rel <= bound)


def test_uniform_box(xs):
    """delta = c everywhere: dT_b is uniform, so every bin has zero power."""
    n, box, z = 32, 64.0, 9.0
    d = np.full((n, n, n), 0.25, dtype=np.float32)
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, 5)
    ctx.prepare("f32", max_walkers=4, max_plain_radii=30)
    walkers = [(20.0, 15.0, 3e4), (1e9, 10.0, 1e4), (2.0, 10.0, 1e5)]
    pk, xhi = ctx.eval_batch([b], walkers)
    pk = pk.cpu().numpy()
    assert np.all(np.abs(pk) <= 1e-6 * (27.0 ** 2) * box ** 3 / n ** 3)
    assert xhi.cpu().numpy()[1, 0] == 0.0     # every cell flagged
    ev = oracle.evaluate(d, box, z, walkers[2], oracle.walker_radii(ctx.radii(b), 10.0), 5, PHYS)
    assert xhi.cpu().numpy()[2, 0] == pytest.approx(ev.xhi_mean, abs=1e-6)
    ctx.close()


def test_batched_equals_plain_and_deterministic(xs):
    """A batched walker equals a plain evaluation on the same radius list; reruns are bitwise equal."""
    n, box, z, nb = 64, 128.0, 9.0, 12
    d = synth.make_box(n, box, z, seed=44, amp=AMP, dtype=np.float32)
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare("f32", max_walkers=16, max_plain_radii=30)
    walkers = synth.draw_walkers(16, 7)
    pk1, x1 = ctx.eval_batch([b], walkers)
    pk2, x2 = ctx.eval_batch([b], walkers)
    assert np.array_equal(pk1.cpu().numpy(), pk2.cpu().numpy())
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    shared = ctx.radii(b)
    for i in (0, 5, 11):
        w = walkers[i]
        out = ctx.eval(b, w, radii=oracle.walker_radii(shared, w[1]), fields=False)
        np.testing.assert_allclose(out["pk"], pk1.cpu().numpy()[i, 0], rtol=1e-6)
        assert out["xhi_mean"] == pytest.approx(x1.cpu().numpy()[i, 0], abs=1e-6)
    ctx.close()


def test_monotonicity(xs):
    """x_HI per cell: non-increasing in zeta and R_mfp, non-decreasing in T_vir."""
    n, box, z = 64, 128.0, 9.0
    d = synth.make_box(n, box, z, seed=45, amp=AMP, dtype=np.float32)
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, 8)
    ctx.prepare("f32", max_walkers=4, max_plain_radii=30)
    base = ctx.materialize(b, (20.0, 10.0, 3e4))[0].cpu().numpy()
    assert np.all(ctx.materialize(b, (40.0, 10.0, 3e4))[0].cpu().numpy() <= base)
    assert np.all(ctx.materialize(b, (20.0, 18.0, 3e4))[0].cpu().numpy() <= base)
    assert np.all(ctx.materialize(b, (20.0, 10.0, 1e5))[0].cpu().numpy() >= base)
    ctx.close()


# ------------------------------------------------------------------ full sizes

def _field_check(tag, fx, fd, res, pk_gpu, xm_gpu):
    """Cell-by-cell check of the x_HI / dT_b boxes a batched launch wrote against an oracle
    result from a worker (flags bit-packed, x_HI and dT_b as float32)."""
    import oracle_jobs
    x = fx.cpu().numpy()
    d = fd.cpu().numpy().astype(np.float64)
    flagged = oracle_jobs.unpack_flags(res)
    same = (x == 0) == flagged
    flips = float(np.mean(~same))
    ok = res["counts"] > 0
    rel = float(np.abs(pk_gpu[ok] / res["pk"][ok] - 1.0).max())
    xo = res["x_hi"].astype(np.float64)
    do = res["dtb"].astype(np.float64)
    dx = float(np.abs(x.astype(np.float64) - xo)[same].max())
    dd = float(np.abs(d - do)[same].max() / np.abs(do).max())
    print(f"[{tag}] flips={flips:.2e} pk_rel_max={rel:.2e} xhi_mean gpu={xm_gpu:.8f} orc={res['xhi_mean']:.8f} "
          f"max|dx_HI|={dx:.2e} max|d dT_b|/max|dT_b|={dd:.2e}", flush=True)
    return flips, rel, dx, dd


def test_batched_256_full_size(xs, ojobs):
    """256^3 x 3 z with 64 walkers (the benchmark launch configuration).  P(k) and mean x_HI
    of 8 seeded walkers on all three boxes against the oracle, and the x_HI and dT_b boxes
    that the batched ionisation launch itself computes for two walkers in the middle of the
    group, cell by cell."""
    import torch
    wl = synth.WORKLOADS["batched-256"]
    walkers = synth.workload_walkers(wl)
    boxes = synth.workload_boxes(wl, AMP)
    ctx = _ctx(xs)
    hs = [ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(boxes, wl.boxes)]
    ctx.prepare("f32", max_walkers=64, max_plain_radii=40)
    assert ctx.radii(hs[0]) == pytest.approx(oracle.shared_radii(256, 250.0, PHYS), rel=1e-15)
    pk_t, xhi_t = ctx.eval_batch(hs, walkers)
    pk = pk_t.cpu().numpy()
    xhi = xhi_t.cpu().numpy()
    assert np.isfinite(pk).all() and np.all((xhi >= 0) & (xhi <= 1))
    fields = {}
    for i, bi in B256_FIELDS:
        pkf, xhf, fx, fd = ctx.eval_batch_fields(hs, walkers, i, bi)
        same_pk = bool(np.array_equal(pkf.cpu().numpy(), pk))
        print(f"[batched-256] P(k) of the field-writing launch bitwise equal: {same_pk}", flush=True)
        np.testing.assert_allclose(pkf.cpu().numpy(), pk, rtol=1e-6)
        np.testing.assert_allclose(xhf.cpu().numpy(), xhi, rtol=0, atol=1e-7)
        fields[(i, bi)] = (fx.cpu(), fd.cpu())
        del fx, fd
    counts = [ctx.bins(h)[1] for h in hs]
    ctx.close()
    torch.cuda.synchronize()
    for (i, bi), (fx, fd) in fields.items():
        res = ojobs[("b256", i, bi)].result()
        flips, rel, dx, dd = _field_check(f"batched-256 fields w{i} z={wl.boxes[bi].z:g}", fx, fd, res, pk[i, bi],
                                          xhi[i, bi])
        assert flips <= 1e-4 and rel <= 1e-3 and dx <= 2e-5 and dd <= 2e-5
    worst = 0.0
    for i in B256_SAMPLE:
        for bi in range(3):
            res = ojobs[("b256", i, bi)].result()
            np.testing.assert_array_equal(counts[bi], res["counts"])
            ok = res["counts"] > 0
            rel = float(np.abs(pk[i, bi][ok] / res["pk"][ok] - 1.0).max())
            worst = max(worst, rel)
            assert rel <= 1e-3, f"walker {i} box {bi}: P(k) relative error {rel:.2e}"
            assert abs(xhi[i, bi] - res["xhi_mean"]) <= 1e-4
    print(f"[batched-256] 8 walkers x 3 boxes: worst P(k) relative error {worst:.2e}", flush=True)


def test_uneven_bf16_storage(xs, ojobs):
    """The uneven workload: 128^3/250 Mpc and 256^3/300 Mpc boxes at z = 8, 9, 10, all
    256 walkers in groups of 64, smoothed boxes stored in BF16 (f_coll in FP32, sigma^2
    and bin sums in FP64).  Against the FP64 oracle for 4 walkers on all 6 boxes (P(k)
    per bin, mean x_HI) and cell by cell for 2 of them (fields from the batched launch).
    BF16 rounding moves cells across their thresholds, so this form is held to its own
    bounds, about 3x the largest observed."""
    wl = synth.WORKLOADS["uneven-mix"]
    walkers = synth.workload_walkers(wl)
    boxes = synth.workload_boxes(wl, AMP)
    ctx = _ctx(xs)
    hs = [ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(boxes, wl.boxes)]
    ctx.prepare("bf16", max_walkers=64, max_plain_radii=40)
    pk_t, xhi_t = ctx.eval_batch(hs, walkers)
    pk = pk_t.cpu().numpy()
    xhi = xhi_t.cpu().numpy()
    assert np.isfinite(pk).all() and np.all((xhi >= 0) & (xhi <= 1))
    fields = {}
    for i, bi in UNEVEN_FIELDS:
        _, _, fx, fd = ctx.eval_batch_fields(hs, walkers, i, bi)
        fields[(i, bi)] = (fx.cpu(), fd.cpu())
    ctx.close()
    for (i, bi), (fx, fd) in fields.items():
        res = ojobs[("uneven", i, bi)].result()
        flips, rel, dx, dd = _field_check(f"uneven-bf16 fields w{i} box{bi}", fx, fd, res, pk[i, bi], xhi[i, bi])
        # observed at most 4.5e-4 flipped cells and 2.9e-3 P(k) relative error
        assert flips <= 1.5e-3 and rel <= 1e-2
    print("[uneven-bf16] walker box   n  flips-n/a  pk_rel_max  |dxhi_mean|", flush=True)
    worst_rel, worst_xm = 0.0, 0.0
    for bi, sp in enumerate(wl.boxes):
        for i in UNEVEN_SAMPLE:
            res = ojobs[("uneven", i, bi)].result()
            ok = res["counts"] > 0
            rel = float(np.abs(pk[i, bi][ok] / res["pk"][ok] - 1.0).max())
            dxm = abs(xhi[i, bi] - res["xhi_mean"])
            print(f"[uneven-bf16] w{i:<4d} box{bi} {sp.n:4d}^3/{sp.box_mpc:g} z={sp.z:g}  pk_rel_max={rel:.2e} "
                  f"|dxhi_mean|={dxm:.2e}", flush=True)
            worst_rel, worst_xm = max(worst_rel, rel), max(worst_xm, dxm)
    print(f"[uneven-bf16] 4 walkers x 6 boxes: worst P(k) rel {worst_rel:.2e}, worst |dx_HI mean| {worst_xm:.2e}",
          flush=True)
    # observed at most 3.5e-3 and 2.5e-4
    assert worst_rel <= 1e-2 and worst_xm <= 8e-4


def test_large_512_box(xs, ojobs):
    """512^3, 400 Mpc (the large workload's geometry): grid limits and FFT length 512.

    Checks a plane wave through the estimator (closed form), one smoothed box
    against the oracle, batched == plain on a sampled walker, and a walker
    group of 64 on one z = 9 box with one walker from the middle of that launch
    against the oracle cell by cell and bin by bin.  The full 1024-walker x
    3-box run is a benchmark case.
    """
    import torch
    n, box, z, nb = 512, 400.0, 9.0, 15
    d = synth.make_box(n, box, z, seed=synth.BOX_SEEDS[(512, 400.0)], amp=AMP, dtype=np.float32)
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare("f32", max_walkers=64, max_plain_radii=40)
    # plane wave: closed-form P in one bin
    g = np.indices((n, n, n), dtype=np.float32)
    m = (3, -5, 7)
    f = (1.3 * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n)).astype(np.float32)
    del g
    pk = ctx.power_spectrum(b, torch.from_numpy(f).cuda())
    _, counts = ctx.bins(b)
    bi = oracle.bin_of_n2(sum(v * v for v in m), n, nb)
    expect = np.zeros(nb)
    expect[bi] = 1.3 ** 2 * box ** 3 / (2 * counts[bi])
    np.testing.assert_allclose(pk, expect, rtol=2e-5, atol=2e-5 * expect.max())
    del f
    # one smoothed box (R = 5 Mpc neighbourhood of the ladder) against the oracle
    radii = ctx.radii(b)
    j = min(range(len(radii)), key=lambda i: abs(radii[i] - 5.0))
    got = ctx.smoothed(b, j).cpu().numpy().astype(np.float64)
    ref = oracle.smooth(np.fft.rfftn(d.astype(np.float64)), n, box, radii[j])
    err = float(np.abs(got - ref).max() / np.abs(d).max())
    print(f"[large-512] smoothed R={radii[j]:.3f}: max err / max|delta| = {err:.2e}", flush=True)
    assert err <= 2e-6
    del got, ref
    walkers = synth.draw_walkers(64, synth.WALKER_SEEDS["large-512"])
    pk, xhi = ctx.eval_batch([b], walkers)
    pk = pk.cpu().numpy()
    xhi = xhi.cpu().numpy()
    assert np.isfinite(pk).all() and np.all((xhi >= 0) & (xhi <= 1))
    w = walkers[5]
    out = ctx.eval(b, w, radii=oracle.walker_radii(radii, w[1]), fields=False)
    np.testing.assert_allclose(out["pk"], pk[5, 0], rtol=1e-6)
    assert out["xhi_mean"] == pytest.approx(xhi[5, 0], abs=1e-6)
    # a walker in the middle of the 64-walker launch (1024-thread ionisation blocks,
    # 8.8.8 radix plan) against the oracle: fields of the batched launch cell by cell
    i, ws = _large_walker()
    assert np.array_equal(ws, walkers)
    _, _, fx, fd = ctx.eval_batch_fields([b], walkers, i, 0)
    fx, fd = fx.cpu(), fd.cpu()
    ctx.close()
    del out
    torch.cuda.synchronize()
    res = ojobs["large"].result()
    flips, rel, dx, dd = _field_check(f"large-512 fields w{i} ({len(oracle.walker_radii(radii, walkers[i][1]))} "
                                      "radii)", fx, fd, res, pk[i, 0], xhi[i, 0])
    assert flips <= 1e-4 and rel <= 1e-3 and dx <= 2e-5 and dd <= 2e-5
    assert abs(xhi[i, 0] - res["xhi_mean"]) <= 1e-4


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_chi2_epilogue(xs, dtype):
    """chi^2 over two redshifts against a mock (the fiducial walker's oracle
    Delta^2), noise on one box: the epilogue on the library's own P(k) to FP64
    round-off, and end to end within the bound that the P(k) tolerance implies."""
    n, box, nb = 64, 128.0, 12
    npd = np.float64 if dtype == "f64" else np.float32
    ptol = 1e-9 if dtype == "f64" else 1e-3
    zs = (8.5, 9.5)
    ctx = _ctx(xs)
    boxes, hs, mocks, noises = [], [], [], []
    for i, z in enumerate(zs):
        d = synth.make_box(n, box, z, seed=47, amp=AMP, dtype=npd)
        boxes.append(d)
        hs.append(ctx.add_box(d, box, z, nb))
    ctx.prepare(dtype, max_walkers=4, max_plain_radii=30)
    shared = ctx.radii(hs[0])
    for i, z in enumerate(zs):
        fid = oracle.evaluate(boxes[i], box, z, (30.0, 15.0, 5e4), oracle.walker_radii(shared, 15.0), nb, PHYS)
        mocks.append(fid.delta2)
        noises.append(np.linspace(1.0, 3.0, nb) if i == 0 else np.zeros(nb))
        ctx.set_mock(hs[i], fid.delta2, noises[i] if i == 0 else None)
    pk_t, _ = ctx.eval_batch(hs, EDGE_WALKERS)
    got = ctx.chi2(hs, pk_t).cpu().numpy()
    pk = pk_t.cpu().numpy()
    for wi, w in enumerate(EDGE_WALKERS):
        own, ref, bound, scale = 0.0, 0.0, 0.0, 0.0
        for i, z in enumerate(zs):
            ev = oracle.evaluate(boxes[i], box, z, w, oracle.walker_radii(shared, w[1]), nb, PHYS)
            use = oracle.likelihood.likelihood_bins(ev.k_mean, ev.counts)
            var = oracle.likelihood.bin_variance(mocks[i], noises[i])
            d2_own = ev.k_mean ** 3 * pk[wi, i, :nb] / (2 * math.pi ** 2)
            own += oracle.likelihood.chi2(d2_own, mocks[i], noises[i], ev.k_mean, ev.counts)
            ref += oracle.likelihood.chi2(ev.delta2, mocks[i], noises[i], ev.k_mean, ev.counts)
            scale += oracle.likelihood.chi2(np.zeros(nb), mocks[i], noises[i], ev.k_mean, ev.counts)
            ok = use & (var > 0)
            r = np.abs(ev.delta2 - mocks[i])[ok]
            dd = ptol * np.abs(ev.delta2)[ok]
            bound += float(np.sum((2 * r * dd + dd * dd) / var[ok]))
        print(f"[chi2-{dtype} w{wi}] gpu={got[wi]:.6e} oracle={ref:.6e} bound={bound:.2e}", flush=True)
        assert got[wi] == pytest.approx(own, rel=1e-12, abs=1e-14 * scale)
        assert abs(got[wi] - ref) <= bound * 1.01 + 1e-12 * scale
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_velocity_factor(xs, dtype):
    """dT_b with the velocity-gradient factor H / (dv_r/dr + H) of eq. (4):
    batched walkers and the plain form against the oracle with velocities."""
    n, box, z, nb = 64, 128.0, 8.0, 12
    npd = np.float64 if dtype == "f64" else np.float32
    d = synth.make_box(n, box, z, seed=53, amp=AMP, dtype=npd)
    phys = oracle.Physics(pk_amp=AMP, velocity=True, dvdr_max=0.2)
    ctx = _ctx(xs, velocity=1, dvdr_max=0.2)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare(dtype, max_walkers=4, max_plain_radii=30)
    walkers = EDGE_WALKERS[:5]
    pk, xhi = ctx.eval_batch([b], walkers)
    pk = pk.cpu().numpy()
    shared = ctx.radii(b)
    plain_off = oracle.evaluate(d, box, z, walkers[0], oracle.walker_radii(shared, walkers[0][1]), nb,
                                oracle.Physics(pk_amp=AMP))
    for i, w in enumerate(walkers):
        ev = oracle.evaluate(d, box, z, w, oracle.walker_radii(shared, w[1]), nb, phys)
        flips, rel = report(f"velocity-{dtype} w{i}", None, ev, pk[i, 0], float(xhi[i, 0]))
        assert rel <= (1e-9 if dtype == "f64" else 1e-3)
        if i == 0:
            # the factor matters: P(k) moves well beyond the tolerance without it
            assert np.abs(ev.pk / plain_off.pk - 1.0)[ev.counts > 0].max() > 1e-2
    out = ctx.eval(b, walkers[0])
    ev = oracle.evaluate(d, box, z, walkers[0], oracle.plain_radii(walkers[0][1], n, box, phys), nb, phys)
    same = (out["x_hi"] == 0) == ev.flagged
    tol = 1e-8 if dtype == "f64" else 2e-3
    assert np.abs(out["dtb"] - ev.dtb)[same].max() <= tol * np.abs(ev.dtb).max()
    ctx.close()


def test_velocity_256_full_size(xs):
    """The velocity-gradient factor at 256^3 x 3 z with 64 walkers (the launch
    configuration the benchmark times for it); one sampled walker on the z = 8
    box checked cell by cell and bin by bin against the oracle with velocities."""
    import torch
    wl = synth.WORKLOADS["batched-256"]
    boxes = synth.workload_boxes(wl, AMP)
    walkers = synth.workload_walkers(wl)
    phys = oracle.Physics(pk_amp=AMP, velocity=True, dvdr_max=0.2)
    ctx = _ctx(xs, velocity=1, dvdr_max=0.2)
    hs = [ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(boxes, wl.boxes)]
    ctx.prepare("f32", max_walkers=64, max_plain_radii=40)
    pk, xhi = ctx.eval_batch(hs, walkers)
    pk = pk.cpu().numpy()
    xhi = xhi.cpu().numpy()
    assert np.isfinite(pk).all() and np.all((xhi >= 0) & (xhi <= 1))
    s0 = wl.boxes[0]
    shared = ctx.radii(hs[0])
    i = 11
    w = walkers[i]
    ev = oracle.evaluate(boxes[0], s0.box_mpc, s0.z, w, oracle.walker_radii(shared, w[1]), s0.n_bins, phys)
    x, _ = ctx.materialize(hs[0], w)
    flips, rel = report(f"velocity-256 w{i} z={s0.z:g}", x.cpu().numpy(), ev, pk[i, 0], xhi[i, 0])
    assert flips <= 1e-4 and rel <= 1e-3
    assert abs(xhi[i, 0] - ev.xhi_mean) <= 1e-4
    ctx.close()
    torch.cuda.synchronize()


# ------------------------------------------------------------------ two-population efficiency (eq. 9)

EDGE2 = [(70.0, 15.0, 10 ** 4.7, 4.0 / 3.0, -1.0 / 3.0),   # the fiducial of Section 4
         (30.0, 15.0, 1e5, 10.0 / 3.0, -4.0 / 3.0),        # bounded flag intervals
         (12.0, 8.0, 3e4, -4.0 / 3.0, 2.0),
         (25.0, 10.0, 2e5, 0.0, 0.0),                      # constant efficiency above 1e4 K
         (0.4, 12.0, 2e4, 1.0, 0.0),                       # F < 1 everywhere
         (200.0, 3.0, 1e6, 2.0, 3.0),
         (60.0, 0.5, 3e4, 1.0, -1.0)]                      # R_mfp below every ladder radius
_ORACLE2 = {}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_population_vs_oracle(xs, dtype):
    """32^3, 64 Mpc, z = 8.5: every edge walker against the oracle (chunks of 3, ragged)."""
    n, box, z, nb = 32, 64.0, 8.5, 6
    d32 = synth.make_box(n, box, z, seed=43, amp=AMP, dtype=np.float32)   # same values for both dtypes
    d = d32.astype(np.float64) if dtype == "f64" else d32
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare(dtype, max_walkers=3, max_plain_radii=30)
    pk, xhi = ctx.eval_batch2([b], EDGE2)
    pk = pk.cpu().numpy()
    xhi = xhi.cpu().numpy()
    shared = ctx.radii(b)
    for i, w in enumerate(EDGE2):
        if i not in _ORACLE2:
            _ORACLE2[i] = oracle.two_population.evaluate(d32.astype(np.float64), box, z, w,
                                                         oracle.walker_radii(shared, w[1]), nb, PHYS)
        ev = _ORACLE2[i]
        x, _ = ctx.materialize2(b, w)
        x = x.cpu().numpy()
        flips, rel = report(f"two-pop-{dtype} w{i}", x, ev, pk[i, 0], xhi[i, 0])
        same = (x == 0) == ev.flagged
        if dtype == "f64":
            # quadrature and table interpolation: x_HI within 2e-7
            assert flips == 0.0 and rel <= 1e-6
            assert np.abs(x - ev.x_hi)[same].max() <= 2e-7
            assert abs(xhi[i, 0] - ev.xhi_mean) <= 2e-7
        else:
            assert flips <= 1e-4 and rel <= 1e-3
            assert np.abs(x - ev.x_hi)[same].max() <= 2e-5
            assert abs(xhi[i, 0] - ev.xhi_mean) <= 1e-4
    ctx.close()


# Walkers whose flag intervals are narrow enough that some cells of the 32^3
# box below skip over them between radii: at those cells only the upper ends
# of the intervals keep the cell unflagged (at least 181 and 263 cells by the
# oracle's per-radius fractions).
NARROW2 = [(15.0, 15.0, 1e5, 10.0 / 3.0, -4.0 / 3.0), (20.0, 15.0, 3e5, 10.0 / 3.0, -10.0 / 3.0)]


def test_two_population_sorted_equals_per_walker(xs):
    """FP32 two-population walkers: the sorted interval test of the team ionisation pass
    (lower ends, and upper ends raised to the next float, two searches per radius slot;
    flag_test 1) flags exactly the cells the per-walker compares flag (flag_test 0):
    the mean x_HI agrees to summation order (one flipped cell of 32^3 would move it by
    3e-5) and P(k) to FP32 rounding, for every edge walker and two walkers whose upper
    interval ends decide cells; those two also against the oracle."""
    n, box, z, nb = 32, 64.0, 8.5, 6
    d = synth.make_box(n, box, z, seed=43, amp=AMP, dtype=np.float32)
    walkers = EDGE2 + NARROW2
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare("f32", max_walkers=len(walkers), max_plain_radii=30)
    ctx.set_tuning(n, flag_test=1)
    pk1, x1 = ctx.eval_batch2([b], walkers)
    ctx.set_tuning(n, flag_test=0)
    pk0, x0 = ctx.eval_batch2([b], walkers)
    ctx.set_tuning(n)
    pk1, x1, pk0, x0 = (t.cpu().numpy() for t in (pk1, x1, pk0, x0))
    print(f"[two-pop sorted vs per-walker] max |dx_HI mean| = {np.abs(x1 - x0).max():.2e}, "
          f"max P(k) rel = {np.max(np.abs(pk1 - pk0) / np.maximum(np.abs(pk0), 1e-30)):.2e}", flush=True)
    np.testing.assert_allclose(x1, x0, rtol=0, atol=1e-7)
    np.testing.assert_allclose(pk1, pk0, rtol=1e-5, atol=1e-5 * np.abs(pk0).max())
    shared = ctx.radii(b)
    for i, w in enumerate(NARROW2):
        wi = len(EDGE2) + i
        ev = oracle.two_population.evaluate(d.astype(np.float64), box, z, w, oracle.walker_radii(shared, w[1]),
                                            nb, PHYS)
        x, _ = ctx.materialize2(b, w)
        flips, rel = report(f"two-pop-narrow w{i}", x.cpu().numpy(), ev, pk1[wi, 0], x1[wi, 0])
        assert flips <= 1e-4 and rel <= 1e-3
        assert abs(x1[wi, 0] - ev.xhi_mean) <= 1e-4
    ctx.close()


def test_two_population_256_sampled(xs):
    """The benchmark geometry (256^3 x 3 z, 64 walkers per launch) with drawn two-population
    walkers: flags and x_HI of sampled cells against the oracle cell by cell, and the
    returned P(k) and mean x_HI against the estimator applied to the materialised field."""
    wl = synth.WORKLOADS["batched-256"]
    boxes = synth.workload_boxes(wl, AMP)
    walkers = synth.draw_walkers2(64, synth.WALKER_SEEDS["two-population-256"])
    ctx = _ctx(xs)
    hs = [ctx.add_box(dd, s.box_mpc, s.z, s.n_bins) for dd, s in zip(boxes, wl.boxes)]
    ctx.prepare("f32", max_walkers=64, max_plain_radii=40)
    pk, xhi = ctx.eval_batch2(hs, walkers)
    pk = pk.cpu().numpy()
    xhi = xhi.cpu().numpy()
    assert np.isfinite(pk).all() and np.all((xhi >= 0) & (xhi <= 1))
    n, box, z = 256, 250.0, 9.0
    shared = ctx.radii(hs[1])
    dh = np.fft.rfftn(boxes[1].astype(np.float64))
    rng = np.random.default_rng(9)
    cells = rng.integers(0, n, size=(20000, 3))
    sampled = {}   # delta_R at the sampled cells, one smoothing per ladder radius
    for r in shared:
        sampled[r] = oracle.smooth(dh, n, box, r)[cells[:, 0], cells[:, 1], cells[:, 2]]
    del dh
    for i in (7, 29):
        w = tuple(float(v) for v in walkers[i])
        flag = np.zeros(len(cells), dtype=bool)
        f_cell = None
        for r in oracle.walker_radii(shared, w[1]):
            f = oracle.two_population.ionizing_fraction(sampled[r], r, z, w, PHYS)
            flag |= f >= 1.0
            f_cell = f
        x_ref = np.where(flag, 0.0, 1.0 - f_cell)
        x, t = ctx.materialize2(hs[1], w)
        x = x.cpu().numpy()
        xs_ = x[cells[:, 0], cells[:, 1], cells[:, 2]].astype(np.float64)
        same = (xs_ == 0) == flag
        print(f"[two-pop-256 w{i}] sampled flips={np.mean(~same):.2e} "
              f"max|dx_HI|={np.abs(xs_ - x_ref)[same].max():.2e}", flush=True)
        assert np.mean(~same) <= 1e-4
        assert np.abs(xs_ - x_ref)[same].max() <= 2e-5
        p_ref = oracle.power_spectrum(t.cpu().numpy(), box, 15)[0]
        np.testing.assert_allclose(pk[i, 1], p_ref, rtol=2e-4)
        assert abs(xhi[i, 1] - float(np.mean(x, dtype=np.float64))) <= 1e-5
    ctx.close()


# ------------------------------------------------------------------ ensemble sampler (Section 2.3)

def _oracle_chain(box_data, specs, mocks, dim, lo, hi, x0, u):
    def loglike(p):
        tot = 0.0
        for d, (n, box, z, nb), mock in zip(box_data, specs, mocks):
            radii = oracle.walker_radii(oracle.shared_radii(n, box, PHYS), p[1])
            if dim == 3:
                ev = oracle.evaluate(d, box, z, (p[0], p[1], 10 ** p[2]), radii, nb, PHYS)
            else:
                ev = oracle.two_population.evaluate(d, box, z, (p[0], p[1], 10 ** p[2], p[3], p[4]), radii, nb,
                                                    PHYS)
            tot += oracle.likelihood.chi2(ev.delta2, mock, np.zeros(nb), ev.k_mean, ev.counts)
        return -0.5 * tot
    lp_fn = oracle.sampler.box_prior(lo, hi, loglike)
    x = x0.copy()
    lp = np.array([lp_fn(v) for v in x])
    xs, lps, accs = [x.copy()], [lp.copy()], []
    for t in range(u.shape[0]):
        accs.append(oracle.sampler.step(x, lp, u[t], lp_fn))
        xs.append(x.copy())
        lps.append(lp.copy())
    return np.array(xs), np.array(lps), np.array(accs)


PRIOR3 = ([5.0, 5.0, 4.0], [100.0, 20.0, 5.3])
PRIOR5 = ([5.0, 5.0, 4.0, -4 / 3, -4 / 3], [100.0, 20.0, 5.3, 10 / 3, 10 / 3])


@pytest.mark.parametrize("dim", [3, 5])
def test_mcmc_chain_vs_oracle(xs, dim):
    """FP64: a few ensemble steps through the C-ABI against the oracle sampler with the
    same uniforms (walker chunks of 3, ragged halves): identical moves, same chain."""
    import torch
    if dim == 3:
        specs = [(32, 64.0, 9.0, 6), (16, 32.0, 8.0, 4)]
        fid, nw, steps = (30.0, 15.0, np.log10(5e4)), 8, 3
        lo, hi = PRIOR3
    else:
        specs = [(16, 32.0, 10.0, 4)]   # the fiducial leaves x_HI ~ 0.5 here
        fid, nw, steps = (70.0, 15.0, 4.7, 4 / 3, -1 / 3), 6, 2
        lo, hi = PRIOR5
    ctx = _ctx(xs)
    data, mocks, hs = [], [], []
    for i, (n, box, z, nb) in enumerate(specs):
        d = synth.make_box(n, box, z, seed=95 + i, amp=AMP, dtype=np.float64)
        data.append(d)
        hs.append(ctx.add_box(d, box, z, nb))
    ctx.prepare("f64", max_walkers=3, max_plain_radii=30)
    for h, d, (n, box, z, nb) in zip(hs, data, specs):
        radii = oracle.walker_radii(oracle.shared_radii(n, box, PHYS), fid[1])
        if dim == 3:
            ev = oracle.evaluate(d, box, z, (fid[0], fid[1], 10 ** fid[2]), radii, nb, PHYS)
        else:
            ev = oracle.two_population.evaluate(d, box, z, (fid[0], fid[1], 10 ** fid[2], fid[3], fid[4]), radii, nb,
                                                PHYS)
        mocks.append(ev.delta2)
        ctx.set_mock(h, ev.delta2)
    # walkers around the fiducial (within 10 % of the prior range), inside the prior
    x0 = np.asarray(fid) + (np.asarray(hi) - np.asarray(lo)) * 0.1 * (synth.uniforms((nw, dim), 210 + dim) - 0.5)
    u = synth.uniforms((steps, 2, nw // 2, 3), 310 + dim)
    spec = xs.sampler(lo, hi)
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    lp = ctx.mcmc_lnprob(hs, spec, x)
    acc = torch.zeros(nw, dtype=torch.int32, device="cuda")
    gx, glp, gacc = [x.cpu().numpy().copy()], [lp.cpu().numpy().copy()], []
    for t in range(steps):
        ctx.mcmc_step(hs, spec, x, lp, torch.tensor(u[t], dtype=torch.float64, device="cuda"), acc)
        gx.append(x.cpu().numpy().copy())
        glp.append(lp.cpu().numpy().copy())
        gacc.append(acc.cpu().numpy().astype(bool))
    ox, olp, oacc = _oracle_chain(data, specs, mocks, dim, lo, hi, x0, u)
    assert np.ptp(olp[0]) > 0.1   # a likelihood that tells the walkers apart
    print(f"[mcmc dim={dim}] accepted {int(np.sum(gacc))}/{nw * steps}; max |dlp| = "
          f"{np.max(np.abs(np.array(glp) - olp)):.2e}", flush=True)
    np.testing.assert_array_equal(np.array(gacc), oacc)
    np.testing.assert_allclose(np.array(gx), ox, rtol=1e-12)
    # ln p to FP64 round-off (3 parameters) or to the two-population table's interpolation
    np.testing.assert_allclose(np.array(glp), olp, rtol=1e-9 if dim == 3 else 1e-5, atol=0 if dim == 3 else 1e-6)
    ctx.close()


@pytest.mark.parametrize("dim", [3, 5])
def test_mcmc_256_consistency(xs, dim):
    """The benchmark geometry (256^3 x 3 z, FP32), 128 walkers of the constant-efficiency
    (dim 3) or two-population (dim 5) model drawn over the prior: device-planned ln p equals
    -chi^2/2 of the host-planned batch; after steps, walkers that did not move keep x and
    ln p, and every ln p equals a fresh evaluation of its walker."""
    import torch
    wl = synth.WORKLOADS["batched-256"]
    boxes = synth.workload_boxes(wl, AMP)
    ctx = _ctx(xs)
    hs = [ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(boxes, wl.boxes)]
    ctx.prepare("f32", max_walkers=64, max_plain_radii=40)
    fid = (30.0, 15.0, 5e4)
    fpk, _ = ctx.eval_batch(hs, [fid])
    fpk = fpk.cpu().numpy()
    for i, h in enumerate(hs):
        km, _ = ctx.bins(h)
        ctx.set_mock(h, km ** 3 * fpk[0, i, :len(km)] / (2 * np.pi ** 2))
    lo, hi = PRIOR3 if dim == 3 else PRIOR5
    nw = 128
    x0 = np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * synth.uniforms((nw, dim), 220 if dim == 3 else 221)
    spec = xs.sampler(lo, hi)
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    lp = ctx.mcmc_lnprob(hs, spec, x)
    walkers = np.column_stack([x0[:, 0], x0[:, 1], 10 ** x0[:, 2], *x0[:, 3:].T])
    pk, _ = (ctx.eval_batch if dim == 3 else ctx.eval_batch2)(hs, walkers)
    ref = -0.5 * ctx.chi2(hs, pk).cpu().numpy()
    np.testing.assert_allclose(lp.cpu().numpy(), ref, rtol=1e-4)
    acc = torch.zeros(nw, dtype=torch.int32, device="cuda")
    for t in range(2):
        xb, lpb = x.clone(), lp.clone()
        ctx.mcmc_step(hs, spec, x, lp, torch.tensor(synth.uniforms((2, nw // 2, 3), 320 + 10 * dim + t),
                                                    device="cuda"), acc)
        moved = acc.cpu().numpy().astype(bool)
        assert 0 < moved.sum() < nw
        np.testing.assert_array_equal(x.cpu().numpy()[~moved], xb.cpu().numpy()[~moved])
        np.testing.assert_array_equal(lp.cpu().numpy()[~moved], lpb.cpu().numpy()[~moved])
        assert np.all(np.any(x.cpu().numpy()[moved] != xb.cpu().numpy()[moved], axis=1))
    xn = x.cpu().numpy()
    assert np.all((xn >= np.asarray(lo)) & (xn <= np.asarray(hi)))
    np.testing.assert_allclose(ctx.mcmc_lnprob(hs, spec, x).cpu().numpy(), lp.cpu().numpy(), rtol=1e-9)
    ctx.close()


def test_mcmc_rejects_bad_arguments(xs):
    import torch
    ctx = _ctx(xs)
    d = synth.make_box(16, 32.0, 9.0, seed=3, amp=AMP, dtype=np.float32)
    h = ctx.add_box(d, 32.0, 9.0, 4)
    ctx.prepare("f32", max_walkers=4, max_plain_radii=30)
    x = torch.tensor([[30.0, 10.0, 4.5]] * 4, dtype=torch.float64, device="cuda")
    lp = torch.zeros(4, dtype=torch.float64, device="cuda")
    u = torch.full((2, 2, 3), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(xs.Xs21Error):
        ctx.mcmc_lnprob([h], xs.sampler(*PRIOR3), x)            # no mock yet
    ctx.set_mock(h, np.ones(4))
    with pytest.raises(xs.Xs21Error):
        ctx.mcmc_lnprob([h], xs.sampler([0.0, 5.0, 4.0], [100.0, 20.0, 5.3]), x)   # zeta >= 0 allowed in prior
    with pytest.raises(xs.Xs21Error):
        ctx.mcmc_step([h], xs.sampler(*PRIOR3), x[:3], lp[:3], u[:, :1].contiguous())   # odd ensemble
    with pytest.raises(ValueError):
        ctx.mcmc_step([h], xs.sampler(*PRIOR3), x, lp, u[:, :1].contiguous())   # uniforms of the wrong shape
    with pytest.raises(xs.Xs21Error):
        ctx.mcmc_step([h], xs.sampler(*PRIOR3, a=1.0), x, lp, u)
    lp = ctx.mcmc_lnprob([h], xs.sampler(*PRIOR3), x)
    assert np.isfinite(lp.cpu().numpy()).all()
    out = ctx.mcmc_lnprob([h], xs.sampler([5.0, 5.0, 4.6], [100.0, 20.0, 5.3]), x)   # walkers below the prior
    assert np.all(np.isneginf(out.cpu().numpy()))
    ctx.close()


def test_two_population_bf16_storage_with_velocity(xs):
    """Two-population walkers on BF16-stored smoothed boxes with the velocity-gradient factor
    of eq. (4) switched on (32^3, 64 Mpc, z = 9): reported against the oracle, loose bounds
    as for BF16 storage with constant efficiency."""
    n, box, z, nb = 32, 64.0, 9.0, 6
    d = synth.make_box(n, box, z, seed=47, amp=AMP, dtype=np.float32)
    phys = oracle.Physics(pk_amp=AMP, velocity=True, dvdr_max=0.2)
    ctx = _ctx(xs, velocity=1, dvdr_max=0.2)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare("bf16", max_walkers=4, max_plain_radii=30)
    walkers = EDGE2[:4]
    pk, xhi = ctx.eval_batch2([b], walkers)
    pk = pk.cpu().numpy()
    xhi = xhi.cpu().numpy()
    shared = ctx.radii(b)
    for i, w in enumerate(walkers):
        ev = oracle.two_population.evaluate(d.astype(np.float64), box, z, w, oracle.walker_radii(shared, w[1]), nb,
                                            phys)
        x, _ = ctx.materialize2(b, w)
        flips, rel = report(f"two-pop-bf16-vel w{i}", x.cpu().numpy(), ev, pk[i, 0], xhi[i, 0])
        assert flips <= 3e-2 and rel <= 5e-2
        assert abs(xhi[i, 0] - ev.xhi_mean) <= 1e-2
    ctx.close()


# ------------------------------------------------------------------ launch shapes and graphs

def test_launch_shapes_and_autotune(xs, tmp_path):
    """Launch shapes change nothing but the order of sums (the two flag tests
    are exact): explicit shapes and the autotuner's choice reproduce the default
    P(k) to the order of FP64 sums and the mean x_HI to the FP32 first level of
    its sums (the two flag tests run different ionisation kernels, which group
    the cells of a partial sum differently); the choice is cached under its key
    and read back by a second context without timing."""
    n, box, z, nb = 64, 128.0, 9.0, 12
    d = synth.make_box(n, box, z, seed=48, amp=AMP, dtype=np.float32)
    walkers = synth.draw_walkers(40, 17)
    cache = str(tmp_path / "tuning.json")
    ctx = _ctx(xs)
    b = ctx.add_box(d, box, z, nb)
    ctx.prepare("f32", max_walkers=40, max_plain_radii=30)
    pk0, x0 = (t.cpu().numpy() for t in ctx.eval_batch([b], walkers))
    res = ctx.autotune([b], walkers, reps=2, cache_path=cache)
    print(f"[autotune 64^3] {res}", flush=True)
    assert not res["from_cache"] and res["best_ms"] > 0
    pk1, x1 = (t.cpu().numpy() for t in ctx.eval_batch([b], walkers))
    np.testing.assert_allclose(pk1, pk0, rtol=1e-12)
    np.testing.assert_allclose(x1, x0, rtol=8 * 2.0 ** -24)
    ctx.set_tuning(n, ion_blocks=500, pipe_blocks=300, bins_blocks=700, flag_test=0, group=7)
    pk2, x2 = (t.cpu().numpy() for t in ctx.eval_batch([b], walkers))
    np.testing.assert_allclose(pk2, pk0, rtol=1e-12)
    np.testing.assert_allclose(x2, x0, rtol=8 * 2.0 ** -24)
    ctx.close()
    ctx2 = _ctx(xs)
    b2 = ctx2.add_box(d, box, z, nb)
    ctx2.prepare("f32", max_walkers=40, max_plain_radii=30)
    res2 = ctx2.autotune([b2], walkers, reps=2, cache_path=cache)
    assert res2["from_cache"] and res2["tuning"] == res["tuning"]
    assert ctx2.get_tuning(n) == res["tuning"]
    ctx2.close()


@pytest.mark.parametrize("dim", [3, 5])
def test_graph_replay_of_sampler_steps(xs, dim):
    """An ensemble step recorded into a launch graph on a created stream, launched
    three times with new uniforms copied in by eager work between the launches,
    against the same steps called directly: every launch gives the same walkers
    and ln p bit for bit; calls that synchronise are refused while capturing."""
    import torch
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):   # torch's work ordered with the context's
        _graph_case(xs, dim, st)
    torch.cuda.synchronize()


def _graph_case(xs, dim, st):
    import torch
    n, box, z, nb = 32, 64.0, 9.0, 6
    d = synth.make_box(n, box, z, seed=49, amp=AMP, dtype=np.float32)
    lo, hi = PRIOR3 if dim == 3 else PRIOR5
    nw, steps = 8, 3
    x0 = np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * synth.uniforms((nw, dim), 500 + dim)
    us = synth.uniforms((steps, 2, nw // 2, 3), 510 + dim)
    ctx = xs.Context(0, stream=st, phys=xs.physics(pk_amp=AMP))
    h = ctx.add_box(d, box, z, nb)
    ctx.prepare("f32", max_walkers=4, max_plain_radii=30)
    fid = (30.0, 15.0, 5e4) if dim == 3 else (70.0, 15.0, 10 ** 4.7, 4 / 3, -1 / 3)
    fpk, _ = (ctx.eval_batch if dim == 3 else ctx.eval_batch2)([h], [fid])
    km, _ = ctx.bins(h)
    ctx.set_mock(h, km ** 3 * fpk.cpu().numpy()[0, 0, :nb] / (2 * np.pi ** 2))
    spec = xs.sampler(lo, hi)
    xe = torch.tensor(x0, dtype=torch.float64, device="cuda")
    xg = xe.clone()
    lpe = torch.empty(nw, dtype=torch.float64, device="cuda")
    lpg = torch.empty(nw, dtype=torch.float64, device="cuda")
    ub = torch.zeros((2, nw // 2, 3), dtype=torch.float64, device="cuda")
    acc = torch.zeros(nw, dtype=torch.int32, device="cuda")
    pk_pre = torch.empty((1, 1, nb), dtype=torch.float64, device="cuda")
    xh_pre = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    ctx.mcmc_lnprob([h], spec, xe, lpe)
    ctx.mcmc_lnprob([h], spec, xg, lpg)
    st.synchronize()
    ctx.capture_begin()
    with pytest.raises(xs.Xs21Error, match="graph capture"):   # host-planned walkers: refused, nothing recorded
        (ctx.eval_batch if dim == 3 else ctx.eval_batch2)([h], [fid], pk_pre, xh_pre)
    ctx.mcmc_step([h], spec, xg, lpg, ub, acc)
    g = ctx.capture_end()
    moved = 0
    for t in range(steps):
        ut = torch.tensor(us[t], dtype=torch.float64, device="cuda")
        ub.copy_(ut)
        ctx.mcmc_step([h], spec, xe, lpe, ut, acc)   # eager reference with the same uniforms
        g.launch()
        st.synchronize()
        moved += int(acc.sum())
        assert torch.equal(xg, xe) and torch.equal(lpg, lpe), f"launch {t} differs from the direct step"
    print(f"[graph dim={dim}] {steps} launches equal to direct steps; accepted {moved}", flush=True)
    g.close()
    ctx.close()
