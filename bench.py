"""Benchmark: walker likelihood evaluations per second at 256^3 x 3 redshifts.

One step = the whole path over one batch: for each of the three boxes
(256^3, 250 Mpc, z = 8, 9, 10) the forward FFT and every sharp-k smoothed box
of the shared radius ladder, then for all 64 walkers the ionisation field,
dT_b and binned P(k) on all three boxes, and each walker's chi^2 against a
synthetic mock (the fiducial walker's Delta^2 on the same boxes, no noise,
25 per cent modelling error, 0.15 <= k <= 1 Mpc^-1).  value = walkers / step
time.

Also reported: the steady-state rate with the smoothed boxes resident (the MCMC
loop), the plain per-walker form (recomputes the forward FFT and all smoothed
boxes of the walker's own radii per evaluation), Gcell-R/s, the roofline of the
dominant kernel (HIP events on the library stream inside the timed steps,
algorithmic bytes against the 8 TB/s HBM peak; VALU instructions from the
committed counter run against the vector instruction rate as a second view),
the project's own HBM probes (read, write, copy and the binning pass's strided
tiles) as practical ceilings, the FP64 CPU oracle timed on a bounded sample,
the same step with the velocity-gradient factor of eq. (4) and with
two-population walkers (eq. (9)), the device-resident ensemble sampler
(Section 2.3), the steady state with 256 and 1024 walkers, the shared smoothing
stage alone, the plain single-walker workloads (64^3 FP64, 128^3 x 3 z FP32)
with the oracle timed beside them, the uneven 128^3/256^3 BF16 workload with
256 walkers, and the 512^3 x 3 z workload with 1024 walkers.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Vector ALU instruction rate without packed FP32 (disabled in this build): 256
# CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-instructions per second (a
# wave64 VALU instruction occupies a SIMD for 4 cycles).  Used for the
# secondary ALU view: SQ_INSTS_VALU x 64 lanes per launch over the launch time.
VALU_PEAK_TLANES = 256 * 4 * 16 * 2.4e9 / 1e12
VALU_FILE = os.path.join(ROOT, "profiles", "valu.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
FIDUCIAL = (30.0, 15.0, 5e4)  # zeta, R_mfp [Mpc], T_vir [K] of the mock
# zeta0, R_mfp [Mpc], T_feed [K], alpha, beta: the two-population fiducial of Section 4
FIDUCIAL2 = (70.0, 15.0, 10 ** 4.7, 4.0 / 3.0, -1.0 / 3.0)

# Sources of the path's kernels (the likelihood epilogue lives apart).
KERNEL_SOURCES = ("kernels.hip", "fft.hpp", "wave.hpp", "common.hpp", "launch.hpp")


def kernel_source_hash() -> str:
    """Hash of the path's kernel sources; counter figures are only reused for the same code."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1501_06576_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def _profile_json(path: str, workload: str):
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    return t


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of kernel class `kernel` from the committed rocprofv3
    counter runs (FETCH_SIZE and WRITE_SIZE scaled by the probes' readings), or
    None if the kernels changed since those counters were taken."""
    t = _profile_json(TRAFFIC_FILE, workload)
    if t is None or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["bytes_per_launch"]


def measured_valu(kernel: str, workload: str):
    """VALU instructions per launch of kernel class `kernel` (SQ_INSTS_VALU summed
    over its waves) from the committed counter run, or None if the kernels changed."""
    t = _profile_json(VALU_FILE, workload)
    if t is None or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["valu_insts_per_launch"]


def measured_valu_busy(kernel: str, workload: str):
    """rocprofv3's VALUBusy (percent) for kernel class `kernel` from the committed run, or None."""
    t = _profile_json(VALU_FILE, workload)
    if t is None or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel].get("valu_busy_pct")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- rocprofv3 summaries

def kernel_class(name: str):
    """The library's kernel class of a kernel symbol (the classes of xs21_profile_read),
    "probe" for the HBM probes, None for kernels outside the library."""
    import re
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    rules = (("k_rows_r2c", "rows_r2c"), ("k_rows_c2r", "rows_c2r"), ("k_axis_bins", "axis_bins"),
             ("k_ion", "ion"), ("k_finalize", "finalize"), ("k_probe", "probe"))
    for pre, cls in rules:
        if re.search(r"\b" + pre, n):
            return cls
    m = re.search(r"\bk_axis(_pipe)?<[^,]+, *\d+, *(-?1)", n)
    if m:
        return "axis_fwd" if m.group(2) == "-1" else "axis_inv"
    if re.search(r"\bk_(plan|walker2|slot_tables)", n):
        return "plan"
    if re.search(r"\bk_", n) and "xs21" in name or re.search(r"\bk_(los_factor|chi2|lnprob|cast|stretch)", n):
        return "other"
    return None


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    return n.replace("xs21::", "").replace("void ", "").strip()[:52]


def _csv_rows(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _counter_runs(directory):
    """{counter: {dispatch: (kernel name, value)}} over every counter-collection CSV below `directory`."""
    import glob
    out = {}
    for f in sorted(glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)):
        for r in _csv_rows(f):
            c = r.get("Counter_Name")
            if not c:
                continue
            key = (f, r.get("Dispatch_Id"))
            cur = out.setdefault(c, {}).get(key)
            val = float(r["Counter_Value"])
            out[c][key] = (r["Kernel_Name"], val + (cur[1] if cur else 0.0))
    return out


def summarize_profiles(directory: str, bench_json: str, workload: str, commands: list, tag: str = None):
    """Writes profiles/traffic.json, profiles/valu.json and their text tables from the
    rocprofv3 counter runs under `directory` (FETCH_SIZE and WRITE_SIZE runs of
    `bench.py --calibrate`, an SQ counter run), and profiles/kernels_<workload>.txt from
    a --kernel-trace --stats run.  Per kernel symbol the median over its dispatches is
    taken (the fiducial mock's single-walker launches are a minority)."""
    import glob
    import statistics
    runs = _counter_runs(directory)
    cal = None
    if bench_json:
        with open(bench_json) as fh:
            cal = json.loads(fh.read().strip().splitlines()[-1]).get("calibration")
    tag = tag or workload.replace("-", "")
    src_hash = kernel_source_hash()
    prof_dir = os.path.join(ROOT, "profiles")

    def per_kernel(counter):
        by = {}
        for name, v in runs.get(counter, {}).values():
            by.setdefault(name, []).append(v)
        return by

    fetch, write = per_kernel("FETCH_SIZE"), per_kernel("WRITE_SIZE")
    if fetch and write and cal:
        def probe(d, kind):
            vals = [v for n, vs in d.items() if f"k_probe_{kind}" in n for v in vs]
            return statistics.median(vals) * 1024.0 if vals else None
        # scale = bytes the probe moves / bytes the counter reports, per access pattern
        scales = {"read": cal["read"] / probe(fetch, "read"), "tile": cal["tile"] / probe(fetch, "tile"),
                  "copy_fetch": 0.5 * cal["copy"] / probe(fetch, "copy"),
                  "write": cal["write"] / probe(write, "write"), "copy_write": 0.5 * cal["copy"] / probe(write, "copy")}
        fs, ws = scales["read"], scales["write"]
        kernels, lines = {}, []
        for name in sorted(set(fetch) | set(write)):
            cls = kernel_class(name)
            if cls in (None, "probe"):
                continue
            f = statistics.median(fetch.get(name, [0.0])) * 1024.0 * fs
            w = statistics.median(write.get(name, [0.0])) * 1024.0 * ws
            lines.append(f"{_short(name):52s} {len(fetch.get(name, [])):5d} {f / 1e6:10.1f} {w / 1e6:10.1f} "
                         f"{(f + w) / 1e6:12.1f}")
            if cls not in kernels or f + w > kernels[cls]["bytes_per_launch"]:
                kernels[cls] = {"bytes_per_launch": f + w, "fetch_bytes": f, "write_bytes": w, "kernel": _short(name)}
        t = {"source_hash": src_hash, "workload": workload, "fetch_scale": fs, "write_scale": ws,
             "scales_by_pattern": scales, "commands": [c for c in commands if "FETCH" in c or "WRITE" in c],
             "kernels": kernels}
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(t, fh, indent=1)
        with open(os.path.join(prof_dir, f"traffic_{tag}.txt"), "w") as fh:
            fh.write(f"# rocprofv3 HBM traffic per dispatch (median over dispatches): {workload} workload\n")
            for c in t["commands"]:
                fh.write(f"# command: {c}\n")
            fh.write("# calibration with the project's probes in the same runs (bytes moved / counter bytes):\n")
            fh.write("#   " + ", ".join(f"{k} {v:.3f}" for k, v in scales.items()) + "\n")
            fh.write(f"#   FETCH_SIZE scaled by {fs:.3f} (streaming read), WRITE_SIZE by {ws:.3f}\n")
            fh.write(f"# kernel source hash: {src_hash}\n\n")
            fh.write(f"{'kernel':52s} {'disp':>5s} {'fetch MB':>10s} {'write MB':>10s} {'total MB/disp':>12s}\n")
            fh.write("\n".join(lines) + "\n")
        log(f"wrote {TRAFFIC_FILE}")

    util = [c for c in ("VALUBusy", "VALUUtilization", "LdsUtil", "LDSBankConflict") if c in runs]
    sq = [c for c in runs if c.startswith("SQ_")]
    if util:
        med = {c: {n: statistics.median(vs) for n, vs in per_kernel(c).items()} for c in util}
        names = sorted(set().union(*(m.keys() for m in med.values())))
        with open(os.path.join(prof_dir, f"utilization_{tag}.txt"), "w") as fh:
            fh.write(f"# rocprofv3 derived metrics per dispatch, percent (median over dispatches): {workload} workload\n")
            for c in commands:
                if "VALUBusy" in c:
                    fh.write(f"# command: {c}\n")
            fh.write("# VALUBusy: share of the kernel's time the CUs' vector ALUs issue; VALUUtilization: active\n"
                     "# lanes per VALU instruction; LdsUtil: share of time LDS is busy; LDSBankConflict: share of\n"
                     "# time LDS is stalled by bank conflicts\n")
            fh.write(f"# kernel source hash: {src_hash}\n\n")
            fh.write(f"{'kernel':52s} " + " ".join(f"{c[:15]:>15s}" for c in util) + "\n")
            for name in names:
                if kernel_class(name) in (None, "probe"):
                    continue
                fh.write(f"{_short(name):52s} " + " ".join(f"{med[c].get(name, 0.0):15.1f}" for c in util) + "\n")
        log(f"wrote utilization_{tag}.txt")
        busy = med.get("VALUBusy", {})
    else:
        busy = {}
    if sq:
        med = {c: {n: statistics.median(vs) for n, vs in per_kernel(c).items()} for c in sq}
        names = sorted(set().union(*(m.keys() for m in med.values())))
        kernels, lines = {}, []
        for name in names:
            cls = kernel_class(name)
            if cls in (None, "probe"):
                continue
            row = {c: med[c].get(name, 0.0) for c in sq}
            waves = row.get("SQ_WAVES", 0.0) or 1.0
            valu = row.get("SQ_INSTS_VALU", 0.0)
            lines.append(f"{_short(name):52s} " + " ".join(f"{row[c] / waves:10.0f}" for c in sq if c != "SQ_WAVES")
                         + f" {waves:9.0f}")
            if cls not in kernels or valu > kernels[cls]["valu_insts_per_launch"]:
                kernels[cls] = {"valu_insts_per_launch": valu, "waves_per_launch": waves, "kernel": _short(name),
                                "per_wave": {c: row[c] / waves for c in sq if c != "SQ_WAVES"},
                                "valu_busy_pct": busy.get(name)}
        t = {"source_hash": src_hash, "workload": workload,
             "commands": [c for c in commands if "SQ_" in c or "VALUBusy" in c], "kernels": kernels}
        with open(VALU_FILE, "w") as fh:
            json.dump(t, fh, indent=1)
        with open(os.path.join(prof_dir, f"sq_counters_{tag}.txt"), "w") as fh:
            fh.write(f"# rocprofv3 SQ counters per wave (median over dispatches): {workload} workload\n")
            for c in t["commands"]:
                fh.write(f"# command: {c}\n")
            fh.write(f"# kernel source hash: {src_hash}\n\n")
            fh.write(f"{'kernel':52s} " + " ".join(f"{c[3:][:10]:>10s}" for c in sq if c != "SQ_WAVES")
                     + f" {'waves':>9s}\n")
            fh.write("\n".join(lines) + "\n")
        log(f"wrote {VALU_FILE}")

    stats = sorted(glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True))
    if stats:
        rows = _csv_rows(stats[-1])
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        with open(os.path.join(prof_dir, f"kernels_{tag}.txt"), "w") as fh:
            fh.write(f"# rocprofv3 kernel statistics: {workload} workload\n")
            for c in commands:
                if "--kernel-trace" in c:
                    fh.write(f"# command: {c}\n")
            fh.write(f"# kernel source hash: {src_hash}\n\n")
            fh.write(f"{'kernel':52s} {'calls':>6s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}\n")
            for r in rows:
                fh.write(f"{_short(r['Name']):52s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                         f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}\n")
        log(f"wrote kernels_{tag}.txt")


def cpu_model() -> str:
    """The host CPU's model name (Linux), or "" where it cannot be read."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def describe(wl, nw):
    geos = {}
    for s in wl.boxes:
        geos.setdefault((s.n, s.box_mpc), []).append(s.z)
    parts = [f"{n}^3 / {L:g} Mpc at z=" + ",".join(f"{z:g}" for z in zs) for (n, L), zs in geos.items()]
    return f"{wl.name}: {len(wl.boxes)} boxes ({'; '.join(parts)}), {nw} walkers, {wl.storage} smoothed boxes"


def roofline(prof, steps, workload):
    """Roofline of the dominant kernel class over the timed launches: algorithmic
    bytes per launch over its average launch time against the HBM peak, and the
    VALU instruction rate from the committed counters beside it."""
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    n = max(d["launches"], 1)
    avg_ms = d["ms"] / n
    bytes_launch = d["bytes"] / n
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    valu = measured_valu(dom, workload)
    out = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, workload),
           "avg_launch_ms": round(avg_ms, 5), "launches_timed": d["launches"],
           "algorithmic_bytes_per_launch": bytes_launch, "source_hash": kernel_source_hash()}
    if valu is not None:
        lanes = valu * 64 / (avg_ms * 1e-3) / 1e12
        out["valu"] = {"insts_per_launch": valu, "achieved": round(lanes, 3), "peak": round(VALU_PEAK_TLANES, 2),
                       "unit": "T lane-instructions/s", "frac": round(lanes / VALU_PEAK_TLANES, 4),
                       "valu_busy_pct_counter": measured_valu_busy(dom, workload)}
    else:
        out["valu"] = None
    return out


def kernel_table(prof, steps):
    return {k: {"ms_per_step": round(v["ms"] / steps, 4), "launches_per_step": v["launches"] / steps,
                "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in prof.items() if v["launches"]}


def cell_radii(ctx, hs, specs, walkers):
    """Sum over walkers and boxes of N^3 x (radii the walker filters at)."""
    tot = 0.0
    for h, s in zip(hs, specs):
        shared = np.array(ctx.radii(h))
        for w in walkers:
            tot += float(s.n) ** 3 * (np.count_nonzero(shared[:-1] <= w[1]) + 1)
    return tot


def tuning_cache() -> str:
    """The autotuner's JSON cache (XS21_TUNING_CACHE, else ~/.cache/xs21/tuning.json)."""
    path = os.environ.get("XS21_TUNING_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "xs21",
                                                                  "tuning.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    return path


class Batch:
    """A prepared context (on its own stream) over one workload's boxes with a mock for
    the chi^2 epilogue."""

    def __init__(self, xs, torch, wl, amp, walkers, phys_kw=None, group=64):
        self.torch = torch
        self.xs = xs
        self.wl = wl
        log(f"workload {wl.name}: generating {len(wl.boxes)} boxes")
        self.boxes = synth.workload_boxes(wl, amp)
        self.walkers = walkers
        self.nw = len(walkers)
        # a stream of its own (a launch graph cannot be recorded on the null stream), made
        # torch's current stream so that tensors and host copies are ordered with the library
        self.stream = torch.cuda.Stream()
        torch.cuda.set_stream(self.stream)
        self.ctx = xs.Context(0, stream=self.stream, phys=xs.physics(pk_amp=amp, **(phys_kw or {})))
        self.hs = [self.ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(self.boxes, wl.boxes)]
        self.ctx.prepare(wl.storage, max_walkers=min(self.nw, group), max_plain_radii=40)
        self.nbmax = max(s.n_bins for s in wl.boxes)
        self.pk = torch.empty((self.nw, len(self.hs), self.nbmax), dtype=torch.float64, device="cuda")
        self.xhi = torch.empty((self.nw, len(self.hs)), dtype=torch.float64, device="cuda")
        self.chi2 = torch.empty(self.nw, dtype=torch.float64, device="cuda")
        self.set_mock(FIDUCIAL)

    def set_mock(self, fid, two=False):
        fpk, _ = (self.ctx.eval_batch2 if two else self.ctx.eval_batch)(self.hs, [fid])
        fpk = fpk.cpu().numpy()
        for i, h in enumerate(self.hs):
            km, _counts = self.ctx.bins(h)
            self.ctx.set_mock(h, km ** 3 * fpk[0, i, : len(km)] / (2 * np.pi ** 2))

    def step(self, walkers=None, two=False):
        for h in self.hs:
            self.ctx.resmooth(h)
        self.steady(walkers, two)

    def steady(self, walkers=None, two=False):
        fn = self.ctx.eval_batch2 if two else self.ctx.eval_batch
        fn(self.hs, self.walkers if walkers is None else walkers, self.pk, self.xhi)
        self.ctx.chi2(self.hs, self.pk, self.chi2)

    def timed(self, fn, reps, warmup=1):
        for _ in range(warmup):
            fn()
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        self.torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    def autotune(self):
        """Launch shapes for each grid size of the workload (autotuner, JSON cache), timed on
        the workload's first walker group."""
        out = {}
        t0 = time.perf_counter()
        for n in sorted({s.n for s in self.wl.boxes}):
            hs = [h for h, s in zip(self.hs, self.wl.boxes) if s.n == n]
            out[str(n)] = self.ctx.autotune(hs, self.walkers[:64], reps=2, cache_path=tuning_cache())
        out["seconds"] = round(time.perf_counter() - t0, 2)
        return out

    def graph_steady(self, reps):
        """The steady state as one launch graph: ln p (chi^2 against the mock) of the walkers
        held on the device, planned and evaluated on the device, recorded once and launched
        `reps` times; also the same call made directly.  Returns ms per batch of both."""
        torch = self.torch
        w = np.asarray(self.walkers, dtype=np.float64)
        x = np.column_stack([w[:, 0], w[:, 1], np.log10(w[:, 2])])
        spec = self.xs.sampler((5.0, 5.0, 4.0), (100.0, 20.0, 6.0))
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        lp = torch.empty(self.nw, dtype=torch.float64, device="cuda")
        ms_direct = self.timed(lambda: self.ctx.mcmc_lnprob(self.hs, spec, xd, lp), reps)
        ref = lp.clone()
        self.ctx.capture_begin()
        self.ctx.mcmc_lnprob(self.hs, spec, xd, lp)
        g = self.ctx.capture_end()
        ms_graph = self.timed(g.launch, reps)
        same = bool(torch.equal(lp, ref))
        g.close()
        return {"ms_per_batch": round(ms_graph, 4), "walker_evals_per_s": round(self.nw / (ms_graph * 1e-3), 2),
                "direct_ms_per_batch": round(ms_direct, 4), "replay_equals_direct": same,
                "note": "ln p = -chi^2/2 of device-resident walkers, planned on the device, one graph launch per batch"}

    def close(self):
        self.ctx.close()
        del self.pk, self.xhi, self.chi2
        self.ctx = None
        self.torch.cuda.synchronize()
        self.torch.cuda.set_stream(self.torch.cuda.default_stream())
        self.torch.cuda.empty_cache()


def hbm_probes(xs, torch):
    """The project's own HBM probes over 4 GiB (the tile probe over 50 spectra of 256^3)."""
    ctx = xs.Context(0, phys=xs.physics())
    out = {}
    for kind, nbytes in (("read", 4 << 30), ("write", 4 << 30), ("copy", 4 << 30), ("tile", 3800 << 20)):
        r = ctx.probe_bandwidth(kind, nbytes + (64 << 10), reps=5)
        out[kind] = {"GBps": round(r["GBps"], 1), "frac_of_peak": round(r["GBps"] / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": r["bytes_per_launch"]}
    ctx.close()
    torch.cuda.empty_cache()
    out["kind"] = ("project-written probe kernels (csrc/probe.hip): streaming 16-byte loads / stores, "
                   "copy = read + write bytes, tile = the binning pass's strided 128-byte segments")
    return out


def section_plain_configs(xs, torch, amp, reps):
    """The plain single-walker workloads (64^3 FP64 at z = 9; 128^3 FP32 at z = 8, 9, 10):
    the literal per-walker method on the GPU (forward FFT and every smoothed box of the
    walker's own radii per evaluation) and the FP64 oracle on the host, full evaluations."""
    import oracle
    phys = oracle.Physics(pk_amp=amp)
    out = {}
    for name in ("plain-f64-64", "plain-f32-128"):
        wl = synth.WORKLOADS[name]
        boxes = synth.workload_boxes(wl, amp)
        w = wl.walkers[0]
        ctx = xs.Context(0, phys=xs.physics(pk_amp=amp))
        hs = [ctx.add_box(d, s.box_mpc, s.z, s.n_bins) for d, s in zip(boxes, wl.boxes)]
        ctx.prepare(wl.storage, max_walkers=1, max_plain_radii=40)
        for h in hs:
            ctx.eval(h, w, fields=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for h in hs:
                ctx.eval(h, w, fields=False)
        torch.cuda.synchronize()
        ms_gpu = (time.perf_counter() - t0) * 1e3 / reps
        ctx.close()
        t0 = time.perf_counter()
        nrad = []
        for d, s in zip(boxes, wl.boxes):
            radii = oracle.plain_radii(w[1], s.n, s.box_mpc, phys)
            nrad.append(len(radii))
            oracle.evaluate(d, s.box_mpc, s.z, w, radii, s.n_bins, phys)
        s_orc = time.perf_counter() - t0
        out[name] = {"workload": describe(wl, 1) + f", walker {w}, {'/'.join(map(str, nrad))} radii",
                     "dtype": wl.dtype, "gpu_ms_per_eval": round(ms_gpu, 3),
                     "gpu_evals_per_s": round(1e3 / ms_gpu, 2),
                     "oracle_s_per_eval": round(s_orc, 3), "oracle_cores": oracle.FFT_WORKERS,
                     "gpu_over_oracle": round(s_orc * 1e3 / ms_gpu, 1),
                     "note": "one eval = the walker on every box of the workload; plain form on both sides"}
    torch.cuda.empty_cache()
    return out


def section_workload(xs, torch, amp, name, reps, group=64, graph=False, oracle_box=False):
    """Full step and steady state of another workload, with its kernel table and roofline;
    oracle_box: the FP64 oracle timed on one walker x the first box beside the GPU's
    steady-state time per walker-box."""
    wl = synth.WORKLOADS[name]
    walkers = synth.workload_walkers(wl)
    b = Batch(xs, torch, wl, amp, walkers, group=group)
    tuning = b.autotune()
    ms_step = b.timed(b.step, reps)
    ms_steady = b.timed(b.steady, reps)
    # kernel table: exactly `reps` further steady-state batches under the
    # library's event timing (after the warm-up above)
    b.ctx.profile(True)
    for _ in range(reps):
        b.steady()
    prof = b.ctx.profile_read()
    b.ctx.profile(False)
    cellr = cell_radii(b.ctx, b.hs, wl.boxes, walkers)
    out = {"workload": describe(wl, b.nw), "walkers": b.nw, "group": min(b.nw, group),
           "ms_per_step": round(ms_step, 3), "walker_evals_per_s": round(b.nw / (ms_step * 1e-3), 2),
           "steady_state": {"ms_per_batch": round(ms_steady, 3),
                            "walker_evals_per_s": round(b.nw / (ms_steady * 1e-3), 2),
                            "gcell_r_per_s": round(cellr / (ms_steady * 1e-3) / 1e9, 2)},
           "kernels_steady": kernel_table(prof, reps), "roofline_steady": roofline(prof, reps, name),
           "tuning": tuning}
    if graph:
        out["steady_state"]["graph"] = b.graph_steady(reps)
    if oracle_box:
        import oracle
        log(f"timing the FP64 CPU oracle on one walker x one box of {name}")
        w, s0 = walkers[0], wl.boxes[0]
        radii = oracle.walker_radii(b.ctx.radii(b.hs[0]), w[1])
        t0 = time.perf_counter()
        oracle.evaluate(b.boxes[0], s0.box_mpc, s0.z, w, radii, s0.n_bins, oracle.Physics(pk_amp=amp))
        dt = time.perf_counter() - t0
        gpu_s = ms_steady * 1e-3 / (b.nw * len(b.hs))
        out["cpu_baseline_walker_box"] = {
            "oracle_s": round(dt, 3), "cores": oracle.FFT_WORKERS, "kind": "oracle",
            "sample": f"walker ({float(w[0]):.4g}, {float(w[1]):.4g} Mpc, {float(w[2]):.4g} K) on box 0 "
                      f"({s0.n}^3 / {s0.box_mpc:g} Mpc, z = {s0.z:g}, {len(radii)} radii)",
            "gpu_steady_s_per_walker_box": round(gpu_s, 7), "gpu_over_oracle": round(dt / gpu_s, 1)}
    b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched-256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-walkers", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-walker form")
    ap.add_argument("--no-velocity", action="store_true",
                    help="skip the variant with the velocity-gradient factor of eq. (4)")
    ap.add_argument("--no-mcmc", action="store_true", help="skip the ensemble-sampler loop")
    ap.add_argument("--no-two-population", action="store_true",
                    help="skip the variant with the two-population efficiency of eq. (9)")
    ap.add_argument("--no-scaling", action="store_true",
                    help="skip the shared-stage timing, the steady state at 256 and 1024 walkers and the probes")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (plain 64^3 / 128^3, uneven BF16 mix, 512^3)")
    ap.add_argument("--no-autotune", action="store_true", help="run with the default launch shapes")
    ap.add_argument("--calibrate", action="store_true",
                    help="end with the HBM probes once each (references for counter scaling)")
    ap.add_argument("--summarize", metavar="DIR",
                    help="no GPU work: write the profiles/ summaries from the rocprofv3 output under DIR")
    ap.add_argument("--bench-json", help="with --summarize: the JSON line of the profiled --calibrate run")
    ap.add_argument("--commands", help="with --summarize: file holding the profiling commands, one a line")
    ap.add_argument("--tag", help="with --summarize: name part of the text summaries (default: the workload)")
    args = ap.parse_args()
    if args.summarize:
        cmds = []
        if args.commands:
            with open(args.commands) as fh:
                cmds = [c.strip() for c in fh if c.strip()]
        summarize_profiles(args.summarize, args.bench_json, args.workload, cmds, args.tag)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards by walkers and "
              "boxes across GPUs, which this build does not run", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1501_06576_amd as xs

    if not os.path.exists(xs.LIB_PATH):
        from paper_1501_06576_amd import build
        build.build()
    wl = synth.WORKLOADS[args.workload]
    amp = synth.reference_amplitude()
    walkers = synth.workload_walkers(wl)
    b = Batch(xs, torch, wl, amp, walkers)
    ctx, hs, nw = b.ctx, b.hs, b.nw
    tuning = None if args.no_autotune else b.autotune()

    for _ in range(args.warmup):
        b.step()
    torch.cuda.synchronize()
    log("timing full steps")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = nw / (ms_step * 1e-3)

    # steady state: smoothed boxes resident, only the per-walker work
    log("timing steady state")
    ms_steady = b.timed(b.steady, args.steps, warmup=2)
    log("timing the steady state as a launch graph")
    graph = b.graph_steady(args.steps)

    shared_stage = walker_scaling = probes = None
    if not args.no_scaling:
        # the shared stage alone (a2 + a3 for each box), as smoothed cells N^3 x N_R per second
        log("timing the shared smoothing stage")
        ms_shared = b.timed(lambda: [ctx.resmooth(h) for h in hs], args.steps, warmup=0)
        shared_cells = sum(float(s.n) ** 3 * len(ctx.radii(h)) for h, s in zip(hs, wl.boxes))
        shared_stage = {"ms_per_step": round(ms_shared, 4), "boxes": len(hs),
                        "gcell_r_per_s": round(shared_cells / (ms_shared * 1e-3) / 1e9, 2)}
        log("timing the steady state at 256 and 1024 walkers")
        walker_scaling = {}
        for wn in (256, 1024):
            ws = synth.draw_walkers(wn, 1000 + wn)
            pkw = torch.empty((wn, len(hs), b.nbmax), dtype=torch.float64, device="cuda")
            xw = torch.empty((wn, len(hs)), dtype=torch.float64, device="cuda")
            cw = torch.empty(wn, dtype=torch.float64, device="cuda")

            def many():
                ctx.eval_batch(hs, ws, pkw, xw)
                ctx.chi2(hs, pkw, cw)
            ms_w = b.timed(many, 3)
            walker_scaling[str(wn)] = {"ms_per_batch": round(ms_w, 3),
                                       "walker_evals_per_s": round(wn / (ms_w * 1e-3), 2)}
            del pkw, xw, cw

    cellR = cell_radii(ctx, hs, wl.boxes, walkers)

    ms_plain = None
    if not args.no_plain and args.plain_walkers > 0:
        log("timing plain per-walker form")
        pw = walkers[: args.plain_walkers]
        for h in hs:
            ctx.eval(h, pw[0], fields=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for w in pw:
            for h in hs:
                ctx.eval(h, w, fields=False)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) * 1e3 / len(pw)

    # the whole step: algorithmic bytes of every kernel over the step's wall time
    step_bytes = sum(v["bytes"] for v in prof.values()) / args.steps
    step_hbm = {"algorithmic_GB": round(step_bytes / 1e9, 3), "GBps": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
                "frac_of_peak": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    result = {
        "metric": "walker likelihood evals/sec at 256^3 x 3 z; ionization Gcell-R/s; %HBM peak",
        "value": round(value, 2),
        "unit": "walker-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.dtype == "f32" else wl.dtype,
        "data": "synthetic",
        "config": {"workload": describe(wl, nw), "walkers": nw, "boxes": len(hs), "grid": wl.boxes[0].n,
                   "parallelism": "single GPU"},
        "gcell_r_per_s": round(cellR / (ms_step * 1e-3) / 1e9, 2),
        "steady_state": {"ms_per_batch": round(ms_steady, 4), "walker_evals_per_s": round(nw / (ms_steady * 1e-3), 2),
                         "gcell_r_per_s": round(cellR / (ms_steady * 1e-3) / 1e9, 2),
                         "more_walkers": walker_scaling, "graph": graph},
        "tuning": tuning,
        "shared_stage": shared_stage,
        "step_hbm": step_hbm,
        "plain_per_walker": None if ms_plain is None else
        {"ms_per_eval": round(ms_plain, 3), "walker_evals_per_s": round(1e3 / ms_plain, 3)},
        "kernels": kernel_table(prof, args.steps),
        "likelihood": {"chi2_min": round(float(b.chi2.min()), 4), "chi2_median": round(float(b.chi2.median()), 4),
                       "mock": "fiducial walker (30, 15, 5e4) on the same boxes"},
        "roofline": roofline(prof, args.steps, wl.name),
    }

    if not args.no_mcmc:
        # the MCMC loop itself: ensemble steps of 2 x nw walkers (stretch move,
        # device-resident walkers, proposals planned and evaluated on the device)
        # on the resident boxes, against the same mock
        log("timing ensemble sampler steps")
        lo, hi = (5.0, 5.0, 4.0), (100.0, 20.0, 5.3)   # zeta, R_mfp, log10 T_vir
        spec = xs.sampler(lo, hi)
        ne = 2 * nw
        x = torch.tensor(np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * synth.uniforms((ne, 3), 401),
                         dtype=torch.float64, device="cuda")
        lp = ctx.mcmc_lnprob(hs, spec, x)
        acc = torch.zeros(ne, dtype=torch.int32, device="cuda")
        nsteps = args.warmup + args.steps
        u = torch.tensor(synth.uniforms((nsteps, 2, nw, 3), 402), dtype=torch.float64, device="cuda")
        for t in range(args.warmup):
            ctx.mcmc_step(hs, spec, x, lp, u[t], acc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.warmup, nsteps):
            ctx.mcmc_step(hs, spec, x, lp, u[t], acc)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t0) * 1e3 / args.steps
        # untimed: acceptance over as many further steps, then one step under
        # the library's per-kernel event timing
        moved = 0
        u2 = torch.tensor(synth.uniforms((args.steps, 2, nw, 3), 403), dtype=torch.float64, device="cuda")
        for t in range(args.steps):
            ctx.mcmc_step(hs, spec, x, lp, u2[t], acc)
            moved += int(acc.sum())
        ctx.profile(True)
        ctx.mcmc_step(hs, spec, x, lp, u[nsteps - 1], acc)
        prof_m = ctx.profile_read()
        ctx.profile(False)
        result["mcmc"] = {"walkers": ne, "ms_per_step": round(ms_m, 4),
                          "walker_evals_per_s": round(ne / (ms_m * 1e-3), 2),
                          "acceptance": round(float(moved) / (ne * args.steps), 4),
                          "vs_steady_eval": round((ne / (ms_m * 1e-3)) / (nw / (ms_steady * 1e-3)), 4),
                          "kernel_ms_per_step": {k: round(v["ms"], 4) for k, v in prof_m.items() if v["launches"]},
                          "note": "stretch move (a = 2) over (zeta, R_mfp, log10 T_vir) in [5,100]x[5,20]x[4,5.3]"}
        # the same loop over two-population walkers (zeta0, R_mfp, log10 T_feed, alpha, beta)
        lo5, hi5 = (5.0, 5.0, 4.0, -4.0 / 3.0, -4.0 / 3.0), (100.0, 20.0, 5.3, 10.0 / 3.0, 10.0 / 3.0)
        spec5 = xs.sampler(lo5, hi5)
        x5 = torch.tensor(np.asarray(lo5) + (np.asarray(hi5) - np.asarray(lo5)) * synth.uniforms((ne, 5), 404),
                          dtype=torch.float64, device="cuda")
        lp5 = ctx.mcmc_lnprob(hs, spec5, x5)
        for t in range(args.warmup):
            ctx.mcmc_step(hs, spec5, x5, lp5, u[t], acc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.warmup, nsteps):
            ctx.mcmc_step(hs, spec5, x5, lp5, u[t], acc)
        torch.cuda.synchronize()
        ms_m5 = (time.perf_counter() - t0) * 1e3 / args.steps
        result["mcmc"]["two_population"] = {"ms_per_step": round(ms_m5, 4),
                                            "walker_evals_per_s": round(ne / (ms_m5 * 1e-3), 2),
                                            "note": "eq. (9) walkers, prior [5,100]x[5,20]x[4,5.3]x[-4/3,10/3]^2"}

    if not args.no_two_population:
        # the same step for two-population walkers (zeta0, R_mfp, T_feed, alpha, beta)
        # drawn from their priors, against the mock of the fiducial of that model
        log("timing the two-population variant")
        walkers2 = synth.draw_walkers2(nw, synth.WALKER_SEEDS["two-population-256"])
        b.set_mock(FIDUCIAL2, two=True)
        ms_2 = b.timed(lambda: b.step(walkers2, two=True), args.steps, warmup=args.warmup)
        ctx.profile(True)
        b.step(walkers2, two=True)
        prof2 = ctx.profile_read()
        ctx.profile(False)
        result["two_population"] = {
            "ms_per_step": round(ms_2, 4), "walker_evals_per_s": round(nw / (ms_2 * 1e-3), 2),
            "plan_ms_per_step": round(prof2["plan"]["ms"], 4),
            "ion_ms_per_step": round(prof2["ion"]["ms"], 4),
            "chi2_median": round(float(b.chi2.median()), 4),
            "note": "eq. (9) walkers drawn from the priors; mock = fiducial (70, 15 Mpc, 10^4.7 K, 4/3, -1/3)"}

    if not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle on a bounded sample")
        import oracle
        phys = oracle.Physics(pk_amp=amp)
        w = walkers[0]
        nrad = []
        # one walker on every box (at 512^3: on the first box only, tens of seconds per box)
        sample = list(zip(hs, b.boxes, wl.boxes))
        if wl.boxes[0].n >= 512:
            sample = sample[:1]
        t0 = time.perf_counter()
        for h, d, s in sample:
            radii = oracle.walker_radii(ctx.radii(h), w[1])
            nrad.append(len(radii))
            oracle.evaluate(d, s.box_mpc, s.z, w, radii, s.n_bins, phys)
        dt = time.perf_counter() - t0
        # one walker-eval covers every box of the workload: scale a partial sample up by box count
        per_eval = dt * len(hs) / len(sample)
        result["cpu_baseline"] = {"value": round(1.0 / per_eval, 6), "unit": "walker-evals/s", "cores":
                                  oracle.FFT_WORKERS, "kind": "oracle",
                                  "sample": f"1 walker (the batch's first) x {len(sample)} of {len(hs)} boxes "
                                            f"({wl.boxes[0].n}^3, {'/'.join(str(n) for n in nrad)} radii) in "
                                            f"{dt:.2f} s" + ("" if len(sample) == len(hs) else
                                                             f", scaled by {len(hs)}/{len(sample)} boxes"),
                                  "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
    b.close()

    if not args.no_velocity:
        # the same step with the velocity-gradient factor H / (dv_r/dr + H) in dT_b
        log("timing the variant with the velocity-gradient factor")
        vb = Batch(xs, torch, wl, amp, walkers, phys_kw={"velocity": 1})
        ms_v = vb.timed(vb.step, args.steps, warmup=args.warmup)
        result["velocity_term"] = {"ms_per_step": round(ms_v, 4), "walker_evals_per_s": round(nw / (ms_v * 1e-3), 2),
                                   "note": "same step with dT_b times H / (dv_r/dr + H), |dv_r/dr| / H <= 0.2"}
        vb.close()

    if not args.no_scaling:
        log("HBM probes")
        probes = hbm_probes(xs, torch)
        result["hbm_probes"] = probes
        for k in ("ion", "axis_fwd", "axis_bins"):
            if k in result["kernels"]:
                result["kernels"][k]["frac_of_copy_probe"] = round(result["kernels"][k]["GBps"] /
                                                                   probes["copy"]["GBps"], 4)

    if not args.no_configs and args.workload == "batched-256":
        log("plain workloads (64^3 FP64, 128^3 x 3 z FP32) with the oracle beside them")
        result["plain_configs"] = section_plain_configs(xs, torch, amp, max(2, args.steps // 2))
        log("uneven BF16 workload (128^3 / 256^3 x 3 z, 256 walkers)")
        result["uneven_mix"] = section_workload(xs, torch, amp, "uneven-mix", max(2, args.steps // 3), graph=True)
        log("large workload (512^3 x 3 z, 1024 walkers)")
        result["large_512"] = section_workload(xs, torch, amp, "large-512", 1, graph=True, oracle_box=True)

    props = torch.cuda.get_device_properties(0)
    result["device"] = {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
                        "compute_units": props.multi_processor_count,
                        "lds_per_block_bytes": props.shared_memory_per_block,
                        "l2_bytes": getattr(props, "L2_cache_size", None),
                        "memory_gib": round(props.total_memory / 2 ** 30, 1)}
    if args.calibrate:
        # each probe launched twice (warm-up and one timed launch); bytes it moves per launch
        c = xs.Context(0, phys=xs.physics())
        result["calibration"] = {kind: c.probe_bandwidth(kind, (3800 << 20) + (64 << 10), reps=1)["bytes_per_launch"]
                                 for kind in ("read", "write", "copy", "tile")}
        c.close()
        log("calibration probes done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
