"""Oracle evaluations of workload walkers in worker processes (test infrastructure).

The FP64 oracle takes seconds per walker and box at 256^3 and minutes at
512^3; full-size parity tests need many such evaluations, so they run in a
process pool beside the GPU work.  Workers regenerate the seeded workload
boxes themselves (the synthetic inputs are deterministic) and return the
binned outputs, and on request the per-cell flags (bit-packed), x_HI and dT_b
(as float32, which adds at most 6e-8 relative to values compared at 2e-5).
Nothing here holds method arithmetic: every value comes from ``oracle``.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor
from typing import Sequence

import numpy as np

_BOXES = {}


def _init(threads: int):
    import oracle.excursion_set as es
    es.FFT_WORKERS = threads


def _box(workload: str, amp: float, box_index: int):
    """One workload box (the whole workload's boxes are made together, as the tests do)."""
    import synth
    key = (workload, amp)
    if key not in _BOXES:
        _BOXES.clear()
        _BOXES[key] = synth.workload_boxes(synth.WORKLOADS[workload], amp)
    return _BOXES[key][box_index]


def _evaluate(args):
    import oracle
    import synth
    workload, amp, box_index, walker, radii, phys_kw, fields = args
    spec = synth.WORKLOADS[workload].boxes[box_index]
    ev = oracle.evaluate(_box(workload, amp, box_index), spec.box_mpc, spec.z, walker, radii, spec.n_bins,
                         oracle.Physics(**phys_kw))
    out = {"pk": ev.pk, "counts": ev.counts, "k_mean": ev.k_mean, "xhi_mean": ev.xhi_mean}
    if fields:
        out["flagged_bits"] = np.packbits(ev.flagged.reshape(-1))
        out["shape"] = ev.flagged.shape
        out["x_hi"] = ev.x_hi.astype(np.float32)
        out["dtb"] = ev.dtb.astype(np.float32)
    return out


def unpack_flags(res) -> np.ndarray:
    n = int(np.prod(res["shape"]))
    return np.unpackbits(res["flagged_bits"], count=n).astype(bool).reshape(res["shape"])


def pool(workers: int | None = None) -> ProcessPoolExecutor:
    """A spawn-context pool sized to the host (16 CPUs at most): 4 threads per worker."""
    cpus = max(1, min(len(os.sched_getaffinity(0)), 16))
    if workers is None:
        workers = max(1, cpus // 4)
    threads = max(1, cpus // workers)
    return ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"), initializer=_init,
                               initargs=(threads,))


def submit(ex: ProcessPoolExecutor, workload: str, amp: float, box_index: int, walker: Sequence[float],
           radii: Sequence[float], phys_kw: dict, fields: bool = False):
    return ex.submit(_evaluate, (workload, amp, box_index, tuple(float(v) for v in walker), list(radii), phys_kw,
                                 fields))
