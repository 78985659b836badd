"""Builds and drives the CPU-emulated xs21 library (test infrastructure only).

The same kernel and host sources as the GPU library are compiled with g++ and
AddressSanitizer against an emulated HIP runtime (tests/emu), then run through
a small driver.  This checks indexing, bounds and host logic without a GPU; it
is never used by the product path.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EMU = os.path.join(HERE, "emu")
# XS21_EMU_DEFINES: extra -D flags (space separated) for checking a build
# variant on the CPU; such builds get a binary of their own
EXTRA_DEFINES = os.environ.get("XS21_EMU_DEFINES", "").split()
BIN = os.path.join(EMU, "_build", "xs21_emu" + ("_" + "_".join(d.lstrip("-D").replace("=", "-")
                                                                for d in EXTRA_DEFINES) if EXTRA_DEFINES else ""))
SRC = [os.path.join(ROOT, "paper_1501_06576_amd", "csrc", f)
       for f in ("kernels.hip", "likelihood.hip", "two_population.hip", "sampler.hip", "probe.hip", "static_scratch.hip",
                 "api.cpp", "plan.cpp")]
NHIP = 6   # leading SRC entries that are HIP sources (compiled as C++ here)
EXTRA = [os.path.join(EMU, "emu_runtime.cpp"), os.path.join(EMU, "driver.cpp")]


def _stale() -> bool:
    if not os.path.exists(BIN):
        return True
    t = os.path.getmtime(BIN)
    deps = SRC + EXTRA + [os.path.join(EMU, "hip", "hip_runtime.h")]
    csrc = os.path.join(ROOT, "paper_1501_06576_amd", "csrc")
    deps += [os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hpp")]
    deps.append(os.path.join(ROOT, "include", "xs21.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build() -> str:
    if not _stale():
        return BIN
    os.makedirs(os.path.dirname(BIN), exist_ok=True)
    # XS21_PIPE_BLOCKS=3 / XS21_ION_BLOCKS=4: grid-stride kernels run 3 or 4
    # blocks, each over many items; XS21_BINS_LDS_BUDGET: FP64 binning at
    # N = 16 runs 1 bin per launch
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-pthread",
           "-DXS21_PIPE_BLOCKS=3", "-DXS21_ION_BLOCKS=4", "-DXS21_BINS_LDS_BUDGET=17664", *EXTRA_DEFINES,
           "-I", EMU, "-I", os.path.join(ROOT, "include"), "-x", "c++", *SRC[:NHIP], "-x", "none", *SRC[NHIP:], *EXTRA,
           "-o", BIN + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("emulation build failed:\n" + res.stderr[-4000:])
    os.replace(BIN + ".tmp", BIN)
    return BIN


class EmuRun:
    """Writes a driver spec, runs it, and reads back the outputs."""

    def __init__(self, storage="f32", max_walkers=8, max_plain=40, phys=None):
        self.dir = tempfile.mkdtemp(prefix="xs21emu_")
        self.lines = [f"storage {storage}", f"max_walkers {max_walkers}", f"max_plain {max_plain}",
                      f"out {self.dir}"]
        for k, v in (phys or {}).items():
            self.lines.append(f"phys {k} {v!r}")
        self.boxes = []
        self.walkers = []
        self.walkers2 = []

    def box(self, delta: np.ndarray, box_mpc: float, z: float, nbins: int):
        i = len(self.boxes)
        path = os.path.join(self.dir, f"box{i}.bin")
        delta.tofile(path)
        dt = "f64" if delta.dtype == np.float64 else "f32"
        self.lines.append(f"box {path} {dt} {delta.shape[0]} {box_mpc!r} {z!r} {nbins}")
        self.boxes.append((delta.shape[0], delta.dtype, nbins))
        return i

    def walker(self, zeta, r_mfp, t_vir):
        self.lines.append(f"walker {zeta!r} {r_mfp!r} {t_vir!r}")
        self.walkers.append((zeta, r_mfp, t_vir))
        return len(self.walkers) - 1

    def walker2(self, zeta0, r_mfp, t_feed, alpha, beta):
        self.lines.append(f"walker2 {zeta0!r} {r_mfp!r} {t_feed!r} {alpha!r} {beta!r}")
        self.walkers2.append((zeta0, r_mfp, t_feed, alpha, beta))
        return len(self.walkers2) - 1

    def cmd(self, line: str):
        self.lines.append(line)

    def write_array(self, name: str, a: np.ndarray) -> str:
        path = os.path.join(self.dir, name)
        a.tofile(path)
        return path

    def run(self, timeout=900):
        spec = os.path.join(self.dir, "spec.txt")
        with open(spec, "w") as fh:
            fh.write("\n".join(self.lines) + "\n")
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        res = subprocess.run([build(), spec], capture_output=True, text=True, timeout=timeout, env=env)
        if res.returncode != 0:
            raise RuntimeError(f"emulated run failed ({res.returncode}):\n{res.stdout[-2000:]}\n{res.stderr[-6000:]}")
        return res.stdout

    def read(self, name: str, dtype, shape=None) -> np.ndarray:
        a = np.fromfile(os.path.join(self.dir, name), dtype=dtype)
        return a.reshape(shape) if shape is not None else a
