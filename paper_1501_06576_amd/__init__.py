"""xs21: excursion-set ionisation -> 21 cm brightness -> P(k) on MI355X (gfx950).

Thin ctypes binding of libxs21.so.  It only marshals arguments: every step of
the path runs in the library's HIP kernels.  PyTorch provides device memory
(the workspace and output tensors) and the HIP stream.  There is no fallback:
if the built library is missing, importing the binding raises.

Paper: Greig & Mesinger 2015, 21CMMC (Section 2.1 ionisation field, eq. 1 and
eq. 3; Section 2.2 brightness temperature eq. 4 and the power spectrum).
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxs21.so")

F32, F64, BF16 = 0, 1, 2
KERNELS = ("rows_r2c", "rows_c2r", "axis_fwd", "axis_inv", "axis_bins", "ion", "finalize", "other", "plan")
_DTYPES = {"f32": F32, "f64": F64, "bf16": BF16}


class Xs21Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"xs21 status {status}: {msg}")
        self.status = status


class Physics(ctypes.Structure):
    _fields_ = [("delta_c", ctypes.c_double), ("omega_m", ctypes.c_double), ("omega_l", ctypes.c_double),
                ("h", ctypes.c_double), ("tb0_mK", ctypes.c_double), ("pk_amp", ctypes.c_double),
                ("pk_k0", ctypes.c_double), ("z_ref", ctypes.c_double), ("radius_step", ctypes.c_double),
                ("ladder_top", ctypes.c_double), ("mu", ctypes.c_double), ("mmin_form", ctypes.c_int32),
                ("velocity", ctypes.c_int32), ("dvdr_max", ctypes.c_double)]


class Walker(ctypes.Structure):
    _fields_ = [("zeta", ctypes.c_double), ("r_mfp", ctypes.c_double), ("t_vir", ctypes.c_double)]


class Sampler(ctypes.Structure):
    """Ensemble sampler settings: dim (3 or 5), uniform prior box lo/hi, stretch scale a."""
    _fields_ = [("dim", ctypes.c_int), ("lo", ctypes.c_double * 5), ("hi", ctypes.c_double * 5),
                ("a", ctypes.c_double)]


def sampler(lo: Sequence[float], hi: Sequence[float], a: float = 2.0) -> Sampler:
    """Sampler settings for walkers of len(lo) parameters (3: eq. 1 walkers, 5: eq. 9 walkers)."""
    s = Sampler()
    s.dim = len(lo)
    for i, (a_, b_) in enumerate(zip(lo, hi)):
        s.lo[i] = float(a_)
        s.hi[i] = float(b_)
    s.a = float(a)
    return s


class Tuning(ctypes.Structure):
    """Launch shapes for one grid size (0 / -1: defaults); see xs21_tuning."""
    _fields_ = [("ion_blocks", ctypes.c_int32), ("pipe_blocks", ctypes.c_int32), ("bins_blocks", ctypes.c_int32),
                ("flag_test", ctypes.c_int32), ("group", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Walker2(ctypes.Structure):
    """Two-population parameter set (zeta0, R_mfp, T_feed, alpha, beta) of eq. (9)."""
    _fields_ = [("zeta0", ctypes.c_double), ("r_mfp", ctypes.c_double), ("t_feed", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)

_SIGNATURES = {
    "xs21_last_error": (ctypes.c_char_p, []),
    "xs21_physics_default": (_I, [ctypes.POINTER(Physics)]),
    "xs21_create": (_I, [ctypes.POINTER(_P), _I, _P, ctypes.POINTER(Physics)]),
    "xs21_destroy": (_I, [_P]),
    "xs21_sync": (_I, [_P]),
    "xs21_add_box": (_I, [_P, _P, _I, _I, _I, _D, _D, _I, ctypes.POINTER(ctypes.c_int32)]),
    "xs21_box_radii": (_I, [_P, _I, _DP, _I, _IP]),
    "xs21_box_bins": (_I, [_P, _I, _DP, _DP]),
    "xs21_workspace_size": (_I, [_P, _I, _I, _I, ctypes.POINTER(ctypes.c_size_t)]),
    "xs21_prepare": (_I, [_P, _P, ctypes.c_size_t, _I, _I, _I]),
    "xs21_eval_batch": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, ctypes.POINTER(Walker), _I, _P, _P]),
    "xs21_eval": (_I, [_P, _I, ctypes.POINTER(Walker), _DP, _I, _P, _P, _DP, _DP, _DP, _DP]),
    "xs21_materialize": (_I, [_P, _I, ctypes.POINTER(Walker), _P, _P]),
    "xs21_eval_batch2": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, ctypes.POINTER(Walker2), _I, _P, _P]),
    "xs21_eval_batch_fields": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, ctypes.POINTER(Walker), _I, _P, _P, _I,
                                    _I, _P, _P]),
    "xs21_mcmc_lnprob": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, ctypes.POINTER(Sampler), _P, _I, _P]),
    "xs21_mcmc_step": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, ctypes.POINTER(Sampler), _P, _P, _I, _P, _P]),
    "xs21_materialize2": (_I, [_P, _I, ctypes.POINTER(Walker2), _P, _P]),
    "xs21_smoothed": (_I, [_P, _I, _I, _P]),
    "xs21_power_spectrum": (_I, [_P, _I, _P, _DP]),
    "xs21_resmooth": (_I, [_P, _I, _P]),
    "xs21_erfc_f32": (_I, [_P, _P, _P, ctypes.c_long]),
    "xs21_power_spectrum_static": (_I, [_P, _I, _P, _P]),
    "xs21_set_tuning": (_I, [_P, _I, _P]),
    "xs21_get_tuning": (_I, [_P, _I, _P]),
    "xs21_autotune": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, _P, _I, _I, ctypes.c_char_p, _P, _DP,
                           ctypes.POINTER(ctypes.c_int)]),
    "xs21_capture_begin": (_I, [_P]),
    "xs21_capture_end": (_I, [_P, ctypes.POINTER(_P)]),
    "xs21_graph_launch": (_I, [_P, _P]),
    "xs21_graph_destroy": (_I, [_P]),
    "xs21_probe_bandwidth": (_I, [_P, _I, _P, ctypes.c_size_t, _I, _DP, _DP]),
    "xs21_set_mock": (_I, [_P, _I, _DP, _DP, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "xs21_chi2": (_I, [_P, ctypes.POINTER(ctypes.c_int32), _I, _P, _I, _P]),
    "xs21_profile": (_I, [_P, _I]),
    "xs21_profile_read": (_I, [_P, _I, _DP, ctypes.POINTER(ctypes.c_longlong), _DP, _DP]),
    "xs21_plan_ladder": (_I, [_D, _D, _D, _DP, _I, _IP]),
    "xs21_plan_sigma2": (_I, [ctypes.POINTER(Physics), _D, _D, _DP]),
    "xs21_plan_walker": (_I, [ctypes.POINTER(Physics), _D, _DP, _I, ctypes.POINTER(Walker), _DP, _DP, _IP, _DP]),
    "xs21_plan_bins": (_I, [_I, _I, ctypes.POINTER(ctypes.c_int8)]),
}

_lib = None


def library() -> ctypes.CDLL:
    """Loads libxs21.so (built by paper_1501_06576_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1501_06576_amd.build` "
                              "(hipcc, gfx950); there is no fallback implementation")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        raise Xs21Error(status, library().xs21_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def physics(**overrides) -> Physics:
    p = Physics()
    _check(library().xs21_physics_default(ctypes.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


# ------------------------------------------------------------------ host planning

def plan_ladder(r_top: float, r_cell: float, step: float) -> List[float]:
    n = ctypes.c_int()
    _check(library().xs21_plan_ladder(r_top, r_cell, step, None, 0, ctypes.byref(n)))
    out = np.zeros(n.value)
    _check(library().xs21_plan_ladder(r_top, r_cell, step, _dptr(out), n.value, ctypes.byref(n)))
    return out.tolist()


def plan_sigma2(phys: Physics, radius: float, z: float) -> float:
    v = ctypes.c_double()
    _check(library().xs21_plan_sigma2(ctypes.byref(phys), radius, z, ctypes.byref(v)))
    return v.value


def plan_walker(phys: Physics, z: float, radii: Sequence[float], walker: Sequence[float]):
    r = np.ascontiguousarray(radii, dtype=np.float64)
    thr = np.zeros(len(r))
    ds = np.zeros(len(r))
    first = ctypes.c_int()
    mmin = ctypes.c_double()
    w = Walker(*map(float, walker))
    _check(library().xs21_plan_walker(ctypes.byref(phys), z, _dptr(r), len(r), ctypes.byref(w), _dptr(thr),
                                      _dptr(ds), ctypes.byref(first), ctypes.byref(mmin)))
    return {"thr": thr, "dsig2": ds, "first": first.value, "m_min": mmin.value}


def plan_bins(n: int, n_bins: int) -> np.ndarray:
    out = np.zeros(3 * (n // 2) ** 2 + 1, dtype=np.int8)
    _check(library().xs21_plan_bins(n, n_bins, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
    return out


# ------------------------------------------------------------------ device context

def _walkers_array(walkers, kind=None) -> Tuple[ctypes.Array, int]:
    kind = kind or Walker
    w = np.ascontiguousarray(np.asarray(walkers, dtype=np.float64).reshape(-1, len(kind._fields_)))
    arr = (kind * len(w))()
    ctypes.memmove(arr, w.ctypes.data, w.nbytes)
    return arr, len(w)


class Context:
    """One xs21 context on one GPU and one HIP stream (torch's current stream by default).

    Device tensors passed in must be ready on the context's stream; tensors the
    methods return are allocated on that stream and written there asynchronously:
    read them on that stream (make it torch's current stream) or after
    synchronising it."""

    def __init__(self, device: int = 0, stream=None, phys: Optional[Physics] = None):
        import torch  # device memory and streams only
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.phys = phys if phys is not None else physics()
        self._ctx = ctypes.c_void_p()
        _check(library().xs21_create(ctypes.byref(self._ctx), device, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(self.phys)))
        self.boxes: List[dict] = []
        self.workspace = None
        self._keep = []

    def _empty(self, shape, dtype):
        """An output tensor allocated on the context's stream, so that the caching
        allocator orders its reuse after the library's work on that stream."""
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(shape, dtype=dtype, device=self.device)

    def close(self):
        if self._ctx:
            library().xs21_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_box(self, delta, box_mpc: float, z: float, n_bins: int) -> int:
        """Registers a density box (numpy array on the host or torch tensor on this GPU)."""
        torch = self.torch
        h = ctypes.c_int32()
        if isinstance(delta, torch.Tensor) and delta.is_cuda:
            t = delta.contiguous()
            dt = F64 if t.dtype == torch.float64 else F32
            self._keep.append(t)  # must outlive prepare
            n = t.shape[0]
            _check(library().xs21_add_box(self._ctx, ctypes.c_void_p(t.data_ptr()), 1, dt, n, box_mpc, z, n_bins,
                                          ctypes.byref(h)))
        else:
            a = np.ascontiguousarray(delta)
            if a.dtype not in (np.float32, np.float64):
                raise TypeError("density box must be float32 or float64")
            dt = F64 if a.dtype == np.float64 else F32
            n = a.shape[0]
            _check(library().xs21_add_box(self._ctx, a.ctypes.data_as(ctypes.c_void_p), 0, dt, n, box_mpc, z,
                                          n_bins, ctypes.byref(h)))
        self.boxes.append({"n": n, "box": box_mpc, "z": z, "n_bins": n_bins, "dtype": dt})
        return h.value

    def radii(self, box: int) -> List[float]:
        n = ctypes.c_int()
        _check(library().xs21_box_radii(self._ctx, box, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value)
        _check(library().xs21_box_radii(self._ctx, box, _dptr(out), n.value, ctypes.byref(n)))
        return out.tolist()

    def bins(self, box: int):
        nb = self.boxes[box]["n_bins"]
        km = np.zeros(nb)
        cn = np.zeros(nb)
        _check(library().xs21_box_bins(self._ctx, box, _dptr(km), _dptr(cn)))
        return km, cn

    def workspace_size(self, storage="f32", max_walkers=64, max_plain_radii=40) -> int:
        v = ctypes.c_size_t()
        _check(library().xs21_workspace_size(self._ctx, _DTYPES[storage], max_walkers, max_plain_radii,
                                             ctypes.byref(v)))
        return v.value

    def prepare(self, storage="f32", max_walkers=64, max_plain_radii=40):
        """Allocates the workspace (one torch uint8 tensor) and builds the resident smoothed boxes."""
        torch = self.torch
        nbytes = self.workspace_size(storage, max_walkers, max_plain_radii)
        ws = self._empty(nbytes + 256, torch.uint8)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        _check(library().xs21_prepare(self._ctx, ctypes.c_void_p(ws.data_ptr() + off), nbytes, _DTYPES[storage],
                                      max_walkers, max_plain_radii))
        self._keep.clear()

    def eval_batch(self, boxes: Sequence[int], walkers, pk=None, xhi=None):
        """Batched evaluation; returns device tensors pk [nw, nb, nbmax] and xhi [nw, nb] (float64)."""
        return self._batch(boxes, walkers, pk, xhi, Walker, library().xs21_eval_batch)

    def eval_batch_fields(self, boxes: Sequence[int], walkers, field_walker: int, field_box: int, pk=None,
                          xhi=None):
        """eval_batch that also returns the x_HI and dT_b boxes of walkers[field_walker] on
        boxes[field_box], written by that walker's batched ionisation launch."""
        torch = self.torch
        bx = (ctypes.c_int32 * len(boxes))(*boxes)
        warr, nw = _walkers_array(walkers, Walker)
        nbmax = max(self.boxes[b]["n_bins"] for b in boxes)
        if pk is None:
            pk = self._empty((nw, len(boxes), nbmax), torch.float64)
        if xhi is None:
            xhi = self._empty((nw, len(boxes)), torch.float64)
        b = self.boxes[boxes[field_box]] if 0 <= field_box < len(boxes) else self.boxes[boxes[0]]
        n = b["n"]
        td = torch.float64 if b["dtype"] == F64 else torch.float32
        fx = self._empty((n, n, n), td)
        fd = self._empty((n, n, n), td)
        _check(library().xs21_eval_batch_fields(self._ctx, bx, len(boxes), warr, nw, ctypes.c_void_p(pk.data_ptr()),
                                                ctypes.c_void_p(xhi.data_ptr()), int(field_walker), int(field_box),
                                                ctypes.c_void_p(fx.data_ptr()), ctypes.c_void_p(fd.data_ptr())))
        return pk, xhi, fx, fd

    def eval_batch2(self, boxes: Sequence[int], walkers, pk=None, xhi=None):
        """eval_batch for two-population walkers (zeta0, R_mfp, T_feed, alpha, beta), eq. (9)."""
        return self._batch(boxes, walkers, pk, xhi, Walker2, library().xs21_eval_batch2)

    def _batch(self, boxes, walkers, pk, xhi, kind, fn):
        torch = self.torch
        bx = (ctypes.c_int32 * len(boxes))(*boxes)
        warr, nw = _walkers_array(walkers, kind)
        nbmax = max(self.boxes[b]["n_bins"] for b in boxes)
        if pk is None:
            pk = self._empty((nw, len(boxes), nbmax), torch.float64)
        if xhi is None:
            xhi = self._empty((nw, len(boxes)), torch.float64)
        _check(fn(self._ctx, bx, len(boxes), warr, nw, ctypes.c_void_p(pk.data_ptr()), ctypes.c_void_p(xhi.data_ptr())))
        return pk, xhi

    def eval(self, box: int, walker, radii=None, fields=True) -> dict:
        """Plain per-walker evaluation (recomputes every smoothed box); host outputs."""
        b = self.boxes[box]
        n, nb = b["n"], b["n_bins"]
        dt = np.float64 if b["dtype"] == F64 else np.float32
        w = Walker(*map(float, walker))
        r = None if radii is None else np.ascontiguousarray(radii, dtype=np.float64)
        x_hi = np.empty((n, n, n), dtype=dt) if fields else None
        dtb = np.empty((n, n, n), dtype=dt) if fields else None
        pk = np.zeros(nb)
        km = np.zeros(nb)
        cn = np.zeros(nb)
        xm = ctypes.c_double()
        _check(library().xs21_eval(self._ctx, box, ctypes.byref(w), None if r is None else _dptr(r),
                                   0 if r is None else len(r),
                                   None if x_hi is None else x_hi.ctypes.data_as(ctypes.c_void_p),
                                   None if dtb is None else dtb.ctypes.data_as(ctypes.c_void_p),
                                   _dptr(pk), _dptr(km), _dptr(cn), ctypes.byref(xm)))
        return {"x_hi": x_hi, "dtb": dtb, "pk": pk, "k_mean": km, "counts": cn, "xhi_mean": xm.value}

    def _dev(self, t, shape, dtype, name):
        """The C-ABI cannot check device buffer sizes: check dtype, device, layout and shape here."""
        if (t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape)):
            raise ValueError(f"{name}: need a contiguous {dtype} device tensor of shape {tuple(shape)}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")

    def mcmc_lnprob(self, boxes: Sequence[int], spec: Sampler, x, lp=None):
        """ln p (-chi^2/2 in the prior, -inf outside) of walkers x (device float64 [nw, dim])."""
        bx = (ctypes.c_int32 * len(boxes))(*boxes)
        nw = int(x.shape[0])
        f64 = self.torch.float64
        self._dev(x, (nw, spec.dim), f64, "x")
        if lp is None:
            lp = self._empty(nw, f64)
        self._dev(lp, (nw,), f64, "lp")
        _check(library().xs21_mcmc_lnprob(self._ctx, bx, len(boxes), ctypes.byref(spec),
                                          ctypes.c_void_p(x.data_ptr()), nw, ctypes.c_void_p(lp.data_ptr())))
        return lp

    def mcmc_step(self, boxes: Sequence[int], spec: Sampler, x, lp, u, accepted=None):
        """One stretch-move ensemble step in place on x / lp (device float64); u: device float64
        [2, nw/2, 3] uniforms; accepted: optional device int32 [nw]."""
        bx = (ctypes.c_int32 * len(boxes))(*boxes)
        nw = int(x.shape[0])
        f64 = self.torch.float64
        self._dev(x, (nw, spec.dim), f64, "x")
        self._dev(lp, (nw,), f64, "lp")
        self._dev(u, (2, nw // 2, 3), f64, "u")
        if accepted is not None:
            self._dev(accepted, (nw,), self.torch.int32, "accepted")
        acc = ctypes.c_void_p(accepted.data_ptr()) if accepted is not None else None
        _check(library().xs21_mcmc_step(self._ctx, bx, len(boxes), ctypes.byref(spec), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(lp.data_ptr()), int(x.shape[0]),
                                        ctypes.c_void_p(u.data_ptr()), acc))

    def materialize(self, box: int, walker):
        """x_HI and dT_b of one walker from the resident smoothed boxes (device tensors)."""
        return self._fields(box, Walker(*map(float, walker)), library().xs21_materialize)

    def materialize2(self, box: int, walker):
        """materialize for one two-population walker (zeta0, R_mfp, T_feed, alpha, beta)."""
        return self._fields(box, Walker2(*map(float, walker)), library().xs21_materialize2)

    def _fields(self, box, w, fn):
        torch = self.torch
        b = self.boxes[box]
        n = b["n"]
        td = torch.float64 if b["dtype"] == F64 else torch.float32
        x = self._empty((n, n, n), td)
        d = self._empty((n, n, n), td)
        _check(fn(self._ctx, box, ctypes.byref(w), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(d.data_ptr())))
        return x, d

    def smoothed(self, box: int, index: int):
        torch = self.torch
        b = self.boxes[box]
        n = b["n"]
        td = torch.float64 if b["dtype"] == F64 else torch.float32
        out = self._empty((n, n, n), td)
        _check(library().xs21_smoothed(self._ctx, box, index, ctypes.c_void_p(out.data_ptr())))
        return out

    def power_spectrum(self, box: int, field) -> np.ndarray:
        b = self.boxes[box]
        pk = np.zeros(b["n_bins"])
        f = field.contiguous()
        _check(library().xs21_power_spectrum(self._ctx, box, ctypes.c_void_p(f.data_ptr()), _dptr(pk)))
        return pk

    def probe_bandwidth(self, kind: str, nbytes: int = 1 << 30, reps: int = 5) -> dict:
        """HBM probe ("read", "write", "copy", "tile"): GB/s of bytes read + written per launch."""
        k = {"read": 0, "write": 1, "copy": 2, "tile": 3}[kind]
        buf = self._empty(nbytes + 256, self.torch.uint8)
        off = (-buf.data_ptr()) % 256
        g = ctypes.c_double()
        m = ctypes.c_double()
        _check(library().xs21_probe_bandwidth(self._ctx, k, ctypes.c_void_p(buf.data_ptr() + off), nbytes, reps,
                                              ctypes.byref(g), ctypes.byref(m)))
        del buf
        return {"GBps": g.value, "bytes_per_launch": m.value}

    def erfc_f32(self, x):
        """erfc of a float32 device tensor by the FP32 routine of the ionisation pass."""
        t = x.contiguous()
        if t.dtype != self.torch.float32 or not t.is_cuda:
            raise ValueError("erfc_f32 needs a float32 device tensor")
        y = self._empty(t.shape, t.dtype)
        _check(library().xs21_erfc_f32(self._ctx, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       t.numel()))
        return y

    def set_tuning(self, n: int, **shapes):
        """Launch shapes for boxes of n^3 cells (keys of Tuning; none given: back to defaults)."""
        if not shapes:
            _check(library().xs21_set_tuning(self._ctx, n, None))
            return
        t = Tuning(0, 0, 0, -1, 0)
        for k, v in shapes.items():
            setattr(t, k, int(v))
        _check(library().xs21_set_tuning(self._ctx, n, ctypes.byref(t)))

    def get_tuning(self, n: int) -> dict:
        t = Tuning()
        _check(library().xs21_get_tuning(self._ctx, n, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, boxes: Sequence[int], walkers, reps: int = 3, cache_path: Optional[str] = None) -> dict:
        """Times candidate launch shapes on eval_batch(boxes, walkers) and sets the best; with a
        cache path, reuses / stores the choice there."""
        bx = (ctypes.c_int32 * len(boxes))(*boxes)
        warr, nw = _walkers_array(walkers, Walker)
        t = Tuning()
        ms = ctypes.c_double()
        cached = ctypes.c_int()
        _check(library().xs21_autotune(self._ctx, bx, len(boxes), warr, nw, reps,
                                       None if cache_path is None else cache_path.encode(), ctypes.byref(t),
                                       ctypes.byref(ms), ctypes.byref(cached)))
        return {"tuning": t.as_dict(), "best_ms": ms.value, "from_cache": bool(cached.value)}

    def capture_begin(self):
        _check(library().xs21_capture_begin(self._ctx))

    def capture_end(self) -> "Graph":
        g = ctypes.c_void_p()
        _check(library().xs21_capture_end(self._ctx, ctypes.byref(g)))
        return Graph(self, g)

    def power_spectrum_static(self, box: int, field, pk=None):
        """P(k) of a device field through the allocation-free entry point (static device
        scratch); returns a device float64 tensor of n_bins (asynchronous)."""
        b = self.boxes[box]
        f = field.contiguous()
        if pk is None:
            pk = self._empty(b["n_bins"], self.torch.float64)
        self._dev(pk, (b["n_bins"],), self.torch.float64, "pk")
        _check(library().xs21_power_spectrum_static(self._ctx, box, ctypes.c_void_p(f.data_ptr()),
                                                    ctypes.c_void_p(pk.data_ptr())))
        return pk

    def set_mock(self, box: int, delta2_mock, noise_sigma=None, model_err=0.25, k_lo=0.15, k_hi=1.0):
        """Mock Delta^2 (and optional noise) of `box` for the chi^2 epilogue; host arrays of n_bins."""
        nb = self.boxes[box]["n_bins"]
        m = np.ascontiguousarray(delta2_mock, dtype=np.float64)
        if m.shape != (nb,):
            raise ValueError(f"mock needs {nb} bins")
        ns = None
        if noise_sigma is not None:
            ns = np.ascontiguousarray(noise_sigma, dtype=np.float64)
            if ns.shape != (nb,):
                raise ValueError(f"noise needs {nb} bins")
        _check(library().xs21_set_mock(self._ctx, box, _dptr(m), None if ns is None else _dptr(ns),
                                       float(model_err), float(k_lo), float(k_hi)))

    def chi2(self, boxes: Sequence[int], pk, out=None):
        """chi^2 per walker (device float64 [nw]) from the pk tensor eval_batch wrote for `boxes`."""
        bx = (ctypes.c_int32 * len(boxes))(*boxes)
        nw = pk.shape[0]
        if out is None:
            out = self._empty(nw, self.torch.float64)
        _check(library().xs21_chi2(self._ctx, bx, len(boxes), ctypes.c_void_p(pk.data_ptr()), nw,
                                   ctypes.c_void_p(out.data_ptr())))
        return out

    def resmooth(self, box: int, new_delta=None):
        """Recomputes the forward FFT and the smoothed boxes of `box` (optionally from new device data)."""
        ptr = None if new_delta is None else ctypes.c_void_p(new_delta.data_ptr())
        _check(library().xs21_resmooth(self._ctx, box, ptr))

    def profile(self, enable: bool = True):
        _check(library().xs21_profile(self._ctx, 1 if enable else 0))

    def profile_read(self) -> dict:
        """Per kernel class: total ms, launches, algorithmic bytes and vector ops since profile(True)."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            by = ctypes.c_double()
            op = ctypes.c_double()
            _check(library().xs21_profile_read(self._ctx, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by),
                                               ctypes.byref(op)))
            out[name] = {"ms": ms.value, "launches": n.value, "bytes": by.value, "ops": op.value}
        return out

    def sync(self):
        _check(library().xs21_sync(self._ctx))


class Graph:
    """A launch graph recorded on a context's stream (xs21_capture_begin / _end)."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self._g = handle

    def launch(self):
        _check(library().xs21_graph_launch(self.ctx._ctx, self._g))

    def close(self):
        if self._g:
            library().xs21_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
