"""ctypes binding of libmclahe.so (argument marshalling only).

Every step of the method runs in the library's HIP kernels; PyTorch provides
device memory and the current stream.  There is no CPU fallback: if the
library is not built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MCLAHE_LIB may name another build of the same library (e.g. an installed one)
LIB_PATH = os.environ.get("MCLAHE_LIB") or os.path.join(_HERE, "libmclahe.so")

SUCCESS, INVALID_VALUE, NOT_SUPPORTED, OUT_OF_MEMORY, WORKSPACE, HIP_ERROR = range(6)
U8, U16, F32 = 0, 1, 2
GLOBAL, KERNEL = 0, 1
# bytes of the static device scratch behind mclahe_run_noalloc (the header's
# MCLAHE_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 128 << 20


class MclaheError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("hist", "clipped", "lut", "range", "scale", "total")]


class Geometry(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32),
                ("pad", ctypes.c_int64 * 8), ("pad0", ctypes.c_int64 * 8),
                ("pad1", ctypes.c_int64 * 8), ("n_kernels_axis", ctypes.c_int64 * 8),
                ("n_kernels", ctypes.c_int64), ("kernel_voxels", ctypes.c_int64),
                ("clip_count", ctypes.c_int64), ("n_voxels", ctypes.c_int64),
                ("n_cells", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("hist_rows_split", "hist_copies", "hist_peel",
                                                "map_rows_split", "map_group", "map_unit_chunks")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Variant(ctypes.Structure):
    _fields_ = [("redistribution", ctypes.c_int32), ("rounds", ctypes.c_int32), ("centre", ctypes.c_int32)]


class PersistOpts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("max_spins", "abort_ticket", "flags", "reserved")]


PERSIST_ABORT_TICKET = 1

REDIST = {"equal": 0, "repeated": 1, "integer": 2}
CENTRE = {"middle": 0, "half": 1}


class MetricsResult(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 2), ("hi", ctypes.c_double * 2), ("mean", ctypes.c_double * 2),
                ("std", ctypes.c_double * 2), ("entropy", ctypes.c_double * 2), ("mse", ctypes.c_double),
                ("psnr", ctypes.c_double), ("count", ctypes.c_uint64)]

    def as_dict(self, two: bool) -> dict:
        k = 2 if two else 1
        d = {n: list(getattr(self, n))[:k] for n in ("lo", "hi", "mean", "std", "entropy")}
        if two:
            d["mse"], d["psnr"] = self.mse, self.psnr
        d["count"] = self.count
        return d


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1906_11355_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname.  Load it first
    # so that the library binds to the runtime that owns torch's streams and
    # allocations: one HIP runtime per process (a stream handle is only valid
    # in the runtime that created it).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "mclahe_plan": [ctypes.POINTER(P), ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_double,
                        ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int],
        "mclahe_plan_destroy": [P],
        "mclahe_plan_geometry": [P, ctypes.POINTER(Geometry)],
        "mclahe_plan_get_tuning": [P, ctypes.POINTER(Tuning)],
        "mclahe_plan_set_tuning": [P, ctypes.POINTER(Tuning)],
        "mclahe_plan_get_variant": [P, ctypes.POINTER(Variant)],
        "mclahe_plan_set_variant": [P, ctypes.POINTER(Variant)],
        "mclahe_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_workspace_layout": [P, ctypes.POINTER(Layout)],
        "mclahe_run": [P, P, P, P, ctypes.c_size_t, P],
        "mclahe_run_noalloc": [P, P, P, P],
        "mclahe_batched_workspace_size": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_batched_workspace_offsets": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_uint64)],
        "mclahe_run_batched": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P,
                               ctypes.c_size_t, P],
        "mclahe_batched_table_size": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_run_batched_split": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t), P, ctypes.c_size_t, P],
        "mclahe_batched_table": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P,
                                 P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_chunked_workspace_size": [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_run_chunked": [P, P, P, ctypes.c_int, P, ctypes.c_size_t, P],
        "mclahe_autotune_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_autotune": [P, P, P, P, ctypes.c_size_t, P],
        "mclahe_run_batched_persistent": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P,
                                          ctypes.c_size_t, ctypes.POINTER(PersistOpts), P],
        "mclahe_persistent_status": [ctypes.c_int, ctypes.POINTER(P), P, ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.POINTER(ctypes.c_uint32), P],
        "mclahe_plan_get_batch_tuning": [P, ctypes.POINTER(Tuning)],
        "mclahe_plan_set_batch_tuning": [P, ctypes.POINTER(Tuning)],
        "mclahe_autotune_batched_workspace_size": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_autotune_batched": [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P,
                                    ctypes.c_size_t, P],
        "mclahe_timer_create": [ctypes.POINTER(P), ctypes.c_int],
        "mclahe_timer_destroy": [P],
        "mclahe_timer_reset": [P],
        "mclahe_run_timed": [P, P, P, P, ctypes.c_size_t, P, P],
        "mclahe_timer_read": [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int)],
        "mclahe_metrics_workspace_size": [ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_gaussian_workspace_size": [ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_gaussian": [P, ctypes.c_int, ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                            P, P, ctypes.c_size_t, P],
        "mclahe_median": [P, ctypes.c_int, ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_int32), P, P],
        "mclahe_metrics": [P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                           P, P, P, ctypes.c_size_t, P],
        "mclahe_run_smoothed_workspace_size": [P, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                               ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_run_smoothed": [P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_double, P, P, P,
                                ctypes.c_size_t, P],
        "mclahe_run_metrics_workspace_size": [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
        "mclahe_run_metrics": [P, P, P, P, ctypes.c_size_t, ctypes.c_int, ctypes.c_double, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.mclahe_status_string.argtypes = [ctypes.c_int]
    lib.mclahe_status_string.restype = ctypes.c_char_p
    lib.mclahe_last_error.argtypes = []
    lib.mclahe_last_error.restype = ctypes.c_char_p
    lib.mclahe_version.argtypes = []
    lib.mclahe_version.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(status: int):
    if status != SUCCESS:
        msg = lib.mclahe_last_error().decode() or lib.mclahe_status_string(status).decode()
        raise MclaheError(status, msg)


def dtype_code(dt) -> int:
    """Map a numpy or torch dtype to the library's dtype code."""
    name = str(dt).replace("torch.", "")
    codes = {"uint8": U8, "uint16": U16, "float32": F32}
    if name not in codes:
        raise TypeError(f"unsupported dtype {dt} (uint8, uint16 or float32)")
    return codes[name]


def _mode_code(mode) -> int:
    if mode in (GLOBAL, "global", "ghr"):
        return GLOBAL
    if mode in (KERNEL, "kernel", "adaptive", "ahr"):
        return KERNEL
    raise ValueError(f"unknown range mode {mode!r}")


class Plan:
    """A validated problem: shape, kernel size, bins, clip limit, range mode, dtypes."""

    def __init__(self, shape: Sequence[int], kernel_size: Sequence[int], n_bins: int = 256,
                 clip_limit: float = 0.01, mode="global", user_range=None,
                 in_dtype="float32", out_dtype="float32"):
        self.shape = tuple(int(s) for s in shape)
        self.kernel_size = tuple(int(b) for b in kernel_size)
        self.n_bins = int(n_bins)
        self.clip_limit = float(clip_limit)
        self.mode = _mode_code(mode)
        self.in_code = in_dtype if isinstance(in_dtype, int) else dtype_code(in_dtype)
        self.out_code = out_dtype if isinstance(out_dtype, int) else dtype_code(out_dtype)
        self.user_range = None if user_range is None else (float(user_range[0]), float(user_range[1]))
        if len(self.kernel_size) != len(self.shape):
            raise MclaheError(INVALID_VALUE, "kernel_size must have one entry per dimension")
        sh = (ctypes.c_int64 * len(self.shape))(*self.shape)
        ks = (ctypes.c_int64 * len(self.kernel_size))(*self.kernel_size)
        ur = None if self.user_range is None else (ctypes.c_float * 2)(*self.user_range)
        h = ctypes.c_void_p()
        _check(lib.mclahe_plan(ctypes.byref(h), len(self.shape), sh, ks, self.n_bins,
                               ctypes.c_double(self.clip_limit), self.mode, ur, self.in_code,
                               self.out_code))
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.mclahe_plan_destroy(h)
            self._h = None

    def geometry(self) -> dict:
        g = Geometry()
        _check(lib.mclahe_plan_geometry(self._h, ctypes.byref(g)))
        D = g.ndim
        return dict(pad=list(g.pad[:D]), pad0=list(g.pad0[:D]), pad1=list(g.pad1[:D]),
                    n_kernels_axis=list(g.n_kernels_axis[:D]), n_kernels=g.n_kernels,
                    kernel_voxels=g.kernel_voxels, clip_count=g.clip_count,
                    n_voxels=g.n_voxels, n_cells=g.n_cells)

    def tuning(self) -> dict:
        t = Tuning()
        _check(lib.mclahe_plan_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{k: int(v) for k, v in kw.items()})
        _check(lib.mclahe_plan_set_tuning(self._h, ctypes.byref(t)))

    def batch_tuning(self) -> dict:
        t = Tuning()
        _check(lib.mclahe_plan_get_batch_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_batch_tuning(self, **kw):
        t = Tuning(**{k: int(v) for k, v in kw.items()})
        _check(lib.mclahe_plan_set_batch_tuning(self._h, ctypes.byref(t)))

    def set_variant(self, redistribution="equal", rounds: int = 1, centre="middle"):
        """Comparison variants of the method (default: the paper's)."""
        v = Variant(REDIST.get(redistribution, redistribution) if isinstance(redistribution, str) else int(redistribution),
                    int(rounds),
                    CENTRE.get(centre, centre) if isinstance(centre, str) else int(centre))
        _check(lib.mclahe_plan_set_variant(self._h, ctypes.byref(v)))

    def variant(self) -> dict:
        v = Variant()
        _check(lib.mclahe_plan_get_variant(self._h, ctypes.byref(v)))
        return {"redistribution": v.redistribution, "rounds": v.rounds, "centre": v.centre}

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(lib.mclahe_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def autotune_workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(lib.mclahe_autotune_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def layout(self) -> dict:
        l = Layout()
        _check(lib.mclahe_workspace_layout(self._h, ctypes.byref(l)))
        return {n: getattr(l, n) for n, _ in Layout._fields_}

    # ---- device calls (pointers are integers; stream is a hipStream_t) ----
    def run_ptr(self, d_in: int, d_out: int, d_ws: int, ws_bytes: int, stream: int = 0):
        _check(lib.mclahe_run(self._h, d_in, d_out, d_ws, ws_bytes, stream))

    def run_noalloc_ptr(self, d_in: int, d_out: int, stream: int = 0):
        """mclahe_run on the library's static device scratch (no workspace)."""
        _check(lib.mclahe_run_noalloc(self._h, d_in, d_out, stream))

    def _sigma(self, sigma):
        if len(sigma) != len(self.shape):
            raise ValueError("one sigma per axis")
        return (ctypes.c_double * len(sigma))(*[float(v) for v in sigma])

    def run_smoothed_workspace_size(self, sigma, truncate: float = 4.0) -> int:
        n = ctypes.c_size_t()
        _check(lib.mclahe_run_smoothed_workspace_size(self._h, self._sigma(sigma), float(truncate), ctypes.byref(n)))
        return n.value

    def run_smoothed_ptr(self, d_in: int, in_code: int, sigma, truncate: float, d_smooth: int, d_out: int,
                         d_ws: int, ws_bytes: int, stream: int = 0):
        """Gaussian smoothing of d_in into d_smooth (float), then the method on it into d_out."""
        _check(lib.mclahe_run_smoothed(self._h, d_in, int(in_code), self._sigma(sigma), float(truncate), d_smooth,
                                       d_out, d_ws, ws_bytes, stream))

    def run_metrics_workspace_size(self, n_bins: int = 256) -> int:
        n = ctypes.c_size_t()
        _check(lib.mclahe_run_metrics_workspace_size(self._h, int(n_bins), ctypes.byref(n)))
        return n.value

    def run_metrics_ptr(self, d_in: int, d_out: int, d_ws: int, ws_bytes: int, n_bins: int, peak: float,
                        d_result: int, d_hist, stream: int = 0):
        """mclahe_run plus the contrast metrics of input and output (one MetricsResult at d_result)."""
        _check(lib.mclahe_run_metrics(self._h, d_in, d_out, d_ws, ws_bytes, int(n_bins), float(peak), d_result,
                                      d_hist, stream))

    def chunked_workspace_size(self, slab_layers: int) -> int:
        n = ctypes.c_size_t()
        _check(lib.mclahe_chunked_workspace_size(self._h, int(slab_layers), ctypes.byref(n)))
        return n.value

    def run_chunked_ptr(self, h_in: int, h_out: int, slab_layers: int, d_ws: int, ws_bytes: int,
                        stream: int = 0):
        """Out-of-core run: h_in / h_out are HOST pointers, d_ws a device workspace."""
        _check(lib.mclahe_run_chunked(self._h, h_in, h_out, int(slab_layers), d_ws, ws_bytes, stream))

    def autotune_ptr(self, d_in: int, d_out: int, d_ws: int, ws_bytes: int, stream: int = 0):
        _check(lib.mclahe_autotune(self._h, d_in, d_out, d_ws, ws_bytes, stream))


class Timer:
    """Per-pass HIP-event timing of mclahe_run calls (range, hist, clip, map)."""

    def __init__(self, max_runs: int):
        h = ctypes.c_void_p()
        _check(lib.mclahe_timer_create(ctypes.byref(h), int(max_runs)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.mclahe_timer_destroy(h)
            self._h = None

    def reset(self):
        _check(lib.mclahe_timer_reset(self._h))

    def run(self, plan: "Plan", d_in: int, d_out: int, d_ws: int, ws_bytes: int, stream: int = 0):
        _check(lib.mclahe_run_timed(plan.handle, d_in, d_out, d_ws, ws_bytes, stream, self._h))

    def read(self):
        ms = (ctypes.c_float * 4)()
        n = ctypes.c_int()
        _check(lib.mclahe_timer_read(self._h, ms, ctypes.byref(n)))
        return dict(range=ms[0], hist=ms[1], clip=ms[2], map=ms[3], runs=n.value)


def _plans_array(plans):
    return (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])


def batched_workspace_size(plans) -> int:
    n = ctypes.c_size_t()
    _check(lib.mclahe_batched_workspace_size(len(plans), _plans_array(plans), ctypes.byref(n)))
    return n.value


def batched_workspace_offsets(plans):
    off = (ctypes.c_uint64 * len(plans))()
    _check(lib.mclahe_batched_workspace_offsets(len(plans), _plans_array(plans), off))
    return list(off)


def run_batched_ptr(plans, d_ins, d_outs, d_ws: int, ws_bytes: int, stream: int = 0):
    n = len(plans)
    ins = (ctypes.c_void_p * n)(*d_ins)
    outs = (ctypes.c_void_p * n)(*d_outs)
    _check(lib.mclahe_run_batched(n, _plans_array(plans), ins, outs, d_ws, ws_bytes, stream))


def autotune_batched_workspace_size(plans) -> int:
    n = ctypes.c_size_t()
    _check(lib.mclahe_autotune_batched_workspace_size(len(plans), _plans_array(plans), ctypes.byref(n)))
    return n.value


def autotune_batched_ptr(plans, d_ins, d_outs, d_ws: int, ws_bytes: int, stream: int = 0):
    """Tune the plans' batch decomposition together on these buffers (overwritten)."""
    n = len(plans)
    ins = (ctypes.c_void_p * n)(*d_ins)
    outs = (ctypes.c_void_p * n)(*d_outs)
    _check(lib.mclahe_autotune_batched(n, _plans_array(plans), ins, outs, d_ws, ws_bytes, stream))


def run_batched_persistent_ptr(plans, d_ins, d_outs, d_ws: int, ws_bytes: int, stream: int = 0,
                               max_spins: int = 0, abort_ticket=None):
    """mclahe_run_batched_persistent: the whole batch as one persistent launch."""
    n = len(plans)
    ins = (ctypes.c_void_p * n)(*d_ins)
    outs = (ctypes.c_void_p * n)(*d_outs)
    o = PersistOpts(int(max_spins), 0 if abort_ticket is None else int(abort_ticket),
                    0 if abort_ticket is None else PERSIST_ABORT_TICKET, 0)
    _check(lib.mclahe_run_batched_persistent(n, _plans_array(plans), ins, outs, d_ws, ws_bytes, ctypes.byref(o),
                                             stream))


def persistent_status(plans, d_ws: int, stream: int = 0):
    """(aborted, tickets) of the last persistent run on d_ws (synchronises the stream)."""
    a, t = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib.mclahe_persistent_status(len(plans), _plans_array(plans), d_ws, ctypes.byref(a), ctypes.byref(t),
                                        stream))
    return a.value, t.value


def batched_table_size(plans) -> int:
    n = ctypes.c_size_t()
    _check(lib.mclahe_batched_table_size(len(plans), _plans_array(plans), ctypes.byref(n)))
    return n.value


def run_batched_split_ptr(plans, d_ins, d_outs, d_wss, ws_bytes, d_table: int, table_bytes: int,
                          stream: int = 0):
    """mclahe_run_batched_split: one workspace per volume plus a table buffer."""
    n = len(plans)
    ins = (ctypes.c_void_p * n)(*d_ins)
    outs = (ctypes.c_void_p * n)(*d_outs)
    wss = (ctypes.c_void_p * n)(*d_wss)
    wsb = (ctypes.c_size_t * n)(*ws_bytes)
    _check(lib.mclahe_run_batched_split(n, _plans_array(plans), ins, outs, wss, wsb, d_table, table_bytes,
                                        stream))


def batched_table(plans, d_ins, d_outs, d_ws: int) -> bytes:
    """Host image of the descriptor table of a batched call (no device call)."""
    n = len(plans)
    ins = (ctypes.c_void_p * n)(*d_ins)
    outs = (ctypes.c_void_p * n)(*d_outs)
    need = ctypes.c_size_t()
    _check(lib.mclahe_batched_table(n, _plans_array(plans), ins, outs, d_ws, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib.mclahe_batched_table(n, _plans_array(plans), ins, outs, d_ws, buf, need.value,
                                    ctypes.byref(need)))
    return buf.raw


def metrics_workspace_size(nvox: int, n_bins: int) -> int:
    n = ctypes.c_size_t()
    _check(lib.mclahe_metrics_workspace_size(int(nvox), int(n_bins), ctypes.byref(n)))
    return n.value


def metrics_ptr(d_x: int, x_code: int, d_y, y_code: int, nvox: int, n_bins: int, peak: float,
                d_result: int, d_hist, d_ws: int, ws_bytes: int, stream: int = 0):
    """mclahe_metrics: d_result receives one MetricsResult (device memory)."""
    _check(lib.mclahe_metrics(d_x, int(x_code), d_y, int(y_code), int(nvox), int(n_bins), float(peak),
                              d_result, d_hist, d_ws, ws_bytes, stream))


def _shape_sigma(shape, sigma):
    D = len(shape)
    sh = (ctypes.c_int64 * D)(*[int(v) for v in shape])
    sg = (ctypes.c_double * D)(*[float(v) for v in sigma])
    return D, sh, sg


def gaussian_workspace_size(shape, sigma) -> int:
    D, sh, sg = _shape_sigma(shape, sigma)
    n = ctypes.c_size_t()
    _check(lib.mclahe_gaussian_workspace_size(D, sh, sg, ctypes.byref(n)))
    return n.value


def gaussian_ptr(d_in: int, in_code: int, shape, sigma, truncate: float, d_out: int, d_ws, ws_bytes: int,
                 stream: int = 0):
    """mclahe_gaussian: separable Gaussian smoothing into a float32 array."""
    D, sh, sg = _shape_sigma(shape, sigma)
    _check(lib.mclahe_gaussian(d_in, int(in_code), D, sh, sg, float(truncate), d_out, d_ws, ws_bytes, stream))


def median_ptr(d_in: int, code: int, shape, window, d_out: int, stream: int = 0):
    """mclahe_median: median filter, output in the input dtype."""
    D = len(shape)
    sh = (ctypes.c_int64 * D)(*[int(v) for v in shape])
    win = (ctypes.c_int32 * D)(*[int(v) for v in window])
    _check(lib.mclahe_median(d_in, int(code), D, sh, win, d_out, stream))


def version() -> str:
    return lib.mclahe_version().decode()


def status_string(s: int) -> str:
    return lib.mclahe_status_string(s).decode()


def last_error() -> str:
    return lib.mclahe_last_error().decode()
