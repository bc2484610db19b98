"""CPU oracle for multidimensional CLAHE -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain C implementation in ``mclahe_oracle.c`` (Algorithm 1,
Eqs. 1-2, Sec. III.C and III.D of Stimper et al., "Multidimensional Contrast
Limited Adaptive Histogram Equalization", 2019), loaded with ctypes.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the product library never does, and this package never imports
the product.  The contrast metrics the paper judges its results by are stated
separately, in plain numpy, in ``oracle/metrics.py``, and the pre-denoising
filters of the paper's experiments in ``oracle/denoise.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mclahe_oracle.c")
_LIB = os.path.join(_HERE, "libmclahe_oracle.so")

U8, U16, F32 = 0, 1, 2
GLOBAL, KERNEL = 0, 1
EQUAL, REPEATED, INTEGER = 0, 1, 2      # redistribution variants
_DT = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16, np.dtype(np.float32): F32}
_NP = {U8: np.uint8, U16: np.uint16, F32: np.float32}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE arithmetic, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    from . import denoise
    denoise.build(force)
    return _LIB


def _bind(lib):
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.mclahe_oracle_geometry.argtypes = [ctypes.c_int, i64p, i64p, i64p, i64p, i64p, i64p]
    lib.mclahe_oracle_geometry.restype = ctypes.c_int
    lib.mclahe_oracle_run.argtypes = [
        ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.mclahe_oracle_run.restype = ctypes.c_int
    lib.mclahe_oracle_run_variant.argtypes = lib.mclahe_oracle_run.argtypes + [ctypes.c_int] * 3
    lib.mclahe_oracle_run_variant.restype = ctypes.c_int
    return lib


def _load(lib=None):
    """The default oracle library, or ``lib`` if one is given."""
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use (from the calling thread)."""
    return int(ctypes.CDLL(_load()._name).omp_get_max_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle's later parallel loops."""
    ctypes.CDLL(_load()._name).omp_set_num_threads(int(n))


def load_library(path: str):
    """Load another build of the oracle source (used by the mutation tests)."""
    return _bind(ctypes.CDLL(path))


def _i64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def geometry(shape, kernel_size, lib=None):
    """Eq. 1-2: (pad, pad0, pad1, n_kernels) per axis."""
    lib = _load(lib)
    D = len(shape)
    sh, shp = _i64(shape)
    ks, ksp = _i64(kernel_size)
    outs = [np.zeros(D, np.int64) for _ in range(4)]
    ptrs = [o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for o in outs]
    rc = lib.mclahe_oracle_geometry(D, shp, ksp, *ptrs)
    if rc:
        raise ValueError("invalid geometry")
    return tuple(outs)


def run(x: np.ndarray, kernel_size, n_bins: int, clip_limit: float,
        mode: int = GLOBAL, user_range=None, out_dtype=np.float32,
        want_f64: bool = False, lib=None, redistribution: int = EQUAL, rounds: int = 1,
        centre_half: bool = False):
    """Run the oracle; returns a dict of hist, clipped, lut, range, out (+out_f64).

    redistribution, rounds and centre_half select the comparison variants
    stated in the C source (defaults: the paper's method)."""
    lib = _load(lib)
    x = np.ascontiguousarray(x)
    if x.dtype not in _DT:
        raise TypeError(f"unsupported input dtype {x.dtype}")
    D = x.ndim
    pad, pad0, pad1, nk = geometry(x.shape, kernel_size, lib)
    nker = int(np.prod(nk))
    od = _DT[np.dtype(out_dtype)]
    out = np.empty(x.shape, dtype=_NP[od])
    hist = np.empty((nker, n_bins), np.int64)
    clipped = np.empty((nker, n_bins), np.int64)
    lut = np.empty((nker, n_bins), np.float32)
    rng = np.empty((nker, 2) if mode == KERNEL else (2,), np.float32)
    f64 = np.empty(x.shape, np.float64) if want_f64 else None
    ur = None
    if user_range is not None:
        ur = np.asarray(user_range, dtype=np.float32)
    sh, shp = _i64(x.shape)
    ks, ksp = _i64(kernel_size)
    rc = lib.mclahe_oracle_run_variant(
        D, shp, ksp, int(n_bins), ctypes.c_double(clip_limit), int(mode),
        None if ur is None else ur.ctypes.data, _DT[x.dtype], x.ctypes.data, od,
        out.ctypes.data, hist.ctypes.data, clipped.ctypes.data, lut.ctypes.data,
        rng.ctypes.data, None if f64 is None else f64.ctypes.data,
        int(redistribution), int(rounds), int(bool(centre_half)))
    if rc == 1:
        raise ValueError("invalid arguments")
    if rc:
        raise MemoryError("oracle allocation failed")
    res = dict(hist=hist, clipped=clipped, lut=lut, range=rng, out=out,
               n_kernels=nk, pad=pad, pad0=pad0, pad1=pad1)
    if f64 is not None:
        res["out_f64"] = f64
    return res
