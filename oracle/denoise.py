"""Pre-denoising filters of the paper's experiments -- TEST INFRASTRUCTURE ONLY.

The paper smooths its data before CLAHE: a Gaussian filter with a standard
deviation per axis for the photoemission volume (Sec. IV.A) and a median
filter of window (2, 2, 2, 1) for the fluorescence microscopy volume
(Sec. IV.B).  The Gaussian is stated in ``denoise_oracle.c`` (plain C, loaded
with ctypes); the median here, in plain numpy.  Only the tests, the smoke
check and the benchmark's CPU leg may import this module; it imports nothing
from the product.

Readings of the median (the paper gives only the window):
  - window of k_a samples per axis at offsets -(k_a // 2) .. k_a - 1 - k_a // 2
    from the output sample (for k = 2: the sample and its predecessor);
  - of the N = prod k_a window values, the one of rank N // 2 (0-based) in
    ascending order: the median for odd N, the upper of the two middle values
    for even N;
  - outside the array the data continue by edge-repeating reflection, as for
    the Gaussian and the CLAHE padding;
  - the output has the input's dtype (a selection, exact).
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "denoise_oracle.c")
_LIB = os.path.join(_HERE, "libdenoise_oracle.so")
_DT = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float32): 2}
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _bind(lib):
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.denoise_oracle_gauss_radius.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.denoise_oracle_gauss_radius.restype = ctypes.c_int
    lib.denoise_oracle_gauss_weights.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    lib.denoise_oracle_gauss_weights.restype = ctypes.c_int
    lib.denoise_oracle_gaussian.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_void_p, f64p,
                                            ctypes.c_double, ctypes.c_void_p]
    lib.denoise_oracle_gaussian.restype = ctypes.c_int
    return lib


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def load_library(path: str):
    """Load another build of the Gaussian source (used by the mutation tests)."""
    return _bind(ctypes.CDLL(path))


def gauss_weights(sigma: float, truncate: float = 4.0, lib=None) -> np.ndarray:
    lib = _load(lib)
    r = lib.denoise_oracle_gauss_radius(sigma, truncate)
    w = np.zeros(2 * r + 1, np.float32)
    if lib.denoise_oracle_gauss_weights(sigma, truncate, w.ctypes.data) != r:
        raise ValueError("radius too large")
    return w


def gaussian(x: np.ndarray, sigma, truncate: float = 4.0, lib=None) -> np.ndarray:
    """Separable Gaussian smoothing (float32 result)."""
    lib = _load(lib)
    x = np.ascontiguousarray(x)
    if x.dtype not in _DT:
        raise TypeError(f"unsupported dtype {x.dtype}")
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float64), (x.ndim,)))
    sh = np.ascontiguousarray(np.asarray(x.shape, np.int64))
    out = np.empty(x.shape, np.float32)
    rc = lib.denoise_oracle_gaussian(x.ndim, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _DT[x.dtype],
                                     x.ctypes.data, sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     float(truncate), out.ctypes.data)
    if rc == 1:
        raise ValueError("invalid arguments")
    if rc:
        raise MemoryError("oracle allocation failed")
    return out


def reflect_index(i: np.ndarray, n: int) -> np.ndarray:
    """Edge-repeating reflection of integer positions into [0, n)."""
    i = np.mod(i, 2 * n)
    return np.where(i < n, i, 2 * n - 1 - i)


def median(x: np.ndarray, size) -> np.ndarray:
    """Median filter with the window and rank stated in the module notes."""
    x = np.asarray(x)
    size = [int(k) for k in size]
    if len(size) != x.ndim or min(size) < 1:
        raise ValueError("one window size >= 1 per axis")
    offsets = [range(-(k // 2), k - k // 2) for k in size]
    views = []
    for off in itertools.product(*offsets):
        idx = np.ix_(*[reflect_index(np.arange(n) + o, n) for n, o in zip(x.shape, off)])
        views.append(x[idx])
    stack = np.stack(views, axis=0)
    N = stack.shape[0]
    return np.sort(stack, axis=0)[N // 2].astype(x.dtype)


def median_at(x: np.ndarray, size, points: np.ndarray) -> np.ndarray:
    """The median filter's output at the given coordinates only ([m, ndim])."""
    x = np.asarray(x)
    size = [int(k) for k in size]
    pts = np.asarray(points, dtype=np.int64)
    offsets = [range(-(k // 2), k - k // 2) for k in size]
    vals = []
    for off in itertools.product(*offsets):
        idx = tuple(reflect_index(pts[:, a] + o, n) for a, (n, o) in enumerate(zip(x.shape, off)))
        vals.append(x[idx])
    stack = np.stack(vals, axis=0)
    return np.sort(stack, axis=0)[stack.shape[0] // 2].astype(x.dtype)
