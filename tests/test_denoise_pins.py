"""Pins of the pre-denoising oracle (oracle/denoise.py, oracle/denoise_oracle.c).

Gaussian: scipy's gaussian_filter (float64, reflect, truncate 4) within the
float32 rounding bound of the oracle's arithmetic; the radius and weight
ratios in closed form; the sum of the data, which an edge-repeating
reflection with a symmetric kernel preserves exactly; the impulse response,
the product of the 1-D kernels, exactly in float32.  Median: scipy's
median_filter, a pure-Python brute force, and hand-worked sequences for the
even window.  The last part plants one-line mistakes in copies of both
oracles and checks that the pins catch each.
"""
import importlib.util
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import denoise as DN

SIGMAS = [(0.7,), (1.3,), (0.7, 0.9), (0.7, 0.7, 0.9, 1.3), (0.0, 1.1, 0.6)]
SHAPES = {1: [(1,), (2,), (37,)], 2: [(2, 3), (19, 23)], 3: [(5, 6, 7), (1, 9, 4)],
          4: [(6, 5, 7, 9), (3, 2, 4, 11)]}


def _gauss_bound(x, sig, truncate=4.0):
    """Float32 error bound of the chained passes: per pass (2r+1) roundings of
    terms no larger than max|x|, plus the rounding of the weights."""
    m = float(np.abs(x).max()) or 1.0
    b = 0.0
    for s in sig:
        if s > 0:
            r = int(truncate * s + 0.5)
            b += (2 * r + 2) * 2.0 ** -24 * m
    return 2 * b + 1e-30


def _gauss_scipy_ok(mod):
    rng = np.random.default_rng(1)
    for sig in SIGMAS:
        for shape in SHAPES[len(sig)]:
            x = (rng.random(shape) * 100).astype(np.float32)
            g = mod.gaussian(x, sig)
            s = ndi.gaussian_filter(x.astype(np.float64), sig, mode="reflect", truncate=4.0)
            if g.dtype != np.float32 or g.shape == () or np.abs(g - s).max() > _gauss_bound(x, sig):
                return False
    return True


def _gauss_closed_forms_ok(mod):
    for s, r in ((0.7, 3), (0.9, 4), (1.3, 5), (0.1, 0), (2.0, 8)):
        w = mod.gauss_weights(s)
        if w.size != 2 * r + 1 or not np.array_equal(w, w[::-1]):
            return False
        if abs(float(w.astype(np.float64).sum()) - 1.0) > (2 * r + 1) * 2.0 ** -24:
            return False
        for j in range(1, r + 1):   # w_j / w_0 = exp(-j^2 / (2 sigma^2))
            if not math.isclose(float(w[r + j]) / float(w[r]), math.exp(-j * j / (2 * s * s)), rel_tol=3e-7):
                return False
    rng = np.random.default_rng(2)
    for sig, shape in (((1.3,), (2,)), ((0.9, 1.3), (7, 3)), ((0.7, 0.7, 0.9, 1.3), (9, 8, 10, 12))):
        x = rng.random(shape).astype(np.float32)
        g = mod.gaussian(x, sig)
        # reflection with a symmetric kernel keeps the sum of the data
        if not math.isclose(float(g.astype(np.float64).sum()), float(x.astype(np.float64).sum()),
                            rel_tol=4 * _gauss_bound(x, sig)):
            return False
    # impulse response: the product of the 1-D kernels, rounded once per pass
    sig = (0.7, 0.9, 1.3)
    x = np.zeros((15, 15, 15), np.float32)
    x[7, 7, 7] = 1
    g = mod.gaussian(x, sig)
    w = [mod.gauss_weights(s) for s in sig]
    exp = np.zeros_like(x)
    for i in range(-3, 4):
        for j in range(-4, 5):
            for k in range(-5, 6):
                exp[7 + i, 7 + j, 7 + k] = np.float32(np.float32(w[0][3 + i] * w[1][4 + j]) * w[2][5 + k])
    if not np.array_equal(g, exp):
        return False
    # integer input converts exactly; a zero sigma leaves its axis alone
    xi = rng.integers(0, 60000, size=(6, 7)).astype(np.uint16)
    if not np.array_equal(mod.gaussian(xi, (0.0, 0.0)), xi.astype(np.float32)):
        return False
    if not np.array_equal(mod.gaussian(xi, (0.8, 0.0)), mod.gaussian(xi.astype(np.float32), (0.8, 0.0))):
        return False
    return True


def _brute_median(x, size):
    out = np.empty_like(x)
    for p in np.ndindex(*x.shape):
        vals = []
        for off in np.ndindex(*size):
            q = []
            for a, (pa, o, k, n) in enumerate(zip(p, off, size, x.shape)):
                i = pa + o - k // 2
                while i < 0 or i >= n:               # edge-repeating reflection
                    i = -i - 1 if i < 0 else 2 * n - 1 - i
                q.append(i)
            vals.append(x[tuple(q)])
        vals.sort()
        out[p] = vals[len(vals) // 2]
    return out


def _median_ok(mod):
    rng = np.random.default_rng(3)
    for size, shape, dt in (((2, 2, 2, 1), (5, 4, 6, 3), np.uint8), ((3, 3), (7, 8), np.float32),
                            ((2,), (9,), np.uint16), ((4, 1, 3), (6, 2, 5), np.float32),
                            ((2, 2, 2, 1), (1, 3, 2, 2), np.uint8)):
        x = rng.integers(0, 200, size=shape).astype(dt)
        m = mod.median(x, size)
        if m.dtype != x.dtype or not np.array_equal(m, _brute_median(x, size)):
            return False
        if not np.array_equal(m, ndi.median_filter(x, size=size, mode="reflect")):
            return False
    # window (2,): the sample and its predecessor, upper value
    up = np.array([0, 10, 20, 30], np.uint8)
    if mod.median(up, (2,)).tolist() != [0, 10, 20, 30]:
        return False
    if mod.median(up[::-1].copy(), (2,)).tolist() != [30, 30, 20, 10]:
        return False
    if mod.median(np.full((3, 4), 7, np.uint8), (2, 2)).tolist() != np.full((3, 4), 7).tolist():
        return False
    return True


def test_gaussian_matches_scipy():
    assert _gauss_scipy_ok(DN)


def test_gaussian_closed_forms():
    assert _gauss_closed_forms_ok(DN)


def test_median_pins():
    assert _median_ok(DN)


def test_median_at_matches_whole_array():
    rng = np.random.default_rng(8)
    x = rng.integers(0, 256, size=(6, 7, 5, 3)).astype(np.uint8)
    full = DN.median(x, (2, 2, 2, 1))
    pts = np.array(list(np.ndindex(*x.shape)))
    assert np.array_equal(DN.median_at(x, (2, 2, 2, 1), pts), full.reshape(-1))


def test_gaussian_rejects():
    with pytest.raises(ValueError):
        DN.gaussian(np.zeros((4, 4), np.float32), (100.0, 1.0))    # radius over the oracle's limit
    with pytest.raises(ValueError):
        DN.median(np.zeros((4, 4), np.uint8), (2,))


# ------------------------------------------------------------------ mutants --
C_MUTANTS = {
    "sigma_not_squared": ("exp(-0.5 / (sigma * sigma) * (double)(j * j))", "exp(-0.5 / sigma * (double)(j * j))"),
    "radius_truncated": ("(int)(truncate * sigma + 0.5)", "(int)(truncate * sigma)"),
    "mirror_not_edge": ("return i < n ? i : period - 1 - i;", "return i < n ? i : period - i;"),
    "not_normalised": ("w[j] = (float)(phi[j] / sum);", "w[j] = (float)(phi[j]);"),
    "one_sided": ("for (int j = -r; j <= r; ++j) acc = __builtin_fmaf(", "for (int j = 0; j <= r; ++j) acc = __builtin_fmaf("),
}
C_SRC = os.path.join(os.path.dirname(DN.__file__), "denoise_oracle.c")


class _CMutant:
    """The oracle module's functions bound to a mutated build of the C source."""

    def __init__(self, name):
        src = open(C_SRC).read()
        old, new = C_MUTANTS[name]
        assert src.count(old) >= 1, f"mutant {name} does not apply"
        src = src.replace(old, new)
        d = tempfile.mkdtemp(prefix="denoise_mutant_")
        c, so = os.path.join(d, "m.c"), os.path.join(d, "m.so")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                               c, "-o", so, "-lm"])
        self.lib = DN.load_library(so)

    def gaussian(self, x, sigma, truncate=4.0):
        return DN.gaussian(x, sigma, truncate, lib=self.lib)

    def gauss_weights(self, sigma, truncate=4.0):
        return DN.gauss_weights(sigma, truncate, lib=self.lib)


PY_MUTANTS = {
    "median_lower": ("return np.sort(stack, axis=0)[N // 2]", "return np.sort(stack, axis=0)[(N - 1) // 2]"),
    "median_window_forward": ("offsets = [range(-(k // 2), k - k // 2) for k in size]",
                              "offsets = [range(0, k) for k in size]"),
    "median_mirror": ("return np.where(i < n, i, 2 * n - 1 - i)", "return np.where(i < n, i, 2 * n - 2 - i)"),
}


def _py_mutant(name):
    src = open(DN.__file__).read()
    old, new = PY_MUTANTS[name]
    assert src.count(old) >= 1, f"mutant {name} does not apply"
    d = tempfile.mkdtemp(prefix="denoise_pymutant_")
    path = os.path.join(d, "denoise_mutant.py")
    open(path, "w").write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("denoise_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _all_gauss(mod):
    try:
        return _gauss_scipy_ok(mod) and _gauss_closed_forms_ok(mod)
    except (ValueError, IndexError):
        return False


def _all_median(mod):
    try:
        return _median_ok(mod)
    except (ValueError, IndexError):
        return False


def test_real_denoise_oracle_passes():
    assert _all_gauss(DN) and _all_median(DN)


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_gaussian_mutant_is_caught(name):
    assert not _all_gauss(_CMutant(name)), f"mutant {name} slipped through the pins"


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_median_mutant_is_caught(name):
    assert not _all_median(_py_mutant(name)), f"mutant {name} slipped through the pins"
