"""Pins of the contrast-metric oracle (oracle/metrics.py).

Checked against what the paper prints (the MSE/PSNR pairs of its two metric
tables, tests/golden/psnr_tables.json), closed forms of ramps and two-level
volumes, the textbook entropy of known distributions, scipy's entropy
routine, invariants (affine invariance, symmetry) and the independent float32
binning model of the CLAHE pins.  A second part plants one-line mistakes in a
copy of the oracle and checks that the pins catch each of them.
"""
import importlib.util
import json
import math
import os
import tempfile

import numpy as np
import pytest
import scipy.stats

from exact_model import f32_bin
from oracle import metrics as M

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "psnr_tables.json")))


def _psnr_rows_ok(mod):
    for name, m, unit, p, mdec, pdec in GOLD["rows"]:
        mse = m * unit
        half = 0.5 * 10.0 ** (-mdec) * unit          # rounding of the printed MSE
        tol = 10 * math.log10(1 + half / (mse - half)) + 0.5 * 10.0 ** (-pdec) + 1e-9
        if not abs(mod.psnr(mse, mod.PAPER_PSNR_PEAK) - p) <= tol:
            return False
    return True


def _closed_forms_ok(mod):
    N = 1001
    ramp = np.arange(N, dtype=np.float32)
    # normalised ramp i/(N-1): variance (N+1) / (12 (N-1))
    if not math.isclose(mod.std(ramp) ** 2, (N + 1) / (12 * (N - 1)), rel_tol=1e-12):
        return False
    # against the reversed ramp the difference is 2u - 1: MSE = (N+1) / (3 (N-1))
    if not math.isclose(mod.mse(ramp, ramp[::-1].copy()), (N + 1) / (3 * (N - 1)), rel_tol=1e-12):
        return False
    # against a constant volume (normalised to 0): mean(u^2) = (2N-1) / (6 (N-1))
    if not math.isclose(mod.mse(ramp, np.full(N, 7, np.float32)), (2 * N - 1) / (6 * (N - 1)),
                        rel_tol=1e-12):
        return False
    # two equal halves at the extremes: std 1/2, entropy 1 bit
    two = np.array([3.0] * 50 + [9.0] * 50, np.float32)
    if not math.isclose(mod.std(two), 0.5, rel_tol=1e-15):
        return False
    if not math.isclose(mod.entropy_bits(mod.grey_histogram(two, 256)), 1.0, rel_tol=1e-15):
        return False
    # one voxel per grey level j = 0..n-1 repeated k times: uniform, log2 n bits
    n, k = 64, 3
    lev = np.repeat(np.arange(n, dtype=np.float32), k)
    if mod.grey_histogram(lev, n).tolist() != [k] * n:
        return False
    if not math.isclose(mod.entropy_bits(mod.grey_histogram(lev, n)), math.log2(n), rel_tol=1e-15):
        return False
    # dyadic distribution 8:4:2:1:1 over 16 voxels: 15/8 bits
    dy = np.array([0] * 8 + [1] * 4 + [2] * 2 + [3] + [4], np.uint8)
    if mod.grey_histogram(dy, 5).tolist() != [8, 4, 2, 1, 1]:
        return False
    if not math.isclose(mod.entropy_bits(mod.grey_histogram(dy, 5)), 15 / 8, rel_tol=1e-15):
        return False
    # constant volume: no contrast, no information
    c = np.full((4, 5), 2.5, np.float32)
    if mod.std(c) != 0.0 or mod.entropy_bits(mod.grey_histogram(c, 16)) != 0.0:
        return False
    return True


def _invariants_ok(mod):
    rng = np.random.default_rng(11)
    x = rng.poisson(3.0, size=(6, 7, 5)).astype(np.float32)
    y = rng.random((6, 7, 5)).astype(np.float32)
    if mod.mse(x, x) != 0.0 or mod.psnr(0.0, 1.0) != float("inf"):
        return False
    if not math.isclose(mod.mse(x, y), mod.mse(y, x), rel_tol=1e-15):
        return False
    # min-max normalisation: positive affine maps of either volume change nothing
    # (the maps are exact in float32 here: powers of two and small integers)
    if not math.isclose(mod.mse(4 * x + 3, y), mod.mse(x, y), rel_tol=1e-12):
        return False
    if not math.isclose(mod.std(0.25 * x - 2), mod.std(x), rel_tol=1e-12):
        return False
    # the histogram is that of the CLAHE float32 binning over the global range
    lo, hi = float(x.min()), float(x.max())
    ref = np.zeros(32, np.int64)
    for v in x.ravel():
        ref[f32_bin(v, lo, hi, 32)] += 1
    if mod.grey_histogram(x, 32).tolist() != ref.tolist():
        return False
    # entropy of a general histogram: scipy's routine
    h = mod.grey_histogram(x, 32)
    if not math.isclose(mod.entropy_bits(h), scipy.stats.entropy(h, base=2), rel_tol=1e-12):
        return False
    # the combined call reports the same numbers as the parts
    r = mod.metrics(x, y, n_bins=32, peak=2.0)
    if r["std"] != [mod.std(x), mod.std(y)] or r["mse"] != mod.mse(x, y):
        return False
    if not math.isclose(r["psnr"], 10 * math.log10(4.0 / r["mse"]), rel_tol=1e-15):
        return False
    return True


def test_psnr_reproduces_both_tables():
    assert _psnr_rows_ok(M)


def test_psnr_rejects_other_peaks():
    # the reading is sharp: one binary order of magnitude either way misses
    class Off:
        PAPER_PSNR_PEAK = 2.0 ** 22
        psnr = staticmethod(M.psnr)
    assert not _psnr_rows_ok(Off)
    Off.PAPER_PSNR_PEAK = 2.0 ** 24
    assert not _psnr_rows_ok(Off)


def test_closed_forms():
    assert _closed_forms_ok(M)


def test_invariants():
    assert _invariants_ok(M)


def test_metrics_shape_mismatch():
    with pytest.raises(ValueError):
        M.mse(np.zeros(3, np.float32), np.zeros(4, np.float32))


# ------------------------------------------------------------------ mutants --
MUTANTS = {
    "psnr_20log": ("10.0 * np.log10(peak * peak / mse_value)", "20.0 * np.log10(peak * peak / mse_value)"),
    "psnr_peak_not_squared": ("peak * peak / mse_value", "peak / mse_value"),
    "entropy_natural_log": ("np.log2(p)", "np.log(p)"),
    "std_sample": ("np.mean((u - u.mean()) ** 2)", "np.sum((u - u.mean()) ** 2) / (u.size - 1)"),
    "std_not_centred": ("np.mean((u - u.mean()) ** 2)", "np.mean(u ** 2)"),
    "mse_not_normalised": ("d = normalise(x) - normalise(y)", "d = np.asarray(x, np.float64) - np.asarray(y, np.float64)"),
    "mse_root": ("return float(np.mean(d * d))", "return float(np.sqrt(np.mean(d * d)))"),
    "normalise_by_max": ("return (x - lo) / (hi - lo)", "return x / hi"),
    "bins_over_n_minus_1": ("scale = np.float32(n_bins) / (hi32 - lo32)",
                            "scale = np.float32(n_bins - 1) / (hi32 - lo32)"),
    "bin_rounding": ("np.minimum(np.floor(t), n_bins - 1)", "np.minimum(np.round(t), n_bins - 1)"),
    "top_bin_wraps": ("np.minimum(np.floor(t), n_bins - 1)", "np.floor(t) % n_bins"),
}


def _mutant(name):
    src = open(M.__file__).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutant {name} does not apply"
    d = tempfile.mkdtemp(prefix="metrics_mutant_")
    path = os.path.join(d, "metrics_mutant.py")
    open(path, "w").write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("metrics_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _all_pins(mod):
    try:
        return _psnr_rows_ok(mod) and _closed_forms_ok(mod) and _invariants_ok(mod)
    except (ValueError, IndexError, ZeroDivisionError):
        return False


def test_real_metrics_oracle_passes():
    assert _all_pins(M)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_metrics_mutant_is_caught(name):
    assert not _all_pins(_mutant(name)), f"mutant {name} slipped through the pins"
