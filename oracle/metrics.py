"""Contrast metrics of a volume and of an enhanced volume against its original
-- TEST INFRASTRUCTURE ONLY.

Plain numpy statement of the four image-contrast metrics the paper uses to
judge its results (Sec. II, related work on contrast metrics; Tables I and
II): the mean squared error (MSE) against the original, the peak
signal-to-noise ratio (PSNR) derived from it, the standard deviation (RMS
contrast) and the Shannon (grey-level) entropy.  All of them are defined for
data of any dimension.  Only the tests, the smoke check and the benchmark's
CPU leg may import this module; the product library never does, and this
module imports nothing from the product.

Readings of points the paper leaves open (normative; the GPU library follows
them):
  - every volume is min-max normalised to [0, 1] first, u = (v - lo)/(hi - lo)
    with lo, hi its own minimum and maximum (u = 0 where hi == lo), so that raw
    data and an enhanced result in [0, 1] are compared on one scale;
  - MSE = mean((u_x - u_y)^2) over all voxels;
  - PSNR = 10 log10(peak^2 / MSE) with the peak a parameter (+inf if MSE = 0);
    both of the paper's tables are consistent with peak = 2^23 (checked
    against every printed MSE/PSNR pair), so that value is named here;
  - STD is the population standard deviation (divide by N) of u;
  - ENT = -sum p_j log2 p_j over an n-bin grey-level histogram of the volume,
    p_j = count_j / N, empty bins contribute 0.  The histogram bins the raw
    values over [lo, hi] exactly as the CLAHE histograms do, in IEEE single
    precision: scale = (float)n / (hi - lo), t = (v - lo) * scale,
    bin = t > 0 ? min(floor(t), n - 1) : 0 (all voxels in bin 0 if hi == lo).
  - inputs are finite.
Arithmetic is float64 except the binning, which is float32 as stated.
"""
from __future__ import annotations

import numpy as np

# The peak value both metric tables of the paper imply (see module notes).
PAPER_PSNR_PEAK = float(2 ** 23)


def value_range(v: np.ndarray) -> tuple[float, float]:
    """Minimum and maximum of the volume (exact; float32 values)."""
    f = np.asarray(v).astype(np.float32, copy=False)
    return float(f.min()), float(f.max())


def normalise(v: np.ndarray) -> np.ndarray:
    """Min-max normalisation to [0, 1] in float64 (0 everywhere if constant)."""
    lo, hi = value_range(v)
    x = np.asarray(v, dtype=np.float64)
    if hi == lo:
        return np.zeros_like(x)
    return (x - lo) / (hi - lo)


def grey_histogram(v: np.ndarray, n_bins: int) -> np.ndarray:
    """n_bins-bin histogram of the raw values over [lo, hi], binned in float32."""
    lo, hi = value_range(v)
    f = np.asarray(v).astype(np.float32, copy=False).ravel()
    if hi == lo:
        idx = np.zeros(f.shape, dtype=np.int64)
    else:
        lo32, hi32 = np.float32(lo), np.float32(hi)
        scale = np.float32(n_bins) / (hi32 - lo32)
        t = (f - lo32) * scale
        idx = np.where(t > 0, np.minimum(np.floor(t), n_bins - 1), 0).astype(np.int64)
    return np.bincount(idx, minlength=n_bins).astype(np.int64)


def entropy_bits(counts: np.ndarray) -> float:
    """Shannon entropy in bits of a histogram (empty bins contribute 0)."""
    c = np.asarray(counts, dtype=np.float64)
    p = c[c > 0] / c.sum()
    return float(-(p * np.log2(p)).sum())


def std(v: np.ndarray) -> float:
    """RMS contrast: population standard deviation of the normalised volume."""
    u = normalise(v)
    return float(np.sqrt(np.mean((u - u.mean()) ** 2)))


def mse(x: np.ndarray, y: np.ndarray) -> float:
    """Mean squared difference of the two normalised volumes."""
    if np.shape(x) != np.shape(y):
        raise ValueError("volumes differ in shape")
    d = normalise(x) - normalise(y)
    return float(np.mean(d * d))


def psnr(mse_value: float, peak: float) -> float:
    """Peak signal-to-noise ratio in dB for a given MSE."""
    if mse_value == 0:
        return float("inf")
    return float(10.0 * np.log10(peak * peak / mse_value))


def metrics(x: np.ndarray, y: np.ndarray | None = None, n_bins: int = 256,
            peak: float = 1.0) -> dict:
    """All metrics of x (and of y against x): the fields the GPU library fills."""
    vols = [x] if y is None else [x, y]
    out = {"lo": [], "hi": [], "mean": [], "std": [], "entropy": []}
    for v in vols:
        lo, hi = value_range(v)
        u = normalise(v)
        out["lo"].append(lo)
        out["hi"].append(hi)
        out["mean"].append(float(u.mean()))
        out["std"].append(std(v))
        out["entropy"].append(entropy_bits(grey_histogram(v, n_bins)))
    if y is not None:
        m = mse(x, y)
        out["mse"] = m
        out["psnr"] = psnr(m, peak)
    return out
