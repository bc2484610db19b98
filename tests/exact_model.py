"""Brute-force exact model of MCLAHE for tiny inputs (a pin for the oracle).

This is deliberately a *different formulation* from the C oracle, so that a
slip in one does not repeat in the other:

* padding uses numpy's ``np.pad(mode="symmetric")`` on an explicit array,
  with the pad lengths of Eq. 1 and the split of Eq. 2 (Sec. III.B);
* kernels are explicit slices of the padded array (Sec. III.A);
* clipping redistributes the excess as the paper states it: every bin gets
  an equal real share ``E / n`` of the excess (Alg. 1, clip step), kept as an
  exact rational instead of the oracle's integer ``n*min(h, C) + E``;
* the CDF normalisation is exact rational arithmetic (Alg. 1, map step);
* interpolation uses the Lagrange coefficients of Sec. III.C literally,
  ``c_i = prod_j (b_j - d_{j i_j}) / b_j``, with the distances ``d`` measured
  from the voxel to the centres of its two bracketing kernels, instead of the
  oracle's integer ``m = 2(x+p0) - (b-1)`` arithmetic.

Only the binning rule is shared as a *specification* (IEEE single precision,
emulated here with numpy float32 scalars), because it is a normative reading
of a point the paper leaves open, not something derivable.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


def pad_lengths(s: int, b: int):
    p = 2 * b - 1 - ((s - 1) % b)       # Eq. 1
    return p, p // 2, (p + 1) // 2      # Eq. 2


def f32_bin(v, lo, hi, n: int) -> int:
    v, lo, hi = np.float32(v), np.float32(lo), np.float32(hi)
    if hi == lo:
        return n - 1 if v > lo else 0
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        scale = np.float32(np.float32(n) / np.float32(hi - lo))
        t = np.float32(np.float32(v - lo) * scale)
    if not (t > np.float32(0)):
        return 0
    if t >= np.float32(n):
        return n - 1
    return int(t)


def decimal_clip_count(clip: float, K: int) -> int:
    """Clip count of a clip limit read as the decimal that was written: the
    shortest decimal that round-trips to the double, times K, floored, and
    capped at K (at K or above nothing is clipped)."""
    return min(math.floor(Fraction(repr(float(clip))) * K), K)


def exact_mclahe(x: np.ndarray, kernel_size, n: int, clip: float,
                 adaptive: bool = False, user_range=None, repeated_rounds: int = 1,
                 centre_half: bool = False):
    """Returns dict(hist, clipped (Fractions, in counts), lut (Fractions), out (Fractions), nk).

    repeated_rounds > 1: the equal sharing is repeated while some bin still
    exceeds the clip level (each round a real share E/n of the new excess);
    centre_half: kernel centres at b//2 instead of (b-1)/2."""
    x = np.asarray(x)
    xf = x.astype(np.float32)
    D = x.ndim
    b = [int(v) for v in kernel_size]
    pads = [pad_lengths(int(s), bb) for s, bb in zip(x.shape, b)]
    padded = np.pad(xf, [(p0, p1) for _, p0, p1 in pads], mode="symmetric")
    nk = [padded.shape[i] // b[i] for i in range(D)]
    assert all(padded.shape[i] == nk[i] * b[i] for i in range(D))
    K = int(np.prod(b))
    C = decimal_clip_count(clip, K)

    if user_range is not None:
        glo, ghi = np.float32(user_range[0]), np.float32(user_range[1])
    else:
        glo, ghi = xf.min(), xf.max()

    hist, lut, rng, clipped = {}, {}, {}, {}
    for kidx in itertools.product(*[range(v) for v in nk]):
        sl = tuple(slice(k * bb, (k + 1) * bb) for k, bb in zip(kidx, b))
        block = padded[sl].ravel()
        lo, hi = (block.min(), block.max()) if adaptive else (glo, ghi)
        rng[kidx] = (lo, hi)
        h = [0] * n
        for v in block:
            h[f32_bin(v, lo, hi, n)] += 1
        hist[kidx] = h
        hp = [Fraction(c) for c in h]
        for r in range(repeated_rounds):
            excess = sum(max(c - C, 0) for c in hp)
            if r > 0 and excess == 0:
                break
            hp = [min(c, Fraction(C)) + Fraction(excess) / n for c in hp]
        clipped[kidx] = hp
        cdf = list(itertools.accumulate(hp))
        if cdf[-1] == cdf[0]:
            lut[kidx] = [Fraction(j, n - 1) for j in range(n)]
        else:
            lut[kidx] = [(c - cdf[0]) / (cdf[-1] - cdf[0]) for c in cdf]

    out = np.empty(x.shape, dtype=object)
    for xi in itertools.product(*[range(s) for s in x.shape]):
        lower, dist = [], []
        for j in range(D):
            q = Fraction(xi[j] + pads[j][1])          # padded position
            half = Fraction(b[j] // 2) if centre_half else Fraction(b[j] - 1, 2)   # centre offset
            klo = math.floor((q - half) / b[j])        # kernel whose centre is below
            c0 = klo * b[j] + half
            c1 = (klo + 1) * b[j] + half
            lower.append(klo)
            dist.append((q - c0, c1 - q))             # d_{j0}, d_{j1}
        v = xf[xi]
        y = Fraction(0)
        for bits in itertools.product((0, 1), repeat=D):
            coef = Fraction(1)
            for j in range(D):
                coef *= (b[j] - dist[j][bits[j]]) / b[j]
            kk = tuple(lower[j] + bits[j] for j in range(D))
            lo, hi = rng[kk]
            y += coef * lut[kk][f32_bin(v, lo, hi, n)]
        out[xi] = y
    return dict(hist=hist, clipped=clipped, lut=lut, out=out, nk=nk, range=rng, C=C)
