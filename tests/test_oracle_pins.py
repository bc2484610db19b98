"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check here is independent of the oracle's own code: hand-derived worked
examples, closed forms of Eq. 1-2, numpy's symmetric padding, an exact
rational brute-force model with a different formulation (tests/exact_model.py),
textbook histogram equalisation (Hall), and invariants of the method.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_model import decimal_clip_count, exact_mclahe, f32_bin, pad_lengths

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- geometry --
# Closed forms of Eq. 1 (p = 2b - 1 - ((s-1) mod b)) and Eq. 2 worked by hand
# for the three benchmark volumes: (pad, pad0, pad1, n_kernels) per axis.
GEOM_TABLE = [
    ((512, 512), (64, 64), [(64, 32, 32, 9)] * 2),
    ((256, 256, 128), (32, 32, 16), [(32, 16, 16, 9), (32, 16, 16, 9), (16, 8, 8, 9)]),
    ((256, 256, 128, 32), (32, 32, 16, 8),
     [(32, 16, 16, 9), (32, 16, 16, 9), (16, 8, 8, 9), (8, 4, 4, 5)]),
    # the paper's own experiment shapes (Sec. IV.A and IV.B processing details)
    ((180, 180, 300, 80), (30, 30, 15, 20),
     [(30, 15, 15, 7), (30, 15, 15, 7), (15, 7, 8, 21), (20, 10, 10, 5)]),
    ((512, 512, 109, 144), (20, 20, 10, 25),
     [(28, 14, 14, 27), (28, 14, 14, 27), (11, 5, 6, 12), (31, 15, 16, 7)]),
]


@pytest.mark.parametrize("shape,ks,expect", GEOM_TABLE)
def test_geometry_table(shape, ks, expect):
    pad, p0, p1, nk = oracle.geometry(shape, ks)
    got = list(zip(pad.tolist(), p0.tolist(), p1.tolist(), nk.tolist()))
    assert got == [tuple(e) for e in expect]


def test_geometry_properties():
    rng = np.random.default_rng(0)
    for _ in range(300):
        s = int(rng.integers(1, 200))
        b = int(rng.integers(1, s + 1))
        pad, p0, p1, nk = oracle.geometry([s], [b])
        p, p0, p1, n = int(pad[0]), int(p0[0]), int(p1[0]), int(nk[0])
        assert (s + p) % b == 0 and b <= p <= 2 * b - 1
        assert p0 + p1 == p and p1 - p0 in (0, 1)
        assert n == -(-s // b) + 1
        # every original voxel has a lower kernel in [0, n-2]
        for x in range(s):
            m = 2 * (x + p0) - (b - 1)
            assert 0 <= m // (2 * b) <= n - 2


def test_geometry_rejects():
    with pytest.raises(ValueError):
        oracle.geometry([4], [5])          # kernel larger than the data
    with pytest.raises(ValueError):
        oracle.geometry([4], [0])


# ---------------------------------------------------------- worked example --
def _golden():
    with open(os.path.join(HERE, "golden", "worked_1d.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _golden()["cases"], ids=lambda c: c["name"])
def test_worked_example(case):
    g = _golden()
    x = np.array(g["input"], np.float32)
    mode = oracle.KERNEL if case["adaptive"] else oracle.GLOBAL
    r = oracle.run(x, g["kernel_size"], g["n_bins"], case["clip"], mode, want_f64=True)
    assert r["pad"].tolist() == [g["geometry"]["pad"]]
    assert r["hist"].tolist() == case["hist"]
    assert r["clipped"].tolist() == case["clipped_times_n"]
    lut = [[float(Fraction(v)) for v in row] for row in case["lut"]]
    np.testing.assert_array_equal(r["lut"], np.array(lut, np.float32))
    out = np.array([float(Fraction(v)) for v in case["out"]])
    # maps are stored in float32 (rounded once from the exact ratio), so the
    # interpolated value carries at most their rounding error (2^-25 relative)
    np.testing.assert_allclose(r["out_f64"], out, rtol=0, atol=3e-8)
    np.testing.assert_allclose(r["out"], out, rtol=0, atol=1e-7)
    # the independent exact model reproduces the hand derivation exactly
    e = exact_mclahe(x, g["kernel_size"], g["n_bins"], case["clip"], case["adaptive"])
    assert [e["hist"][(k,)] for k in range(3)] == case["hist"]
    assert [e["lut"][(k,)] for k in range(3)] == [[Fraction(v) for v in row] for row in case["lut"]]
    assert list(e["out"]) == [Fraction(v) for v in case["out"]]
    padded = np.pad(x, (1, 1), mode="symmetric")
    assert padded.tolist() == g["padded"]


# ------------------------------------------------ exact model vs the oracle --
def _random_case(rng):
    D = int(rng.integers(1, 4))
    shape = [int(rng.integers(1, 9 if D < 3 else 6)) for _ in range(D)]
    ks = [int(rng.integers(1, s + 1)) for s in shape]
    dtype = [np.uint8, np.uint16, np.float32][int(rng.integers(0, 3))]
    kind = int(rng.integers(0, 4))
    if kind == 0:
        x = rng.integers(0, 4, size=shape)                 # heavy collisions
    elif kind == 1:
        x = rng.poisson(2.0, size=shape)                   # count data
    elif kind == 2:
        x = rng.integers(0, 60000 if dtype == np.uint16 else 256, size=shape)
    else:
        x = np.full(shape, 7)                              # constant input
    if dtype == np.float32:
        x = x.astype(np.float32) * np.float32(rng.choice([1.0, 0.37, -2.5]))
    else:
        x = np.clip(x, 0, np.iinfo(dtype).max).astype(dtype)
    n = int(rng.choice([2, 3, 4, 7, 16]))
    clip = float(rng.choice([0.0, 0.01, 0.1, 0.25, 0.5, 1.0, 5.0]))
    adaptive = bool(rng.integers(0, 2))
    return np.ascontiguousarray(x), ks, n, clip, adaptive


@pytest.mark.parametrize("seed", range(60))
def test_oracle_matches_exact_model(seed):
    rng = np.random.default_rng(1000 + seed)
    x, ks, n, clip, adaptive = _random_case(rng)
    mode = oracle.KERNEL if adaptive else oracle.GLOBAL
    r = oracle.run(x, ks, n, clip, mode, want_f64=True)
    e = exact_mclahe(x, ks, n, clip, adaptive)
    nk = e["nk"]
    keys = list(np.ndindex(*nk))
    assert r["hist"].tolist() == [e["hist"][k] for k in keys]
    # integer clipped histogram == n * (exact real-valued redistribution)
    K = int(np.prod(ks))
    for i, k in enumerate(keys):
        h = e["hist"][k]
        exc = sum(max(c - e["C"], 0) for c in h)
        hp = [Fraction(min(c, e["C"])) + Fraction(exc, n) for c in h]
        assert [Fraction(int(v)) for v in r["clipped"][i]] == [n * v for v in hp]
        assert int(r["clipped"][i].sum()) == n * K
        # map rounded to float32 from the exact rational (<= 1 ulp)
        ex = np.array([float(v) for v in e["lut"][k]], np.float64)
        np.testing.assert_allclose(r["lut"][i], ex, rtol=0, atol=6e-8)
    ex = np.vectorize(float)(e["out"]).astype(np.float64)
    # float32 maps: error of the weighted sum <= max map rounding (2^-25)
    np.testing.assert_allclose(r["out_f64"], ex, rtol=0, atol=3e-8)


# ------------------------------------------- numpy symmetric-padding pin --
@pytest.mark.parametrize("seed", range(8))
def test_histograms_sum_to_padded_bincount(seed):
    """Sum over kernels of h_k == bincount of the bins of np.pad(symmetric)."""
    rng = np.random.default_rng(seed)
    D = 1 + seed % 3
    shape = [int(rng.integers(3, 14)) for _ in range(D)]
    ks = [int(rng.integers(1, s + 1)) for s in shape]
    x = rng.poisson(3.0, size=shape).astype(np.float32)
    n = 8
    r = oracle.run(x, ks, n, 1.0, oracle.GLOBAL)
    pads = [pad_lengths(s, b) for s, b in zip(shape, ks)]
    padded = np.pad(x, [(p0, p1) for _, p0, p1 in pads], mode="symmetric")
    lo, hi = x.min(), x.max()
    bins = [f32_bin(v, lo, hi, n) for v in padded.ravel()]
    np.testing.assert_array_equal(r["hist"].sum(0), np.bincount(bins, minlength=n))
    assert (r["hist"].sum(1) == int(np.prod(ks))).all()


# ------------------------------------------------------------ closed forms --
def test_bin_edges_closed_form():
    # range [0, n): integer values land exactly in their own bin; the top
    # value goes to the last bin (reading of the histogram step)
    n = 16
    x = np.arange(n, dtype=np.float32).reshape(4, 4)
    x[3, 3] = 16.0      # hi = 16 -> scale = 1
    r = oracle.run(x, (4, 4), n, 1.0, oracle.GLOBAL)
    expect = np.bincount(np.minimum(x.ravel().astype(int), n - 1), minlength=n)
    # the kernel grid is 2x2 of fully mirrored 4x4 blocks; each kernel holds
    # each quadrant value 4 times -> totals are 4x the raw counts
    np.testing.assert_array_equal(r["hist"].sum(0), 4 * expect)


def test_clip_closed_forms():
    rng = np.random.default_rng(5)
    x = rng.poisson(4.0, size=(12, 10)).astype(np.float32)
    ks, n = (4, 5), 8
    K = 20
    r1 = oracle.run(x, ks, n, 1.0)
    assert (r1["clipped"] == n * r1["hist"]).all()          # clip >= 1: no-op
    r5 = oracle.run(x, ks, n, 5.0)
    assert (r5["clipped"] == n * r5["hist"]).all()
    r0 = oracle.run(x, ks, n, 0.0)
    assert (r0["clipped"] == K).all()                       # clip 0: uniform
    rc = oracle.run(x, ks, n, 0.1)
    assert (rc["clipped"].sum(1) == n * K).all()
    C = 2                                                    # floor(0.1*20)
    for h, H in zip(rc["hist"], rc["clipped"]):
        E = np.maximum(h - C, 0).sum()
        assert (H == n * np.minimum(h, C) + E).all()


def _oracle_clip_count(clip, K):
    """C read back from the oracle: a constant 1D volume with kernel K puts all
    K voxels of every kernel in bin 0, so every other bin holds the excess
    share K - C (in units of 1/n)."""
    r = oracle.run(np.full(K, 7.0, np.float32), (K,), 4, clip)
    return K - int(r["clipped"][0, 1])


@pytest.mark.parametrize("clip,K,C", [
    (0.02, 270000, 5400),    # the photoemission experiment's clip limit and kernel (Sec. IV.A)
    (0.01, 100, 1),          # float32(0.01) * 100 would floor to 0
    (0.29, 100, 29),         # the double product 28.999999999999996 floors to 28
    (0.25, 1000, 250),       # the fluorescence experiment's clip limit (Sec. IV.B), exact in binary
    (0.7, 10, 7),
    (1.0, 64, 64), (3.5, 64, 64),   # at or above K nothing is clipped: C is reported as K
    (0.0, 64, 0),
])
def test_clip_count_of_decimal_limits(clip, K, C):
    assert decimal_clip_count(clip, K) == C
    assert _oracle_clip_count(clip, K) == C


def test_clip_count_random_decimals():
    """The oracle's count equals the written decimal's exact count, floored,
    for decimals of 1-4 significant digits (exact rational arithmetic)."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        digits = int(rng.integers(1, 5))
        clip = float(f"{rng.uniform(0.001, 0.999):.{digits}g}")
        K = int(rng.choice([7, 64, 100, 300, 1000, 4096, 12000]))
        assert _oracle_clip_count(clip, K) == decimal_clip_count(clip, K), (clip, K)


def test_lut_invariants():
    rng = np.random.default_rng(6)
    x = (rng.exponential(5.0, size=(20, 17, 6)) * 3).astype(np.float32)
    for mode in (oracle.GLOBAL, oracle.KERNEL):
        for clip in (0.0, 0.02, 0.3, 1.0):
            r = oracle.run(x, (5, 4, 3), 32, clip, mode)
            lut = r["lut"]
            assert (np.diff(lut, axis=1) >= 0).all()
            assert (lut[:, 0] == 0).all() and (lut[:, -1] == 1).all()
            assert ((lut >= 0) & (lut <= 1)).all()


def test_degenerate_kernel_gives_ramp():
    x = np.zeros((6, 6), np.float32)
    x[0, 0] = 5.0
    r = oracle.run(x, (3, 3), 5, 1.0, oracle.GLOBAL)
    ramp = (np.arange(5) / 4).astype(np.float32)
    # kernels far from the single bright voxel hold only zeros: flat cdf
    flat = [k for k in range(r["hist"].shape[0]) if r["hist"][k, 0] == 9]
    assert flat
    for k in flat:
        np.testing.assert_array_equal(r["lut"][k], ramp)


@pytest.mark.parametrize("mode", [oracle.GLOBAL, oracle.KERNEL])
def test_constant_input_maps_to_zero(mode):
    for dt, val in ((np.float32, 3.5), (np.uint8, 200), (np.uint16, 9)):
        x = np.full((7, 5, 3), val, dtype=dt)
        r = oracle.run(x, (3, 2, 3), 16, 0.02, mode)
        assert (r["out"] == 0).all()


def test_clip_zero_global_is_linear_in_bin():
    rng = np.random.default_rng(7)
    x = rng.normal(0, 1, size=(9, 11)).astype(np.float32)
    n = 10
    r = oracle.run(x, (4, 3), n, 0.0, oracle.GLOBAL)
    lo, hi = x.min(), x.max()
    bins = np.array([f32_bin(v, lo, hi, n) for v in x.ravel()]).reshape(x.shape)
    np.testing.assert_allclose(r["out"], bins / (n - 1), rtol=0, atol=1e-7)


@pytest.mark.parametrize("mode", [oracle.GLOBAL, oracle.KERNEL])
def test_reduces_to_global_histogram_equalisation(mode):
    """Textbook HE (Hall 1974) as the single-kernel limit.

    With b = s (even) and data periodic with period s/2 on every axis, every
    padded kernel holds exactly the multiset of the data, so without clipping
    each map is the global equalisation map and the output equals it.
    """
    rng = np.random.default_rng(8)
    half = rng.poisson(6.0, size=(3, 4, 2)).astype(np.float32)
    x = np.tile(half, (2, 2, 2))
    n = 12
    r = oracle.run(x, x.shape, n, 1.0, mode, want_f64=True)
    lo, hi = x.min(), x.max()
    bins = np.array([f32_bin(v, lo, hi, n) for v in x.ravel()])
    cdf = np.cumsum(np.bincount(bins, minlength=n))
    he = ((cdf - cdf[0]) / (cdf[-1] - cdf[0])).astype(np.float32)  # maps are float32
    np.testing.assert_array_equal(r["lut"], np.broadcast_to(he, r["lut"].shape))
    np.testing.assert_allclose(r["out_f64"].ravel(), he[bins], rtol=0, atol=1e-12)


# --------------------------------------------------------------- symmetries --
@pytest.mark.parametrize("mode", [oracle.GLOBAL, oracle.KERNEL])
def test_flip_equivariance(mode):
    rng = np.random.default_rng(9)
    # axis sizes chosen so that every pad length is even
    x = rng.poisson(3.0, size=(16, 12, 9)).astype(np.float32)
    ks = (4, 4, 5)
    pad = oracle.geometry(x.shape, ks)[0]
    assert (pad % 2 == 0).all()
    r = oracle.run(x, ks, 16, 0.05, mode, want_f64=True)
    for ax in range(3):
        rf = oracle.run(np.flip(x, ax).copy(), ks, 16, 0.05, mode, want_f64=True)
        np.testing.assert_allclose(rf["out_f64"], np.flip(r["out_f64"], ax), rtol=0, atol=1e-12)


def test_axis_permutation_equivariance():
    rng = np.random.default_rng(10)
    x = rng.poisson(3.0, size=(9, 7, 5)).astype(np.float32)
    ks = (4, 3, 2)
    r = oracle.run(x, ks, 8, 0.1, oracle.KERNEL, want_f64=True)
    perm = (2, 0, 1)
    rp = oracle.run(np.transpose(x, perm).copy(), [ks[p] for p in perm], 8, 0.1,
                    oracle.KERNEL, want_f64=True)
    np.testing.assert_allclose(rp["out_f64"], np.transpose(r["out_f64"], perm), rtol=0, atol=1e-12)


@pytest.mark.parametrize("where", ["front", "back"])
def test_singleton_axis_lifting_is_bit_identical(where):
    rng = np.random.default_rng(11)
    x = rng.poisson(3.0, size=(10, 9)).astype(np.float32)
    ks = (4, 3)
    r = oracle.run(x, ks, 16, 0.05, oracle.GLOBAL, want_f64=True)
    if where == "front":
        xl, kl = x[None], (1,) + ks
    else:
        xl, kl = x[..., None], ks + (1,)
    rl = oracle.run(np.ascontiguousarray(xl), kl, 16, 0.05, oracle.GLOBAL, want_f64=True)
    np.testing.assert_array_equal(rl["out_f64"].reshape(x.shape), r["out_f64"])


def test_power_of_two_scaling_is_bit_identical():
    rng = np.random.default_rng(12)
    x = rng.gamma(2.0, 3.0, size=(11, 13)).astype(np.float32)
    for mode in (oracle.GLOBAL, oracle.KERNEL):
        r = oracle.run(x, (4, 5), 64, 0.03, mode, want_f64=True)
        for k in (-3, 5):
            rs = oracle.run(x * np.float32(2.0 ** k), (4, 5), 64, 0.03, mode, want_f64=True)
            np.testing.assert_array_equal(rs["hist"], r["hist"])
            np.testing.assert_array_equal(rs["out_f64"], r["out_f64"])


def test_kernel_centre_voxel_takes_its_own_map():
    """With odd b, a voxel at a kernel centre has weight 1 on that kernel."""
    rng = np.random.default_rng(13)
    x = rng.poisson(3.0, size=(15,)).astype(np.float32)
    b = 5
    r = oracle.run(x, (b,), 8, 0.2, oracle.GLOBAL, want_f64=True)
    p0 = int(r["pad0"][0])
    lo, hi = x.min(), x.max()
    for xi in range(15):
        q = xi + p0
        if (q - (b - 1) // 2) % b == 0:
            k = (q - (b - 1) // 2) // b
            assert r["out_f64"][xi] == r["lut"][k, f32_bin(x[xi], lo, hi, 8)]


def test_integer_output_quantisation():
    rng = np.random.default_rng(14)
    x = rng.integers(0, 256, size=(20, 24)).astype(np.uint8)
    rf = oracle.run(x, (8, 8), 64, 0.02, out_dtype=np.float32)
    r8 = oracle.run(x, (8, 8), 64, 0.02, out_dtype=np.uint8)
    r16 = oracle.run(x, (8, 8), 64, 0.02, out_dtype=np.uint16)
    y = rf["out"].astype(np.float32)
    np.testing.assert_array_equal(r8["out"], np.minimum(255, np.floor(y * np.float32(255) + np.float32(0.5))))
    np.testing.assert_array_equal(r16["out"], np.minimum(65535, np.floor(y * np.float32(65535) + np.float32(0.5))))


def test_user_range_matches_data_range():
    rng = np.random.default_rng(15)
    x = rng.normal(0, 1, size=(10, 10)).astype(np.float32)
    r = oracle.run(x, (4, 4), 32, 0.05)
    ru = oracle.run(x, (4, 4), 32, 0.05, user_range=(x.min(), x.max()))
    np.testing.assert_array_equal(r["out"], ru["out"])
    # a wider user range clamps nothing and shifts bins: differs in general
    rw = oracle.run(x, (4, 4), 32, 0.05, user_range=(-10.0, 10.0))
    assert not np.array_equal(rw["hist"], r["hist"])
