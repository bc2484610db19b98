"""Pins of the oracle's comparison variants (repeated and integer
redistribution, centres at b//2).

Hand-derived clip results and outputs (tests/golden/variants_1d.json); the
exact rational model (tests/exact_model.py), whose repeated sharing adds
real shares E/n instead of the oracle's scaled integers and whose centres
are measured as distances; conservation of the kernel's count; and the
identities with the paper's method (one round, odd kernel sizes).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_model import decimal_clip_count, exact_mclahe

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "variants_1d.json")))


@pytest.mark.parametrize("case", GOLD["clip_cases"], ids=lambda c: c["name"])
def test_clip_variants_hand_derived(case):
    x = np.zeros(case["input_len"], np.float32)
    r = oracle.run(x, [case["kernel"]], case["n_bins"], case["clip"], redistribution=case["redistribution"],
                   rounds=case["rounds"])
    for row in r["clipped"]:
        assert row.tolist() == case["clipped"]


def test_centre_half_hand_derived():
    c = GOLD["centre_case"]
    r = oracle.run(np.array(c["input"], np.float32), c["kernel"], c["n_bins"], c["clip"], want_f64=True,
                   centre_half=True)
    np.testing.assert_allclose(r["out_f64"], [float(Fraction(v)) for v in c["out"]], atol=3e-8)


def _rand(seed):
    rng = np.random.default_rng(seed)
    D = 1 + seed % 3
    shape = [int(rng.integers(2, [9, 6, 4][D - 1] + 1)) for _ in range(D)]
    ks = [int(rng.integers(1, s + 1)) for s in shape]
    x = rng.poisson(2.0, size=shape).astype(np.float32)
    return x, ks


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("rounds", [2, 3])
def test_repeated_against_exact_model(seed, rounds):
    x, ks = _rand(seed)
    n, clip = 5, 0.15
    ad = bool(seed % 2)
    r = oracle.run(x, ks, n, clip, oracle.KERNEL if ad else oracle.GLOBAL, want_f64=True,
                   redistribution=oracle.REPEATED, rounds=rounds)
    e = exact_mclahe(x, ks, n, clip, ad, repeated_rounds=rounds)
    keys = list(np.ndindex(*e["nk"]))
    K = int(np.prod(ks))
    for i, k in enumerate(keys):
        row = [int(v) for v in r["clipped"][i]]
        tot = sum(row)
        # scaled integers and real shares agree once both are normalised by the count
        assert [Fraction(v, tot) for v in row] == [v / K for v in e["clipped"][k]]
        assert sum(e["clipped"][k]) == K
    ex = np.vectorize(float)(e["out"]).astype(np.float64)
    np.testing.assert_allclose(r["out_f64"], ex, atol=3e-8, rtol=0)


@pytest.mark.parametrize("seed", range(8))
def test_centre_half_against_exact_model(seed):
    x, ks = _rand(seed + 20)
    ks = [k if k % 2 == 0 or k == 1 else k - 1 for k in ks]   # mostly even sizes
    r = oracle.run(x, ks, 6, 0.3, want_f64=True, centre_half=True)
    e = exact_mclahe(x, ks, 6, 0.3, centre_half=True)
    ex = np.vectorize(float)(e["out"]).astype(np.float64)
    np.testing.assert_allclose(r["out_f64"], ex, atol=3e-8, rtol=0)


@pytest.mark.parametrize("seed", range(6))
def test_integer_redistribution_invariants(seed):
    x, ks = _rand(seed + 40)
    n, clip = 7, 0.1
    r = oracle.run(x, ks, n, clip, redistribution=oracle.INTEGER)
    K = int(np.prod(ks))
    C = decimal_clip_count(clip, K)
    for h, H in zip(r["hist"], r["clipped"]):
        base = np.minimum(h, C)
        E = int((h - base).sum())
        share = H - base
        assert int(H.sum()) == K                                   # every count kept
        assert set(share.tolist()) <= {E // n, E // n + 1}         # equal integer share
        assert int((share == E // n + 1).sum()) == E % n           # remainder one each


def test_identities_with_the_papers_method():
    rng = np.random.default_rng(3)
    x = rng.poisson(3.0, size=(9, 7, 5)).astype(np.float32)
    base = oracle.run(x, (3, 5, 3), 16, 0.1)
    one = oracle.run(x, (3, 5, 3), 16, 0.1, redistribution=oracle.REPEATED, rounds=1)
    odd = oracle.run(x, (3, 5, 3), 16, 0.1, centre_half=True)   # odd b: same centres
    assert len({tuple(r) for r in base["lut"].tolist()}) > 1     # the kernels differ
    for k in ("clipped", "lut", "out"):
        assert np.array_equal(base[k], one[k]) and np.array_equal(base[k], odd[k])
    # a clip level no bin reaches: every variant is the plain equalisation
    big = [oracle.run(x, (3, 5, 3), 16, 1.0, redistribution=v, rounds=3) for v in (0, 1, 2)]
    assert np.array_equal(big[0]["lut"], big[1]["lut"]) and np.array_equal(big[0]["lut"], big[2]["lut"])


# ------------------------------------------------------------------ mutants --
VARIANT_MUTANTS = {
    "integer_remainder_step": ("const int64_t s = R ? (n / R > 1 ? n / R : 1) : 1;", "const int64_t s = 1;"),
    "integer_share_rounded": ("const int64_t q = E / n, R = E % n;", "const int64_t q = (E + n / 2) / n, R = E % n;"),
    "repeated_level_fixed": ("                Cr *= n;\n", "\n"),
    "repeated_no_stop": ("if (r > 1 && E == 0) break;", ""),
    "centre_half_odd": ("(centre_half ? 2 * (ksize[i] / 2) : ksize[i] - 1)", "(centre_half ? ksize[i] : ksize[i] - 1)"),
}


def _variant_pins_pass(lib):
    try:
        for case in GOLD["clip_cases"]:
            x = np.zeros(case["input_len"], np.float32)
            r = oracle.run(x, [case["kernel"]], case["n_bins"], case["clip"], lib=lib,
                           redistribution=case["redistribution"], rounds=case["rounds"])
            if any(row.tolist() != case["clipped"] for row in r["clipped"]):
                return False
        c = GOLD["centre_case"]
        r = oracle.run(np.array(c["input"], np.float32), c["kernel"], c["n_bins"], c["clip"], want_f64=True,
                       centre_half=True, lib=lib)
        if not np.allclose(r["out_f64"], [float(Fraction(v)) for v in c["out"]], atol=3e-8):
            return False
        # odd kernel sizes: the two centre conventions coincide
        xo = np.random.default_rng(3).poisson(3.0, size=(9, 7)).astype(np.float32)
        a = oracle.run(xo, (3, 5), 16, 0.5, lib=lib)
        b = oracle.run(xo, (3, 5), 16, 0.5, centre_half=True, lib=lib)
        if not np.array_equal(a["out"], b["out"]):
            return False
        for seed in range(4):
            x, ks = _rand(seed)
            r = oracle.run(x, ks, 5, 0.15, want_f64=True, redistribution=oracle.REPEATED, rounds=3, lib=lib)
            e = exact_mclahe(x, ks, 5, 0.15, repeated_rounds=3)
            if not np.allclose(r["out_f64"], np.vectorize(float)(e["out"]).astype(np.float64), atol=3e-8):
                return False
        return True
    except (ValueError, KeyError, IndexError):
        return False


def test_real_oracle_passes_variant_pins():
    assert _variant_pins_pass(None)


@pytest.mark.parametrize("name", sorted(VARIANT_MUTANTS))
def test_variant_mutant_is_caught(name):
    import subprocess
    import tempfile
    src = open(os.path.join(os.path.dirname(oracle.__file__), "mclahe_oracle.c")).read()
    old, new = VARIANT_MUTANTS[name]
    assert src.count(old) == 1, f"mutant {name} does not apply"
    d = tempfile.mkdtemp(prefix="variant_mutant_")
    c, so = os.path.join(d, "m.c"), os.path.join(d, "m.so")
    open(c, "w").write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", c,
                           "-o", so, "-lm"])
    assert not _variant_pins_pass(oracle.load_library(so)), f"mutant {name} slipped through the pins"
