"""The pins catch plausible mistakes: plant one in a copy of the oracle.

Each mutant is a one-line slip in the oracle source (a dropped term, a flipped
sign, a swapped operand, a wrong convention).  The copy is compiled on the CPU
and the pin checks below are run against it; every mutant must fail at least
one of them.  The real oracle is never modified.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from exact_model import exact_mclahe

SRC = os.path.join(os.path.dirname(oracle.__file__), "mclahe_oracle.c")

MUTANTS = {
    "eq1_sign": ("2 * b - 1 - ((s - 1) % b)", "2 * b - 1 + ((s - 1) % b)"),
    "eq2_split_swapped": ("pad0[i] = p / 2;", "pad0[i] = (p + 1) / 2;"),
    "reflect_not_symmetric": ("if (x < 0) x = -x - 1;", "if (x < 0) x = -x;"),
    "excess_dropped": ("H[j] = (int64_t)n * (H[j] < Cr ? H[j] : Cr) + E;",
                       "H[j] = (int64_t)n * (H[j] < Cr ? H[j] : Cr);"),
    "clip_ceil": ("int64_t C = (int64_t)floor(c);", "int64_t C = (int64_t)ceil(c);"),
    "cdf_exclusive": ("acc += H[j];\n            double m", "double m"),
    "weights_swapped": ("coef *= bit ? w[i] : 1.0 - w[i];", "coef *= bit ? 1.0 - w[i] : w[i];"),
    "centre_b_over_2": ("(centre_half ? 2 * (ksize[i] / 2) : ksize[i] - 1)",
                        "(centre_half ? 2 * (ksize[i] / 2) : 2 * (ksize[i] / 2))"),
    "bin_round_not_trunc": ("return (int)t;", "return (int)(t + 0.5f) < n ? (int)(t + 0.5f) : n - 1;"),
    "ahr_map_uses_global": ("float sc = mode == ORC_KERNEL ? (float)n / (hi - lo) : gscale;",
                            "float sc = gscale; lo = glo; hi = ghi;"),
    "corner_axis_transposed": ("kidx = kidx * nk[i] + k0[i] + bit;",
                               "kidx = kidx * nk[i] + k0[i] + ((c >> i) & 1);"),
    "top_bin_dropped": ("if (t >= (float)n) return n - 1;", "if (t >= (float)n) return 0;"),
}


def _build(name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutant {name} does not apply"
    src = src.replace(old, new, 1)
    d = tempfile.mkdtemp(prefix="mclahe_mutant_")
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "m.so")
    open(c, "w").write(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off",
                           "-shared", "-fPIC", c, "-o", so, "-lm"])
    return oracle.load_library(so)


def _pins_pass(lib):
    """A compact subset of the pin suite; returns False on the first failure."""
    try:
        # worked 1D example (hand-derived values)
        x = np.array([0, 1, 2, 3], np.float32)
        r = oracle.run(x, [2], 4, 0.5, oracle.GLOBAL, want_f64=True, lib=lib)
        if not np.allclose(r["out_f64"], [0, 11 / 24, 23 / 28, 1], atol=3e-8):
            return False
        r = oracle.run(x, [2], 4, 1.0, oracle.KERNEL, want_f64=True, lib=lib)
        if not np.allclose(r["out_f64"], [0, 1 / 4, 3 / 4, 1 / 4], atol=3e-8):
            return False
        # exact brute-force model on small random cases
        for seed in range(6):
            rng = np.random.default_rng(seed)
            shape = [5, 4, 3][: 1 + seed % 3]
            ks = [int(rng.integers(1, s + 1)) for s in shape]
            xx = rng.poisson(2.0, size=shape).astype(np.float32)
            ad = bool(seed % 2)
            r = oracle.run(xx, ks, 5, 0.2, oracle.KERNEL if ad else oracle.GLOBAL,
                           want_f64=True, lib=lib)
            e = exact_mclahe(xx, ks, 5, 0.2, ad)
            keys = list(np.ndindex(*e["nk"]))
            if r["hist"].shape[0] != len(keys):
                return False
            if r["hist"].tolist() != [e["hist"][k] for k in keys]:
                return False
            ex = np.vectorize(float)(e["out"]).astype(np.float64)
            if not np.allclose(r["out_f64"], ex, atol=3e-8, rtol=0):
                return False
        return True
    except (ValueError, KeyError, IndexError):
        return False


def test_real_oracle_passes_the_subset():
    assert _pins_pass(None)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    lib = _build(name)
    assert not _pins_pass(lib), f"mutant {name} slipped through the pins"
