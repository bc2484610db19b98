"""GPU parity of the contrast metrics (mclahe_metrics) against the oracle.

The oracle is oracle/metrics.py (plain numpy, float64, binning in float32).
Histogram counts and the value range must match exactly; means, standard
deviations and the MSE are float64 sums of up to 2^28 terms in another order,
so they must agree to a relative 1e-9; entropies (same counts, another
summation order and log2) to a relative 1e-12; the PSNR to 1e-8 dB.
Cases: every dtype pair, one volume or two, ragged tails, misaligned bases
(the element-load path), 2 to 8192 bins, constant and two-level volumes, and
the 4D benchmark volume against its CLAHE result at full size.
"""
import ctypes
import math

import numpy as np
import pytest

from gpu_util import to_device_bytes
from oracle import metrics as M

pytestmark = pytest.mark.gpu
CODE = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float32): 2}


def gpu_metrics(x, y=None, n_bins=256, peak=1.0, x_off=0, y_off=0):
    import torch
    from paper_1906_11355_amd import _lib
    xb, xp = to_device_bytes(x, x_off)
    yb, yp = (None, None) if y is None else to_device_bytes(y, y_off)
    n = x.size
    need = _lib.metrics_workspace_size(n, n_bins)
    ws = torch.full((need,), 0xAB, dtype=torch.uint8, device="cuda")     # poisoned
    res = torch.zeros(ctypes.sizeof(_lib.MetricsResult), dtype=torch.uint8, device="cuda")
    hist = torch.full((2 * n_bins,), -1, dtype=torch.int64, device="cuda")
    _lib.metrics_ptr(xp, CODE[x.dtype], yp, CODE[y.dtype] if y is not None else 0, n, n_bins, peak,
                     res.data_ptr(), hist.data_ptr(), ws.data_ptr(), need,
                     torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    r = _lib.MetricsResult.from_buffer_copy(bytes(res.cpu().numpy()))
    h = hist.cpu().numpy()
    return r, h


def close(a, b, rel, what):
    assert math.isclose(a, b, rel_tol=rel, abs_tol=1e-300), f"{what}: {a!r} vs {b!r}"


def check(x, y=None, n_bins=256, peak=1.0, **kw):
    r, h = gpu_metrics(x, y, n_bins, peak, **kw)
    e = M.metrics(x, y, n_bins, peak)
    vols = [x] if y is None else [x, y]
    for v, vol in enumerate(vols):
        tag = f"vol{v} {vol.dtype} n={vol.size} nb={n_bins}"
        assert r.lo[v] == e["lo"][v] and r.hi[v] == e["hi"][v], tag
        np.testing.assert_array_equal(h[v * n_bins:(v + 1) * n_bins], M.grey_histogram(vol, n_bins),
                                      err_msg=tag)
        close(r.mean[v], e["mean"][v], 1e-9, tag + " mean")
        close(r.std[v], e["std"][v], 1e-9, tag + " std")
        close(r.entropy[v], e["entropy"][v], 1e-12, tag + " entropy")
    if y is None:
        assert r.mse == 0.0 and r.psnr == 0.0 and r.lo[1] == 0.0 and r.std[1] == 0.0
    else:
        close(r.mse, e["mse"], 1e-9, "mse")
        if math.isinf(e["psnr"]):
            assert math.isinf(r.psnr)
        else:
            assert abs(r.psnr - e["psnr"]) <= 1e-8, (r.psnr, e["psnr"])
    assert r.count == x.size
    return r


def _vol(rng, dt, n, kind):
    if kind == "poisson":
        v = rng.poisson(3.0, size=n)
    elif kind == "wide":
        v = rng.integers(0, 60000 if dt == np.uint16 else 256, size=n)
    else:
        v = rng.normal(50, 20, size=n)
    if dt == np.float32:
        return v.astype(np.float32) * np.float32(0.37)
    return np.clip(v, 0, np.iinfo(dt).max).astype(dt)


DTS = [np.uint8, np.uint16, np.float32]


@pytest.mark.parametrize("xdt", DTS)
@pytest.mark.parametrize("ydt", DTS + [None])
def test_dtype_pairs(xdt, ydt):
    rng = np.random.default_rng(10 * DTS.index(xdt) + (DTS.index(ydt) if ydt else 3))
    n = 3 * 256 * 8 * 4 + 5          # several work-groups and a ragged tail
    x = _vol(rng, xdt, n, "poisson")
    y = None if ydt is None else _vol(rng, ydt, n, "wide")
    check(x, y)


@pytest.mark.parametrize("n", [1, 7, 8, 9, 2047, 8 * 256 * 2048 + 13])
def test_sizes(n):
    rng = np.random.default_rng(n)
    x = _vol(rng, np.float32, n, "normal")
    y = _vol(rng, np.float32, n, "poisson")
    check(x, y)


@pytest.mark.parametrize("x_off,y_off", [(4, 0), (0, 2), (1, 3)])
def test_misaligned_bases(x_off, y_off):
    rng = np.random.default_rng(7)
    n = 100003
    x = _vol(rng, np.uint8, n, "wide")
    y = _vol(rng, np.uint16, n, "wide") if y_off % 2 == 0 else _vol(rng, np.uint8, n, "poisson")
    check(x, y, x_off=x_off, y_off=y_off)


@pytest.mark.parametrize("nb", [2, 3, 255, 256, 4096, 8192])
def test_bins(nb):
    rng = np.random.default_rng(nb)
    x = _vol(rng, np.float32, 200000, "normal")
    y = _vol(rng, np.uint16, 200000, "wide")
    check(x, y, n_bins=nb)


def test_degenerate_volumes():
    n = 4099
    c = np.full(n, 3.5, np.float32)
    r = check(c, c.copy())
    assert r.std[0] == 0.0 and r.entropy[0] == 0.0 and r.mse == 0.0 and math.isinf(r.psnr)
    two = np.where(np.arange(n) % 2 == 0, 0, 255).astype(np.uint8)
    r = check(two, c)
    assert abs(r.entropy[0] - M.entropy_bits([2050, 2049])) < 1e-12
    check(np.array([5.0], np.float32))


def test_paper_peak():
    rng = np.random.default_rng(3)
    x = _vol(rng, np.float32, 50000, "poisson")
    y = _vol(rng, np.float32, 50000, "normal")
    check(x, y, peak=M.PAPER_PSNR_PEAK)


@pytest.mark.timeout(300)
def test_against_clahe_result_full_size():
    """The 4D benchmark volume (256x256x128x32 float) against its CLAHE result."""
    import torch
    from paper_1906_11355_amd import api, synth
    x = synth.gen_4d()
    xt = torch.from_numpy(x).cuda()
    y = api.enhance(xt, (32, 32, 16, 8), 512, 0.02).cpu().numpy()
    r = check(x, y, n_bins=256, peak=M.PAPER_PSNR_PEAK)
    # the result is contrast-enhanced: more spread and more grey-level entropy
    assert r.std[1] > r.std[0] and r.entropy[1] > r.entropy[0]


def test_api_metrics_matches_abi():
    import torch
    from paper_1906_11355_amd import api
    rng = np.random.default_rng(5)
    x = _vol(rng, np.float32, 70001, "poisson")
    y = _vol(rng, np.float32, 70001, "normal")
    d = api.metrics(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), n_bins=64, with_hist=True)
    r, h = gpu_metrics(x, y, 64)
    assert d["mse"] == r.mse and d["std"] == [r.std[0], r.std[1]]
    np.testing.assert_array_equal(d["hist"][1], h[64:])
