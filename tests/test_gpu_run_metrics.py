"""mclahe_run_metrics: a CLAHE run that computes the contrast metrics of its
input and output on the way (the interpolation units write the minimum,
maximum and sum of both; one pass over both volumes adds the centred sums
and the grey-level histograms).

The output must be bit-identical to mclahe_run's; the metrics must agree
with the oracle (oracle/metrics.py) within the tolerances of the standalone
metric tests: ranges and histogram counts exact, means, standard deviations
and the MSE within a relative 1e-9, entropies within 1e-12, the PSNR within
1e-8 dB.  The metrics are those of the stored output (integer codes for
8- and 16-bit output).
"""
import ctypes

import numpy as np
import pytest

from gpu_util import NP_CODE, from_device_bytes, to_device_bytes
from oracle import metrics as M
from test_gpu_metrics import close

pytestmark = pytest.mark.gpu

# shape, kernel, clip bins, clip, mode, input dtype, output dtype, metric bins, (in, out) offsets
CASES = [
    ((40, 36, 20, 8), (10, 9, 5, 4), 256, 0.02, "global", np.float32, np.float32, 256, (0, 0)),
    ((40, 36, 20, 8), (10, 9, 5, 4), 128, 0.03, "kernel", np.float32, np.float32, 256, (0, 0)),
    ((61, 47, 33), (13, 9, 7), 128, 0.03, "kernel", np.float32, np.uint8, 64, (4, 0)),
    ((300, 517), (64, 50), 256, 0.01, "global", np.uint8, np.uint8, 256, (1, 3)),
    ((257, 1000), (64, 100), 256, 0.02, "global", np.uint16, np.uint16, 4096, (0, 0)),
    ((9, 8, 7, 6, 5), (3, 3, 3, 3, 3), 64, 0.05, "global", np.float32, np.float32, 32, (0, 0)),   # generic map
    ((17, 33, 9), (5, 7, 3), 64, 0.0, "kernel", np.float32, np.float32, 2, (8, 4)),
]


def _input(shape, dt, seed):
    rng = np.random.default_rng(seed)
    x = rng.poisson(3.0, size=shape) + (rng.random(shape) < 0.02) * rng.integers(0, 200, size=shape)
    if dt == np.uint16:
        x = x * 250
    return x.astype(dt)


def run_with_metrics(x, ks, nb, clip, mode, odt, mbins, peak, off=(0, 0)):
    import torch
    from paper_1906_11355_amd import _lib
    plan = _lib.Plan(x.shape, ks, nb, clip, mode, in_dtype=NP_CODE[x.dtype], out_dtype=NP_CODE[np.dtype(odt)])
    st = torch.cuda.current_stream().cuda_stream
    ib, ip = to_device_bytes(x, off[0])
    nbytes = x.size * np.dtype(odt).itemsize
    ob = torch.zeros(nbytes + off[1] + 64, dtype=torch.uint8, device="cuda")
    op = ob.data_ptr() + off[1]
    rb = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    need = plan.run_metrics_workspace_size(mbins)
    assert need >= plan.workspace_size()
    ws = torch.full((need,), 0xAB, dtype=torch.uint8, device="cuda")      # poisoned
    res = torch.zeros(ctypes.sizeof(_lib.MetricsResult), dtype=torch.uint8, device="cuda")
    hist = torch.full((2 * mbins,), -1, dtype=torch.int64, device="cuda")
    plan.run_metrics_ptr(ip, op, ws.data_ptr(), need, mbins, peak, res.data_ptr(), hist.data_ptr(), st)
    ws2 = torch.empty(plan.workspace_size(), dtype=torch.uint8, device="cuda")
    plan.run_ptr(ip, rb.data_ptr(), ws2.data_ptr(), ws2.numel(), st)
    torch.cuda.synchronize()
    y = from_device_bytes(ob, op, x.shape, odt)
    ref = from_device_bytes(rb, rb.data_ptr(), x.shape, odt)
    r = _lib.MetricsResult.from_buffer_copy(bytes(res.cpu().numpy()))
    return y, ref, r, hist.cpu().numpy()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_run_metrics_matches_run_and_oracle(case):
    shape, ks, nb, clip, mode, dt, odt, mbins, off = CASES[case]
    print(f"run-metrics case {case}: {CASES[case]}", flush=True)
    x = _input(shape, dt, 90 + case)
    peak = M.PAPER_PSNR_PEAK
    y, ref, r, h = run_with_metrics(x, ks, nb, clip, mode, odt, mbins, peak, off)
    np.testing.assert_array_equal(y, ref, err_msg="output differs from mclahe_run")
    e = M.metrics(x, y, mbins, peak)
    for v, vol in enumerate((x, y)):
        tag = f"case {case} vol{v}"
        assert r.lo[v] == e["lo"][v] and r.hi[v] == e["hi"][v], tag
        np.testing.assert_array_equal(h[v * mbins:(v + 1) * mbins], M.grey_histogram(vol, mbins), err_msg=tag)
        close(r.mean[v], e["mean"][v], 1e-9, tag + " mean")
        close(r.std[v], e["std"][v], 1e-9, tag + " std")
        close(r.entropy[v], e["entropy"][v], 1e-12, tag + " entropy")
    close(r.mse, e["mse"], 1e-9, "mse")
    assert abs(r.psnr - e["psnr"]) <= 1e-8, (r.psnr, e["psnr"])
    assert r.count == x.size


def test_run_metrics_full_4d_volume():
    """The 256x256x128x32 photoemission-like volume (both range modes)."""
    from paper_1906_11355_amd import synth
    x = synth.gen_4d()
    for mode in ("global", "kernel"):
        y, ref, r, h = run_with_metrics(x, (32, 32, 16, 8), 512, 0.02, mode, np.float32, 256, M.PAPER_PSNR_PEAK)
        np.testing.assert_array_equal(y, ref, err_msg=mode)
        e = M.metrics(x, y, 256, M.PAPER_PSNR_PEAK)
        for v in range(2):
            assert r.lo[v] == e["lo"][v] and r.hi[v] == e["hi"][v]
            close(r.std[v], e["std"][v], 1e-9, f"{mode} std{v}")
            close(r.entropy[v], e["entropy"][v], 1e-12, f"{mode} entropy{v}")
        close(r.mse, e["mse"], 1e-9, f"{mode} mse")


def test_run_metrics_rejects_in_place_and_bad_arguments():
    import torch
    from paper_1906_11355_amd import _lib
    x = _input((32, 40), np.float32, 1)
    plan = _lib.Plan(x.shape, (8, 10), 64, 0.02)
    xt = torch.from_numpy(x).cuda()
    need = plan.run_metrics_workspace_size(64)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    res = torch.zeros(ctypes.sizeof(_lib.MetricsResult), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(xt)
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(_lib.MclaheError) as ei:
        plan.run_metrics_ptr(xt.data_ptr(), xt.data_ptr(), ws.data_ptr(), need, 64, 1.0, res.data_ptr(), None, st)
    assert ei.value.status == _lib.INVALID_VALUE
    with pytest.raises(_lib.MclaheError) as ei:
        plan.run_metrics_ptr(xt.data_ptr(), out.data_ptr(), ws.data_ptr(), need - 256, 64, 1.0, res.data_ptr(),
                             None, st)
    assert ei.value.status == _lib.WORKSPACE
    with pytest.raises(_lib.MclaheError) as ei:
        plan.run_metrics_ptr(xt.data_ptr(), out.data_ptr(), ws.data_ptr(), need, 64, 0.0, res.data_ptr(), None, st)
    assert ei.value.status == _lib.INVALID_VALUE
    torch.cuda.synchronize()
