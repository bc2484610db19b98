"""Largest sizes: a volume of more than 2^32 voxels through mclahe_run.

A 65536 x 65600 uint8 image (4.30 G voxels, so element offsets need 64
bits) with 256x256 kernels, 256 bins, clip 0.01, global range and uint8
output, against the full CPU oracle: histograms and clipped counts
bit-exact, output within one level.  Needs about 35 GB of host memory and
a minute of CPU time for the oracle.
"""
import numpy as np
import pytest

import oracle
from gpu_util import collect

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_more_than_2e32_voxels():
    import torch
    from paper_1906_11355_amd import _lib
    shape, ks, nb, clip = (65536, 65600), (256, 256), 256, 0.01
    print(f"large case: {shape} u8 kernel {ks}", flush=True)
    rng = np.random.default_rng(31)
    # noise plus a gradient along both axes, so that the kernels' histograms
    # differ (built in row blocks to bound the host memory)
    x = np.empty(shape, np.uint8)
    colg = (np.arange(shape[1]) // 1024).astype(np.int16)
    for r0 in range(0, shape[0], 4096):
        r1 = min(shape[0], r0 + 4096)
        rowg = (np.arange(r0, r1) // 1024).astype(np.int16)[:, None]
        x[r0:r1] = rng.integers(0, 160, size=(r1 - r0, shape[1]), dtype=np.uint8) + ((rowg + colg) // 2).astype(np.uint8)
    plan = _lib.Plan(shape, ks, nb, clip, "global", in_dtype="uint8", out_dtype="uint8")
    xt = torch.from_numpy(x).cuda()
    ob = torch.empty(x.size, dtype=torch.uint8, device="cuda")
    ws = torch.empty(plan.workspace_size(), dtype=torch.uint8, device="cuda")
    plan.run_ptr(xt.data_ptr(), ob.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    del xt
    g = collect(plan, ws, 0, ob, ob.data_ptr(), shape, np.uint8)
    del ob, ws
    torch.cuda.empty_cache()
    print("gpu done; oracle", flush=True)
    r = oracle.run(x, ks, nb, clip, oracle.GLOBAL, out_dtype=np.uint8)
    np.testing.assert_array_equal(g["hist"], r["hist"])
    np.testing.assert_array_equal(g["clipped"], r["clipped"])
    assert np.abs(g["lut"].astype(np.float64) - r["lut"]).max() <= 1e-5
    d = np.abs(g["out"].astype(np.int16) - r["out"].astype(np.int16))
    assert int(d.max()) <= 1, int(d.max())
