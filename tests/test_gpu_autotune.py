"""Autotuner: picks a decomposition on the GPU, never changes a bit of the
result, and is remembered for later plans of the same problem."""
import numpy as np
import pytest

from gpu_util import NP_CODE, gpu_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["global", "kernel"])
def test_autotune_keeps_bits_and_is_cached(mode):
    import torch
    from paper_1906_11355_amd import _lib, synth
    x = synth.gen_4d((96, 80, 64, 16), 31, slab=8)
    ks = (24, 20, 16, 8)
    before = gpu_run(x, ks, 256, 0.02, mode)
    p = _lib.Plan(x.shape, ks, 256, 0.02, mode, in_dtype=NP_CODE[x.dtype])
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    ws = torch.empty(p.autotune_workspace_size(), dtype=torch.uint8, device="cuda")
    p.autotune_ptr(xt.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    t = p.tuning()
    assert t["hist_copies"] in (1, 2, 4, 8) and 1 <= t["hist_peel"] <= 3
    assert 1 <= t["map_unit_chunks"] <= t["map_rows_split"]
    after = gpu_run(x, ks, 256, 0.02, mode, plan=p)
    for k in ("out", "hist", "clipped", "lut", "range"):
        np.testing.assert_array_equal(after[k], before[k], err_msg=f"{k} changed by autotuning")
    q = _lib.Plan(x.shape, ks, 256, 0.02, mode, in_dtype=NP_CODE[x.dtype])
    assert q.tuning() == t          # later plans of the same problem start tuned
