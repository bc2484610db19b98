"""mclahe_run under stream capture: the library only enqueues kernels (no
allocation, no memset, no synchronisation), so a caller can capture a run in
a hipGraph and replay it.  Every replay, with the program's own eager work
and synchronisations between replays, must equal the eager result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["global", "kernel"])
def test_captured_run_replays_match_eager(mode):
    import torch
    from paper_1906_11355_amd import _lib, synth
    x = synth.gen_4d((64, 48, 32, 16), 41, slab=8)
    p = _lib.Plan(x.shape, (16, 12, 8, 8), 256, 0.02, mode)
    xt = torch.from_numpy(x).cuda()
    eager = torch.empty_like(xt)
    ws = torch.empty(p.workspace_size(), dtype=torch.uint8, device="cuda")
    p.run_ptr(xt.data_ptr(), eager.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = torch.zeros_like(xt)
    ws2 = torch.full((p.workspace_size(),), 0xAB, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            p.run_ptr(xt.data_ptr(), out.data_ptr(), ws2.data_ptr(), ws2.numel(), s.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(4):
        out.zero_()
        a = torch.randn(1 << 20, device="cuda")
        (a * 2).sum().item()                   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep} differs"
