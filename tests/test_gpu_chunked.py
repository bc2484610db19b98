"""Out-of-core (chunked) runs: host-resident input and output streamed through
the device in slabs of kernel layers along axis 0 must give bit-identical
outputs to the whole-volume run, for every slab size, both range modes, a
caller range, every dimensionality from 2 to 5 and every dtype; and the
oracle agrees within the parity tolerance.
"""
import numpy as np
import pytest

from gpu_util import NP_CODE, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


def _chunked(x, ks, nb, clip, mode, L, user_range=None, out_dtype=np.float32):
    import torch
    from paper_1906_11355_amd import _lib
    p = _lib.Plan(x.shape, ks, nb, clip, mode, user_range, in_dtype=NP_CODE[x.dtype],
                  out_dtype=NP_CODE[np.dtype(out_dtype)])
    hin = torch.from_numpy(np.ascontiguousarray(x).view(np.uint8).reshape(-1)).pin_memory()
    hout = torch.full((x.size * np.dtype(out_dtype).itemsize,), 0xEE, dtype=torch.uint8).pin_memory()
    wsb = p.chunked_workspace_size(L)
    ws = torch.full((wsb,), 0xAB, dtype=torch.uint8, device="cuda")
    p.run_chunked_ptr(hin.data_ptr(), hout.data_ptr(), L, ws.data_ptr(), wsb,
                      torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return hout.numpy().view(out_dtype).reshape(x.shape)


CASES = [
    # shape, kernel, bins, clip, mode, dtype
    ((300, 257), (64, 50), 256, 0.02, "global", np.uint16),
    ((61, 47, 33), (13, 9, 7), 128, 0.03, "global", np.float32),
    ((61, 47, 33), (13, 9, 7), 128, 0.03, "kernel", np.float32),
    ((40, 24, 20, 8), (8, 6, 5, 4), 512, 0.02, "global", np.float32),
    ((40, 24, 20, 8), (9, 6, 5, 3), 64, 0.05, "kernel", np.float32),
    ((37, 30), (5, 7), 64, 0.1, "global", np.uint8),
    ((12, 5, 4, 3, 7), (3, 2, 2, 2, 3), 16, 0.1, "kernel", np.float32),
]


def _data(shape, dtype, seed):
    rng = np.random.default_rng(seed)
    if dtype == np.uint8:
        return rng.integers(0, 256, size=shape).astype(np.uint8)
    if dtype == np.uint16:
        return rng.integers(0, 60000, size=shape).astype(np.uint16)
    return rng.poisson(3.0, size=shape).astype(np.float32)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_chunked_bit_identical_to_whole_volume(case):
    shape, ks, nb, clip, mode, dt = CASES[case]
    x = _data(shape, dt, case)
    whole = gpu_run(x, ks, nb, clip, mode)["out"]
    n0 = (shape[0] - 1) // ks[0] + 2
    for L in sorted({1, 2, 3, n0 - 1, n0, n0 + 5}):
        if L < 1:
            continue
        got = _chunked(x, ks, nb, clip, mode, L)
        np.testing.assert_array_equal(got, whole, err_msg=f"case {case} slab_layers={L}")


def test_chunked_user_range_and_integer_output():
    x = _data((50, 70), np.float32, 11) * 0.37
    whole = gpu_run(x, (10, 12), 64, 0.05, "global", user_range=(0.2, 2.0), out_dtype=np.uint8)["out"]
    for L in (1, 2, 4):
        got = _chunked(x, (10, 12), 64, 0.05, "global", L, user_range=(0.2, 2.0), out_dtype=np.uint8)
        np.testing.assert_array_equal(got, whole, err_msg=f"slab_layers={L}")


def test_chunked_matches_oracle():
    from paper_1906_11355_amd import synth
    x = synth.gen_4d((48, 40, 32, 8), 21, slab=8)
    for mode in ("global", "kernel"):
        r = oracle_run(x, (12, 10, 8, 4), 256, 0.02, mode)
        got = _chunked(x, (12, 10, 8, 4), 256, 0.02, mode, 2)
        d = np.abs(got.astype(np.float64) - r["out"]).max()
        assert d <= 1e-5, f"{mode}: max |diff| {d}"
