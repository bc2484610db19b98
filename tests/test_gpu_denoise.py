"""GPU parity of the pre-denoising filters (mclahe_gaussian, mclahe_median).

Both sides follow one stated arithmetic (float32 fused multiply-add chain in
tap order; the median is a selection), so the GPU results must equal the
oracle's bit for bit.  Cases: every dtype, 1 to 5 axes, zero sigmas, radii
longer than the axis (repeated reflection), radii beyond the register ring
(direct taps), vector and element paths (strides not a multiple of 4,
misaligned bases), the paper's sigmas on the 256x256x128x32 volume at full
size, CLAHE on the smoothed volume, and median windows up to 64 values.
"""
import numpy as np
import pytest

from gpu_util import NP_CODE, to_device_bytes
from oracle import denoise as DN

pytestmark = pytest.mark.gpu


def gpu_gaussian(x, sigma, truncate=4.0, in_off=0, out_off=0):
    import torch
    from paper_1906_11355_amd import _lib
    ib, ip = to_device_bytes(x, in_off)
    ob = torch.full((x.size * 4 + out_off + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    op = ob.data_ptr() + out_off
    need = _lib.gaussian_workspace_size(x.shape, sigma)
    ws = torch.full((max(need, 1),), 0xCD, dtype=torch.uint8, device="cuda")
    _lib.gaussian_ptr(ip, NP_CODE[x.dtype], x.shape, sigma, truncate, op, ws.data_ptr() if need else None, need,
                      torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return ob[out_off:out_off + x.size * 4].cpu().numpy().view(np.float32).reshape(x.shape)


def gpu_median(x, window, in_off=0, out_off=0):
    import torch
    from paper_1906_11355_amd import _lib
    ib, ip = to_device_bytes(x, in_off)
    nb = x.size * x.itemsize
    ob = torch.full((nb + out_off + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    op = ob.data_ptr() + out_off
    _lib.median_ptr(ip, NP_CODE[x.dtype], x.shape, window, op, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return ob[out_off:out_off + nb].cpu().numpy().view(x.dtype).reshape(x.shape)


def _data(rng, shape, dt):
    if dt == np.uint8:
        return rng.integers(0, 256, size=shape).astype(np.uint8)
    if dt == np.uint16:
        return rng.integers(0, 65536, size=shape).astype(np.uint16)
    return (rng.poisson(3.0, size=shape) * np.float32(0.37) + rng.random(shape)).astype(np.float32)


GAUSS_CASES = [
    ((1000,), (1.3,), np.float32),
    ((2,), (1.3,), np.float32),                        # radius 5 on 2 samples
    ((1,), (0.7,), np.uint8),
    ((37, 41), (0.7, 0.9), np.float32),               # strides not a multiple of 4
    ((40, 44), (0.7, 0.9), np.uint16),
    ((9, 8, 12), (0.7, 0.9, 1.3), np.uint8),
    ((7, 5, 3), (1.3, 0.0, 0.9), np.float32),
    ((6, 5, 7, 9), (0.7, 0.7, 0.9, 1.3), np.float32),
    ((16, 12, 20, 8), (0.7, 0.7, 0.9, 1.3), np.float32),
    ((5, 3, 4, 2, 6), (0.6, 1.0, 0.0, 1.7, 0.8), np.uint16),
    ((33, 70), (2.5, 3.1), np.float32),                # radii 10 and 12: direct taps
    ((12, 3000), (0.0, 0.0), np.uint16),               # nothing to smooth: conversion
    ((3, 4096 * 3 + 5), (1.9, 1.1), np.float32),       # several last-axis tiles, ragged
    ((5000,), (2.5,), np.uint8),                       # long row, radius 10: flat tile, any radius
    ((3000, 1), (0.0, 5.0), np.float32),               # rows of one sample, radius 20
    ((7, 2048), (0.0, 0.9), np.float32),               # one row per work-group
    ((20, 500), (16.0, 16.0), np.float32),             # radius 64: too wide to fuse the last two axes
    ((3, 2, 512), (0.0, 1.4, 0.6), np.uint8),          # fused last two axes, longest fused rows, first pass
    ((4, 9, 1), (0.8, 2.2, 3.0), np.float32),          # fused, rows of one sample, generic radii
    # two leading strided axes in one pass
    ((3, 40, 30, 6), (0.9, 1.3, 0.0, 0.7), np.float32),  # radii 4 and 5, two row tiles, wide vectors
    ((70, 3, 5, 4), (0.7, 1.3, 0.9, 0.0), np.uint8),     # second axis shorter than its radius, first pass
    ((3, 11, 9, 2, 5), (0.0, 0.7, 0.9, 0.0, 1.1), np.float32),  # pair after an outer axis, scalar columns
    ((130, 27, 2, 8), (0.4, 0.7, 0.0, 0.0), np.uint16),  # radii 2 and 3, segments of the first axis
]


@pytest.mark.parametrize("shape,sigma,dt", GAUSS_CASES)
def test_gaussian_bit_exact(shape, sigma, dt):
    rng = np.random.default_rng(sum(shape) + 7 * len(shape))
    x = _data(rng, shape, dt)
    g = gpu_gaussian(x, sigma)
    r = DN.gaussian(x, sigma)
    np.testing.assert_array_equal(g, r, err_msg=f"{shape} {sigma} {dt}")


@pytest.mark.parametrize("in_off,out_off", [(4, 0), (0, 4), (2, 8)])
def test_gaussian_misaligned(in_off, out_off):
    rng = np.random.default_rng(5)
    x = _data(rng, (12, 16, 20), np.uint16 if in_off == 2 else np.float32)
    np.testing.assert_array_equal(gpu_gaussian(x, (0.9, 0.7, 1.3), in_off=in_off, out_off=out_off),
                                  DN.gaussian(x, (0.9, 0.7, 1.3)))
    # the two-axis pass with unaligned buffers (single-element columns)
    x4 = _data(rng, (8, 9, 6, 8), np.uint16 if in_off == 2 else np.float32)
    np.testing.assert_array_equal(gpu_gaussian(x4, (0.7, 0.7, 0.9, 1.3), in_off=in_off, out_off=out_off),
                                  DN.gaussian(x4, (0.7, 0.7, 0.9, 1.3)))


@pytest.mark.timeout(300)
def test_gaussian_full_size_and_clahe():
    """The paper's photoemission sigmas on the 256x256x128x32 volume (bit-exact),
    then CLAHE of both smoothed volumes: histograms equal."""
    import torch
    from gpu_util import assert_parity, gpu_run, oracle_run
    from paper_1906_11355_amd import synth
    sig = (0.7, 0.7, 0.9, 1.3)
    x = synth.gen_4d()
    g = gpu_gaussian(x, sig)
    r = DN.gaussian(x, sig)
    assert np.array_equal(g, r)
    torch.cuda.empty_cache()
    # CLAHE of the smoothed 3D-per-frame sized block (bit-exact inputs -> exact histograms)
    xs = r[:64, :64, :64, :8].copy()
    gr = gpu_run(xs, (16, 16, 16, 4), 256, 0.02, "global")
    assert_parity(gr, oracle_run(xs, (16, 16, 16, 4), 256, 0.02, "global"), what="smoothed clahe")


MEDIAN_CASES = [
    ((5, 4, 6, 3), (2, 2, 2, 1), np.uint8),
    ((17, 9, 11, 4), (2, 2, 2, 1), np.uint8),
    ((1, 3, 2, 2), (2, 2, 2, 1), np.uint8),
    ((7, 8), (3, 3), np.float32),
    ((1000,), (2,), np.uint16),
    ((6, 2, 5), (4, 1, 3), np.float32),
    ((9, 9, 9), (4, 4, 4), np.uint16),                # 64 values
    ((10, 11, 12), (3, 3, 3), np.uint8),              # 27 values, padded to 32
    ((1,), (5,), np.float32),
]


@pytest.mark.parametrize("shape,window,dt", MEDIAN_CASES)
def test_median_exact(shape, window, dt):
    rng = np.random.default_rng(sum(shape) + len(window))
    x = _data(rng, shape, dt)
    np.testing.assert_array_equal(gpu_median(x, window), DN.median(x, window), err_msg=f"{shape} {window}")


@pytest.mark.timeout(300)
def test_median_over_2e31_voxels_sampled():
    """The microscopy window on a uint8 volume of 512x512x109x80 voxels (over
    2^31: 64-bit coordinates), checked at sampled voxels, all borders
    included, and as a whole against the 32-bit path on its first frames."""
    import torch
    shape = (512, 512, 109, 80)
    g = torch.Generator(device="cpu").manual_seed(21)
    x = torch.randint(0, 256, shape, dtype=torch.uint8, generator=g)
    xt = x.cuda()
    out = torch.empty_like(xt)
    from paper_1906_11355_amd import _lib
    _lib.median_ptr(xt.data_ptr(), _lib.U8, shape, (2, 2, 2, 1), out.data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    rng = np.random.default_rng(22)
    pts = np.stack([rng.integers(0, n, 20000) for n in shape], axis=1)
    pts[:64, 0] = 0
    pts[64:128, 1] = 0
    pts[128:192, 2] = 0
    pts[192:256] = [[0, 0, 0, 0], [511, 511, 108, 79]] * 32
    xn = x.numpy()
    got = out[tuple(torch.from_numpy(pts[:, a]).cuda() for a in range(4))].cpu().numpy()
    np.testing.assert_array_equal(got, DN.median_at(xn, (2, 2, 2, 1), pts))
    del out, xt
    torch.cuda.empty_cache()


def test_median_misaligned():
    rng = np.random.default_rng(9)
    x = _data(rng, (8, 7, 6, 5), np.uint8)
    np.testing.assert_array_equal(gpu_median(x, (2, 2, 2, 1), in_off=1, out_off=3),
                                  DN.median(x, (2, 2, 2, 1)))


def test_api_wrappers():
    import torch
    from paper_1906_11355_amd import api
    rng = np.random.default_rng(4)
    x = _data(rng, (11, 13, 6), np.uint8)
    xt = torch.from_numpy(x).cuda()
    np.testing.assert_array_equal(api.gaussian(xt, (0.7, 0.9, 0.0)).cpu().numpy(), DN.gaussian(x, (0.7, 0.9, 0.0)))
    np.testing.assert_array_equal(api.median(xt, (2, 2, 1)).cpu().numpy(), DN.median(x, (2, 2, 1)))
