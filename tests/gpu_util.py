"""Helpers for the GPU parity tests: run the C-ABI library on numpy inputs and
compare every intermediate with the CPU oracle.

Inputs come from the tests (seeded numpy); expected values come only from the
oracle.  The library is called through its C ABI with raw device buffers
(torch tensors of bytes), so the comparison covers exactly what the ABI does.
"""
from __future__ import annotations

import numpy as np

import oracle

NP_CODE = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float32): 2}
ORACLE_MODE = {"global": oracle.GLOBAL, "kernel": oracle.KERNEL}


def _torch():
    import torch
    return torch


def to_device_bytes(a: np.ndarray, offset: int = 0):
    """Copy an array into a fresh device byte buffer, optionally at a byte offset."""
    torch = _torch()
    raw = np.ascontiguousarray(a).view(np.uint8).reshape(-1)
    buf = torch.empty(raw.size + offset + 64, dtype=torch.uint8, device="cuda")
    buf[offset:offset + raw.size].copy_(torch.from_numpy(raw))
    return buf, buf.data_ptr() + offset


def from_device_bytes(buf, ptr: int, shape, dtype) -> np.ndarray:
    n = int(np.prod(shape)) * np.dtype(dtype).itemsize
    off = ptr - buf.data_ptr()
    return buf[off:off + n].cpu().numpy().view(dtype).reshape(shape)


def gpu_run(x: np.ndarray, ks, nb, clip, mode="global", user_range=None, out_dtype=np.float32,
            tuning=None, in_offset=0, out_offset=0, plan=None, inplace=False):
    """Run mclahe_run; returns out plus every workspace array as numpy."""
    torch = _torch()
    from paper_1906_11355_amd import _lib
    if plan is None:
        plan = _lib.Plan(x.shape, ks, nb, clip, mode, user_range,
                         in_dtype=NP_CODE[x.dtype], out_dtype=NP_CODE[np.dtype(out_dtype)])
    if tuning:
        plan.set_tuning(**tuning)
    ib, ip = to_device_bytes(x, in_offset)
    if inplace:
        ob, op = ib, ip
    else:
        nbytes = x.size * np.dtype(out_dtype).itemsize
        ob = torch.zeros(nbytes + out_offset + 64, dtype=torch.uint8, device="cuda")
        op = ob.data_ptr() + out_offset
    wsz = plan.workspace_size()
    ws = torch.full((wsz,), 0xAB, dtype=torch.uint8, device="cuda")   # poisoned workspace
    plan.run_ptr(ip, op, ws.data_ptr(), wsz, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return collect(plan, ws, 0, ob, op, x.shape, out_dtype)


def collect(plan, ws, base, ob, op, shape, out_dtype):
    lay = plan.layout()
    g = plan.geometry()
    nk, nb = g["n_kernels"], plan.n_bins
    w = ws[base:base + lay["total"]].cpu().numpy()

    def arr(off, count, dt):
        return w[off:off + count * np.dtype(dt).itemsize].view(dt)

    ahr = plan.mode == 1
    return dict(
        out=from_device_bytes(ob, op, shape, out_dtype),
        hist=arr(lay["hist"], nk * nb, np.uint32).reshape(nk, nb).astype(np.int64),
        clipped=arr(lay["clipped"], nk * nb, np.uint64).reshape(nk, nb).astype(np.int64),
        lut=arr(lay["lut"], nk * nb, np.float32).reshape(nk, nb),
        range=arr(lay["range"], nk * 2 if ahr else 2, np.float32).reshape((nk, 2) if ahr else (2,)),
        scale=arr(lay["scale"], nk if ahr else 1, np.float32),
    )


def oracle_run(x, ks, nb, clip, mode="global", user_range=None, out_dtype=np.float32):
    return oracle.run(x, ks, nb, clip, ORACLE_MODE[mode], user_range=user_range, out_dtype=out_dtype)


def assert_parity(g, r, out_dtype=np.float32, tol=1e-5, what=""):
    """Histograms, clipped counts, ranges and LUTs bit-exact; output within
    tolerance.  A LUT entry is one double division of exact integers rounded
    once to float, so it has exactly one correct value (compared bit for bit,
    beside the tolerance the output is held to)."""
    np.testing.assert_array_equal(g["hist"], r["hist"], err_msg=f"{what}: histograms")
    np.testing.assert_array_equal(g["clipped"], r["clipped"], err_msg=f"{what}: clipped counts")
    np.testing.assert_array_equal(g["range"], r["range"], err_msg=f"{what}: ranges")
    dl = np.abs(g["lut"].astype(np.float64) - r["lut"].astype(np.float64)).max()
    assert dl <= tol, f"{what}: LUT max |diff| {dl}"
    np.testing.assert_array_equal(g["lut"].view(np.uint32), np.asarray(r["lut"], np.float32).view(np.uint32),
                                  err_msg=f"{what}: LUT bits")
    if np.dtype(out_dtype) == np.float32:
        do = np.abs(g["out"].astype(np.float64) - r["out"].astype(np.float64)).max()
        assert do <= tol, f"{what}: output max |diff| {do}"
    else:
        do = np.abs(g["out"].astype(np.int64) - r["out"].astype(np.int64)).max()
        assert do <= 1, f"{what}: integer output max |diff| {do} levels"
    return dl, do
