"""PyTorch-facing entry points: tensors in, tensors out, on the current stream.

PyTorch only supplies device memory and streams; the work is done by the
library's HIP kernels through the C ABI (see ``_lib``).
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib
from ._lib import F32, KERNEL, U8, U16, Plan

TORCH_DTYPE = {U8: torch.uint8, U16: torch.uint16, F32: torch.float32}


def stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def plan_for(x: torch.Tensor, kernel_size: Sequence[int], n_bins: int = 256, clip_limit: float = 0.01,
             mode="global", user_range=None, out_dtype=torch.float32) -> Plan:
    return Plan(tuple(x.shape), kernel_size, n_bins, clip_limit, mode, user_range,
                in_dtype=x.dtype, out_dtype=out_dtype)


def _check_tensor(x: torch.Tensor, name: str):
    if not x.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check_against_plan(plan: Plan, x: torch.Tensor, out: torch.Tensor | None, what: str = ""):
    """The C ABI receives raw pointers only: make sure the tensors are what the
    plan describes, so that no kernel reads or writes past them."""
    if tuple(x.shape) != plan.shape:
        raise ValueError(f"{what}input shape {tuple(x.shape)} differs from the plan's {plan.shape}")
    if _lib.dtype_code(x.dtype) != plan.in_code:
        raise ValueError(f"{what}input dtype {x.dtype} differs from the plan's {TORCH_DTYPE[plan.in_code]}")
    if out is not None:
        if tuple(out.shape) != plan.shape:
            raise ValueError(f"{what}output shape {tuple(out.shape)} differs from the plan's {plan.shape}")
        if out.dtype != TORCH_DTYPE[plan.out_code]:
            raise ValueError(f"{what}output dtype {out.dtype} differs from the plan's {TORCH_DTYPE[plan.out_code]}")
        if out.device != x.device:
            raise ValueError(f"{what}output is on {out.device}, input on {x.device}")


def _check_workspace(ws: torch.Tensor, need: int, device):
    if ws.device != device:
        raise ValueError(f"workspace is on {ws.device}, input on {device}")
    if ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace holds {ws.numel() * ws.element_size()} bytes, {need} needed")


def enhance(x: torch.Tensor, kernel_size: Sequence[int], n_bins: int = 256, clip_limit: float = 0.01,
            mode="global", user_range=None, out_dtype=torch.float32, plan: Plan | None = None,
            workspace: torch.Tensor | None = None, out: torch.Tensor | None = None,
            return_workspace: bool = False):
    """Multidimensional CLAHE of one volume (asynchronous on the current stream)."""
    _check_tensor(x, "input")
    if plan is None:
        plan = plan_for(x, kernel_size, n_bins, clip_limit, mode, user_range, out_dtype)
    need = plan.workspace_size()
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    _check_tensor(workspace, "workspace")
    _check_workspace(workspace, need, x.device)
    if out is None:
        out = torch.empty(x.shape, dtype=TORCH_DTYPE[plan.out_code], device=x.device)
    _check_tensor(out, "output")
    _check_against_plan(plan, x, out)
    plan.run_ptr(x.data_ptr(), out.data_ptr(), workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                 stream_handle(x.device))
    return (out, workspace, plan) if return_workspace else out


def read_workspace(plan: Plan, ws: torch.Tensor, base: int = 0) -> dict:
    """Views of the intermediate arrays (hist, clipped, lut, range, scale)."""
    lay = plan.layout()
    g = plan.geometry()
    nk, nb = g["n_kernels"], plan.n_bins
    ahr = plan.mode == KERNEL

    def view(off, count, dtype, esize):
        return ws[base + off: base + off + count * esize].view(dtype)

    return dict(
        hist=view(lay["hist"], nk * nb, torch.int32, 4).view(nk, nb),
        clipped=view(lay["clipped"], nk * nb, torch.int64, 8).view(nk, nb),
        lut=view(lay["lut"], nk * nb, torch.float32, 4).view(nk, nb),
        range=view(lay["range"], (nk * 2 if ahr else 2), torch.float32, 4).view(-1, 2) if ahr
        else view(lay["range"], 2, torch.float32, 4),
        scale=view(lay["scale"], nk if ahr else 1, torch.float32, 4),
    )


def make_plans(xs: Sequence[torch.Tensor], params: Sequence[dict]) -> list:
    return [plan_for(x, **p) for x, p in zip(xs, params)]


def enhance_batched(xs: Sequence[torch.Tensor], params: Sequence[dict] | None = None, plans=None,
                    outs=None, workspace: torch.Tensor | None = None, return_workspace: bool = False):
    """Enhance many volumes as one batch: one launch per pass over all volumes (hipGraph)."""
    if plans is None:
        plans = make_plans(xs, params)
    if len(plans) != len(xs) or (outs is not None and len(outs) != len(xs)):
        raise ValueError("one plan (and one output) per input volume")
    dev = xs[0].device
    for i, x in enumerate(xs):
        _check_tensor(x, f"input {i}")
        if x.device != dev:
            raise ValueError(f"input {i} is on {x.device}, input 0 on {dev}")
    need = _lib.batched_workspace_size(plans)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _check_tensor(workspace, "workspace")
    _check_workspace(workspace, need, dev)
    if outs is None:
        outs = [torch.empty(x.shape, dtype=TORCH_DTYPE[p.out_code], device=x.device)
                for x, p in zip(xs, plans)]
    for i, (p, x, o) in enumerate(zip(plans, xs, outs)):
        _check_tensor(o, f"output {i}")
        _check_against_plan(p, x, o, f"volume {i}: ")
    _lib.run_batched_ptr(plans, [x.data_ptr() for x in xs], [o.data_ptr() for o in outs],
                         workspace.data_ptr(), workspace.numel() * workspace.element_size(), stream_handle(dev))
    return (outs, workspace, plans) if return_workspace else outs


def autotune(plan: Plan, x: torch.Tensor, out: torch.Tensor | None = None):
    """Pick the fastest work decomposition for this plan on the current GPU."""
    _check_tensor(x, "input")
    ws = torch.empty(plan.autotune_workspace_size(), dtype=torch.uint8, device=x.device)
    if out is None:
        out = torch.empty(x.shape, dtype=TORCH_DTYPE[plan.out_code], device=x.device)
    plan.autotune_ptr(x.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(), stream_handle(x.device))
    return plan.tuning()


def metrics(x: torch.Tensor, y: torch.Tensor | None = None, n_bins: int = 256, peak: float = 1.0,
            workspace: torch.Tensor | None = None, with_hist: bool = False) -> dict:
    """Contrast metrics of x, and of y against x (MSE, PSNR, STD, entropy).

    Runs the library's metric kernels on the current stream and waits for the
    result (a few dozen bytes copied back).
    """
    _check_tensor(x, "x")
    if y is not None:
        _check_tensor(y, "y")
        if y.numel() != x.numel():
            raise ValueError("x and y must have the same number of voxels")
    n = x.numel()
    need = _lib.metrics_workspace_size(n, n_bins)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    res = torch.empty(ctypes.sizeof(_lib.MetricsResult), dtype=torch.uint8, device=x.device)
    hist = torch.empty(2 * n_bins, dtype=torch.int64, device=x.device) if with_hist else None
    _lib.metrics_ptr(x.data_ptr(), _lib.dtype_code(x.dtype), None if y is None else y.data_ptr(),
                     _lib.dtype_code(y.dtype) if y is not None else 0, n, n_bins, peak, res.data_ptr(),
                     None if hist is None else hist.data_ptr(), workspace.data_ptr(), workspace.numel(),
                     stream_handle(x.device))
    r = _lib.MetricsResult.from_buffer_copy(bytes(res.cpu().numpy()))
    out = r.as_dict(y is not None)
    if with_hist:
        h = hist.cpu().numpy()
        out["hist"] = [h[:n_bins], h[n_bins:]] if y is not None else [h[:n_bins]]
    return out


def gaussian(x: torch.Tensor, sigma, truncate: float = 4.0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Separable Gaussian smoothing (one sigma per axis, 0 = leave the axis) into float32."""
    _check_tensor(x, "input")
    sigma = [float(s) for s in (sigma if hasattr(sigma, "__len__") else [sigma] * x.dim())]
    if len(sigma) != x.dim():
        raise ValueError("one sigma per axis")
    if out is None:
        out = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    _check_tensor(out, "output")
    need = _lib.gaussian_workspace_size(x.shape, sigma)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    _lib.gaussian_ptr(x.data_ptr(), _lib.dtype_code(x.dtype), x.shape, sigma, truncate, out.data_ptr(),
                      ws.data_ptr() if need else None, need, stream_handle(x.device))
    return out


def median(x: torch.Tensor, window, out: torch.Tensor | None = None) -> torch.Tensor:
    """Median filter over a window per axis (even sizes: upper middle value)."""
    _check_tensor(x, "input")
    if len(window) != x.dim():
        raise ValueError("one window size per axis")
    if out is None:
        out = torch.empty_like(x)
    _check_tensor(out, "output")
    _lib.median_ptr(x.data_ptr(), _lib.dtype_code(x.dtype), x.shape, window, out.data_ptr(),
                    stream_handle(x.device))
    return out
