"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and builds arrays; it holds none of the
method's arithmetic.  Tests, the benchmark and the serving demo take their
inputs from here, and the same arrays feed both the GPU library and the CPU
oracle.  All generators use numpy's PCG64 (``np.random.default_rng(seed)``).

Workloads (stand-ins for the paper's datasets, which are not available):

* ``gen_2d``  -- 2D uint8 image, linear background 20..60, Gaussian blobs,
  Poisson noise (a generic scientific 2D image).
* ``gen_3d``  -- 3D float fluorescence-like volume (stand-in for the light-sheet
  embryo data of Sec. IV.B): exponential background, anisotropic Gaussian spots
  with log-normal amplitudes, shot noise.
* ``gen_4d``  -- 4D float photoemission-like volume (k_x, k_y, E, t) (stand-in
  for the WSe2 data of Sec. IV.A): a paraboloid valence band with a
  Fermi-Dirac cut-off and a cone conduction band whose population decays in
  time, Lorentzian line width, Poisson counts with mean 0.5..50.
* ``gen_mix`` -- a seeded mix of 2D uint16 / 3D float / 4D float volumes with
  per-volume kernel sizes and clip limits.
* ``arrivals`` -- open-loop Poisson arrival times for the serving loop.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def gen_2d(shape=(512, 512), seed=1, dtype=np.uint8, scale=1.0):
    rng = np.random.default_rng(seed)
    H, W = shape
    nblob = max(1, int(round(40 * H * W / (512 * 512))))
    cy = rng.uniform(0, H, nblob)
    cx = rng.uniform(0, W, nblob)
    sig = rng.uniform(3, 25, nblob)
    amp = rng.uniform(30, 180, nblob)
    yy = np.arange(H, dtype=np.float32)[:, None]
    xx = np.arange(W, dtype=np.float32)[None, :]
    lam = np.broadcast_to(20.0 + 40.0 * xx / max(W - 1, 1), (H, W)).astype(np.float32).copy()
    for i in range(nblob):
        r = int(math.ceil(4 * sig[i]))
        y0, y1 = max(0, int(cy[i]) - r), min(H, int(cy[i]) + r + 1)
        x0, x1 = max(0, int(cx[i]) - r), min(W, int(cx[i]) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        d2 = (yy[y0:y1] - cy[i]) ** 2 + (xx[:, x0:x1] - cx[i]) ** 2
        lam[y0:y1, x0:x1] += amp[i] * np.exp(-d2 / (2 * sig[i] ** 2))
    img = rng.poisson(lam).astype(np.float64) * scale
    hi = np.iinfo(dtype).max
    return np.clip(img, 0, hi).astype(dtype)


def gen_3d(shape=(256, 256, 128), seed=2):
    rng = np.random.default_rng(seed)
    X, Y, Z = shape
    nspot = max(1, int(round(2000 * X * Y * Z / (256 * 256 * 128))))
    lam = rng.exponential(5.0, size=shape).astype(np.float32)
    c = rng.uniform(0, 1, (nspot, 3)) * np.array(shape)
    sxy = rng.uniform(1.5, 4.0, nspot)
    sz = rng.uniform(3.0, 8.0, nspot)
    amp = rng.lognormal(4.0, 1.0, nspot)
    for i in range(nspot):
        sig = (sxy[i], sxy[i], sz[i])
        lo = [max(0, int(c[i, a] - 4 * sig[a])) for a in range(3)]
        hi = [min(shape[a], int(c[i, a] + 4 * sig[a]) + 1) for a in range(3)]
        if any(l >= h for l, h in zip(lo, hi)):
            continue
        g = [np.exp(-((np.arange(lo[a], hi[a]) - c[i, a]) ** 2) / (2 * sig[a] ** 2)).astype(np.float32)
             for a in range(3)]
        lam[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += np.float32(amp[i]) * (
            g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :])
    return rng.poisson(lam).astype(np.float32)


def gen_4d(shape=(256, 256, 128, 32), seed=3, slab=16):
    """Photoemission-like (k_x, k_y, E, t); t is the fastest axis."""
    rng = np.random.default_rng(seed)
    NX, NY, NE, NT = shape
    kx = np.linspace(-1, 1, NX, dtype=np.float32)
    ky = np.linspace(-1, 1, NY, dtype=np.float32)
    e = np.arange(NE, dtype=np.float32)
    sE = NE / 128.0
    t = np.arange(NT, dtype=np.float32)
    mt = (np.exp(-t / 10.0) * (1 + np.cos(2 * np.pi * t / 16.0)) / 2).astype(np.float32)

    def lor(x):
        return 1.0 / (1.0 + (x / 2.0) ** 2)

    fermi = 1.0 / (1.0 + np.exp((e - 70.4 * sE) / 2.0))
    # the maximum of I over the volume, for the normalisation of the mean
    def slab_I(x0, x1):
        r2 = kx[x0:x1, None] ** 2 + ky[None, :] ** 2
        Ev = 57.6 * sE - 38.4 * sE * r2
        Ec = 79.36 * sE + 32.0 * sE * np.sqrt(r2)
        A = lor(e[None, None, :] - Ev[..., None]) * fermi[None, None, :]
        B = 0.3 * lor(e[None, None, :] - Ec[..., None])
        return A.astype(np.float32), B.astype(np.float32)

    imax = 0.0
    for x0 in range(0, NX, slab):
        A, B = slab_I(x0, min(NX, x0 + slab))
        imax = max(imax, float((A[..., None] + B[..., None] * mt).max()))
    out = np.empty(shape, np.float32)
    for x0 in range(0, NX, slab):
        x1 = min(NX, x0 + slab)
        A, B = slab_I(x0, x1)
        I = A[..., None] + B[..., None] * mt
        lam = 0.5 + 49.5 * I / imax
        out[x0:x1] = rng.poisson(lam)
    return out


def gen_fm4d_torch(shape=(512, 512, 109, 144), seed=6, device="cuda"):
    """Fluorescence-like 3D+t uint8 volume (x, y, z, t), t the fastest axis,
    generated on the device: a fluorescence-like 3D frame (gen_3d) as the
    rate, brightening linearly over time by 0.8..1.2, shot noise per frame,
    clipped to [0, 255].  Returns a torch tensor on `device`."""
    import torch
    X, Y, Z, T = shape
    base = torch.from_numpy(gen_3d((X, Y, Z), seed)).to(device)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty(shape, dtype=torch.uint8, device=device)
    for t in range(T):
        lam = base * (0.8 + 0.4 * t / max(1, T - 1))
        out[..., t] = torch.poisson(lam, generator=g).clamp_(0, 255).to(torch.uint8)
    return out


@dataclass
class MixItem:
    kind: str                 # "2d" | "3d" | "4d"
    x: np.ndarray
    kernel_size: tuple
    clip_limit: float
    n_bins: int = 256
    adaptive: bool = False
    seed: int = 0
    meta: dict = field(default_factory=dict)


def mix_spec(n=64, seed=4):
    """Shapes and parameters of the mixed batch, without drawing the data."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        kind = ["2d", "3d", "4d"][int(rng.integers(0, 3))]
        if kind == "2d":
            shape = tuple(int(v) for v in rng.integers(256, 2049, 2))
        elif kind == "3d":
            shape = tuple(int(v) for v in rng.integers(64, 257, 3))
        else:
            shape = tuple(int(v) for v in rng.integers(64, 129, 3)) + (int(rng.integers(8, 17)),)
        tiles = [int(rng.integers(2, 9)) for _ in shape]
        if kind == "4d":
            tiles[-1] = int(rng.integers(1, 3))
        ks = tuple(int(math.ceil(s / t)) for s, t in zip(shape, tiles))
        clip = float(rng.uniform(0.01, 0.05))
        specs.append(dict(kind=kind, shape=shape, kernel_size=ks, clip_limit=clip,
                          adaptive=(kind == "3d"), seed=seed * 1000 + i))
    return specs


def gen_item(spec, scale=1.0):
    kind, shape, sd = spec["kind"], spec["shape"], spec["seed"]
    if kind == "2d":
        x = gen_2d(shape, sd, dtype=np.uint16, scale=256.0)
    elif kind == "3d":
        x = gen_3d(shape, sd)
    else:
        x = gen_4d(shape, sd, slab=8)
    return MixItem(kind=kind, x=x, kernel_size=spec["kernel_size"],
                   clip_limit=spec["clip_limit"], adaptive=spec["adaptive"], seed=sd)


def gen_mix(n=64, seed=4):
    return [gen_item(s) for s in mix_spec(n, seed)]


def arrivals(rate_hz: float, n: int, seed=5):
    """Open-loop Poisson arrival times (seconds from 0)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))
