"""Seeded synthetic fields generated on the device with torch (large
benchmark inputs that would take minutes to synthesise on the host).

Same recipes as ``inputs.fields`` (power-law Gaussian random fields, tanh
fronts with log-normal spikes, sorted jittered positions, uneven batches),
drawn from torch's counter-based device generator, so the values differ
from the numpy versions; tests that compare against the CPU oracle use
``inputs.fields``.  No compression arithmetic here.
"""
from __future__ import annotations

import math
import sys

import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _pow2(n: int) -> int:
    return 1 << max(0, (int(n) - 1).bit_length())


def grf(shape, alpha=3.0, seed=2, device="cuda") -> torch.Tensor:
    """P(k) ~ k^-alpha Gaussian random field scaled to [0, 1], float32.

    The periodic field is synthesised on the power-of-two grid that covers
    ``shape`` and cropped (the FFT library builds kernels for each new
    length at run time; power-of-two lengths are precompiled)."""
    shape = tuple(int(s) for s in shape)
    full = tuple(_pow2(s) for s in shape)
    f = _grf_periodic(full, alpha, seed, device)
    f = f[tuple(slice(0, s) for s in shape)]
    lo, hi = f.min(), f.max()
    return ((f - lo) / (hi - lo)).contiguous() if hi > lo else torch.zeros(shape, device=device)


def _grf_periodic(shape, alpha, seed, device) -> torch.Tensor:
    g = _gen(seed, device)
    noise = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    spec = torch.fft.rfftn(noise)
    del noise
    k2 = None
    for a, n in enumerate(shape):
        k = torch.fft.rfftfreq(n, device=device) if a == len(shape) - 1 else torch.fft.fftfreq(n, device=device)
        view = [1] * len(shape)
        view[a] = k.numel()
        kk = (k.to(torch.float32) ** 2).reshape(view)
        k2 = kk if k2 is None else k2 + kk
    amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (-alpha / 4.0), torch.zeros_like(k2))
    spec *= amp
    del amp, k2
    f = torch.fft.irfftn(spec, s=shape)
    del spec
    return f


def fronts_spikes(shape=(1024, 1024, 1024), seed=3, n_fronts=64, spike_frac=0.01, spike_sigma=2.0,
                  alpha=11.0 / 3.0, device="cuda", with_base_range=False):
    """k^-11/3 field in [0, 1] + ``n_fronts`` tanh steps (width ~2 cells) +
    ``spike_frac`` of the cells replaced by exp(sigma Z).  With
    ``with_base_range`` also returns max - min of the field before the
    spikes are set (float)."""
    f = grf(shape, alpha=alpha, seed=seed * 7919 + 1, device=device)
    g = _gen(seed, device)
    nz, ny, nx = shape
    zc = torch.arange(nz, device=device, dtype=torch.float32).reshape(nz, 1, 1)
    yc = torch.arange(ny, device=device, dtype=torch.float32).reshape(1, ny, 1)
    xc = torch.arange(nx, device=device, dtype=torch.float32).reshape(1, 1, nx)
    for _ in range(n_fronts):
        v = torch.randn(3, generator=g, device=device, dtype=torch.float64)
        v = v / v.norm()
        p = torch.rand(3, generator=g, device=device, dtype=torch.float64) * torch.tensor(
            [nx, ny, nz], device=device, dtype=torch.float64)
        sgn = 1.0 if float(torch.rand(1, generator=g, device=device)) < 0.5 else -1.0
        amp = sgn * (0.5 + 0.5 * float(torch.rand(1, generator=g, device=device)))
        vx, vy, vz = (float(t) for t in v)
        px, py, pz = (float(t) for t in p)
        d = (xc - px) * vx + (yc - py) * vy + (zc - pz) * vz
        f += amp * torch.tanh(d * 0.5)
    base_range = float(f.max()) - float(f.min()) if with_base_range else None
    m = int(math.floor(spike_frac * f.numel()))
    if m:
        idx = torch.randint(0, f.numel(), (m,), generator=g, device=device)
        vals = torch.exp(spike_sigma * torch.randn(m, generator=g, device=device))
        f.view(-1)[idx] = vals
    return (f.contiguous(), base_range) if with_base_range else f.contiguous()


def sorted_positions(n, seed=5, box=256.0, device="cuda") -> torch.Tensor:
    g = _gen(seed, device)
    x = torch.sort(torch.rand(int(n), generator=g, device=device, dtype=torch.float64) * box).values
    x += torch.randn(int(n), generator=g, device=device, dtype=torch.float64) * (box / n)
    return x.to(torch.float32).contiguous()


def _log_uniform(g, lo, hi, device):
    u = float(torch.rand(1, generator=g, device=device, dtype=torch.float64))
    return math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))


def batch_2d(n_fields=64, seed=4000, hmin=256, hmax=3600, wmin=256, wmax=1800, device="cuda"):
    """Uneven 2D k^-3 fields with per-field offset and scale (log-uniform
    1e-3..1e3) and relative bound (log-uniform 1e-5..1e-2)."""
    out = []
    for i in range(n_fields):
        g = _gen(seed + i, device)
        h = int(torch.randint(hmin, hmax + 1, (1,), generator=g, device=device))
        w = int(torch.randint(wmin, wmax + 1, (1,), generator=g, device=device))
        off = _log_uniform(g, 1e-3, 1e3, device)
        scale = _log_uniform(g, 1e-3, 1e3, device)
        eb = _log_uniform(g, 1e-5, 1e-2, device)
        f = (off + scale * grf((h, w), alpha=3.0, seed=seed + 100000 + i, device=device).double()).float()
        out.append((f.contiguous(), eb))
        if (i + 1) % 16 == 0:
            print(f"[fields_gpu] {i + 1}/{n_fields} fields", file=sys.stderr, flush=True)
    return out


def batch_mixed(n_fields=256, seed=5000, max_1d=1 << 26, max_3d_edge=384, device="cuda"):
    """Field i: 1D sorted positions (1M..max_1d values, log-uniform) when
    i mod 3 = 0, a 2D field as in ``batch_2d`` when 1, a 3D k^-3..k^-5
    field of edge 64..max_3d_edge when 2; relative bound log-uniform in
    1e-5..1e-2."""
    out = []
    for i in range(n_fields):
        g = _gen(seed + i, device)
        eb = _log_uniform(g, 1e-5, 1e-2, device)
        t = i % 3
        if t == 0:
            n = int(_log_uniform(g, 1 << 20, max_1d, device))
            f = sorted_positions(n, seed=seed + 200000 + i, device=device)
        elif t == 1:
            h = int(torch.randint(256, 3601, (1,), generator=g, device=device))
            w = int(torch.randint(256, 1801, (1,), generator=g, device=device))
            off = _log_uniform(g, 1e-3, 1e3, device)
            scale = _log_uniform(g, 1e-3, 1e3, device)
            f = (off + scale * grf((h, w), alpha=3.0, seed=seed + 100000 + i, device=device).double()).float()
        else:
            e = int(torch.randint(64, max_3d_edge + 1, (1,), generator=g, device=device))
            a = 3.0 + 2.0 * float(torch.rand(1, generator=g, device=device))
            f = grf((e, e, e), alpha=a, seed=seed + 100000 + i, device=device)
        out.append((f.contiguous(), eb))
        if (i + 1) % 16 == 0:
            print(f"[fields_gpu] {i + 1}/{n_fields} fields", file=sys.stderr, flush=True)
    return out
