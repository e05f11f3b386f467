"""Seeded synthetic float32 fields shaped like the paper's workloads.

This module only draws random numbers and synthesises fields; it holds none
of the compression method's arithmetic.  Both the CPU oracle side and the
GPU side of every test and benchmark take their inputs from here.

The paper evaluates on SDRBench datasets (Sec. 4.1, Table 2: CESM-ATM
3600x1800x26 climate slices, HACC 1D particle arrays, HURR 500x500x100,
Nyx 512^3).  Those files are not available here; these seeded fields stand
in for their shapes and smoothness:

* ``sinusoid_field``  - sum of seeded plane waves plus a little noise;
* ``grf``             - Gaussian random field with power spectrum P(k) ~ k^-alpha,
                        synthesised by filtering white noise in Fourier space,
                        scaled to [0, 1] (stands in for Nyx / HURR 3D fields and
                        CESM-ATM 2D slices);
* ``fronts_spikes``   - a k^-11/3 field plus tanh fronts and log-normal spikes;
* ``sorted_positions``- sorted uniform positions with Gaussian jitter (HACC-like 1D);
* ``batch_2d`` / ``batch_mixed`` - batches of uneven fields with per-field
                        offsets, scales and relative error bounds.

All arrays are C-ordered with the last axis fastest (x), i.e. shape (nz, ny, nx).
"""
from __future__ import annotations

import math

import numpy as np

try:  # multi-threaded FFT when available; results do not depend on the thread count
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sinusoid_field(shape=(64, 64, 64), seed=1, n_waves=4, noise_sigma=1e-3) -> np.ndarray:
    """Sum of ``n_waves`` plane waves with integer per-axis frequencies 1..8
    cycles per domain and random phases (amplitude 1), plus Gaussian noise."""
    r = rng(seed)
    nd = len(shape)
    axes = [np.arange(n, dtype=np.float64) / n for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    f = np.zeros(shape, np.float64)
    for _ in range(n_waves):
        freqs = r.integers(1, 9, size=nd)
        phase = r.uniform(0.0, 2.0 * math.pi)
        arg = phase
        for a in range(nd):
            arg = arg + 2.0 * math.pi * freqs[a] * grids[a]
        f += np.sin(arg)
    f += r.normal(0.0, noise_sigma, size=shape)
    return f.astype(np.float32)


def grf(shape, alpha=3.0, seed=2, scale01=True, dtype=np.float32) -> np.ndarray:
    """Gaussian random field with isotropic P(k) ~ k^-alpha.

    White N(0,1) noise -> real FFT -> amplitude k^(-alpha/2) with k measured
    in cycles per cell on each axis (so non-cubic grids stay isotropic) ->
    zero mean mode -> inverse FFT -> min-max scaling to [0, 1].
    """
    r = rng(seed)
    shape = tuple(int(s) for s in shape)
    noise = r.standard_normal(size=shape)
    spec = _rfftn(noise)
    del noise
    k2 = None
    for a, n in enumerate(shape):
        if a == len(shape) - 1:
            k = np.fft.rfftfreq(n)
        else:
            k = np.fft.fftfreq(n)
        view = [1] * len(shape)
        view[a] = k.size
        kk = (k ** 2).reshape(view)
        k2 = kk if k2 is None else k2 + kk
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-alpha / 4.0), 0.0)
    spec *= amp
    del amp, k2
    f = _irfftn(spec, s=shape)
    del spec
    if scale01:
        lo, hi = f.min(), f.max()
        f = (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)
    return f.astype(dtype)


def fronts_spikes(shape=(1024, 1024, 1024), seed=3, n_fronts=64, spike_frac=0.01,
                  spike_sigma=2.0, alpha=11.0 / 3.0, include_spikes=True) -> np.ndarray:
    """k^-11/3 field in [0,1] plus ``n_fronts`` tanh steps (width about 2 cells)
    and ``spike_frac`` of the cells replaced by log-normal values exp(sigma Z)."""
    r = rng(seed)
    base = grf(shape, alpha=alpha, seed=seed * 7919 + 1, dtype=np.float32)
    nz, ny, nx = shape
    f = base
    zc = np.arange(nz, dtype=np.float32).reshape(nz, 1, 1)
    yc = np.arange(ny, dtype=np.float32).reshape(1, ny, 1)
    xc = np.arange(nx, dtype=np.float32).reshape(1, 1, nx)
    for _ in range(n_fronts):
        v = r.standard_normal(3)
        v /= np.linalg.norm(v)
        p = r.uniform(0, 1, 3) * np.array([nx, ny, nz])
        amp = r.choice([-1.0, 1.0]) * r.uniform(0.5, 1.0)
        # signed distance to the plane through p with normal v, in cells
        d = (xc - p[0]) * np.float32(v[0]) + (yc - p[1]) * np.float32(v[1]) + (zc - p[2]) * np.float32(v[2])
        f += np.float32(amp) * np.tanh(d * np.float32(0.5))
    if include_spikes:
        n = f.size
        m = int(math.floor(spike_frac * n))
        idx = r.choice(n, size=m, replace=False)
        vals = np.exp(spike_sigma * r.standard_normal(m)).astype(np.float32)
        f.reshape(-1)[idx] = vals
    return f.astype(np.float32)


def sorted_positions(n, seed=5, box=256.0) -> np.ndarray:
    """Sorted uniform positions in [0, box) plus Gaussian jitter of box/n (HACC-like 1D)."""
    r = rng(seed)
    x = np.sort(r.uniform(0.0, box, size=n))
    x += r.normal(0.0, box / n, size=n)
    return x.astype(np.float32)


def log_uniform(r, lo, hi, size=None):
    return np.exp(r.uniform(math.log(lo), math.log(hi), size=size))


def batch_2d(n_fields=64, seed=4000, hmin=256, hmax=3600, wmin=256, wmax=1800):
    """Uneven 2D fields: shapes, offsets, scales and relative bounds per field.

    Returns a list of (field float32 (H, W), rel_eb)."""
    out = []
    for i in range(n_fields):
        r = rng(seed + i)
        h = int(r.integers(hmin, hmax + 1))
        w = int(r.integers(wmin, wmax + 1))
        off = log_uniform(r, 1e-3, 1e3)
        scale = log_uniform(r, 1e-3, 1e3)
        eb = log_uniform(r, 1e-5, 1e-2)
        g = grf((h, w), alpha=3.0, seed=seed + 100000 + i, dtype=np.float64)
        out.append(((off + scale * g).astype(np.float32), float(eb)))
    return out


def batch_mixed(n_fields=256, seed=5000, max_1d=1 << 26, max_3d_edge=384):
    """Mixed 1D / 2D / 3D batch; field i has type i mod 3.

    Returns a list of (field float32, rel_eb)."""
    out = []
    for i in range(n_fields):
        r = rng(seed + i)
        eb = float(log_uniform(r, 1e-5, 1e-2))
        t = i % 3
        if t == 0:
            n = int(log_uniform(r, 1 << 20, max_1d))
            f = sorted_positions(n, seed=seed + 200000 + i)
        elif t == 1:
            h = int(r.integers(256, 3601))
            w = int(r.integers(256, 1801))
            off = log_uniform(r, 1e-3, 1e3)
            scale = log_uniform(r, 1e-3, 1e3)
            g = grf((h, w), alpha=3.0, seed=seed + 100000 + i, dtype=np.float64)
            f = (off + scale * g).astype(np.float32)
        else:
            e = int(r.integers(64, max_3d_edge + 1))
            a = float(r.uniform(3.0, 5.0))
            f = grf((e, e, e), alpha=a, seed=seed + 100000 + i)
        out.append((f, eb))
    return out


def random_small(shape, seed, kind="smooth"):
    """Small test fields: 'smooth' (GRF), 'noise' (i.i.d. uniform), 'const',
    'steps' (piecewise constant), 'wide' (values spanning many magnitudes)."""
    r = rng(seed)
    if kind == "smooth":
        return grf(shape, alpha=3.0, seed=seed)
    if kind == "noise":
        return r.uniform(-1, 1, size=shape).astype(np.float32)
    if kind == "const":
        return np.full(shape, np.float32(r.uniform(-10, 10)), np.float32)
    if kind == "steps":
        return np.round(grf(shape, alpha=2.0, seed=seed) * 8).astype(np.float32)
    if kind == "wide":
        mag = np.exp(r.uniform(-30, 30, size=shape))
        return (mag * r.choice([-1.0, 1.0], size=shape)).astype(np.float32)
    raise ValueError(kind)
