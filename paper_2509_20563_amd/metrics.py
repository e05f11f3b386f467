"""Evaluation metrics of Sec. 4.2 (FZModules): compression ratio, throughput,
overall speedup (Eq. 1), bit-rate and PSNR."""
from __future__ import annotations

import math

import numpy as np


def compression_ratio(n_values: int, compressed_bytes: int) -> float:
    """Input size divided by compressed size (Sec. 4.2), float32 input."""
    return 4.0 * n_values / compressed_bytes


def throughput_gbps(n_values: int, seconds: float) -> float:
    """Input bytes processed per second, in GB/s (10^9 B/s)."""
    return 4.0 * n_values / seconds / 1e9


def overall_speedup(bw_gbps: float, cr: float, throughput_gbps: float) -> float:
    """Eq. (1): 1 / (((BW * CR)^-1 + T^-1) * BW).

    BW is the bandwidth of the link the data crosses, CR the compression
    ratio and T the compressor throughput, both rates in the same unit."""
    return 1.0 / ((1.0 / (bw_gbps * cr) + 1.0 / throughput_gbps) * bw_gbps)


def bit_rate(n_values: int, compressed_bytes: int) -> float:
    """Average compressed bits per input value (Sec. 4.2 rate-distortion)."""
    return 8.0 * compressed_bytes / n_values


def psnr(original: np.ndarray, reconstructed: np.ndarray) -> float:
    """20 log10(value range / RMSE), RMSE in double precision."""
    a = np.asarray(original, dtype=np.float64).ravel()
    b = np.asarray(reconstructed, dtype=np.float64).ravel()
    rng = float(a.max() - a.min())
    mse = float(np.mean((a - b) ** 2))
    if mse == 0.0:
        return math.inf
    if rng == 0.0:
        return -math.inf
    return 20.0 * math.log10(rng / math.sqrt(mse))
