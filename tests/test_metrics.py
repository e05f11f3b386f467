"""Eq. (1) overall speedup and the other Sec. 4.2 metrics."""
import json
import math
import os

import numpy as np

from paper_2509_20563_amd import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_eq1_worked_example():
    with open(os.path.join(GOLDEN, "eq1_speedup.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        s = metrics.overall_speedup(c["bw_gbps"], c["cr"], c["throughput_gbps"])
        if c["relation"] == "eq":
            assert math.isclose(s, c["speedup"], rel_tol=1e-12)
        elif c["relation"] == "gt":
            assert s > c["speedup"]
        else:
            assert s < c["speedup"]


def test_eq1_limits():
    # infinitely fast compressor: speedup -> CR; no compression (CR 1): speedup < 1
    assert math.isclose(metrics.overall_speedup(35.7, 10.0, 1e12), 10.0, rel_tol=1e-9)
    assert metrics.overall_speedup(35.7, 1.0, 1000.0) < 1.0


def test_ratio_rate_psnr():
    assert metrics.compression_ratio(1000, 400) == 10.0
    assert metrics.bit_rate(1000, 400) == 3.2
    a = np.linspace(0, 1, 1001)
    b = a + 1e-3
    assert math.isclose(metrics.psnr(a, b), 60.0, rel_tol=1e-9)
    assert metrics.psnr(a, a) == math.inf
