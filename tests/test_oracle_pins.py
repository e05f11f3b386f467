"""Pins for the CPU oracle: each test ties one oracle step to something other
than the oracle itself - brute force on tiny inputs, closed forms, a textbook
Huffman construction, invariants, or values worked out by hand."""
import heapq
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from inputs import fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- eb (step 1)
def test_eb_abs_closed_form():
    x = fields.random_small((9, 10, 11), 1, "wide")
    lo, hi = float(x.min()), float(x.max())
    assert oracle.eb_abs(x, 0, 1e-3) == 1e-3
    assert oracle.eb_abs(x, 1, 1e-3) == 1e-3 * (hi - lo)


def test_eb_abs_constant_field_uses_eb():
    x = np.full((4, 5), 3.25, np.float32)
    assert oracle.eb_abs(x, 1, 1e-2) == 1e-2


@pytest.mark.parametrize("bad", [0.0, -1e-3, float("inf"), float("nan")])
def test_eb_invalid(bad):
    x = np.zeros(10, np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x, bad, 0)
    assert e.value.code == oracle.ERR_EB


@pytest.mark.parametrize("v", [np.nan, np.inf, -np.inf])
def test_nonfinite_rejected(v):
    x = np.zeros(100, np.float32)
    x[37] = v
    for mode in (0, 1):
        with pytest.raises(oracle.OracleError) as e:
            oracle.compress(x, 1e-3, mode)
        assert e.value.code == oracle.ERR_NONFINITE


# ------------------------------------------------------- prequant (step 2)
def test_prequant_worked_examples():
    # eb_abs = 0.5 -> grid step 1: q is x rounded half to even
    x = np.array([2.5, 3.5, -2.5, 0.7, -0.5, 0.5, 1.49999988], np.float32)
    q, p = oracle.prequant(x, 0.5)
    assert q.tolist() == [2, 4, -2, 1, 0, 0, 1]
    # error exactly eb (2.5 -> 2.0, 0.5 -> 0.0) is inside the inclusive bound
    assert not p.any()


def test_prequant_out_of_range_is_patch_with_zero_q():
    x = np.array([1000.0, -1000.0, 1e-3], np.float32)
    q, p = oracle.prequant(x, 1e-9)
    assert q.tolist() == [0, 0, 0] or q[2] != 0
    assert p[0] and p[1] and q[0] == 0 and q[1] == 0
    # 1e-3 / 2e-9 = 5e5 < 2^24: regular grid value
    assert q[2] == 500000


def test_prequant_brute_force_interval():
    # every float32 in [100, 100 + 2^-8): the decoded value must be within eb_abs
    lo = np.float32(100.0)
    start = lo.view(np.uint32)
    x = (start + np.arange(1 << 15, dtype=np.uint32)).view(np.float32)
    for eb in (5e-6, 3e-6, 1e-4, 0.37):
        c = oracle.compress(x, eb, 0)
        y = oracle.decompress(c)
        assert np.all(np.abs(x.astype(np.float64) - y.astype(np.float64)) <= eb)


def test_prequant_is_nearest_grid_point():
    r = fields.rng(11)
    x = r.uniform(-50, 50, 5000).astype(np.float32)
    e = 0.013
    q, p = oracle.prequant(x, e)
    t = x.astype(np.float64) / (2 * e)
    # nearest integer up to the rounding of x * (1 / 2e)
    assert np.all(np.abs(t - q) <= 0.5 + 1e-9)


# -------------------------------------------------------- Lorenzo (step 3)
def _block_shape(nd):
    return {1: (512,), 2: (16, 32), 3: (8, 8, 8)}[nd]


def _composed_differences(q):
    """Backward difference along every axis, neighbour outside the block = 0,
    applied one axis at a time (independent of the oracle's 8-term formula)."""
    q = q.astype(np.int64)
    bs = _block_shape(q.ndim)
    out = q.copy()
    for a in range(q.ndim):
        prev = np.zeros_like(out)
        sl_dst = [slice(None)] * q.ndim
        sl_src = [slice(None)] * q.ndim
        sl_dst[a] = slice(1, None)
        sl_src[a] = slice(0, -1)
        prev[tuple(sl_dst)] = out[tuple(sl_src)]
        local = np.arange(q.shape[a]) % bs[a]
        view = [1] * q.ndim
        view[a] = q.shape[a]
        prev = prev * (local.reshape(view) > 0)
        out = out - prev
    return out


@pytest.mark.parametrize("shape", [(1100,), (512,), (1,), (40, 70), (16, 32), (17, 33), (9, 10, 11),
                                   (8, 8, 8), (16, 24, 8), (3, 5, 2)])
def test_lorenzo_matches_composed_differences(shape):
    r = fields.rng(sum(shape))
    q = r.integers(-2 ** 20, 2 ** 20, size=shape).astype(np.int32)
    d = oracle.lorenzo1(q)
    assert np.array_equal(d.astype(np.int64), _composed_differences(q))


@pytest.mark.parametrize("shape", [(1100,), (40, 70), (9, 10, 11), (17, 9, 25)])
def test_lorenzo_inverse_identity(shape):
    r = fields.rng(7 + len(shape))
    q = r.integers(-2 ** 23, 2 ** 23, size=shape).astype(np.int32)
    assert np.array_equal(oracle.lorenzo1_inverse(oracle.lorenzo1(q)), q)


def test_lorenzo_constant_block():
    q = np.full((8, 8, 8), 37, np.int32)
    d = oracle.lorenzo1(q)
    assert d[0, 0, 0] == 37
    d[0, 0, 0] = 0
    assert not d.any()


def test_lorenzo_separable_sum_vanishes_off_lower_faces():
    # q = f(x,y) + g(y,z) + h(x,z): each term is constant along one axis
    r = fields.rng(3)
    f = r.integers(-100, 100, (8, 8))
    g = r.integers(-100, 100, (8, 8))
    h = r.integers(-100, 100, (8, 8))
    z, y, x = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    q = (f[y, x] + g[z, y] + h[z, x]).astype(np.int32)
    d = oracle.lorenzo1(q)
    assert not d[1:, 1:, 1:].any()


# ----------------------------------------- post-quant + histogram (steps 4-5)
def test_postquant_radius_edges():
    # eb_abs = 0.5 -> q = x; 1D residual d[i] = q[i] - q[i-1] inside a block
    deltas = [5, 511, -511, 512, -512, 0, 1000, -1]
    x = np.cumsum(deltas).astype(np.float32)
    codes, pos, hist, e = oracle.stage_codes(x, 0.5, 0)
    assert codes.tolist() == [517, 1023, 1, 0, 0, 512, 0, 511]
    c = oracle.compress(x, 0.5, 0)
    h = oracle.header(c)
    assert h["flags"] & 1 or h["n_outliers"] == 3
    assert np.array_equal(oracle.decompress(c), x)


def test_histogram_counts():
    x = fields.grf((20, 30, 40), seed=5)
    codes, pos, hist, e = oracle.stage_codes(x, 1e-4, 1)
    assert hist.sum() == x.size
    assert np.array_equal(hist, np.bincount(codes, minlength=1024))
    c = oracle.compress(x, 1e-4, 1)
    h = oracle.header(c)
    if not h["flags"] & 1:
        assert h["n_outliers"] == hist[0]


def test_block_major_positions():
    shape = (11, 13, 19)  # ragged in every axis
    x = fields.grf(shape, seed=9)
    codes, pos, hist, e = oracle.stage_codes(x, 1e-3, 1)
    nz, ny, nx = shape
    nbx, nby = -(-nx // 8), -(-ny // 8)
    expect = []
    for bz in range(-(-nz // 8)):
        for by in range(nby):
            for bx in range(nbx):
                b = bx + nbx * (by + nby * bz)
                for lz in range(8):
                    for ly in range(8):
                        for lx in range(8):
                            if bx * 8 + lx < nx and by * 8 + ly < ny and bz * 8 + lz < nz:
                                expect.append(b * 512 + lx + 8 * ly + 64 * lz)
    assert pos.tolist() == expect


# ------------------------------------------------------- codebook (step 6)
def _heap_huffman_cost(w):
    w = [int(v) for v in w if v > 0]
    if len(w) == 1:
        return w[0]
    heapq.heapify(w)
    cost = 0
    while len(w) > 1:
        a = heapq.heappop(w)
        b = heapq.heappop(w)
        cost += a + b
        heapq.heappush(w, a + b)
    return cost


def _heap_huffman_depth(w):
    items = [(int(v), i, 0) for i, v in enumerate(w) if v > 0]
    heapq.heapify(items)
    k = len(w)
    while len(items) > 1:
        a = heapq.heappop(items)
        b = heapq.heappop(items)
        heapq.heappush(items, (a[0] + b[0], k, max(a[2], b[2]) + 1))
        k += 1
    return items[0][2]


def _kraft(lengths):
    return sum(2.0 ** -int(l) for l in lengths if l > 0)


def _cost(hist, lengths):
    return int(sum(int(h) * int(l) for h, l in zip(hist, lengths)))


def test_codebook_golden():
    with open(os.path.join(GOLDEN, "huffman_examples.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        hist = np.zeros(1024, np.uint32)
        for s, v in c["hist"].items():
            hist[int(s)] = v
        ln = oracle.codebook(hist)
        got = {str(s): int(ln[s]) for s in np.nonzero(ln)[0]}
        assert got == c["lengths"]
        cw = oracle.canonical(ln)
        codes = {str(s): format(int(cw[s]), "0%db" % ln[s]) for s in np.nonzero(ln)[0]}
        assert codes == c["codes"]
        assert _cost(hist, ln) == c["cost"]
        if "encode" in c:
            words, nb = oracle.encode_symbols(c["encode"]["symbols"], ln)
            assert nb == len(c["encode"]["bits"])
            assert int(words[0]) == c["encode"]["first_word"]


def test_codebook_matches_heap_huffman_cost():
    r = fields.rng(17)
    for trial in range(200):
        n = int(r.integers(2, 300))
        hist = np.zeros(1024, np.uint32)
        syms = r.choice(1024, n, replace=False)
        kind = trial % 3
        if kind == 0:
            hist[syms] = r.integers(1, 1000, n)
        elif kind == 1:
            hist[syms] = np.maximum(1, (1e6 * np.exp(-np.abs(r.normal(0, 3, n)))).astype(np.uint32))
        else:
            hist[syms] = r.integers(1, 4, n)  # many ties
        ln = oracle.codebook(hist)
        assert abs(_kraft(ln) - 1.0) < 1e-12
        assert ln.max() <= 12
        assert set(np.nonzero(ln)[0]) == set(np.nonzero(hist)[0])
        if _heap_huffman_depth(hist) <= 12:
            assert _cost(hist, ln) == _heap_huffman_cost(hist)


def test_codebook_brute_force_length_limited():
    r = fields.rng(23)
    for trial in range(60):
        n = int(r.integers(2, 7))
        lmax = int(r.integers(max(1, math.ceil(math.log2(n))), 5))
        w = r.integers(1, 60, n)
        if trial % 2:
            w = np.array([int(1.9 ** i) + 1 for i in range(n)])  # skewed: limiter binds
        best = None
        for ls in itertools.product(range(1, lmax + 1), repeat=n):
            if sum(2.0 ** -l for l in ls) <= 1.0:
                c = sum(int(a) * b for a, b in zip(w, ls))
                best = c if best is None else min(best, c)
        hist = np.zeros(n, np.uint32)
        hist[:] = w
        ln = oracle.codebook(hist, lmax=lmax)
        assert ln.max() <= lmax
        assert abs(_kraft(ln) - 1.0) < 1e-12
        assert _cost(hist, ln) == best


def test_codebook_limiter_binds_at_12():
    # Fibonacci counts force an unrestricted Huffman depth far above 12
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    hist = np.zeros(1024, np.uint32)
    hist[100:130] = fib
    assert _heap_huffman_depth(hist) > 12
    ln = oracle.codebook(hist)
    assert ln.max() == 12
    assert abs(_kraft(ln) - 1.0) < 1e-12
    assert _cost(hist, ln) >= _heap_huffman_cost(hist)


def test_canonical_prefix_free_and_ordered():
    r = fields.rng(5)
    hist = np.zeros(1024, np.uint32)
    hist[r.choice(1024, 500, replace=False)] = r.integers(1, 10000, 500)
    ln = oracle.codebook(hist)
    cw = oracle.canonical(ln)
    used = [s for s in range(1024) if ln[s]]
    strs = {s: format(int(cw[s]), "0%db" % ln[s]) for s in used}
    allc = sorted(strs.values())
    for a, b in zip(allc, allc[1:]):
        assert not b.startswith(a)
    # canonical order: (length, symbol) order equals numeric order of left-aligned codes
    order = sorted(used, key=lambda s: (ln[s], s))
    vals = [int(cw[s]) << (12 - int(ln[s])) for s in order]
    assert vals == sorted(vals) and len(set(vals)) == len(vals)


# ------------------------------------------------ container and round trip
@pytest.mark.parametrize("shape,kind", [((64, 64, 64), "smooth"), ((13, 17, 29), "smooth"), ((3, 600), "steps"),
                                        ((2000,), "smooth"), ((8, 8, 8), "const"), ((1,), "const"),
                                        ((5, 7, 9), "wide"), ((33, 65), "noise")])
@pytest.mark.parametrize("eb", [1e-2, 1e-4])
def test_round_trip_bound(shape, kind, eb):
    if len(shape) == 1 and kind == "smooth":
        x = fields.sorted_positions(shape[0], seed=3)
    else:
        x = fields.random_small(shape, 3, kind)
    c = oracle.compress(x, eb, 1)
    h = oracle.header(c)
    assert h["magic"] == 0x314D5A46 and h["total"] == len(c)
    y = oracle.decompress(c)
    err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
    assert err <= h["eb_abs"]
    assert len(c) <= oracle.compress_bound(x.shape)


def test_sinusoid_field_round_trip():
    x = fields.sinusoid_field()
    for mode, eb in ((1, 1e-3), (0, 1e-3 * float(x.max() - x.min()))):
        c = oracle.compress(x, eb, mode)
        y = oracle.decompress(c)
        assert np.abs(x.astype(np.float64) - y).max() <= oracle.header(c)["eb_abs"]


def test_rel_equals_abs_except_header_mode():
    x = fields.grf((16, 24, 40), seed=4)
    rel = bytearray(oracle.compress(x, 1e-3, 1))
    e = oracle.header(rel)["eb_abs"]
    ab = bytearray(oracle.compress(x, e, 0))
    assert len(rel) == len(ab)
    # header differs only in eb_mode (40..44) and the user eb (48..56)
    diff = [i for i in range(len(rel)) if rel[i] != ab[i]]
    assert all(40 <= i < 44 or 48 <= i < 56 for i in diff)


def test_verbatim_when_incompressible():
    x = fields.random_small((64, 64), 8, "noise")
    c = oracle.compress(x, 1e-7, 1)
    h = oracle.header(c)
    assert h["flags"] & 1 and len(c) == 128 + 4 * x.size
    assert np.array_equal(oracle.decompress(c), x)


def test_denormals_and_signed_zero():
    x = np.array([0.0, -0.0, 1e-45, -1e-45, 1e-40, 3e-39, -2e-38, 1.0], np.float32)
    for eb in (1e-44, 1e-3):
        c = oracle.compress(x, eb, 0)
        y = oracle.decompress(c)
        assert np.all(np.abs(x.astype(np.float64) - y) <= oracle.header(c)["eb_abs"])


def test_corruption_detected():
    x = fields.grf((16, 16, 16), seed=6)
    good = oracle.compress(x, 1e-3, 1)
    assert oracle.decompress_rc(good) == 0
    bad = bytearray(good)
    bad[0] ^= 1
    assert oracle.decompress_rc(bad) == oracle.ERR_CORRUPT
    assert oracle.decompress_rc(good[: len(good) - 16]) == oracle.ERR_CORRUPT
    h = oracle.header(good)
    chunk_off = 128 + 512
    bad = bytearray(good)
    bad[chunk_off] ^= 0x01  # first block's bit count off by one
    assert oracle.decompress_rc(bad) == oracle.ERR_CORRUPT
    bad = bytearray(good)
    bad[128] = 0xFF  # code length 15 > 12
    assert oracle.decompress_rc(bad) == oracle.ERR_CORRUPT
    assert h["n_outliers"] >= 0
