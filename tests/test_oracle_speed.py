"""Pins for the oracle's bit-shuffle codec (the FZMod-Speed lossless stage:
bit-shuffle plus zero-word elimination of the quantisation symbols, in place
of Huffman coding).  Residuals are steered exactly with 1D integer fields at
absolute bound 0.5 (grid step 1, so q = x and the first-order residual is
the difference of neighbours, the block's first value standing alone); the
symbols, the shuffled words and the container are then checked against hand
values, closed forms and brute force."""
import numpy as np
import pytest

import oracle
from inputs import fields


def _field_from_residuals(d):
    """1D float32 field whose first-order residuals (blocks of 512, zero
    before each block) are d, at absolute bound 0.5."""
    d = np.asarray(d, np.int64)
    x = np.empty(d.size, np.float64)
    for b in range(0, d.size, 512):
        x[b:b + 512] = np.cumsum(d[b:b + 512])
    assert np.abs(x).max() < 2 ** 23
    return x.astype(np.float32)


def _expected_symbols(d):
    s = []
    for v in d:
        if abs(v) >= 512:
            s.append(1023)
        elif v >= 0:
            s.append(2 * v)
        else:
            s.append(-2 * v - 1)
    return np.array(s, np.uint16)


def test_symbols_worked_example():
    # residuals 0, -1, 1, -2, 2, 511, -511, 512, -512, 3 -> folded symbols,
    # 1023 marking the two outliers; the rest of the block holds zeros
    d = [0, -1, 1, -2, 2, 511, -511, 512, -512, 3]
    x = _field_from_residuals(d)
    sym, _ = oracle.speed_stage(x, 0.5, 0)
    assert sym.shape == (1, 512)
    assert sym[0, :10].tolist() == [0, 1, 2, 3, 4, 1022, 1021, 1023, 1023, 6]
    assert not sym[0, 10:].any()


def test_shuffle_worked_example():
    # symbols 1, 2, 3 in slots 0..2 (residuals -1, 1, -2): plane 0 has bits
    # 0 and 2 set (5), plane 1 bits 1 and 2 (6); every other word is zero
    x = _field_from_residuals([-1, 1, -2])
    sym, words = oracle.speed_stage(x, 0.5, 0)
    assert sym[0, :3].tolist() == [1, 2, 3]
    assert words[0, 0, 0] == 5 and words[0, 0, 1] == 6
    w = words.copy()
    w[0, 0, 0] = w[0, 0, 1] = 0
    assert not w.any()


def test_shuffle_is_a_bit_transpose():
    r = np.random.default_rng(7)
    d = r.integers(-700, 700, size=3 * 512 + 77)
    small = r.random(d.size) < 0.6
    d[small] = r.integers(-3, 4, size=int(small.sum()))
    x = _field_from_residuals(d)
    sym, words = oracle.speed_stage(x, 0.5, 0)
    exp = np.zeros(sym.size, np.uint16)
    exp[: d.size] = _expected_symbols(d)
    assert np.array_equal(sym.reshape(-1), exp)
    # each word: bit j = bit p of symbol 32 g + j, by unpacking to bits
    bits = ((exp.reshape(-1, 16, 32)[..., None] >> np.arange(10)) & 1).astype(np.uint64)  # (b, g, j, p)
    ref = (bits << np.arange(32, dtype=np.uint64)[None, None, :, None]).sum(axis=2).astype(np.uint32)
    assert np.array_equal(words, ref)


def _sections(buf):
    h = oracle.header(buf)
    nb, words = h["nblocks"], h["stream_words"]
    a16 = lambda v: (v + 15) & ~15
    masks_at = 128
    words_at = a16(masks_at + 20 * nb)
    b = np.frombuffer(buf, np.uint8)
    masks = b[masks_at:masks_at + 20 * nb].view(np.uint32).reshape(nb, 5)
    kept = b[words_at:words_at + 4 * words].view(np.uint32)
    return h, masks, kept


@pytest.mark.parametrize("shape,eb", [((37, 45, 29), 1e-2), ((1001, 777), 1e-3), ((70001,), 1e-3),
                                      ((20, 12, 512), 1e-3)])
def test_container_masks_and_kept_words(shape, eb):
    x = fields.grf(shape, 3.0, seed=11) if len(shape) > 1 else fields.sorted_positions(shape[0], seed=4)
    buf = oracle.speed_compress(x, eb, 1)
    h, masks, kept = _sections(buf)
    assert h["flags"] == 2 and h["pred"] == 0 and h["stream_bits"] == 0
    _, words = oracle.speed_stage(x, eb, 1)
    flat = words.reshape(h["nblocks"], 160)
    nz = flat != 0
    # the mask bit of word k of a block is set exactly for the non-zero words
    mbits = ((masks[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(h["nblocks"], 160).astype(bool)
    assert np.array_equal(mbits, nz)
    # the kept words are the non-zero words in (block, mask bit) order
    assert np.array_equal(kept, flat[nz])
    assert h["stream_words"] == int(nz.sum())


@pytest.mark.parametrize("c", [0.0, 1.0, -3.0, 37.0, -300.0, 600.0])
def test_constant_field_closed_form(c):
    # a constant field on the grid: per 8^3 block only the corner keeps a
    # residual (q = c); its symbol has popcount(symbol) non-zero planes, so
    # the kept words are nblocks * popcount, and |c| >= 512 is an outlier
    # per block (symbol 1023: 10 words)
    shape = (19, 17, 23)
    x = np.full(shape, c, np.float32)
    buf = oracle.speed_compress(x, 0.5, 0)
    h = oracle.header(buf)
    nb = oracle.nblocks_of(shape)
    s = 1023 if abs(c) >= 512 else (int(2 * c) if c >= 0 else int(-2 * c - 1))
    if h["flags"] & 1:
        pytest.skip("verbatim")
    assert h["stream_words"] == nb * bin(s).count("1")
    assert h["n_outliers"] == (nb if abs(c) >= 512 else 0)
    assert np.array_equal(oracle.decompress(buf), x)


SHAPES = [((37, 45, 29), 1e-2), ((37, 45, 29), 1e-3), ((70, 33, 130), 1e-4), ((40, 64, 1), 1e-3),
          ((1, 64, 40), 1e-3), ((1001, 777), 1e-3), ((257, 1800), 1e-5), ((3, 5), 1e-2), ((1000003,), 1e-4),
          ((1,), 1e-3), ((513,), 1e-3), ((24, 24, 24), 1e-3)]


@pytest.mark.parametrize("shape,eb", SHAPES)
def test_round_trip_matches_huffman_path(shape, eb):
    if len(shape) == 1 and shape[0] > 1000:
        x = fields.sorted_positions(shape[0], seed=5)
    elif shape == (24, 24, 24):
        x = fields.random_small(shape, 3, "wide")
    else:
        x = fields.grf(shape, 3.0, seed=len(shape) + shape[0]) if shape[0] > 1 or len(shape) > 1 else \
            np.array([0.375], np.float32)
    s = oracle.speed_compress(x, eb, 1)
    hs = oracle.header(s)
    y = oracle.decompress(s)
    eb_abs = oracle.eb_abs(x, 1, eb)
    assert np.abs(y.astype(np.float64) - x).max() <= eb_abs
    hh = oracle.compress(x, eb, 1)
    if not (hs["flags"] & 1) and not (oracle.header(hh)["flags"] & 1):
        # the same quantisation: identical reconstructions and side lists
        assert np.array_equal(y.view(np.uint32), oracle.decompress(hh).view(np.uint32))
        assert hs["n_outliers"] == oracle.header(hh)["n_outliers"]
        assert hs["n_patches"] == oracle.header(hh)["n_patches"]


def test_verbatim_on_noise():
    x = fields.random_small((20, 30, 40), 4, "noise")
    buf = oracle.speed_compress(x, 1e-7, 1)
    h = oracle.header(buf)
    assert h["flags"] == 3 and len(buf) == 128 + 4 * x.size
    assert np.array_equal(oracle.decompress(buf), x)


def test_corruption_detected():
    x = fields.grf((40, 40, 40), 3.0, seed=9)
    buf = bytearray(oracle.speed_compress(x, 1e-3, 1))
    h, masks, _ = _sections(bytes(buf))
    assert oracle.decompress_rc(bytes(buf), x.size) == 0
    # a mask bit flipped: the kept words no longer add up
    bad = bytearray(buf)
    bad[128] ^= 1 << 3
    assert oracle.decompress_rc(bytes(bad), x.size) == oracle.ERR_CORRUPT
    # truncated container
    assert oracle.decompress_rc(bytes(buf[:-16]), x.size) == oracle.ERR_CORRUPT
    # an unknown flag bit
    bad = bytearray(buf)
    bad[6] |= 4
    assert oracle.decompress_rc(bytes(bad), x.size) == oracle.ERR_CORRUPT


def test_outlier_list_must_match_symbols():
    d = [0] * 100 + [700] + [0] * 50 + [-900]
    x = _field_from_residuals(d)
    buf = bytearray(oracle.speed_compress(x, 0.5, 0))
    h = oracle.header(bytes(buf))
    assert h["n_outliers"] == 2
    assert np.array_equal(oracle.decompress(bytes(buf)), x)
    # move the first listed outlier position by one
    words_at = (128 + 20 * h["nblocks"] + 15) & ~15
    opos_at = (words_at + 4 * h["stream_words"] + 15) & ~15
    p = int.from_bytes(buf[opos_at:opos_at + 4], "little")
    assert p == 100
    buf[opos_at:opos_at + 4] = (p + 1).to_bytes(4, "little")
    assert oracle.decompress_rc(bytes(buf), x.size) == oracle.ERR_CORRUPT
