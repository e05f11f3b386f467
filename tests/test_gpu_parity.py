"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Containers must be byte-identical (codes, outliers, patches, code lengths,
chunk table and Huffman stream all live in it), reconstructions bit-identical,
and every reconstructed value within the absolute bound."""
import numpy as np
import pytest
import torch

import oracle
from inputs import fields

pytestmark = pytest.mark.gpu


def _field(kind, shape, seed):
    if kind == "sinusoid":
        return fields.sinusoid_field(shape, seed=seed)
    if kind == "positions":
        return fields.sorted_positions(shape[0], seed=seed)
    if kind == "zeros":
        return np.zeros(shape, np.float32)
    if kind == "denormal":
        r = fields.rng(seed)
        return (r.uniform(-1, 1, shape) * 1e-38).astype(np.float32)
    return fields.random_small(shape, seed, kind)


CASES = [
    # name, kind, shape, eb, mode
    ("c1-sinusoid-64^3", "sinusoid", (64, 64, 64), 1e-3, 1),
    ("3d-ragged-smooth", "smooth", (37, 45, 29), 1e-2, 1),
    ("3d-ragged-smooth-1e-3", "smooth", (37, 45, 29), 1e-3, 1),
    ("3d-ragged-tight", "smooth", (70, 33, 130), 1e-4, 1),
    ("3d-thin-x", "smooth", (40, 64, 1), 1e-3, 1),
    ("3d-thin-z", "smooth", (1, 64, 40), 1e-3, 1),
    ("3d-steps", "steps", (48, 40, 56), 1e-3, 1),
    ("3d-abs", "smooth", (32, 48, 64), 2e-4, 0),
    ("3d-wide-patches", "wide", (24, 24, 24), 1e-3, 1),
    ("3d-zeros-one-symbol", "zeros", (16, 16, 16), 1e-3, 0),
    ("3d-denormal", "denormal", (16, 16, 16), 1e-44, 0),
    ("3d-noise-verbatim", "noise", (20, 30, 40), 1e-7, 1),
    # x extent a multiple of 512: the fast decoder's staged row stores (a
    # wave = one run of 64 blocks along x), with inactive waves in the last
    # workgroup, ragged y/z edge blocks beside it, and a tight bound
    ("3d-x512-partial-waves", "smooth", (20, 12, 512), 1e-3, 1),
    ("3d-x1024-ragged-yz", "smooth", (9, 17, 1024), 1e-2, 1),
    ("3d-x512-tight", "smooth", (16, 24, 512), 1e-5, 1),
    ("2d-ragged", "smooth", (1001, 777), 1e-3, 1),
    ("2d-tight", "smooth", (257, 1800), 1e-5, 1),
    ("2d-small", "smooth", (3, 5), 1e-2, 1),
    ("1d-positions", "positions", (1000003,), 1e-4, 1),
    ("1d-positions-loose", "positions", (70001,), 1e-2, 1),
    ("1d-one", "const", (1,), 1e-3, 1),
    ("1d-ragged", "smooth", (513,), 1e-3, 1),
]


@pytest.fixture(scope="module")
def ctx(fz):
    return fz.Context(0)


def _round_trip(fz, ctx, x, eb, mode, name):
    print(f"[gpu parity] {name} shape={x.shape} eb={eb} mode={mode}", flush=True)
    ref = oracle.compress(x, eb, mode)
    d = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    c = ctx.compress(d, eb, mode)
    got = c.cpu().numpy().tobytes()
    h = oracle.header(ref)
    assert len(got) == len(ref), f"{name}: size {len(got)} vs oracle {len(ref)}"
    if got != ref:
        a = np.frombuffer(got, np.uint8)
        b = np.frombuffer(ref, np.uint8)
        first = int(np.nonzero(a != b)[0][0])
        raise AssertionError(f"{name}: container differs first at byte {first} (header {h})")
    if not h["flags"] & 1:
        codes, pos, hist, e = oracle.stage_codes(x, eb, mode)
        assert np.array_equal(ctx.last_histogram(), hist), f"{name}: histogram differs"
    y = ctx.decompress(c).cpu().numpy()
    yo = oracle.decompress(ref)
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), f"{name}: reconstruction differs"
    err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
    assert err <= h["eb_abs"], f"{name}: max error {err} > {h['eb_abs']}"
    return ref


@pytest.mark.parametrize("name,kind,shape,eb,mode", CASES, ids=[c[0] for c in CASES])
def test_parity_small(fz, ctx, name, kind, shape, eb, mode):
    x = _field(kind, shape, seed=len(name))
    _round_trip(fz, ctx, x, eb, mode, name)


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_parity_full_512cubed(fz, ctx, eb):
    """The benchmarked workload: 512^3 k^-3 Gaussian random field, whole
    container and whole reconstruction against the oracle."""
    x = fields.grf((512, 512, 512), alpha=3.0, seed=2)
    _round_trip(fz, ctx, x, eb, 1, f"512^3 grf rel {eb}")


def test_repeat_calls_identical(fz, ctx):
    x = fields.grf((64, 96, 80), seed=12)
    d = torch.from_numpy(x).cuda()
    a = ctx.compress(d, 1e-4, 1).cpu().numpy().tobytes()
    for _ in range(5):
        assert ctx.compress(d, 1e-4, 1).cpu().numpy().tobytes() == a


def test_shrinking_then_growing_sizes(fz, ctx):
    for shape in [(96, 96, 96), (8, 8, 8), (130, 17, 65), (4,)]:
        x = fields.random_small(shape, 5, "smooth") if len(shape) > 1 else np.arange(4, dtype=np.float32)
        _round_trip(fz, ctx, x, 1e-3, 1, f"resize {shape}")


@pytest.mark.parametrize("mode", [0, 1])
def test_nonfinite_rejected(fz, ctx, mode):
    x = fields.grf((16, 16, 16), seed=3)
    x[3, 4, 5] = np.nan
    with pytest.raises(fz.FZError) as e:
        ctx.compress(torch.from_numpy(x).cuda(), 1e-3, mode)
    assert e.value.code == -3


def test_bad_eb_rejected(fz, ctx):
    x = torch.zeros(100, device="cuda")
    for eb in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(fz.FZError) as e:
            ctx.compress(x, eb, 0)
        assert e.value.code == -2


def test_corrupt_containers_rejected(fz, ctx):
    x = fields.grf((24, 40, 56), seed=8)
    d = torch.from_numpy(x).cuda()
    good = ctx.compress(d, 1e-3, 1).clone()
    h = oracle.header(good.cpu().numpy().tobytes())
    chunks = 128 + 512
    stream = (chunks + 2 * h["nblocks"] + 15) // 16 * 16
    cases = {
        "chunk bits": (chunks, 0x01),
        "code length nibble": (128 + 256, 0xF0),
        "stream word": (stream + 7, 0xFF),
    }
    for what, (off, xor) in cases.items():
        bad = good.clone()
        bad[off] ^= xor
        print(f"[gpu parity] corrupt {what}", flush=True)
        try:
            y = ctx.decompress(bad).cpu().numpy()
        except fz.FZError as e:
            assert e.code == -5, what
            continue
        # a flipped stream bit may still decode to a valid code sequence;
        # then the values differ but the call must not crash
        assert what == "stream word" and y.shape == x.shape


def test_stage_timing(fz, ctx):
    x = torch.from_numpy(fields.grf((64, 64, 64), seed=1)).cuda()
    ctx.set_timing(True)
    c = ctx.compress(x, 1e-3, 1)
    names = [n for n, _ in ctx.stage_times()]
    assert names == ["reset", "minmax", "quant", "scan_counts", "codebook", "encode", "finalize"]
    ctx.decompress(c)
    names = [n for n, _ in ctx.stage_times()]
    assert names == ["lut", "scan", "oindex", "decode", "patch"]
    # one stage timed: an event before and after it, nothing for calls without it
    ctx.set_timing_stage("decode")
    c2 = ctx.compress(x, 1e-3, 1)
    assert ctx.stage_times() == []
    ctx.decompress(c2)
    t = ctx.stage_times()
    assert [n for n, _ in t] == ["decode"] and t[0][1] > 0
    ctx.set_timing_stage("quant")
    ctx.compress(x, 1e-3, 1)
    assert [n for n, _ in ctx.stage_times()] == ["quant"]
    with pytest.raises(fz.FZError):
        ctx.set_timing_stage("x" * 32)
    # the whole call as one stage: one event before the first kernel, one after the last
    ctx.set_timing_stage("call")
    c3 = ctx.compress(x, 1e-3, 1)
    t = ctx.stage_times()
    assert [n for n, _ in t] == ["call"] and t[0][1] > 0
    y = ctx.decompress(c3)
    t = ctx.stage_times()
    assert [n for n, _ in t] == ["call"] and t[0][1] > 0
    assert torch.equal(y, ctx.decompress(c))
    ctx.set_timing_stage(None)
    ctx.compress(x, 1e-3, 1)
    assert len(ctx.stage_times()) == 7
    ctx.set_timing(False)
