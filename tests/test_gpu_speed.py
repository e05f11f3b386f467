"""GPU parity of the bit-shuffle codec (the FZMod-Speed pipeline) through the
C ABI: containers byte for byte and reconstructions bit for bit against the
oracle, on cases spanning several workgroups of 32 blocks, ragged edges in
every axis, 1D/2D/3D, outliers, patches and verbatim fields; the 512^3
benchmark field at three bounds; decoding through the batch call and the
allocation-free entry point; corrupt containers."""
import numpy as np
import pytest
import torch

import oracle
from inputs import fields

pytestmark = pytest.mark.gpu

CASES = [
    ("c1-sinusoid-64^3", "sinusoid", (64, 64, 64), 1e-3, 1),
    ("3d-ragged-smooth", "smooth", (37, 45, 29), 1e-2, 1),
    ("3d-ragged-tight", "smooth", (70, 33, 130), 1e-4, 1),
    ("3d-thin-x", "smooth", (40, 64, 1), 1e-3, 1),
    ("3d-thin-z", "smooth", (1, 64, 40), 1e-3, 1),
    ("3d-steps", "steps", (48, 40, 56), 1e-3, 1),
    ("3d-abs", "smooth", (32, 48, 64), 2e-4, 0),
    ("3d-wide-patches", "wide", (24, 24, 24), 1e-3, 1),
    ("3d-zeros", "zeros", (16, 16, 16), 1e-3, 0),
    ("3d-noise-verbatim", "noise", (20, 30, 40), 1e-7, 1),
    ("3d-x512-tight", "smooth", (16, 24, 512), 1e-5, 1),
    ("3d-column", "smooth", (700, 1, 1), 1e-3, 1),
    ("2d-ragged", "smooth", (1001, 777), 1e-3, 1),
    ("2d-tight", "smooth", (257, 1800), 1e-5, 1),
    ("2d-small", "smooth", (3, 5), 1e-2, 1),
    ("1d-positions", "positions", (1000003,), 1e-4, 1),
    ("1d-positions-loose", "positions", (70001,), 1e-2, 1),
    ("1d-one", "const", (1,), 1e-3, 1),
    ("1d-ragged", "smooth", (513,), 1e-3, 1),
]


def _field(kind, shape, seed):
    if kind == "sinusoid":
        return fields.sinusoid_field(shape, seed=seed)
    if kind == "positions":
        return fields.sorted_positions(shape[0], seed=seed)
    if kind == "zeros":
        return np.zeros(shape, np.float32)
    return fields.random_small(shape, seed, kind)


@pytest.fixture(scope="module")
def ctx(fz):
    return fz.Context(0)


def _check(fz, ctx, x, eb, mode, name):
    print(f"[gpu speed] {name} shape={x.shape} eb={eb} mode={mode}", flush=True)
    ref = oracle.speed_compress(x, eb, mode)
    d = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    c = ctx.compress(d, eb, mode, codec="shuffle")
    got = c.cpu().numpy().tobytes()
    h = oracle.header(ref)
    assert len(got) == len(ref), f"{name}: size {len(got)} vs oracle {len(ref)} (header {h})"
    if got != ref:
        a = np.frombuffer(got, np.uint8)
        b = np.frombuffer(ref, np.uint8)
        first = int(np.nonzero(a != b)[0][0])
        raise AssertionError(f"{name}: container differs first at byte {first} (header {h})")
    y = ctx.decompress(c).cpu().numpy()
    yo = oracle.decompress(ref)
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), f"{name}: reconstruction differs"
    err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
    assert err <= h["eb_abs"], f"{name}: max error {err} > {h['eb_abs']}"
    return c, y


@pytest.mark.parametrize("name,kind,shape,eb,mode", CASES, ids=[c[0] for c in CASES])
def test_speed_parity_small(fz, ctx, name, kind, shape, eb, mode):
    _check(fz, ctx, _field(kind, shape, seed=len(name)), eb, mode, name)


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_speed_parity_full_512cubed(fz, ctx, eb):
    x = fields.grf((512, 512, 512), alpha=3.0, seed=2)
    _check(fz, ctx, x, eb, 1, f"512^3 grf rel {eb}")


def test_speed_repeat_and_resize(fz, ctx):
    x = fields.grf((64, 96, 80), seed=12)
    d = torch.from_numpy(x).cuda()
    a = ctx.compress(d, 1e-4, 1, codec="shuffle").cpu().numpy().tobytes()
    for _ in range(3):
        assert ctx.compress(d, 1e-4, 1, codec="shuffle").cpu().numpy().tobytes() == a
    for shape in [(96, 96, 96), (8, 8, 8), (130, 17, 65), (4,)]:
        y = fields.random_small(shape, 5, "smooth") if len(shape) > 1 else np.arange(4, dtype=np.float32)
        _check(fz, ctx, y, 1e-3, 1, f"resize {shape}")


def test_speed_decode_noalloc_and_batch(fz, ctx):
    xs = [fields.grf((40, 56, 72), seed=31), fields.random_small((1001, 777), 9, "smooth"),
          fields.sorted_positions(70001, seed=6)]
    conts, refs = [], []
    for x in xs:
        c, y = _check(fz, ctx, x, 1e-3, 1, f"batch member {x.shape}")
        conts.append(c.clone())
        refs.append(y)
        out = torch.empty(x.size, dtype=torch.float32, device="cuda:0")
        fz.decompress_noalloc(c, out)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), y.reshape(-1).view(np.uint32))
    # packed back to back (16-byte aligned) and decoded by one batch call
    offs = [0]
    for c in conts:
        offs.append(offs[-1] + (c.numel() + 15) // 16 * 16)
    packed = torch.zeros(offs[-1], dtype=torch.uint8, device="cuda:0")
    for c, o in zip(conts, offs):
        packed[o:o + c.numel()] = c
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda:0") for x in xs]
    ctx.decompress_batch(packed, offs, outs)
    for o, y in zip(outs, refs):
        assert np.array_equal(o.cpu().numpy().view(np.uint32), y.view(np.uint32))


def test_speed_rejects_other_predictors(fz, ctx):
    x = torch.from_numpy(fields.grf((32, 32, 32), seed=4)).cuda()
    for pred in (1, 2, 4, 5, 6):
        with pytest.raises(fz.FZError) as e:
            ctx.compress(x, 1e-3, 1, pred=pred, codec="shuffle")
        assert e.value.code == -8


def test_speed_corrupt_containers(fz, ctx):
    x = fields.grf((24, 40, 56), seed=8)
    x[3, 5, 7] = 50.0  # an outlier at the absolute bound 1e-3
    d = torch.from_numpy(x).cuda()
    good = ctx.compress(d, 1e-3, 0, codec="shuffle").clone()
    h = oracle.header(good.cpu().numpy().tobytes())
    assert h["n_outliers"] > 0
    words_at = (128 + 20 * h["nblocks"] + 15) // 16 * 16
    opos_at = (words_at + 4 * h["stream_words"] + 15) // 16 * 16
    cases = {"mask bit": (128, 0x08), "outlier position": (opos_at, 0x01)}
    for what, (off, xor) in cases.items():
        bad = good.clone()
        bad[off] ^= xor
        print(f"[gpu speed] corrupt {what}", flush=True)
        with pytest.raises(fz.FZError) as e:
            ctx.decompress(bad)
        assert e.value.code == -5, what
        assert oracle.decompress_rc(bad.cpu().numpy().tobytes(), x.size) == oracle.ERR_CORRUPT
