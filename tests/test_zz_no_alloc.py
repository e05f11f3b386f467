"""fz_decompress_noalloc (the allocation-free decompression, static per-GPU
scratch) against fz_decompress on the same containers: bit-identical
reconstructions, two calls in a row with the second smaller, verbatim
containers, and the host-side rejections (other predictors, more blocks than
the scratch holds)."""
import numpy as np
import pytest
import torch

from inputs import fields, fields_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(fz):
    return fz.Context(0)


def _roundtrip(fz, ctx, x, eb, mode=1, pred=0):
    d = x if isinstance(x, torch.Tensor) else torch.from_numpy(x).to("cuda:0")
    c = ctx.compress(d, eb, mode, pred=pred)
    ref = ctx.decompress(c)
    return d, c, ref


def _noalloc(fz, c, n, header=True):
    out = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda:0")
    hdr = c[:fz.HDR_BYTES].cpu().numpy().tobytes() if header else None
    fz.decompress_noalloc(c, out, hdr)
    torch.cuda.synchronize()
    return out


def _same(a, b):
    return np.array_equal(a.cpu().numpy().reshape(-1).view(np.uint32), b.cpu().numpy().reshape(-1).view(np.uint32))


def test_noalloc_matches_decompress_twice(fz, ctx):
    print("[noalloc] scratch bytes", fz.noalloc_scratch_bytes(), flush=True)
    assert fz.noalloc_scratch_bytes() < 8 << 20
    # a large field with outliers and patches at a tight bound, then a
    # smaller, ragged one: the second call reuses the scratch the first left
    big = fields.grf((128, 160, 192), 3.0, seed=21)
    small = fields.random_small((37, 45, 29), 5, "smooth")
    for x, eb, hdr in ((big, 1e-5, True), (small, 1e-3, False)):
        print(f"[noalloc] shape {x.shape} eb {eb}", flush=True)
        d, c, ref = _roundtrip(fz, ctx, x, eb)
        got = _noalloc(fz, c, x.size, header=hdr)
        assert _same(got, ref)
        assert float((got.view(x.shape).double() - d.double()).abs().max()) <= fz.header_fields(
            c[:fz.HDR_BYTES].cpu().numpy().tobytes())["eb_abs"]


def test_noalloc_full_scratch_and_tail(fz, ctx):
    # exactly the maximum block count (a 1D field of 2^26 values), then a
    # ragged 2D field and a one-value field
    n = 131072 * 512
    x = fields_gpu.sorted_positions(n, seed=3, device="cuda:0")
    assert x.numel() == n
    for y, eb in ((x, 1e-4), (fields.random_small((1001, 777), 9, "smooth"), 1e-3),
                  (np.array([0.25], np.float32), 1e-3)):
        print(f"[noalloc] shape {tuple(y.shape)} eb {eb}", flush=True)
        _, c, ref = _roundtrip(fz, ctx, y, eb)
        nb = fz.header_fields(c[:fz.HDR_BYTES].cpu().numpy().tobytes())["nblocks"]
        assert nb <= 131072
        assert _same(_noalloc(fz, c, int(np.prod(y.shape))), ref)


def test_noalloc_verbatim(fz, ctx):
    x = fields.random_small((20, 30, 40), 4, "noise")
    _, c, ref = _roundtrip(fz, ctx, x, 1e-7)
    assert fz.header_fields(c[:fz.HDR_BYTES].cpu().numpy().tobytes())["flags"] & 1
    assert _same(_noalloc(fz, c, x.size), ref)


def test_noalloc_rejects(fz, ctx):
    x = fields.random_small((32, 32, 32), 6, "smooth")
    d = torch.from_numpy(x).to("cuda:0")
    for pred in (1, 2, 4, 5, 6):
        c = ctx.compress(d, 1e-3, 1, pred=pred)
        with pytest.raises(fz.FZError) as e:
            _noalloc(fz, c, x.size)
        assert e.value.code == -8
    # one block more than the scratch holds: a (N, 1, 1) 3D field has one
    # 8x8x8 block per 8 values along z
    y = fields.random_small((8 * 131073, 1, 1), 7, "smooth")
    _, c, _ = _roundtrip(fz, ctx, y, 1e-3)
    with pytest.raises(fz.FZError) as e:
        _noalloc(fz, c, y.size)
    assert e.value.code == -10
    c = ctx.compress(d, 1e-3, 1)
    with pytest.raises(fz.FZError) as e:
        _noalloc(fz, c, x.size - 1)
    assert e.value.code == -4
