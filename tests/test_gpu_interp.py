"""GPU parity of the interpolation predictor (the FZMod-Quality front end,
predictor 5) with the oracle: byte-identical containers (codes, outliers,
patches, stream), bit-identical reconstructions within the bound, on 3D,
2D and 1D fields with ragged edges, thin and tiny extents, outliers,
lossless patches and the verbatim fallback; graph mode and the batch call;
a 512^3 field at three bounds (containers byte for byte; reconstructions
against the prequantised values, which dual quantisation reproduces
exactly at any size)."""
import numpy as np
import pytest
import torch

import oracle
from inputs import fields, fields_gpu

pytestmark = pytest.mark.gpu

PI = oracle.P_INTERP

CASES = [
    # name, kind, shape, eb, mode
    ("3d-sinusoid-64^3", "sinusoid", (64, 64, 64), 1e-3, 1),
    ("3d-ragged", "smooth", (37, 45, 29), 1e-3, 1),
    ("3d-ragged-tight", "smooth", (70, 33, 130), 1e-4, 1),
    ("3d-grf-1e-2", "grf", (96, 80, 72), 1e-2, 1),
    ("3d-grf-abs", "grf", (96, 80, 72), 3e-4, 0),
    ("3d-steps", "steps", (48, 40, 56), 1e-3, 1),
    ("3d-wide", "wide", (24, 24, 24), 1e-3, 1),
    ("3d-noise", "noise", (20, 30, 40), 1e-2, 1),
    ("3d-noise-verbatim", "noise", (20, 30, 40), 1e-7, 1),
    ("3d-thin", "smooth", (3, 64, 40), 1e-3, 1),
    ("3d-tiny", "smooth", (2, 3, 5), 1e-3, 1),
    ("3d-const", "const", (17, 9, 33), 1e-3, 1),
    # rows longer than one workgroup's 512 values: the even points of the
    # neighbouring workgroups' pairs rebuilt at the range edges
    ("3d-long-rows", "smooth", (20, 21, 1100), 1e-3, 1),
    ("3d-long-rows-odd", "smooth", (18, 17, 1025), 1e-4, 1),
    # rows of several 512-point chunks on the stride-4 and stride-2 lattices
    ("3d-rows-3-chunks", "smooth", (6, 13, 2301), 1e-4, 1),
    ("2d-rows-3-chunks", "smooth", (9, 2500), 1e-3, 1),
    # degenerate lattices: one row per plane, rows of one to three values
    ("3d-one-row", "smooth", (19, 1, 37), 1e-3, 1),
    ("3d-narrow-x", "smooth", (21, 18, 3), 1e-3, 1),
    ("3d-one-x", "smooth", (13, 11, 1), 1e-3, 1),
    ("2d-one-column", "smooth", (37, 1), 1e-3, 1),
    ("3d-one-plane", "smooth", (1, 20, 30), 1e-3, 1),
    ("3d-two-planes-long-rows", "smooth", (2, 9, 1500), 1e-4, 1),
    ("2d-ragged", "smooth", (1001, 777), 1e-3, 1),
    ("2d-small", "smooth", (3, 5), 1e-2, 1),
    ("1d-positions", "positions", (300007,), 1e-4, 1),
    ("1d-ragged", "smooth", (513,), 1e-3, 1),
    ("1d-one", "const", (1,), 1e-3, 1),
]


def _field(kind, shape, seed):
    if kind == "sinusoid":
        return fields.sinusoid_field(shape, seed=seed)
    if kind == "positions":
        return fields.sorted_positions(shape[0], seed=seed)
    if kind == "grf":
        return fields.grf(shape, alpha=3.0, seed=seed)
    return fields.random_small(shape, seed, kind)


@pytest.fixture(scope="module")
def ctx(fz):
    return fz.Context(0)


def _first_diff(a, b):
    a = np.frombuffer(a, np.uint8)
    b = np.frombuffer(b, np.uint8)
    n = min(a.size, b.size)
    d = np.nonzero(a[:n] != b[:n])[0]
    return int(d[0]) if d.size else n


@pytest.mark.parametrize("name,kind,shape,eb,mode", CASES, ids=[c[0] for c in CASES])
def test_interp_parity(fz, ctx, name, kind, shape, eb, mode):
    x = _field(kind, shape, seed=len(name) + 11)
    print(f"[gpu interp] {name} shape={x.shape} eb={eb} mode={mode}", flush=True)
    ref = oracle.compress(x, eb, mode, pred=PI)
    h = oracle.header(ref)
    d = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    got = ctx.compress(d, eb, mode, pred=PI).cpu().numpy().tobytes()
    assert len(got) == len(ref) and got == ref, \
        f"{name}: {len(got)} vs {len(ref)} bytes, first difference at {_first_diff(got, ref)} ({h})"
    c = torch.from_numpy(np.frombuffer(ref, np.uint8).copy()).to("cuda:0")
    y = ctx.decompress(c).cpu().numpy()
    yo = oracle.decompress(ref)
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), f"{name}: reconstruction differs"
    err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max() if x.size else 0.0
    assert err <= h["eb_abs"], f"{name}: max error {err} > {h['eb_abs']}"
    if name == "3d-noise-verbatim":
        assert h["flags"] & 1
    if name == "3d-ragged-tight":
        assert h["n_outliers"] > 0
    if name in ("3d-steps", "1d-positions"):
        assert h["n_patches"] > 0


def test_interp_in_graph_mode(fz, ctx):
    g = fz.Context(0)
    g.set_graph_mode(True)
    x = fields.grf((48, 40, 56), alpha=3.0, seed=21)
    d = torch.from_numpy(x).cuda()
    ref = oracle.compress(x, 1e-4, 1, pred=PI)
    yo = oracle.decompress(ref)
    for rep in range(3):
        print(f"[gpu interp] graph mode replay {rep}", flush=True)
        c = g.compress(d, 1e-4, 1, pred=PI)
        assert c.cpu().numpy().tobytes() == ref, f"graph container (replay {rep})"
        # eager work between replays
        assert ctx.compress(d, 1e-4, 1, pred=PI).cpu().numpy().tobytes() == ref
        y = g.decompress(c).cpu().numpy()
        assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), f"graph reconstruction (replay {rep})"
    # the residual decode feeds the interpolation passes
    tasks, _, _, _ = g.graph_info(0)
    assert tasks == 7
    tasks, _, _, _ = g.graph_info(1)
    assert tasks == 6


def test_interp_in_batch(fz, ctx):
    xs = [fields.grf((40, 48, 56), alpha=3.0, seed=31), fields.random_small((1001, 777), 32, "smooth"),
          fields.sorted_positions(70001, seed=33), fields.grf((64, 64, 64), alpha=4.0, seed=34)]
    ebs = [1e-3, 1e-3, 1e-4, 1e-4]
    preds = [PI, PI, 0, PI]
    print("[gpu interp] batch of 4 (three interpolation members)", flush=True)
    ds = [torch.from_numpy(x).cuda() for x in xs]
    packed, offs = ctx.compress_batch(ds, ebs, preds=preds)
    host = packed.cpu().numpy()
    outs = [torch.empty_like(d) for d in ds]
    ctx.decompress_batch(packed, offs, outs)
    for i, x in enumerate(xs):
        ref = oracle.compress(x, ebs[i], 1, pred=preds[i])
        got = host[offs[i]:offs[i + 1]].tobytes()
        assert got[:len(ref)] == ref, f"member {i}: container differs at byte {_first_diff(got, ref)}"
        y = outs[i].cpu().numpy()
        assert np.array_equal(y.view(np.uint32), oracle.decompress(ref).view(np.uint32)), f"member {i}"


@pytest.fixture(scope="module")
def f512():
    return fields_gpu.grf((512, 512, 512), alpha=3.0, seed=512, device="cuda")


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_interp_512cubed(fz, ctx, f512, eb):
    print(f"[gpu interp] 512^3 k^-3 field rel {eb}", flush=True)
    xh = f512.cpu().numpy()
    ref = oracle.compress(xh, eb, 1, pred=PI)
    h = oracle.header(ref)
    c = ctx.compress(f512, eb, 1, pred=PI)
    got = c.cpu().numpy().tobytes()
    print(f"[gpu interp] 512^3 rel {eb}: {len(ref)} bytes (ratio {xh.nbytes / len(ref):.2f}), "
          f"{h['n_outliers']} outliers", flush=True)
    assert len(got) == len(ref) and got == ref, f"container differs at byte {_first_diff(got, ref)}"
    y = ctx.decompress(c).cpu().numpy()
    # dual quantisation: decompression returns the prequantised values
    q, patch = oracle.prequant(xh, h["eb_abs"])
    e2 = 2.0 * h["eb_abs"]
    want = (q.astype(np.float64) * e2).astype(np.float32).reshape(xh.shape)
    pm = patch.reshape(xh.shape).astype(bool)
    want[pm] = xh[pm]
    assert np.array_equal(y.view(np.uint32), want.view(np.uint32))
    assert np.abs(y.astype(np.float64) - xh).max() <= h["eb_abs"]
