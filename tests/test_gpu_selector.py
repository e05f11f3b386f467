"""GPU parity of the per-block predictor choice against the CPU oracle:
block features (bit-identical floats), the selector network's predictions
and choices (bit-identical), the exhaustive trial's choices and costs, and
containers compressed with the selector's choice."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from inputs import fields

pytestmark = pytest.mark.gpu

SHAPES = [
    ("3d-64^3", (64, 64, 64), "grf", 1e-3, 1),
    ("3d-ragged", (37, 45, 29), "grf", 1e-4, 1),
    ("3d-steps", (24, 40, 56), "steps", 1e-3, 1),
    ("3d-wide", (16, 24, 24), "wide", 1e-3, 1),
    ("3d-abs", (40, 33, 17), "grf", 2e-4, 0),
    ("2d-ragged", (301, 777), "grf", 1e-3, 1),
    # x a multiple of the block, y/z not: whole rows, empty segments
    ("3d-yz-ragged", (21, 30, 48), "grf", 1e-3, 1),
    ("2d-y-ragged", (45, 96), "grf", 1e-3, 1),
    ("1d", (100003,), "positions", 1e-4, 1),
    ("1d-tiny", (5,), "grf", 1e-2, 1),
]


def _field(kind, shape, seed):
    if kind == "positions":
        return fields.sorted_positions(shape[0], seed=seed)
    if kind == "grf":
        return fields.grf(shape, alpha=3.0, seed=seed)
    return fields.random_small(shape, seed, kind)


def random_selector(seed):
    """A seeded selector with standardisation taken from a feature sample."""
    r = np.random.default_rng(seed)
    w = np.zeros(oracle.NPARAM, np.float32)
    for name, scale in (("W1", 0.5), ("b1", 0.1), ("W2", 0.2), ("b2", 0.1), ("W3", 0.3), ("b3", 0.1)):
        o, n = oracle.OFF[name]
        w[o:o + n] = r.normal(0, scale, n)
    o, n = oracle.OFF["mu"]
    w[o:o + n] = r.uniform(0, 4, n)
    o, n = oracle.OFF["rs"]
    w[o:o + n] = r.uniform(0.2, 1.5, n)
    return w


@pytest.fixture(scope="module")
def ctx(fz):
    return fz.Context(0)


@pytest.mark.parametrize("name,shape,kind,eb,mode", SHAPES, ids=[s[0] for s in SHAPES])
def test_features_bit_exact(fz, ctx, name, shape, kind, eb, mode):
    print(f"[gpu selector] features {name} {shape}", flush=True)
    x = _field(kind, shape, seed=len(name))
    f = ctx.block_features(torch.from_numpy(x).cuda(), eb, mode).cpu().numpy()
    fo = oracle.features(x, eb, mode)
    assert f.shape == fo.shape
    bad = np.nonzero(f.view(np.uint32) != fo.view(np.uint32))
    assert bad[0].size == 0, f"{name}: {bad[0].size} features differ, first block {bad[0][0]} feature {bad[1][0]}"


@pytest.mark.parametrize("name,shape,kind,eb,mode", SHAPES, ids=[s[0] for s in SHAPES])
def test_selector_bit_exact(fz, ctx, name, shape, kind, eb, mode):
    print(f"[gpu selector] network {name} {shape}", flush=True)
    x = _field(kind, shape, seed=len(name) + 1)
    w = random_selector(len(name))
    ctx.selector_set(w)
    ch, y = ctx.block_select(torch.from_numpy(x).cuda(), eb, mode)
    yo, cho = oracle.mlp_infer(w, oracle.features(x, eb, mode))
    assert np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32)), f"{name}: predictions differ"
    assert np.array_equal(ch.cpu().numpy(), cho), f"{name}: choices differ"


@pytest.mark.parametrize("name,shape,kind,eb,mode", SHAPES[:6], ids=[s[0] for s in SHAPES[:6]])
def test_compress_with_selector(fz, ctx, name, shape, kind, eb, mode):
    print(f"[gpu selector] compress {name} {shape}", flush=True)
    x = _field(kind, shape, seed=len(name) + 2)
    w = random_selector(len(name) + 5)
    ctx.selector_set(w)
    _, cho = oracle.mlp_infer(w, oracle.features(x, eb, mode))
    ref = oracle.compress(x, eb, mode, pred=oracle.P_SELECTED, choice=cho)
    c = ctx.compress(torch.from_numpy(x).cuda(), eb, mode, pred=3)
    got = c.cpu().numpy().tobytes()
    assert len(got) == len(ref)
    assert got == ref, f"{name}: container differs"
    y = ctx.decompress(c).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), oracle.decompress(ref).view(np.uint32))


@pytest.mark.parametrize("name,shape,kind,eb,mode", SHAPES, ids=[s[0] for s in SHAPES])
def test_trial_choices_and_costs(fz, ctx, name, shape, kind, eb, mode):
    print(f"[gpu selector] trial {name} {shape}", flush=True)
    x = _field(kind, shape, seed=len(name) + 3)
    ch, costs = ctx.block_trial(torch.from_numpy(x).cuda(), eb, mode)
    cho, co = oracle.trial(x, eb, mode)
    assert np.array_equal(costs.cpu().numpy().astype(np.uint32), co)
    assert np.array_equal(ch.cpu().numpy(), cho)


def test_selector_full_1024cubed(fz, ctx):
    """The selector workload at its full size and in the launch configuration
    the benchmark times (1024^3 fronts + spikes field, rel 1e-4): features and
    network outputs of 512 sampled blocks (the first and last among them)
    against the oracle block by block.  Features are block-local, so each
    sampled 8^3 block goes through the oracle alone at the field's absolute
    bound (resolved by the oracle from the whole field)."""
    from inputs import fields_gpu
    n, eb = 1024, 1e-4
    print(f"[gpu selector] full {n}^3 fronts/spikes rel {eb}", flush=True)
    x = fields_gpu.fronts_spikes((n, n, n), seed=3, device="cuda")
    w = random_selector(n)
    ctx.selector_set(w)
    f = ctx.block_features(x, eb, 1)
    ch, y = ctx.block_select(x, eb, 1)
    nb = n // 8
    picks = np.unique(np.concatenate([[0, nb ** 3 - 1], np.random.default_rng(11).choice(nb ** 3, 510, replace=False)]))
    f = f[torch.from_numpy(picks).cuda()].cpu().numpy()
    y = y[torch.from_numpy(picks).cuda()].cpu().numpy()
    ch = ch[torch.from_numpy(picks).cuda()].cpu().numpy()
    xh = x.cpu().numpy()
    del x
    e = oracle.eb_abs(xh, 1, eb)
    fo = np.empty((picks.size, 16), np.float32)
    for k, b in enumerate(picks):
        bz, by, bx = b // (nb * nb), (b // nb) % nb, b % nb
        blk = np.ascontiguousarray(xh[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8])
        fo[k] = oracle.features(blk, e, 0)[0]
    del xh
    bad = np.nonzero(f.view(np.uint32) != fo.view(np.uint32))
    assert bad[0].size == 0, f"{bad[0].size} features differ, first block {picks[bad[0][0]]} feature {bad[1][0]}"
    yo, cho = oracle.mlp_infer(w, fo)
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), "predictions differ"
    assert np.array_equal(ch, cho), "choices differ"


def test_selector_file_round_trip(fz, ctx):
    w = random_selector(99)
    ctx.selector_set(w)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "sel.bin")
        ctx.selector_save(path)
        other = fz.Context(0)
        other.selector_load(path)
        assert np.array_equal(other.selector_get().view(np.uint32), w.view(np.uint32))
        raw = bytearray(open(path, "rb").read())
        raw[8] = 1  # another feature-set version (the first)
        bad = os.path.join(d, "bad.bin")
        open(bad, "wb").write(bytes(raw))
        with pytest.raises(fz.FZError) as e:
            other.selector_load(bad)
        assert e.value.code == -5


def test_selector_required(fz):
    c = fz.Context(0)
    x = torch.zeros((16, 16, 16), device="cuda")
    with pytest.raises(fz.FZError) as e:
        c.compress(x, 1e-3, 1, pred=3)
    assert e.value.code == -8
    with pytest.raises(fz.FZError):
        c.selector_set(np.full(5475, np.nan, np.float32))
