"""Bit-exact parity with the oracle at the sizes of the benchmarked
configurations:
  - the 1024^3 fronts/spikes field's per-GPU share (a 1024x1024x128 slab,
    the z-slab one of eight GPUs would hold), compressed as a field of its
    own at rel 1e-4 with first-order Lorenzo, exhaustive trial and a
    selector network: whole containers and reconstructions;
  - all 64 uneven 2D fields of the batch configuration (one graph-captured
    batch call), every container and reconstruction;
  - a mixed batch shaped like the 256-field configuration's members (a 1D
    field of 2^24 sorted positions, 2D and 3D fields) with the selector.
Inputs come from the seeded device generators and are copied to the host
for the oracle."""
import numpy as np
import pytest
import torch

import oracle
from inputs import fields_gpu

pytestmark = pytest.mark.gpu


def random_selector(seed):
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


@pytest.fixture(scope="module")
def slab():
    x = fields_gpu.fronts_spikes((1024, 1024, 1024), seed=3, device="cuda")
    s = x[:128].contiguous()
    del x
    torch.cuda.empty_cache()
    return s


def _first_diff(a, b):
    a = np.frombuffer(a, np.uint8)
    b = np.frombuffer(b, np.uint8)
    n = min(a.size, b.size)
    d = np.nonzero(a[:n] != b[:n])[0]
    return int(d[0]) if d.size else n


@pytest.mark.parametrize("mode", ["lorenzo1", "trial", "selector"])
def test_fronts_spikes_slab(fz, ctx, slab, mode):
    eb = 1e-4
    print(f"[gpu configs] 1024x1024x128 fronts/spikes slab rel {eb} {mode}", flush=True)
    xh = slab.cpu().numpy()
    if mode == "selector":
        w = random_selector(77)
        ctx.selector_set(w)
        _, cho = oracle.mlp_infer(w, oracle.features(xh, eb, 1))
        ref = oracle.compress(xh, eb, 1, pred=oracle.P_SELECTED, choice=cho)
        c = ctx.compress(slab, eb, 1, pred=3)
    else:
        pred = 0 if mode == "lorenzo1" else 4
        ref = oracle.compress(xh, eb, 1, pred=pred)
        c = ctx.compress(slab, eb, 1, pred=pred)
    got = c.cpu().numpy().tobytes()
    h = oracle.header(ref)
    print(f"[gpu configs] {mode}: {len(ref)} bytes, {h['n_outliers']} outliers, {h['n_reg']} regression blocks",
          flush=True)
    assert len(got) == len(ref) and got == ref, f"{mode}: container differs at byte {_first_diff(got, ref)}"
    y = ctx.decompress(c).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), oracle.decompress(ref).view(np.uint32)), f"{mode}: reconstruction"
    assert np.abs(y.astype(np.float64) - xh).max() <= h["eb_abs"]


@pytest.fixture(scope="module")
def batch2d(fz, ctx):
    batch = fields_gpu.batch_2d(n_fields=64, device="cuda")
    xs = [f for f, _ in batch]
    ebs = [eb for _, eb in batch]
    packed, offs = ctx.compress_batch(xs, ebs)
    outs = [torch.empty_like(x) for x in xs]
    ctx.decompress_batch(packed, offs, outs)
    return xs, ebs, packed.cpu().numpy(), offs, [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("part", range(4))
def test_batch2d_all_fields(fz, batch2d, part):
    xs, ebs, host, offs, outs = batch2d
    for i in range(16 * part, 16 * part + 16):
        xh = xs[i].cpu().numpy()
        print(f"[gpu configs] 2D batch field {i} {xh.shape} rel {ebs[i]:.3g}", flush=True)
        ref = oracle.compress(xh, ebs[i], 1)
        got = host[offs[i]:offs[i + 1]].tobytes()
        assert got[:len(ref)] == ref, f"field {i}: container differs at byte {_first_diff(got, ref)}"
        assert len(got) == (len(ref) + 15) // 16 * 16 and not any(got[len(ref):])
        assert np.array_equal(outs[i].view(np.uint32), oracle.decompress(ref).view(np.uint32)), f"field {i}"


def test_mixed_batch_with_selector(fz, ctx):
    w = random_selector(5)
    ctx.selector_set(w)
    members = [
        (fields_gpu.sorted_positions(1 << 24, seed=5100, device="cuda"), 3e-5),
        (fields_gpu.batch_2d(n_fields=1, seed=5101, device="cuda")[0][0], 1e-3),
        (fields_gpu.grf((96, 96, 96), alpha=4.0, seed=5102, device="cuda"), 1e-4),
        (fields_gpu.grf((200, 200, 200), alpha=3.0, seed=5103, device="cuda"), 1e-2),
        (fields_gpu.grf((64, 64, 64), alpha=5.0, seed=5104, device="cuda"), 1e-5),
    ]
    xs = [m for m, _ in members]
    ebs = [eb for _, eb in members]
    packed, offs = ctx.compress_batch(xs, ebs, preds=[3] * len(xs))
    outs = [torch.empty_like(x) for x in xs]
    ctx.decompress_batch(packed, offs, outs)
    host = packed.cpu().numpy()
    for i, (x, eb) in enumerate(members):
        xh = x.cpu().numpy()
        print(f"[gpu configs] mixed member {i} {xh.shape} rel {eb}", flush=True)
        _, cho = oracle.mlp_infer(w, oracle.features(xh, eb, 1))
        ref = oracle.compress(xh, eb, 1, pred=oracle.P_SELECTED, choice=cho)
        got = host[offs[i]:offs[i + 1]].tobytes()
        assert got[:len(ref)] == ref, f"member {i}: container differs at byte {_first_diff(got, ref)}"
        y = outs[i].cpu().numpy()
        assert np.array_equal(y.view(np.uint32), oracle.decompress(ref).view(np.uint32)), f"member {i}"
