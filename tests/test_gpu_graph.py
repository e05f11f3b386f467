"""Graph mode (stage tasks with declared accesses, dependencies inferred,
independent stages on concurrent branches, captured once and replayed)
against the eager calls and the oracle: containers byte for byte,
reconstructions bit for bit, for every predictor mode, both codecs and a
verbatim field; replays with eager work in between; the captured graphs'
shape (two concurrent branches in compression and in decompression)."""
import time

import numpy as np
import pytest
import torch

import oracle
from inputs import fields

pytestmark = pytest.mark.gpu

CASES = [
    # name, shape, eb, mode, pred, codec
    ("3d-ragged", (37, 45, 29), 1e-3, 1, 0, "huffman"),
    ("3d-tight-outliers", (70, 33, 130), 1e-4, 1, 0, "huffman"),
    ("3d-abs", (32, 48, 64), 2e-4, 0, 0, "huffman"),
    ("2d", (1001, 777), 1e-3, 1, 0, "huffman"),
    ("1d", (70001,), 1e-3, 1, 0, "huffman"),
    ("3d-noise-verbatim", (20, 30, 40), 1e-7, 1, 0, "huffman"),
    ("3d-lorenzo2", (48, 40, 56), 1e-3, 1, 1, "huffman"),
    ("3d-regression", (48, 40, 56), 1e-3, 1, 2, "huffman"),
    ("3d-trial", (48, 40, 56), 1e-4, 1, 4, "huffman"),
    ("3d-shuffle", (37, 45, 29), 1e-3, 1, 0, "shuffle"),
    ("2d-shuffle-tight", (257, 1800), 1e-5, 1, 0, "shuffle"),
]


def _field(name, shape):
    if name.startswith("1d"):
        return fields.sorted_positions(shape[0], seed=7)
    if "noise" in name:
        return fields.random_small(shape, 4, "noise")
    return fields.grf(shape, 3.0, seed=len(name))


@pytest.fixture(scope="module")
def ctxs(fz):
    eager = fz.Context(0)
    graph = fz.Context(0)
    graph.set_graph_mode(True)
    return eager, graph


@pytest.mark.parametrize("name,shape,eb,mode,pred,codec", CASES, ids=[c[0] for c in CASES])
def test_graph_mode_matches_eager_and_oracle(fz, ctxs, name, shape, eb, mode, pred, codec):
    eager, graph = ctxs
    print(f"[gpu graph] {name} shape={shape} eb={eb} pred={pred} codec={codec}", flush=True)
    x = _field(name, shape)
    d = torch.from_numpy(x).cuda()
    ref = oracle.speed_compress(x, eb, mode) if codec == "shuffle" else oracle.compress(x, eb, mode, pred=pred)
    ce = eager.compress(d, eb, mode, pred=pred, codec=codec)
    for rep in range(3):
        cg = graph.compress(d, eb, mode, pred=pred, codec=codec)
        assert cg.cpu().numpy().tobytes() == ref, f"{name}: graph container differs (replay {rep})"
        # eager work on the same device between replays
        assert eager.compress(d, eb, mode, pred=pred, codec=codec).cpu().numpy().tobytes() == ref
    assert ce.cpu().numpy().tobytes() == ref
    ye = eager.decompress(ce).cpu().numpy()
    for rep in range(3):
        yg = graph.decompress(cg).cpu().numpy()
        assert np.array_equal(yg.view(np.uint32), ye.view(np.uint32)), f"{name}: graph reconstruction (replay {rep})"
        eager.decompress(ce)
    assert np.array_equal(ye.view(np.uint32), oracle.decompress(ref).view(np.uint32))


def test_graph_shapes(fz, ctxs):
    _, graph = ctxs
    x = torch.from_numpy(fields.grf((64, 64, 64), 3.0, seed=3)).cuda()
    c = graph.compress(x, 1e-3, 1)
    # reset, minmax, quant, scan_counts, codebook, encode, finalize: the
    # outlier-count scan beside the code and encoder
    tasks, streams, width, edges = graph.graph_info(0)
    print(f"[gpu graph] compress graph: {tasks} tasks, {streams} streams, width {width}, {edges} edges", flush=True)
    assert (tasks, width, streams) == (7, 2, 2) and edges == 7
    graph.decompress(c)
    # lut, scan, oindex, decode, patch: the outlier index beside the scan
    tasks, streams, width, edges = graph.graph_info(1)
    print(f"[gpu graph] decompress graph: {tasks} tasks, {streams} streams, width {width}, {edges} edges", flush=True)
    assert (tasks, width, streams) == (5, 2, 2)
    with pytest.raises(fz.FZError):
        fz.Context(0).graph_info(0)


def test_graph_recaptures_on_new_buffers(fz, ctxs):
    eager, graph = ctxs
    xs = [fields.grf((40, 48, 56), 3.0, seed=s) for s in (1, 2)]
    for x in xs + xs:
        d = torch.from_numpy(x).cuda()
        assert graph.compress(d, 1e-3, 1).cpu().numpy().tobytes() == oracle.compress(x, 1e-3, 1)
    # a larger field grows the scratch: the next call must not replay a
    # graph that holds the old buffers
    big = fields.grf((96, 96, 96), 3.0, seed=4)
    d = torch.from_numpy(big).cuda()
    assert graph.compress(d, 1e-3, 1).cpu().numpy().tobytes() == oracle.compress(big, 1e-3, 1)
    d = torch.from_numpy(xs[0]).cuda()
    assert graph.compress(d, 1e-3, 1).cpu().numpy().tobytes() == oracle.compress(xs[0], 1e-3, 1)


def test_graph_small_field_latency(fz, ctxs):
    """Report only: call latency of the 64^3 field eager vs graph mode."""
    eager, graph = ctxs
    x = torch.from_numpy(fields.sinusoid_field((64, 64, 64), seed=1)).cuda()
    out = torch.empty(eager.compress_bound(x.shape), dtype=torch.uint8, device="cuda")
    res = {}
    for name, ctx in (("eager", eager), ("graph", graph)):
        c = ctx.compress(x, 1e-3, 1, out=out)
        hdr = c[:128].cpu().numpy().tobytes()
        y = torch.empty_like(x)
        for _ in range(3):
            ctx.compress(x, 1e-3, 1, out=out)
            ctx.decompress(c, header=hdr, out=y)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(20):
            ctx.compress(x, 1e-3, 1, out=out)
        tc = (time.perf_counter() - t) / 20
        t = time.perf_counter()
        for _ in range(20):
            ctx.decompress(c, header=hdr, out=y)
        td = (time.perf_counter() - t) / 20
        res[name] = (tc * 1e6, td * 1e6)
    print(f"[gpu graph] 64^3 call latency us (compress, decompress): {res}", flush=True)
