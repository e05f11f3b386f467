"""GPU parity of the per-block predictors (second-order Lorenzo, linear
regression, and the per-block choice by exhaustive trial) against the CPU
oracle: byte-identical containers (map, coefficients, codes, outliers,
patches, stream), bit-identical reconstructions within the bound."""
import numpy as np
import pytest
import torch

import oracle
from inputs import fields

pytestmark = pytest.mark.gpu

P1, P2, PT = oracle.P1, oracle.P2, oracle.P_TRIAL

CASES = [
    # name, kind, shape, eb, mode
    ("3d-sinusoid-64^3", "sinusoid", (64, 64, 64), 1e-3, 1),
    ("3d-ragged", "smooth", (37, 45, 29), 1e-3, 1),
    ("3d-ragged-tight", "smooth", (70, 33, 130), 1e-4, 1),
    ("3d-steps", "steps", (48, 40, 56), 1e-3, 1),
    ("3d-wide-patches", "wide", (24, 24, 24), 1e-3, 1),
    ("3d-noise", "noise", (20, 30, 40), 1e-2, 1),
    ("3d-thin", "smooth", (3, 64, 40), 1e-3, 1),
    ("2d-ragged", "smooth", (1001, 777), 1e-3, 1),
    ("2d-small", "smooth", (3, 5), 1e-2, 1),
    ("1d-positions", "positions", (300007,), 1e-4, 1),
    ("1d-ragged", "smooth", (513,), 1e-3, 1),
    ("1d-one", "const", (1,), 1e-3, 1),
    ("3d-grf-abs", "grf", (96, 80, 72), 3e-4, 0),
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


def _check(fz, ctx, x, eb, mode, pred, name):
    print(f"[gpu predictors] {name} pred={pred} shape={x.shape} eb={eb} mode={mode}", flush=True)
    ref = oracle.compress(x, eb, mode, pred=pred)
    d = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    c = ctx.compress(d, eb, mode, pred=pred)
    got = c.cpu().numpy().tobytes()
    h = oracle.header(ref)
    assert len(got) == len(ref), f"{name}: size {len(got)} vs oracle {len(ref)} ({h})"
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
    return h


@pytest.mark.parametrize("pred", [P1, P2, PT], ids=["lorenzo2", "regression", "trial"])
@pytest.mark.parametrize("name,kind,shape,eb,mode", CASES, ids=[c[0] for c in CASES])
def test_predictor_parity(fz, ctx, name, kind, shape, eb, mode, pred):
    x = _field(kind, shape, seed=len(name) + 7)
    _check(fz, ctx, x, eb, mode, pred, name)


def test_trial_full_256cubed(fz, ctx):
    """Trial mode on a 256^3 k^-3 field: every block's choice (the map) and
    the whole container against the oracle; the choice must not cost more
    than plain first-order Lorenzo."""
    x = fields.grf((256, 256, 256), alpha=3.0, seed=21)
    h = _check(fz, ctx, x, 1e-3, 1, PT, "256^3 grf trial")
    h0 = oracle.header(ctx.compress(torch.from_numpy(x).cuda(), 1e-3, 1).cpu().numpy().tobytes())
    assert h["total"] <= h0["total"] * 1.001


def test_mixed_modes_one_context(fz, ctx):
    """Switching predictors on one context leaves no state behind."""
    x = fields.grf((40, 48, 56), seed=4)
    for pred in (0, P2, PT, P1, 0, PT):
        _check(fz, ctx, x, 1e-3, 1, pred, f"mixed {pred}")
