"""Pins for the per-block predictors (first- and second-order Lorenzo,
fixed-point linear regression), the predictor map in the container and the
exhaustive per-block trial selection."""
import itertools

import numpy as np
import pytest

import oracle
from inputs import fields

BS = {1: (512,), 2: (16, 32), 3: (8, 8, 8)}


def _local(shape):
    """Per-axis in-block coordinate grids (C order)."""
    bs = BS[len(shape)]
    grids = np.meshgrid(*[np.arange(n) % b for n, b in zip(shape, bs)], indexing="ij")
    return grids


def _backdiff(a, axis, bs):
    """Backward difference along one axis with zero outside the block."""
    prev = np.zeros_like(a)
    dst = [slice(None)] * a.ndim
    src = [slice(None)] * a.ndim
    dst[axis] = slice(1, None)
    src[axis] = slice(0, -1)
    prev[tuple(dst)] = a[tuple(src)]
    local = np.arange(a.shape[axis]) % bs
    view = [1] * a.ndim
    view[axis] = a.shape[axis]
    return a - prev * (local.reshape(view) > 0)


@pytest.mark.parametrize("shape", [(1100,), (40, 70), (17, 33), (9, 10, 11), (16, 24, 8), (3, 5, 2)])
def test_second_order_is_twice_composed_differences(shape):
    r = fields.rng(31 + sum(shape))
    q = r.integers(-2 ** 18, 2 ** 18, size=shape).astype(np.int32)
    d, _ = oracle.residual(q, oracle.P1)
    ref = q.astype(np.int64)
    bs = BS[len(shape)]
    for axis in range(len(shape)):
        ref = _backdiff(_backdiff(ref, axis, bs[axis]), axis, bs[axis])
    assert np.array_equal(d.astype(np.int64), ref)


@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("shape", [(1100,), (40, 70), (9, 10, 11), (17, 9, 25)])
def test_inverse_identity(p, shape):
    r = fields.rng(5 + p + len(shape))
    q = r.integers(-2 ** 22, 2 ** 22, size=shape).astype(np.int32)
    d, coef = oracle.residual(q, p)
    assert np.array_equal(oracle.residual_inverse(d, p, coef), q)


def test_second_order_annihilates_linear_along_x():
    z, y, x = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    q = (7 + 3 * x + 0 * y).astype(np.int32)
    d, _ = oracle.residual(q, oracle.P1)
    lx = x % 8
    assert not d[lx >= 2].any()
    assert d[lx < 2].any()


@pytest.mark.parametrize("shape", [(16, 16, 16), (13, 11, 9), (40, 37), (1030,)])
def test_regression_exact_on_planes(shape):
    grids = _local(shape)
    r = fields.rng(9)
    c = r.integers(-50, 50, size=len(shape) + 1)
    q = c[0] + sum(ci * g for ci, g in zip(c[1:], grids))
    q = q.astype(np.int32)
    d, coef = oracle.residual(q, oracle.P2)
    assert not d.any()


def test_regression_matches_least_squares():
    r = fields.rng(10)
    q = r.integers(-1000, 1000, size=(8, 8, 8)).astype(np.int32)
    d, coef = oracle.residual(q, oracle.P2)
    w, v, u = [2 * g - 7 for g in _local(q.shape)]
    A = np.stack([np.ones(q.size), u.ravel(), v.ravel(), w.ravel()], axis=1).astype(np.float64)
    sol, *_ = np.linalg.lstsq(A, q.ravel().astype(np.float64), rcond=None)
    assert np.all(np.abs(coef[0] - np.rint(256 * sol)) <= 1)


def test_regression_rounds_half_away_from_zero():
    # one full 1D block whose sum is +-1: mean * 256 = +-0.5 -> +-1
    for s in (1, -1):
        q = np.zeros(512, np.int32)
        q[0] = s
        d, coef = oracle.residual(q, oracle.P2)
        # slope term: sum(u q) / sum(u^2) with u = 2i - 511 at i = 0 -> -511 s / 44739200
        assert coef[0, 0] == s


def test_trial_costs_and_choice():
    x = fields.grf((24, 20, 28), seed=14)
    eb = 1e-3
    choice, costs = oracle.trial(x, eb, 1)
    assert np.array_equal(choice, np.argmin(costs, axis=1))  # ties -> lowest index (argmin)
    # independent recomputation of the costs from residuals and the reference code
    e = oracle.eb_abs(x, 1, eb)
    q, _ = oracle.prequant(x, e)
    codes0, pos, hist, _ = oracle.stage_codes(x, eb, 1)
    ln = oracle.codebook(hist).astype(np.int64)
    ln[ln == 0] = 13
    blk = (pos // 512).astype(np.int64)
    order = np.argsort(pos, kind="stable")
    # row-major index of each block-major entry
    nz, ny, nx = x.shape
    local = pos % 512
    b = pos // 512
    nbx, nby = -(-nx // 8), -(-ny // 8)
    bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
    xi = bx * 8 + local % 8
    yi = by * 8 + (local // 8) % 8
    zi = bz * 8 + local // 64
    rmi = xi + nx * (yi + ny * zi)
    for p in range(3):
        d, _ = oracle.residual(q, p)
        dv = d.ravel()[rmi].astype(np.int64)
        code = np.where(np.abs(dv) < 512, dv + 512, 0)
        bits = ln[code] + 64 * (code == 0)
        cost = np.bincount(blk, weights=bits, minlength=costs.shape[0]) + (128 if p == 2 else 0)
        assert np.array_equal(cost.astype(np.int64), costs[:, p].astype(np.int64)), p
    assert len(set(choice.tolist())) >= 1 and order.size == x.size


@pytest.mark.parametrize("pred", [1, 2, 3, 4])
@pytest.mark.parametrize("shape,eb", [((24, 20, 28), 1e-3), ((130, 70), 1e-4), ((3000,), 1e-3), ((9, 7, 5), 1e-2)])
def test_round_trip_with_predictors(pred, shape, eb):
    x = fields.grf(shape, seed=sum(shape)) if len(shape) > 1 else fields.sorted_positions(shape[0], seed=2)
    choice = None
    if pred == 3:
        choice = fields.rng(1).integers(0, 3, oracle.nblocks_of(shape)).astype(np.uint8)
    c = oracle.compress(x, eb, 1, pred=pred, choice=choice)
    h = oracle.header(c)
    y = oracle.decompress(c)
    assert np.abs(x.astype(np.float64) - y).max() <= h["eb_abs"]
    if not h["flags"] & 1:
        # the map is kept only when at least one block in 64 leaves
        # first-order Lorenzo; otherwise a first-order container
        want = pred
        nb = oracle.nblocks_of(shape)
        if pred == 3 and 64 * int((choice != 0).sum()) < nb:
            want = 0
        if pred == 4 and 64 * int((oracle.trial(x, eb, 1)[0] != 0).sum()) < nb:
            want = 0
        assert h["pred"] == want
        if pred == 2:
            assert h["n_reg"] == oracle.nblocks_of(shape)
        if pred == 3:
            assert h["n_reg"] == int((choice == 2).sum())


def test_trial_never_worse_than_fixed_by_reference_cost():
    x = fields.fronts_spikes((32, 32, 32), seed=3, n_fronts=4, spike_frac=0.001)
    for eb in (1e-2, 1e-4):
        choice, costs = oracle.trial(x, eb, 1)
        best = costs[np.arange(costs.shape[0]), choice].sum()
        assert best <= costs[:, 0].sum() and best <= costs[:, 1].sum() and best <= costs[:, 2].sum()


def test_all_first_order_choice_is_a_first_order_container():
    # no map when every block keeps first-order Lorenzo: the same bytes as
    # the first-order container, for the selector's and trial's choices;
    # likewise when fewer than one block in 64 leaves it (those blocks are
    # coded first-order too)
    x = fields.grf((130, 70), seed=200)
    nb = oracle.nblocks_of(x.shape)
    for eb in (1e-2, 1e-4):
        ref = oracle.compress(x, eb, 1, pred=0)
        assert oracle.compress(x, eb, 1, pred=3, choice=np.zeros(nb, np.uint8)) == ref
        ch, _ = oracle.trial(x, eb, 1)
        if not ch.any():
            assert oracle.compress(x, eb, 1, pred=4) == ref
    # one block off first-order among the 27 keeps the map
    ch = np.zeros(nb, np.uint8)
    ch[3] = 1
    h = oracle.header(oracle.compress(x, 1e-2, 1, pred=3, choice=ch))
    assert h["pred"] == 3 and nb == 27
    # 3D, 512 blocks: 7 switched blocks (64 * 7 < 512) drop the map, 8 keep it
    y = fields.grf((64, 64, 64), seed=201)
    ch = np.zeros(512, np.uint8)
    ch[:7] = 2
    assert oracle.compress(y, 1e-3, 1, pred=3, choice=ch) == oracle.compress(y, 1e-3, 1, pred=0)
    ch[7] = 1
    h = oracle.header(oracle.compress(y, 1e-3, 1, pred=3, choice=ch))
    assert h["pred"] == 3 and h["n_reg"] == 7
