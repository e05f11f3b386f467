"""Pins for the oracle's global (non-blocked) first-order Lorenzo predictor
(Sec. 3.1's Lorenzo predictor with neighbours anywhere in the field): the
residual field against backward differences composed independently with
numpy along each axis over the whole field, a hand-worked 2x2 example, the
closed form for sums of one-axis functions, agreement with the block-local
predictor away from block faces, the inverse against numpy cumulative sums,
inverse-after-forward identity (also modulo 2^32), round trips within the
bound and smaller containers than the block-local predictor on smooth
fields (one corner outlier for the field instead of one per block)."""
import numpy as np
import pytest

import oracle
from inputs import fields

PG = oracle.P_GLOBAL


def _numpy_lorenzo(q):
    d = q.astype(np.int64)
    for ax in range(q.ndim):
        d = np.diff(d, axis=ax, prepend=0)
    return d


@pytest.mark.parametrize("shape", [(19, 13, 22), (8, 8, 8), (40, 33), (1001,), (1, 9, 17), (3, 1, 5), (1,)])
def test_residual_is_backward_difference_along_every_axis(shape):
    r = np.random.default_rng(sum(shape))
    q = r.integers(-5000, 5000, size=shape).astype(np.int32)
    d, _ = oracle.residual(q, PG)
    assert np.array_equal(d.astype(np.int64), _numpy_lorenzo(q))


def test_worked_example_2x2():
    q = np.array([[1, 2], [3, 5]], np.int32)  # q[y, x]
    d, _ = oracle.residual(q, PG)
    assert d.tolist() == [[1, 1], [2, 1]]


def test_sum_of_one_axis_functions():
    # q = f(x) + g(y) + h(z): the mixed difference vanishes wherever at most
    # one coordinate is 0; only the coordinate axes keep residuals
    r = np.random.default_rng(3)
    nz, ny, nx = 11, 14, 17
    f, g, h = (r.integers(-100, 100, n) for n in (nx, ny, nz))
    q = (f[None, None, :] + g[None, :, None] + h[:, None, None]).astype(np.int32)
    d, _ = oracle.residual(q, PG)
    z, y, x = np.indices(q.shape)
    zeros = (x == 0).astype(int) + (y == 0) + (z == 0)
    assert not d[zeros <= 1].any()
    # on the x axis (y = z = 0) the residual is f's backward difference
    assert np.array_equal(d[0, 0, 1:], np.diff(f))
    assert d[0, 0, 0] == f[0] + g[0] + h[0]


@pytest.mark.parametrize("shape", [(19, 13, 22), (40, 70), (1500,)])
def test_equals_block_local_away_from_block_faces(shape):
    r = np.random.default_rng(7)
    q = r.integers(-3000, 3000, size=shape).astype(np.int32)
    dg, _ = oracle.residual(q, PG)
    d0, _ = oracle.residual(q, oracle.P0)
    bs = {1: (512,), 2: (16, 32), 3: (8, 8, 8)}[len(shape)]
    idx = np.indices(shape)
    inner = np.ones(shape, bool)
    for a, b in enumerate(bs):
        inner &= idx[a] % b != 0
    assert np.array_equal(dg[inner], d0[inner])
    # and they differ somewhere on the faces
    assert not np.array_equal(dg, d0)


@pytest.mark.parametrize("shape", [(19, 13, 22), (40, 33), (1001,), (2, 1, 1)])
def test_inverse_is_cumulative_sum_and_undoes_the_residual(shape):
    r = np.random.default_rng(len(shape) * 11)
    d = r.integers(-50, 50, size=shape).astype(np.int32)
    q = oracle.residual_inverse(d, PG)
    want = d.astype(np.int64)
    for ax in range(d.ndim):
        want = np.cumsum(want, axis=ax)
    assert np.array_equal(q.astype(np.int64), want)
    # inverse after forward, also where sums wrap modulo 2^32
    for lo in (2000, 2 ** 24):
        qq = r.integers(-lo, lo, size=shape).astype(np.int32)
        dd, _ = oracle.residual(qq, PG)
        assert np.array_equal(oracle.residual_inverse(dd, PG), qq)


@pytest.mark.parametrize("shape,eb", [((37, 45, 29), 1e-3), ((64, 64, 64), 1e-4), ((1001, 777), 1e-3),
                                      ((70001,), 1e-4), ((24, 24, 24), 1e-3), ((1,), 1e-3)])
def test_round_trip_within_bound(shape, eb):
    if shape == (24, 24, 24):
        x = fields.random_small(shape, 3, "wide")
    elif len(shape) == 1 and shape[0] > 1:
        x = fields.sorted_positions(shape[0], seed=5)
    elif shape == (1,):
        x = np.array([0.25], np.float32)
    else:
        x = fields.grf(shape, 3.0, seed=7)
    c = oracle.compress(x, eb, 1, pred=PG)
    h = oracle.header(c)
    assert h["pred"] == PG or h["flags"] & 1
    y = oracle.decompress(c)
    assert np.abs(y.astype(np.float64) - x).max() <= oracle.eb_abs(x, 1, eb)


def test_smaller_than_block_local_on_smooth_fields():
    # the reason for the predictor: no residuals at block faces and corners.
    # On a smooth field the block-local corners keep the value itself (an
    # outlier once it exceeds the radius); globally only the field's origin
    # does.  (On noise-dominated fields at tight bounds the 8-term residual
    # is wider than the block faces' 4- and 2-term ones, so global is not
    # smaller there.)
    x = fields.sinusoid_field((64, 64, 64), seed=1)
    for eb in (1e-2, 1e-3, 1e-4):
        assert len(oracle.compress(x, eb, 1, pred=PG)) < len(oracle.compress(x, eb, 1, pred=oracle.P0))
    y = fields.grf((64, 64, 64), 4.0, seed=9) + np.float32(10)
    hg = oracle.header(oracle.compress(y, 1e-2, 1, pred=PG))
    h0 = oracle.header(oracle.compress(y, 1e-2, 1, pred=oracle.P0))
    assert hg["n_outliers"] == 1 and h0["n_outliers"] >= 500
