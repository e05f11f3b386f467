"""Pins for the oracle's interpolation predictor (the FZMod-Quality front
end, G-Interp on the prequantised integers): the level and axis of every
point worked out by hand, closed forms (a constant field leaves one
non-zero residual in the whole field; a linear ramp is predicted exactly
except where only the lower neighbour exists; cubic interpolation is exact
on cubic polynomials), inverse-after-forward identity on random integer
fields, and round trips within the bound."""
import numpy as np
import pytest

import oracle
from inputs import fields


def test_classes_worked_examples():
    ax, st = oracle.interp_classes((16, 16, 16))  # numpy order (z, y, x); axis 0 = x
    cases = {
        # (x, y, z): (axis, stride)
        (0, 0, 0): (-1, 8), (8, 8, 8): (-1, 8), (8, 0, 8): (-1, 8),
        (4, 0, 0): (0, 4), (0, 4, 0): (1, 4), (0, 0, 4): (2, 4), (4, 4, 0): (0, 4), (0, 4, 4): (1, 4),
        (12, 8, 0): (0, 4), (2, 0, 0): (0, 2), (0, 2, 4): (1, 2), (4, 4, 2): (2, 2), (6, 2, 2): (0, 2),
        (1, 2, 3): (0, 1), (2, 1, 0): (1, 1), (2, 4, 1): (2, 1), (15, 15, 15): (0, 1),
    }
    for (x, y, z), (a, s) in cases.items():
        assert (int(ax[z, y, x]), int(st[z, y, x])) == (a, s), (x, y, z)
    # anchors: every coordinate a multiple of 8
    n = 19
    ax, _ = oracle.interp_classes((n, n, n))
    assert int((ax == -1).sum()) == 3 ** 3


def _q_field(shape, fn):
    """float32 field of integers (absolute bound 0.5: grid step 1, q = x)."""
    idx = np.indices(shape)
    v = fn(*idx[::-1])  # fn(x, y, z...) with x the last numpy axis
    assert np.abs(v).max() < 2 ** 23
    return v.astype(np.float32)


def _residuals(x):
    q, _ = oracle.prequant(x, 0.5)
    d, _ = oracle.residual(q.reshape(x.shape), oracle.P_INTERP)
    return q.reshape(x.shape), d


@pytest.mark.parametrize("shape", [(19, 13, 22), (40, 33), (1001,), (8, 8, 8), (1, 1, 9)])
def test_constant_field_one_residual(shape):
    x = np.full(shape, 37.0, np.float32)
    _, d = _residuals(x)
    assert d.reshape(-1)[0] == 37
    assert np.count_nonzero(d) == 1


def test_linear_ramp_closed_form():
    n = 45
    x = _q_field((n,), lambda x: 3 * x + 5)
    q, d = _residuals(x)
    ax, st = oracle.interp_classes((n,))
    for i in range(n):
        s = int(st[i])
        if ax[i] == -1:
            exp = 5 if i == 0 else 3 * 8  # Lorenzo on the anchor grid
        elif i + s < n:
            exp = 0  # cubic or linear: exact on a line
        else:
            exp = 3 * s  # only the lower neighbour: q - q[-s]
        assert d[i] == exp, i


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cubic_exact_on_cubics(axis):
    shape = (40, 40, 40)
    x = _q_field(shape, lambda x, y, z: ([x, y, z][axis] - 20) ** 3 // 8)
    _, d = _residuals(x)
    ax, st = oracle.interp_classes(shape)
    # the cubic points along the varying axis: both 3s neighbours inside
    coord = np.indices(shape)[::-1][axis]
    cubic = (ax == axis) & (coord >= 3 * st.astype(int)) & (coord + 3 * st.astype(int) < 40)
    # q is the integer cubic itself only where (c - 20)^3 is divisible by 8
    # (even c); elsewhere the floor makes it a cubic plus a periodic term, so
    # check the even-coordinate points of strides 2 and 4
    sel = cubic & (st >= 2)
    assert sel.sum() > 100
    assert not d[sel].any()
    # points interpolated along another axis see a constant line: exact
    other = (ax >= 0) & (ax != axis)
    coord_o = [np.indices(shape)[::-1][a] for a in range(3)]
    inside = np.zeros(shape, bool)
    for a in range(3):
        m = (ax == a)
        inside |= m & (coord_o[a] + st.astype(int) < 40)
    assert not d[other & inside].any()


@pytest.mark.parametrize("shape", [(19, 13, 22), (40, 33), (1001,), (9, 8, 17), (3, 5), (1,), (2, 1, 1)])
def test_inverse_after_forward_identity(shape):
    r = np.random.default_rng(len(shape) + shape[0])
    q = r.integers(-2000, 2000, size=shape).astype(np.int32)
    d, _ = oracle.residual(q, oracle.P_INTERP)
    assert np.array_equal(oracle.residual_inverse(d, oracle.P_INTERP), q)
    # large values wrap consistently (residuals modulo 2^32)
    q2 = r.integers(-2 ** 24, 2 ** 24, size=shape).astype(np.int32)
    d2, _ = oracle.residual(q2, oracle.P_INTERP)
    assert np.array_equal(oracle.residual_inverse(d2, oracle.P_INTERP), q2)


@pytest.mark.parametrize("shape,eb", [((37, 45, 29), 1e-2), ((37, 45, 29), 1e-4), ((64, 64, 64), 1e-3),
                                      ((1001, 777), 1e-3), ((70001,), 1e-4), ((24, 24, 24), 1e-3), ((1,), 1e-3)])
def test_round_trip_within_bound(shape, eb):
    if shape == (24, 24, 24):
        x = fields.random_small(shape, 3, "wide")
    elif len(shape) == 1 and shape[0] > 1:
        x = fields.sorted_positions(shape[0], seed=5)
    elif shape == (1,):
        x = np.array([0.25], np.float32)
    else:
        x = fields.grf(shape, 3.0, seed=7)
    c = oracle.compress(x, eb, 1, pred=oracle.P_INTERP)
    h = oracle.header(c)
    assert h["pred"] == oracle.P_INTERP or h["flags"] & 1
    y = oracle.decompress(c)
    assert np.abs(y.astype(np.float64) - x).max() <= oracle.eb_abs(x, 1, eb)


def test_smooth_fields_compress_better_than_lorenzo():
    # the reason for the predictor: on smooth 3D fields the interpolation
    # residuals are smaller than block-local first-order Lorenzo's
    x = fields.grf((64, 64, 64), 4.0, seed=9)
    for eb in (1e-3, 1e-4):
        assert len(oracle.compress(x, eb, 1, pred=oracle.P_INTERP)) < len(oracle.compress(x, eb, 1, pred=0))


def test_rounding_worked_examples():
    # 1D, 32 values, q = 1 at x = 4, 8 and 28, else 0 (absolute bound 0.5)
    x = np.zeros(32, np.float32)
    x[[4, 8, 28]] = 1.0
    _, d = _residuals(x)
    # x = 5, cubic from 2, 4, 6, 8: -0 + 9 + 9*0 - 1 = 8 -> floor((8 + 8) / 16) = 1
    assert d[5] == -1
    # x = 3, cubic from 0, 2, 4, 6: 9 -> floor(17 / 16) = 1
    assert d[3] == -1
    # x = 29, linear from 28 and 30 (29 + 3 is outside): floor((1 + 0 + 1) / 2) = 1
    assert d[29] == -1
    # x = 31, only the lower neighbour: q[30] = 0
    assert d[31] == 0
    # x = 7, cubic from 4, 6, 8, 10: 9 + 0 + 9 * 1 - 0 = 18 -> floor(26 / 16) = 1
    assert d[7] == -1
