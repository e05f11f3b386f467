"""Pins of the oracle's block features, selector network and training
arithmetic against closed forms, hand-built networks, finite differences
and the first Adam step."""
import numpy as np
import pytest

import oracle

F = oracle.NFEAT


def _plog2_1p(v):
    # piecewise-linear log2 of (1 + v): exponent + mantissa fraction of the
    # float 1 + v, the sum rounded to float as one int-to-float conversion
    a = np.float32(1.0) + np.float32(v)
    m, e = np.frexp(np.float64(a))  # a = m 2^e, m in [0.5, 1)
    exact = (e - 1) + (2 * m - 1)  # multiple of 2^-23
    return np.float32(np.float32(exact * 2.0 ** 23) * np.float32(2.0 ** -23))


def test_plog2_closed_forms():
    q = np.zeros((8, 8, 8), np.int32)
    for v, want in [(0, 0.0), (1, 1.0), (2, 1.5), (3, 2.0), (5.25, 2.5625), (7, 3.0), (1023, 10.0)]:
        assert _plog2_1p(v) == want
    f = oracle.features_q(q)
    assert np.all(f == 0)


def test_ramp_x_3d():
    """q = lx in every 8^3 block (features over the two lowest z-planes):
    variance 63/12, range 7, unit first differences along x only, no
    curvature, max |q| 7, mean 3.5."""
    lx = np.arange(16, dtype=np.int32) % 8
    q = np.broadcast_to(lx, (8, 16, 16)).copy()
    f = oracle.features_q(q)
    assert f.shape == (4, F)
    for b in range(4):
        assert f[b, 0] == _plog2_1p(63 / 12) == 2.5625
        assert f[b, 1] == 3.0
        assert f[b, 2] == 1.0 and f[b, 3] == 0 and f[b, 4] == 0
        assert np.all(f[b, 5:11] == 0)
        assert f[b, 14] == _plog2_1p(7) == 3.0
        assert f[b, 15] == _plog2_1p(3.5)


def test_quadratic_y_2d():
    """q = ly^2 (2D, 32x16 blocks; features over the four lowest rows):
    first differences 2 ly - 1 (1, 3, 5) have mean 3 along y, second
    differences are 2, nothing along x."""
    ly = np.arange(16, dtype=np.int64) ** 2
    q = np.broadcast_to(ly[:, None], (16, 32)).astype(np.int32).copy()
    f = oracle.features_q(q)
    assert f.shape == (1, F)
    assert f[0, 2] == 0.0 and f[0, 3] == _plog2_1p(3.0) == 2.0
    assert f[0, 5] == 0.0 and f[0, 6] == _plog2_1p(2.0) == 1.5
    assert f[0, 4] == 0 and f[0, 7] == 0 and np.all(f[0, 8:11] == 0)


def test_mixed_difference_xy():
    """q = lx * ly: the mixed xy difference is 1 everywhere it is defined,
    the yz and xz ones vanish."""
    l = np.arange(8)
    q = np.broadcast_to(l[None, :, None] * l[None, None, :], (8, 8, 8)).astype(np.int32).copy()
    f = oracle.features_q(q)
    assert f[0, 8] == 1.0 and f[0, 9] == 0 and f[0, 10] == 0


def test_constant_block_residual_features():
    """A constant c: only the block's first point has a first-order residual
    (c, zero outside the block); c >= 512 is one outlier in the 128 sampled
    values; max |q| and |mean| are |c|."""
    for c in (3, 700, -900):
        q = np.full((8, 8, 8), c, np.int32)
        f = oracle.features_q(q)[0]
        assert f[0] == 0 and f[1] == 0
        assert f[11] == _plog2_1p(abs(c) / 128)
        assert f[12] == _plog2_1p(abs(c))
        assert f[13] == np.float32((abs(c) >= 512) / 128)
        assert f[14] == _plog2_1p(abs(c)) and f[15] == _plog2_1p(abs(c))


def test_residual_features_match_residual_fields():
    """Residual features of random blocks equal the statistics of the
    oracle's own first-order residual field (pinned elsewhere) over each
    block's sample, its first 128 row-major positions (a lower box), block
    by block, ragged edges included; so do range, max |q| and |mean|."""
    r = np.random.default_rng(5)
    for shape in [(11, 13, 9), (20, 45), (1100,)]:
        q = r.integers(-2000, 2000, size=shape).astype(np.int32)
        f = oracle.features_q(q)
        d0, _ = oracle.residual(q, oracle.P0)
        bs = {1: (512,), 2: (16, 32), 3: (8, 8, 8)}[len(shape)]
        keep = {1: (128,), 2: (4, 32), 3: (2, 8, 8)}[len(shape)]  # numpy axis order
        nb = [-(-s // b) for s, b in zip(shape, bs)]
        k = 0
        for idx in np.ndindex(*nb):
            sl = tuple(slice(i * b, i * b + m) for i, b, m in zip(idx, bs, keep))
            blk = q[sl].astype(np.int64)
            res = np.abs(d0[sl]).astype(np.int64)
            assert f[k, 11] == _plog2_1p(res.sum() / blk.size)
            assert f[k, 12] == _plog2_1p(res.max())
            assert f[k, 13] == np.float32(np.count_nonzero(res >= 512) / blk.size)
            assert f[k, 1] == _plog2_1p(blk.max() - blk.min())
            assert f[k, 14] == _plog2_1p(np.abs(blk).max())
            assert f[k, 15] == _plog2_1p(abs(blk.sum() / blk.size))
            k += 1
        # block order: x fastest (numpy's last axis)
        assert k == f.shape[0]


def test_features_from_field_use_prequantised_values():
    x = (np.arange(8, dtype=np.float32)[None, None, :] * np.ones((8, 8, 1), np.float32)) * 0.02
    f = oracle.features(x, 0.01, 0)  # step 0.02: q = lx
    assert f[0, 0] == 2.5625 and f[0, 2] == 1.0


def _net_permutation():
    """z = f; h1_j = relu(z_j) (j < 16); h2_j = h1_{(j + 1) mod 16}
    (j < 16); y_k = h2 at index (11, 14, 15)[k] - 1 (mod 16)."""
    W1 = np.zeros((64, 16))
    W1[np.arange(16), np.arange(16)] = 1
    W2 = np.zeros((64, 64))
    W2[np.arange(16), (np.arange(16) + 1) % 16] = 1
    W3 = np.zeros((3, 64))
    for k, i in enumerate((11, 14, 15)):
        W3[k, (i - 1) % 16] = 1
    return oracle.pack_params(mu=np.zeros(16), rs=np.ones(16), W1=W1, W2=W2, W3=W3)


def test_mlp_permutation_network():
    r = np.random.default_rng(1)
    feat = r.uniform(0, 10, size=(50, 16)).astype(np.float32)
    y, ch = oracle.mlp_infer(_net_permutation(), feat)
    want = feat[:, [11, 14, 15]]
    assert np.array_equal(y, want)
    # scores: first-order Lorenzo its output, the others output + 1/128
    score = want.astype(np.float32) + np.array([0, 0.0078125, 0.0078125], np.float32)
    assert np.array_equal(ch, np.argmin(score, axis=1))


def test_mlp_bias_only_ties_lowest():
    feat = np.ones((3, 16), np.float32)
    # ties to the lower index; other predictors need to beat first-order
    # Lorenzo by more than the margin of 1/128 (exact in float32)
    for b3, c in [((1, 1, 0), 2), ((0, 0, 1), 0), ((2, 1, 1), 1), ((5, 5, 5), 0), ((1, 0.995, 2), 0),
                  ((1, 0.9921875, 2), 0), ((1, 0.99, 2), 1), ((1, 2, 0.5), 2), ((1, 0.99, 0.985), 2)]:
        y, ch = oracle.mlp_infer(oracle.pack_params(b3=b3), feat)
        assert np.all(ch == c) and np.all(y == np.float32(b3))


def test_mlp_standardisation_and_relu():
    """mu/rs shift and scale; a negative pre-activation is cut by the ReLU."""
    W1 = np.zeros((64, 16))
    W1[0, 3] = 1.0
    W1[1, 3] = -1.0
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    W2[1, 1] = 1.0
    W3 = np.zeros((3, 64))
    W3[0, 0] = 1.0
    W3[1, 1] = 1.0
    mu = np.zeros(16)
    mu[3] = 2.0
    rs = np.ones(16)
    rs[3] = 0.5
    w = oracle.pack_params(mu=mu, rs=rs, W1=W1, W2=W2, W3=W3, b3=(0, 0, 0.25))
    feat = np.zeros((2, 16), np.float32)
    feat[0, 3] = 6.0  # z = 2: y = (2, 0, .25)
    feat[1, 3] = 0.0  # z = -1: y = (0, 1, .25)
    y, ch = oracle.mlp_infer(w, feat)
    assert y.tolist() == [[2.0, 0.0, 0.25], [0.0, 1.0, 0.25]]
    assert ch.tolist() == [1, 0]


def test_mlp_terms_are_fused_multiply_adds():
    """Each term of a dot product is one fused multiply-add: with z = w =
    1 + 2^-12 and bias -1, w z + b = 2^-11 + 2^-24 exactly (representable),
    where a separately rounded product (1 + 2^-11, the tie to even) would
    give 2^-11.  Passed through identity rows of layers 2 and 3."""
    a = 1.0 + 2.0 ** -12
    W1 = np.zeros((64, 16))
    W1[0, 0] = a
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    W3 = np.zeros((3, 64))
    W3[1, 0] = 1.0
    b1 = np.zeros(64)
    b1[0] = -1.0
    w = oracle.pack_params(mu=np.zeros(16), rs=np.ones(16), W1=W1, b1=b1, W2=W2, W3=W3, b3=(0.5, 0, 0.5))
    feat = np.zeros((1, 16), np.float32)
    feat[0, 0] = a
    y, ch = oracle.mlp_infer(w, feat)
    assert y[0, 1] == np.float32(2.0 ** -11 + 2.0 ** -24)
    assert y[0, 0] == 0.5 and y[0, 2] == 0.5 and ch[0] == 1


def _random_net(seed):
    r = np.random.default_rng(seed)
    w = r.normal(0, 0.3, oracle.NPARAM)
    o, n = oracle.OFF["mu"]
    w[o:o + n] = r.uniform(0, 1, n)
    o, n = oracle.OFF["rs"]
    w[o:o + n] = r.uniform(0.5, 2, n)
    return w


def test_loss_closed_form_zero_weights():
    feat = np.random.default_rng(2).uniform(0, 5, (7, 16)).astype(np.float32)
    t = np.random.default_rng(3).uniform(0, 12, (7, 3))
    b3 = np.array([1.0, 2.0, 3.0])
    loss, g = oracle.mlp_loss_grad(oracle.pack_params(b3=b3), feat, t)
    assert loss == pytest.approx(np.mean((b3[None, :] - t) ** 2), rel=1e-14)
    o, n = oracle.OFF["b3"]
    assert np.allclose(g[o:o + n], 2 * (b3[None, :] - t).sum(0) / (3 * 7), rtol=1e-13)


def test_gradient_matches_central_differences():
    """Every learned parameter of a random network: backpropagated
    gradient against central differences of the loss."""
    w = _random_net(7)
    feat = np.random.default_rng(8).uniform(0, 4, (6, 16)).astype(np.float32)
    t = np.random.default_rng(9).uniform(0, 10, (6, 3))
    _, g = oracle.mlp_loss_grad(w, feat, t)
    h = 1e-6
    o1 = oracle.OFF["W1"][0]
    fd = np.zeros(oracle.NPARAM)
    for i in range(o1, oracle.NPARAM):
        wp = w.copy()
        wp[i] += h
        wm = w.copy()
        wm[i] -= h
        fd[i] = (oracle.mlp_loss_grad(wp, feat, t, False)[0] - oracle.mlp_loss_grad(wm, feat, t, False)[0]) / (2 * h)
    assert np.all(g[:o1] == 0)
    err = np.abs(g[o1:] - fd[o1:])
    assert err.max() <= 1e-6 * max(1.0, np.abs(fd).max())
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        o, n = oracle.OFF[name]
        assert np.any(g[o:o + n] != 0), name


def test_adam_first_step_closed_form():
    """First Adam step: bias corrections make m_hat = g and v_hat = g^2, so
    every learned weight moves by -lr g / (|g| + eps); mu and rs stay."""
    w = _random_net(3)
    g = np.random.default_rng(4).normal(0, 1, oracle.NPARAM)
    m = np.zeros(oracle.NPARAM)
    v = np.zeros(oracle.NPARAM)
    w1 = w.copy()
    oracle.adam_step(w1, m, v, g, 1, lr=1e-3)
    o1 = oracle.OFF["W1"][0]
    assert np.array_equal(w1[:o1], w[:o1])
    assert np.allclose(w1[o1:] - w[o1:], -1e-3 * g[o1:] / (np.abs(g[o1:]) + 1e-8), rtol=1e-9, atol=1e-15)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    w2 = w1.copy()
    oracle.adam_step(w2, m, v, g, 2, lr=1e-3)
    assert np.allclose(w2[o1:] - w1[o1:], -1e-3 * g[o1:] / (np.abs(g[o1:]) + 1e-8), rtol=1e-9, atol=1e-15)


def _block3(fn):
    """One 8^3 block with q[lz, ly, lx] = fn(lx, ly, lz)."""
    l = np.arange(8)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    return np.ascontiguousarray(fn(lx, ly, lz).astype(np.int32))


def test_ramp_z_3d():
    """q = lz: the 3D sample is the two lowest z-planes, so the only z pairs
    are (lz = 1, lz = 0), each with difference 1; nothing varies along x or
    y.  A y/z stride mix-up in the oracle would read 0 here."""
    f = oracle.features_q(_block3(lambda x, y, z: z))[0]
    assert f[4] == _plog2_1p(1.0) == 1.0
    assert f[2] == 0 and f[3] == 0
    assert np.all(f[5:11] == 0)
    assert f[0] == _plog2_1p(0.25)  # lz in {0, 1}, 64 values each: variance 1/4
    assert f[14] == _plog2_1p(1) and f[15] == _plog2_1p(0.5)


def test_second_difference_z_is_outside_the_3d_sample():
    """Feature 7 (mean |second difference along z|) needs three z-planes;
    the 3D sample holds two, so it is 0 for every 3D block: a z-quadratic
    (lz^2), a z-cubic and random blocks.  Their first z difference at
    lz = 1 is q(1) - q(0): 1 for lz^2, 1 for lz^3."""
    for fn in (lambda x, y, z: z * z, lambda x, y, z: z ** 3):
        f = oracle.features_q(_block3(fn))[0]
        assert f[7] == 0.0 and f[4] == 1.0
        assert f[2] == 0 and f[3] == 0 and f[5] == 0 and f[6] == 0
    r = np.random.default_rng(9)
    q = r.integers(-500, 500, size=(13, 17, 19)).astype(np.int32)
    assert np.all(oracle.features_q(q)[:, 7] == 0)


def test_mixed_difference_yz():
    """q = ly * lz: the yz mixed difference is 1 wherever ly, lz >= 1; the
    xy and xz ones vanish.  Along z the difference is ly (mean 3.5 over the
    64 pairs at lz = 1); along y it is lz (0 on the lz = 0 plane, 1 on
    lz = 1: mean 1/2 over 112 pairs)."""
    f = oracle.features_q(_block3(lambda x, y, z: y * z))[0]
    assert f[9] == 1.0 and f[8] == 0 and f[10] == 0
    assert f[4] == _plog2_1p(3.5)
    assert f[3] == _plog2_1p(0.5) == 0.5
    assert f[2] == 0 and f[5] == 0 and f[6] == 0 and f[7] == 0


def test_mixed_difference_xz():
    """q = lx * lz: the xz mixed difference is 1 wherever lx, lz >= 1; the
    xy and yz ones vanish; along z the difference is lx (mean 3.5)."""
    f = oracle.features_q(_block3(lambda x, y, z: x * z))[0]
    assert f[10] == 1.0 and f[8] == 0 and f[9] == 0
    assert f[4] == _plog2_1p(3.5)
    assert f[3] == 0 and f[6] == 0 and f[7] == 0


def test_axis_features_follow_the_axis_not_the_stride():
    """The same 1D profile put along x, then y, then z moves its first
    difference feature from index 2 to 3 to 4 (ramps of slope 3, so the
    mean |difference| is 3 and the feature plog2(4) = 2)."""
    for a, fn in enumerate((lambda x, y, z: 3 * x, lambda x, y, z: 3 * y, lambda x, y, z: 3 * z)):
        f = oracle.features_q(_block3(fn))[0]
        want = np.zeros(3, np.float32)
        want[a] = 2.0
        assert np.array_equal(f[2:5], want), (a, f[2:5])
