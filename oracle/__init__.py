"""Python access to the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never does.

Arrays follow numpy C order: a field of shape (nz, ny, nx) has x fastest,
which the oracle calls dims = (nx, ny, nz).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

OK, ERR_ARG, ERR_EB, ERR_NONFINITE, ERR_CAPACITY, ERR_CORRUPT = 0, -1, -2, -3, -4, -5
ERR_NOMEM, ERR_UNSUPPORTED = -7, -8
HDR = 128
NBINS = 1024
RADIUS = 512
LMAX = 12


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        vp = ctypes.c_void_p
        L.orc_eb_abs.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double)]
        L.orc_prequant.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, vp, vp]
        L.orc_prequant.restype = None
        L.orc_lorenzo1.argtypes = [vp, ctypes.c_int, u64p, vp]
        L.orc_lorenzo1.restype = None
        L.orc_lorenzo1_inverse.argtypes = [vp, ctypes.c_int, u64p, vp]
        L.orc_lorenzo1_inverse.restype = None
        L.orc_histogram.argtypes = [vp, ctypes.c_uint64, vp]
        L.orc_histogram.restype = None
        L.orc_codebook_lmax.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
        L.orc_codebook.argtypes = [vp, vp]
        L.orc_canonical.argtypes = [vp, ctypes.c_int, vp]
        L.orc_canonical.restype = None
        L.orc_compress_bound.argtypes = [ctypes.c_int, u64p]
        L.orc_compress_bound.restype = ctypes.c_uint64
        L.orc_compress.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, vp,
                                   ctypes.c_uint64, u64p]
        L.orc_decompress.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_uint64]
        L.orc_stage_codes.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, vp, vp,
                                      vp, ctypes.POINTER(ctypes.c_double)]
        L.orc_residual.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, vp, vp]
        L.orc_residual.restype = None
        L.orc_residual_inverse.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, vp, vp]
        L.orc_residual_inverse.restype = None
        L.orc_compress_ex.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, ctypes.c_int, vp, vp,
                                      ctypes.c_uint64, u64p]
        L.orc_trial.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, vp, vp]
        L.orc_encode_symbols.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_int, vp]
        L.orc_encode_symbols.restype = ctypes.c_uint64
        L.orc_features.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, vp]
        L.orc_features_q.argtypes = [vp, ctypes.c_int, u64p, vp]
        L.orc_mlp_nparam.argtypes = []
        L.orc_mlp_infer.argtypes = [vp, vp, ctypes.c_uint64, vp, vp]
        L.orc_mlp_infer.restype = None
        L.orc_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_uint64, vp]
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double]
        L.orc_adam_step.restype = None
        L.orc_speed_compress.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, vp,
                                         ctypes.c_uint64, u64p]
        L.orc_speed_stage.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, ctypes.c_double, vp, vp]
        L.orc_interp_classes.argtypes = [ctypes.c_int, u64p, vp, vp]
        L.orc_interp_classes.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def dims_of(shape):
    """numpy shape (C order) -> (ndim, dims[3]) with dims[0] fastest."""
    nd = len(shape)
    if nd < 1 or nd > 3:
        raise ValueError("1-3 dimensions")
    d = list(reversed([int(s) for s in shape])) + [1] * (3 - nd)
    return nd, (ctypes.c_uint64 * 3)(*d)


def eb_abs(x, mode, eb):
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = ctypes.c_double()
    rc = lib().orc_eb_abs(_ptr(x), x.size, int(mode), float(eb), ctypes.byref(out))
    if rc:
        raise OracleError(rc)
    return out.value


def prequant(x, eb_abs_value):
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.empty(x.shape, np.int32)
    p = np.empty(x.shape, np.uint8)
    lib().orc_prequant(_ptr(x), x.size, float(eb_abs_value), _ptr(q), _ptr(p))
    return q, p.astype(bool)


def lorenzo1(q):
    q = np.ascontiguousarray(q, dtype=np.int32)
    nd, d = dims_of(q.shape)
    out = np.empty_like(q)
    lib().orc_lorenzo1(_ptr(q), nd, d, _ptr(out))
    return out


def lorenzo1_inverse(delta):
    delta = np.ascontiguousarray(delta, dtype=np.int32)
    nd, d = dims_of(delta.shape)
    out = np.empty_like(delta)
    lib().orc_lorenzo1_inverse(_ptr(delta), nd, d, _ptr(out))
    return out


def histogram(codes):
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    h = np.empty(NBINS, np.uint32)
    lib().orc_histogram(_ptr(codes), codes.size, _ptr(h))
    return h


def codebook(hist, lmax=LMAX):
    hist = np.ascontiguousarray(hist, dtype=np.uint32)
    ln = np.zeros(hist.size, np.uint8)
    rc = lib().orc_codebook_lmax(_ptr(hist), hist.size, int(lmax), _ptr(ln))
    if rc:
        raise OracleError(rc)
    return ln


def canonical(lengths):
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    c = np.zeros(lengths.size, np.uint32)
    lib().orc_canonical(_ptr(lengths), lengths.size, _ptr(c))
    return c


def compress_bound(shape):
    nd, d = dims_of(shape)
    return int(lib().orc_compress_bound(nd, d))


P0, P1, P2, P_SELECTED, P_TRIAL, P_INTERP, P_GLOBAL = 0, 1, 2, 3, 4, 5, 6


def nblocks_of(shape):
    nd = len(shape)
    bs = {1: (512,), 2: (16, 32), 3: (8, 8, 8)}[nd]
    n = 1
    for s, b in zip(shape, bs):
        n *= -(-s // b)
    return n


def compress(x, eb, mode=1, pred=P0, choice=None):
    """Compress a float32 field; returns the container as bytes.  mode 0 =
    absolute, 1 = relative; pred 0/1/2 = that predictor everywhere, 3 = the
    per-block choice given, 4 = per-block choice by exhaustive trial."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, d = dims_of(x.shape)
    cap = compress_bound(x.shape)
    out = np.zeros(max(cap, HDR), np.uint8)
    n = ctypes.c_uint64(0)
    ch = None
    if pred == P_SELECTED:
        ch = np.ascontiguousarray(choice, dtype=np.uint8)
        assert ch.size == nblocks_of(x.shape)
    rc = lib().orc_compress_ex(_ptr(x), nd, d, int(mode), float(eb), int(pred),
                               _ptr(ch) if ch is not None else None, _ptr(out), out.size, ctypes.byref(n))
    if rc:
        raise OracleError(rc)
    return out[: n.value].tobytes()


def residual(q, p):
    """Residual field with predictor p in every block; (delta, coef[nblocks, 4])."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    nd, d = dims_of(q.shape)
    delta = np.empty_like(q)
    coef = np.zeros((nblocks_of(q.shape), 4), np.int32)
    lib().orc_residual(_ptr(q), nd, d, int(p), _ptr(delta), _ptr(coef))
    return delta, coef


def residual_inverse(delta, p, coef=None):
    delta = np.ascontiguousarray(delta, dtype=np.int32)
    nd, d = dims_of(delta.shape)
    q = np.empty_like(delta)
    cf = None if coef is None else np.ascontiguousarray(coef, dtype=np.int32)
    lib().orc_residual_inverse(_ptr(delta), nd, d, int(p), _ptr(cf) if cf is not None else None, _ptr(q))
    return q


def trial(x, eb, mode=1):
    """Per-block exhaustive-trial choice and the three costs (bits) per block."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, d = dims_of(x.shape)
    nb = nblocks_of(x.shape)
    choice = np.zeros(nb, np.uint8)
    costs = np.zeros((nb, 3), np.uint32)
    rc = lib().orc_trial(_ptr(x), nd, d, int(mode), float(eb), _ptr(choice), _ptr(costs))
    if rc:
        raise OracleError(rc)
    return choice, costs


def header(buf):
    """Parse the container header into a dict (fields used by the tests)."""
    b = np.frombuffer(bytes(buf[:HDR]), np.uint8)

    def u(o, n):
        return int.from_bytes(bytes(b[o:o + n]), "little")

    return dict(magic=u(0, 4), version=u(4, 2), flags=u(6, 2), ndim=u(8, 4), pred=u(12, 4),
                dims=(u(16, 8), u(24, 8), u(32, 8)), eb_mode=u(40, 4), radius=u(44, 4),
                eb=np.frombuffer(bytes(b[48:56]), np.float64)[0],
                eb_abs=np.frombuffer(bytes(b[56:64]), np.float64)[0],
                total=u(64, 8), nblocks=u(72, 4), n_outliers=u(76, 4), n_patches=u(80, 4),
                stream_words=u(84, 4), stream_bits=u(88, 8), n_reg=u(96, 4))


def shape_of(h):
    nd = h["ndim"]
    return tuple(reversed(h["dims"][:nd]))


def decompress(buf):
    buf = np.frombuffer(bytes(buf), np.uint8)
    h = header(buf)
    shape = shape_of(h)
    out = np.empty(shape, np.float32)
    rc = lib().orc_decompress(_ptr(buf), buf.size, _ptr(out), out.size)
    if rc:
        raise OracleError(rc)
    return out


def decompress_rc(buf, out_elems=None):
    """Return code only (for corruption tests); never raises."""
    buf = np.frombuffer(bytes(buf), np.uint8)
    n = out_elems if out_elems is not None else (1 << 20)
    out = np.empty(max(n, 1), np.float32)
    return int(lib().orc_decompress(_ptr(buf), buf.size, _ptr(out), out.size))


def stage_codes(x, eb, mode=1):
    """Codes (block-major), their positions, the histogram and eb_abs."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, d = dims_of(x.shape)
    codes = np.empty(x.size, np.uint16)
    pos = np.empty(x.size, np.uint32)
    hist = np.empty(NBINS, np.uint32)
    e = ctypes.c_double()
    rc = lib().orc_stage_codes(_ptr(x), nd, d, int(mode), float(eb), _ptr(codes), _ptr(pos), _ptr(hist),
                               ctypes.byref(e))
    if rc:
        raise OracleError(rc)
    return codes, pos, hist, e.value


def encode_symbols(syms, lengths):
    """Bits of a symbol sequence under the canonical code of ``lengths``: (words u32, nbits)."""
    syms = np.ascontiguousarray(syms, dtype=np.uint16)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    nbits_max = int(sum(int(lengths[s]) for s in syms))
    words = np.zeros(nbits_max // 32 + 2, np.uint32)
    nb = lib().orc_encode_symbols(_ptr(syms), syms.size, _ptr(lengths), lengths.size, _ptr(words))
    return words[: (nb + 31) // 32], int(nb)


# ------------------------------------------------------------ selector
NFEAT, NHID, NOUT = 16, 64, 3
OFF = {}
_o = 0
for _name, _n in (("mu", NFEAT), ("rs", NFEAT), ("W1", NHID * NFEAT), ("b1", NHID), ("W2", NHID * NHID),
                  ("b2", NHID), ("W3", NOUT * NHID), ("b3", NOUT)):
    OFF[_name] = (_o, _n)
    _o += _n
NPARAM = _o


def features(x, eb, mode=1):
    """Block features (nblocks, 16) float32 of a float32 field."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, d = dims_of(x.shape)
    f = np.zeros((nblocks_of(x.shape), NFEAT), np.float32)
    rc = lib().orc_features(_ptr(x), nd, d, int(mode), float(eb), _ptr(f))
    if rc:
        raise OracleError(rc)
    return f


def features_q(q):
    """Block features of a grid-value field q (int32)."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    nd, d = dims_of(q.shape)
    f = np.zeros((nblocks_of(q.shape), NFEAT), np.float32)
    rc = lib().orc_features_q(_ptr(q), nd, d, _ptr(f))
    if rc:
        raise OracleError(rc)
    return f


def pack_params(**parts):
    """Parameter vector from named parts (missing parts are zero)."""
    w = np.zeros(NPARAM, np.float64)
    for k, v in parts.items():
        o, n = OFF[k]
        w[o:o + n] = np.asarray(v, np.float64).reshape(-1)
    return w


def mlp_infer(w, feat):
    """float32 inference: (y (n, 3) float32, choice (n,) uint8)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    assert w.size == NPARAM
    feat = np.ascontiguousarray(feat, dtype=np.float32).reshape(-1, NFEAT)
    n = feat.shape[0]
    y = np.zeros((n, NOUT), np.float32)
    ch = np.zeros(n, np.uint8)
    lib().orc_mlp_infer(_ptr(w), _ptr(feat), n, _ptr(y), _ptr(ch))
    return y, ch


def mlp_loss_grad(w, feat, target, with_grad=True):
    """Double-precision MSE loss and gradient (NPARAM,)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    feat = np.ascontiguousarray(feat, dtype=np.float32).reshape(-1, NFEAT)
    target = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, NOUT)
    g = np.zeros(NPARAM, np.float64) if with_grad else None
    loss = lib().orc_mlp_loss_grad(_ptr(w), _ptr(feat), _ptr(target), feat.shape[0],
                                   _ptr(g) if g is not None else None)
    return loss, g


def adam_step(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adam_step(_ptr(w), _ptr(m), _ptr(v), _ptr(g), int(t), lr, b1, b2, eps)


# ----------------------------------------------------- bit-shuffle codec
FLAG_SHUFFLE = 2
SYM_OUTLIER = 1023


def speed_compress(x, eb, mode=1):
    """Bit-shuffle (FZMod-Speed) container of a float32 field, as bytes."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, d = dims_of(x.shape)
    cap = compress_bound(x.shape)
    out = np.zeros(max(cap, HDR), np.uint8)
    n = ctypes.c_uint64(0)
    rc = lib().orc_speed_compress(_ptr(x), nd, d, int(mode), float(eb), _ptr(out), out.size, ctypes.byref(n))
    if rc:
        raise OracleError(rc)
    return out[: n.value].tobytes()


def speed_stage(x, eb, mode=1):
    """(symbols (nblocks, 512) uint16, shuffled words (nblocks, 16, 10)
    uint32) of a field, as the bit-shuffle codec computes them."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, d = dims_of(x.shape)
    nb = nblocks_of(x.shape)
    sym = np.zeros((nb, 512), np.uint16)
    words = np.zeros((nb, 16, 10), np.uint32)
    rc = lib().orc_speed_stage(_ptr(x), nd, d, int(mode), float(eb), _ptr(sym), _ptr(words))
    if rc:
        raise OracleError(rc)
    return sym, words


def interp_classes(shape):
    """(axis, stride) per point of the interpolation predictor: axis in
    numpy order of dims (0 = x) or -1 for an anchor; stride 8 for anchors."""
    nd, d = dims_of(shape)
    ax = np.zeros(shape, np.int8)
    st = np.zeros(shape, np.uint8)
    lib().orc_interp_classes(nd, d, _ptr(ax), _ptr(st))
    return ax, st
