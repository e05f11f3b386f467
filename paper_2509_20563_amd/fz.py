"""Python binding of libfz (include/fz.h): argument marshalling only.

Every step of compression and decompression runs in the library's HIP
kernels; PyTorch supplies device memory and the current HIP stream.  There is
no fallback: if libfz.so is missing or cannot be loaded, every call raises.

Field tensors are float32, C-contiguous, on a ROCm device, shape
(nz, ny, nx), (ny, nx) or (nx,) - the library's dims[0] is the last axis.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfz.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "fz.h")

EB_ABS, EB_REL = 0, 1
PRED_LORENZO1, PRED_LORENZO2, PRED_REGRESSION, PRED_AUTO_MLP, PRED_AUTO_TRIAL, PRED_INTERP, PRED_GLOBAL = \
    0, 1, 2, 3, 4, 5, 6
HDR_BYTES = 128
NFEAT = 16
SELECTOR_PARAMS = 5475

STATUS = {
    0: "FZ_OK", -1: "FZ_ERR_ARG", -2: "FZ_ERR_EB", -3: "FZ_ERR_NONFINITE", -4: "FZ_ERR_CAPACITY",
    -5: "FZ_ERR_CORRUPT", -6: "FZ_ERR_HIP", -7: "FZ_ERR_NOMEM", -8: "FZ_ERR_UNSUPPORTED", -9: "FZ_ERR_INTERNAL",
    -10: "FZ_ERR_SCRATCH",
}


class FZError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)} ({_strerror(code)})")


class TrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class Params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_uint32), ("dims", ctypes.c_uint64 * 3), ("eb_mode", ctypes.c_uint32),
                ("eb", ctypes.c_double), ("pred", ctypes.c_uint32), ("radius", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    P = ctypes.POINTER(Params)
    L.fz_ctx_create.argtypes = [ctypes.POINTER(vp), i32, u64]
    L.fz_ctx_create.restype = i32
    L.fz_ctx_destroy.argtypes = [vp]
    L.fz_ctx_destroy.restype = None
    L.fz_compress_bound.argtypes = [P]
    L.fz_compress_bound.restype = u64
    L.fz_compress.argtypes = [vp, P, vp, vp, u64, ctypes.POINTER(u64), vp]
    L.fz_compress.restype = i32
    L.fz_header_read.argtypes = [vp, u64, P, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.fz_header_read.restype = i32
    L.fz_decompress.argtypes = [vp, vp, u64, vp, vp, u64, vp]
    L.fz_decompress.restype = i32
    L.fz_strerror.argtypes = [i32]
    L.fz_strerror.restype = ctypes.c_char_p
    L.fz_set_timing.argtypes = [vp, i32]
    L.fz_set_timing.restype = i32
    L.fz_set_timing_stage.argtypes = [vp, ctypes.c_char_p]
    L.fz_set_timing_stage.restype = i32
    L.fz_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)]
    L.fz_stage_times.restype = i32
    L.fz_stage_name.argtypes = [vp, i32]
    L.fz_stage_name.restype = ctypes.c_char_p
    L.fz_last_histogram.argtypes = [vp, vp]
    L.fz_last_histogram.restype = i32
    L.fz_block_count.argtypes = [P]
    L.fz_block_count.restype = u64
    L.fz_block_features.argtypes = [vp, P, vp, vp, u64, vp]
    L.fz_block_features.restype = i32
    L.fz_block_select.argtypes = [vp, P, vp, vp, vp, vp]
    L.fz_block_select.restype = i32
    L.fz_block_trial.argtypes = [vp, P, vp, vp, vp, vp]
    L.fz_block_trial.restype = i32
    L.fz_selector_set.argtypes = [vp, vp, u64]
    L.fz_selector_set.restype = i32
    L.fz_selector_get.argtypes = [vp, vp, u64]
    L.fz_selector_get.restype = i32
    L.fz_selector_save.argtypes = [vp, ctypes.c_char_p]
    L.fz_selector_save.restype = i32
    L.fz_selector_load.argtypes = [vp, ctypes.c_char_p]
    L.fz_selector_load.restype = i32
    PP = ctypes.POINTER(Params)
    L.fz_compress_batch_bound.argtypes = [ctypes.c_uint32, PP]
    L.fz_compress_batch_bound.restype = u64
    L.fz_compress_batch.argtypes = [vp, ctypes.c_uint32, PP, vp, vp, u64, vp, vp]
    L.fz_compress_batch.restype = i32
    L.fz_decompress_batch.argtypes = [vp, ctypes.c_uint32, vp, vp, vp, vp, vp]
    L.fz_decompress_batch.restype = i32
    L.fz_batch_autotune.argtypes = [vp, ctypes.c_uint32, PP, vp, vp, u64, vp]
    L.fz_batch_autotune.restype = i32
    L.fz_batch_tuning.argtypes = [vp, ctypes.c_uint32, PP, vp, vp]
    L.fz_batch_tuning.restype = i32
    L.fz_selector_train.argtypes = [vp, vp, vp, u64, ctypes.POINTER(TrainParams), vp, vp]
    L.fz_selector_train.restype = i32
    L.fz_selector_grad.argtypes = [vp, vp, vp, u64, vp, vp, vp]
    L.fz_selector_grad.restype = i32
    L.fz_selector_adam_step.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, vp]
    L.fz_selector_adam_step.restype = i32
    L.fz_set_graph_mode.argtypes = [vp, i32]
    L.fz_set_graph_mode.restype = i32
    L.fz_graph_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(i32)]
    L.fz_graph_info.restype = i32
    L.fz_compress_speed.argtypes = [vp, P, vp, vp, u64, ctypes.POINTER(u64), vp]
    L.fz_compress_speed.restype = i32
    L.fz_decompress_noalloc.argtypes = [vp, u64, vp, vp, u64, vp]
    L.fz_decompress_noalloc.restype = i32
    L.fz_noalloc_scratch_bytes.argtypes = []
    L.fz_noalloc_scratch_bytes.restype = u64
    _lib = L
    return L


def declared_functions() -> list[str]:
    """Names of the functions include/fz.h declares."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fz_[a-z_0-9]+)\s*\(", text)))


def _strerror(code: int) -> str:
    try:
        return lib().fz_strerror(code).decode()
    except Exception:
        return "?"


def _check(rc: int, what: str):
    if rc != 0:
        raise FZError(rc, what)


def params_for(shape, eb: float, mode: int = EB_REL, pred: int = PRED_LORENZO1) -> Params:
    nd = len(shape)
    if nd < 1 or nd > 3:
        raise ValueError("fields have 1 to 3 dimensions")
    dims = list(reversed([int(s) for s in shape])) + [1] * (3 - nd)
    return Params(nd, (ctypes.c_uint64 * 3)(*dims), int(mode), float(eb), int(pred), 512)


def header_fields(hdr: bytes) -> dict:
    """Counts recorded in a container header (little-endian fields of the
    128-byte header described in include/fz.h)."""
    b = bytes(hdr[:HDR_BYTES])

    def u(o, n):
        return int.from_bytes(b[o:o + n], "little")

    return dict(flags=u(6, 2), ndim=u(8, 4), dims=(u(16, 8), u(24, 8), u(32, 8)), eb_mode=u(40, 4),
                eb=ctypes.c_double.from_buffer_copy(b[48:56]).value,
                eb_abs=ctypes.c_double.from_buffer_copy(b[56:64]).value, total=u(64, 8),
                nblocks=u(72, 4), n_outliers=u(76, 4), n_patches=u(80, 4), stream_words=u(84, 4),
                stream_bits=u(88, 8), pred=u(12, 4), n_reg=u(96, 4))


def shape_of(p: Params):
    return tuple(reversed([int(p.dims[a]) for a in range(p.ndim)]))


def _stream_handle(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """An fz context bound to one device; owns the library's scratch memory."""

    def __init__(self, device: int | torch.device = 0, max_elems: int = 0):
        if isinstance(device, torch.device):
            device = device.index or 0
        self.device = torch.device("cuda", int(device))
        h = ctypes.c_void_p()
        _check(lib().fz_ctx_create(ctypes.byref(h), int(device), int(max_elems)), "fz_ctx_create")
        # marshalled arguments reused across calls (small caches)
        self._pcache: dict = {}
        self._hcache: dict = {}
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().fz_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ---------------------------------------------------------------- compress
    def compress_bound(self, shape) -> int:
        return int(lib().fz_compress_bound(ctypes.byref(params_for(shape, 1.0))))

    def compress(self, x: torch.Tensor, eb: float, mode: int = EB_REL, out: torch.Tensor | None = None,
                 pred: int = PRED_LORENZO1, codec: str = "huffman") -> torch.Tensor:
        """Compress a float32 device field; returns a uint8 device tensor (view
        of `out`).  codec "huffman" (fz_compress) or "shuffle" (the
        bit-shuffle codec, fz_compress_speed)."""
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 device tensor")
        key = (tuple(x.shape), float(eb), int(mode), int(pred))
        p = self._pcache.get(key)
        if p is None:
            if len(self._pcache) > 256:
                self._pcache.clear()
            p = self._pcache[key] = params_for(x.shape, eb, mode, pred)
        if out is None:
            cap = self.compress_bound(x.shape)
            if cap == 0:
                raise FZError(-1, "fz_compress_bound")
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        n = ctypes.c_uint64(0)
        if codec == "huffman":
            fn, name = lib().fz_compress, "fz_compress"
        elif codec == "shuffle":
            fn, name = lib().fz_compress_speed, "fz_compress_speed"
        else:
            raise ValueError("codec is 'huffman' or 'shuffle'")
        rc = fn(self._h, ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                out.numel(), ctypes.byref(n), _stream_handle(x.device))
        _check(rc, name)
        return out[: n.value]

    # -------------------------------------------------------------- decompress
    @staticmethod
    def read_header(hdr: bytes):
        """(params, n_elems, total_bytes) from a host copy of the header."""
        buf = (ctypes.c_uint8 * HDR_BYTES).from_buffer_copy(bytes(hdr[:HDR_BYTES]).ljust(HDR_BYTES, b"\0"))
        p = Params()
        n = ctypes.c_uint64()
        tot = ctypes.c_uint64()
        _check(lib().fz_header_read(buf, len(hdr), ctypes.byref(p), ctypes.byref(n), ctypes.byref(tot)),
               "fz_header_read")
        return p, n.value, tot.value

    def decompress(self, buf: torch.Tensor, header: bytes | None = None, out: torch.Tensor | None = None):
        """Decompress a uint8 device container; returns a float32 device field."""
        if buf.dtype != torch.uint8 or not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("buf must be a contiguous uint8 device tensor")
        if header is None:
            header = buf[:HDR_BYTES].cpu().numpy().tobytes()
        hb = bytes(header[:HDR_BYTES])
        cached = self._hcache.get(hb)
        if cached is None:
            if len(self._hcache) > 256:
                self._hcache.clear()
            p, n, _ = self.read_header(hb)
            cached = self._hcache[hb] = (p, n, (ctypes.c_uint8 * HDR_BYTES).from_buffer_copy(hb))
        p, n, h = cached
        if out is None:
            out = torch.empty(shape_of(p), dtype=torch.float32, device=buf.device)
        rc = lib().fz_decompress(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel(), h,
                                 ctypes.c_void_p(out.data_ptr()), out.numel(), _stream_handle(buf.device))
        _check(rc, "fz_decompress")
        return out

    # ------------------------------------------------------------ graph mode
    def set_graph_mode(self, streams: int | bool = True):
        """Graph mode with at most `streams` streams (True = 4, False/0 = eager calls)."""
        n = (4 if streams else 0) if isinstance(streams, bool) else int(streams)
        _check(lib().fz_set_graph_mode(self._h, n), "fz_set_graph_mode")

    def graph_info(self, which: int):
        """(tasks, streams, width, edges) of the last captured graph of a kind
        (0 = compression, 1 = decompression)."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().fz_graph_info(self._h, int(which), *[ctypes.byref(x) for x in v]), "fz_graph_info")
        return tuple(x.value for x in v)

    # ------------------------------------------------------------ diagnostics
    def set_timing(self, on: bool = True):
        _check(lib().fz_set_timing(self._h, 1 if on else 0), "fz_set_timing")

    def set_timing_stage(self, stage: str | None):
        """Time only the named stage (None: every stage)."""
        _check(lib().fz_set_timing_stage(self._h, None if stage is None else stage.encode()), "fz_set_timing_stage")

    def stage_times(self) -> list[tuple[str, float]]:
        ms = (ctypes.c_float * 16)()
        n = ctypes.c_int()
        _check(lib().fz_stage_times(self._h, ms, 16, ctypes.byref(n)), "fz_stage_times")
        return [(lib().fz_stage_name(self._h, i).decode(), float(ms[i])) for i in range(min(n.value, 16))]

    # -------------------------------------------------------------- batches
    @staticmethod
    def _batch_params(xs, ebs, modes, preds):
        n = len(xs)
        P = (Params * n)()
        for i, x in enumerate(xs):
            if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
                raise ValueError("fields must be contiguous float32 device tensors")
            P[i] = params_for(x.shape, ebs[i], modes[i], preds[i])
        return P

    def compress_batch_bound(self, shapes, preds=None) -> int:
        n = len(shapes)
        P = (Params * n)()
        for i, sh in enumerate(shapes):
            P[i] = params_for(sh, 1.0, EB_REL, 0 if preds is None else preds[i])
        return int(lib().fz_compress_batch_bound(n, P))

    def compress_batch(self, xs, ebs, modes=None, preds=None, out: torch.Tensor | None = None):
        """Compress a list of fields in one call: (packed uint8 device tensor, offsets list)."""
        n = len(xs)
        modes = [EB_REL] * n if modes is None else list(modes)
        preds = [PRED_LORENZO1] * n if preds is None else list(preds)
        P = self._batch_params(xs, list(ebs), modes, preds)
        cap = int(lib().fz_compress_batch_bound(n, P))
        if cap == 0:
            raise FZError(-1, "fz_compress_batch_bound")
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=xs[0].device)
        ptrs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        offs = (ctypes.c_uint64 * (n + 1))()
        _check(lib().fz_compress_batch(self._h, n, P, ptrs, ctypes.c_void_p(out.data_ptr()), out.numel(), offs,
                                       _stream_handle(xs[0].device)), "fz_compress_batch")
        return out[: offs[n]], list(offs)

    def decompress_batch(self, buf: torch.Tensor, offsets, outs):
        """Decompress a packed batch into the given float32 device tensors."""
        n = len(outs)
        offs = (ctypes.c_uint64 * (n + 1))(*[int(o) for o in offsets])
        ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        ne = (ctypes.c_uint64 * n)(*[o.numel() for o in outs])
        _check(lib().fz_decompress_batch(self._h, n, ctypes.c_void_p(buf.data_ptr()), offs, ptrs, ne,
                                         _stream_handle(buf.device)), "fz_decompress_batch")
        return outs

    def batch_autotune(self, xs, ebs, modes=None, preds=None):
        n = len(xs)
        modes = [EB_REL] * n if modes is None else list(modes)
        preds = [PRED_LORENZO1] * n if preds is None else list(preds)
        P = self._batch_params(xs, list(ebs), modes, preds)
        cap = int(lib().fz_compress_batch_bound(n, P))
        out = torch.empty(cap, dtype=torch.uint8, device=xs[0].device)
        ptrs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        _check(lib().fz_batch_autotune(self._h, n, P, ptrs, ctypes.c_void_p(out.data_ptr()), cap,
                                       _stream_handle(xs[0].device)), "fz_batch_autotune")
        return self.batch_tuning(xs, ebs, modes, preds)

    def batch_tuning(self, xs, ebs, modes=None, preds=None):
        """(chains, workgroups per CU of each field) the batch would run with."""
        n = len(xs)
        modes = [EB_REL] * n if modes is None else list(modes)
        preds = [PRED_LORENZO1] * n if preds is None else list(preds)
        P = self._batch_params(xs, list(ebs), modes, preds)
        k = ctypes.c_uint32()
        w = (ctypes.c_uint32 * n)()
        _check(lib().fz_batch_tuning(self._h, n, P, ctypes.byref(k), w), "fz_batch_tuning")
        return k.value, list(w)

    # ------------------------------------------------- per-block predictors
    def block_count(self, shape) -> int:
        return int(lib().fz_block_count(ctypes.byref(params_for(shape, 1.0))))

    def _field_args(self, x, eb, mode):
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 device tensor")
        return params_for(x.shape, eb, mode), self.block_count(x.shape)

    def block_features(self, x: torch.Tensor, eb: float, mode: int = EB_REL) -> torch.Tensor:
        """(nblocks, 16) float32 device tensor of block features."""
        p, nb = self._field_args(x, eb, mode)
        f = torch.empty((nb, NFEAT), dtype=torch.float32, device=x.device)
        _check(lib().fz_block_features(self._h, ctypes.byref(p), ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(f.data_ptr()), f.numel(), _stream_handle(x.device)),
               "fz_block_features")
        return f

    def block_select(self, x: torch.Tensor, eb: float, mode: int = EB_REL):
        """(choice uint8 (nblocks,), predictions float32 (nblocks, 3)) by the selector."""
        p, nb = self._field_args(x, eb, mode)
        ch = torch.empty(nb, dtype=torch.uint8, device=x.device)
        y = torch.empty((nb, 3), dtype=torch.float32, device=x.device)
        _check(lib().fz_block_select(self._h, ctypes.byref(p), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(ch.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     _stream_handle(x.device)), "fz_block_select")
        return ch, y

    def block_trial(self, x: torch.Tensor, eb: float, mode: int = EB_REL):
        """(choice uint8 (nblocks,), costs int32 (nblocks, 3) in bits) by exhaustive trial."""
        p, nb = self._field_args(x, eb, mode)
        ch = torch.empty(nb, dtype=torch.uint8, device=x.device)
        costs = torch.empty((nb, 3), dtype=torch.int32, device=x.device)
        _check(lib().fz_block_trial(self._h, ctypes.byref(p), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(ch.data_ptr()), ctypes.c_void_p(costs.data_ptr()),
                                    _stream_handle(x.device)), "fz_block_trial")
        return ch, costs

    def selector_set(self, params):
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().fz_selector_set(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size), "fz_selector_set")

    def selector_get(self):
        import numpy as np
        a = np.zeros(SELECTOR_PARAMS, np.float32)
        _check(lib().fz_selector_get(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size), "fz_selector_get")
        return a

    def selector_train(self, feat: torch.Tensor, costs: torch.Tensor, epochs: int = 10, batch: int = 4096,
                       lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                       seed: int = 0):
        """Train the selector on device features (n, 16) and trial costs (n, 3); returns the
        mean minibatch loss of every epoch."""
        import numpy as np
        if feat.dtype != torch.float32 or not feat.is_cuda or not feat.is_contiguous() or feat.shape[-1] != NFEAT:
            raise ValueError("feat must be a contiguous (n, 16) float32 device tensor")
        if costs.dtype not in (torch.int32,) or not costs.is_cuda or not costs.is_contiguous():
            raise ValueError("costs must be a contiguous (n, 3) int32 device tensor")
        n = feat.shape[0]
        if costs.shape != (n, 3):
            raise ValueError("costs must be (n, 3)")
        tp = TrainParams(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed))
        loss = np.zeros(int(epochs), np.float32)
        _check(lib().fz_selector_train(self._h, ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(costs.data_ptr()),
                                       n, ctypes.byref(tp), loss.ctypes.data_as(ctypes.c_void_p),
                                       _stream_handle(feat.device)), "fz_selector_train")
        return loss

    def selector_grad(self, feat: torch.Tensor, target: torch.Tensor):
        """(gradient (5475,) float32, loss) of the current selector's MSE on device samples."""
        import numpy as np
        if feat.dtype != torch.float32 or target.dtype != torch.float32:
            raise ValueError("float32 tensors")
        feat = feat.contiguous()
        target = target.contiguous()
        g = np.zeros(SELECTOR_PARAMS, np.float32)
        loss = ctypes.c_float()
        _check(lib().fz_selector_grad(self._h, ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                      feat.shape[0], g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss),
                                      _stream_handle(feat.device)), "fz_selector_grad")
        return g, loss.value

    def selector_adam_step(self, w, m, v, g, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step of the training kernel on copies of host float32
        arrays (5475,): returns the new (w, m, v)."""
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float32).copy() for a in (w, m, v, g)]
        if any(a.shape != (SELECTOR_PARAMS,) for a in arrs):
            raise ValueError(f"arrays of {SELECTOR_PARAMS} floats")
        ptr = [a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
        _check(lib().fz_selector_adam_step(self._h, *ptr, int(t), lr, beta1, beta2, eps,
                                           _stream_handle(self.device)), "fz_selector_adam_step")
        return arrs[0], arrs[1], arrs[2]

    def selector_save(self, path: str):
        _check(lib().fz_selector_save(self._h, os.fsencode(path)), "fz_selector_save")

    def selector_load(self, path: str):
        _check(lib().fz_selector_load(self._h, os.fsencode(path)), "fz_selector_load")

    def last_histogram(self):
        import numpy as np
        h = np.zeros(1024, np.uint32)
        _check(lib().fz_last_histogram(self._h, h.ctypes.data_as(ctypes.c_void_p)), "fz_last_histogram")
        return h


_default: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def compress(x: torch.Tensor, eb: float, mode: int = EB_REL) -> torch.Tensor:
    return context(x.device.index or 0).compress(x, eb, mode)


def decompress(buf: torch.Tensor, header: bytes | None = None) -> torch.Tensor:
    return context(buf.device.index or 0).decompress(buf, header)


def decompress_noalloc(buf: torch.Tensor, out: torch.Tensor, header: bytes | None = None) -> torch.Tensor:
    """fz_decompress_noalloc: decompress a first-order Lorenzo (or verbatim)
    container into the caller's float32 device tensor `out`, with no device
    allocation (the library's static per-GPU scratch)."""
    if buf.dtype != torch.uint8 or not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous uint8 device tensor")
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 device tensor")
    h = None
    if header is not None:
        h = (ctypes.c_uint8 * HDR_BYTES).from_buffer_copy(bytes(header[:HDR_BYTES]))
    with torch.cuda.device(buf.device):
        rc = lib().fz_decompress_noalloc(ctypes.c_void_p(buf.data_ptr()), buf.numel(), h,
                                         ctypes.c_void_p(out.data_ptr()), out.numel(), _stream_handle(buf.device))
    _check(rc, "fz_decompress_noalloc")
    return out


def noalloc_scratch_bytes() -> int:
    return int(lib().fz_noalloc_scratch_bytes())
