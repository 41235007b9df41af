"""ctypes binding of libfc.so: argument marshalling only.

Every step of the FC chain runs in the library's HIP kernels; this module
checks tensor shapes/dtypes/devices, passes raw pointers and the current HIP
stream, and converts status codes into exceptions. It raises if the library
is not built: there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfc.so")

CONT_OLA, CONT_OLS, SYNC_OLA, SYNC_OLS = 0, 1, 2, 3
MODES = {"cont_ola": CONT_OLA, "cont_ols": CONT_OLS, "sync_ola": SYNC_OLA, "sync_ols": SYNC_OLS}
IO_C64, IO_F16, IO_BF16 = 0, 1, 2
IOS = {"c64": IO_C64, "f16": IO_F16, "bf16": IO_BF16}
OP_TX, OP_RX, OP_ADJ, OP_RXD, OP_TXG = 0, 1, 2, 3, 4

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_F32P = ctypes.POINTER(ctypes.c_float)


class FcSubband(ctypes.Structure):
    _fields_ = [("scs_khz", _I32), ("first_symbol", _I32), ("n_symbols", _I32), ("n_active", _I32),
                ("n_tb", _I32), ("n_short", _I32), ("n_long", _I32), ("center_bin", _I32),
                ("overlap_num", _I32), ("overlap_den", _I32), ("mode", _I32), ("stream", _I32),
                ("ncp_high", _I32P), ("taper", _I32)]


EXPORTS = {
    "fc_plan_create": (_I32, [ctypes.POINTER(FcSubband), _I32, _I32, _I32, ctypes.POINTER(_P)]),
    "fc_plan_destroy": (None, [_P]),
    "fc_plan_counts": (_I32, [_P, _I32P, _I32P]),
    "fc_plan_layout": (_I32, [_P, _I32, _I64P, _I64P]),
    "fc_plan_symbols": (_I32, [_P, _I32, _I32P, _I32P, _I64P]),
    "fc_plan_stats": (_I32, [_P, _I32, _I64P, _I64P, _I64P]),
    "fc_set_weights": (_I32, [_P, _I32, _F32P, _I32, _P]),
    "fc_set_weights_device": (_I32, [_P, _I32, _P, _I32, _P]),
    "fc_get_weights": (_I32, [_P, _I32, _F32P, _I32]),
    "fc_tx_synthesize": (_I32, [_P, _P, _P, _P]),
    "fc_rx_analyze": (_I32, [_P, _P, _P, _P]),
    "fc_tx_adjoint": (_I32, [_P, _P, _P, _P]),
    "fc_rx_demodulate": (_I32, [_P, _P, _P, _P]),
    "fc_tx_modulate": (_I32, [_P, _P, _P, _P]),
    "fc_tx_weight_grad": (_I32, [_P, _P, _P, _P, _P]),
    "fc_tx_weight_grad_noalloc": (_I32, [_P, _P, _P, _P, _P]),
    "fc_plan_set_tuning": (_I32, [_P, _I32, _I32, _I32]),
    "fc_plan_get_tuning": (_I32, [_P, _I32, _I32P, _I32P]),
    "fc_plan_set_transform_plan": (_I32, [_P, _I32, _I32]),
    "fc_plan_get_transform_plan": (_I32, [_P, _I32, _I32P]),
    "fc_plan_get_class_plans": (_I32, [_P, _I32, _I32P, _I32P]),
    "fc_plan_autotune": (_I32, [_P, _I32, _P, _P, _P, _I32P, _I32P, ctypes.POINTER(ctypes.c_float)]),
    "fc_graph_begin": (_I32, [_P]),
    "fc_graph_end": (_I32, [_P, ctypes.POINTER(_P)]),
    "fc_graph_launch": (_I32, [_P, _P]),
    "fc_graph_destroy": (None, [_P]),
    "fc_status_str": (ctypes.c_char_p, [_I32]),
    "fc_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libfc.so (built in-tree by paper_2008_00672_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfc.so is not built (run paper_2008_00672_amd.build or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FcError(RuntimeError):
    def __init__(self, status, what):
        msg = lib().fc_status_str(status).decode()
        super().__init__("%s failed: %s (%d)" % (what, msg, status))
        self.status = status


def _check(status, what):
    if status != 0:
        raise FcError(status, what)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A plan over a list of subband dicts (see fcsynth.workloads.subband)."""

    def __init__(self, subbands, io="c64", device=0):
        self.subbands = [dict(s) for s in subbands]
        self.io = io
        self.device = device
        arr = (FcSubband * len(subbands))()
        self._cp_keep = []
        for i, s in enumerate(subbands):
            num, den = s.get("overlap", (1, 2))
            cp = s.get("ncp_high")
            cp_ptr = None
            if cp is not None:
                buf = (ctypes.c_int32 * len(cp))(*cp)
                self._cp_keep.append(buf)
                cp_ptr = ctypes.cast(buf, _I32P)
            arr[i] = FcSubband(s["scs_khz"], s.get("first_symbol", 0), s["n_symbols"], s["n_active"],
                               s["n_tb"], s["n_short"], s["n_long"], s["center_bin"], num, den,
                               MODES[s["mode"]] if isinstance(s["mode"], str) else s["mode"],
                               s.get("stream", 0), cp_ptr, s.get("taper", 0))
        h = ctypes.c_void_p()
        _check(lib().fc_plan_create(arr, len(subbands), IOS[io], device, ctypes.byref(h)), "fc_plan_create")
        self._h = h
        nsb, nst = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fc_plan_counts(h, ctypes.byref(nsb), ctypes.byref(nst)), "fc_plan_counts")
        self.n_sb, self.n_streams = nsb.value, nst.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.fc_plan_destroy(h)
            self._h = None

    # ---------------------------------------------------------- queries --
    def layout(self, op=OP_TX):
        cache = self.__dict__.setdefault("_layouts", {})
        if op in cache:
            return cache[op]
        cache[op] = self._layout(op)
        return cache[op]

    def _layout(self, op):
        lo = (ctypes.c_int64 * (self.n_sb + 1))()
        hi = (ctypes.c_int64 * (self.n_streams + 1))()
        _check(lib().fc_plan_layout(self._h, op, lo, hi), "fc_plan_layout")
        return np.array(lo[:], dtype=np.int64), np.array(hi[:], dtype=np.int64)

    def symbols(self, sb):
        n = self.subbands[sb]["n_symbols"]
        a, b = (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)()
        off = ctypes.c_int64()
        _check(lib().fc_plan_symbols(self._h, sb, a, b, ctypes.byref(off)), "fc_plan_symbols")
        return list(a), list(b), off.value

    def stats(self, op=OP_TX):
        nb, nt, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fc_plan_stats(self._h, op, ctypes.byref(nb), ctypes.byref(nt), ctypes.byref(nl)),
               "fc_plan_stats")
        return dict(blocks=nb.value, tasks=nt.value, launches=nl.value)

    # ---------------------------------------------------------- weights --
    def set_weights(self, sb, w, stream=None):
        """w: host array-like (copied) or a float32 CUDA tensor (device copy)."""
        L = self.subbands[sb]["n_short"]
        try:
            import torch
            is_dev = isinstance(w, torch.Tensor) and w.is_cuda
        except ImportError:  # pragma: no cover
            is_dev = False
        if is_dev:
            if w.dtype != torch.float32 or w.numel() != L or not w.is_contiguous():
                raise ValueError("weights must be a contiguous float32 tensor of n_short values")
            # the library does not read device weights on the host: the
            # finiteness check that fc_set_weights makes is made here
            if not bool(torch.isfinite(w).all()):
                raise ValueError("weights must be finite")
            _check(lib().fc_set_weights_device(self._h, sb, _ptr(w), L, _stream_handle(stream)),
                   "fc_set_weights_device")
            return
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32).ravel())
        if a.size != L:
            raise ValueError("need %d weights" % L)
        st = None if self.device < 0 else _stream_handle(stream)
        _check(lib().fc_set_weights(self._h, sb, a.ctypes.data_as(_F32P), L, st), "fc_set_weights")

    def set_all_weights(self, w, stream=None):
        """Every subband's weights at once from a float32 CUDA tensor holding
        them concatenated in plan order (one device copy; checked finite)."""
        import torch
        total = sum(s["n_short"] for s in self.subbands)
        if not (isinstance(w, torch.Tensor) and w.is_cuda):
            raise ValueError("set_all_weights takes a CUDA tensor")
        if w.dtype != torch.float32 or w.numel() != total or not w.is_contiguous():
            raise ValueError("weights must be a contiguous float32 tensor of %d values" % total)
        if not bool(torch.isfinite(w).all()):
            raise ValueError("weights must be finite")
        _check(lib().fc_set_weights_device(self._h, -1, _ptr(w), total, _stream_handle(stream)),
               "fc_set_weights_device")

    def get_weights(self, sb):
        L = self.subbands[sb]["n_short"]
        a = np.zeros(L, dtype=np.float32)
        _check(lib().fc_get_weights(self._h, sb, a.ctypes.data_as(_F32P), L), "fc_get_weights")
        return a

    # ------------------------------------------------------------- I/O --
    def _dtype(self):
        import torch
        return {"c64": torch.complex64, "f16": torch.float16, "bf16": torch.bfloat16}[self.io]

    def empty(self, n):
        """Device tensor for n complex samples in this plan's I/O type."""
        import torch
        dev = torch.device("cuda", self.device)
        if self.io == "c64":
            return torch.empty(n, dtype=torch.complex64, device=dev)
        return torch.empty((n, 2), dtype=self._dtype(), device=dev)

    def _check_buf(self, t, n, what):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % what)
        if t.device.index != self.device:
            raise ValueError("%s is on the wrong device" % what)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % what)
        if self.io == "c64":
            ok = t.dtype == torch.complex64 and t.numel() == n
        else:
            ok = t.dtype == self._dtype() and t.numel() == 2 * n
        if not ok:
            raise ValueError("%s must hold %d samples of I/O type %s" % (what, n, self.io))

    def tx(self, x, out=None, stream=None):
        lo, hi = self.layout(OP_TX)
        self._check_buf(x, int(lo[-1]), "low-rate input")
        if out is None:
            out = self.empty(int(hi[-1]))
        self._check_buf(out, int(hi[-1]), "high-rate output")
        _check(lib().fc_tx_synthesize(self._h, _ptr(x), _ptr(out), _stream_handle(stream)), "fc_tx_synthesize")
        return out

    def rx(self, y, out=None, stream=None):
        lo, hi = self.layout(OP_RX)
        self._check_buf(y, int(hi[-1]), "high-rate input")
        if out is None:
            out = self.empty(int(lo[-1]))
        self._check_buf(out, int(lo[-1]), "low-rate output")
        _check(lib().fc_rx_analyze(self._h, _ptr(y), _ptr(out), _stream_handle(stream)), "fc_rx_analyze")
        return out

    def tx_grid(self, grid, out=None, stream=None):
        """CP-OFDM modulation + synchronised FC TX of QAM grids (per subband
        n_symbols x n_active values, concatenated in plan order)."""
        lo, hi = self.layout(OP_TXG)
        self._check_buf(grid, int(lo[-1]), "QAM grid")
        if out is None:
            out = self.empty(int(hi[-1]))
        self._check_buf(out, int(hi[-1]), "high-rate output")
        _check(lib().fc_tx_modulate(self._h, _ptr(grid), _ptr(out), _stream_handle(stream)), "fc_tx_modulate")
        return out

    def rx_demod(self, y, out=None, stream=None):
        """Synchronised RX + OFDM demodulation: subcarrier values per symbol."""
        lo, hi = self.layout(OP_RXD)
        self._check_buf(y, int(hi[-1]), "high-rate input")
        if out is None:
            out = self.empty(int(lo[-1]))
        self._check_buf(out, int(lo[-1]), "subcarrier output")
        _check(lib().fc_rx_demodulate(self._h, _ptr(y), _ptr(out), _stream_handle(stream)), "fc_rx_demodulate")
        return out

    def adjoint(self, y, out=None, stream=None):
        lo, hi = self.layout(OP_ADJ)
        self._check_buf(y, int(hi[-1]), "high-rate input")
        if out is None:
            out = self.empty(int(lo[-1]))
        self._check_buf(out, int(lo[-1]), "low-rate output")
        _check(lib().fc_tx_adjoint(self._h, _ptr(y), _ptr(out), _stream_handle(stream)), "fc_tx_adjoint")
        return out

    def weight_grad(self, x, g, out=None, stream=None):
        import torch
        lo, hi = self.layout(OP_TX)
        self._check_buf(x, int(lo[-1]), "low-rate input")
        self._check_buf(g, int(hi[-1]), "high-rate gradient")
        total = sum(s["n_short"] for s in self.subbands)
        if out is None:
            out = torch.empty(total, dtype=torch.float32, device=x.device)
        if (not out.is_cuda or out.device.index != self.device or out.dtype != torch.float32
                or out.numel() != total or not out.is_contiguous()):
            raise ValueError("grad_w must be a contiguous float32 tensor of sum(n_short) values on the plan's device")
        _check(lib().fc_tx_weight_grad(self._h, _ptr(x), _ptr(g), _ptr(out), _stream_handle(stream)),
               "fc_tx_weight_grad")
        return out

    def weight_grad_noalloc(self, x, g, out, stream=None):
        """fc_tx_weight_grad_noalloc: the weight gradient into the caller's
        `out` with the library's fixed device scratch (no allocation, also
        none here: `out` is required)."""
        import torch
        lo, hi = self.layout(OP_TX)
        self._check_buf(x, int(lo[-1]), "low-rate input")
        self._check_buf(g, int(hi[-1]), "high-rate gradient")
        total = sum(s["n_short"] for s in self.subbands)
        if (out is None or not out.is_cuda or out.device.index != self.device or out.dtype != torch.float32
                or out.numel() != total or not out.is_contiguous()):
            raise ValueError("grad_w must be a contiguous float32 tensor of sum(n_short) values on the plan's device")
        _check(lib().fc_tx_weight_grad_noalloc(self._h, _ptr(x), _ptr(g), _ptr(out), _stream_handle(stream)),
               "fc_tx_weight_grad_noalloc")
        return out

    # ----------------------------------------------------------- tuning --
    def set_tuning(self, op, run_len=0, conc=4):
        _check(lib().fc_plan_set_tuning(self._h, op, run_len, conc), "fc_plan_set_tuning")

    def get_tuning(self, op):
        r, c = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fc_plan_get_tuning(self._h, op, ctypes.byref(r), ctypes.byref(c)), "fc_plan_get_tuning")
        return dict(run_len=r.value, conc=c.value)

    def set_transform_plan(self, op, tplan):
        _check(lib().fc_plan_set_transform_plan(self._h, op, tplan), "fc_plan_set_transform_plan")

    def get_transform_plan(self, op):
        t = ctypes.c_int32()
        _check(lib().fc_plan_get_transform_plan(self._h, op, ctypes.byref(t)), "fc_plan_get_transform_plan")
        return t.value

    def get_class_plans(self, op):
        """(kernel classes of op with two transform plans, how many run plan 1)."""
        n, n1 = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fc_plan_get_class_plans(self._h, op, ctypes.byref(n), ctypes.byref(n1)),
               "fc_plan_get_class_plans")
        return n.value, n1.value

    def autotune(self, op, inp, out, stream=None):
        """Time the op's work splits and transform plans on these buffers (out
        is overwritten) and keep the fastest; returns the choice and its time
        per call."""
        lo, hi = self.layout(op)
        n_in, n_out = (int(lo[-1]), int(hi[-1])) if op in (OP_TX, OP_TXG) else (int(hi[-1]), int(lo[-1]))
        self._check_buf(inp, n_in, "input")
        self._check_buf(out, n_out, "output")
        r, c, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        _check(lib().fc_plan_autotune(self._h, op, _ptr(inp), _ptr(out), _stream_handle(stream), ctypes.byref(r),
                                      ctypes.byref(c), ctypes.byref(ms)), "fc_plan_autotune")
        n, n1 = self.get_class_plans(op)
        return dict(run_len=r.value, conc=c.value, plan=self.get_transform_plan(op), classes_plan1=n1,
                    classes_two_plans=n, ms=ms.value)


class Graph:
    """A HIP graph of FC calls: ``with Graph(stream) as g: plan.tx(...)``
    records the calls made on ``stream`` (a non-default torch stream) inside
    the block; ``g.launch()`` replays them."""

    def __init__(self, stream):
        if stream is None or stream.cuda_stream == 0:
            raise ValueError("capture needs a non-default stream")
        self.stream = stream
        self._g = None

    def __enter__(self):
        import torch
        self._prev = torch.cuda.current_stream(self.stream.device)
        torch.cuda.set_stream(self.stream)
        _check(lib().fc_graph_begin(_stream_handle(self.stream)), "fc_graph_begin")
        return self

    def __exit__(self, et, ev, tb):
        import torch
        h = _P()
        st = lib().fc_graph_end(_stream_handle(self.stream), ctypes.byref(h))
        torch.cuda.set_stream(self._prev)
        if et is None:
            _check(st, "fc_graph_end")
            self._g = h
        elif h.value:
            lib().fc_graph_destroy(h)
        return False

    def launch(self, stream=None):
        if self._g is None:
            raise RuntimeError("graph not captured")
        _check(lib().fc_graph_launch(self._g, _stream_handle(stream or self.stream)), "fc_graph_launch")

    def close(self):
        if self._g is not None and _lib is not None:
            lib().fc_graph_destroy(self._g)
        self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
