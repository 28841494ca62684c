"""Thin Python binding of libpbp (include/pbp.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors on a ROCm device (torch supplies memory and
streams, nothing else); every step of decoding runs in the HIP library.
There is no CPU fallback: without the built library, or given host tensors
where device memory is required, these functions raise.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbp.so")

PBP_OK = 0

_P = ctypes.c_void_p


class pbp_decode_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("early_stop", ctypes.c_int32),
                ("freezing", ctypes.c_int32), ("freeze_input", ctypes.c_int32),
                ("freeze_walk", ctypes.c_int32), ("alpha", ctypes.c_float)]


class pbp_mixed_config(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32)]


class PbpError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn} failed: {status_string(status)} ({status})")


_lib = None

# (name, restype, argtypes) of every exported entry point
_SIGNATURES = [
    ("pbp_status_string", ctypes.c_char_p, [ctypes.c_int32]),
    ("pbp_construct", ctypes.c_int32,
     [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P]),
    ("pbp_code_create", ctypes.c_int32,
     [ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    ("pbp_code_destroy", None, [_P]),
    ("pbp_code_dims", ctypes.c_int32, [_P, _P, _P]),
    ("pbp_encode", ctypes.c_int32, [_P, _P, ctypes.c_int64, _P, _P]),
    ("pbp_decode", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.POINTER(pbp_decode_opts), _P, _P, _P, _P,
      _P]),
    ("pbp_decode_noalloc", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.POINTER(pbp_decode_opts), _P, _P, _P, _P,
      _P]),
    ("pbp_workspace_release", ctypes.c_int32, [_P]),
    ("pbp_decode_round_trip", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.POINTER(pbp_decode_opts), _P, _P, _P, _P,
      _P]),
    ("pbp_decode_quant", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.POINTER(pbp_decode_opts), ctypes.c_int32,
      ctypes.c_int32, _P, _P, _P, _P, _P]),
    ("pbp_decode_sc", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, _P, _P, _P]),
    ("pbp_mixed_plan_create", ctypes.c_int32,
     [_P, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(_P)]),
    ("pbp_mixed_plan_destroy", None, [_P]),
    ("pbp_mixed_plan_get_config", ctypes.c_int32,
     [_P, ctypes.POINTER(pbp_mixed_config)]),
    ("pbp_mixed_plan_set_config", ctypes.c_int32,
     [_P, ctypes.POINTER(pbp_mixed_config)]),
    ("pbp_decode_mixed", ctypes.c_int32,
     [_P, _P, _P, _P, ctypes.c_int64, _P, ctypes.POINTER(pbp_decode_opts), _P,
      _P, _P, _P]),
    ("pbp_mixed_plan_tune", ctypes.c_int32,
     [_P, _P, _P, _P, ctypes.c_int64, _P, ctypes.POINTER(pbp_decode_opts), _P,
      _P, _P, ctypes.c_int32, _P, ctypes.POINTER(pbp_mixed_config)]),
    ("pbp_mixed_plan_fill", ctypes.c_int32,
     [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    ("pbp_unrolled_forward", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P, _P]),
    ("pbp_unrolled_backward", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P]),
]


def lib():
    """Load libpbp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing; build it with "
                "`python -m paper_1505_04979_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [s[0] for s in _SIGNATURES]


def status_string(status):
    return lib().pbp_status_string(int(status)).decode()


def _check(fn, status):
    if status != PBP_OK:
        raise PbpError(fn, status)


def _dev_ptr(t, dtype, shape, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def pbp_construct(N, K, design_ebn0_db=0.0):
    """Frozen mask (numpy uint8, 1 = frozen) of an (N, K) code."""
    out = np.zeros(int(N), np.uint8)
    _check("pbp_construct", lib().pbp_construct(
        int(N), int(K), float(design_ebn0_db), out.ctypes.data_as(_P)))
    return out


class Code:
    """Owns a pbp_code handle (pbp_code_create / pbp_code_destroy)."""

    def __init__(self, N, K, frozen):
        frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
        if frozen.shape != (int(N),):
            raise ValueError("frozen must have N entries")
        h = _P()
        _check("pbp_code_create", lib().pbp_code_create(
            int(N), int(K), frozen.ctypes.data_as(_P), ctypes.byref(h)))
        self._h = h
        self.N, self.K = int(N), int(K)
        self.m = self.N.bit_length() - 1
        self.frozen = frozen.copy()

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pbp_code_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pbp_code_create(N, K, frozen):
    return Code(N, K, frozen)


def pbp_code_dims(code):
    n = ctypes.c_int32()
    k = ctypes.c_int32()
    _check("pbp_code_dims", lib().pbp_code_dims(code.handle, ctypes.byref(n),
                                                ctypes.byref(k)))
    return n.value, k.value


def pbp_encode(code, info, codeword=None, stream=None):
    """Codewords (B, N) uint8 of information bits ``info`` (B, K) uint8."""
    import torch
    B = int(info.shape[0])
    if codeword is None:
        codeword = torch.empty((B, code.N), dtype=torch.uint8, device=info.device)
    _check("pbp_encode", lib().pbp_encode(
        code.handle, _dev_ptr(info, torch.uint8, (B, code.K), "info"), B,
        _dev_ptr(codeword, torch.uint8, (B, code.N), "codeword"),
        _stream(stream)))
    return codeword


def make_opts(max_iter=40, early_stop=True, freezing=False, freeze_input=1,
              freeze_walk=0, alpha=0.9375):
    return pbp_decode_opts(int(max_iter), int(bool(early_stop)),
                           int(bool(freezing)), int(freeze_input),
                           int(freeze_walk), float(alpha))


def pbp_decode(code, llr, opts=None, pe=True, soft=False, out=None,
               stream=None, schedule="single", **kw):
    """Decode FP32 LLRs (B, N) on the device.

    Returns a dict of device tensors: ``info`` (B, K) uint8, ``iters`` (B,)
    int32, ``pe`` (B,) int64 when asked, ``soft`` (B, N) float32 when asked.
    ``opts`` is a pbp_decode_opts or None (then keyword options apply).
    Pass ``out`` (a dict of preallocated tensors) to avoid allocation.
    ``schedule``: "single" (pbp_decode), "round_trip"
    (pbp_decode_round_trip: no freezing, N <= 2048) or "noalloc"
    (pbp_decode_noalloc: the single sweep with static scratch).
    """
    import torch
    if opts is None:
        opts = make_opts(**kw)
    B = int(llr.shape[0])
    dev = llr.device
    o = dict(out or {})
    if "info" not in o:
        o["info"] = torch.empty((B, code.K), dtype=torch.uint8, device=dev)
    if "iters" not in o:
        o["iters"] = torch.empty((B,), dtype=torch.int32, device=dev)
    if pe and "pe" not in o:
        o["pe"] = torch.empty((B,), dtype=torch.int64, device=dev)
    if soft and "soft" not in o:
        o["soft"] = torch.empty((B, code.N), dtype=torch.float32, device=dev)
    names = {"single": "pbp_decode", "round_trip": "pbp_decode_round_trip",
             "noalloc": "pbp_decode_noalloc"}
    if schedule not in names:
        raise ValueError(f"unknown schedule {schedule!r}")
    name = names[schedule]
    _check(name, getattr(lib(), name)(
        code.handle, _dev_ptr(llr, torch.float32, (B, code.N), "llr"), B,
        ctypes.byref(opts),
        _dev_ptr(o["info"], torch.uint8, (B, code.K), "info"),
        _dev_ptr(o["iters"], torch.int32, (B,), "iters"),
        _dev_ptr(o.get("pe") if pe else None, torch.int64, (B,), "pe"),
        _dev_ptr(o.get("soft") if soft else None, torch.float32, (B, code.N),
                 "soft"),
        _stream(stream)))
    return o


def pbp_decode_round_trip(code, llr, opts=None, pe=True, soft=False, out=None,
                          stream=None, **kw):
    """pbp_decode with the round-trip schedule (the C entry point
    pbp_decode_round_trip): same arguments and outputs; no freezing,
    N <= 2048."""
    return pbp_decode(code, llr, opts=opts, pe=pe, soft=soft, out=out,
                      stream=stream, schedule="round_trip", **kw)


def pbp_decode_noalloc(code, llr, opts=None, pe=True, soft=False, out=None,
                       stream=None, **kw):
    """pbp_decode through the C entry point pbp_decode_noalloc (its scratch
    is a static device array; the library allocates nothing): same
    arguments and outputs.  Pass ``out`` to allocate nothing here either."""
    return pbp_decode(code, llr, opts=opts, pe=pe, soft=soft, out=out,
                      stream=stream, schedule="noalloc", **kw)


def pbp_workspace_release(stream=None):
    """Free the library's decoder workspace of ``stream`` (default: torch's
    current stream) on the current device, after synchronising it."""
    _check("pbp_workspace_release", lib().pbp_workspace_release(
        _stream(stream)))


def pbp_decode_quant(code, llr, bits=8, frac=3, opts=None, pe=True, soft=False,
                     out=None, stream=None, **kw):
    """pbp_decode with saturating ``bits``-bit fixed-point messages (channel
    quantized with ``frac`` fraction bits).  Returns ``info``, ``iters``,
    ``pe`` and, when asked, ``soft`` (B, N) int8."""
    import torch
    if opts is None:
        opts = make_opts(**kw)
    B = int(llr.shape[0])
    dev = llr.device
    o = dict(out or {})
    if "info" not in o:
        o["info"] = torch.empty((B, code.K), dtype=torch.uint8, device=dev)
    if "iters" not in o:
        o["iters"] = torch.empty((B,), dtype=torch.int32, device=dev)
    if pe and "pe" not in o:
        o["pe"] = torch.empty((B,), dtype=torch.int64, device=dev)
    if soft and "soft" not in o:
        o["soft"] = torch.empty((B, code.N), dtype=torch.int8, device=dev)
    _check("pbp_decode_quant", lib().pbp_decode_quant(
        code.handle, _dev_ptr(llr, torch.float32, (B, code.N), "llr"), B,
        ctypes.byref(opts), int(bits), int(frac),
        _dev_ptr(o["info"], torch.uint8, (B, code.K), "info"),
        _dev_ptr(o["iters"], torch.int32, (B,), "iters"),
        _dev_ptr(o.get("pe") if pe else None, torch.int64, (B,), "pe"),
        _dev_ptr(o.get("soft") if soft else None, torch.int8, (B, code.N),
                 "soft"),
        _stream(stream)))
    return o


def pbp_decode_sc(code, llr, leaf=False, out=None, stream=None):
    """Successive-cancellation decoding of FP32 LLRs (B, N) on the device.

    Returns a dict of device tensors: ``info`` (B, K) uint8 and, when asked,
    ``leaf`` (B, N) float32, the LLR reaching each leaf."""
    import torch
    B = int(llr.shape[0])
    dev = llr.device
    o = dict(out or {})
    if "info" not in o:
        o["info"] = torch.empty((B, code.K), dtype=torch.uint8, device=dev)
    if leaf and "leaf" not in o:
        o["leaf"] = torch.empty((B, code.N), dtype=torch.float32, device=dev)
    _check("pbp_decode_sc", lib().pbp_decode_sc(
        code.handle, _dev_ptr(llr, torch.float32, (B, code.N), "llr"), B,
        _dev_ptr(o["info"], torch.uint8, (B, code.K), "info"),
        _dev_ptr(o.get("leaf") if leaf else None, torch.float32, (B, code.N),
                 "leaf"),
        _stream(stream)))
    return o


def pbp_unrolled_forward(code, llr, alpha, ckpt=True, out=None, stream=None):
    """Unrolled BP with scales ``alpha`` (T, m, 2) float32 on the device.

    Returns ``(out, ckpt)``: R^T at column m+1, (B, N) float32, and the
    per-iteration L checkpoints (T, B, m-1, N) float32 for the backward call
    (``ckpt=False``: none are written and None is returned; a tensor: it is
    filled).
    """
    import torch
    B, T = int(llr.shape[0]), int(alpha.shape[0])
    m, N, dev = code.m, code.N, llr.device
    if out is None:
        out = torch.empty((B, N), dtype=torch.float32, device=dev)
    if ckpt is True:
        ckpt = torch.empty((T, B, max(m - 1, 0), N), dtype=torch.float32,
                           device=dev)
    elif ckpt is False:
        ckpt = None
    _check("pbp_unrolled_forward", lib().pbp_unrolled_forward(
        code.handle, _dev_ptr(llr, torch.float32, (B, N), "llr"), B, T,
        _dev_ptr(alpha, torch.float32, (T, m, 2), "alpha"),
        _dev_ptr(out, torch.float32, (B, N), "out"),
        _dev_ptr(ckpt, torch.float32, (T, B, max(m - 1, 0), N), "ckpt"),
        _stream(stream)))
    return out, ckpt


def pbp_unrolled_backward(code, llr, alpha, ckpt, dout, dllr=True,
                          stream=None):
    """Gradients of sum(dout * out) of pbp_unrolled_forward.

    Returns ``(dalpha, dllr, dalpha_frame)``: (T, m, 2), (B, N) or None,
    and each frame's share of dalpha, (B, T, m, 2); all float32.
    """
    import torch
    B, T = int(llr.shape[0]), int(alpha.shape[0])
    m, N, dev = code.m, code.N, llr.device
    dalpha = torch.empty((T, m, 2), dtype=torch.float32, device=dev)
    dframe = torch.empty((B, T, m, 2), dtype=torch.float32, device=dev)
    if dllr is True:
        dllr = torch.empty((B, N), dtype=torch.float32, device=dev)
    elif dllr is False:
        dllr = None
    _check("pbp_unrolled_backward", lib().pbp_unrolled_backward(
        code.handle, _dev_ptr(llr, torch.float32, (B, N), "llr"), B, T,
        _dev_ptr(alpha, torch.float32, (T, m, 2), "alpha"),
        _dev_ptr(ckpt, torch.float32, (T, B, max(m - 1, 0), N), "ckpt"),
        _dev_ptr(dout, torch.float32, (B, N), "dout"),
        _dev_ptr(dframe, torch.float32, (B, T, m, 2), "dalpha_frame"),
        _dev_ptr(dalpha, torch.float32, (T, m, 2), "dalpha"),
        _dev_ptr(dllr, torch.float32, (B, N), "dllr"),
        _stream(stream)))
    return dalpha, dllr, dframe


class MixedPlan:
    """Owns a pbp_mixed_plan over a list of Code objects (kept alive here)."""

    def __init__(self, codes, max_frames):
        self.codes = list(codes)
        arr = (_P * len(self.codes))(*[c.handle for c in self.codes])
        h = _P()
        _check("pbp_mixed_plan_create", lib().pbp_mixed_plan_create(
            arr, len(self.codes), int(max_frames), ctypes.byref(h)))
        self._h = h
        self.max_frames = int(max_frames)

    @property
    def handle(self):
        return self._h

    @property
    def config(self):
        c = pbp_mixed_config()
        _check("pbp_mixed_plan_get_config",
               lib().pbp_mixed_plan_get_config(self._h, ctypes.byref(c)))
        return (c.order, c.waves_per_cu)

    @config.setter
    def config(self, value):
        c = pbp_mixed_config(int(value[0]), int(value[1]))
        _check("pbp_mixed_plan_set_config",
               lib().pbp_mixed_plan_set_config(self._h, ctypes.byref(c)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pbp_mixed_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pbp_mixed_plan_create(codes, max_frames):
    return MixedPlan(codes, max_frames)


def _mixed_args(plan, code_of_frame, llr_off, info_off, llr, info_bytes,
                opts, pe, out, kw):
    import torch
    if opts is None:
        opts = make_opts(**kw)
    B = int(code_of_frame.shape[0])
    dev = code_of_frame.device
    o = dict(out or {})
    if "info" not in o:
        o["info"] = torch.empty((int(info_bytes),), dtype=torch.uint8,
                                device=dev)
    if "iters" not in o:
        o["iters"] = torch.empty((B,), dtype=torch.int32, device=dev)
    if pe and "pe" not in o:
        o["pe"] = torch.empty((B,), dtype=torch.int64, device=dev)
    if llr.dim() != 1:
        raise ValueError("llr must be a flat buffer")
    args = (_dev_ptr(code_of_frame, torch.int32, (B,), "code_of_frame"),
            _dev_ptr(llr_off, torch.int64, (B,), "llr_off"),
            _dev_ptr(info_off, torch.int64, (B,), "info_off"), B,
            _dev_ptr(llr, torch.float32, tuple(llr.shape), "llr"),
            ctypes.byref(opts),
            _dev_ptr(o["info"], torch.uint8, tuple(o["info"].shape), "info"),
            _dev_ptr(o["iters"], torch.int32, (B,), "iters"),
            _dev_ptr(o.get("pe") if pe else None, torch.int64, (B,), "pe"))
    return args, o


def pbp_decode_mixed(plan, code_of_frame, llr_off, info_off, llr,
                     info_bytes=None, opts=None, pe=True, out=None,
                     stream=None, **kw):
    """Decode a mixed batch: frame f of code ``codes[code_of_frame[f]]`` has
    its LLRs at ``llr[llr_off[f]:]`` (flat float32 buffer) and its decided
    information bits go to ``info[info_off[f]:]`` (flat uint8 buffer of
    ``info_bytes`` bytes, or ``out["info"]``).  Returns a dict of device
    tensors ``info``, ``iters`` and (when asked) ``pe``."""
    args, o = _mixed_args(plan, code_of_frame, llr_off, info_off, llr,
                          info_bytes, opts, pe, out, kw)
    _check("pbp_decode_mixed", lib().pbp_decode_mixed(
        plan.handle, *args, _stream(stream)))
    return o


def pbp_mixed_plan_tune(plan, code_of_frame, llr_off, info_off, llr,
                        info_bytes=None, opts=None, pe=True, out=None,
                        reps=2, stream=None, **kw):
    """Choose the plan's configuration by timing the candidates on this
    batch (outputs overwritten); returns (order, waves_per_cu)."""
    args, o = _mixed_args(plan, code_of_frame, llr_off, info_off, llr,
                          info_bytes, opts, pe, out, kw)
    best = pbp_mixed_config()
    _check("pbp_mixed_plan_tune", lib().pbp_mixed_plan_tune(
        plan.handle, *args, int(reps), _stream(stream), ctypes.byref(best)))
    return (best.order, best.waves_per_cu)


def pbp_mixed_plan_fill(plan, stream=None):
    """Fill efficiency of the plan's last launch (synchronises the stream)."""
    v = ctypes.c_double()
    _check("pbp_mixed_plan_fill", lib().pbp_mixed_plan_fill(
        plan.handle, _stream(stream), ctypes.byref(v)))
    return v.value
