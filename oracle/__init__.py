"""CPU oracle of the polar BP decoder -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product never does.  It shares no
code with the HIP path: the C library (bp_oracle.c) is built with gcc in two
precisions, and the construction (construct.py) is high-precision Python.

Functions and the passages they follow:
  construct          Section II (reliable/unreliable split); Bhattacharyya
                     recursion for the ranking.
  encode             Section II, Fig. 1 (x = u F^{(x)m}).
  csfg_check         eqs. (2)-(4), Lemma 1.
  decode             Section II-A eq. (1) and schedule (single sweep, or the
                     round trip: an L pass then an R pass); Section III
                     freezing; G-matrix stop; Section IV PE count.
  unrolled_forward   eq. (1) with per-(iteration, stage, direction) scales.
  unrolled_grad      reverse-mode derivative of unrolled_forward.
  unrolled_grad_mag  the magnitude sums of unrolled_grad's terms (sizes the
                     rounding error of a gradient computed in FP32).
  sc_decode          successive cancellation, the decoder whose scheduling
                     tree Section III maps onto the factor graph (min-sum f).
  decode_quant       decode with saturating b-bit fixed-point messages (the
                     hardware cost framing of Sections I and V).
  quantize           the channel quantizer of decode_quant.
"""

import ctypes
import os

import numpy as np

from .construct import construct, bhattacharyya, design_z0, logits  # noqa

HERE = os.path.dirname(os.path.abspath(__file__))

WALK_ONE_PER_ITER = 0
WALK_ONE_PER_STAGE = 1
WALK_GREEDY = 2
INPUT_R = 0
INPUT_TOTAL = 1
SCHEDULE_SINGLE = 0
SCHEDULE_ROUND_TRIP = 1


class Opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("early_stop", ctypes.c_int32),
                ("freezing", ctypes.c_int32), ("freeze_input", ctypes.c_int32),
                ("freeze_walk", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("schedule", ctypes.c_int32)]


class QFmt(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_int32), ("frac", ctypes.c_int32)]


_libs = {}


def _lib(prec):
    if prec not in _libs:
        path = os.path.join(HERE, f"liboracle_{prec}.so")
        if not os.path.exists(path):
            from .build import build
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_decode.argtypes = [ctypes.c_int, P, ctypes.c_int64, P,
                                      ctypes.POINTER(Opts), P, P, P, P, P,
                                      ctypes.c_int32, P]
        lib.oracle_decode.restype = ctypes.c_int
        lib.oracle_encode_batch.argtypes = [ctypes.c_int, ctypes.c_int64, P, P]
        lib.oracle_csfg_check.argtypes = [ctypes.c_int, P, P, P, P]
        lib.oracle_csfg_check.restype = ctypes.c_int
        lib.oracle_unrolled_forward.argtypes = [ctypes.c_int, P, ctypes.c_int64,
                                                P, ctypes.c_int, P, P]
        lib.oracle_unrolled_messages.argtypes = [
            ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int, P, P, P]
        lib.oracle_unrolled_grad.argtypes = [ctypes.c_int, P, ctypes.c_int64,
                                             P, ctypes.c_int, P, P, P, P]
        lib.oracle_unrolled_grad_mag.argtypes = \
            lib.oracle_unrolled_grad.argtypes
        lib.oracle_sc_decode.argtypes = [ctypes.c_int, P, ctypes.c_int64, P,
                                         P, P]
        lib.oracle_sc_decode.restype = ctypes.c_int
        lib.oracle_decode_q.argtypes = [ctypes.c_int, P, ctypes.c_int64, P,
                                        ctypes.POINTER(Opts),
                                        ctypes.POINTER(QFmt), P, P, P, P]
        lib.oracle_decode_q.restype = ctypes.c_int
        lib.oracle_quantize.argtypes = [ctypes.c_float, ctypes.c_int32,
                                        ctypes.c_int32]
        lib.oracle_quantize.restype = ctypes.c_int32
        expect = 4 if prec == "f32" else 8
        assert lib.oracle_real_bytes() == expect
        _libs[prec] = lib
    return _libs[prec]


def _real(prec):
    return np.float32 if prec == "f32" else np.float64


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _m_of(N):
    m = int(N).bit_length() - 1
    if N < 2 or (1 << m) != N:
        raise ValueError("N must be a power of two >= 2")
    return m


def encode(u):
    """x = u F^{(x)m}; u is (N,) or (B, N) uint8."""
    u = np.ascontiguousarray(u, dtype=np.uint8)
    shape = u.shape
    u2 = u.reshape(-1, shape[-1])
    x = np.empty_like(u2)
    _lib("f32").oracle_encode_batch(_m_of(shape[-1]), u2.shape[0], _ptr(u2),
                                    _ptr(x))
    return x.reshape(shape)


def csfg_check(msgs, frozen, prec="f64"):
    """eqs. (2)-(4) on one CSFG: returns (pass, xhat, uhat)."""
    msgs = np.ascontiguousarray(msgs, dtype=_real(prec))
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    n = msgs.shape[0]
    xh = np.empty(n, np.uint8)
    uh = np.empty(n, np.uint8)
    ok = _lib(prec).oracle_csfg_check(_m_of(n) if n > 1 else 0, _ptr(msgs),
                                      _ptr(frozen), _ptr(xh), _ptr(uh))
    return bool(ok), xh, uh


def decode(llr, frozen, max_iter=40, early_stop=True, freezing=False,
           freeze_input=INPUT_TOTAL, freeze_walk=WALK_ONE_PER_ITER,
           alpha=0.9375, prec="f32", soft=False, trace=False, trace_cap=1 << 16,
           schedule=SCHEDULE_SINGLE):
    """Decode a batch of FP32 LLRs (B, N).

    Returns a dict with ``uhat`` (B, N) source-word decisions, ``info``
    (B, K) the information bits, ``iters`` (B,), ``pe`` (B,), and when asked
    ``soft`` (B, N) posterior LLRs of u and ``trace`` (n, 5) freezing checks
    (frame, t, j, k, pass).
    """
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim == 1:
        llr = llr[None, :]
    B, N = llr.shape
    m = _m_of(N)
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    assert frozen.shape == (N,)
    o = Opts(int(max_iter), int(bool(early_stop)), int(bool(freezing)),
             int(freeze_input), int(freeze_walk), float(alpha), int(schedule))
    uhat = np.empty((B, N), np.uint8)
    iters = np.empty(B, np.int32)
    pe = np.empty(B, np.int64)
    sf = np.empty((B, N), _real(prec)) if soft else None
    tr = np.empty((trace_cap, 5), np.int32) if trace else None
    tl = ctypes.c_int32(0)
    rc = _lib(prec).oracle_decode(m, _ptr(frozen), B, _ptr(llr),
                                  ctypes.byref(o), _ptr(uhat), _ptr(iters),
                                  _ptr(pe), _ptr(sf), _ptr(tr),
                                  trace_cap if trace else 0, ctypes.byref(tl))
    if rc != 0:
        raise ValueError("oracle_decode rejected its arguments")
    out = {"uhat": uhat, "info": uhat[:, frozen == 0], "iters": iters, "pe": pe}
    if soft:
        out["soft"] = sf
    if trace:
        out["trace"] = tr[:tl.value].copy()
    return out


def unrolled_forward(llr, frozen, alpha, prec="f64"):
    """R^T at column m+1, (B, N), of the unrolled decoder; alpha is (T, m, 2)."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    B, N = llr.shape
    m = _m_of(N)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    T = alpha.shape[0]
    assert alpha.shape == (T, m, 2)
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    out = np.empty((B, N), _real(prec))
    _lib(prec).oracle_unrolled_forward(m, _ptr(frozen), B, _ptr(llr), T,
                                       _ptr(alpha), _ptr(out))
    return out


def unrolled_messages(llr, frozen, alpha, prec="f64"):
    """Every message of the unrolled decoder: (L, R), each (B, T+1, m+2, N),
    column c of iteration t at [f, t, c] (t = 0: the initial state; column 0
    unused).  Section II-A, eq. (1), applied as in unrolled_forward."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    B, N = llr.shape
    m = _m_of(N)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    T = alpha.shape[0]
    assert alpha.shape == (T, m, 2)
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    L = np.empty((B, T + 1, m + 2, N), _real(prec))
    R = np.empty_like(L)
    _lib(prec).oracle_unrolled_messages(m, _ptr(frozen), B, _ptr(llr), T,
                                        _ptr(alpha), _ptr(L), _ptr(R))
    return L, R


def unrolled_grad(llr, frozen, alpha, dout, prec="f64"):
    """Gradients (dalpha (T, m, 2), dllr (B, N)) of sum(dout * forward)."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    B, N = llr.shape
    m = _m_of(N)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    T = alpha.shape[0]
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    dout = np.ascontiguousarray(dout, dtype=np.float64)
    assert dout.shape == (B, N)
    da = np.empty((T, m, 2), np.float64)
    dl = np.empty((B, N), np.float64)
    _lib(prec).oracle_unrolled_grad(m, _ptr(frozen), B, _ptr(llr), T,
                                    _ptr(alpha), _ptr(dout), _ptr(da), _ptr(dl))
    return da, dl


def unrolled_grad_mag(llr, frozen, alpha, dout, prec="f64"):
    """(A_alpha (T, m, 2), A_llr (B, N)): for every element of unrolled_grad's
    result, the sum of the magnitudes of the path terms it adds up (|dout|,
    scales, |g0| for the scale gradients; no sign factors).  An FP32
    accumulation of those terms in any order is within n u A of the exact
    sum, n the roundings along the longest path and u = 2^-24."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    B, N = llr.shape
    m = _m_of(N)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    if not (alpha > 0).all():
        raise ValueError("scales must be positive")
    T = alpha.shape[0]
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    dout = np.ascontiguousarray(dout, dtype=np.float64)
    assert dout.shape == (B, N)
    da = np.empty((T, m, 2), np.float64)
    dl = np.empty((B, N), np.float64)
    _lib(prec).oracle_unrolled_grad_mag(m, _ptr(frozen), B, _ptr(llr), T,
                                        _ptr(alpha), _ptr(dout), _ptr(da),
                                        _ptr(dl))
    return da, dl


def sc_decode(llr, frozen, prec="f32", leaf=False):
    """Successive-cancellation decisions (B, N) uint8 of FP32 LLRs (B, N);
    with ``leaf`` also the LLR reaching each leaf, (B, N)."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim == 1:
        llr = llr[None, :]
    B, N = llr.shape
    m = _m_of(N)
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    uhat = np.empty((B, N), np.uint8)
    lf = np.empty((B, N), _real(prec)) if leaf else None
    rc = _lib(prec).oracle_sc_decode(m, _ptr(frozen), B, _ptr(llr), _ptr(uhat),
                                     _ptr(lf))
    assert rc == 0
    return (uhat, lf) if leaf else uhat


def quantize(llr, bits=8, frac=3):
    """decode_quant's channel quantizer: clamp(round(LLR 2^F), -Q, Q)."""
    f = _lib("f64").oracle_quantize
    a = np.asarray(llr, np.float32)
    return np.array([f(float(v), int(bits), int(frac)) for v in a.ravel()],
                    np.int32).reshape(a.shape)


def decode_quant(llr, frozen, bits=8, frac=3, max_iter=40, early_stop=True,
                 freezing=False, freeze_input=INPUT_TOTAL,
                 freeze_walk=WALK_ONE_PER_ITER, alpha=0.9375, soft=False):
    """decode() with saturating fixed-point messages (single sweep).  Returns
    the same dict; ``soft`` holds sat(R + L) at column m+1 as int32."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim == 1:
        llr = llr[None, :]
    B, N = llr.shape
    m = _m_of(N)
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    o = Opts(int(max_iter), int(bool(early_stop)), int(bool(freezing)),
             int(freeze_input), int(freeze_walk), float(alpha), 0)
    qf = QFmt(int(bits), int(frac))
    uhat = np.empty((B, N), np.uint8)
    iters = np.empty(B, np.int32)
    pe = np.empty(B, np.int64)
    sf = np.empty((B, N), np.int32) if soft else None
    rc = _lib("f64").oracle_decode_q(m, _ptr(frozen), B, _ptr(llr),
                                     ctypes.byref(o), ctypes.byref(qf),
                                     _ptr(uhat), _ptr(iters), _ptr(pe),
                                     _ptr(sf))
    if rc != 0:
        raise ValueError("oracle_decode_q rejected its arguments")
    out = {"uhat": uhat, "info": uhat[:, frozen == 0], "iters": iters, "pe": pe}
    if soft:
        out["soft"] = sf
    return out
