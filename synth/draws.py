"""Per-frame draws and the BPSK/AWGN channel.

All functions take ``frame0`` (the first frame index) and a count ``B`` so
that any slice of a workload can be regenerated on its own.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .philox import (PURPOSE_BITS, PURPOSE_NOISE, PURPOSE_UNIFORM, SEED,
                     philox4x32_10, u53)

_CHUNK_WORDS = 1 << 20  # Philox calls per chunk (bounds host memory)
_THREADS = max(1, min(16, os.cpu_count() or 1))


def _run_blocks(B, words, fn):
    """Run fn(lo, hi) over frame blocks; numpy releases the GIL inside its
    array kernels, so the blocks proceed in parallel threads."""
    blocks = list(_blocks(B, words))
    if len(blocks) <= 1 or _THREADS == 1:
        for lo, hi in blocks:
            fn(lo, hi)
        return
    with ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(lambda b: fn(*b), blocks))


def stream_id(config, point):
    """Stream key of one operating point of one workload."""
    return (int(config) << 16) + int(point)


def _frames(frame0, B):
    f = np.arange(frame0, frame0 + B, dtype=np.uint64)
    return f & np.uint64(0xFFFFFFFF), f >> np.uint64(32)


def _blocks(B, words):
    """Split B frames into frame blocks of at most _CHUNK_WORDS calls."""
    per = max(1, _CHUNK_WORDS // max(1, words))
    for lo in range(0, B, per):
        yield lo, min(B, lo + per)


def info_bits(K, B, frame0=0, seed=SEED, stream=0):
    """Uniform information bits, shape (B, K) uint8.

    Call w of a frame yields info bits 128w .. 128w+127; bit b of output
    word q is info bit 128w + 32q + b.
    """
    out = np.zeros((B, K), dtype=np.uint8)
    if K == 0 or B == 0:
        return out
    words = (K + 127) // 128
    w = np.arange(words, dtype=np.uint64)
    shifts = np.arange(32, dtype=np.uint64)
    def blk(lo, hi):
        flo, fhi = _frames(frame0 + lo, hi - lo)
        r = philox4x32_10(w[None, :], flo[:, None], fhi[:, None],
                          PURPOSE_BITS, seed, stream)
        # (b, words, 4, 32) bits -> (b, words*128)
        bits = (np.stack(r, axis=-1)[..., None] >> shifts) & np.uint64(1)
        out[lo:hi] = bits.reshape(hi - lo, words * 128)[:, :K]

    _run_blocks(B, words * 32, blk)
    return out


def normals(N, B, frame0=0, seed=SEED, stream=0):
    """Standard normals, shape (B, N) float64, by Box-Muller.

    Call w of a frame yields positions 2w (cosine branch) and 2w+1 (sine
    branch) from u1 = u53(r0, r1) and u2 = u53(r2, r3):
    n = sqrt(-2 ln(1 - u1)) * (cos, sin)(2 pi u2).
    """
    assert N % 2 == 0
    out = np.empty((B, N), dtype=np.float64)
    if B == 0:
        return out
    words = N // 2
    w = np.arange(words, dtype=np.uint64)
    def blk(lo, hi):
        flo, fhi = _frames(frame0 + lo, hi - lo)
        r0, r1, r2, r3 = philox4x32_10(w[None, :], flo[:, None], fhi[:, None],
                                       PURPOSE_NOISE, seed, stream)
        u1 = u53(r0, r1)
        u2 = u53(r2, r3)
        rad = np.sqrt(-2.0 * np.log(1.0 - u1))
        th = (2.0 * np.pi) * u2
        o = out[lo:hi]
        o[:, 0::2] = rad * np.cos(th)
        o[:, 1::2] = rad * np.sin(th)

    _run_blocks(B, words, blk)
    return out


def uniform(B, frame0=0, seed=SEED, stream=0, word=0):
    """One uniform double in [0, 1) per frame, shape (B,).  Different
    ``word`` values give independent draws of the same frame."""
    flo, fhi = _frames(frame0, B)
    r0, r1, _, _ = philox4x32_10(word, flo, fhi, PURPOSE_UNIFORM, seed, stream)
    return u53(r0, r1)


def ebn0_to_sigma2(ebn0_db, rate):
    """Noise variance of BPSK at the given Eb/N0 (dB) and code rate:
    sigma^2 = 1 / (2 R 10^(Eb/N0 / 10))."""
    return 1.0 / (2.0 * rate * np.power(10.0, np.asarray(ebn0_db,
                                                         dtype=np.float64) / 10.0))


def channel_llr(codeword, noise, ebn0_db, rate):
    """BPSK s = 1 - 2x over AWGN, y = s + sigma*n, LLR = 2y/sigma^2.

    ``codeword`` (B, N) uint8, ``noise`` (B, N) float64 standard normals,
    ``ebn0_db`` a scalar or a (B,) array.  Computed in FP64 and rounded once
    to FP32.  A positive LLR favours bit 0.
    """
    codeword = np.asarray(codeword)
    sigma2 = np.asarray(ebn0_to_sigma2(ebn0_db, rate), dtype=np.float64)
    if sigma2.ndim == 1:
        sigma2 = sigma2[:, None]
    sigma = np.sqrt(sigma2)
    s = 1.0 - 2.0 * codeword.astype(np.float64)
    y = s + sigma * noise
    return (2.0 * y / sigma2).astype(np.float32)
