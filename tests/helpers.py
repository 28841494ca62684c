"""Test-side input recipe: seeded draws from ``synth`` placed and encoded by
the oracle.  Nothing here comes from the HIP path."""

import functools

import numpy as np

import oracle
import synth


@functools.lru_cache(maxsize=None)
def frozen_mask(N, K, design_db=0.0):
    fz, _ = oracle.construct(N, K, design_db)
    return np.array(fz, dtype=np.uint8)


def make_frames(N, K, B, ebn0_db, stream, frame0=0, frozen=None):
    """(u, x, llr): source words (B, N), codewords (B, N) and FP32 LLRs of
    a BPSK/AWGN transmission at ``ebn0_db`` (scalar or (B,) array)."""
    if frozen is None:
        frozen = frozen_mask(N, K)
    u = np.zeros((B, N), np.uint8)
    u[:, frozen == 0] = synth.info_bits(K, B, frame0=frame0, stream=stream)
    x = oracle.encode(u)
    nz = synth.normals(N, B, frame0=frame0, stream=stream)
    # a rate-0 code has no Eb; its channel is set as if it carried one bit
    llr = synth.channel_llr(x, nz, ebn0_db, max(K, 1) / N)
    return u, x, llr


def noiseless_llr(x, mag=4.0):
    return (mag * (1.0 - 2.0 * x.astype(np.float64))).astype(np.float32)


def wilson(k, n, z=1.959963984540054):
    """Wilson score interval of a binomial proportion."""
    if n == 0:
        return 0.0, 1.0
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h
