"""Philox4x32-10 (Salmon et al., SC'11), vectorised over numpy arrays.

One round maps counter (c0, c1, c2, c3) under key (k0, k1) to

    hi0:lo0 = M0 * c0,  hi1:lo1 = M1 * c2           (32x32 -> 64-bit products)
    (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)

and the key is bumped by the Weyl constants (W0, W1) between rounds; ten
rounds make Philox4x32-10.  Arithmetic is done in uint64 holding 32-bit
values so that the products are exact.
"""

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF

#: default seed of every synthetic workload (the arXiv number of the paper)
SEED = 150504979

PURPOSE_BITS = 0      # information bits
PURPOSE_NOISE = 1     # channel noise
PURPOSE_UNIFORM = 2   # per-frame uniforms (Eb/N0, code choice, ...)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit outputs (as uint64 arrays) for the given
    counters and keys; arguments broadcast against each other."""
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & _MASK
                              for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3 = (np.array(v) for v in (c0, c1, c2, c3))
    k0 = np.array(k0)
    k1 = np.array(k1)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    w0 = np.uint64(W0)
    w1 = np.uint64(W1)
    mask = np.uint64(_MASK)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def u53(a, b):
    """Uniform double in [0, 1) from two 32-bit words (53 random bits)."""
    a = np.asarray(a, dtype=np.uint64) >> np.uint64(5)
    b = np.asarray(b, dtype=np.uint64) >> np.uint64(6)
    return (a.astype(np.float64) * 67108864.0 + b.astype(np.float64)) \
        * (1.0 / 9007199254740992.0)
