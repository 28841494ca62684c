"""Pins of the oracle's fixed-point decoder (saturating b-bit messages):

* the channel quantizer: exact values, halves rounded away from zero,
  saturation at +-(2^(b-1) - 1);
* N = 2 closed forms in every mode: with position 0 frozen the prior at
  column 2 never changes (a freeze of row 0 keeps +Q), so every iteration
  gives u1 = [sat(q1 + gq(Q, q0)) < 0]; with both free, the first
  iteration gives u0 = [gq(q0, q1) < 0] and u1 = [q1 < 0], with
  gq(x, y) = sign(x) sign(y) ((15 min(|x|, |y|) + 8) >> 4);
* noiseless decoding in every mode;
* codeword symmetry of the messages: every operation is odd in its message
  arguments and the range is symmetric, so without decisions inside the
  loop (plain BP) the posterior of codeword x's LLRs, sign-flipped by x, is
  the posterior times (1 - 2u), exactly (decisions on exact zeros, frequent
  at this resolution, are not symmetric, so the bits are not compared);
* at 16 bits with 8 fraction bits it decides as the FP32 decoder does on
  all but a few frames (the quantization error is below the messages'
  resolution that matters).
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames, noiseless_llr

MODES = [dict(early_stop=False), dict(early_stop=True),
         dict(early_stop=True, freezing=True),
         dict(early_stop=False, freezing=True),
         dict(early_stop=True, freezing=True, freeze_walk=1),
         dict(early_stop=True, freezing=True, freeze_input=0)]


def test_quantizer():
    q = oracle.quantize
    assert q(1.5, 8, 3) == 12 and q(-1.5, 8, 3) == -12
    assert q(0.0625, 8, 3) == 1 and q(-0.0625, 8, 3) == -1   # halves away
    assert q(0.06, 8, 3) == 0 and q(0.07, 8, 3) == 1
    assert q(100.0, 8, 3) == 127 and q(-100.0, 8, 3) == -127
    assert q(15.5, 6, 1) == 31 and q(16.0, 6, 1) == 31 and q(-40, 6, 1) == -31
    assert q(np.inf, 8, 3) == 127


def _gq(x, y):
    return int(np.sign(x) * np.sign(y)) * ((15 * min(abs(x), abs(y)) + 8) >> 4)


@pytest.mark.parametrize("bits,frac", [(8, 3), (6, 1), (5, 2)])
@pytest.mark.parametrize("mode", MODES)
def test_n2_closed_forms(bits, frac, mode):
    Q = (1 << (bits - 1)) - 1
    rng = np.random.default_rng(bits * 10 + frac)
    y = (rng.standard_normal((300, 2)) * 4).astype(np.float32)
    q = oracle.quantize(y, bits, frac)
    r = oracle.decode_quant(y, np.array([1, 0], np.uint8), bits=bits,
                            frac=frac, max_iter=5, **mode)
    sat = lambda v: max(-Q, min(Q, v))
    want = [int(sat(b + _gq(Q, a)) < 0) for a, b in q]
    assert r["uhat"][:, 0].sum() == 0
    assert r["uhat"][:, 1].tolist() == want
    r = oracle.decode_quant(y, np.array([0, 0], np.uint8), bits=bits,
                            frac=frac, max_iter=1, **mode)
    assert r["uhat"][:, 0].tolist() == [int(_gq(a, b) < 0) for a, b in q]
    assert r["uhat"][:, 1].tolist() == [int(b < 0) for a, b in q]


@pytest.mark.parametrize("N,K", [(8, 4), (64, 32), (1024, 512), (4096, 1365)])
def test_noiseless_and_symmetry(N, K):
    fz = frozen_mask(N, K)
    u, x, _ = make_frames(N, K, 20, 2.0, stream=41)
    for mode in MODES:
        r = oracle.decode_quant(noiseless_llr(x), fz, **mode)
        assert np.array_equal(r["uhat"], u), mode
    _, _, llr = make_frames(N, K, 20, 1.5, stream=42)
    flip = llr * (1 - 2 * x.astype(np.float32))
    for bits, frac in ((8, 3), (6, 1)):
        a = oracle.decode_quant(llr, fz, bits=bits, frac=frac,
                                early_stop=False, soft=True)
        b = oracle.decode_quant(flip, fz, bits=bits, frac=frac,
                                early_stop=False, soft=True)
        assert np.array_equal(b["soft"], a["soft"] * (1 - 2 * u.astype(np.int32)))


def test_fine_format_decides_as_fp32():
    N, K = 1024, 512
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, 200, 2.5, stream=43)
    for mode in (dict(early_stop=False), dict(early_stop=True, freezing=True)):
        a = oracle.decode_quant(llr, fz, bits=16, frac=8, **mode)
        b = oracle.decode(llr, fz, **mode)
        same = (a["uhat"] == b["uhat"]).all(axis=1)
        assert same.mean() >= 0.95, mode
