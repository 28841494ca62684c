"""Pins of the oracle's round-trip schedule (an L pass over stages m..1, then
an R pass over stages 1..m, per iteration; the other common reading of the
schedule of Section II-A), against what the mathematics fixes:

- the repetition code (K = 1): the frozen rows carry +inf, so one round trip
  with alpha = 1 delivers the information bit's ML posterior, the sum of the
  channel LLRs (the single sweep does not, in its first iteration);
- N = 2: one stage, so both schedules compute the same messages and only the
  PE count doubles;
- the rate-1 code: every L is 0, so the decisions are the channel's hard
  decisions re-encoded (F is an involution over GF(2)), and the stop test
  holds after one iteration;
- channel symmetry: flipping the LLR signs along a codeword flips every
  decision along its source word and leaves the iterations unchanged;
- the PE count: m N per iteration.
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames

RT = oracle.SCHEDULE_ROUND_TRIP


@pytest.mark.parametrize("N", [2, 4, 8, 64, 1024])
def test_repetition_code_posterior_is_the_llr_sum(N):
    rng = np.random.default_rng(N)
    frozen = np.ones(N, np.uint8)
    frozen[N - 1] = 0
    llr = rng.normal(0.0, 2.0, size=(8, N)).astype(np.float32)
    o = oracle.decode(llr, frozen, max_iter=1, early_stop=False, alpha=1.0,
                      prec="f64", soft=True, schedule=RT)
    want = llr.astype(np.float64).sum(axis=1)
    np.testing.assert_allclose(o["soft"][:, N - 1], want, rtol=1e-12,
                               atol=1e-12)
    assert np.array_equal(o["info"][:, 0], (want < 0).astype(np.uint8))
    assert (o["pe"] == (N.bit_length() - 1) * N).all()
    if N >= 4:
        # the single sweep's first iteration has seen only part of the LLRs
        s = oracle.decode(llr, frozen, max_iter=1, early_stop=False,
                          alpha=1.0, prec="f64", soft=True)
        assert not np.allclose(s["soft"][:, N - 1], want)


@pytest.mark.parametrize("K", [0, 1, 2])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_n2_equals_the_single_sweep(K, prec):
    rng = np.random.default_rng(K)
    frozen = np.array([1, 1] if K == 0 else ([1, 0] if K == 1 else [0, 0]),
                      np.uint8)
    llr = rng.normal(0.0, 1.5, size=(300, 2)).astype(np.float32)
    for es in (False, True):
        a = oracle.decode(llr, frozen, max_iter=5, early_stop=es, prec=prec,
                          soft=True, schedule=RT)
        b = oracle.decode(llr, frozen, max_iter=5, early_stop=es, prec=prec,
                          soft=True)
        assert np.array_equal(a["uhat"], b["uhat"])
        assert np.array_equal(a["iters"], b["iters"])
        assert np.array_equal(a["pe"], 2 * b["pe"])
        assert np.array_equal(a["soft"], b["soft"])


@pytest.mark.parametrize("N", [4, 16, 256])
def test_rate_one_closed_form(N):
    rng = np.random.default_rng(7)
    frozen = np.zeros(N, np.uint8)
    llr = rng.normal(0.0, 1.0, size=(50, N)).astype(np.float32)
    o = oracle.decode(llr, frozen, max_iter=10, early_stop=True, schedule=RT)
    hard = (llr < 0).astype(np.uint8)
    assert np.array_equal(o["uhat"], oracle.encode(hard))
    assert (o["iters"] == 1).all()


@pytest.mark.parametrize("N,K,ebn0", [(64, 32, 2.0), (256, 128, 2.5),
                                      (1024, 512, 2.0)])
def test_codeword_symmetry(N, K, ebn0):
    frozen = frozen_mask(N, K)
    u, x, llr = make_frames(N, K, 40, ebn0, stream=(9 << 16) + N)
    # the same noise around the all-zero codeword
    llr0 = (llr * (1.0 - 2.0 * x.astype(np.float32))).astype(np.float32)
    a = oracle.decode(llr0, frozen, max_iter=30, soft=True, schedule=RT)
    b = oracle.decode(llr, frozen, max_iter=30, soft=True, schedule=RT)
    assert np.array_equal(b["uhat"], a["uhat"] ^ u)
    assert np.array_equal(b["iters"], a["iters"])
    sign = 1.0 - 2.0 * u.astype(np.float32)
    assert np.array_equal(b["soft"], a["soft"] * sign)


def test_pe_count_and_rejected_options():
    N, K = 128, 64
    frozen = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, 30, 2.5, stream=(9 << 16) + 1)
    o = oracle.decode(llr, frozen, max_iter=20, schedule=RT)
    assert np.array_equal(o["pe"], o["iters"].astype(np.int64) * 7 * N)
    with pytest.raises(ValueError):
        oracle.decode(llr, frozen, freezing=True, schedule=RT)


def test_fp32_and_fp64_agree_statistically():
    """The FP32 round trip (what the GPU reproduces bit for bit) has its
    frame error rate inside the FP64 round trip's 95% interval."""
    from helpers import wilson
    N, K, B = 256, 128, 3000
    u, _, llr = make_frames(N, K, B, 2.5, stream=(9 << 16) + 77)
    fz = frozen_mask(N, K)
    a = oracle.decode(llr, fz, prec="f32", schedule=RT)
    b = oracle.decode(llr, fz, prec="f64", schedule=RT)
    ea = int(np.sum(np.any(a["uhat"] != u, axis=1)))
    eb = int(np.sum(np.any(b["uhat"] != u, axis=1)))
    lo, hi = wilson(eb, B)
    assert lo <= ea / B <= hi
    assert np.mean(np.all(a["uhat"] == b["uhat"], axis=1)) > 0.97
