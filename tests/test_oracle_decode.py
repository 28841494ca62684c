"""Pins of the oracle decoder, against what the paper and the mathematics fix.

* N = 2 closed forms of eq. (1) in every mode (the PE equations, alpha,
  operand order).
* Noiseless channel: correct bits, and closed forms for iterations and PE
  activations in every mode (schedule, skipping, walk, termination, count).
* Codeword symmetry: decoding LLR * (1 - 2x) for a codeword x gives the
  decisions of the original LLRs XOR u with identical iterations and PE
  counts (sign errors anywhere break it).
* Lemma 1 by brute force: a CSFG that passes eqs. (2)-(4) holds the ML
  source word of its constituent code.
* The walk of Section III and Fig. 5: checks follow decoded-bit order,
  a failed check moves to the next stage, and the (8,4) sequence of
  Fig. 5 (a)-(c) occurs.
* FP32 and FP64 builds agree statistically.
* Context from Section IV (not a pin of exact values): G-matrix early stop
  at 3 dB averages about 26 iterations for the (1024, 512) code.
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames, noiseless_llr, wilson

ALPHA = 0.9375
MODES = {
    "plain": dict(early_stop=False, freezing=False),
    "es": dict(early_stop=True, freezing=False),
    "es_frz_total": dict(early_stop=True, freezing=True, freeze_input=1),
    "es_frz_r": dict(early_stop=True, freezing=True, freeze_input=0),
    "frz_total": dict(early_stop=False, freezing=True, freeze_input=1),
    "es_frz_stage": dict(early_stop=True, freezing=True, freeze_walk=1),
    "es_frz_greedy": dict(early_stop=True, freezing=True, freeze_walk=2),
}


def _pairs(prec, n=400, seed=0):
    rng = np.random.default_rng(seed)
    y = (rng.standard_normal((n, 2)) * 3).astype(np.float32)
    return y


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mode", list(MODES))
def test_n2_rate_half_closed_form(prec, mode):
    # u0 frozen, u1 information: R at (1, column 2) = y1 + alpha*y0
    y = _pairs(prec)
    fz = np.array([1, 0], np.uint8)
    r = oracle.decode(y, fz, max_iter=7, prec=prec, **MODES[mode])
    dt = np.float32 if prec == "f32" else np.float64
    y0, y1 = y[:, 0].astype(dt), y[:, 1].astype(dt)
    u1 = (y1 + dt(ALPHA) * y0 < 0).astype(np.uint8)
    assert np.array_equal(r["uhat"][:, 0], np.zeros_like(u1))
    assert np.array_equal(r["uhat"][:, 1], u1)
    # the G-matrix stop holds at t = 1 iff both channel-side decisions agree
    x0 = (y0 + dt(ALPHA) * y1 < 0)
    es_ok = x0 == (u1 == 1)
    kw = MODES[mode]
    if not kw["early_stop"] and not kw["freezing"]:
        want = np.full(len(y), 7)
    elif not kw["freezing"]:
        want = np.where(es_ok, 1, 7)
    else:
        # row 0 can be frozen from the first check on unless eq. (2) is
        # taken on R alone and g(y0, y1) < 0; the second check (row 1, an
        # information bit) always passes and ends the decoding
        row0 = np.ones(len(y), bool) if kw.get("freeze_input", 1) == 1 \
            else (y0 * y1 >= 0)
        if kw.get("freeze_walk", 0) == 2:
            done = np.where(row0, 1, 7)     # both rows in one sweep
        else:
            done = np.where(row0, 2, 7)
        want = np.minimum(np.where(es_ok, 1, 7), done) if kw["early_stop"] else done
    assert np.array_equal(r["iters"], want)
    assert np.array_equal(r["pe"], want)    # one PE, never skipped at stage 1


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mode", list(MODES))
def test_n2_rate_one_closed_form(prec, mode):
    # no frozen bit: plain hard-decision decoding, u = (x0 ^ x1, x1)
    y = _pairs(prec, seed=1)
    r = oracle.decode(y, np.zeros(2, np.uint8), max_iter=5, prec=prec,
                      **MODES[mode])
    x = (y < 0).astype(np.uint8)
    assert np.array_equal(r["uhat"][:, 0], x[:, 0] ^ x[:, 1])
    assert np.array_equal(r["uhat"][:, 1], x[:, 1])


def noiseless_closed_form(mode, N, max_iter):
    m = N.bit_length() - 1
    kw = MODES[mode]
    walk = kw.get("freeze_walk", 0)
    if not kw["freezing"]:
        it = 1 if kw["early_stop"] else max_iter
        return it, it * m * N // 2
    if walk == 2:                       # greedy: both stage-1 CSFGs at once
        return 1, N // 2
    if walk == 1:                       # one freeze per stage
        return (1, N - 1) if kw["early_stop"] else (2, N - 1 + N // 2)
    one = N // 2 + (m - 1) * N // 4     # stage 1, then half of every stage
    return (1, one) if kw["early_stop"] else (2, one + N // 2)


@pytest.mark.parametrize("N", [2, 4, 8, 64, 1024])
@pytest.mark.parametrize("mode", list(MODES))
def test_noiseless_closed_forms(N, mode):
    K = N // 2
    u, x, _ = make_frames(N, K, 8, 3.0, stream=7)
    llr = noiseless_llr(x)
    r = oracle.decode(llr, frozen_mask(N, K), max_iter=40, **MODES[mode])
    it, pe = noiseless_closed_form(mode, N, 40)
    assert np.array_equal(r["uhat"], u)
    assert np.all(r["iters"] == it)
    assert np.all(r["pe"] == pe)


@pytest.mark.parametrize("N,K,ebn0,B", [(64, 32, 2.5, 300), (1024, 512, 2.5, 40)])
@pytest.mark.parametrize("mode", ["plain", "es", "es_frz_total", "es_frz_r",
                                  "es_frz_stage", "frz_total"])
def test_codeword_symmetry(N, K, ebn0, B, mode):
    fz = frozen_mask(N, K)
    zero = np.zeros((B, N), np.uint8)
    _, _, llr0 = make_frames(N, K, B, ebn0, stream=21)
    # llr0 belongs to a random codeword; strip it to the all-zero word
    u, x, _ = make_frames(N, K, B, ebn0, stream=21)
    llr_zero = (llr0 * (1 - 2 * x.astype(np.float32))).astype(np.float32)
    u2, x2, _ = make_frames(N, K, B, ebn0, stream=22)
    llr_flip = (llr_zero * (1 - 2 * x2.astype(np.float32))).astype(np.float32)
    kw = dict(max_iter=40, **MODES[mode])
    a = oracle.decode(llr_zero, fz, soft=True, **kw)
    b = oracle.decode(llr_flip, fz, soft=True, **kw)
    # hard decisions on exactly-zero messages break the symmetry; there are
    # none on these inputs
    assert not np.any(a["soft"] == 0)
    assert np.array_equal(a["uhat"] ^ u2, b["uhat"])
    assert np.array_equal(a["iters"], b["iters"])
    assert np.array_equal(a["pe"], b["pe"])
    assert np.array_equal(np.abs(a["soft"]), np.abs(b["soft"]))
    del zero


def _ml_value(msgs, frozen, nlog):
    """Largest correlation sum((1 - 2x) R) over every codeword x = uG of
    the constituent code (frozen rows of u fixed to 0), by enumeration with
    the explicit Kronecker matrix."""
    n = 1 << nlog
    G = np.ones((1, 1), np.int64)
    for _ in range(nlog):
        G = np.kron(G, np.array([[1, 0], [1, 1]], np.int64))
    us = (np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1
    us = us[~np.any(us & frozen[None, :].astype(np.int64), axis=1)]
    xs = (us @ G) % 2
    return float(np.max((1 - 2 * xs) @ msgs))


def test_lemma1_brute_force():
    rng = np.random.default_rng(5)
    passed = 0
    for trial in range(1500):
        nlog = int(rng.integers(1, 5))
        n = 1 << nlog
        frozen = (rng.random(n) < rng.random()).astype(np.uint8)
        msgs = rng.standard_normal(n) * rng.uniform(0.2, 4)
        ok, xh, uh = oracle.csfg_check(msgs, frozen)
        assert np.array_equal(xh, (msgs < 0).astype(np.uint8))
        assert np.array_equal(uh, oracle.encode(xh))
        assert ok == (not np.any(uh & frozen))
        if ok:
            passed += 1
            val = float(np.sum((1 - 2 * xh.astype(np.float64)) * msgs))
            assert np.isclose(val, np.sum(np.abs(msgs)))
            assert val >= _ml_value(msgs, frozen, nlog) - 1e-12
    assert passed > 100


def _walk_invariants(trace, m, greedy=False, one_per_iter=True):
    """Checks of one frame's freezing trace against Section III's rules:
    at stage j the checked CSFG is the first one not yet frozen, where the
    frozen CSFGs of a stage are those passed there or lying inside a CSFG
    passed at an earlier stage; stages are visited left to right."""
    frozen_upto = {j: 0 for j in range(1, m + 1)}
    last_t, last_j, passed_in_t = 0, 0, False
    for (_, t, j, k, ok) in trace:
        if t != last_t:
            last_t, last_j, passed_in_t = t, 0, False
        assert j >= last_j
        if one_per_iter:
            assert not passed_in_t
        for jj in range(1, j + 1):
            for j0 in range(1, jj):
                frozen_upto[jj] = max(frozen_upto[jj],
                                      frozen_upto[j0] << (jj - j0))
        assert k == frozen_upto[j]
        if ok:
            frozen_upto[j] = k + 1
            passed_in_t = True
        last_j = j


def test_walk_follows_section3_and_fig5():
    N, K = 8, 4
    fz = frozen_mask(N, K)
    assert list(np.flatnonzero(fz == 0)) == [3, 5, 6, 7]
    fig5 = None
    for stream, ebn0 in ((31, 1.0), (32, 2.0), (33, 3.0)):
        u, x, llr = make_frames(N, K, 400, ebn0, stream=stream)
        r = oracle.decode(llr, fz, early_stop=False, freezing=True, trace=True)
        tr = r["trace"]
        for f in range(len(llr)):
            ft = tr[tr[:, 0] == f]
            _walk_invariants(ft, 3)
            seq = [tuple(e[1:]) for e in ft[:3]]
            if fig5 is None and len(seq) == 3 and seq[0] == (1, 1, 0, 1) \
                    and seq[1] == (2, 1, 1, 0) and seq[2][:3] == (2, 2, 2):
                fig5 = (stream, f)
    # Fig. 5: iteration 1 freezes the first CSFG at stage 1; iteration 2
    # fails on the second CSFG at stage 1 and moves on to the third CSFG at
    # stage 2
    assert fig5 is not None


@pytest.mark.parametrize("mode", ["es_frz_total", "es_frz_r", "es_frz_stage"])
def test_walk_invariants_n64(mode):
    N, K = 64, 32
    _, _, llr = make_frames(N, K, 200, 2.0, stream=41)
    r = oracle.decode(llr, frozen_mask(N, K), trace=True, **MODES[mode])
    for f in range(len(llr)):
        _walk_invariants(r["trace"][r["trace"][:, 0] == f], 6,
                         one_per_iter=MODES[mode].get("freeze_walk", 0) == 0)


def test_fp32_and_fp64_agree_statistically():
    N, K, B = 64, 32, 3000
    u, _, llr = make_frames(N, K, B, 2.5, stream=51)
    fz = frozen_mask(N, K)
    a = oracle.decode(llr, fz, prec="f32")
    b = oracle.decode(llr, fz, prec="f64")
    ea = int(np.sum(np.any(a["uhat"] != u, axis=1)))
    eb = int(np.sum(np.any(b["uhat"] != u, axis=1)))
    lo, hi = wilson(eb, B)
    assert lo <= ea / B <= hi
    assert np.mean(np.all(a["uhat"] == b["uhat"], axis=1)) > 0.97


def test_section4_context_iterations_at_3db():
    # Section IV: at 3 dB the proposed scheme needs 46% fewer iterations
    # than 40-iteration BP and 17% fewer than the G-matrix stop, which puts
    # the G-matrix stop near 0.54 * 40 / 0.83 = 26 iterations.
    N, K, B = 1024, 512, 200
    u, _, llr = make_frames(N, K, B, 3.0, stream=61)
    fz = frozen_mask(N, K)
    es = oracle.decode(llr, fz)
    frz = oracle.decode(llr, fz, freezing=True)
    plain = oracle.decode(llr, fz, early_stop=False)
    assert 23.0 < es["iters"].mean() < 29.0
    assert frz["iters"].mean() < es["iters"].mean()
    assert frz["pe"].mean() < 0.8 * es["pe"].mean()
    # no error-rate degradation (one-sided, loose at this sample size)
    e_plain = int(np.sum(np.any(plain["uhat"] != u, axis=1)))
    e_frz = int(np.sum(np.any(frz["uhat"] != u, axis=1)))
    assert e_frz <= e_plain + 3 * np.sqrt(max(e_plain, 1)) + 2
