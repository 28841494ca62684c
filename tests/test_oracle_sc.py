"""Pins of the oracle's successive-cancellation (SC) decoder, the decoder
whose scheduling tree Section III maps onto the BP factor graph.

* N = 2 closed forms: u0 from f(y0, y1), u1 from y1 + (1 - 2 u0) y0.
* Binary erasure channel, every erasure pattern of N <= 8 weighted exactly:
  the probability that the LLR reaching leaf i is an erasure equals the
  Bhattacharyya parameter z_i of the construction's recursion (SC with
  min-sum f and this g is exact on the BEC, and with the all-zero word every
  decision is correct, so the leaf statistics are the genie's).
* Rate-1 codes: SC decides u = xhat G, the re-encoded hard decisions.
* Repetition codes (only the last position free): the leaf LLR is the sum
  of the channel LLRs, the ML decision.
* Noiseless channel: every code decodes correctly; codeword symmetry.
"""

import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames, noiseless_llr


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_n2_closed_forms(prec):
    rng = np.random.default_rng(11)
    y = (rng.standard_normal((400, 2)) * 3).astype(np.float32)
    for frozen in ([0, 0], [1, 0]):
        fz = np.array(frozen, np.uint8)
        u = oracle.sc_decode(y, fz, prec=prec)
        y0, y1 = y[:, 0].astype(np.float64), y[:, 1].astype(np.float64)
        fv = np.sign(y0) * np.sign(y1) * np.minimum(abs(y0), abs(y1))
        u0 = np.zeros(400, np.uint8) if frozen[0] else (fv < 0).astype(np.uint8)
        assert np.array_equal(u[:, 0], u0)
        if prec == "f64":
            g = y1 + np.where(u0 == 1, -y0, y0)
        else:
            g = (y[:, 1] + np.where(u0 == 1, -y[:, 0], y[:, 0])).astype(np.float64)
        assert np.array_equal(u[:, 1], (g < 0).astype(np.uint8))


def _bhattacharyya_bec(m, eps):
    """z_i of x = u F^(x)m on BEC(eps), natural order (exact rationals)."""
    z = [eps]
    for _ in range(m):
        z = [v for a in z for v in (2 * a - a * a, a * a)]
    return z


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("eps", [Fraction(1, 2), Fraction(3, 10)])
def test_bec_leaf_erasure_probability_equals_bhattacharyya(m, eps):
    n = 1 << m
    pats = np.array(list(itertools.product([0, 1], repeat=n)), np.uint8)
    llr = np.where(pats == 1, 0.0, np.inf).astype(np.float32)  # 1 = erased
    fz = np.zeros(n, np.uint8)                                # all free
    u, leaf = oracle.sc_decode(llr, fz, prec="f64", leaf=True)
    assert not u.any()                  # the all-zero word is always decoded
    w = [eps ** int(p.sum()) * (1 - eps) ** int(n - p.sum()) for p in pats]
    erased = leaf == 0
    assert np.all((leaf == 0) | (leaf == np.inf))
    got = [sum((wi for wi, e in zip(w, erased[:, i]) if e), Fraction(0))
           for i in range(n)]
    want = _bhattacharyya_bec(m, eps)
    assert got == want
    # and the same values from the construction module's recursion
    zc, _ = oracle.bhattacharyya(m, str(float(eps)))
    assert np.allclose(np.array(zc, np.float64), [float(v) for v in want],
                       rtol=0, atol=1e-12)


@pytest.mark.parametrize("N", [4, 64, 1024])
def test_rate_one_decides_reencoded_hard_decisions(N):
    rng = np.random.default_rng(N)
    llr = (rng.standard_normal((50, N)) * 2).astype(np.float32)
    llr[llr == 0] = 1.0
    u = oracle.sc_decode(llr, np.zeros(N, np.uint8))
    assert np.array_equal(u, oracle.encode((llr < 0).astype(np.uint8)))


@pytest.mark.parametrize("N", [2, 16, 256])
def test_repetition_code_is_ml(N):
    rng = np.random.default_rng(N + 1)
    llr = (rng.standard_normal((300, N)) + 0.3).astype(np.float32)
    fz = np.ones(N, np.uint8)
    fz[-1] = 0
    u, leaf = oracle.sc_decode(llr, fz, prec="f64", leaf=True)
    s = llr.astype(np.float64).sum(axis=1)
    assert np.allclose(leaf[:, -1], s, rtol=1e-12, atol=1e-9)
    clear = np.abs(s) > 1e-6
    assert np.array_equal(u[clear, -1], (s[clear] < 0).astype(np.uint8))
    assert not u[:, :-1].any()


@pytest.mark.parametrize("N,K", [(8, 4), (64, 32), (1024, 512), (4096, 1365)])
def test_noiseless_and_codeword_symmetry(N, K):
    fz = frozen_mask(N, K)
    u, x, _ = make_frames(N, K, 40, 2.0, stream=31)
    for prec in ("f32", "f64"):
        assert np.array_equal(oracle.sc_decode(noiseless_llr(x), fz,
                                               prec=prec), u)
    # symmetry: the LLRs of codeword x, sign-flipped by x, decode to u ^ uhat
    # of the all-zero word's LLRs (exact; ties at exact zeros excepted)
    _, _, llr = make_frames(N, K, 40, 1.5, stream=32)
    z = np.zeros((40, N), np.uint8)
    u0 = oracle.sc_decode(llr * (1 - 2 * x.astype(np.float32)), fz)
    u1 = oracle.sc_decode(llr, fz)
    assert np.array_equal(u1 ^ u0, u ^ z) or np.any(llr == 0)
