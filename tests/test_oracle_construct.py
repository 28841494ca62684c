"""Pins of the oracle's code construction.

* Exact successive-cancellation erasure probabilities on the binary erasure
  channel, by brute force over every erasure pattern, equal the recursion's
  Bhattacharyya values (on the BEC they coincide), which fixes the index
  orientation (natural order, no bit reversal) and the 2i / 2i+1 branches.
* The decimal form (carrying w = 1 - z) equals the literal recursion
  z -> 2z - z^2, z -> z^2 evaluated exactly in rationals, and the literal
  recursion at several hundred digits at the full configuration sizes.
"""

from decimal import Decimal
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle


def gen_rows(m):
    """Rows of F^{(x)m} as bit masks: row i has bit j iff j is a subset of i."""
    n = 1 << m
    return [sum(1 << j for j in range(n) if (j & ~i) == 0) for i in range(n)]


def sc_erasure_probs(m, eps):
    """P(u_i undetermined | channel outputs, u_0..u_{i-1}) on BEC(eps), exact.

    u_i is undetermined iff row i of G restricted to the unerased positions
    lies in the GF(2) span of the restricted rows l > i.
    """
    n = 1 << m
    rows = gen_rows(m)
    probs = [Fraction(0)] * n
    for unerased in range(1 << n):
        k = bin(unerased).count("1")
        w = (1 - eps) ** k * eps ** (n - k)
        basis = {}  # leading bit -> vector
        for i in range(n - 1, -1, -1):
            v = rows[i] & unerased
            while v:
                hb = v.bit_length() - 1
                if hb in basis:
                    v ^= basis[hb]
                else:
                    break
            if v == 0:
                probs[i] += w          # in the span: erased
            else:
                basis[v.bit_length() - 1] = v
    return probs


def literal_recursion(m, z0):
    z = [z0]
    for _ in range(m):
        z = [v for zi in z for v in (2 * zi - zi * zi, zi * zi)]
    return z


@pytest.mark.parametrize("m", [1, 2, 3, 4])
@pytest.mark.parametrize("eps", [Fraction(1, 2), Fraction(1, 3)])
def test_recursion_equals_bec_sc_erasure(m, eps):
    assert sc_erasure_probs(m, eps) == literal_recursion(m, eps)


def test_hand_values_n8():
    # BEC(1/2), N = 8: z = [255, 225, 207, 81, 175, 49, 31, 1] / 256 and the
    # four best positions {3, 5, 6, 7}
    z = literal_recursion(3, Fraction(1, 2))
    assert z == [Fraction(v, 256) for v in (255, 225, 207, 81, 175, 49, 31, 1)]
    zd, wd = oracle.bhattacharyya(3, "0.5")
    assert [float(v) for v in zd] == [float(v) for v in z]
    order = sorted(range(8), key=lambda i: (-z[i], i))
    assert sorted(order[4:]) == [3, 5, 6, 7]


@pytest.mark.parametrize("m", [2, 5, 7])
def test_decimal_form_equals_exact_rationals(m):
    z0 = Fraction(1, 3)
    exact = literal_recursion(m, z0)
    zd, wd = oracle.bhattacharyya(m, Decimal(1) / Decimal(3))
    for e, zi, wi in zip(exact, zd, wd):
        ez = float(e)
        assert abs(float(zi) - ez) <= 1e-15 * max(ez, 1e-300)
        assert abs(float(wi) - float(1 - e)) <= 1e-15 * max(float(1 - e), 1e-300)


@pytest.mark.parametrize("N,K", [(64, 32), (128, 64), (256, 85), (256, 128),
                                 (256, 213), (1024, 341), (1024, 512),
                                 (1024, 853)])
def test_ranking_equals_literal_recursion_high_precision(N, K):
    m = N.bit_length() - 1
    with mpmath.workdps(600):
        z0 = mpmath.exp(-mpmath.mpf(K) / N)
        z = literal_recursion(m, z0)
        order = sorted(range(N), key=lambda i: (-z[i], i))
    want = np.zeros(N, np.uint8)
    want[order[:N - K]] = 1
    got, gap = oracle.construct(N, K, 0.0)
    assert np.array_equal(np.array(got, np.uint8), want)
    assert gap is not None and gap > 1e-4


@pytest.mark.parametrize("N,K,dps,gap_want", [
    (4096, 1365, 2500, 9.560243e-4), (4096, 2048, 2500, 3.328686e-2),
    (4096, 3413, 2500, 2.350008e-2), (16384, 8192, 8000, 2.259419e-3)])
def test_long_code_ranking_equals_literal_recursion(N, K, dps, gap_want):
    """The long codes of the mixed and long-code workloads: the literal
    recursion on z alone, at enough digits that no z rounds to 1 (1 - z
    reaches 1e-2243 at (4096, 1365) and 1e-6637 at (16384, 8192)), ranks
    the positions as the oracle's logit recursion does; the boundary gap in
    logits is recorded (the smallest of all configured codes is 9.6e-4)."""
    m = N.bit_length() - 1
    with mpmath.workdps(dps):
        z0 = mpmath.exp(-mpmath.mpf(K) / N)
        z = literal_recursion(m, z0)
        assert min(1 - v for v in z) > 0
        order = sorted(range(N), key=lambda i: (-z[i], i))
        lo, hi = z[order[N - K - 1]], z[order[N - K]]
        gap = float(mpmath.log(lo / (1 - lo)) - mpmath.log(hi / (1 - hi)))
    want = np.zeros(N, np.uint8)
    want[order[:N - K]] = 1
    got, ogap = oracle.construct(N, K, 0.0)
    assert np.array_equal(np.array(got, np.uint8), want)
    assert abs(gap - gap_want) <= 1e-6 * gap_want
    assert abs(ogap - gap) <= 1e-9 * gap


def test_config_code_facts():
    fz, gap = oracle.construct(64, 32, 0.0)
    assert sum(fz) == 32
    fz = np.array(oracle.construct(1024, 512, 0.0)[0])
    info = np.flatnonzero(fz == 0)
    assert info.size == 512 and info[0] == 127 and info[-1] == 1023
    fz = np.array(oracle.construct(16384, 8192, 0.0)[0])
    assert fz.sum() == 8192 and fz[-1] == 0 and fz[0] == 1


def test_degenerate_rates():
    assert oracle.construct(8, 0)[0] == [1] * 8
    assert oracle.construct(8, 8)[0] == [0] * 8
    assert oracle.construct(2, 1)[0] == [1, 0]
