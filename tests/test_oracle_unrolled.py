"""Pins of the oracle's unrolled (trainable) decoder and its gradient.

* With every scale at 0.9375 the unrolled forward equals plain T-iteration
  BP of eq. (1) (bit-exact in FP32 and FP64).
* N = 2 closed forms: R(1, column 2) = y1 + aR * y0 in the last iteration,
  so d/d aR = y0, d/d y0 = aR, d/d y1 = 1 and every other scale has zero
  gradient.
* Central finite differences of the FP64 forward (h = 1e-4), with kinks of
  the min screened out by comparing against a half step.
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("N,K,T", [(8, 4, 3), (64, 32, 5), (128, 64, 20),
                                   (1024, 512, 4)])
def test_unrolled_at_default_scale_equals_plain_bp(prec, N, K, T):
    m = N.bit_length() - 1
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, 20, 2.0, stream=71)
    alpha = np.full((T, m, 2), 0.9375)
    out = oracle.unrolled_forward(llr, fz, alpha, prec=prec)
    ref = oracle.decode(llr, fz, max_iter=T, early_stop=False, soft=True,
                        prec=prec)
    info = fz == 0
    assert np.array_equal(out[:, info], ref["soft"][:, info])


def test_n2_gradient_closed_form():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((50, 2)).astype(np.float32) * 2
    fz = np.array([1, 0], np.uint8)
    T = 4
    alpha = rng.uniform(0.5, 1.2, size=(T, 1, 2))
    out = oracle.unrolled_forward(y, fz, alpha)
    aR = alpha[T - 1, 0, 1]
    y0 = y[:, 0].astype(np.float64)
    assert np.allclose(out[:, 1], y[:, 1] + aR * y0, rtol=1e-15, atol=0)
    dout = np.zeros((50, 2))
    dout[:, 1] = rng.standard_normal(50)
    da, dl = oracle.unrolled_grad(y, fz, alpha, dout)
    want = np.zeros_like(da)
    want[T - 1, 0, 1] = np.sum(dout[:, 1] * y0)
    assert np.allclose(da, want, rtol=1e-13, atol=1e-13)
    assert np.allclose(dl[:, 1], dout[:, 1], rtol=1e-15)
    assert np.allclose(dl[:, 0], dout[:, 1] * aR, rtol=1e-15)


def _fd_check(N, K, T, B, seed):
    m = N.bit_length() - 1
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, 1.5, stream=seed)
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(0.7, 1.1, size=(T, m, 2))
    dout = rng.standard_normal((B, N)) * (fz == 0)

    def loss(a):
        return float(np.sum(dout * oracle.unrolled_forward(llr, fz, a)))

    da, _ = oracle.unrolled_grad(llr, fz, alpha, dout)
    h = 1e-4
    checked = 0
    for idx in np.ndindex(alpha.shape):
        e = np.zeros_like(alpha)
        e[idx] = h
        fd1 = (loss(alpha + e) - loss(alpha - e)) / (2 * h)
        fd2 = (loss(alpha + e / 2) - loss(alpha - e / 2)) / h
        if abs(fd1 - fd2) > 1e-6 * max(1.0, abs(fd1)):
            continue                    # a min switched inside the step
        checked += 1
        assert abs(da[idx] - fd1) <= 1e-6 * max(1.0, abs(fd1)), idx
    return checked, alpha.size


@pytest.mark.parametrize("N,K,T,B", [(8, 4, 3, 4), (16, 8, 4, 3), (64, 32, 3, 2)])
def test_alpha_gradient_matches_central_differences(N, K, T, B):
    checked, total = _fd_check(N, K, T, B, seed=80 + N)
    assert checked >= 0.8 * total


def test_llr_gradient_matches_central_differences():
    N, K, T, B = 16, 8, 4, 2
    m = 4
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, 1.5, stream=91)
    llr = llr.astype(np.float64)
    rng = np.random.default_rng(91)
    alpha = rng.uniform(0.7, 1.1, size=(T, m, 2))
    dout = rng.standard_normal((B, N)) * (fz == 0)
    _, dl = oracle.unrolled_grad(llr.astype(np.float32), fz, alpha, dout)
    # the forward takes FP32 LLRs, so differentiate with a step that FP32
    # represents exactly around each value
    checked = 0
    for f in range(B):
        for i in range(N):
            x = np.float32(llr[f, i])
            h = np.float32(2.0 ** (np.floor(np.log2(abs(x) + 1e-30)) - 12))
            vals = []
            for s in (h, -h, h / 2, -h / 2):
                l2 = llr.astype(np.float32).copy()
                l2[f, i] = x + s
                vals.append(float(np.sum(dout * oracle.unrolled_forward(l2, fz, alpha))))
            fd1 = (vals[0] - vals[1]) / (2 * float(h))
            fd2 = (vals[2] - vals[3]) / float(h)
            if abs(fd1 - fd2) > 1e-6 * max(1.0, abs(fd1)):
                continue
            checked += 1
            assert abs(dl[f, i] - fd1) <= 1e-5 * max(1.0, abs(fd1)), (f, i)
    assert checked >= 0.8 * B * N


def test_magnitude_sums_n2_closed_form_and_bound():
    """unrolled_grad_mag: at N = 2 the only terms are dout * y0 (scale),
    dout (y1) and dout * aR (y0), so the sums are their magnitudes; at any
    size every sum is at least the gradient's magnitude (triangle
    inequality), with the same zero pattern, and equals it when every
    term has one sign (dout >= 0 on a noiseless all-zero word, where every
    message is positive)."""
    rng = np.random.default_rng(4)
    y = rng.standard_normal((40, 2)).astype(np.float32) * 2
    fz = np.array([1, 0], np.uint8)
    T = 3
    alpha = rng.uniform(0.5, 1.2, size=(T, 1, 2))
    dout = np.zeros((40, 2))
    dout[:, 1] = rng.standard_normal(40)
    Aa, Al = oracle.unrolled_grad_mag(y, fz, alpha, dout, prec="f64")
    aR = alpha[T - 1, 0, 1]
    want = np.zeros_like(Aa)
    want[T - 1, 0, 1] = np.sum(np.abs(dout[:, 1] * y[:, 0]))
    assert np.allclose(Aa, want, rtol=1e-13, atol=0)
    assert np.allclose(Al[:, 1], np.abs(dout[:, 1]), rtol=1e-15)
    assert np.allclose(Al[:, 0], np.abs(dout[:, 1]) * aR, rtol=1e-15)

    N, K, T, B = 64, 32, 5, 6
    m = 6
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, 1.5, stream=92)
    alpha = rng.uniform(0.7, 1.1, size=(T, m, 2))
    dout = rng.standard_normal((B, N)) * (fz == 0)
    da, dl = oracle.unrolled_grad(llr, fz, alpha, dout)
    Aa, Al = oracle.unrolled_grad_mag(llr, fz, alpha, dout)
    for g, A in ((da, Aa), (dl, Al)):
        assert (A >= np.abs(g) * (1 - 1e-12)).all()
        assert np.array_equal(A == 0, g == 0)
    # one sign throughout: the all-zero codeword without noise
    pos = np.full((2, N), 3.0, np.float32)
    dpos = np.abs(rng.standard_normal((2, N))) * (fz == 0)
    da, dl = oracle.unrolled_grad(pos, fz, alpha, dpos)
    Aa, Al = oracle.unrolled_grad_mag(pos, fz, alpha, dpos)
    assert np.allclose(Aa, da, rtol=1e-12, atol=0)
    assert np.allclose(Al, dl, rtol=1e-12, atol=0)


def test_messages_n2_closed_forms():
    """Every message of the N = 2 graph, iteration by iteration: with the
    frozen prior +inf at row 0 and 0 at row 1, L(column 1) = (aL y1, aL y0),
    R(column 2) = (aR g(y0, y1), y1 + aR y0), g(x, y) = sign(x) sign(y)
    min(|x|, |y|); the channel column and the prior column never change."""
    rng = np.random.default_rng(11)
    y = (rng.standard_normal((40, 2)) * 2).astype(np.float32)
    fz = np.array([1, 0], np.uint8)
    T = 3
    alpha = rng.uniform(0.5, 1.2, size=(T, 1, 2))
    L, R = oracle.unrolled_messages(y, fz, alpha)
    y0, y1 = y[:, 0].astype(np.float64), y[:, 1].astype(np.float64)
    g = np.sign(y0) * np.sign(y1) * np.minimum(np.abs(y0), np.abs(y1))
    # the initial state: zeros but for the prior column
    assert np.all(L[:, 0, :2] == 0) and np.all(R[:, 0] == 0)
    assert np.all(L[:, 0, 2, 0] == np.inf) and np.all(L[:, 0, 2, 1] == 0)
    for t in range(1, T + 1):
        aL, aR = alpha[t - 1, 0]
        assert np.all(L[:, t, 2, 0] == np.inf) and np.all(L[:, t, 2, 1] == 0)
        assert np.array_equal(R[:, t, 1], y.astype(np.float64))
        assert np.allclose(L[:, t, 1, 0], aL * y1, rtol=1e-15, atol=0)
        assert np.allclose(L[:, t, 1, 1], aL * y0, rtol=1e-15, atol=0)
        assert np.allclose(R[:, t, 2, 0], aR * g, rtol=1e-15, atol=0)
        assert np.allclose(R[:, t, 2, 1], y1 + aR * y0, rtol=1e-15, atol=0)


def _column_bits(u):
    """Bits carried at every column of the graph for source words u (B, N):
    column m+1 holds u; stage j maps column j+1 to column j by
    v_j[a] = v_{j+1}[a] ^ v_{j+1}[a + h], v_j[a + h] = v_{j+1}[a + h] with
    h = N / 2^j, so column 1 holds the codeword."""
    B, N = u.shape
    m = N.bit_length() - 1
    v = np.zeros((B, m + 2, N), np.uint8)
    v[:, m + 1] = u
    for j in range(m, 0, -1):
        h = N >> j
        v[:, j] = v[:, j + 1]
        for a in range(N):
            if not a & h:
                v[:, j, a] ^= v[:, j + 1, a + h]
    return v


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("N,K,T", [(8, 4, 3), (64, 32, 4), (256, 128, 3)])
def test_messages_follow_codeword_symmetry(prec, N, K, T):
    """Flipping the channel LLRs by a codeword x = u G flips every message at
    column c, row i, by the bit the graph carries there (eq. (1) is odd in
    each operand and the frozen bits of u are 0), exactly, in every
    iteration; the last column's R equals the forward's output."""
    m = N.bit_length() - 1
    fz = frozen_mask(N, K)
    rng = np.random.default_rng(N)
    _, _, llr = make_frames(N, K, 6, 1.5, stream=72)
    u = np.zeros((6, N), np.uint8)
    u[:, fz == 0] = rng.integers(0, 2, size=(6, K))
    v = _column_bits(u)
    x = v[:, 1]
    assert np.array_equal(x, oracle.encode(u))
    alpha = rng.uniform(0.7, 1.1, size=(T, m, 2))
    L0, R0 = oracle.unrolled_messages(llr, fz, alpha, prec=prec)
    flip = llr * (1 - 2 * x.astype(np.float32))
    L1, R1 = oracle.unrolled_messages(flip, fz, alpha, prec=prec)
    s = (1 - 2 * v.astype(np.float64))[:, None]          # (B, 1, m+2, N)
    assert np.array_equal(L1, L0 * s)
    assert np.array_equal(R1, R0 * s)
    out = oracle.unrolled_forward(llr, fz, alpha, prec=prec)
    assert np.array_equal(R0[:, T, m + 1], out)
