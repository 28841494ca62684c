"""GPU parity of the unrolled decoder and its adjoint against the oracle,
through the C-ABI.

Bar: forward outputs equal to the FP32 oracle's (same operation order, so
the same values).  Gradients element by element, for every (t, j, dir) of
the scale gradient and every LLR gradient:

    |g - r| <= 1e-3 |r| + n (u A + eta)

r is the oracle's gradient (of the same FP32 forward, accumulated in FP64;
and, separately, the FP64 oracle's), A the oracle's sum of the magnitudes of
the terms that element adds up (``oracle.unrolled_grad_mag``), u = 2^-24 and
n = 6 m T + log2(N) + 16 the roundings along the longest path of the FP32
adjoint (an alpha product and up to five sums per stage and iteration, the
per-frame tree sum and the final product), and eta = 2^-126 the absolute
error of a rounding in FP32's subnormal range (terms below it underflow).
The second term is the worst-case FP32 rounding of that element's sum: it
is a small fraction of |r| for well-conditioned elements and only grows
where the terms cancel.
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_04979_amd as pbp
    pbp.lib()
    return pbp, torch


_codes = {}


def code_of(pbp, N, K):
    if (N, K) not in _codes:
        _codes[(N, K)] = pbp.Code(N, K, frozen_mask(N, K))
    return _codes[(N, K)]


U32 = 2.0 ** -24
ETA32 = 2.0 ** -126
RTOL = 1e-3


def n_roundings(N, T):
    m = N.bit_length() - 1
    return 6 * m * T + m + 16


def check_elementwise(name, g, r, A, N, T, extra=0):
    """Every element within RTOL |r| + n (u A + eta) (n grown by ``extra``
    roundings of the inputs); prints the worst one."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    A = np.asarray(A, np.float64)
    assert g.shape == r.shape == A.shape
    tol = RTOL * np.abs(r) + (n_roundings(N, T) + extra) * (U32 * A + ETA32)
    err = np.abs(g - r)
    ratio = np.where(tol > 0, err / np.where(tol > 0, tol, 1.0),
                     np.where(err > 0, np.inf, 0.0))
    i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    print(f"  {name}: worst element {tuple(int(v) for v in i)}: gpu {g[i]!r} "
          f"oracle {r[i]!r} |err| {err[i]:.3e} tol {tol[i]:.3e} "
          f"(err/tol {ratio[i]:.3f})", flush=True)
    assert ratio[i] <= 1.0, f"{name} element {i} outside tolerance"


def run_gpu(env, N, K, llr, alpha, dout):
    pbp, torch = env
    code = code_of(pbp, N, K)
    d_llr = torch.from_numpy(llr).cuda()
    d_alpha = torch.from_numpy(alpha.astype(np.float32)).cuda()
    out, ck = pbp.pbp_unrolled_forward(code, d_llr, d_alpha)
    da, dl, dfr = pbp.pbp_unrolled_backward(
        code, d_llr, d_alpha, ck, torch.from_numpy(dout.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return (out.cpu().numpy(), da.cpu().numpy(), dl.cpu().numpy(),
            dfr.cpu().numpy())


CASES = [
    # N, K, T, B, Eb/N0
    (2, 1, 4, 64, 1.0),
    (8, 4, 3, 100, 2.0),
    (64, 32, 5, 100, 1.5),
    (128, 64, 20, 64, 2.0),
    (256, 128, 7, 32, 2.0),
    (1024, 512, 20, 16, 2.5),
]


@pytest.mark.parametrize("N,K,T,B,ebn0", CASES)
def test_forward_and_gradient_parity(env, N, K, T, B, ebn0):
    print(f"[unrolled] N={N} K={K} T={T} B={B}", flush=True)
    m = N.bit_length() - 1
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, ebn0, stream=500 + N)
    rng = np.random.default_rng(N + T)
    alpha = rng.uniform(0.6, 1.1, size=(T, m, 2)).astype(np.float32)
    dout = (rng.standard_normal((B, N)) * (fz == 0)).astype(np.float32)
    out, da, dl, dfr = run_gpu(env, N, K, llr, alpha, dout)
    a64 = alpha.astype(np.float64)
    ref = oracle.unrolled_forward(llr, fz, a64, prec="f32")
    assert np.array_equal(out, ref)
    # same FP32 forward, FP64 adjoint
    rda, rdl = oracle.unrolled_grad(llr, fz, a64, dout, prec="f32")
    Ada, Adl = oracle.unrolled_grad_mag(llr, fz, a64, dout, prec="f32")
    check_elementwise("dalpha", da, rda, Ada, N, T)
    check_elementwise("dllr", dl, rdl, Adl, N, T)
    # per-frame shares add up to the total
    check_elementwise("sum of per-frame dalpha",
                      dfr.astype(np.float64).sum(axis=0), rda, Ada, N, T)
    # FP64 forward and adjoint
    rda64, rdl64 = oracle.unrolled_grad(llr, fz, a64, dout, prec="f64")
    check_elementwise("dalpha vs FP64", da, rda64, Ada, N, T)
    check_elementwise("dllr vs FP64", dl, rdl64, Adl, N, T)


@pytest.mark.parametrize("N,K,T", [(64, 32, 6), (1024, 512, 10)])
def test_default_scale_equals_plain_decode(env, N, K, T):
    """With every scale at 0.9375 the unrolled output equals pbp_decode's
    posterior at the information positions after T plain iterations."""
    pbp, torch = env
    m = N.bit_length() - 1
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, 40, 2.0, stream=88)
    code = code_of(pbp, N, K)
    d = torch.from_numpy(llr).cuda()
    alpha = torch.full((T, m, 2), 0.9375, dtype=torch.float32, device="cuda")
    out, _ = pbp.pbp_unrolled_forward(code, d, alpha, ckpt=False)
    dec = pbp.pbp_decode(code, d, max_iter=T, early_stop=False, soft=True)
    torch.cuda.synchronize()
    info = torch.from_numpy(fz == 0).cuda()
    assert torch.equal(out[:, info], dec["soft"][:, info])


def test_autograd_matches_direct_calls(env):
    pbp, torch = env
    N, K, T, B = 128, 64, 20, 256
    m = 7
    fz = frozen_mask(N, K)
    ebn0 = np.random.default_rng(5).uniform(1.0, 4.0, size=B)
    u, _, llr = make_frames(N, K, B, ebn0, stream=89)
    code = code_of(pbp, N, K)
    d_llr = torch.from_numpy(llr).cuda().requires_grad_(True)
    alpha = torch.full((T, m, 2), 0.9375, dtype=torch.float32,
                       device="cuda", requires_grad=True)
    info_pos = torch.from_numpy(np.flatnonzero(fz == 0)).cuda()
    u_info = torch.from_numpy(u[:, fz == 0].astype(np.float32)).cuda()
    out = pbp.unrolled_bp(d_llr, alpha, code)
    loss = pbp.info_bce(out, u_info, info_pos)
    loss.backward()
    # the same gradient through the oracle: dloss/dout of the mean BCE
    z = out.detach().cpu().numpy().astype(np.float64)[:, fz == 0]
    s = 1.0 - 2.0 * u[:, fz == 0]
    dz = -s / (1.0 + np.exp(s * z)) / z.size
    dout = np.zeros((B, N))
    dout[:, fz == 0] = dz
    a0 = np.full((T, m, 2), 0.9375)
    rda, rdl = oracle.unrolled_grad(llr, fz, a0, dout, prec="f32")
    Ada, Adl = oracle.unrolled_grad_mag(llr, fz, a0, dout, prec="f32")
    # torch forms the loss gradient in FP32 (a few roundings per element)
    # before the adjoint kernel sees it
    check_elementwise("dalpha (autograd)", alpha.grad.cpu().numpy(), rda, Ada,
                      N, T, extra=8)
    check_elementwise("dllr (autograd)", d_llr.grad.cpu().numpy(), rdl, Adl,
                      N, T, extra=8)


def test_training_steps_reduce_the_loss(env):
    """A few plain gradient steps on the scales lower the BCE of a fixed
    batch (the use the unrolled form exists for)."""
    pbp, torch = env
    N, K, T, B = 128, 64, 20, 512
    m = 7
    fz = frozen_mask(N, K)
    ebn0 = np.random.default_rng(6).uniform(1.0, 4.0, size=B)
    u, _, llr = make_frames(N, K, B, ebn0, stream=90)
    code = code_of(pbp, N, K)
    d_llr = torch.from_numpy(llr).cuda()
    alpha = torch.full((T, m, 2), 0.9375, dtype=torch.float32,
                       device="cuda", requires_grad=True)
    info_pos = torch.from_numpy(np.flatnonzero(fz == 0)).cuda()
    u_info = torch.from_numpy(u[:, fz == 0].astype(np.float32)).cuda()
    opt = torch.optim.SGD([alpha], lr=0.05)
    losses = []
    for _ in range(8):
        opt.zero_grad()
        loss = pbp.info_bce(pbp.unrolled_bp(d_llr, alpha, code), u_info,
                            info_pos)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    assert losses[-1] < losses[0]


@pytest.mark.parametrize("N,K", [(128, 64), (1024, 512)])
def test_training_batch_shape_sampled(env, N, K):
    """The training configurations (N = 128 and 1024, T = 20, 4096 frames,
    Eb/N0 uniform in [1, 4] dB): outputs and per-frame scale gradients of
    sampled frames against the oracle, and the frame sum."""
    pbp, torch = env
    T, B = 20, 4096
    m = N.bit_length() - 1
    print(f"[unrolled] training batch N={N} B={B}", flush=True)
    fz = frozen_mask(N, K)
    ebn0 = np.random.default_rng(7).uniform(1.0, 4.0, size=B)
    u, _, llr = make_frames(N, K, B, ebn0, stream=91)
    rng = np.random.default_rng(8)
    alpha = rng.uniform(0.8, 1.0, size=(T, m, 2)).astype(np.float32)
    dout = (rng.standard_normal((B, N)) * (fz == 0)).astype(np.float32)
    out, da, dl, dfr = run_gpu(env, N, K, llr, alpha, dout)
    idx = rng.choice(B, 12, replace=False)
    a64 = alpha.astype(np.float64)
    ref = oracle.unrolled_forward(llr[idx], fz, a64, prec="f32")
    assert np.array_equal(out[idx], ref)
    for f in idx[:6]:
        rda, rdl = oracle.unrolled_grad(llr[f:f + 1], fz, a64, dout[f:f + 1],
                                        prec="f32")
        Ada, Adl = oracle.unrolled_grad_mag(llr[f:f + 1], fz, a64,
                                            dout[f:f + 1], prec="f32")
        check_elementwise(f"frame {f} dalpha", dfr[f], rda, Ada, N, T)
        check_elementwise(f"frame {f} dllr", dl[f:f + 1], rdl, Adl, N, T)
    tot = dfr.astype(np.float64).sum(axis=0)
    assert np.allclose(da, tot, rtol=1e-6, atol=1e-6 * np.abs(tot).max())


def test_rejects_bad_arguments(env):
    pbp, torch = env
    code = code_of(pbp, 64, 32)
    llr = torch.zeros((4, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        pbp.pbp_unrolled_forward(code, llr, torch.ones((3, 5, 2),
                                                       device="cuda"))
    big = code_of(pbp, 2048, 1024)
    with pytest.raises(pbp.PbpError):
        pbp.pbp_unrolled_forward(
            big, torch.zeros((1, 2048), dtype=torch.float32, device="cuda"),
            torch.ones((2, 11, 2), dtype=torch.float32, device="cuda"),
            ckpt=False)
    out, _ = pbp.pbp_unrolled_forward(
        code, torch.zeros((0, 64), dtype=torch.float32, device="cuda"),
        torch.ones((2, 6, 2), dtype=torch.float32, device="cuda"), ckpt=False)
    assert out.shape == (0, 64)


@pytest.mark.parametrize("N,K,T,B", [(8, 4, 3, 30), (64, 32, 5, 20),
                                     (1024, 512, 6, 4)])
def test_intermediate_messages(env, N, K, T, B):
    """The L messages the forward checkpoints (columns 2..m at the start of
    every iteration) against the FP32 oracle's, element by element at every
    (iteration, column, row): the same operation order gives the same
    values, so they are compared for equality, inside the 1e-5 relative bar
    everywhere; infinite (frozen) messages compare as infinities."""
    pbp, torch = env
    print(f"[unrolled] messages N={N} T={T} B={B}", flush=True)
    m = N.bit_length() - 1
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, 2.0, stream=600 + N)
    rng = np.random.default_rng(N + 7)
    alpha = rng.uniform(0.6, 1.1, size=(T, m, 2)).astype(np.float32)
    code = code_of(pbp, N, K)
    _, ck = pbp.pbp_unrolled_forward(code, torch.from_numpy(llr).cuda(),
                                     torch.from_numpy(alpha).cuda())
    torch.cuda.synchronize()
    ck = ck.cpu().numpy()                                  # (T, B, m-1, N)
    L, _ = oracle.unrolled_messages(llr, fz, alpha.astype(np.float64),
                                    prec="f32")
    ref = L[:, :T, 2:m + 1].transpose(1, 0, 2, 3)          # (T, B, m-1, N)
    assert ck.shape == ref.shape
    bad = ck != ref
    assert not bad.any(), np.argwhere(bad)[:5]
    fin = np.isfinite(ref)
    rel = np.abs(ck[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1e-30)
    assert rel.max(initial=0.0) <= 1e-5


def test_backward_leaves_checkpoints_unchanged(env):
    """The backward reads the checkpoints and keeps the adjoint state on
    chip: a second backward call on the same checkpoints gives the same
    gradients, bit for bit, and the checkpoints are unchanged."""
    pbp, torch = env
    N, K, T, B = 256, 128, 6, 24
    m = N.bit_length() - 1
    print(f"[unrolled] backward twice N={N} T={T}", flush=True)
    _, _, llr = make_frames(N, K, B, 2.0, stream=612)
    rng = np.random.default_rng(5)
    alpha = torch.from_numpy(rng.uniform(0.6, 1.1, size=(T, m, 2)).astype(
        np.float32)).cuda()
    dout = torch.from_numpy(rng.standard_normal((B, N)).astype(np.float32)).cuda()
    code = code_of(pbp, N, K)
    d_llr = torch.from_numpy(llr).cuda()
    _, ck = pbp.pbp_unrolled_forward(code, d_llr, alpha)
    ck0 = ck.clone()
    g1 = pbp.pbp_unrolled_backward(code, d_llr, alpha, ck, dout)
    g2 = pbp.pbp_unrolled_backward(code, d_llr, alpha, ck, dout)
    torch.cuda.synchronize()
    assert torch.equal(ck, ck0)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
