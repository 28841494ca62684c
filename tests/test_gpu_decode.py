"""GPU parity of the HIP path against the FP32 oracle, through the C-ABI.

Bar: information bits, iteration counts and PE counts bit-exact; posterior
(soft) outputs equal as FP32 values (the same operation order gives the
same bits; -0 and +0 compare equal); error rates of the GPU inside the FP64
oracle's 95% interval.
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames, noiseless_llr, wilson

pytestmark = pytest.mark.gpu

MODES = {
    "plain": dict(early_stop=False, freezing=False),
    "es": dict(early_stop=True, freezing=False),
    "es_frz_total": dict(early_stop=True, freezing=True, freeze_input=1),
    "es_frz_r": dict(early_stop=True, freezing=True, freeze_input=0),
    "frz_total": dict(early_stop=False, freezing=True, freeze_input=1),
    "es_frz_stage": dict(early_stop=True, freezing=True, freeze_walk=1),
    "es_frz_greedy": dict(early_stop=True, freezing=True, freeze_walk=2),
}


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


def gpu_decode(env, N, K, llr, max_iter=40, alpha=0.9375, **mode):
    pbp, torch = env
    code = code_of(pbp, N, K)
    d = torch.from_numpy(llr).cuda()
    o = pbp.pbp_decode(code, d, max_iter=max_iter, alpha=alpha, soft=True,
                       **mode)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def assert_parity(g, r, K, frozen):
    assert np.array_equal(g["info"], r["uhat"][:, frozen == 0])
    assert np.array_equal(g["iters"], r["iters"])
    assert np.array_equal(g["pe"], r["pe"])
    gs, rs = g["soft"], r["soft"]
    same = (gs == rs) | (np.isnan(gs) & np.isnan(rs))
    assert same.all(), np.argwhere(~same)[:5]


CASES = [
    # N, K, Eb/N0, frames
    (2, 1, 1.0, 64),
    (8, 4, 2.0, 200),
    (16, 8, 2.0, 200),
    (32, 11, 2.0, 200),
    (64, 32, 2.5, 400),
    (128, 64, 2.0, 200),
    (256, 85, 2.0, 100),
    (512, 256, 2.5, 60),
    (1024, 512, 3.0, 160),
    (1024, 512, 1.5, 64),
    (2048, 1024, 2.5, 16),
    (4096, 2048, 2.5, 12),
    (16384, 8192, 2.0, 3),
]


@pytest.mark.parametrize("N,K,ebn0,B", CASES)
@pytest.mark.parametrize("mode", list(MODES))
def test_decode_parity(env, N, K, ebn0, B, mode):
    print(f"[parity] N={N} K={K} ebn0={ebn0} B={B} mode={mode}", flush=True)
    fz = frozen_mask(N, K)
    u, x, llr = make_frames(N, K, B, ebn0, stream=1000 + N)
    kw = MODES[mode]
    mi = 60 if N >= 4096 else 40
    r = oracle.decode(llr, fz, max_iter=mi, soft=True, **kw)
    g = gpu_decode(env, N, K, llr, max_iter=mi, **kw)
    assert_parity(g, r, K, fz)


@pytest.mark.parametrize("N,K", [(16, 0), (16, 16), (64, 1), (64, 63)])
@pytest.mark.parametrize("mode", ["plain", "es", "es_frz_total", "es_frz_greedy"])
def test_degenerate_rates(env, N, K, mode):
    fz = frozen_mask(N, K)
    u, x, llr = make_frames(N, K, 50, 1.0, stream=77)
    r = oracle.decode(llr, fz, soft=True, **MODES[mode])
    g = gpu_decode(env, N, K, llr, **MODES[mode])
    assert_parity(g, r, K, fz)


@pytest.mark.parametrize("max_iter,alpha", [(1, 0.9375), (3, 1.0), (17, 0.5),
                                            (40, 0.8125)])
def test_options(env, max_iter, alpha):
    N, K = 256, 128
    fz = frozen_mask(N, K)
    u, x, llr = make_frames(N, K, 64, 2.0, stream=78)
    for mode in ("plain", "es_frz_total"):
        r = oracle.decode(llr, fz, max_iter=max_iter, alpha=alpha, soft=True,
                          **MODES[mode])
        g = gpu_decode(env, N, K, llr, max_iter=max_iter, alpha=alpha,
                       **MODES[mode])
        assert_parity(g, r, K, fz)


@pytest.mark.parametrize("N", [64, 1024, 16384])
def test_noiseless_closed_forms(env, N):
    K = N // 2
    u, x, _ = make_frames(N, K, 4, 3.0, stream=79)
    llr = noiseless_llr(x)
    m = N.bit_length() - 1
    g = gpu_decode(env, N, K, llr, **MODES["es_frz_total"])
    assert np.array_equal(g["info"], u[:, frozen_mask(N, K) == 0])
    assert np.all(g["iters"] == 1)
    assert np.all(g["pe"] == N // 2 + (m - 1) * N // 4)
    g = gpu_decode(env, N, K, llr, **MODES["plain"])
    assert np.all(g["pe"] == 40 * m * N // 2)


def test_encode_parity(env):
    pbp, torch = env
    for N, K in ((2, 1), (8, 4), (64, 32), (1024, 512), (4096, 1365),
                 (16384, 8192), (32, 0), (32, 32)):
        code = code_of(pbp, N, K)
        fz = frozen_mask(N, K)
        rng = np.random.default_rng(N + K)
        info = rng.integers(0, 2, size=(37, K)).astype(np.uint8)
        u = np.zeros((37, N), np.uint8)
        u[:, fz == 0] = info
        cw = pbp.pbp_encode(code, torch.from_numpy(info).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(cw.cpu().numpy(), oracle.encode(u))


def test_large_batch_sampled_parity(env):
    """The benchmark's launch shape (10^6 frames of the (1024, 512) code at
    3 dB, early stop + freezing, one launch), checked on sampled frames.  The
    inputs are made a chunk of frames at a time (the draws are per frame)."""
    pbp, torch = env
    N, K, B, chunk = 1024, 512, 10 ** 6, 1 << 17
    kw = MODES["es_frz_total"]
    fz = frozen_mask(N, K)
    code = code_of(pbp, N, K)
    idx = np.sort(np.random.default_rng(0).choice(B, 96, replace=False))
    llr_s = np.empty((len(idx), N), np.float32)
    u_s = np.empty((len(idx), N), np.uint8)
    d_llr = torch.empty((B, N), dtype=torch.float32, device="cuda")
    for lo in range(0, B, chunk):
        hi = min(B, lo + chunk)
        u, x, llr = make_frames(N, K, hi - lo, 3.0, stream=2024, frame0=lo,
                                frozen=fz)
        d_llr[lo:hi].copy_(torch.from_numpy(llr))
        sel = (idx >= lo) & (idx < hi)
        llr_s[sel] = llr[idx[sel] - lo]
        u_s[sel] = u[idx[sel] - lo]
    print(f"[parity] bench batch N={N} B={B}", flush=True)
    o = pbp.pbp_decode(code, d_llr, soft=True, **kw)
    torch.cuda.synchronize()
    ti = torch.from_numpy(idx).cuda()
    sub = {k: v[ti].cpu().numpy() for k, v in o.items()}
    del d_llr, o
    r = oracle.decode(llr_s, fz, soft=True, **kw)
    assert_parity(sub, r, K, fz)
    # error rate within the FP64 oracle's interval on the sample
    r64 = oracle.decode(llr_s, fz, prec="f64", **kw)
    e64 = int(np.sum(np.any(r64["uhat"] != u_s, axis=1)))
    lo_, hi_ = wilson(e64, len(idx))
    eg = float(np.mean(np.any(sub["info"] != u_s[:, fz == 0], axis=1)))
    assert lo_ - 0.02 <= eg <= hi_ + 0.02


def test_repeatable(env):
    N, K = 1024, 512
    u, x, llr = make_frames(N, K, 256, 2.5, stream=81)
    a = gpu_decode(env, N, K, llr, **MODES["es_frz_total"])
    b = gpu_decode(env, N, K, llr, **MODES["es_frz_total"])
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_rejects_bad_arguments(env):
    pbp, torch = env
    code = code_of(pbp, 64, 32)
    llr = torch.zeros((4, 64), dtype=torch.float32, device="cuda")
    for bad in (dict(max_iter=0), dict(freeze_input=2), dict(freeze_walk=3),
                dict(alpha=0.0), dict(alpha=float("inf"))):
        with pytest.raises(pbp.PbpError):
            pbp.pbp_decode(code, llr, **bad)
    with pytest.raises(TypeError):
        pbp.pbp_decode(code, llr.cpu())
    with pytest.raises(ValueError):
        pbp.pbp_decode(code, torch.zeros((4, 32), dtype=torch.float32,
                                         device="cuda"))
    # an empty batch enqueues nothing
    o = pbp.pbp_decode(code, torch.zeros((0, 64), dtype=torch.float32,
                                         device="cuda"))
    assert o["info"].shape == (0, 32)


@pytest.mark.parametrize("N,K,B", [(256, 128, 40), (1024, 512, 40),
                                   (4096, 2048, 6)])
def test_unaligned_buffers(env, N, K, B):
    """LLRs and posteriors at addresses that are not 16-byte aligned: the
    N = 1024 register decoder reads and writes them by words instead of
    16-byte vectors, and the generic kernel's first stage reads them one PE
    at a time instead of in 16-byte groups, with the same results."""
    pbp, torch = env
    fz = frozen_mask(N, K)
    u, x, llr = make_frames(N, K, B, 2.5, stream=83)
    code = code_of(pbp, N, K)
    buf = torch.zeros(B * N + 1, dtype=torch.float32, device="cuda")
    view = buf[1:].view(B, N)
    view.copy_(torch.from_numpy(llr))
    assert view.data_ptr() % 16 != 0
    sbuf = torch.zeros(B * N + 3, dtype=torch.float32, device="cuda")
    soft = sbuf[3:].view(B, N)
    kw = MODES["es_frz_total"]
    o = pbp.pbp_decode(code, view, soft=True, out={"soft": soft}, **kw)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in o.items()}
    r = oracle.decode(llr, fz, soft=True, **kw)
    assert_parity(g, r, K, fz)


def test_long_code_batch_sampled_parity(env):
    """The long-code benchmark's launch shape ((16384, 8192) code, 2.0 dB,
    10^5 frames in one launch, 60 iterations, early stop + freezing),
    checked on sampled frames; inputs made a chunk of frames at a time."""
    pbp, torch = env
    N, K, B, chunk = 16384, 8192, 10 ** 5, 1 << 13
    kw = MODES["es_frz_total"]
    fz = frozen_mask(N, K)
    code = code_of(pbp, N, K)
    idx = np.sort(np.random.default_rng(1).choice(B, 3, replace=False))
    llr_s = np.empty((len(idx), N), np.float32)
    d_llr = torch.empty((B, N), dtype=torch.float32, device="cuda")
    for lo in range(0, B, chunk):
        hi = min(B, lo + chunk)
        _, _, llr = make_frames(N, K, hi - lo, 2.0, stream=2025, frame0=lo,
                                frozen=fz)
        d_llr[lo:hi].copy_(torch.from_numpy(llr))
        sel = (idx >= lo) & (idx < hi)
        llr_s[sel] = llr[idx[sel] - lo]
    print(f"[parity] long batch N={N} B={B}", flush=True)
    o = pbp.pbp_decode(code, d_llr, max_iter=60, soft=True, **kw)
    torch.cuda.synchronize()
    ti = torch.from_numpy(idx).cuda()
    sub = {k: v[ti].cpu().numpy() for k, v in o.items()}
    del d_llr, o
    r = oracle.decode(llr_s, fz, max_iter=60, soft=True, **kw)
    assert_parity(sub, r, K, fz)


@pytest.mark.parametrize("N,K,B", [(1024, 512, 96), (2048, 1024, 24)])
def test_graph_capture_replays(env, N, K, B):
    """pbp_decode captured once in a graph and replayed on new LLRs (copied
    into the captured buffer between replays) matches eager calls and the
    oracle, replay after replay: the persistent kernel's frame counter and
    the long-code state slots are left ready for the next launch."""
    pbp, torch = env
    print(f"[parity] graph replay N={N} B={B}", flush=True)
    fz = frozen_mask(N, K)
    code = code_of(pbp, N, K)
    kw = MODES["es_frz_total"]
    u, x, llr0 = make_frames(N, K, B, 2.5, stream=97)
    static_llr = torch.from_numpy(llr0).cuda()
    out = pbp.pbp_decode(code, static_llr, soft=True, **kw)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pbp.pbp_decode(code, static_llr, soft=True, out=out, stream=s, **kw)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pbp.pbp_decode(code, static_llr, soft=True, out=out, stream=s, **kw)
    torch.cuda.synchronize()
    for rep in range(4):
        _, _, llr = make_frames(N, K, B, 2.0 + 0.5 * rep, stream=98 + rep)
        static_llr.copy_(torch.from_numpy(llr))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        eager = gpu_decode(env, N, K, llr, **kw)
        for k in got:
            assert np.array_equal(got[k], eager[k]), (rep, k)
        idx = np.arange(0, B, max(1, B // 6))
        r = oracle.decode(llr[idx], fz, soft=True, **kw)
        assert_parity({k: v[idx] for k, v in got.items()}, r, K, fz)


@pytest.mark.parametrize("mode", ["es_frz_total", "es", "frz_total",
                                  "es_frz_stage", "es_frz_r"])
def test_long_code_converging_frames(env, mode):
    """(16384, 8192) at 4.0 dB with 60 iterations: the frames converge (34
    to 41 iterations on the oracle), so the m = 14 kernel's freezing walk,
    its all-frozen exit and its early stop all act on noisy frames; bits,
    iterations, PE counts and posteriors against the FP32 oracle."""
    N, K = 16384, 8192
    print(f"[decode] N={N} 4.0 dB mode={mode}", flush=True)
    fz = frozen_mask(N, K)
    u, _, llr = make_frames(N, K, 6, 4.0, stream=77)
    g = gpu_decode(env, N, K, llr, max_iter=60, **MODES[mode])
    r = oracle.decode(llr, fz, max_iter=60, soft=True, **MODES[mode])
    assert_parity(g, r, K, fz)
    if mode == "es_frz_total":
        assert (r["iters"] < 60).all()
        assert (r["pe"] < 60 * 7 * N).all()
        assert np.array_equal(g["info"], u[:, fz == 0])


@pytest.mark.parametrize("N,K,B", [(1024, 512, 4096), (4096, 2048, 384)])
def test_one_handle_on_two_streams(env, N, K, B):
    """One handle decoding on two streams at once: each stream has its own
    workspace (the persistent kernel's frame counter, the long-code state
    slots), so overlapping decodes equal the same decodes made one after the
    other, repeat after repeat, and the oracle on sampled frames."""
    pbp, torch = env
    print(f"[decode] two streams N={N} B={B}", flush=True)
    fz = frozen_mask(N, K)
    code = code_of(pbp, N, K)
    kw = MODES["es_frz_total"]
    _, _, l1 = make_frames(N, K, B, 2.5, stream=131)
    _, _, l2 = make_frames(N, K, B, 3.0, stream=132)
    d1, d2 = torch.from_numpy(l1).cuda(), torch.from_numpy(l2).cuda()
    ref1 = pbp.pbp_decode(code, d1, soft=True, **kw)
    ref2 = pbp.pbp_decode(code, d2, soft=True, **kw)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(s1):
            o1 = pbp.pbp_decode(code, d1, soft=True, stream=s1, **kw)
        with torch.cuda.stream(s2):
            o2 = pbp.pbp_decode(code, d2, soft=True, stream=s2, **kw)
        torch.cuda.synchronize()
        for o, ref in ((o1, ref1), (o2, ref2)):
            for k in ref:
                assert torch.equal(o[k], ref[k]), (rep, k)
    idx = np.arange(0, B, B // 8)
    for llr, o in ((l1, o1), (l2, o2)):
        r = oracle.decode(llr[idx], fz, soft=True, **kw)
        assert_parity({k: v.cpu().numpy()[idx] for k, v in o.items()}, r, K,
                      fz)
    pbp.pbp_workspace_release(s1)
    pbp.pbp_workspace_release(s2)
    # a released stream gets a fresh workspace on its next decode
    with torch.cuda.stream(s1):
        o1 = pbp.pbp_decode(code, d1, soft=True, stream=s1, **kw)
    torch.cuda.synchronize()
    for k in ref1:
        assert torch.equal(o1[k], ref1[k]), k


def test_small_code_many_frames(env):
    """N = 64 without freezing runs one wavefront per frame in registers:
    a batch of 20000 frames (more wavefronts than the chip holds at once),
    both stop rules, every frame against the oracle, posteriors included."""
    N, K, B = 64, 32, 20000
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, 2.5, stream=2600)
    for mode in ("plain", "es"):
        print(f"[decode] small code, {B} frames, mode={mode}", flush=True)
        r = oracle.decode(llr, fz, max_iter=40, soft=True, **MODES[mode])
        g = gpu_decode(env, N, K, llr, max_iter=40, **MODES[mode])
        assert_parity(g, r, K, fz)
