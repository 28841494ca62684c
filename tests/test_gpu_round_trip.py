"""GPU parity of the round-trip schedule (pbp_decode_round_trip) against the
FP32 oracle's round trip, through the C-ABI.

Bar, as for the single sweep: information bits, iteration counts and PE
counts bit-exact; posteriors equal as FP32 values (-0 and +0 compare equal).
"""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames

pytestmark = pytest.mark.gpu

RT = oracle.SCHEDULE_ROUND_TRIP


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_04979_amd as pbp
    pbp.lib()
    return pbp, torch


_codes = {}


def code_of(pbp, N, K, frozen=None):
    key = (N, K, None if frozen is None else frozen.tobytes())
    if key not in _codes:
        _codes[key] = pbp.Code(N, K, frozen_mask(N, K) if frozen is None
                               else frozen)
    return _codes[key]


def run_both(env, N, K, llr, frozen=None, max_iter=40, alpha=0.9375,
             early_stop=True):
    pbp, torch = env
    fz = frozen_mask(N, K) if frozen is None else frozen
    code = code_of(pbp, N, K, frozen)
    d = torch.from_numpy(llr).cuda()
    g = pbp.pbp_decode_round_trip(code, d, max_iter=max_iter, alpha=alpha,
                                  early_stop=early_stop, soft=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    r = oracle.decode(llr, fz, max_iter=max_iter, early_stop=early_stop,
                      alpha=alpha, soft=True, schedule=RT)
    return g, r, fz


def assert_parity(g, r, fz):
    assert np.array_equal(g["info"], r["uhat"][:, fz == 0])
    assert np.array_equal(g["iters"], r["iters"])
    assert np.array_equal(g["pe"], r["pe"])
    assert (g["soft"] == r["soft"]).all(), np.argwhere(g["soft"] != r["soft"])[:5]


CASES = [
    (2, 1, 1.0, 64),
    (4, 2, 1.5, 100),
    (8, 4, 2.0, 200),
    (16, 8, 2.0, 200),
    (32, 16, 2.0, 200),
    (64, 32, 2.5, 300),
    (128, 64, 2.0, 200),
    (256, 85, 2.0, 100),
    (512, 256, 2.5, 80),
    (1024, 512, 3.0, 160),
    (1024, 512, 1.5, 64),
    (2048, 1024, 2.5, 40),
]


@pytest.mark.parametrize("N,K,ebn0,B", CASES)
@pytest.mark.parametrize("early_stop", [False, True])
def test_round_trip_parity(env, N, K, ebn0, B, early_stop):
    _, _, llr = make_frames(N, K, B, ebn0, stream=(11 << 16) + N + K)
    g, r, fz = run_both(env, N, K, llr, early_stop=early_stop)
    assert_parity(g, r, fz)


@pytest.mark.parametrize("N,K", [(16, 0), (16, 16), (64, 1), (64, 63),
                                 (1024, 1), (1024, 1024)])
def test_degenerate_rates(env, N, K):
    _, _, llr = make_frames(N, K, 40, 2.0, stream=(11 << 16) + 500 + K)
    g, r, fz = run_both(env, N, K, llr, max_iter=12)
    assert_parity(g, r, fz)


@pytest.mark.parametrize("max_iter,alpha", [(1, 0.9375), (3, 1.0), (17, 0.5)])
def test_options(env, max_iter, alpha):
    N, K = 256, 128
    _, _, llr = make_frames(N, K, 64, 1.5, stream=(11 << 16) + 900 + max_iter)
    g, r, fz = run_both(env, N, K, llr, max_iter=max_iter, alpha=alpha)
    assert_parity(g, r, fz)


def test_repetition_code_delivers_the_llr_sum(env):
    """One round trip of the K = 1 code with alpha = 1 gives the ML
    posterior (the sum of the LLRs), on the GPU as in the oracle."""
    N = 1024
    fz = np.ones(N, np.uint8)
    fz[N - 1] = 0
    rng = np.random.default_rng(3)
    llr = rng.normal(0.0, 2.0, size=(32, N)).astype(np.float32)
    g, r, _ = run_both(env, N, 1, llr, frozen=fz, max_iter=1, alpha=1.0,
                       early_stop=False)
    assert_parity(g, r, fz)
    np.testing.assert_allclose(g["soft"][:, N - 1],
                               llr.astype(np.float64).sum(axis=1), rtol=1e-4,
                               atol=1e-3)


def test_rejects_what_it_does_not_run(env):
    pbp, torch = env
    code = code_of(pbp, 1024, 512)
    d = torch.zeros((4, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(pbp.PbpError):
        pbp.pbp_decode(code, d, freezing=True, schedule="round_trip")
    long = code_of(pbp, 4096, 2048)
    d2 = torch.zeros((2, 4096), dtype=torch.float32, device="cuda")
    with pytest.raises(pbp.PbpError):
        pbp.pbp_decode(long, d2, schedule="round_trip")
    # an empty batch is a no-op
    e = pbp.pbp_decode(code, d[:0], schedule="round_trip")
    assert e["iters"].shape == (0,)


def test_large_batch_sampled_parity(env):
    """2^17 frames in one launch (several frames per workgroup); 256 sampled
    frames against the oracle."""
    pbp, torch = env
    N, K, B = 1024, 512, 1 << 17
    fz = frozen_mask(N, K)
    code = code_of(pbp, N, K)
    d = torch.empty((B, N), dtype=torch.float32, device="cuda")
    chunk = 1 << 14
    for lo in range(0, B, chunk):
        _, _, llr = make_frames(N, K, chunk, 3.0, stream=(11 << 16) + 7,
                                frame0=lo)
        d[lo:lo + chunk] = torch.from_numpy(llr).cuda()
    g = pbp.pbp_decode(code, d, soft=True, schedule="round_trip")
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(B, 256, replace=False))
    sel = torch.from_numpy(idx).cuda()
    gs = {k: v[sel].cpu().numpy() for k, v in g.items()}
    r = oracle.decode(d[sel].cpu().numpy(), fz, soft=True, schedule=RT)
    assert_parity(gs, r, fz)


def test_graph_capture_replays(env):
    """pbp_decode_round_trip captured once in a graph and replayed on new
    LLRs matches eager calls and the oracle, replay after replay: the frame
    counter the workgroups take frames from is left at zero for the next
    launch."""
    pbp, torch = env
    N, K, B = 1024, 512, 600
    print(f"[parity] round-trip graph replay N={N} B={B}", flush=True)
    fz = frozen_mask(N, K)
    code = code_of(pbp, N, K)
    _, _, llr0 = make_frames(N, K, B, 2.5, stream=(11 << 16) + 97)
    static_llr = torch.from_numpy(llr0).cuda()
    out = pbp.pbp_decode_round_trip(code, static_llr, soft=True)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pbp.pbp_decode_round_trip(code, static_llr, soft=True, out=out,
                                  stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pbp.pbp_decode_round_trip(code, static_llr, soft=True, out=out,
                                  stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        _, _, llr = make_frames(N, K, B, 2.0 + 0.5 * rep,
                                stream=(11 << 16) + 98 + rep)
        static_llr.copy_(torch.from_numpy(llr))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        eager = pbp.pbp_decode_round_trip(code, torch.from_numpy(llr).cuda(),
                                          soft=True)
        torch.cuda.synchronize()
        for k in got:
            assert np.array_equal(got[k], eager[k].cpu().numpy()), (rep, k)
        idx = np.arange(0, B, 50)
        r = oracle.decode(llr[idx], fz, soft=True, schedule=RT)
        assert_parity({k: v[idx] for k, v in got.items()}, r, fz)
