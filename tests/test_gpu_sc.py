"""GPU parity of the successive-cancellation decoder (pbp_decode_sc) with the
oracle's, through the C-ABI: decided bits equal to the FP32 oracle's, and the
LLR reaching every leaf equal as an FP32 value (f is a selection and g one
rounding in both), on seeded frames of the benchmark's recipe, for lengths
across the kernel's tiling (one to 256 LDS passes per step) and degenerate
rates; the error rate inside the FP64 oracle's 95% interval."""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames, noiseless_llr, wilson

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_04979_amd as pbp
    pbp.lib()
    return pbp, torch


CASES = [
    # N, K, Eb/N0, frames
    (2, 1, 2.0, 300), (2, 2, 2.0, 300), (4, 2, 2.0, 200), (8, 4, 2.5, 200),
    (64, 32, 2.5, 300), (128, 64, 2.0, 200), (256, 128, 2.5, 150),
    (1024, 512, 3.0, 120), (1024, 0, 3.0, 20), (1024, 1024, 3.0, 20),
    (4096, 2048, 2.5, 30), (16384, 8192, 2.0, 6),
]


@pytest.mark.parametrize("N,K,ebn0,B", CASES)
def test_sc_parity(env, N, K, ebn0, B):
    pbp, torch = env
    print(f"[sc] N={N} K={K} B={B}", flush=True)
    fz = frozen_mask(N, K)
    code = pbp.Code(N, K, fz)
    u, x, llr = make_frames(N, K, B, ebn0, stream=900 + N + K)
    out = pbp.pbp_decode_sc(code, torch.from_numpy(llr).cuda(), leaf=True)
    torch.cuda.synchronize()
    ref, leaf = oracle.sc_decode(llr, fz, leaf=True)
    assert np.array_equal(out["info"].cpu().numpy(), ref[:, fz == 0])
    assert np.array_equal(out["leaf"].cpu().numpy(), leaf)


def test_sc_noiseless(env):
    pbp, torch = env
    for N, K in ((64, 32), (1024, 512), (16384, 8192)):
        fz = frozen_mask(N, K)
        code = pbp.Code(N, K, fz)
        u, x, _ = make_frames(N, K, 8, 2.0, stream=910)
        out = pbp.pbp_decode_sc(code, torch.from_numpy(noiseless_llr(x)).cuda())
        assert np.array_equal(out["info"].cpu().numpy(), u[:, fz == 0])


def test_sc_error_rate_inside_fp64_interval(env):
    """(1024, 512) at 2.5 dB, 3000 frames: the FP32 GPU decoder's frame
    error rate inside the FP64 oracle's 95% Wilson interval."""
    pbp, torch = env
    N, K, B = 1024, 512, 3000
    fz = frozen_mask(N, K)
    code = pbp.Code(N, K, fz)
    u, _, llr = make_frames(N, K, B, 2.5, stream=920)
    got = pbp.pbp_decode_sc(code, torch.from_numpy(llr).cuda())["info"]
    err = (got.cpu().numpy() != u[:, fz == 0]).any(axis=1)
    ref = oracle.sc_decode(llr, fz, prec="f64")
    err64 = (ref != u).any(axis=1)
    lo, hi = wilson(int(err64.sum()), B)
    assert lo <= err.mean() <= hi


def test_sc_rejects_bad_arguments(env):
    pbp, torch = env
    code = pbp.Code(64, 32, frozen_mask(64, 32))
    out = pbp.pbp_decode_sc(code, torch.zeros((0, 64), device="cuda"))
    assert out["info"].shape == (0, 32)
