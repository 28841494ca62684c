"""GPU parity of the fixed-point decoder (pbp_decode_quant) with the
oracle's, through the C-ABI: decided bits, iteration counts, PE counts and
the saturated posteriors all equal (integer arithmetic, so exact), in every
mode and three message formats, for N = 2 to 4096 (every decoder the
lengths use) including degenerate
rates and noiseless frames; the long-code limit is rejected."""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask, make_frames, noiseless_llr

pytestmark = pytest.mark.gpu

MODES = {
    "plain": dict(max_iter=20, early_stop=False, freezing=False),
    "es": dict(max_iter=40, early_stop=True, freezing=False),
    "es_frz": dict(max_iter=40, early_stop=True, freezing=True),
    "frz": dict(max_iter=30, early_stop=False, freezing=True),
    "es_frz_R": dict(max_iter=40, early_stop=True, freezing=True,
                     freeze_input=0),
    "stage": dict(max_iter=40, early_stop=True, freezing=True, freeze_walk=1),
    "greedy": dict(max_iter=40, early_stop=True, freezing=True, freeze_walk=2),
}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_04979_amd as pbp
    pbp.lib()
    return pbp, torch


def run(env, N, K, llr, bits, frac, mode):
    pbp, torch = env
    fz = frozen_mask(N, K)
    code = pbp.Code(N, K, fz)
    o = dict(freeze_input=1, freeze_walk=0)
    o.update(MODES[mode])
    got = pbp.pbp_decode_quant(code, torch.from_numpy(llr).cuda(), bits=bits,
                               frac=frac, soft=True, **o)
    torch.cuda.synchronize()
    ref = oracle.decode_quant(llr, fz, bits=bits, frac=frac, soft=True, **o)
    assert np.array_equal(got["info"].cpu().numpy(), ref["info"]), "bits"
    assert np.array_equal(got["iters"].cpu().numpy(), ref["iters"]), "iters"
    assert np.array_equal(got["pe"].cpu().numpy(), ref["pe"]), "pe"
    assert np.array_equal(got["soft"].cpu().numpy().astype(np.int32),
                          ref["soft"]), "soft"


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("N,K,ebn0,B", [(2, 1, 2.0, 100), (8, 4, 2.0, 100),
                                        (32, 16, 2.0, 200),
                                        (64, 32, 2.5, 200), (128, 64, 2.5, 100),
                                        (256, 128, 2.5, 100), (512, 256, 2.5, 60),
                                        (1024, 512, 3.0, 60),
                                        (2048, 1024, 2.5, 12),
                                        (4096, 2048, 2.5, 8)])
def test_quant_parity(env, N, K, ebn0, B, mode):
    print(f"[quant] N={N} K={K} mode={mode}", flush=True)
    _, _, llr = make_frames(N, K, B, ebn0, stream=1000 + N)
    run(env, N, K, llr, 8, 3, mode)


@pytest.mark.parametrize("bits,frac", [(6, 1), (7, 2), (8, 1)])
def test_quant_formats(env, bits, frac):
    N, K = 1024, 512
    _, _, llr = make_frames(N, K, 40, 2.5, stream=1100 + bits)
    for mode in ("plain", "es_frz"):
        run(env, N, K, llr, bits, frac, mode)


@pytest.mark.parametrize("N,K", [(1024, 0), (1024, 1024), (64, 1), (64, 63)])
def test_quant_degenerate_rates(env, N, K):
    _, _, llr = make_frames(N, K, 20, 2.0, stream=1200 + K)
    for mode in ("es", "es_frz"):
        run(env, N, K, llr, 8, 3, mode)


def test_quant_noiseless(env):
    pbp, torch = env
    N, K = 1024, 512
    fz = frozen_mask(N, K)
    u, x, _ = make_frames(N, K, 10, 2.0, stream=1300)
    llr = noiseless_llr(x)
    for mode in MODES:
        run(env, N, K, llr, 8, 3, mode)


def test_quant_rejects(env):
    pbp, torch = env
    code = pbp.Code(8192, 4096, frozen_mask(8192, 4096))
    with pytest.raises(pbp.PbpError):
        pbp.pbp_decode_quant(code, torch.zeros((1, 8192), device="cuda"))
    code = pbp.Code(64, 32, frozen_mask(64, 32))
    with pytest.raises(pbp.PbpError):
        pbp.pbp_decode_quant(code, torch.zeros((1, 64), device="cuda"),
                             bits=9)


@pytest.mark.parametrize("N,K,B", [(64, 32, 200), (256, 128, 60),
                                   (1024, 512, 40), (4096, 2048, 6)])
def test_quant_alpha_above_one(env, N, K, B):
    """alpha = 1.25 (a = 20) with 8-bit messages: a scaled minimum reaches
    (20 * 127 + 8) >> 4 = 159 > Q.  The oracle keeps it unsaturated, and
    every decoder holds it exactly in FP32 registers or LDS words."""
    pbp, torch = env
    fz = frozen_mask(N, K)
    _, _, llr = make_frames(N, K, B, 2.5, stream=1400 + N)
    code = pbp.Code(N, K, fz)
    for mode in ("plain", "es_frz"):
        o = dict(freeze_input=1, freeze_walk=0, alpha=1.25)
        o.update(MODES[mode])
        got = pbp.pbp_decode_quant(code, torch.from_numpy(llr).cuda(), bits=8,
                                   frac=3, soft=True, **o)
        ref = oracle.decode_quant(llr, fz, bits=8, frac=3, soft=True, **o)
        assert np.array_equal(got["info"].cpu().numpy(), ref["info"])
        assert np.array_equal(got["iters"].cpu().numpy(), ref["iters"])
        assert np.array_equal(got["pe"].cpu().numpy(), ref["pe"])
        assert np.array_equal(got["soft"].cpu().numpy().astype(np.int32),
                              ref["soft"])


def test_quant_unaligned_and_many_frames(env):
    """N = 1024: LLR rows that are not 16-byte aligned (scalar loads), and a
    batch of more frames than resident wavefronts, so each wavefront takes
    several frames from the stream's counter; a second call on the same
    stream starts from a rewound counter."""
    pbp, torch = env
    N, K = 1024, 512
    fz = frozen_mask(N, K)
    code = pbp.Code(N, K, fz)
    _, _, llr = make_frames(N, K, 64, 3.0, stream=1500)
    buf = torch.zeros(64 * N + 1, device="cuda")
    buf[1:] = torch.from_numpy(llr).cuda().reshape(-1)
    o = dict(MODES["es_frz"], freeze_input=1, freeze_walk=0)
    got = pbp.pbp_decode_quant(code, buf[1:].view(64, N), bits=8, frac=3, **o)
    ref = oracle.decode_quant(llr, fz, bits=8, frac=3, **o)
    assert np.array_equal(got["info"].cpu().numpy(), ref["info"])
    assert np.array_equal(got["iters"].cpu().numpy(), ref["iters"])
    assert np.array_equal(got["pe"].cpu().numpy(), ref["pe"])
    B = 20000
    rep = np.tile(llr, (B // 64 + 1, 1))[:B]
    d = torch.from_numpy(rep).cuda()
    for _ in range(2):
        got = pbp.pbp_decode_quant(code, d, bits=8, frac=3, **o)
        idx = np.arange(B) % 64
        assert np.array_equal(got["info"].cpu().numpy(), ref["info"][idx])
        assert np.array_equal(got["iters"].cpu().numpy(), ref["iters"][idx])
        assert np.array_equal(got["pe"].cpu().numpy(), ref["pe"][idx])
