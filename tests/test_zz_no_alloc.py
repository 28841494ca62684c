"""pbp_decode_noalloc, the decode entry point for callers that cannot
allocate, against pbp_decode on the same inputs, through the C-ABI: two calls
in a row on one GPU (the second with a smaller batch, so the shared scratch
still holds the first call's state), for the three scratch uses: the
N = 1024 kernel's counter pair, the message-state slots of a code longer
than 1024 (more frames than slots fit in the scratch), and a code that needs
no scratch.  Bits, iteration counts, PE counts and posteriors must be equal.
"""

import numpy as np
import pytest

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


CASES = [
    # N, K, Eb/N0, first batch, second batch, options
    (1024, 512, 2.5, 3000, 700, dict(max_iter=40, early_stop=True,
                                     freezing=True, freeze_input=1,
                                     freeze_walk=0)),
    (4096, 2048, 2.0, 400, 90, dict(max_iter=30, early_stop=True,
                                    freezing=True, freeze_input=1,
                                    freeze_walk=0)),
    (64, 32, 2.5, 500, 37, dict(max_iter=40, early_stop=True, freezing=False,
                                freeze_input=1, freeze_walk=0)),
    # message state in the static array's slots
    (8192, 4096, 2.5, 40, 9, dict(max_iter=20, early_stop=True, freezing=True,
                                  freeze_input=1, freeze_walk=0)),
]


@pytest.mark.parametrize("N,K,ebn0,B1,B2,opts", CASES)
def test_noalloc_matches_decode(env, N, K, ebn0, B1, B2, opts):
    pbp, torch = env
    code = pbp.Code(N, K, frozen_mask(N, K))
    for call, B in enumerate((B1, B2)):
        print(f"[noalloc] N={N} K={K} call={call} B={B}", flush=True)
        _, _, llr = make_frames(N, K, B, ebn0, stream=700 + 10 * N + call)
        d = torch.from_numpy(llr).cuda()
        ref = pbp.pbp_decode(code, d, soft=True, **opts)
        got = pbp.pbp_decode_noalloc(code, d, soft=True, **opts)
        torch.cuda.synchronize()
        for k in ("info", "iters", "pe", "soft"):
            assert torch.equal(got[k], ref[k]), (k, call)


def test_noalloc_rejects_bad_arguments(env):
    pbp, torch = env
    code = pbp.Code(64, 32, frozen_mask(64, 32))
    d = torch.zeros((4, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(pbp.PbpError):
        pbp.pbp_decode_noalloc(code, d, max_iter=0)
    out = pbp.pbp_decode_noalloc(code, d[:0], max_iter=5)
    assert out["iters"].shape == (0,)
