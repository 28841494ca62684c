"""GPU parity of the mixed-code persistent decoder against the FP32 oracle,
through the C-ABI: every frame's bits, iteration count and PE count equal
the oracle's for that frame's code, under every launch configuration, in a
replayed graph, and after autotuning."""

import numpy as np
import pytest

import oracle
from helpers import frozen_mask
from mixed_helpers import MIX, make_mixed

pytestmark = pytest.mark.gpu

MODES = {
    "es_frz": dict(early_stop=True, freezing=True, freeze_input=1,
                   freeze_walk=0),
    "es": dict(early_stop=True, freezing=False),
    "plain": dict(early_stop=False, freezing=False),
    "frz": dict(early_stop=False, freezing=True),
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


def codes_of(pbp, dims):
    out = []
    for N, K in dims:
        if (N, K) not in _codes:
            _codes[(N, K)] = pbp.Code(N, K, frozen_mask(N, K))
        out.append(_codes[(N, K)])
    return out


def upload(torch, batch):
    cof, ebn0, lo, io, llr, info = batch
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return d(cof), d(lo), d(io), d(llr), int(sum(len(i) for i in info))


def oracle_check(dims, batch, out, mode, max_iter, frames=None):
    cof, ebn0, lo, io, llr, info = batch
    bits = out["info"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    pe = out["pe"].cpu().numpy()
    sel = np.arange(len(cof)) if frames is None else np.asarray(frames)
    for c, (N, K) in enumerate(dims):
        idx = sel[cof[sel] == c]
        if len(idx) == 0:
            continue
        fz = frozen_mask(N, K)
        L = np.stack([llr[lo[f]:lo[f] + N] for f in idx])
        r = oracle.decode(L, fz, max_iter=max_iter, **MODES[mode])
        got = np.stack([bits[io[f]:io[f] + K] for f in idx])
        assert np.array_equal(got, r["info"]), (N, K, mode)
        assert np.array_equal(iters[idx], r["iters"]), (N, K, mode)
        assert np.array_equal(pe[idx], r["pe"]), (N, K, mode)


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("mode", list(MODES))
def test_mixed_parity(env, mode, order):
    """Both schedules: one launch in the caller's order (0), one launch per
    code after the device sort (1)."""
    pbp, torch = env
    print(f"[mixed] mode={mode} order={order}", flush=True)
    dims = MIX
    batch = make_mixed(dims, 360, stream=40)
    cof, lo, io, llr, nbits = upload(torch, batch)
    plan = pbp.MixedPlan(codes_of(pbp, dims), 360)
    plan.config = (order, 16)
    out = pbp.pbp_decode_mixed(plan, cof, lo, io, llr, info_bytes=nbits,
                               max_iter=60, alpha=0.9375, **MODES[mode])
    torch.cuda.synchronize()
    oracle_check(dims, batch, out, mode, 60)


@pytest.mark.parametrize("cfg", [(0, 1), (0, 3), (1, 2), (1, 8), (1, 16)])
def test_configs_give_identical_results(env, cfg):
    pbp, torch = env
    dims = [(64, 32), (1024, 512), (2048, 1024), (128, 100), (1024, 300)]
    batch = make_mixed(dims, 300, stream=41)
    cof, lo, io, llr, nbits = upload(torch, batch)
    plan = pbp.MixedPlan(codes_of(pbp, dims), 1000)
    plan.config = cfg
    assert plan.config == cfg
    out = pbp.pbp_decode_mixed(plan, cof, lo, io, llr, info_bytes=nbits,
                               max_iter=40, **MODES["es_frz"])
    torch.cuda.synchronize()
    oracle_check(dims, batch, out, "es_frz", 40)
    fill = pbp.pbp_mixed_plan_fill(plan)
    assert 0.0 < fill <= 1.0


@pytest.mark.parametrize("order", [0, 1])
def test_frames_not_decoded(env, order):
    """A frame naming no code of the plan gets zero iterations and is not
    decoded; an N = 1024 frame whose LLRs are not 16-byte aligned decodes
    like the others (the register decoder reads it by words)."""
    pbp, torch = env
    dims = [(256, 128), (1024, 512)]
    batch = make_mixed(dims, 40, stream=42)
    cof, ebn0, lo, io, llr, info = batch
    cof = cof.copy()
    lo = lo.copy()
    bad_code = 3
    cof[bad_code] = 7
    j = int(np.flatnonzero(cof == 1)[0])
    # shift one N = 1024 frame by one element (its LLRs move with it)
    big = np.zeros(len(llr) + 4, np.float32)
    big[:len(llr)] = llr
    big[lo[j] + 1:lo[j] + 1 + 1024] = llr[lo[j]:lo[j] + 1024]
    lo[j] += 1
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = pbp.MixedPlan(codes_of(pbp, dims), 40)
    plan.config = (order, 16)
    out = pbp.pbp_decode_mixed(plan, d(cof), d(lo), d(io), d(big),
                               info_bytes=int(sum(len(i) for i in info)),
                               **MODES["es_frz"])
    torch.cuda.synchronize()
    it = out["iters"].cpu().numpy()
    assert it[bad_code] == 0 and it[j] > 0
    keep = [f for f in range(40) if f != bad_code]
    oracle_check(dims, (cof, ebn0, lo, io, big, info), out, "es_frz", 40,
                 frames=keep)


def test_graph_capture_replays(env):
    """The mixed decode captured once in a graph and replayed on new LLRs
    (copied into the captured buffer between replays) matches eager calls,
    replay after replay."""
    pbp, torch = env
    dims = [(256, 85), (1024, 512), (4096, 2048)]
    batches = [make_mixed(dims, 120, stream=43 + i) for i in range(3)]
    # one layout (codes and offsets) for every replay: reuse the first
    cof, ebn0, lo, io, llr0, info0 = batches[0]
    plan = pbp.MixedPlan(codes_of(pbp, dims), 120)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d_cof, d_lo, d_io = d(cof), d(lo), d(io)
    nbits = int(sum(len(i) for i in info0))
    static_llr = d(llr0)
    out = {"info": torch.empty(nbits, dtype=torch.uint8, device="cuda"),
           "iters": torch.empty(120, dtype=torch.int32, device="cuda"),
           "pe": torch.empty(120, dtype=torch.int64, device="cuda")}
    opts = pbp.make_opts(max_iter=60, **MODES["es_frz"])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pbp.pbp_decode_mixed(plan, d_cof, d_lo, d_io, static_llr, opts=opts,
                             out=out, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pbp.pbp_decode_mixed(plan, d_cof, d_lo, d_io, static_llr, opts=opts,
                             out=out, stream=s)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    for rep in range(4):
        # new channel realisations with the same layout
        llr = llr0 * rng.uniform(0.5, 1.5, size=llr0.shape).astype(np.float32)
        static_llr.copy_(torch.from_numpy(llr))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.clone() for k, v in out.items()}
        eager = pbp.pbp_decode_mixed(plan, d_cof, d_lo, d_io, d(llr),
                                     info_bytes=nbits, opts=opts)
        torch.cuda.synchronize()
        for k in got:
            assert torch.equal(got[k], eager[k]), (rep, k)
        oracle_check(dims, (cof, ebn0, lo, io, llr, info0), got, "es_frz", 60)


def test_tune_picks_and_caches(env):
    pbp, torch = env
    import time
    dims = [(256, 128), (1024, 512), (4096, 1365)]
    batch = make_mixed(dims, 600, stream=47)
    cof, lo, io, llr, nbits = upload(torch, batch)
    plan = pbp.MixedPlan(codes_of(pbp, dims), 600)
    best = pbp.pbp_mixed_plan_tune(plan, cof, lo, io, llr, info_bytes=nbits,
                                   max_iter=60, reps=1, **MODES["es_frz"])
    assert best[0] in (0, 1) and best[1] in (4, 8, 12, 16)
    assert plan.config == best
    # a second plan with the same codes and mode takes the cached result
    plan2 = pbp.MixedPlan(codes_of(pbp, dims), 600)
    t0 = time.perf_counter()
    best2 = pbp.pbp_mixed_plan_tune(plan2, cof, lo, io, llr,
                                    info_bytes=nbits, max_iter=60, reps=1,
                                    **MODES["es_frz"])
    assert best2 == best
    out = pbp.pbp_decode_mixed(plan2, cof, lo, io, llr, info_bytes=nbits,
                               max_iter=60, **MODES["es_frz"])
    torch.cuda.synchronize()
    assert time.perf_counter() - t0 < 5.0
    oracle_check(dims, batch, out, "es_frz", 60)


def test_rejects_bad_arguments(env):
    pbp, torch = env
    codes = codes_of(pbp, [(64, 32)])
    with pytest.raises(pbp.PbpError):
        pbp.MixedPlan(codes, 0)
    with pytest.raises(pbp.PbpError):
        pbp.MixedPlan(codes * 17, 10)
    plan = pbp.MixedPlan(codes, 10)
    with pytest.raises(pbp.PbpError):
        plan.config = (2, 4)
    with pytest.raises(pbp.PbpError):
        plan.config = (1, 17)
    z = torch.zeros(11, dtype=torch.int32, device="cuda")
    zl = torch.zeros(11, dtype=torch.int64, device="cuda")
    buf = torch.zeros(64 * 11, dtype=torch.float32, device="cuda")
    with pytest.raises(pbp.PbpError):   # more frames than the plan holds
        pbp.pbp_decode_mixed(plan, z, zl, zl, buf, info_bytes=64)


def test_full_size_mixed_batch_sampled(env):
    """The mixed workload at full size (2^20 frames over the nine codes,
    Eb/N0 uniform in [1, 4] dB, 60 iterations) in the tuned launch
    configuration.  To keep input generation short, 2^16 distinct frames are
    repeated 16 times (each copy with its own offsets): every copy must
    decode identically, and sampled frames of every code match the oracle."""
    pbp, torch = env
    U, REP = 1 << 16, 16
    B = U * REP
    print(f"[mixed] full size B={B}", flush=True)
    batch = make_mixed(MIX, U, stream=48)
    cof, ebn0, lo, io, llr, info = batch
    nllr, nbits = len(llr), int(sum(len(i) for i in info))
    k = np.repeat(np.arange(REP, dtype=np.int64), U)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d_cof = d(np.tile(cof, REP))
    d_lo = d(np.tile(lo, REP) + k * nllr)
    d_io = d(np.tile(io, REP) + k * nbits)
    d_llr = d(llr).repeat(REP)
    plan = pbp.MixedPlan(codes_of(pbp, MIX), B)
    plan.config = (1, 16)
    out = pbp.pbp_decode_mixed(plan, d_cof, d_lo, d_io, d_llr,
                               info_bytes=nbits * REP, max_iter=60,
                               **MODES["es_frz"])
    torch.cuda.synchronize()
    for key in ("iters", "pe", "info"):
        v = out[key].view(REP, -1)
        assert torch.equal(v, v[:1].expand_as(v)), key
    first = {key: v[:U] if key != "info" else v[:nbits]
             for key, v in out.items()}
    rng = np.random.default_rng(2)
    frames = np.concatenate([rng.choice(np.flatnonzero(cof == c), 3,
                                        replace=False)
                             for c in range(len(MIX))])
    oracle_check(MIX, batch, first, "es_frz", 60, frames=frames)
    fill = pbp.pbp_mixed_plan_fill(plan)
    print(f"[mixed] fill {fill:.4f}", flush=True)
    assert 0.5 < fill <= 1.0
