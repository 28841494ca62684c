"""Throughput of the polar BP decoder on one MI355X.

Workload: the (1024, 512) polar code (design Eb/N0 0 dB), BPSK over AWGN at
Eb/N0 = 3.0 dB, scaled min-sum with alpha = 0.9375, at most 40 iterations,
G-matrix early stop plus CSFG freezing (eq. (2) on the total belief, one
freeze per iteration).  A step decodes one batch of frames already resident
in device memory; the metric is decoded information bits per second.

Prints one JSON line.  Beside the headline it reports: PE activations per
frame; the same batch under 40-iteration BP and under early stop alone
(speed-up and error-rate match); the decoder kernel's fraction of the VALU
roofline; and the CPU oracle timed on the host's cores on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("decoded info Mbit/s at N=1024 R=1/2 3.0dB, FER-matched; "
          "PE updates/frame")

# FP32 VALU roofline of gfx950 without packed FP32: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz FP32 lane operations per second (the published FP64 vector
# rate, 78.6 TFLOP/s, is these lanes at two flops per FMA; the published FP32
# figure counts packed FP32, which these kernels do not use).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic work of one PE activation of eq. (1): three distinct min-sum
# terms (each a sign product, a magnitude minimum and a scaling) and three
# additions, 12 operations.  gfx950 issues about 11 VALU instructions for
# them (a median of three is the clamped minimum and carries one sign), so
# the kernel's issued-instruction rate is reported beside this fraction.
OPS_PER_PE = 12

# the kernel one step launches (one launch per step)
KERNEL = "bp_decode_r10_kernel<true, true>"

# Measured HBM traffic of a workload's roofline kernel: the profile summary
# that records it, and the kernel's sources (a record is valid while they
# are unchanged).
def _csrc(*names):
    return [os.path.join(ROOT, "paper_1505_04979_amd", "csrc", f) for f in names]


TRAFFIC_RECORDS = {
    "n1024": ("traffic_bp_decode_r10_n1024_3db.txt",
              _csrc("pbp_r10.hip", "pbp_r10_decoder.h", "pbp_r10.h",
                    "pbp_arith.h")),
    "n16384": ("traffic_bp_decode_n16384_2db.txt",
               _csrc("pbp_decode.hip", "pbp_generic_decoder.h", "pbp_lanes.h")),
    "unrolled": ("traffic_unrolled_backward_n1024.txt",
                 _csrc("pbp_unrolled.hip")),
    # the mixed batch's N = 4096 frames decoded alone: three class kernels
    # (one per rate) per decode, summed
    "mixed": ("traffic_class_pair_n4096_mixed.txt",
              _csrc("pbp_mixed.hip", "pbp_pair_decoder.h",
                    "pbp_generic_decoder.h", "pbp_arith.h", "pbp_lanes.h")),
}
KERNEL_SRCS = TRAFFIC_RECORDS["n1024"][1]

# Kernel-trace summaries (rocprofv3 --kernel-trace --stats of the workload's
# own bench command): the roofline kernel's average dispatch duration, valid
# while its sources are unchanged; plus, for the headline, the VALU
# instructions the counters run issued per launch.
TRACE_RECORDS = {
    "n1024": ("bp_decode_r10_n1024_3db_trace.md", KERNEL_SRCS),
    "c1": ("bp_decode_n64_c1_trace.md",
           _csrc("pbp_decode.hip", "pbp_wave_decoder.h", "pbp_arith.h",
                 "pbp_generic_decoder.h", "pbp_lanes.h")),
    "n16384": ("n16384_trace.md", TRAFFIC_RECORDS["n16384"][1]),
    "sc": ("sc_decode_n1024_trace.md", _csrc("pbp_sc.hip")),
    "quant": ("quant_decode_n1024_3db_trace.md",
              _csrc("pbp_quant.hip", "pbp_r10_decoder.h", "pbp_r10.h",
                    "pbp_arith.h")),
    "round_trip": ("round_trip_trace.md", _csrc("pbp_roundtrip.hip")),
    "mixed": ("mixed_trace.md", TRAFFIC_RECORDS["mixed"][1]),
    "unrolled": ("unrolled_trace.md", TRAFFIC_RECORDS["unrolled"][1]),
}
COUNTER_RECORDS = {
    "n1024": ("counters_bp_decode_r10_n1024_3db.md", KERNEL_SRCS),
    "unrolled": ("counters_unrolled_backward_n1024.md",
                 TRAFFIC_RECORDS["unrolled"][1]),
}

MODES = {
    "es_frz": dict(early_stop=True, freezing=True, freeze_input=1, freeze_walk=0),
    "es": dict(early_stop=True, freezing=False),
    "plain": dict(early_stop=False, freezing=False),
}


def wilson(k, n, z):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h


def make_inputs(pbp, torch, code, frozen, N, K, B, ebn0, stream, chunk=None):
    """Seeded info bits and noise (host), encoding on the device, channel
    LLRs (host, FP64 rounded once), uploaded to device memory.  The noise
    and LLRs are made a chunk of frames at a time (the draws are counter-based
    per frame, so chunking does not change them)."""
    import synth
    if chunk is None:
        chunk = max(1, (1 << 27) // N)      # 1 GB of FP64 noise at a time
    info = synth.info_bits(K, B, stream=stream)
    d_info = torch.from_numpy(info).cuda()
    cw = pbp.pbp_encode(code, d_info)
    torch.cuda.synchronize()
    del d_info
    d_llr = torch.empty((B, N), dtype=torch.float32, device="cuda")
    for lo in range(0, B, chunk):
        hi = min(B, lo + chunk)
        noise = synth.normals(N, hi - lo, frame0=lo, stream=stream)
        llr = synth.channel_llr(cw[lo:hi].cpu().numpy(), noise, ebn0, K / N)
        d_llr[lo:hi].copy_(torch.from_numpy(llr))
        del noise, llr
    del cw
    torch.cuda.synchronize()
    return info, d_llr


def time_mode(pbp, torch, code, d_llr, opts, steps, warmup):
    out = pbp.pbp_decode(code, d_llr, **opts)
    torch.cuda.synchronize()
    for _ in range(warmup):
        pbp.pbp_decode(code, d_llr, out=out, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record()
    for i in range(steps):
        pbp.pbp_decode(code, d_llr, out=out, **opts)
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = evs[0].elapsed_time(evs[-1]) / steps
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    median = per_step[steps // 2] if steps % 2 else \
        0.5 * (per_step[steps // 2 - 1] + per_step[steps // 2])
    # end to end: one more decode plus the copy of its decided bits and
    # iteration counts to the host
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pbp.pbp_decode(code, d_llr, out=out, **opts)
    host = {k: v.cpu().numpy() for k, v in out.items()}
    e2e = (time.perf_counter() - t1) * 1e3
    return ms, wall, host, median, e2e


def source_digest(srcs=None):
    import hashlib
    h = hashlib.sha256()
    for src in srcs or KERNEL_SRCS:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _record(name, srcs, frames=None):
    """The machine-read lines (``@key = value``) of a profile summary, or
    None when it is missing, was taken on other kernel sources, or (frames
    given) on another number of frames per launch."""
    vals = {}
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            for ln in f:
                if ln.startswith("@") and "=" in ln:
                    k, v = ln[1:].split("=", 1)
                    vals[k.strip()] = v.strip()
    except OSError:
        return None
    if vals.get("source_sha256_16") != source_digest(srcs):
        return None
    if frames is not None and vals.get("frames_per_launch") != str(frames):
        return None
    return vals


def _record_float(vals, key):
    try:
        return float(vals[key]) if vals is not None else None
    except (KeyError, ValueError):
        return None


def measured_traffic(workload="n1024", frames=None):
    """HBM bytes per launch of a workload's roofline kernel from the
    FETCH_SIZE and WRITE_SIZE counter runs recorded in its profile summary,
    scaled by what the same counters read for a plain copy of known size;
    None when the kernel source has changed since the counters were taken."""
    name, srcs = TRAFFIC_RECORDS[workload]
    return _record_float(_record(name, srcs, frames),
                         "traffic_bytes_per_launch")


def traced_kernel_ms(workload, kernel, frames):
    """The duration (ms) of `kernel` per launch of the workload in its
    committed kernel trace (the average dispatch times the dispatches one
    launch makes), or None (missing, stale or other frames)."""
    name, srcs = TRACE_RECORDS[workload]
    rec = _record(name, srcs, frames)
    v = _record_float(rec, f"avg_ns[{kernel}]")
    n = _record_float(rec, f"dispatches_per_launch[{kernel}]") or 1.0
    return None if v is None else v * n / 1e6


def valu_issue(workload, kernel, frames, ms):
    """Fraction of the VALU lane rate the kernel's issued VALU instructions
    fill: SQ_INSTS_VALU x 64 lanes over (lane peak x launch time), from the
    committed counters run (None when missing or stale)."""
    if workload not in COUNTER_RECORDS:
        return None
    name, srcs = COUNTER_RECORDS[workload]
    n = _record_float(_record(name, srcs, frames),
                      f"sq_insts_valu_per_launch[{kernel}]")
    if n is None or not ms:
        return None
    return n * 64 / (VALU_PEAK_TOPS * 1e12 * ms / 1e3)


def copy_calibration(torch, nbytes, reps):
    """A plain device-to-device copy of nbytes, reps times: the yardstick for
    the HBM byte counters (reads nbytes, writes nbytes per launch)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "launches": reps}), flush=True)


def _oracle_frozen(N, K):
    """The frozen set of the oracle's own construction (the oracle's inputs
    come from the oracle and the seeded draws, not from the library)."""
    import oracle
    fz, _ = oracle.construct(N, K, 0.0)
    return np.array(fz, dtype=np.uint8)


def host_cpu():
    """(CPU model, logical CPUs this process may run on, threads an all-core
    run uses: at most 16, the CPU share of one GPU on a shared host)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return model, avail, max(1, min(16, avail))


def _oracle_timed(llr, frozen, opts, threads, seconds, chunk,
                  decode=None):
    """Decode chunks of llr (host) with the oracle on `threads` threads, in
    order and wrapping round, until `seconds` have passed (every thread
    finishes its chunk).  Returns (frames decoded, wall seconds, {first
    frame of a chunk: oracle result} for the first pass)."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    if decode is None:
        def decode(x):
            return oracle.decode(x, frozen, **opts)
    B = len(llr)
    nxt = [0]
    lock = threading.Lock()
    first = {}
    count = [0]
    t0 = time.perf_counter()
    deadline = t0 + seconds

    def worker():
        while time.perf_counter() < deadline:
            with lock:
                k = nxt[0]
                nxt[0] += 1
            lo = (k * chunk) % B if B > chunk else 0
            hi = min(B, lo + chunk)
            r = decode(llr[lo:hi])
            with lock:
                count[0] += hi - lo
                if k * chunk < B:
                    first[lo] = r
    with ThreadPoolExecutor(threads) as ex:
        for f in [ex.submit(worker) for _ in range(threads)]:
            f.result()
    return count[0], time.perf_counter() - t0, first


def cpu_baseline(llr, K, info_ref, opts, seconds, chunk=16, decode=None,
                 key="info", what="FP32 oracle"):
    """The oracle on the host over a bounded sample of the same frames,
    single-threaded for half the time budget and on all the cores it may use
    for the other half; each leg's first pass is checked against the GPU's
    bits (`info_ref`, rows of the sample)."""
    model, avail, threads = host_cpu()
    frozen = _oracle_frozen(llr.shape[1], K)
    legs = {}
    mism = 0
    for name, nt in (("single_thread", 1), ("all_cores", threads)):
        n, wall, first = _oracle_timed(llr, frozen, opts, nt, seconds / 2,
                                       chunk, decode)
        mism += sum(int(np.sum(np.any(r[key] != info_ref[lo:lo + len(r[key])],
                                      axis=1)))
                    for lo, r in first.items())
        legs[name] = {"value": round(n * K / wall / 1e6, 4),
                      "frames_per_s": round(n / wall, 1), "threads": nt,
                      "frames": n, "seconds": round(wall, 2)}
    a = legs["all_cores"]
    return {"value": a["value"], "unit": "Mbit/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{what} over the first {len(llr)} frames of the "
                      f"timed batch (wrapping round), {seconds / 2:g} s "
                      f"single-threaded then {seconds / 2:g} s on {threads} "
                      "threads",
            "cpu_model": model, "host_cpus_visible": avail,
            "single_thread": legs["single_thread"], "all_cores": a,
            "gpu_mismatches": mism}


def _oracle_all(llr, frozen, opts, threads, chunk=256):
    """The oracle over every frame of llr (host FP32 array), in chunks on a
    thread pool; returns the concatenated info bits, iterations and PE
    counts."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    B = len(llr)
    parts = {}

    def job(lo):
        parts[lo] = oracle.decode(llr[lo:lo + chunk], frozen, **opts)
        return lo

    with ThreadPoolExecutor(threads) as ex:
        done = 0
        for _ in ex.map(job, range(0, B, chunk)):
            done += 1
            if done % 512 == 0:
                print(f"[parity] {min(B, done * chunk)} / {B} frames",
                      file=sys.stderr, flush=True)
    keys = sorted(parts)
    return {k: np.concatenate([parts[lo][k] for lo in keys])
            for k in ("info", "iters", "pe")}


def _compare(o, info, iters, pe):
    """Frames where the oracle's outputs o differ from the given GPU outputs
    in information bits, iteration count or PE count."""
    return int(np.sum(np.any(o["info"] != info, axis=1) |
                      (o["iters"] != iters) | (o["pe"] != pe)))


def full_parity(d_llr, info_ref, res, K):
    """Every frame of the timed batch through the FP32 oracle in each mode
    (bits, iterations and PE counts against the GPU's, frame by frame), and
    through the FP64 oracle in the headline mode (the GPU's error rate
    against the FP64 oracle's 95% interval).  Part of the CPU baseline leg."""
    threads = max(1, min(16, os.cpu_count() or 1))
    llr = d_llr.cpu().numpy()
    B = len(llr)
    frozen = _oracle_frozen(llr.shape[1], K)
    out = {"frames": B, "threads": threads}
    t0 = time.perf_counter()
    for name, r in res.items():
        print(f"[parity] mode {name}: FP32 oracle on {B} frames",
              file=sys.stderr, flush=True)
        o = _oracle_all(llr, frozen, r["opts"], threads)
        g = r["out"]
        bad = (np.any(o["info"] != g["info"], axis=1) |
               (o["iters"] != g["iters"]) | (o["pe"] != g["pe"]))
        out[name] = {"mismatched_frames": int(bad.sum())}
    h = res["es_frz"]
    print(f"[parity] FP64 oracle on {B} frames", file=sys.stderr, flush=True)
    o64 = _oracle_all(llr, frozen, dict(h["opts"], prec="f64"), threads)
    e64 = int(np.sum(np.any(o64["info"] != info_ref, axis=1)))
    lo, hi = wilson(e64, B, 1.959963984540054)
    out["fp64_es_frz"] = {"fer": e64 / B, "fer_ci95": [lo, hi],
                          "gpu_fer": h["fer"],
                          "gpu_inside": bool(lo <= h["fer"] <= hi)}
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=0,
                    help="frames per step (0: the workload's default)")
    ap.add_argument("--ebn0", type=float, default=None,
                    help="Eb/N0 in dB (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU baseline time budget, split between a "
                         "single-threaded and an all-core run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference-modes", action="store_true")
    ap.add_argument("--full-parity", action="store_true",
                    help="also decode every frame of the batch with the FP32 "
                         "oracle in each mode (bits, iterations and PE "
                         "counts compared) and with the FP64 oracle in the "
                         "headline mode (error-rate interval); takes minutes")
    ap.add_argument("--workload", default="n1024",
                    choices=["n1024", "c1", "n16384", "mixed", "unrolled",
                             "sweep", "round_trip", "sc", "quant"],
                    help="n1024: the headline line (default); c1: the "
                         "(64,32) code with every frame checked; n16384: the "
                         "long-code decoder; mixed: the mixed-code persistent "
                         "decoder; unrolled: one training step of the "
                         "unrolled decoder; sweep: every mode over Eb/N0; "
                         "round_trip: the round-trip schedule on the "
                         "headline's frames; sc: successive cancellation; "
                         "quant: 8-bit fixed-point BP")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter "
                         "yardstick) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(frames are independent: a multi-GPU run would shard the batch "
              "by frame and only sum counters)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1505_04979_amd as pbp
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration, max(1, args.steps))
        return
    if args.workload != "n1024":
        fn = {"c1": bench_c1, "n16384": bench_long_code,
              "mixed": bench_mixed, "unrolled": bench_unrolled,
              "sweep": bench_sweep, "round_trip": bench_round_trip,
              "sc": bench_sc, "quant": bench_quant}[args.workload]
        print(json.dumps(fn(args, pbp, torch)), flush=True)
        return

    # 10^6 frames per step: the frame count of the (1024, 512) workload's
    # error-rate points
    N, K, B, max_iter, alpha = 1024, 512, args.batch or 10 ** 6, 40, 0.9375
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    t0 = time.perf_counter()
    if args.ebn0 is None:
        args.ebn0 = 3.0
    info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, args.ebn0,
                              stream=(2 << 16) + 5)
    gen_s = time.perf_counter() - t0

    res = {}
    for name in (["es_frz"] if args.no_reference_modes else ["es_frz", "es", "plain"]):
        opts = dict(MODES[name], max_iter=max_iter, alpha=alpha)
        steps = args.steps
        ms, wall, out, med, e2e = time_mode(pbp, torch, code, d_llr, opts,
                                            steps, args.warmup)
        errs = int(np.sum(np.any(out["info"] != info, axis=1)))
        res[name] = dict(ms=ms, wall=wall, steps=steps, errors=errs,
                         fer=errs / B, iters=float(out["iters"].mean()),
                         pe=float(out["pe"].mean()),
                         mbps=B * K / (ms / 1e3) / 1e6, info=out["info"],
                         median_ms=med, e2e_ms=e2e, out=out, opts=opts)

    h = res["es_frz"]
    line = {
        "metric": METRIC,
        "value": round(h["mbps"], 2),
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": h["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "polar BP decode, (1024,512) code, BPSK/AWGN "
                               f"Eb/N0 {args.ebn0} dB, early stop + CSFG "
                               "freezing",
                   "N": N, "K": K, "ebn0_db": args.ebn0,
                   "frames_per_step": B, "max_iter": max_iter, "alpha": alpha,
                   "freeze_input": "total", "freeze_walk": "one_per_iter"},
        "pe_per_frame": round(h["pe"], 1),
        "avg_iters": round(h["iters"], 3),
        "fer": h["fer"],
        "ms_per_step_median": round(h["median_ms"], 4),
        # one decode plus the copy of its bits and iteration counts to the host
        "end_to_end_ms": round(h["e2e_ms"], 3),
    }
    pe_total = h["pe"] * B
    achieved = OPS_PER_PE * pe_total / (h["ms"] / 1e3) / 1e12
    line["roofline"] = _alu_roofline(achieved, "n1024", KERNEL, B, h["ms"],
                                     "12 operations per PE activation")
    if "plain" in res:
        p, e = res["plain"], res["es"]
        lo_f, _ = wilson(h["errors"], B, 1.6448536269514722)
        _, hi_p = wilson(p["errors"], B, 1.6448536269514722)
        line["reference_modes"] = {
            k: {"mbps": round(v["mbps"], 2), "ms_per_step": round(v["ms"], 4),
                "fer": v["fer"], "avg_iters": round(v["iters"], 3),
                "pe_per_frame": round(v["pe"], 1)}
            for k, v in (("plain40", p), ("early_stop", e))}
        line["speedup_vs_plain40"] = round(p["ms"] / h["ms"], 3)
        line["fer_matched"] = bool(lo_f <= hi_p)
    if not args.no_cpu_baseline:
        # a bounded sample: the oracle gets through well under 2^19 frames
        # in its time budget
        d_host = d_llr[:min(B, 1 << 19)].cpu().numpy()
        opts = dict(MODES["es_frz"], max_iter=max_iter, alpha=alpha)
        line["cpu_baseline"] = cpu_baseline(d_host, K, h["info"], opts,
                                            args.cpu_seconds)
        if args.full_parity:
            line["cpu_baseline"]["full_parity"] = full_parity(d_llr, info,
                                                              res, K)
    line["input_generation_s"] = round(gen_s, 2)
    print(json.dumps(line), flush=True)


def _alu_roofline(achieved, workload, kernel, frames, event_ms, note):
    """The roofline object of a VALU-bound kernel: `achieved` algorithmic
    TOP/s over the launch time measured live (`event_ms`, HIP events on the
    launch stream); `kernel_ms` is the average dispatch duration in the
    workload's committed kernel trace (None when stale), and
    `valu_issue_frac` the issued VALU instructions' share of the lane rate
    from the committed counters run, where one exists."""
    tr = TRACE_RECORDS.get(workload)
    r = {"bound": "alu", "achieved": round(achieved, 4),
         "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
         "frac": round(achieved / VALU_PEAK_TOPS, 5),
         "traffic": (measured_traffic(workload, frames)
                     if workload in TRAFFIC_RECORDS else None),
         "kernel": kernel,
         "kernel_ms": (None if tr is None else
                       _round(traced_kernel_ms(workload, kernel, frames), 4)),
         "event_ms": round(event_ms, 4),
         "valu_issue_frac": _round(valu_issue(workload, kernel, frames,
                                              event_ms), 4),
         "note": note}
    return r


def _round(v, nd):
    return None if v is None else round(v, nd)


# ---------------------------------------------------------------------------
# Other workloads (one JSON line each; not the headline)

HBM_PEAK_GBS = 8000.0


def _line(metric, value, unit, steps, warmup, ms, config, **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1,
         "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
         "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": "f32", "data": "synthetic", "config": config}
    d.update(extra)
    return d


def _timed(torch, fn, steps, warmup):
    fn()
    torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def bench_long_code(args, pbp, torch):
    """(16384, 8192) code at 2.0 dB, early stop + freezing, 60 iterations:
    the message state of each frame lives in device memory, so the decoder
    is bound by HBM traffic (16 B per active PE: two L messages read, two
    written; plus the channel LLRs once per iteration)."""
    N, K, max_iter, alpha = 16384, 8192, 60, 0.9375
    ebn0 = 2.0 if args.ebn0 is None else args.ebn0
    B = args.batch or 10 ** 5      # the long-code workload's frame count
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, ebn0,
                              stream=(5 << 16) + 1)
    opts = dict(MODES["es_frz"], max_iter=max_iter, alpha=alpha)
    out = pbp.pbp_decode(code, d_llr, **opts)
    steps = max(1, args.steps // 3)
    ms = _timed(torch, lambda: pbp.pbp_decode(code, d_llr, out=out, **opts),
                steps, 1)
    iters = out["iters"].cpu().numpy().astype(np.float64)
    pe = out["pe"].cpu().numpy().astype(np.float64)
    errs = int(np.sum(np.any(out["info"].cpu().numpy() != info, axis=1)))
    extra = {}
    if args.full_parity:
        # CPU baseline leg: the first 10^4 frames of the batch through the
        # FP32 oracle, timed, and compared frame by frame
        S = min(B, 10 ** 4)
        threads = max(1, min(16, os.cpu_count() or 1))
        print(f"[parity] long code: FP32 oracle on {S} frames", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        o = _oracle_all(d_llr[:S].cpu().numpy(), _oracle_frozen(N, K), opts,
                        threads, chunk=16)
        wall = time.perf_counter() - t0
        extra["cpu_baseline"] = {
            "value": round(S * K / wall / 1e6, 3), "unit": "Mbit/s",
            "cores": threads, "kind": "oracle",
            "sample": f"the first {S} frames of the batch, FP32 oracle, "
                      f"{threads} threads, {wall:.1f} s",
            "frames": S, "gpu_mismatches": _compare(
                o, out["info"][:S].cpu().numpy(),
                out["iters"][:S].cpu().numpy(), out["pe"][:S].cpu().numpy())}
    alg_bytes = 16.0 * pe.sum() + 4.0 * N * iters.sum() + B * (K + 12)
    gbs = alg_bytes / (ms / 1e3) / 1e9
    ops = OPS_PER_PE * pe.sum() / (ms / 1e3) / 1e12
    return _line(
        "decoded info Mbit/s, N=16384 R=1/2 2.0dB", round(B * K / ms / 1e3, 2),
        "Mbit/s", steps, 1, ms,
        {"workload": "polar BP decode, (16384,8192) code, BPSK/AWGN Eb/N0 "
                     f"{ebn0} dB, early stop + CSFG freezing, max 60 "
                     "iterations, message state in device memory",
         "N": N, "K": K, "ebn0_db": ebn0, "frames_per_step": B,
         "max_iter": max_iter},
        avg_iters=round(float(iters.mean()), 3),
        pe_per_frame=round(float(pe.mean()), 1), fer=errs / B,
        roofline={"bound": "hbm", "achieved": round(gbs, 1),
                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(gbs / HBM_PEAK_GBS, 4),
                  "traffic": measured_traffic("n16384", B),
                  "kernel": "bp_decode_kernel<14, true>",
                  "kernel_ms": _round(traced_kernel_ms(
                      "n16384", "bp_decode_kernel<14, true>", B), 4),
                  "event_ms": round(ms, 4)},
        valu={"achieved": round(ops, 3), "peak": round(VALU_PEAK_TOPS, 3),
              "unit": "TOP/s", "frac": round(ops / VALU_PEAK_TOPS, 4)},
        **extra)


def bench_c1(args, pbp, torch):
    """The (64, 32) code (design Eb/N0 0 dB) at Eb/N0 2.5 dB, early stop, at
    most 40 iterations, 10^4 frames.  Every frame is checked against the
    FP32 oracle (bits, iterations, PE counts), and the error rate against the
    FP64 oracle's 95% interval."""
    N, K, max_iter, alpha = 64, 32, 40, 0.9375
    ebn0 = 2.5 if args.ebn0 is None else args.ebn0
    B = args.batch or 10 ** 4
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, ebn0,
                              stream=(1 << 16) + 1)
    opts = dict(MODES["es"], max_iter=max_iter, alpha=alpha)
    # a launch decodes 10^4 short frames in tens of microseconds: more steps
    steps = args.steps * 10
    ms, _, out, med, e2e = time_mode(pbp, torch, code, d_llr, opts, steps,
                                     args.warmup)
    errs = int(np.sum(np.any(out["info"] != info, axis=1)))
    pe = out["pe"].astype(np.float64)
    llr = d_llr.cpu().numpy()
    fz = _oracle_frozen(N, K)
    _, _, threads = host_cpu()
    print(f"[parity] C1: FP32 and FP64 oracle on {B} frames", file=sys.stderr,
          flush=True)
    o = _oracle_all(llr, fz, opts, threads)
    o64 = _oracle_all(llr, fz, dict(opts, prec="f64"), threads)
    e64 = int(np.sum(np.any(o64["info"] != info, axis=1)))
    lo, hi = wilson(e64, B, 1.959963984540054)
    parity = {"frames": B,
              "fp32_mismatched_frames": _compare(o, out["info"], out["iters"],
                                                 out["pe"]),
              "fp64_fer": e64 / B, "fp64_fer_ci95": [lo, hi],
              "gpu_inside_fp64_ci95": bool(lo <= errs / B <= hi)}
    achieved = OPS_PER_PE * pe.sum() / (ms / 1e3) / 1e12
    line = _line(
        "decoded info Mbit/s, N=64 R=1/2 2.5dB, early stop",
        round(B * K / ms / 1e3, 3), "Mbit/s", steps, args.warmup, ms,
        {"workload": "polar BP decode, (64,32) code, BPSK/AWGN Eb/N0 "
                     f"{ebn0} dB, G-matrix early stop, no freezing",
         "N": N, "K": K, "ebn0_db": ebn0, "frames_per_step": B,
         "max_iter": max_iter, "alpha": alpha},
        avg_iters=round(float(out["iters"].mean()), 3),
        pe_per_frame=round(float(pe.mean()), 1), fer=errs / B,
        ms_per_step_median=round(med, 4), end_to_end_ms=round(e2e, 3),
        parity=parity,
        roofline=_alu_roofline(achieved, "c1", "bp_decode_wave_kernel<6, false, F32>",
                               B, ms, "12 operations per PE activation"))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(llr, K, out["info"], opts,
                                            args.cpu_seconds, chunk=256)
    return line


# Operations of one SC frame: m N / 2 evaluations of f (magnitude minimum,
# sign product) and m N / 2 of g (sign flip by the partial sum, addition)
def sc_ops_per_frame(N):
    return 2 * (N.bit_length() - 1) * N


def bench_sc(args, pbp, torch):
    """Successive-cancellation decoding of the (1024, 512) code on the
    headline's frames (3.0 dB, 10^6 frames): decode rate, error rate beside
    BP with early stop and freezing on the same frames, and the decisions
    against the SC oracle frame by frame (a sample of 2^16 frames, or every
    frame with --full-parity)."""
    import oracle
    N, K = 1024, 512
    ebn0 = 3.0 if args.ebn0 is None else args.ebn0
    B = args.batch or 10 ** 6
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, ebn0,
                              stream=(2 << 16) + 5)
    out = pbp.pbp_decode_sc(code, d_llr)
    ms = _timed(torch, lambda: pbp.pbp_decode_sc(code, d_llr, out=out),
                args.steps, args.warmup)
    got = out["info"].cpu().numpy()
    errs = int(np.sum(np.any(got != info, axis=1)))
    bp = pbp.pbp_decode(code, d_llr, max_iter=40, alpha=0.9375,
                        **MODES["es_frz"])
    bp_errs = int(np.sum(np.any(bp["info"].cpu().numpy() != info, axis=1)))
    z = 1.959963984540054
    fz = _oracle_frozen(N, K)

    def sc_oracle(x):
        return {"info": oracle.sc_decode(x, fz)[:, fz == 0]}

    S = B if args.full_parity else min(B, 1 << 16)
    _, _, threads = host_cpu()
    print(f"[parity] SC oracle on {S} frames", file=sys.stderr, flush=True)
    llr_s = d_llr[:S].cpu().numpy()
    parts = {}
    from concurrent.futures import ThreadPoolExecutor

    def job(lo):
        parts[lo] = sc_oracle(llr_s[lo:lo + 1024])["info"]
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(job, range(0, S, 1024)))
    ref = np.concatenate([parts[k] for k in sorted(parts)])
    mism = int(np.sum(np.any(ref != got[:S], axis=1)))
    achieved = sc_ops_per_frame(N) * B / (ms / 1e3) / 1e12
    line = _line(
        "decoded info Mbit/s, N=1024 R=1/2 3.0dB, successive cancellation",
        round(B * K / ms / 1e3, 2), "Mbit/s", args.steps, args.warmup, ms,
        {"workload": "polar SC decode, (1024,512) code, BPSK/AWGN Eb/N0 "
                     f"{ebn0} dB, the headline's frames",
         "N": N, "K": K, "ebn0_db": ebn0, "frames_per_step": B},
        fer=errs / B, fer_ci95=list(wilson(errs, B, z)),
        bp_es_freeze_fer=bp_errs / B,
        bp_es_freeze_fer_ci95=list(wilson(bp_errs, B, z)),
        parity={"frames": S, "mismatched_frames": mism},
        roofline=_alu_roofline(
            achieved, "sc", "sc_decode64_kernel<10>", B, ms,
            "2 m N operations per frame (m N / 2 f and m N / 2 g "
            "evaluations); one wavefront walks a frame's leaves in order"))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(
            llr_s[:1 << 16], K, got, {}, args.cpu_seconds, chunk=64,
            decode=sc_oracle, what="FP32 SC oracle")
    return line


def bench_quant(args, pbp, torch):
    """BP with saturating 8-bit fixed-point messages (3 fraction bits) on the
    headline's frames and mode (3.0 dB, 10^6 frames, early stop + freezing):
    decode rate, error rate beside FP32 BP on the same frames, and bits,
    iterations and PE counts against the fixed-point oracle frame by frame
    (a sample of 2^15 frames, or every frame with --full-parity)."""
    import oracle
    N, K, max_iter, alpha, bits, frac = 1024, 512, 40, 0.9375, 8, 3
    ebn0 = 3.0 if args.ebn0 is None else args.ebn0
    B = args.batch or 10 ** 6
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, ebn0,
                              stream=(2 << 16) + 5)
    opts = dict(MODES["es_frz"], max_iter=max_iter, alpha=alpha)
    out = pbp.pbp_decode_quant(code, d_llr, bits=bits, frac=frac, **opts)
    ms = _timed(torch, lambda: pbp.pbp_decode_quant(
        code, d_llr, bits=bits, frac=frac, out=out, **opts),
        args.steps, args.warmup)
    got = {k: v.cpu().numpy() for k, v in out.items()}
    errs = int(np.sum(np.any(got["info"] != info, axis=1)))
    bp = pbp.pbp_decode(code, d_llr, **opts)
    bp_errs = int(np.sum(np.any(bp["info"].cpu().numpy() != info, axis=1)))
    z = 1.959963984540054
    fz = _oracle_frozen(N, K)

    def q_oracle(x):
        return oracle.decode_quant(x, fz, bits=bits, frac=frac, **opts)

    S = B if args.full_parity else min(B, 1 << 15)
    _, _, threads = host_cpu()
    print(f"[parity] fixed-point oracle on {S} frames", file=sys.stderr,
          flush=True)
    llr_s = d_llr[:S].cpu().numpy()
    parts = {}
    from concurrent.futures import ThreadPoolExecutor

    def job(lo):
        parts[lo] = q_oracle(llr_s[lo:lo + 256])
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(job, range(0, S, 256)))
    o = {k: np.concatenate([parts[lo][k] for lo in sorted(parts)])
         for k in ("info", "iters", "pe")}
    mism = _compare(o, got["info"][:S], got["iters"][:S], got["pe"][:S])
    pe = got["pe"].astype(np.float64)
    achieved = OPS_PER_PE * pe.sum() / (ms / 1e3) / 1e12
    line = _line(
        "decoded info Mbit/s, N=1024 R=1/2 3.0dB, 8-bit fixed-point BP",
        round(B * K / ms / 1e3, 2), "Mbit/s", args.steps, args.warmup, ms,
        {"workload": "polar BP decode with saturating 8-bit messages (3 "
                     "fraction bits), (1024,512) code, BPSK/AWGN Eb/N0 "
                     f"{ebn0} dB, early stop + CSFG freezing, the headline's "
                     "frames",
         "N": N, "K": K, "ebn0_db": ebn0, "frames_per_step": B,
         "max_iter": max_iter, "alpha": alpha, "bits": bits, "frac": frac},
        avg_iters=round(float(got["iters"].mean()), 3),
        pe_per_frame=round(float(pe.mean()), 1),
        fer=errs / B, fer_ci95=list(wilson(errs, B, z)),
        fp32_fer=bp_errs / B, fp32_fer_ci95=list(wilson(bp_errs, B, z)),
        parity={"frames": S, "mismatched_frames": mism},
        roofline=_alu_roofline(achieved, "quant",
                               "quant_r10_kernel<true, true>", B, ms,
                               "12 operations per PE activation, as for FP32; "
                               "the saturations and roundings come on top"),
        messages="saturating 8-bit integers, carried exactly in FP32 "
                 "registers")
    # the integer messages are computed by FP32 instructions (exact here)
    line["dtype"] = "f32"
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(
            llr_s, K, got["info"], {}, args.cpu_seconds, chunk=16,
            decode=q_oracle, what="fixed-point oracle")
    return line


def bench_mixed(args, pbp, torch):
    """2^20 frames mixing N in {256, 1024, 4096} and R in {1/3, 1/2, 5/6}
    uniformly, Eb/N0 uniform in [1, 4] dB per frame, early stop + freezing,
    60 iterations, one mixed-code decode per step (autotuned first)."""
    import synth
    dims = [(n, int(n * r)) for n in (256, 1024, 4096)
            for r in (1 / 3, 1 / 2, 5 / 6)]
    B = args.batch or (1 << 20)
    stream = (3 << 16) + 1
    t0 = time.perf_counter()
    u = synth.uniform(B, stream=stream, word=0)
    cof = np.minimum((u * len(dims)).astype(np.int32), len(dims) - 1)
    ebn0 = 1.0 + 3.0 * synth.uniform(B, stream=stream, word=1)
    Ns = np.array([dims[c][0] for c in cof], np.int64)
    Ks = np.array([dims[c][1] for c in cof], np.int64)
    llr_off = np.concatenate([[0], np.cumsum(Ns)[:-1]]).astype(np.int64)
    info_off = np.concatenate([[0], np.cumsum(Ks)[:-1]]).astype(np.int64)
    d_llr = torch.empty(int(Ns.sum()), dtype=torch.float32, device="cuda")
    codes = []
    info_ref = {}
    for c, (N, K) in enumerate(dims):
        frozen = pbp.pbp_construct(N, K, 0.0)
        code = pbp.Code(N, K, frozen)
        codes.append(code)
        idx = np.flatnonzero(cof == c)
        info = synth.info_bits(K, len(idx), stream=stream * 16 + c + 1)
        info_ref[c] = (idx, info)
        cw = pbp.pbp_encode(code, torch.from_numpy(info).cuda()).cpu().numpy()
        # channel LLRs in chunks (bounded host memory), scattered to the
        # frames' offsets on the device
        for lo in range(0, len(idx), 16384):
            sl = slice(lo, lo + 16384)
            nz = synth.normals(N, len(idx[sl]), frame0=lo,
                               stream=stream * 16 + c + 1)
            llr = torch.from_numpy(synth.channel_llr(
                cw[sl], nz, ebn0[idx[sl]], K / N)).cuda()
            pos = torch.from_numpy(llr_off[idx[sl]]).cuda()[:, None] + \
                torch.arange(N, device="cuda")[None, :]
            d_llr[pos.reshape(-1)] = llr.reshape(-1)
    gen_s = time.perf_counter() - t0
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d_cof, d_lo, d_io = d(cof), d(llr_off), d(info_off)
    plan = pbp.MixedPlan(codes, B)
    opts = pbp.make_opts(max_iter=60, **MODES["es_frz"])
    nbits = int(Ks.sum())
    out = {"info": torch.empty(nbits, dtype=torch.uint8, device="cuda"),
           "iters": torch.empty(B, dtype=torch.int32, device="cuda"),
           "pe": torch.empty(B, dtype=torch.int64, device="cuda")}
    t1 = time.perf_counter()
    cfg = pbp.pbp_mixed_plan_tune(plan, d_cof, d_lo, d_io, d_llr, opts=opts,
                                  out=out, reps=1)
    tune_s = time.perf_counter() - t1
    steps = max(1, args.steps // 3)
    # both schedules at 16 wavefronts per compute unit: one launch over the
    # batch in the caller's order (order 0), and one launch per code,
    # longest first, after the device sort (order 1)
    schedules = {}
    for order in (0, 1):
        plan.config = (order, 16)
        ms_o = _timed(torch, lambda: pbp.pbp_decode_mixed(
            plan, d_cof, d_lo, d_io, d_llr, opts=opts, out=out), steps, 1)
        schedules[["single_launch", "per_code"][order]] = {
            "ms_per_step": round(ms_o, 3),
            "fill": round(pbp.pbp_mixed_plan_fill(plan), 4)}
    plan.config = cfg
    # the tuned step captured in a graph and replayed (the timed value)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        pbp.pbp_decode_mixed(plan, d_cof, d_lo, d_io, d_llr, opts=opts,
                             out=out, stream=side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        pbp.pbp_decode_mixed(plan, d_cof, d_lo, d_io, d_llr, opts=opts,
                             out=out, stream=side)
    torch.cuda.synchronize()
    ms = _timed(torch, graph.replay, steps, 1)
    ms_eager = _timed(torch, lambda: pbp.pbp_decode_mixed(
        plan, d_cof, d_lo, d_io, d_llr, opts=opts, out=out), steps, 1)
    fill = pbp.pbp_mixed_plan_fill(plan)
    pe_i = out["pe"].cpu().numpy()
    pe = pe_i.astype(np.float64)
    iters = out["iters"].cpu().numpy()
    bits = out["info"].cpu().numpy()
    extra = {}
    if args.full_parity:
        # CPU baseline leg: a seeded sample of 10^4 frames of the batch
        # through the FP32 oracle, code by code, timed and compared frame by
        # frame
        S = min(B, 10 ** 4)
        samp = np.sort(np.random.default_rng(2).choice(B, S, replace=False))
        threads = max(1, min(16, os.cpu_count() or 1))
        print(f"[parity] mixed: FP32 oracle on {S} sampled frames",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        bad = 0
        for c, (N, K) in enumerate(dims):
            fs = samp[cof[samp] == c]
            if len(fs) == 0:
                continue
            pos = torch.from_numpy(llr_off[fs]).cuda()[:, None] + \
                torch.arange(N, device="cuda")[None, :]
            llr_c = d_llr[pos.reshape(-1)].reshape(len(fs), N).cpu().numpy()
            o = _oracle_all(llr_c, _oracle_frozen(N, K),
                            dict(MODES["es_frz"], max_iter=60, alpha=0.9375),
                            threads, chunk=16)
            got = bits[info_off[fs][:, None] + np.arange(K)[None, :]]
            bad += _compare(o, got, iters[fs], pe_i[fs])
        wall = time.perf_counter() - t0
        extra["cpu_baseline"] = {
            "value": round(float(Ks[samp].sum()) / wall / 1e6, 3),
            "unit": "Mbit/s", "cores": threads, "kind": "oracle",
            "sample": f"{S} seeded frames of the batch, FP32 oracle, "
                      f"{threads} threads, {wall:.1f} s",
            "frames": S, "gpu_mismatches": bad}
    errs = 0
    for c, (idx, info) in info_ref.items():
        K = dims[c][1]
        got = bits[info_off[idx][:, None] + np.arange(K)[None, :]]
        errs += int(np.sum(np.any(got != info, axis=1)))
    ops = OPS_PER_PE * pe.sum() / (ms / 1e3) / 1e12
    # the dominant kernels: the N = 4096 codes' frames alone (the others
    # named as no code of the plan, so they are skipped), same plan
    long_codes = [c for c, (n, _) in enumerate(dims) if n == 4096]
    sel = np.isin(cof, long_codes)
    d_cof_long = d(np.where(sel, cof, np.int32(len(dims))).astype(np.int32))
    ms_long = _timed(torch, lambda: pbp.pbp_decode_mixed(
        plan, d_cof_long, d_lo, d_io, d_llr, opts=opts, out=out), steps, 1)
    pe_long = pe[sel]
    it_long = iters[sel].astype(np.float64)
    # messages stay on chip: the channel is read once per frame
    long_bytes = 4.0 * 4096 * sel.sum() + float(Ks[sel].sum()) + 12.0 * sel.sum()
    long_gbs = long_bytes / (ms_long / 1e3) / 1e9
    long_ops = OPS_PER_PE * pe_long.sum() / (ms_long / 1e3) / 1e12
    return _line(
        "decoded info Mbit/s, mixed N in {256,1024,4096} x R in "
        "{1/3,1/2,5/6}, Eb/N0 U[1,4] dB", round(nbits / ms / 1e3, 2),
        "Mbit/s", steps, 1, ms,
        {"workload": "mixed-code persistent decode, 2^20 frames, (N, R) "
                     "uniform over 9 codes, early stop + CSFG freezing, max "
                     "60 iterations", "frames_per_step": B,
         "codes": [list(x) for x in dims]},
        frames_per_s=round(B / ms * 1e3, 1), fill_efficiency=round(fill, 4),
        tuned_config={"order": cfg[0], "waves_per_cu": cfg[1]},
        timed="replays of the tuned step captured in a HIP graph",
        eager_ms_per_step=round(ms_eager, 3), schedules=schedules,
        avg_iters=round(float(iters.mean()), 3),
        pe_per_frame=round(float(pe.mean()), 1), fer=errs / B,
        roofline=dict(
            _alu_roofline(long_ops, "mixed", "class_pair_kernel<12>", B,
                          ms_long, "12 operations per PE activation of the "
                          "N = 4096 frames decoded alone (three launches, "
                          "one per rate, messages on chip)"),
            hbm_gbs=round(long_gbs, 1)),
        step_valu={"achieved": round(ops, 3),
                   "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
                   "frac": round(ops / VALU_PEAK_TOPS, 4)},
        input_generation_s=round(gen_s, 2), tune_s=round(tune_s, 2),
        **extra)


# Operations per PE activation of one round-trip pass, counted as for the
# single sweep: each pass computes two outputs of eq. (1), each a min-sum
# term (sign product, magnitude minimum, scaling) and an addition
OPS_PER_PE_PASS = 8


def bench_round_trip(args, pbp, torch):
    """The round-trip schedule (an L pass over stages m..1, then an R pass
    over stages 1..m, per iteration; early stop, no freezing) on the
    headline's frames: (1024, 512) code, 3.0 dB, 10^6 frames.  The single
    sweep with early stop is timed on the same frames beside it."""
    import oracle
    N, K, B, max_iter, alpha = 1024, 512, args.batch or 10 ** 6, 40, 0.9375
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    ebn0 = 3.0 if args.ebn0 is None else args.ebn0
    info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, ebn0,
                              stream=(2 << 16) + 5)
    base = dict(early_stop=True, freezing=False, max_iter=max_iter,
                alpha=alpha)
    res = {}
    for name, sched, es in (("round_trip", "round_trip", True),
                            ("single", "single", True),
                            ("plain40", "single", False)):
        ms, _, out, med, _ = time_mode(pbp, torch, code, d_llr,
                                       dict(base, schedule=sched,
                                            early_stop=es),
                                       args.steps, args.warmup)
        errs = int(np.sum(np.any(out["info"] != info, axis=1)))
        res[name] = dict(ms=ms, median=med, errors=errs, fer=errs / B,
                         iters=float(out["iters"].mean()),
                         pe=float(out["pe"].mean()),
                         mbps=B * K / (ms / 1e3) / 1e6, info=out["info"])
    r, s1, p40 = res["round_trip"], res["single"], res["plain40"]
    achieved = OPS_PER_PE_PASS * r["pe"] * B / (r["ms"] / 1e3) / 1e12
    line = _line(
        "decoded info Mbit/s at N=1024 R=1/2 3.0dB, round-trip BP schedule "
        "with early stop", round(r["mbps"], 2), "Mbit/s", args.steps,
        args.warmup, r["ms"],
        {"workload": f"polar BP decode, (1024,512) code, BPSK/AWGN Eb/N0 "
                     f"{ebn0} dB, round-trip schedule, early stop",
         "N": N, "K": K, "ebn0_db": ebn0, "frames_per_step": B,
         "max_iter": max_iter, "alpha": alpha},
        ms_per_step_median=round(r["median"], 4),
        avg_iters=round(r["iters"], 3), pe_per_frame=round(r["pe"], 1),
        fer=r["fer"], fer_ci95=list(wilson(r["errors"], B, 1.959963984540054)),
        single_sweep_early_stop={
            "mbps": round(s1["mbps"], 2), "ms_per_step": round(s1["ms"], 4),
            "fer": s1["fer"],
            "fer_ci95": list(wilson(s1["errors"], B, 1.959963984540054)),
            "avg_iters": round(s1["iters"], 3),
            "pe_per_frame": round(s1["pe"], 1)},
        plain40={
            "mbps": round(p40["mbps"], 2), "ms_per_step": round(p40["ms"], 4),
            "fer": p40["fer"],
            "fer_ci95": list(wilson(p40["errors"], B, 1.959963984540054)),
            "avg_iters": round(p40["iters"], 3),
            "pe_per_frame": round(p40["pe"], 1)},
        # context only: the round trip has no freezing, so this is not the
        # freezing decoder's speed-up (that is the headline line's)
        speedup_vs_plain40_context=round(r["mbps"] / p40["mbps"], 3),
        roofline=_alu_roofline(achieved, "round_trip",
                               "bp_round_trip_kernel<10>", B, r["ms"],
                               "8 operations per PE activation of one pass, "
                               "m N activations per iteration"))
    if not args.no_cpu_baseline:
        d_host = d_llr[:min(B, 1 << 19)].cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(
            d_host, K, r["info"],
            dict(base, schedule=oracle.SCHEDULE_ROUND_TRIP),
            args.cpu_seconds)
    return line


def _training_step_ms(pbp, torch, N, K, T, B, steps, stream):
    """Time one training step (forward, BCE, backward, SGD update) of the
    unrolled decoder on a fresh batch of the (N, K) code."""
    import synth
    m = N.bit_length() - 1
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    ebn0 = 1.0 + 3.0 * synth.uniform(B, stream=stream, word=1)
    info = synth.info_bits(K, B, stream=stream)
    cw = pbp.pbp_encode(code, torch.from_numpy(info).cuda()).cpu().numpy()
    llr = synth.channel_llr(cw, synth.normals(N, B, stream=stream), ebn0,
                            K / N)
    d_llr = torch.from_numpy(llr).cuda()
    info_pos = torch.from_numpy(np.flatnonzero(frozen == 0)).cuda()
    u_info = torch.from_numpy(info.astype(np.float32)).cuda()
    alpha = torch.full((T, m, 2), 0.9375, dtype=torch.float32, device="cuda",
                       requires_grad=True)
    opt = torch.optim.SGD([alpha], lr=0.01)

    def step():
        opt.zero_grad(set_to_none=False)
        loss = pbp.info_bce(pbp.unrolled_bp(d_llr, alpha, code), u_info,
                            info_pos)
        loss.backward()
        opt.step()

    return _timed(torch, step, steps, 2)


def bench_unrolled(args, pbp, torch):
    """One training step of the unrolled decoder: (1024, 512) code, T = 20,
    4096 frames at Eb/N0 uniform in [1, 4] dB: forward with checkpoints,
    BCE of the information bits, backward to the 400 scales.  The (128, 64)
    code's step is timed beside it."""
    import synth
    N, K, T = 1024, 512, 20
    m = 10
    B = args.batch or 4096
    stream = (4 << 16) + 1
    ms128 = _training_step_ms(pbp, torch, 128, 64, T, B, max(1, args.steps),
                              (4 << 16) + 2)
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    ebn0 = 1.0 + 3.0 * synth.uniform(B, stream=stream, word=1)
    info = synth.info_bits(K, B, stream=stream)
    cw = pbp.pbp_encode(code, torch.from_numpy(info).cuda()).cpu().numpy()
    llr = synth.channel_llr(cw, synth.normals(N, B, stream=stream), ebn0,
                            K / N)
    d_llr = torch.from_numpy(llr).cuda()
    info_pos = torch.from_numpy(np.flatnonzero(frozen == 0)).cuda()
    u_info = torch.from_numpy(info.astype(np.float32)).cuda()
    alpha = torch.full((T, m, 2), 0.9375, dtype=torch.float32, device="cuda",
                       requires_grad=True)
    opt = torch.optim.SGD([alpha], lr=0.01)

    def step():
        opt.zero_grad(set_to_none=False)
        loss = pbp.info_bce(pbp.unrolled_bp(d_llr, alpha, code), u_info,
                            info_pos)
        loss.backward()
        opt.step()

    steps = max(1, args.steps)
    ms = _timed(torch, step, steps, 2)
    # forward and backward kernels alone
    a = alpha.detach().clone()
    ck = torch.empty((T, B, m - 1, N), dtype=torch.float32, device="cuda")
    o = torch.empty((B, N), dtype=torch.float32, device="cuda")
    fwd_ms = _timed(torch, lambda: pbp.pbp_unrolled_forward(
        code, d_llr, a, ckpt=ck, out=o), steps, 1)
    dout = torch.randn((B, N), device="cuda")
    bwd_ms = _timed(torch, lambda: pbp.pbp_unrolled_backward(
        code, d_llr, a, ck, dout), steps, 1)
    ck_bytes = 4.0 * T * B * (m - 1) * N
    fwd_gbs = (ck_bytes + 8.0 * B * N) / (fwd_ms / 1e3) / 1e9
    # backward: checkpoints read once, LLRs and output gradients read,
    # channel gradients and per-frame scale gradients written
    bwd_bytes = ck_bytes + 12.0 * B * N + 4.0 * B * T * m * 2
    bwd_gbs = bwd_bytes / (bwd_ms / 1e3) / 1e9
    pe = float(T) * m * N / 2 * B
    return _line(
        "unrolled BP training step, frames/s (N=1024, T=20)",
        round(B / ms * 1e3, 1), "frames/s", steps, 2, ms,
        {"workload": "unrolled BP training step, (1024,512) code, T=20, "
                     "400 scales, 4096 frames, Eb/N0 U[1,4] dB",
         "N": N, "K": K, "T": T, "frames_per_step": B},
        forward_ms=round(fwd_ms, 4), backward_ms=round(bwd_ms, 4),
        n128_training_step={"ms_per_step": round(ms128, 4),
                            "frames_per_s": round(B / ms128 * 1e3, 1),
                            "code": [128, 64], "T": T, "frames_per_step": B},
        roofline={"bound": "hbm", "achieved": round(bwd_gbs, 1),
                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(bwd_gbs / HBM_PEAK_GBS, 4),
                  "traffic": measured_traffic("unrolled", B),
                  "kernel": "unrolled_backward_kernel<10>",
                  "kernel_ms": _round(traced_kernel_ms(
                      "unrolled", "unrolled_backward_kernel<10>", B), 4),
                  "event_ms": round(bwd_ms, 4),
                  "valu_issue_frac": _round(valu_issue(
                      "unrolled", "unrolled_backward_kernel<10>", B, bwd_ms), 4),
                  "note": "checkpoint reads (T x B x (m-1) x N x 4 B), LLR "
                          "and output-gradient reads, gradient writes; the "
                          "kernel issues VALU at valu_issue_frac of the lane "
                          "rate, which bounds it before HBM does"},
        forward_roofline={"bound": "hbm", "achieved": round(fwd_gbs, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(fwd_gbs / HBM_PEAK_GBS, 4),
                          "kernel": "unrolled_forward_kernel<10>"},
        valu_forward={"achieved": round(OPS_PER_PE * pe / (fwd_ms / 1e3) / 1e12, 3),
                      "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s"})


SWEEP_MODES = {
    "plain40": dict(early_stop=False, freezing=False),
    "early_stop": dict(early_stop=True, freezing=False),
    "es_freeze_total": dict(early_stop=True, freezing=True, freeze_input=1,
                            freeze_walk=0),
    "es_freeze_r": dict(early_stop=True, freezing=True, freeze_input=0,
                        freeze_walk=0),
    "freeze_only": dict(early_stop=False, freezing=True, freeze_input=1,
                        freeze_walk=0),
    "es_freeze_stage": dict(early_stop=True, freezing=True, freeze_input=1,
                            freeze_walk=1),
    "es_freeze_greedy": dict(early_stop=True, freezing=True, freeze_input=1,
                             freeze_walk=2),
    # the round-trip schedule with early stop (pbp_decode_round_trip)
    "round_trip_es": dict(early_stop=True, freezing=False,
                          schedule="round_trip"),
}


def bench_sweep(args, pbp, torch):
    """The (1024, 512) code over Eb/N0 1.0 .. 3.5 dB: every decoding mode
    (plain, early stop, early stop with each freezing reading, freezing
    alone) on the same LLRs per point; error rate, iterations, PE updates
    per frame and decode rate."""
    N, K, max_iter, alpha = 1024, 512, 40, 0.9375
    B = args.batch or 10 ** 6
    frozen = pbp.pbp_construct(N, K, 0.0)
    code = pbp.Code(N, K, frozen)
    points = [1.0, 1.5, 2.0, 2.5, 3.0, 3.5]
    fz_oracle = _oracle_frozen(N, K) if args.full_parity else None
    table = []
    total_ms = 0.0
    for k, eb in enumerate(points):
        info, d_llr = make_inputs(pbp, torch, code, frozen, N, K, B, eb,
                                  stream=(2 << 16) + k)
        row = {"ebn0_db": eb}
        for name, mode in SWEEP_MODES.items():
            opts = dict(mode, max_iter=max_iter, alpha=alpha)
            out = pbp.pbp_decode(code, d_llr, **opts)
            ms = _timed(torch, lambda: pbp.pbp_decode(code, d_llr, out=out,
                                                      **opts), 1, 0)
            total_ms += ms
            errs = int(np.sum(np.any(out["info"].cpu().numpy() != info,
                                     axis=1)))
            lo, hi = wilson(errs, B, 1.959963984540054)
            row[name] = {"fer": errs / B, "fer_ci95": [lo, hi],
                         "avg_iters": round(float(out["iters"].float().mean()), 3),
                         "pe_per_frame": round(float(out["pe"].double().mean()), 1),
                         "mbps": round(B * K / ms / 1e3, 1)}
            if args.full_parity and name in ("plain40", "early_stop",
                                             "es_freeze_total",
                                             "round_trip_es"):
                # CPU baseline leg: the first 10^5 frames of the point
                # through the FP32 oracle, compared frame by frame
                S = min(B, 10 ** 5)
                print(f"[parity] {eb} dB {name}: FP32 oracle on {S} frames",
                      file=sys.stderr, flush=True)
                oo = dict(opts)
                if oo.pop("schedule", "single") == "round_trip":
                    import oracle
                    oo["schedule"] = oracle.SCHEDULE_ROUND_TRIP
                o = _oracle_all(d_llr[:S].cpu().numpy(), fz_oracle, oo,
                                max(1, min(16, os.cpu_count() or 1)))
                row[name]["oracle_frames"] = S
                row[name]["oracle_mismatched_frames"] = _compare(
                    o, out["info"][:S].cpu().numpy(),
                    out["iters"][:S].cpu().numpy(), out["pe"][:S].cpu().numpy())
        # successive cancellation on the same LLRs
        sc = pbp.pbp_decode_sc(code, d_llr)
        ms = _timed(torch, lambda: pbp.pbp_decode_sc(code, d_llr, out=sc), 1, 0)
        errs = int(np.sum(np.any(sc["info"].cpu().numpy() != info, axis=1)))
        lo, hi = wilson(errs, B, 1.959963984540054)
        row["sc"] = {"fer": errs / B, "fer_ci95": [lo, hi],
                     "mbps": round(B * K / ms / 1e3, 1)}
        table.append(row)
        del d_llr
        print(f"[sweep] {eb} dB done", file=sys.stderr, flush=True)
    at3 = next(r for r in table if r["ebn0_db"] == 3.0)
    base, es, fz = at3["plain40"], at3["early_stop"], at3["es_freeze_total"]
    ctx = {"iterations_vs_plain40": round(1 - fz["avg_iters"] / base["avg_iters"], 4),
           "iterations_vs_early_stop": round(1 - fz["avg_iters"] / es["avg_iters"], 4),
           "pe_vs_plain40": round(1 - fz["pe_per_frame"] / base["pe_per_frame"], 4),
           "pe_vs_early_stop": round(1 - fz["pe_per_frame"] / es["pe_per_frame"], 4)}
    return _line(
        "FER / iterations / PE updates per frame over Eb/N0, N=1024 R=1/2, "
        "all decoding modes", round(fz["mbps"], 2), "Mbit/s (3.0 dB, early "
        "stop + freezing)", 1, 0, total_ms,
        {"workload": "(1024,512) code, Eb/N0 1.0-3.5 dB, "
                     f"{B} frames per point, {len(SWEEP_MODES)} BP modes "
                     "and SC decoding on the same LLRs",
         "frames_per_point": B, "max_iter": max_iter, "alpha": alpha},
        reductions_at_3db=ctx,
        paper_reductions_at_3db={"iterations_vs_plain40": 0.46,
                                 "iterations_vs_early_stop": 0.17,
                                 "pe_vs_plain40": 0.65,
                                 "pe_vs_early_stop": 0.46},
        table=table)


if __name__ == "__main__":
    main()
