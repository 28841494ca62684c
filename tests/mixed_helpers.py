"""Test-side recipe of a mixed batch: frames of several codes, each frame's
code and Eb/N0 drawn from seeded generators, its LLRs at a 16-byte aligned
offset of one flat buffer and its information bits at an offset of one flat
byte buffer.  Inputs come from ``synth`` and the oracle's encoder only."""

import numpy as np

import oracle
import synth
from helpers import frozen_mask

# the (N, K) set of the mixed workload: N in {256, 1024, 4096} x rate in
# {1/3, 1/2, 5/6}, K = floor(N R)
MIX = [(256, 85), (256, 128), (256, 213), (1024, 341), (1024, 512),
       (1024, 853), (4096, 1365), (4096, 2048), (4096, 3413)]


def layout(codes, code_of_frame):
    Ns = np.array([codes[c][0] for c in code_of_frame], np.int64)
    Ks = np.array([codes[c][1] for c in code_of_frame], np.int64)
    pad = (Ns + 3) // 4 * 4
    llr_off = np.concatenate([[0], np.cumsum(pad)[:-1]]).astype(np.int64)
    info_off = np.concatenate([[0], np.cumsum(Ks)[:-1]]).astype(np.int64)
    return llr_off, info_off, int(pad.sum()), int(Ks.sum())


def make_mixed(codes, B, stream, ebn0_range=(1.0, 4.0), seed=0):
    """Returns code_of_frame, ebn0 per frame, llr_off, info_off, the flat LLR
    buffer (float32) and each frame's information bits (list)."""
    u = synth.uniform(B, stream=stream, word=0)
    code_of_frame = np.minimum((u * len(codes)).astype(np.int32),
                               len(codes) - 1)
    e = synth.uniform(B, stream=stream, word=1)
    ebn0 = ebn0_range[0] + (ebn0_range[1] - ebn0_range[0]) * e
    llr_off, info_off, nllr, ninfo = layout(codes, code_of_frame)
    llr = np.zeros(nllr, np.float32)
    info = [None] * B
    for c, (N, K) in enumerate(codes):
        idx = np.flatnonzero(code_of_frame == c)
        if len(idx) == 0:
            continue
        fz = frozen_mask(N, K)
        # each code's frames draw from their own stream, in batch order
        st = stream * 16 + c + 1
        bits = synth.info_bits(K, len(idx), stream=st)
        uw = np.zeros((len(idx), N), np.uint8)
        uw[:, fz == 0] = bits
        x = oracle.encode(uw)
        nz = synth.normals(N, len(idx), stream=st)
        l = synth.channel_llr(x, nz, ebn0[idx], max(K, 1) / N)
        for j, f in enumerate(idx):
            llr[llr_off[f]:llr_off[f] + N] = l[j]
            info[f] = bits[j]
    return code_of_frame, ebn0, llr_off, info_off, llr, info
