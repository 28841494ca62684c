"""The seeded input generator: pinned to the published Philox4x32-10
known-answer vectors and to the moments of its distributions."""

import numpy as np

import synth

# Known-answer vectors of Philox4x32-10 published with the Random123
# library of Salmon et al. (SC'11): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2,
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def test_philox_known_answers():
    for ctr, key, want in KAT:
        got = synth.philox4x32_10(*ctr, *key)
        assert tuple(int(v) for v in got) == want


def test_philox_vectorised_matches_scalar():
    c0 = np.arange(50, dtype=np.uint64)
    v = synth.philox4x32_10(c0, 7, 9, 1, 12345, 678)
    for i in range(50):
        s = synth.philox4x32_10(i, 7, 9, 1, 12345, 678)
        assert all(int(v[q][i]) == int(s[q]) for q in range(4))


def test_frame_slices_are_independent_of_batching():
    a = synth.normals(64, 40, frame0=0, stream=3)
    b = synth.normals(64, 15, frame0=25, stream=3)
    assert np.array_equal(a[25:], b)
    ia = synth.info_bits(300, 40, frame0=0, stream=3)
    ib = synth.info_bits(300, 5, frame0=35, stream=3)
    assert np.array_equal(ia[35:], ib)
    assert not np.array_equal(synth.normals(64, 4, stream=3),
                              synth.normals(64, 4, stream=4))


def test_normal_and_bit_moments():
    z = synth.normals(1024, 200, stream=11).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(z ** 4) - 3) < 0.05
    bits = synth.info_bits(512, 400, stream=11)
    assert abs(bits.mean() - 0.5) < 5 * 0.5 / np.sqrt(bits.size)
    u = synth.uniform(100000, stream=2)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.005


def test_channel_llr_statistics():
    # BPSK of the all-zero word: LLR ~ N(2/sigma^2, 4/sigma^2)
    N, B, ebn0 = 1024, 200, 3.0
    s2 = synth.ebn0_to_sigma2(ebn0, 0.5)
    assert abs(s2 - 0.5011872336272722) < 1e-15
    llr = synth.channel_llr(np.zeros((B, N), np.uint8),
                            synth.normals(N, B, stream=5), ebn0, 0.5)
    assert llr.dtype == np.float32
    assert abs(llr.mean() - 2 / s2) < 0.02
    assert abs(llr.std() - 2 / np.sqrt(s2)) < 0.02
    # a one bit flips the sign of the noiseless term
    ones = synth.channel_llr(np.ones((1, 4), np.uint8), np.zeros((1, 4)), ebn0, 0.5)
    assert np.allclose(ones, -2 / s2)
