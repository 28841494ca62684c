"""Seeded synthetic inputs for the polar BP decoder and its oracle.

This module is the only code shared by the CPU oracle and the GPU path.  It
draws random numbers and applies the channel model; it holds none of the
decoder's arithmetic (no construction, no encoding, no message passing):

* ``philox4x32_10`` -- the Philox4x32-10 counter-based generator of Salmon,
  Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
  (SC'11), written from its published definition.
* ``info_bits``      -- uniform information bits per frame.
* ``normals``        -- standard normals by the Box-Muller transform in FP64.
* ``channel_llr``    -- BPSK over AWGN and the channel LLR 2y/sigma^2, the
  simulation setup of the paper's Section IV (BPSK, AWGN), with
  sigma^2 = 1 / (2 R Eb/N0) and R = K/N.
* ``uniform``        -- per-frame uniform doubles (mixed-workload Eb/N0 and
  code choice).

Counter layout, per draw: ``ctr = (word, frame_lo, frame_hi, purpose)`` and
``key = (seed, stream)``.  Every frame's draws depend only on
(seed, stream, frame, word), so any frame range can be regenerated alone.
"""

from .philox import (PURPOSE_BITS, PURPOSE_NOISE, PURPOSE_UNIFORM, SEED,
                     philox4x32_10)
from .draws import (channel_llr, ebn0_to_sigma2, info_bits, normals, uniform,
                    stream_id)

__all__ = [
    "SEED", "PURPOSE_BITS", "PURPOSE_NOISE", "PURPOSE_UNIFORM",
    "philox4x32_10", "info_bits", "normals", "uniform", "channel_llr",
    "ebn0_to_sigma2", "stream_id",
]
