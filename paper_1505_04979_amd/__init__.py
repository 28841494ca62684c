"""MI355X-native belief-propagation decoding of polar codes with
sub-factor-graph freezing (Abbas, Fan, Chen, Tsui).

The decoder is hand-written HIP for gfx950 behind the C-ABI of
include/pbp.h; this package is its Python binding (device memory and streams
come from torch).  Build the library with ``python -m
paper_1505_04979_amd.build``.
"""

from .binding import (Code, MixedPlan, PbpError, exported_symbols, lib,  # noqa
                      make_opts, pbp_code_create, pbp_code_dims, pbp_construct,
                      pbp_decode, pbp_decode_mixed, pbp_decode_opts,
                      pbp_decode_noalloc, pbp_decode_quant,
                      pbp_decode_round_trip, pbp_decode_sc,
                      pbp_encode, pbp_mixed_config, pbp_mixed_plan_create,
                      pbp_mixed_plan_fill, pbp_mixed_plan_tune,
                      pbp_unrolled_backward, pbp_unrolled_forward,
                      pbp_workspace_release, status_string)
from .unrolled import UnrolledBP, info_bce, unrolled_bp  # noqa
