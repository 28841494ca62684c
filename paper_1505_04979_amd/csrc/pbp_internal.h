// Internal declarations shared by the host and kernel translation units of
// libpbp (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pbp.h"

struct pbp_code {
    int32_t N = 0, K = 0, m = 0;
    int device = 0;
    std::vector<uint8_t> frozen;       // host, N bytes
    std::vector<int32_t> info_pos;     // host, K positions, increasing
    uint64_t *d_frozen_words = nullptr;  // device, frozen bit mask, row i is
                                         // bit (i & 63) of word i >> 6
    int32_t *d_info_pos = nullptr;     // device, K entries (at least 1)
    int64_t state_slots = 0;           // message-state slots of codes whose
    int64_t state_floats_per_slot = 0; // state does not fit in LDS
    int cus = 0;                       // compute units of the device
    uint64_t *d_fzw10 = nullptr;       // N = 1024: frozen ballot words [4][16]
};

namespace pbp {

inline bool valid_n(int32_t N)
{
    return N >= 2 && N <= 16384 && (N & (N - 1)) == 0;
}

inline int log2i(int32_t N)
{
    int m = 0;
    while ((1 << m) < N)
        m++;
    return m;
}

// Largest code length whose full message state lives in LDS (the generic
// and register decoders), and largest whose messages stay on chip (the
// workgroup decoder of N = 2048 and 4096 keeps half its L columns in VGPRs).
constexpr int kMaxLdsLog = 10;
constexpr int kMaxOnChipLog = 12;

// Device scratch of the decoders on one (device, stream): the [frame, exit]
// counters of the persistent kernels (zero between launches) and the
// message-state slots of codes longer than 1024.  Owned by the library, not
// the code handle, so that one handle serves several streams at once.
struct Workspace {
    int *counter = nullptr;
    float *state = nullptr;
};

// The workspace of `stream` on the handle's device, created on first use and
// grown (after synchronising that stream) when a longer code needs more
// state.  Calls on one stream are ordered, so they share it safely.
int32_t stream_workspace(const pbp_code *code, hipStream_t stream,
                         Workspace *out);

}  // namespace pbp
