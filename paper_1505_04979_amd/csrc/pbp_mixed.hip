// Persistent decoding of a batch that mixes codes (lengths and rates).
//
// Two schedules, both a work queue of frames drained by persistent
// wavefronts that each take the next entry from a device counter when they
// finish a frame, and both decoding each frame exactly as pbp_decode does:
//
// order 0 -- one launch for the whole batch, frames in the caller's order.
//   One kernel dispatches on the frame's code length: N = 1024 frames run
//   the register-resident decoder, N <= 512 the generic decoder with its
//   state in the wavefront's LDS, N >= 2048 the generic decoder on one
//   wavefront with L in that wavefront's device-memory slot.
//
// order 1 -- frames grouped by code, longest code first.  A device counting
//   sort builds the queue (an order array of frame indices, one contiguous
//   segment per code); each code's segment is then drained by a kernel
//   specialised for its length: N = 2048 and 4096 by workgroups of N / 4
//   threads with every message on chip (pbp_pair_decoder.h), longer codes
//   by 256-thread workgroups that share one slot per frame.
//
// The last wavefront out of a launch rewinds its counters, so the enqueued
// work needs no host-side or memset reset and can be captured in a graph and
// replayed.  The order and the number of resident wavefronts per compute
// unit are set by the caller or chosen by timing the candidates on a sample
// batch (pbp_mixed_plan_tune), with results cached per device, code set and
// mode for the life of the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "pbp.h"
#include "pbp_generic_decoder.h"
#include "pbp_internal.h"
#include "pbp_pair_decoder.h"
#include "pbp_r10.h"
#include "pbp_r10_decoder.h"

namespace {

constexpr int kMaxCodes = 16;
constexpr int kMaxWavesPerCu = 16;
constexpr int kMaxLongGroupsPerCu = 4;   // 256-thread groups of long codes
constexpr int64_t kMaxFrames = 1ll << 30;

struct CodeDesc {
    int32_t m, K;
    const uint64_t *frozen_words;
    const int32_t *info_pos;
    const uint64_t *fzw10;      // N = 1024 register decoder words, or null
};

// One code's share of a mixed launch.
struct ClassParams {
    CodeDesc code;
    const int *bounds;          // bucket starts (bounds[b] .. bounds[b+1])
    int32_t bucket;
    const int32_t *order;       // queue position -> frame
    const int64_t *llr_off;
    const int64_t *info_off;
    const float *llr;
    int32_t max_iter, early_stop, freezing, freeze_input, freeze_walk;
    float alpha;
    uint8_t *info_out;
    int32_t *iters_out;
    int64_t *pe_out;
    int *counter;               // [queue head, waves out] of this code
    float *state;               // device slots (long codes)
    int64_t slot_floats;
    int64_t *stats;             // per wavefront: start, end, busy (ticks)
};

using pbp::generic::DecodeParams;
using pbp::generic::decode_frame;

// One wavefront per frame.  PATH: 0 = generic decoder, state in LDS;
// 10 = register decoder with early stop; 11 = register decoder without early
// stop (freezing switched at run time)
template <int M, int PATH>
__global__ __launch_bounds__(64, 2) void class_kernel(ClassParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = (int)__builtin_amdgcn_workitem_id_x();
    const int64_t wave = blockIdx.x;
    const int lo = P.bounds[P.bucket], hi = P.bounds[P.bucket + 1];
    const int64_t t_start = wall_clock64();
    int64_t busy = 0;
    for (;;) {
        int q = 0;
        if (lane == 0)
            q = atomicAdd(P.counter, 1);
        q = __builtin_amdgcn_readfirstlane(__shfl(q, 0, 64)) + lo;
        if (q >= hi)
            break;
        const int64_t t0 = wall_clock64();
        const int f = __builtin_amdgcn_readfirstlane(P.order[q]);
        const float *llr = P.llr + P.llr_off[f];
        uint8_t *info = P.info_out + P.info_off[f];
        if constexpr (PATH >= 10) {
            pbp::r10::Params R{};
            R.llr = llr;
            R.B = 1;
            R.fzw = P.code.fzw10;
            R.info_pos = P.code.info_pos;
            R.K = P.code.K;
            R.max_iter = P.max_iter;
            R.freezing = P.freezing;
            R.freeze_input = P.freeze_input;
            R.freeze_walk = P.freeze_walk;
            R.alpha = P.alpha;
            R.info_out = info;
            R.iters_out = P.iters_out + f;
            R.pe_out = P.pe_out ? P.pe_out + f : nullptr;
            R.soft_out = nullptr;
            pbp::r10::Decoder<true, PATH == 10> D(
                R, *reinterpret_cast<pbp::r10::Smem *>(smem), lane);
            D.decode(0);
        } else {
            DecodeParams D{};
            D.llr = llr;
            D.B = 1;
            D.frozen_words = P.code.frozen_words;
            D.info_pos = P.code.info_pos;
            D.K = P.code.K;
            D.max_iter = P.max_iter;
            D.early_stop = P.early_stop;
            D.freezing = P.freezing;
            D.freeze_input = P.freeze_input;
            D.freeze_walk = P.freeze_walk;
            D.alpha = P.alpha;
            D.info_out = info;
            D.iters_out = P.iters_out + f;
            D.pe_out = P.pe_out ? P.pe_out + f : nullptr;
            D.soft_out = nullptr;
            decode_frame<M, PATH, true>(D, 0, smem, nullptr, lane, 64);
        }
        busy += wall_clock64() - t0;
    }
    if (lane == 0) {
        P.stats[wave * 3] = t_start;
        P.stats[wave * 3 + 1] = wall_clock64();
        P.stats[wave * 3 + 2] = busy;
        // every wavefront has taken its last queue entry before it counts
        // itself out; the last one out rewinds both counters
        if (atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(P.counter, 0);
            atomicExch(P.counter + 1, 0);
        }
    }
}

// Long codes: a 256-thread workgroup decodes each frame (L in the
// workgroup's device slot, the working R column in LDS).
constexpr int kWgThreads = 256;

// at m = 14 two groups fit a compute unit's LDS, as in the batch kernel
template <int M>
__global__ __launch_bounds__(kWgThreads, M >= 14 ? 2 : 4) void class_wg_kernel(ClassParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_q;
    const int tid = (int)threadIdx.x;
    const int64_t wg = blockIdx.x;
    float *gslot = P.state + wg * P.slot_floats;
    const int lo = P.bounds[P.bucket], hi = P.bounds[P.bucket + 1];
    const int64_t t_start = wall_clock64();
    int64_t busy = 0;
    for (;;) {
        if (tid == 0)
            s_q = atomicAdd(P.counter, 1) + lo;
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= hi)
            break;
        const int64_t t0 = wall_clock64();
        const int f = P.order[q];
        DecodeParams D{};
        D.llr = P.llr + P.llr_off[f];
        D.B = 1;
        D.frozen_words = P.code.frozen_words;
        D.info_pos = P.code.info_pos;
        D.K = P.code.K;
        D.max_iter = P.max_iter;
        D.early_stop = P.early_stop;
        D.freezing = P.freezing;
        D.freeze_input = P.freeze_input;
        D.freeze_walk = P.freeze_walk;
        D.alpha = P.alpha;
        D.info_out = P.info_out + P.info_off[f];
        D.iters_out = P.iters_out + f;
        D.pe_out = P.pe_out ? P.pe_out + f : nullptr;
        D.soft_out = nullptr;
        decode_frame<M, 1, false>(D, 0, smem, gslot, tid, kWgThreads);
        busy += wall_clock64() - t0;
    }
    if (tid == 0) {
        P.stats[wg * 3] = t_start;
        P.stats[wg * 3 + 1] = wall_clock64();
        P.stats[wg * 3 + 2] = busy;
        if (atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(P.counter, 0);
            atomicExch(P.counter + 1, 0);
        }
    }
}

// N = 2048 and 4096: the workgroup-resident decoder, N / 4 threads per
// frame, every message on chip.
template <int M>
__global__ __launch_bounds__(pbp::pair::Shape<M>::NT) void class_pair_kernel(ClassParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_q;
    const int tid = (int)threadIdx.x;
    const int64_t wg = blockIdx.x;
    const int lo = P.bounds[P.bucket], hi = P.bounds[P.bucket + 1];
    const int64_t t_start = wall_clock64();
    int64_t busy = 0;
    for (;;) {
        if (tid == 0)
            s_q = atomicAdd(P.counter, 1) + lo;
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= hi)
            break;
        const int64_t t0 = wall_clock64();
        const int f = P.order[q];
        DecodeParams D{};
        D.llr = P.llr + P.llr_off[f];
        D.B = 1;
        D.frozen_words = P.code.frozen_words;
        D.info_pos = P.code.info_pos;
        D.K = P.code.K;
        D.max_iter = P.max_iter;
        D.early_stop = P.early_stop;
        D.freezing = P.freezing;
        D.freeze_input = P.freeze_input;
        D.freeze_walk = P.freeze_walk;
        D.alpha = P.alpha;
        D.info_out = P.info_out + P.info_off[f];
        D.iters_out = P.iters_out + f;
        D.pe_out = P.pe_out ? P.pe_out + f : nullptr;
        D.soft_out = nullptr;
        pbp::pair::Decoder<M> dec(D, smem, tid);
        dec.decode(0);
        busy += wall_clock64() - t0;
    }
    if (tid == 0) {
        P.stats[wg * 3] = t_start;
        P.stats[wg * 3 + 1] = wall_clock64();
        P.stats[wg * 3 + 2] = busy;
        if (atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(P.counter, 0);
            atomicExch(P.counter + 1, 0);
        }
    }
}

// ---- order 0: one persistent kernel for the whole batch ----

struct MixedParams {
    CodeDesc code[kMaxCodes];
    int32_t ncodes;
    const int32_t *code_of_frame;
    const int64_t *llr_off;
    const int64_t *info_off;
    const float *llr;
    int64_t B;
    int32_t max_iter, early_stop, freezing, freeze_input, freeze_walk;
    float alpha;
    uint8_t *info_out;
    int32_t *iters_out;
    int64_t *pe_out;
    int *counter;               // [queue head, waves out]
    float *state;               // one slot per wavefront (long codes)
    int64_t slot_floats;
    int64_t *stats;             // per wavefront: start, end, busy (ticks)
};

// the generic decoder of code length 2^M on one wavefront (state in LDS up
// to N = 512, in the wavefront's slot above 1024)
template <int M>
__device__ __forceinline__ void mixed_generic(const MixedParams &P,
                                              const CodeDesc &cd, int f,
                                              unsigned char *smem, float *slot,
                                              int lane)
{
    DecodeParams D{};
    D.llr = P.llr + P.llr_off[f];
    D.B = 1;
    D.frozen_words = cd.frozen_words;
    D.info_pos = cd.info_pos;
    D.K = cd.K;
    D.max_iter = P.max_iter;
    D.early_stop = P.early_stop;
    D.freezing = P.freezing;
    D.freeze_input = P.freeze_input;
    D.freeze_walk = P.freeze_walk;
    D.alpha = P.alpha;
    D.info_out = P.info_out + P.info_off[f];
    D.iters_out = P.iters_out + f;
    D.pe_out = P.pe_out ? P.pe_out + f : nullptr;
    D.soft_out = nullptr;
    decode_frame<M, (M > pbp::kMaxLdsLog ? 1 : 0), true>(D, 0, smem, slot,
                                                         lane, 64);
}

// ES: early stop (the register decoder's instantiation; the generic decoder
// takes it at run time)
template <bool ES>
__global__ __launch_bounds__(64, 2) void mixed_kernel(MixedParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = (int)__builtin_amdgcn_workitem_id_x();
    const int64_t wave = blockIdx.x;
    float *slot = P.state ? P.state + wave * P.slot_floats : nullptr;
    const int64_t t_start = wall_clock64();
    int64_t busy = 0;
    for (;;) {
        int f = 0;
        if (lane == 0)
            f = atomicAdd(P.counter, 1);
        f = __builtin_amdgcn_readfirstlane(__shfl(f, 0, 64));
        if (f >= P.B)
            break;
        const int64_t t0 = wall_clock64();
        const int c = __builtin_amdgcn_readfirstlane(P.code_of_frame[f]);
        if (c < 0 || c >= P.ncodes) {
            // a frame naming no code of the plan is not decoded
            if (lane == 0) {
                P.iters_out[f] = 0;
                if (P.pe_out)
                    P.pe_out[f] = 0;
            }
            continue;
        }
        const CodeDesc cd = P.code[c];
        switch (cd.m) {
        case pbp::r10::M: {
            pbp::r10::Params R{};
            R.llr = P.llr + P.llr_off[f];
            R.B = 1;
            R.fzw = cd.fzw10;
            R.info_pos = cd.info_pos;
            R.K = cd.K;
            R.max_iter = P.max_iter;
            R.freezing = P.freezing;
            R.freeze_input = P.freeze_input;
            R.freeze_walk = P.freeze_walk;
            R.alpha = P.alpha;
            R.info_out = P.info_out + P.info_off[f];
            R.iters_out = P.iters_out + f;
            R.pe_out = P.pe_out ? P.pe_out + f : nullptr;
            R.soft_out = nullptr;
            pbp::r10::Decoder<true, ES> D(
                R, *reinterpret_cast<pbp::r10::Smem *>(smem), lane);
            D.decode(0);
            break;
        }
        case 1: mixed_generic<1>(P, cd, f, smem, slot, lane); break;
        case 2: mixed_generic<2>(P, cd, f, smem, slot, lane); break;
        case 3: mixed_generic<3>(P, cd, f, smem, slot, lane); break;
        case 4: mixed_generic<4>(P, cd, f, smem, slot, lane); break;
        case 5: mixed_generic<5>(P, cd, f, smem, slot, lane); break;
        case 6: mixed_generic<6>(P, cd, f, smem, slot, lane); break;
        case 7: mixed_generic<7>(P, cd, f, smem, slot, lane); break;
        case 8: mixed_generic<8>(P, cd, f, smem, slot, lane); break;
        case 9: mixed_generic<9>(P, cd, f, smem, slot, lane); break;
        case 11: mixed_generic<11>(P, cd, f, smem, slot, lane); break;
        case 12: mixed_generic<12>(P, cd, f, smem, slot, lane); break;
        case 13: mixed_generic<13>(P, cd, f, smem, slot, lane); break;
        case 14: mixed_generic<14>(P, cd, f, smem, slot, lane); break;
        default: break;
        }
        busy += wall_clock64() - t0;
    }
    if (lane == 0) {
        P.stats[wave * 3] = t_start;
        P.stats[wave * 3 + 1] = wall_clock64();
        P.stats[wave * 3 + 2] = busy;
        // every wavefront has taken its last queue entry before it counts
        // itself out; the last one out rewinds both counters
        if (atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(P.counter, 0);
            atomicExch(P.counter + 1, 0);
        }
    }
}

// LDS of the single kernel for code length 2^m
size_t mixed_lds(int m)
{
    switch (m) {
    case 1: return pbp::generic::lds_bytes<1>(0);
    case 2: return pbp::generic::lds_bytes<2>(0);
    case 3: return pbp::generic::lds_bytes<3>(0);
    case 4: return pbp::generic::lds_bytes<4>(0);
    case 5: return pbp::generic::lds_bytes<5>(0);
    case 6: return pbp::generic::lds_bytes<6>(0);
    case 7: return pbp::generic::lds_bytes<7>(0);
    case 8: return pbp::generic::lds_bytes<8>(0);
    case 9: return pbp::generic::lds_bytes<9>(0);
    case 10: return pbp::r10::smem_bytes();
    case 11: return pbp::generic::lds_bytes<11>(1);
    case 12: return pbp::generic::lds_bytes<12>(1);
    case 13: return pbp::generic::lds_bytes<13>(1);
    case 14: return pbp::generic::lds_bytes<14>(1);
    default: return 0;
    }
}

// ---- the work queue: frames grouped by code (counting sort) ----

struct CodeSet {
    int32_t m[kMaxCodes];
    int32_t ncodes;
};

// frame f's bucket: its code, or ncodes for a frame that names no code of
// the plan (not decoded: it gets zero iterations and PE updates here)
__device__ __forceinline__ int bucket_of(const CodeSet &cs, const int32_t *code_of_frame,
                                         const int64_t *llr_off, const float *llr,
                                         int f)
{
    const int c = code_of_frame[f];
    if (c < 0 || c >= cs.ncodes)
        return cs.ncodes;
    return c;
}

// cnt[0..nb] := 0 (a kernel, not a memset, so that graphs replay it)
__global__ void clear_kernel(int *cnt, int n)
{
    if ((int)threadIdx.x < n)
        cnt[threadIdx.x] = 0;
}

// Bucket counts: each workgroup counts its frames in LDS, then adds one total
// per bucket to the device counts (one frame one device atomic would queue
// every frame of the batch on the same few counters).
__global__ void count_kernel(CodeSet cs, const int32_t *code_of_frame,
                             const int64_t *llr_off, const float *llr,
                             int32_t B, int *cnt, int32_t *iters_out,
                             int64_t *pe_out)
{
    __shared__ int h[kMaxCodes + 1];
    const int nb = cs.ncodes + 1;
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        h[i] = 0;
    __syncthreads();
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < B;
         f += gridDim.x * blockDim.x) {
        const int b = bucket_of(cs, code_of_frame, llr_off, llr, f);
        if (b == cs.ncodes) {
            iters_out[f] = 0;
            if (pe_out)
                pe_out[f] = 0;
        }
        atomicAdd(&h[b], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (h[i])
            atomicAdd(&cnt[i], h[i]);
}

// bounds[b] := start of bucket b (exclusive prefix of the counts), with
// bounds[nb] = B; cursor[b] := bounds[b] for the scatter
__global__ void scan_kernel(const int *cnt, int nb, int *bounds, int *cursor)
{
    if (threadIdx.x == 0) {
        int s = 0;
        for (int b = 0; b < nb; b++) {
            bounds[b] = s;
            cursor[b] = s;
            s += cnt[b];
        }
        bounds[nb] = s;
    }
}

// Frames into their buckets, one block of frames at a time: ranks within the
// block from LDS counters, then one device atomic per bucket reserves the
// block's range.  Frames of a bucket end up in no fixed order (nothing
// depends on it: each frame's results are its own).
__global__ void scatter_kernel(CodeSet cs, const int32_t *code_of_frame,
                               const int64_t *llr_off, const float *llr,
                               int32_t B, int *cursor, int32_t *order)
{
    __shared__ int h[kMaxCodes + 1];
    __shared__ int base[kMaxCodes + 1];
    const int nb = cs.ncodes + 1;
    for (int64_t f0 = (int64_t)blockIdx.x * blockDim.x; f0 < B;
         f0 += (int64_t)gridDim.x * blockDim.x) {
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            h[i] = 0;
        __syncthreads();
        const int64_t f = f0 + threadIdx.x;
        int b = 0, r = 0;
        if (f < B) {
            b = bucket_of(cs, code_of_frame, llr_off, llr, (int)f);
            r = atomicAdd(&h[b], 1);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            base[i] = h[i] ? atomicAdd(&cursor[i], h[i]) : 0;
        __syncthreads();
        if (f < B)
            order[base[b] + r] = (int32_t)f;
        __syncthreads();
    }
}

// ---- tuner cache: (device, codes, mode) -> configuration ----

using TuneKey = std::tuple<int, std::vector<std::pair<int, int>>, int, int>;

std::mutex g_tune_mu;
std::map<TuneKey, pbp_mixed_config> g_tune_cache;

}  // namespace

struct pbp_mixed_plan {
    int device = 0;
    int cus = 0;
    int ncodes = 0;
    int64_t max_frames = 0;
    CodeDesc codes[kMaxCodes];
    CodeSet cs{};
    std::vector<std::pair<int, int>> dims;   // (N, K) per code
    int *d_counters = nullptr;      // [head, waves out] per code
    int *d_cnt = nullptr;           // ncodes + 1 bucket counts
    int *d_bounds = nullptr;        // ncodes + 2 bucket bounds
    int *d_cursor = nullptr;        // ncodes + 1 scatter cursors
    int32_t *d_order = nullptr;     // max_frames
    float *d_state = nullptr;       // slots of long codes
    int64_t slot_floats = 0;
    int64_t *d_stats = nullptr;     // 3 per wavefront per code
    int last_waves[kMaxCodes] = {};   // resident groups of each launch
    int last_threads[kMaxCodes] = {}; // and their size
    int last_launches = 0;            // launches of the last call
    int64_t slots = 0;                // state slots (long codes)
    pbp_mixed_config cfg{0, 16};
};

namespace {

struct Launch {
    const void *kern;
    size_t lds;
    int threads;
};

template <int M, int PATH>
Launch launch_of()
{
    if constexpr (PATH == 2) {
        return Launch{(const void *)class_pair_kernel<M>,
                      pbp::pair::lds_bytes<M>(), pbp::pair::Shape<M>::NT};
    } else if constexpr (PATH == 1) {
        return Launch{(const void *)class_wg_kernel<M>,
                      pbp::generic::lds_bytes<M>(1), kWgThreads};
    } else {
        size_t lds = PATH >= 10 ? pbp::r10::smem_bytes()
                                : pbp::generic::lds_bytes<M>(PATH);
        return Launch{(const void *)class_kernel<M, PATH>, lds, 64};
    }
}

Launch class_launch(int m, int early_stop)
{
    switch (m) {
    case 1: return launch_of<1, 0>();
    case 2: return launch_of<2, 0>();
    case 3: return launch_of<3, 0>();
    case 4: return launch_of<4, 0>();
    case 5: return launch_of<5, 0>();
    case 6: return launch_of<6, 0>();
    case 7: return launch_of<7, 0>();
    case 8: return launch_of<8, 0>();
    case 9: return launch_of<9, 0>();
    case 10: return early_stop ? launch_of<10, 10>() : launch_of<10, 11>();
    case 11: return launch_of<11, 2>();
    case 12: return launch_of<12, 2>();
    case 13: return launch_of<13, 1>();
    case 14: return launch_of<14, 1>();
    default: return Launch{nullptr, 0};
    }
}

void free_plan(pbp_mixed_plan *p)
{
    if (!p)
        return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->d_counters) (void)hipFree(p->d_counters);
    if (p->d_cnt) (void)hipFree(p->d_cnt);
    if (p->d_bounds) (void)hipFree(p->d_bounds);
    if (p->d_cursor) (void)hipFree(p->d_cursor);
    if (p->d_order) (void)hipFree(p->d_order);
    if (p->d_state) (void)hipFree(p->d_state);
    if (p->d_stats) (void)hipFree(p->d_stats);
    (void)hipSetDevice(prev);
    delete p;
}

bool valid_opts(const pbp_decode_opts *o)
{
    return o && o->max_iter >= 1 && (o->early_stop == 0 || o->early_stop == 1) &&
           (o->freezing == 0 || o->freezing == 1) &&
           (o->freeze_input == 0 || o->freeze_input == 1) &&
           o->freeze_walk >= 0 && o->freeze_walk <= 2 && o->alpha > 0.0f &&
           o->alpha < __builtin_inff();
}

bool valid_cfg(const pbp_mixed_config *c)
{
    return c && (c->order == 0 || c->order == 1) && c->waves_per_cu >= 1 &&
           c->waves_per_cu <= kMaxWavesPerCu;
}

// order 0: the single persistent kernel over the batch in the caller's order
hipError_t enqueue_single(pbp_mixed_plan *p, const pbp_mixed_config &cfg,
                          const int32_t *code_of_frame, const int64_t *llr_off,
                          const int64_t *info_off, int32_t B, const float *llr,
                          const pbp_decode_opts *o, uint8_t *info_out,
                          int32_t *iters_out, int64_t *pe_out, hipStream_t st)
{
    size_t lds = 0;
    for (int c = 0; c < p->ncodes; c++)
        lds = std::max(lds, mixed_lds(p->codes[c].m));
    const void *kern = o->early_stop ? (const void *)mixed_kernel<true>
                                     : (const void *)mixed_kernel<false>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    int per_cu = cfg.waves_per_cu;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, lds) ==
            hipSuccess && occ >= 1 && occ < per_cu)
        per_cu = occ;
    int64_t grid = (int64_t)p->cus * per_cu;
    if (p->slots > 0 && grid > p->slots)
        grid = p->slots;
    if (grid > B)
        grid = B;
    MixedParams P{};
    for (int c = 0; c < p->ncodes; c++)
        P.code[c] = p->codes[c];
    P.ncodes = p->ncodes;
    P.code_of_frame = code_of_frame;
    P.llr_off = llr_off;
    P.info_off = info_off;
    P.llr = llr;
    P.B = B;
    P.max_iter = o->max_iter;
    P.early_stop = o->early_stop;
    P.freezing = o->freezing;
    P.freeze_input = o->freeze_input;
    P.freeze_walk = o->freeze_walk;
    P.alpha = o->alpha;
    P.info_out = info_out;
    P.iters_out = iters_out;
    P.pe_out = pe_out;
    P.counter = p->d_counters;
    P.state = p->d_state;
    P.slot_floats = p->slot_floats;
    P.stats = p->d_stats;
    p->last_launches = 1;
    p->last_waves[0] = (int)grid;
    p->last_threads[0] = 64;
    void *args[] = {&P};
    return hipLaunchKernel(kern, dim3((unsigned)grid), dim3(64), args, lds, st);
}

hipError_t enqueue(pbp_mixed_plan *p, const pbp_mixed_config &cfg,
                   const int32_t *code_of_frame, const int64_t *llr_off,
                   const int64_t *info_off, int32_t B, const float *llr,
                   const pbp_decode_opts *o, uint8_t *info_out,
                   int32_t *iters_out, int64_t *pe_out, hipStream_t st)
{
    if (cfg.order == 0)
        return enqueue_single(p, cfg, code_of_frame, llr_off, info_off, B, llr,
                              o, info_out, iters_out, pe_out, st);
    const int nb = p->ncodes + 1;
    const int g = (int)std::min<int64_t>((B + 255) / 256, 4096);
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(64), 0, st, p->d_cnt, nb);
    hipLaunchKernelGGL(count_kernel, dim3(g), dim3(256), 0, st, p->cs,
                       code_of_frame, llr_off, llr, B, p->d_cnt, iters_out,
                       pe_out);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, st, p->d_cnt, nb,
                       p->d_bounds, p->d_cursor);
    hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(256), 0, st, p->cs,
                       code_of_frame, llr_off, llr, B, p->d_cursor, p->d_order);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // codes by decreasing length, stable
    std::vector<int> seq(p->ncodes);
    for (int c = 0; c < p->ncodes; c++)
        seq[c] = c;
    std::stable_sort(seq.begin(), seq.end(), [&](int a, int b) {
        return p->codes[a].m > p->codes[b].m;
    });
    const int64_t max_waves = (int64_t)p->cus * kMaxWavesPerCu;
    p->last_launches = 0;
    for (int c : seq) {
        const Launch L = class_launch(p->codes[c].m, o->early_stop);
        if (!L.kern)
            return hipErrorInvalidValue;
        // resident groups per compute unit: waves_per_cu one-wavefront
        // groups, or half as many 256-thread groups (their wavefronts wait
        // on memory, so twice the wavefronts are resident, and at most one
        // per device slot), never more than the kernel's occupancy allows
        int per_cu = L.threads == 64
                         ? cfg.waves_per_cu
                         : std::min(kMaxLongGroupsPerCu,
                                    std::max(1, cfg.waves_per_cu / 2));
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, L.kern, L.threads,
                                                         L.lds) == hipSuccess &&
            occ >= 1 && occ < per_cu)
            per_cu = occ;
        int64_t grid = (int64_t)p->cus * per_cu;
        if (grid > B)
            grid = B;
        ClassParams P{};
        P.code = p->codes[c];
        P.bounds = p->d_bounds;
        P.bucket = c;
        P.order = p->d_order;
        P.llr_off = llr_off;
        P.info_off = info_off;
        P.llr = llr;
        P.max_iter = o->max_iter;
        P.early_stop = o->early_stop;
        P.freezing = o->freezing;
        P.freeze_input = o->freeze_input;
        P.freeze_walk = o->freeze_walk;
        P.alpha = o->alpha;
        P.info_out = info_out;
        P.iters_out = iters_out;
        P.pe_out = pe_out;
        P.counter = p->d_counters + 2 * c;
        P.state = p->d_state;
        P.slot_floats = p->slot_floats;
        P.stats = p->d_stats + (int64_t)c * max_waves * 3;
        p->last_waves[c] = (int)grid;
        p->last_threads[c] = L.threads;
        p->last_launches = p->ncodes;
        e = hipFuncSetAttribute(L.kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)L.lds);
        if (e != hipSuccess)
            return e;
        void *args[] = {&P};
        e = hipLaunchKernel(L.kern, dim3((unsigned)grid), dim3(L.threads), args,
                            L.lds, st);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" int32_t pbp_mixed_plan_create(const pbp_code *const *codes,
                                         int32_t ncodes, int64_t max_frames,
                                         pbp_mixed_plan **out)
{
    if (!out)
        return PBP_EINVAL;
    *out = nullptr;
    if (!codes || ncodes < 1 || ncodes > kMaxCodes || max_frames < 1 ||
        max_frames > kMaxFrames)
        return PBP_EINVAL;
    for (int c = 0; c < ncodes; c++)
        if (!codes[c] || codes[c]->device != codes[0]->device ||
            codes[c]->m < 1 || codes[c]->m > 14)
            return PBP_EINVAL;
    pbp_mixed_plan *p = new (std::nothrow) pbp_mixed_plan();
    if (!p)
        return PBP_ENOMEM;
    p->device = codes[0]->device;
    p->cus = codes[0]->cus;
    p->ncodes = ncodes;
    p->max_frames = max_frames;
    p->cs.ncodes = ncodes;
    int max_long = 0;
    for (int c = 0; c < ncodes; c++) {
        const pbp_code *k = codes[c];
        p->codes[c] = CodeDesc{k->m, k->K, k->d_frozen_words, k->d_info_pos,
                               k->d_fzw10};
        p->cs.m[c] = k->m;
        p->dims.emplace_back(k->N, k->K);
        if (k->m > pbp::r10::M)
            max_long = std::max(max_long, k->m);
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(p->device) != hipSuccess) {
        delete p;
        return PBP_EDEVICE;
    }
    const int64_t waves = (int64_t)p->cus * kMaxWavesPerCu;
    int32_t st = PBP_OK;
    // codes longer than 1024 keep L in a slot per wavefront of the single
    // kernel (order 0); in the per-code kernels (order 1) N = 2048 and 4096
    // decode on chip and longer codes use the slots of their 256-thread
    // groups
    if (max_long) {
        p->slot_floats = (int64_t)(max_long + 1) << max_long;
        p->slots = waves;
    }
    if (hipMalloc(&p->d_counters, 2 * kMaxCodes * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_cnt, (kMaxCodes + 1) * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_bounds, (kMaxCodes + 2) * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_cursor, (kMaxCodes + 1) * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_order, max_frames * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&p->d_stats, ncodes * waves * 3 * sizeof(int64_t)) != hipSuccess ||
        (max_long && hipMalloc(&p->d_state, p->slots * p->slot_floats *
                                                sizeof(float)) != hipSuccess))
        st = PBP_ENOMEM;
    else if (hipMemset(p->d_counters, 0, 2 * kMaxCodes * sizeof(int)) != hipSuccess ||
             hipDeviceSynchronize() != hipSuccess)
        st = PBP_EDEVICE;
    (void)hipSetDevice(prev);
    if (st != PBP_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    return PBP_OK;
}

extern "C" void pbp_mixed_plan_destroy(pbp_mixed_plan *plan)
{
    free_plan(plan);
}

extern "C" int32_t pbp_mixed_plan_get_config(const pbp_mixed_plan *plan,
                                             pbp_mixed_config *cfg)
{
    if (!plan || !cfg)
        return PBP_EINVAL;
    *cfg = plan->cfg;
    return PBP_OK;
}

extern "C" int32_t pbp_mixed_plan_set_config(pbp_mixed_plan *plan,
                                             const pbp_mixed_config *cfg)
{
    if (!plan || !valid_cfg(cfg))
        return PBP_EINVAL;
    plan->cfg = *cfg;
    return PBP_OK;
}

extern "C" int32_t pbp_decode_mixed(pbp_mixed_plan *plan,
                                    const int32_t *code_of_frame,
                                    const int64_t *llr_off,
                                    const int64_t *info_off, int64_t B,
                                    const float *llr,
                                    const pbp_decode_opts *opts,
                                    uint8_t *info_out, int32_t *iters_out,
                                    int64_t *pe_out, void *stream)
{
    if (!plan || B < 0 || B > plan->max_frames || !valid_opts(opts))
        return PBP_EINVAL;
    if (B == 0)
        return PBP_OK;
    if (!code_of_frame || !llr_off || !info_off || !llr || !info_out ||
        !iters_out)
        return PBP_EINVAL;
    return enqueue(plan, plan->cfg, code_of_frame, llr_off, info_off,
                   (int32_t)B, llr, opts, info_out, iters_out, pe_out,
                   (hipStream_t)stream) == hipSuccess
               ? PBP_OK
               : PBP_EDEVICE;
}

extern "C" int32_t pbp_mixed_plan_fill(pbp_mixed_plan *plan, void *stream,
                                       double *fill)
{
    if (!plan || !fill)
        return PBP_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return PBP_EDEVICE;
    // busy wavefront-time of every launch of the last call over (resident
    // wavefronts x the call's whole span, from the first wavefront's start
    // to the last one's end): kernel tails and the gaps between the
    // per-code launches count as idle
    const int64_t max_waves = (int64_t)plan->cus * kMaxWavesPerCu;
    double busy = 0.0;
    int64_t t0 = INT64_MAX, t1 = INT64_MIN, cap = 0;
    for (int c = 0; c < plan->last_launches; c++) {
        const int w = plan->last_waves[c];
        if (w <= 0)
            continue;
        const int per = plan->last_threads[c] / 64;
        std::vector<int64_t> s((size_t)w * 3);
        if (hipMemcpy(s.data(), plan->d_stats + (int64_t)c * max_waves * 3,
                      s.size() * sizeof(int64_t),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return PBP_EDEVICE;
        for (int i = 0; i < w; i++) {
            t0 = std::min(t0, s[3 * i]);
            t1 = std::max(t1, s[3 * i + 1]);
            busy += (double)s[3 * i + 2] * per;
        }
        cap = std::max(cap, (int64_t)w * per);
    }
    *fill = (cap > 0 && t1 > t0) ? busy / ((double)cap * (double)(t1 - t0)) : 0.0;
    return PBP_OK;
}

extern "C" int32_t pbp_mixed_plan_tune(pbp_mixed_plan *plan,
                                       const int32_t *code_of_frame,
                                       const int64_t *llr_off,
                                       const int64_t *info_off, int64_t B,
                                       const float *llr,
                                       const pbp_decode_opts *opts,
                                       uint8_t *info_out, int32_t *iters_out,
                                       int64_t *pe_out, int32_t reps,
                                       void *stream, pbp_mixed_config *best)
{
    if (!plan || B < 1 || B > plan->max_frames || !valid_opts(opts) ||
        reps < 1 || !code_of_frame || !llr_off || !info_off || !llr ||
        !info_out || !iters_out)
        return PBP_EINVAL;
    TuneKey key{plan->device, plan->dims, opts->early_stop, opts->freezing};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            plan->cfg = it->second;
            if (best)
                *best = plan->cfg;
            return PBP_OK;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return PBP_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PBP_EDEVICE;
    }
    pbp_mixed_config cand[] = {{0, 4}, {0, 8}, {0, 12}, {0, 16},
                               {1, 4}, {1, 8}, {1, 12}, {1, 16}};
    float best_ms = 0.0f;
    pbp_mixed_config best_cfg = plan->cfg;
    int32_t status = PBP_OK;
    for (const pbp_mixed_config &c : cand) {
        // one untimed launch, then reps timed
        if (enqueue(plan, c, code_of_frame, llr_off, info_off, (int32_t)B,
                    llr, opts, info_out, iters_out, pe_out, st) != hipSuccess ||
            hipEventRecord(e0, st) != hipSuccess) {
            status = PBP_EDEVICE;
            break;
        }
        bool ok = true;
        for (int r = 0; r < reps && ok; r++)
            ok = enqueue(plan, c, code_of_frame, llr_off, info_off, (int32_t)B,
                         llr, opts, info_out, iters_out, pe_out, st) ==
                 hipSuccess;
        float ms = 0.0f;
        if (!ok || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            status = PBP_EDEVICE;
            break;
        }
        if (best_ms == 0.0f || ms < best_ms) {
            best_ms = ms;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != PBP_OK)
        return status;
    plan->cfg = best_cfg;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = best_cfg;
    }
    if (best)
        *best = best_cfg;
    return PBP_OK;
}
