// BP decoding of polar codes on gfx950: encoder and batch decoder.
//
// Batch decoder: one workgroup decodes one frame at a time (grid-stride over
// the batch) with the generic decoder of pbp_generic_decoder.h, its message
// state in LDS (N <= 512) or in a per-workgroup slot of device memory
// (N >= 8192).  N = 1024 goes to the register-resident decoder and N = 2048
// and 4096 to the workgroup-resident decoder (pbp_pair_decoder.h), both
// taking frames from the stream's counter.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pbp_generic_decoder.h"
#include "pbp_internal.h"
#include "pbp_pair_decoder.h"
#include "pbp_wave_decoder.h"
#include "pbp_r10.h"

namespace {

using namespace pbp::generic;

// At m = 14 the working column (64 KB of LDS) leaves room for two groups per
// compute unit, so each group may take twice the registers.
template <int M, bool GSTATE>
__global__ __launch_bounds__(256, M >= 14 ? 2 : 4) void bp_decode_kernel(DecodeParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *gslot = GSTATE ? P.state + (int64_t)blockIdx.x * P.state_stride
                          : nullptr;
    for (int64_t frame = blockIdx.x; frame < P.B; frame += gridDim.x)
        decode_frame<M, GSTATE ? 1 : 0, false>(P, frame, smem, gslot,
                                               (int)threadIdx.x,
                                               (int)blockDim.x);
}

// N = 2048 and 4096: one workgroup of N / 4 threads per frame, messages on
// chip; frames come from the counter pair (next frame, groups out), which
// the last group out rewinds, or by grid stride when there is none.
template <int M>
__global__ __launch_bounds__(pbp::pair::Shape<M>::NT) void bp_decode_pair_kernel(
    DecodeParams P, int *counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_frame;
    const int tid = (int)threadIdx.x;
    pbp::pair::Decoder<M> D(P, smem, tid);
    int64_t frame = blockIdx.x;
    for (;;) {
        if (counter) {
            if (tid == 0)
                s_frame = atomicAdd(counter, 1);
            __syncthreads();
            frame = s_frame;
            __syncthreads();
        }
        if (frame >= P.B)
            break;
        D.decode(frame);
        if (!counter)
            frame += gridDim.x;
    }
    if (counter && tid == 0 &&
        atomicAdd(counter + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(counter, 0);
        atomicExch(counter + 1, 0);
    }
}

// ---------------------------------------------------------------------------
// Encoder: x = u F^{(x)m}, one workgroup per frame, bytes in LDS.
__global__ void encode_kernel(const uint8_t *info, int64_t B, int N, int K,
                              const int32_t *info_pos, uint8_t *cw)
{
    extern __shared__ uint8_t ub[];
    const int tid = threadIdx.x, NT = blockDim.x;
    for (int64_t f = blockIdx.x; f < B; f += gridDim.x) {
        for (int i = tid; i < N; i += NT)
            ub[i] = 0;
        __syncthreads();
        for (int k = tid; k < K; k += NT)
            ub[info_pos[k]] = info[f * K + k] & 1;
        __syncthreads();
        for (int h = 1; h < N; h <<= 1) {
            for (int q = tid; q < N / 2; q += NT) {
                const int a = ((q / h) * 2 * h) + (q % h);
                ub[a] ^= ub[a + h];
            }
            __syncthreads();
        }
        for (int i = tid; i < N; i += NT)
            cw[f * N + i] = ub[i];
        __syncthreads();
    }
}

template <int M>
size_t decode_lds_bytes(bool gstate)
{
    return lds_bytes<M>(gstate ? 1 : 0);
}

// state, slots: the message state of codes longer than 4096 (one slot of
// (m + 1) N floats per resident workgroup, so at most `slots` groups)
template <int M>
hipError_t launch_decode(const pbp_code *c, DecodeParams &P, float *state,
                         int64_t slots, hipStream_t st)
{
    constexpr int N = 1 << M;
    constexpr bool G = M > pbp::kMaxLdsLog;
    const int nt = N >= 512 ? 256 : (N / 2 >= 64 ? N / 2 : 64);
    const size_t lds = decode_lds_bytes<M>(G);
    int64_t grid = P.B;
    if (G) {
        P.state = state;
        P.state_stride = c->state_floats_per_slot;
        if (grid > slots)
            grid = slots;
    }
    if (grid > (1ll << 30))
        grid = 1ll << 30;
    auto kern = bp_decode_kernel<M, G>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(nt), lds, st, P);
    return hipGetLastError();
}

template <int M>
hipError_t launch_wave(DecodeParams &P, hipStream_t st)
{
    constexpr int W = pbp::wave::kWaves;
    int64_t grid = (P.B + W - 1) / W;
    if (grid > (1ll << 30))
        grid = 1ll << 30;
    if (P.freezing)
        hipLaunchKernelGGL((pbp::wave::bp_decode_wave_kernel<M, true>),
                           dim3((unsigned)grid), dim3(64 * W), 0, st, P);
    else
        hipLaunchKernelGGL((pbp::wave::bp_decode_wave_kernel<M, false>),
                           dim3((unsigned)grid), dim3(64 * W), 0, st, P);
    return hipGetLastError();
}

// counter: the frame counter pair (zero), or null for a grid-stride launch
template <int M>
hipError_t launch_pair(const pbp_code *c, DecodeParams &P, int *counter,
                       hipStream_t st)
{
    using S = pbp::pair::Shape<M>;
    const size_t lds = pbp::pair::lds_bytes<M>();
    auto kern = bp_decode_pair_kernel<M>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    // resident groups per compute unit (once per process: LDS bound)
    static int occ = 0;
    if (occ < 1) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void *)kern,
                                                         S::NT, lds) != hipSuccess)
            return hipGetLastError();
        occ = o < 1 ? 1 : o;
    }
    int64_t grid = (int64_t)c->cus * occ;
    if (grid > P.B)
        grid = P.B;
    int *ctr = P.B <= (int64_t(1) << 30) ? counter : nullptr;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(S::NT), lds, st, P, ctr);
    return hipGetLastError();
}

}  // namespace

extern "C" int32_t pbp_encode(const pbp_code *code, const uint8_t *info,
                              int64_t B, uint8_t *codeword, void *stream)
{
    if (!code || B < 0 || (B > 0 && (!codeword || (!info && code->K > 0))))
        return PBP_EINVAL;
    if (B == 0)
        return PBP_OK;
    const int N = code->N;
    const int nt = N >= 256 ? 256 : 64;
    int64_t grid = B < (1ll << 30) ? B : (1ll << 30);
    hipLaunchKernelGGL(encode_kernel, dim3((unsigned)grid), dim3(nt), N,
                       (hipStream_t)stream, info, B, N, code->K,
                       code->d_info_pos, codeword);
    return hipGetLastError() == hipSuccess ? PBP_OK : PBP_EDEVICE;
}

namespace {

// Device scratch of one decode call: the [frame, exit] counter pair of the
// N = 1024, 2048 and 4096 kernels and the message-state slots of codes
// longer than 4096.
struct Scratch {
    int *counter;
    float *state;
    int64_t slots;
};

// sc == nullptr: check the arguments only, enqueue nothing

int32_t decode_impl(const pbp_code *code, const float *llr, int64_t B,
                    const pbp_decode_opts *opts, uint8_t *info_out,
                    int32_t *iters_out, int64_t *pe_out, float *soft_out,
                    void *stream, const Scratch *sc)
{
    if (!code || !opts || B < 0)
        return PBP_EINVAL;
    if (opts->max_iter < 1 || (opts->early_stop != 0 && opts->early_stop != 1) ||
        (opts->freezing != 0 && opts->freezing != 1) ||
        (opts->freeze_input != 0 && opts->freeze_input != 1) ||
        opts->freeze_walk < 0 || opts->freeze_walk > 2 ||
        !(opts->alpha > 0.0f) || !(opts->alpha < kInf))
        return PBP_EINVAL;
    if (B == 0)
        return PBP_OK;
    if (!llr || !iters_out || (!info_out && code->K > 0))
        return PBP_EINVAL;
    if (!sc)            // arguments checked, nothing to enqueue
        return PBP_OK;
    DecodeParams P{};
    P.llr = llr;
    P.B = B;
    P.frozen_words = code->d_frozen_words;
    P.info_pos = code->d_info_pos;
    P.K = code->K;
    P.max_iter = opts->max_iter;
    P.early_stop = opts->early_stop;
    P.freezing = opts->freezing;
    P.freeze_input = opts->freeze_input;
    P.freeze_walk = opts->freeze_walk;
    P.alpha = opts->alpha;
    P.info_out = info_out;
    P.iters_out = iters_out;
    P.pe_out = pe_out;
    P.soft_out = soft_out;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    // the register-resident N = 1024 kernel numbers frames with a 32-bit
    // device counter
    if (code->m == pbp::r10::M && code->d_fzw10 && B <= (int64_t(1) << 30)) {
        e = pbp::r10::launch(code, llr, B, opts, info_out, iters_out, pe_out,
                             soft_out, sc->counter, st);
        return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
    }
    // codes up to 64: one wavefront per frame in registers
    if (code->m <= 6) {
        switch (code->m) {
        case 1: e = launch_wave<1>(P, st); break;
        case 2: e = launch_wave<2>(P, st); break;
        case 3: e = launch_wave<3>(P, st); break;
        case 4: e = launch_wave<4>(P, st); break;
        case 5: e = launch_wave<5>(P, st); break;
        default: e = launch_wave<6>(P, st); break;
        }
        return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
    }
    switch (code->m) {
    case 1: e = launch_decode<1>(code, P, sc->state, sc->slots, st); break;
    case 2: e = launch_decode<2>(code, P, sc->state, sc->slots, st); break;
    case 3: e = launch_decode<3>(code, P, sc->state, sc->slots, st); break;
    case 4: e = launch_decode<4>(code, P, sc->state, sc->slots, st); break;
    case 5: e = launch_decode<5>(code, P, sc->state, sc->slots, st); break;
    case 6: e = launch_decode<6>(code, P, sc->state, sc->slots, st); break;
    case 7: e = launch_decode<7>(code, P, sc->state, sc->slots, st); break;
    case 8: e = launch_decode<8>(code, P, sc->state, sc->slots, st); break;
    case 9: e = launch_decode<9>(code, P, sc->state, sc->slots, st); break;
    case 10: e = launch_decode<10>(code, P, sc->state, sc->slots, st); break;
    case 11: e = launch_pair<11>(code, P, sc->counter, st); break;
    case 12: e = launch_pair<12>(code, P, sc->counter, st); break;
    case 13: e = launch_decode<13>(code, P, sc->state, sc->slots, st); break;
    case 14: e = launch_decode<14>(code, P, sc->state, sc->slots, st); break;
    default: return PBP_EUNSUPPORTED;
    }
    return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
}

}  // namespace

extern "C" int32_t pbp_decode(const pbp_code *code, const float *llr, int64_t B,
                              const pbp_decode_opts *opts, uint8_t *info_out,
                              int32_t *iters_out, int64_t *pe_out,
                              float *soft_out, void *stream)
{
    if (!code)
        return PBP_EINVAL;
    // argument errors first: a rejected call allocates nothing either
    const int32_t chk = decode_impl(code, llr, B, opts, info_out, iters_out,
                                    pe_out, soft_out, stream, nullptr);
    if (chk != PBP_OK || B == 0)
        return chk;
    pbp::Workspace ws;
    const int32_t st = pbp::stream_workspace(code, (hipStream_t)stream, &ws);
    if (st != PBP_OK)
        return st;
    const Scratch sc{ws.counter, ws.state, code->state_slots};
    return decode_impl(code, llr, B, opts, info_out, iters_out, pe_out,
                       soft_out, stream, &sc);
}

// ---- Decoding without allocation (pbp_decode_noalloc) --------------------
//
// The scratch of these calls is one static device array per GPU, so a call
// needs no allocation: its first 256 bytes hold the counter pair, the rest
// the message-state slots of codes longer than 4096.
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchHead = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The device address of this GPU's scratch, looked up once per device with
// that device current.  (In host code the array's name is only a stand-in:
// every kernel argument, fill and copy uses this address.)
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

int32_t scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return PBP_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return PBP_EDEVICE;
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return PBP_OK;
}

// the counter pair starts each call at zero (a kernel, not a memset, so that
// a caller may capture the call in a graph)
__global__ void clear_counters_kernel(int *counter)
{
    if (threadIdx.x < 2)
        counter[threadIdx.x] = 0;
}

// message-state slots that fit the scratch (codes longer than 4096)
int64_t scratch_slots(const pbp_code *code)
{
    if (code->m <= pbp::kMaxOnChipLog)
        return INT64_MAX;
    const int64_t slot = (int64_t)sizeof(float) * code->state_floats_per_slot;
    return (int64_t)((kScratchBytes - kScratchHead) / slot);
}

}  // namespace

extern "C" int32_t pbp_decode_noalloc(const pbp_code *code, const float *llr,
                                      int64_t B, const pbp_decode_opts *opts,
                                      uint8_t *info_out, int32_t *iters_out,
                                      int64_t *pe_out, float *soft_out,
                                      void *stream)
{
    if (!code || !opts || B < 0)
        return PBP_EINVAL;
    // the N = 1024 kernel numbers frames with a 32-bit counter
    if (B > (int64_t(1) << 30))
        return PBP_EINVAL;
    void *base = nullptr;
    const int32_t st = scratch_address(&base);
    if (st != PBP_OK)
        return st;
    Scratch sc{};
    sc.counter = reinterpret_cast<int *>(base);
    sc.state = reinterpret_cast<float *>(static_cast<unsigned char *>(base) +
                                         kScratchHead);
    sc.slots = scratch_slots(code);
    if (code->m > pbp::kMaxOnChipLog && sc.slots < 1)
        return PBP_EUNSUPPORTED;
    // the persistent kernels (N = 1024, 2048, 4096) take frames from the
    // counter pair
    if (B > 0 && code->m >= pbp::r10::M && code->m <= pbp::kMaxOnChipLog) {
        hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0,
                           (hipStream_t)stream, sc.counter);
        if (hipGetLastError() != hipSuccess)
            return PBP_EDEVICE;
    }
    return decode_impl(code, llr, B, opts, info_out, iters_out, pe_out,
                       soft_out, stream, &sc);
}
