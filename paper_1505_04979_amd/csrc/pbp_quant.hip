// BP decoding with saturating b-bit fixed-point messages: the decoder of
// pbp_decode (single sweep, G-matrix early stop, CSFG freezing) in the
// integer arithmetic of a hardware decoder, the setting in which the paper
// counts a PE's cost (Sections I and V).  Every message lies in [-Q, Q],
// Q = 2^(b-1) - 1; the channel is clamp(round(LLR 2^F)); the scaled minimum
// of eq. (1) is (a min(|x|, |y|) + 8) >> 4 with a = round(16 alpha); every
// sum of eq. (1) saturates; +-Q stands for the +-inf of the frozen prior and
// of a frozen CSFG's messages; hard decisions take the exact sum's sign.
//
// Every length runs the decoder pbp_decode uses for it (pbp_wave_decoder.h
// for N <= 64, pbp_generic_decoder.h for N = 128..512, pbp_r10_decoder.h for
// N = 1024, pbp_pair_decoder.h for N = 2048, 4096) with the fixed-point
// arithmetic policy (pbp_arith.h): messages are integers held exactly in
// FP32 registers and LDS words, so the PE is the FP32 one plus a saturation
// per sum and a rounding per scaled minimum.
#include <hip/hip_runtime.h>

#include "pbp_internal.h"
#include "pbp_pair_decoder.h"
#include "pbp_r10.h"
#include "pbp_r10_decoder.h"
#include "pbp_wave_decoder.h"

namespace {

// the call's validated arguments, before they go to one decoder's parameters
struct QParams {
    const float *llr;
    int64_t B;
    const int32_t *info_pos;
    int32_t K;
    int32_t max_iter, early_stop, freezing, freeze_input, freeze_walk;
    int32_t Q;       // 2^(b-1) - 1
    int32_t frac;    // fraction bits of the channel quantizer
    int32_t a16;     // round(16 alpha)
    uint8_t *info_out;
    int32_t *iters_out;
    int64_t *pe_out;
    int8_t *soft_out;   // B x N or null: sat(R + L) at column m+1
};

// N = 1024: persistent wavefronts take frames from the stream's counter
template <bool FRZ, bool ES>
__global__ __launch_bounds__(64, 2) void quant_r10_kernel(pbp::r10::Params P)
{
    __shared__ pbp::r10::Smem S;
    const int lane = (int)__builtin_amdgcn_workitem_id_x();
    pbp::r10::Decoder<FRZ, ES, pbp::r10::ArithFixed> D(P, S, lane);
    for (;;) {
        int frame = 0;
        if (lane == 0)
            frame = atomicAdd(P.counter, 1);
        frame = __shfl(frame, 0, 64);
        if (frame >= P.B)
            break;
        D.decode(frame);
    }
    // the last wavefront out rewinds both counters for the next launch
    if (lane == 0 && atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(P.counter, 0);
        atomicExch(P.counter + 1, 0);
    }
}

hipError_t launch_quant_r10(const pbp_code *c, const QParams &Q, float alpha_q,
                            int *counter, hipStream_t st)
{
    pbp::r10::Params P{};
    P.llr = Q.llr;
    P.B = Q.B;
    P.counter = counter;
    P.fzw = c->d_fzw10;
    P.info_pos = Q.info_pos;
    P.K = Q.K;
    P.max_iter = Q.max_iter;
    P.freezing = Q.freezing;
    P.freeze_input = Q.freeze_input;
    P.freeze_walk = Q.freeze_walk;
    P.alpha = alpha_q;
    P.info_out = Q.info_out;
    P.iters_out = Q.iters_out;
    P.pe_out = Q.pe_out;
    P.soft_out = nullptr;
    P.qmax = (float)Q.Q;
    P.frac = Q.frac;
    P.soft_q = Q.soft_out;
    int64_t grid = (int64_t)c->cus * 8;
    if (grid > Q.B)
        grid = Q.B;
    // as in pbp_decode: early stop without freezing runs the freezing kernel
    // with the walk switched off
    if (Q.early_stop)
        hipLaunchKernelGGL((quant_r10_kernel<true, true>), dim3(grid), dim3(64), 0, st, P);
    else if (Q.freezing)
        hipLaunchKernelGGL((quant_r10_kernel<true, false>), dim3(grid), dim3(64), 0, st, P);
    else
        hipLaunchKernelGGL((quant_r10_kernel<false, false>), dim3(grid), dim3(64), 0, st, P);
    return hipGetLastError();
}

// the generic parameter block of the wavefront and workgroup decoders
pbp::generic::DecodeParams decode_params(const pbp_code *c, const QParams &Q,
                                         float alpha_q)
{
    pbp::generic::DecodeParams P{};
    P.llr = Q.llr;
    P.B = Q.B;
    P.frozen_words = c->d_frozen_words;
    P.info_pos = Q.info_pos;
    P.K = Q.K;
    P.max_iter = Q.max_iter;
    P.early_stop = Q.early_stop;
    P.freezing = Q.freezing;
    P.freeze_input = Q.freeze_input;
    P.freeze_walk = Q.freeze_walk;
    P.alpha = alpha_q;
    P.info_out = Q.info_out;
    P.iters_out = Q.iters_out;
    P.pe_out = Q.pe_out;
    P.soft_out = nullptr;
    P.qmax = (float)Q.Q;
    P.frac = Q.frac;
    P.soft_q = Q.soft_out;
    return P;
}

// N <= 64: one wavefront per frame, every message in registers
template <int M>
hipError_t launch_quant_wave(const pbp_code *c, const QParams &Q, float alpha_q,
                             hipStream_t st)
{
    const pbp::generic::DecodeParams P = decode_params(c, Q, alpha_q);
    constexpr int W = pbp::wave::kWaves;
    int64_t grid = (P.B + W - 1) / W;
    if (grid > (1ll << 30))
        grid = 1ll << 30;
    if (P.freezing)
        hipLaunchKernelGGL((pbp::wave::bp_decode_wave_kernel<M, true, pbp::arith::Fixed>),
                           dim3((unsigned)grid), dim3(64 * W), 0, st, P);
    else
        hipLaunchKernelGGL((pbp::wave::bp_decode_wave_kernel<M, false, pbp::arith::Fixed>),
                           dim3((unsigned)grid), dim3(64 * W), 0, st, P);
    return hipGetLastError();
}

// N = 128..512: one workgroup per frame, every message in LDS
template <int M>
__global__ __launch_bounds__(256, 4) void quant_generic_kernel(pbp::generic::DecodeParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    for (int64_t frame = blockIdx.x; frame < P.B; frame += gridDim.x)
        pbp::generic::decode_frame<M, 0, false, pbp::arith::Fixed>(
            P, frame, smem, nullptr, (int)threadIdx.x, (int)blockDim.x);
}

template <int M>
hipError_t launch_quant_generic(const pbp_code *c, const QParams &Q, float alpha_q,
                                hipStream_t st)
{
    constexpr int N = 1 << M;
    const int nt = N >= 512 ? 256 : N / 2;
    const size_t lds = pbp::generic::lds_bytes<M>(0);
    const pbp::generic::DecodeParams P = decode_params(c, Q, alpha_q);
    int64_t grid = P.B;
    if (grid > (1ll << 30))
        grid = 1ll << 30;
    auto kern = quant_generic_kernel<M>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(nt), lds, st, P);
    return hipGetLastError();
}

// N = 2048, 4096: one workgroup of N/4 threads per frame, messages on chip;
// frames from the stream's counter pair, which the last group out rewinds
template <int M>
__global__ __launch_bounds__(pbp::pair::Shape<M>::NT) void quant_pair_kernel(
    pbp::generic::DecodeParams P, int *counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_frame;
    const int tid = (int)threadIdx.x;
    pbp::pair::Decoder<M, pbp::arith::Fixed> D(P, smem, tid);
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

template <int M>
hipError_t launch_quant_pair(const pbp_code *c, const QParams &Q, float alpha_q,
                             int *counter, hipStream_t st)
{
    using S = pbp::pair::Shape<M>;
    const pbp::generic::DecodeParams P = decode_params(c, Q, alpha_q);
    const size_t lds = pbp::pair::lds_bytes<M>();
    auto kern = quant_pair_kernel<M>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
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

extern "C" int32_t pbp_decode_quant(const pbp_code *code, const float *llr,
                                    int64_t B, const pbp_decode_opts *opts,
                                    int32_t bits, int32_t frac,
                                    uint8_t *info_out, int32_t *iters_out,
                                    int64_t *pe_out, int8_t *soft_out,
                                    void *stream)
{
    if (!code || !opts || B < 0)
        return PBP_EINVAL;
    if (opts->max_iter < 1 || (opts->early_stop != 0 && opts->early_stop != 1) ||
        (opts->freezing != 0 && opts->freezing != 1) ||
        (opts->freeze_input != 0 && opts->freeze_input != 1) ||
        opts->freeze_walk < 0 || opts->freeze_walk > 2 ||
        !(opts->alpha > 0.0f) || !(opts->alpha < 2.0f) || bits < 2 ||
        bits > 8 || frac < 0 || frac > 16)
        return PBP_EINVAL;
    if (code->m > 12)
        return PBP_EUNSUPPORTED;
    if (B == 0)
        return PBP_OK;
    if (!llr || !iters_out || (!info_out && code->K > 0))
        return PBP_EINVAL;
    QParams P{};
    P.llr = llr;
    P.B = B;
    P.info_pos = code->d_info_pos;
    P.K = code->K;
    P.max_iter = opts->max_iter;
    P.early_stop = opts->early_stop;
    P.freezing = opts->freezing;
    P.freeze_input = opts->freeze_input;
    P.freeze_walk = opts->freeze_walk;
    P.Q = (1 << (bits - 1)) - 1;
    P.frac = frac;
    P.a16 = (int32_t)lrintf(opts->alpha * 16.0f);
    P.info_out = info_out;
    P.iters_out = iters_out;
    P.pe_out = pe_out;
    P.soft_out = soft_out;
    hipStream_t st = (hipStream_t)stream;
    const float alpha_q = (float)P.a16 / 16.0f;     // exact
    // on-chip decoders with every message an integer in an FP32 register
    if (code->m <= 6) {
        hipError_t e;
        switch (code->m) {
        case 1: e = launch_quant_wave<1>(code, P, alpha_q, st); break;
        case 2: e = launch_quant_wave<2>(code, P, alpha_q, st); break;
        case 3: e = launch_quant_wave<3>(code, P, alpha_q, st); break;
        case 4: e = launch_quant_wave<4>(code, P, alpha_q, st); break;
        case 5: e = launch_quant_wave<5>(code, P, alpha_q, st); break;
        default: e = launch_quant_wave<6>(code, P, alpha_q, st); break;
        }
        return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
    }
    if (code->m == pbp::r10::M || code->m == 11 || code->m == 12) {
        pbp::Workspace ws;
        const int32_t rc = pbp::stream_workspace(code, st, &ws);
        if (rc != PBP_OK)
            return rc;
        const hipError_t e =
            code->m == pbp::r10::M ? launch_quant_r10(code, P, alpha_q, ws.counter, st)
            : code->m == 11      ? launch_quant_pair<11>(code, P, alpha_q, ws.counter, st)
                                 : launch_quant_pair<12>(code, P, alpha_q, ws.counter, st);
        return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
    }
    hipError_t e;
    switch (code->m) {
    case 7: e = launch_quant_generic<7>(code, P, alpha_q, st); break;
    case 8: e = launch_quant_generic<8>(code, P, alpha_q, st); break;
    case 9: e = launch_quant_generic<9>(code, P, alpha_q, st); break;
    default: return PBP_EUNSUPPORTED;
    }
    return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
}
