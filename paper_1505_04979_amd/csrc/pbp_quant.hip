// BP decoding with saturating b-bit fixed-point messages: the decoder of
// pbp_decode (single sweep, G-matrix early stop, CSFG freezing) in the
// integer arithmetic of a hardware decoder, the setting in which the paper
// counts a PE's cost (Sections I and V).  Every message lies in [-Q, Q],
// Q = 2^(b-1) - 1; the channel is clamp(round(LLR 2^F)); the scaled minimum
// of eq. (1) is (a min(|x|, |y|) + 8) >> 4 with a = round(16 alpha); every
// sum of eq. (1) saturates; +-Q stands for the +-inf of the frozen prior and
// of a frozen CSFG's messages; hard decisions take the exact sum's sign.
//
// N <= 64, 1024, 2048 and 4096 run the on-chip decoders of pbp_decode
// (pbp_wave_decoder.h, pbp_r10_decoder.h, pbp_pair_decoder.h) with the
// fixed-point arithmetic policy (pbp_arith.h): messages are integers held
// exactly in FP32 registers, so the PE is the FP32 one plus a saturation per
// sum and a rounding per scaled minimum.
//
// N = 128..512: one wavefront per frame, persistent over a grid stride,
// with the whole state in LDS, one signed byte per message (L at columns
// 1..m+1, the working R column updated in place stage by stage, the
// quantized channel, the kept decisions and two bit-byte scratch columns):
// (m + 6) N bytes and the frozen prefixes.  PEs go four at a time where a
// stage's offset is at least 4 (rows a..a+3 are one 32-bit LDS word in every
// column), one at a time at the last two stages.  The CSFG check and the
// stop test transform their decision bytes by F^{(x)s} in LDS, one butterfly
// level per step.
#include <hip/hip_runtime.h>

#include "pbp_internal.h"
#include "pbp_pair_decoder.h"
#include "pbp_r10.h"
#include "pbp_r10_decoder.h"
#include "pbp_wave_decoder.h"

namespace {

struct QParams {
    const float *llr;
    int64_t B;
    const uint64_t *frozen_words;
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

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int sat(int v, int Q)
{
    return min(max(v, -Q), Q);
}

// sign(x) sign(y) ((a16 min(|x|, |y|) + 8) >> 4); a zero operand gives 0
__device__ __forceinline__ int gq(int x, int y, int a16)
{
    const int mn = min(abs(x), abs(y));
    const int r = (a16 * mn + 8) >> 4;
    const int s = (x ^ y) >> 31;            // -1 when the signs differ
    return (r ^ s) - s;
}

__device__ __forceinline__ bool frozen_bit(const uint64_t *fw, int i)
{
    return (fw[i >> 6] >> (i & 63)) & 1;
}

// one PE of eq. (1) in fixed point
__device__ __forceinline__ void pe_q(int La, int Lb, int Ra, int Rb, int Q,
                                     int a16, int &oLa, int &oLb, int &oRa,
                                     int &oRb)
{
    const int s = sat(Lb + Rb, Q);
    const int g1 = gq(La, Ra, a16);
    oLa = gq(La, s, a16);
    oLb = sat(Lb + g1, Q);
    oRa = gq(Ra, s, a16);
    oRb = sat(Rb + g1, Q);
}

__device__ __forceinline__ int sbyte(uint32_t w, int k)
{
    return (int)(int8_t)(uint8_t)(w >> (8 * k));
}

__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d)
{
    return (uint32_t)(uint8_t)a | ((uint32_t)(uint8_t)b << 8) |
           ((uint32_t)(uint8_t)c << 16) | ((uint32_t)(uint8_t)d << 24);
}

// x := x F^{(x)s} over n = 2^s bytes: level hh, position i with bit hh clear
// takes x[i] ^ x[i + hh]
__device__ __forceinline__ void transform(uint8_t *x, int n, int lane)
{
    for (int hh = 1; hh < n; hh <<= 1) {
        for (int q = lane; q < n / 2; q += 64) {
            const int i = ((q / hh) * 2 * hh) + (q % hh);
            x[i] ^= x[i + hh];
        }
        wave_sync();
    }
}

template <int M>
__global__ __launch_bounds__(64) void quant_decode_kernel(QParams P)
{
    constexpr int N = 1 << M;
    extern __shared__ __align__(16) unsigned char smem[];
    int8_t *Lall = reinterpret_cast<int8_t *>(smem);     // columns 1..M+1
    int8_t *Rw = Lall + (M + 1) * N;
    int8_t *ch = Rw + N;
    uint8_t *dec = reinterpret_cast<uint8_t *>(ch + N);
    uint8_t *uh = dec + N;
    uint8_t *tb = uh + N;
    int *p = reinterpret_cast<int *>(tb + N);   // frozen prefix per stage
    auto Lc = [&](int c) { return Lall + (c - 1) * N; };
    const int lane = (int)threadIdx.x;
    const int Q = P.Q, a16 = P.a16;

    for (int64_t frame = blockIdx.x; frame < P.B; frame += gridDim.x) {
        const float *llr = P.llr + frame * N;
        for (int i = lane; i < N; i += 64) {
            // LLR 2^F is exact; roundf rounds halves away from zero
            const float v = roundf(ldexpf(llr[i], P.frac));
            ch[i] = (int8_t)(int)fminf(fmaxf(v, (float)-Q), (float)Q);
            for (int c = 1; c <= M; c++)
                Lc(c)[i] = 0;
            Lc(M + 1)[i] = frozen_bit(P.frozen_words, i) ? (int8_t)Q : 0;
            dec[i] = 0;
        }
        if (lane <= M)
            p[lane] = 0;
        wave_sync();

        int64_t pe = 0;
        int t = 1;
        for (; t <= P.max_iter; t++) {
            bool walking = true;
            for (int j = 1; j <= M; j++) {
                const int s = M - j;
                const int h = 1 << s;
                const int f = __builtin_amdgcn_readfirstlane(p[j - 1]) << (s + 1);
                int8_t *Lj = Lc(j);
                const int8_t *Lj1 = Lc(j + 1);
                const int8_t *Rin = j == 1 ? ch : Rw;
                if (h >= 4) {
                    // four PEs a..a+3 (consecutive rows, one word per column)
                    for (int q = (f >> 1) + 4 * lane; q < N / 2; q += 256) {
                        const int a = ((q >> s) << (s + 1)) | (q & (h - 1));
                        const int b = a + h;
                        const uint32_t wLa = *reinterpret_cast<const uint32_t *>(Lj1 + a);
                        const uint32_t wLb = *reinterpret_cast<const uint32_t *>(Lj1 + b);
                        const uint32_t wRa = *reinterpret_cast<const uint32_t *>(Rin + a);
                        const uint32_t wRb = *reinterpret_cast<const uint32_t *>(Rin + b);
                        int la[4], lb[4], ra[4], rb[4];
#pragma unroll
                        for (int k = 0; k < 4; k++)
                            pe_q(sbyte(wLa, k), sbyte(wLb, k), sbyte(wRa, k),
                                 sbyte(wRb, k), Q, a16, la[k], lb[k], ra[k], rb[k]);
                        *reinterpret_cast<uint32_t *>(Lj + a) = pack4(la[0], la[1], la[2], la[3]);
                        *reinterpret_cast<uint32_t *>(Lj + b) = pack4(lb[0], lb[1], lb[2], lb[3]);
                        *reinterpret_cast<uint32_t *>(Rw + a) = pack4(ra[0], ra[1], ra[2], ra[3]);
                        *reinterpret_cast<uint32_t *>(Rw + b) = pack4(rb[0], rb[1], rb[2], rb[3]);
                    }
                } else {
                    for (int q = (f >> 1) + lane; q < N / 2; q += 64) {
                        const int a = ((q >> s) << (s + 1)) | (q & (h - 1));
                        const int b = a + h;
                        int la, lb, ra, rb;
                        pe_q(Lj1[a], Lj1[b], Rin[a], Rin[b], Q, a16, la, lb, ra, rb);
                        Lj[a] = (int8_t)la;
                        Lj[b] = (int8_t)lb;
                        Rw[a] = (int8_t)ra;
                        Rw[b] = (int8_t)rb;
                    }
                }
                pe += (N - f) / 2;
                wave_sync();
                if (!P.freezing)
                    continue;
                // ---- CSFG freezing walk at stage j (eqs. (2)-(4)) ----
                int pj = __builtin_amdgcn_readfirstlane(max(p[j], 2 * p[j - 1]));
                while (pj < (1 << j)) {
                    if (P.freeze_walk == 0 && !walking)
                        break;
                    const int r0 = pj * h;
                    int8_t *Lb1 = Lc(j + 1);
                    for (int r = lane; r < h; r += 64) {
                        const int v = P.freeze_input ? (int)Rw[r0 + r] + (int)Lb1[r0 + r]
                                                     : (int)Rw[r0 + r];
                        tb[r] = v < 0;
                    }
                    wave_sync();
                    // keep xhat (for the fixed messages) before the transform
                    for (int r = lane; r < h; r += 64)
                        uh[r] = tb[r];
                    wave_sync();
                    transform(tb, h, lane);
                    bool bad = false;
                    for (int r = lane; r < h; r += 64)
                        bad |= tb[r] && frozen_bit(P.frozen_words, r0 + r);
                    if (__ballot(bad))
                        break;
                    for (int r = lane; r < h; r += 64) {
                        Lb1[r0 + r] = uh[r] ? (int8_t)(-Q) : (int8_t)Q;
                        dec[r0 + r] = tb[r];
                    }
                    wave_sync();
                    pj++;
                    if (P.freeze_walk == 0) {
                        walking = false;
                        break;
                    }
                    if (P.freeze_walk == 1)
                        break;
                }
                if (lane == 0)
                    p[j] = pj;
                wave_sync();
            }
            // decisions at column m+1
            const int fm = P.freezing ? __builtin_amdgcn_readfirstlane(p[M]) : 0;
            for (int i = lane; i < N; i += 64) {
                const uint8_t u = i < fm ? dec[i]
                                         : (frozen_bit(P.frozen_words, i) ? 0 : (Rw[i] < 0));
                uh[i] = u;
                tb[i] = u;
            }
            wave_sync();
            if (P.freezing && fm == N)
                break;
            if (P.early_stop) {
                // G-matrix test: uhat G against [R + L < 0] at column 1
                transform(tb, N, lane);
                bool diff = false;
                for (int i = lane; i < N; i += 64)
                    diff |= tb[i] != (uint8_t)((int)ch[i] + (int)Lc(1)[i] < 0);
                if (!__ballot(diff))
                    break;
                wave_sync();
            }
        }
        if (t > P.max_iter)
            t = P.max_iter;
        uint8_t *out = P.info_out + frame * P.K;
        for (int k = lane; k < P.K; k += 64)
            out[k] = uh[P.info_pos[k]];
        if (P.soft_out) {
            const int fm = P.freezing ? p[M] : 0;
            for (int i = lane; i < N; i += 64)
                P.soft_out[frame * N + i] =
                    i < fm ? (dec[i] ? (int8_t)(-Q) : (int8_t)Q)
                           : (int8_t)sat((int)Rw[i] + (int)Lc(M + 1)[i], Q);
        }
        if (lane == 0) {
            P.iters_out[frame] = t;
            if (P.pe_out)
                P.pe_out[frame] = pe;
        }
        wave_sync();
    }
}

template <int M>
hipError_t launch_quant(const pbp_code *c, QParams &P, hipStream_t st)
{
    constexpr int N = 1 << M;
    const size_t lds = (size_t)(M + 6) * N + 64;
    int64_t grid = P.B;
    const int64_t cap = (int64_t)c->cus * 32;
    if (grid > cap)
        grid = cap;
    auto kern = quant_decode_kernel<M>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), lds, st, P);
    return hipGetLastError();
}

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
    int64_t grid = P.B;
    if (grid > (1ll << 30))
        grid = 1ll << 30;
    if (P.freezing)
        hipLaunchKernelGGL((pbp::wave::bp_decode_wave_kernel<M, true, pbp::arith::Fixed>),
                           dim3((unsigned)grid), dim3(64), 0, st, P);
    else
        hipLaunchKernelGGL((pbp::wave::bp_decode_wave_kernel<M, false, pbp::arith::Fixed>),
                           dim3((unsigned)grid), dim3(64), 0, st, P);
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
    P.frozen_words = code->d_frozen_words;
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
    // N = 128..512 keep messages as bytes: a scaled minimum must fit (8-bit
    // messages with alpha above 1 can reach 246)
    if ((P.a16 * P.Q + 8) >> 4 > 127)
        return PBP_EUNSUPPORTED;
    hipError_t e;
    switch (code->m) {
    case 7: e = launch_quant<7>(code, P, st); break;
    case 8: e = launch_quant<8>(code, P, st); break;
    case 9: e = launch_quant<9>(code, P, st); break;
    default: return PBP_EUNSUPPORTED;
    }
    return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
}
