// BP decoding of polar codes on gfx950: encoder and batch decoder.
//
// Decoder layout: one workgroup decodes one frame at a time (grid-stride
// over the batch).  The left-to-right messages live in one working column
// of LDS that is updated in place stage by stage (stage j reads R at column
// j and writes R at column j+1 on the same rows), the channel LLRs in a
// second LDS column, and the right-to-left messages L at columns 1..m+1 in
// LDS (N <= 2048) or in a per-workgroup slot of device memory (larger N).
// Hard decisions are packed 64 to a word with wavefront ballots; the
// transform by F^{(x)s} runs on those words (shift/mask/xor inside a word,
// xor across words by cross-lane shuffles).
#include <hip/hip_runtime.h>

#include "pbp_internal.h"
#include "pbp_r10.h"

namespace {

constexpr float kInf = __builtin_inff();

// The min-sum term of eq. (1): alpha * sign(x) * sign(y) * min(|x|, |y|).
// A zero result may carry either sign; no value or decision depends on it.
__device__ __forceinline__ float gmin(float x, float y, float alpha)
{
    // sign(x) sign(y) min(|x|, |y|) is y, its sign flipped when x < 0,
    // clamped to [-|x|, |x|]: one median of three (exact, a selection); the
    // product with alpha then rounds once, symmetrically in sign
    const float t = __uint_as_float(__float_as_uint(y) ^
                                    (__float_as_uint(x) & 0x80000000u));
    return alpha * __builtin_amdgcn_fmed3f(-fabsf(x), t, fabsf(x));
}

// x F^{(x)6} over the 64 bits of a word (bit i = position i): at each level
// hh, position i with bit hh clear takes x[i] ^ x[i + hh].
__device__ __forceinline__ uint64_t ffx_word(uint64_t x)
{
    x ^= (x >> 1) & 0x5555555555555555ull;
    x ^= (x >> 2) & 0x3333333333333333ull;
    x ^= (x >> 4) & 0x0F0F0F0F0F0F0F0Full;
    x ^= (x >> 8) & 0x00FF00FF00FF00FFull;
    x ^= (x >> 16) & 0x0000FFFF0000FFFFull;
    x ^= (x >> 32) & 0x00000000FFFFFFFFull;
    return x;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask)
{
    const int lo = __shfl_xor((int)(uint32_t)v, mask, 64);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Up to 4 words per lane: blocks of at most 16384 bits.
constexpr int kMaxWordsPerLane = 4;

// In-register F^{(x)s} transform of nw words (nw a power of two, word w =
// lane + 64 q held in r[q]); each word already transformed internally.
__device__ __forceinline__ void ffx_cross(uint64_t (&r)[kMaxWordsPerLane],
                                          int nw, int lane)
{
    for (int L = 1; L < nw && L < 64; L <<= 1) {
#pragma unroll
        for (int q = 0; q < kMaxWordsPerLane; q++) {
            const uint64_t o = shfl_xor64(r[q], L);
            if (!(lane & L))
                r[q] ^= o;
        }
    }
    if (nw > 64) {
        // word distance 64: q with bit 0 clear takes q+1; distance 128: q in
        // {0,1} takes q+2
        r[0] ^= r[1];
        r[2] ^= r[3];
        if (nw > 128) {
            r[0] ^= r[2];
            r[1] ^= r[3];
        }
    }
}

struct DecodeParams {
    const float *llr;
    int64_t B;
    const uint64_t *frozen_words;
    const int32_t *info_pos;
    int32_t K;
    int32_t max_iter, early_stop, freezing, freeze_input, freeze_walk;
    float alpha;
    uint8_t *info_out;
    int32_t *iters_out;
    int64_t *pe_out;
    float *soft_out;
    float *state;          // global L state (when not in LDS)
    int64_t state_stride;  // floats per workgroup slot
};

// Control words kept in LDS.
struct Ctl {
    int p[16];        // p[j]: number of frozen CSFGs at stage j (p[0] = 0)
    int stop;
    int walking;
};

template <int M>
struct Layout {
    static constexpr int N = 1 << M;
    static constexpr int NW = N >= 64 ? N / 64 : 1;   // bit words per frame
};

__device__ __forceinline__ bool frozen_bit(const uint64_t *fw, int i)
{
    return (fw[i >> 6] >> (i & 63)) & 1;
}

template <int M, bool GSTATE>
__global__ void bp_decode_kernel(DecodeParams P)
{
    constexpr int N = 1 << M;
    constexpr int NW = Layout<M>::NW;
    extern __shared__ __align__(16) unsigned char smem[];

    // LDS carve-up: [u64 xw NW][u64 dw NW][Ctl][f32 Rw N][f32 ch N][L...]
    uint64_t *xw = reinterpret_cast<uint64_t *>(smem);
    uint64_t *dw = xw + NW;
    Ctl *ctl = reinterpret_cast<Ctl *>(dw + NW);
    float *Rw = reinterpret_cast<float *>(ctl + 1);
    float *ch = Rw + N;
    float *Lbase = GSTATE ? P.state + (int64_t)blockIdx.x * P.state_stride
                          : ch + N;
    // L at column c (1..M+1)
    auto Lc = [&](int c) { return Lbase + (size_t)(c - 1) * N; };

    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int lane = tid & 63;
    const bool wave0 = tid < 64;
    const float alpha = P.alpha;

    for (int64_t frame = blockIdx.x; frame < P.B; frame += gridDim.x) {
        const float *llr = P.llr + frame * N;
        // ---- initial messages ----
        for (int i = tid; i < N; i += NT) {
            ch[i] = llr[i];
            for (int c = 1; c <= M; c++)
                Lc(c)[i] = 0.0f;
            Lc(M + 1)[i] = frozen_bit(P.frozen_words, i) ? kInf : 0.0f;
        }
        for (int w = tid; w < NW; w += NT)
            dw[w] = 0;
        if (tid == 0) {
            for (int j = 0; j <= M; j++)
                ctl->p[j] = 0;
            ctl->stop = 0;
        }
        __syncthreads();

        int64_t pe = 0;
        int t = 1;
        for (; t <= P.max_iter; t++) {
            if (tid == 0)
                ctl->walking = 1;
            for (int j = 1; j <= M; j++) {
                const int s = M - j;
                const int h = 1 << s;
                const int f = ctl->p[j - 1] << (s + 1);  // frozen rows, column j
                const float *Rin = (j == 1) ? ch : Rw;
                float *Lj = Lc(j);
                const float *Lj1 = Lc(j + 1);
                // ---- PE updates, eq. (1) ----
                for (int q = (f >> 1) + tid; q < N / 2; q += NT) {
                    const int a = ((q >> s) << (s + 1)) | (q & (h - 1));
                    const int b = a + h;
                    const float La = Lj1[a], Lb = Lj1[b];
                    const float Ra = Rin[a], Rb = Rin[b];
                    const float sm = Lb + Rb;
                    const float g1 = gmin(La, Ra, alpha);
                    Lj[a] = gmin(La, sm, alpha);
                    Lj[b] = Lb + g1;
                    Rw[a] = gmin(Ra, sm, alpha);
                    Rw[b] = Rb + g1;
                }
                pe += (N - f) >> 1;
                __syncthreads();
                if (!P.freezing)
                    continue;
                // ---- CSFG freezing walk (Section III), wavefront 0 ----
                if (wave0) {
                    int pj = max(ctl->p[j], 2 * ctl->p[j - 1]);
                    int walking = ctl->walking;
                    float *L1 = Lc(j + 1);
                    const int nw = h >= 64 ? h >> 6 : 1;
                    while (pj < (1 << j) && (P.freeze_walk != 0 || walking)) {
                        const int r0 = pj << s;
                        // eq. (2): hard decisions of the CSFG's inputs
                        for (int w = 0; w < nw; w++) {
                            const int i = 64 * w + lane;
                            bool x = false;
                            if (i < h) {
                                const float v = P.freeze_input
                                                    ? Rw[r0 + i] + L1[r0 + i]
                                                    : Rw[r0 + i];
                                x = v < 0.0f;
                            }
                            const uint64_t bal = __ballot(x);
                            if (lane == 0)
                                xw[w] = bal;
                        }
                        wave_sync();
                        // eq. (3): uhat = xhat F^{(x)s}
                        uint64_t r[kMaxWordsPerLane];
#pragma unroll
                        for (int q = 0; q < kMaxWordsPerLane; q++) {
                            const int w = lane + 64 * q;
                            r[q] = w < nw ? ffx_word(xw[w]) : 0;
                        }
                        ffx_cross(r, nw, lane);
                        // eq. (4): no frozen position may decode to 1
                        bool bad = false;
#pragma unroll
                        for (int q = 0; q < kMaxWordsPerLane; q++) {
                            const int w = lane + 64 * q;
                            if (w < nw) {
                                uint64_t fz;
                                if (h >= 64) {
                                    fz = P.frozen_words[(r0 >> 6) + w];
                                } else {
                                    fz = (P.frozen_words[r0 >> 6] >> (r0 & 63)) &
                                         ((1ull << h) - 1);
                                }
                                bad |= (r[q] & fz) != 0;
                            }
                        }
                        if (__any(bad))
                            break;
                        // freeze: L at column j+1 := (-1)^xhat inf, keep uhat
#pragma unroll
                        for (int q = 0; q < kMaxWordsPerLane; q++) {
                            const int w = lane + 64 * q;
                            if (w < nw) {
                                // a CSFG may cover sub-CSFGs of later
                                // stages frozen before it: its decisions
                                // replace theirs
                                if (h >= 64) {
                                    dw[(r0 >> 6) + w] = r[q];
                                } else {
                                    const uint64_t msk = ((1ull << h) - 1)
                                                         << (r0 & 63);
                                    dw[r0 >> 6] = (dw[r0 >> 6] & ~msk) |
                                                  (r[q] << (r0 & 63));
                                }
                            }
                        }
                        for (int i = lane; i < h; i += 64) {
                            const bool x = (xw[i >> 6] >> (i & 63)) & 1;
                            L1[r0 + i] = x ? -kInf : kInf;
                        }
                        wave_sync();
                        pj++;
                        if (P.freeze_walk == 0) {
                            walking = 0;
                            break;
                        }
                        if (P.freeze_walk == 1)
                            break;
                    }
                    if (lane == 0) {
                        ctl->p[j] = pj;
                        ctl->walking = walking;
                    }
                }
                __syncthreads();
            }

            // ---- decisions, termination ----
            const int fm = P.freezing ? ctl->p[M] : 0;
            if (wave0) {
                int stop = P.freezing && fm == N;
                if (!stop && P.early_stop) {
                    // G-matrix criterion: uhat F^{(x)m} == hard(R + L) at
                    // column 1
                    const float *L1 = Lc(1);
                    uint64_t r[kMaxWordsPerLane];
                    for (int w = 0; w < NW; w++) {
                        const int i = 64 * w + lane;
                        bool u = false;
                        if (i < N) {
                            if (i < fm)
                                u = (dw[i >> 6] >> (i & 63)) & 1;
                            else
                                u = !frozen_bit(P.frozen_words, i) && Rw[i] < 0.0f;
                        }
                        const uint64_t bal = __ballot(u);
                        if (lane == 0)
                            xw[w] = bal;
                    }
                    wave_sync();
#pragma unroll
                    for (int q = 0; q < kMaxWordsPerLane; q++) {
                        const int w = lane + 64 * q;
                        r[q] = w < NW ? ffx_word(xw[w]) : 0;
                    }
                    ffx_cross(r, NW, lane);
                    bool diff = false;
                    for (int w = 0; w < NW; w++) {
                        const int i = 64 * w + lane;
                        const bool x = i < N && (ch[i] + L1[i] < 0.0f);
                        const uint64_t bal = __ballot(x);
                        // the lane holding word w compares it
                        if ((w & 63) == lane) {
                            const int q = w >> 6;
                            uint64_t mine = r[0];
                            if (q == 1) mine = r[1];
                            if (q == 2) mine = r[2];
                            if (q == 3) mine = r[3];
                            diff |= mine != bal;
                        }
                    }
                    stop = !__any(diff);
                }
                if (lane == 0)
                    ctl->stop = stop;
            }
            __syncthreads();
            if (ctl->stop)
                break;
        }
        if (t > P.max_iter)
            t = P.max_iter;

        // ---- outputs ----
        const int fm = P.freezing ? ctl->p[M] : 0;
        uint8_t *out = P.info_out + frame * P.K;
        for (int k = tid; k < P.K; k += NT) {
            const int i = P.info_pos[k];
            out[k] = i < fm ? (uint8_t)((dw[i >> 6] >> (i & 63)) & 1)
                            : (uint8_t)(Rw[i] < 0.0f);
        }
        if (P.soft_out) {
            float *so = P.soft_out + frame * N;
            const float *Lm = Lc(M + 1);
            for (int i = tid; i < N; i += NT)
                so[i] = i < fm ? (((dw[i >> 6] >> (i & 63)) & 1) ? -kInf : kInf)
                               : Rw[i] + Lm[i];
        }
        if (tid == 0) {
            P.iters_out[frame] = t;
            if (P.pe_out)
                P.pe_out[frame] = pe;
        }
        __syncthreads();
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
    constexpr int N = 1 << M;
    size_t b = 2 * sizeof(uint64_t) * Layout<M>::NW + sizeof(Ctl) +
               2 * sizeof(float) * N;
    if (!gstate)
        b += sizeof(float) * (size_t)(M + 1) * N;
    return b;
}

template <int M>
hipError_t launch_decode(const pbp_code *c, DecodeParams &P, hipStream_t st)
{
    constexpr int N = 1 << M;
    constexpr bool G = M > pbp::kMaxLdsLog;
    const int nt = N >= 512 ? 256 : (N / 2 >= 64 ? N / 2 : 64);
    const size_t lds = decode_lds_bytes<M>(G);
    int64_t grid = P.B;
    if (G) {
        P.state = c->d_state;
        P.state_stride = c->state_floats_per_slot;
        if (grid > c->state_slots)
            grid = c->state_slots;
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

extern "C" int32_t pbp_decode(const pbp_code *code, const float *llr, int64_t B,
                              const pbp_decode_opts *opts, uint8_t *info_out,
                              int32_t *iters_out, int64_t *pe_out,
                              float *soft_out, void *stream)
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
    // the register-resident N = 1024 kernel moves LLRs and posteriors as
    // 16-byte vectors
    const bool aligned16 = !(reinterpret_cast<uintptr_t>(llr) & 15) &&
                           !(reinterpret_cast<uintptr_t>(soft_out) & 15);
    if (code->m == pbp::r10::M && code->d_fzw10 && aligned16) {
        e = pbp::r10::launch(code, llr, B, opts, info_out, iters_out, pe_out,
                             soft_out, st);
        return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
    }
    switch (code->m) {
    case 1: e = launch_decode<1>(code, P, st); break;
    case 2: e = launch_decode<2>(code, P, st); break;
    case 3: e = launch_decode<3>(code, P, st); break;
    case 4: e = launch_decode<4>(code, P, st); break;
    case 5: e = launch_decode<5>(code, P, st); break;
    case 6: e = launch_decode<6>(code, P, st); break;
    case 7: e = launch_decode<7>(code, P, st); break;
    case 8: e = launch_decode<8>(code, P, st); break;
    case 9: e = launch_decode<9>(code, P, st); break;
    case 10: e = launch_decode<10>(code, P, st); break;
    case 11: e = launch_decode<11>(code, P, st); break;
    case 12: e = launch_decode<12>(code, P, st); break;
    case 13: e = launch_decode<13>(code, P, st); break;
    case 14: e = launch_decode<14>(code, P, st); break;
    default: return PBP_EUNSUPPORTED;
    }
    return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
}
