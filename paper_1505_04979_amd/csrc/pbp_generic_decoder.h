// Generic BP decoder of one frame (any N = 2^m, m <= 14), shared by the
// batch kernel (pbp_decode.hip) and the mixed-code persistent kernel
// (pbp_mixed.hip).
//
// The left-to-right messages live in one working column updated in place
// stage by stage (stage j reads R at column j and writes R at column j+1 on
// the same rows), the channel LLRs in a second column, and the
// right-to-left messages L at columns 1..m+1.  Placement (STATE): 0 = all in
// LDS; 1 = L in a device-memory slot, the working R column in LDS, channel
// LLRs read in place; 2 = L and the working R column in the slot, channel
// LLRs read in place.  Hard
// decisions are packed 64 to a word with wavefront ballots; the transform by
// F^{(x)s} runs on those words (shift/mask/xor inside a word, xor across
// words by cross-lane shuffles).  The CSFG walk and the stop test run on
// wavefront 0.  WAVE: the frame is decoded by one wavefront alone (ordering
// by wavefront barriers), else by the whole workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbp_arith.h"
#include "pbp_lanes.h"
#include "pbp_internal.h"

namespace pbp {
namespace generic {
namespace {

constexpr float kInf = __builtin_inff();

// The min-sum term of eq. (1), alpha * sign(x) * sign(y) * min(|x|, |y|),
// is gmin(ax, x, y) with ax = salpha(x): y clamped to [-|x|, |x|] (one
// median of three: exact, a selection) times alpha carrying the sign of x
// (one product, rounded once and symmetrically in sign).  The two terms of a
// PE with the same first operand share ax.  A zero result may carry either
// sign; no value or decision depends on it.
__device__ __forceinline__ float salpha(float x, float alpha)
{
    return __builtin_copysignf(alpha, x);
}

__device__ __forceinline__ float gmin(float ax, float x, float y)
{
    return ax * __builtin_amdgcn_fmed3f(-fabsf(x), y, fabsf(x));
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

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Up to 4 words per lane: blocks of at most 16384 bits.
constexpr int kMaxWordsPerLane = 4;

// Words whose input loads are issued together before their ballots (with L
// in device memory, one dependent load per word would serialise the walk
// and the stop test on memory latency).
constexpr int kBatch = 8;

// Groups of four PEs per thread whose 16-byte loads are issued together in
// the vector sweep.
constexpr int kBatch4 = 4;

__device__ __forceinline__ float4 ld4(const float *p)
{
    return *reinterpret_cast<const float4 *>(p);
}

__device__ __forceinline__ void st4(float *p, float4 v)
{
    *reinterpret_cast<float4 *>(p) = v;
}

// one PE of eq. (1): inputs L_a, L_b (column j+1), R_a, R_b (column j)
__device__ __forceinline__ void pe_eq1(float La, float Lb, float Ra, float Rb,
                                       float alpha, float &oLa, float &oLb,
                                       float &oRa, float &oRb)
{
    const float sm = Lb + Rb;
    const float aLa = salpha(La, alpha);
    const float g1 = gmin(aLa, La, Ra);
    oLa = gmin(aLa, La, sm);
    oLb = Lb + g1;
    oRa = gmin(salpha(Ra, alpha), Ra, sm);
    oRb = Rb + g1;
}

// In-register F^{(x)s} transform of nw words (nw a power of two, word w =
// lane + 64 q held in r[q]); each word already transformed internally.
__device__ __forceinline__ void ffx_cross(uint64_t (&r)[kMaxWordsPerLane],
                                          int nw, int lane)
{
#pragma unroll
    for (int L = 1; L < 64; L <<= 1) {
        if (L >= nw)
            break;
#pragma unroll
        for (int q = 0; q < kMaxWordsPerLane; q++) {
            const uint64_t o = lanes::down_u64(r[q], L);
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
    // fixed-point messages only (decoders with the Fixed arithmetic policy)
    float qmax;            // Q = 2^(b-1) - 1
    int32_t frac;          // fraction bits of the channel quantizer
    int8_t *soft_q;        // B x N or null: sat(R + L) at column m+1
};

// Control words kept in LDS (16-byte aligned size, so the float columns after
// it take 16-byte accesses).
struct alignas(16) Ctl {
    int p[16];        // p[j]: number of frozen CSFGs at stage j (p[0] = 0)
    int walking;      // the walk may still check in this sweep
    int bad;          // the last check failed
    int ndiff;        // some word differs in the stop test
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

template <bool WAVE>
__device__ __forceinline__ void sync()
{
    if constexpr (WAVE)
        wave_sync();
    else
        __syncthreads();
}

// Barrier between stages: only the working R column (and the walk's words
// and control) must be ordered there.  When R is in LDS, the L messages a
// stage stores to device memory are next read in the following iteration,
// after the full barrier that ends each sweep, so they stay in flight.
template <bool WAVE, int STATE>
__device__ __forceinline__ void sync_stage()
{
    if constexpr (WAVE || STATE == 2) {
        sync<WAVE>();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}

// LDS bytes of one decoder instance: [u64 xw NW][u64 dw NW][Ctl], then
// [f32 Rw N] unless STATE == 2, then [f32 ch N] and L (m+1 columns) if
// STATE == 0
template <int M>
__host__ __device__ constexpr size_t lds_bytes(int state)
{
    return 2 * sizeof(uint64_t) * Layout<M>::NW + sizeof(Ctl) +
           (state < 2 ? sizeof(float) * (1u << M) : 0) +
           (state == 0 ? sizeof(float) * (size_t)(M + 2) * (1u << M) : 0);
}

// floats of a device-memory slot: L (m+1 columns), plus the working R
// column when STATE == 2
template <int M>
__host__ __device__ constexpr int64_t slot_floats(int state)
{
    return (int64_t)(M + 1 + (state == 2 ? 1 : 0)) << M;
}

// Decode frame `frame` of P (LLRs at P.llr + frame N, outputs at index
// frame).  smem: this instance's LDS (lds_bytes); gslot: its device slot
// (slot_floats, STATE > 0).  tid, NT: thread index and count of the group
// decoding the frame (NT = 64 when WAVE).
// Ar: the message arithmetic (pbp_arith.h); arith::Fixed decodes b-bit
// integers (state in LDS only), +-Q standing for the +-inf of frozen rows
template <int M, int STATE, bool WAVE, class Ar = arith::F32>
__device__ __forceinline__ void decode_frame(const DecodeParams &P,
                                             int64_t frame,
                                             unsigned char *smem,
                                             float *gslot, int tid, int NT)
{
    constexpr int N = 1 << M;
    constexpr int NW = Layout<M>::NW;
    uint64_t *xw = reinterpret_cast<uint64_t *>(smem);
    uint64_t *dw = xw + NW;
    Ctl *ctl = reinterpret_cast<Ctl *>(dw + NW);
    float *Rw = STATE == 2 ? gslot + (int64_t)(M + 1) * N
                           : reinterpret_cast<float *>(ctl + 1);
    float *chl = reinterpret_cast<float *>(ctl + 1) + N;
    float *Lbase = STATE == 0 ? chl + N : gslot;
    // L at column c (1..M+1)
    auto Lc = [&](int c) { return Lbase + (size_t)(c - 1) * N; };
    const int lane = tid & 63;
    const bool wave0 = tid < 64;
    const int wv = tid >> 6;       // wavefront of the group
    const int nwv = NT >> 6;       // wavefronts in the group
    const float alpha = P.alpha;
    const float big = Ar::big(P.qmax);     // inf, or Q in fixed point
    static_assert(!Ar::kFixed || STATE == 0, "fixed point keeps its state in LDS");
    // an opaque thread count keeps the strided loops rolled (a known count
    // of 64 would unroll them N/64 times over and exhaust the registers)
    NT = __builtin_amdgcn_readfirstlane(NT);
    asm volatile("" : "+s"(NT));

    const float *llr = P.llr + frame * N;
    const float *ch = STATE != 0 ? llr : chl;
    const bool ch_aligned = (reinterpret_cast<uintptr_t>(ch) & 15) == 0;
    // ---- initial messages ----
    for (int i = tid; i < N; i += NT) {
        if (STATE == 0)
            chl[i] = Ar::channel(llr[i], P.frac, P.qmax);
        for (int c = 1; c <= M; c++)
            Lc(c)[i] = 0.0f;
        Lc(M + 1)[i] = frozen_bit(P.frozen_words, i) ? big : 0.0f;
    }
    for (int w = tid; w < NW; w += NT)
        dw[w] = 0;
    if (tid == 0) {
        for (int j = 0; j <= M; j++)
            ctl->p[j] = 0;
    }
    sync<WAVE>();

    int64_t pe = 0;
    int t = 1;
    for (; t <= P.max_iter; t++) {
        if (tid == 0)
            ctl->walking = 1;
        for (int j = 1; j <= M; j++) {
            const int s = M - j;
            const int h = 1 << s;
            const int f = ctl->p[j - 1] << (s + 1);  // frozen rows, column j
            float *Lj = Lc(j);
            const float *Lj1 = Lc(j + 1);
            // The walk's first check of this stage starts on the last word of
            // its block (below); its L inputs (column j+1, which the sweep
            // does not write) are loaded now, so the latency overlaps the
            // sweep.
            const int pj0 = max(ctl->p[j], 2 * ctl->p[j - 1]);
            const int hl = h < 64 ? h : 64;      // rows of the last word
            float lpre = 0.0f;
            if (P.freezing && P.freeze_input && pj0 < (1 << j) && lane < hl)
                lpre = Lj1[(pj0 << s) + h - hl + lane];
            // ---- PE updates, eq. (1) ----
            // kBatch PEs per thread at a time: all their loads are issued
            // before any of their stores (which may alias as far as the
            // compiler can tell), so their latencies overlap.  Stage 1 reads
            // the channel column, the others the working column: two copies
            // of the loop, so that each pointer keeps its address space.
            auto sweep = [&](const float *Rin) {
#pragma unroll 1
                for (int q0 = (f >> 1) + tid; q0 < N / 2; q0 += kBatch * NT) {
                    float La[kBatch], Lb[kBatch], Ra[kBatch], Rb[kBatch];
                    int ia[kBatch];
#pragma unroll
                    for (int u = 0; u < kBatch; u++) {
                        const int q = q0 + u * NT;
                        const int a = ((q >> s) << (s + 1)) | (q & (h - 1));
                        ia[u] = a;
                        if (q < N / 2) {
                            La[u] = Lj1[a];
                            Lb[u] = Lj1[a + h];
                            Ra[u] = Rin[a];
                            Rb[u] = Rin[a + h];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kBatch; u++) {
                        if (q0 + u * NT < N / 2) {
                            const int a = ia[u], b = a + h;
                            float oLa, oLb, oRa, oRb;
                            Ar::pe(La[u], Lb[u], Ra[u], Rb[u], alpha, P.qmax,
                                   oLa, oLb, oRa, oRb);
                            Lj[a] = oLa;
                            Lj[b] = oLb;
                            Rw[a] = oRa;
                            Rw[b] = oRb;
                        }
                    }
                }
            };
            // h >= 4: four consecutive PEs per thread, rows a..a+3 and
            // b..b+3 each one 16-byte access (columns are 16-byte aligned;
            // the caller's channel column may not be)
            auto sweep4 = [&](const float *Rin) {
#pragma unroll 1
                for (int g0 = (f >> 3) + tid; g0 < N / 8; g0 += kBatch4 * NT) {
                    float4 La[kBatch4], Lb[kBatch4], Ra[kBatch4], Rb[kBatch4];
                    int ia[kBatch4];
#pragma unroll
                    for (int u = 0; u < kBatch4; u++) {
                        const int q = 4 * (g0 + u * NT);
                        const int a = ((q >> s) << (s + 1)) | (q & (h - 1));
                        ia[u] = a;
                        if (g0 + u * NT < N / 8) {
                            La[u] = ld4(Lj1 + a);
                            Lb[u] = ld4(Lj1 + a + h);
                            Ra[u] = ld4(Rin + a);
                            Rb[u] = ld4(Rin + a + h);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kBatch4; u++) {
                        if (g0 + u * NT < N / 8) {
                            const int a = ia[u], b = a + h;
                            float4 oLa, oLb, oRa, oRb;
                            Ar::pe(La[u].x, Lb[u].x, Ra[u].x, Rb[u].x, alpha, P.qmax,
                                   oLa.x, oLb.x, oRa.x, oRb.x);
                            Ar::pe(La[u].y, Lb[u].y, Ra[u].y, Rb[u].y, alpha, P.qmax,
                                   oLa.y, oLb.y, oRa.y, oRb.y);
                            Ar::pe(La[u].z, Lb[u].z, Ra[u].z, Rb[u].z, alpha, P.qmax,
                                   oLa.z, oLb.z, oRa.z, oRb.z);
                            Ar::pe(La[u].w, Lb[u].w, Ra[u].w, Rb[u].w, alpha, P.qmax,
                                   oLa.w, oLb.w, oRa.w, oRb.w);
                            st4(Lj + a, oLa);
                            st4(Lj + b, oLb);
                            st4(Rw + a, oRa);
                            st4(Rw + b, oRb);
                        }
                    }
                }
            };
            if (j > 1) {
                if (h >= 4)
                    sweep4(Rw);
                else
                    sweep(Rw);
            } else {
                if (h >= 4 && ch_aligned)
                    sweep4(ch);
                else
                    sweep(ch);
            }
            pe += (N - f) >> 1;
            sync_stage<WAVE, STATE>();
            if (!P.freezing)
                continue;
            // ---- CSFG freezing walk (Section III) ----
            // Each check first tests the block's last word: its positions
            // have every higher in-block row bit set, so eq. (3) maps that
            // word onto itself, and a frozen 1 there fails the block.  Every
            // wavefront computes this test alike (no barrier); when the block
            // is one word (h <= 64) it is the whole check.  Otherwise the
            // full check follows: its ballots and the freeze writes are
            // shared out over the group's wavefronts, and wavefront 0
            // transforms and tests.
            {
                int pj = pj0;
                int walking = ctl->walking;
                float *L1 = Lc(j + 1);
                const int nw = h >= 64 ? h >> 6 : 1;
                while (pj < (1 << j) && (P.freeze_walk != 0 || walking)) {
                    const int r0 = pj << s;
                    {
                        const int rl = r0 + h - hl;      // first row of the word
                        float v = 0.0f;
                        if (lane < hl) {
                            const float lv = pj == pj0 ? lpre : L1[rl + lane];
                            v = P.freeze_input ? Rw[rl + lane] + lv : Rw[rl + lane];
                        }
                        const uint64_t xl = __ballot(v < 0.0f);
                        const uint64_t ul = ffx_word(xl);
                        const uint64_t fz =
                            h >= 64 ? P.frozen_words[rl >> 6]
                                    : (P.frozen_words[r0 >> 6] >> (r0 & 63)) &
                                          ((1ull << h) - 1);
                        if (ul & fz)
                            break;
                        if (h <= 64) {
                            // passed: keep uhat, L at column j+1 := (-1)^xhat inf
                            if (tid < h)
                                L1[r0 + tid] = ((xl >> tid) & 1) ? -big : big;
                            if (tid == 0) {
                                const uint64_t msk = (h == 64 ? ~0ull : ((1ull << h) - 1))
                                                     << (r0 & 63);
                                dw[r0 >> 6] = (dw[r0 >> 6] & ~msk) | (ul << (r0 & 63));
                            }
                            pj++;
                            if (P.freeze_walk == 0) {
                                walking = 0;
                                break;
                            }
                            if (P.freeze_walk == 1)
                                break;
                            continue;
                        }
                    }
                    // eq. (2): hard decisions of the CSFG's inputs, the
                    // loads of kBatch words in flight before their ballots
#pragma unroll 1
                    for (int w0 = wv * kBatch; w0 < nw; w0 += nwv * kBatch) {
                        float v[kBatch];
#pragma unroll
                        for (int u = 0; u < kBatch; u++) {
                            const int i = 64 * (w0 + u) + lane;
                            v[u] = 0.0f;
                            if (w0 + u < nw && i < h)
                                v[u] = P.freeze_input ? Rw[r0 + i] + L1[r0 + i]
                                                      : Rw[r0 + i];
                        }
#pragma unroll
                        for (int u = 0; u < kBatch; u++) {
                            const uint64_t bal = __ballot(v[u] < 0.0f);
                            if (lane == 0 && w0 + u < nw)
                                xw[w0 + u] = bal;
                        }
                    }
                    sync_stage<WAVE, STATE>();
                    if (wave0) {
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
                        bad = __any(bad);
                        if (!bad) {
                            // keep uhat; a CSFG may cover sub-CSFGs of
                            // later stages frozen before it: its decisions
                            // replace theirs
#pragma unroll
                            for (int q = 0; q < kMaxWordsPerLane; q++) {
                                const int w = lane + 64 * q;
                                if (w < nw) {
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
                        }
                        if (lane == 0)
                            ctl->bad = bad;
                    }
                    sync_stage<WAVE, STATE>();
                    if (ctl->bad)
                        break;
                    // freeze: L at column j+1 := (-1)^xhat inf
                    for (int i = tid; i < h; i += NT) {
                        const bool x = (xw[i >> 6] >> (i & 63)) & 1;
                        L1[r0 + i] = x ? -big : big;
                    }
                    pj++;
                    if (P.freeze_walk == 0) {
                        walking = 0;
                        break;
                    }
                    if (P.freeze_walk == 1)
                        break;
                    // the next check's ballots reuse the words read above
                    sync_stage<WAVE, STATE>();
                }
                // every thread computed the same pj and walking
                if (tid == 0) {
                    ctl->p[j] = pj;
                    ctl->walking = walking;
                }
            }
            sync_stage<WAVE, STATE>();
        }
        // the sweep's L stores complete before the stop test reads column 1
        // and before the next sweep reads them
        sync<WAVE>();

        // ---- decisions, termination ----
        const int fm = P.freezing ? ctl->p[M] : 0;
        int stop = P.freezing && fm == N;
        if (!stop && P.early_stop) {
            // G-matrix criterion: uhat F^{(x)m} == hard(R + L) at column 1;
            // the ballots are shared out over the wavefronts, wavefront 0
            // transforms
            const float *L1 = Lc(1);
#pragma unroll 1
            for (int w0 = wv * kBatch; w0 < NW; w0 += nwv * kBatch) {
                float rv[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; u++) {
                    const int i = 64 * (w0 + u) + lane;
                    rv[u] = (w0 + u < NW && i < N) ? Rw[i] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kBatch; u++) {
                    const int w = w0 + u;
                    const int i = 64 * w + lane;
                    bool x = false;
                    if (w < NW && i < N) {
                        if (i < fm)
                            x = (dw[w] >> (i & 63)) & 1;
                        else
                            x = !frozen_bit(P.frozen_words, i) && rv[u] < 0.0f;
                    }
                    const uint64_t bal = __ballot(x);
                    if (lane == 0 && w < NW)
                        xw[w] = bal;
                }
            }
            sync_stage<WAVE, STATE>();
            if (wave0) {
                uint64_t r[kMaxWordsPerLane];
#pragma unroll
                for (int q = 0; q < kMaxWordsPerLane; q++) {
                    const int w = lane + 64 * q;
                    r[q] = w < NW ? ffx_word(xw[w]) : 0;
                }
                ffx_cross(r, NW, lane);
                // the transformed words replace the source words
                sync<true>();
#pragma unroll
                for (int q = 0; q < kMaxWordsPerLane; q++) {
                    const int w = lane + 64 * q;
                    if (w < NW)
                        xw[w] = r[q];
                }
                if (lane == 0)
                    ctl->ndiff = 0;
            }
            sync_stage<WAVE, STATE>();
            bool diff = false;
#pragma unroll 1
            for (int w0 = wv * kBatch; w0 < NW; w0 += nwv * kBatch) {
                float v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; u++) {
                    const int i = 64 * (w0 + u) + lane;
                    v[u] = (w0 + u < NW && i < N) ? ch[i] + L1[i] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kBatch; u++) {
                    const int w = w0 + u;
                    const uint64_t bal = __ballot(v[u] < 0.0f);
                    if (w < NW)
                        diff |= xw[w] != bal;
                }
            }
            if (lane == 0 && diff)
                ctl->ndiff = 1;
            sync_stage<WAVE, STATE>();
            stop = ctl->ndiff == 0;
        }
        // end of the sweep: every thread has read the control words before
        // the next sweep changes them
        sync<WAVE>();
        if (stop)
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
    if constexpr (Ar::kFixed) {
        if (P.soft_q) {
            // sat(R + L) at column m+1 (+-Q inside frozen CSFGs), as bytes
            int8_t *so = P.soft_q + frame * N;
            const float *Lm = Lc(M + 1);
            for (int i = tid; i < N; i += NT)
                so[i] = (int8_t)(int)(i < fm ? (((dw[i >> 6] >> (i & 63)) & 1) ? -big : big)
                                             : Ar::sat(Rw[i] + Lm[i], P.qmax));
        }
    } else if (P.soft_out) {
        float *so = P.soft_out + frame * N;
        const float *Lm = Lc(M + 1);
        for (int i = tid; i < N; i += NT)
            so[i] = i < fm ? (((dw[i >> 6] >> (i & 63)) & 1) ? -big : big)
                           : Rw[i] + Lm[i];
    }
    if (tid == 0) {
        P.iters_out[frame] = t;
        if (P.pe_out)
            P.pe_out[frame] = pe;
    }
    sync<WAVE>();
}

}  // namespace
}  // namespace generic
}  // namespace pbp
