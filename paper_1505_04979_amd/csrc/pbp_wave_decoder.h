// One-wavefront BP decoder for N <= 64 (m <= 6): every message of a frame in
// registers, one row per lane.  Used by pbp_decode (FP32) and by
// pbp_decode_quant (fixed point), through the arithmetic policy of
// pbp_arith.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbp_arith.h"
#include "pbp_generic_decoder.h"

namespace pbp {
namespace wave {
namespace {

// N <= 64: one wavefront per frame, row i on lane i, every message in
// registers.  Stage j pairs lanes i and i ^ h (h = N / 2^j): each lane reads
// its partner's L (column j+1) and R (column j) across lanes, evaluates
// eq. (1) as the other kernels do, and keeps its own row's two outputs, so a
// sweep needs neither LDS nor barriers.  A CSFG of stage j is a run of N/2^j
// lanes: its check (eqs. (2)-(4)) is one ballot, and lane i's bit of
// x F^{(x)s} is the parity of the ballot over the block lanes whose index
// contains i; a freeze writes +-inf into the block lanes' own L register and
// their decisions into one uniform word.  Rows below a stage's frozen prefix
// keep their L (their R is not read again in the sweep).  The stop test is
// the same parity over the whole word.
// This lane's two outputs of eq. (1) at a PE of stage j.  The PE joins rows
// a and b = a + h; lane a (up false) keeps L_a and R_a, lane b (up true) L_b
// and R_b.  Lin, R: this lane's L (column j+1) and R (column j); Lp, Rp: the
// partner's.  Each output is the policy's own expression on the same
// operands (so the results are those of Ar::pe), but only this row's two
// are evaluated: the a row's term aLa clampm(La, .) is L_a at the a lane
// and g1 at the b lane.
template <class Ar>
__device__ __forceinline__ void half_pe(bool up, float Lin, float Lp, float R,
                                        float Rp, float alpha, float q,
                                        float &oL, float &oR)
{
    const float La = up ? Lp : Lin;
    if constexpr (Ar::kFixed) {
        const float s = Ar::sat(Lp + Rp, q);             // a lane: Lb + Rb
        const float t = Ar::term(alpha, La, up ? Rp : s); // g1, or L_a
        oL = up ? Ar::sat(Lin + t, q) : t;
        oR = up ? Ar::sat(R + t, q) : Ar::term(alpha, R, s);
    } else {
        const float aLa = arith::salpha(La, alpha);
        const float s = Lp + Rp;                         // a lane: Lb + Rb
        const float t = aLa * arith::clampm(La, up ? Rp : s);
        oL = up ? Lin + t : t;
        oR = up ? R + t : arith::salpha(R, alpha) * arith::clampm(R, s);
    }
}

// Wavefronts per workgroup, each decoding its own frames (a compute unit
// holds at most 16 workgroups: groups of one wavefront would cap it at 16)
constexpr int kWaves = 4;

template <int M, bool FRZ, class Ar = arith::F32>
__global__ __launch_bounds__(64 * kWaves) void bp_decode_wave_kernel(generic::DecodeParams P)
{
    constexpr int N = 1 << M;
    static_assert(M >= 1 && M <= 6, "one row per lane");
    const int lane = (int)__builtin_amdgcn_workitem_id_x() & 63;
    const int wv = (int)__builtin_amdgcn_workitem_id_x() >> 6;
    const bool act = lane < N;
    const bool frz = act && ((P.frozen_words[0] >> lane) & 1);
    // lanes whose index contains this lane's index bits
    uint64_t sup = ~0ull;
#pragma unroll
    for (int lb = 0; lb < 6; lb++)
        if ((lane >> lb) & 1)
            sup &= (lb == 0 ? 0xAAAAAAAAAAAAAAAAull : lb == 1 ? 0xCCCCCCCCCCCCCCCCull
                    : lb == 2 ? 0xF0F0F0F0F0F0F0F0ull : lb == 3 ? 0xFF00FF00FF00FF00ull
                    : lb == 4 ? 0xFFFF0000FFFF0000ull : 0xFFFFFFFF00000000ull);
    // parity over the lanes of w that contain this lane's index
    auto par = [&](uint64_t w) {
        const uint64_t x = w & sup;
        return (uint32_t)(__builtin_popcount((uint32_t)x) +
                          __builtin_popcount((uint32_t)(x >> 32))) & 1u;
    };
    const float big = Ar::big(P.qmax);      // inf, or Q in fixed point
    const float prior = frz ? big : 0.0f;
    const float alpha = P.alpha;
    for (int64_t frame = (int64_t)blockIdx.x * kWaves + wv; frame < P.B;
         frame += (int64_t)gridDim.x * kWaves) {
        const float ch = act ? Ar::channel(P.llr[frame * N + lane], P.frac, P.qmax) : 0.0f;
        float L[M + 1];                // L at columns 1..m+1 (index c - 1)
#pragma unroll
        for (int c = 0; c < M; c++)
            L[c] = 0.0f;
        L[M] = prior;
        int p[M + 1];                  // frozen CSFG prefix per stage
#pragma unroll
        for (int j = 0; j <= M; j++)
            p[j] = 0;
        uint64_t dw = 0;               // kept decisions of frozen rows
        int64_t pe = 0;
        float R = 0.0f;                // R at column m+1 after a sweep
        int t = 1;
        for (; t <= P.max_iter; t++) {
            R = ch;
            uint64_t xw = 0;
            int walking = 1;
#pragma unroll
            for (int j = 1; j <= M; j++) {
                const int h = N >> j;
                const int f = FRZ ? p[j - 1] << (M - j + 1) : 0;
                const float Lin = L[j];
                const float Lp = __shfl_xor(Lin, h, 64);
                const float Rp = __shfl_xor(R, h, 64);
                const bool up = (lane & h) != 0;
                float lo, ro;
                half_pe<Ar>(up, Lin, Lp, R, Rp, alpha, P.qmax, lo, ro);
                L[j - 1] = (!FRZ || lane >= f) ? lo : L[j - 1];
                // channel-side decisions of the stop test: R + L at column 1
                if (j == 1 && P.early_stop)
                    xw = __ballot(act && R + L[0] < 0.0f);
                R = ro;
                pe += (N - f) >> 1;
                if constexpr (FRZ) {
                    // ---- CSFG walk at stage j (eqs. (2)-(4)) ----
                    const int SH = M - j;              // a block has 2^SH rows
                    int pj = max(p[j], 2 * p[j - 1]);
                    while (pj < (1 << j) && (P.freeze_walk != 0 || walking)) {
                        const int r0 = pj << SH;
                        const uint64_t lm = ((1ull << (1 << SH)) - 1) << r0;  // 2^SH <= 32
                        const bool in = (lm >> lane) & 1;
                        const float v = P.freeze_input ? R + L[j] : R;
                        const uint64_t w = __ballot(v < 0.0f) & lm;
                        const uint32_t ub = par(w);
                        if (__ballot(in && ub && frz) != 0)
                            break;
                        if (in)
                            L[j] = ((w >> lane) & 1) ? -big : big;
                        dw = (dw & ~lm) | (__ballot(in && ub) & lm);
                        pj++;
                        if (P.freeze_walk == 0) {
                            walking = 0;
                            break;
                        }
                        if (P.freeze_walk == 1)
                            break;
                    }
                    p[j] = pj;
                }
            }
            // source-word decisions: kept ones below the prefix of stage m
            const int fm = FRZ ? p[M] : 0;
            const uint64_t below = fm >= 64 ? ~0ull : ((1ull << fm) - 1);
            const uint64_t u = (dw & below) | (__ballot(act && !frz && R < 0.0f) & ~below);
            if (FRZ && fm == N)
                break;
            if (P.early_stop &&
                __ballot(act && par(u) != (uint32_t)((xw >> lane) & 1)) == 0)
                break;
        }
        if (t > P.max_iter)
            t = P.max_iter;
        const int fm = FRZ ? p[M] : 0;
        const uint64_t below = fm >= 64 ? ~0ull : ((1ull << fm) - 1);
        const uint64_t dec = (dw & below) | (__ballot(act && R < 0.0f) & ~below);
        uint8_t *out = P.info_out + frame * P.K;
        if (lane < P.K)
            out[lane] = (uint8_t)((dec >> P.info_pos[lane]) & 1);
        if constexpr (Ar::kFixed) {
            if (P.soft_q && act)
                P.soft_q[frame * N + lane] = (int8_t)(int)(
                    lane < fm ? (((dw >> lane) & 1) ? -big : big)
                              : Ar::sat(R + L[M], P.qmax));
        } else if (P.soft_out && act) {
            P.soft_out[frame * N + lane] =
                lane < fm ? (((dw >> lane) & 1) ? -big : big) : R + L[M];
        }
        if (lane == 0) {
            P.iters_out[frame] = t;
            if (P.pe_out)
                P.pe_out[frame] = pe;
        }
    }
}

}  // namespace
}  // namespace wave
}  // namespace pbp
