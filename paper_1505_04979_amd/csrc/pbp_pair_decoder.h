// Workgroup-resident BP decoder for N = 2048 and N = 4096 (m = 11, 12): one
// workgroup of N / 4 threads decodes one frame with every message on chip.
// Shared by the batch kernel (pbp_decode.hip) and the mixed-code class
// kernels (pbp_mixed.hip).
//
// Stages are taken in pairs (j, j+1), j odd (Section II-A: stage j joins
// columns j and j+1).  Within a pair, thread t owns the four rows x + k h,
// k = 0..3, with h = 2^(m-j-1) and x the thread index with a zero pair of
// row bits inserted at bit m-j-1 (the pair's radix-4 group): stage j joins
// rows k and k+2 (distance 2h) and stage j+1 rows k and k+1 (distance h),
// so both stages' butterflies stay in the thread's registers.  Hence
//  - L at the even columns j+1 (written by stage j+1 and read by stage j of
//    the next iteration, on the same rows) lives in VGPRs, 4 per column;
//  - L at the odd columns 3, 5, ... (written by the first stage of one pair
//    and read by the second stage of the previous pair) lives in LDS;
//  - R flows through registers within a pair and through one LDS column
//    between pairs (a transpose onto the next pair's rows);
//  - L at column 1 is never stored: stage 1 ballots the channel-side
//    decisions of the stop test at once; L at column m+1 (the prior) is
//    computed where it is read: +inf at frozen rows, 0 at information rows,
//    (-1)^u inf on rows frozen at stage m (from the kept decisions).
// With m odd the last stage runs alone on rows 4t .. 4t+3.
//
// The schedule, the PE arithmetic (eq. (1) through the arithmetic policy), the CSFG walk and the stop test
// are those of the generic decoder, so results agree bit for bit.  LDS: the
// odd columns ((m-1)/2 columns of N floats), two R columns and two columns
// of check inputs used in turn, four bit words per 64 rows (one of them the
// frozen mask) and the published check words: 147.0 KB at N = 4096, 73.5 KB
// at N = 2048.  The channel
// LLRs stay in registers.  A pair of stages costs one barrier.  Checks of
// small blocks (at most 64 rows) run their test on the one wavefront that
// holds the block's word in registers, before that barrier; only a check that
// passes it runs the walk on the whole group.  Checks of large blocks are
// published: each wavefront ballots its words of the block before the
// barrier, and every wavefront transforms and tests them after it, so a
// failed check costs no further barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbp_arith.h"
#include "pbp_lanes.h"
#include "pbp_generic_decoder.h"
#include "pbp_internal.h"

namespace pbp {
namespace pair {
namespace {

using generic::Ctl;
using generic::DecodeParams;
using generic::ffx_cross;
using generic::ffx_word;
using generic::kBatch;
using generic::kMaxWordsPerLane;

template <int M>
struct Shape {
    static constexpr int N = 1 << M;
    static constexpr int NT = N / 4;          // threads of the workgroup
    static constexpr int NW = N / 64;         // bit words per frame
    static constexpr int NP = M / 2;          // stage pairs
    static constexpr int NL = (M - 1) / 2;    // odd columns 3, 5, .. <= m
};

// LDS bytes of one decoder: [u64 xw NW][u64 dw NW][u64 cw NW][u64 fw NW]
// [u64 published check words, 2 (pair parity) x 2 (stage of the pair) x
// N/128][Ctl][int first-test flags 2 x 2][f32 R, two columns of N, and the
// walk's check inputs, two columns of N][f32 L at the odd columns, NL x N]
template <int M>
__host__ __device__ constexpr size_t lds_bytes()
{
    return 4 * sizeof(uint64_t) * Shape<M>::NW +
           4 * sizeof(uint64_t) * (Shape<M>::N / 128) + sizeof(Ctl) +
           4 * sizeof(int) +
           sizeof(float) * (size_t)(4 + Shape<M>::NL) * Shape<M>::N;
}

// Ar: the message arithmetic (pbp_arith.h); arith::Fixed decodes b-bit
// integers, +-Q standing for the +-inf of frozen rows
template <int M, class Ar = arith::F32>
struct Decoder {
    using S = Shape<M>;
    static constexpr int N = S::N, NT = S::NT, NW = S::NW, NP = S::NP;
    static constexpr int NWV = NT / 64;       // wavefronts of the group
    // the R column pair PI reads (PI > 0) and the one it writes; with m odd
    // the last stage reads column NP and writes column NP + 1 (mod 2)
    static constexpr int RIN(int pi) { return pi & 1; }
    static constexpr int ROUT(int pi) { return (pi + 1) & 1; }
    static constexpr int RFINAL = (M & 1) ? ROUT(NP) : ROUT(NP - 1);

    const DecodeParams &P;
    uint64_t *xw;         // check and stop-test words
    uint64_t *dw;         // kept source decisions of frozen rows
    uint64_t *cw;         // channel-side decisions of the stop test
    uint64_t *fw;         // the frozen mask (bit i of word i >> 6)
    uint64_t *xp;         // published check words (see run_pair)
    Ctl *ctl;
    int *fl;              // first-test results, [pair parity][stage of pair]
    float *Rb;            // two R columns used in turn by the pairs, and the
                          // check inputs of the register-column walks
    float *Lo;            // L at the odd columns
    const int tid, lane, wv;
    float Lr[NP][4];      // L at column 2 pi + 2, rows of pair pi
    float Rv[4];          // R at the current column, rows of the pair
    float chv[4];         // the frame's channel LLRs, rows of pair 0
    int p[M + 1];         // frozen CSFG prefix per stage (same in all threads)
    int walking;
    int64_t pe;

    __device__ __forceinline__ Decoder(const DecodeParams &P_,
                                       unsigned char *smem, int tid_)
        : P(P_), tid(tid_), lane(tid_ & 63), wv(tid_ >> 6)
    {
        xw = reinterpret_cast<uint64_t *>(smem);
        dw = xw + NW;
        cw = dw + NW;
        fw = cw + NW;
        xp = fw + NW;
        ctl = reinterpret_cast<Ctl *>(xp + 4 * (N / 128));
        fl = reinterpret_cast<int *>(ctl + 1);
        Rb = reinterpret_cast<float *>(fl + 4);
        Lo = Rb + 4 * N;
    }

    __device__ __forceinline__ float *rcol(int b) const { return Rb + b * N; }

    // the message standing for inf: +inf, or Q in fixed point
    __device__ __forceinline__ float big() const { return Ar::big(P.qmax); }

    // L at odd column c, 3 <= c <= m
    __device__ __forceinline__ float *lcol(int c) const
    {
        return Lo + (size_t)((c - 3) >> 1) * N;
    }

    // row of register k in the radix-4 group whose finer butterfly is on
    // row bit SB.  The thread index is made opaque at each use: rows and LDS
    // addresses of all pairs would otherwise be hoisted out of the loops
    // and kept in registers.
    template <int SB>
    __device__ __forceinline__ void rows_of(int (&rows)[4]) const
    {
        int t = tid;
        asm volatile("" : "+v"(t));
        const int x = ((t >> SB) << (SB + 2)) | (t & ((1 << SB) - 1));
#pragma unroll
        for (int k = 0; k < 4; k++)
            rows[k] = x + (k << SB);
    }

    // L at column m+1
    __device__ __forceinline__ float prior(int i) const
    {
        if (i < p[M])
            return ((dw[i >> 6] >> (i & 63)) & 1) ? -big() : big();
        return ((fw[i >> 6] >> (i & 63)) & 1) ? big() : 0.0f;
    }

    // ---- CSFG walk at stage J (Section III, eqs. (2)-(4)) ----
    //
    // vin(i): the input of eq. (2) at row i of column J+1, read from LDS
    // (written before the last barrier; the caller keeps what it reads
    // unchanged until the next barrier); fix(i, x): freeze L at column J+1,
    // row i, to (-1)^x inf when that column is in LDS (register columns are
    // fixed by their owners after the walk).  Every thread runs the walk and
    // computes the same prefix.  Each check first tests the block's last word
    // (positions with every higher in-block row bit set, which eq. (3) maps
    // onto themselves): every wavefront ballots it alike, so a failed test,
    // the common case, ends the walk with no barrier and no shared write.
    // It is the whole check when the block is one word; otherwise all words
    // are ballotted and wavefront 0 transforms and tests eq. (4).
    template <int J, class VIN, class FIX>
    __device__ __forceinline__ void walk(int pj0, VIN vin, FIX fix)
    {
        constexpr int s = M - J, h = 1 << s;
        constexpr int hl = h < 64 ? h : 64;
        constexpr int nw = h >= 64 ? h >> 6 : 1;
        int pj = pj0;
        bool wrote = false;
        while (pj < (1 << J) && (P.freeze_walk != 0 || walking)) {
            const int r0 = pj << s;
            {
                const int rl = r0 + h - hl;
                const float v = lane < hl ? vin(rl + lane) : 0.0f;
                const uint64_t xl = __ballot(v < 0.0f);
                const uint64_t ul = ffx_word(xl);
                const uint64_t fz =
                    h >= 64 ? fw[rl >> 6]
                            : (fw[r0 >> 6] >> (r0 & 63)) & ((1ull << h) - 1);
                if (ul & fz)
                    break;
                if constexpr (h <= 64) {
                    if (tid < h)
                        fix(r0 + tid, (xl >> tid) & 1);
                    if (tid == 0) {
                        const uint64_t msk = (h == 64 ? ~0ull : ((1ull << h) - 1))
                                             << (r0 & 63);
                        dw[r0 >> 6] = (dw[r0 >> 6] & ~msk) | (ul << (r0 & 63));
                    }
                    wrote = true;
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
            if constexpr (h > 64) {
                // eq. (2) over the block, kBatch words per wavefront at a time
#pragma unroll 1
                for (int w0 = wv * kBatch; w0 < nw; w0 += NWV * kBatch) {
                    float v[kBatch];
#pragma unroll
                    for (int u = 0; u < kBatch; u++)
                        v[u] = w0 + u < nw ? vin(r0 + 64 * (w0 + u) + lane) : 0.0f;
#pragma unroll
                    for (int u = 0; u < kBatch; u++) {
                        const uint64_t bal = __ballot(v[u] < 0.0f);
                        if (lane == 0 && w0 + u < nw)
                            xw[w0 + u] = bal;
                    }
                }
                __syncthreads();
                if (wv == 0) {
                    // eq. (3): uhat = xhat F^{(x)s}; eq. (4) on the frozen rows
                    uint64_t r[kMaxWordsPerLane];
#pragma unroll
                    for (int q = 0; q < kMaxWordsPerLane; q++) {
                        const int w = lane + 64 * q;
                        r[q] = w < nw ? ffx_word(xw[w]) : 0;
                    }
                    ffx_cross(r, nw, lane);
                    bool bad = false;
#pragma unroll
                    for (int q = 0; q < kMaxWordsPerLane; q++) {
                        const int w = lane + 64 * q;
                        if (w < nw)
                            bad |= (r[q] & fw[(r0 >> 6) + w]) != 0;
                    }
                    bad = __any(bad);
                    if (!bad) {
                        // the CSFG's decisions replace those of any sub-CSFG
                        // of a later stage frozen before it
#pragma unroll
                        for (int q = 0; q < kMaxWordsPerLane; q++) {
                            const int w = lane + 64 * q;
                            if (w < nw)
                                dw[(r0 >> 6) + w] = r[q];
                        }
                    }
                    if (lane == 0)
                        ctl->bad = bad;
                }
                __syncthreads();
                if (ctl->bad)
                    break;
                for (int i = tid; i < h; i += NT)
                    fix(r0 + i, (xw[i >> 6] >> (i & 63)) & 1);
                wrote = true;
                pj++;
                if (P.freeze_walk == 0) {
                    walking = 0;
                    break;
                }
                if (P.freeze_walk == 1)
                    break;
                // the next check's ballots reuse xw
                __syncthreads();
            }
        }
        p[J] = pj;
        // a freeze's LDS writes (fixed messages, kept decisions) before
        // anything reads them
        if (wrote)
            __syncthreads();
    }

    // The first test of a check (its block's last word, which eq. (3) maps
    // onto itself), computed before the barrier by the one wavefront that
    // holds that word in registers, and published in *flag (1: the word
    // decodes to no frozen 1, so the full check must run).  v: the check
    // inputs of the thread's rows in the radix-4 group with finer row bit
    // SB; the block is CSFG pj of the group's first stage (FIRST, 2^(SB+1)
    // rows) or second stage (2^SB rows).  Row r is register (r >> SB) & 3 of
    // thread ((r >> (SB + 2)) << SB) | (r & (2^SB - 1)).  The result equals
    // the walk's own first test, which every wavefront would otherwise
    // repeat on the scalar unit that a compute unit's wavefronts share.
    template <int SB, bool FIRST>
    __device__ __forceinline__ void owner_test(int pj, const float (&v)[4],
                                               int *flag) const
    {
        constexpr int LB = FIRST ? SB + 1 : SB;     // log2 of the block rows
        constexpr int h = 1 << LB;
        constexpr int hl = h < 64 ? h : 64;
        const int r0 = pj << LB;
        const int rl = r0 + h - hl;                 // first row of the word
        int tb;                                     // thread of its bit 0
        if constexpr (SB >= 6)
            tb = ((rl >> (SB + 2)) << SB) | (rl & ((1 << SB) - 1));
        else
            tb = (r0 >> (SB + 2)) << SB;
        if (wv != (tb >> 6))
            return;
        uint64_t word;
        if constexpr (SB >= 6) {
            // 64 rows of one register on 64 consecutive threads
            const int k = (rl >> SB) & 3;
            word = __ballot(v[k] < 0.0f);
        } else {
            // 2^SB threads from lane tb & 63; a first-stage block spans two
            // registers (row bit SB), a second-stage block one
            constexpr uint64_t m = SB == 5 ? 0xFFFFFFFFull
                                           : ((1ull << (1 << SB)) - 1);
            const int lb = tb & 63;
            const int k = (r0 >> SB) & 3;
            word = (__ballot(v[k] < 0.0f) >> lb) & m;
            if constexpr (FIRST)
                word |= ((__ballot(v[k + 1] < 0.0f) >> lb) & m) << (1 << SB);
        }
        const uint64_t fz =
            h >= 64 ? fw[rl >> 6] : (fw[r0 >> 6] >> (r0 & 63)) & ((1ull << h) - 1);
        if (lane == 0)
            *flag = (ffx_word(word) & fz) == 0;
    }

    // Published checks.  Where a check's block is made of whole 64-row words
    // and each word is one register of one wavefront (pair row bit SB >= 6),
    // every wavefront ballots its words of the block before the pair's
    // barrier into buf, and after it every wavefront transforms all of the
    // block's words (at most N/128: one per lane) and tests eq. (4) alike.
    // A failed check, the common case for large blocks, then costs no
    // barrier and no shared write.  (The first test on the block's last word
    // is no filter there: a large block's last rows are mostly information
    // rows, so that word nearly always passes.)
    //
    // publish: the words of CSFG pj (2^LB rows) held by this wavefront
    template <int LB>
    __device__ __forceinline__ void publish(int pj, const float (&v)[4],
                                            const int (&rows)[4], uint64_t *buf) const
    {
        constexpr int NB = 1 << (LB - 6);
        const int w0 = pj << (LB - 6);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            // the wavefront's 64 rows of register k are one aligned word
            const int o = (__builtin_amdgcn_readfirstlane(rows[k]) >> 6) - w0;
            if (o >= 0 && o < NB) {
                const uint64_t b = __ballot(v[k] < 0.0f);
                if (lane == 0)
                    buf[o] = b;
            }
        }
    }

    // eqs. (3)-(4) on the published words of CSFG pj: true when it passes;
    // u: this lane's transformed word (lane w, word w of the block)
    template <int LB>
    __device__ __forceinline__ bool published_check(int pj, const uint64_t *buf,
                                                    uint64_t &u) const
    {
        constexpr int NB = 1 << (LB - 6);
        const int w0 = pj << (LB - 6);
        const bool in = lane < NB;
        uint64_t x = in ? ffx_word(buf[lane]) : 0;
#pragma unroll
        for (int L = 1; L < NB; L <<= 1) {
            const uint64_t o = lanes::down_u64(x, L);
            if (!(lane & L))
                x ^= o;
        }
        u = x;
        return !__any(in && (x & fw[w0 + (in ? lane : 0)]) != 0);
    }

    // after a published check of CSFG pj passed: the CSFG's decisions replace
    // those of any sub-CSFG frozen before it (wavefront 0 writes them)
    template <int LB>
    __device__ __forceinline__ void keep_published(int pj, uint64_t u) const
    {
        constexpr int NB = 1 << (LB - 6);
        if (wv == 0 && lane < NB)
            dw[(pj << (LB - 6)) + lane] = u;
    }

    // One pair of stages: J = 2 PI + 1 and J + 1, with one barrier.
    //  - R at column J comes from the channel (PI = 0) or the R column the
    //    previous pair wrote; R at column J+2 goes to the other R column,
    //    whose last readers passed the previous pair's barrier.
    //  - The L outputs of stage J (odd column J) are stored after the
    //    barrier: the previous pair's walk reads that column after its own
    //    barrier, with no barrier behind it when it freezes nothing.
    //  - The walk of stage J runs after stage J+1, on the check inputs kept
    //    from stage J.  This is the same computation: stage J+1's butterflies
    //    stay inside each CSFG of stage J, so on rows that the walk freezes
    //    stage J+1 only writes L at column J+1, which the freeze then
    //    overwrites, and R at column J+2, which is never read on frozen rows;
    //    the PE count takes stage J+1's prefix after the walk.
    template <int PI>
    __device__ __forceinline__ void run_pair()
    {
        constexpr int J = 2 * PI + 1;
        constexpr int SB = M - J - 1;         // row bit of stage J+1's butterfly
        const float alpha = P.alpha;
        float *Rout = rcol(ROUT(PI));
        // check inputs of stage J's walk: one of two columns by pair parity
        // (the previous pair's walk may still read the other one)
        float *Vb = rcol(2 + (PI & 1));
        int rows[4];
        rows_of<SB>(rows);
        if constexpr (PI == 0) {
#pragma unroll
            for (int k = 0; k < 4; k++)
                Rv[k] = chv[k];
        } else {
            const float *Rin = rcol(RIN(PI));
#pragma unroll
            for (int k = 0; k < 4; k++)
                Rv[k] = Rin[rows[k]];
        }

        // ---- stage J: rows (k, k+2) ----
        const int fJ = p[J - 1] << (M - J + 1);    // rows frozen at stage J-1
        float lj[4];                               // L at column J (J == 1:
                                                   // R + L there)
        bool ran[2];
#pragma unroll
        for (int e = 0; e < 2; e++) {
            const int ka = e, kb = e + 2;
            ran[e] = J == 1 || rows[ka] >= fJ;
            if (ran[e]) {
                float oLa, oLb, oRa, oRb;
                Ar::pe(Lr[PI][ka], Lr[PI][kb], Rv[ka], Rv[kb], alpha, P.qmax, oLa, oLb,
                       oRa, oRb);
                lj[ka] = J == 1 ? Rv[ka] + oLa : oLa;
                lj[kb] = J == 1 ? Rv[kb] + oLb : oLb;
                Rv[ka] = oRa;
                Rv[kb] = oRb;
            }
        }
        pe += (N - fJ) >> 1;
        if constexpr (J == 1) {
            // channel-side decisions of the stop test: the rows of register
            // k on wavefront w are the 64 rows of word w + k N / 256
            if (P.early_stop) {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint64_t b = __ballot(lj[k] < 0.0f);
                    if (lane == 0)
                        cw[wv + k * (N / 256)] = b;
                }
            }
        }
        // stage J's walk starts at CSFG pj0; its inputs at column J+1
        const int pj0 = P.freezing ? max(p[J], 2 * p[J - 1]) : 0;
        const bool walkJ = P.freezing && pj0 < (1 << J) &&
                           (P.freeze_walk != 0 || walking);
        float vv[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            vv[k] = P.freeze_input ? Rv[k] + Lr[PI][k] : Rv[k];

        // ---- stage J+1: rows (k, k+1), from the prefix before the walk ----
        const int fJ1 = pj0 << (M - J);
        float Lin[4];                              // L at column J+2
        {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                if constexpr (J + 2 <= M)
                    Lin[k] = lcol(J + 2)[rows[k]];
                else
                    Lin[k] = prior(rows[k]);
            }
#pragma unroll
            for (int e = 0; e < 2; e++) {
                const int ka = 2 * e, kb = 2 * e + 1;
                if (rows[ka] >= fJ1) {
                    float oLa, oLb, oRa, oRb;
                    Ar::pe(Lin[ka], Lin[kb], Rv[ka], Rv[kb], alpha, P.qmax, oLa, oLb,
                           oRa, oRb);
                    Lr[PI][ka] = oLa;
                    Lr[PI][kb] = oLb;
                    Rv[ka] = oRa;
                    Rv[kb] = oRb;
                }
            }
        }
        // first tests of both walks, stage J+1's assuming stage J freezes
        // nothing (else its walk runs in full below)
        int *flags = fl + 2 * (PI & 1);
        // published words, by pair parity: stage J's block, then stage J+1's
        uint64_t *xpJ = xp + (PI & 1) * (2 * (N / 128));
        uint64_t *xpJ1 = xpJ + N / 128;
        constexpr bool PUBJ = SB >= 6, PUB1 = SB >= 7;
        const int pj1s = P.freezing ? max(p[J + 1], 2 * pj0) : 0;
        if (walkJ) {
            if constexpr (PUBJ)
                publish<SB + 1>(pj0, vv, rows, xpJ);
            else
                owner_test<SB, true>(pj0, vv, flags);
        }
        if (P.freezing && pj1s < (1 << (J + 1)) &&
            (P.freeze_walk != 0 || walking)) {
            float v1[4];
#pragma unroll
            for (int k = 0; k < 4; k++)
                v1[k] = P.freeze_input ? Rv[k] + Lin[k] : Rv[k];
            if constexpr (PUB1)
                publish<SB>(pj1s, v1, rows, xpJ1);
            else
                owner_test<SB, false>(pj1s, v1, flags + 1);
        }
        // R at column J+2 and the walk's inputs, in row order; then the
        // barrier; then stage J's L outputs
#pragma unroll
        for (int k = 0; k < 4; k++) {
            Rout[rows[k]] = Rv[k];
            if (walkJ)
                Vb[rows[k]] = vv[k];
        }
        __syncthreads();
        if constexpr (J >= 3) {
#pragma unroll
            for (int e = 0; e < 2; e++) {
                if (ran[e]) {
                    lcol(J)[rows[e]] = lj[e];
                    lcol(J)[rows[e + 2]] = lj[e + 2];
                }
            }
        }

        // ---- walk at stage J: column J+1 is held in registers ----
        auto vinJ = [&](int i) { return Vb[i]; };
        bool ranJ = false;
        if constexpr (PUBJ) {
            p[J] = pj0;
            uint64_t u;
            if (walkJ && published_check<SB + 1>(pj0, xpJ, u)) {
                keep_published<SB + 1>(pj0, u);
                p[J] = pj0 + 1;
                if (P.freeze_walk == 0)
                    walking = 0;
                // the kept decisions before any reader
                __syncthreads();
                if (P.freeze_walk == 2)
                    walk<J>(pj0 + 1, vinJ, [](int, bool) {});
                ranJ = true;
            }
        } else {
            if (walkJ && flags[0]) {
                walk<J>(pj0, vinJ, [](int, bool) {});
                ranJ = true;
            } else {
                p[J] = pj0;
            }
        }
        if (ranJ) {
            const int lo = pj0 << (M - J), hi = p[J] << (M - J);
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (rows[k] >= lo && rows[k] < hi)
                    Lr[PI][k] = vv[k] < 0.0f ? -big() : big();
        }
        pe += (N - (p[J] << (M - J))) >> 1;

        // ---- walk at stage J+1: column J+2 is in LDS, or the prior ----
        // (skipped when its first test failed on the blocks assumed above;
        // with large blocks, the published check when stage J froze nothing)
        bool done1 = false;
        if constexpr (PUB1) {
            if (P.freezing && p[J] == pj0) {
                done1 = true;
                p[J + 1] = pj1s;
                uint64_t u;
                if (pj1s < (1 << (J + 1)) && (P.freeze_walk != 0 || walking) &&
                    published_check<SB>(pj1s, xpJ1, u)) {
                    keep_published<SB>(pj1s, u);
                    // L at column J+2 := (-1)^xhat inf on the block's rows
                    if constexpr (J + 2 <= M) {
                        float *Lc = lcol(J + 2);
                        const int r0 = pj1s << SB;
                        for (int i = tid; i < (1 << SB); i += NT)
                            Lc[r0 + i] = ((xpJ1[i >> 6] >> (i & 63)) & 1) ? -big() : big();
                    }
                    p[J + 1] = pj1s + 1;
                    if (P.freeze_walk == 0)
                        walking = 0;
                    __syncthreads();
                    if (P.freeze_walk == 2) {
                        if constexpr (J + 2 <= M) {
                            float *Lc = lcol(J + 2);
                            auto vin = [&](int i) {
                                return P.freeze_input ? Rout[i] + Lc[i] : Rout[i];
                            };
                            walk<J + 1>(pj1s + 1, vin,
                                        [&](int i, bool x) { Lc[i] = x ? -big() : big(); });
                        } else {
                            auto vin = [&](int i) {
                                return P.freeze_input ? Rout[i] + prior(i) : Rout[i];
                            };
                            walk<J + 1>(pj1s + 1, vin, [](int, bool) {});
                        }
                    }
                }
            }
        }
        if (!done1) {
            if (P.freezing &&
                (p[J] != pj0 || pj1s >= (1 << (J + 1)) || flags[1] || PUB1)) {
                const int pj1 = max(p[J + 1], 2 * p[J]);
                if constexpr (J + 2 <= M) {
                    float *Lc = lcol(J + 2);
                    auto vin = [&](int i) {
                        return P.freeze_input ? Rout[i] + Lc[i] : Rout[i];
                    };
                    walk<J + 1>(pj1, vin,
                                [&](int i, bool x) { Lc[i] = x ? -big() : big(); });
                } else {
                    auto vin = [&](int i) {
                        return P.freeze_input ? Rout[i] + prior(i) : Rout[i];
                    };
                    walk<J + 1>(pj1, vin, [](int, bool) {});
                }
            } else if (P.freezing) {
                p[J + 1] = pj1s;
            }
        }
    }

    template <int PI>
    __device__ __forceinline__ void run_pairs()
    {
        if constexpr (PI < NP) {
            run_pair<PI>();
            run_pairs<PI + 1>();
        }
    }

    // m odd: stage m alone on rows 4t .. 4t+3 (L at column m+1 is the prior,
    // L at column m an odd LDS column, stored after the barrier)
    __device__ __forceinline__ void run_last()
    {
        constexpr int J = M;
        const float alpha = P.alpha;
        const float *Rin = rcol(ROUT(NP - 1));
        float *Rout = rcol(RFINAL);
        int rows[4];
        rows_of<0>(rows);
#pragma unroll
        for (int k = 0; k < 4; k++)
            Rv[k] = Rin[rows[k]];
        const int fJ = p[J - 1] << 1;
        float Lin[4], lj[4];
        bool ran[2];
#pragma unroll
        for (int k = 0; k < 4; k++)
            Lin[k] = prior(rows[k]);
#pragma unroll
        for (int e = 0; e < 2; e++) {
            const int ka = 2 * e, kb = 2 * e + 1;
            ran[e] = rows[ka] >= fJ;
            if (ran[e]) {
                float oLa, oLb, oRa, oRb;
                Ar::pe(Lin[ka], Lin[kb], Rv[ka], Rv[kb], alpha, P.qmax, oLa, oLb, oRa,
                       oRb);
                lj[ka] = oLa;
                lj[kb] = oLb;
                Rv[ka] = oRa;
                Rv[kb] = oRb;
            }
        }
        pe += (N - fJ) >> 1;
        int *flags = fl + 2 * (NP & 1);
        const int pj = P.freezing ? max(p[J], 2 * p[J - 1]) : 0;
        if (P.freezing && pj < (1 << J)) {
            float v1[4];
#pragma unroll
            for (int k = 0; k < 4; k++)
                v1[k] = P.freeze_input ? Rv[k] + Lin[k] : Rv[k];
            owner_test<0, false>(pj, v1, flags);
        }
#pragma unroll
        for (int k = 0; k < 4; k++)
            Rout[rows[k]] = Rv[k];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 2; e++) {
            if (ran[e]) {
                lcol(J)[rows[2 * e]] = lj[2 * e];
                lcol(J)[rows[2 * e + 1]] = lj[2 * e + 1];
            }
        }
        if (P.freezing) {
            if (pj >= (1 << J) || flags[0]) {
                auto vin = [&](int i) {
                    return P.freeze_input ? Rout[i] + prior(i) : Rout[i];
                };
                walk<J>(pj, vin, [](int, bool) {});
            } else {
                p[J] = pj;
            }
        }
    }

    // G-matrix stop test: uhat F^{(x)m} == the channel-side decisions
    __device__ __forceinline__ bool stop_test(int fm)
    {
        const float *Rf = rcol(RFINAL);
#pragma unroll 1
        for (int w = wv; w < NW; w += NWV) {
            const int i = 64 * w + lane;
            const bool x = i < fm ? ((dw[w] >> lane) & 1)
                                  : (!((fw[w] >> lane) & 1) && Rf[i] < 0.0f);
            const uint64_t bal = __ballot(x);
            if (lane == 0)
                xw[w] = bal;
        }
        __syncthreads();
        if (wv == 0) {
            uint64_t r[kMaxWordsPerLane];
#pragma unroll
            for (int q = 0; q < kMaxWordsPerLane; q++) {
                const int w = lane + 64 * q;
                r[q] = w < NW ? ffx_word(xw[w]) : 0;
            }
            ffx_cross(r, NW, lane);
            bool diff = false;
#pragma unroll
            for (int q = 0; q < kMaxWordsPerLane; q++) {
                const int w = lane + 64 * q;
                if (w < NW)
                    diff |= r[q] != cw[w];
            }
            diff = __any(diff);
            if (lane == 0)
                ctl->ndiff = diff;
        }
        __syncthreads();
        return ctl->ndiff == 0;
    }

    __device__ __forceinline__ void decode(int64_t frame)
    {
        // the channel LLRs stay in registers for the whole frame (rows of
        // pair 0: t + k N / 4, coalesced), the frozen mask in LDS
        {
            const float *ch = P.llr + frame * N;
            int rows[4];
            rows_of<M - 2>(rows);
#pragma unroll
            for (int k = 0; k < 4; k++)
                chv[k] = Ar::channel(ch[rows[k]], P.frac, P.qmax);
        }
        for (int w = tid; w < NW; w += NT)
            fw[w] = P.frozen_words[w];
        // initial messages: L = 0 except the prior
#pragma unroll
        for (int pi = 0; pi < NP; pi++)
#pragma unroll
            for (int k = 0; k < 4; k++)
                Lr[pi][k] = 0.0f;
        for (int i = tid; i < S::NL * N; i += NT)
            Lo[i] = 0.0f;
        for (int w = tid; w < NW; w += NT)
            dw[w] = 0;
#pragma unroll
        for (int j = 0; j <= M; j++)
            p[j] = 0;
        pe = 0;
        __syncthreads();

        int t = 1;
        for (; t <= P.max_iter; t++) {
            walking = 1;
            run_pairs<0>();
            if constexpr (M & 1)
                run_last();
            // the last R column holds R at column m+1
            const int fm = P.freezing ? p[M] : 0;
            bool stop = P.freezing && fm == N;
            if (!stop && P.early_stop)
                stop = stop_test(fm);
            // every thread has read R and the control words before the
            // next sweep writes them
            __syncthreads();
            if (stop)
                break;
        }
        if (t > P.max_iter)
            t = P.max_iter;

        const int fm = P.freezing ? p[M] : 0;
        const float *Rf = rcol(RFINAL);
        uint8_t *out = P.info_out + frame * P.K;
        for (int k = tid; k < P.K; k += NT) {
            const int i = P.info_pos[k];
            out[k] = i < fm ? (uint8_t)((dw[i >> 6] >> (i & 63)) & 1)
                            : (uint8_t)(Rf[i] < 0.0f);
        }
        if constexpr (Ar::kFixed) {
            if (P.soft_q) {
                // sat(R + L) at column m+1 (+-Q inside frozen CSFGs), as bytes
                int8_t *so = P.soft_q + frame * N;
                for (int i = tid; i < N; i += NT)
                    so[i] = (int8_t)(int)(i < fm ? (((dw[i >> 6] >> (i & 63)) & 1) ? -big() : big())
                                                 : Ar::sat(Rf[i] + prior(i), P.qmax));
            }
        } else if (P.soft_out) {
            float *so = P.soft_out + frame * N;
            for (int i = tid; i < N; i += NT)
                so[i] = i < fm ? (((dw[i >> 6] >> (i & 63)) & 1) ? -big() : big())
                               : Rf[i] + prior(i);
        }
        if (tid == 0) {
            P.iters_out[frame] = t;
            if (P.pe_out)
                P.pe_out[frame] = pe;
        }
        __syncthreads();
    }
};

}  // namespace
}  // namespace pair
}  // namespace pbp
