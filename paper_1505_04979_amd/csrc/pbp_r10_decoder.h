// Register-resident BP decoder for N = 1024 (m = 10): one wavefront per frame.
// Shared by the batch kernel (pbp_r10.hip) and the mixed-code persistent
// kernel (pbp_mixed.hip).
//
//
// One wavefront decodes one frame at a time; persistent wavefronts take
// frames from a device counter.  Each lane owns 16 rows of the factor
// graph.  Stages are taken in pairs (radix-4 groups); within a group the
// butterflies of both stages are register-local because the two butterfly
// row bits are register bits of that group's row-to-(register, lane)
// mapping.  The other two register bits are always the top row bits 9 and
// 8, so a frozen prefix of rows skips whole registers, uniformly over the
// wavefront (the frozen prefixes of Section III are coarse: 256-row
// granularity keeps most of the skipped PE work off the VALU).
//
//   mapping  register bits (q3 q2 q1 q0)   lane bits (l5..l0)   stages
//   MA       9 8 1 0                        7 6 5 4 3 2          1 2 9 10
//   MB       9 8 7 6                        5 4 3 2 1 0          3 4
//   MC       9 8 5 4                        7 6 3 2 1 0          5 6
//   MD       9 8 3 2                        7 6 5 4 1 0          7 8
//
// L columns written and read by the same group (2, 4, 6, 8, 10) and the
// source prior (11) stay in VGPRs; the columns between groups (3, 5, 7, 9)
// live in LDS; R crosses a group boundary through an LDS transpose.  The
// hard decisions of the CSFG checks (eqs. (2)-(4)) and of the G-matrix stop
// are ballot words (bit = lane) per register; the transform by F^{(x)s} is
// word XORs along free register bits, and along the lane bits each lane
// reads its own output as a parity over the word (two ANDs and two
// popcounts, in every lane at once).  A stage's check reads only the
// selected block's registers, through a branch tree ending in one ballot.
// Stages 1 and 10 share mapping MA, so the stop compares u G with the
// channel-side decisions without any reshuffle.
#pragma once

#include <hip/hip_runtime.h>

#include "pbp_arith.h"
#include "pbp_internal.h"
#include "pbp_r10.h"

namespace pbp {
namespace r10 {
namespace {

constexpr float kInf = __builtin_inff();

using arith::clampm;
using arith::salpha;
using ArithF32 = arith::F32;
using ArithFixed = arith::Fixed;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lanes whose lane-index bit b is set / clear
__device__ constexpr uint64_t kLaneSet[6] = {
    0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
    0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};

// a uniform bound the compiler may not fold back into per-lane operands
// (lane >= bound - c would otherwise become lane + c >= bound, with one
// live register per c)
__device__ __forceinline__ int opaque_s(int v)
{
    asm volatile("" : "+s"(v));
    return v;
}

__device__ __forceinline__ uint64_t ballot(bool p)
{
    return __ballot(p);
}

// The frozen ballot words are read-only for the whole launch: reading them
// through the constant address space lets them come in by scalar loads.
typedef const uint64_t __attribute__((address_space(4))) *const_u64_ptr;

struct Params {
    const float *llr;
    int64_t B;
    int *counter;
    const uint64_t *fzw;   // [4][16] frozen ballot words per mapping
    const int32_t *info_pos;
    int32_t K;
    int32_t max_iter, freezing, freeze_input, freeze_walk;
    float alpha;
    uint8_t *info_out;
    int32_t *iters_out;
    int64_t *pe_out;
    float *soft_out;
    // fixed-point messages only
    float qmax;            // Q = 2^(b-1) - 1
    int32_t frac;          // fraction bits of the channel quantizer
    int8_t *soft_q;        // B x N or null: sat(R + L) at column M+1
};

// LDS per wavefront
struct Smem {
    float lb[4][N];      // L at columns 3, 5, 7, 9
    float tb[N / 2];     // transpose buffer (half a frame at a time)
    uint8_t dec[N];      // decided source bits of frozen rows
};

// Stage j: its mapping and the register bit of its butterfly.
__host__ __device__ constexpr int smap(int j)
{
    return (j <= 2 || j >= 9) ? MA : (j <= 4 ? MB : (j <= 6 ? MC : MD));
}
__host__ __device__ constexpr int sqb(int j)
{
    return j == 1 ? 3 : j == 2 ? 2 : ((j & 1) ? 1 : 0);
}
// boundary LDS column index of L at column c (3, 5, 7, 9), else -1
__host__ __device__ constexpr int lbcol(int c)
{
    return c == 3 ? 0 : c == 5 ? 1 : c == 7 ? 2 : c == 9 ? 3 : -1;
}

// LDS word of row r in a boundary column or the transpose buffer.  With rows
// stored in order, one access of mapping MA puts lanes 4 rows apart (4 lanes
// per bank), and MC and MD are as strided.  XOR-ing row bits 5, 6 and 7 into
// the low five bits sends the lanes of every mapping to distinct banks (32
// lanes at a time, and all 64 over 64 banks).  The map is a bijection on
// rows 0..2^b - 1 for every b >= 8 and is linear over XOR.
__host__ __device__ constexpr int swz(int r)
{
    return r ^ (((r >> 5) & 1) ? 0x05 : 0) ^ (((r >> 6) & 1) ? 0x1a : 0) ^
           (((r >> 7) & 1) ? 0x20 : 0);
}

// address bits that the lane part of a mapping's rows can reach under swz
__host__ __device__ constexpr int swz_lane_bits(int mp)
{
    int m = 0;
    for (int lb = 0; lb < 6; lb++)
        m |= swz(1 << lrow(mp, lb));
    return m;
}

template <bool FRZ, bool ES, class Ar = ArithF32>
struct Decoder {
    const Params &P;
    Smem &S;
    const int lane;
    int lr[4];            // row bits contributed by this lane, per mapping
    int sl[4];            // swz(lr[mp]): the lane part of an LDS word
    float ch[Q];          // channel LLRs (MA) for the next stage 1, reloaded
                          // from device memory each iteration
    float L2[Q], L4[Q], L6[Q], L8[Q], L10[Q];
    float R[Q];
    float Lt[Q];          // boundary column read for the current stage
    uint64_t X[Q];        // channel-side hard decisions (MA ballot words)
    int p[M + 1];         // frozen CSFG prefix length per stage
    int l11lo, l11hi;     // rows that may be frozen at stage 10 and read
    int walking;
    int64_t pe;
    int pskip;            // PEs of this sweep below the frozen prefixes
    // frozen mask as per-lane bits: bit 16 (mp & 1) + q of fzb[mp >> 1] says
    // whether the row of register q in mapping mp is frozen on this lane
    // (two registers, so the checks need no scalar loads and their waits)
    uint32_t fzb[2];
    // lanes whose index contains this lane's index bits (bit l of
    // sup_hi:sup_lo): the lane part of the transform by F^{(x)s}
    uint32_t sup_lo, sup_hi;

    // frozen ballot word [mapping mp][register q] as stored by the host
    __device__ __forceinline__ uint64_t fz_word(int mp, int q) const
    {
        uint64_t base = reinterpret_cast<uint64_t>(P.fzw);
        asm volatile("" : "+s"(base));
        return reinterpret_cast<const_u64_ptr>(base)[mp * Q + q];
    }

    // this lane's frozen bit of register q in mapping mp
    __device__ __forceinline__ bool fzbit(int mp, int q) const
    {
        return (fzb[mp >> 1] >> ((mp & 1) * 16 + q)) & 1;
    }

    __device__ __forceinline__ Decoder(const Params &P_, Smem &S_, int lane_)
        : P(P_), S(S_), lane(lane_)
    {
#pragma unroll
        for (int mp = 0; mp < 4; mp++) {
            int r = 0;
#pragma unroll
            for (int lb = 0; lb < 6; lb++)
                if ((lane >> lb) & 1)
                    r |= 1 << lrow(mp, lb);
            lr[mp] = r;
            sl[mp] = swz(r);
        }
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint32_t b = 0;
#pragma unroll
            for (int k = 0; k < 2 * Q; k++)
                b |= (uint32_t)((fz_word(2 * h + k / Q, k % Q) >> lane) & 1) << k;
            fzb[h] = b;
        }
        uint64_t sup = ~0ull;
#pragma unroll
        for (int lb = 0; lb < 6; lb++)
            if ((lane >> lb) & 1)
                sup &= kLaneSet[lb];
        sup_lo = (uint32_t)sup;
        sup_hi = (uint32_t)(sup >> 32);
    }

    template <int MP>
    __device__ __forceinline__ int row(int q) const { return lr[MP] + rowq(MP, q); }

    // LDS word swz(row) of register q in mapping MP, within the first WMASK+1
    // words.  swz(row) = sl ^ swz(rowq); the part of swz(rowq) outside the
    // lane part's bits adds without carries, so it becomes an instruction
    // offset, and only the part inside (two register bits' worth) needs a XOR.
    template <int MP, int WMASK = N - 1>
    __device__ __forceinline__ int lds_word(int q) const
    {
        const int c = swz(rowq(MP, q));
        const int in = c & swz_lane_bits(MP);
        return (sl[MP] ^ in) + (c & ~swz_lane_bits(MP) & WMASK);
    }

    // largest row offset a lane contributes in mapping mp
    static constexpr int lanemax(int mp)
    {
        int r = 0;
        for (int lb = 0; lb < 6; lb++)
            r |= 1 << lrow(mp, lb);
        return r;
    }

    // L at column 11 (MA): +inf at frozen rows, 0 at information rows, and
    // (-1)^u inf at rows frozen at stage 10 (single-row CSFGs, whose kept
    // decision is u).  Only rows in [lo, hi) can be frozen at stage 10 and
    // still be read, so only those consult the kept decisions.
    __device__ __forceinline__ float l11(int q, int lo, int hi) const
    {
        const float big = Ar::big(P.qmax);
        float v = fzbit(MA, q) ? big : 0.0f;
        if (FRZ) {
            const int rq = rowq(MA, q);
            if (rq + 252 >= lo && rq < hi) {
                // row >= lo and row < hi, compared as the lane part against
                // uniform bounds (no per-register row value stays live)
                if (lr[MA] >= opaque_s(lo - rq) && lr[MA] < opaque_s(hi - rq))
                    v = S.dec[row<MA>(q)] ? -big : big;
            }
        }
        return v;
    }

    // register array holding L at column c in its group's mapping
    template <int C>
    __device__ __forceinline__ float *lreg()
    {
        if constexpr (C == 2) return L2;
        else if constexpr (C == 4) return L4;
        else if constexpr (C == 6) return L6;
        else if constexpr (C == 8) return L8;
        else if constexpr (C == 10) return L10;
        else if constexpr (C == 3 || C == 5 || C == 7 || C == 9) return Lt;
        else return nullptr;
    }

    // channel LLRs of a frame in mapping MA: register (qh, ql) of lane l is
    // row 256 qh + 4 l + ql, so each lane reads four 16-byte vectors (four
    // words each where the caller's buffer is not 16-byte aligned)
    __device__ __forceinline__ void load_channel(int64_t frame)
    {
        const float *src = P.llr + frame * N;
        if (__builtin_expect((reinterpret_cast<uintptr_t>(src) & 15) == 0, 1)) {
#pragma unroll
            for (int qh = 0; qh < 4; qh++) {
                const float4 v = *reinterpret_cast<const float4 *>(src + qh * 256 + lane * 4);
                ch[qh * 4 + 0] = Ar::channel(v.x, P.frac, P.qmax);
                ch[qh * 4 + 1] = Ar::channel(v.y, P.frac, P.qmax);
                ch[qh * 4 + 2] = Ar::channel(v.z, P.frac, P.qmax);
                ch[qh * 4 + 3] = Ar::channel(v.w, P.frac, P.qmax);
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; q++)
                ch[q] = Ar::channel(src[(q >> 2) * 256 + lane * 4 + (q & 3)], P.frac, P.qmax);
        }
    }

    __device__ __forceinline__ void load_frame(int64_t frame)
    {
        load_channel(frame);
#pragma unroll
        for (int q = 0; q < Q; q++)
            L2[q] = L4[q] = L6[q] = L8[q] = L10[q] = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; c++)
#pragma unroll
            for (int i = 0; i < N / 64; i++)
                S.lb[c][i * 64 + lane] = 0.0f;
#pragma unroll
        for (int i = 0; i < N / 256; i++)
            reinterpret_cast<uint32_t *>(S.dec)[i * 64 + lane] = 0u;
#pragma unroll
        for (int j = 0; j <= M; j++)
            p[j] = 0;
        pe = 0;
        wave_sync();
    }

    // R crosses from mapping A to mapping B, half a frame (row bit 9) at a
    // time through the transpose buffer.
    template <int A, int Bm>
    __device__ __forceinline__ void transpose_r()
    {
#pragma unroll
        for (int h = 0; h < 2; h++) {
#pragma unroll
            for (int q = h * 8; q < h * 8 + 8; q++)
                S.tb[lds_word<A, N / 2 - 1>(q)] = R[q];
            wave_sync();
#pragma unroll
            for (int q = h * 8; q < h * 8 + 8; q++)
                R[q] = S.tb[lds_word<Bm, N / 2 - 1>(q)];
            wave_sync();
        }
    }

    // One PE of eq. (1) on registers qa (row a) and qb = qa | BIT (row a + h).
    // Lin = L at column J+1; the outputs L at column J go to registers, to
    // LDS (boundary column) or into the channel-side decisions (J = 1).
    // KEPT: stage M may read rows frozen at stage M (their kept decisions)
    template <int J, int QA, bool KEPT, bool MASKED = false>
    __device__ __forceinline__ void pe_update(bool keep = true)
    {
        constexpr int MP = smap(J);
        constexpr int QB = QA | (1 << sqb(J));
        float La, Lb;
        if constexpr (J == M) {
            La = KEPT ? l11(QA, l11lo, l11hi) : l11(QA, 0, 0);
            Lb = KEPT ? l11(QB, l11lo, l11hi) : l11(QB, 0, 0);
        } else {
            float *Lin = lreg<J + 1>();
            La = Lin[QA];
            Lb = Lin[QB];
        }
        const float Ra = (J == 1) ? ch[QA] : R[QA];
        const float Rb = (J == 1) ? ch[QB] : R[QB];
        float la, lbv, ra, rb;
        Ar::pe(La, Lb, Ra, Rb, P.alpha, P.qmax, la, lbv, ra, rb);
        R[QA] = ra;
        R[QB] = rb;
        if constexpr (J == 1) {
            if constexpr (ES) {
                X[QA] = ballot(Ra + la < 0.0f);
                X[QB] = ballot(Rb + lbv < 0.0f);
            }
        } else if constexpr (lbcol(J) >= 0) {
            if (!MASKED || keep) {
                S.lb[lbcol(J)][lds_word<MP>(QA)] = la;
                S.lb[lbcol(J)][lds_word<MP>(QB)] = lbv;
            }
        } else {
            float *Lout = lreg<J>();
            Lout[QA] = (!MASKED || keep) ? la : Lout[QA];
            Lout[QB] = (!MASKED || keep) ? lbv : Lout[QB];
        }
        // one PE at a time: dependent VALU operations issue back to back, so
        // interleaving PEs buys nothing but register pressure
        __builtin_amdgcn_sched_barrier(0);
    }

    // Register slots of a stage: PEs are grouped by the top two row bits of
    // their upper row (register bits 3 and 2), except at stage 2, where the
    // butterfly itself is on row bit 8 and the groups are the two halves.
    template <int J>
    static constexpr int slot_of(int qa) { return J == 2 ? (qa >> 3) * 2 : (qa >> 2); }

    // PEs of stage J in register slot SLOT, all lanes active
    template <int J, int QA, int SLOT, bool KEPT>
    __device__ __forceinline__ void pe_slot()
    {
        if constexpr (QA < Q) {
            if constexpr (!((QA >> sqb(J)) & 1) && slot_of<J>(QA) == SLOT)
                pe_update<J, QA, KEPT>();
            pe_slot<J, QA + 1, SLOT, KEPT>();
        }
    }

    // the same, each PE masked to the lanes whose row is >= f
    template <int J, int QA, int SLOT, bool KEPT>
    __device__ __forceinline__ void pe_slot_masked(int f)
    {
        if constexpr (QA < Q) {
            if constexpr (!((QA >> sqb(J)) & 1) && slot_of<J>(QA) == SLOT) {
                constexpr int MP = smap(J);
                // R of rows below f is not read again in this sweep, so
                // only the L outputs keep their old values there
                pe_update<J, QA, KEPT, true>(lr[MP] >= opaque_s(f - rowq(MP, QA)));
            }
            pe_slot_masked<J, QA + 1, SLOT, KEPT>(f);
        }
    }

    template <int J, int SLOT, bool KEPT>
    __device__ __forceinline__ void run_slot() { pe_slot<J, 0, SLOT, KEPT>(); }

    // Rows of slot s are [256 s, 256 s + 256).  Frozen prefix f: a slot
    // entirely >= f runs unmasked, the slot holding f runs masked per lane,
    // slots entirely below f are skipped.
    template <int J, int SLOT, bool KEPT>
    __device__ __forceinline__ void slot_step(int f)
    {
        // the common case (nothing of the slot frozen) falls through
        if (__builtin_expect(f <= SLOT * 256, 1))
            run_slot<J, SLOT, KEPT>();
        else if (f < SLOT * 256 + 256)
            pe_slot_masked<J, 0, SLOT, KEPT>(f);
    }

    // With no frozen prefix at the stage (every stage while nothing is
    // frozen, and stage 1 always) all slots run unmasked behind one branch.
    template <int J, bool KEPT>
    __device__ __forceinline__ void stage_pes(int f)
    {
        if (J == 1 || !FRZ || f == 0) {
            run_slot<J, 0, KEPT>(); run_slot<J, 1, KEPT>();
            run_slot<J, 2, KEPT>(); run_slot<J, 3, KEPT>();
        } else {
            slot_step<J, 0, KEPT>(f);
            slot_step<J, 1, KEPT>(f);
            slot_step<J, 2, KEPT>(f);
            slot_step<J, 3, KEPT>(f);
        }
    }

    // stage J runs (N - f) / 2 PEs: N / 2 less the prefix's f / 2, which is
    // summed per iteration in 32 bits (at most M N / 2 a sweep).  Stage M
    // consults the kept decisions only while some row frozen at stage M
    // lies at or above its own frozen prefix (rarely, and for a row or two).
    template <int J>
    __device__ __forceinline__ void stage(int f)
    {
        if (FRZ && J == M && l11hi > l11lo)
            stage_pes<J, true>(f);
        else
            stage_pes<J, false>(f);
        if constexpr (FRZ && J > 1)
            pskip += p[J - 1] << (M - J);
    }

    // the boundary column L at column J+1 (J even, J < 10) into Lt
    template <int J>
    __device__ __forceinline__ void load_lt()
    {
        constexpr int MP = smap(J);
#pragma unroll
        for (int q = 0; q < Q; q++)
            Lt[q] = S.lb[lbcol(J + 1)][lds_word<MP>(q)];
    }

    // ---- CSFG freezing walk at stage J (Section III, eqs. (2)-(4)) ----
    //
    // The block of CSFG k at stage J is the set of rows whose top J bits are
    // k.  In the stage's mapping its rows are the registers whose fixed
    // register bits (row bits >= 10 - J) match k, on the lanes whose fixed
    // lane bits match k.  The register part is dispatched at compile time,
    // so only the block's registers are touched.

    template <int J>
    static constexpr int fixed_qmask()
    {
        int fm = 0;
        for (int qb = 0; qb < 4; qb++)
            if (qrow(smap(J), qb) >= M - J)
                fm |= 1 << qb;
        return fm;
    }

    // value of register q's input to eq. (2)
    template <int J>
    __device__ __forceinline__ float check_input(int q)
    {
        if constexpr (J == M) {
            return P.freeze_input ? R[q] + l11(q, 0, 0) : R[q];
        } else {
            const float *Ln = lreg<J + 1>();
            return P.freeze_input ? R[q] + Ln[q] : R[q];
        }
    }

    // The lane part of the transform by F^{(x)s}, read at this lane: output
    // bit i of x F^{(x)s} is the XOR of the inputs whose index contains i,
    // so along the lane-index bits it is the parity of the ballot word w over
    // the lanes whose index contains this lane's (the mask sup).  A block's
    // free lane bits are the low ones and w is zero outside the block, so the
    // same mask serves every stage.  Returns the count; bit 0 is the parity.
    __device__ __forceinline__ uint32_t lane_fx(uint64_t w) const
    {
        return (uint32_t)__builtin_popcount((uint32_t)w & sup_lo) +
               (uint32_t)__builtin_popcount((uint32_t)(w >> 32) & sup_hi);
    }

    // lanes where the transformed word w is 1 at a frozen row of register q
    // (uniform, run time) in mapping MP: eq. (4) fails on any of the block's
    __device__ __forceinline__ uint64_t frozen_hits(int mp, uint64_t w, int q) const
    {
        const uint32_t f = fzb[mp >> 1] >> ((mp & 1) * 16 + q);
        return ballot(((lane_fx(w) & f) & 1u) != 0u);
    }

    // candidates of a register branch tree: registers in [LO, HI) whose bits
    // under CM equal CV
    template <int CM, int CV, int LO, int HI>
    static constexpr bool has_cand()
    {
        for (int q = LO; q < HI; q++)
            if ((q & CM) == CV)
                return true;
        return false;
    }

    // eq. (2)'s decisions at register q of stage J as a ballot word; q is
    // uniform and known at run time only, and is one of the registers whose
    // bits under CM equal CV.  A branch tree over those candidates ends in
    // one ballot per leaf, so only the selected register is read.
    template <int J, int CM, int CV, int LO = 0, int HI = Q>
    __device__ __forceinline__ uint64_t input_word(int q)
    {
        if constexpr (HI - LO == 1) {
            return ballot(check_input<J>(LO) < 0.0f);
        } else {
            constexpr int MID = (LO + HI) / 2;
            if constexpr (!has_cand<CM, CV, LO, MID>())
                return input_word<J, CM, CV, MID, HI>(q);
            else if constexpr (!has_cand<CM, CV, MID, HI>())
                return input_word<J, CM, CV, LO, MID>(q);
            else if (q < MID)
                return input_word<J, CM, CV, LO, MID>(q);
            else
                return input_word<J, CM, CV, MID, HI>(q);
        }
    }

    // row bits contributed by register index q (uniform, run time)
    template <int MP>
    static __device__ __forceinline__ int rowq_rt(int q)
    {
        return ((q & 1) << qrow(MP, 0)) | (((q >> 1) & 1) << qrow(MP, 1)) |
               (((q >> 2) & 1) << qrow(MP, 2)) | (((q >> 3) & 1) << qrow(MP, 3));
    }

    // input words of the block's registers t | I other than t | FREE
    template <int J, int I>
    __device__ __forceinline__ void rest_words(int t, uint64_t lm, uint64_t *X0)
    {
        if constexpr (I < Q) {
            constexpr int FREE = ~fixed_qmask<J>() & (Q - 1);
            if constexpr ((I & FREE) == I && I != FREE)
                X0[I] = input_word<J, FREE, I>(t | I) & lm;
            rest_words<J, I + 1>(t, lm, X0);
        }
    }

    // The rest of a block's check once its register with every free register
    // bit set has passed (rare): the block's other registers t | i, eq. (3)
    // along the free register bits as word XORs, eq. (4) per word, and on
    // success the freeze.  wl is the passed word's input; lm the block's
    // lanes.  Returns true when frozen.
    template <int J>
    __device__ __forceinline__ bool check_rest(int t, uint64_t lm, uint64_t wl)
    {
        constexpr int MP = smap(J);
        constexpr int FREE = ~fixed_qmask<J>() & (Q - 1);
        uint64_t X0[Q], W[Q];
        X0[FREE] = wl;
        rest_words<J, 0>(t, lm, X0);
#pragma unroll
        for (int i = 0; i < Q; i++)
            if ((i & FREE) == i)
                W[i] = X0[i];
#pragma unroll
        for (int qb = 0; qb < 4; qb++)
            if ((FREE >> qb) & 1)
#pragma unroll
                for (int i = 0; i < Q; i++)
                    if ((i & FREE) == i && !((i >> qb) & 1))
                        W[i] ^= W[i | (1 << qb)];
        uint64_t bad = 0;
#pragma unroll
        for (int i = 0; i < Q; i++)
            if ((i & FREE) == i && i != FREE)
                bad |= frozen_hits(MP, W[i], t | i);
        if (bad & lm)
            return false;
        // freeze: keep uhat; when L at column J+1 lives in LDS, fix it to
        // (-1)^xhat inf there (register columns are fixed after the walk)
        if ((lm >> lane) & 1) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if ((i & FREE) == i) {
                    const int rq = rowq_rt<MP>(t | i);
                    S.dec[lr[MP] + rq] = (uint8_t)(lane_fx(W[i]) & 1u);
                    if constexpr (lbcol(J + 1) >= 0)
                        S.lb[lbcol(J + 1)][sl[MP] ^ swz(rq)] =
                            ((X0[i] >> lane) & 1) ? -Ar::big(P.qmax) : Ar::big(P.qmax);
                }
            }
        }
        wave_sync();
        return true;
    }

    // L at column J+1 := (-1)^xhat inf on rows [lo, hi) when that column is
    // held in registers (after the walk, so that the walk loop carries no
    // register state)
    template <int J>
    __device__ __forceinline__ void fix_range(int lo, int hi)
    {
        constexpr int MP = smap(J);
        if constexpr (lbcol(J + 1) < 0 && J < M) {
            float *Ln = lreg<J + 1>();
#pragma unroll
            for (int q = 0; q < Q; q++) {
                const int rq = rowq(MP, q);
                if (rq + lanemax(MP) >= lo && rq < hi) {
                    const float fixed = check_input<J>(q) < 0.0f ? -Ar::big(P.qmax) : Ar::big(P.qmax);
                    Ln[q] = (lr[MP] >= opaque_s(lo - rq) && lr[MP] < opaque_s(hi - rq))
                                ? fixed : Ln[q];
                }
            }
        }
    }

    // lane bits whose row bit is below the stage's block size
    template <int J>
    static constexpr int free_lanes()
    {
        int n = 0;
        for (int lb = 0; lb < 6; lb++)
            if (lrow(smap(J), lb) < M - J)
                n++;
        return n;
    }

    // the lane bits of fixed row bits are the top ones, with consecutive rows
    template <int J>
    static constexpr bool fixed_lanes_top()
    {
        const int nf = free_lanes<J>();
        for (int lb = 0; lb < 6; lb++) {
            if ((lb < nf) != (lrow(smap(J), lb) < M - J))
                return false;
            if (lb > nf && lrow(smap(J), lb) != lrow(smap(J), nf) + (lb - nf))
                return false;
        }
        return true;
    }

    // check CSFG k of stage J (and freeze it on success)
    template <int J>
    __device__ __forceinline__ bool check_k(int k)
    {
        constexpr int MP = smap(J);
        constexpr int SH = M - J;          // row bits below SH are free
        constexpr int FM = fixed_qmask<J>();
        constexpr int FREE = ~FM & (Q - 1);
        // lanes inside block k.  In every stage's mapping the lane bits of
        // the fixed row bits are the top NF.. 5 and carry consecutive row
        // bits, so the block's lanes are one run of 2^NF lanes.
        constexpr int NF = free_lanes<J>();
        static_assert(fixed_lanes_top<J>(), "block lanes must form one run");
        uint64_t lm = ~0ull;
        if constexpr (NF < 6) {
            const int v = (k >> (lrow(MP, NF) - SH)) & ((1 << (6 - NF)) - 1);
            lm = (NF == 0 ? 1ull : ((1ull << (1 << NF)) - 1)) << (v << NF);
        }
        // fixed register bits of block k
        int t = 0;
#pragma unroll
        for (int qb = 0; qb < 4; qb++)
            if ((FM >> qb) & 1)
                t |= ((k >> (qrow(MP, qb) - SH)) & 1) << qb;
        // Along the register bits the output word of the block's register
        // with every free bit set is its own input, so eqs. (3)-(4) are tested
        // on it first; most checks fail there.
        const uint64_t wl = input_word<J, FREE, FREE>(t | FREE) & lm;
        if (__builtin_expect((frozen_hits(MP, wl, t | FREE) & lm) != 0, 1))
            return false;
        return check_rest<J>(t, lm, wl);
    }

    template <int J>
    __device__ __forceinline__ void freeze_walk()
    {
        constexpr int SH = M - J;
        if (__builtin_expect(!P.freezing, 0))
            return;
        int pj = max(p[J], 2 * p[J - 1]);
        const int k0 = pj;
        // At most one freeze per stage unless the walk is greedy; the common
        // path is loop-free so that no check input is hoisted out of a loop.
        if (pj < (1 << J) && (P.freeze_walk != 0 || walking)) {
            if (check_k<J>(pj)) {
                pj++;
                if (P.freeze_walk == 0)
                    walking = 0;
                if (P.freeze_walk == 2)
                    while (pj < (1 << J) && check_k<J>(pj))
                        pj++;
            }
        }
        if (pj > k0)
            fix_range<J>(k0 << SH, pj << SH);
        p[J] = pj;
    }

    template <int J>
    __device__ __forceinline__ void step()
    {
        int f = 0;
        if constexpr (FRZ)
            f = p[J - 1] << (M - J + 1);
        if constexpr (J == M) {
            l11lo = f;                       // rows below f are not read
            l11hi = FRZ ? p[M] : 0;          // rows frozen at stage 10 so far
        }
        // keep each stage's LDS reads inside the stage (hoisting them ahead
        // only lengthens register lifetimes)
        asm volatile("" ::: "memory");
        if constexpr ((J & 1) == 0 && J < M)
            load_lt<J>();
        stage<J>(f);
        if constexpr (FRZ)
            freeze_walk<J>();
    }

    // source-word decisions of register q (MA) as a ballot word: the hard
    // decision of R at column 11, 0 at frozen rows, and the kept CSFG
    // decisions on rows below the frozen prefix fm
    __device__ __forceinline__ uint64_t u_word(int q, int fm)
    {
        uint64_t u = ballot(R[q] < 0.0f && !fzbit(MA, q));
        if (FRZ) {
            const int base = rowq(MA, q);         // lane l holds row base + 4l
            if (fm > base) {
                const uint64_t d = ballot(S.dec[row<MA>(q)] != 0);
                if (fm > base + 252) {
                    u = d;
                } else {
                    const int T = (fm - base + 3) >> 2;   // lanes below fm
                    const uint64_t pm = (1ull << T) - 1;
                    u = (u & ~pm) | (d & pm);
                }
            }
        }
        return u;
    }

    // decisions at column 11 and the stop test; returns true to stop
    __device__ __forceinline__ bool decide()
    {
        const int fm = FRZ ? p[M] : 0;
        if (FRZ && fm == N)
            return true;
        if constexpr (!ES)
            return false;
        // G-matrix test: u F^{(x)10} == xhat.  Output word 15 (all register
        // bits set) depends on input word 15 alone: test it first.
        if (__builtin_expect(ballot(lane_fx(u_word(Q - 1, fm)) & 1u) != X[Q - 1], 1))
            return false;
        uint64_t U[Q];
#pragma unroll
        for (int q = 0; q < Q; q++)
            U[q] = u_word(q, fm);
#pragma unroll
        for (int qb = 0; qb < 4; qb++)
#pragma unroll
            for (int q = 0; q < Q; q++)
                if (!((q >> qb) & 1))
                    U[q] ^= U[q | (1 << qb)];
        uint64_t diff = 0;
#pragma unroll
        for (int q = 0; q < Q - 1; q++)
            diff |= ballot(lane_fx(U[q]) & 1u) ^ X[q];
        return diff == 0;
    }

    __device__ __forceinline__ void write_outputs(int64_t frame, int iters)
    {
        const int fm = FRZ ? p[M] : 0;
        // source-word decisions of the non-frozen rows into the LDS table
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int r = row<MA>(q);
            if (r >= fm)
                S.dec[r] = (uint8_t)(R[q] < 0.0f);
        }
        wave_sync();
        uint8_t *out = P.info_out + frame * P.K;
        for (int k = lane; k < P.K; k += 64)
            out[k] = S.dec[P.info_pos[k]];
        if constexpr (Ar::kFixed) {
            if (P.soft_q) {
                // sat(R + L) at column M+1 (+-Q at frozen CSFG rows), as bytes
                const float q = P.qmax;
                int8_t *so = P.soft_q + frame * N;
#pragma unroll
                for (int qh = 0; qh < 4; qh++) {
#pragma unroll
                    for (int ql = 0; ql < 4; ql++) {
                        const int qq = qh * 4 + ql;
                        const int r = row<MA>(qq);
                        const float v = r < fm ? (S.dec[r] ? -q : q)
                                               : Ar::sat(R[qq] + l11(qq, 0, 0), q);
                        so[qh * 256 + lane * 4 + ql] = (int8_t)(int)v;
                    }
                }
            }
        } else if (P.soft_out) {
            float *so = P.soft_out + frame * N;
#pragma unroll
            for (int qh = 0; qh < 4; qh++) {
                float v[4];
#pragma unroll
                for (int ql = 0; ql < 4; ql++) {
                    const int q = qh * 4 + ql;
                    const int r = row<MA>(q);
                    v[ql] = r < fm ? (S.dec[r] ? -kInf : kInf) : R[q] + l11(q, 0, 0);
                }
                float *dst = so + qh * 256 + lane * 4;
                if ((reinterpret_cast<uintptr_t>(so) & 15) == 0) {
                    *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int ql = 0; ql < 4; ql++)
                        dst[ql] = v[ql];
                }
            }
        }
        if (lane == 0) {
            P.iters_out[frame] = iters;
            if (P.pe_out)
                P.pe_out[frame] = pe;
        }
        wave_sync();
    }

    __device__ __forceinline__ void decode(int64_t frame)
    {
        load_frame(frame);
        int t = 1;
        for (; t <= P.max_iter; t++) {
            walking = 1;
            pskip = 0;
            step<1>();
            step<2>();
            transpose_r<MA, MB>();
            step<3>();
            step<4>();
            transpose_r<MB, MC>();
            step<5>();
            step<6>();
            transpose_r<MC, MD>();
            step<7>();
            step<8>();
            transpose_r<MD, MA>();
            load_channel(frame);        // for the next iteration's stage 1
            step<9>();
            step<10>();
            pe += M * N / 2 - pskip;
            if (decide())
                break;
        }
        if (t > P.max_iter)
            t = P.max_iter;
        write_outputs(frame, t);
    }
};

}  // namespace
}  // namespace r10
}  // namespace pbp
