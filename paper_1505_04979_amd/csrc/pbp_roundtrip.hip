// Round-trip BP schedule for codes up to N = 2048.
//
// The other common reading of Section II-A's schedule: each iteration first
// computes every L output of eq. (1), stage m down to stage 1 (from the L
// just computed at column j+1 and the R of the previous pass at column j),
// then every R output, stage 1 up to stage m (from the R just computed at
// column j and this pass's L at column j+1).  No freezing; the G-matrix stop
// and the outputs are those of the single sweep.  Each pass activates every
// PE once (m N PE activations per iteration).
//
// One workgroup decodes one frame at a time (grid-stride over frames), one
// thread per PE of a stage.  A thread's PE at stage j has the same rows in
// both passes, so the L pass keeps the two L inputs it read at stage j for
// the R pass, and the R pass keeps the two R inputs it read at stage j for
// the next L pass: 4 m values per thread in registers.  LDS holds only a
// ping-pong pair of columns per direction, the decisions and the encoder's
// bits (about 19 KB at N = 1024, 37 KB at N = 2048).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbp.h"
#include "pbp_internal.h"

namespace {

constexpr float kInf = __builtin_inff();

// longest code: one thread per PE of a stage (N / 2 <= 1024 threads)
constexpr int kMaxRoundTripLog = 11;

// alpha g(x, y) of eq. (1): y with the sign of x folded in, clamped to
// [-|x|, |x|] (a selection, exact), then scaled once
__device__ __forceinline__ float gsc(float x, float y, float alpha)
{
    const float t = __uint_as_float(__float_as_uint(y) ^
                                    (__float_as_uint(x) & 0x80000000u));
    return alpha * __builtin_amdgcn_fmed3f(-fabsf(x), t, fabsf(x));
}

__device__ __forceinline__ void sync_group_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void sync_wave_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// LDS ordering between consecutive stages with offsets h1 and h2: with one
// thread per PE, wavefront w's PEs at a stage with offset <= 64 lie in rows
// [128 w, 128 w + 128), so when both offsets are that small (or the group is
// one wavefront) the words the second stage touches were last touched by the
// same wavefront
template <int NW>
__device__ __forceinline__ void sync_stages(int h1, int h2)
{
    if (NW == 1 || (h1 <= 64 && h2 <= 64))
        sync_wave_lds();
    else
        sync_group_lds();
}

struct RtParams {
    const float *llr;
    int64_t B;
    const uint64_t *frozen;   // frozen bit words, row i is bit i & 63 of i >> 6
    const int32_t *info_pos;
    int32_t K;
    int32_t max_iter, early_stop;
    float alpha;
    uint8_t *info_out;
    int32_t *iters_out;
    int64_t *pe_out;
    float *soft_out;
    int *counter;             // [frame, exit] counters, zero between
                              // launches; null: frames by grid stride
};

template <int M>
struct RtShape {
    static constexpr int N = 1 << M;
    static constexpr int H = N / 2;                 // PEs per stage
    static constexpr int NT = H < 64 ? 64 : H;      // threads per workgroup
    static constexpr int NW = NT / 64;
};

template <int M>
struct RtSmem {
    float L[2][RtShape<M>::N];    // L at columns j (parity of j), 2 <= j <= m
    float R[2][RtShape<M>::N];    // R at columns j+1 (parity of j+1)
    uint8_t xh[RtShape<M>::N];    // hard decisions of R + L at column 1
    uint8_t u[RtShape<M>::N];     // source-word decisions, then u F^{(x)m}
};

template <int M>
__global__ __launch_bounds__(RtShape<M>::NT, 8) void bp_round_trip_kernel(RtParams P)
{
    using S = RtShape<M>;
    constexpr int N = S::N, H = S::H, NW = S::NW;
    __shared__ RtSmem<M> sm;
    const int tid = (int)threadIdx.x;
    const bool act = tid < H;
    const float alpha = P.alpha;

    auto frozen_at = [&](int i) { return (P.frozen[i >> 6] >> (i & 63)) & 1; };
    // the frozen bits of this thread's rows at stage m (offset 1: rows 2 t
    // and 2 t + 1), read once for the launch
    const int fz_m = act ? (int)(frozen_at(2 * tid) | (frozen_at(2 * tid + 1) << 1)) : 0;

    // Frames come from the stream workspace's counter, so that groups whose
    // frames stop early take more of them; the counter numbers frames in 32
    // bits, so batches beyond 2^30 frames are split by grid stride instead.
    __shared__ int64_t next;
    auto take = [&](int64_t prev) -> int64_t {
        if (!P.counter)
            return prev < 0 ? (int64_t)blockIdx.x : prev + gridDim.x;
        if (tid == 0)
            next = atomicAdd(P.counter, 1);
        __syncthreads();
        const int64_t f = next;
        // every thread has read it before thread 0 takes the next one
        __syncthreads();
        return f;
    };
    for (int64_t f = take(-1); f < P.B; f = take(f)) {
        // R inputs of each stage's PE (R at column j, rows a and b), as the
        // R pass last read them: the channel at column 1, 0 elsewhere
        float kRa[M + 1], kRb[M + 1];
        // L inputs of each stage's PE (L at column j+1), from the L pass
        float kLa[M + 1], kLb[M + 1];
#pragma unroll
        for (int j = 1; j <= M; j++)
            kRa[j] = kRb[j] = kLa[j] = kLb[j] = 0.0f;
        if (act) {
            kRa[1] = P.llr[f * N + tid];
            kRb[1] = P.llr[f * N + tid + H];
        }
        int t = 1;
        for (; t <= P.max_iter; t++) {
            // rows of this thread's PE at stage j, from a copy of the thread
            // index made opaque per iteration (the rows of all stages would
            // otherwise be kept in registers across iterations)
            int tt = tid;
            asm volatile("" : "+v"(tt));
            auto row_a = [&](int j) {
                const int sh = M - j;
                return ((tt >> sh) << (sh + 1)) | (tt & ((1 << sh) - 1));
            };
            // ---- L pass: stages m .. 1 ----
#pragma unroll
            for (int j = M; j >= 1; j--) {
                const int h = 1 << (M - j);
                if (act) {
                    const int a = row_a(j), b = a + h;
                    float La, Lb;
                    if (j == M) {
                        La = (fz_m & 1) ? kInf : 0.0f;
                        Lb = (fz_m & 2) ? kInf : 0.0f;
                    } else {
                        La = sm.L[(j + 1) & 1][a];
                        Lb = sm.L[(j + 1) & 1][b];
                    }
                    kLa[j] = La;
                    kLb[j] = Lb;
                    const float Ra = kRa[j], Rb = kRb[j];
                    const float lb = Lb + gsc(La, Ra, alpha);
                    const float la = gsc(La, Lb + Rb, alpha);
                    if (j >= 2) {
                        sm.L[j & 1][a] = la;
                        sm.L[j & 1][b] = lb;
                    } else {
                        sm.xh[a] = (uint8_t)(Ra + la < 0.0f);
                        sm.xh[b] = (uint8_t)(Rb + lb < 0.0f);
                    }
                }
                if (j > 1)
                    sync_stages<NW>(h, h << 1);
            }
            // ---- R pass: stages 1 .. m ----
#pragma unroll
            for (int j = 1; j <= M; j++) {
                const int h = 1 << (M - j);
                if (act) {
                    const int a = row_a(j), b = a + h;
                    float Ra, Rb;
                    if (j == 1) {
                        Ra = kRa[1];
                        Rb = kRb[1];
                    } else {
                        Ra = sm.R[j & 1][a];
                        Rb = sm.R[j & 1][b];
                        kRa[j] = Ra;
                        kRb[j] = Rb;
                    }
                    const float La = kLa[j], Lb = kLb[j];
                    const float ra = gsc(Ra, Lb + Rb, alpha);
                    const float rb = Rb + gsc(La, Ra, alpha);
                    sm.R[(j + 1) & 1][a] = ra;
                    sm.R[(j + 1) & 1][b] = rb;
                    if (j == M) {
                        // h = 1: rows a, a + 1; decisions at column m+1
                        sm.u[a] = (fz_m & 1) ? 0 : (uint8_t)(ra < 0.0f);
                        sm.u[b] = (fz_m & 2) ? 0 : (uint8_t)(rb < 0.0f);
                    }
                }
                if (j < M)
                    sync_stages<NW>(h, h >> 1);
            }
            if (!P.early_stop) {
                sync_group_lds();
                continue;
            }
            // ---- G-matrix stop: u F^{(x)m} against xh, in place over u,
            // stage m (offset 1) first; any order of the stages gives the
            // same product ----
#pragma unroll
            for (int j = M; j >= 1; j--) {
                const int h = 1 << (M - j);
                // after the R pass's last stage (offset 1, the same rows) or
                // the previous product stage (offset h / 2)
                sync_stages<NW>(j == M ? 1 : h >> 1, h);
                if (act) {
                    const int a = row_a(j);
                    sm.u[a] ^= sm.u[a + h];
                }
            }
            sync_group_lds();
            int bad = 0;
            if (act) {
                const int a = row_a(1), b = a + H;
                bad = (sm.u[a] != sm.xh[a]) | (sm.u[b] != sm.xh[b]);
            }
            const bool stop = !__syncthreads_or(bad);
            // the decisions overwritten by the product are needed at exit
            if (stop)
                break;
        }
        if (t > P.max_iter)
            t = P.max_iter;
        // decisions at column m+1 (the stop test overwrote u in place)
        sync_group_lds();
        const float *Rfin = sm.R[(M + 1) & 1];
        for (int i = tid; i < N; i += S::NT)
            sm.u[i] = frozen_at(i) ? 0 : (uint8_t)(Rfin[i] < 0.0f);
        sync_group_lds();
        uint8_t *out = P.info_out + f * P.K;
        for (int k = tid; k < P.K; k += S::NT)
            out[k] = sm.u[P.info_pos[k]];
        if (P.soft_out)
            for (int i = tid; i < N; i += S::NT)
                P.soft_out[f * N + i] = Rfin[i] + (frozen_at(i) ? kInf : 0.0f);
        if (tid == 0) {
            P.iters_out[f] = t;
            if (P.pe_out)
                P.pe_out[f] = (int64_t)t * M * N;
        }
        __syncthreads();
    }
    // every group has taken its last frame number before it counts itself
    // out; the last one out rewinds both counters for the next launch
    if (P.counter && tid == 0 &&
        atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(P.counter, 0);
        atomicExch(P.counter + 1, 0);
    }
}

template <int M>
hipError_t launch_rt(const pbp_code *c, const RtParams &P, hipStream_t st)
{
    using S = RtShape<M>;
    // at most 64 VGPRs: eight wavefronts per SIMD, 32 per compute unit
    const int per_cu = 32 / S::NW;
    int64_t grid = (int64_t)(c->cus > 0 ? c->cus : 256) * per_cu;
    if (grid > P.B)
        grid = P.B;
    hipLaunchKernelGGL(bp_round_trip_kernel<M>, dim3((unsigned)grid),
                       dim3(S::NT), 0, st, P);
    return hipGetLastError();
}

}  // namespace

extern "C" int32_t pbp_decode_round_trip(const pbp_code *code, const float *llr,
                                         int64_t B, const pbp_decode_opts *opts,
                                         uint8_t *info_out, int32_t *iters_out,
                                         int64_t *pe_out, float *soft_out,
                                         void *stream)
{
    if (!code || !opts || B < 0)
        return PBP_EINVAL;
    if (opts->max_iter < 1 || (opts->early_stop != 0 && opts->early_stop != 1) ||
        (opts->freezing != 0 && opts->freezing != 1) ||
        (opts->freeze_input != 0 && opts->freeze_input != 1) ||
        opts->freeze_walk < 0 || opts->freeze_walk > 2 ||
        !(opts->alpha > 0.0f) || !(opts->alpha < kInf))
        return PBP_EINVAL;
    if (opts->freezing || code->m > kMaxRoundTripLog)
        return PBP_EUNSUPPORTED;
    if (B == 0)
        return PBP_OK;
    if (!llr || !iters_out || (!info_out && code->K > 0))
        return PBP_EINVAL;
    RtParams P{};
    P.llr = llr;
    P.B = B;
    P.frozen = code->d_frozen_words;
    P.info_pos = code->d_info_pos;
    P.K = code->K;
    P.max_iter = opts->max_iter;
    P.early_stop = opts->early_stop;
    P.alpha = opts->alpha;
    P.info_out = info_out;
    P.iters_out = iters_out;
    P.pe_out = pe_out;
    P.soft_out = soft_out;
    if (B <= (int64_t(1) << 30)) {
        pbp::Workspace ws;
        const int32_t wst = pbp::stream_workspace(code, (hipStream_t)stream, &ws);
        if (wst != PBP_OK)
            return wst;
        P.counter = ws.counter;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    switch (code->m) {
    case 1: e = launch_rt<1>(code, P, st); break;
    case 2: e = launch_rt<2>(code, P, st); break;
    case 3: e = launch_rt<3>(code, P, st); break;
    case 4: e = launch_rt<4>(code, P, st); break;
    case 5: e = launch_rt<5>(code, P, st); break;
    case 6: e = launch_rt<6>(code, P, st); break;
    case 7: e = launch_rt<7>(code, P, st); break;
    case 8: e = launch_rt<8>(code, P, st); break;
    case 9: e = launch_rt<9>(code, P, st); break;
    case 10: e = launch_rt<10>(code, P, st); break;
    case 11: e = launch_rt<11>(code, P, st); break;
    default: return PBP_EUNSUPPORTED;
    }
    return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
}
