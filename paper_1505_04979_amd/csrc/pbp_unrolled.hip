// Unrolled BP with trainable scales, and its adjoint.
//
// T single left-to-right sweeps of eq. (1) with no early stop and no
// freezing; the scale of stage j in iteration t is split by direction:
//   L^t_{a,j}   = aL g(L_a, L_b + R_b)     L^t_{b,j}   = L_b + aL g(L_a, R_a)
//   R^t_{a,j+1} = aR g(R_a, L_b + R_b)     R^t_{b,j+1} = R_b + aR g(L_a, R_a)
// with g(x, y) = sign(x) sign(y) min(|x|, |y|) and L = L^{t-1} at column j+1
// (Section II-A, eq. (1); with every scale equal to alpha this is plain
// T-iteration BP).  The output is R^T at column m+1.
//
// One workgroup owns one frame at a time (grid-stride over frames), one
// thread per PE of a stage.  The forward keeps the message columns in LDS
// and writes the L state at the start of every iteration (columns 2..m) to a
// caller buffer.  The backward recomputes each iteration's R sweep from
// that checkpoint, then runs the stages in reverse; the adjoint of L takes
// the place of the checkpoint it was computed from.  Scale gradients are
// reduced per frame in a fixed order, then over frames in FP64, so results
// do not depend on scheduling.
//
// Derivatives: d g(x,y)/dx = sign(y) when |x| <= |y| (ties go to x), else
// 0; d g(x,y)/dy = sign(x) when |x| > |y|, else 0; d(a g)/da = g.  An
// infinite message (the frozen prior and what it produces) is a constant: it
// takes no adjoint and adds nothing to the scale gradients.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pbp.h"
#include "pbp_internal.h"

namespace {

constexpr float kInf = __builtin_inff();

// g(x, y) exactly: y with the sign of x folded in, clamped to [-|x|, |x|]
__device__ __forceinline__ float g0(float x, float y)
{
    const float t = __uint_as_float(__float_as_uint(y) ^
                                    (__float_as_uint(x) & 0x80000000u));
    return __builtin_amdgcn_fmed3f(-fabsf(x), t, fabsf(x));
}

__device__ __forceinline__ bool finite(float v) { return fabsf(v) < kInf; }

// +-1 with the sign of v, 0 for +-0
__device__ __forceinline__ float sgn(float v)
{
    return v == 0.0f ? 0.0f : __builtin_copysignf(1.0f, v);
}

// adjoint d of g(x, y) routed to x or y; an infinite operand takes nothing
// (selects, not branches, so that both accumulators stay in registers)
__device__ __forceinline__ void g0_back(float x, float y, float d, float &dx,
                                        float &dy)
{
    const bool to_x = fabsf(x) <= fabsf(y);
    const float cx = to_x && finite(x) ? d * sgn(y) : 0.0f;
    const float cy = !to_x && finite(y) ? d * sgn(x) : 0.0f;
    dx += cx;
    dy += cy;
}

// The scales are read-only for the whole launch: reading them through the
// constant address space makes them scalar loads, which do not wait behind
// the vector loads in flight.
typedef const float __attribute__((address_space(4))) *const_f32_ptr;

__device__ __forceinline__ float scale_at(const float *alpha, int64_t i)
{
    return reinterpret_cast<const_f32_ptr>(reinterpret_cast<uintptr_t>(alpha))[i];
}

__device__ __forceinline__ bool frozen_at(const uint64_t *fw, int i)
{
    return (fw[i >> 6] >> (i & 63)) & 1;
}

template <int M>
struct Shape {
    static constexpr int N = 1 << M;
    static constexpr int H = N / 2;                 // PEs per stage
    static constexpr int NT = H < 64 ? 64 : H;      // threads per workgroup
    static constexpr int NW = NT / 64;              // wavefronts
    static constexpr int YR = (N + NT - 1) / NT;    // LLRs per thread
};

struct FwdParams {
    const float *llr;
    int64_t B;
    int T;
    const float *alpha;       // T x m x 2
    const uint64_t *frozen;   // frozen bit words
    float *out;               // B x N
    float *ckpt;              // T x B x (m-1) x N, or null
};

struct BwdParams {
    const float *llr;
    int64_t B;
    int T;
    const float *alpha;
    const uint64_t *frozen;
    const float *ckpt;        // L checkpoints, read only
    const float *dout;        // B x N
    float *dalpha_frame;      // B x T x m x 2
    float *dllr;              // B x N, or null
};

template <int M>
size_t fwd_lds_bytes()
{
    return sizeof(float) * (size_t)(M + 2) * Shape<M>::N;
}

// [adjoint of L, columns 2..m][R, two columns][adjoint of R, two columns]
// [partial scale sums]
template <int M>
size_t bwd_lds_bytes()
{
    using S = Shape<M>;
    return sizeof(float) * ((size_t)(M + 3) * S::N + (size_t)M * S::NW * 2);
}

// Barrier that orders LDS only (device-memory accesses of a stage are
// ordered by the full barrier that ends each iteration).
__device__ __forceinline__ void sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS ordering between two consecutive stages.  With one thread per PE, the
// PEs of wavefront w at a stage whose offset is at most 64 all lie in rows
// [128 w, 128 w + 128); when both stages have such offsets (or the group is
// one wavefront) every LDS word the second stage touches was last touched by
// the same wavefront, so ordering within the wavefront is enough.
__device__ __forceinline__ void sync_wave_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// v from the lane that DPP control CTRL names (a pattern inside each row of
// 16 lanes, so every lane has a source)
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v plus lane 15 of the previous row, in rows 1 and 3 (rows 0 and 2 keep v).
// The s_nop gives the two wait states a DPP read of a VGPR needs after a
// VALU write of it.
__device__ __forceinline__ float add_bcast15(float v)
{
    asm("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf"
        : "+v"(v));
    return v;
}

// v plus lane 31, in rows 2 and 3 (rows 0 and 1 keep v)
__device__ __forceinline__ float add_bcast31(float v)
{
    asm("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(v));
    return v;
}

// Sums of a and b over the wavefront, complete in lane 63.  Within each row
// of 16 lanes a butterfly by DPP (the lane i ^ 1, i ^ 2, then the mirrored
// quad of the 8-lane half and the mirrored half of the row) leaves the row's
// sum r in all its lanes; lane 15 of each row is then added into rows 1 and
// 3, and lane 31 into rows 2 and 3, so lane 63 holds (r3 + r2) + (r1 + r0).
// No LDS; the order is the same in every call.  The two sums are
// interleaved so that each covers the other's DPP wait.
__device__ __forceinline__ void wave_sum2(float &a, float &b)
{
    a += dpp_f<0xB1>(a);            // quad_perm [1, 0, 3, 2]
    b += dpp_f<0xB1>(b);
    a += dpp_f<0x4E>(a);            // quad_perm [2, 3, 0, 1]
    b += dpp_f<0x4E>(b);
    a += dpp_f<0x141>(a);           // row_half_mirror
    b += dpp_f<0x141>(b);
    a += dpp_f<0x140>(a);           // row_mirror
    b += dpp_f<0x140>(b);
    a = add_bcast15(a);
    b = add_bcast15(b);
    a = add_bcast31(a);
    b = add_bcast31(b);
}

template <int NW>
__device__ __forceinline__ void sync_stages(int h_first, int h_second)
{
    if (NW == 1 || (h_first <= 64 && h_second <= 64))
        sync_wave_lds();
    else
        sync_lds();
}

template <int M>
__global__ __launch_bounds__(Shape<M>::NT) void unrolled_forward_kernel(FwdParams P)
{
    using S = Shape<M>;
    constexpr int N = S::N, H = S::H, NT = S::NT;
    extern __shared__ __align__(16) float sm[];
    float *L = sm;               // column c (2..m+1) at (c-2)*N
    float *R = sm + M * N;       // two columns, ping-pong by stage parity
    const int tid = (int)threadIdx.x;

    for (int64_t f = blockIdx.x; f < P.B; f += gridDim.x) {
        // the frame's LLRs stay in registers for all T iterations
        float yv[S::YR];
#pragma unroll
        for (int k = 0; k < S::YR; k++) {
            const int i = tid + k * NT;
            yv[k] = i < N ? P.llr[f * N + i] : 0.0f;
        }
        for (int i = tid; i < N; i += NT) {
            for (int c = 0; c < M - 1; c++)
                L[c * N + i] = 0.0f;
            L[(M - 1) * N + i] = frozen_at(P.frozen, i) ? kInf : 0.0f;
        }
        __syncthreads();
        for (int t = 0; t < P.T; t++) {
            if (P.ckpt) {
                float *ck = P.ckpt + ((int64_t)t * P.B + f) * (M - 1) * N;
                for (int i = tid; i < (M - 1) * N; i += NT)
                    ck[i] = L[i];
            }
#pragma unroll
            for (int k = 0; k < S::YR; k++) {
                const int i = tid + k * NT;
                if (i < N)
                    R[i] = yv[k];
            }
            __syncthreads();
            for (int j = 1; j <= M; j++) {
                const float aL = scale_at(P.alpha, ((int64_t)t * M + (j - 1)) * 2);
                const float aR = scale_at(P.alpha, ((int64_t)t * M + (j - 1)) * 2 + 1);
                const int sh = M - j, h = 1 << sh;
                if (tid < H) {
                    const int a = ((tid >> sh) << (sh + 1)) | (tid & (h - 1));
                    const int b = a + h;
                    const float *Lc = L + (j - 1) * N;
                    const float *Ri = R + ((j - 1) & 1) * N;
                    float *Ro = R + (j & 1) * N;
                    const float La = Lc[a], Lb = Lc[b];
                    const float Ra = Ri[a], Rb = Ri[b];
                    const float s = Lb + Rb;
                    const float g1 = g0(La, Ra);
                    if (j >= 2) {
                        float *Lw = L + (j - 2) * N;
                        Lw[a] = aL * g0(La, s);
                        Lw[b] = Lb + aL * g1;
                    }
                    Ro[a] = aR * g0(Ra, s);
                    Ro[b] = Rb + aR * g1;
                }
                if (j < M)
                    sync_stages<S::NW>(h, h >> 1);
                else
                    __syncthreads();
            }
        }
        for (int i = tid; i < N; i += NT)
            P.out[f * N + i] = R[(M & 1) * N + i];
        __syncthreads();
    }
}


// Backward pass.  L^{t-1} is read once from the checkpoint of iteration t
// (device memory) and R^t is recomputed from it; each thread keeps the L
// and R inputs of its PE at every stage in registers for the adjoint stages
// (the same rows), so R needs only two LDS columns in turn.  The adjoint of
// L (columns 2..m) stays in LDS across iterations: stage j reads the
// adjoint of L^t at column j and then writes that of L^{t-1} at column j+1
// over the values stage j+1 read, so device memory sees only the
// checkpoints, the LLRs and the gradients.  LDS: m + 3 columns (53 KB at
// m = 10); at most 102 VGPRs (no spills) keep five wavefronts per SIMD, so
// two groups of eight wavefronts per compute unit, and the grid is sized to
// what is resident.
template <int M>
__global__ __launch_bounds__(Shape<M>::NT, 5) void unrolled_backward_kernel(BwdParams P)
{
    using S = Shape<M>;
    constexpr int N = S::N, H = S::H, NT = S::NT, NW = S::NW;
    extern __shared__ __align__(16) float sm[];
    float *dA = sm;                     // adjoint of L, column c (2..m) at
                                        // (c-2)*N
    float *Rc = dA + (M - 1) * N;       // R^t, two columns by parity
    float *dR = Rc + 2 * N;             // adjoint of R, two columns by parity
    float *red = dR + 2 * N;            // [m][NW][2] wavefront partial sums
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;

    for (int64_t f = blockIdx.x; f < P.B; f += gridDim.x) {
        // the frame's LLRs, output gradient and channel gradient stay in
        // registers
        float yv[S::YR], dv[S::YR], dc[S::YR];
#pragma unroll
        for (int k = 0; k < S::YR; k++) {
            const int i = tid + k * NT;
            yv[k] = i < N ? P.llr[f * N + i] : 0.0f;
            dv[k] = i < N ? P.dout[f * N + i] : 0.0f;
            dc[k] = 0.0f;
        }
        // the adjoint of L after the last iteration is zero
        for (int i = tid; i < (M - 1) * N; i += NT)
            dA[i] = 0.0f;
        for (int t = P.T - 1; t >= 0; t--) {
            // L^{t-1} at columns 2..m
            const float *ck = P.ckpt + ((int64_t)t * P.B + f) * (M - 1) * N;
            auto lprev = [&](int c, int r) -> float {
                return c == M + 1 ? (frozen_at(P.frozen, r) ? kInf : 0.0f)
                                  : ck[(c - 2) * N + r];
            };
            // rows of this thread's PE at stage j, from a copy of the thread
            // index made opaque per iteration: the rows and offsets of all
            // stages would otherwise be kept in registers across iterations
            int tt = tid;
            asm volatile("" : "+v"(tt));
            auto row_a = [&](int j) {
                const int sh = M - j;
                return ((tt >> sh) << (sh + 1)) | (tt & ((1 << sh) - 1));
            };
            // L^{t-1} at columns 2..m for the R sweep of iteration t+1, all
            // requested at once so that their latencies overlap, and kept for
            // the adjoint stages (one read of the checkpoint per iteration)
            float keepLa[M], keepLb[M];
#pragma unroll
            for (int j = 1; j < M; j++) {
                keepLa[j - 1] = 0.0f;
                keepLb[j - 1] = 0.0f;
                if (tid < H) {
                    const int a = row_a(j);
                    keepLa[j - 1] = lprev(j + 1, a);
                    keepLb[j - 1] = lprev(j + 1, a + (1 << (M - j)));
                }
            }
#pragma unroll
            for (int k = 0; k < S::YR; k++) {
                const int i = tid + k * NT;
                if (i < N)
                    Rc[i] = yv[k];
            }
            sync_lds();
            // R^t at column j on this thread's rows of stage j, kept for the
            // adjoint stages (column j at parity (j - 1) & 1)
            float keepRa[M], keepRb[M];
#pragma unroll
            for (int j = 1; j < M; j++) {
                const float aR = scale_at(P.alpha, ((int64_t)t * M + (j - 1)) * 2 + 1);
                const int sh = M - j, h = 1 << sh;
                keepRa[j - 1] = 0.0f;
                keepRb[j - 1] = 0.0f;
                if (tid < H) {
                    const int a = row_a(j);
                    const int b = a + h;
                    const float *Ri = Rc + ((j - 1) & 1) * N;
                    float *Ro = Rc + (j & 1) * N;
                    const float La = keepLa[j - 1], Lb = keepLb[j - 1];
                    const float Ra = Ri[a], Rb = Ri[b];
                    keepRa[j - 1] = Ra;
                    keepRb[j - 1] = Rb;
                    const float s = Lb + Rb;
                    Ro[a] = aR * g0(Ra, s);
                    Ro[b] = Rb + aR * g0(La, Ra);
                }
                sync_stages<NW>(h, h >> 1);
            }
            keepRa[M - 1] = 0.0f;
            keepRb[M - 1] = 0.0f;
            if (tid < H) {
                const int a = row_a(M);
                const float *Ri = Rc + ((M - 1) & 1) * N;
                keepRa[M - 1] = Ri[a];
                keepRb[M - 1] = Ri[a + 1];
            }
            {
                float *d = dR + ((M + 1) & 1) * N;
#pragma unroll
                for (int k = 0; k < S::YR; k++) {
                    const int i = tid + k * NT;
                    if (i < N)
                        d[i] = t == P.T - 1 ? dv[k] : 0.0f;
                }
            }
            sync_lds();
            // the adjoint of L^t at column j, stage j's input (LDS)
            float qiLa = 0.0f, qiLb = 0.0f;
            auto fetch = [&](int j) {
                const int a = row_a(j), b = a + (1 << (M - j));
                qiLa = 0.0f;
                qiLb = 0.0f;
                if (j >= 2) {
                    qiLa = dA[(j - 2) * N + a];                   // column j
                    qiLb = dA[(j - 2) * N + b];
                }
            };
#pragma unroll
            for (int j = M; j >= 1; j--) {
                const float aL = scale_at(P.alpha, ((int64_t)t * M + (j - 1)) * 2);
                const float aR = scale_at(P.alpha, ((int64_t)t * M + (j - 1)) * 2 + 1);
                const int sh = M - j, h = 1 << sh;
                // sums start at -0, the identity of the addition (the first
                // term is then taken as it is)
                float daL = -0.0f, daR = -0.0f;
                if (tid < H) {
                    const int a = row_a(j);
                    const int b = a + h;
                    const float *dRi = dR + ((j + 1) & 1) * N;   // column j+1
                    float *dRo = dR + (j & 1) * N;               // column j
                    // L^{t-1} at column j+1: kept from the R sweep, or the
                    // frozen prior at column m+1
                    const float La = j < M ? keepLa[j - 1] : lprev(M + 1, a);
                    const float Lb = j < M ? keepLb[j - 1] : lprev(M + 1, b);
                    fetch(j);
                    const float iLa = qiLa, iLb = qiLb;
                    float oLa = 0.0f, oLb = 0.0f;
                    const float Ra = keepRa[j - 1], Rb = keepRb[j - 1];
                    const float s = Lb + Rb;
                    const float gA = g0(La, s), g1 = g0(La, Ra), gB = g0(Ra, s);
                    // adjoints of the four outputs; infinite outputs are constants
                    const bool fLa = finite(aL * gA), fLb = finite(Lb + aL * g1);
                    const bool fRa = finite(aR * gB), fRb = finite(Rb + aR * g1);
                    oLa = fLa ? iLa : 0.0f;
                    oLb = fLb ? iLb : 0.0f;
                    const float oRa = fRa ? dRi[a] : 0.0f;
                    const float oRb = fRb ? dRi[b] : 0.0f;
                    if (fLa)
                        daL += oLa * gA;
                    if (fLb)
                        daL += oLb * g1;
                    if (fRa)
                        daR += oRa * gB;
                    if (fRb)
                        daR += oRb * g1;
                    const float dgA = aL * oLa;
                    const float dg1 = aL * oLb + aR * oRb;
                    const float dgB = aR * oRa;
                    float dLa = -0.0f, dLb = oLb, dRa = -0.0f, dRb = oRb, ds = -0.0f;
                    g0_back(La, s, dgA, dLa, ds);
                    g0_back(La, Ra, dg1, dLa, dRa);
                    g0_back(Ra, s, dgB, dRa, ds);
                    if (finite(s)) {
                        dLb += ds;
                        dRb += ds;
                    }
                    if (j + 1 <= M) {
                        // the adjoint of L^{t-1} at column j+1 replaces that
                        // of L^t there, which stage j+1 read before the
                        // barrier
                        dA[(j - 1) * N + a] = finite(La) ? dLa : 0.0f;
                        dA[(j - 1) * N + b] = finite(Lb) ? dLb : 0.0f;
                    }
                    dRo[a] = dRa;
                    dRo[b] = dRb;
                }
                // this stage's scale gradients, summed over the wavefront
                // (the group's sum is taken once per iteration)
                {
                    float vL = daL, vR = daR;
                    wave_sum2(vL, vR);
                    if (lane == 63) {
                        red[((j - 1) * NW + wv) * 2] = vL;
                        red[((j - 1) * NW + wv) * 2 + 1] = vR;
                    }
                }
                // after stage 1 the channel gradient is read in another
                // thread order
                if (j > 1)
                    sync_stages<NW>(h, h << 1);
                else
                    sync_lds();
            }
#pragma unroll
            for (int k = 0; k < S::YR; k++) {
                const int i = tid + k * NT;
                if (i < N)
                    dc[k] += dR[(1 & 1) * N + i];
            }
            sync_lds();
            if (tid < 2 * M) {
                float acc = 0.0f;
                for (int w = 0; w < NW; w++)
                    acc += red[((tid >> 1) * NW + w) * 2 + (tid & 1)];
                P.dalpha_frame[((f * P.T + t) * M) * 2 + tid] = acc;
            }
            // the adjoint of L written in this iteration is read by other
            // threads in the next one
            __syncthreads();
        }
        if (P.dllr) {
#pragma unroll
            for (int k = 0; k < S::YR; k++) {
                const int i = tid + k * NT;
                if (i < N)
                    P.dllr[f * N + i] = dc[k];
            }
        }
        __syncthreads();
    }
}

// dalpha[k] = sum over frames of dalpha_frame[f][k], in FP64, fixed order
__global__ __launch_bounds__(256) void reduce_frames_kernel(const float *part,
                                                            int64_t B, int K,
                                                            float *out)
{
    __shared__ double acc[256];
    const int k = (int)blockIdx.x, tid = (int)threadIdx.x;
    double s = 0.0;
    for (int64_t f = tid; f < B; f += 256)
        s += (double)part[f * K + k];
    acc[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w)
            acc[tid] += acc[tid + w];
        __syncthreads();
    }
    if (tid == 0)
        out[k] = (float)acc[0];
}

int64_t frames_grid(const pbp_code *c, int64_t B, int per_cu)
{
    int64_t g = (int64_t)(c->cus > 0 ? c->cus : 256) * per_cu;
    return B < g ? B : g;
}

template <int M>
hipError_t launch_forward(const pbp_code *c, FwdParams &P, hipStream_t st)
{
    auto kern = unrolled_forward_kernel<M>;
    const size_t lds = fwd_lds_bytes<M>();
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)frames_grid(c, P.B, 8)),
                       dim3(Shape<M>::NT), lds, st, P);
    return hipGetLastError();
}

template <int M>
hipError_t launch_backward(const pbp_code *c, BwdParams &P, hipStream_t st)
{
    auto kern = unrolled_backward_kernel<M>;
    const size_t lds = bwd_lds_bytes<M>();
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    // as many groups per compute unit as are resident (a grid stride over
    // more would leave the extra groups a tail of their own)
    static int occ = 0;
    if (occ < 1) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void *)kern,
                                                         Shape<M>::NT, lds) != hipSuccess)
            return hipGetLastError();
        occ = o < 1 ? 1 : o;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)frames_grid(c, P.B, occ)),
                       dim3(Shape<M>::NT), lds, st, P);
    return hipGetLastError();
}

template <template <int> class Fn, typename Prm>
hipError_t dispatch_m(int m, const pbp_code *c, Prm &P, hipStream_t st)
{
    switch (m) {
    case 1: return Fn<1>::run(c, P, st);
    case 2: return Fn<2>::run(c, P, st);
    case 3: return Fn<3>::run(c, P, st);
    case 4: return Fn<4>::run(c, P, st);
    case 5: return Fn<5>::run(c, P, st);
    case 6: return Fn<6>::run(c, P, st);
    case 7: return Fn<7>::run(c, P, st);
    case 8: return Fn<8>::run(c, P, st);
    case 9: return Fn<9>::run(c, P, st);
    case 10: return Fn<10>::run(c, P, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M>
struct Fwd {
    static hipError_t run(const pbp_code *c, FwdParams &P, hipStream_t st)
    {
        return launch_forward<M>(c, P, st);
    }
};

template <int M>
struct Bwd {
    static hipError_t run(const pbp_code *c, BwdParams &P, hipStream_t st)
    {
        return launch_backward<M>(c, P, st);
    }
};

constexpr int kMaxUnrolledLog = 10;
constexpr int kMaxT = 1 << 16;

}  // namespace

extern "C" int32_t pbp_unrolled_forward(const pbp_code *code, const float *llr,
                                        int64_t B, int32_t T,
                                        const float *alpha, float *out,
                                        float *ckpt, void *stream)
{
    if (!code || B < 0 || T < 1 || T > kMaxT)
        return PBP_EINVAL;
    if (code->m > kMaxUnrolledLog)
        return PBP_EUNSUPPORTED;
    if (B == 0)
        return PBP_OK;
    if (!llr || !alpha || !out)
        return PBP_EINVAL;
    FwdParams P{};
    P.llr = llr;
    P.B = B;
    P.T = T;
    P.alpha = alpha;
    P.frozen = code->d_frozen_words;
    P.out = out;
    P.ckpt = code->m >= 2 ? ckpt : nullptr;
    return dispatch_m<Fwd>(code->m, code, P, (hipStream_t)stream) == hipSuccess
               ? PBP_OK
               : PBP_EDEVICE;
}

extern "C" int32_t pbp_unrolled_backward(const pbp_code *code, const float *llr,
                                         int64_t B, int32_t T,
                                         const float *alpha, const float *ckpt,
                                         const float *dout, float *dalpha_frame,
                                         float *dalpha, float *dllr,
                                         void *stream)
{
    if (!code || B < 0 || T < 1 || T > kMaxT)
        return PBP_EINVAL;
    if (code->m > kMaxUnrolledLog)
        return PBP_EUNSUPPORTED;
    if (!dalpha)
        return PBP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int K = T * code->m * 2;
    if (B > 0) {
        if (!llr || !alpha || !dout || !dalpha_frame ||
            (code->m >= 2 && !ckpt))
            return PBP_EINVAL;
        BwdParams P{};
        P.llr = llr;
        P.B = B;
        P.T = T;
        P.alpha = alpha;
        P.frozen = code->d_frozen_words;
        P.ckpt = ckpt;
        P.dout = dout;
        P.dalpha_frame = dalpha_frame;
        P.dllr = dllr;
        if (dispatch_m<Bwd>(code->m, code, P, st) != hipSuccess)
            return PBP_EDEVICE;
    }
    hipLaunchKernelGGL(reduce_frames_kernel, dim3((unsigned)K), dim3(256), 0,
                       st, dalpha_frame, B, K, dalpha);
    return hipGetLastError() == hipSuccess ? PBP_OK : PBP_EDEVICE;
}
