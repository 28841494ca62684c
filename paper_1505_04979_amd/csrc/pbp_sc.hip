// Successive-cancellation (SC) decoding on the GPU: the decoder whose
// scheduling tree Section III maps onto the BP factor graph.  It decodes the
// same codes as pbp_decode (natural order, G = F^{(x)m}) and serves as the
// error-rate reference of Section III's comparison of a frozen CSFG's ML
// decision with SC.
//
// One wavefront per frame, persistent over a grid stride; a workgroup holds
// up to four such wavefronts, each with its own LDS.  The node at
// depth d of the SC tree covers 2^(m-d) consecutive source bits; its LLRs
// live in LDS (alpha: depth d at offset N - 2^(m-d+1), 2^(m-d) values; the
// channel LLRs of depth 0 are read in place).  The re-encoded bits of every
// completed subtree are kept in place in one byte per source position
// (beta): the subtree over positions [s, s + n) holds x = u G_n there, so
// completing a right subtree turns its parent's bits into
// [x_left ^ x_right | x_right] by n XORs.  Leaf i follows leaf i - 1 by one
// g step at the depth where the path turns right (the depth of the lowest
// set bit of i) and f steps down to the leaf.
//
// From N = 64 on, the bottom six levels run in registers: the subtrees of 64
// positions are the leaves of the LDS walk above, and each is decoded with
// one position per lane, its node LLRs moving between lanes by DPP and
// cross-lane shuffles and its re-encoded bits in one 64-bit mask, every
// index known at compile time.  The arithmetic is the same f and g.
#include <hip/hip_runtime.h>

#include "pbp_internal.h"

namespace {

// LDS of one wavefront: node LLRs (N floats) and re-encoded bits (N bytes)
__host__ __device__ constexpr size_t lds_per_wave(int N)
{
    return (sizeof(float) * (size_t)N + (size_t)N + 15) & ~(size_t)15;
}

// Independent wavefronts per workgroup, each decoding its own frames in its
// own LDS slice.  A compute unit holds at most 16 workgroups, so groups of
// one wavefront would cap it at 16 wavefronts; up to four per group (within
// 128 KB of LDS per group) let the register and LDS budgets set the
// occupancy.
template <int M>
__host__ __device__ constexpr int sc_waves()
{
    return lds_per_wave(1 << M) * 4 <= 131072 ? 4
         : lds_per_wave(1 << M) * 2 <= 131072 ? 2 : 1;
}

// f: the min-sum check-node rule sign(a) sign(b) min(|a|, |b|), exact (a
// selection: b clamped to [-|a|, |a|] with the sign of a applied)
__device__ __forceinline__ float sc_f(float a, float b)
{
    const float t = __uint_as_float(__float_as_uint(b) ^
                                    (__float_as_uint(a) & 0x80000000u));
    return __builtin_amdgcn_fmed3f(-fabsf(a), t, fabsf(a));
}

// g: b + (1 - 2c) a, one rounding (the sign flip is exact)
__device__ __forceinline__ float sc_g(float a, float b, uint8_t c)
{
    return b + (c ? -a : a);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SCParams {
    const float *llr;
    int64_t B;
    const uint64_t *frozen_words;   // bit i of word i >> 6: position i frozen
    const int32_t *info_pos;
    int32_t K;
    uint8_t *info_out;
    float *leaf_out;                // B x N or null: the LLR at each leaf
};

// N < 64: every level in LDS
template <int M>
__global__ __launch_bounds__(64 * sc_waves<M>()) void sc_decode_kernel(SCParams P)
{
    constexpr int N = 1 << M;
    extern __shared__ __align__(16) unsigned char smem_all[];
    // each wavefront of the group decodes its own frames in its own LDS
    const int wv = (int)threadIdx.x >> 6;
    unsigned char *smem = smem_all + wv * lds_per_wave(N);
    float *alpha = reinterpret_cast<float *>(smem);          // N - 1 floats
    uint8_t *beta = smem + sizeof(float) * N;                // N bytes
    const int lane = (int)threadIdx.x & 63;

    constexpr int W = sc_waves<M>();
    for (int64_t frame = (int64_t)blockIdx.x * W + wv; frame < P.B;
         frame += (int64_t)gridDim.x * W) {
        const float *ch = P.llr + frame * N;
        // depth d >= 1 starts at N - 2^(m-d+1); depth 0 is the channel
        auto col = [&](int d) -> float * { return alpha + (N - (N >> (d - 1))); };
        for (int i = 0; i < N; i++) {
            // the depth whose node turns right at leaf i (0 for leaf 0: the
            // path starts at the root with f steps)
            int p = 0;
            if (i > 0) {
                const int t = __builtin_ctz(i);
                p = M - 1 - t;
                const int n = 1 << t;                // child size
                const float *src = p == 0 ? ch : col(p);
                float *dst = col(p + 1);
                const uint8_t *c = beta + (i - n);
                for (int j = lane; j < n; j += 64)
                    dst[j] = sc_g(src[j], src[j + n], c[j]);
                wave_sync();
                p++;
            }
            for (int d = p; d < M; d++) {
                const int n = N >> (d + 1);
                const float *src = d == 0 ? ch : col(d);
                float *dst = col(d + 1);
                for (int j = lane; j < n; j += 64)
                    dst[j] = sc_f(src[j], src[j + n]);
                wave_sync();
            }
            // leaf decision: 0 at a frozen position, else [LLR < 0]
            const float v = M == 0 ? ch[0] : col(M)[0];
            const bool fz = (P.frozen_words[i >> 6] >> (i & 63)) & 1;
            if (lane == 0) {
                beta[i] = fz ? 0 : (v < 0.0f ? 1 : 0);
                if (P.leaf_out)
                    P.leaf_out[frame * N + i] = v;
            }
            wave_sync();
            // completed right subtrees: parent bits [x_l ^ x_r | x_r]
            for (int t = 0; t < M && ((i >> t) & 1); t++) {
                const int n = 1 << t;
                const int s = i + 1 - 2 * n;
                for (int j = lane; j < n; j += 64)
                    beta[s + j] ^= beta[s + n + j];
                wave_sync();
            }
        }
        // beta now holds x = u G, the re-encoded word; the decided source
        // bits are its transform (G is its own inverse)
        for (int l = 0; (1 << l) < N; l++) {
            const int h = 1 << l;
            for (int q = lane; q < N / 2; q += 64) {
                const int a = ((q >> l) << (l + 1)) | (q & (h - 1));
                beta[a] ^= beta[a + h];
            }
            wave_sync();
        }
        uint8_t *out = P.info_out + frame * P.K;
        for (int k = lane; k < P.K; k += 64)
            out[k] = beta[P.info_pos[k]];
        wave_sync();
    }
}


// node LLRs held one per lane: lane j (< n) takes lane j + n
template <int n>
__device__ __forceinline__ float from_lane_plus(float v)
{
    if constexpr (n <= 8) {
        // row_shl:n within each row of 16 lanes (lanes j < n stay in row 0)
        return __int_as_float(__builtin_amdgcn_update_dpp(
            0, __float_as_int(v), 0x100 | n, 0xf, 0xf, false));
    } else {
        return __shfl_down(v, n, 64);
    }
}

// The 64 positions of one subtree, root LLRs a0 (lane i = position i):
// decisions and leaf LLRs in position order, re-encoded bits returned as a
// mask (bit i = x_i of x = u G_64).  fz: the subtree's frozen bits.  Leaf
// i's LLR is written to leaf (when not null) by lane 0.
struct Sub64 {
    float a[7];           // the current path's node LLRs, level k has 64 >> k
    uint64_t x;           // decided, then re-encoded bits
    uint64_t fz;
    float *leaf;
    int lane;

    // level K+1 from level K: left child (f) or right child (g)
    template <int K>
    __device__ __forceinline__ void step_f()
    {
        constexpr int n = 32 >> K;           // child size
        const float b = from_lane_plus<n>(a[K]);
        a[K + 1] = sc_f(a[K], b);
    }
    template <int K, int I>
    __device__ __forceinline__ void step_g()
    {
        constexpr int n = 32 >> K;           // child size; left sibling at
                                             // positions I - n .. I - 1
        const float b = from_lane_plus<n>(a[K]);
        const uint8_t c = (uint8_t)((x >> (I - n)) >> lane) & 1;
        a[K + 1] = sc_g(a[K], b, c);
    }
    template <int K, int I>
    __device__ __forceinline__ void down_f()
    {
        if constexpr (K < 6) {
            step_f<K>();
            down_f<K + 1, I>();
        }
    }
    template <int I>
    __device__ __forceinline__ void leaf_step()
    {
        if constexpr (I < 64) {
            if constexpr (I == 0) {
                down_f<0, 0>();
            } else {
                constexpr int t = __builtin_ctz(I);
                constexpr int K = 5 - t;          // level of the turning node
                step_g<K, I>();
                down_f<K + 1, I>();
            }
            // leaf decision: 0 at a frozen position, else [LLR < 0]
            const float lv = __int_as_float(__builtin_amdgcn_readfirstlane(
                __float_as_int(a[6])));
            const bool u = !((fz >> I) & 1) && lv < 0.0f;
            if (leaf && lane == 0)
                leaf[I] = lv;
            x |= (uint64_t)u << I;
            // completed right subtrees: [x_l ^ x_r | x_r]
#pragma unroll
            for (int tt = 0; tt < 6; tt++) {
                if (((I >> tt) & 1) == 0)
                    break;
                const int n = 1 << tt;
                const int s0 = I + 1 - 2 * n;
                const uint64_t m = (n == 64 ? ~0ull : ((1ull << n) - 1)) << s0;
                x ^= (x >> n) & m;
            }
            leaf_step<I + 1>();
        }
    }
};

// N >= 64: the levels above the 64-position subtrees in LDS, the subtrees in
// registers
template <int M>
__global__ __launch_bounds__(64 * sc_waves<M>()) void sc_decode64_kernel(SCParams P)
{
    constexpr int N = 1 << M;
    constexpr int MS = M - 6;                 // depth of the 64-position nodes
    extern __shared__ __align__(16) unsigned char smem_all[];
    // each wavefront of the group decodes its own frames in its own LDS
    const int wv = (int)threadIdx.x >> 6;
    unsigned char *smem = smem_all + wv * lds_per_wave(N);
    float *alpha = reinterpret_cast<float *>(smem);          // N - 1 floats
    uint8_t *beta = smem + sizeof(float) * N;                // N bytes
    const int lane = (int)threadIdx.x & 63;

    constexpr int W = sc_waves<M>();
    for (int64_t frame = (int64_t)blockIdx.x * W + wv; frame < P.B;
         frame += (int64_t)gridDim.x * W) {
        const float *ch = P.llr + frame * N;
        auto col = [&](int d) -> float * { return alpha + (N - (N >> (d - 1))); };
        for (int s = 0; s < (N >> 6); s++) {
            // the path to subtree s: one g step where it turns right, f steps
            // down to depth MS (every node there has at least 128 positions)
            int p = 0;
            if (s > 0) {
                const int t = __builtin_ctz(s) + 6;
                p = M - 1 - t;
                const int n = 1 << t;
                const float *src = p == 0 ? ch : col(p);
                float *dst = col(p + 1);
                const uint8_t *c = beta + (64 * s - n);
                for (int j = lane; j < n; j += 64)
                    dst[j] = sc_g(src[j], src[j + n], c[j]);
                wave_sync();
                p++;
            }
            for (int d = p; d < MS; d++) {
                const int n = N >> (d + 1);
                const float *src = d == 0 ? ch : col(d);
                float *dst = col(d + 1);
                for (int j = lane; j < n; j += 64)
                    dst[j] = sc_f(src[j], src[j + n]);
                wave_sync();
            }
            Sub64 sub;
            sub.a[0] = MS == 0 ? ch[lane] : col(MS)[lane];
            sub.x = 0;
            sub.fz = P.frozen_words[s];
            sub.leaf = P.leaf_out ? P.leaf_out + frame * N + 64 * s : nullptr;
            sub.lane = lane;
            sub.leaf_step<0>();
            beta[64 * s + lane] = (uint8_t)((sub.x >> lane) & 1);
            wave_sync();
            // completed right subtrees above the 64-position level
            for (int t = 6; t < M && ((s >> (t - 6)) & 1); t++) {
                const int n = 1 << t;
                const int s0 = 64 * (s + 1) - 2 * n;
                for (int j = lane; j < n; j += 64)
                    beta[s0 + j] ^= beta[s0 + n + j];
                wave_sync();
            }
        }
        // beta holds x = u G; the decided source bits are its transform
        for (int l = 0; (1 << l) < N; l++) {
            const int h = 1 << l;
            for (int q = lane; q < N / 2; q += 64) {
                const int a = ((q >> l) << (l + 1)) | (q & (h - 1));
                beta[a] ^= beta[a + h];
            }
            wave_sync();
        }
        uint8_t *out = P.info_out + frame * P.K;
        for (int k = lane; k < P.K; k += 64)
            out[k] = beta[P.info_pos[k]];
        wave_sync();
    }
}

// as many wavefronts per compute unit as are resident (occ, looked up once
// per kernel): a grid stride over more would leave the extra ones a tail
template <class Kern>
hipError_t launch_k(Kern kern, const pbp_code *c, SCParams &P, int waves,
                    size_t lds, int &occ, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    if (occ < 1) {
        int o = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void *)kern,
                                                         64 * waves, lds);
        if (e != hipSuccess)
            return e;
        occ = o < 1 ? 1 : o;
    }
    int64_t grid = (P.B + waves - 1) / waves;
    const int64_t cap = (int64_t)c->cus * occ;
    if (grid > cap)
        grid = cap;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * waves), lds, st, P);
    return hipGetLastError();
}

template <int M>
hipError_t launch_sc(const pbp_code *c, SCParams &P, hipStream_t st)
{
    constexpr int N = 1 << M;
    constexpr int W = sc_waves<M>();
    const size_t lds = W * lds_per_wave(N);
    static int occ = 0;
    if constexpr (M >= 6)
        return launch_k(sc_decode64_kernel<M>, c, P, W, lds, occ, st);
    else
        return launch_k(sc_decode_kernel<M>, c, P, W, lds, occ, st);
}

}  // namespace

extern "C" int32_t pbp_decode_sc(const pbp_code *code, const float *llr,
                                 int64_t B, uint8_t *info_out, float *leaf_out,
                                 void *stream)
{
    if (!code || B < 0)
        return PBP_EINVAL;
    if (B == 0)
        return PBP_OK;
    if (!llr || (!info_out && code->K > 0))
        return PBP_EINVAL;
    SCParams P{};
    P.llr = llr;
    P.B = B;
    P.frozen_words = code->d_frozen_words;
    P.info_pos = code->d_info_pos;
    P.K = code->K;
    P.info_out = info_out;
    P.leaf_out = leaf_out;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    switch (code->m) {
    case 1: e = launch_sc<1>(code, P, st); break;
    case 2: e = launch_sc<2>(code, P, st); break;
    case 3: e = launch_sc<3>(code, P, st); break;
    case 4: e = launch_sc<4>(code, P, st); break;
    case 5: e = launch_sc<5>(code, P, st); break;
    case 6: e = launch_sc<6>(code, P, st); break;
    case 7: e = launch_sc<7>(code, P, st); break;
    case 8: e = launch_sc<8>(code, P, st); break;
    case 9: e = launch_sc<9>(code, P, st); break;
    case 10: e = launch_sc<10>(code, P, st); break;
    case 11: e = launch_sc<11>(code, P, st); break;
    case 12: e = launch_sc<12>(code, P, st); break;
    case 13: e = launch_sc<13>(code, P, st); break;
    case 14: e = launch_sc<14>(code, P, st); break;
    default: return PBP_EUNSUPPORTED;
    }
    return e == hipSuccess ? PBP_OK : PBP_EDEVICE;
}
