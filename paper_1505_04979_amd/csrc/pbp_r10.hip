// Batch kernel of the register-resident N = 1024 decoder: persistent
// wavefronts take frames from a device counter (pbp_r10_decoder.h).
#include <hip/hip_runtime.h>

#include "pbp_internal.h"
#include "pbp_r10.h"
#include "pbp_r10_decoder.h"

namespace pbp {
namespace r10 {
namespace {

template <bool FRZ, bool ES>
__global__ __launch_bounds__(64, 2) void bp_decode_r10_kernel(Params P)
{
    __shared__ Smem S;
    const int lane = (int)__builtin_amdgcn_workitem_id_x();
    Decoder<FRZ, ES> D(P, S, lane);
    for (;;) {
        int frame = 0;
        if (lane == 0)
            frame = atomicAdd(P.counter, 1);
        frame = __shfl(frame, 0, 64);
        if (frame >= P.B)
            break;
        D.decode(frame);
    }
    // every wave has taken its last frame number before it counts itself out;
    // the last one out rewinds both counters for the next launch on the stream
    if (lane == 0 && atomicAdd(P.counter + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(P.counter, 0);
        atomicExch(P.counter + 1, 0);
    }
}

}  // namespace

size_t smem_bytes() { return sizeof(Smem); }

hipError_t launch(const pbp_code *c, const float *llr, int64_t B,
                  const pbp_decode_opts *o, uint8_t *info_out,
                  int32_t *iters_out, int64_t *pe_out, float *soft_out,
                  int *counter, hipStream_t st)
{
    Params P{};
    P.llr = llr;
    P.B = B;
    P.counter = counter;
    P.fzw = c->d_fzw10;
    P.info_pos = c->d_info_pos;
    P.K = c->K;
    P.max_iter = o->max_iter;
    P.freezing = o->freezing;
    P.freeze_input = o->freeze_input;
    P.freeze_walk = o->freeze_walk;
    P.alpha = o->alpha;
    P.info_out = info_out;
    P.iters_out = iters_out;
    P.pe_out = pe_out;
    P.soft_out = soft_out;
    int64_t grid = (int64_t)c->cus * 8;
    if (grid > B)
        grid = B;
    // early stop without freezing runs the freezing kernel with the walk
    // switched off (the frozen prefix stays empty, so no PE is skipped)
    if (o->early_stop)
        hipLaunchKernelGGL((bp_decode_r10_kernel<true, true>), dim3(grid), dim3(64), 0, st, P);
    else if (o->freezing)
        hipLaunchKernelGGL((bp_decode_r10_kernel<true, false>), dim3(grid), dim3(64), 0, st, P);
    else
        hipLaunchKernelGGL((bp_decode_r10_kernel<false, false>), dim3(grid), dim3(64), 0, st, P);
    return hipGetLastError();
}

void frozen_words(const uint8_t *frozen, uint64_t *fzw)
{
    for (int mp = 0; mp < 4; mp++)
        for (int q = 0; q < Q; q++) {
            uint64_t w = 0;
            for (int l = 0; l < 64; l++) {
                int r = rowq(mp, q);
                for (int lb = 0; lb < 6; lb++)
                    if ((l >> lb) & 1)
                        r |= 1 << lrow(mp, lb);
                if (frozen[r])
                    w |= 1ull << l;
            }
            fzw[mp * Q + q] = w;
        }
}

}  // namespace r10
}  // namespace pbp
