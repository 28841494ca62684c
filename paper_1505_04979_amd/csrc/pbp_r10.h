// Row mappings of the register-resident N = 1024 decoder (see pbp_r10.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbp.h"

struct pbp_code;

namespace pbp {
namespace r10 {

constexpr int M = 10;
constexpr int N = 1 << M;
constexpr int Q = N / 64;   // rows per lane

enum Mapping { MA = 0, MB = 1, MC = 2, MD = 3 };

// the upper butterfly row bit of a mapping's stage pair
__host__ __device__ constexpr int map_x(int mp)
{
    return mp == MA ? 1 : mp == MB ? 7 : mp == MC ? 5 : 3;
}

// row bit held by register-index bit qb (0..3)
__host__ __device__ constexpr int qrow(int mp, int qb)
{
    return qb == 3 ? 9 : qb == 2 ? 8 : qb == 1 ? map_x(mp) : map_x(mp) - 1;
}

// row bit held by lane-index bit lb (0..5): the six bits of 0..7 that are
// not register bits, in increasing order
__host__ __device__ constexpr int lrow(int mp, int lb)
{
    int n = 0;
    for (int b = 0; b < 8; ++b) {
        if (b == map_x(mp) || b == map_x(mp) - 1)
            continue;
        if (n == lb)
            return b;
        ++n;
    }
    return -1;
}

// row bits contributed by register index q
__host__ __device__ constexpr int rowq(int mp, int q)
{
    int r = 0;
    for (int qb = 0; qb < 4; ++qb)
        if ((q >> qb) & 1)
            r |= 1 << qrow(mp, qb);
    return r;
}

// Ballot words of the frozen mask, [mapping][register index]: bit l is set
// when the row held by lane l is frozen.
void frozen_words(const uint8_t *frozen, uint64_t *fzw);

size_t smem_bytes();

hipError_t launch(const pbp_code *c, const float *llr, int64_t B,
                  const pbp_decode_opts *o, uint8_t *info_out,
                  int32_t *iters_out, int64_t *pe_out, float *soft_out,
                  int *counter, hipStream_t st);

}  // namespace r10
}  // namespace pbp
