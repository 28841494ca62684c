// Host side of libpbp: status strings, code construction, code handles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <utility>
#include <vector>

#include "pbp_internal.h"
#include "pbp_r10.h"

extern "C" const char *pbp_status_string(int32_t status)
{
    switch (status) {
    case PBP_OK: return "ok";
    case PBP_EINVAL: return "invalid argument";
    case PBP_ENOMEM: return "out of memory";
    case PBP_EDEVICE: return "HIP runtime error";
    case PBP_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

// Code construction: Bhattacharyya parameters of the synthetic channels of
// G = F^{(x)m} in natural order, z_{2i} = 2z - z^2 and z_{2i+1} = z^2, from
// z_0 = exp(-R Eb/N0).  Tracked as (ln z, ln(1 - z)) so that neither loses
// relative precision near 0 or 1:
//   index 2i:   z' = z (1 + w),  w' = w^2
//   index 2i+1: z' = z^2,        w' = w (1 + z)
// with w = 1 - z.  Positions are ranked by ln z - ln w (monotone in z).
extern "C" int32_t pbp_construct(int32_t N, int32_t K, double design_ebn0_db,
                                 uint8_t *frozen_out)
{
    if (!pbp::valid_n(N) || K < 0 || K > N || !frozen_out ||
        !std::isfinite(design_ebn0_db))
        return PBP_EINVAL;
    try {
        const double rate = (double)K / (double)N;
        const double z0 = std::exp(-rate * std::pow(10.0, design_ebn0_db / 10.0));
        std::vector<double> lz(N), lw(N), nz(N), nw(N);
        lz[0] = std::log(z0);
        lw[0] = std::log1p(-z0);
        for (int size = 1; size < N; size <<= 1) {
            for (int i = 0; i < size; i++) {
                const double z = std::exp(lz[i]), w = std::exp(lw[i]);
                nz[2 * i] = lz[i] + std::log1p(w);
                nw[2 * i] = 2.0 * lw[i];
                nz[2 * i + 1] = 2.0 * lz[i];
                nw[2 * i + 1] = lw[i] + std::log1p(z);
            }
            std::copy(nz.begin(), nz.begin() + 2 * size, lz.begin());
            std::copy(nw.begin(), nw.begin() + 2 * size, lw.begin());
        }
        std::vector<double> logit(N);
        for (int i = 0; i < N; i++)
            logit[i] = lz[i] - lw[i];
        std::vector<int> order(N);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return logit[a] > logit[b]; });
        std::fill(frozen_out, frozen_out + N, 0);
        for (int r = 0; r < N - K; r++)
            frozen_out[order[r]] = 1;
    } catch (const std::bad_alloc &) {
        return PBP_ENOMEM;
    }
    return PBP_OK;
}

namespace {

void free_code(pbp_code *c)
{
    if (!c)
        return;
    if (c->d_frozen_words)
        (void)hipFree(c->d_frozen_words);
    if (c->d_info_pos)
        (void)hipFree(c->d_info_pos);
    if (c->d_fzw10)
        (void)hipFree(c->d_fzw10);
    delete c;
}

}  // namespace

extern "C" int32_t pbp_code_create(int32_t N, int32_t K, const uint8_t *frozen,
                                   pbp_code **out)
{
    if (!out)
        return PBP_EINVAL;
    *out = nullptr;
    if (!pbp::valid_n(N) || K < 0 || K > N || !frozen)
        return PBP_EINVAL;
    int32_t nfrozen = 0;
    for (int i = 0; i < N; i++)
        nfrozen += frozen[i] != 0;
    if (nfrozen != N - K)
        return PBP_EINVAL;

    pbp_code *c = new (std::nothrow) pbp_code;
    if (!c)
        return PBP_ENOMEM;
    try {
        c->N = N;
        c->K = K;
        c->m = pbp::log2i(N);
        c->frozen.assign(frozen, frozen + N);
        for (auto &v : c->frozen)
            v = v ? 1 : 0;
        for (int i = 0; i < N; i++)
            if (!c->frozen[i])
                c->info_pos.push_back(i);
    } catch (const std::bad_alloc &) {
        delete c;
        return PBP_ENOMEM;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        free_code(c);
        return PBP_EDEVICE;
    }
    const int nwords = N >= 64 ? N / 64 : 1;
    std::vector<uint64_t> words(nwords, 0);
    for (int i = 0; i < N; i++)
        if (c->frozen[i])
            words[i >> 6] |= 1ull << (i & 63);
    std::vector<int32_t> pos(c->info_pos);
    if (pos.empty())
        pos.push_back(0);
    if (hipMalloc(&c->d_frozen_words, nwords * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&c->d_info_pos, pos.size() * sizeof(int32_t)) != hipSuccess) {
        free_code(c);
        return PBP_ENOMEM;
    }
    if (hipMemcpy(c->d_frozen_words, words.data(), nwords * sizeof(uint64_t),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_info_pos, pos.data(), pos.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
        free_code(c);
        return PBP_EDEVICE;
    }
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount,
                              c->device) != hipSuccess) {
        free_code(c);
        return PBP_EDEVICE;
    }
    if (c->m == pbp::r10::M) {
        uint64_t fzw[4 * pbp::r10::Q];
        pbp::r10::frozen_words(c->frozen.data(), fzw);
        if (hipMalloc(&c->d_fzw10, sizeof(fzw)) != hipSuccess) {
            free_code(c);
            return PBP_ENOMEM;
        }
        if (hipMemcpy(c->d_fzw10, fzw, sizeof(fzw), hipMemcpyHostToDevice) !=
            hipSuccess) {
            free_code(c);
            return PBP_EDEVICE;
        }
    }
    if (c->m > pbp::kMaxOnChipLog) {
        // message state of codes too long for the chip: one slot per resident
        // workgroup, (m + 1) columns of N floats each, in the workspace of
        // the decoding stream.  The workgroups hold the working R column and
        // two bit words per 64 rows in LDS, so as many as fit in 160 KB (at
        // most 4) are resident per compute unit.
        const int64_t lds = 4 * (int64_t)N + 16 * (int64_t)(N / 64) + 128;
        int64_t per_cu = (160 * 1024) / lds;
        per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
        c->state_slots = (int64_t)c->cus * per_cu;
        c->state_floats_per_slot = (int64_t)(c->m + 1) * N;
    }
    *out = c;
    return PBP_OK;
}

extern "C" void pbp_code_destroy(pbp_code *code)
{
    if (!code)
        return;
    const int dev = code->device;
    int prev = dev;
    if (hipGetDevice(&prev) == hipSuccess && prev != dev)
        (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    free_code(code);
    if (prev != dev)
        (void)hipSetDevice(prev);
}

// ---- Per-stream workspaces -------------------------------------------------

namespace {

struct WsEntry {
    int *counter = nullptr;
    float *state = nullptr;
    int64_t state_floats = 0;   // capacity of state
};

std::mutex g_ws_mu;
std::map<std::pair<int, uintptr_t>, WsEntry> g_ws;

// Run fn with `dev` current, restoring the caller's device afterwards.
template <class Fn>
int32_t on_device(int dev, Fn fn)
{
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess)
        return PBP_EDEVICE;
    if (prev != dev && hipSetDevice(dev) != hipSuccess)
        return PBP_EDEVICE;
    const int32_t st = fn();
    if (prev != dev)
        (void)hipSetDevice(prev);
    return st;
}

}  // namespace

int32_t pbp::stream_workspace(const pbp_code *code, hipStream_t stream,
                              Workspace *out)
{
    const int64_t need = code->state_slots * code->state_floats_per_slot;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    WsEntry *e;
    try {
        e = &g_ws[{code->device, reinterpret_cast<uintptr_t>(stream)}];
    } catch (const std::bad_alloc &) {
        return PBP_ENOMEM;
    }
    const int32_t st = on_device(code->device, [&]() -> int32_t {
        if (!e->counter) {
            // zero here; each persistent launch's last wave rewinds it
            if (hipMalloc(&e->counter, 2 * sizeof(int)) != hipSuccess) {
                e->counter = nullptr;
                return PBP_ENOMEM;
            }
            if (hipMemset(e->counter, 0, 2 * sizeof(int)) != hipSuccess ||
                hipDeviceSynchronize() != hipSuccess)
                return PBP_EDEVICE;
        }
        if (need > e->state_floats) {
            // earlier calls on this stream may still read the old slots
            if (e->state) {
                if (hipStreamSynchronize(stream) != hipSuccess)
                    return PBP_EDEVICE;
                (void)hipFree(e->state);
                e->state = nullptr;
                e->state_floats = 0;
            }
            if (hipMalloc(&e->state, sizeof(float) * need) != hipSuccess) {
                e->state = nullptr;
                return PBP_ENOMEM;
            }
            e->state_floats = need;
        }
        return PBP_OK;
    });
    if (st != PBP_OK)
        return st;
    out->counter = e->counter;
    out->state = e->state;
    return PBP_OK;
}

extern "C" int32_t pbp_workspace_release(void *stream)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return PBP_EDEVICE;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto it = g_ws.find({dev, reinterpret_cast<uintptr_t>(stream)});
    if (it == g_ws.end())
        return PBP_OK;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return PBP_EDEVICE;
    if (it->second.counter)
        (void)hipFree(it->second.counter);
    if (it->second.state)
        (void)hipFree(it->second.state);
    g_ws.erase(it);
    return PBP_OK;
}

extern "C" int32_t pbp_code_dims(const pbp_code *code, int32_t *N, int32_t *K)
{
    if (!code)
        return PBP_EINVAL;
    if (N)
        *N = code->N;
    if (K)
        *K = code->K;
    return PBP_OK;
}
