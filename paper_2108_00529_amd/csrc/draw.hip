// Drawing attributes of the supernodes: radius by the square root of the size
// (Section 4.1) and 11 colour groups by size share (Section 4.3).
//   1. keys (size << b) | sid with b = bits for K: the stable LSD radix sort orders the
//      supernodes by size, equal sizes by id
//   2. exclusive scan of the sorted sizes (uint64): each supernode's running total
//   3. per sorted position: the group from the running total, the radius from the size
#include "common.h"

namespace bgv {

constexpr int kDrThreads = 256;

static int dr_bits(int32_t K) {
    int b = 1;
    while (b < 31 && (1 << b) < K) ++b;
    return b;
}

__global__ void k_draw_keys(const uint32_t *__restrict__ size, int32_t K, int kb, uint64_t *__restrict__ keys) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        keys[i] = ((uint64_t)size[i] << kb) | (uint64_t)i;
}

__global__ void k_draw_sizes(const uint64_t *__restrict__ skeys, int32_t K, int kb, uint64_t *__restrict__ ssize) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < K; q += (int64_t)gridDim.x * blockDim.x)
        ssize[q] = skeys[q] >> kb;
}

// Correctly rounded float square root of x >= 0: the hardware estimate (within an ulp)
// moved to the neighbour on the far side of a midpoint m when x lies beyond m^2.  A
// midpoint of two floats has at most 25 significant bits, so m^2 and the comparison
// are exact in FP64, and x is never exactly m^2 (that would need more bits than x has).
__device__ __forceinline__ float dr_sqrt_rn(float x) {
    float s = __builtin_sqrtf(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float up = __uint_as_float(__float_as_uint(s) + 1u);
        const float dn = s > 0.f ? __uint_as_float(__float_as_uint(s) - 1u) : 0.f;
        const double mu = 0.5 * ((double)s + (double)up), md = 0.5 * ((double)s + (double)dn);
        if ((double)x > mu * mu)
            s = up;
        else if (s > 0.f && (double)x < md * md)
            s = dn;
    }
    return s;
}

// Group of the supernode at sorted position q with running total P (itself included):
// 0 when 2P <= alpha, else ceil(10 * (2P - alpha) / alpha) (at most 10); the product
// is formed in 128 bits.
__global__ void k_draw_groups(const uint64_t *__restrict__ skeys, const uint64_t *__restrict__ excl,
                              const uint64_t *__restrict__ total, int32_t K, int kb, int32_t *__restrict__ group,
                              float *__restrict__ radius) {
    const uint64_t alpha = *total;
    const uint64_t mask = (1ull << kb) - 1ull;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < K; q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = skeys[q];
        const uint32_t sid = (uint32_t)(key & mask);
        const uint32_t sz = (uint32_t)(key >> kb);
        const uint64_t P = excl[q] + sz;
        int32_t g = 0;
        if (2 * P > alpha) {
            const unsigned __int128 num = (unsigned __int128)10 * (2 * P - alpha);
            const uint64_t c = (uint64_t)((num + alpha - 1) / alpha);
            g = c < 1 ? 1 : (c > 10 ? 10 : (int32_t)c);
        }
        group[sid] = g;
        radius[sid] = dr_sqrt_rn(__uint2float_rn(sz));
    }
}

struct DrWs {
    uint64_t *keys, *keys_alt, *ssize, *excl, *total;
    void *sort_scratch, *scan_scratch;
};

static size_t dr_layout(Carver &c, int32_t K, DrWs *w) {
    const size_t k = (size_t)(K > 0 ? K : 1);
    w->keys = c.take<uint64_t>(k);
    w->keys_alt = c.take<uint64_t>(k);
    w->ssize = c.take<uint64_t>(k);
    w->excl = c.take<uint64_t>(k);
    w->total = c.take<uint64_t>(1);
    w->sort_scratch = c.take<char>(radix_workspace((int64_t)k));
    w->scan_scratch = c.take<char>(scan_workspace((int64_t)k));
    return c.size();
}

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_draw_workspace(int32_t K) {
    if (K < 1) return 0;
    Carver c(nullptr);
    DrWs w;
    return dr_layout(c, K, &w);
}

extern "C" bgv_status bgv_draw_supernodes(int32_t K, const uint32_t *super_size, int32_t *group, float *radius,
                                          void *ws, size_t ws_bytes, bgv_stream_t stream) {
    clear_error();
    if (K < 1) {
        set_error("bgv_draw_supernodes: K must be >= 1 (got %d)", K);
        return BGV_E_INVALID;
    }
    if (!super_size || !group || !radius) {
        set_error("bgv_draw_supernodes: null pointer");
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_draw_workspace(K)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Carver c(ws);
    DrWs w;
    dr_layout(c, K, &w);
    const int kb = dr_bits(K);
    const unsigned g = grid_for(K, kDrThreads, 65536);
    BGV_LAUNCH(k_draw_keys, dim3(g), dim3(kDrThreads), 0, s, super_size, K, kb, w.keys);
    uint64_t *sk;
    BGV_TRY(radix_sort_u64(w.keys, w.keys_alt, nullptr, nullptr, K, 32 + kb, &sk, nullptr, w.sort_scratch, s));
    BGV_LAUNCH(k_draw_sizes, dim3(g), dim3(kDrThreads), 0, s, sk, K, kb, w.ssize);
    BGV_TRY(exclusive_scan<uint64_t>(w.ssize, w.excl, K, w.total, w.scan_scratch, s));
    BGV_LAUNCH(k_draw_groups, dim3(g), dim3(kDrThreads), 0, s, sk, w.excl, w.total, K, kb, group, radius);
    return BGV_OK;
}
