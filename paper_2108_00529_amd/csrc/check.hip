// Device-side id range checks (opt-in): a read-only scan of an id list that raises one
// flag, read back on the host before any kernel indexes by those ids.
#include <cstdlib>

#include "common.h"

namespace bgv {

constexpr int kChkThreads = 256;

// flag = 1 if any of the 2m ids of the int32 pairs lies outside [0, n).
__global__ void __launch_bounds__(kChkThreads) k_check_ids(const int2 *__restrict__ e, int64_t m, int32_t n,
                                                           int32_t *__restrict__ flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kChkThreads + threadIdx.x; i < m; i += (int64_t)gridDim.x * kChkThreads) {
        const int2 v = e[i];
        bad |= (uint32_t)v.x >= (uint32_t)n || (uint32_t)v.y >= (uint32_t)n;
    }
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) *flag = 1;
}

// flag = 1 if any of the n ids lies outside [0, bound).
__global__ void __launch_bounds__(kChkThreads) k_check_list(const int32_t *__restrict__ id, int64_t n, int32_t bound,
                                                            int32_t *__restrict__ flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kChkThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kChkThreads)
        bad |= (uint32_t)id[i] >= (uint32_t)bound;
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) *flag = 1;
}

// Concatenated graphs: the offsets start at 0, never decrease and end at the totals,
// and every edge of graph g has local ids in [0, n_g).  An offset error stops the id
// test (the graph of an edge is then undefined).
__global__ void __launch_bounds__(kChkThreads) k_check_batched(const int2 *__restrict__ e, int64_t m_total,
                                                               int64_t n_total, const int64_t *__restrict__ node_off,
                                                               const int64_t *__restrict__ edge_off, int32_t G,
                                                               int32_t *__restrict__ flag) {
    const int64_t tid = (int64_t)blockIdx.x * kChkThreads + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kChkThreads;
    bool bad = false;
    for (int64_t g = tid; g <= G; g += stride) {
        if (g == 0) bad |= node_off[0] != 0 || edge_off[0] != 0;
        if (g == G) bad |= node_off[G] != n_total || edge_off[G] != m_total;
        if (g > 0) bad |= node_off[g] < node_off[g - 1] || edge_off[g] < edge_off[g - 1];
        if (g > 0 && node_off[g] - node_off[g - 1] > INT32_MAX) bad = true;
    }
    if (__any(bad)) {
        if ((threadIdx.x & (kWave - 1)) == 0) *flag = 1;
        return;
    }
    for (int64_t i = tid; i < m_total; i += stride) {
        int32_t lo = 0, hi = G;  // the graph g with edge_off[g] <= i < edge_off[g + 1]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (edge_off[mid] <= i) lo = mid; else hi = mid;
        }
        const int64_t ng = node_off[lo + 1] - node_off[lo];
        const int2 v = e[i];
        bad |= v.x < 0 || v.y < 0 || (int64_t)v.x >= ng || (int64_t)v.y >= ng;
    }
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) *flag = 1;
}

bool range_check_on() {
    const char *v = std::getenv("BGV_CHECK");
    return v && v[0] == '1' && v[1] == '\0';
}

static bgv_status read_flag(int32_t *flag, hipStream_t s, const char *what) {
    int32_t h = 0;
    BGV_CHECK_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s));
    BGV_CHECK_HIP(hipStreamSynchronize(s));
    if (h) {
        set_error("%s", what);
        return BGV_E_RANGE;
    }
    return BGV_OK;
}

bgv_status check_edge_ids(int32_t n, int64_t m, const int32_t *edges, int32_t *flag, hipStream_t s) {
    BGV_TRY(fill<int32_t>(flag, 0, 1, s));
    if (m > 0)
        BGV_LAUNCH(k_check_ids, dim3(grid_for(m, kChkThreads, 4096)), dim3(kChkThreads), 0, s,
                   reinterpret_cast<const int2 *>(edges), m, n, flag);
    return read_flag(flag, s, "edge ids outside [0, n)");
}

bgv_status check_id_list(int64_t count, const int32_t *id, int32_t bound, int32_t *flag, hipStream_t s) {
    BGV_TRY(fill<int32_t>(flag, 0, 1, s));
    if (count > 0)
        BGV_LAUNCH(k_check_list, dim3(grid_for(count, kChkThreads, 4096)), dim3(kChkThreads), 0, s, id, count, bound,
                   flag);
    return read_flag(flag, s, "ids outside their range");
}

bgv_status check_batched_ids(int32_t G, int64_t n_total, int64_t m_total, const int64_t *node_off,
                             const int64_t *edge_off, const int32_t *edges, int32_t *flag, hipStream_t s) {
    BGV_TRY(fill<int32_t>(flag, 0, 1, s));
    BGV_LAUNCH(k_check_batched, dim3(grid_for(m_total > G ? m_total : G + 1, kChkThreads, 4096)), dim3(kChkThreads),
               0, s, reinterpret_cast<const int2 *>(edges), m_total, n_total, node_off, edge_off, G, flag);
    return read_flag(flag, s, "graph offsets inconsistent or local edge ids outside [0, n_g)");
}

}  // namespace bgv

using namespace bgv;

extern "C" bgv_status bgv_validate_edges(int32_t n, int64_t m, const int32_t *edges, int32_t *flag,
                                         bgv_stream_t stream) {
    clear_error();
    if (n < 1 || m < 0 || m > INT32_MAX || (m > 0 && !edges) || !flag) {
        set_error("bgv_validate_edges: invalid arguments (n=%d m=%lld)", n, (long long)m);
        return BGV_E_INVALID;
    }
    return check_edge_ids(n, m, edges, flag, reinterpret_cast<hipStream_t>(stream));
}
