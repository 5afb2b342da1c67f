// Streaming community detection (Section 3.2 rule, Section 3.2.1 / Algorithm 3 passes),
// batch-synchronous form.  Per chunk of the edge stream:
//   kernel A  = apply(previous chunk) + counter increments(this chunk)
//   kernel B  = decide(this chunk): every edge reads the chunk-end counters and the
//               chunk-start labels and proposes with a 64-bit atomicMin keyed by its
//               stream index (smallest index wins)
// The apply of chunk k only touches labels/proposal slots and the increments of chunk
// k+1 only touch counters, so the two are fused into one launch.
//
// Per-node state is one 16-byte record {counter, label, proposal}: the counter
// atomics, the decision gathers and the proposal atomic of a node hit one cache line.
#include "common.h"

namespace bgv {

struct __align__(16) NodeState {
    int32_t cnt;     // degree counter (accumulates over passes)
    int32_t label;   // community label
    uint64_t win;    // smallest (edge index << 32 | proposed label) this chunk, ~0 if none
};
static_assert(sizeof(NodeState) == 16, "node record must be 16 bytes");

constexpr int kCdThreads = 256;
constexpr uint64_t kNoProposal = ~0ull;

__global__ void __launch_bounds__(kCdThreads) k_cd_init(NodeState *st, int32_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        NodeState s;
        s.cnt = 0;
        s.label = (int32_t)v;
        s.win = kNoProposal;
        st[v] = s;
    }
}

// Apply the winning proposals of chunk [ps, pe) (prop[i-ps] = proposing target or -1),
// then add the counter increments of chunk [cs, ce).
__global__ void __launch_bounds__(kCdThreads) k_cd_apply_hist(NodeState *__restrict__ st,
                                                               const int2 *__restrict__ edges,
                                                               const int32_t *__restrict__ prop,
                                                               int64_t ps, int64_t pe, int64_t cs, int64_t ce) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = ps + tid; i < pe; i += stride) {
        const int32_t x = prop[i - ps];
        if (x >= 0) {
            const uint64_t w = st[x].win;
            if ((int64_t)(w >> 32) == i) {
                st[x].label = (int32_t)(uint32_t)(w & 0xffffffffu);
                st[x].win = kNoProposal;
            }
        }
    }
    for (int64_t i = cs + tid; i < ce; i += stride) {
        const int2 e = edges[i];
        if (e.x != e.y) {
            atomicAdd(&st[e.x].cnt, 1);
            atomicAdd(&st[e.y].cnt, 1);
        }
    }
}

__global__ void __launch_bounds__(kCdThreads) k_cd_decide(NodeState *__restrict__ st,
                                                           const int2 *__restrict__ edges,
                                                           int32_t *__restrict__ prop, int64_t cs, int64_t ce,
                                                           int32_t D) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = cs + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ce; i += stride) {
        const int2 e = edges[i];
        int32_t target = -1;
        if (e.x != e.y) {
            const int2 su = *reinterpret_cast<const int2 *>(&st[e.x]);  // {cnt, label}
            const int2 sv = *reinterpret_cast<const int2 *>(&st[e.y]);
            if (su.x <= D && sv.x <= D && su.x != sv.x) {
                const bool u_low = su.x < sv.x;
                target = u_low ? e.x : e.y;
                const int32_t lab = u_low ? sv.y : su.y;
                atomicMin(reinterpret_cast<unsigned long long *>(&st[target].win),
                          (unsigned long long)(((uint64_t)i << 32) | (uint32_t)lab));
            }
        }
        prop[i - cs] = target;
    }
}

__global__ void __launch_bounds__(kCdThreads) k_cd_finish(const NodeState *__restrict__ st, int32_t n,
                                                           int32_t passes, int32_t *__restrict__ labels,
                                                           int32_t *__restrict__ degree,
                                                           unsigned long long *__restrict__ volume) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int2 s = *reinterpret_cast<const int2 *>(&st[v]);
        const int32_t d = s.x / passes;
        labels[v] = s.y;
        degree[v] = d;
        if (volume && d) atomicAdd(&volume[s.y], (unsigned long long)d);
    }
}

static int32_t pass_threshold(int32_t D1, int32_t growth, int32_t p) {
    int64_t D = D1;
    for (int32_t k = 0; k < p; ++k) {
        D *= growth;
        if (D > INT32_MAX) return INT32_MAX;
    }
    return (int32_t)D;
}

static bool cd_valid(int32_t n, int64_t m, const bgv_cd_params *p) {
    return p && n >= 1 && m >= 0 && m <= INT32_MAX && p->threshold >= 0 && p->passes >= 1 && p->growth >= 1 &&
           p->chunk >= 1 && p->reserved == 0;
}

static size_t cd_layout(Carver &c, int32_t n, int64_t m, const bgv_cd_params *p, NodeState **st, int32_t **prop) {
    *st = c.take<NodeState>((size_t)n);
    const int64_t b = p->chunk < m ? p->chunk : m;
    *prop = c.take<int32_t>((size_t)(b > 0 ? b : 1));
    return c.size();
}

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_community_workspace(int32_t n, int64_t m, const bgv_cd_params *p) {
    if (!cd_valid(n, m, p)) return 0;
    Carver c(nullptr);
    NodeState *st;
    int32_t *prop;
    return cd_layout(c, n, m, p, &st, &prop);
}

extern "C" bgv_status bgv_community(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                                    int32_t *labels, int32_t *degree, int64_t *volume, void *ws,
                                    size_t ws_bytes, bgv_stream_t stream) {
    clear_error();
    if (!cd_valid(n, m, p)) {
        set_error("bgv_community: invalid arguments (n=%d m=%lld)", n, (long long)m);
        return BGV_E_INVALID;
    }
    if ((m > 0 && !edges) || !labels || !degree) {
        set_error("bgv_community: null pointer");
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_community_workspace(n, m, p)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Carver c(ws);
    NodeState *st;
    int32_t *prop;
    cd_layout(c, n, m, p, &st, &prop);
    const int2 *e2 = reinterpret_cast<const int2 *>(edges);

    BGV_LAUNCH(k_cd_init, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, st, n);
    if (volume) BGV_TRY(fill<int64_t>(volume, 0, n, s));

    const int64_t B = p->chunk;
    const int64_t nchunk = (m + B - 1) / B;
    int64_t ps = 0, pe = 0;  // pending (not yet applied) chunk
    for (int32_t pass = 0; pass < p->passes && m > 0; ++pass) {
        const int32_t D = pass_threshold(p->threshold, p->growth, pass);
        for (int64_t k = 0; k < nchunk; ++k) {
            const int64_t cs = k * B, ce = (cs + B < m) ? cs + B : m;
            const int64_t work = (pe - ps) > (ce - cs) ? (pe - ps) : (ce - cs);
            BGV_LAUNCH(k_cd_apply_hist, dim3(grid_for(work, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                               st, e2, prop, ps, pe, cs, ce);
            BGV_LAUNCH(k_cd_decide, dim3(grid_for(ce - cs, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                               st, e2, prop, cs, ce, D);
            ps = cs;
            pe = ce;
        }
    }
    if (pe > ps) {
        BGV_LAUNCH(k_cd_apply_hist, dim3(grid_for(pe - ps, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                           st, e2, prop, ps, pe, (int64_t)0, (int64_t)0);
    }
    BGV_LAUNCH(k_cd_finish, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, st, n, p->passes,
                       labels, degree, reinterpret_cast<unsigned long long *>(volume));
    return BGV_OK;
}
