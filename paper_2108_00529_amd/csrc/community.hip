// Streaming community detection (Section 3.2 rule, Section 3.2.1 / Algorithm 3 passes),
// batch-synchronous form.  Per chunk of the edge stream:
//   kernel A  = apply(previous chunk) + counter increments(this chunk, pass 0 only)
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

// Decide phase.  Pass 0 reads the chunk-end counters from the node records; with more
// passes it also stores them per edge (c1[i] = counters of the two endpoints at the end
// of edge i's chunk in pass 0).  From pass 1 on, counters are no longer incremented: a
// node's counter at the end of chunk k of pass p is p * d(v) + its pass-0 value at the
// end of chunk k, where d(v) (the record's counter once pass 0 is complete) is the true
// degree, so the counter atomics of later passes are replaced by that closed form.
template <int kMode>  // 0: only pass; 1: pass 0 of several; 2: a later pass
__global__ void __launch_bounds__(kCdThreads) k_cd_decide(NodeState *__restrict__ st,
                                                           const int2 *__restrict__ edges,
                                                           int32_t *__restrict__ prop, int2 *__restrict__ c1,
                                                           int64_t cs, int64_t ce, int32_t D, int32_t pass) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = cs + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ce; i += stride) {
        const int2 e = edges[i];
        int32_t target = -1;
        if (e.x != e.y) {
            const int2 su = *reinterpret_cast<const int2 *>(&st[e.x]);  // {counter, label}
            const int2 sv = *reinterpret_cast<const int2 *>(&st[e.y]);
            int32_t cu = su.x, cv = sv.x;
            if (kMode == 1) c1[i] = make_int2(cu, cv);
            if (kMode == 2) {
                const int2 c = c1[i];
                cu = pass * su.x + c.x;
                cv = pass * sv.x + c.y;
            }
            if (cu <= D && cv <= D && cu != cv) {
                const bool u_low = cu < cv;
                target = u_low ? e.x : e.y;
                const int32_t lab = u_low ? sv.y : su.y;
                atomicMin(reinterpret_cast<unsigned long long *>(&st[target].win),
                          (unsigned long long)(((uint64_t)i << 32) | (uint32_t)lab));
            }
        }
        prop[i - cs] = target;
    }
}

// Counting stops after pass 0, so each record's counter is d(v), the true degree.
__global__ void __launch_bounds__(kCdThreads) k_cd_finish(const NodeState *__restrict__ st, int32_t n,
                                                           int32_t *__restrict__ labels, int32_t *__restrict__ degree,
                                                           unsigned long long *__restrict__ volume) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int2 s = *reinterpret_cast<const int2 *>(&st[v]);
        labels[v] = s.y;
        degree[v] = s.x;
        if (volume && s.x) atomicAdd(&volume[s.y], (unsigned long long)s.x);
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

static size_t cd_layout(Carver &c, int32_t n, int64_t m, const bgv_cd_params *p, NodeState **st, int32_t **prop,
                        int2 **c1) {
    *st = c.take<NodeState>((size_t)n);
    const int64_t b = p->chunk < m ? p->chunk : m;
    *prop = c.take<int32_t>((size_t)(b > 0 ? b : 1));
    *c1 = p->passes > 1 && m > 0 ? c.take<int2>((size_t)m) : nullptr;
    return c.size();
}

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_community_workspace(int32_t n, int64_t m, const bgv_cd_params *p) {
    if (!cd_valid(n, m, p)) return 0;
    Carver c(nullptr);
    NodeState *st;
    int32_t *prop;
    int2 *c1;
    return cd_layout(c, n, m, p, &st, &prop, &c1);
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
    int2 *c1;
    cd_layout(c, n, m, p, &st, &prop, &c1);
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
            // counters are incremented in pass 0 only (later passes use the closed form)
            const int64_t hs = pass == 0 ? cs : 0, he = pass == 0 ? ce : 0;
            const int64_t work = (pe - ps) > (he - hs) ? (pe - ps) : (he - hs);
            if (work > 0)
                BGV_LAUNCH(k_cd_apply_hist, dim3(grid_for(work, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                           st, e2, prop, ps, pe, hs, he);
            const dim3 grid(grid_for(ce - cs, kCdThreads * 4, 16384));
            if (p->passes == 1)
                BGV_LAUNCH(k_cd_decide<0>, grid, dim3(kCdThreads), 0, s, st, e2, prop, c1, cs, ce, D, pass);
            else if (pass == 0)
                BGV_LAUNCH(k_cd_decide<1>, grid, dim3(kCdThreads), 0, s, st, e2, prop, c1, cs, ce, D, pass);
            else
                BGV_LAUNCH(k_cd_decide<2>, grid, dim3(kCdThreads), 0, s, st, e2, prop, c1, cs, ce, D, pass);
            ps = cs;
            pe = ce;
        }
    }
    if (pe > ps) {
        BGV_LAUNCH(k_cd_apply_hist, dim3(grid_for(pe - ps, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                           st, e2, prop, ps, pe, (int64_t)0, (int64_t)0);
    }
    BGV_LAUNCH(k_cd_finish, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, st, n, labels, degree,
               reinterpret_cast<unsigned long long *>(volume));
    return BGV_OK;
}
