// Streaming community detection (Section 3.2 rule, Section 3.2.1 / Algorithm 3 passes),
// batch-synchronous form: per chunk of the edge stream, every edge reads its endpoints'
// counters at the end of the chunk and their labels at its start; an edge whose two
// counters are at most the pass threshold and differ proposes that the endpoint with
// the smaller counter join the other's community, and of the proposals to one node the
// one from the smallest stream index wins.
//
// Three implementations give the same integers: the two chunk-by-chunk forms below
// and, for many chunks, the back-pointer resolution of community_jump.hip (no barrier
// per chunk; chosen by bgv_cd_params.method).
//
// Bucketed (n <= 2^24): counters and labels in two int32 arrays and no global atomics.
// Nodes fall into buckets of 2^kB consecutive ids (kB = cd_bucket_bits(n)).
//   group (pass 0)  each 2048-edge tile of a chunk writes its endpoints grouped by
//                   bucket, one segment per (tile, bucket), offsets in a per-tile table
//   decide          each 2048-edge tile writes its proposals (target, stream index,
//                   label) grouped by the target's bucket in the same way
//   resolve         one workgroup per bucket reads its segments from every tile: the
//                   smallest proposing index per target by LDS atomicMin, the winners'
//                   labels written, and in pass 0 the next chunk's counter increments
//                   summed in LDS and added to the records, which no other workgroup
//                   touches.
// Per chunk: resolve(previous proposals, this chunk's increments), then one launch that
// decides this chunk and, in pass 0, groups the next chunk's endpoints.
// Device-scope atomics run at a small fraction of the LDS rate on this chip, and the
// grouping costs two coalesced streams per chunk instead.
//
// Atomic (larger n): one 16-byte record {counter, label, proposal} per node;
//   kernel A  = apply(previous chunk) + counter atomics(this chunk, pass 0 only)
//   kernel B  = decide(this chunk), proposals by a 64-bit atomicMin keyed by the
//               stream index.
#include <algorithm>
#include <type_traits>

#include "block_scan.h"
#include "common.h"
#include "community_jump.h"

namespace bgv {

struct __align__(16) NodeState {
    int32_t cnt;     // degree counter (accumulates over passes)
    int32_t label;   // community label
    uint64_t win;    // smallest (edge index << 32 | proposed label) this chunk, ~0 if none
};
static_assert(sizeof(NodeState) == 16, "node record must be 16 bytes");

constexpr int kCdThreads = 1024;
constexpr uint64_t kNoProposal = ~0ull;

// Records: counter 0, label lab0[v] (a resumed run's labels) or v, no proposal.
__global__ void __launch_bounds__(kCdThreads) k_cd_init(NodeState *st, int32_t n, const int32_t *__restrict__ lab0) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        NodeState s;
        s.cnt = 0;
        s.label = lab0 ? lab0[v] : (int32_t)v;
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
                                                           int64_t cs, int64_t ce, int32_t D, int32_t pass,
                                                           int32_t tie) {
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
            if (cu <= D && cv <= D && (cu != cv || tie)) {
                const bool u_low = cu <= cv;  // a tie (rule 1): the first endpoint joins
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
// Records are kRecInts int32 apart ({counter, label} first).
template <int kRecInts>
__global__ void __launch_bounds__(kCdThreads) k_cd_finish(const int32_t *__restrict__ st, int32_t n,
                                                           int32_t *__restrict__ labels, int32_t *__restrict__ degree,
                                                           unsigned long long *__restrict__ volume) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int2 s = *reinterpret_cast<const int2 *>(st + kRecInts * v);
        labels[v] = s.y;
        degree[v] = s.x;
        if (volume && s.x) atomicAdd(&volume[s.y], (unsigned long long)s.x);
    }
}

// ------------------------------------------------------------ bucketed path -------
// Buckets of 2^12 consecutive node ids, or 2^13 from 2^21 nodes on: larger buckets halve
// the (tile, bucket) segments each resolve walks but leave half as many resolve
// workgroups (measured over the community passes and sketch: 3.2M nodes and 34M edges,
// 13 bits 0.33 ms faster; 1M nodes and 10M edges, 12 bits 0.13 ms faster).
constexpr int32_t kCdMaxNodes = 1 << 24;           // bucketed path up to here
constexpr int32_t kCdMaxBuckets = kCdMaxNodes >> 12;  // bucket histogram held in LDS
inline int cd_bucket_bits(int32_t n) { return n >= (1 << 21) ? 13 : 12; }
// 2048-edge tiles of 1024 threads x 2 edges: fewer segments per resolve than 1024-edge
// tiles, and shorter per-thread chains in the decide than 256 x 8 or 512 x 4 (community
// passes on a 10M-edge stream: 0.87 ms; 256 x 8: 0.94; 256 x 4: 0.98; 256 x 16: 1.06)
constexpr int kCdItems = 2;
constexpr int32_t kCdTile = kCdThreads * kCdItems;  // edges per tile

inline int32_t cd_buckets(int32_t n, int bits) { return (int32_t)(((int64_t)n + (1 << bits) - 1) >> bits); }
inline bool cd_bucketed(int32_t n) { return n <= kCdMaxNodes; }

// Tile-local grouping by bucket: hist[0, nb) holds each bucket's entry count; turns it
// into exclusive offsets in place, writes them (and the total at [nb]) to the tile's
// table row, and returns the total.
__device__ __forceinline__ uint32_t cd_offsets(uint32_t *hist, int32_t nb, uint32_t *__restrict__ row) {
    const int32_t per = (nb + kCdThreads - 1) / kCdThreads;
    const int32_t b0 = min(nb, (int32_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    uint32_t sum = 0;
    for (int32_t b = b0; b < b1; ++b) sum += hist[b];
    uint32_t total;
    uint32_t run = block_excl_scan<uint32_t>(sum, &total);  // synchronises the block
    for (int32_t b = b0; b < b1; ++b) {
        const uint32_t c = hist[b];
        hist[b] = run;
        row[b] = run;
        run += c;
    }
    if (threadIdx.x == 0) row[nb] = total;
    __syncthreads();
    return total;
}

__global__ void __launch_bounds__(kCdThreads) k_cd_init_b(int32_t *cnt, int32_t *lab, int32_t n,
                                                           const int32_t *__restrict__ lab0, uint8_t *cnt8,
                                                           uint16_t *cnt16) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        cnt[v] = 0;
        if (cnt8) cnt8[v] = 0;
        if (cnt16) cnt16[v] = 0;
        lab[v] = lab0 ? lab0[v] : (int32_t)v;
    }
}

// Counting stops after pass 0, so each counter is d(v), the true degree.
__global__ void __launch_bounds__(kCdThreads) k_cd_finish_b(const int32_t *__restrict__ cnt,
                                                             const int32_t *__restrict__ lab, int32_t n,
                                                             int32_t *__restrict__ labels,
                                                             int32_t *__restrict__ degree,
                                                             unsigned long long *__restrict__ volume) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = cnt[v], l = lab[v];
        labels[v] = l;
        degree[v] = d;
        if (volume && d) atomicAdd(&volume[l], (unsigned long long)d);
    }
}

// Endpoints of the non-loop edges of tile `tile` of chunk [cs, ce), grouped by bucket:
// ends[tile * 2 * kCdTile + ...] holds their offsets within the bucket.
template <int kB>
__device__ __forceinline__ void cd_group_tile(const int2 *__restrict__ edges, int64_t cs, int64_t ce, int32_t tile,
                                              int32_t nb, uint16_t *__restrict__ ends, uint32_t *__restrict__ etab,
                                              uint32_t *hist, uint16_t *stage) {
    for (int32_t b = threadIdx.x; b < nb; b += kCdThreads) hist[b] = 0;
    __syncthreads();
    const int64_t t0 = cs + (int64_t)tile * kCdTile;
    int32_t node[2 * kCdItems];
    uint32_t rank[2 * kCdItems];
#pragma unroll
    for (int j = 0; j < kCdItems; ++j) {
        const int64_t i = t0 + j * kCdThreads + threadIdx.x;
        node[2 * j] = node[2 * j + 1] = -1;
        if (i < ce) {
            const int2 e = edges[i];
            if (e.x != e.y) {
                node[2 * j] = e.x;
                node[2 * j + 1] = e.y;
                rank[2 * j] = atomicAdd(&hist[e.x >> kB], 1u);
                rank[2 * j + 1] = atomicAdd(&hist[e.y >> kB], 1u);
            }
        }
    }
    __syncthreads();
    const uint32_t total = cd_offsets(hist, nb, etab + (int64_t)tile * (nb + 1));
#pragma unroll
    for (int q = 0; q < 2 * kCdItems; ++q)
        if (node[q] >= 0)
            stage[hist[node[q] >> kB] + rank[q]] = (uint16_t)(node[q] & ((1 << kB) - 1));
    __syncthreads();
    uint16_t *out = ends + (int64_t)tile * (2 * kCdTile);
    for (uint32_t k = threadIdx.x; k < total; k += kCdThreads) out[k] = stage[k];
}

// Decide, tile `tile` of chunk [cs, ce): the rule above (counters as in the atomic
// path's decide: pass-0 values stored per edge in c1 when more passes follow,
// p * d(v) + c1 in later passes), each proposal (offset of the target in its bucket,
// stream index, label) grouped by the target's bucket.  Counters and labels are
// separate arrays: every edge gathers two 4-byte counters (at a million nodes the
// counter array fits one XCD's L2), and only proposing edges gather a label.
// From pass 1 on every counter is known in closed form, so pass 1 (mode 2 with `mask`)
// also settles passes 2 .. 1 + nlater (thresholds in `later`): mask[i] holds, per such
// pass q, bit 2(q-2) = the edge proposes and bit 2(q-2)+1 = its first endpoint is the
// target.  Those passes (mode 3) read that byte instead of the stored counters and
// the two counter gathers.
struct CdLater {
    int32_t D[4];  // thresholds of passes 2..5
    int32_t n;     // how many of them the mask covers
};

// Whether a node whose degree is at least dlow (stored pass-0 counter c) could still
// pass the threshold of pass `pass` or of one of the passes the mask decides.
__device__ __forceinline__ bool cd_may_pass(int32_t dlow, int32_t c, int32_t pass, int32_t D, const CdLater &later,
                                            bool masked) {
    if (pass * dlow + c <= D) return true;
    if (masked)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < later.n && (q + 2) * dlow + c <= later.D[q]) return true;
    return false;
}

template <int kMode, int kB, typename CT>  // kMode 0: only pass; 1: pass 0 of several; 2: a later pass; 3: a pass in the mask
__device__ __forceinline__ void cd_decide_tile(const CT *__restrict__ cnt, const int32_t *__restrict__ exact,
                                               const int32_t *__restrict__ labv,
                                               const int2 *__restrict__ edges,
                                               int2 *__restrict__ c1, uint8_t *__restrict__ mask, CdLater later,
                                               int64_t cs, int64_t ce, int32_t D,
                                               int32_t pass, int32_t tie, int32_t tile, int32_t nb,
                                               uint3 *__restrict__ props, uint32_t *__restrict__ ptab,
                                               uint32_t *hist, uint3 *stage) {
    for (int32_t b = threadIdx.x; b < nb; b += kCdThreads) hist[b] = 0;
    __syncthreads();
    const int64_t t0 = cs + (int64_t)tile * kCdTile;
    int32_t target[kCdItems], lab[kCdItems];
    uint32_t rank[kCdItems];
#pragma unroll
    for (int j = 0; j < kCdItems; ++j) {
        const int64_t i = t0 + j * kCdThreads + threadIdx.x;
        target[j] = -1;
        if (i < ce) {
            const int2 e = edges[i];
            if (e.x != e.y) {
                bool go, u_low;
                if (kMode == 3) {
                    const uint32_t mb = (uint32_t)mask[i] >> (2 * (pass - 2));
                    go = mb & 1u;
                    u_low = (mb >> 1) & 1u;
                } else {
                    int32_t du = (int32_t)cnt[e.x], dv = (int32_t)cnt[e.y];
                    int2 c = make_int2(0, 0);
                    if (kMode == 2) c = c1[i];
                    if (kMode == 2 && sizeof(CT) == 1) {
                        // 255 stands for a degree of 255 or more: the exact degree is read
                        // only where such a degree could still pass a threshold
                        if (du == 255 && cd_may_pass(255, c.x, pass, D, later, mask != nullptr)) du = exact[e.x];
                        if (dv == 255 && cd_may_pass(255, c.y, pass, D, later, mask != nullptr)) dv = exact[e.y];
                    }
                    int32_t cu = du, cv = dv;
                    if (kMode == 1) c1[i] = make_int2(cu, cv);
                    if (kMode == 2) {
                        cu = pass * du + c.x;
                        cv = pass * dv + c.y;
                        if (mask) {
                            uint32_t mb = 0;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const int32_t a = (q + 2) * du + c.x, b = (q + 2) * dv + c.y;
                                if (q < later.n && a <= later.D[q] && b <= later.D[q] && (a != b || tie))
                                    mb |= (a <= b ? 3u : 1u) << (2 * q);
                            }
                            mask[i] = (uint8_t)mb;
                        }
                    }
                    go = cu <= D && cv <= D && (cu != cv || tie);
                    u_low = cu <= cv;  // a tie (rule 1): the first endpoint joins
                }
                if (go) {
                    target[j] = u_low ? e.x : e.y;
                    lab[j] = labv[u_low ? e.y : e.x];
                    rank[j] = atomicAdd(&hist[target[j] >> kB], 1u);
                }
            }
        }
    }
    __syncthreads();
    const uint32_t total = cd_offsets(hist, nb, ptab + (int64_t)tile * (nb + 1));
#pragma unroll
    for (int j = 0; j < kCdItems; ++j)
        if (target[j] >= 0)
            stage[hist[target[j] >> kB] + rank[j]] =
                make_uint3((uint32_t)(target[j] & ((1 << kB) - 1)),
                           (uint32_t)(t0 + j * kCdThreads + threadIdx.x), (uint32_t)lab[j]);
    __syncthreads();
    uint3 *out = props + (int64_t)tile * kCdTile;
    for (uint32_t k = threadIdx.x; k < total; k += kCdThreads) out[k] = stage[k];
}

// One launch per chunk: decide chunk [cs, ce) (kMode >= 0) and, in pass 0, group the
// endpoints of the next chunk [gs, ge) for the counter increments of the resolve that
// follows; workgroup x takes tile x of each.
template <int kMode, int kB, typename CT>  // kMode -1: grouping only
__global__ void __launch_bounds__(kCdThreads) k_cd_step(const CT *__restrict__ cnt,
                                                         const int32_t *__restrict__ exact,
                                                         const int32_t *__restrict__ labv,
                                                         const int2 *__restrict__ edges,
                                                         int2 *__restrict__ c1, uint8_t *__restrict__ mask,
                                                         CdLater later, int64_t cs, int64_t ce, int32_t D,
                                                         int32_t pass, int32_t tie, int32_t nb,
                                                         uint3 *__restrict__ props,
                                                         uint32_t *__restrict__ ptab, int64_t gs, int64_t ge,
                                                         uint16_t *__restrict__ ends, uint32_t *__restrict__ etab) {
    __shared__ uint32_t hist[kCdMaxBuckets];
    __shared__ uint3 pstage[kCdTile];
    __shared__ uint16_t estage[2 * kCdTile];
    const int32_t tile = (int32_t)blockIdx.x;
    if (kMode >= 0 && cs + (int64_t)tile * kCdTile < ce)  // uniform over the workgroup
        cd_decide_tile<kMode < 0 ? 0 : kMode, kB, CT>(cnt, exact, labv, edges, c1, mask, later, cs, ce, D, pass, tie,
                                                      tile, nb, props, ptab, hist, pstage);
    if (gs + (int64_t)tile * kCdTile < ge) {
        __syncthreads();  // hist is reused
        cd_group_tile<kB>(edges, gs, ge, tile, nb, ends, etab, hist, estage);
    }
}

// Resolve, one workgroup per bucket: proposals from ptiles decide tiles and counter
// increments from etiles grouped tiles.  The winner of a target is the smallest
// (stream index, label) key (stream indices are distinct), found by LDS atomicMin;
// then one sweep over the bucket's records writes the winners' labels and adds the
// counts.  Only this workgroup writes the bucket's records.  Each tile's segment goes
// to a group of `lanes` threads (a power of two: kCdResolveThreads / tiles, at least
// 1), which load its entries in batches before applying them, so that few tiles with
// long segments and many tiles with short ones both leave every thread few memory
// round trips.
constexpr int kCdResolveThreads = 1024;

// Workgroups are dealt to the chip's eight XCDs (each with its own L2) in turn, so
// workgroup x runs on XCD x mod 8.  Neighbouring buckets share cache lines of the
// offset rows and of the grouped segments (a tile writes its buckets' segments one
// after another), so the resolve gives each XCD a contiguous range of buckets: every
// line is then fetched into one L2 instead of into all eight.
constexpr int32_t kXcds = 8;
inline int32_t cd_resolve_grid(int32_t nb) { return (nb + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int32_t cd_resolve_bucket(int32_t x, int32_t nb) {
    return (x % kXcds) * ((nb + kXcds - 1) / kXcds) + x / kXcds;
}

inline int32_t cd_resolve_lanes(int32_t tiles, int32_t nb) {
    // an average endpoint segment (2 * kCdTile / nb entries) in one batch of eight loads
    // per lane, and at least about kCdResolveThreads / tiles lanes
    const int64_t seg = 2 * (int64_t)kCdTile / (nb > 0 ? nb : 1);
    int32_t g = 1;
    while (g < 64 && (int64_t)g * 8 < seg) g *= 2;
    while (g < kCdResolveThreads && (int64_t)g * 2 * (tiles > 0 ? tiles : 1) <= kCdResolveThreads) g *= 2;
    return g;
}

__device__ __forceinline__ void cd_segment(const uint32_t *__restrict__ tab, int32_t nb, int32_t t, int32_t b,
                                           uint32_t *q0, uint32_t *q1) {
    const uint32_t *row = tab + (int64_t)t * (nb + 1);
    *q0 = row[b];
    *q1 = row[b + 1];
}

// kEnds: the launch also adds grouped endpoint increments (pass 0); without them the
// workgroup needs no increment array and two fit a compute unit's LDS.
template <int kB, bool kEnds>
__global__ void __launch_bounds__(kCdResolveThreads) k_cd_resolve(int32_t *__restrict__ cnt,
                                                                   int32_t *__restrict__ lab, int32_t n, int32_t nb,
                                                                   const uint3 *__restrict__ props,
                                                                   const uint32_t *__restrict__ ptab, int32_t ptiles,
                                                                   const uint16_t *__restrict__ ends,
                                                                   const uint32_t *__restrict__ etab, int32_t etiles,
                                                                   int32_t lanes, uint8_t *__restrict__ cnt8,
                                                                   uint16_t *__restrict__ cnt16) {
    __shared__ unsigned long long win[1 << kB];
    __shared__ uint32_t inc[kEnds ? (1 << kB) : 1];
    const int32_t b = cd_resolve_bucket((int32_t)blockIdx.x, nb);
    if (b >= nb) return;  // the grid is rounded up to a multiple of the XCD count
    for (int32_t k = threadIdx.x; k < (1 << kB); k += kCdResolveThreads) {
        win[k] = ~0ull;
        if (kEnds) inc[k] = 0u;
    }
    __syncthreads();
    const int32_t tiles = max(ptiles, etiles);
    const int32_t groups = kCdResolveThreads / lanes;
    const uint32_t sub = threadIdx.x % lanes, L = (uint32_t)lanes;
    for (int32_t t = threadIdx.x / lanes; t < tiles; t += groups) {
        uint32_t p0 = 0, p1 = 0, e0 = 0, e1 = 0;
        if (t < ptiles) cd_segment(ptab, nb, t, b, &p0, &p1);
        if (t < etiles) cd_segment(etab, nb, t, b, &e0, &e1);
        const uint3 *ps = props + (int64_t)t * kCdTile;
        for (uint32_t q = p0 + sub; q < p1; q += 4 * L) {
            uint3 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u * L < p1) v[u] = ps[q + u * L];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u * L < p1) atomicMin(&win[v[u].x], ((unsigned long long)v[u].y << 32) | v[u].z);
        }
        if (!kEnds) continue;
        const uint16_t *es = ends + (int64_t)t * (2 * kCdTile);
        for (uint32_t q = e0 + sub; q < e1; q += 8 * L) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u * L < e1) v[u] = es[q + u * L];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u * L < e1) atomicAdd(&inc[v[u]], 1u);
        }
    }
    __syncthreads();
    const int64_t base = (int64_t)b << kB;
    const int32_t span = min(1 << kB, n - (b << kB));
    for (int32_t k = threadIdx.x; k < span; k += kCdResolveThreads) {
        const unsigned long long w = win[k];
        const uint32_t c = kEnds ? inc[k] : 0u;
        if (w != ~0ull) lab[base + k] = (int32_t)(uint32_t)w;
        if (c) {
            const int32_t v = cnt[base + k] + (int32_t)c;
            cnt[base + k] = v;
            if (cnt8) cnt8[base + k] = (uint8_t)min(v, 255);
            if (cnt16) cnt16[base + k] = (uint16_t)min(v, 65535);
        }
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
    if (!(p && n >= 1 && m >= 0 && m <= INT32_MAX && p->threshold >= 0 && p->passes >= 1 && p->growth >= 1 &&
          p->chunk >= 1 && p->method >= 0 && p->method <= 2 && (p->tie == 0 || p->tie == 1) &&
          (p->rule == 0 || p->rule == 1)))
        return false;
    if (p->rule == 1 && (p->tie != 0 || p->method == 2)) return false;
    return p->method != 2 || m == 0 || sq_fits(n, m, p);
}

// 1: chunk by chunk; 2: back-pointer resolution.  Automatic: measured on a 10M-edge
// stream, a chunk step costs about 12 us and back-pointer resolution about 150 us plus
// 0.09 ns more per (pass, edge) than the chunk steps' streaming, so the second wins past
// about 16 + passes * m / 2^17 chunk steps (245 at 3 x 10M edges, 16 on small graphs).
static int cd_method(int32_t n, int64_t m, const bgv_cd_params *p) {
    if (m == 0 || p->rule == 1) return 1;
    if (p->method != 0) return p->method;
    const int64_t steps = (int64_t)p->passes * ((m + p->chunk - 1) / p->chunk);
    return steps > 16 + ((int64_t)p->passes * m >> 17) && sq_fits(n, m, p) ? 2 : 1;
}

struct CdWs {
    NodeState *st;      // atomic path
    int32_t *prop;      // atomic path
    int32_t *cnt, *lab; // bucketed path: counters and labels
    uint8_t *cnt8;      // bucketed path: saturated copies of the counters (see cd_counter_widths)
    uint16_t *cnt16;
    uint3 *props;       // bucketed: proposals grouped per tile
    uint16_t *ends;     // bucketed: endpoints grouped per tile
    uint32_t *ptab, *etab;
    int2 *c1;
    uint8_t *mask;  // bucketed, passes > 2: decisions of passes 2..5 per edge
};

static size_t cd_layout(Carver &c, int32_t n, int64_t m, const bgv_cd_params *p, CdWs *w) {
    const int64_t b = p->chunk < m ? p->chunk : m;
    const size_t bb = (size_t)(b > 0 ? b : 1);
    *w = CdWs{};
    if (cd_bucketed(n)) {
        const size_t tiles = (bb + kCdTile - 1) / kCdTile;
        const size_t nb = (size_t)cd_buckets(n, 12);  // the larger of the two bucket counts
        w->cnt = c.take<int32_t>((size_t)n);
        w->cnt8 = c.take<uint8_t>((size_t)n);
        w->cnt16 = c.take<uint16_t>((size_t)n);
        w->lab = c.take<int32_t>((size_t)n);
        w->props = c.take<uint3>(tiles * kCdTile);
        w->ends = c.take<uint16_t>(tiles * 2 * kCdTile);
        w->ptab = c.take<uint32_t>(tiles * (nb + 1));
        w->etab = c.take<uint32_t>(tiles * (nb + 1));
    } else {
        w->st = c.take<NodeState>((size_t)n);
        w->prop = c.take<int32_t>(bb);
    }
    w->c1 = p->passes > 1 && m > 0 ? c.take<int2>((size_t)m) : nullptr;
    w->mask = cd_bucketed(n) && p->passes > 2 && m > 0 ? c.take<uint8_t>((size_t)m) : nullptr;
    return c.size();
}

// ------------------------------------------------------------ volume rule ----
// SCoDA's community-volume rule, batch-synchronous, on the per-node records plus
// V[label] (64-bit): per chunk
//   inc     counters and V of the chunk-start labels of both endpoints (atomics)
//   decide  both counters at most D and labels different: the endpoint whose
//           community has the smaller or equal V moves; proposals by a 64-bit
//           atomicMin keyed by the stream index
//   apply   winners take their label and carry their counter from the old V to the new
// Integer atomics only, so the result does not depend on timing.  Counters are raised
// in every pass (V needs the increments), so a counter ends at passes * d(v).
// Adds `v` to vol[key] for the active lanes of a wave with one atomic per distinct key
// (a few giant communities would otherwise serialise most of a chunk's atomics on a
// handful of addresses).  Called by every lane of the wave that is still running.
__device__ __forceinline__ void vr_wave_add(unsigned long long *vol, int32_t key, unsigned long long v, bool active) {
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t k = __shfl(key, leader, kWave);
        const uint64_t same = __ballot(active && key == k) & pending;
        unsigned long long sum = (same >> lane) & 1ull ? v : 0ull;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, kWave);
        if (lane == leader) atomicAdd(&vol[k], sum);
        pending &= ~same;
    }
}

// The grid-stride loops below advance whole workgroups together, so every lane of a
// wave reaches the wave-wide steps.
__global__ void __launch_bounds__(kCdThreads) k_vr_inc(NodeState *__restrict__ st, unsigned long long *vol,
                                                       const int2 *__restrict__ edges, int64_t cs, int64_t ce) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = cs + blockIdx.x * (int64_t)blockDim.x; b < ce; b += stride) {
        const int64_t i = b + threadIdx.x;
        const int2 e = i < ce ? edges[i] : make_int2(0, 0);
        const bool act = i < ce && e.x != e.y;
        int32_t lx = 0, ly = 0;
        if (act) {
            atomicAdd(&st[e.x].cnt, 1);
            atomicAdd(&st[e.y].cnt, 1);
            lx = st[e.x].label;
            ly = st[e.y].label;
        }
        vr_wave_add(vol, lx, 1ull, act);
        vr_wave_add(vol, ly, 1ull, act);
    }
}

__global__ void __launch_bounds__(kCdThreads) k_vr_decide(NodeState *__restrict__ st,
                                                          const unsigned long long *__restrict__ vol,
                                                          const int2 *__restrict__ edges, int32_t *__restrict__ prop,
                                                          int64_t cs, int64_t ce, int32_t D) {
    for (int64_t i = cs + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ce; i += (int64_t)gridDim.x * blockDim.x) {
        const int2 e = edges[i];
        int32_t target = -1;
        if (e.x != e.y) {
            const int2 su = *reinterpret_cast<const int2 *>(&st[e.x]);  // {counter, label}
            const int2 sv = *reinterpret_cast<const int2 *>(&st[e.y]);
            if (su.x <= D && sv.x <= D && su.y != sv.y) {
                const bool u_moves = vol[su.y] <= vol[sv.y];
                target = u_moves ? e.x : e.y;
                const int32_t lab = u_moves ? sv.y : su.y;
                atomicMin(reinterpret_cast<unsigned long long *>(&st[target].win),
                          (unsigned long long)(((uint64_t)i << 32) | (uint32_t)lab));
            }
        }
        prop[i - cs] = target;
    }
}

__global__ void __launch_bounds__(kCdThreads) k_vr_apply(NodeState *__restrict__ st, unsigned long long *vol,
                                                         const int32_t *__restrict__ prop, int64_t cs, int64_t ce) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = cs + blockIdx.x * (int64_t)blockDim.x; b < ce; b += stride) {
        const int64_t i = b + threadIdx.x;
        const int32_t x = i < ce ? prop[i - cs] : -1;
        bool won = false;
        int32_t old = 0, nw = 0;
        unsigned long long d = 0;
        if (x >= 0) {
            const uint64_t w = st[x].win;
            if ((int64_t)(w >> 32) == i) {
                won = true;
                old = st[x].label;
                nw = (int32_t)(uint32_t)(w & 0xffffffffu);
                d = (unsigned long long)st[x].cnt;
                st[x].label = nw;
                st[x].win = kNoProposal;
            }
        }
        vr_wave_add(vol, nw, d, won);
        vr_wave_add(vol, old, 0ull - d, won);
    }
}

__global__ void __launch_bounds__(kCdThreads) k_vr_finish(const NodeState *__restrict__ st, int32_t n, int32_t passes,
                                                          int32_t *__restrict__ labels, int32_t *__restrict__ degree,
                                                          unsigned long long *__restrict__ volume) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = st[v].cnt / passes, l = st[v].label;
        labels[v] = l;
        degree[v] = d;
        if (volume && d) atomicAdd(&volume[l], (unsigned long long)d);
    }
}

struct VrWs {
    NodeState *st;
    unsigned long long *vol;
    int32_t *prop;
};

static size_t vr_layout(Carver &c, int32_t n, int64_t m, const bgv_cd_params *p, VrWs *w) {
    const int64_t b = p->chunk < m ? p->chunk : m;
    VrWs t;
    t.st = c.take<NodeState>((size_t)n);
    t.vol = c.take<unsigned long long>((size_t)n);
    t.prop = c.take<int32_t>((size_t)(b > 0 ? b : 1));
    if (w) *w = t;
    return c.size();
}

static bgv_status vr_run(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p, int32_t *labels,
                         int32_t *degree, int64_t *volume, int32_t *pass_labels, int32_t first,
                         const int32_t *lab0, void *ws, hipStream_t s);

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_community_workspace(int32_t n, int64_t m, const bgv_cd_params *p) {
    if (!cd_valid(n, m, p)) return 0;
    Carver c(nullptr);
    if (cd_method(n, m, p) == 2) return sq_layout(c, n, m, p, nullptr);
    if (p->rule == 1) return vr_layout(c, n, m, p, nullptr);
    CdWs w;
    return cd_layout(c, n, m, p, &w);
}

namespace bgv {

__global__ void k_cd_copy_labels(const int32_t *__restrict__ src, int32_t stride, int32_t n,
                                 int32_t *__restrict__ dst) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        dst[v] = src[(int64_t)stride * v];
}

// Width of the counter copies the decisions gather.  A decision only compares counters
// with the pass threshold and with each other when both are within it, so a copy that
// saturates above every threshold decides the same: 16 bits when every threshold is
// below 65,535.  Pass 0 may use 8 bits when its own threshold is below 255 and no later
// pass p can accept an edge whose stored pass-0 counter c1 saturated: there the
// counter p*d(v) + c1 >= (p + 1) * c1 (c1 <= d(v)), so every threshold must be below
// (p + 1) * 255.  Later passes gather the 8-bit copy of the degrees and read the exact
// degree only where a saturated one (255 or more) could still pass a threshold
// (cd_may_pass).  Returns 8 (pass 0 in 8 bits), 16 or 32 (exact counters throughout).
static int cd_counter_widths(const bgv_cd_params *p, int32_t first) {
    const int64_t D0 = first > 0 ? -1 : p->threshold;
    bool w8 = D0 < 255, w16 = true;
    int64_t D = p->threshold;
    for (int32_t q = 0; q < p->passes; ++q) {
        if (q > 0) D = std::min<int64_t>(D * p->growth, INT32_MAX);
        if (D >= 65535) w16 = false;
        if (q > 0 && D >= (int64_t)(q + 1) * 255) w8 = false;
    }
    return w16 ? (w8 ? 8 : 16) : 32;
}

// The bucketed form, buckets of 2^kB node ids; the decisions of pass 0 gather counters
// of type C0 and those of later passes degrees of type C1 (uint8_t: the saturated copy
// with the exact degree read where needed; see cd_counter_widths).
template <int kB, typename C0, typename C1>
static bgv_status cd_run_bucketed(int32_t n, int64_t m, const int2 *e2, const bgv_cd_params *p, const CdWs &w,
                                  int32_t first, const int32_t *lab0, int32_t *labels, int32_t *degree,
                                  int64_t *volume, int32_t *pass_labels, hipStream_t s) {
    const int64_t B = p->chunk;
    const int64_t nchunk = (m + B - 1) / B;
    const int32_t nb = cd_buckets(n, kB);
    // one profiler name per kernel, whatever the bucket size
    const auto k_cd_resolve = bgv::k_cd_resolve<kB, true>;
    const auto k_cd_resolve_props = bgv::k_cd_resolve<kB, false>;  // no endpoint increments
    const auto k_cd_group = k_cd_step<-1, kB, int32_t>;
    const auto k_cd_step0 = k_cd_step<0, kB, C0>;
    const auto k_cd_step1 = k_cd_step<1, kB, C0>;
    const auto k_cd_step2 = k_cd_step<2, kB, C1>;
    const auto k_cd_step3 = k_cd_step<3, kB, int32_t>;
    // the counter arrays the decisions gather: the exact one, or a saturated copy that
    // the resolve keeps beside it
    uint8_t *const cnt8 = std::is_same<C0, uint8_t>::value || std::is_same<C1, uint8_t>::value ? w.cnt8 : nullptr;
    uint16_t *const cnt16 = std::is_same<C0, uint16_t>::value ? w.cnt16 : nullptr;
    const C0 *const g0 = std::is_same<C0, uint8_t>::value    ? reinterpret_cast<const C0 *>(w.cnt8)
                         : std::is_same<C0, uint16_t>::value ? reinterpret_cast<const C0 *>(w.cnt16)
                                                             : reinterpret_cast<const C0 *>(w.cnt);
    const C1 *const g1 = std::is_same<C1, uint8_t>::value ? reinterpret_cast<const C1 *>(w.cnt8)
                                                          : reinterpret_cast<const C1 *>(w.cnt);
    BGV_LAUNCH(k_cd_init_b, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, w.cnt, w.lab, n, lab0,
               cnt8, cnt16);
    int32_t ptiles = 0;  // decide tiles whose proposals are not yet resolved
    int32_t etiles = 0;  // grouped endpoint tiles whose increments are not yet added
    auto tiles_of = [&](int64_t k) {
        const int64_t len = (k + 1) * B < m ? B : m - k * B;
        return (int32_t)((len + kCdTile - 1) / kCdTile);
    };
    if (nchunk > 0) {
        // pass 0, chunk 0: its endpoints grouped before anything is decided
        etiles = tiles_of(0);
        BGV_LAUNCH(k_cd_group, dim3(etiles), dim3(kCdThreads), 0, s, w.cnt, w.cnt, w.lab, e2, w.c1,
                   (uint8_t *)nullptr, CdLater{}, (int64_t)0, (int64_t)0, 0, 0, 0, nb, w.props, w.ptab, (int64_t)0,
                   std::min<int64_t>(B, m), w.ends, w.etab);
    }
    // passes 2 .. 1 + later.n are decided in pass 1 (their counters are known there);
    // a run resumed after two or more passes has no pass 1 and decides each pass itself
    CdLater later{};
    later.n = w.mask && first <= 1 ? std::min(p->passes - 2, 4) : 0;
    for (int q = 0; q < later.n; ++q) later.D[q] = pass_threshold(p->threshold, p->growth, q + 2);
    for (int32_t pass = 0; pass < p->passes && (m > 0 || pass_labels); ++pass) {
        // resumed after `first` passes: pass 0 only counts (threshold -1: no edge
        // proposes), which yields the degrees and the per-edge pass-0 counters of the
        // closed form; passes 1 .. first-1 are skipped
        if (pass > 0 && pass < first) continue;
        const int32_t D = pass == 0 && first > 0 ? -1 : pass_threshold(p->threshold, p->growth, pass);
        for (int64_t k = 0; k < nchunk; ++k) {
            const int64_t cs = k * B, ce = (cs + B < m) ? cs + B : m;
            const int32_t tiles = tiles_of(k);
            // proposals of the previous chunk and, in pass 0, this chunk's increments
            if (etiles > 0)
                BGV_LAUNCH(k_cd_resolve, dim3(cd_resolve_grid(nb)), dim3(kCdResolveThreads), 0, s, w.cnt, w.lab, n, nb, w.props, w.ptab,
                           ptiles, w.ends, w.etab, etiles, cd_resolve_lanes(std::max(ptiles, etiles), nb), cnt8, cnt16);
            else if (ptiles > 0)
                BGV_LAUNCH(k_cd_resolve_props, dim3(cd_resolve_grid(nb)), dim3(kCdResolveThreads), 0, s, w.cnt, w.lab, n, nb,
                           w.props, w.ptab, ptiles, w.ends, w.etab, 0, cd_resolve_lanes(ptiles, nb), cnt8, cnt16);
            // counters are incremented in pass 0 only (later passes use the closed form):
            // the next chunk's endpoints are grouped by this launch in pass 0
            const bool group_next = pass == 0 && k + 1 < nchunk;
            const int64_t gs = group_next ? ce : 0, ge = group_next ? std::min<int64_t>(ce + B, m) : 0;
            const int32_t gtiles = group_next ? tiles_of(k + 1) : 0;
            const dim3 grid((unsigned)std::max(tiles, gtiles));
            if (p->passes == 1)
                BGV_LAUNCH(k_cd_step0, grid, dim3(kCdThreads), 0, s, g0, w.cnt, w.lab, e2, w.c1, (uint8_t *)nullptr,
                           later, cs, ce, D, pass, p->tie, nb, w.props, w.ptab, gs, ge, w.ends, w.etab);
            else if (pass == 0)
                BGV_LAUNCH(k_cd_step1, grid, dim3(kCdThreads), 0, s, g0, w.cnt, w.lab, e2, w.c1, (uint8_t *)nullptr,
                           later, cs, ce, D, pass, p->tie, nb, w.props, w.ptab, gs, ge, w.ends, w.etab);
            else if (pass >= 2 && pass < 2 + later.n)
                BGV_LAUNCH(k_cd_step3, grid, dim3(kCdThreads), 0, s, w.cnt, w.cnt, w.lab, e2, w.c1, w.mask, later, cs,
                           ce, D, pass, p->tie, nb, w.props, w.ptab, gs, ge, w.ends, w.etab);
            else
                BGV_LAUNCH(k_cd_step2, grid, dim3(kCdThreads), 0, s, g1, w.cnt, w.lab, e2, w.c1,
                           pass == 1 && later.n > 0 ? w.mask : (uint8_t *)nullptr, later, cs, ce, D, pass, p->tie,
                           nb, w.props, w.ptab, gs, ge, w.ends, w.etab);
            ptiles = tiles;
            etiles = gtiles;
        }
        if (pass_labels) {
            if (ptiles > 0)
                BGV_LAUNCH(k_cd_resolve_props, dim3(cd_resolve_grid(nb)), dim3(kCdResolveThreads), 0, s, w.cnt, w.lab, n,
                           nb, w.props, w.ptab, ptiles, w.ends, w.etab, 0, cd_resolve_lanes(ptiles, nb), cnt8, cnt16);
            ptiles = 0;
            BGV_LAUNCH(k_cd_copy_labels, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, w.lab, 1,
                       n, pass_labels + (int64_t)pass * n);
        }
    }
    if (ptiles > 0)
        BGV_LAUNCH(k_cd_resolve_props, dim3(cd_resolve_grid(nb)), dim3(kCdResolveThreads), 0, s, w.cnt, w.lab, n, nb,
                   w.props, w.ptab, ptiles, w.ends, w.etab, 0, cd_resolve_lanes(ptiles, nb), cnt8, cnt16);
    BGV_LAUNCH(k_cd_finish_b, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, w.cnt, w.lab, n,
               labels, degree, reinterpret_cast<unsigned long long *>(volume));
    return BGV_OK;
}

// The passes; with pass_labels, the labels after each pass are copied to row p (the
// last chunk's proposals are then resolved at the end of its pass rather than with the
// next pass's first chunk, which adds no counter increments, so nothing changes).
static bgv_status cd_run(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p, int32_t *labels,
                         int32_t *degree, int64_t *volume, int32_t *pass_labels, int32_t first,
                         const int32_t *lab0, void *ws, size_t ws_bytes, bgv_stream_t stream, const char *who) {
    clear_error();
    if (!cd_valid(n, m, p)) {
        set_error("%s: invalid arguments (n=%d m=%lld)", who, n, (long long)m);
        return BGV_E_INVALID;
    }
    if ((m > 0 && !edges) || !labels || !degree) {
        set_error("%s: null pointer", who);
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_community_workspace(n, m, p)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (range_check_on()) {
        BGV_TRY(check_edge_ids(n, m, edges, labels, s));  // labels[0]: overwritten below
        if (lab0) BGV_TRY(check_id_list(n, lab0, n, labels, s));
    }
    if (volume) BGV_TRY(fill<int64_t>(volume, 0, n, s));
    if (cd_method(n, m, p) == 2)
        return sq_run(n, m, edges, p, labels, degree, volume, pass_labels, first, lab0, ws, s);
    if (p->rule == 1) return vr_run(n, m, edges, p, labels, degree, volume, pass_labels, first, lab0, ws, s);
    Carver c(ws);
    CdWs w;
    cd_layout(c, n, m, p, &w);
    const int2 *e2 = reinterpret_cast<const int2 *>(edges);
    const int64_t B = p->chunk;
    const int64_t nchunk = (m + B - 1) / B;

    if (cd_bucketed(n)) {
        const int wd = cd_counter_widths(p, first);
        if (cd_bucket_bits(n) == 13) {
            if (wd == 8)
                return cd_run_bucketed<13, uint8_t, uint8_t>(n, m, e2, p, w, first, lab0, labels, degree, volume,
                                                              pass_labels, s);
            if (wd == 16)
                return cd_run_bucketed<13, uint16_t, uint8_t>(n, m, e2, p, w, first, lab0, labels, degree, volume,
                                                               pass_labels, s);
            return cd_run_bucketed<13, int32_t, int32_t>(n, m, e2, p, w, first, lab0, labels, degree, volume,
                                                         pass_labels, s);
        }
        if (wd == 8)
            return cd_run_bucketed<12, uint8_t, uint8_t>(n, m, e2, p, w, first, lab0, labels, degree, volume,
                                                          pass_labels, s);
        if (wd == 16)
            return cd_run_bucketed<12, uint16_t, uint8_t>(n, m, e2, p, w, first, lab0, labels, degree, volume,
                                                           pass_labels, s);
        return cd_run_bucketed<12, int32_t, int32_t>(n, m, e2, p, w, first, lab0, labels, degree, volume,
                                                     pass_labels, s);
    }

    NodeState *st = w.st;
    int32_t *prop = w.prop;
    int2 *c1 = w.c1;
    BGV_LAUNCH(k_cd_init, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s, st, n, lab0);
    int64_t ps = 0, pe = 0;  // pending (not yet applied) chunk
    for (int32_t pass = 0; pass < p->passes && (m > 0 || pass_labels); ++pass) {
        if (pass > 0 && pass < first) continue;  // resumed: as in the bucketed form above
        const int32_t D = pass == 0 && first > 0 ? -1 : pass_threshold(p->threshold, p->growth, pass);
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
                BGV_LAUNCH(k_cd_decide<0>, grid, dim3(kCdThreads), 0, s, st, e2, prop, c1, cs, ce, D, pass, p->tie);
            else if (pass == 0)
                BGV_LAUNCH(k_cd_decide<1>, grid, dim3(kCdThreads), 0, s, st, e2, prop, c1, cs, ce, D, pass, p->tie);
            else
                BGV_LAUNCH(k_cd_decide<2>, grid, dim3(kCdThreads), 0, s, st, e2, prop, c1, cs, ce, D, pass, p->tie);
            ps = cs;
            pe = ce;
        }
        if (pass_labels) {
            if (pe > ps)
                BGV_LAUNCH(k_cd_apply_hist, dim3(grid_for(pe - ps, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                           st, e2, prop, ps, pe, (int64_t)0, (int64_t)0);
            ps = pe = 0;
            BGV_LAUNCH(k_cd_copy_labels, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s,
                       reinterpret_cast<const int32_t *>(st) + 1, 4, n, pass_labels + (int64_t)pass * n);
        }
    }
    if (pe > ps) {
        BGV_LAUNCH(k_cd_apply_hist, dim3(grid_for(pe - ps, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s,
                           st, e2, prop, ps, pe, (int64_t)0, (int64_t)0);
    }
    BGV_LAUNCH(k_cd_finish<4>, dim3(grid_for(n, kCdThreads, 65536)), dim3(kCdThreads), 0, s,
               reinterpret_cast<const int32_t *>(st), n, labels, degree,
               reinterpret_cast<unsigned long long *>(volume));
    return BGV_OK;
}

static bgv_status vr_run(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p, int32_t *labels,
                         int32_t *degree, int64_t *volume, int32_t *pass_labels, int32_t first,
                         const int32_t *lab0, void *ws, hipStream_t s) {
    Carver c(ws);
    VrWs w;
    vr_layout(c, n, m, p, &w);
    const int2 *e2 = reinterpret_cast<const int2 *>(edges);
    const unsigned gn = grid_for(n, kCdThreads, 65536);
    BGV_LAUNCH(k_cd_init, dim3(gn), dim3(kCdThreads), 0, s, w.st, n, lab0);
    BGV_TRY(fill<uint64_t>(reinterpret_cast<uint64_t *>(w.vol), 0ull, n, s));
    const int64_t B = p->chunk;
    // a resumed run: after `first` passes every counter is first * d(v) and V[c] the sum
    // of the counters labelled c; the increments of `first` sweeps over the stream with
    // the labels held at lab0 build exactly that
    for (int32_t q = 0; q < first && m > 0; ++q)
        BGV_LAUNCH(k_vr_inc, dim3(grid_for(m, kCdThreads * 4, 16384)), dim3(kCdThreads), 0, s, w.st, w.vol, e2,
                   (int64_t)0, m);
    for (int32_t pass = first; pass < p->passes; ++pass) {
        const int32_t D = pass_threshold(p->threshold, p->growth, pass);
        for (int64_t cs = 0; cs < m; cs += B) {
            const int64_t ce = cs + B < m ? cs + B : m;
            const dim3 grid(grid_for(ce - cs, kCdThreads * 4, 16384));
            BGV_LAUNCH(k_vr_inc, grid, dim3(kCdThreads), 0, s, w.st, w.vol, e2, cs, ce);
            BGV_LAUNCH(k_vr_decide, grid, dim3(kCdThreads), 0, s, w.st, w.vol, e2, w.prop, cs, ce, D);
            BGV_LAUNCH(k_vr_apply, grid, dim3(kCdThreads), 0, s, w.st, w.vol, w.prop, cs, ce);
        }
        if (pass_labels)
            BGV_LAUNCH(k_cd_copy_labels, dim3(gn), dim3(kCdThreads), 0, s, reinterpret_cast<const int32_t *>(w.st) + 1,
                       4, n, pass_labels + (int64_t)pass * n);
    }
    BGV_LAUNCH(k_vr_finish, dim3(gn), dim3(kCdThreads), 0, s, w.st, n, p->passes, labels, degree,
               reinterpret_cast<unsigned long long *>(volume));
    return BGV_OK;
}

}  // namespace bgv

extern "C" bgv_status bgv_community(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                                    int32_t *labels, int32_t *degree, int64_t *volume, void *ws,
                                    size_t ws_bytes, bgv_stream_t stream) {
    return cd_run(n, m, edges, p, labels, degree, volume, nullptr, 0, nullptr, ws, ws_bytes, stream, "bgv_community");
}

extern "C" bgv_status bgv_community_resume(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                                           int32_t done, const int32_t *labels_in, int32_t *labels,
                                           int32_t *degree, int64_t *volume, void *ws, size_t ws_bytes,
                                           bgv_stream_t stream) {
    if (!p || done < 1 || done >= p->passes || !labels_in || labels_in == labels) {
        clear_error();
        set_error("bgv_community_resume: invalid arguments (done=%d, passes=%d, labels_in %p, labels %p)", done,
                  p ? p->passes : 0, (const void *)labels_in, (void *)labels);
        return BGV_E_INVALID;
    }
    return cd_run(n, m, edges, p, labels, degree, volume, nullptr, done, labels_in, ws, ws_bytes, stream,
                  "bgv_community_resume");
}

extern "C" bgv_status bgv_community_passes(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                                           int32_t *labels, int32_t *degree, int64_t *volume,
                                           int32_t *pass_labels, void *ws, size_t ws_bytes,
                                           bgv_stream_t stream) {
    if (!pass_labels) {
        clear_error();
        set_error("bgv_community_passes: null pointer");
        return BGV_E_INVALID;
    }
    return cd_run(n, m, edges, p, labels, degree, volume, pass_labels, 0, nullptr, ws, ws_bytes, stream,
                  "bgv_community_passes");
}
