// Batched form of the whole path: many independent graphs in one persistent launch.
// Each workgroup pops graphs from a queue (in the caller's order, e.g. largest first)
// and runs, with workgroup barriers only:
//   community passes (Section 3.2 rule, batch-synchronous chunks as in community.hip)
//   -> supernodes (ascending labels) -> sketch 1 in LDS -> inter-community keys ->
//   workgroup LSD radix sort -> superedges, sketch 2 in LDS, weights -> directed CSR ->
//   exact ForceAtlas2 iterations (Section 3.1 / Algorithm 1).
// The layout reproduces the plain exact path operation for operation: repulsion summed
// over j in order, the same per-row attraction wavefront, per-256-node partial sums of
// swing and traction in the plain kernels' fixed order, the same speed and move
// arithmetic (fa2_math.h).  Integer results equal the plain path's by construction.
#include "block_scan.h"
#include "common.h"
#include "fa2_math.h"
#include "sketch_hash.h"

namespace bgv {

constexpr int kBtMaxCells = 8192;  // rows*cols of a per-graph sketch, held in LDS
// Largest supergraph laid out by the multi-workgroup kernels after the persistent launch,
// and the repulsion segments it has at most (segment sums: that many per node).
constexpr int32_t kBtBigMax = 4096;
constexpr int32_t kBtMaxSeg = kBtBigMax / kRepSegment;

struct BtArgs {
    int32_t G;
    const int64_t *node_off, *edge_off;  // device, G+1
    const int32_t *order;                // device, G, or null for 0..G-1
    const int2 *edges;                   // concatenated, local ids
    int32_t threshold, passes, growth, tie;
    int64_t chunk;
    int32_t rows;
    uint32_t cols;
    HashRows h1, h2;
    int32_t iters;
    float kr, kg, tau, ks, ksmax;
    // outputs (per-node arrays at node_off, per-edge arrays at edge_off)
    int32_t *labels, *degree, *K, *E, *super_label;
    uint32_t *super_size;
    int2 *superedges;
    uint32_t *se_weight;
    float2 *pos, *fprev;
    float *speed;
    // workspace
    int32_t *cnt, *lab, *prop, *row_base;
    unsigned long long *win;
    uint32_t *sid, *row;
    uint64_t *keyA, *keyB;  // 2 * m_total each
    int2 *cw;               // 2 * m_total
    float *mass;
    float2 *F, *att;
    double2 *vpart;         // floor(n_total/256) + G + 1
    unsigned int *queue;
    // graphs with more than big_k and at most kBtBigMax supernodes are listed in
    // big[0, *nbig) and laid out afterwards by the k_bt_* kernels; 0: none
    int32_t big_k;
    int32_t *big;
    unsigned int *nbig;
};

// Exclusive scan of in[0, n) into out (may alias); returns the total.
template <int NT>
__device__ uint32_t wg_scan(const uint32_t *in, uint32_t *out, int64_t n) {
    uint32_t carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += NT) {
        const int64_t i = t0 + threadIdx.x;
        const uint32_t v = i < n ? in[i] : 0u;
        uint32_t tot;
        const uint32_t e = block_excl_scan<uint32_t>(v, &tot);
        if (i < n) out[i] = carry + e;
        carry += tot;
    }
    return carry;
}

// Stable LSD radix sort of keys[0, n) on bits [0, nbits) by one workgroup (8-bit digits;
// ranks within a round of NT keys from wavefront ballots).  Returns the buffer holding
// the result (keys or alt).
template <int NT>
__device__ uint64_t *wg_radix_sort(uint64_t *keys, uint64_t *alt, int64_t n, int nbits, uint32_t *hist,
                                   uint32_t *running, uint32_t (*wcnt)[256]) {
    constexpr int NW = NT / kWave;
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t *src = keys, *dst = alt;
    for (int shift = 0; shift < nbits; shift += 8) {
        for (int d = t; d < 256; d += NT) hist[d] = 0;
        __syncthreads();
        for (int64_t i = t; i < n; i += NT) atomicAdd(&hist[(uint32_t)(src[i] >> shift) & 255u], 1u);
        __syncthreads();
        uint32_t tot;
        const uint32_t e = block_excl_scan<uint32_t>(t < 256 ? hist[t] : 0u, &tot);
        if (t < 256) running[t] = e;
        for (int q = 0; q < NW; ++q)
            for (int d = t; d < 256; d += NT) wcnt[q][d] = 0;
        __syncthreads();
        for (int64_t r0 = 0; r0 < n; r0 += NT) {
            const int64_t i = r0 + t;
            const bool valid = i < n;
            const uint64_t key = valid ? src[i] : 0ull;
            const uint32_t d = (uint32_t)(key >> shift) & 255u;
            uint64_t match = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                match &= bit ? bb : ~bb;
            }
            const uint32_t rank = __popcll(match & lt);
            if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(match);
            __syncthreads();
            if (valid) {
                uint32_t p = running[d] + rank;
                for (int q = 0; q < w; ++q) p += wcnt[q][d];
                dst[p] = key;
            }
            __syncthreads();
            for (int d2 = t; d2 < 256; d2 += NT) {
                uint32_t add = 0;
                for (int q = 0; q < NW; ++q) {
                    add += wcnt[q][d2];
                    wcnt[q][d2] = 0;
                }
                running[d2] += add;
            }
            __syncthreads();
        }
        uint64_t *tmp = src;
        src = dst;
        dst = tmp;
    }
    return src;
}

__device__ __forceinline__ int32_t bt_threshold(int32_t D1, int32_t growth, int32_t p) {
    int64_t D = D1;
    for (int32_t k = 0; k < p; ++k) {
        D *= growth;
        if (D > INT32_MAX) return INT32_MAX;
    }
    return (int32_t)D;
}

template <int NT>
__global__ void __launch_bounds__(NT) k_batched(BtArgs a) {
    constexpr int NW = NT / kWave;
    constexpr int NV = NT / 256;  // 256-node groups handled side by side in the layout
    static_assert(NT % 256 == 0 && NT <= 1024, "workgroup of 256, 512 or 1024 threads");
    static_assert(NT % kRepSegment == 0 || kRepSegment % NT == 0, "segment boundaries fall on LDS tile halves");
    __shared__ uint32_t sk[kBtMaxCells];
    __shared__ uint32_t hist[256], running[256];
    __shared__ uint32_t wcnt[NW][256];
    __shared__ float4 tile[NT];
    __shared__ double2 ws[NW];
    __shared__ int s_g;
    __shared__ uint32_t s_count;
    __shared__ float s_speed;
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;

    for (;;) {
        if (t == 0) s_g = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int qi = s_g;
        __syncthreads();
        if (qi >= a.G) break;
        const int g = a.order ? a.order[qi] : qi;
        const int64_t n0 = a.node_off[g], e0 = a.edge_off[g];
        const int32_t n = (int32_t)(a.node_off[g + 1] - n0);
        const int64_t m = a.edge_off[g + 1] - e0;
        const int2 *edges = a.edges + e0;
        int32_t *cnt = a.cnt + n0, *lab = a.lab + n0, *prop = a.prop + e0;
        unsigned long long *win = a.win + n0;
        uint32_t *sid = a.sid + n0;

        // ---- community passes, chunk by chunk -------------------------------------
        for (int32_t v = t; v < n; v += NT) {
            cnt[v] = 0;
            lab[v] = v;
            win[v] = ~0ull;
        }
        __syncthreads();
        for (int32_t pass = 0; pass < a.passes; ++pass) {
            const int32_t D = bt_threshold(a.threshold, a.growth, pass);
            for (int64_t cs = 0; cs < m; cs += a.chunk) {
                const int64_t ce = cs + a.chunk < m ? cs + a.chunk : m;
                for (int64_t i = cs + t; i < ce; i += NT) {
                    const int2 e = edges[i];
                    if (e.x != e.y) {
                        __hip_atomic_fetch_add(&cnt[e.x], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_fetch_add(&cnt[e.y], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                __syncthreads();
                for (int64_t i = cs + t; i < ce; i += NT) {
                    const int2 e = edges[i];
                    int32_t target = -1;
                    if (e.x != e.y) {
                        const int32_t du = cnt[e.x], dv = cnt[e.y];
                        if (du <= D && dv <= D && (du != dv || a.tie)) {
                            const bool u_low = du <= dv;  // a tie (rule 1): the first endpoint joins
                            target = u_low ? e.x : e.y;
                            const int32_t l = u_low ? lab[e.y] : lab[e.x];
                            __hip_atomic_fetch_min(&win[target], ((unsigned long long)i << 32) | (uint32_t)l,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                    prop[i] = target;
                }
                __syncthreads();
                for (int64_t i = cs + t; i < ce; i += NT) {
                    const int32_t x = prop[i];
                    if (x >= 0) {
                        const unsigned long long wv = win[x];
                        if ((int64_t)(wv >> 32) == i) {
                            lab[x] = (int32_t)(uint32_t)(wv & 0xffffffffull);
                            win[x] = ~0ull;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int32_t v = t; v < n; v += NT) {
            a.labels[n0 + v] = lab[v];
            a.degree[n0 + v] = cnt[v] / a.passes;
            sid[v] = 0u;
        }
        __syncthreads();

        // ---- supernodes: distinct labels in ascending order ---------------------
        for (int32_t v = t; v < n; v += NT) sid[lab[v]] = 1u;
        __syncthreads();
        uint32_t *flag = reinterpret_cast<uint32_t *>(win);  // free after the passes
        for (int32_t v = t; v < n; v += NT) flag[v] = sid[v];
        __syncthreads();
        const uint32_t K = wg_scan<NT>(sid, sid, n);
        int kb = 1;
        while (kb < 31 && (1u << kb) < K) ++kb;
        for (int32_t c = t; c < n; c += NT)
            if (flag[c]) a.super_label[n0 + sid[c]] = c;
        const int32_t cells = a.rows * (int32_t)a.cols;
        for (int32_t c = t; c < cells; c += NT) sk[c] = 0u;
        __syncthreads();

        // ---- sketch 1: community weights ------------------------------------------
        for (int32_t v = t; v < n; v += NT) {
            const uint32_t d = (uint32_t)(cnt[v] / a.passes);
            if (d == 0) continue;
            const uint32_t l = (uint32_t)lab[v];
            for (int r = 0; r < a.rows; ++r) atomicAdd(&sk[r * a.cols + col_key(a.h1.a[r], a.h1.b[r], l, a.cols)], d);
        }
        __syncthreads();
        for (uint32_t k = t; k < K; k += NT) {
            const uint32_t l = (uint32_t)a.super_label[n0 + k];
            uint32_t best = 0xffffffffu;
            for (int r = 0; r < a.rows; ++r) best = min(best, sk[r * a.cols + col_key(a.h1.a[r], a.h1.b[r], l, a.cols)]);
            a.super_size[n0 + k] = best;
        }
        __syncthreads();  // every read of sketch 1 is done before it is cleared for sketch 2
        if (t == 0) s_count = 0u;
        for (int32_t c = t; c < cells; c += NT) sk[c] = 0u;
        __syncthreads();

        // ---- inter-community keys, sorted -----------------------------------------
        uint64_t *keyA = a.keyA + 2 * e0, *keyB = a.keyB + 2 * e0;
        for (int64_t i = t; i < m; i += NT) {
            const int2 e = edges[i];
            if (e.x == e.y) continue;
            const int32_t la = lab[e.x], lb = lab[e.y];
            if (la == lb) continue;
            const uint32_t lo = (uint32_t)min(la, lb), hi = (uint32_t)max(la, lb);
            const uint32_t at = atomicAdd(&s_count, 1u);
            keyA[at] = ((uint64_t)sid[lo] << kb) | (uint64_t)sid[hi];
        }
        __syncthreads();
        const uint32_t nk = s_count;
        __syncthreads();
        const uint64_t *sorted = wg_radix_sort<NT>(keyA, keyB, nk, 2 * kb, hist, running, wcnt);

        // ---- superedges: distinct keys, multiplicities into sketch 2, weights -----
        const uint64_t lowmask = (1ull << kb) - 1ull;
        int2 *se = a.superedges + e0;
        uint32_t *run = reinterpret_cast<uint32_t *>(prop);  // run starts; prop is free now
        uint32_t E = 0;
        for (int64_t t0 = 0; t0 < nk; t0 += NT) {
            const int64_t i = t0 + t;
            const bool first = i < nk && (i == 0 || sorted[i] != sorted[i - 1]);
            uint32_t tot;
            const uint32_t j = E + block_excl_scan<uint32_t>(first ? 1u : 0u, &tot);
            if (first) {
                const uint64_t k = sorted[i];
                se[j] = make_int2((int32_t)(k >> kb), (int32_t)(k & lowmask));
                run[j] = (uint32_t)i;
            }
            E += tot;
        }
        __syncthreads();
        for (uint32_t j = t; j < E; j += NT) {
            const uint32_t c = (j + 1 < E ? run[j + 1] : nk) - run[j];
            const uint32_t la = (uint32_t)a.super_label[n0 + se[j].x], lb = (uint32_t)a.super_label[n0 + se[j].y];
            for (int r = 0; r < a.rows; ++r)
                atomicAdd(&sk[r * a.cols + col_pair(a.h2.a[r], a.h2.b[r], a.h2.c[r], la, lb, a.cols)], c);
        }
        __syncthreads();
        for (uint32_t j = t; j < E; j += NT) {
            const uint32_t la = (uint32_t)a.super_label[n0 + se[j].x], lb = (uint32_t)a.super_label[n0 + se[j].y];
            uint32_t best = 0xffffffffu;
            for (int r = 0; r < a.rows; ++r)
                best = min(best, sk[r * a.cols + col_pair(a.h2.a[r], a.h2.b[r], a.h2.c[r], la, lb, a.cols)]);
            a.se_weight[e0 + j] = best;
        }
        if (t == 0) {
            a.K[g] = (int32_t)K;
            a.E[g] = (int32_t)E;
        }

        // ---- directed CSR of the supergraph (neighbours ascending) ----------------
        for (uint32_t j = t; j < E; j += NT) {
            const int2 p = se[j];
            keyA[2 * j] = ((uint64_t)(uint32_t)p.x << kb) | (uint32_t)p.y;
            keyA[2 * j + 1] = ((uint64_t)(uint32_t)p.y << kb) | (uint32_t)p.x;
        }
        __syncthreads();
        const uint64_t *dk = wg_radix_sort<NT>(keyA, keyB, 2 * (int64_t)E, 2 * kb, hist, running, wcnt);
        uint32_t *row = a.row + n0 + g;
        int2 *cw = a.cw + 2 * e0;
        const int64_t nent = 2 * (int64_t)E;
        for (int64_t k = t; k < nent; k += NT) {
            const uint64_t key = dk[k];
            const int64_t src = (int64_t)(key >> kb);
            cw[k] = make_int2((int32_t)(key & lowmask), __float_as_int(1.0f));
            const int64_t prev = k ? (int64_t)(dk[k - 1] >> kb) : -1;
            for (int64_t r = prev + 1; r <= src; ++r) row[r] = (uint32_t)k;
            if (k == nent - 1)
                for (int64_t r = src + 1; r <= (int64_t)K; ++r) row[r] = (uint32_t)nent;
        }
        if (nent == 0)
            for (uint32_t r = t; r <= K; r += NT) row[r] = 0u;
        __syncthreads();
        float *mass = a.mass + n0;
        for (uint32_t i = t; i < K; i += NT) mass[i] = (float)(row[i + 1] - row[i]) + 1.0f;
        if (a.big_k > 0 && a.iters > 0 && K > (uint32_t)a.big_k && K <= (uint32_t)kBtBigMax) {
            // a large supergraph is laid out by the multi-workgroup kernels afterwards,
            // so that it does not hold one compute unit for the whole layout
            if (t == 0) a.big[atomicAdd(a.nbig, 1u)] = g;
            __syncthreads();
            continue;
        }

        // ---- exact ForceAtlas2 iterations -------------------------------------------
        float2 *pos = a.pos + n0, *fprev = a.fprev + n0, *F = a.F + n0, *att = a.att + n0;
        double2 *vpart = a.vpart + (n0 / 256) + g;
        if (t == 0) s_speed = a.speed[g];
        __syncthreads();
        const int32_t nvb = (int32_t)((K + 255) / 256);
        for (int32_t it = 0; it < a.iters; ++it) {
            for (uint32_t i = w; i < K; i += NW) {
                const float2 f = fa2_row_attraction(pos, cw, row[i], row[i + 1], pos[i], lane);
                if (lane == 0) att[i] = f;
            }
            __syncthreads();
            for (int32_t vb0 = 0; vb0 < nvb; vb0 += NV) {
                const int32_t vb = vb0 + t / 256;
                const uint32_t i = (uint32_t)vb * 256u + (uint32_t)(t & 255);
                const bool live = vb < nvb && i < K;
                const float2 xi = live ? pos[i] : make_float2(0.f, 0.f);
                const float mi = live ? mass[i] : 0.f;
                // the plain kernels' order: segments of kRepSegment bodies, each summed
                // from zero, then added in order; a segment boundary can fall inside a tile
                float rx = 0.f, ry = 0.f, sx = 0.f, sy = 0.f;
                for (uint32_t j0 = 0; j0 < K; j0 += NT) {
                    const uint32_t j = j0 + t;
                    if (j < K) {
                        const float2 xj = pos[j];
                        tile[t] = make_float4(xj.x, xj.y, mass[j], 0.f);
                    }
                    __syncthreads();
                    const uint32_t c = min((uint32_t)NT, K - j0);
                    for (uint32_t q0 = 0; q0 < c;) {
                        const uint32_t jj = j0 + q0;
                        if (jj != 0 && jj % (uint32_t)kRepSegment == 0) {
                            if (jj == (uint32_t)kRepSegment) {
                                rx = sx;
                                ry = sy;
                            } else {
                                rx += sx;
                                ry += sy;
                            }
                            sx = sy = 0.f;
                        }
                        const uint32_t q1 = min(c, (jj / (uint32_t)kRepSegment + 1u) * (uint32_t)kRepSegment - j0);
                        const uint32_t n8 = (q1 - q0) & ~7u;  // groups of eight LDS reads in flight
                        fa2_rep_run(xi, tile + q0, (int)n8, sx, sy);
                        for (uint32_t q = q0 + n8; q < q1; ++q) fa2_rep_term(xi, tile[q], sx, sy);
                        q0 = q1;
                    }
                    __syncthreads();
                }
                if (K <= (uint32_t)kRepSegment) {
                    rx = sx;
                    ry = sy;
                } else {
                    rx += sx;
                    ry += sy;
                }
                double2 st = make_double2(0.0, 0.0);
                if (live) {
                    const float2 f = fa2_net_force(xi, mi, a.kr, rx, ry, att[i], a.kg);
                    F[i] = f;
                    st = fa2_swing_traction(f, fprev[i], mi);
                }
                st = fa2_sum256(st, ws);
                if ((t & 255) == 0 && vb < nvb) vpart[vb] = st;
            }
            __syncthreads();
            double2 acc = make_double2(0.0, 0.0);
            if (t < 256)
                for (int32_t p = t; p < nvb; p += 256) {
                    acc.x += vpart[p].x;
                    acc.y += vpart[p].y;
                }
            acc = fa2_sum256(acc, ws);
            if (t == 0) s_speed = fa2_global_speed(acc.x, acc.y, s_speed, a.tau);
            __syncthreads();
            const float s = s_speed;
            for (uint32_t i = t; i < K; i += NT) {
                const float2 f = F[i];
                pos[i] = fa2_move(pos[i], f, fprev[i], s, a.ks, a.ksmax);
                fprev[i] = f;
            }
            __syncthreads();
        }
        if (t == 0) a.speed[g] = s_speed;
        __syncthreads();
    }
}

// ---- layout of the listed large graphs, all of them per launch ------------------
// Work items are the listed graphs' CSR rows (attraction), (256-node tile, repulsion
// segment) pairs (repulsion) or tiles (segment sums, update), numbered through
// exclusive prefix sums over the list; an item finds its graph by a table made once
// per call.  Each graph goes through exactly the plain path's tile functions, so its
// result equals a plain layout of it bit for bit.
struct BtBig {
    const int64_t *node_off, *edge_off;
    const int32_t *K;
    const int32_t *big;
    const unsigned int *nbig;
    uint32_t *tile_off, *row_off;  // G+1 each: prefix sums of tiles / rows over the list
    uint32_t *fitem_off;           // G+1: prefix sums of wave tiles x segments over the list
    uint32_t *tile_slot;           // list slot of every tile item
    uint32_t *fitem_slot;          // list slot of every (wave tile, segment) item
    uint4 *row_desc;               // per row item: CSR entries [x, y) in cw, node z, graph base w
    const uint32_t *row;
    const int2 *cw;
    const float *mass;
    float2 *pos, *fprev, *F, *att;
    float2 *seg;                   // segment sums: kBtMaxSeg per node from the graph's first node
    double2 *vpart;
    float *speed;                  // caller's per-graph speeds (initial and final)
    float *bspeed;                 // 2 per graph: ping-pong across iterations
    float kr, kg, tau, ks, ksmax;
};

// Prefix sums of tiles, rows and (tile, segment) items over the list; initial speeds
// into the ping-pong pair.
__global__ void __launch_bounds__(1024) k_bt_plan(BtBig b) {
    const uint32_t nb = *b.nbig;
    uint32_t ct = 0, cr = 0, cf = 0;
    for (uint32_t s0 = 0; s0 < nb; s0 += 1024) {
        const uint32_t sl = s0 + threadIdx.x;
        uint32_t tiles = 0, rows = 0, fitems = 0;
        if (sl < nb) {
            const int32_t g = b.big[sl];
            rows = (uint32_t)b.K[g];
            tiles = (rows + kFa2Tile - 1) / kFa2Tile;
            fitems = ((rows + kWave - 1) / kWave) * (uint32_t)fa2_rep_segments((int32_t)rows);
            b.bspeed[2 * g] = b.speed[g];
        }
        uint32_t tt, tr, tf;
        const uint32_t et = block_excl_scan<uint32_t>(tiles, &tt);
        const uint32_t er = block_excl_scan<uint32_t>(rows, &tr);
        const uint32_t ef = block_excl_scan<uint32_t>(fitems, &tf);
        if (sl < nb) {
            b.tile_off[sl] = ct + et;
            b.row_off[sl] = cr + er;
            b.fitem_off[sl] = cf + ef;
        }
        ct += tt;
        cr += tr;
        cf += tf;
    }
    if (threadIdx.x == 0) {
        b.tile_off[nb] = ct;
        b.row_off[nb] = cr;
        b.fitem_off[nb] = cf;
    }
}

// Largest slot s with off[s] <= x (off ascending, off[0] = 0, x < off[nb]).
__device__ __forceinline__ uint32_t bt_slot(const uint32_t *off, uint32_t nb, uint32_t x) {
    uint32_t lo = 0, hi = nb;  // off[lo] <= x < off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Per-call maps: each row item's descriptor and each tile and (tile, segment) item's
// slot, found once instead of once per iteration.
__global__ void __launch_bounds__(kFa2Tile) k_bt_maps(BtBig b) {
    const uint32_t nb = *b.nbig;
    const uint32_t R = b.row_off[nb], T = b.tile_off[nb], FI = b.fitem_off[nb];
    const uint32_t stride = gridDim.x * kFa2Tile;
    for (uint32_t r = blockIdx.x * kFa2Tile + threadIdx.x; r < R; r += stride) {
        const uint32_t sl = bt_slot(b.row_off, nb, r);
        const int32_t g = b.big[sl];
        const uint32_t i = r - b.row_off[sl];
        const int64_t n0 = b.node_off[g];
        const uint32_t *row = b.row + n0 + g;
        const uint32_t c0 = (uint32_t)(2 * b.edge_off[g]);
        b.row_desc[r] = make_uint4(c0 + row[i], c0 + row[i + 1], (uint32_t)n0 + i, (uint32_t)n0);
    }
    for (uint32_t x = blockIdx.x * kFa2Tile + threadIdx.x; x < T; x += stride) b.tile_slot[x] = bt_slot(b.tile_off, nb, x);
    for (uint32_t x = blockIdx.x * kFa2Tile + threadIdx.x; x < FI; x += stride)
        b.fitem_slot[x] = bt_slot(b.fitem_off, nb, x);
}

// Repulsion of one (64-target wave tile, segment) item by one wavefront: the segment's
// bodies pass through the wavefront's own LDS slice 64 at a time and every lane adds
// them in ascending order, the same additions as the 256-target tiles of the plain path
// (a target's sum does not depend on which targets share its tile), into the segment
// sums seg[s * K + i].  Targets are grouped by 64 so that small supergraphs leave few
// lanes idle.
__device__ __forceinline__ void bt_wave_repulsion(int32_t wt, int32_t sgm, int32_t K, const float2 *__restrict__ pos,
                                                  const float *__restrict__ mass, float2 *__restrict__ seg,
                                                  float4 *slab) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t i = wt * kWave + lane;
    const bool live = i < K;
    const float2 xi = live ? pos[i] : make_float2(0.f, 0.f);
    const int32_t jb = sgm * kRepSegment, je = min(K, jb + kRepSegment);
    float fx = 0.f, fy = 0.f;
    for (int32_t t0 = jb; t0 < je; t0 += kWave) {
        const int32_t j = t0 + lane;
        if (j < je) {
            const float2 xj = pos[j];
            slab[lane] = make_float4(xj.x, xj.y, mass[j], 0.f);
        }
        __builtin_amdgcn_wave_barrier();
        const int cnt = min(kWave, je - t0);
        if (cnt == kWave) {
            fa2_rep_run(xi, slab, kWave, fx, fy);
        } else {
            for (int q = 0; q < cnt; ++q) fa2_rep_term(xi, slab[q], fx, fy);
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (live) seg[(int64_t)sgm * K + i] = make_float2(fx, fy);
}

// All (wave tile, segment) items, one per wavefront, then the attraction of the listed
// graphs' rows, one wavefront per row as in the persistent kernel (the row descriptor:
// absolute CSR range, node, graph base, in one load).  A graph of one segment takes the
// same path: its one segment sum is its repulsion.
__global__ void __launch_bounds__(kFa2Tile) k_bt_force(BtBig b) {
    __shared__ float4 slab[kFa2Tile];
    const uint32_t nb = *b.nbig;
    const uint32_t FI = b.fitem_off[nb], R = b.row_off[nb];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t nw = gridDim.x * (kFa2Tile / kWave);
    for (uint32_t x = blockIdx.x * (kFa2Tile / kWave) + w; x < FI; x += nw) {
        const uint32_t sl = b.fitem_slot[x];
        const int32_t g = b.big[sl];
        const int64_t n0 = b.node_off[g];
        const int32_t K = b.K[g];
        const uint32_t wtiles = (uint32_t)((K + kWave - 1) / kWave);
        const uint32_t q = x - b.fitem_off[sl];
        bt_wave_repulsion((int32_t)(q % wtiles), (int32_t)(q / wtiles), K, b.pos + n0, b.mass + n0,
                          b.seg + kBtMaxSeg * n0, slab + w * kWave);
    }
    for (uint32_t r = (blockIdx.x * kFa2Tile + threadIdx.x) / kWave; r < R; r += nw) {
        const uint4 d = b.row_desc[r];  // (first entry, end entry, node, graph's first node)
        const float2 *pos = b.pos + d.w;
        const float2 f = fa2_row_attraction(pos, b.cw, d.x, d.y, b.pos[d.z], lane);
        if (lane == 0) b.att[d.z] = f;
    }
}

// Segment sums added in order, then the rest of every force and the tiles' partials.
__global__ void __launch_bounds__(kFa2Tile) k_bt_combine(BtBig b) {
    const uint32_t nb = *b.nbig;
    const uint32_t T = b.tile_off[nb];
    for (uint32_t x = blockIdx.x; x < T; x += gridDim.x) {
        const uint32_t sl = b.tile_slot[x];
        const int32_t g = b.big[sl];
        const int64_t n0 = b.node_off[g];
        const int32_t K = b.K[g];
        fa2_combine_tile((int32_t)(x - b.tile_off[sl]), K, fa2_rep_segments(K), b.seg + kBtMaxSeg * n0, b.pos + n0,
                         b.mass + n0, b.att + n0, nullptr, b.kr, b.kg, b.fprev + n0, b.F + n0,
                         b.vpart + (n0 / 256) + g);
        __syncthreads();  // the tile function's LDS is reused by the next item
    }
}

__global__ void __launch_bounds__(kFa2Tile) k_bt_update(BtBig b, int32_t it) {
    const uint32_t nb = *b.nbig;
    const uint32_t T = b.tile_off[nb];
    for (uint32_t x = blockIdx.x; x < T; x += gridDim.x) {
        const uint32_t sl = b.tile_slot[x];
        const int32_t g = b.big[sl];
        const int64_t n0 = b.node_off[g];
        const int32_t ntiles = (int32_t)(b.tile_off[sl + 1] - b.tile_off[sl]);
        fa2_update_tile((int32_t)(x - b.tile_off[sl]), ntiles, b.K[g], b.pos + n0, b.fprev + n0, b.F + n0,
                        b.vpart + (n0 / 256) + g, ntiles, b.bspeed + 2 * g + (it & 1),
                        b.bspeed + 2 * g + ((it + 1) & 1), b.tau, b.ks, b.ksmax);
        __syncthreads();  // the tile function's LDS is reused by the next item
    }
}

__global__ void k_bt_finish(BtBig b, int32_t iters) {
    const uint32_t nb = *b.nbig;
    for (uint32_t sl = blockIdx.x * blockDim.x + threadIdx.x; sl < nb; sl += gridDim.x * blockDim.x) {
        const int32_t g = b.big[sl];
        b.speed[g] = b.bspeed[2 * g + (iters & 1)];
    }
}

struct BtWs {
    int32_t *cnt, *lab, *prop;
    unsigned long long *win;
    uint32_t *sid, *row;
    uint64_t *keyA, *keyB;
    int2 *cw;
    float *mass;
    float2 *F, *att;
    double2 *vpart;
    unsigned int *queue;
    int32_t *big;
    unsigned int *nbig;
    uint32_t *tile_off, *row_off, *fitem_off, *tile_slot, *fitem_slot;
    uint4 *row_desc;
    float2 *seg;
    float *bspeed;
};

static size_t bt_layout(Carver &c, int32_t G, int64_t n_total, int64_t m_total, BtWs *w) {
    const size_t n = (size_t)(n_total > 0 ? n_total : 1), m = (size_t)(m_total > 0 ? m_total : 1);
    w->cnt = c.take<int32_t>(n);
    w->lab = c.take<int32_t>(n);
    w->win = c.take<unsigned long long>(n);
    w->sid = c.take<uint32_t>(n);
    w->prop = c.take<int32_t>(m);
    w->keyA = c.take<uint64_t>(2 * m);
    w->keyB = c.take<uint64_t>(2 * m);
    w->cw = c.take<int2>(2 * m);
    w->row = c.take<uint32_t>(n + (size_t)G);
    w->mass = c.take<float>(n);
    w->F = c.take<float2>(n);
    w->att = c.take<float2>(n);
    w->vpart = c.take<double2>(n / 256 + (size_t)G + 1);
    w->queue = c.take<unsigned int>(1);
    w->big = c.take<int32_t>((size_t)G);
    w->nbig = c.take<unsigned int>(1);
    w->tile_off = c.take<uint32_t>((size_t)G + 1);
    w->row_off = c.take<uint32_t>((size_t)G + 1);
    w->fitem_off = c.take<uint32_t>((size_t)G + 1);
    w->tile_slot = c.take<uint32_t>(n / kFa2Tile + (size_t)G + 1);
    // a listed graph has K <= kBtBigMax supernodes, at most kBtMaxSeg segments of them
    // a listed graph has K <= kBtBigMax supernodes: at most kBtMaxSeg segments of K / 64 + 1 wave tiles
    w->fitem_slot = c.take<uint32_t>((size_t)kBtMaxSeg * (n / kWave + (size_t)G + 1));
    w->row_desc = c.take<uint4>(n);
    w->seg = c.take<float2>((size_t)kBtMaxSeg * n);
    w->bspeed = c.take<float>(2 * (size_t)G);
    return c.size();
}

static bool bt_valid(int32_t G, int64_t n_total, int64_t m_total, const bgv_cd_params *cd,
                     const bgv_sketch_params *sk, const bgv_fa2_params *fa) {
    return G >= 1 && n_total >= 0 && n_total <= INT32_MAX && m_total >= 0 && m_total <= INT32_MAX && cd && sk &&
           fa && cd->threshold >= 0 && cd->passes >= 1 && cd->growth >= 1 && cd->chunk >= 1 && cd->method == 0 &&
           (cd->tie == 0 || cd->tie == 1) && cd->rule == 0 &&
           sk->rows >= 1 && sk->rows <= kMaxRows && sk->cols >= 1 && (int64_t)sk->rows * sk->cols <= kBtMaxCells &&
           sk->coef1 && sk->coef2 && fa->iters >= 0 && fa->exact == 1 && fa->tau > 0.f && fa->ks >= 0.f &&
           fa->ksmax > 0.f;
}

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_batched_workspace(int32_t G, int64_t n_total, int64_t m_total) {
    if (G < 1 || n_total < 0 || m_total < 0) return 0;
    Carver c(nullptr);
    BtWs w;
    return bt_layout(c, G, n_total, m_total, &w);
}

extern "C" bgv_status bgv_batched(int32_t G, int64_t n_total, int64_t m_total, const int64_t *node_off,
                                  const int64_t *edge_off, const int32_t *order, const int32_t *edges,
                                  const bgv_cd_params *cd, const bgv_sketch_params *sk, const bgv_fa2_params *fa,
                                  int32_t wg_threads, int32_t big_k, int32_t *labels, int32_t *degree, int32_t *K, int32_t *E_S,
                                  int32_t *super_label, uint32_t *super_size, int32_t *superedges,
                                  uint32_t *se_weight, float *pos, float *fprev, float *speed, void *ws,
                                  size_t ws_bytes, bgv_stream_t stream) {
    clear_error();
    if (!bt_valid(G, n_total, m_total, cd, sk, fa)) {
        set_error("bgv_batched: invalid arguments (G=%d n_total=%lld m_total=%lld)", G, (long long)n_total,
                  (long long)m_total);
        return BGV_E_INVALID;
    }
    if (big_k < 0) {
        set_error("bgv_batched: big_k must be >= 0 (got %d)", big_k);
        return BGV_E_INVALID;
    }
    if (wg_threads == 0) wg_threads = 512;
    if (wg_threads != 256 && wg_threads != 512 && wg_threads != 1024) {
        set_error("bgv_batched: wg_threads must be 0, 256, 512 or 1024 (got %d)", wg_threads);
        return BGV_E_INVALID;
    }
    if (!node_off || !edge_off || (m_total > 0 && (!edges || !superedges || !se_weight)) || !labels || !degree ||
        !K || !E_S || !super_label || !super_size || !pos || !fprev || !speed) {
        set_error("bgv_batched: null pointer");
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_batched_workspace(G, n_total, m_total)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (range_check_on()) {  // K[0] holds the flag; it is written below
        BGV_TRY(check_batched_ids(G, n_total, m_total, node_off, edge_off, edges, K, s));
        if (order) BGV_TRY(check_id_list(G, order, G, K, s));
    }
    Carver c(ws);
    BtWs w;
    bt_layout(c, G, n_total, m_total, &w);

    BtArgs a{};
    a.G = G;
    a.node_off = node_off;
    a.edge_off = edge_off;
    a.order = order;
    a.edges = reinterpret_cast<const int2 *>(edges);
    a.threshold = cd->threshold;
    a.passes = cd->passes;
    a.growth = cd->growth;
    a.tie = cd->tie;
    a.chunk = cd->chunk;
    a.rows = sk->rows;
    a.cols = (uint32_t)sk->cols;
    a.h1 = make_hash_rows(sk->coef1, sk->rows);
    a.h2 = make_hash_rows(sk->coef2, sk->rows);
    a.iters = fa->iters;
    a.kr = fa->kr;
    a.kg = fa->kg;
    a.tau = fa->tau;
    a.ks = fa->ks;
    a.ksmax = fa->ksmax;
    a.labels = labels;
    a.degree = degree;
    a.K = K;
    a.E = E_S;
    a.super_label = super_label;
    a.super_size = super_size;
    a.superedges = reinterpret_cast<int2 *>(superedges);
    a.se_weight = se_weight;
    a.pos = reinterpret_cast<float2 *>(pos);
    a.fprev = reinterpret_cast<float2 *>(fprev);
    a.speed = speed;
    a.cnt = w.cnt;
    a.lab = w.lab;
    a.prop = w.prop;
    a.win = w.win;
    a.sid = w.sid;
    a.row = w.row;
    a.keyA = w.keyA;
    a.keyB = w.keyB;
    a.cw = w.cw;
    a.mass = w.mass;
    a.F = w.F;
    a.att = w.att;
    a.vpart = w.vpart;
    a.queue = w.queue;
    a.big_k = big_k;
    a.big = w.big;
    a.nbig = w.nbig;

    int cus = 1;
    BGV_TRY(device_cu_count(&cus));
    const int per_cu = wg_threads == 1024 ? 1 : 2;
    const int grid = G < cus * per_cu ? G : cus * per_cu;
    BGV_TRY(fill<uint32_t>(w.queue, 0u, 1, s));
    BGV_TRY(fill<uint32_t>(w.nbig, 0u, 1, s));
    switch (wg_threads) {
        case 256: BGV_LAUNCH(k_batched<256>, dim3(grid), dim3(256), 0, s, a); break;
        case 512: BGV_LAUNCH(k_batched<512>, dim3(grid), dim3(512), 0, s, a); break;
        default: BGV_LAUNCH(k_batched<1024>, dim3(grid), dim3(1024), 0, s, a); break;
    }
    if (big_k > 0 && fa->iters > 0) {
        // the listed large graphs: a fixed sequence of launches whose sizes are read on
        // the device, so the whole call can still be captured in a graph
        BtBig b{};
        b.node_off = node_off;
        b.edge_off = edge_off;
        b.K = K;
        b.big = w.big;
        b.nbig = w.nbig;
        b.tile_off = w.tile_off;
        b.row_off = w.row_off;
        b.fitem_off = w.fitem_off;
        b.tile_slot = w.tile_slot;
        b.fitem_slot = w.fitem_slot;
        b.row_desc = w.row_desc;
        b.seg = w.seg;
        b.row = w.row;
        b.cw = w.cw;
        b.mass = w.mass;
        b.pos = a.pos;
        b.fprev = a.fprev;
        b.F = w.F;
        b.att = w.att;
        b.vpart = w.vpart;
        b.speed = speed;
        b.bspeed = w.bspeed;
        b.kr = fa->kr;
        b.kg = fa->kg;
        b.tau = fa->tau;
        b.ks = fa->ks;
        b.ksmax = fa->ksmax;
        // item bounds known on the host (tiles <= n_total/256 + G, rows <= n_total); wide
        // grids, since a workgroup holding two items of a large graph doubles the path
        // (measured: 512 workgroups looping over the items were 1.4x slower than 4096)
        const unsigned tiles_bound = (unsigned)(n_total / kFa2Tile + G);
        const unsigned gt = tiles_bound < 4096u ? (tiles_bound > 0 ? tiles_bound : 1u) : 4096u;
        // force items are wavefronts: four per workgroup
        const unsigned gf = gt * (unsigned)kBtMaxSeg < 16384u ? gt * (unsigned)kBtMaxSeg : 16384u;
        BGV_LAUNCH(k_bt_plan, dim3(1), dim3(1024), 0, s, b);
        BGV_LAUNCH(k_bt_maps, dim3(grid_for(n_total > 0 ? n_total : 1, kFa2Tile, 4096)), dim3(kFa2Tile), 0, s, b);
        for (int32_t it = 0; it < fa->iters; ++it) {
            BGV_LAUNCH(k_bt_force, dim3(gf), dim3(kFa2Tile), 0, s, b);
            BGV_LAUNCH(k_bt_combine, dim3(gt), dim3(kFa2Tile), 0, s, b);
            BGV_LAUNCH(k_bt_update, dim3(gt), dim3(kFa2Tile), 0, s, b, it);
        }
        BGV_LAUNCH(k_bt_finish, dim3(1), dim3(256), 0, s, b, fa->iters);
    }
    return BGV_OK;
}
