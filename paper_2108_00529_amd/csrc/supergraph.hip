// Count-min-sketch supergraph (Section 3.3 / Algorithm 2, Section 4.1, Algorithm 3).
//   1. flag used labels, exclusive scan -> sid (supernodes numbered by ascending label)
//   2. sketch 1: every node adds its degree at column h_r(label) of each row
//   3. every inter-community edge emits its packed (sid_lo, sid_hi) key
//   4. LSD radix sort of the keys, unique -> superedges; sketch 2 gets each distinct
//      pair's multiplicity at g_r(min label, max label); weights = min over rows of
//      sketch 2; supernode sizes = min over rows of sketch 1
#include "block_scan.h"
#include "common.h"
#include "sketch_hash.h"

namespace bgv {

constexpr int kSgThreads = 256;

__global__ void k_sg_flag(const int32_t *__restrict__ labels, int32_t n, uint32_t *__restrict__ flag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[labels[v]] = 1u;
}

// Flags as above, plus each community's volume vol[c] = sum of d(v) over its nodes
// (below 2^32: at most twice the number of edges).
__global__ void k_sg_flag_volume(const int32_t *__restrict__ labels, const int32_t *__restrict__ degree, int32_t n,
                                 uint32_t *__restrict__ flag, uint32_t *__restrict__ vol) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t lab = labels[v];
        flag[lab] = 1u;
        const uint32_t d = (uint32_t)degree[v];
        if (d) atomicAdd(&vol[lab], d);
    }
}

// The same without device atomics (labels below kLbMaxBuckets * kLbBucket): each tile of
// kLbTile nodes writes (label offset in bucket, degree) entries grouped by 4096-label
// bucket, one segment per (tile, bucket), offsets in a per-tile row; one workgroup per
// bucket then sums its segments from every tile in LDS and writes the bucket's flags and
// volumes, all of them, so neither array needs clearing.  Same integers.
constexpr int kLbBucketBits = 12;
constexpr int32_t kLbBucket = 1 << kLbBucketBits;
constexpr int32_t kLbMaxBuckets = 4096;
constexpr int kLbItems = 4;
constexpr int32_t kLbTile = kSgThreads * kLbItems;
constexpr int kLbResolveThreads = 1024;

inline int32_t lb_buckets(int32_t n) { return (n + kLbBucket - 1) / kLbBucket; }

__global__ void __launch_bounds__(kSgThreads) k_sg_group_nodes(const int32_t *__restrict__ labels,
                                                                const int32_t *__restrict__ degree, int32_t n,
                                                                int32_t nb, uint2 *__restrict__ ent,
                                                                uint32_t *__restrict__ etab) {
    __shared__ uint32_t hist[kLbMaxBuckets];
    __shared__ uint2 stage[kLbTile];
    for (int32_t b = threadIdx.x; b < nb; b += kSgThreads) hist[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kLbTile;
    int32_t lab[kLbItems];
    uint32_t d[kLbItems], rank[kLbItems];
#pragma unroll
    for (int u = 0; u < kLbItems; ++u) {
        const int64_t v = base + u * kSgThreads + threadIdx.x;
        lab[u] = -1;
        if (v < n) {
            lab[u] = labels[v];
            d[u] = (uint32_t)degree[v];
            rank[u] = atomicAdd(&hist[lab[u] >> kLbBucketBits], 1u);
        }
    }
    __syncthreads();
    uint32_t *row = etab + (int64_t)blockIdx.x * (nb + 1);
    const int32_t per = (nb + kSgThreads - 1) / kSgThreads;
    const int32_t b0 = min(nb, (int32_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    uint32_t sum = 0;
    for (int32_t b = b0; b < b1; ++b) sum += hist[b];
    uint32_t total;
    uint32_t run = block_excl_scan<uint32_t>(sum, &total);
    for (int32_t b = b0; b < b1; ++b) {
        const uint32_t c = hist[b];
        hist[b] = run;
        row[b] = run;
        run += c;
    }
    if (threadIdx.x == 0) row[nb] = total;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kLbItems; ++u)
        if (lab[u] >= 0)
            stage[hist[lab[u] >> kLbBucketBits] + rank[u]] = make_uint2((uint32_t)(lab[u] & (kLbBucket - 1)), d[u]);
    __syncthreads();
    uint2 *out = ent + (int64_t)blockIdx.x * kLbTile;
    for (uint32_t k = threadIdx.x; k < total; k += kSgThreads) out[k] = stage[k];
}

// One workgroup per label bucket; each tile's segment goes to a group of `lanes`
// threads (a power of two sized by the tile count).
__global__ void __launch_bounds__(kLbResolveThreads) k_sg_sum_labels(const uint2 *__restrict__ ent,
                                                                      const uint32_t *__restrict__ etab, int32_t tiles,
                                                                      int32_t nb, int32_t n, int32_t lanes,
                                                                      uint32_t *__restrict__ flag,
                                                                      uint32_t *__restrict__ vol) {
    __shared__ uint32_t svol[kLbBucket];
    __shared__ uint32_t sflag[kLbBucket];
    const int32_t b = blockIdx.x;
    for (int32_t k = threadIdx.x; k < kLbBucket; k += kLbResolveThreads) {
        svol[k] = 0u;
        sflag[k] = 0u;
    }
    __syncthreads();
    const int32_t groups = kLbResolveThreads / lanes;
    const uint32_t sub = threadIdx.x % lanes, L = (uint32_t)lanes;
    for (int32_t t = threadIdx.x / lanes; t < tiles; t += groups) {
        const uint32_t *row = etab + (int64_t)t * (nb + 1);
        const uint32_t q0 = row[b], q1 = row[b + 1];
        const uint2 *seg = ent + (int64_t)t * kLbTile;
        for (uint32_t q = q0 + sub; q < q1; q += 4 * L) {
            uint2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u * L < q1) v[u] = seg[q + u * L];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u * L < q1) {
                    atomicOr(&sflag[v[u].x], 1u);
                    if (v[u].y) atomicAdd(&svol[v[u].x], v[u].y);
                }
        }
    }
    __syncthreads();
    const int64_t base = (int64_t)b << kLbBucketBits;
    const int32_t span = (int32_t)min((int64_t)kLbBucket, (int64_t)n - base);
    for (int32_t k = threadIdx.x; k < span; k += kLbResolveThreads) {
        flag[base + k] = sflag[k];
        vol[base + k] = svol[k];
    }
}

inline int32_t lb_lanes(int32_t tiles) {
    int32_t g = 1;
    while (g < kLbResolveThreads && (int64_t)g * 2 * (tiles > 0 ? tiles : 1) <= kLbResolveThreads) g *= 2;
    return g;
}

// flag[] still holds the 0/1 flags; sid[] is its exclusive scan.
__global__ void k_sg_compact(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ sid, int32_t n,
                             int32_t *__restrict__ super_label) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        if (flag[c]) super_label[sid[c]] = (int32_t)c;
}

// Sketch 1 with the whole sketch privatised in LDS (rows*cols <= kLdsCounters).
constexpr int kLdsCounters = 16384;
__global__ void __launch_bounds__(kSgThreads) k_sg_sketch_nodes_lds(const int32_t *__restrict__ labels,
                                                                     const int32_t *__restrict__ degree, int32_t n,
                                                                     HashRows h, int32_t rows, uint32_t cols,
                                                                     uint32_t *__restrict__ M1) {
    __shared__ uint32_t loc[kLdsCounters];
    const int total = rows * (int)cols;
    for (int i = threadIdx.x; i < total; i += blockDim.x) loc[i] = 0;
    __syncthreads();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t d = (uint32_t)degree[v];
        if (d == 0) continue;
        const uint32_t lab = (uint32_t)labels[v];
        for (int r = 0; r < rows; ++r) atomicAdd(&loc[r * cols + col_key(h.a[r], h.b[r], lab, cols)], d);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < total; i += blockDim.x)
        if (loc[i]) atomicAdd(&M1[i], loc[i]);
}

// Sketch 1 from the community volumes: M1[r][h_r(c)] += vol[c] once per community c,
// the same integer sums as adding d(v) once per node (a quarter of the atomics and
// fewer: one per community and row instead of one per node and row).
__global__ void k_sg_sketch_volumes(const int32_t *__restrict__ super_label, const uint32_t *__restrict__ Kp,
                                    const uint32_t *__restrict__ vol, HashRows h, int32_t rows, uint32_t cols,
                                    uint32_t *__restrict__ M1) {
    const int64_t K = *Kp;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t lab = (uint32_t)super_label[k];
        const uint32_t v = vol[lab];
        if (v == 0) continue;
        for (int r = 0; r < rows; ++r) atomicAdd(&M1[(size_t)r * cols + col_key(h.a[r], h.b[r], lab, cols)], v);
    }
}

__global__ void k_sg_super_size(const int32_t *__restrict__ super_label, const uint32_t *__restrict__ Kp,
                                HashRows h, int32_t rows, uint32_t cols, const uint32_t *__restrict__ M1,
                                uint32_t *__restrict__ super_size) {
    const int64_t K = *Kp;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t lab = (uint32_t)super_label[k];
        uint32_t best = 0xffffffffu;
        for (int r = 0; r < rows; ++r) best = min(best, M1[(size_t)r * cols + col_key(h.a[r], h.b[r], lab, cols)]);
        super_size[k] = best;
    }
}

// Inter-community edges: emit the packed (sid_lo, sid_hi) key of each; a block
// compacts its tile with a block scan and reserves output space with one atomic (the
// order of tiles is arbitrary; the sort below makes the result deterministic).
// Sketch 2 is filled after the keys are sorted: each
// distinct key adds its multiplicity once (the same integer sums as one increment per
// edge, without same-address contention on popular community pairs).
constexpr int kKeyItems = 16;  // edges per thread; a block compacts kSgThreads*kKeyItems edges
// nsid[v] = sid of node v's community: an edge is inter-community iff its endpoints'
// sids differ, and since sids ascend with labels, (min, max) of the two sids is
// (sid of the smaller label, sid of the larger).
// 32-bit keys when 2 * kbits <= 32; then the supernode ids are gathered as 16-bit values
// (half the footprint of the random gathers, which bound this kernel)
// With bcnt, each workgroup also counts the digits of its keys for the one-sweep sort
// (8-bit digits, `passes` of them) and writes its counts as row blockIdx.x of bcnt.
constexpr int kKeyMaxPasses = 8;
template <typename KT, typename NT>
__global__ void __launch_bounds__(kSgThreads) k_sg_edge_keys(const int2 *__restrict__ edges, int64_t m,
                                                              const NT *__restrict__ nsid, int kbits,
                                                              KT *__restrict__ keys,
                                                              unsigned long long *__restrict__ nkeys,
                                                              uint32_t *__restrict__ bcnt, int passes) {
    __shared__ unsigned long long s_base;
    __shared__ uint32_t hist[kKeyMaxPasses * 256];
    if (bcnt)
        for (int q = 0; q < passes; ++q) hist[q * 256 + threadIdx.x] = 0u;
    const int64_t tile = (int64_t)blockIdx.x * (kSgThreads * kKeyItems);
    KT k[kKeyItems];
    uint32_t flags = 0, cnt = 0;
#pragma unroll
    for (int j = 0; j < kKeyItems; ++j) {
        const int64_t i = tile + (int64_t)j * kSgThreads + threadIdx.x;
        k[j] = 0;
        if (i < m) {
            const int2 e = edges[i];
            if (e.x != e.y) {
                const uint32_t a = (uint32_t)nsid[e.x], b = (uint32_t)nsid[e.y];
                if (a != b) {
                    k[j] = ((KT)min(a, b) << kbits) | (KT)max(a, b);
                    flags |= 1u << j;
                    ++cnt;
                }
            }
        }
    }
    uint32_t total;
    const uint32_t pre = block_excl_scan<uint32_t>(cnt, &total);
    if (threadIdx.x == 0) s_base = total ? atomicAdd(nkeys, (unsigned long long)total) : 0ull;
    __syncthreads();
    unsigned long long at = s_base + pre;
#pragma unroll
    for (int j = 0; j < kKeyItems; ++j)
        if ((flags >> j) & 1u) keys[at++] = k[j];
    if (bcnt) {  // uniform
#pragma unroll
        for (int j = 0; j < kKeyItems; ++j)
            if ((flags >> j) & 1u)
                for (int q = 0; q < passes; ++q) atomicAdd(&hist[q * 256 + ((uint32_t)(k[j] >> (8 * q)) & 255u)], 1u);
        __syncthreads();
        for (int q = 0; q < passes; ++q)
            bcnt[((int64_t)blockIdx.x * passes + q) * 256 + threadIdx.x] = hist[q * 256 + threadIdx.x];
    }
}

// Distinct sorted keys, in tiles of kUqTile: k_sg_unique_count counts each tile's run
// starts (key differs from its predecessor), an exclusive scan of the tile counts gives
// each tile's first superedge, and k_sg_unique_write numbers the run starts inside the
// tile (a block scan in key order) and writes superedge j = (sid_lo, sid_hi) with the
// position of its run.  Two reads of the keys instead of a device-wide scan of one flag
// per key.
constexpr int kUqItems = 16;
constexpr int kUqTile = kSgThreads * kUqItems;
constexpr int kUqWaves = kSgThreads / kWave;

// The keys of wavefront w of a tile: kUqItems rounds of 64 consecutive keys from
// tile * kUqTile + w * 64 * kUqItems, with the run-start flag of each (its key differs
// from the one before it: the lane below, the last lane of the previous round, or for
// the wavefront's first key the key before it in memory).
template <typename KT>
__device__ __forceinline__ void uq_load(const KT *__restrict__ keys, int64_t nk, int64_t wbase, int lane, KT *k,
                                        bool *start) {
    KT before = (lane == 0 && wbase > 0 && wbase - 1 < nk) ? keys[wbase - 1] : KT(0);
#pragma unroll
    for (int u = 0; u < kUqItems; ++u) {
        const int64_t i = wbase + (int64_t)u * kWave + lane;
        k[u] = i < nk ? keys[i] : KT(0);
    }
#pragma unroll
    for (int u = 0; u < kUqItems; ++u) {
        const int64_t i = wbase + (int64_t)u * kWave + lane;
        KT prev = __shfl_up(k[u], 1, kWave);
        const KT last_prev_round = __shfl(u > 0 ? k[u > 0 ? u - 1 : 0] : before, kWave - 1, kWave);
        if (lane == 0) prev = u > 0 ? last_prev_round : before;
        start[u] = i < nk && (i == 0 || k[u] != prev);
    }
}

template <typename KT>
__global__ void __launch_bounds__(kSgThreads) k_sg_unique_count(const KT *__restrict__ keys,
                                                                 const unsigned long long *__restrict__ nkp,
                                                                 uint32_t *__restrict__ tile_count) {
    const int64_t nk = (int64_t)*nkp;  // the grid covers a bound of it
    __shared__ uint32_t ws[kUqWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t wbase = (int64_t)blockIdx.x * kUqTile + (int64_t)w * (kWave * kUqItems);
    KT k[kUqItems];
    bool start[kUqItems];
    uq_load(keys, nk, wbase, lane, k, start);
    uint32_t c = 0;
#pragma unroll
    for (int u = 0; u < kUqItems; ++u) c += (uint32_t)__popcll(__ballot(start[u]));
    if (lane == 0) ws[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int q = 0; q < kUqWaves; ++q) t += ws[q];
        tile_count[blockIdx.x] = t;
    }
}

template <typename KT>
__global__ void __launch_bounds__(kSgThreads) k_sg_unique_write(const KT *__restrict__ keys,
                                                                 const unsigned long long *__restrict__ nkp,
                                                                 const uint32_t *__restrict__ tile_first, int kbits,
                                                                 int32_t *__restrict__ superedges,
                                                                 uint32_t *__restrict__ run_start) {
    const int64_t nk = (int64_t)*nkp;  // the grid covers a bound of it
    __shared__ uint32_t ws[kUqWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t wbase = (int64_t)blockIdx.x * kUqTile + (int64_t)w * (kWave * kUqItems);
    KT k[kUqItems];
    bool start[kUqItems];
    uq_load(keys, nk, wbase, lane, k, start);
    uint32_t c = 0;
#pragma unroll
    for (int u = 0; u < kUqItems; ++u) c += (uint32_t)__popcll(__ballot(start[u]));
    if (lane == 0) ws[w] = c;
    __syncthreads();
    uint32_t j = tile_first[blockIdx.x];
    for (int q = 0; q < w; ++q) j += ws[q];  // the wavefronts before this one, in key order
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t lowmask = (1ull << kbits) - 1ull;
#pragma unroll
    for (int u = 0; u < kUqItems; ++u) {
        const uint64_t m = __ballot(start[u]);
        if (start[u]) {
            const uint32_t at = j + (uint32_t)__popcll(m & lt);
            superedges[2 * (int64_t)at] = (int32_t)((uint64_t)k[u] >> kbits);
            superedges[2 * (int64_t)at + 1] = (int32_t)((uint64_t)k[u] & lowmask);
            run_start[at] = (uint32_t)(wbase + (int64_t)u * kWave + lane);
        }
        j += (uint32_t)__popcll(m);
    }
}

// Sketch 2: each distinct key adds its multiplicity (run length) at g_r(key).
__global__ void k_sg_sketch_pairs(const int32_t *__restrict__ superedges, const uint32_t *__restrict__ run_start,
                                  const uint32_t *__restrict__ Ep, const unsigned long long *__restrict__ nkp,
                                  const int32_t *__restrict__ super_label,
                                  HashRows h, int32_t rows, uint32_t cols, uint32_t *__restrict__ M2,
                                  uint32_t *__restrict__ se_count) {
    const int64_t E = *Ep;
    const uint32_t nk = (uint32_t)*nkp;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t cnt = (j + 1 < E ? run_start[j + 1] : nk) - run_start[j];
        const uint32_t la = (uint32_t)super_label[superedges[2 * j]];
        const uint32_t lb = (uint32_t)super_label[superedges[2 * j + 1]];
        for (int r = 0; r < rows; ++r)
            atomicAdd(&M2[(size_t)r * cols + col_pair(h.a[r], h.b[r], h.c[r], la, lb, cols)], cnt);
        if (se_count) se_count[j] = cnt;
    }
}

// Sketch 2 without global atomics, for sketches of at most kSkMaxCells cells, in buckets
// of 2^kB consecutive cells (cell = row * cols + column).  Each tile of distinct pairs
// (4,096 of them, 2,048 with more than five rows) writes one 4-byte entry per (pair,
// row) grouped by bucket, one segment per (tile, bucket), offsets in a per-tile table
// row; then one workgroup per bucket sums its segments from every tile in LDS and
// writes the bucket's cells, all of them, so the sketch needs no clearing.  Same
// integer sums.  An entry packs the cell's offset in its bucket (kB bits), the pair's
// multiplicity when below 31 (5 bits; 31: look it up in the tile's count row) and the
// pair's index in its tile (12 bits).
// Buckets of 2^14 cells, or 2^15 from 2^23 cells on (the 128 KiB of LDS counters leave
// one resolve workgroup per compute unit, but halve the (tile, bucket) segments and the
// grouping's per-tile bucket table).
constexpr int32_t kSkMaxCells = 1 << 26;             // grouped sketch 2 up to here
constexpr int32_t kSkMaxBuckets = kSkMaxCells >> 14;  // bucket histogram held in LDS
inline int sk_bucket_bits(int64_t cells) { return cells >= (1 << 23) ? 15 : 14; }
constexpr int kSkThreads = 1024;                      // grouping workgroup
constexpr int32_t kSkStage = 20480;                   // entries a tile stages in LDS
inline int32_t sk_tile_pairs(int32_t rows) { return rows <= 5 ? 4096 : 2048; }
constexpr int kSkCodeBits = 5;
constexpr uint32_t kSkEscape = (1u << kSkCodeBits) - 1;
constexpr int kSkResolveThreads = 1024;

inline int64_t sk_buckets(int64_t cells, int bits) { return (cells + (1ll << bits) - 1) >> bits; }

template <int kB>
__global__ void __launch_bounds__(kSkThreads) k_sg_group_pairs(const int32_t *__restrict__ superedges,
                                                                const uint32_t *__restrict__ run_start,
                                                                const uint32_t *__restrict__ Ep,
                                                                const unsigned long long *__restrict__ nkp,
                                                                const int32_t *__restrict__ super_label, HashRows h,
                                                                int32_t rows, uint32_t cols, int32_t nb, int32_t tp,
                                                                uint32_t *__restrict__ ent, uint32_t *__restrict__ etab,
                                                                uint32_t *__restrict__ pcnt,
                                                                uint32_t *__restrict__ se_count) {
    static_assert(kB + kSkCodeBits + 12 <= 32, "entry fields must fit 32 bits");
    constexpr int kItems = 4096 / kSkThreads;  // pairs per thread at most
    __shared__ uint32_t hist[kSkMaxBuckets];
    __shared__ uint32_t stage[kSkStage];
    const int64_t E = *Ep;
    const uint32_t nk = (uint32_t)*nkp;
    const int64_t j0 = (int64_t)blockIdx.x * tp;
    if (j0 >= E) return;  // the grid covers a bound of E
    for (int32_t b = threadIdx.x; b < nb; b += kSkThreads) hist[b] = 0;
    __syncthreads();
    const int items = tp / kSkThreads;
    uint32_t la[kItems], lb[kItems], cnt[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t j = j0 + u * kSkThreads + threadIdx.x;
        cnt[u] = 0;
        if (u < items && j < E) {
            cnt[u] = (j + 1 < E ? run_start[j + 1] : nk) - run_start[j];
            la[u] = (uint32_t)super_label[superedges[2 * j]];
            lb[u] = (uint32_t)super_label[superedges[2 * j + 1]];
            pcnt[j] = cnt[u];
            if (se_count) se_count[j] = cnt[u];
            for (int r = 0; r < rows; ++r) {
                const uint32_t cell = (uint32_t)r * cols + col_pair(h.a[r], h.b[r], h.c[r], la[u], lb[u], cols);
                atomicAdd(&hist[cell >> kB], 1u);
            }
        }
    }
    __syncthreads();
    // exclusive offsets of the tile's buckets, in place and into the table row
    uint32_t *row = etab + (int64_t)blockIdx.x * (nb + 1);
    const int32_t per = (nb + kSkThreads - 1) / kSkThreads;
    const int32_t b0 = min(nb, (int32_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    uint32_t sum = 0;
    for (int32_t b = b0; b < b1; ++b) sum += hist[b];
    uint32_t total;
    uint32_t run = block_excl_scan<uint32_t>(sum, &total);
    for (int32_t b = b0; b < b1; ++b) {
        const uint32_t c = hist[b];
        hist[b] = run;
        row[b] = run;
        run += c;
    }
    if (threadIdx.x == 0) row[nb] = total;
    __syncthreads();
    // the entries placed in their buckets' segments (the order inside a segment does not
    // matter: sums and minima)
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        if (cnt[u]) {
            const uint32_t pair = (uint32_t)(u * kSkThreads + threadIdx.x);
            const uint32_t code = cnt[u] < kSkEscape ? cnt[u] : kSkEscape;
            for (int r = 0; r < rows; ++r) {
                const uint32_t cell = (uint32_t)r * cols + col_pair(h.a[r], h.b[r], h.c[r], la[u], lb[u], cols);
                const uint32_t at = atomicAdd(&hist[cell >> kB], 1u);
                stage[at] = (pair << (kB + kSkCodeBits)) | (code << kB) | (cell & ((1u << kB) - 1));
            }
        }
    __syncthreads();
    uint32_t *out = ent + (int64_t)blockIdx.x * ((int64_t)tp * rows);  // a tile's region holds tp * rows
    for (uint32_t k = threadIdx.x; k < total; k += kSkThreads) out[k] = stage[k];
}

// Each tile's segment goes to a group of `lanes` threads (a power of two): enough that
// a segment of average length takes one batch of eight loads per lane, and at least
// about kSkResolveThreads / tiles, so that few tiles with long segments still spread
// over the workgroup.  (3.2M-node bench graph, 32-entry segments: 4 lanes 348 us per
// resolve, 16 lanes 393, 1 lane 968.)
inline int32_t sk_sum_lanes(int64_t tiles, int32_t tp, int32_t rows, int32_t nb) {
    const int64_t seg = (int64_t)tp * rows / (nb > 0 ? nb : 1);  // entries per (tile, bucket) on average
    int32_t g = 1;
    while (g < 64 && (int64_t)g * 8 < seg) g *= 2;
    while (g < kSkResolveThreads && (int64_t)g * 2 * (tiles > 0 ? tiles : 1) <= kSkResolveThreads) g *= 2;
    return g;
}

// One workgroup per bucket of sketch-2 cells: the bucket's entries from every tile are
// summed into its cells in LDS and the cells written whole; then every entry's cell
// value is written beside it (est, the same position), so that each tile finds its
// pairs' row estimates in its own region (k_sg_pair_min) instead of gathering them from
// the sketch.  Buckets are dealt to the XCDs in contiguous ranges (as in the community
// resolve): neighbouring buckets' segments share cache lines.
constexpr int32_t kSgXcds = 8;

template <int kB>
__global__ void __launch_bounds__(kSkResolveThreads) k_sg_sum_cells(const uint32_t *__restrict__ ent,
                                                                     uint32_t *__restrict__ est,
                                                                     const uint32_t *__restrict__ etab,
                                                                     const uint32_t *__restrict__ pcnt,
                                                                     const uint32_t *__restrict__ Ep, int32_t rows,
                                                                     int32_t nb, int32_t tp, int64_t cells,
                                                                     int32_t lanes, uint32_t *__restrict__ M2) {
    __shared__ uint32_t acc[1 << kB];
    const int32_t x = (int32_t)blockIdx.x;
    const int32_t b = (x % kSgXcds) * ((nb + kSgXcds - 1) / kSgXcds) + x / kSgXcds;
    if (b >= nb) return;  // the grid is rounded up to a multiple of the XCD count
    for (int32_t k = threadIdx.x; k < (1 << kB); k += kSkResolveThreads) acc[k] = 0u;
    __syncthreads();
    const int64_t tiles = ((int64_t)*Ep + tp - 1) / tp;
    const int64_t groups = kSkResolveThreads / lanes;
    const uint32_t sub = threadIdx.x % lanes, L = (uint32_t)lanes;
    constexpr uint32_t kCell = (1u << kB) - 1;
    const int64_t region = (int64_t)tp * rows;
    for (int64_t t = threadIdx.x / lanes; t < tiles; t += groups) {
        const uint32_t *row = etab + t * (nb + 1);
        const uint32_t q0 = row[b], q1 = row[b + 1];
        const uint32_t *seg = ent + t * region;
        for (uint32_t q = q0 + sub; q < q1; q += 8 * L) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u * L < q1) v[u] = seg[q + u * L];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u * L < q1) {
                    uint32_t c = (v[u] >> kB) & kSkEscape;
                    if (c == kSkEscape) c = pcnt[t * tp + (v[u] >> (kB + kSkCodeBits))];
                    atomicAdd(&acc[v[u] & kCell], c);
                }
        }
    }
    __syncthreads();
    const int64_t base = (int64_t)b << kB;
    const int32_t span = (int32_t)min((int64_t)1 << kB, cells - base);
    for (int32_t k = threadIdx.x; k < span; k += kSkResolveThreads) M2[base + k] = acc[k];
    for (int64_t t = threadIdx.x / lanes; t < tiles; t += groups) {
        const uint32_t *row = etab + t * (nb + 1);
        const uint32_t q0 = row[b], q1 = row[b + 1];
        const uint32_t *seg = ent + t * region;
        uint32_t *eseg = est + t * region;
        for (uint32_t q = q0 + sub; q < q1; q += 8 * L) {
            uint32_t c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u * L < q1) c[u] = seg[q + u * L];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u * L < q1) eseg[q + u * L] = acc[c[u] & kCell];
        }
    }
}

inline unsigned sg_sum_grid(int32_t nb) { return (unsigned)((nb + kSgXcds - 1) / kSgXcds * kSgXcds); }

// Superedge weight = count-min estimate, the minimum over the rows of the final cell
// values k_sg_sum_cells left beside the tile's entries (one per pair and row).
template <int kB>
__global__ void __launch_bounds__(kSgThreads) k_sg_pair_min(const uint32_t *__restrict__ ent,
                                                             const uint32_t *__restrict__ est,
                                                             const uint32_t *__restrict__ etab,
                                                             const uint32_t *__restrict__ Ep, int32_t rows, int32_t nb,
                                                             int32_t tp, uint32_t *__restrict__ se_weight) {
    __shared__ uint32_t best[4096];
    const int64_t E = *Ep;
    const int64_t j0 = (int64_t)blockIdx.x * tp;
    if (j0 >= E) return;  // the grid covers a bound of E
    for (int k = threadIdx.x; k < tp; k += kSgThreads) best[k] = 0xffffffffu;
    __syncthreads();
    const uint32_t total = etab[(int64_t)blockIdx.x * (nb + 1) + nb];
    const int64_t region = (int64_t)blockIdx.x * ((int64_t)tp * rows);
    for (uint32_t k = threadIdx.x; k < total; k += kSgThreads)
        atomicMin(&best[ent[region + k] >> (kB + kSkCodeBits)], est[region + k]);
    __syncthreads();
    const int32_t cnt = (int32_t)min((int64_t)tp, E - j0);
    for (int k = threadIdx.x; k < cnt; k += kSgThreads) se_weight[j0 + k] = best[k];
}

// Superedge weight = count-min estimate (minimum over the rows of sketch 2).
__global__ void k_sg_pair_weights(const int32_t *__restrict__ superedges, const uint32_t *__restrict__ Ep,
                                  const int32_t *__restrict__ super_label, HashRows h, int32_t rows, uint32_t cols,
                                  const uint32_t *__restrict__ M2, uint32_t *__restrict__ se_weight) {
    const int64_t E = *Ep;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t la = (uint32_t)super_label[superedges[2 * j]];
        const uint32_t lb = (uint32_t)super_label[superedges[2 * j + 1]];
        uint32_t best = 0xffffffffu;
        for (int r = 0; r < rows; ++r)
            best = min(best, M2[(size_t)r * cols + col_pair(h.a[r], h.b[r], h.c[r], la, lb, cols)]);
        se_weight[j] = best;
    }
}

// nsid[v] = sid of node v's community (and the caller's copy when asked for).
// nsid16: the same ids in 16 bits (saturated; exact whenever K <= 65536, the only case
// that reads it), written before K is known on the host.
__global__ void k_sg_node_super(const int32_t *__restrict__ labels, const uint32_t *__restrict__ sid, int32_t n,
                                uint32_t *__restrict__ nsid, uint16_t *__restrict__ nsid16,
                                int32_t *__restrict__ node_super) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = sid[labels[v]];
        nsid[v] = x;
        nsid16[v] = (uint16_t)(x < 65535u ? x : 65535u);
        if (node_super) node_super[v] = (int32_t)x;
    }
}

struct SgWs {
    uint32_t *flag, *sid, *vol, *nsid, *counters, *utile, *run_start;
    uint16_t *nsid16;
    uint64_t *keys, *keys_alt;
    uint32_t *ent;    // grouped sketch-2 entries (bucketed sketch only)
    uint32_t *est;    // beside each entry, its cell's final value
    uint32_t *pcnt;   // multiplicity of each distinct pair
    uint32_t *etab;   // their per-tile offset rows
    uint2 *lent;      // grouped (label, degree) entries (volumes without atomics)
    uint32_t *ltab;   // their per-tile offset rows
    void *scan_scratch, *sort_scratch;
};

// The inter-community keys are sorted by the one-sweep sort of keys alone (one read and
// one write of the keys per 8-bit pass, after one counting read), below 2^30 edges;
// beyond, by the reduce-then-scan radix sort.
static bool sg_onesweep(int64_t m) { return m < ((int64_t)1 << 30) - 1; }

static size_t sg_layout(Carver &c, int32_t n, int64_t m, int32_t rows, int64_t cells, SgWs *w) {
    const int64_t mm = m > 0 ? m : 1;
    w->ent = w->est = w->pcnt = nullptr;
    w->etab = nullptr;
    w->lent = nullptr;
    w->ltab = nullptr;
    w->flag = c.take<uint32_t>((size_t)n);
    w->nsid = c.take<uint32_t>((size_t)n);
    w->nsid16 = c.take<uint16_t>((size_t)n);
    w->sid = c.take<uint32_t>((size_t)n);
    w->vol = c.take<uint32_t>((size_t)n);
    w->counters = c.take<uint32_t>(8);  // [0] K, [1] E_S, [2..3] key count (u64, 8-byte aligned)
    w->keys = c.take<uint64_t>((size_t)mm);
    w->keys_alt = c.take<uint64_t>((size_t)mm);
    w->utile = c.take<uint32_t>((size_t)mm / kUqTile + 1);  // unique counts, then first superedge, per tile
    w->run_start = c.take<uint32_t>((size_t)mm);
    const int64_t big = n > mm ? n : mm;
    w->scan_scratch = c.take<char>(scan_workspace(big));
    w->sort_scratch = c.take<char>(sg_onesweep(mm) ? onesweep_keys_workspace(mm, 64) : radix_workspace(mm));
    if (cells > kLdsCounters && lb_buckets(n) <= kLbMaxBuckets) {
        const size_t tiles = ((size_t)n + kLbTile - 1) / kLbTile;
        w->lent = c.take<uint2>(tiles * kLbTile);
        w->ltab = c.take<uint32_t>(tiles * (size_t)(lb_buckets(n) + 1));
    }
    const int64_t nb = sk_buckets(cells, 14);  // the larger of the two bucket counts
    if (cells <= kSkMaxCells) {
        // distinct pairs <= m: a tile bound, rows entries per pair
        const size_t tp = (size_t)sk_tile_pairs(rows);
        const size_t tiles = ((size_t)mm + tp - 1) / tp;
        w->ent = c.take<uint32_t>(tiles * tp * (size_t)rows);
        w->est = c.take<uint32_t>(tiles * tp * (size_t)rows);
        w->pcnt = c.take<uint32_t>(tiles * tp);
        w->etab = c.take<uint32_t>(tiles * (size_t)(nb + 1));
    }
    return c.size();
}

// A small pinned host buffer and an event per host thread, for device-to-host reads of
// counts that run asynchronously while later work is already queued.
struct SgReadback {
    uint32_t *host = nullptr;
    hipEvent_t ev = nullptr;
};
static bgv_status sg_readback(SgReadback **out) {
    static thread_local SgReadback rb;
    if (!rb.host) {
        BGV_CHECK_HIP(hipHostMalloc(reinterpret_cast<void **>(&rb.host), 64, hipHostMallocDefault));
        BGV_CHECK_HIP(hipEventCreateWithFlags(&rb.ev, hipEventDisableTiming));
    }
    *out = &rb;
    return BGV_OK;
}

// Waits for the readback event by polling it: the two readbacks wait on work this call
// has just queued (well under a millisecond for K), and a blocking wait would add the
// host thread's wake-up time to each.
static bgv_status sg_wait(hipEvent_t ev) {
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return BGV_OK;
        if (e != hipErrorNotReady) {
            set_error("hipEventQuery failed: %s", hipGetErrorString(e));
            return BGV_E_HIP;
        }
    }
}

// Sketch 2 by grouped entries (buckets of 2^kB cells) and the superedge weights.
template <int kB>
static bgv_status sg_sketch2_grouped(int64_t m, const SgWs &w, const int32_t *superedges,
                                     const unsigned long long *nkeys_d, const int32_t *super_label, HashRows h2,
                                     int32_t rows, uint32_t cols, int64_t cells, uint32_t *se_count, uint32_t *M2,
                                     uint32_t *se_weight, hipStream_t s) {
    const int32_t nb = (int32_t)sk_buckets(cells, kB);
    const int32_t tp = sk_tile_pairs(rows);
    const unsigned tiles = (unsigned)((m + tp - 1) / tp);  // a bound: the pair count is on the device
    const auto k_sg_group_pairs = bgv::k_sg_group_pairs<kB>;  // one profiler name per kernel
    const auto k_sg_sum_cells = bgv::k_sg_sum_cells<kB>;
    const auto k_sg_pair_min = bgv::k_sg_pair_min<kB>;
    BGV_LAUNCH(k_sg_group_pairs, dim3(tiles), dim3(kSkThreads), 0, s, superedges, w.run_start, &w.counters[1],
               nkeys_d, super_label, h2, rows, cols, nb, tp, w.ent, w.etab, w.pcnt, se_count);
    BGV_LAUNCH(k_sg_sum_cells, dim3(sg_sum_grid(nb)), dim3(kSkResolveThreads), 0, s, w.ent, w.est, w.etab, w.pcnt,
               &w.counters[1], rows, nb, tp, cells, sk_sum_lanes(tiles, tp, rows, nb), M2);
    BGV_LAUNCH(k_sg_pair_min, dim3(tiles), dim3(kSgThreads), 0, s, w.ent, w.est, w.etab, &w.counters[1], rows, nb,
               tp, se_weight);
    return BGV_OK;
}

static bool sg_valid(int32_t n, int64_t m, const bgv_sketch_params *s) {
    return s && n >= 1 && m >= 0 && m <= INT32_MAX && s->rows >= 1 && s->rows <= kMaxRows && s->cols >= 1 &&
           s->coef1 && s->coef2;
}


}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_supergraph_workspace(int32_t n, int64_t m, const bgv_sketch_params *s) {
    if (!sg_valid(n, m, s)) return 0;
    Carver c(nullptr);
    SgWs w;
    return sg_layout(c, n, m, s->rows, (int64_t)s->rows * s->cols, &w);
}

extern "C" bgv_status bgv_supergraph(int32_t n, int64_t m, const int32_t *edges, const int32_t *labels,
                                     const int32_t *degree, const bgv_sketch_params *sp, int32_t *K_out,
                                     int64_t *E_out, int32_t *super_label, uint32_t *super_size,
                                     int32_t *node_super, int32_t *superedges, uint32_t *se_weight,
                                     uint32_t *se_count, uint32_t *M1, uint32_t *M2, void *ws, size_t ws_bytes,
                                     bgv_stream_t stream) {
    clear_error();
    if (!sg_valid(n, m, sp)) {
        set_error("bgv_supergraph: invalid arguments (n=%d m=%lld)", n, (long long)m);
        return BGV_E_INVALID;
    }
    if ((m > 0 && (!edges || !superedges || !se_weight)) || !labels || !degree || !K_out || !E_out ||
        !super_label || !super_size || !M1 || !M2) {
        set_error("bgv_supergraph: null pointer");
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_supergraph_workspace(n, m, sp)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (range_check_on()) {  // super_label[0] holds the flag; it is written below
        BGV_TRY(check_edge_ids(n, m, edges, super_label, s));
        BGV_TRY(check_id_list(n, labels, n, super_label, s));
    }
    Carver c(ws);
    SgWs w;
    sg_layout(c, n, m, sp->rows, (int64_t)sp->rows * sp->cols, &w);
    const int rows = sp->rows;
    const uint32_t cols = (uint32_t)sp->cols;
    const HashRows h1 = make_hash_rows(sp->coef1, rows), h2 = make_hash_rows(sp->coef2, rows);
    const int2 *e2 = reinterpret_cast<const int2 *>(edges);
    const unsigned gn = grid_for(n, kSgThreads, 65536);

    // supernodes
    // a sketch small enough for LDS takes the node degrees directly; a larger one is
    // filled from the communities' volumes
    const int64_t cells = (int64_t)rows * cols;
    const bool lds_sketch = cells <= kLdsCounters;
    BGV_TRY(fill<uint32_t>(w.counters, 0u, 8, s));
    if (lds_sketch) {
        BGV_TRY(fill<uint32_t>(w.flag, 0u, n, s));
        BGV_LAUNCH(k_sg_flag, dim3(gn), dim3(kSgThreads), 0, s, labels, n, w.flag);
    } else if (w.lent) {
        // flags and volumes grouped by label bucket, written whole
        const int32_t lnb = lb_buckets(n);
        const int32_t ltiles = (int32_t)(((int64_t)n + kLbTile - 1) / kLbTile);
        BGV_LAUNCH(k_sg_group_nodes, dim3((unsigned)ltiles), dim3(kSgThreads), 0, s, labels, degree, n, lnb, w.lent,
                   w.ltab);
        BGV_LAUNCH(k_sg_sum_labels, dim3((unsigned)lnb), dim3(kLbResolveThreads), 0, s, w.lent, w.ltab, ltiles, lnb,
                   n, lb_lanes(ltiles), w.flag, w.vol);
    } else {
        BGV_TRY(fill<uint32_t>(w.flag, 0u, n, s));
        BGV_TRY(fill<uint32_t>(w.vol, 0u, n, s));
        BGV_LAUNCH(k_sg_flag_volume, dim3(gn), dim3(kSgThreads), 0, s, labels, degree, n, w.flag, w.vol);
    }
    BGV_TRY(exclusive_scan_u32(w.flag, w.sid, n, &w.counters[0], w.scan_scratch, s));
    BGV_LAUNCH(k_sg_compact, dim3(gn), dim3(kSgThreads), 0, s, w.flag, w.sid, n, super_label);
    // K sizes the packed superedge keys: read it back while the sketch-1 work below runs
    SgReadback *rb;
    BGV_TRY(sg_readback(&rb));
    BGV_CHECK_HIP(hipMemcpyAsync(rb->host, &w.counters[0], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    BGV_CHECK_HIP(hipEventRecord(rb->ev, s));

    // sketch 1 and sizes
    BGV_TRY(fill<uint32_t>(M1, 0u, cells, s));
    const bool grouped_sketch = w.ent != nullptr;  // sketch 2 written whole by k_sg_sum_cells
    if (!grouped_sketch) BGV_TRY(fill<uint32_t>(M2, 0u, cells, s));
    if (lds_sketch) {
        BGV_LAUNCH(k_sg_sketch_nodes_lds, dim3(grid_for(n, kSgThreads * 16, 1024)), dim3(kSgThreads), 0, s,
                   labels, degree, n, h1, rows, cols, M1);
    } else {
        BGV_LAUNCH(k_sg_sketch_volumes, dim3(gn), dim3(kSgThreads), 0, s, super_label, &w.counters[0], w.vol, h1,
                   rows, cols, M1);
    }
    BGV_LAUNCH(k_sg_super_size, dim3(gn), dim3(kSgThreads), 0, s, super_label, &w.counters[0], h1, rows, cols,
                       M1, super_size);
    BGV_LAUNCH(k_sg_node_super, dim3(gn), dim3(kSgThreads), 0, s, labels, w.sid, n, w.nsid, w.nsid16, node_super);

    BGV_TRY(sg_wait(rb->ev));
    const uint32_t Kh = rb->host[0];
    *K_out = (int32_t)Kh;
    int kbits = 1;
    while (kbits < 31 && (1u << kbits) < Kh) ++kbits;

    // inter-community keys, sorted and made unique, then sketch 2 and the weights
    unsigned long long *nkeys_d = reinterpret_cast<unsigned long long *>(&w.counters[2]);
    // one profiler name per key width
    const auto k_sg_edge_keys_32 = k_sg_edge_keys<uint32_t, uint16_t>;
    const auto k_sg_edge_keys_64 = k_sg_edge_keys<uint64_t, uint32_t>;
    const bool k32 = 2 * kbits <= 32;  // keys in 32 bits: half the sort traffic
    uint32_t *keys32 = reinterpret_cast<uint32_t *>(w.keys), *keys32_alt = reinterpret_cast<uint32_t *>(w.keys_alt);
    // the one-sweep sort's digit counts come from the key launch, its workgroups' counts
    // written into the sort's second key buffer (free until the first pass; 256 words
    // per workgroup and pass, at most 2 words per edge)
    const int64_t nkb = (m + kSgThreads * kKeyItems - 1) / (kSgThreads * kKeyItems);
    const int passes = onesweep_key_passes(2 * kbits);
    const bool fused_count = sg_onesweep(m) && nkb * passes * 256 <= 2 * m;
    uint32_t *bcnt = fused_count ? reinterpret_cast<uint32_t *>(w.keys_alt) : nullptr;
    if (m > 0) {
        const dim3 gkey((unsigned)nkb);
        if (k32)
            BGV_LAUNCH(k_sg_edge_keys_32, gkey, dim3(kSgThreads), 0, s, e2, m, w.nsid16, kbits, keys32, nkeys_d, bcnt,
                       passes);
        else
            BGV_LAUNCH(k_sg_edge_keys_64, gkey, dim3(kSgThreads), 0, s, e2, m, w.nsid, kbits, w.keys, nkeys_d, bcnt,
                       passes);
        if (fused_count) BGV_TRY(onesweep_keys_counted(bcnt, nkb, m, 2 * kbits, !k32, w.sort_scratch, s));
    }
    // the key count stays on the device: everything below is sized by the edge count m,
    // which bounds it, and reads the count itself, so no host round trip is needed here
    int64_t E = 0;
    if (m == 0 && grouped_sketch) BGV_TRY(fill<uint32_t>(M2, 0u, cells, s));
    if (m > 0) {
        uint64_t *sorted = nullptr;
        uint32_t *sorted32 = nullptr;
        if (sg_onesweep(m)) {
            if (k32)
                BGV_TRY(onesweep_sort_keys<uint32_t>(keys32, keys32_alt, m, nkeys_d, 2 * kbits, &sorted32,
                                                     w.sort_scratch, s, fused_count));
            else
                BGV_TRY(onesweep_sort_keys<uint64_t>(w.keys, w.keys_alt, m, nkeys_d, 2 * kbits, &sorted,
                                                     w.sort_scratch, s, fused_count));
        } else if (k32) {
            BGV_TRY(radix_sort_u32(keys32, keys32_alt, nullptr, nullptr, m, 2 * kbits, &sorted32, nullptr,
                                   w.sort_scratch, s, false, nkeys_d));
        } else {
            BGV_TRY(radix_sort_u64(w.keys, w.keys_alt, nullptr, nullptr, m, 2 * kbits, &sorted, nullptr,
                                   w.sort_scratch, s, false, nkeys_d));
        }
        const unsigned gk = grid_for(m, kSgThreads, 65536);
        const unsigned ut = (unsigned)((m + kUqTile - 1) / kUqTile);
        if (k32)
            BGV_LAUNCH(k_sg_unique_count<uint32_t>, dim3(ut), dim3(kSgThreads), 0, s, sorted32, nkeys_d, w.utile);
        else
            BGV_LAUNCH(k_sg_unique_count<uint64_t>, dim3(ut), dim3(kSgThreads), 0, s, sorted, nkeys_d, w.utile);
        BGV_TRY(exclusive_scan_u32(w.utile, w.utile, (int64_t)ut, &w.counters[1], w.scan_scratch, s));
        if (k32)
            BGV_LAUNCH(k_sg_unique_write<uint32_t>, dim3(ut), dim3(kSgThreads), 0, s, sorted32, nkeys_d, w.utile,
                       kbits, superedges, w.run_start);
        else
            BGV_LAUNCH(k_sg_unique_write<uint64_t>, dim3(ut), dim3(kSgThreads), 0, s, sorted, nkeys_d, w.utile,
                       kbits, superedges, w.run_start);
        if (grouped_sketch) {
            if (sk_bucket_bits(cells) == 15)
                BGV_TRY(sg_sketch2_grouped<15>(m, w, superedges, nkeys_d, super_label, h2, rows, cols, cells, se_count,
                                               M2, se_weight, s));
            else
                BGV_TRY(sg_sketch2_grouped<14>(m, w, superedges, nkeys_d, super_label, h2, rows, cols, cells, se_count,
                                               M2, se_weight, s));
        } else {
            BGV_LAUNCH(k_sg_sketch_pairs, dim3(gk), dim3(kSgThreads), 0, s, superedges, w.run_start, &w.counters[1],
                       nkeys_d, super_label, h2, rows, cols, M2, se_count);
            BGV_LAUNCH(k_sg_pair_weights, dim3(gk), dim3(kSgThreads), 0, s, superedges, &w.counters[1], super_label,
                       h2, rows, cols, M2, se_weight);
        }
        BGV_CHECK_HIP(hipMemcpyAsync(rb->host + 4, &w.counters[1], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        BGV_CHECK_HIP(hipEventRecord(rb->ev, s));
        BGV_TRY(sg_wait(rb->ev));
        E = rb->host[4];
    }
    *E_out = E;
    return BGV_OK;
}
