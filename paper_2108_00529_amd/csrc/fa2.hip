// ForceAtlas2 layout (Section 3.1 / Algorithm 1; force and speed laws of the cited
// ForceAtlas2 publication) on gfx950.
//
// Setup: directed CSR of the undirected edge list (own LSD radix sort, so neighbour
// order and therefore every FP sum is deterministic).
// Per iteration:
//   both:   k_attract       attraction, one wavefront per CSR row
//   exact:  k_force_exact   LDS-tiled all-pairs repulsion (split into 512-body segments
//                           summed by k_force_combine when K is larger) + attraction +
//                           gravity, swing/traction, FP64 block partials of the two sums
//   BH:     k_bh_bbox -> k_bh_codes -> radix sort -> k_bh_gather -> FP64 prefix sums
//           -> k_bh_build_attract (binary radix tree: centre of mass of a node =
//           difference of prefix sums over its body range, so no atomics; the
//           attraction in the same launch) -> k_bh_force (traversal with a shared
//           stack per body)
//   exact:  k_update        global speed from the partials (every block reduces them in
//                           the same order), local speeds, displacement
//   BH:     k_bh_speed      global speed from the partials (one per 8 bodies) in one block
//           k_bh_update     local speeds, displacement, bounding-box partials
// No floating-point atomics anywhere: results are identical run to run.
#include <algorithm>
#include <climits>
#include <cstddef>
#include <cstring>
#include <mutex>

#include "block_scan.h"
#include "common.h"
#include "fa2_internal.h"
#include "fa2_math.h"

namespace bgv {

constexpr int kFaThreads = 256;
static_assert(kFaThreads == kFa2Tile, "the layout kernels work on 256-node tiles");

// Column-blocked attraction (CsrWs::cols): blocks of kAttCol consecutive neighbour ids,
// whose positions fill 128 KiB of LDS; items of at most kAttCap entries of one row in
// one block, summed by kAttColLanes lanes each.
constexpr int kAttColBits = 14;
constexpr int32_t kAttCol = 1 << kAttColBits;
constexpr uint32_t kAttCap = 256;
constexpr int kAttLenBits = 9;  // kAttCap - length, in the low bits of an item's sort key
static_assert(kAttCap < (1u << kAttLenBits), "item lengths must fit the key field");
constexpr int kAttColLanes = 8;
constexpr int kAttColThreads = 1024;
inline int32_t att_col_blocks(int32_t K) { return (K + kAttCol - 1) / kAttCol; }

// ------------------------------------------------------------------------ CSR ----
template <typename KT>  // 32-bit keys when 2 * kb <= 32
__global__ void k_csr_keys(const int2 *__restrict__ edges, int64_t E, int kb, KT *__restrict__ keys,
                           uint32_t *__restrict__ vals) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const int2 p = edges[e];
        keys[2 * e] = ((KT)(uint32_t)p.x << kb) | (KT)(uint32_t)p.y;
        keys[2 * e + 1] = ((KT)(uint32_t)p.y << kb) | (KT)(uint32_t)p.x;
        vals[2 * e] = (uint32_t)e;
        vals[2 * e + 1] = (uint32_t)e;
    }
}

template <typename KT>
__global__ void k_csr_fill(const KT *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t nent,
                           int kb, int32_t K, const float *__restrict__ attr_w, int fmt, uint32_t *__restrict__ row,
                           int2 *__restrict__ cw) {
    const uint64_t mask = (1ull << kb) - 1ull;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nent; k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[k];
        const int64_t src = (int64_t)(key >> kb);
        const int32_t nb = (int32_t)(key & mask);
        if (fmt == kCsrWeighted)
            cw[k] = make_int2(nb, __float_as_int(attr_w[vals[k]]));
        else if (fmt == kCsrIds32)
            reinterpret_cast<uint32_t *>(cw)[k] = (uint32_t)nb;
        else
            reinterpret_cast<uint16_t *>(cw)[k] = (uint16_t)nb;
        const int64_t prev = k ? (int64_t)(keys[k - 1] >> kb) : -1;
        for (int64_t r = prev + 1; r <= src; ++r) row[r] = (uint32_t)k;
        if (k == nent - 1)
            for (int64_t r = src + 1; r <= K; ++r) row[r] = (uint32_t)nent;
    }
}

__global__ void k_csr_mass(const uint32_t *__restrict__ row, int32_t K, float *__restrict__ mass) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        mass[i] = (float)(row[i + 1] - row[i]) + 1.0f;
}

static int bits_for(int64_t K) {
    int kb = 1;
    while (kb < 31 && (1ll << kb) < K) ++kb;
    return kb;
}

int64_t att_items_cap(int32_t K, int64_t E, bool cols) {
    if (!cols) return (int64_t)K + (2 * E) / kAttBlock + 1;
    // every row one item, every further block run one more, every kAttCap entries of a
    // run one more
    const int64_t runs = std::min<int64_t>(2 * E, (int64_t)K * att_col_blocks(K));
    return (int64_t)K + runs + (2 * E) / kAttCap + 1;
}

size_t csr_layout(Carver &c, int32_t K, int64_t E, CsrWs *w, bool allow_cols) {
    const int64_t nent = 2 * E > 0 ? 2 * E : 1;
    w->row = c.take<uint32_t>((size_t)K + 1);
    w->cw = c.take<int2>((size_t)nent);
    w->mass = c.take<float>((size_t)K);
    w->cols = allow_cols && att_cols(K);
    w->items_bound = att_items_cap(K, E, w->cols);
    w->item_of = c.take<uint32_t>((size_t)K + 1);
    w->item_row = c.take<uint32_t>((size_t)w->items_bound);
    const bool cols = w->cols;
    const int64_t nblk = cols ? att_col_blocks(K) : 0;
    // column-blocked entries: nent plus the padding of each block's groups, at most one
    // group's worth per block (lengths fall within a block, so a group's padding is at
    // most the previous group's entries)
    const int64_t cwb_slots = nent + nblk * kWave * (int64_t)kAttCap;
    w->keys = c.take<uint64_t>((size_t)std::max<int64_t>(nent, cols ? cwb_slots : 0));
    size_t scratch = std::max(radix_workspace(nent), scan_workspace((int64_t)K + 1));
    w->it = w->ir = w->cstart = w->gfirst = w->gbase = w->wg_first = nullptr;
    w->il = nullptr;
    w->item_beg = w->ikeys = w->ikeys_alt = w->ivals = w->ivals_alt = w->ilen = nullptr;
    w->cwb = nullptr;
    w->nitems = nullptr;
    const int64_t T = w->items_bound;
    const int64_t ngroups = T / kWave + nblk + 1;  // bound on the groups of 64
    if (cols) {
        w->it = c.take<uint32_t>((size_t)T);
        w->ir = c.take<uint32_t>((size_t)T);
        w->il = c.take<uint16_t>((size_t)T);
        w->cstart = c.take<uint32_t>((size_t)nblk + 1);
        w->gfirst = c.take<uint32_t>((size_t)nblk + 1);
        w->gbase = c.take<uint32_t>((size_t)ngroups + 1);
        w->wg_first = c.take<uint32_t>((size_t)nblk + 1);
        w->nitems = c.take<unsigned long long>(1);
        w->cwb = w->keys;  // free once the CSR is filled
    }
    // the CSR sort's other buffers and the item setup's are both dead once the CSR is
    // built, so they share one region
    char *const r0 = c.base ? c.base + c.size() : nullptr;
    Carver a(r0);
    w->keys_alt = a.take<uint64_t>((size_t)nent);
    w->vals = a.take<uint32_t>((size_t)nent);
    w->vals_alt = a.take<uint32_t>((size_t)nent);
    size_t region = a.size();
    if (cols) {
        Carver b(r0);
        w->item_beg = b.take<uint32_t>((size_t)T + 1);
        w->ikeys = b.take<uint32_t>((size_t)T);
        w->ikeys_alt = b.take<uint32_t>((size_t)T);
        w->ivals = b.take<uint32_t>((size_t)T);
        w->ivals_alt = b.take<uint32_t>((size_t)T);
        w->ilen = b.take<uint32_t>((size_t)std::max<int64_t>(T, ngroups + 1));
        region = std::max(region, b.size());
        scratch = std::max(scratch, std::max(radix_workspace(T), scan_workspace(std::max<int64_t>(T, ngroups + 1))));
    }
    c.take<char>(region);
    w->sort_scratch = c.take<char>(scratch);
    return c.size();
}

// Work items of the attraction: max(1, ceil(row length / kAttBlock)) per row, turned
// into first-item offsets by an exclusive scan, then each item's row.
__global__ void k_att_item_counts(const uint32_t *__restrict__ row, int32_t K, uint32_t *__restrict__ item_of) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= K; i += (int64_t)gridDim.x * blockDim.x) {
        if (i == K) {
            item_of[i] = 0u;
        } else {
            const uint32_t len = row[i + 1] - row[i];
            item_of[i] = len > kAttBlock ? (len + kAttBlock - 1) / kAttBlock : 1u;
        }
    }
}

__global__ void k_att_item_rows(const uint32_t *__restrict__ item_of, int32_t K, uint32_t *__restrict__ item_row) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        for (uint32_t t = item_of[i]; t < item_of[i + 1]; ++t) item_row[t] = (uint32_t)i;
}

// --------------------------------------------------- column-blocked item setup ----
// Item starts of row r (entries [r0, r1), neighbours ascending, so a row's column
// blocks come in runs in ascending order), one wavefront per row: entry k starts an
// item when it opens a block run or lies a multiple of kAttCap entries after the start
// of its run.  f(k, j) is called by the lane holding each start, j = the start's rank
// in the row.  Returns the number of starts.
template <typename E, typename F>
__device__ __forceinline__ uint32_t attc_walk(const E *__restrict__ cw, uint32_t r0, uint32_t r1, int lane, F f) {
    uint32_t run = r0, count = 0;
    int32_t prev_blk = -1;
    for (uint32_t c0 = r0; c0 < r1; c0 += kWave) {
        const uint32_t k = c0 + (uint32_t)lane;
        const bool in = k < r1;
        const int32_t blk = in ? (fa2_entry_id(cw[k]) >> kAttColBits) : INT_MAX;
        int32_t before = __shfl_up(blk, 1, kWave);
        if (lane == 0) before = prev_blk;
        // latest run start at or before each lane: an inclusive max-scan
        uint32_t rs = (in && blk != before) ? k : run;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t v = __shfl_up(rs, o, kWave);
            if (lane >= o) rs = max(rs, v);
        }
        const bool start = in && ((k - rs) & (kAttCap - 1)) == 0;
        const uint64_t m = __ballot(start);
        if (start) f(k, count + (uint32_t)__popcll(m & ((1ull << lane) - 1ull)));
        count += (uint32_t)__popcll(m);
        run = __shfl(rs, kWave - 1, kWave);
        prev_blk = __shfl(blk, kWave - 1, kWave);
    }
    return count;
}

// item_of[r] = items of row r (at least one: an empty row has one empty item);
// item_of[K] = 0 for the scan that follows.
template <typename E>
__global__ void __launch_bounds__(kFaThreads) k_attc_count(const uint32_t *__restrict__ row, const E *__restrict__ cw,
                                                            int32_t K, uint32_t *__restrict__ item_of) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (kFaThreads / kWave);
    for (int64_t r = (blockIdx.x * (int64_t)kFaThreads + threadIdx.x) / kWave; r <= K; r += nw) {
        if (r == K) {
            if (lane == 0) item_of[K] = 0u;
            continue;
        }
        const uint32_t n = attc_walk(cw, row[r], row[r + 1], lane, [](uint32_t, uint32_t) {});
        if (lane == 0) item_of[r] = n ? n : 1u;
    }
}

// item_row and item_beg of every item (item_of now holds first-item offsets), the item
// count in *nitems and item_beg[count] = nent.
template <typename E>
__global__ void __launch_bounds__(kFaThreads) k_attc_fill(const uint32_t *__restrict__ row, const E *__restrict__ cw,
                                                           int32_t K, const uint32_t *__restrict__ item_of,
                                                           uint32_t nent, uint32_t *__restrict__ item_row,
                                                           uint32_t *__restrict__ item_beg,
                                                           unsigned long long *__restrict__ nitems) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (kFaThreads / kWave);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        item_beg[item_of[K]] = nent;
        *nitems = item_of[K];
    }
    for (int64_t r = (blockIdx.x * (int64_t)kFaThreads + threadIdx.x) / kWave; r < K; r += nw) {
        const uint32_t r0 = row[r], r1 = row[r + 1], base = item_of[r];
        if (r0 == r1) {
            if (lane == 0) {
                item_row[base] = (uint32_t)r;
                item_beg[base] = r0;
            }
            continue;
        }
        attc_walk(cw, r0, r1, lane, [&](uint32_t k, uint32_t j) {
            item_row[base + j] = (uint32_t)r;
            item_beg[base + j] = k;
        });
    }
}

// Sort keys of the items: column block above, kAttCap - length below (so each block's
// items come longest first); an empty item goes with block 0.
template <typename E>
__global__ void k_attc_keys(const E *__restrict__ cw, const uint32_t *__restrict__ item_beg,
                            const unsigned long long *__restrict__ nitems, uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ vals) {
    const uint32_t T = (uint32_t)*nitems;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
        const uint32_t b = item_beg[t], len = item_beg[t + 1] - b;
        const uint32_t blk = len ? (uint32_t)fa2_entry_id(cw[b]) >> kAttColBits : 0u;
        keys[t] = (blk << kAttLenBits) | (kAttCap - len);
        vals[t] = t;
    }
}

// The first schedule position of every column block (items sorted by their keys).
__global__ void k_attc_order(const uint32_t *__restrict__ skeys, const unsigned long long *__restrict__ nitems,
                             int32_t nblk, uint32_t *__restrict__ cstart) {
    const uint32_t T = (uint32_t)*nitems;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < T; q += gridDim.x * blockDim.x) {
        const int32_t c = (int32_t)(skeys[q] >> kAttLenBits);
        const int32_t before = q ? (int32_t)(skeys[q - 1] >> kAttLenBits) : -1;
        for (int32_t x = before + 1; x <= c; ++x) cstart[x] = q;
        if (q == T - 1)
            for (int32_t x = c + 1; x <= nblk; ++x) cstart[x] = T;
    }
}

// gfirst[c] = first group of block c (groups of kWave consecutive items of a block).
__global__ void k_attc_gfirst(int32_t nblk, const uint32_t *__restrict__ cstart, uint32_t *__restrict__ gfirst) {
    if (threadIdx.x != 0) return;
    uint32_t g = 0;
    for (int32_t c = 0; c < nblk; ++c) {
        gfirst[c] = g;
        g += (cstart[c + 1] - cstart[c] + kWave - 1) / kWave;
    }
    gfirst[nblk] = g;
}

__device__ __forceinline__ int32_t attc_block_of(const uint32_t *__restrict__ first, int32_t nblk, uint32_t x) {
    int32_t lo = 0, hi = nblk - 1;  // the last c with first[c] <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// gsize[gi] = kWave * (length of the group's first item, its longest); 0 past the groups.
__global__ void k_attc_gsize(const uint32_t *__restrict__ svals, const uint32_t *__restrict__ item_beg,
                             int32_t nblk, const uint32_t *__restrict__ cstart, const uint32_t *__restrict__ gfirst,
                             int64_t bound, uint32_t *__restrict__ gsize) {
    const uint32_t NG = gfirst[nblk];
    for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < bound; gi += (int64_t)gridDim.x * blockDim.x) {
        if (gi >= NG) {
            gsize[gi] = 0u;
            continue;
        }
        const int32_t c = attc_block_of(gfirst, nblk, (uint32_t)gi);
        const uint32_t q0 = cstart[c] + ((uint32_t)gi - gfirst[c]) * kWave;
        const uint32_t t = svals[q0];
        gsize[gi] = kWave * (item_beg[t + 1] - item_beg[t]);
    }
}

// The schedule arrays and the entries, copied transposed per group (gbase = exclusive
// sums of gsize), neighbour ids replaced by their offsets in the block; kAttColLanes
// lanes per item.
__device__ __forceinline__ uint16_t attc_local(uint32_t e, int32_t base) { return (uint16_t)((int32_t)e - base); }
__device__ __forceinline__ uint16_t attc_local(uint16_t e, int32_t base) { return (uint16_t)((int32_t)e - base); }
__device__ __forceinline__ int2 attc_local(int2 e, int32_t base) { return make_int2(e.x - base, e.y); }

template <typename E, typename EC>
__global__ void k_attc_copy(const E *__restrict__ cw, const uint32_t *__restrict__ skeys,
                            const uint32_t *__restrict__ svals, const unsigned long long *__restrict__ nitems,
                            const uint32_t *__restrict__ item_beg, const uint32_t *__restrict__ item_row,
                            const uint32_t *__restrict__ cstart, const uint32_t *__restrict__ gfirst,
                            const uint32_t *__restrict__ gbase, uint32_t *__restrict__ it, uint32_t *__restrict__ ir,
                            uint16_t *__restrict__ il, EC *__restrict__ cwb) {
    const uint32_t T = (uint32_t)*nitems;
    const uint32_t L = threadIdx.x % kAttColLanes;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kAttColLanes);
    for (int64_t q = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kAttColLanes; q < T; q += groups) {
        const int32_t c = (int32_t)(skeys[q] >> kAttLenBits);
        const uint32_t off = (uint32_t)q - cstart[c];
        const uint32_t lane = off % kWave;
        const uint32_t eb = gbase[gfirst[c] + off / kWave];
        const uint32_t t = svals[q], b = item_beg[t], len = item_beg[t + 1] - b;
        const int32_t base = c << kAttColBits;
        for (uint32_t k = L; k < len; k += kAttColLanes) cwb[eb + k * kWave + lane] = attc_local(cw[b + k], base);
        if (L == 0) {
            it[q] = t;
            ir[q] = item_row[t];
            il[q] = (uint16_t)len;
        }
    }
}

// Workgroups of the column-blocked attraction per block: one each, and the other
// G - nblk shared out in proportion to the block's work (the longest entry of each of
// its groups, plus 8 per group), so that the blocks finish together.
__global__ void k_attc_plan(int32_t nblk, int32_t G, const uint32_t *__restrict__ gfirst,
                            const uint32_t *__restrict__ gbase, uint32_t *__restrict__ wg_first) {
    if (threadIdx.x != 0) return;
    uint64_t total = 0;
    for (int32_t c = 0; c < nblk; ++c)
        total += (gbase[gfirst[c + 1]] - gbase[gfirst[c]]) / kWave + 8ull * (gfirst[c + 1] - gfirst[c]);
    const uint64_t spare = (uint64_t)(G - nblk);
    uint64_t run = 0;
    for (int32_t c = 0; c < nblk; ++c) {
        wg_first[c] = (uint32_t)c + (uint32_t)(total ? spare * run / total : 0);
        run += (gbase[gfirst[c + 1]] - gbase[gfirst[c]]) / kWave + 8ull * (gfirst[c + 1] - gfirst[c]);
    }
    wg_first[nblk] = (uint32_t)G;
}

static bgv_status att_col_grid(int32_t K, int32_t *G) {
    int cus = 1;
    BGV_TRY(device_cu_count(&cus));
    *G = std::max(cus, att_col_blocks(K));
    return BGV_OK;
}

template <typename E, typename EC>
static bgv_status attc_setup(int32_t K, int64_t nent, CsrWs &w, hipStream_t s) {
    const E *cw = reinterpret_cast<const E *>(w.cw);
    const int64_t T = w.items_bound;
    const int32_t nblk = att_col_blocks(K);
    const int64_t ngroups = T / kWave + nblk + 1;
    const dim3 gr(grid_for((int64_t)K + 1, kFaThreads / kWave, 65536));
    BGV_LAUNCH(k_attc_count<E>, gr, dim3(kFaThreads), 0, s, w.row, cw, K, w.item_of);
    BGV_TRY(exclusive_scan_u32(w.item_of, w.item_of, (int64_t)K + 1, nullptr, w.sort_scratch, s));
    BGV_LAUNCH(k_attc_fill<E>, gr, dim3(kFaThreads), 0, s, w.row, cw, K, w.item_of, (uint32_t)nent, w.item_row,
               w.item_beg, w.nitems);
    const dim3 gt(grid_for(T, kFaThreads, 65536));
    BGV_LAUNCH(k_attc_keys<E>, gt, dim3(kFaThreads), 0, s, cw, w.item_beg, w.nitems, w.ikeys, w.ivals);
    int kbits = kAttLenBits + 1;
    while ((1ll << (kbits - kAttLenBits)) < nblk) ++kbits;
    uint32_t *sk, *sv;
    BGV_TRY(radix_sort_u32(w.ikeys, w.ikeys_alt, w.ivals, w.ivals_alt, T, kbits, &sk, &sv, w.sort_scratch, s, false,
                           w.nitems));
    BGV_LAUNCH(k_attc_order, gt, dim3(kFaThreads), 0, s, sk, w.nitems, nblk, w.cstart);
    BGV_LAUNCH(k_attc_gfirst, dim3(1), dim3(64), 0, s, nblk, w.cstart, w.gfirst);
    BGV_LAUNCH(k_attc_gsize, dim3(grid_for(ngroups + 1, kFaThreads, 65536)), dim3(kFaThreads), 0, s, sv, w.item_beg,
               nblk, w.cstart, w.gfirst, ngroups + 1, w.ilen);
    BGV_TRY(exclusive_scan_u32(w.ilen, w.gbase, ngroups + 1, nullptr, w.sort_scratch, s));
    const auto k_attc_copy_ = k_attc_copy<E, EC>;
    BGV_LAUNCH(k_attc_copy_, dim3(grid_for(T, kFaThreads / kAttColLanes, 65536)), dim3(kFaThreads), 0, s, cw, sk, sv,
               w.nitems, w.item_beg, w.item_row, w.cstart, w.gfirst, w.gbase, w.it, w.ir, w.il,
               reinterpret_cast<EC *>(w.cwb));
    int32_t G = 1;
    BGV_TRY(att_col_grid(K, &G));
    BGV_LAUNCH(k_attc_plan, dim3(1), dim3(64), 0, s, nblk, G, w.gfirst, w.gbase, w.wg_first);
    return BGV_OK;
}

bgv_status build_csr(int32_t K, int64_t E, const int32_t *edges, const float *attr_w, const float *mass_in,
                     CsrWs &w, hipStream_t s, const float **mass_out) {
    w.fmt = attr_w ? kCsrWeighted : (K <= 65536 ? kCsrIds16 : kCsrIds32);
    if (E == 0) {
        BGV_TRY(fill<uint32_t>(w.row, 0u, (int64_t)K + 1, s));
    } else {
        const int kb = bits_for(K);
        const int2 *e2 = reinterpret_cast<const int2 *>(edges);
        const dim3 ge(grid_for(E, kFaThreads, 65536)), gf(grid_for(2 * E, kFaThreads, 65536));
        uint32_t *sv;
        if (2 * kb <= 32) {  // keys in 32 bits: half the sort traffic
            uint32_t *k32 = reinterpret_cast<uint32_t *>(w.keys), *k32_alt = reinterpret_cast<uint32_t *>(w.keys_alt);
            uint32_t *sk;
            BGV_LAUNCH(k_csr_keys<uint32_t>, ge, dim3(kFaThreads), 0, s, e2, E, kb, k32, w.vals);
            BGV_TRY(radix_sort_u32(k32, k32_alt, w.vals, w.vals_alt, 2 * E, 2 * kb, &sk, &sv, w.sort_scratch, s));
            BGV_LAUNCH(k_csr_fill<uint32_t>, gf, dim3(kFaThreads), 0, s, sk, sv, 2 * E, kb, K, attr_w, w.fmt, w.row,
                       w.cw);
        } else {
            uint64_t *sk;
            BGV_LAUNCH(k_csr_keys<uint64_t>, ge, dim3(kFaThreads), 0, s, e2, E, kb, w.keys, w.vals);
            BGV_TRY(radix_sort_u64(w.keys, w.keys_alt, w.vals, w.vals_alt, 2 * E, 2 * kb, &sk, &sv, w.sort_scratch,
                                   s));
            BGV_LAUNCH(k_csr_fill<uint64_t>, gf, dim3(kFaThreads), 0, s, sk, sv, 2 * E, kb, K, attr_w, w.fmt, w.row,
                       w.cw);
        }
    }
    if (w.cols) {
        if (w.fmt == kCsrWeighted)
            BGV_TRY((attc_setup<int2, int2>(K, 2 * E, w, s)));
        else if (w.fmt == kCsrIds32)
            BGV_TRY((attc_setup<uint32_t, uint16_t>(K, 2 * E, w, s)));
        else
            BGV_TRY((attc_setup<uint16_t, uint16_t>(K, 2 * E, w, s)));
    } else {
        BGV_LAUNCH(k_att_item_counts, dim3(grid_for((int64_t)K + 1, kFaThreads, 65536)), dim3(kFaThreads), 0, s,
                   w.row, K, w.item_of);
        BGV_TRY(exclusive_scan_u32(w.item_of, w.item_of, (int64_t)K + 1, nullptr, w.sort_scratch, s));
        BGV_LAUNCH(k_att_item_rows, dim3(grid_for(K, kFaThreads, 65536)), dim3(kFaThreads), 0, s, w.item_of, K,
                   w.item_row);
    }
    if (mass_in) {
        *mass_out = mass_in;
    } else {
        BGV_LAUNCH(k_csr_mass, dim3(grid_for(K, kFaThreads, 65536)), dim3(kFaThreads), 0, s, w.row, K,
                           w.mass);
        *mass_out = w.mass;
    }
    return BGV_OK;
}

// --------------------------------------------------------------- reductions ------
// Deterministic block sum of a double2 (fixed shuffle pattern, fixed wave order).
__device__ __forceinline__ double2 block_sum2(double2 v) {
    __shared__ double2 ws[kFaThreads / kWave];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        v.x += __shfl_down(v.x, o, kWave);
        v.y += __shfl_down(v.y, o, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
            r.x += ws[q].x;
            r.y += ws[q].y;
        }
    __syncthreads();
    return r;  // valid in thread 0
}

// Attraction: one wavefront per node; lanes stride over the CSR row and the partial
// sums are combined by a fixed butterfly, so the result does not depend on timing.
// Power-law supernode degrees (rows of thousands of entries next to rows of a few)
// are why a row is not given to a single thread.
// Attraction items wave0, wave0 + nwaves, ... (one per wavefront), positions from pos
// (global memory or an LDS copy).
template <typename E>
__device__ __forceinline__ void att_items(int32_t K, const float2 *__restrict__ pos, const uint32_t *__restrict__ row,
                                          const E *__restrict__ cw, const uint32_t *__restrict__ item_of,
                                          const uint32_t *__restrict__ item_row, float2 *__restrict__ A,
                                          int64_t wave0, int64_t nwaves) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t T = item_of[K];
    for (int64_t t = wave0; t < T; t += nwaves) {
        const uint32_t r = item_row[t];
        const uint32_t r1 = row[r + 1];
        const uint32_t b0 = row[r] + ((uint32_t)t - item_of[r]) * kAttBlock;
        const uint32_t b1 = r1 - b0 > kAttBlock ? b0 + kAttBlock : r1;
        const float2 a = fa2_block_attraction(pos, cw, b0, b1, pos[r], lane);
        if (lane == 0) A[t] = a;
    }
}

template <typename E>
__global__ void __launch_bounds__(kFaThreads) k_attract(int32_t K, const float2 *__restrict__ pos,
                                                         const uint32_t *__restrict__ row, const E *__restrict__ cw,
                                                         const uint32_t *__restrict__ item_of,
                                                         const uint32_t *__restrict__ item_row,
                                                         float2 *__restrict__ A) {
    att_items(K, pos, row, cw, item_of, item_row, A, (blockIdx.x * (int64_t)kFaThreads + threadIdx.x) / kWave,
              (int64_t)gridDim.x * (kFaThreads / kWave));
}

// The same with all K positions staged in LDS first (kAttLdsMin <= K <= kAttLdsMax):
// the gathers of the neighbours' positions then read LDS instead of L2.  One workgroup
// of 16 wavefronts per compute unit, so each position array is loaded once per unit.
// Smaller supergraphs keep the plain kernel: their positions stay in L2 anyway and a
// 1024-thread workgroup per unit only adds dispatch time to their short iterations.
constexpr int32_t kAttLdsMin = 4096;  // up to kAttLdsMax: dynamic LDS of K * 8 bytes
constexpr int kAttLdsThreads = 1024;

template <typename E>
__global__ void __launch_bounds__(kAttLdsThreads) k_attract_lds(int32_t K, const float2 *__restrict__ pos,
                                                                 const uint32_t *__restrict__ row,
                                                                 const E *__restrict__ cw,
                                                                 const uint32_t *__restrict__ item_of,
                                                                 const uint32_t *__restrict__ item_row,
                                                                 float2 *__restrict__ A) {
    extern __shared__ float2 sp[];  // K entries
    for (int32_t i = threadIdx.x; i < K; i += kAttLdsThreads) sp[i] = pos[i];
    __syncthreads();
    att_items(K, sp, row, cw, item_of, item_row, A, (blockIdx.x * (int64_t)kAttLdsThreads + threadIdx.x) / kWave,
              (int64_t)gridDim.x * (kAttLdsThreads / kWave));
}

// Column-blocked attraction: the workgroups [wg_first[c], wg_first[c + 1]) of column
// block c (one per compute unit: the block's positions take 128 KiB of LDS) stage the
// block's positions, then their wavefronts take the block's groups in turn, one item
// per lane: the lane adds its item's entries in order, reading them from the group's
// transposed run (coalesced) and the positions from LDS.  Every item sum, and so
// every node's attraction, is identical run to run.
template <typename EC>
__global__ void __launch_bounds__(kAttColThreads) k_attract_cols(int32_t K, int32_t nblk,
                                                                  const uint32_t *__restrict__ wg_first,
                                                                  const float2 *__restrict__ pos,
                                                                  const uint32_t *__restrict__ it,
                                                                  const uint32_t *__restrict__ ir,
                                                                  const uint16_t *__restrict__ il,
                                                                  const uint32_t *__restrict__ cstart,
                                                                  const uint32_t *__restrict__ gfirst,
                                                                  const uint32_t *__restrict__ gbase,
                                                                  const EC *__restrict__ cwb, float2 *__restrict__ A) {
    extern __shared__ float2 sp[];  // kAttCol entries
    const uint32_t x = blockIdx.x;
    const int32_t c = attc_block_of(wg_first, nblk, x);
    const uint32_t g = x - wg_first[c], wpb = wg_first[c + 1] - wg_first[c];
    const int32_t base = c << kAttColBits;
    const int32_t nb = min(kAttCol, K - base);
    for (int32_t i = threadIdx.x; i < nb; i += kAttColThreads) sp[i] = pos[base + i];
    __syncthreads();
    constexpr uint32_t kWaves = kAttColThreads / kWave;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t g0 = gfirst[c], g1 = gfirst[c + 1], qs = cstart[c], qe = cstart[c + 1];
    for (uint32_t gi = g0 + g * kWaves + threadIdx.x / kWave; gi < g1; gi += wpb * kWaves) {
        const uint32_t q = qs + (gi - g0) * kWave + lane;
        if (q >= qe) continue;
        const uint32_t t = it[q], len = il[q];
        const float2 xi = pos[ir[q]];
        const EC *e = cwb + gbase[gi] + lane;
        float ax = 0.f, ay = 0.f;
        uint32_t k = 0;
        for (; k + 4 <= len; k += 4) {
            EC v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = e[(k + u) * kWave];
            float2 xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = sp[fa2_entry_id(v[u])];
#pragma unroll
            for (int u = 0; u < 4; ++u) fa2_entry_add(v[u], xv[u], xi, ax, ay);
        }
        for (; k < len; ++k) {
            const EC v = e[k * kWave];
            fa2_entry_add(v, sp[fa2_entry_id(v)], xi, ax, ay);
        }
        A[t] = make_float2(ax, ay);
    }
}

static bgv_status attraction_cols(int32_t K, const float2 *pos, const CsrWs &csr, float2 *A, hipStream_t s) {
    int32_t G = 1;
    BGV_TRY(att_col_grid(K, &G));
    const int32_t nblk = att_col_blocks(K);
    const size_t lds = sizeof(float2) * (size_t)kAttCol;
    if (csr.fmt == kCsrWeighted)
        BGV_LAUNCH(k_attract_cols<int2>, dim3((unsigned)G), dim3(kAttColThreads), lds, s, K, nblk, csr.wg_first, pos,
                   csr.it, csr.ir, csr.il, csr.cstart, csr.gfirst, csr.gbase, reinterpret_cast<const int2 *>(csr.cwb),
                   A);
    else
        BGV_LAUNCH(k_attract_cols<uint16_t>, dim3((unsigned)G), dim3(kAttColThreads), lds, s, K, nblk, csr.wg_first,
                   pos, csr.it, csr.ir, csr.il, csr.cstart, csr.gfirst, csr.gbase,
                   reinterpret_cast<const uint16_t *>(csr.cwb), A);
    return BGV_OK;
}

bgv_status attraction(int32_t K, const float2 *pos, const CsrWs &csr, float2 *A, hipStream_t s) {
    if (csr.cols) return attraction_cols(K, pos, csr, A, s);
    if (K >= kAttLdsMin && K <= kAttLdsMax) {
        int cus = 1;
        BGV_TRY(device_cu_count(&cus));
        const unsigned wg = (unsigned)((csr.items_bound + kAttLdsThreads / kWave - 1) / (kAttLdsThreads / kWave));
        const dim3 grid(wg < (unsigned)cus ? (wg > 0 ? wg : 1u) : (unsigned)cus);
        const size_t lds = sizeof(float2) * (size_t)K;
        if (csr.fmt == kCsrWeighted)
            BGV_LAUNCH(k_attract_lds<int2>, grid, dim3(kAttLdsThreads), lds, s, K, pos, csr.row, csr.cw, csr.item_of,
                       csr.item_row, A);
        else if (csr.fmt == kCsrIds32)
            BGV_LAUNCH(k_attract_lds<uint32_t>, grid, dim3(kAttLdsThreads), lds, s, K, pos, csr.row,
                       reinterpret_cast<const uint32_t *>(csr.cw), csr.item_of, csr.item_row, A);
        else
            BGV_LAUNCH(k_attract_lds<uint16_t>, grid, dim3(kAttLdsThreads), lds, s, K, pos, csr.row,
                       reinterpret_cast<const uint16_t *>(csr.cw), csr.item_of, csr.item_row, A);
        return BGV_OK;
    }
    // one wavefront per item; the item count is only known on the device, so the grid
    // covers the bound and the kernel reads the count
    const dim3 grid(grid_for(csr.items_bound, kFaThreads / kWave, 16384));
    if (csr.fmt == kCsrWeighted)
        BGV_LAUNCH(k_attract<int2>, grid, dim3(kFaThreads), 0, s, K, pos, csr.row, csr.cw, csr.item_of, csr.item_row, A);
    else if (csr.fmt == kCsrIds32)
        BGV_LAUNCH(k_attract<uint32_t>, grid, dim3(kFaThreads), 0, s, K, pos, csr.row,
                   reinterpret_cast<const uint32_t *>(csr.cw), csr.item_of, csr.item_row, A);
    else
        BGV_LAUNCH(k_attract<uint16_t>, grid, dim3(kFaThreads), 0, s, K, pos, csr.row,
                   reinterpret_cast<const uint16_t *>(csr.cw), csr.item_of, csr.item_row, A);
    return BGV_OK;
}

// ------------------------------------------------------------------ exact ------
// Repulsion of the i tile of block x over the j segment of block y (all of [0, K) when
// kSegmented is false), bodies staged through LDS 256 at a time.  With one segment the
// kernel finishes the force (attraction, gravity, swing, traction and the block's FP64
// partials); with several it stores the segment sums for k_force_combine.
template <bool kSegmented>
__global__ void __launch_bounds__(kFaThreads) k_force_exact(int32_t K, const float2 *__restrict__ pos,
                                                             const float *__restrict__ mass,
                                                             const float2 *__restrict__ att,
                                                             const uint32_t *__restrict__ item_of, float kr, float kg,
                                                             const float2 *__restrict__ fprev, float2 *__restrict__ F,
                                                             double2 *__restrict__ part, float2 *__restrict__ seg) {
    fa2_exact_force_tile<kSegmented>((int32_t)blockIdx.x, (int32_t)blockIdx.y, K, pos, mass, att, item_of, kr, kg,
                                     fprev, F, part, seg);
}

// Segment sums of body i added in ascending segment order, then the rest of the force.
__global__ void __launch_bounds__(kFaThreads) k_force_combine(int32_t K, int32_t nseg,
                                                               const float2 *__restrict__ seg,
                                                               const float2 *__restrict__ pos,
                                                               const float *__restrict__ mass,
                                                               const float2 *__restrict__ att,
                                                               const uint32_t *__restrict__ item_of, float kr, float kg,
                                                               const float2 *__restrict__ fprev,
                                                               float2 *__restrict__ F, double2 *__restrict__ part) {
    fa2_combine_tile((int32_t)blockIdx.x, K, nseg, seg, pos, mass, att, item_of, kr, kg, fprev, F, part);
}

static bgv_status exact_forces(int32_t K, const float2 *pos, const float *mass, const float2 *A,
                               const uint32_t *item_of, float kr, float kg, const float2 *fprev, float2 *F,
                               double2 *part, float2 *seg, hipStream_t s) {
    const unsigned nb = (unsigned)((K + kFaThreads - 1) / kFaThreads);
    const int32_t nseg = fa2_rep_segments(K);
    if (nseg <= 1) {
        BGV_LAUNCH(k_force_exact<false>, dim3(nb), dim3(kFaThreads), 0, s, K, pos, mass, A, item_of, kr, kg, fprev,
                   F, part, seg);
    } else {
        BGV_LAUNCH(k_force_exact<true>, dim3(nb, (unsigned)nseg), dim3(kFaThreads), 0, s, K, pos, mass, A, item_of,
                   kr, kg, fprev, F, part, seg);
        BGV_LAUNCH(k_force_combine, dim3(nb), dim3(kFaThreads), 0, s, K, nseg, seg, pos, mass, A, item_of, kr, kg,
                   fprev, F, part);
    }
    return BGV_OK;
}

// ----------------------------------------------------------------- update ------
// Bounding box (xmin, xmax, ymin, ymax) of the block's points; result in every thread.
// min/max are order-independent, so any reduction order gives the same box.
__device__ __forceinline__ float4 block_bbox(float4 b) {
    __shared__ float4 ws[kFaThreads / kWave];
    __shared__ float4 res;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        b.x = fminf(b.x, __shfl_down(b.x, o, kWave));
        b.y = fmaxf(b.y, __shfl_down(b.y, o, kWave));
        b.z = fminf(b.z, __shfl_down(b.z, o, kWave));
        b.w = fmaxf(b.w, __shfl_down(b.w, o, kWave));
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        float4 r = ws[0];
        for (int q = 1; q < kFaThreads / kWave; ++q) {
            r.x = fminf(r.x, ws[q].x);
            r.y = fmaxf(r.y, ws[q].y);
            r.z = fminf(r.z, ws[q].z);
            r.w = fmaxf(r.w, ws[q].w);
        }
        res = r;
    }
    __syncthreads();
    return res;
}

constexpr float kInf = __builtin_huge_valf();

// Global speed, local speeds, displacement.  With bbox_part != nullptr each block also
// writes the bounding box of the positions it just moved (for the next tree build).
__global__ void __launch_bounds__(kFaThreads) k_update(int32_t K, float2 *__restrict__ pos,
                                                        float2 *__restrict__ fprev, const float2 *__restrict__ F,
                                                        const double2 *__restrict__ part, int32_t nparts,
                                                        const float *__restrict__ speed_in,
                                                        float *__restrict__ speed_out, float tau, float ks,
                                                        float ksmax, float4 *__restrict__ bbox_part) {
    float4 bb = fa2_update_tile((int32_t)blockIdx.x, (int32_t)gridDim.x, K, pos, fprev, F, part, nparts, speed_in,
                                speed_out, tau, ks, ksmax);
    if (bbox_part) {
        bb = block_bbox(bb);
        if (threadIdx.x == 0) bbox_part[blockIdx.x] = bb;
    }
}

__global__ void k_copy_f32(const float *__restrict__ a, float *__restrict__ b) { *b = *a; }

// Barnes-Hut iterations have one force partial per 8 bodies, too many for every update
// block to reduce: one 1024-thread block reduces them (each thread its strided share in
// ascending order, eight loads in flight; then the waves in order) ...
constexpr int kBhSpeedThreads = 1024;

// Also clears the force launch's redo count for the next iteration (adding it to a
// running tally that the profiler can read).
__device__ unsigned long long g_bh_redo_blocks;

__global__ void __launch_bounds__(kBhSpeedThreads) k_bh_speed(const double2 *__restrict__ part, int32_t nparts,
                                                               const float *__restrict__ speed_in,
                                                               float *__restrict__ speed_out, float tau,
                                                               uint32_t *__restrict__ redo) {
    __shared__ double2 ws[kBhSpeedThreads / kWave];
    double2 acc = make_double2(0.0, 0.0);
    int32_t p = threadIdx.x;
    for (; p + 7 * kBhSpeedThreads < nparts; p += 8 * kBhSpeedThreads) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[p + u * kBhSpeedThreads];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
        }
    }
    for (; p < nparts; p += kBhSpeedThreads) {
        acc.x += part[p].x;
        acc.y += part[p].y;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        acc.x += __shfl_down(acc.x, o, kWave);
        acc.y += __shfl_down(acc.y, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 r = ws[0];
        for (int q = 1; q < kBhSpeedThreads / kWave; ++q) {
            r.x += ws[q].x;
            r.y += ws[q].y;
        }
        *speed_out = fa2_global_speed(r.x, r.y, *speed_in, tau);
        g_bh_redo_blocks += redo[0];
        redo[0] = 0u;
    }
}

// ... and the update blocks read the result; each writes the bounding box of the
// positions it moved.
// The Morton sort's digit totals, which the next encoding launch adds into, cleared by
// the launch before it (the bounding box before the first iteration, the update after
// each one).
__device__ __forceinline__ void bh_clear_totals(uint32_t *__restrict__ totals) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kOsTotals; i += blockDim.x) totals[i] = 0u;
}

__global__ void __launch_bounds__(kFaThreads) k_bh_update(int32_t K, float2 *__restrict__ pos,
                                                           float2 *__restrict__ fprev, const float2 *__restrict__ F,
                                                           const float *__restrict__ speed, float ks, float ksmax,
                                                           float4 *__restrict__ bbox_part, uint32_t *__restrict__ totals) {
    float4 bb = fa2_move_tile((int32_t)blockIdx.x, (int32_t)gridDim.x, K, pos, fprev, F, *speed, ks, ksmax);
    bb = block_bbox(bb);
    if (threadIdx.x == 0) bbox_part[blockIdx.x] = bb;
    bh_clear_totals(totals);
}

// ------------------------------------------------------------------ Barnes-Hut --
// One bounding-box partial per block of kFaThreads positions (same grid as k_update).
__global__ void __launch_bounds__(kFaThreads) k_bh_bbox(int32_t K, const float2 *__restrict__ pos,
                                                         float4 *__restrict__ part, uint32_t *__restrict__ totals) {
    bh_clear_totals(totals);
    float4 bb = make_float4(kInf, -kInf, kInf, -kInf);
    for (int32_t i = blockIdx.x * kFaThreads + threadIdx.x; i < K; i += gridDim.x * kFaThreads) {
        const float2 p = pos[i];
        bb = make_float4(fminf(bb.x, p.x), fmaxf(bb.y, p.x), fminf(bb.z, p.y), fmaxf(bb.w, p.y));
    }
    bb = block_bbox(bb);
    if (threadIdx.x == 0) part[blockIdx.x] = bb;
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// The bounding square of the positions (from the per-block boxes): origin and side s0.
// Every thread of the block gets the result; block 0 stores s0.
__device__ __forceinline__ void bh_frame(const float4 *__restrict__ part, int nparts, float *xmin, float *ymin,
                                         float *s0, float *__restrict__ s0_out) {
    float4 bb = make_float4(kInf, -kInf, kInf, -kInf);
    for (int q = threadIdx.x; q < nparts; q += kFaThreads) {
        const float4 r = part[q];
        bb = make_float4(fminf(bb.x, r.x), fmaxf(bb.y, r.y), fminf(bb.z, r.z), fmaxf(bb.w, r.w));
    }
    bb = block_bbox(bb);
    *xmin = bb.x;
    *ymin = bb.z;
    const float ex = bb.y - bb.x, ey = bb.w - bb.z;
    float s = ex > ey ? ex : ey;
    if (!(s > 0.f)) s = 1.0f;
    *s0 = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) *s0_out = s;
}

// Quantise on the 2^16 grid over the bounding square and Morton-encode (x even bits).
__device__ __forceinline__ uint32_t bh_morton(float2 p, float xmin, float ymin, float s0) {
    const float tx = __fdiv_rn(__fsub_rn(p.x, xmin), s0);
    const float ty = __fdiv_rn(__fsub_rn(p.y, ymin), s0);
    int32_t qx = (int32_t)__fmul_rn(tx, 65536.0f);
    int32_t qy = (int32_t)__fmul_rn(ty, 65536.0f);
    qx = qx > 65535 ? 65535 : qx;
    qy = qy > 65535 ? 65535 : qy;
    return spread16((uint32_t)qx) | (spread16((uint32_t)qy) << 1);
}

__global__ void __launch_bounds__(kFaThreads) k_bh_codes(int32_t K, const float2 *__restrict__ pos,
                                                          const float4 *__restrict__ part, int nparts,
                                                          uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                          float *__restrict__ s0_out) {
    float xmin, ymin, s0;
    bh_frame(part, nparts, &xmin, &ymin, &s0, s0_out);
    for (int32_t i = blockIdx.x * kFaThreads + threadIdx.x; i < K; i += gridDim.x * kFaThreads) {
        keys[i] = bh_morton(pos[i], xmin, ymin, s0);
        vals[i] = (uint32_t)i;
    }
}

// The codes and the one-sweep sort's counts in one launch: workgroup t encodes the
// bodies of sort tile t (256 * ITEMS consecutive ones), counts the four 8-bit digits
// of their codes in LDS into counts[t*1024 + pass*256 + d], and clears its share
// of the sort's look-back words.
template <int ITEMS>
__global__ void __launch_bounds__(kFaThreads) k_bh_codes_os(int32_t K, const float2 *__restrict__ pos,
                                                             const float4 *__restrict__ part, int nparts,
                                                             uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                             float *__restrict__ s0_out,
                                                             uint32_t *__restrict__ totals,
                                                             uint32_t *__restrict__ status, int64_t status_words) {
    __shared__ uint32_t hist[4][256];
    float xmin, ymin, s0;
    bh_frame(part, nparts, &xmin, &ymin, &s0, s0_out);
#pragma unroll
    for (int q = 0; q < 4; ++q) hist[q][threadIdx.x] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * kFaThreads + threadIdx.x; i < status_words;
         i += (int64_t)gridDim.x * kFaThreads)
        status[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kFaThreads * ITEMS);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * kFaThreads + threadIdx.x;
        if (i < K) {
            const uint32_t c = bh_morton(pos[i], xmin, ymin, s0);
            keys[i] = c;
            vals[i] = (uint32_t)i;
#pragma unroll
            for (int q = 0; q < 4; ++q) atomicAdd(&hist[q][(c >> (8 * q)) & 255u], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (hist[q][threadIdx.x]) atomicAdd(&totals[q * 256 + threadIdx.x], hist[q][threadIdx.x]);
}

// Bodies [256 g, 256 g + 256) in Morton order (one per thread) and the group totals of
// the FP64 mass moments m, m*x, m*y into part3[3 g ..].
__device__ __forceinline__ void bh_gather_group(int32_t g, int32_t K, const float2 *__restrict__ pos,
                                                const float *__restrict__ mass, const uint32_t *__restrict__ order,
                                                uint32_t key_of_k, float4 *__restrict__ body,
                                                uint32_t *__restrict__ code, double *__restrict__ part3) {
    const int32_t k = g * kFaThreads + threadIdx.x;
    double m = 0.0, mx = 0.0, my = 0.0;
    if (k < K) {
        const uint32_t b = order[k];
        const float2 p = pos[b];
        const float mf = mass[b];
        body[k] = make_float4(p.x, p.y, mf, __int_as_float((int)b));
        code[k] = key_of_k;
        m = (double)mf;
        mx = m * (double)p.x;
        my = m * (double)p.y;
    }
    double t0, t1, t2;
    block_excl_scan<double>(m, &t0);
    block_excl_scan<double>(mx, &t1);
    block_excl_scan<double>(my, &t2);
    if (threadIdx.x == 0) {
        part3[3 * g] = t0;
        part3[3 * g + 1] = t1;
        part3[3 * g + 2] = t2;
    }
}

__global__ void __launch_bounds__(kFaThreads) k_bh_gather(int32_t K, const float2 *__restrict__ pos,
                                                           const float *__restrict__ mass,
                                                           const uint32_t *__restrict__ skeys,
                                                           const uint32_t *__restrict__ order,
                                                           float4 *__restrict__ body, uint32_t *__restrict__ code,
                                                           double *__restrict__ part3) {
    const int32_t k = blockIdx.x * kFaThreads + threadIdx.x;
    bh_gather_group((int32_t)blockIdx.x, K, pos, mass, order, k < K ? skeys[k] : 0u, body, code, part3);
}

// Exclusive FP64 prefix sums PM/PX/PY (K+1 entries) of the mass moments in Morton
// order: block offset = fixed-order sum of the preceding block totals, then a block scan.
__global__ void __launch_bounds__(kFaThreads) k_bh_prefix(int32_t K, const float4 *__restrict__ body,
                                                           const double *__restrict__ part3,
                                                           double *__restrict__ PM, double *__restrict__ PX,
                                                           double *__restrict__ PY) {
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int q = threadIdx.x; q < (int)blockIdx.x; q += kFaThreads) {
        b0 += part3[3 * q];
        b1 += part3[3 * q + 1];
        b2 += part3[3 * q + 2];
    }
    double base0, base1, base2;
    block_excl_scan<double>(b0, &base0);
    block_excl_scan<double>(b1, &base1);
    block_excl_scan<double>(b2, &base2);
    const int32_t k = blockIdx.x * kFaThreads + threadIdx.x;
    double m = 0.0, mx = 0.0, my = 0.0;
    if (k < K) {
        const float4 bd = body[k];
        m = (double)bd.z;
        mx = m * (double)bd.x;
        my = m * (double)bd.y;
    }
    double t0, t1, t2;
    const double e0 = block_excl_scan<double>(m, &t0);
    const double e1 = block_excl_scan<double>(mx, &t1);
    const double e2 = block_excl_scan<double>(my, &t2);
    if (k < K) {
        PM[k] = base0 + e0;
        PX[k] = base1 + e1;
        PY[k] = base2 + e2;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        PM[K] = base0 + t0;
        PX[K] = base1 + t1;
        PY[K] = base2 + t2;
    }
}

// Common-prefix length of sorted positions i and j; index bits break ties between
// equal codes (values >= 32 mean equal codes); -1 when j is outside [0, K) (only j is
// checked: i must be a valid position).
__device__ __forceinline__ int delta(const uint32_t *__restrict__ code, int32_t K, int32_t i, int32_t j) {
    if (j < 0 || j >= K) return -1;
    const uint32_t a = code[i], b = code[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

// A node's own record: (centre of mass, mass, size^2) and (left, right, first, last) in
// 32 bytes (the tree export reads these).
struct __align__(32) BhNode {
    float4 a;
    int4 b;
};

// What a traversal step needs about the two children of an opened node, so that the
// step that pops the node decides both children without loading their own records:
// per child its (centre of mass, mass, size^2) — a body's (x, y, m, unused) —, its
// body range and its index (>= 0 internal node, < 0 leaf ~body).  64 bytes: one line.
struct __align__(64) BhKids {
    float4 a[2];
    int4 range;  // first and last body of the left child, then of the right one
    int2 idx;    // left, right
    int2 pad;
};

// (centre of mass, mass, size^2) of the internal node over bodies [first, last]
// (first < last); size^2 < 0 for a node whose codes are all equal (a leaf cell).
//
// The radix tree refines the compressed quadtree of Section 3.1's hierarchical
// partition: a node whose codes share a 2d-bit prefix and differ in the next bit is
// the quadtree cell of depth d (side s0 / 2^d) whose bodies occupy quadrants in both
// of its y halves; a node with a (2d+1)-bit prefix holds bodies in two quadrants of one
// y half.  When its parent has the 2d-bit prefix, that node is only half of the
// parent's cell, not a quadtree cell: it gets size^2 = +inf, so the traversal always
// opens it and reaches the quadrant nodes below it.  Every other node is a quadtree
// cell with its own side, so the opening decisions are those of the quadtree.  The
// parent of the node over [first, last] has the longer of the prefixes shared across
// the range's two ends (Karras' tree: the parent extends the range on that side).
__device__ __forceinline__ float4 bh_range_data(int32_t K, const uint32_t *__restrict__ code,
                                                const double *__restrict__ PM, const double *__restrict__ PX,
                                                const double *__restrict__ PY, float s0, int first, int last) {
    const int dnode = delta(code, K, first, last);
    const double M = PM[last + 1] - PM[first];
    const double cx = (PX[last + 1] - PX[first]) / M;
    const double cy = (PY[last + 1] - PY[first]) / M;
    float size2;
    if (dnode >= 32) {
        size2 = -1.0f;
    } else if ((dnode & 1) && max(delta(code, K, first, first - 1), delta(code, K, last, last + 1)) == dnode - 1) {
        size2 = __builtin_inff();  // half of the parent's cell: always opened
    } else {
        const int lev = min(dnode >> 1, 16);
        const float sz = s0 / (float)(1u << lev);
        size2 = sz * sz;
    }
    return make_float4((float)cx, (float)cy, (float)M, size2);
}

// Internal node i of the binary radix tree over the sorted codes (Karras' parallel
// construction): the record of its two children that the traversal reads and, when
// `node` is given (the tree export), its own record (children >= 0 internal node, < 0
// leaf ~child).
__device__ __forceinline__ void bh_build_nodes(int32_t K, const uint32_t *__restrict__ code,
                                               const double *__restrict__ PM, const double *__restrict__ PX,
                                               const double *__restrict__ PY, const float *__restrict__ s0p,
                                               const float4 *__restrict__ body, BhNode *__restrict__ node,
                                               BhKids *__restrict__ kids, int32_t i0, int32_t stride) {
    const float s0 = *s0p;
    for (int32_t i = i0; i < K - 1; i += stride) {
        const int d = (delta(code, K, i, i + 1) - delta(code, K, i, i - 1)) >= 0 ? 1 : -1;
        const int dmin = delta(code, K, i, i - d);
        int lmax = 2;
        while (delta(code, K, i, i + lmax * d) > dmin) lmax <<= 1;
        int l = 0;
        for (int t = lmax >> 1; t >= 1; t >>= 1)
            if (delta(code, K, i, i + (l + t) * d) > dmin) l += t;
        const int j = i + l * d;
        const int dnode = delta(code, K, i, j);
        int sgap = 0;
        int t = l;
        do {
            t = (t + 1) >> 1;
            if (delta(code, K, i, i + (sgap + t) * d) > dnode) sgap += t;
        } while (t > 1);
        const int gamma = i + sgap * d + (d < 0 ? -1 : 0);
        const int first = min(i, j), last = max(i, j);
        const int left = (first == gamma) ? ~gamma : gamma;
        const int right = (last == gamma + 1) ? ~(gamma + 1) : gamma + 1;
        if (node) {  // the tree export only: the traversal reads the children records
            BhNode nd;
            nd.a = bh_range_data(K, code, PM, PX, PY, s0, first, last);
            nd.b = make_int4(left, right, first, last);
            node[i] = nd;
        }
        BhKids kd;
        kd.a[0] = left < 0 ? body[first] : bh_range_data(K, code, PM, PX, PY, s0, first, gamma);
        kd.a[1] = right < 0 ? body[last] : bh_range_data(K, code, PM, PX, PY, s0, gamma + 1, last);
        kd.range = make_int4(first, gamma, gamma + 1, last);
        kd.idx = make_int2(left, right);
        kd.pad = make_int2(0, 0);
        kids[i] = kd;
    }
}

__global__ void k_bh_build(int32_t K, const uint32_t *__restrict__ code, const double *__restrict__ PM,
                           const double *__restrict__ PX, const double *__restrict__ PY,
                           const float *__restrict__ s0p, const float4 *__restrict__ body,
                           BhNode *__restrict__ node, BhKids *__restrict__ kids) {
    bh_build_nodes(K, code, PM, PX, PY, s0p, body, node, kids, blockIdx.x * blockDim.x + threadIdx.x,
                   gridDim.x * blockDim.x);
}

// The tree build and the attraction in one launch: workgroups [0, build_blocks) build
// the tree (a few dozen for a supergraph of some ten thousand bodies), the others take
// the attraction items, which do not depend on the tree, so the two latency-bound jobs
// overlap instead of following each other.  With kLds the attraction workgroups stage
// the positions in (dynamic) LDS first, as k_attract_lds does.
template <typename E, int NT, bool kLds>
__global__ void __launch_bounds__(NT) k_bh_build_attract(int32_t K, const uint32_t *__restrict__ code,
                                                          const double *__restrict__ PM,
                                                          const double *__restrict__ PX,
                                                          const double *__restrict__ PY,
                                                          const float *__restrict__ s0p,
                                                          const float4 *__restrict__ body, BhNode *__restrict__ node,
                                                          BhKids *__restrict__ kids, int32_t build_blocks,
                                                          const float2 *__restrict__ pos,
                                                          const uint32_t *__restrict__ row, const E *__restrict__ cw,
                                                          const uint32_t *__restrict__ item_of,
                                                          const uint32_t *__restrict__ item_row,
                                                          float2 *__restrict__ A) {
    if ((int32_t)blockIdx.x < build_blocks) {  // uniform over the workgroup
        bh_build_nodes(K, code, PM, PX, PY, s0p, body, node, kids, blockIdx.x * NT + threadIdx.x,
                       build_blocks * NT);
        return;
    }
    const int64_t wave0 = ((int64_t)(blockIdx.x - build_blocks) * NT + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)(gridDim.x - build_blocks) * (NT / kWave);
    if (kLds) {
        extern __shared__ float2 sp[];  // K entries
        for (int32_t i = threadIdx.x; i < K; i += NT) sp[i] = pos[i];
        __syncthreads();
        att_items(K, sp, row, cw, item_of, item_row, A, wave0, nwaves);
    } else {
        att_items(K, pos, row, cw, item_of, item_row, A, wave0, nwaves);
    }
}


__device__ __forceinline__ void add_pair(float2 xi, float4 bj, float &fx, float &fy, uint32_t &ic) {
    ++ic;
    fa2_rep_term(xi, bj, fx, fy);
}

constexpr int kBhThreads = 64;
// Lanes per body: few, so that few lanes idle when a body's stack is short, but enough
// that the bodies' wavefronts fill the chip.  Measured on the 171,724-body lfr_3m
// supergraph: 8 lanes 93 us per launch, 4 lanes 72, 2 lanes 71; on the 17,724-body
// lfr_1m supergraph 8 lanes beat 16 and 32.
static int bh_lanes(int32_t K) { return K >= 131072 ? 2 : K >= 65536 ? 4 : 8; }

// Barnes-Hut repulsion.  Bodies are taken in Morton order, so the bodies of a wavefront
// walk similar paths.  Each body has a shared stack of opened nodes and G lanes: they
// pop the top (up to) G nodes of the body's LDS stack together, and each lane decides
// both children of its node from the node's children record, exactly as a single
// traversal would (a body or a cell of equal codes is summed directly, a node far
// enough away by its centre of mass, any other node is opened and pushed).  So a
// step costs one dependent load per lane and settles two entries: the accepted
// nodes and the bodies are never loaded on their own.  Work is shared out afresh every
// step, so no lane waits on another's subtree.  Children are pushed in reverse lane
// order, so the deepest entries stay on top and the stack is sorted by depth; a step
// that pops an entry of depth d then pops every deeper entry, so at most 2G entries of
// any one depth are ever on the stack, and 2G per level of the tree bounds it: a
// node's prefix is longer than its parent's, so the tree has at most 34 levels (root,
// 32 prefix lengths, bodies) and the stack never exceeds that.  The order of the
// additions depends only on G and the tree: results are identical run to run.
constexpr int kBhTreeLevels = 34;  // 32-bit Morton codes: root, 32 prefix lengths, equal-code cells

// One force workgroup's bodies (block `blk`) with a stack of C entries per body.  A step
// whose pushes would not fit stops the body's walk and returns true (the caller then
// redoes the whole workgroup with the full stack); otherwise the forces, the
// workgroup's speed partial and its interaction tally are written and false returned.
template <int G, int C>
__device__ __forceinline__ bool bh_force_block(int32_t blk, int32_t K, const float4 *__restrict__ body,
                                               const BhKids *__restrict__ kids, float theta2, const float2 *__restrict__ att,
                                               const uint32_t *__restrict__ item_of, float kr, float kg,
                                               const float2 *__restrict__ fprev, float2 *__restrict__ F,
                                               double2 *__restrict__ part, uint32_t *__restrict__ icount) {
    static_assert(G >= 2 && G <= kWave && (G & (G - 1)) == 0, "lanes per body: power of two in [2, 64]");
    constexpr int kGroups = kBhThreads / G;
    __shared__ int stk[kGroups][C];
    const int64_t tid = (int64_t)blk * kBhThreads + threadIdx.x;
    const int32_t r = (int32_t)(tid / G);
    const int L = (int)(tid % G);
    int *st_g = stk[threadIdx.x / G];
    double2 st = make_double2(0.0, 0.0);
    float fx = 0.f, fy = 0.f;
    uint32_t ic = 0;
    float4 me = make_float4(0.f, 0.f, 0.f, 0.f);
    int size = 0;
    bool overflow = false;
    if (r < K) {
        me = body[r];
        if (K > 1) size = 1;
    }
    if (L == 0) st_g[0] = 0;  // the root
    const float2 xi = make_float2(me.x, me.y);
    while (__any(size > 0)) {
        const int take = size < G ? size : G;
        const bool has = L < take;
        const int e = has ? st_g[size - 1 - L] : 0;
        size -= take;
        int c_left = 0, c_right = 0, np = 0;
        if (has) {
            // an opened node: decide both children from its children's record
            const BhKids kd = kids[e];
            bool open[2] = {false, false};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float4 A = kd.a[q];
                const int c = q ? kd.idx.y : kd.idx.x;
                const int f = q ? kd.range.z : kd.range.x, l = q ? kd.range.w : kd.range.y;
                if (c < 0) {
                    if (~c != r) add_pair(xi, A, fx, fy, ic);  // a body
                } else if (A.w < 0.f) {  // a cell of equal codes: direct sum
                    for (int k = f; k <= l; ++k)
                        if (k != r) add_pair(xi, body[k], fx, fy, ic);
                } else {
                    bool o = r >= f && r <= l;
                    if (!o) {
                        const float dx = xi.x - A.x, dy = xi.y - A.y;
                        const float d2 = dx * dx + dy * dy;
                        if (d2 > 0.f && A.w < theta2 * d2) {
                            const float fr = A.z * __builtin_amdgcn_rcpf(d2);
                            fx += fr * dx;
                            fy += fr * dy;
                            ++ic;
                        } else {
                            o = true;
                        }
                    }
                    open[q] = o;
                }
            }
            if (open[0] && open[1]) {
                c_left = kd.idx.x;
                c_right = kd.idx.y;
                np = 2;
            } else if (open[0] || open[1]) {
                c_left = open[0] ? kd.idx.x : kd.idx.y;
                np = 1;
            }
        }
        // inclusive scan of the pushes from the highest lane down, so lane 0 (the
        // deepest popped entry) writes last, on top
        int incl = np;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            const int v = __shfl_down(incl, o, G);
            if (L + o < G) incl += v;
        }
        const int total = __shfl(incl, 0, G);
        if (size + total > C) {  // uniform over the body's lanes
            overflow = true;
            size = 0;
        } else {
            if (np == 2) {
                const int at = size + incl - np;  // this lane's two slots: at, at + 1
                st_g[at] = c_right;
                st_g[at + 1] = c_left;  // left on top: popped first
            } else if (np == 1) {
                st_g[size + incl - 1] = c_left;
            }
            size += total;
        }
    }
    if (__any(overflow)) return true;  // uniform: the workgroup is one wavefront
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, kWave);
        fy += __shfl_xor(fy, o, kWave);
    }
    if (r < K && L == 0) {
        const float mi = me.z;
        const int32_t b = __float_as_int(me.w);
        const float2 f = fa2_net_force(xi, mi, kr, fx, fy, fa2_att_combine(att, item_of, b), kg);
        F[b] = f;
        st = fa2_swing_traction(f, fprev[b], mi);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) ic += __shfl_xor(ic, o, kWave);
    st = block_sum2(st);
    if (threadIdx.x == 0) {
        part[blk] = st;
        icount[blk] += ic;
    }
    return false;
}

// The full stack: at most 2G entries of one depth (see above) on at most kBhTreeLevels
// depths.  The fast launch gives each body 20 entries per lane (5 KiB of LDS per
// wavefront whatever G is), so that several times more wavefronts fit a compute unit's
// LDS than with the full stack; a workgroup whose walk would not fit
// appends itself to a list, and k_bh_force_full redoes it with the full stack (the same
// steps, so the same bits: results never depend on the capacity).
template <int G>
struct BhStack {
    static constexpr int kFull = 2 * G * kBhTreeLevels;
    static constexpr int kFast = 20 * G;
};

constexpr int32_t kBhXcds = 8;

template <int G>
__global__ void __launch_bounds__(kBhThreads) k_bh_force(int32_t K, const float4 *__restrict__ body,
                                                          const BhKids *__restrict__ kids, float theta2,
                                                          const float2 *__restrict__ att,
                                                          const uint32_t *__restrict__ item_of, float kr, float kg,
                                                          const float2 *__restrict__ fprev, float2 *__restrict__ F,
                                                          double2 *__restrict__ part, uint32_t *__restrict__ icount,
                                                          uint32_t *__restrict__ redo) {
    // workgroups are dealt to the eight XCDs in turn; each XCD takes a contiguous eighth
    // of the bodies (in Morton order: a region of the plane), so its L2 holds the nodes
    // that region's walks visit rather than the whole tree
    const int32_t nblk = (int32_t)((K * (int64_t)G + kBhThreads - 1) / kBhThreads);
    const int32_t per = (nblk + kBhXcds - 1) / kBhXcds;
    const int32_t blk = ((int32_t)blockIdx.x % kBhXcds) * per + (int32_t)blockIdx.x / kBhXcds;
    if (blk >= nblk) return;  // the grid is rounded up to a multiple of the XCD count
    const bool ovf = bh_force_block<G, BhStack<G>::kFast>(blk, K, body, kids, theta2, att, item_of, kr, kg, fprev,
                                                           F, part, icount);
    if (ovf && threadIdx.x == 0) redo[1 + atomicAdd(&redo[0], 1u)] = (uint32_t)blk;
}

// The listed workgroups again with the full stack; redo[0] counts them.
template <int G>
__global__ void __launch_bounds__(kBhThreads) k_bh_force_full(int32_t K, const float4 *__restrict__ body,
                                                               const BhKids *__restrict__ kids, float theta2,
                                                               const float2 *__restrict__ att,
                                                               const uint32_t *__restrict__ item_of, float kr,
                                                               float kg, const float2 *__restrict__ fprev,
                                                               float2 *__restrict__ F, double2 *__restrict__ part,
                                                               uint32_t *__restrict__ icount,
                                                               const uint32_t *__restrict__ redo) {
    const uint32_t n = redo[0];
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x)
        bh_force_block<G, BhStack<G>::kFull>((int32_t)redo[1 + i], K, body, kids, theta2, att, item_of, kr,
                                             kg, fprev, F, part, icount);
}

static_assert(kBhThreads == kWave, "the interaction tally reduces over one wavefront per workgroup");

// Profiling only: total Barnes-Hut interactions, readable with bgv_profile_counter().
__device__ unsigned long long g_bh_interactions;

__global__ void __launch_bounds__(kFaThreads) k_count_total(const uint32_t *__restrict__ icount, int32_t n) {
    unsigned long long acc = 0;
    for (int32_t i = threadIdx.x; i < n; i += kFaThreads) acc += icount[i];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&g_bh_interactions, acc);
}

int prof_read_counter(const char *name, uint64_t *value) {
    unsigned long long v = 0;
    if (std::strcmp(name, "bh_interactions") == 0) {
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bh_interactions), sizeof v) != hipSuccess) return -1;
    } else if (std::strcmp(name, "bh_redo_blocks") == 0) {
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bh_redo_blocks), sizeof v) != hipSuccess) return -1;
    } else {
        return -1;
    }
    *value = v;
    return 0;
}

void prof_reset_counters() {
    const unsigned long long z = 0;
    (void)hipMemcpyToSymbol(HIP_SYMBOL(g_bh_interactions), &z, sizeof z);
    (void)hipMemcpyToSymbol(HIP_SYMBOL(g_bh_redo_blocks), &z, sizeof z);
}

static int32_t bh_force_blocks(int32_t K) {
    return (int32_t)(((int64_t)K * bh_lanes(K) + kBhThreads - 1) / kBhThreads);
}
constexpr int kBhFullBlocks = 64;  // workgroups of the full-stack redo launch (grid-stride over its list)

// Blocks of the Barnes-Hut update, and so the number of bounding-box partials the next
// tree build reduces (min/max, so any count gives the same box).
constexpr int32_t kBhUpdateMaxBlocks = 256;
static int32_t bh_update_blocks(int32_t K) {
    const int32_t nb = (K + kFaThreads - 1) / kFaThreads;
    return nb < kBhUpdateMaxBlocks ? nb : kBhUpdateMaxBlocks;
}

struct BhWs {
    float4 *bbox;
    float *s0;
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
    float4 *body;
    uint32_t *code;
    double *part3, *PM, *PX, *PY;
    BhNode *node;
    BhKids *kids;      // the children's records of each internal node (what the traversal reads)
    uint32_t *icount;  // interactions per force workgroup, summed over the call's iterations
    uint32_t *redo;    // [0]: force workgroups to redo with the full stack, [1..]: their ids
    void *sort_scratch;
};

struct FaWs {
    CsrWs csr;
    float2 *F, *A;
    float2 *seg;  // exact repulsion: per-segment sums [segments][K] when K spans several segments
    double2 *part;
    float *speed;  // [2] ping-pong
    int32_t *flag;  // id range check
    BhWs bh;
};

static size_t fa_layout(Carver &c, int32_t K, int64_t E, const bgv_fa2_params *p, FaWs *w) {
    csr_layout(c, K, E, &w->csr, true);
    const int64_t nb = (K + kFaThreads - 1) / kFaThreads;
    w->F = c.take<float2>((size_t)K);
    w->A = c.take<float2>((size_t)w->csr.items_bound);
    w->part = c.take<double2>((size_t)(nb > bh_force_blocks(K) ? nb : bh_force_blocks(K)));
    w->speed = c.take<float>(2);
    w->flag = c.take<int32_t>(1);
    w->seg = nullptr;
    if (p->exact && fa2_rep_segments(K) > 1) w->seg = c.take<float2>((size_t)fa2_rep_segments(K) * (size_t)K);
    if (!p->exact) {
        BhWs &b = w->bh;
        b.bbox = c.take<float4>((size_t)nb);
        b.s0 = c.take<float>(1);
        b.keys = c.take<uint64_t>((size_t)K);
        b.keys_alt = c.take<uint64_t>((size_t)K);
        b.vals = c.take<uint32_t>((size_t)K);
        b.vals_alt = c.take<uint32_t>((size_t)K);
        b.body = c.take<float4>((size_t)K);
        b.code = c.take<uint32_t>((size_t)K);
        b.part3 = c.take<double>(3 * (size_t)nb);
        b.PM = c.take<double>((size_t)K + 1);
        b.PX = c.take<double>((size_t)K + 1);
        b.PY = c.take<double>((size_t)K + 1);
        b.node = c.take<BhNode>((size_t)K);
        b.kids = c.take<BhKids>((size_t)K);
        b.icount = c.take<uint32_t>((size_t)bh_force_blocks(K));
        b.redo = c.take<uint32_t>((size_t)bh_force_blocks(K) + 1);
        b.sort_scratch = c.take<char>(onesweep_workspace(K));
    }
    return c.size();
}

static bool fa_valid(int32_t K, int64_t E, const bgv_fa2_params *p) {
    return p && K >= 1 && E >= 0 && E <= INT32_MAX && p->iters >= 0 && (p->exact == 0 || p->exact == 1) &&
           p->theta >= 0.f && p->tau > 0.f && p->ks >= 0.f && p->ksmax > 0.f;
}

// One Barnes-Hut repulsion + force evaluation into w.F / w.part.
template <typename E, int NT, bool kLds>
static bgv_status launch_build_attract(int32_t K, const BhWs &b, unsigned build_blocks, unsigned att_blocks,
                                       size_t lds, const float2 *pos, const CsrWs &csr, float2 *A, hipStream_t s) {
    const auto k_bh_build_att = k_bh_build_attract<E, NT, kLds>;  // one name for the profiler
    BGV_LAUNCH(k_bh_build_att, dim3(build_blocks + att_blocks), dim3(NT), lds, s, K, b.code,
               b.PM, b.PX, b.PY, b.s0, b.body, (BhNode *)nullptr, b.kids, (int32_t)build_blocks, pos, csr.row,
               reinterpret_cast<const E *>(csr.cw), csr.item_of, csr.item_row, A);
    return BGV_OK;
}

template <int NT, bool kLds>
static bgv_status build_attract(int32_t K, const BhWs &b, unsigned att_blocks, size_t lds, const float2 *pos,
                                const CsrWs &csr, float2 *A, hipStream_t s) {
    const unsigned build_blocks = grid_for(K - 1, NT, 65536);
    if (csr.fmt == kCsrWeighted)
        return launch_build_attract<int2, NT, kLds>(K, b, build_blocks, att_blocks, lds, pos, csr, A, s);
    if (csr.fmt == kCsrIds32)
        return launch_build_attract<uint32_t, NT, kLds>(K, b, build_blocks, att_blocks, lds, pos, csr, A, s);
    return launch_build_attract<uint16_t, NT, kLds>(K, b, build_blocks, att_blocks, lds, pos, csr, A, s);
}

// The Morton sort's digit totals in the layout's sort scratch.
static uint32_t *bh_sort_totals(const BhWs &b, int32_t K) {
    OsBuffers ob;
    onesweep_layout(b.sort_scratch, K, os_items(K), &ob);
    return ob.totals;
}

// Morton codes of the positions, sorted, the bodies gathered in Morton order and the
// FP64 prefix sums of their mass moments: everything the node build reads.
static bgv_status bh_sorted_bodies(int32_t K, const float2 *pos, const float *mass, BhWs &b, hipStream_t s) {
    const unsigned nb = (unsigned)((K + kFaThreads - 1) / kFaThreads);
    // b.bbox holds one box per update block (written by k_bh_bbox before the first
    // iteration and by k_bh_update after each one)
    const int nbox = bh_update_blocks(K);
    // 32-bit Morton codes, sorted as 32-bit keys (the index buffers hold them)
    uint32_t *keys = reinterpret_cast<uint32_t *>(b.keys), *keys_alt = reinterpret_cast<uint32_t *>(b.keys_alt);
    uint32_t *sk = keys;
    uint32_t *sv = b.vals;
    if (K > 1) {
        // codes and the sort's digit counts in one launch, then the one-sweep passes
        OsBuffers ob;
        onesweep_layout(b.sort_scratch, K, os_items(K), &ob);
        if (ob.items == 4)
            BGV_LAUNCH(k_bh_codes_os<4>, dim3((unsigned)ob.tiles), dim3(kFaThreads), 0, s, K, pos, b.bbox, nbox, keys,
                       b.vals, b.s0, ob.totals, ob.status, ob.status_words);
        else if (ob.items == 8)
            BGV_LAUNCH(k_bh_codes_os<8>, dim3((unsigned)ob.tiles), dim3(kFaThreads), 0, s, K, pos, b.bbox, nbox, keys,
                       b.vals, b.s0, ob.totals, ob.status, ob.status_words);
        else
            BGV_LAUNCH(k_bh_codes_os<16>, dim3((unsigned)ob.tiles), dim3(kFaThreads), 0, s, K, pos, b.bbox, nbox, keys,
                       b.vals, b.s0, ob.totals, ob.status, ob.status_words);
        BGV_TRY(onesweep_sort_u32(keys, keys_alt, b.vals, b.vals_alt, K, &sk, &sv, b.sort_scratch, s, true));
    } else {
        BGV_LAUNCH(k_bh_codes, dim3(1), dim3(kFaThreads), 0, s, K, pos, b.bbox, nbox, keys, b.vals, b.s0);
    }
    BGV_LAUNCH(k_bh_gather, dim3(nb), dim3(kFaThreads), 0, s, K, pos, mass, sk, sv, b.body, b.code, b.part3);
    BGV_LAUNCH(k_bh_prefix, dim3(nb), dim3(kFaThreads), 0, s, K, b.body, b.part3, b.PM, b.PX, b.PY);
    return BGV_OK;
}

// The force launch and the redo of the workgroups whose walk outgrew the fast stack.
template <int G>
static bgv_status bh_force_launch(int32_t K, const BhWs &b, float theta, float kr, float kg, const float2 *fprev,
                                  const CsrWs &csr, FaWs &w, hipStream_t s) {
    const auto k_bh_force_g = k_bh_force<G>;  // one profiler name for every lane count
    const auto k_bh_force_full_g = k_bh_force_full<G>;
    const unsigned grid = (unsigned)((bh_force_blocks(K) + kBhXcds - 1) / kBhXcds * kBhXcds);
    BGV_LAUNCH(k_bh_force_g, dim3(grid), dim3(kBhThreads), 0, s, K, b.body, b.kids, theta * theta, w.A,
               csr.item_of, kr, kg, fprev, w.F, w.part, b.icount, b.redo);
    BGV_LAUNCH(k_bh_force_full_g, dim3(kBhFullBlocks), dim3(kBhThreads), 0, s, K, b.body, b.kids, theta * theta, w.A,
               csr.item_of, kr, kg, fprev, w.F, w.part, b.icount, b.redo);
    return BGV_OK;
}

// Streams of one layout call: the caller's, and (when the call may use it) a second one
// on which the column-blocked attraction of an iteration runs beside that iteration's
// sort and tree build, which leave most compute units idle; fork and join are two
// events of the call.
struct FaStreams {
    hipStream_t s;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

static bgv_status bh_forces(int32_t K, const float2 *pos, const float *mass, const CsrWs &csr, float theta, float kr,
                            float kg, const float2 *fprev, FaWs &w, const FaStreams &st) {
    hipStream_t s = st.s;
    BhWs &b = w.bh;
    const bool side = st.side && csr.cols && K > 1;
    if (side) {  // the attraction reads only the positions: it can start at once
        BGV_CHECK_HIP(hipEventRecord(st.fork, s));
        BGV_CHECK_HIP(hipStreamWaitEvent(st.side, st.fork, 0));
        BGV_TRY(attraction_cols(K, pos, csr, w.A, st.side));
        BGV_CHECK_HIP(hipEventRecord(st.join, st.side));
    }
    BGV_TRY(bh_sorted_bodies(K, pos, mass, b, s));
    // the tree and the attraction (which the force kernel combines), in one launch
    if (K > 1) {
        if (csr.cols) {
            // the tree, and the column-blocked attraction in a launch of its own (its
            // workgroups take most of a compute unit's LDS)
            BGV_LAUNCH(k_bh_build, dim3(grid_for(K - 1, kFaThreads, 65536)), dim3(kFaThreads), 0, s, K, b.code, b.PM,
                       b.PX, b.PY, b.s0, b.body, (BhNode *)nullptr, b.kids);
            if (side)
                BGV_CHECK_HIP(hipStreamWaitEvent(s, st.join, 0));
            else
                BGV_TRY(attraction_cols(K, pos, csr, w.A, s));
        } else if (K >= kAttLdsMin && K <= kAttLdsMax) {
            int cus = 1;
            BGV_TRY(device_cu_count(&cus));
            const unsigned wg = (unsigned)((csr.items_bound + kAttLdsThreads / kWave - 1) / (kAttLdsThreads / kWave));
            BGV_TRY((build_attract<kAttLdsThreads, true>(K, b, wg < (unsigned)cus ? (wg > 0 ? wg : 1u) : (unsigned)cus,
                                                         sizeof(float2) * (size_t)K, pos, csr, w.A, s)));
        } else {
            BGV_TRY((build_attract<kFaThreads, false>(K, b, grid_for(csr.items_bound, kFaThreads / kWave, 16384), 0,
                                                      pos, csr, w.A, s)));
        }
    } else {
        BGV_TRY(attraction(K, pos, csr, w.A, s));
    }
    switch (bh_lanes(K)) {
        case 2: return bh_force_launch<2>(K, b, theta, kr, kg, fprev, csr, w, s);
        case 4: return bh_force_launch<4>(K, b, theta, kr, kg, fprev, csr, w, s);
        default: return bh_force_launch<8>(K, b, theta, kr, kg, fprev, csr, w, s);
    }
}

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_fa2_workspace(int32_t K, int64_t E, const bgv_fa2_params *p) {
    if (!fa_valid(K, E, p)) return 0;
    Carver c(nullptr);
    FaWs w;
    return fa_layout(c, K, E, p, &w);
}

namespace bgv {

// The second stream of each device (see FaStreams), created on first use outside graph
// capture, at the default priority, kept until the process ends.  nullptr when it
// cannot be had: the call then runs on the caller's stream alone, with the same results.
static hipStream_t side_stream(hipStream_t main) {
    static std::mutex mu;
    static hipStream_t side[64] = {};
    static bool tried[64] = {};
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(main, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!tried[dev]) {
        tried[dev] = true;
        hipStream_t q = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) == hipSuccess) side[dev] = q;
    }
    return side[dev];
}

// The iterations of one layout call (the loop of Algorithm 1).
static bgv_status fa2_iterations(int32_t K, float2 *x, float2 *fp, const float *m, const bgv_fa2_params *p, FaWs &w,
                                 int32_t nb, const FaStreams &st) {
    hipStream_t s = st.s;
    float4 *bbox = p->exact ? nullptr : w.bh.bbox;
    if (bbox && p->iters > 0)
        BGV_LAUNCH(k_bh_bbox, dim3(bh_update_blocks(K)), dim3(kFaThreads), 0, s, K, x, bbox, bh_sort_totals(w.bh, K));
    for (int32_t it = 0; it < p->iters; ++it) {
        if (p->exact) {
            BGV_TRY(attraction(K, x, w.csr, w.A, s));
            BGV_TRY(exact_forces(K, x, m, w.A, w.csr.item_of, p->kr, p->kg, fp, w.F, w.part, w.seg, s));
        } else {
            BGV_TRY(bh_forces(K, x, m, w.csr, p->theta, p->kr, p->kg, fp, w, st));  // attraction included
        }
        const int32_t nparts = p->exact ? nb : bh_force_blocks(K);
        if (p->exact) {
            BGV_LAUNCH(k_update, dim3(nb), dim3(kFaThreads), 0, s, K, x, fp, w.F, w.part, nparts, w.speed + (it & 1),
                       w.speed + ((it + 1) & 1), p->tau, p->ks, p->ksmax, (float4 *)nullptr);
        } else {
            BGV_LAUNCH(k_bh_speed, dim3(1), dim3(kBhSpeedThreads), 0, s, w.part, nparts, w.speed + (it & 1),
                       w.speed + ((it + 1) & 1), p->tau, w.bh.redo);
            BGV_LAUNCH(k_bh_update, dim3(bh_update_blocks(K)), dim3(kFaThreads), 0, s, K, x, fp, w.F,
                       w.speed + ((it + 1) & 1), p->ks, p->ksmax, bbox, bh_sort_totals(w.bh, K));
        }
    }
    return BGV_OK;
}

}  // namespace bgv

extern "C" bgv_status bgv_fa2_layout(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                                     const float *mass, float *pos, float *fprev, float *speed,
                                     const bgv_fa2_params *p, void *ws, size_t ws_bytes, bgv_stream_t stream) {
    return fa2_layout_run(K, E, edges, attr_w, mass, pos, fprev, speed, p, ws, ws_bytes, stream, true);
}

// One layout call; with may_fork the column-blocked attraction may run on the device's
// second stream (the allocation-free entry point passes false: it creates nothing).
bgv_status bgv::fa2_layout_run(int32_t K, int64_t E, const int32_t *edges, const float *attr_w, const float *mass,
                               float *pos, float *fprev, float *speed, const bgv_fa2_params *p, void *ws,
                               size_t ws_bytes, bgv_stream_t stream, bool may_fork) {
    clear_error();
    if (!fa_valid(K, E, p)) {
        set_error("bgv_fa2_layout: invalid arguments (K=%d E=%lld)", K, (long long)E);
        return BGV_E_INVALID;
    }
    if ((E > 0 && !edges) || !pos || !fprev || !speed) {
        set_error("bgv_fa2_layout: null pointer");
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_fa2_workspace(K, E, p)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Carver c(ws);
    FaWs w;
    fa_layout(c, K, E, p, &w);
    if (range_check_on()) BGV_TRY(check_edge_ids(K, E, edges, w.flag, s));
    const float *m = nullptr;
    BGV_TRY(build_csr(K, E, edges, attr_w, mass, w.csr, s, &m));
    if (!p->exact) {
        BGV_TRY(fill<uint32_t>(w.bh.icount, 0u, bh_force_blocks(K), s));
        BGV_TRY(fill<uint32_t>(w.bh.redo, 0u, 1, s));
    }

    float2 *x = reinterpret_cast<float2 *>(pos);
    float2 *fp = reinterpret_cast<float2 *>(fprev);
    const int32_t nb = (K + kFaThreads - 1) / kFaThreads;
    BGV_LAUNCH(k_copy_f32, dim3(1), dim3(1), 0, s, speed, w.speed);
    FaStreams st;
    st.s = s;
    if (may_fork && !p->exact && w.csr.cols && K > 1 && p->iters > 0) {
        st.side = side_stream(s);
        if (st.side && (hipEventCreateWithFlags(&st.fork, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&st.join, hipEventDisableTiming) != hipSuccess)) {
            if (st.fork) (void)hipEventDestroy(st.fork);
            st = FaStreams{};
            st.s = s;
        }
    }
    const bgv_status rc = fa2_iterations(K, x, fp, m, p, w, nb, st);
    if (st.fork) (void)hipEventDestroy(st.fork);
    if (st.join) (void)hipEventDestroy(st.join);
    BGV_TRY(rc);
    BGV_LAUNCH(k_copy_f32, dim3(1), dim3(1), 0, s, w.speed + (p->iters & 1), speed);
    if (!p->exact && p->iters > 0 && prof_on())
        BGV_LAUNCH(k_count_total, dim3(1), dim3(kFaThreads), 0, s, w.bh.icount, bh_force_blocks(K));
    return BGV_OK;
}

// Diagnostics: the Barnes-Hut tree of one set of positions (the tree an iteration builds).
extern "C" size_t bgv_bh_tree_workspace(int32_t K) {
    if (K < 1) return 0;
    bgv_fa2_params p{};
    p.exact = 0;
    p.theta = 1.f;
    p.tau = 1.f;
    p.ksmax = 1.f;
    return bgv_fa2_workspace(K, 0, &p);
}

extern "C" bgv_status bgv_bh_tree(int32_t K, const float *pos, const float *mass, uint32_t *codes, float *body,
                                  float *nodeA, int32_t *nodeB, float *s0, void *ws, size_t ws_bytes,
                                  bgv_stream_t stream) {
    clear_error();
    if (K < 1 || !pos || !mass || !codes || !body || !s0 || (K > 1 && (!nodeA || !nodeB))) {
        set_error("bgv_bh_tree: invalid arguments (K=%d)", K);
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_bh_tree_workspace(K)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    bgv_fa2_params p{};
    p.exact = 0;
    Carver c(ws);
    FaWs w;
    fa_layout(c, K, 0, &p, &w);
    BhWs &b = w.bh;
    const float2 *x = reinterpret_cast<const float2 *>(pos);
    const unsigned nb = (unsigned)((K + kFaThreads - 1) / kFaThreads);
    BGV_LAUNCH(k_bh_bbox, dim3(bh_update_blocks(K)), dim3(kFaThreads), 0, s, K, x, b.bbox, bh_sort_totals(b, K));
    BGV_TRY(bh_sorted_bodies(K, x, mass, b, s));
    if (K > 1)
        BGV_LAUNCH(k_bh_build, dim3(grid_for(K - 1, kFaThreads, 65536)), dim3(kFaThreads), 0, s, K, b.code, b.PM,
                   b.PX, b.PY, b.s0, b.body, b.node, b.kids);
    BGV_CHECK_HIP(hipMemcpyAsync(codes, b.code, sizeof(uint32_t) * (size_t)K, hipMemcpyDeviceToDevice, s));
    BGV_CHECK_HIP(hipMemcpyAsync(body, b.body, sizeof(float4) * (size_t)K, hipMemcpyDeviceToDevice, s));
    BGV_CHECK_HIP(hipMemcpyAsync(s0, b.s0, sizeof(float), hipMemcpyDeviceToDevice, s));
    if (K > 1) {
        // the two halves of the node records, each to its own packed array
        BGV_CHECK_HIP(hipMemcpy2DAsync(nodeA, sizeof(float4), reinterpret_cast<const char *>(b.node) + offsetof(BhNode, a), sizeof(BhNode), sizeof(float4),
                                       (size_t)(K - 1), hipMemcpyDeviceToDevice, s));
        BGV_CHECK_HIP(hipMemcpy2DAsync(nodeB, sizeof(int4), reinterpret_cast<const char *>(b.node) + offsetof(BhNode, b), sizeof(BhNode), sizeof(int4),
                                       (size_t)(K - 1), hipMemcpyDeviceToDevice, s));
    }
    return BGV_OK;
}
