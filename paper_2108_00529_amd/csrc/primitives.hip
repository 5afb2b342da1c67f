// Device-wide primitives written for gfx950: fill, exclusive scan (reduce-then-scan)
// and a stable LSD radix sort (8-bit digits, per-tile histograms, wave-ballot ranking).
#include <stdarg.h>
#include <stdio.h>

#include "common.h"
#include "block_scan.h"

namespace bgv {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = '\0'; }
const char *last_error() { return g_err; }

// ------------------------------------------------------------------------ fill ---
template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
bgv_status fill(T *p, T value, int64_t count, hipStream_t s) {
    if (count <= 0) return BGV_OK;
    BGV_LAUNCH(k_fill<T>, dim3(grid_for(count, 256 * 4, 8192)), dim3(256), 0, s, p, value, count);
    return BGV_OK;
}
template bgv_status fill<int32_t>(int32_t *, int32_t, int64_t, hipStream_t);
template bgv_status fill<uint32_t>(uint32_t *, uint32_t, int64_t, hipStream_t);
template bgv_status fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);
template bgv_status fill<uint64_t>(uint64_t *, uint64_t, int64_t, hipStream_t);
template bgv_status fill<float>(float *, float, int64_t, hipStream_t);
template bgv_status fill<double>(double *, double, int64_t, hipStream_t);

// ------------------------------------------------------------------------ scan ---
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const T *in, int64_t n, T *part) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) acc += in[base + j];
    T tot;
    block_excl_scan<T>(acc, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <class T>
__global__ void __launch_bounds__(1024) k_scan_partials(T *part, int64_t nb, T *total) {
    const int64_t per = (nb + blockDim.x - 1) / blockDim.x;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    T acc = T(0);
    for (int64_t i = lo; i < hi; ++i) acc += part[i];
    T tot;
    T pre = block_excl_scan<T>(acc, &tot);
    for (int64_t i = lo; i < hi; ++i) {
        T v = part[i];
        part[i] = pre;
        pre += v;
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const T *in, T *out, int64_t n, const T *part) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? in[base + j] : T(0);
        acc += v[j];
    }
    T tot;
    T pre = block_excl_scan<T>(acc, &tot) + part[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = pre;
        pre += v[j];
    }
}

size_t scan_workspace(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return align_up(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
}

template <class T>
bgv_status exclusive_scan(const T *in, T *out, int64_t n, T *total, void *scratch, hipStream_t s) {
    if (n <= 0) {
        if (total) BGV_TRY(fill<T>(total, T(0), 1, s));
        return BGV_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    T *part = static_cast<T *>(scratch);
    BGV_LAUNCH(k_scan_reduce<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, part);
    BGV_LAUNCH(k_scan_partials<T>, dim3(1), dim3(1024), 0, s, part, nb, total);
    BGV_LAUNCH(k_scan_down<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, part);
    return BGV_OK;
}
template bgv_status exclusive_scan<uint32_t>(const uint32_t *, uint32_t *, int64_t, uint32_t *, void *, hipStream_t);
template bgv_status exclusive_scan<double>(const double *, double *, int64_t, double *, void *, hipStream_t);
template bgv_status exclusive_scan<uint64_t>(const uint64_t *, uint64_t *, int64_t, uint64_t *, void *, hipStream_t);

bgv_status exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *scratch,
                              hipStream_t s) {
    return exclusive_scan<uint32_t>(in, out, n, total, scratch, s);
}

// ------------------------------------------------------------------ radix sort ---
constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / kWave;
constexpr int kRsLocalOffsetTiles = kRsFewTiles;  // up to this many tiles the scatter kernel scans the counts itself
// Keys per thread: 16 for large sorts; 4 for sorts of at most kRsSmallN keys, so that
// small sorts (the per-iteration Morton sort) spread over 4x more workgroups.
constexpr int kRsItemsLarge = 16;
constexpr int kRsItemsSmall = 4;
constexpr int64_t kRsSmallN = (int64_t)kRsLocalOffsetTiles * kRsThreads * kRsItemsSmall;

static int64_t rs_items(int64_t n) { return n <= kRsSmallN ? kRsItemsSmall : kRsItemsLarge; }

// Per-tile digit counts (counts[digit * nb + tile]).  `zero` (or null): a 256 x nb count
// buffer this launch clears for the next pass.  With n_dev the key count is *n_dev and n
// only bounds it (the grid covers n).
template <int ITEMS, typename KT>
__global__ void __launch_bounds__(kRsThreads) k_rs_upsweep(const KT *keys, int64_t n, int shift,
                                                            uint32_t *counts, int64_t nb, uint32_t *zero,
                                                            const unsigned long long *n_dev) {
    if (n_dev) n = (int64_t)*n_dev;
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    if (zero) zero[(int64_t)blockIdx.x * 256 + threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kRsThreads * ITEMS);
#pragma unroll 4
    for (int j = 0; j < ITEMS; ++j) {
        int64_t i = base + (int64_t)j * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&hist[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter of one tile of kRsThreads * ITEMS consecutive keys.  Wave w owns the
// tile's w-th quarter and reads it in rounds of 64 consecutive keys; a key's rank among
// the equal digits of its wave = (equal digits in the wave's earlier rounds, kept in a
// per-wave LDS histogram) + (equal-digit lanes below it in its round, from 8 ballots).
// Ranks are turned into tile positions (digits in order, waves in order within a digit),
// the tile is reordered by digit in LDS, and written out in that order: each digit's
// keys leave as one contiguous run, so the stores coalesce.
// With `next` (raw-count mode only), the launch also counts the next pass's digit of
// every key it writes into next[digit * nb + destination tile] (integer atomics, so the
// counts do not depend on timing), which replaces the next pass's counting launch;
// `zero` (or null) is a count buffer it clears for the pass after that.
template <int ITEMS, typename KT>
__global__ void __launch_bounds__(kRsThreads) k_rs_downsweep(const KT *keys, KT *keys_out,
                                                              const uint32_t *vals, uint32_t *vals_out,
                                                              int64_t n, int shift, const uint32_t *offsets,
                                                              int64_t nb, int raw_counts, uint32_t *next,
                                                              int next_shift, uint32_t *zero,
                                                              const unsigned long long *n_dev) {
    if (n_dev) n = (int64_t)*n_dev;  // n bounds it
    constexpr int kTile = kRsThreads * ITEMS;
    __shared__ uint32_t running[256];  // where each digit of this tile starts in the output
    __shared__ uint32_t lstart[256];   // where each digit starts inside the tile
    __shared__ uint32_t hist[kRsWaves][256];
    __shared__ KT skey[kTile];
    __shared__ uint32_t sval[kTile];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    if (raw_counts) {
        // few tiles: derive this tile's digit offsets from the raw per-tile counts here
        // instead of a separate device-wide scan
        // 32 independent loads at a time: one L2 round trip for up to 32 tiles (a
        // dependent chain of round trips otherwise dominates small sorts)
        uint32_t tot = 0, pre = 0;
        const uint32_t *row = offsets + (int64_t)t * nb;
        for (int64_t b0 = 0; b0 < nb; b0 += 32) {
            uint32_t c[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) c[u] = b0 + u < nb ? row[b0 + u] : 0u;
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                if (b0 + u < (int64_t)blockIdx.x) pre += c[u];
                tot += c[u];
            }
        }
        uint32_t all;
        running[t] = block_excl_scan<uint32_t>(tot, &all) + pre;
    } else {
        running[t] = offsets[(int64_t)t * nb + blockIdx.x];
    }
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) hist[q][t] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int64_t wbase = base + (int64_t)w * (kWave * ITEMS);
    KT key[ITEMS];
    uint32_t val[ITEMS], rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        key[j] = i < n ? keys[i] : KT(0);
        val[j] = (i < n && vals) ? vals[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = wbase + (int64_t)j * kWave + lane < n;
        const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(match & lt_mask);
        const uint32_t before = hist[w][d];
        rk[j] = before + below;
        // every lane of the round has read the histogram; the lowest lane of each digit
        // group then adds the group's size (LDS operations of a wave take effect in order)
        if (valid && below == 0) hist[w][d] = before + (uint32_t)__popcll(match);
    }
    __syncthreads();
    {
        uint32_t acc = 0;
#pragma unroll
        for (int q = 0; q < kRsWaves; ++q) {
            const uint32_t c = hist[q][t];
            hist[q][t] = acc;  // equal digits in lower waves of the tile
            acc += c;
        }
        uint32_t all;
        lstart[t] = block_excl_scan<uint32_t>(acc, &all);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (wbase + (int64_t)j * kWave + lane < n) {
            const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
            const uint32_t lp = lstart[d] + hist[w][d] + rk[j];
            skey[lp] = key[j];
            sval[lp] = val[j];
        }
    }
    __syncthreads();
    const int cnt = (int)((n - base) < kTile ? (n - base) : kTile);
    for (int p = t; p < cnt; p += kRsThreads) {
        const KT k = skey[p];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t dst = running[d] + ((uint32_t)p - lstart[d]);
        keys_out[dst] = k;
        if (vals) vals_out[dst] = sval[p];
        if (next) atomicAdd(&next[(int64_t)((k >> next_shift) & 255u) * nb + dst / (uint32_t)kTile], 1u);
    }
    if (zero) zero[(int64_t)blockIdx.x * 256 + t] = 0u;
}

// Tile count bound for any sort of at most n keys: small sorts use more (smaller)
// tiles than a large sort of n keys would, so both tile counts are covered.
static int64_t radix_tiles_bound(int64_t n) {
    const int64_t ns = n < kRsSmallN ? n : kRsSmallN;
    const int64_t nb_small = (ns + kRsThreads * kRsItemsSmall - 1) / (kRsThreads * kRsItemsSmall);
    int64_t nb_large = (n + kRsThreads * kRsItemsLarge - 1) / (kRsThreads * kRsItemsLarge);
    if (nb_large < 1) nb_large = 1;
    return nb_small > nb_large ? nb_small : nb_large;
}

// Layout: per-tile counts [256][tiles], scan scratch, three [256][64] count buffers for
// the few-tile path.
size_t radix_workspace(int64_t n) {
    const int64_t nb = radix_tiles_bound(n);
    return align_up(sizeof(uint32_t) * 256 * (size_t)nb) + scan_workspace(256 * nb) +
           align_up(3 * sizeof(uint32_t) * 256 * (size_t)kRsLocalOffsetTiles);
}

bool radix_few_tiles(int64_t n, int64_t *tiles, int *items) {
    if (n <= 1) return false;
    const int it = (int)rs_items(n);
    const int64_t nb = (n + (int64_t)kRsThreads * it - 1) / ((int64_t)kRsThreads * it);
    if (nb > kRsLocalOffsetTiles) return false;
    *tiles = nb;
    *items = it;
    return true;
}

// The three rotating count buffers of the few-tile path sit after the per-tile counts
// and the scan scratch.
static uint32_t *rs_few_buffers(void *scratch, int64_t n) {
    const size_t counts_bytes = align_up(sizeof(uint32_t) * 256 * (size_t)radix_tiles_bound(n));
    return reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) + counts_bytes +
                                        scan_workspace(256 * radix_tiles_bound(n)));
}

void radix_pass0_buffers(void *scratch, int64_t n, uint32_t **counts0, uint32_t **clear1) {
    uint32_t *cb = rs_few_buffers(scratch, n);
    *counts0 = cb;
    *clear1 = cb + 256 * kRsLocalOffsetTiles;
}

template <typename KT>
static bgv_status radix_sort(KT *keys, KT *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t n, int nbits,
                             KT **keys_out, uint32_t **vals_out, void *scratch, hipStream_t s, bool counted,
                             const unsigned long long *n_dev) {
    // one name per kernel shape for the profiler (the key width is not part of it)
    const auto k_rs_upsweep_small = k_rs_upsweep<kRsItemsSmall, KT>;
    const auto k_rs_upsweep_large = k_rs_upsweep<kRsItemsLarge, KT>;
    const auto k_rs_downsweep_small = k_rs_downsweep<kRsItemsSmall, KT>;
    const auto k_rs_downsweep_large = k_rs_downsweep<kRsItemsLarge, KT>;
    KT *src = keys, *dst = keys_alt;
    uint32_t *vsrc = vals, *vdst = vals_alt;
    if (counted) {
        int64_t t;
        int it;
        if (!radix_few_tiles(n, &t, &it)) {
            set_error("radix sort: pass-0 counts given for a sort that is not on the few-tile path");
            return BGV_E_INVALID;
        }
    }
    if (n > 1) {
        const bool small = rs_items(n) == kRsItemsSmall;
        const int64_t tile = kRsThreads * rs_items(n);
        const int64_t nb = (n + tile - 1) / tile;
        const size_t counts_bytes = align_up(sizeof(uint32_t) * 256 * (size_t)radix_tiles_bound(n));
        uint32_t *counts = static_cast<uint32_t *>(scratch);
        void *scan_scratch = static_cast<char *>(scratch) + counts_bytes;
        const int npass = (nbits + 7) / 8;
        if (nb <= kRsLocalOffsetTiles) {
            // few tiles: every scatter derives its offsets from the raw counts and counts
            // the next pass's digits itself, so only pass 0 has a counting launch; three
            // count buffers rotate (read by pass i, filled during pass i-1, cleared two
            // passes ahead)
            uint32_t *cb = rs_few_buffers(scratch, n);
            uint32_t *buf[3] = {cb, cb + 256 * kRsLocalOffsetTiles, cb + 2 * 256 * kRsLocalOffsetTiles};
            uint32_t *zero1 = npass > 1 ? buf[1] : nullptr;
            if (counted) {
                // the caller counted pass 0 into buf[0] and cleared buf[1]
            } else if (small)
                BGV_LAUNCH(k_rs_upsweep_small, dim3((unsigned)nb), dim3(kRsThreads), 0, s, src, n, 0,
                           buf[0], nb, zero1, n_dev);
            else
                BGV_LAUNCH(k_rs_upsweep_large, dim3((unsigned)nb), dim3(kRsThreads), 0, s, src, n, 0,
                           buf[0], nb, zero1, n_dev);
            for (int pass = 0; pass < npass; ++pass) {
                const int shift = 8 * pass;
                uint32_t *next = pass + 1 < npass ? buf[(pass + 1) % 3] : nullptr;
                uint32_t *zero = pass + 2 < npass ? buf[(pass + 2) % 3] : nullptr;
                if (small)
                    BGV_LAUNCH(k_rs_downsweep_small, dim3((unsigned)nb), dim3(kRsThreads), 0, s, src, dst,
                               vsrc, vdst, n, shift, buf[pass % 3], nb, 1, next, shift + 8, zero, n_dev);
                else
                    BGV_LAUNCH(k_rs_downsweep_large, dim3((unsigned)nb), dim3(kRsThreads), 0, s, src, dst,
                               vsrc, vdst, n, shift, buf[pass % 3], nb, 1, next, shift + 8, zero, n_dev);
                KT *tk = src; src = dst; dst = tk;
                uint32_t *tv = vsrc; vsrc = vdst; vdst = tv;
            }
        } else {
            for (int pass = 0; pass < npass; ++pass) {
                const int shift = 8 * pass;
                BGV_LAUNCH(k_rs_upsweep_large, dim3((unsigned)nb), dim3(kRsThreads), 0, s, src, n, shift,
                           counts, nb, (uint32_t *)nullptr, n_dev);
                BGV_TRY(exclusive_scan_u32(counts, counts, 256 * nb, nullptr, scan_scratch, s));
                BGV_LAUNCH(k_rs_downsweep_large, dim3((unsigned)nb), dim3(kRsThreads), 0, s, src, dst, vsrc,
                           vdst, n, shift, counts, nb, 0, (uint32_t *)nullptr, 0, (uint32_t *)nullptr, n_dev);
                KT *tk = src; src = dst; dst = tk;
                uint32_t *tv = vsrc; vsrc = vdst; vdst = tv;
            }
        }
    }
    *keys_out = src;
    if (vals_out) *vals_out = vsrc;
    return BGV_OK;
}

bgv_status radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t n,
                          int nbits, uint64_t **keys_out, uint32_t **vals_out, void *scratch, hipStream_t s,
                          bool counted, const unsigned long long *n_dev) {
    return radix_sort<uint64_t>(keys, keys_alt, vals, vals_alt, n, nbits, keys_out, vals_out, scratch, s, counted,
                                n_dev);
}

bgv_status radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t n,
                          int nbits, uint32_t **keys_out, uint32_t **vals_out, void *scratch, hipStream_t s,
                          bool counted, const unsigned long long *n_dev) {
    if (nbits > 32) {
        set_error("radix_sort_u32: %d key bits", nbits);
        return BGV_E_INVALID;
    }
    return radix_sort<uint32_t>(keys, keys_alt, vals, vals_alt, n, nbits, keys_out, vals_out, scratch, s, counted,
                                n_dev);
}

// ----------------------------------------------------------- one-sweep radix sort ---
// Stable LSD sort of 32-bit keys (with 32-bit values) in four 8-bit passes, one launch
// per pass and no per-key device atomics.  Before the passes, every key's four digits
// are counted per tile and each tile adds its counts into the totals per (pass, digit)
// (os_count, or a producer of the keys doing the same: one device atomic per tile and
// digit); a pass's tiles scan the 256 totals of their pass for the digit bases.  In a pass each
// tile takes its index in launch order from a counter (so every earlier tile has
// started), ranks its keys by digit as the scatter above does, publishes its digit
// counts, and finds how many keys of each digit precede it by walking back over the
// published words of earlier tiles: a word holds either that tile's own count
// (kOsAgg) or its inclusive prefix (kOsInc), so the walk adds counts until it meets an
// inclusive prefix (decoupled look-back).  Tile 0 publishes its counts as inclusive, so
// every walk ends; no tile waits on a later one.  The words and counters are cleared
// by the counting launch.
constexpr uint32_t kOsAgg = 1u << 30;
constexpr uint32_t kOsInc = 2u << 30;
constexpr uint32_t kOsCountMask = (1u << 30) - 1;
constexpr int kOsPasses = 4;
// A walk step waits for a word that an earlier, already started tile publishes right
// after ranking its keys; the bound only keeps a broken invariant from hanging the GPU
// (the sort's output is then wrong, which the callers' tests would show).
constexpr uint32_t kOsMaxSpins = 1u << 20;
constexpr int kOsWindow = 8;  // earlier tiles' words read at once by a walk step

__device__ __forceinline__ void os_publish(uint32_t *w, uint32_t v) {
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t os_peek(const uint32_t *w) {
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static int64_t os_tiles(int64_t n, int items) { return (n + kRsThreads * items - 1) / (kRsThreads * items); }

void onesweep_layout(void *scratch, int64_t n, int items, OsBuffers *b) {
    const int64_t tiles = os_tiles(n, items);
    char *p = static_cast<char *>(scratch);
    b->tiles = tiles;
    b->items = items;
    b->totals = reinterpret_cast<uint32_t *>(p);
    p += align_up(sizeof(uint32_t) * kOsTotals);
    b->status = reinterpret_cast<uint32_t *>(p);  // passes x tiles x 256 words, then the pass counters
    b->status_words = (int64_t)kOsPasses * tiles * 256 + kOsPasses;
}

size_t onesweep_workspace(int64_t n) {
    const int64_t tiles = os_tiles(n > 0 ? n : 1, os_items(n));
    return align_up(sizeof(uint32_t) * kOsTotals) +
           align_up(sizeof(uint32_t) * ((size_t)kOsPasses * tiles * 256 + kOsPasses));
}

// Digit counts of one tile's keys for all four passes, added into the totals, and,
// spread over the grid, the clearing of the look-back words.
template <int ITEMS>
__global__ void __launch_bounds__(kRsThreads) k_os_count(const uint32_t *__restrict__ keys, int64_t n,
                                                          uint32_t *__restrict__ totals,
                                                          uint32_t *__restrict__ status, int64_t status_words) {
    __shared__ uint32_t hist[kOsPasses][256];
#pragma unroll
    for (int q = 0; q < kOsPasses; ++q) hist[q][threadIdx.x] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * kRsThreads + threadIdx.x; i < status_words;
         i += (int64_t)gridDim.x * kRsThreads)
        status[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kRsThreads * ITEMS);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * kRsThreads + threadIdx.x;
        if (i < n) {
            const uint32_t k = keys[i];
#pragma unroll
            for (int q = 0; q < kOsPasses; ++q) atomicAdd(&hist[q][(k >> (8 * q)) & 255u], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kOsPasses; ++q)
        if (hist[q][threadIdx.x]) atomicAdd(&totals[q * 256 + threadIdx.x], hist[q][threadIdx.x]);
}

template <int ITEMS>
__global__ void __launch_bounds__(kRsThreads) k_os_pass(const uint32_t *__restrict__ keys, uint32_t *__restrict__ keys_out,
                                                         const uint32_t *__restrict__ vals,
                                                         uint32_t *__restrict__ vals_out, int64_t n, int64_t tiles,
                                                         int shift, const uint32_t *__restrict__ totals,
                                                         uint32_t *status, uint32_t *counter) {
    constexpr int kTile = kRsThreads * ITEMS;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t running[256];
    __shared__ uint32_t lstart[256];
    __shared__ uint32_t hist[kRsWaves][256];
    __shared__ uint32_t skey[kTile];
    __shared__ uint32_t sval[kTile];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    if (t == 0) s_tile = atomicAdd(counter, 1u);
    const uint32_t tot = totals[t];  // keys of digit t in this pass
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) hist[q][t] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= tiles) return;  // only if the counter was not cleared (uniform)
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = tile * kTile;
    const int64_t wbase = base + (int64_t)w * (kWave * ITEMS);
    uint32_t key[ITEMS], val[ITEMS], rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        key[j] = i < n ? keys[i] : 0u;
        val[j] = i < n ? vals[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = wbase + (int64_t)j * kWave + lane < n;
        const uint32_t d = (key[j] >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(match & lt_mask);
        const uint32_t before = hist[w][d];
        rk[j] = before + below;
        if (valid && below == 0) hist[w][d] = before + (uint32_t)__popcll(match);
    }
    __syncthreads();
    uint32_t cnt_d = 0;  // this tile's keys of digit t
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) {
        const uint32_t c = hist[q][t];
        hist[q][t] = cnt_d;
        cnt_d += c;
    }
    os_publish(&status[tile * 256 + t], (tile == 0 ? kOsInc : kOsAgg) | cnt_d);
    uint32_t all;
    lstart[t] = block_excl_scan<uint32_t>(cnt_d, &all);
    uint32_t excl = 0;
    if (tile > 0) {
        // the walk reads the words of kOsWindow earlier tiles at once (independent loads),
        // then adds them nearest first up to the first inclusive prefix; below tile 0 a
        // word reads as an inclusive zero and is not loaded
        uint32_t spins = 0;
        bool done = false;
        for (int64_t j = tile - 1; !done; j -= kOsWindow) {
            uint32_t v[kOsWindow];
#pragma unroll
            for (int q = 0; q < kOsWindow; ++q) v[q] = j - q >= 0 ? os_peek(&status[(j - q) * 256 + t]) : kOsInc;
#pragma unroll
            for (int q = 0; q < kOsWindow; ++q) {
                if (done) break;
                uint32_t x = v[q];
                while ((x & ~kOsCountMask) == 0u && ++spins < kOsMaxSpins) x = os_peek(&status[(j - q) * 256 + t]);
                excl += x & kOsCountMask;
                if (x & kOsInc) done = true;
            }
        }
        os_publish(&status[tile * 256 + t], kOsInc | (excl + cnt_d));
    }
    uint32_t all_keys;
    running[t] = block_excl_scan<uint32_t>(tot, &all_keys) + excl;  // keys of lower digits, then earlier tiles
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (wbase + (int64_t)j * kWave + lane < n) {
            const uint32_t d = (key[j] >> shift) & 255u;
            const uint32_t lp = lstart[d] + hist[w][d] + rk[j];
            skey[lp] = key[j];
            sval[lp] = val[j];
        }
    }
    __syncthreads();
    const int cnt = (int)((n - base) < kTile ? (n - base) : kTile);
    for (int p = t; p < cnt; p += kRsThreads) {
        const uint32_t k = skey[p];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t dst = running[d] + ((uint32_t)p - lstart[d]);
        keys_out[dst] = k;
        vals_out[dst] = sval[p];
    }
}

// ------------------------------------------------ one-sweep sort of keys alone ---
// The same passes for keys without values (32 or 64 bits, the low nbits significant:
// ceil(nbits / 8) passes), whose count may be known only on the device (*n_dev <= the
// bound n): every launch is sized by the bound and reads the count itself.  One
// counting launch first reads the keys once, adds the digit counts of every pass into
// the totals and clears the look-back words and tile counters; then each pass is one
// launch that reads and writes every key once.
constexpr int kOs64Items = 16;  // keys per thread for 64-bit keys
template <typename KT>
struct OsKeyShape {
    static constexpr int kItems = sizeof(KT) == 8 ? kOs64Items : 16;  // keys per thread
    static constexpr int kTile = kRsThreads * kItems;
};
constexpr int kOsMaxPasses = 8;
constexpr unsigned kOsCountBlocks = 1024;
constexpr int kOsCountLoads = 8;
constexpr int kOsKeyWindow = 8;  // earlier tiles' words read at once by a look-back step

static int os_key_passes(int nbits) { return nbits <= 0 ? 1 : (nbits + 7) / 8; }
template <typename KT>
static int64_t os_key_tiles(int64_t n) {
    return (n + OsKeyShape<KT>::kTile - 1) / OsKeyShape<KT>::kTile;
}

size_t onesweep_keys_workspace(int64_t n, int nbits) {
    const int64_t t32 = os_key_tiles<uint32_t>(n > 0 ? n : 1), t64 = os_key_tiles<uint64_t>(n > 0 ? n : 1);
    const int64_t tiles = t32 > t64 ? t32 : t64;
    const int passes = os_key_passes(nbits);
    return align_up(sizeof(uint32_t) * kOsMaxPasses * 256) +
           align_up(sizeof(uint32_t) * ((size_t)passes * tiles * 256 + passes));
}

__device__ __forceinline__ int64_t os_key_count(const unsigned long long *n_dev, int64_t n) {
    if (!n_dev) return n;
    const int64_t c = (int64_t)*n_dev;
    return c < n ? c : n;
}

template <typename KT>
__global__ void __launch_bounds__(kRsThreads) k_os_count_keys(const KT *__restrict__ keys,
                                                               const unsigned long long *__restrict__ n_dev,
                                                               int64_t n_bound, int passes,
                                                               uint32_t *__restrict__ totals,
                                                               uint32_t *__restrict__ status, int64_t status_words) {
    __shared__ uint32_t hist[kOsMaxPasses][256];
    for (int q = 0; q < passes; ++q) hist[q][threadIdx.x] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * kRsThreads + threadIdx.x; i < status_words;
         i += (int64_t)gridDim.x * kRsThreads)
        status[i] = 0u;
    __syncthreads();
    const int64_t n = os_key_count(n_dev, n_bound);
    // kOsCountLoads keys per thread and round, all loaded before any is counted
    const int64_t stride = (int64_t)gridDim.x * kRsThreads;
    for (int64_t i0 = (int64_t)blockIdx.x * kRsThreads + threadIdx.x; i0 < n; i0 += stride * kOsCountLoads) {
        KT k[kOsCountLoads];
#pragma unroll
        for (int u = 0; u < kOsCountLoads; ++u) {
            const int64_t i = i0 + u * stride;
            k[u] = i < n ? keys[i] : (KT)0;
        }
#pragma unroll
        for (int u = 0; u < kOsCountLoads; ++u)
            if (i0 + u * stride < n)
                for (int q = 0; q < passes; ++q) atomicAdd(&hist[q][(uint32_t)(k[u] >> (8 * q)) & 255u], 1u);
    }
    __syncthreads();
    for (int q = 0; q < passes; ++q)
        if (hist[q][threadIdx.x]) atomicAdd(&totals[q * 256 + threadIdx.x], hist[q][threadIdx.x]);
}

template <typename KT>
__global__ void __launch_bounds__(kRsThreads, 4) k_os_pass_keys(const KT *__restrict__ keys, KT *__restrict__ keys_out,
                                                              const unsigned long long *__restrict__ n_dev,
                                                              int64_t n_bound, int shift,
                                                              const uint32_t *__restrict__ totals, uint32_t *status,
                                                              uint32_t *counter) {
    constexpr int ITEMS = OsKeyShape<KT>::kItems;
    constexpr int kTile = OsKeyShape<KT>::kTile;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t running[256];
    __shared__ uint32_t lstart[256];
    __shared__ uint32_t hist[kRsWaves][256];
    __shared__ KT skey[kTile];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    if (t == 0) s_tile = atomicAdd(counter, 1u);
    const uint32_t tot = totals[t];  // keys of digit t in this pass
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) hist[q][t] = 0;
    __syncthreads();
    const int64_t n = os_key_count(n_dev, n_bound);
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int64_t tile = s_tile;
    if (tile >= tiles) return;  // uniform: tiles past the count take no part
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = tile * kTile;
    const int64_t wbase = base + (int64_t)w * (kWave * ITEMS);
    KT key[ITEMS];
    uint32_t rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        key[j] = i < n ? keys[i] : (KT)0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = wbase + (int64_t)j * kWave + lane < n;
        const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(match & lt_mask);
        const uint32_t before = hist[w][d];
        rk[j] = before + below;
        if (valid && below == 0) hist[w][d] = before + (uint32_t)__popcll(match);
    }
    __syncthreads();
    uint32_t cnt_d = 0;  // this tile's keys of digit t
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) {
        const uint32_t c = hist[q][t];
        hist[q][t] = cnt_d;
        cnt_d += c;
    }
    os_publish(&status[tile * 256 + t], (tile == 0 ? kOsInc : kOsAgg) | cnt_d);
    uint32_t all;
    lstart[t] = block_excl_scan<uint32_t>(cnt_d, &all);
    __syncthreads();
    // the tile's keys in digit order in LDS before the look-back, so that no key is held
    // in registers while it waits
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (wbase + (int64_t)j * kWave + lane < n) {
            const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
            skey[lstart[d] + hist[w][d] + rk[j]] = key[j];
        }
    }
    uint32_t excl = 0;
    if (tile > 0) {
        uint32_t spins = 0;
        bool done = false;
        for (int64_t j = tile - 1; !done; j -= kOsKeyWindow) {
            uint32_t v[kOsKeyWindow];
#pragma unroll
            for (int q = 0; q < kOsKeyWindow; ++q)
                v[q] = j - q >= 0 ? os_peek(&status[(j - q) * 256 + t]) : kOsInc;
#pragma unroll
            for (int q = 0; q < kOsKeyWindow; ++q) {
                if (done) break;
                uint32_t x = v[q];
                while ((x & ~kOsCountMask) == 0u && ++spins < kOsMaxSpins) x = os_peek(&status[(j - q) * 256 + t]);
                excl += x & kOsCountMask;
                if (x & kOsInc) done = true;
            }
        }
        os_publish(&status[tile * 256 + t], kOsInc | (excl + cnt_d));
    }
    uint32_t all_keys;
    running[t] = block_excl_scan<uint32_t>(tot, &all_keys) + excl;  // keys of lower digits, then earlier tiles
    __syncthreads();
    const int cnt = (int)((n - base) < kTile ? (n - base) : kTile);
    for (int p = t; p < cnt; p += kRsThreads) {
        const KT k = skey[p];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        keys_out[running[d] + ((uint32_t)p - lstart[d])] = k;
    }
}

// The totals from per-block digit counts that a producer of the keys wrote
// (bcnt[block * passes * 256 + pass * 256 + d]), and the clearing of the look-back
// words: workgroup (c, q) sums the counts of digit threadIdx.x in pass q over its share
// of the blocks.
constexpr int kOsSumRows = 16;
__global__ void __launch_bounds__(kRsThreads) k_os_sum_block_counts(const uint32_t *__restrict__ bcnt, int64_t nblocks,
                                                                     int passes, uint32_t *__restrict__ totals,
                                                                     uint32_t *__restrict__ status, int64_t status_words) {
    const int q = blockIdx.y;
    const int64_t b0 = (int64_t)blockIdx.x * kOsSumRows;
    uint32_t acc = 0;
#pragma unroll 8
    for (int r = 0; r < kOsSumRows; ++r) {
        const int64_t b = b0 + r;
        if (b < nblocks) acc += bcnt[(b * passes + q) * 256 + threadIdx.x];
    }
    if (acc) atomicAdd(&totals[q * 256 + threadIdx.x], acc);
    const int64_t nthreads = (int64_t)gridDim.x * gridDim.y * kRsThreads;
    for (int64_t i = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kRsThreads + threadIdx.x; i < status_words;
         i += nthreads)
        status[i] = 0u;
}

int onesweep_key_passes(int nbits) { return os_key_passes(nbits); }

bgv_status onesweep_keys_counted(const uint32_t *bcnt, int64_t nblocks, int64_t n, int nbits, bool wide,
                                 void *scratch, hipStream_t s) {
    const int passes = os_key_passes(nbits);
    const int64_t tiles = wide ? os_key_tiles<uint64_t>(n) : os_key_tiles<uint32_t>(n);
    uint32_t *totals = static_cast<uint32_t *>(scratch);
    uint32_t *status = reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) +
                                                    align_up(sizeof(uint32_t) * kOsMaxPasses * 256));
    const int64_t status_words = (int64_t)passes * tiles * 256 + passes;
    BGV_TRY(fill<uint32_t>(totals, 0u, passes * 256, s));
    const dim3 grid((unsigned)((nblocks + kOsSumRows - 1) / kOsSumRows), (unsigned)passes);
    BGV_LAUNCH(k_os_sum_block_counts, grid, dim3(kRsThreads), 0, s, bcnt, nblocks, passes, totals, status,
               status_words);
    return BGV_OK;
}

template <typename KT>
bgv_status onesweep_sort_keys(KT *keys, KT *keys_alt, int64_t n, const unsigned long long *n_dev, int nbits,
                              KT **keys_out, void *scratch, hipStream_t s, bool counted) {
    const int passes = os_key_passes(nbits);
    if (passes > (int)sizeof(KT) || n > (int64_t)kOsCountMask) {
        set_error("onesweep_sort_keys: %d key bits, %lld keys", nbits, (long long)n);
        return BGV_E_INVALID;
    }
    KT *src = keys, *dst = keys_alt;
    if (n > 0) {
        const int64_t tiles = os_key_tiles<KT>(n);
        char *p = static_cast<char *>(scratch);
        uint32_t *totals = reinterpret_cast<uint32_t *>(p);
        p += align_up(sizeof(uint32_t) * kOsMaxPasses * 256);
        uint32_t *status = reinterpret_cast<uint32_t *>(p);
        const int64_t status_words = (int64_t)passes * tiles * 256 + passes;
        uint32_t *counters = status + (int64_t)passes * tiles * 256;
        if (!counted) {
            BGV_TRY(fill<uint32_t>(totals, 0u, passes * 256, s));
            const unsigned gc = grid_for(n, kRsThreads * 16, kOsCountBlocks);
            BGV_LAUNCH(k_os_count_keys<KT>, dim3(gc), dim3(kRsThreads), 0, s, keys, n_dev, n, passes, totals, status,
                       status_words);
        }
        for (int pass = 0; pass < passes; ++pass) {
            BGV_LAUNCH(k_os_pass_keys<KT>, dim3((unsigned)tiles), dim3(kRsThreads), 0, s, src, dst, n_dev, n,
                       8 * pass, totals + 256 * pass, status + (int64_t)pass * tiles * 256, counters + pass);
            KT *tk = src;
            src = dst;
            dst = tk;
        }
    }
    *keys_out = src;
    return BGV_OK;
}
template bgv_status onesweep_sort_keys<uint32_t>(uint32_t *, uint32_t *, int64_t, const unsigned long long *, int,
                                                 uint32_t **, void *, hipStream_t, bool);
template bgv_status onesweep_sort_keys<uint64_t>(uint64_t *, uint64_t *, int64_t, const unsigned long long *, int,
                                                 uint64_t **, void *, hipStream_t, bool);

int os_items(int64_t n) { return n <= (int64_t)(1 << 16) ? 4 : n <= (int64_t)(1 << 20) ? 8 : 16; }

bgv_status onesweep_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t n,
                             uint32_t **keys_out, uint32_t **vals_out, void *scratch, hipStream_t s, bool counted) {
    OsBuffers b;
    onesweep_layout(scratch, n, os_items(n), &b);
    uint32_t *src = keys, *dst = keys_alt, *vsrc = vals, *vdst = vals_alt;
    if (n > 1) {
        const unsigned tiles = (unsigned)b.tiles;
        if (!counted) {
            BGV_TRY(fill<uint32_t>(b.totals, 0u, kOsTotals, s));
            if (b.items == 4)
                BGV_LAUNCH(k_os_count<4>, dim3(tiles), dim3(kRsThreads), 0, s, src, n, b.totals, b.status,
                           b.status_words);
            else if (b.items == 8)
                BGV_LAUNCH(k_os_count<8>, dim3(tiles), dim3(kRsThreads), 0, s, src, n, b.totals, b.status,
                           b.status_words);
            else
                BGV_LAUNCH(k_os_count<16>, dim3(tiles), dim3(kRsThreads), 0, s, src, n, b.totals, b.status,
                           b.status_words);
        }
        uint32_t *counters = b.status + (int64_t)kOsPasses * b.tiles * 256;
        for (int pass = 0; pass < kOsPasses; ++pass) {
            uint32_t *st = b.status + (int64_t)pass * b.tiles * 256;
            if (b.items == 4)
                BGV_LAUNCH(k_os_pass<4>, dim3(tiles), dim3(kRsThreads), 0, s, src, dst, vsrc, vdst, n, b.tiles,
                           8 * pass, b.totals + 256 * pass, st, counters + pass);
            else if (b.items == 8)
                BGV_LAUNCH(k_os_pass<8>, dim3(tiles), dim3(kRsThreads), 0, s, src, dst, vsrc, vdst, n, b.tiles,
                           8 * pass, b.totals + 256 * pass, st, counters + pass);
            else
                BGV_LAUNCH(k_os_pass<16>, dim3(tiles), dim3(kRsThreads), 0, s, src, dst, vsrc, vdst, n, b.tiles,
                           8 * pass, b.totals + 256 * pass, st, counters + pass);
            uint32_t *tk = src; src = dst; dst = tk;
            uint32_t *tv = vsrc; vsrc = vdst; vdst = tv;
        }
    }
    *keys_out = src;
    *vals_out = vsrc;
    return BGV_OK;
}

}  // namespace bgv

extern "C" const char *bgv_status_string(bgv_status s) {
    switch (s) {
        case BGV_OK: return "BGV_OK";
        case BGV_E_INVALID: return "BGV_E_INVALID";
        case BGV_E_RANGE: return "BGV_E_RANGE";
        case BGV_E_WORKSPACE: return "BGV_E_WORKSPACE";
        case BGV_E_HIP: return "BGV_E_HIP";
        default: return "BGV_E_UNKNOWN";
    }
}

extern "C" const char *bgv_last_error(void) { return bgv::last_error(); }
