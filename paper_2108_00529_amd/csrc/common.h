// Internal helpers shared by the HIP translation units of libbgv (gfx950 only).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bgv.h"

namespace bgv {

constexpr int kWave = 64;  // CDNA wavefront width

// Thread-local error message behind bgv_last_error().
void set_error(const char *fmt, ...);
void clear_error();

#define BGV_CHECK_HIP(call)                                                              \
    do {                                                                                 \
        hipError_t _e = (call);                                                          \
        if (_e != hipSuccess) {                                                          \
            ::bgv::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),      \
                             __FILE__, __LINE__);                                        \
            return BGV_E_HIP;                                                            \
        }                                                                                \
    } while (0)

#define BGV_CHECK_LAUNCH() BGV_CHECK_HIP(hipGetLastError())

// Optional per-kernel event timing and counters (include/bgv_profile.h).
struct ProfPair {
    hipEvent_t start, stop;
    void *stat;
};
bool prof_on();
int prof_read_counter(const char *name, uint64_t *value);
void prof_reset_counters();
// True if this launch of `name` is to be timed; then *p holds the two events.
bool prof_take(const char *name, ProfPair *p);
void prof_commit(const ProfPair &p);

// Launch + error check.  A timed launch passes its events to the launch itself
// (hipExtLaunchKernelGGL), so they carry the kernel's own start and end times and no
// host-side gap before the dispatch.
#define BGV_LAUNCH(kernel, grid, block, shmem, stream, ...)                                              \
    do {                                                                                                 \
        ::bgv::ProfPair _bgv_p;                                                                          \
        const bool _bgv_t = ::bgv::prof_on() && ::bgv::prof_take(#kernel, &_bgv_p);                      \
        if (_bgv_t)                                                                                      \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, _bgv_p.start, _bgv_p.stop, 0u,     \
                                  __VA_ARGS__);                                                          \
        else                                                                                             \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                         \
        BGV_CHECK_LAUNCH();                                                                              \
        if (_bgv_t) ::bgv::prof_commit(_bgv_p);                                                          \
    } while (0)

#define BGV_TRY(expr)                                                                    \
    do {                                                                                 \
        bgv_status _s = (expr);                                                          \
        if (_s != BGV_OK) return _s;                                                     \
    } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Carves 256-byte-aligned sub-buffers out of a caller workspace.  With base == nullptr
// it only counts, so the same code computes the workspace size and the layout.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += align_up(sizeof(T) * (count ? count : 1));
        return p;
    }
    size_t size() const { return off; }
};

inline bgv_status check_ws(void *ws, size_t have, size_t need) {
    if (need == 0) return BGV_OK;
    if (ws == nullptr || have < need || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) {
        set_error("workspace: need %zu bytes, 256-byte aligned (got %zu at %p)", need, have, ws);
        return BGV_E_WORKSPACE;
    }
    return BGV_OK;
}

// Compute units of the current device, queried once per device, so that a launch
// sequence captured in a graph makes no query.
inline bgv_status device_cu_count(int *out) {
    static int cached[64] = {0};
    int dev = 0;
    BGV_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) dev = 0;
    if (cached[dev] == 0) {
        int c = 0;
        BGV_CHECK_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
        cached[dev] = c > 0 ? c : 1;
    }
    *out = cached[dev];
    return BGV_OK;
}

inline unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

// ------------------------------------------------------------- id range checks ----
// Opt-in device checks (BGV_CHECK=1 in the environment): a read-only scan of the ids
// raises a device flag (one int32 the caller's call is about to overwrite), read back
// on the host; BGV_E_RANGE when set.  They synchronise the stream.
bool range_check_on();
bgv_status check_edge_ids(int32_t n, int64_t m, const int32_t *edges, int32_t *flag, hipStream_t s);
bgv_status check_id_list(int64_t count, const int32_t *id, int32_t bound, int32_t *flag, hipStream_t s);
bgv_status check_batched_ids(int32_t G, int64_t n_total, int64_t m_total, const int64_t *node_off,
                             const int64_t *edge_off, const int32_t *edges, int32_t *flag, hipStream_t s);

// ---------------------------------------------------------------- primitives ----
// Device-wide fill (a kernel, so it is safe inside captured graphs).
template <class T>
bgv_status fill(T *p, T value, int64_t count, hipStream_t s);

// Exclusive prefix sum of `in[0..n)` into `out` (may alias `in`); writes the total
// to *total (device) if non-null.  Scratch from scan_workspace(n).
size_t scan_workspace(int64_t n);
bgv_status exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                              void *scratch, hipStream_t s);
template <class T>  // instantiated for uint32_t, uint64_t and double
bgv_status exclusive_scan(const T *in, T *out, int64_t n, T *total, void *scratch, hipStream_t s);

// Stable LSD radix sort of keys below 2^nbits, with an optional uint32 payload.
// keys/alt (and vals/vals_alt) are ping-pong buffers of n entries; the sorted result
// ends in *keys_out/*vals_out (one of the two).  Scratch from radix_workspace(n).  With
// n_dev the key count is read on the device (*n_dev <= n) and n is only its bound, so
// the sort can be queued before the count is known on the host.
size_t radix_workspace(int64_t n);
bgv_status radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                          int64_t n, int nbits, uint64_t **keys_out, uint32_t **vals_out,
                          void *scratch, hipStream_t s, bool counted = false,
                          const unsigned long long *n_dev = nullptr);
// The same for keys below 2^nbits <= 2^32 held in 32 bits (half the traffic per pass).
bgv_status radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                          int64_t n, int nbits, uint32_t **keys_out, uint32_t **vals_out,
                          void *scratch, hipStream_t s, bool counted = false,
                          const unsigned long long *n_dev = nullptr);

// Sorts of at most kRsFewTiles tiles (n > 1) count pass 0's digits in one launch ahead
// of the scatters.  A producer of the keys can do that count itself: for such an n,
// radix_few_tiles gives the tile shape (tiles of 256 * items consecutive keys) and
// radix_pass0_buffers where the counts go (counts0[digit * tiles + tile], the low 8
// bits of each key) and a [256 * tiles] buffer to clear; radix_sort_u64 with
// counted = true then skips its own count.
constexpr int kRsFewTiles = 64;
bool radix_few_tiles(int64_t n, int64_t *tiles, int *items);
void radix_pass0_buffers(void *scratch, int64_t n, uint32_t **counts0, uint32_t **clear1);

// One-sweep sort of 32-bit keys with 32-bit values (all 32 bits, four 8-bit passes, one
// launch per pass after a counting launch; see primitives.hip).  keys/alt and
// vals/vals_alt are ping-pong buffers of n entries; after the four passes the result is
// back in keys/vals.  Scratch from onesweep_workspace(n).  With counted = true a
// producer of the keys has already done what the counting launch would, for tiles of
// 256 * os_items(n) consecutive keys: added each tile's digit counts of all four passes
// into OsBuffers::totals[pass*256 + d] (which the caller had cleared before, in an
// earlier launch) and written zeros over OsBuffers::status (status_words words).
struct OsBuffers {
    int64_t tiles;
    int items;
    uint32_t *totals;  // kOsTotals words: keys per (pass, digit)
    uint32_t *status;
    int64_t status_words;
};
constexpr int kOsTotals = 4 * 256;
int os_items(int64_t n);
size_t onesweep_workspace(int64_t n);
void onesweep_layout(void *scratch, int64_t n, int items, OsBuffers *b);
bgv_status onesweep_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t n,
                             uint32_t **keys_out, uint32_t **vals_out, void *scratch, hipStream_t s, bool counted);

// One-sweep sort of keys alone (uint32_t or uint64_t; the low nbits significant,
// ceil(nbits / 8) <= sizeof(KT) passes; stable, so equal keys keep their order).
// keys/keys_alt are ping-pong buffers of n entries; the sorted keys end in *keys_out
// (one of the two).  With n_dev the key count is read on the device (*n_dev <= n) and
// n is only its bound, so the sort can be queued before the count is known on the
// host.  Scratch from onesweep_keys_workspace(n, nbits); n < 2^30.
// With counted = true a producer of the keys has done the counting launch's work: it
// wrote the digit counts of its blocks' keys (bcnt[block * passes * 256 + pass * 256 +
// d], passes = onesweep_key_passes(nbits)) and onesweep_keys_counted summed them into
// the scratch's totals and cleared its look-back words (wide: 64-bit keys).
size_t onesweep_keys_workspace(int64_t n, int nbits);
int onesweep_key_passes(int nbits);
bgv_status onesweep_keys_counted(const uint32_t *bcnt, int64_t nblocks, int64_t n, int nbits, bool wide,
                                 void *scratch, hipStream_t s);
template <class KT>
bgv_status onesweep_sort_keys(KT *keys, KT *keys_alt, int64_t n, const unsigned long long *n_dev, int nbits,
                              KT **keys_out, void *scratch, hipStream_t s, bool counted = false);

}  // namespace bgv
