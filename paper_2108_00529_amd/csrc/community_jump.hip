// Streaming community detection without a barrier per chunk (the rule of Section 3.2,
// the passes of Section 3.2.1 / Algorithm 3, batch-synchronous as in community.hip:
// the same integers for every chunk size, chunk = 1 being the sequential rule).
//
// Under the degree rule an edge's decision in a pass (whether it proposes, and which
// endpoint is the target) depends only on counters, and those follow in closed form
// from the stream: in pass p at the end of chunk k the counter of x is p d(x) + c(x, k),
// with c(x, k) the occurrences of x as an endpoint of a non-loop edge in chunks 0..k.
// Labels enter only as the value a proposal carries (its source's label when the chunk
// began).  So every pass's proposals are known up front; a target's winner in a chunk
// is its proposal of smallest stream index; and the label a winner carries is the one
// its source got from its own latest winner in an earlier chunk (the source's id if it
// had none).  Those links point strictly back in time, and pointer jumping over them
// labels every winner in O(log chunks) bulk steps:
//   1. endpoint occurrences sorted by node (stable): d(x) = run length, c(x, k) of each
//      occurrence by a binary search in its node's run;
//   2. the proposals of every (pass, edge), compacted in stream order, sorted stably
//      by (target, global chunk): the first of each run is the winner;
//   3. winners compacted; each one's link = the last winner into its source with an
//      earlier chunk (a binary search in the source's run of winners);
//   4. pointer jumping along the links, in place on packed (link, label) words, each
//      round skipped once a round has left nothing unresolved; a node's label = its
//      last winner's label.
// About 20 launches whatever the number of chunks, against two per chunk and pass for
// the chunk-by-chunk form: the choice for small chunks.
#include <algorithm>

#include "common.h"
#include "community_jump.h"

namespace bgv {

constexpr int kSqThreads = 256;
constexpr int kSqMaxRounds = 66;  // ceil(log2 chunks) + 1 <= 34 for 32-bit proposal indices

static int bits_for(uint64_t x) {  // bits needed to hold values 0..x
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

// D1 * growth^p, saturating at INT32_MAX (at most ~31 products before it saturates).
__host__ __device__ inline int32_t sq_threshold(int32_t D1, int32_t growth, int32_t p) {
    if (growth == 1 || D1 == 0) return D1;
    int64_t D = D1;
    for (int32_t k = 0; k < p; ++k) {
        D *= growth;
        if (D > INT32_MAX) return INT32_MAX;
    }
    return (int32_t)D;
}

bool sq_fits(int32_t n, int64_t m, const bgv_cd_params *p) {
    if (m < 1) return false;
    const int64_t nchunk = (m + p->chunk - 1) / p->chunk;
    if ((int64_t)p->passes * m > INT32_MAX) return false;  // proposals indexed in 32 bits
    const uint64_t G = (uint64_t)p->passes * (uint64_t)nchunk;
    return bits_for((uint64_t)(n - 1)) + bits_for(G - 1) <= 64;
}

struct SqWs {
    uint32_t *okey, *okey_alt, *oval, *oval_alt;  // endpoint occurrences [2m]
    uint32_t *beg, *end;                          // run of each node in the sorted occurrences [n]
    int4 *cd;                                     // per edge {c(e.x), d(e.x), c(e.y), d(e.y)}
    uint32_t *flag;                               // [P m]: proposals, then winners
    void *evk, *evk_alt;                          // proposal keys (target, chunk) [P m], 32 or 64 bits
    uint32_t *evv, *evv_alt;                      // their edge indices
    void *wk;                                     // winners' keys [P m]
    uint32_t *wv;                                 // winners' edge indices
    unsigned long long *jv;                       // per winner: label << 32 | link (link ~0: resolved) [P m]
    int32_t *go;                                  // [kSqMaxRounds + 1]: round r runs if go[r]
    uint32_t *tot;                                // [4]: proposals, winners
    unsigned long long *tot64;                    // proposals, as the sort's device count
    void *sort_scratch, *scan_scratch;
};

static bool sq_wide(int32_t n, int64_t m, const bgv_cd_params *p) {
    const int64_t nchunk = (m + p->chunk - 1) / p->chunk;
    return bits_for((uint64_t)(n - 1)) + bits_for((uint64_t)p->passes * (uint64_t)nchunk - 1) > 32;
}

size_t sq_layout(Carver &c, int32_t n, int64_t m, const bgv_cd_params *p, void *out) {
    SqWs w{};
    const size_t no = 2 * (size_t)m, pm = (size_t)p->passes * (size_t)m;
    const size_t kw = sq_wide(n, m, p) ? sizeof(uint64_t) : sizeof(uint32_t);
    w.okey = c.take<uint32_t>(no);
    w.okey_alt = c.take<uint32_t>(no);
    w.oval = c.take<uint32_t>(no);
    w.oval_alt = c.take<uint32_t>(no);
    w.beg = c.take<uint32_t>((size_t)n);
    w.end = c.take<uint32_t>((size_t)n);
    w.cd = c.take<int4>((size_t)m);
    w.flag = c.take<uint32_t>(pm);
    w.evk = c.take<char>(pm * kw);
    w.evk_alt = c.take<char>(pm * kw);
    w.evv = c.take<uint32_t>(pm);
    w.evv_alt = c.take<uint32_t>(pm);
    w.wk = c.take<char>(pm * kw);
    w.wv = c.take<uint32_t>(pm);
    w.jv = c.take<unsigned long long>(pm);
    w.go = c.take<int32_t>(kSqMaxRounds + 1);
    w.tot = c.take<uint32_t>(4);
    w.tot64 = c.take<unsigned long long>(2);
    w.sort_scratch = c.take<char>(radix_workspace((int64_t)std::max(no, pm)));
    w.scan_scratch = c.take<char>(scan_workspace((int64_t)pm));
    if (out) *static_cast<SqWs *>(out) = w;
    return c.size();
}

// ------------------------------------------------------------------ kernels ----
#define SQ_LOOP(i, count) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (count); i += (int64_t)gridDim.x * blockDim.x)

// Occurrence 2i + s is endpoint s of edge i, keyed by its node (self-loops by n, past
// every node: they raise no counter).
__global__ void __launch_bounds__(kSqThreads) k_sq_occ(const int2 *__restrict__ edges, int64_t m, int32_t n,
                                                       uint32_t *__restrict__ okey, uint32_t *__restrict__ oval) {
    SQ_LOOP(i, m) {
        const int2 e = edges[i];
        const bool loop = e.x == e.y;
        okey[2 * i] = loop ? (uint32_t)n : (uint32_t)e.x;
        okey[2 * i + 1] = loop ? (uint32_t)n : (uint32_t)e.y;
        oval[2 * i] = (uint32_t)(2 * i);
        oval[2 * i + 1] = (uint32_t)(2 * i + 1);
    }
}

__global__ void __launch_bounds__(kSqThreads) k_sq_runs(const uint32_t *__restrict__ sk, int64_t no, int32_t n,
                                                        uint32_t *__restrict__ beg, uint32_t *__restrict__ end) {
    SQ_LOOP(j, no) {
        const uint32_t x = sk[j];
        if (x >= (uint32_t)n) continue;
        if (j == 0 || sk[j - 1] != x) beg[x] = (uint32_t)j;
        if (j + 1 == no || sk[j + 1] != x) end[x] = (uint32_t)(j + 1);
    }
}

// c(x, k) of each occurrence: the occurrences of x before the end of its chunk, i.e.
// the first place in x's run (occurrences in stream order) at or past that end.
__global__ void __launch_bounds__(kSqThreads) k_sq_counts(const uint32_t *__restrict__ sk,
                                                          const uint32_t *__restrict__ sv, int64_t no, int32_t n,
                                                          const uint32_t *__restrict__ beg,
                                                          const uint32_t *__restrict__ end, int64_t m, int64_t B,
                                                          int4 *__restrict__ cd) {
    SQ_LOOP(j, no) {
        const uint32_t x = sk[j];
        if (x >= (uint32_t)n) continue;
        const uint32_t o = sv[j];
        const int64_t i = o >> 1;
        const int64_t ce = std::min<int64_t>((i / B + 1) * B, m);
        const uint64_t lim = 2 * (uint64_t)ce;
        // gallop from j (the chunk's run of x is usually short), then bisect
        const uint32_t e = end[x];
        uint32_t lo = (uint32_t)j + 1, hi = e;
        uint64_t step = 1;
        while (true) {
            const uint64_t probe = (uint64_t)j + step;
            if (probe >= e || (uint64_t)sv[probe] >= lim) {
                hi = probe < e ? (uint32_t)probe : e;
                break;
            }
            lo = (uint32_t)probe + 1;
            step <<= 1;
        }
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if ((uint64_t)sv[mid] < lim) lo = mid + 1;
            else hi = mid;
        }
        // one 8-byte store per occurrence: {c, d} of this endpoint
        reinterpret_cast<int2 *>(cd + i)[o & 1u] = make_int2((int32_t)(lo - beg[x]), (int32_t)(e - beg[x]));
    }
}

// Target of edge e in pass p (threshold D), or -1: both counters at most D and unequal,
// the endpoint with the smaller one is the target; equal ones with tie rule 1: e.x.
__device__ __forceinline__ int32_t sq_target(int2 e, int4 c, int32_t p, int32_t D, int32_t tie) {
    if (e.x == e.y) return -1;
    const int32_t cu = p * c.y + c.x, cv = p * c.w + c.z;
    if (cu <= D && cv <= D && (cu != cv || tie)) return cu <= cv ? e.x : e.y;
    return -1;
}

// flag[p m + i] = edge i proposes in pass p (passes before `first` propose nothing)
__global__ void __launch_bounds__(kSqThreads) k_sq_flags(const int2 *__restrict__ edges, const int4 *__restrict__ cd,
                                                         int64_t m, int32_t P, int32_t D1, int32_t growth,
                                                         int32_t tie, int32_t first, uint32_t *__restrict__ flag) {
    SQ_LOOP(t, (int64_t)P * m) {
        const int32_t p = (int32_t)(t / m);
        const int64_t i = t - (int64_t)p * m;
        flag[t] = p >= first && sq_target(edges[i], cd[i], p, sq_threshold(D1, growth, p), tie) >= 0 ? 1u : 0u;
    }
}

// Proposal (p, i) at its place pos[p m + i]: key (target, global chunk), value i.
template <class KT>
__global__ void __launch_bounds__(kSqThreads) k_sq_emit(const int2 *__restrict__ edges, const int4 *__restrict__ cd,
                                                        int64_t m, int32_t P, int32_t D1, int32_t growth,
                                                        int32_t tie, int32_t first, int64_t B,
                                                        int64_t nchunk, int gbits, const uint32_t *__restrict__ pos,
                                                        KT *__restrict__ key, uint32_t *__restrict__ val) {
    SQ_LOOP(t, (int64_t)P * m) {
        const int32_t p = (int32_t)(t / m);
        const int64_t i = t - (int64_t)p * m;
        if (p < first) continue;
        const int32_t v = sq_target(edges[i], cd[i], p, sq_threshold(D1, growth, p), tie);
        if (v < 0) continue;
        const uint64_t g = (uint64_t)p * (uint64_t)nchunk + (uint64_t)(i / B);
        const uint32_t q = pos[t];
        key[q] = (KT)(((uint64_t)v << gbits) | g);
        val[q] = (uint32_t)i;
    }
}

__global__ void __launch_bounds__(kSqThreads) k_sq_widen(const uint32_t *__restrict__ a, unsigned long long *b) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *b = *a;
}

// flag[q] = sorted proposal q is the first of its (target, chunk) run
template <class KT>
__global__ void __launch_bounds__(kSqThreads) k_sq_first(const KT *__restrict__ sk, int64_t bound,
                                                         const uint32_t *__restrict__ count,
                                                         uint32_t *__restrict__ flag) {
    const int64_t E = *count;
    SQ_LOOP(q, bound) flag[q] = (q < E && (q == 0 || sk[q - 1] != sk[q])) ? 1u : 0u;
}

template <class KT>
__global__ void __launch_bounds__(kSqThreads) k_sq_compact(const KT *__restrict__ sk, const uint32_t *__restrict__ sv,
                                                           const uint32_t *__restrict__ count,
                                                           const uint32_t *__restrict__ pos, KT *__restrict__ wk,
                                                           uint32_t *__restrict__ wv) {
    const int64_t E = *count;
    SQ_LOOP(q, E) {
        if (q == 0 || sk[q - 1] != sk[q]) {
            wk[pos[q]] = sk[q];
            wv[pos[q]] = sv[q];
        }
    }
}

// The run of each node in the sorted winners (beg/end cleared before).
template <class KT>
__global__ void __launch_bounds__(kSqThreads) k_sq_wruns(const KT *__restrict__ wk,
                                                         const uint32_t *__restrict__ wcount, int gbits,
                                                         uint32_t *__restrict__ beg, uint32_t *__restrict__ end) {
    const int64_t W = *wcount;
    SQ_LOOP(r, W) {
        const uint32_t v = (uint32_t)((uint64_t)wk[r] >> gbits);
        if (r == 0 || (uint32_t)((uint64_t)wk[r - 1] >> gbits) != v) beg[v] = (uint32_t)r;
        if (r + 1 == W || (uint32_t)((uint64_t)wk[r + 1] >> gbits) != v) end[v] = (uint32_t)(r + 1);
    }
}

// Winner r's link: the last winner into its source with an earlier chunk, or none
// (~0); packed with the label it carries when it has no link: the source's starting
// label (its id, or lab0 of a resumed run).
template <class KT>
__global__ void __launch_bounds__(kSqThreads) k_sq_links(const int2 *__restrict__ edges, const KT *__restrict__ wk,
                                                         const uint32_t *__restrict__ wv,
                                                         const uint32_t *__restrict__ wcount, int gbits,
                                                         const uint32_t *__restrict__ beg,
                                                         const uint32_t *__restrict__ end,
                                                         const int32_t *__restrict__ lab0,
                                                         unsigned long long *__restrict__ jv) {
    const int64_t W = *wcount;
    SQ_LOOP(r, W) {
        const uint64_t key = (uint64_t)wk[r];
        const uint64_t gmask = gbits >= 64 ? ~0ull : ((1ull << gbits) - 1ull);
        const int32_t v = (int32_t)(key >> gbits);
        const int2 e = edges[wv[r]];
        const int32_t u = e.x == v ? e.y : e.x;
        const uint64_t want = ((uint64_t)u << gbits) | (key & gmask);
        const uint32_t b0 = beg[u];
        uint32_t lo = b0, hi = end[u];  // u's winners (empty: beg = end = 0); first key >= want
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if ((uint64_t)wk[mid] < want) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t link = lo > b0 ? lo - 1 : 0xffffffffu;
        const int32_t l0 = lab0 ? lab0[u] : u;
        jv[r] = ((unsigned long long)(uint32_t)l0 << 32) | link;
    }
}

// One pointer-jumping round, in place: a winner whose link is resolved takes its
// label; any other skips to its link's link.  Each 8-byte word is read and written by
// one instruction, so a concurrent reader sees a link and label that belong together
// (older or newer, both true of the chain: its label is that of its link's), and the
// final label is copied only from a resolved word; every word read is at least as new
// as the round's start, so each round at least halves every remaining chain.  The
// round does nothing if the previous one left nothing unresolved (*go_in == 0), and
// sets *go_out when it did not resolve everything.
__global__ void __launch_bounds__(kSqThreads) k_sq_jump(unsigned long long *jv, const uint32_t *__restrict__ wcount,
                                                        const int32_t *go_in, int32_t *go_out) {
    if (*go_in == 0) return;  // the same value for every thread of the grid
    const int64_t W = *wcount;
    bool more = false;
    SQ_LOOP(r, W) {
        const unsigned long long w0 = __hip_atomic_load(&jv[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t a = (uint32_t)w0;
        if (a == 0xffffffffu) continue;
        const unsigned long long wa = __hip_atomic_load(&jv[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t b = (uint32_t)wa;
        const unsigned long long nw = b == 0xffffffffu ? wa : ((w0 & 0xffffffff00000000ull) | b);
        more |= b != 0xffffffffu;
        __hip_atomic_store(&jv[r], nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (__syncthreads_or(more) && threadIdx.x == 0) *go_out = 1;
}

__global__ void __launch_bounds__(kSqThreads) k_sq_init(int32_t n, int32_t rows, int32_t *__restrict__ labels,
                                                        int32_t *__restrict__ pass_labels,
                                                        const uint32_t *__restrict__ beg,
                                                        const uint32_t *__restrict__ end,
                                                        const int32_t *__restrict__ lab0,
                                                        int32_t *__restrict__ degree) {
    SQ_LOOP(v, n) {
        labels[v] = lab0 ? lab0[v] : (int32_t)v;
        degree[v] = (int32_t)(end[v] - beg[v]);
        for (int32_t p = 0; p < rows; ++p) pass_labels[(int64_t)p * n + v] = (int32_t)v;
    }
}

// A node's label after pass p: the label of its last winner in a chunk of passes 0..p.
template <class KT>
__global__ void __launch_bounds__(kSqThreads) k_sq_labels(const KT *__restrict__ wk,
                                                          const uint32_t *__restrict__ wcount, int gbits,
                                                          int64_t nchunk, int32_t P,
                                                          const unsigned long long *__restrict__ jv,
                                                          int32_t n, int32_t *__restrict__ labels,
                                                          int32_t *__restrict__ pass_labels) {
    const int64_t W = *wcount;
    SQ_LOOP(r, W) {
        const uint64_t key = (uint64_t)wk[r];
        const uint64_t gmask = gbits >= 64 ? ~0ull : ((1ull << gbits) - 1ull);
        const int32_t v = (int32_t)(key >> gbits);
        const bool more = r + 1 < W && (int32_t)((uint64_t)wk[r + 1] >> gbits) == v;
        const int32_t lab = (int32_t)(jv[r] >> 32);
        if (!more) labels[v] = lab;
        if (pass_labels) {
            const int32_t p0 = (int32_t)((key & gmask) / (uint64_t)nchunk);
            const int32_t p1 = more ? (int32_t)(((uint64_t)wk[r + 1] & gmask) / (uint64_t)nchunk) : P;
            for (int32_t p = p0; p < p1; ++p) pass_labels[(int64_t)p * n + v] = lab;
        }
    }
}

__global__ void __launch_bounds__(kSqThreads) k_sq_volume(const int32_t *__restrict__ labels,
                                                          const int32_t *__restrict__ degree, int32_t n,
                                                          unsigned long long *__restrict__ volume) {
    SQ_LOOP(v, n) {
        const int32_t d = degree[v];
        if (d) atomicAdd(&volume[labels[v]], (unsigned long long)d);
    }
}

// ------------------------------------------------------------------- driver ----
template <class KT>
static bgv_status sq_sort_events(SqWs &w, int64_t pm, int nbits, KT **sk, uint32_t **sv, hipStream_t s);

template <>
bgv_status sq_sort_events<uint32_t>(SqWs &w, int64_t pm, int nbits, uint32_t **sk, uint32_t **sv, hipStream_t s) {
    return radix_sort_u32(static_cast<uint32_t *>(w.evk), static_cast<uint32_t *>(w.evk_alt), w.evv, w.evv_alt, pm,
                          nbits, sk, sv, w.sort_scratch, s, false, w.tot64);
}

template <>
bgv_status sq_sort_events<uint64_t>(SqWs &w, int64_t pm, int nbits, uint64_t **sk, uint32_t **sv, hipStream_t s) {
    return radix_sort_u64(static_cast<uint64_t *>(w.evk), static_cast<uint64_t *>(w.evk_alt), w.evv, w.evv_alt, pm,
                          nbits, sk, sv, w.sort_scratch, s, false, w.tot64);
}

template <class KT>
static bgv_status sq_events(const int2 *e2, int32_t n, int64_t m, const bgv_cd_params *p, SqWs &w, int32_t *labels,
                            int32_t *pass_labels, int32_t first, const int32_t *lab0, hipStream_t s) {
    const int32_t P = p->passes;
    const int64_t B = p->chunk, nchunk = (m + B - 1) / B, pm = (int64_t)P * m;
    const int gbits = bits_for((uint64_t)P * (uint64_t)nchunk - 1);
    const int nbits = std::max(1, bits_for((uint64_t)(n - 1)) + gbits);
    const unsigned grid = grid_for(pm, kSqThreads, 65536);
    // proposals of every pass, in (pass, stream) order
    BGV_LAUNCH(k_sq_flags, dim3(grid), dim3(kSqThreads), 0, s, e2, w.cd, m, P, p->threshold, p->growth, p->tie,
               first, w.flag);
    BGV_TRY(exclusive_scan_u32(w.flag, w.flag, pm, w.tot, w.scan_scratch, s));
    BGV_LAUNCH(k_sq_emit<KT>, dim3(grid), dim3(kSqThreads), 0, s, e2, w.cd, m, P, p->threshold, p->growth, p->tie,
               first, B, nchunk,
               gbits, w.flag, static_cast<KT *>(w.evk), w.evv);
    BGV_LAUNCH(k_sq_widen, dim3(1), dim3(kSqThreads), 0, s, w.tot, w.tot64);
    KT *sk = nullptr;
    uint32_t *sv = nullptr;
    BGV_TRY(sq_sort_events<KT>(w, pm, nbits, &sk, &sv, s));
    // winners: first of each (target, chunk) run
    BGV_LAUNCH(k_sq_first<KT>, dim3(grid), dim3(kSqThreads), 0, s, sk, pm, w.tot, w.flag);
    BGV_TRY(exclusive_scan_u32(w.flag, w.flag, pm, w.tot + 1, w.scan_scratch, s));
    KT *wk = static_cast<KT *>(w.wk);
    BGV_LAUNCH(k_sq_compact<KT>, dim3(grid), dim3(kSqThreads), 0, s, sk, sv, w.tot, w.flag, wk, w.wv);
    // each winner's link: a search in its source's run of winners (the occurrence runs'
    // arrays, free by now, hold the winner runs)
    BGV_TRY(fill<uint32_t>(w.beg, 0u, n, s));
    BGV_TRY(fill<uint32_t>(w.end, 0u, n, s));
    BGV_LAUNCH(k_sq_wruns<KT>, dim3(grid), dim3(kSqThreads), 0, s, wk, w.tot + 1, gbits, w.beg, w.end);
    BGV_LAUNCH(k_sq_links<KT>, dim3(grid), dim3(kSqThreads), 0, s, e2, wk, w.wv, w.tot + 1, gbits, w.beg, w.end,
               lab0, w.jv);
    // a chain of links visits at most one winner per chunk: ceil(log2 chunks) + 1 rounds
    const int rounds = bits_for((uint64_t)P * (uint64_t)nchunk) + 1;
    BGV_TRY(fill<int32_t>(w.go, 0, rounds + 1, s));
    BGV_TRY(fill<int32_t>(w.go, 1, 1, s));
    for (int r = 0; r < rounds; ++r)
        BGV_LAUNCH(k_sq_jump, dim3(grid), dim3(kSqThreads), 0, s, w.jv, w.tot + 1, w.go + r, w.go + r + 1);
    BGV_LAUNCH(k_sq_labels<KT>, dim3(grid), dim3(kSqThreads), 0, s, wk, w.tot + 1, gbits, nchunk, P, w.jv, n, labels,
               pass_labels);
    return BGV_OK;
}

bgv_status sq_run(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p, int32_t *labels,
                  int32_t *degree, int64_t *volume, int32_t *pass_labels, int32_t first, const int32_t *lab0,
                  void *ws, hipStream_t s) {
    Carver c(ws);
    SqWs w;
    sq_layout(c, n, m, p, &w);
    const int2 *e2 = reinterpret_cast<const int2 *>(edges);
    const int64_t no = 2 * m;
    const unsigned go = grid_for(no, kSqThreads, 65536), gn = grid_for(n, kSqThreads, 65536);
    BGV_LAUNCH(k_sq_occ, dim3(grid_for(m, kSqThreads, 65536)), dim3(kSqThreads), 0, s, e2, m, n, w.okey, w.oval);
    uint32_t *sk = nullptr, *sv = nullptr;
    BGV_TRY(radix_sort_u32(w.okey, w.okey_alt, w.oval, w.oval_alt, no, bits_for((uint64_t)n), &sk, &sv,
                           w.sort_scratch, s));
    BGV_TRY(fill<uint32_t>(w.beg, 0u, n, s));
    BGV_TRY(fill<uint32_t>(w.end, 0u, n, s));
    BGV_LAUNCH(k_sq_runs, dim3(go), dim3(kSqThreads), 0, s, sk, no, n, w.beg, w.end);
    BGV_LAUNCH(k_sq_counts, dim3(go), dim3(kSqThreads), 0, s, sk, sv, no, n, w.beg, w.end, m, p->chunk, w.cd);
    BGV_LAUNCH(k_sq_init, dim3(gn), dim3(kSqThreads), 0, s, n, pass_labels ? p->passes : 0, labels, pass_labels,
               w.beg, w.end, lab0, degree);
    if (sq_wide(n, m, p))
        BGV_TRY(sq_events<uint64_t>(e2, n, m, p, w, labels, pass_labels, first, lab0, s));
    else
        BGV_TRY(sq_events<uint32_t>(e2, n, m, p, w, labels, pass_labels, first, lab0, s));
    if (volume)
        BGV_LAUNCH(k_sq_volume, dim3(gn), dim3(kSqThreads), 0, s, labels, degree, n,
                   reinterpret_cast<unsigned long long *>(volume));
    return BGV_OK;
}

}  // namespace bgv
