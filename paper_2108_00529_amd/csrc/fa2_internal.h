// Shared between the ForceAtlas2 layout and the energy/gradient translation units.
#pragma once
#include "common.h"

namespace bgv {

// Directed CSR of an undirected edge list: row[K+1]; cw[2E] = node i's entries in
// ascending (neighbour, edge index) order, as (neighbour, weight bits) when weights are
// given and as bare neighbour ids (16-bit when K <= 65536) when they are all 1;
// mass[K] = row length + 1.
enum CsrFormat { kCsrWeighted = 0, kCsrIds32 = 1, kCsrIds16 = 2 };

struct CsrWs {
    uint32_t *row;
    int2 *cw;        // room for 2E int2 entries; holds the format below
    int fmt;         // kCsrWeighted: int2 (id, weight bits); kCsrIds32 / kCsrIds16: ids only (unit weights)
    float *mass;
    // attraction work items: row i's entries are cut into blocks of kAttBlock entries
    // (at least one block per row); item_of[i] = first item of row i (K+1 entries,
    // item_of[K] = number of items), item_row[t] = row of item t
    uint32_t *item_of, *item_row;
    int64_t items_bound;  // att_items_cap(K, E, cols)
    // With cols (chosen by csr_layout: above kAttLdsMax rows, for callers that run many
    // iterations on one CSR) items are cut by column block too (see
    // attraction).  Schedule order q: block by block, each block's items longest first,
    // in groups of 64 (one wavefront; group gi of block c at gfirst[c] + j holds the
    // block's items cstart[c] + 64 j ..).  it/ir/il[q] = item, row and length; cwb holds
    // each group's entries transposed from gbase[gi] (entry k of the group's lane l at
    // gbase[gi] + 64 k + l) as in-block offsets (uint16, or (offset, weight bits) when
    // weighted), in the sort keys' buffer, free once the CSR is built.
    bool cols;
    uint32_t *it, *ir;
    uint16_t *il;
    uint32_t *cstart, *gfirst, *gbase;
    uint32_t *wg_first;  // block c's workgroups: [wg_first[c], wg_first[c + 1])
    void *cwb;
    // setup scratch
    uint32_t *item_beg;  // first entry of each item, items + 1 entries
    uint32_t *ikeys, *ikeys_alt, *ivals, *ivals_alt, *ilen;
    unsigned long long *nitems;
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
    void *sort_scratch;
};

// Upper bound on the number of attraction work items (block sums) of K rows holding 2E
// entries.
int64_t att_items_cap(int32_t K, int64_t E, bool cols);
// Rows above which the attraction's positions no longer fit in LDS and its items are
// cut by column block as well.
constexpr int32_t kAttLdsMax = 19456;  // 152 KiB of float2
inline bool att_cols(int32_t K) { return K > kAttLdsMax; }
// allow_cols: the column-blocked items may be used (their setup costs about as much as
// a few iterations, so callers that evaluate the attraction once pass false).
size_t csr_layout(Carver &c, int32_t K, int64_t E, CsrWs *w, bool allow_cols);
// A[t] = attraction block sum of work item t (att_items_cap(K, E) entries), one
// wavefront per item; node i's attraction is fa2_att_combine(A, csr.item_of, i).
bgv_status attraction(int32_t K, const float2 *pos, const CsrWs &csr, float2 *A, hipStream_t s);
// Builds the CSR; *mass_out = mass_in if given, else the degree-based masses.
bgv_status build_csr(int32_t K, int64_t E, const int32_t *edges, const float *attr_w, const float *mass_in,
                     CsrWs &w, hipStream_t s, const float **mass_out);

// bgv_fa2_layout; may_fork lets the call run part of each iteration on a second stream
// of the device (created once, on first use outside graph capture); results do not
// depend on it.
bgv_status fa2_layout_run(int32_t K, int64_t E, const int32_t *edges, const float *attr_w, const float *mass,
                          float *pos, float *fprev, float *speed, const bgv_fa2_params *p, void *ws, size_t ws_bytes,
                          bgv_stream_t stream, bool may_fork);

}  // namespace bgv
