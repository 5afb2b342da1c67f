// Shared between the ForceAtlas2 layout and the energy/gradient translation units.
#pragma once
#include "common.h"

namespace bgv {

// Directed CSR of an undirected edge list: row[K+1], col/wt[2E] (neighbours of node i
// in ascending (neighbour, edge index) order), mass[K] = row length + 1.
struct CsrWs {
    uint32_t *row;
    int32_t *col;
    float *wt;
    float *mass;
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
    void *sort_scratch;
};

size_t csr_layout(Carver &c, int32_t K, int64_t E, CsrWs *w);
// Builds the CSR; *mass_out = mass_in if given, else the degree-based masses.
bgv_status build_csr(int32_t K, int64_t E, const int32_t *edges, const float *attr_w, const float *mass_in,
                     CsrWs &w, hipStream_t s, const float **mass_out);

}  // namespace bgv
