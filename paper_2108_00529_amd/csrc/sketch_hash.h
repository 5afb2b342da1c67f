// Count-min sketch row hashes (Section 3.3: one pairwise-independent hash per row).
// Multiply-add-shift to 32 bits (Dietzfelbinger), then Lemire's multiply-high range
// reduction to [0, cols); arithmetic mod 2^64.  The coefficients are inputs.
#pragma once
#include "common.h"

namespace bgv {

constexpr int kMaxRows = 8;

struct HashRows {
    uint64_t a[kMaxRows], b[kMaxRows], c[kMaxRows];
};

// Column of a 32-bit key x in the row with coefficients (A, B).
__device__ __forceinline__ uint32_t col_key(uint64_t A, uint64_t B, uint32_t x, uint32_t cols) {
    const uint64_t t = A * (uint64_t)x + B;
    return (uint32_t)(((t >> 32) * (uint64_t)cols) >> 32);
}

// Column of an unordered pair key (lo < hi) in the row with coefficients (A, B, C).
__device__ __forceinline__ uint32_t col_pair(uint64_t A, uint64_t B, uint64_t C, uint32_t lo, uint32_t hi,
                                             uint32_t cols) {
    const uint64_t t = A * (uint64_t)lo + C * (uint64_t)hi + B;
    return (uint32_t)(((t >> 32) * (uint64_t)cols) >> 32);
}

inline HashRows make_hash_rows(const uint64_t *coef, int rows) {
    HashRows h{};
    for (int r = 0; r < rows && r < kMaxRows; ++r) {
        h.a[r] = coef[3 * r];
        h.b[r] = coef[3 * r + 1];
        h.c[r] = coef[3 * r + 2];
    }
    return h;
}

}  // namespace bgv
