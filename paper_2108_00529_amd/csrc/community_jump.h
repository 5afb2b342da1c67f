// Community detection by back-pointer resolution (community_jump.hip): the same
// integers as the chunk-by-chunk form, in a fixed number of bulk launches.
#pragma once
#include "common.h"

namespace bgv {

// Whether the form applies: m >= 1 and passes * m < 2^31 (proposals indexed in 32 bits).
bool sq_fits(int32_t n, int64_t m, const bgv_cd_params *p);
// Workspace layout (out: the internal layout, or nullptr); returns the bytes used.
size_t sq_layout(Carver &c, int32_t n, int64_t m, const bgv_cd_params *p, void *out);
// The passes; arguments as bgv_community_passes (pass_labels may be null).  volume, if
// given, must be zero-filled.  A run resumed after `first` passes (first >= 1, then
// pass_labels null) starts from labels lab0 and forms the proposals of passes first..
// only; first = 0 and lab0 null for a run from the start.
bgv_status sq_run(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p, int32_t *labels,
                  int32_t *degree, int64_t *volume, int32_t *pass_labels, int32_t first, const int32_t *lab0,
                  void *ws, hipStream_t s);

}  // namespace bgv
