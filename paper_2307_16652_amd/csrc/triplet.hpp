// triplet.hpp -- the triplet (symmetry) variant of PaLD.  Not implemented yet:
// requests for it are rejected with PALD_ERR_UNSUPPORTED.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pald.h"

namespace pald {

inline size_t triplet_workspace_bytes(int64_t) { return 0; }

inline pald_status triplet_cohesion(const float *, int64_t, int64_t, int32_t *, int64_t, float *, int64_t, void *,
                                    size_t, hipStream_t, bool, bool) {
    return PALD_ERR_UNSUPPORTED;
}

}  // namespace pald
