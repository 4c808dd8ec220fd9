// Launchers of the DET-stage elimination kernel, one per (order N, lanes per matrix GL);
// the kernel is in det_impl.h and its instantiations are spread over det_part.hip builds.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "modarith.h"

namespace pd {

template <int N, int GL>
hipError_t det_launch(const uint32_t* eval, uint32_t* detv, int64_t npts, int pn,
                      const PrimeConst* pcs, hipStream_t st);

}  // namespace pd
