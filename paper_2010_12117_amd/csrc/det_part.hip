// One slice of the (order, lanes-per-matrix) instantiations of the elimination kernel,
// selected by DET_PART at compile time so that the slices build in parallel.
#include "det_impl.h"

#ifndef DET_PART
#error "DET_PART must be defined"
#endif

namespace pd {

#define PD_DET(N, GL)                                                                  \
  template hipError_t det_launch<N, GL>(const uint32_t*, uint32_t*, uint32_t*, int64_t,  \
                                        int, const PrimeConst*, hipStream_t);         \
  template hipError_t det_fused_launch<N, GL>(const FusedDetArgs&, hipStream_t);          \
  template hipError_t det_fused_batch_launch<N, GL>(const BDet*, int, int64_t, size_t,    \
                                                    uint8_t*, int, bool, hipStream_t);
#define PD_LL(N)                                                                       \
  template hipError_t det_ll_launch<N>(const FusedDetArgs&, hipStream_t);              \
  template hipError_t det_ll_batch_launch<N>(const BDet*, int, int64_t, size_t, uint8_t*, \
                                             hipStream_t);

#if DET_PART == 0
PD_DET(1, 1) PD_DET(2, 1) PD_DET(3, 1) PD_DET(4, 1) PD_DET(5, 1) PD_DET(6, 1)
PD_DET(7, 1) PD_DET(8, 1) PD_DET(9, 1) PD_DET(10, 1) PD_DET(11, 1) PD_DET(12, 1)
PD_LL(1) PD_LL(2) PD_LL(3) PD_LL(4) PD_LL(5) PD_LL(6)
PD_LL(7) PD_LL(8) PD_LL(9) PD_LL(10) PD_LL(11) PD_LL(12)
#elif DET_PART == 1
PD_LL(13) PD_LL(14) PD_LL(15) PD_LL(16)
PD_DET(2, 2) PD_DET(3, 2) PD_DET(4, 2) PD_DET(5, 2) PD_DET(6, 2) PD_DET(7, 2)
PD_DET(8, 2) PD_DET(9, 2) PD_DET(10, 2) PD_DET(11, 2) PD_DET(12, 2) PD_DET(13, 2)
PD_DET(14, 2) PD_DET(15, 2) PD_DET(16, 2)
#elif DET_PART == 2
PD_DET(4, 4) PD_DET(5, 4) PD_DET(6, 4) PD_DET(7, 4) PD_DET(8, 4) PD_DET(9, 4)
PD_DET(10, 4) PD_DET(11, 4) PD_DET(12, 4) PD_DET(13, 4) PD_DET(14, 4) PD_DET(15, 4)
PD_DET(16, 4)
#elif DET_PART == 3
PD_DET(17, 4) PD_DET(18, 4) PD_DET(19, 4) PD_DET(20, 4) PD_DET(21, 4) PD_DET(22, 4)
PD_DET(23, 4) PD_DET(24, 4)
#elif DET_PART == 4
PD_DET(8, 8) PD_DET(9, 8) PD_DET(10, 8) PD_DET(11, 8) PD_DET(12, 8) PD_DET(13, 8)
PD_DET(14, 8) PD_DET(15, 8) PD_DET(16, 8) PD_DET(17, 8) PD_DET(18, 8) PD_DET(19, 8)
PD_DET(20, 8) PD_DET(21, 8) PD_DET(22, 8)
#elif DET_PART == 5
PD_DET(23, 8) PD_DET(24, 8) PD_DET(25, 8) PD_DET(26, 8) PD_DET(27, 8) PD_DET(28, 8)
PD_DET(29, 8) PD_DET(30, 8) PD_DET(31, 8) PD_DET(32, 8)
#elif DET_PART == 6
PD_DET(16, 16) PD_DET(17, 16) PD_DET(18, 16) PD_DET(19, 16) PD_DET(20, 16) PD_DET(21, 16)
PD_DET(22, 16) PD_DET(23, 16) PD_DET(24, 16) PD_DET(25, 16) PD_DET(26, 16)
#elif DET_PART == 7
PD_DET(27, 16) PD_DET(28, 16) PD_DET(29, 16) PD_DET(30, 16) PD_DET(31, 16) PD_DET(32, 16)
#else
#error "unknown DET_PART"
#endif

}  // namespace pd
