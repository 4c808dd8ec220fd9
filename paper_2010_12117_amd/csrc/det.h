// Launchers of the DET-stage elimination kernel, one per (order N, lanes per matrix GL);
// the kernel is in det_impl.h and its instantiations are spread over det_part.hip builds.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "modarith.h"

namespace pd {

// Arguments of the fused evaluation + elimination launch (det_impl.h, det_fused_kernel).
struct FusedDetArgs {
  const uint32_t* pre;   // [pn][nslot][m0][R]
  uint32_t* detv;        // [pn][N0 * R] numerators of the determinants
  uint32_t* denv;        // [pn][N0 * R] denominators
  int64_t R;             // grid points of the other variables
  int N0, m0;            // grid size and coefficient count of the first variable
  int Q, S;              // points per LDS tile, first-variable values per block
  const uint32_t* tw0;   // w_0^t (Montgomery), t < N0, at prime * tw_stride
  int64_t tw_stride;
  const PrimeConst* pcs;
  const uint8_t* zero;   // [n*n] zero-entry flags or null
  const int32_t* slot;   // [n*n] pre-tensor slot of each entry (elimination order)
  int64_t nslot;         // slots per prime in the pre-tensor
  int pn;
  bool fixup;            // repair launch: recompute only the points with den = 0
  // A slab of the grid (capped plans): the R points of the pre-tensor are the local points
  // r < seg at global r + off1 and r >= seg at global r + off2, of Rout per first-variable
  // value in detv / denv. The whole grid: Rout = seg = R, off1 = off2 = 0.
  int64_t Rout, seg, off1, off2;
};

template <int N, int GL>
hipError_t det_fused_launch(const FusedDetArgs& f, hipStream_t st);

// Left-looking form, one lane per matrix (det_impl.h, det_ll_kernel); points with a zero
// pivot are left with den = 0 for a repair launch of det_fused_launch with fixup = true.
template <int N>
hipError_t det_ll_launch(const FusedDetArgs& f, hipStream_t st);

template <int N, int GL>
hipError_t det_launch(const uint32_t* eval, uint32_t* detv, uint32_t* denv, int64_t npts, int pn,
                      const PrimeConst* pcs, hipStream_t st);

}  // namespace pd
