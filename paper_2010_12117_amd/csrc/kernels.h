// Stage launchers of one solve (all asynchronous on the given stream). The workspace
// layout and the device tables come from the plan (plan.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include "plan.h"

namespace pd {

constexpr int kTileElems = 8192;  // interpolation tile: at most 32 KB of LDS per block (plus
                                  // the line's twiddles)
constexpr int kFuseBatch = 8;     // denominators a thread of the first interpolation pass
                                  // inverts together (one exponentiation)
constexpr int kInttRegLines = 32; // lines per block of the register-form 64-point pass

// Whether an elimination kernel is compiled for this order and lanes-per-matrix.
bool det_config_supported(int n, int lanes);

// Launch shapes shared by the single and the batched paths.
int expand_outputs_per_thread(int Nv, int64_t inner, int m);
int intt_lines_per_block(int64_t lines, int Nv, int pn);
// Whether an interpolation pass of Nv points per line, inner points apart, takes the register
// form (32, 64, 128 or 256 points along an axis of at least kInttRegLines contiguous lines).
bool intt_register_pass(int Nv, int64_t inner);
int64_t finalize_threads(int64_t G, int pn);  // threads of the det = num / den launch

hipError_t run_reduce(const MatPlan& P, const int64_t* coeffs, uint8_t* ws, hipStream_t st);
hipError_t run_evaluate(const MatPlan& P, uint8_t* ws, hipStream_t st);
// S1 and S2 together: the first evaluation pass reduces the integer coefficients as it loads
// them (and stores the residues as S1 does), one launch fewer (run_reduce then run_evaluate
// where there is no evaluation pass).
hipError_t run_reduce_evaluate(const MatPlan& P, const int64_t* coeffs, uint8_t* ws,
                               hipStream_t st);
hipError_t run_det(const MatPlan& P, uint8_t* ws, hipStream_t st);       // numerators, denominators
// Grid slabs (MatPlan::slabs > 1, fused plans with two or more variables): the passes over
// variables k-1 .. 2 once, then for each slab b the pass over variable 1 for its points and
// their determinants.
hipError_t run_evaluate_upper(const MatPlan& P, uint8_t* ws, hipStream_t st);
hipError_t run_evaluate_slab(const MatPlan& P, uint8_t* ws, int slab, hipStream_t st);
hipError_t run_det_slab(const MatPlan& P, uint8_t* ws, int slab, hipStream_t st);
// det = num / den: a launch of its own only without variables; otherwise run_interpolate's
// first pass divides as it loads
hipError_t run_finalize(const MatPlan& P, uint8_t* ws, hipStream_t st);
hipError_t run_interpolate(const MatPlan& P, uint8_t* ws, hipStream_t st);
hipError_t run_reconstruct(const MatPlan& P, uint8_t* ws, uint32_t* out, hipStream_t st);
// S4 and S5 together: the last interpolation pass also reconstructs the coefficients it
// produces (and stores their residues as S4 does), one launch fewer; run_interpolate then
// run_reconstruct where the pass's tiles for every prime do not fit in LDS or there is a
// single variable.
hipError_t run_interpolate_reconstruct(const MatPlan& P, uint8_t* ws, uint32_t* out,
                                       hipStream_t st);

}  // namespace pd
