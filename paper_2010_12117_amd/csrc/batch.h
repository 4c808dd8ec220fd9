// Batched solve: thousands of matrices of different orders, variable counts and degrees run
// as a short sequence of persistent launches per chunk of matrices, one launch per stage
// (one per matrix order for the elimination). Each launch reads a table of per-matrix
// descriptors; a block walks its share of virtual blocks and finds the matrix of each by a
// binary search on the descriptors' first virtual block.
//
// Offsets in the descriptors are relative to the solve's base pointers: workspace offsets in
// bytes (a chunk's matrices occupy disjoint workspace regions, chunks reuse the workspace in
// turn), coefficient and output offsets through the per-matrix offset arrays that
// polydet_solve_batch copies to the device.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

#include "modarith.h"

namespace pd {

struct BReduce {
  int64_t block0;  // first virtual block of this matrix
  int64_t count;   // nslot * T coefficients
  int64_t T;
  int64_t res_off;
  int32_t mat, pn;
  const PrimeConst* pc;
  const int32_t* slot_src;
};

struct BExpand {
  int64_t block0;
  int64_t in_off, out_off, B, outer, inner, nent, tw_stride;
  int32_t m, Nv, JC, pad;
  const uint32_t* tw;  // already offset to this variable
  const PrimeConst* pc;
  const uint8_t* zero;
};

struct BDet {
  int64_t block0;
  int64_t pre_off, detv_off, den_off, R, tw_stride, rtiles, jtiles, nslot;
  int32_t N0, m0, Q, S;
  const uint32_t* tw0;
  const PrimeConst* pc;
  const uint8_t* zero;
  const int32_t* slot;
};

struct BIntt {
  int64_t block0;
  int64_t in_off, out_off, outer, inner, tw_stride, tiles;
  int64_t den_off;  // the first pass: the denominators, divided into the numerators as they load
                    // (-1 for the later passes)
  int32_t pn, Nv, logN, Dv1, W;
  int32_t reg;      // the register form: Nv / 8 = 4, 8 or 16 (intt_reg_body, kInttRegLines
                    // lines a tile), or 0
  const uint32_t* itw;
  const PrimeConst* pc;
};

struct BGarner {
  int64_t block0;
  int64_t coef_off, C;
  int32_t mat, pn, L, pad;
  const PrimeConst* pc;
  const uint32_t *gw, *gc, *ml, *hl;
};

// One launch of a batched solve.
struct BLaunch {
  enum Kind { kReduce, kExpand, kDet, kIntt, kGarner } kind;
  size_t desc_off;     // byte offset of its descriptors in the plan's descriptor buffer
  int32_t ndesc;
  int64_t vblocks;     // virtual blocks in total
  int32_t n, lanes;    // elimination launches: order and lanes per matrix
  int32_t ll;          // elimination launches: left-looking form (lanes = 1) or repair pass
  int32_t pair;        // elimination launches: terms per lane of the paired first-variable
                       // evaluation (fused_pair_terms), 0 when unpaired
  int32_t each;        // elimination launches: one single-matrix launch per descriptor in
                       // place of the batched kernel (batch_det_each)
  int32_t pnmax;       // reconstruction launches: largest prime count
  int32_t chunk;       // the chunk of matrices the launch belongs to
  size_t lds;          // dynamic LDS per block
};

// Launchers (kernels.hip and det_part.hip). `desc` points to device descriptors;
// the launches walk `vblocks` virtual blocks.
hipError_t batch_reduce(const BReduce* desc, int ndesc, int64_t vblocks, const int64_t* coeffs,
                        const int64_t* coeff_offsets, uint8_t* ws, hipStream_t st);
hipError_t batch_expand(const BExpand* desc, int ndesc, int64_t vblocks, uint8_t* ws,
                        hipStream_t st);
hipError_t batch_intt(const BIntt* desc, int ndesc, int64_t vblocks, size_t lds, uint8_t* ws,
                      hipStream_t st);
hipError_t batch_garner(const BGarner* desc, int ndesc, int64_t vblocks, int pnmax, uint8_t* ws,
                        uint32_t* out, const int64_t* out_offsets, hipStream_t st);
// ll = 1: left-looking launch; ll = 2: repair launch of the exchanging kernel (fixup);
// ll = 0: the exchanging kernel. pair: every matrix of the launch has fused_paired(m0) with
// that many fused_pair_terms, or 0: none has.
hipError_t batch_det(int n, int lanes, int ll, int pair, const BDet* desc, int ndesc,
                     int64_t vblocks, size_t lds, uint8_t* ws, hipStream_t st);
// The same elimination as batch_det (ll = 0 or 2) as one launch of the single-matrix kernel
// per matrix. `host_desc` is the host copy of the launch's descriptors; the kernels read the
// workspace `ws` on the device.
hipError_t batch_det_each(int n, int lanes, bool fixup, const BDet* host_desc, int ndesc,
                          int64_t vblocks, uint8_t* ws, hipStream_t st);

template <int N, int GL>
hipError_t det_fused_batch_launch(const BDet* desc, int ndesc, int64_t vblocks, size_t lds,
                                  uint8_t* ws, int pair, bool fixup, hipStream_t st);
template <int N>
hipError_t det_ll_batch_launch(const BDet* desc, int ndesc, int64_t vblocks, size_t lds,
                               uint8_t* ws, hipStream_t st);

// Virtual blocks are walked by at most this many resident blocks per launch (all but the
// elimination launches, which take one block per virtual block, at most kMaxGridBlocks).
constexpr int64_t kPersistentBlocks = 256 * 8;
constexpr int64_t kMaxGridBlocks = 0x7FFFFFFF;
// Coefficients per variable handled by the batched evaluation (registers).
constexpr int kBatchMaxM = 8;

// Index of the descriptor whose [block0, next block0) range holds vb.
template <typename D>
PD_HD int find_desc(const D* desc, int ndesc, int64_t vb) {
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].block0 <= vb) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace pd
