// Elimination kernels of the DET stage, included by the det_part.hip translation units that
// instantiate them for each (order, lanes-per-matrix) pair (det.h declares the launchers).
#pragma once

#include <hip/hip_runtime.h>

#include "batch.h"
#include "det.h"
#include "modarith.h"
#include "plan.h"

namespace pd {

constexpr int kDetBlock = 256;
constexpr int kEvalChunk = 8;  // entries per scheduling window of the fused evaluation

// ------------------------------------------------------------------------------------
// S3: determinant of the n x n matrix at every (prime, grid point).
//
// Division-free condensation, two columns per step. The paper's DET step (Section 3.2)
// condenses one column at a time (Chio's rule: with pivot pi = A[k][k], every later entry
// becomes pi A[i][j] - A[i][k] A[k][j]). Here two columns go at once, by Sylvester's
// determinant identity as used in Bareiss's two-step fraction-free elimination (Bareiss 1968):
// with the 2 x 2 leading minor D = A[k][k] A[k+1][k+1] - A[k][k+1] A[k+1][k], every entry
// i, j >= k + 2 becomes the 3 x 3 minor bordered by row i and column j,
//   A[i][j] <- D A[i][j] - A[i][k+1] u_j + A[i][k] v_j,
//   u_j = A[k][k] A[k+1][j] - A[k+1][k] A[k][j],   v_j = A[k][k+1] A[k+1][j] - A[k+1][k+1] A[k][j],
// and the condensed matrix of order m - 2 has determinant det(A) D^(m-3) (m = n - k, the
// order before the step). Three products under one Montgomery reduction replace the two
// reductions of two single steps. The last one or two rows finish directly (an entry, or a
// 2 x 2 determinant), so det = sign * last / prod_s D_s^(m_s - 3), and the denominator is
// accumulated with prefix products of the D_s. One inverse (Fermat) per determinant remains.
// Pivoting: the first nonzero entry scanning down column k becomes A[k][k]; if then D = 0,
// the first later row i whose single-step value A[k][k] A[i][k+1] - A[i][k] A[k][k+1] is
// nonzero takes the place of row k + 1 (D becomes that value). Each exchange flips the sign;
// no such row (or no pivot in column k) gives determinant 0.
//
// Mapping: GL lanes cooperate on one matrix (GL = 1: one matrix per lane). Lane t of a
// group holds columns t, t + GL, t + 2 GL, ... of all n rows in registers (a[c][i] is
// A[i][c GL + t]), so every index below is static after unrolling. The owners of columns k
// and k + 1 broadcast the pivot rows' and each row's two factors to their group with DPP
// moves; row exchanges are register selects.
// ------------------------------------------------------------------------------------

// Lane `src` of each aligned group of GL lanes to the whole group, as DPP moves (VALU, no
// LDS round trip). `src` is a constant after unrolling, so each switch folds to one case.
// GL = 2, 4: quad_perm within each quad. GL = 16: row_newbcast (lane src of each 16-lane
// row). GL = 8: row_newbcast of lane src into lanes 0-7 of the row (banks 0-1), then of lane
// 8 + src into lanes 8-15 (banks 2-3). Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
template <int O>
__device__ __forceinline__ uint32_t bcast8(uint32_t v) {
  const int lo = __builtin_amdgcn_update_dpp((int)v, (int)v, 0x150 + O, 0xF, 0x3, false);
  return (uint32_t)__builtin_amdgcn_update_dpp(lo, (int)v, 0x158 + O, 0xF, 0xC, false);
}

template <int GL>
__device__ __forceinline__ uint32_t bcast(uint32_t v, int src) {
  if constexpr (GL == 1) {
    return v;
  } else if constexpr (GL == 2) {
    return src == 0 ? dpp_mov<0xA0>(v) : dpp_mov<0xF5>(v);  // [0,0,2,2] / [1,1,3,3]
  } else if constexpr (GL == 4) {
    switch (src) {
      case 0: return dpp_mov<0x00>(v);
      case 1: return dpp_mov<0x55>(v);
      case 2: return dpp_mov<0xAA>(v);
      default: return dpp_mov<0xFF>(v);
    }
  } else if constexpr (GL == 8) {
    switch (src) {
      case 0: return bcast8<0>(v);
      case 1: return bcast8<1>(v);
      case 2: return bcast8<2>(v);
      case 3: return bcast8<3>(v);
      case 4: return bcast8<4>(v);
      case 5: return bcast8<5>(v);
      case 6: return bcast8<6>(v);
      default: return bcast8<7>(v);
    }
  } else {
    static_assert(GL == 16, "lane groups of 1, 2, 4, 8 or 16");
    switch (src) {
      case 0: return dpp_mov<0x150>(v);
      case 1: return dpp_mov<0x151>(v);
      case 2: return dpp_mov<0x152>(v);
      case 3: return dpp_mov<0x153>(v);
      case 4: return dpp_mov<0x154>(v);
      case 5: return dpp_mov<0x155>(v);
      case 6: return dpp_mov<0x156>(v);
      case 7: return dpp_mov<0x157>(v);
      case 8: return dpp_mov<0x158>(v);
      case 9: return dpp_mov<0x159>(v);
      case 10: return dpp_mov<0x15A>(v);
      case 11: return dpp_mov<0x15B>(v);
      case 12: return dpp_mov<0x15C>(v);
      case 13: return dpp_mov<0x15D>(v);
      case 14: return dpp_mov<0x15E>(v);
      default: return dpp_mov<0x15F>(v);
    }
  }
}

// The determinant of the matrix held by the lane group as a quotient num / den (Montgomery
// form): num = sign * (the last entry, or the last 2 x 2 determinant), 0 when the matrix is
// singular; den = prod_s D_s^(m_s - 3) (the representative of 1 for a singular matrix, so
// that den is never 0). The division is left to a later pass (the first interpolation pass,
// or finalize_kernel for integer matrices), which inverts the denominators of
// several points with one exponentiation. Every lane of the group returns the pair; all lanes
// of the wave must call this together (lane broadcasts).
// Entries may come in unreduced, in [0, 2p), and stay so: each step reduces only its two
// pivot columns (for the zero tests, the exchanges and the row factors), the column factors
// u_j, v_j are reduced, and the update sums three products with one unreduced factor
// (mm3_lazy: below 4 p^2 < p R for p < 2^30).
struct DetFrac {
  uint32_t num, den;
};

// Makes A[k][k] nonzero by exchanging row k with the first later row whose column-k entry is
// nonzero (column k reduced); no such row marks the matrix dead.
template <int N, int GL>
__device__ __forceinline__ void pivot_column(uint32_t (&a)[(N + GL - 1) / GL][N], int k,
                                             uint32_t& flip, bool& dead) {
  constexpr int C = (N + GL - 1) / GL;
  const int s = k / GL, o = k % GL;
  const uint32_t zero_piv = bcast<GL>(a[s][k] == 0u ? 1u : 0u, o);
  if (__any(zero_piv != 0u)) {
    int r = N;
#pragma unroll
    for (int i = N - 1; i > k; --i) r = (a[s][i] != 0u) ? i : r;
    r = (int)bcast<GL>((uint32_t)r, o);
    if (!zero_piv) r = k;
    dead = dead || (r == N);
    flip ^= (r != k && r != N) ? 1u : 0u;
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const bool sw = (r == i);
#pragma unroll
      for (int c = s; c < C; ++c) {
        const uint32_t x = a[c][k], y = a[c][i];
        a[c][k] = sw ? y : x;
        a[c][i] = sw ? x : y;
      }
    }
  }
}

template <int N, int GL>
__device__ __forceinline__ DetFrac eliminate(uint32_t (&a)[(N + GL - 1) / GL][N], uint32_t p,
                                             uint32_t pinv, uint32_t one) {
  constexpr int C = (N + GL - 1) / GL;
  uint32_t flip = 0;
  bool dead = false;
  uint32_t e = one, Q = one;  // e = D_0 .. D_s; Q accumulates the denominator
#pragma unroll
  for (int k = 0; k + 2 < N; k += 2) {
    const int s0 = k / GL, o0 = k % GL;
    const int s1 = (k + 1) / GL, o1 = (k + 1) % GL;
    // reduce the two pivot columns (with them the other columns of their slots, harmlessly)
#pragma unroll
    for (int i = k; i < N; ++i) {
      a[s0][i] = fold(a[s0][i], p);
      if (s1 != s0) a[s1][i] = fold(a[s1][i], p);
    }
    pivot_column<N, GL>(a, k, flip, dead);
    const uint32_t a00 = bcast<GL>(a[s0][k], o0), a01 = bcast<GL>(a[s1][k], o1);
    uint32_t a10 = bcast<GL>(a[s0][k + 1], o0), a11 = bcast<GL>(a[s1][k + 1], o1);
    uint32_t D = mm2(a00, a11, p - a10, a01, p, pinv);
    if (__any(D == 0u && !dead)) {
      // a vanishing 2 x 2 minor: bring up the first row whose single-step value is nonzero
      int r = N;
#pragma unroll
      for (int i = N - 1; i > k + 1; --i) {
        const uint32_t b = mm2(a00, bcast<GL>(a[s1][i], o1), p - bcast<GL>(a[s0][i], o0), a01,
                               p, pinv);
        r = (b != 0u) ? i : r;
      }
      if (D != 0u) r = k + 1;
      dead = dead || (r == N);
      flip ^= (r != k + 1 && r != N) ? 1u : 0u;
#pragma unroll
      for (int i = k + 2; i < N; ++i) {
        const bool sw = (r == i);
#pragma unroll
        for (int c = s0; c < C; ++c) {
          const uint32_t x = a[c][k + 1], y = a[c][i];
          a[c][k + 1] = sw ? y : x;
          a[c][i] = sw ? x : y;
        }
      }
      a10 = bcast<GL>(a[s0][k + 1], o0);
      a11 = bcast<GL>(a[s1][k + 1], o1);
      D = mm2(a00, a11, p - a10, a01, p, pinv);
    }
    // the slots that hold columns >= k + 2 (a slot's lanes below that column compute values
    // nobody reads)
    const int sf = (k + 2) / GL;
    if constexpr (GL == 1) {
      // one lane per matrix: column by column, so that only one column's factors are live
#pragma unroll
      for (int c = k + 2; c < N; ++c) {
        const uint32_t nu = p - fold(mm2_lazy(a00, a[c][k + 1], p - a10, a[c][k], p, pinv), p);
        const uint32_t v = fold(mm2_lazy(a01, a[c][k + 1], p - a11, a[c][k], p, pinv), p);
#pragma unroll
        for (int i = k + 2; i < N; ++i)
          a[c][i] = mm3_lazy(D, a[c][i], a[k + 1][i], nu, a[k][i], v, p, pinv);
      }
    } else {
      uint32_t nu[C], v[C];
#pragma unroll
      for (int c = sf; c < C; ++c) {
        nu[c] = p - fold(mm2_lazy(a00, a[c][k + 1], p - a10, a[c][k], p, pinv), p);
        v[c] = fold(mm2_lazy(a01, a[c][k + 1], p - a11, a[c][k], p, pinv), p);
      }
#pragma unroll
      for (int i = k + 2; i < N; ++i) {
        const uint32_t f0 = bcast<GL>(a[s0][i], o0), f1 = bcast<GL>(a[s1][i], o1);
#pragma unroll
        for (int c = sf; c < C; ++c) a[c][i] = mm3_lazy(D, a[c][i], f1, nu[c], f0, v[c], p, pinv);
      }
    }
    // den = prod_s D_s^(m_s - 3) as prod_s e_s^(w_s), e_s = D_0 .. D_s: w_s = 2 while another
    // two-column step follows, and m_s - 3 (0 or 1) for the last one
    e = mm(e, D, p, pinv);
    if (k + 4 < N) {
      Q = mm(Q, e, p, pinv);
      Q = mm(Q, e, p, pinv);
    } else if (N - k == 4) {
      Q = mm(Q, e, p, pinv);
    }
  }
  constexpr int kl = (N - 1) & ~1;  // first row of the last block: N - 1 (odd N) or N - 2
  uint32_t last;
  if constexpr (N - kl == 2) {
    // the remaining 2 x 2 block: its determinant directly
    constexpr int s0 = kl / GL, o0 = kl % GL, s1 = (kl + 1) / GL, o1 = (kl + 1) % GL;
    const uint32_t a00 = fold(bcast<GL>(a[s0][kl], o0), p);
    const uint32_t a10 = fold(bcast<GL>(a[s0][kl + 1], o0), p);
    const uint32_t a01 = fold(bcast<GL>(a[s1][kl], o1), p);
    const uint32_t a11 = fold(bcast<GL>(a[s1][kl + 1], o1), p);
    last = mm2(a00, a11, p - a10, a01, p, pinv);
  } else {
    constexpr int sl = kl / GL, ol = kl % GL;
    last = fold(bcast<GL>(a[sl][kl], ol), p);
  }
  dead = dead || (last == 0u);
  DetFrac f;
  f.num = dead ? 0u : (flip ? negm(last, p) : last);
  f.den = dead ? one : Q;
  return f;
}

// Waves per SIMD asked of the compiler for the elimination kernels (single-matrix and batched)
// where it lands just above an occupancy step by itself. With one lane per matrix (paired
// kernel) the request is the lane's n^2 values plus kDetRegMargin, out of 512 registers per
// lane: 168 at n = 12 (169 unasked: two waves) without spills. At n = 32 with 8 lanes (171-175
// unasked) three waves cost a few spilled values and were measured 7-8% faster; at n = 31 they
// were not. Every other kernel gets no request (1: the launch bounds alone).
constexpr int kDetRegMargin = 24;
template <int N, int GL, bool PAIR>
constexpr int det_waves() {
  if (GL == 8 && N == 32) return 3;
  // 4 lanes from order 21: the kernels land at 164-187 VGPRs (2 waves); asked for 3 they spill
  // up to 14 values and ran the 4096-matrix batch 5% faster, batched and plain alike
  if (GL == 4 && N >= 21) return 3;
  // 2 lanes at orders 13 and 16 (133-135 and 176-178 VGPRs unasked: 3 and 2 waves): asked for 4
  // and 3 they spill 7-11 values and ran those classes of the batch 4% and 7-11% faster
  if (GL == 2 && N == 16) return 3;
  if (GL == 2 && N == 13) return 4;
  if (GL != 1 || !PAIR) return 1;
  constexpr int regs = ((N * N + kDetRegMargin + 7) / 8) * 8;
  constexpr int w = 512 / regs;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// Unfused form: the matrix at each point is read from the full evaluation tensor
// eval[pn][n*n][npts].
template <int N, int GL>
__global__ __launch_bounds__(kDetBlock) void det_kernel(const uint32_t* __restrict__ eval,
                                                        uint32_t* __restrict__ detv,
                                                        uint32_t* __restrict__ denv, int64_t npts,
                                                        const PrimeConst* __restrict__ pcs) {
  constexpr int C = (N + GL - 1) / GL;
  constexpr int PER_BLOCK = kDetBlock / GL;
  const int prime = blockIdx.y;
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv, one = pcs[prime].r1;
  const int t = (int)(threadIdx.x % GL);
  const int64_t pt = (int64_t)blockIdx.x * PER_BLOCK + threadIdx.x / GL;
  const bool valid = pt < npts;
  const int64_t ptc = valid ? pt : npts - 1;
  const uint32_t* src = eval + (int64_t)prime * N * N * npts + ptc;

  uint32_t a[C][N];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int col = c * GL + t;
    const int colc = col < N ? col : N - 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const uint32_t v = src[(int64_t)(i * N + colc) * npts];
      a[c][i] = col < N ? v : 0u;
    }
  }
  const DetFrac d = eliminate<N, GL>(a, p, pinv, one);
  if (valid && t == 0) {
    detv[(int64_t)prime * npts + pt] = d.num;
    denv[(int64_t)prime * npts + pt] = d.den;
  }
}

// Stages columns r0 .. r0+Q-1 of the pre-tensor pre[nslot][m0][R] (one prime) in LDS as
// tile[m][q][i * NCP + col] with NCP >= n columns per row (the columns past n-1 hold zeros,
// so that every lane of a lane group reads the same offsets) and row stride
// NEP = n*NCP | 1 (odd, so lanes reading different q hit different banks, and the entry
// offset is an immediate). Entry e is read from pre-tensor slot slot[e] (entries with equal
// coefficients share a slot). Zero entries and points past R are stored as zeros without
// reading memory.
template <int N, int NCP>
__device__ __forceinline__ void fill_tile(uint32_t* tile, const uint32_t* __restrict__ src,
                                          int64_t R, int m0, int Q, int64_t r0,
                                          const uint8_t* __restrict__ zero,
                                          const int32_t* __restrict__ slot) {
  constexpr int NEC = N * NCP;
  constexpr int NEP = NEC | 1;
  // Q is a power of two: q = idx mod Q by mask, the padded entry index ec = idx / Q by shift;
  // every thread then copies its (ec, q) for each of the m0 coefficients
  const int qs = __builtin_ctz((unsigned)Q);
  for (int idx = threadIdx.x; idx < NEC * Q; idx += kDetBlock) {
    const int q = idx & (Q - 1);
    const int ec = idx >> qs;
    const int i = ec / NCP, col = ec - i * NCP;
    const int e = i * N + col;
    const bool live = col < N && !(zero && zero[e]) && r0 + q < R;
    uint32_t* d = tile + q * NEP + ec;
    if (live) {
      const uint32_t* s = src + (int64_t)slot[e] * m0 * R + r0 + q;
      for (int m = 0; m < m0; ++m) d[m * Q * NEP] = s[(int64_t)m * R];
    } else {
      for (int m = 0; m < m0; ++m) d[m * Q * NEP] = 0u;
    }
  }
}

// In a repair launch (fixup = true) a block recomputes only the points whose denominator an
// earlier launch left at 0 (a zero pivot the left-looking kernel cannot exchange away).
// Returns whether this block has such a point; every thread of the block gets the answer.
// Where the local point r of a slab lies on the grid (FusedDetArgs: seg, off1, off2).
__device__ __forceinline__ int64_t slab_point(int64_t r, int64_t seg, int64_t off1,
                                              int64_t off2) {
  return r + (r < seg ? off1 : off2);
}

__device__ __forceinline__ bool block_needs_fixup(const uint32_t* __restrict__ denv, int64_t R,
                                                  int N0, int NJ, int Q, int S, int64_t r0,
                                                  int jbase, int prime, int64_t Rout,
                                                  int64_t seg, int64_t off1, int64_t off2) {
  int any = 0;
  const int halves = N0 / NJ;  // 2 when the points j0 and j0 + N0/2 are taken in pairs
  const int pts = Q * S * halves;
  for (int idx = threadIdx.x; idx < pts; idx += kDetBlock) {
    const int q = idx % Q, jo = (idx / Q) % S, hh = idx / (Q * S);
    const int j0 = jbase + jo;
    if (r0 + q < R && j0 < NJ &&
        denv[(int64_t)prime * N0 * Rout + (int64_t)(j0 + hh * NJ) * Rout +
             slab_point(r0 + q, seg, off1, off2)] == 0u)
      any = 1;
  }
  return __syncthreads_or(any) != 0;
}

// Fused form: the last evaluation axis (the first variable, whose grid index j0 is the
// slowest) runs inside the elimination kernel, so the full evaluation tensor never exists.
// pre[pn][nslot][m0][R] holds every evaluated entry (slot) already evaluated along the other
// variables (R points) with its m0 coefficients in the first variable. A block stages the columns
// r0 .. r0+Q-1 in LDS (fill_tile) and then, for S values of j0, each lane group rebuilds its
// matrix at the point (j0, r0 + q) as sum_m x_m w0^{m j0} (the evaluation of Section 2 along
// x1) and eliminates it with row exchanges. Point index = j0 R + r.
//
// PT > 0 (paired, 2 <= m0 <= 2 PT, fused_paired): j0 runs over [0, N0/2) and lanes l and
// l + 32 of a wave build the points j0 and j0 + N0/2 of the same (slot, r) together. The
// lower lane sums the even terms E = x0 + x2 w0^{2 j0} (+ x4 w0^{4 j0}), the upper one the odd
// terms O = x1 w0^{j0} + x3 w0^{3 j0} (+ x5 w0^{5 j0}), PT products under one reduction each;
// they exchange the sums, and since w0^{N0/2} = -1 the values are E + O and E - O: half the
// products and LDS reads of the unpaired form, and one reduction instead of m0 / 2.
// One block's share of the fused kernel: prime `prime`, tile `bx` = (j-range, r-range).
template <int N, int GL, int PT>
__device__ __forceinline__ void det_fused_body(
    uint32_t* tile, const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv,
    uint32_t* __restrict__ denv, int64_t R,
    int N0, int m0, int Q, int S, const uint32_t* __restrict__ tw0, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero,
    const int32_t* __restrict__ entry_slot, int64_t nslot, int prime, int64_t bx, bool fixup,
    int64_t Rout, int64_t seg, int64_t off1, int64_t off2) {
  constexpr bool PAIR = PT > 0;
  static_assert(PT == 0 || PT == 2 || PT == 3, "two or three terms per lane when paired");
  constexpr int C = (N + GL - 1) / GL;
  constexpr int NE = N * N;
  constexpr int NCP = C * GL;  // tile columns per row, padded for the last lane slot
  constexpr int NEP = (N * NCP) | 1;
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv, one = pcs[prime].r1;
  const int64_t rtiles = (R + Q - 1) / Q;
  const int64_t r0 = (bx % rtiles) * Q;
  const int jbase = (int)(bx / rtiles) * S;
  const uint32_t* src = pre + (int64_t)prime * nslot * m0 * R;
  const int NJ = PAIR ? N0 / 2 : N0;
  if (fixup && !block_needs_fixup(denv, R, N0, NJ, Q, S, r0, jbase, prime, Rout, seg, off1, off2))
    return;
  fill_tile<N, NCP>(tile, src, R, m0, Q, r0, zero, entry_slot);
  // Structurally zero entries as a wave-uniform bit mask (one lane per matrix only): the
  // paired evaluation branches around them (scalar branches; their registers are set to 0).
  uint64_t zm[(NE + 63) / 64];
#pragma unroll
  for (int w = 0; w < (NE + 63) / 64; ++w) {
    const int e = w * 64 + (int)(threadIdx.x & 63);
    zm[w] = (GL == 1 && zero) ? __ballot(e < NE && zero[e] != 0) : 0ull;
  }
  __syncthreads();

  // lane -> (half, pair index): lanes l and l + 32 of a wave share (slot, r, j0) when paired
  const int lane = (int)(threadIdx.x & 63);
  const int half = PAIR ? (lane >> 5) : 0;
  const int pidx = PAIR ? (int)(((threadIdx.x >> 6) << 5) | (unsigned)(lane & 31))
                        : (int)threadIdx.x;
  const int t = pidx % GL;
  const int slot = pidx / GL;
  const int q = slot % Q;
  const int J = ((PAIR ? kDetBlock / 2 : kDetBlock) / GL) / Q;
  const int jj = slot / Q;
  const bool qvalid = r0 + q < R;
  const uint32_t* w0 = tw0 + (int64_t)prime * tw_stride;
  // lanes of the last slot past column n - 1 read the tile's zero columns: their registers
  // evaluate to 0, which the elimination expects

  for (int j = jbase; j < jbase + S && j < NJ; j += J) {
    const int j0 = j + jj;
    const bool valid = qvalid && j0 < NJ && j0 < jbase + S;
    const int j0c = j0 < NJ ? j0 : NJ - 1;
    uint32_t a[C][N];
    if constexpr (PAIR) {
      // an opaque copy per point keeps the compiler from hoisting all n^2 branch conditions
      // out of the loop (they would be spilled to VGPR lanes and read back one by one)
#pragma unroll
      for (int w = 0; w < (NE + 63) / 64; ++w) asm volatile("" : "+s"(zm[w]));
      // terms m = half, half + 2 (and half + 4 when PT = 3) of every entry, weight
      // w0^{m j0} (0 past m0 - 1, where the row index is clamped to a valid row); w0^0 is
      // the representative of 1
      const int ma = half, mb = half + 2, mc = half + 4;
      const uint32_t wa = ma < m0 ? w0[(ma * j0c) & (N0 - 1)] : 0u;
      const uint32_t wb = mb < m0 ? w0[(mb * j0c) & (N0 - 1)] : 0u;
      const uint32_t wc = PT == 3 && mc < m0 ? w0[(mc * j0c) & (N0 - 1)] : 0u;
      const uint32_t* ra = tile + ((ma < m0 ? ma : m0 - 1) * Q + q) * NEP + t;
      const uint32_t* rb = tile + ((mb < m0 ? mb : m0 - 1) * Q + q) * NEP + t;
      const uint32_t* rc = tile + ((mc < m0 ? mc : m0 - 1) * Q + q) * NEP + t;
      const uint32_t sm = half ? ~0u : 0u, sc = half ? p + 1u : 0u;
#pragma unroll
      for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const int off = i * NCP + c * GL;
          const int e = i * N + c;  // the entry's index when GL == 1
          if (GL == 1 && ((zm[e >> 6] >> (e & 63)) & 1ull)) {
            a[c][i] = 0u;
          } else {
            const uint32_t v = PT == 3 ? mm3(ra[off], wa, rb[off], wb, rc[off], wc, p, pinv)
                                       : mm2(ra[off], wa, rb[off], wb, p, pinv);
            // every lane now holds E (the lower lane's v) and O (the upper lane's v). Keep
            // E + O (lower lane) or E + (p - O) (upper lane), as E + (O ^ sm) + sc: with
            // sm = -1 and sc = p + 1, (O ^ sm) + sc = p - O. Both lie below 2p and are left
            // unreduced for the elimination.
            const auto eo = __builtin_amdgcn_permlane32_swap(v, v, false, false);
            a[c][i] = eo[0] + (eo[1] ^ sm) + sc;
          }
          // without a branch per entry (GL > 1) the scheduler would run every product first
          // and keep all of them live until their exchanges: bound its window
          if (GL > 1 && (c * N + i) % kEvalChunk == kEvalChunk - 1)
            __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      // a[c][i] = sum_{m < m0} x_m w0^{m j0}, two terms per reduction (mm2). With m0 even
      // the constant term pairs with x_1 (its factor is R mod p, the representative of 1);
      // with m0 odd it stands alone. The loop over m is uniform and sits outside the
      // unrolled loops over the entries held by the lane.
      int mstart;
      if ((m0 & 1) == 0) {
        const uint32_t w1 = w0[j0c & (N0 - 1)];
        const uint32_t* r0w = tile + q * NEP + t;
        const uint32_t* r1w = r0w + Q * NEP;
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const int off = i * NCP + c * GL;
            a[c][i] = mm2(r0w[off], one, r1w[off], w1, p, pinv);
            if ((c * N + i) % kEvalChunk == kEvalChunk - 1) __builtin_amdgcn_sched_barrier(0);
          }
        }
        mstart = 2;
      } else {
        const uint32_t* r0w = tile + q * NEP + t;
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int i = 0; i < N; ++i) a[c][i] = r0w[i * NCP + c * GL];
        }
        mstart = 1;
      }
      for (int m = mstart; m < m0; m += 2) {
        const uint32_t wa = w0[(m * j0c) & (N0 - 1)];
        const uint32_t wb = w0[((m + 1) * j0c) & (N0 - 1)];
        const uint32_t* ra = tile + (m * Q + q) * NEP + t;
        const uint32_t* rb = ra + Q * NEP;
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const int off = i * NCP + c * GL;
            a[c][i] = addm(a[c][i], mm2(ra[off], wa, rb[off], wb, p, pinv), p);
            // bound the scheduler's window so that the LDS reads (one register each) are
            // not all hoisted ahead of the arithmetic
            if ((c * N + i) % kEvalChunk == kEvalChunk - 1) __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
    const DetFrac d = eliminate<N, GL>(a, p, pinv, one);
    const int64_t o = (int64_t)prime * N0 * Rout + (int64_t)(j0 + half * NJ) * Rout +
                      slab_point(r0 + q, seg, off1, off2);
    if (valid && t == 0 && (!fixup || denv[o] == 0u)) {
      detv[o] = d.num;
      denv[o] = d.den;
    }
  }
}

// The hardware hands a launch's workgroups to the 8 XCDs of the chip in turn (linear id mod
// 8), and each XCD has its own L2. Neighbouring tiles read neighbouring 32-byte pieces of the
// same 128-byte lines of the pre-tensor, so within every 32 consecutive workgroups the 4 that
// an XCD receives take 4 consecutive tiles: block 32 g + 8 q + x takes tile 32 g + 4 x + q.
// The order over the whole launch stays interleaved, which keeps the XCDs evenly loaded when
// tiles differ in cost (a batch puts its largest grids first). The last nb mod 32 blocks (in
// a grid row of nb) keep the identity.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  if (b >= (nb & ~(int64_t)31)) return b;
  return (b & ~(int64_t)31) | ((b & 7) << 2) | ((b >> 3) & 3);
}

template <int N, int GL>
__global__ __launch_bounds__(kDetBlock) __attribute__((amdgpu_waves_per_eu(det_waves<N, GL, false>())))
void det_fused_kernel(
    const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv, uint32_t* __restrict__ denv,
    int64_t R, int N0, int m0, int Q, int S, const uint32_t* __restrict__ tw0, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero,
    const int32_t* __restrict__ slot, int64_t nslot, bool fixup, int64_t Rout, int64_t seg,
    int64_t off1, int64_t off2) {
  extern __shared__ uint32_t tile[];  // [m0][Q][n*n | 1]
  det_fused_body<N, GL, 0>(tile, pre, detv, denv, R, N0, m0, Q, S, tw0, tw_stride, pcs, zero,
                               slot, nslot, blockIdx.y, xcd_tile(blockIdx.x, gridDim.x), fixup,
                               Rout, seg, off1, off2);
}

template <int N, int GL, int PT>
__global__ __launch_bounds__(kDetBlock) __attribute__((amdgpu_waves_per_eu(det_waves<N, GL, true>())))
void det_fused_pair_kernel(
    const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv, uint32_t* __restrict__ denv,
    int64_t R, int N0, int m0, int Q, int S, const uint32_t* __restrict__ tw0, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero,
    const int32_t* __restrict__ slot, int64_t nslot, bool fixup, int64_t Rout, int64_t seg,
    int64_t off1, int64_t off2) {
  extern __shared__ uint32_t tile[];  // [m0][Q][n*n | 1]
  det_fused_body<N, GL, PT>(tile, pre, detv, denv, R, N0, m0, Q, S, tw0, tw_stride, pcs, zero,
                              slot, nslot, blockIdx.y, xcd_tile(blockIdx.x, gridDim.x), fixup,
                              Rout, seg, off1, off2);
}

// Batched form: blocks walk the virtual blocks of every matrix of this order in the launch;
// virtual block vb of matrix d is (prime, tile) = divmod(vb - block0, rtiles * jtiles).
template <int N, int GL, int PT>
__device__ __forceinline__ void det_fused_batch_body(uint32_t* tile, const BDet* __restrict__ desc,
                                                     int ndesc, int64_t vblocks,
                                                     uint8_t* __restrict__ ws, bool fixup) {
  // One block per virtual block (no persistent loop: the loop's state costs registers that
  // the elimination needs), consecutive virtual blocks on one XCD.
  const int64_t vb = xcd_tile(blockIdx.x, gridDim.x);
  if (vb >= vblocks) return;
  const BDet& d = desc[find_desc(desc, ndesc, vb)];
  const int64_t local = vb - d.block0;
  const int64_t per_prime = d.rtiles * d.jtiles;
  const int prime = (int)(local / per_prime);
  det_fused_body<N, GL, PT>(tile, (const uint32_t*)(ws + d.pre_off),
                              (uint32_t*)(ws + d.detv_off), (uint32_t*)(ws + d.den_off), d.R,
                              d.N0, d.m0, d.Q, d.S, d.tw0, d.tw_stride, d.pc, d.zero, d.slot,
                              d.nslot, prime, local - (int64_t)prime * per_prime, fixup, d.R,
                              d.R, 0, 0);
}

template <int N, int GL>
__global__ __launch_bounds__(kDetBlock) __attribute__((amdgpu_waves_per_eu(det_waves<N, GL, false>())))
void det_fused_batch_kernel(
    const BDet* __restrict__ desc, int ndesc, int64_t vblocks, uint8_t* __restrict__ ws,
    bool fixup) {
  extern __shared__ uint32_t tile[];
  det_fused_batch_body<N, GL, 0>(tile, desc, ndesc, vblocks, ws, fixup);
}

template <int N, int GL, int PT>
__global__ __launch_bounds__(kDetBlock) __attribute__((amdgpu_waves_per_eu(det_waves<N, GL, true>())))
void det_fused_pair_batch_kernel(
    const BDet* __restrict__ desc, int ndesc, int64_t vblocks, uint8_t* __restrict__ ws,
    bool fixup) {
  extern __shared__ uint32_t tile[];
  det_fused_batch_body<N, GL, PT>(tile, desc, ndesc, vblocks, ws, fixup);
}

// ------------------------------------------------------------------------------------
// Left-looking form of the same condensation, one lane per matrix. Row i is evaluated from
// the LDS tile when it is needed and reduced against the stored pivot rows k < i in order,
//   r[c] <- pi_k r[c] - r[k] U[k][c]   (c > k),
// which are exactly the updates the right-looking form applies to row i at steps 0..i-1, so
// the pivots and the quotient num / den are the same. Only the pivots pi_k and the strict
// upper parts U[k][c] stay in registers (n(n+1)/2 - 1 values instead of n^2), which leaves
// room for four waves per SIMD at n = 12. Rows cannot be exchanged here: a zero pivot (the
// plan's row order removes the structural ones, so it happens only when a value vanishes
// mod p) marks the point with den = 0 and the exchanging kernel recomputes it in a repair
// launch (fixup = true in det_fused_body).
// ------------------------------------------------------------------------------------

// Columns evaluated between scheduling barriers: the row is evaluated while every earlier
// pivot row is live, so its loads and 64-bit products are kept to a few at a time.
constexpr int kLLEvalChunk = 4;

template <int N>
__device__ __forceinline__ void eval_row(uint32_t (&r)[N], const uint32_t* tile, int i, int q,
                                         int Q, int m0, const uint32_t* __restrict__ w0, int j0,
                                         int mask, uint32_t one, uint32_t p, uint32_t pinv) {
  constexpr int NEP = (N * N) | 1;
  const uint32_t* b0 = tile + q * NEP + i * N;
  const int step = Q * NEP;
  // sum_{m < m0} x_m w^m, two terms per reduction; m0 even pairs the constant term with x_1
  int m;
  if ((m0 & 1) == 0) {
    const uint32_t w1 = w0[j0 & mask];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      r[c] = mm2(b0[c], one, b0[step + c], w1, p, pinv);
      if (c % kLLEvalChunk == kLLEvalChunk - 1) __builtin_amdgcn_sched_barrier(0);
    }
    m = 2;
  } else {
#pragma unroll
    for (int c = 0; c < N; ++c) r[c] = b0[c];
    m = 1;
  }
#pragma unroll 1
  for (; m + 1 < m0; m += 2) {
    const uint32_t wa = w0[(m * j0) & mask], wb = w0[((m + 1) * j0) & mask];
    const uint32_t* ra = b0 + m * step;
    const uint32_t* rb = ra + step;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      r[c] = addm(r[c], mm2(ra[c], wa, rb[c], wb, p, pinv), p);
      if (c % kLLEvalChunk == kLLEvalChunk - 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Row I of the left-looking pass: evaluate row I at the point, apply the I earlier pivot
// rows in order (each a Chio step with its pivot), and keep the result as the next pivot row.
// Recursion over I keeps every register index a compile-time constant.
template <int N, int I>
__device__ __forceinline__ void ll_rows(uint32_t (&piv)[N], uint32_t (&U)[N][N], uint32_t& e,
                                        uint32_t& den, bool& bad, const uint32_t* tile, int q,
                                        int Q, int m0, const uint32_t* __restrict__ w0, int j0,
                                        int mask, uint32_t one, uint32_t p, uint32_t pinv) {
  if constexpr (I < N) {
    // keep the scheduler from hoisting later rows' LDS reads (register pressure)
    __builtin_amdgcn_sched_barrier(0);
    uint32_t r[N];
    eval_row<N>(r, tile, I, q, Q, m0, w0, j0, mask, one, p, pinv);
#pragma unroll
    for (int k = 0; k < I; ++k) {
      const uint32_t mk = p - r[k];  // -A[I][k]; p stands for 0
#pragma unroll
      for (int c = 0; c < N; ++c)
        if (c > k) r[c] = mm2(piv[k], r[c], mk, U[k][c], p, pinv);
    }
    // Pin the finished row in place: otherwise the compiler sinks each row's elimination
    // to where its results are first used, behind the evaluation of the later rows, and all
    // n evaluated rows end up live together.
#pragma unroll
    for (int c = I; c < N; ++c) asm volatile("" : "+v"(r[c]));
    piv[I] = r[I];
    if constexpr (I < N - 1) {
      bad = bad || (r[I] == 0u);
#pragma unroll
      for (int c = I + 1; c < N; ++c) U[I][c] = r[c];
      if constexpr (I <= N - 3) {
        e = mm(e, r[I], p, pinv);
        den = mm(den, e, p, pinv);
      }
    }
    ll_rows<N, I + 1>(piv, U, e, den, bad, tile, q, Q, m0, w0, j0, mask, one, p, pinv);
  }
}

template <int N>
__device__ __forceinline__ void det_ll_body(
    uint32_t* tile, const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv,
    uint32_t* __restrict__ denv, int64_t R, int N0, int m0, int Q, int S,
    const uint32_t* __restrict__ tw0, int64_t tw_stride, const PrimeConst* __restrict__ pcs,
    const uint8_t* __restrict__ zero, const int32_t* __restrict__ slot, int64_t nslot, int prime,
    int64_t bx) {
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv, one = pcs[prime].r1;
  // The exchanging kernel's tiles (Q points, S values of j0 in [0, N0/2) with their partners
  // j0 + N0/2 when paired) cover the same points as these: S' = 2 S values of j0 in [0, N0).
  S = fused_paired(m0) ? 2 * S : S;
  const int64_t rtiles = (R + Q - 1) / Q;
  const int64_t r0 = (bx % rtiles) * Q;
  const int jbase = (int)(bx / rtiles) * S;
  fill_tile<N, N>(tile, pre + (int64_t)prime * nslot * m0 * R, R, m0, Q, r0, zero, slot);
  __syncthreads();

  const int q = (int)(threadIdx.x % Q);
  const int J = kDetBlock / Q;
  const int jj = (int)(threadIdx.x / Q);
  const bool qvalid = r0 + q < R;
  const uint32_t* w0 = tw0 + (int64_t)prime * tw_stride;

  for (int j = jbase; j < jbase + S && j < N0; j += J) {
    const int j0 = j + jj;
    const bool valid = qvalid && j0 < N0 && j0 < jbase + S;
    const int j0c = j0 < N0 ? j0 : N0 - 1;
    uint32_t piv[N];
    uint32_t U[N][N];  // U[k][c] for c > k only
    uint32_t e = one, den = one;
    bool bad = false;
    // The tile does not change inside this loop; an opaque copy of its offset keeps the
    // compiler from hoisting all n^2 constant-term reads out of the loop into registers.
    int qoff = q;
    asm volatile("" : "+v"(qoff));
    ll_rows<N, 0>(piv, U, e, den, bad, tile, qoff, Q, m0, w0, j0c, N0 - 1, one, p, pinv);
    // Without this the compiler sinks the whole elimination into the store branch below,
    // after all n rows have been evaluated, and every row is then live at once.
    uint32_t last = piv[N - 1];
    asm volatile("" : "+v"(last), "+v"(den));
    uint32_t num = last;
    if (bad) {
      num = 0u;
      den = 0u;  // repair marker
    } else if (last == 0u) {
      den = one;  // singular mod p
    }
    if (valid) {
      const int64_t o = (int64_t)prime * N0 * R + (int64_t)j0 * R + r0 + q;
      detv[o] = num;
      denv[o] = den;
    }
  }
}

template <int N>
__global__ __launch_bounds__(kDetBlock) void det_ll_kernel(
    const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv, uint32_t* __restrict__ denv,
    int64_t R, int N0, int m0, int Q, int S, const uint32_t* __restrict__ tw0, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero,
    const int32_t* __restrict__ slot, int64_t nslot) {
  extern __shared__ uint32_t tile[];
  det_ll_body<N>(tile, pre, detv, denv, R, N0, m0, Q, S, tw0, tw_stride, pcs, zero, slot, nslot,
                 blockIdx.y, blockIdx.x);
}

template <int N>
__global__ __launch_bounds__(kDetBlock) void det_ll_batch_kernel(
    const BDet* __restrict__ desc, int ndesc, int64_t vblocks, uint8_t* __restrict__ ws) {
  extern __shared__ uint32_t tile[];
  const int64_t vb = blockIdx.x;  // one block per virtual block, as in the exchanging kernel
  if (vb >= vblocks) return;
  const BDet& d = desc[find_desc(desc, ndesc, vb)];
  const int64_t local = vb - d.block0;
  const int64_t per_prime = d.rtiles * d.jtiles;
  const int prime = (int)(local / per_prime);
  det_ll_body<N>(tile, (const uint32_t*)(ws + d.pre_off), (uint32_t*)(ws + d.detv_off),
                 (uint32_t*)(ws + d.den_off), d.R, d.N0, d.m0, d.Q, d.S, d.tw0, d.tw_stride,
                 d.pc, d.zero, d.slot, d.nslot, prime, local - (int64_t)prime * per_prime);
}

template <int N, int GL>
hipError_t det_launch(const uint32_t* eval, uint32_t* detv, uint32_t* denv, int64_t npts, int pn,
                      const PrimeConst* pcs, hipStream_t st) {
  constexpr int per_block = kDetBlock / GL;
  const int64_t bx = (npts + per_block - 1) / per_block;
  hipLaunchKernelGGL((det_kernel<N, GL>), dim3((unsigned)bx, (unsigned)pn), dim3(kDetBlock), 0, st,
                     eval, detv, denv, npts, pcs);
  return hipGetLastError();
}

template <int N, int GL>
hipError_t det_fused_batch_launch(const BDet* desc, int ndesc, int64_t vblocks, size_t lds,
                                  uint8_t* ws, int pair, bool fixup, hipStream_t st) {
  if (vblocks < 1) return hipSuccess;
  if (vblocks > kMaxGridBlocks) return hipErrorInvalidConfiguration;
  const dim3 g((unsigned)vblocks);
  if (pair == 2)
    hipLaunchKernelGGL((det_fused_pair_batch_kernel<N, GL, 2>), g, dim3(kDetBlock), lds, st,
                       desc, ndesc, vblocks, ws, fixup);
  else if (pair == 3)
    hipLaunchKernelGGL((det_fused_pair_batch_kernel<N, GL, 3>), g, dim3(kDetBlock), lds, st,
                       desc, ndesc, vblocks, ws, fixup);
  else if (pair == 0)
    hipLaunchKernelGGL((det_fused_batch_kernel<N, GL>), g, dim3(kDetBlock), lds, st, desc, ndesc,
                       vblocks, ws, fixup);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int N>
hipError_t det_ll_launch(const FusedDetArgs& f, hipStream_t st) {
  const int64_t rtiles = (f.R + f.Q - 1) / f.Q;
  const int Sl = fused_paired(f.m0) ? 2 * f.S : f.S;
  const int64_t jtiles = (f.N0 + Sl - 1) / Sl;
  const size_t lds = fused_tile_words(N, 1, f.m0, f.Q) * sizeof(uint32_t);
  hipLaunchKernelGGL((det_ll_kernel<N>), dim3((unsigned)(rtiles * jtiles), (unsigned)f.pn),
                     dim3(kDetBlock), lds, st, f.pre, f.detv, f.denv, f.R, f.N0, f.m0, f.Q, f.S,
                     f.tw0, f.tw_stride, f.pcs, f.zero, f.slot, f.nslot);
  return hipGetLastError();
}

template <int N>
hipError_t det_ll_batch_launch(const BDet* desc, int ndesc, int64_t vblocks, size_t lds,
                               uint8_t* ws, hipStream_t st) {
  if (vblocks < 1) return hipSuccess;
  if (vblocks > kMaxGridBlocks) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((det_ll_batch_kernel<N>), dim3((unsigned)vblocks), dim3(kDetBlock), lds, st,
                     desc, ndesc, vblocks, ws);
  return hipGetLastError();
}

template <int N, int GL>
hipError_t det_fused_launch(const FusedDetArgs& f, hipStream_t st) {
  const int64_t rtiles = (f.R + f.Q - 1) / f.Q;
  const int64_t jtiles = (fused_jrange(f.N0, f.m0) + f.S - 1) / f.S;
  const size_t lds = fused_tile_words(N, GL, f.m0, f.Q) * sizeof(uint32_t);
  const dim3 g((unsigned)(rtiles * jtiles), (unsigned)f.pn);
  if (fused_paired(f.m0) && fused_pair_terms(f.m0) == 2)
    hipLaunchKernelGGL((det_fused_pair_kernel<N, GL, 2>), g, dim3(kDetBlock), lds, st, f.pre,
                       f.detv, f.denv, f.R, f.N0, f.m0, f.Q, f.S, f.tw0, f.tw_stride, f.pcs,
                       f.zero, f.slot, f.nslot, f.fixup, f.Rout, f.seg, f.off1, f.off2);
  else if (fused_paired(f.m0))
    hipLaunchKernelGGL((det_fused_pair_kernel<N, GL, 3>), g, dim3(kDetBlock), lds, st, f.pre,
                       f.detv, f.denv, f.R, f.N0, f.m0, f.Q, f.S, f.tw0, f.tw_stride, f.pcs,
                       f.zero, f.slot, f.nslot, f.fixup, f.Rout, f.seg, f.off1, f.off2);
  else
    hipLaunchKernelGGL((det_fused_kernel<N, GL>), g, dim3(kDetBlock), lds, st, f.pre, f.detv,
                       f.denv, f.R, f.N0, f.m0, f.Q, f.S, f.tw0, f.tw_stride, f.pcs, f.zero,
                       f.slot, f.nslot, f.fixup, f.Rout, f.seg, f.off1, f.off2);
  return hipGetLastError();
}

}  // namespace pd
