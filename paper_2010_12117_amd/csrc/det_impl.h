// Elimination kernel of the DET stage, included by the det_part.hip translation units that
// instantiate it for each (order, lanes-per-matrix) pair (det.h declares the launchers).
#pragma once

#include <hip/hip_runtime.h>

#include "det.h"
#include "modarith.h"

namespace pd {

constexpr int kDetBlock = 256;

// ------------------------------------------------------------------------------------
// S3: determinant of the n x n matrix at every (prime, grid point).
//
// Division-free condensation (Chio's rule, the condensation the paper adopts in its
// DET step, Section 3.2): with pivot pi = A[k][k], every later row becomes
//   A[i][j] <- pi A[i][j] - A[i][k] A[k][j]   (j > k),
// which multiplies the determinant by pi once per updated row. After n - 1 steps the
// pivots pi_0..pi_{n-1} are the diagonal of a triangular matrix, so
//   det = sign * pi_{n-1} / prod_{k <= n-3} pi_k^{n-k-2},
// and the denominator is the product of the prefix products e_j = pi_0 .. pi_j for
// j <= n-3. One inverse (Fermat) per determinant replaces one per step. The pivot is the
// first nonzero entry scanning down column k; each exchange flips the sign; a column with
// no pivot gives determinant 0. Each update is one reduction of two products (mm2).
//
// Mapping: GL lanes cooperate on one matrix (GL = 1: one matrix per lane). Lane t of a
// group holds columns t, t + GL, t + 2 GL, ... of all n rows in registers (a[c][i] is
// A[i][c GL + t]), so every index below is static after unrolling. The owner of column k
// (lane k mod GL) finds the pivot row and broadcasts the row index, the pivot and the
// multipliers to its group with lane shuffles; row exchanges are register selects.
// ------------------------------------------------------------------------------------
template <int GL>
__device__ __forceinline__ uint32_t bcast(uint32_t v, int src) {
  if constexpr (GL == 1) {
    return v;
  } else {
    return (uint32_t)__shfl((int)v, src, GL);
  }
}

template <int N, int GL>
__global__ __launch_bounds__(kDetBlock) void det_kernel(const uint32_t* __restrict__ eval,
                                                     uint32_t* __restrict__ detv, int64_t npts,
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

  uint32_t flip = 0;
  bool dead = false;
  uint32_t e = one, Q = one;
#pragma unroll
  for (int k = 0; k < N - 1; ++k) {
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
    const uint32_t piv = bcast<GL>(a[s][k], o);
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const uint32_t mi = p - bcast<GL>(a[s][i], o);  // -A[i][k]; p stands for 0
#pragma unroll
      for (int c = s; c < C; ++c) a[c][i] = mm2(piv, a[c][i], mi, a[c][k], p, pinv);
    }
    if (k <= N - 3) {
      e = mm(e, piv, p, pinv);
      Q = mm(Q, e, p, pinv);
    }
  }
  constexpr int sl = (N - 1) / GL, ol = (N - 1) % GL;
  const uint32_t last = bcast<GL>(a[sl][N - 1], ol);
  dead = dead || (last == 0u);
  uint32_t d = mm(last, minv(Q, one, p, pinv), p, pinv);
  if (flip) d = negm(d, p);
  if (dead) d = 0u;
  if (valid && t == 0) detv[(int64_t)prime * npts + pt] = d;
}

template <int N, int GL>
hipError_t det_launch(const uint32_t* eval, uint32_t* detv, int64_t npts, int pn,
                      const PrimeConst* pcs, hipStream_t st) {
  constexpr int per_block = kDetBlock / GL;
  const int64_t bx = (npts + per_block - 1) / per_block;
  hipLaunchKernelGGL((det_kernel<N, GL>), dim3((unsigned)bx, (unsigned)pn), dim3(kDetBlock), 0, st,
                     eval, detv, npts, pcs);
  return hipGetLastError();
}

}  // namespace pd
