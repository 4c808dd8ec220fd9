// Elimination kernels of the DET stage, included by the det_part.hip translation units that
// instantiate them for each (order, lanes-per-matrix) pair (det.h declares the launchers).
#pragma once

#include <hip/hip_runtime.h>

#include "batch.h"
#include "det.h"
#include "modarith.h"

namespace pd {

constexpr int kDetBlock = 256;
constexpr int kEvalChunk = 8;  // entries per scheduling window of the fused evaluation

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

// The determinant of the matrix held by the lane group as a quotient num / den (Montgomery
// form): num = sign * pi_{n-1} (0 when some column has no pivot) and den = prod_{k<=n-3}
// pi_k^{n-k-2} (the representative of 1 for a singular matrix, so that den is never 0).
// The division is left to finalize_kernel, which inverts the denominators of many points
// with one exponentiation. Every lane of the group returns the pair; all lanes of the wave
// must call this together (lane shuffles).
struct DetFrac {
  uint32_t num, den;
};

template <int N, int GL>
__device__ __forceinline__ DetFrac eliminate(uint32_t (&a)[(N + GL - 1) / GL][N], uint32_t p,
                                             uint32_t pinv, uint32_t one) {
  constexpr int C = (N + GL - 1) / GL;
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
  DetFrac f;
  f.num = dead ? 0u : (flip ? negm(last, p) : last);
  f.den = dead ? one : Q;
  return f;
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

// Fused form: the last evaluation axis (the first variable, whose grid index j0 is the
// slowest) runs inside the elimination kernel, so the full evaluation tensor never exists.
// pre[pn][n*n][m0][R] holds every entry already evaluated along the other variables (R
// points) with its m0 coefficients in the first variable. A block stages the columns
// r0 .. r0+Q-1 of every nonzero entry in LDS as tile[m][q][e] (row stride NEP = n*n | 1, odd,
// so lanes reading different q hit different banks and the entry index is an immediate
// offset) and then, for S values of j0, each lane group rebuilds its matrix at the point
// (j0, r0 + q) by Horner's rule in w0^j0 (the evaluation of Section 2 along x1) and
// eliminates it. Point index = j0 R + r.
// One block's share of the fused kernel: prime `prime`, tile `bx` = (j-range, r-range).
template <int N, int GL>
__device__ __forceinline__ void det_fused_body(
    uint32_t* tile, const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv,
    uint32_t* __restrict__ denv, int64_t R,
    int N0, int m0, int Q, int S, const uint32_t* __restrict__ tw0, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero, int prime, int64_t bx) {
  constexpr int C = (N + GL - 1) / GL;
  constexpr int NE = N * N;
  constexpr int NEP = NE | 1;
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv, one = pcs[prime].r1;
  const int64_t rtiles = (R + Q - 1) / Q;
  const int64_t r0 = (bx % rtiles) * Q;
  const int jbase = (int)(bx / rtiles) * S;
  const uint32_t* src = pre + (int64_t)prime * NE * m0 * R;

  const int mq = m0 * Q;
  for (int idx = threadIdx.x; idx < NE * mq; idx += kDetBlock) {
    const int e = idx / mq;
    const int rem = idx - e * mq;  // = m Q + q
    const int q = rem % Q;
    const int m = rem / Q;
    uint32_t v = 0u;
    if (!(zero && zero[e]) && r0 + q < R) v = src[((int64_t)e * m0 + m) * R + r0 + q];
    tile[rem * NEP + e] = v;
  }
  __syncthreads();

  const int t = (int)(threadIdx.x % GL);
  const int slot = (int)(threadIdx.x / GL);
  const int q = slot % Q;
  const int J = (kDetBlock / GL) / Q;
  const int jj = slot / Q;
  const bool qvalid = r0 + q < R;
  const uint32_t* w0 = tw0 + (int64_t)prime * tw_stride;
  // column offset of the lane within its slot, clamped for the padded columns of the last
  // slot (their registers are zeroed after the evaluation)
  const int tl = t < N - (C - 1) * GL ? t : N - 1 - (C - 1) * GL;
  const int dl = tl - t;

  for (int j = jbase; j < jbase + S && j < N0; j += J) {
    const int j0 = j + jj;
    const bool valid = qvalid && j0 < N0 && j0 < jbase + S;
    const int j0c = j0 < N0 ? j0 : N0 - 1;
    uint32_t a[C][N];
    // a[c][i] = sum_{m < m0} x_m w0^{m j0}, two terms per reduction (mm2). With m0 even the
    // constant term pairs with x_1 (its factor is R mod p, the representative of 1); with
    // m0 odd it stands alone. The loop over m is uniform and sits outside the unrolled
    // loops over the entries held by the lane.
    int mstart;
    if ((m0 & 1) == 0) {
      const uint32_t w1 = w0[j0c & (N0 - 1)];
      const uint32_t* r0w = tile + q * NEP + t;
      const uint32_t* r1w = r0w + Q * NEP;
#pragma unroll
      for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const int off = i * N + c * GL + (c == C - 1 ? dl : 0);
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
        for (int i = 0; i < N; ++i) a[c][i] = r0w[i * N + c * GL + (c == C - 1 ? dl : 0)];
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
          const int off = i * N + c * GL + (c == C - 1 ? dl : 0);
          a[c][i] = addm(a[c][i], mm2(ra[off], wa, rb[off], wb, p, pinv), p);
          // bound the scheduler's window so that the LDS reads (one register each) are
          // not all hoisted ahead of the arithmetic
          if ((c * N + i) % kEvalChunk == kEvalChunk - 1) __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    if constexpr (C * GL > N) {
      if ((C - 1) * GL + t >= N) {
#pragma unroll
        for (int i = 0; i < N; ++i) a[C - 1][i] = 0u;
      }
    }
    const DetFrac d = eliminate<N, GL>(a, p, pinv, one);
    if (valid && t == 0) {
      const int64_t o = (int64_t)prime * N0 * R + (int64_t)j0 * R + r0 + q;
      detv[o] = d.num;
      denv[o] = d.den;
    }
  }
}

template <int N, int GL>
__global__ __launch_bounds__(kDetBlock) void det_fused_kernel(
    const uint32_t* __restrict__ pre, uint32_t* __restrict__ detv, uint32_t* __restrict__ denv,
    int64_t R, int N0, int m0, int Q, int S, const uint32_t* __restrict__ tw0, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero) {
  extern __shared__ uint32_t tile[];  // [m0][Q][n*n | 1]
  det_fused_body<N, GL>(tile, pre, detv, denv, R, N0, m0, Q, S, tw0, tw_stride, pcs, zero,
                        blockIdx.y, blockIdx.x);
}

// Batched form: blocks walk the virtual blocks of every matrix of this order in the launch;
// virtual block vb of matrix d is (prime, tile) = divmod(vb - block0, rtiles * jtiles).
template <int N, int GL>
__global__ __launch_bounds__(kDetBlock) void det_fused_batch_kernel(
    const BDet* __restrict__ desc, int ndesc, int64_t vblocks, uint8_t* __restrict__ ws) {
  extern __shared__ uint32_t tile[];
  for (int64_t vb = blockIdx.x; vb < vblocks; vb += gridDim.x) {
    const BDet& d = desc[find_desc(desc, ndesc, vb)];
    const int64_t local = vb - d.block0;
    const int64_t per_prime = d.rtiles * d.jtiles;
    const int prime = (int)(local / per_prime);
    det_fused_body<N, GL>(tile, (const uint32_t*)(ws + d.pre_off), (uint32_t*)(ws + d.detv_off),
                          (uint32_t*)(ws + d.den_off), d.R, d.N0, d.m0, d.Q, d.S, d.tw0,
                          d.tw_stride, d.pc, d.zero, prime,
                          local - (int64_t)prime * per_prime);
    __syncthreads();  // the next virtual block refills the tile
  }
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
                                  uint8_t* ws, hipStream_t st) {
  const int64_t grid = vblocks < kPersistentBlocks ? vblocks : kPersistentBlocks;
  hipLaunchKernelGGL((det_fused_batch_kernel<N, GL>), dim3((unsigned)(grid < 1 ? 1 : grid)),
                     dim3(kDetBlock), lds, st, desc, ndesc, vblocks, ws);
  return hipGetLastError();
}

template <int N, int GL>
hipError_t det_fused_launch(const FusedDetArgs& f, hipStream_t st) {
  const int64_t rtiles = (f.R + f.Q - 1) / f.Q;
  const int64_t jtiles = (f.N0 + f.S - 1) / f.S;
  const size_t lds = (size_t)((N * N) | 1) * f.m0 * f.Q * sizeof(uint32_t);
  hipLaunchKernelGGL((det_fused_kernel<N, GL>), dim3((unsigned)(rtiles * jtiles), (unsigned)f.pn),
                     dim3(kDetBlock), lds, st, f.pre, f.detv, f.denv, f.R, f.N0, f.m0, f.Q, f.S, f.tw0,
                     f.tw_stride, f.pcs, f.zero);
  return hipGetLastError();
}

}  // namespace pd
