// HIP kernels for gfx950 of the modular determinant (Wei & Chen, arXiv 2010.12117,
// Algorithm 1): reduction of the integer coefficients, evaluation on the grid of roots of
// unity (the FFT stage), interpolation (the IFFT stage) and mixed-radix reconstruction (the
// CRT stage); the elimination (the DET stage) is in det_impl.h.
//
// Each stage is a device-side body shared by a single-matrix kernel (parameters as kernel
// arguments) and a batched kernel (parameters from a per-matrix descriptor table, batch.h).
// Every value below is a Montgomery representative (modarith.h) until the reconstruction.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <utility>

#include "batch.h"
#include "det.h"
#include "kernels.h"
#include "modarith.h"

namespace pd {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t work, int per_block = kBlock) {
  int64_t b = (work + per_block - 1) / per_block;
  return (unsigned)(b < 1 ? 1 : b);
}

inline unsigned persistent_grid(int64_t vblocks) {
  return (unsigned)(vblocks < kPersistentBlocks ? (vblocks < 1 ? 1 : vblocks) : kPersistentBlocks);
}

// ------------------------------------------------------------------------------------
// S1: int64 coefficient -> representative of (c mod p) for every prime.
// |c| = hi 2^32 + lo with hi <= 2^31, so c~ = mm(hi, R^3) + mm(lo, R^2), negated for c < 0.
// The residues are laid out by slot: slot u holds input entry slot_src[u] (the entries in
// elimination row order, or only the distinct nonzero ones).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t reduce_coeff(int64_t c, uint32_t p, uint32_t pinv,
                                                 uint32_t r2, uint32_t r3) {
  const bool neg = c < 0;
  const uint64_t a = neg ? (uint64_t)(-(c + 1)) + 1u : (uint64_t)c;
  const uint32_t hi = (uint32_t)(a >> 32), lo = (uint32_t)a;
  const uint32_t r = addm(mm(hi, r3, p, pinv), mm(lo, r2, p, pinv), p);
  return neg ? negm(r, p) : r;
}

__device__ __forceinline__ void reduce_body(const int64_t* __restrict__ in,
                                            uint32_t* __restrict__ out, int64_t i, int64_t count,
                                            int pn, int64_t T,
                                            const int32_t* __restrict__ slot_src,
                                            const PrimeConst* __restrict__ pcs) {
  const int64_t u = i / T;
  const int64_t c = in[(int64_t)slot_src[u] * T + (i - u * T)];
  for (int q = 0; q < pn; ++q) {
    const PrimeConst P = pcs[q];
    out[(int64_t)q * count + i] = reduce_coeff(c, P.p, P.pinv, P.r2, P.r3);
  }
}

__global__ __launch_bounds__(kBlock) void reduce_kernel(const int64_t* __restrict__ in,
                                                        uint32_t* __restrict__ out,
                                                        int64_t count, int pn, int64_t T,
                                                        const int32_t* __restrict__ slot_src,
                                                        const PrimeConst* __restrict__ pcs) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) reduce_body(in, out, i, count, pn, T, slot_src, pcs);
}

__global__ __launch_bounds__(kBlock) void reduce_batch_kernel(
    const BReduce* __restrict__ desc, int ndesc, int64_t vblocks, const int64_t* __restrict__ coeffs,
    const int64_t* __restrict__ coeff_offsets, uint8_t* __restrict__ ws) {
  for (int64_t vb = blockIdx.x; vb < vblocks; vb += gridDim.x) {
    const BReduce& d = desc[find_desc(desc, ndesc, vb)];
    const int64_t i = (vb - d.block0) * kBlock + threadIdx.x;
    if (i < d.count) {
      reduce_body(coeffs + coeff_offsets[d.mat], (uint32_t*)(ws + d.res_off), i, d.count, d.pn,
                  d.T, d.slot_src, d.pc);
    }
  }
}

// ------------------------------------------------------------------------------------
// S2: evaluation along one variable. For every line (b, o, q) of
//   in  [B][outer][m][inner]   (coefficients of x_v^e, e < m, other axes as given)
//   out [B][outer][Nv][inner]  out[j] = sum_e in[e] w_v^{e j}
// the values at the Nv-th roots of unity (the DFT over Z/pZ of Section 2, restricted to the
// m nonzero leading coefficients of the zero-padded line). b = prime * nent + slot.
// With m >= 2 the outputs come in pairs: since w^{Nv/2} = -1, out[j] = E + O and
// out[j + Nv/2] = E - O, with E the even terms and O the odd terms at j, so a thread takes
// j in [0, Nv/2) and half the products. A thread computes JC consecutive j of one line;
// consecutive lanes take consecutive q (coalesced when inner >= 64) and, for small inner,
// consecutive j-chunks. M >= m bounds the coefficients held in registers; terms e >= m are
// skipped (a uniform test). Lines of structurally zero entries are written as zeros only when
// the output is read without the zero flags (write_zero: the full evaluation tensor).
// UJ (inner >= 64, a multiple of the wave): the 64 lanes of a wave share the line's position
// r and so j, the prime and the entry; they are taken from the wave's first index, which lets
// the twiddle, constant and zero-flag loads be scalar.
// ------------------------------------------------------------------------------------
//
// A slab of the grid (capped plans, one prime's pass over variable 1 in parts): the output
// holds Nout < Nv values per line, the points jbase + j and, paired, jbase + j + Nv/2 for
// j in [0, Nout/2), stored at j and j + Nout/2. jbase = 0 and Nout = Nv give the whole line.
//
// RED (the first pass, over the last variable: inner = 1): the line's coefficients are read
// from the integer input and reduced as they load (S1 in the same launch): slot `entry` is
// input entry slot_src[entry], whose T = outer * m coefficients start at slot_src[entry] * T.
// The line's first thread also stores the residues where S1 puts them (`res`, laid out like
// `in`), so that every later stage can be run again from them.
template <int M, bool UJ, bool EXACT, bool RED = false>
__device__ __forceinline__ void expand_body(
    const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t idx, int64_t B,
    int64_t outer, int m, int Nv, int JC, int64_t inner, int64_t nent,
    const uint32_t* __restrict__ tw, int64_t tw_stride, const PrimeConst* __restrict__ pcs,
    const uint8_t* __restrict__ zero, bool write_zero, int jbase, int Nout, int64_t idx_wave,
    const int64_t* __restrict__ coeffs = nullptr, const int32_t* __restrict__ slot_src = nullptr,
    uint32_t* __restrict__ res = nullptr) {
  const bool paired = expand_paired(Nv, m);
  const int NJ = paired ? Nout / 2 : Nout;
  const int nJB = NJ / JC;
  if (idx >= B * outer * nJB * inner) return;
  // inner and nJB are powers of two
  const int li = __builtin_ctzll((unsigned long long)inner);
  const int64_t q = idx & (inner - 1);
  int64_t r;
  if constexpr (UJ) {
    r = idx_wave >> li;  // the wave's first index (uniform across the wave)
  } else {
    r = idx >> li;
  }
  const int jb = (int)(r & (nJB - 1));
  const int64_t bo = r >> __builtin_ctz((unsigned)nJB);
  const int64_t b = bo / outer;
  const int prime = (int)(b / nent);
  const int64_t entry = b - (int64_t)prime * nent;
  uint32_t* dst = out + bo * Nout * inner + q;
  const int j0 = jb * JC;
  if (zero && zero[entry]) {
    if (write_zero) {
      for (int j = j0; j < j0 + JC; ++j) {
        dst[(int64_t)j * inner] = 0u;
        if (paired) dst[(int64_t)(j + NJ) * inner] = 0u;
      }
    }
    return;
  }
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv;
  const uint32_t* w = tw + (int64_t)prime * tw_stride;
  uint32_t x[M];
  if constexpr (RED) {
    const uint32_t r2 = pcs[prime].r2, r3 = pcs[prime].r3;
    const int64_t* src = coeffs + (int64_t)slot_src[entry] * outer * m + (bo - b * outer) * m;
#pragma unroll
    for (int e = 0; e < M; ++e) x[e] = e < m ? reduce_coeff(src[e], p, pinv, r2, r3) : 0u;
    if (jb == 0) {
#pragma unroll
      for (int e = 0; e < M; ++e)
        if (e < m) res[bo * m + e] = x[e];
    }
  } else {
    const uint32_t* src = in + bo * m * inner + q;
#pragma unroll
    for (int e = 0; e < M; ++e) x[e] = e < m ? src[(int64_t)e * inner] : 0u;
  }
  const int mask = Nv - 1;
  if (paired) {
    // unrolled so that the twiddle loads of several points are in flight together
#pragma unroll 4
    for (int j = j0; j < j0 + JC; ++j) {
      // E = x0 + (x2 w^2j + x4 w^4j) + ..., O = (x1 w^j + x3 w^3j) + ..., two per reduction
      // With EXACT (m == M) the loop over e has no runtime condition, and the twiddle loads
      // of the unrolled points are issued together. Otherwise the terms past m - 1 (x[e] = 0,
      // adding nothing) are skipped.
      const int jg = jbase + j;  // the point's index on the whole line
      uint32_t E = x[0], O = 0u;
#pragma unroll
      for (int e = 2; e < M; e += 4) {
        if (EXACT || e < m) {
          if (e + 2 < M && (EXACT || e + 2 < m))
            E = addm(E, mm2(x[e], w[(e * jg) & mask], x[e + 2], w[((e + 2) * jg) & mask], p, pinv), p);
          else
            E = addm(E, mm(x[e], w[(e * jg) & mask], p, pinv), p);
        }
      }
#pragma unroll
      for (int e = 1; e < M; e += 4) {
        if (EXACT || e < m) {
          if (e + 2 < M && (EXACT || e + 2 < m))
            O = addm(O, mm2(x[e], w[(e * jg) & mask], x[e + 2], w[((e + 2) * jg) & mask], p, pinv), p);
          else
            O = addm(O, mm(x[e], w[(e * jg) & mask], p, pinv), p);
        }
      }
      // streaming stores: each output is written once and read by the next launch (at the
      // 12 x 12 trivariate workload the pre-tensor pass took 12.5 against 13.8 us)
      __builtin_nontemporal_store(addm(E, O, p), &dst[(int64_t)j * inner]);
      __builtin_nontemporal_store(subm(E, O, p), &dst[(int64_t)(j + NJ) * inner]);
    }
  } else {
    // m == 1: the line is its constant term at every point
    for (int j = j0; j < j0 + JC; ++j) dst[(int64_t)j * inner] = x[0];
  }
}

// The first pass with the reduction of the integer coefficients (RED in expand_body).
template <int M>
__global__ __launch_bounds__(kBlock) void expand_reduce_kernel(
    const int64_t* __restrict__ coeffs, const int32_t* __restrict__ slot_src,
    uint32_t* __restrict__ res, uint32_t* __restrict__ out, int64_t B, int64_t outer, int m,
    int Nv, int JC, int64_t nent, const uint32_t* __restrict__ tw, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero, bool write_zero) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  expand_body<M, false, (M <= 8), true>(nullptr, out, idx, B, outer, m, Nv, JC, 1, nent, tw,
                                        tw_stride, pcs, zero, write_zero, 0, Nv, idx, coeffs,
                                        slot_src, res);
}

template <int M, bool UJ>
__global__ __launch_bounds__(kBlock) void expand_kernel(
    const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t B, int64_t outer,
    int m, int Nv, int JC, int64_t inner, int64_t nent, const uint32_t* __restrict__ tw,
    int64_t tw_stride, const PrimeConst* __restrict__ pcs, const uint8_t* __restrict__ zero,
    bool write_zero, int jbase, int Nout) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t idx_wave =
      (int64_t)blockIdx.x * kBlock + 64 * __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // the single-matrix launches pick M = m up to 8 (launch_expand)
  expand_body<M, UJ, (M <= 8)>(in, out, idx, B, outer, m, Nv, JC, inner, nent, tw, tw_stride, pcs, zero,
                     write_zero, jbase, Nout, idx_wave);
}

// One virtual block of the batched pass, with the coefficient count M = d.m known at compile
// time (the loop over the terms then has no runtime condition) and, for d.inner >= 64, the
// wave-uniform form (UJ); both are uniform per virtual block.
template <int M>
__device__ __forceinline__ void expand_batch_vb(const BExpand& d, int64_t local, uint8_t* ws) {
  const int64_t idx = local * kBlock + threadIdx.x;
  const int64_t idx_wave = local * kBlock + 64 * __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t* in = (const uint32_t*)(ws + d.in_off);
  uint32_t* out = (uint32_t*)(ws + d.out_off);
  if (d.inner >= 64)
    expand_body<M, true, true>(in, out, idx, d.B, d.outer, d.m, d.Nv, d.JC, d.inner, d.nent, d.tw,
                               d.tw_stride, d.pc, d.zero, false, 0, d.Nv, idx_wave);
  else
    expand_body<M, false, true>(in, out, idx, d.B, d.outer, d.m, d.Nv, d.JC, d.inner, d.nent,
                                d.tw, d.tw_stride, d.pc, d.zero, false, 0, d.Nv, idx_wave);
}

__global__ __launch_bounds__(kBlock) void expand_batch_kernel(const BExpand* __restrict__ desc,
                                                              int ndesc, int64_t vblocks,
                                                              uint8_t* __restrict__ ws) {
  static_assert(kBatchMaxM == 8, "the dispatch below covers 1..8 coefficients");
  for (int64_t vb = blockIdx.x; vb < vblocks; vb += gridDim.x) {
    const BExpand& d = desc[find_desc(desc, ndesc, vb)];
    const int64_t local = vb - d.block0;
    switch (d.m) {
      case 1: expand_batch_vb<1>(d, local, ws); break;
      case 2: expand_batch_vb<2>(d, local, ws); break;
      case 3: expand_batch_vb<3>(d, local, ws); break;
      case 4: expand_batch_vb<4>(d, local, ws); break;
      case 5: expand_batch_vb<5>(d, local, ws); break;
      case 6: expand_batch_vb<6>(d, local, ws); break;
      case 7: expand_batch_vb<7>(d, local, ws); break;
      default: expand_batch_vb<8>(d, local, ws); break;
    }
  }
}

// ------------------------------------------------------------------------------------
// S3 (end): det = num / den at every point, written to quot (which may be detv itself). A
// thread takes kFinalPoints points of one prime, chunks apart (so that a wave's loads and
// stores are contiguous), and inverts their denominators together (Montgomery's simultaneous
// inversion: prefix products, one Fermat inverse, then back-substitution), which costs one
// exponentiation per kFinalPoints points instead of one per point. Every den is nonzero.
// ------------------------------------------------------------------------------------
constexpr int kFinalPoints = 8;

__device__ __forceinline__ void finalize_body(const uint32_t* detv,
                                              const uint32_t* __restrict__ denv, uint32_t* quot,
                                              int64_t t, int64_t G,
                                              const PrimeConst* __restrict__ pcs) {
  const int64_t chunks = (G + kFinalPoints - 1) / kFinalPoints;
  const int prime = (int)(t / chunks);
  const int64_t c = t - (int64_t)prime * chunks;  // points c, c + chunks, c + 2 chunks, ...
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv, one = pcs[prime].r1;
  const uint32_t* num = detv + (int64_t)prime * G + c;
  uint32_t* q = quot + (int64_t)prime * G + c;
  const uint32_t* den = denv + (int64_t)prime * G + c;
  uint32_t d[kFinalPoints], pre[kFinalPoints];
  uint32_t acc = one;
#pragma unroll
  for (int i = 0; i < kFinalPoints; ++i) {
    d[i] = (c + i * chunks < G) ? den[i * chunks] : one;
    pre[i] = acc;  // product of the denominators before i
    acc = mm(acc, d[i], p, pinv);
  }
  uint32_t inv = minv(acc, one, p, pinv);  // inverse of the product of all
#pragma unroll
  for (int i = kFinalPoints - 1; i >= 0; --i) {
    const uint32_t di = mm(inv, pre[i], p, pinv);  // 1 / d[i]
    inv = mm(inv, d[i], p, pinv);                   // 1 / (d[0] .. d[i-1])
    if (c + i * chunks < G) q[i * chunks] = mm(num[i * chunks], di, p, pinv);
  }
}

__global__ __launch_bounds__(kBlock) void finalize_kernel(const uint32_t* detv,
                                                          const uint32_t* __restrict__ denv,
                                                          uint32_t* quot, int64_t G, int pn,
                                                          const PrimeConst* __restrict__ pcs) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < (int64_t)pn * ((G + kFinalPoints - 1) / kFinalPoints))
    finalize_body(detv, denv, quot, t, G, pcs);
}


// ------------------------------------------------------------------------------------
// S4: interpolation along one variable (inverse DFT: opposite sign in the exponent; the
// 1/N factor is applied once in the reconstruction). A block loads a tile of W lines of
// length Nv into LDS in bit-reversed order (with the Nv/2 twiddles it needs after it), runs
// log2 Nv radix-2 decimation-in-time stages and writes the first D_v + 1 outputs of each line:
//   in  [pn][outer][Nv][inner] -> out [pn][outer][Dv1][inner];  tile index = prime * tiles + t.
// ------------------------------------------------------------------------------------
//
// With `den` set (the first pass, over the points' numerators and denominators), the load
// also takes the division of the finalize step: each thread inverts the denominators of
// kFuseBatch points with one exponentiation (simultaneous inversion) and puts num / den in the
// tile. The numerators and denominators are left as they are (every stage reads only earlier
// stages' outputs, so a stage can be run again).

__device__ __forceinline__ void intt_body(uint32_t* tile, const uint32_t* __restrict__ in,
                                          uint32_t* __restrict__ out, int64_t block,
                                          int64_t outer, int Nv, int logN, int64_t inner, int Dv1,
                                          int W, const uint32_t* __restrict__ itw,
                                          int64_t tw_stride, const PrimeConst* __restrict__ pcs,
                                          const uint32_t* __restrict__ den = nullptr) {
  const int64_t lines = outer * inner;
  const int64_t tiles_per_prime = (lines + W - 1) / W;
  const int prime = (int)(block / tiles_per_prime);
  const int64_t line0 = (block - (int64_t)prime * tiles_per_prime) * W;
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv;
  const uint32_t* w = itw + (int64_t)prime * tw_stride;
  const uint32_t* src = in + (int64_t)prime * outer * Nv * inner;
  uint32_t* dst = out + (int64_t)prime * outer * Dv1 * inner;
  const int nW = (int)((lines - line0) < W ? (lines - line0) : W);
  const int total = Nv * W;
  // W, Nv and inner are powers of two: the index arithmetic below is shifts and masks
  const int lW = __builtin_ctz((unsigned)W);
  const int lI = __builtin_ctzll((unsigned long long)inner);
  const int64_t imask = inner - 1;
  // twiddles w^t, t < Nv/2, after the tile (the stages read w^{pos N / 2^s} with
  // pos < 2^{s-1})
  uint32_t* twl = tile + total;
  for (int t = threadIdx.x; t < Nv / 2; t += kBlock) twl[t] = w[t];
  // load: element j of local line l goes to tile[brev(j) * W + l]
  if (den == nullptr) {
    for (int idx = threadIdx.x; idx < total; idx += kBlock) {
      int j, l;
      if (inner >= W) { j = idx >> lW; l = idx & (W - 1); } else { l = idx >> logN; j = idx & (Nv - 1); }
      uint32_t v = 0u;
      if (l < nW) {
        const int64_t line = line0 + l;
        const int64_t o = line >> lI, q = line & imask;
        v = src[(o * Nv + j) * inner + q];
      }
      const int rj = logN ? (int)(__brev((unsigned)j) >> (32 - logN)) : 0;
      tile[rj * W + l] = v;
    }
  } else {
    const uint32_t one = pcs[prime].r1;
    const uint32_t* dsrc = den + (int64_t)prime * outer * Nv * inner;
    for (int base = threadIdx.x; base < total; base += kFuseBatch * kBlock) {
      uint32_t v[kFuseBatch], d[kFuseBatch], pre[kFuseBatch];
      int64_t gi[kFuseBatch];
      int ti[kFuseBatch];
      uint32_t acc = one;
#pragma unroll
      for (int i = 0; i < kFuseBatch; ++i) {
        const int idx = base + i * kBlock;
        int j, l;
        if (inner >= W) { j = idx >> lW; l = idx & (W - 1); } else { l = idx >> logN; j = idx & (Nv - 1); }
        const int rj = logN ? (int)(__brev((unsigned)j) >> (32 - logN)) : 0;
        ti[i] = idx < total ? rj * W + l : -1;
        gi[i] = -1;
        v[i] = 0u;
        d[i] = one;
        if (idx < total && l < nW) {
          const int64_t line = line0 + l;
          const int64_t o = line >> lI, q = line & imask;
          gi[i] = (o * Nv + j) * inner + q;
          v[i] = src[gi[i]];
          d[i] = dsrc[gi[i]];
        }
        pre[i] = acc;  // product of the denominators before i
        acc = mm(acc, d[i], p, pinv);
      }
      uint32_t inv = minv(acc, one, p, pinv);  // inverse of the product of all
#pragma unroll
      for (int i = kFuseBatch - 1; i >= 0; --i) {
        const uint32_t di = mm(inv, pre[i], p, pinv);  // 1 / d[i]
        inv = mm(inv, d[i], p, pinv);                   // 1 / (d[0] .. d[i-1])
        if (ti[i] >= 0) tile[ti[i]] = mm(v[i], di, p, pinv);
      }
    }
  }
  __syncthreads();
  int s = 1;
  // Two stages per pass over the tile while two remain: a thread takes the four elements
  // i0 + {0, h, 2h, 3h} (h = 2^{s-1}) that stages s and s+1 combine among themselves. Stage s
  // pairs (0, h) and (2h, 3h) with the twiddle w^{pos N / 2^s}; stage s+1 pairs (0, 2h) with
  // w^{pos N / 2^{s+1}} and (h, 3h) with w^{(pos + h) N / 2^{s+1}}. Half the barriers.
  for (; s + 1 <= logN; s += 2) {
    const int h = 1 << (s - 1);
    const int st1 = Nv >> s, st2 = Nv >> (s + 1);
    for (int bi = threadIdx.x; bi < (Nv / 4) * W; bi += kBlock) {
      const int l = bi & (W - 1);
      const int b = bi >> lW;
      const int grp = b >> (s - 1), pos = b & (h - 1);
      const int i0 = grp * 4 * h + pos;
      uint32_t* e0 = tile + i0 * W + l;
      const uint32_t x0 = e0[0], x1 = e0[h * W], x2 = e0[2 * h * W], x3 = e0[3 * h * W];
      const uint32_t t1 = twl[pos * st1];
      const uint32_t v1 = mm(x1, t1, p, pinv), v3 = mm(x3, t1, p, pinv);
      const uint32_t u0 = addm(x0, v1, p), u1 = subm(x0, v1, p);
      const uint32_t u2 = addm(x2, v3, p), u3 = subm(x2, v3, p);
      const uint32_t y2 = mm(u2, twl[pos * st2], p, pinv);
      const uint32_t y3 = mm(u3, twl[(pos + h) * st2], p, pinv);
      e0[0] = addm(u0, y2, p);
      e0[2 * h * W] = subm(u0, y2, p);
      e0[h * W] = addm(u1, y3, p);
      e0[3 * h * W] = subm(u1, y3, p);
    }
    __syncthreads();
  }
  for (; s <= logN; ++s) {  // the last stage when log2 Nv is odd
    const int half = 1 << (s - 1);
    const int stride = Nv >> s;  // twiddle index step: w^{pos * N / 2^s}
    for (int bi = threadIdx.x; bi < (Nv / 2) * W; bi += kBlock) {
      const int l = bi & (W - 1);
      const int b = bi >> lW;
      const int grp = b >> (s - 1), pos = b & (half - 1);
      const int i0 = grp * 2 * half + pos, i1 = i0 + half;
      const uint32_t u = tile[i0 * W + l];
      const uint32_t v = mm(tile[i1 * W + l], twl[pos * stride], p, pinv);
      tile[i0 * W + l] = addm(u, v, p);
      tile[i1 * W + l] = subm(u, v, p);
    }
    __syncthreads();
  }
  const int otot = Dv1 * W;
  for (int idx = threadIdx.x; idx < otot; idx += kBlock) {
    int e, l;
    if (inner >= W) { e = idx >> lW; l = idx & (W - 1); } else { l = idx / Dv1; e = idx - l * Dv1; }
    if (l < nW) {
      const int64_t line = line0 + l;
      const int64_t o = line >> lI, q = line & imask;
      dst[(o * Dv1 + e) * inner + q] = tile[e * W + l];
    }
  }
}

// ------------------------------------------------------------------------------------
// The same pass for lines of Nv = 8 M points (M = 4, 8, 16, 32) that run along a contiguous
// axis (inner >= 32), with the transform in registers (Cooley-Tukey, Nv = M x 8). A block
// takes 32 lines of one prime; thread (t, l), t < 8, l < 32, holds the points j = 8 i + t of
// line l (i < M), takes their M-point transform (root w^8), multiplies entry k1 by w^{t k1},
// and writes the entries to LDS; after one barrier it takes, for each k1 = t + 8 c < M, the
// 8-point transform (root w^M) of entry k1 of the eight threads of its line: outputs
// e = k1 + M k2. One LDS exchange and one barrier per pass, against log2(Nv)/2 barrier-
// separated stages in LDS (intt_body). With `den` the first pass divides as intt_body does
// (M points per thread share one exponentiation).
// ------------------------------------------------------------------------------------

// In-place M-point transform a[k] <- sum_i a[i] r^{i k}, r a primitive M-th root of unity, with
// rt[i] = r^i (i < M/2, Montgomery form): decimation in frequency, whose outputs come in
// bit-reversed order, which the static index permutation at the end undoes.
template <int M>
__device__ __forceinline__ void dft_reg(uint32_t (&a)[M], const uint32_t (&rt)[M / 2],
                                        uint32_t p, uint32_t pinv) {
#pragma unroll
  for (int span = M / 2; span >= 1; span >>= 1) {
    const int step = (M / 2) / span;  // the twiddle of position i is r^{i step}
#pragma unroll
    for (int blk = 0; blk < M; blk += 2 * span) {
#pragma unroll
      for (int i = 0; i < span; ++i) {
        const uint32_t u = a[blk + i], v = a[blk + i + span];
        a[blk + i] = addm(u, v, p);
        a[blk + i + span] = i == 0 ? subm(u, v, p) : mm(subm(u, v, p), rt[i * step], p, pinv);
      }
    }
  }
  uint32_t b[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    int r = 0;
#pragma unroll
    for (int bit = 1; bit < M; bit <<= 1) r = (r << 1) | ((k & bit) ? 1 : 0);
    b[k] = a[r];
  }
#pragma unroll
  for (int k = 0; k < M; ++k) a[k] = b[k];
}

template <int M>
__device__ __forceinline__ void intt_reg_body(uint32_t* xch, const uint32_t* __restrict__ in,
                                              uint32_t* __restrict__ out, int64_t block,
                                              int64_t outer, int64_t inner, int Dv1,
                                              const uint32_t* __restrict__ itw, int64_t tw_stride,
                                              const PrimeConst* __restrict__ pcs,
                                              const uint32_t* __restrict__ den) {
  constexpr int Nv = 8 * M;
  const int64_t lines = outer * inner;
  const int64_t tiles_per_prime = lines / kInttRegLines;  // inner >= 32: lines % 32 == 0
  const int prime = (int)(block / tiles_per_prime);
  const int64_t line0 = (block - (int64_t)prime * tiles_per_prime) * kInttRegLines;
  const int t = (int)(threadIdx.x >> 5), l = (int)(threadIdx.x & 31);
  const uint32_t p = pcs[prime].p, pinv = pcs[prime].pinv;
  const uint32_t* w = itw + (int64_t)prime * tw_stride;
  const int64_t line = line0 + l;
  const int lI = __builtin_ctzll((unsigned long long)inner);
  const int64_t o = line >> lI, q = line & (inner - 1);
  const int64_t base = (int64_t)prime * outer * Nv * inner + o * Nv * inner + q;
  uint32_t v[M];
#pragma unroll
  for (int i = 0; i < M; ++i) v[i] = in[base + (int64_t)(8 * i + t) * inner];
  uint32_t rin[M / 2];  // roots of the inner transform: w^{8 i}
#pragma unroll
  for (int i = 0; i < M / 2; ++i) rin[i] = w[8 * i];
  if (den) {
    const uint32_t one = pcs[prime].r1;
    uint32_t d[M], pre[M];
    uint32_t acc = one;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      d[i] = den[base + (int64_t)(8 * i + t) * inner];
      pre[i] = acc;  // product of the denominators before i
      acc = mm(acc, d[i], p, pinv);
    }
    uint32_t inv = minv(acc, one, p, pinv);  // inverse of the product of all
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
      const uint32_t di = mm(inv, pre[i], p, pinv);  // 1 / d[i]
      inv = mm(inv, d[i], p, pinv);
      v[i] = mm(v[i], di, p, pinv);
    }
  }
  dft_reg<M>(v, rin, p, pinv);  // over i: entry k1 of the inner transform (n2 = t)
#pragma unroll
  for (int k = 1; k < M; ++k) v[k] = mm(v[k], w[(t * k) & (Nv - 1)], p, pinv);
  // exchange: row (n2, k1) of 32 lines
#pragma unroll
  for (int k = 0; k < M; ++k) xch[(t * M + k) * kInttRegLines + l] = v[k];
  __syncthreads();
  const uint32_t rout[4] = {w[0], w[M], w[2 * M], w[3 * M]};  // the 8th roots w^{M j}
#pragma unroll
  for (int c = 0; c < (M + 7) / 8; ++c) {
    const int k1 = t + 8 * c;
    if (k1 < M) {
      uint32_t z[8];
#pragma unroll
      for (int n2 = 0; n2 < 8; ++n2) z[n2] = xch[(n2 * M + k1) * kInttRegLines + l];
      dft_reg<8>(z, rout, p, pinv);  // over n2: output e = k1 + M k2
      uint32_t* dst = out + (int64_t)prime * outer * Dv1 * inner + o * Dv1 * inner + q;
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) {
        const int e = k1 + M * k2;
        if (e < Dv1) dst[(int64_t)e * inner] = z[k2];
      }
    }
  }
}

// The register-form pass for Nv = 8 M (intt_reg_body); xch holds Nv x 32 words.
template <int M>
__global__ __launch_bounds__(kBlock) void intt_reg_kernel(
    const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t outer, int64_t inner,
    int Dv1, const uint32_t* __restrict__ itw, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint32_t* __restrict__ den) {
  __shared__ uint32_t xch[8 * M * kInttRegLines];
  intt_reg_body<M>(xch, in, out, blockIdx.x, outer, inner, Dv1, itw, tw_stride, pcs, den);
}

__global__ __launch_bounds__(kBlock) void intt_kernel(
    const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t outer, int Nv, int logN,
    int64_t inner, int Dv1, int W, const uint32_t* __restrict__ itw, int64_t tw_stride,
    const PrimeConst* __restrict__ pcs, const uint32_t* __restrict__ den) {
  extern __shared__ uint32_t tile[];  // [Nv][W]
  intt_body(tile, in, out, blockIdx.x, outer, Nv, logN, inner, Dv1, W, itw, tw_stride, pcs, den);
}

__global__ __launch_bounds__(kBlock) void intt_batch_kernel(const BIntt* __restrict__ desc,
                                                            int ndesc, int64_t vblocks,
                                                            uint8_t* __restrict__ ws) {
  extern __shared__ uint32_t tile[];
  for (int64_t vb = blockIdx.x; vb < vblocks; vb += gridDim.x) {
    const BIntt& d = desc[find_desc(desc, ndesc, vb)];
    const uint32_t* den = d.den_off >= 0 ? (const uint32_t*)(ws + d.den_off) : nullptr;
    const uint32_t* src = (const uint32_t*)(ws + d.in_off);
    uint32_t* dst = (uint32_t*)(ws + d.out_off);
    const int64_t b = vb - d.block0;
    if (d.reg == 4)
      intt_reg_body<4>(tile, src, dst, b, d.outer, d.inner, d.Dv1, d.itw, d.tw_stride, d.pc, den);
    else if (d.reg == 8)
      intt_reg_body<8>(tile, src, dst, b, d.outer, d.inner, d.Dv1, d.itw, d.tw_stride, d.pc, den);
    else if (d.reg == 16)
      intt_reg_body<16>(tile, src, dst, b, d.outer, d.inner, d.Dv1, d.itw, d.tw_stride, d.pc, den);
    else
      intt_body(tile, (const uint32_t*)(ws + d.in_off), (uint32_t*)(ws + d.out_off), vb - d.block0,
                d.outer, d.Nv, d.logN, d.inner, d.Dv1, d.W, d.itw, d.tw_stride, d.pc, den);
    __syncthreads();  // the next virtual block reuses the tile
  }
}

// ------------------------------------------------------------------------------------
// S5: mixed-radix conversion (Section 3.4, Algorithm 4; one lane per coefficient, as the
// paper parallelises over coefficients rather than digits). With x_i the residue mod p_i:
//   alpha_0 = x_0,  alpha_i = (x_i - sum_{j<i} alpha_j (p_0..p_{j-1} mod p_i)) c_i mod p_i,
//   c_i = (p_0..p_{i-1})^{-1} mod p_i,  X = sum_i alpha_i p_0..p_{i-1} (Horner, top down),
// then the symmetric range: X - M when X > (M-1)/2, written as L two's-complement limbs.
// ------------------------------------------------------------------------------------
template <int PN>
struct GarnerShared {
  uint32_t gw[PN * PN];
  uint32_t p[PN], pinv[PN], gc[PN], scale[PN], m[PN], h[PN];
};

template <int PN>
__device__ __forceinline__ void garner_load(GarnerShared<PN>& s, int pn, int L,
                                            const PrimeConst* __restrict__ pcs,
                                            const uint32_t* __restrict__ gw,
                                            const uint32_t* __restrict__ gc,
                                            const uint32_t* __restrict__ mlimbs,
                                            const uint32_t* __restrict__ hlimbs) {
  for (int i = threadIdx.x; i < pn * pn; i += kBlock) s.gw[(i / pn) * PN + i % pn] = gw[i];
  for (int i = threadIdx.x; i < pn; i += kBlock) {
    s.p[i] = pcs[i].p;
    s.pinv[i] = pcs[i].pinv;
    s.gc[i] = gc[i];
    s.scale[i] = pcs[i].scale;
  }
  for (int i = threadIdx.x; i < L; i += kBlock) {
    s.m[i] = mlimbs[i];
    s.h[i] = hlimbs[i];
  }
}

// Coefficient c from its residues r[i] (Montgomery form, i < pn), written as L limbs at out.
template <int PN>
__device__ __forceinline__ void garner_residues(const GarnerShared<PN>& s,
                                                const uint32_t (&r)[PN],
                                                uint32_t* __restrict__ out, int64_t c, int pn,
                                                int L) {
  uint32_t alpha[PN];
#pragma unroll
  for (int i = 0; i < PN; ++i) {
    if (i < pn) {
      const uint32_t p = s.p[i], pinv = s.pinv[i];
      // residue out of Montgomery form and divided by G (the inverse-DFT factor)
      const uint32_t x = mm(r[i], s.scale[i], p, pinv);
      uint32_t acc = 0u;
#pragma unroll
      for (int j = 0; j < PN; ++j) {
        if (j < i) acc = addm(acc, mm(alpha[j], s.gw[i * PN + j], p, pinv), p);
      }
      alpha[i] = mm(subm(x, acc, p), s.gc[i], p, pinv);
    } else {
      alpha[i] = 0u;
    }
  }
  // Horner: X = alpha_{pn-1}; X = X p_i + alpha_i for i = pn-2 .. 0
  uint32_t X[PN];
#pragma unroll
  for (int l = 0; l < PN; ++l) X[l] = 0u;
#pragma unroll
  for (int i = PN - 1; i >= 0; --i) {
    if (i < pn) {
      const uint32_t pi = (i == pn - 1) ? 0u : s.p[i];
      uint64_t carry = alpha[i];
#pragma unroll
      for (int l = 0; l < PN; ++l) {
        const uint64_t tt = (uint64_t)X[l] * pi + carry;
        X[l] = (uint32_t)tt;
        carry = tt >> 32;
      }
    }
  }
  // X > (M-1)/2 ?  compare from the top limb
  int cmp = 0;
#pragma unroll
  for (int l = PN - 1; l >= 0; --l) {
    if (l < L && cmp == 0) cmp = (X[l] > s.h[l]) ? 1 : (X[l] < s.h[l] ? -1 : 0);
  }
  if (cmp > 0) {
    uint32_t borrow = 0u;
#pragma unroll
    for (int l = 0; l < PN; ++l) {
      if (l < L) {
        const uint64_t d = (uint64_t)X[l] - s.m[l] - borrow;
        X[l] = (uint32_t)d;
        borrow = (uint32_t)(d >> 63);
      }
    }
  }
  uint32_t* o = out + c * L;
#pragma unroll
  for (int l = 0; l < PN; ++l) {
    if (l < L) o[l] = X[l];
  }
}

template <int PN>
__device__ __forceinline__ void garner_body(const GarnerShared<PN>& s,
                                            const uint32_t* __restrict__ coef,
                                            uint32_t* __restrict__ out, int64_t c, int64_t C,
                                            int pn, int L) {
  uint32_t r[PN];
#pragma unroll
  for (int i = 0; i < PN; ++i) r[i] = i < pn ? coef[(int64_t)i * C + c] : 0u;
  garner_residues<PN>(s, r, out, c, pn, L);
}

// ------------------------------------------------------------------------------------
// S4 (last pass) + S5 in one launch: a block takes W lines of the last variable for every
// prime (lines along the last variable are contiguous: inner = 1), runs each prime's inverse
// transform in LDS as intt_body does, stores the trimmed coefficient residues where S4 puts
// them (so that S5 can be run again from them), and reconstructs the block's coefficients from
// the residues still in LDS. Tile of prime q: [Nv][W] in bit-reversed rows, then its Nv/2
// twiddles w^{-t}, at q * (Nv W + Nv/2) words.
// ------------------------------------------------------------------------------------
template <int PN>
__global__ __launch_bounds__(kBlock) void intt_garner_kernel(
    const uint32_t* __restrict__ in, uint32_t* __restrict__ coef, uint32_t* __restrict__ out,
    int64_t outer, int Nv, int logN, int Dv1, int W, int pn, int L,
    const uint32_t* __restrict__ itw, int64_t tw_stride, const PrimeConst* __restrict__ pcs,
    const uint32_t* __restrict__ gw, const uint32_t* __restrict__ gc,
    const uint32_t* __restrict__ mlimbs, const uint32_t* __restrict__ hlimbs) {
  __shared__ GarnerShared<PN> s;
  extern __shared__ uint32_t tiles[];
  const int per = Nv * W + Nv / 2;  // words per prime
  const int total = Nv * W;
  const int lW = __builtin_ctz((unsigned)W);
  const int64_t line0 = (int64_t)blockIdx.x * W;
  const int nW = (int)((outer - line0) < W ? (outer - line0) : W);
  garner_load<PN>(s, pn, L, pcs, gw, gc, mlimbs, hlimbs);
  for (int t = threadIdx.x; t < pn * (Nv / 2); t += kBlock) {
    const int q = t / (Nv / 2), i = t - q * (Nv / 2);
    tiles[q * per + total + i] = itw[(int64_t)q * tw_stride + i];
  }
  // load: element j of local line l of prime q goes to row brev(j), column l
  for (int idx = threadIdx.x; idx < pn * total; idx += kBlock) {
    const int q = idx / total, r = idx - q * total;
    const int l = r >> logN, j = r & (Nv - 1);
    uint32_t v = 0u;
    if (l < nW) v = in[((int64_t)q * outer + line0 + l) * Nv + j];
    const int rj = logN ? (int)(__brev((unsigned)j) >> (32 - logN)) : 0;
    tiles[q * per + rj * W + l] = v;
  }
  __syncthreads();
  int st = 1;
  for (; st + 1 <= logN; st += 2) {  // two radix-2 stages per pass (intt_body)
    const int h = 1 << (st - 1);
    const int st1 = Nv >> st, st2 = Nv >> (st + 1);
    const int quarter = (Nv / 4) * W;
    for (int bi = threadIdx.x; bi < pn * quarter; bi += kBlock) {
      const int q = bi / quarter, bq = bi - q * quarter;
      const uint32_t p = s.p[q], pinv = s.pinv[q];
      uint32_t* tile = tiles + q * per;
      const uint32_t* twl = tile + total;
      const int l = bq & (W - 1);
      const int b = bq >> lW;
      const int grp = b >> (st - 1), pos = b & (h - 1);
      const int i0 = grp * 4 * h + pos;
      uint32_t* e0 = tile + i0 * W + l;
      const uint32_t x0 = e0[0], x1 = e0[h * W], x2 = e0[2 * h * W], x3 = e0[3 * h * W];
      const uint32_t t1 = twl[pos * st1];
      const uint32_t v1 = mm(x1, t1, p, pinv), v3 = mm(x3, t1, p, pinv);
      const uint32_t u0 = addm(x0, v1, p), u1 = subm(x0, v1, p);
      const uint32_t u2 = addm(x2, v3, p), u3 = subm(x2, v3, p);
      const uint32_t y2 = mm(u2, twl[pos * st2], p, pinv);
      const uint32_t y3 = mm(u3, twl[(pos + h) * st2], p, pinv);
      e0[0] = addm(u0, y2, p);
      e0[2 * h * W] = subm(u0, y2, p);
      e0[h * W] = addm(u1, y3, p);
      e0[3 * h * W] = subm(u1, y3, p);
    }
    __syncthreads();
  }
  for (; st <= logN; ++st) {  // the last stage when log2 Nv is odd
    const int half = 1 << (st - 1);
    const int stride = Nv >> st;
    const int halfw = (Nv / 2) * W;
    for (int bi = threadIdx.x; bi < pn * halfw; bi += kBlock) {
      const int q = bi / halfw, bq = bi - q * halfw;
      const uint32_t p = s.p[q], pinv = s.pinv[q];
      uint32_t* tile = tiles + q * per;
      const uint32_t* twl = tile + total;
      const int l = bq & (W - 1);
      const int b = bq >> lW;
      const int grp = b >> (st - 1), pos = b & (half - 1);
      const int i0 = grp * 2 * half + pos, i1 = i0 + half;
      const uint32_t u = tile[i0 * W + l];
      const uint32_t v = mm(tile[i1 * W + l], twl[pos * stride], p, pinv);
      tile[i0 * W + l] = addm(u, v, p);
      tile[i1 * W + l] = subm(u, v, p);
    }
    __syncthreads();
  }
  // the coefficient residues (S4's output) and the reconstruction (S5) of each coefficient
  const int64_t C = outer * Dv1;
  for (int idx = threadIdx.x; idx < nW * Dv1; idx += kBlock) {
    const int l = idx / Dv1, e = idx - l * Dv1;
    const int64_t c = (line0 + l) * Dv1 + e;
    uint32_t r[PN];
#pragma unroll
    for (int q = 0; q < PN; ++q) {
      r[q] = 0u;
      if (q < pn) {
        r[q] = tiles[q * per + e * W + l];
        coef[(int64_t)q * C + c] = r[q];
      }
    }
    garner_residues<PN>(s, r, out, c, pn, L);
  }
}

template <int PN>
__global__ __launch_bounds__(kBlock) void garner_kernel(
    const uint32_t* __restrict__ coef, uint32_t* __restrict__ out, int64_t C, int pn, int L,
    const PrimeConst* __restrict__ pcs, const uint32_t* __restrict__ gw,
    const uint32_t* __restrict__ gc, const uint32_t* __restrict__ mlimbs,
    const uint32_t* __restrict__ hlimbs) {
  __shared__ GarnerShared<PN> s;
  garner_load<PN>(s, pn, L, pcs, gw, gc, mlimbs, hlimbs);
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c < C) garner_body<PN>(s, coef, out, c, C, pn, L);
}

template <int PN>
__global__ __launch_bounds__(kBlock) void garner_batch_kernel(
    const BGarner* __restrict__ desc, int ndesc, int64_t vblocks, uint8_t* __restrict__ ws,
    uint32_t* __restrict__ out, const int64_t* __restrict__ out_offsets) {
  __shared__ GarnerShared<PN> s;
  for (int64_t vb = blockIdx.x; vb < vblocks; vb += gridDim.x) {
    const BGarner& d = desc[find_desc(desc, ndesc, vb)];
    garner_load<PN>(s, d.pn, d.L, d.pc, d.gw, d.gc, d.ml, d.hl);
    __syncthreads();
    const int64_t c = (vb - d.block0) * kBlock + threadIdx.x;
    if (c < d.C) {
      garner_body<PN>(s, (const uint32_t*)(ws + d.coef_off), out + out_offsets[d.mat], c, d.C,
                      d.pn, d.L);
    }
    __syncthreads();  // the next virtual block reloads the tables
  }
}

// ------------------------------------------------------------------------------------
// launch helpers
// ------------------------------------------------------------------------------------
template <int M>
hipError_t launch_expand_m(const MatPlan& P, const uint32_t* in, uint32_t* out, int64_t outer,
                           int v, int64_t inner, int jbase, int Nout, hipStream_t st,
                           const int64_t* coeffs) {
  const int64_t B = (int64_t)P.pn * P.nslot;
  if (B == 0) return hipSuccess;  // every entry is zero
  const int JC = expand_outputs_per_thread(Nout, inner, P.m[v]);
  const int64_t work = B * outer * (expand_jrange(Nout, P.m[v]) / JC) * inner;
  // the full evaluation tensor (last pass of the unfused path) is read without zero flags
  const bool write_zero = v == 0;
  if (coeffs) {  // the first pass (inner = 1, the whole line): reduce as the line loads
    if (inner != 1 || jbase != 0 || Nout != P.N[v]) return hipErrorInvalidValue;
    hipLaunchKernelGGL((expand_reduce_kernel<M>), dim3(blocks_for(work)), dim3(kBlock), 0, st,
                       coeffs, P.d_slot_src, const_cast<uint32_t*>(in), out, B, outer, P.m[v],
                       P.N[v], JC, P.nslot,
                       P.d_tw + P.tw_off[v], P.tw_stride, P.d_pc, P.d_slot_zero, write_zero);
    return hipGetLastError();
  }
  if (inner >= 64)
    hipLaunchKernelGGL((expand_kernel<M, true>), dim3(blocks_for(work)), dim3(kBlock), 0, st, in,
                       out, B, outer, P.m[v], P.N[v], JC, inner, P.nslot, P.d_tw + P.tw_off[v],
                       P.tw_stride, P.d_pc, P.d_slot_zero, write_zero, jbase, Nout);
  else
    hipLaunchKernelGGL((expand_kernel<M, false>), dim3(blocks_for(work)), dim3(kBlock), 0, st, in,
                       out, B, outer, P.m[v], P.N[v], JC, inner, P.nslot, P.d_tw + P.tw_off[v],
                       P.tw_stride, P.d_pc, P.d_slot_zero, write_zero, jbase, Nout);
  return hipGetLastError();
}

// The pass over variable v; with jbase, Nout a slab of its grid (expand_body); with coeffs
// the first pass, reading the integer coefficients instead of the residues.
hipError_t launch_expand(const MatPlan& P, const uint32_t* in, uint32_t* out, int64_t outer,
                         int v, int64_t inner, hipStream_t st, int jbase = 0, int Nout = 0,
                         const int64_t* coeffs = nullptr) {
  const int m = P.m[v];
  if (Nout == 0) Nout = P.N[v];
  switch (m) {
    case 1: return launch_expand_m<1>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 2: return launch_expand_m<2>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 3: return launch_expand_m<3>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 4: return launch_expand_m<4>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 5: return launch_expand_m<5>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 6: return launch_expand_m<6>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 7: return launch_expand_m<7>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    case 8: return launch_expand_m<8>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
    default:
      if (m <= 16) return launch_expand_m<16>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
      return launch_expand_m<32>(P, in, out, outer, v, inner, jbase, Nout, st, coeffs);
  }
}

// The points of slab b (of P.slabs) along variable 1: h = N_1 / (2 slabs) values j_1 from
// b h and as many from N_1 / 2 + b h, whose pass over variable 1 is paired (expand_body).
struct SlabMap {
  int jbase, Nout;                // that pass's output: Nout = 2h values per line from jbase
  int64_t R, seg, off1, off2;     // the elimination's local points (FusedDetArgs)
};

SlabMap slab_map(const MatPlan& P, int b) {
  const int64_t R = P.G / P.N[0];
  SlabMap s;
  if (b < 0 || P.slabs <= 1) {
    s.jbase = 0;
    s.Nout = P.k >= 2 ? P.N[1] : 1;
    s.R = s.seg = R;
    s.off1 = s.off2 = 0;
    return s;
  }
  const int64_t R1 = R / P.N[1];  // points of the variables after the first two
  const int h = P.N[1] / (2 * P.slabs);
  s.jbase = b * h;
  s.Nout = 2 * h;
  s.R = 2 * h * R1;
  s.seg = h * R1;
  s.off1 = (int64_t)b * h * R1;
  s.off2 = ((int64_t)P.N[1] / 2 + (int64_t)b * h - h) * R1;
  return s;
}

template <int N, int GL>
hipError_t launch_det_ng(const MatPlan& P, const uint8_t* ws, uint32_t* detv, int slab,
                         hipStream_t st) {
  uint32_t* denv = (uint32_t*)(const_cast<uint8_t*>(ws) + P.off_den);
  if (!P.fused) {
    return det_launch<N, GL>((const uint32_t*)(ws + P.off_eval), detv, denv, P.G, P.pn, P.d_pc, st);
  }
  const SlabMap sm = slab_map(P, slab);
  FusedDetArgs f;
  f.pre = (const uint32_t*)(ws + P.off_pre);
  f.detv = detv;
  f.denv = denv;
  f.R = sm.R;
  f.Rout = P.G / P.N[0];
  f.seg = sm.seg;
  f.off1 = sm.off1;
  f.off2 = sm.off2;
  f.N0 = P.N[0];
  f.m0 = P.m[0];
  f.Q = P.fuse_Q;
  f.S = P.fuse_S;
  f.tw0 = P.d_tw + P.tw_off[0];
  f.tw_stride = P.tw_stride;
  f.pcs = P.d_pc;
  f.zero = P.d_zero;
  f.slot = P.d_entry_slot;
  f.nslot = P.nslot;
  f.pn = P.pn;
  f.fixup = false;
  if constexpr (N <= kLLMaxN) {
    if (P.det_ll) {
      // left-looking pass, then the exchanging kernel repairs the points it could not do
      const hipError_t e = det_ll_launch<N>(f, st);
      if (e != hipSuccess) return e;
      f.fixup = true;
    }
  }
  return det_fused_launch<N, GL>(f, st);
}

template <int N, int GL>
struct SingleDet {
  static hipError_t run(const MatPlan& P, const uint8_t* ws, uint32_t* detv, int slab,
                        hipStream_t st) {
    return launch_det_ng<N, GL>(P, ws, detv, slab, st);
  }
};

template <int N, int GL>
struct BatchDet {
  static hipError_t run(int ll, int pair, const BDet* desc, int ndesc, int64_t vblocks,
                        size_t lds, uint8_t* ws, hipStream_t st) {
    if (ll == 1) {
      if constexpr (N <= kLLMaxN) return det_ll_batch_launch<N>(desc, ndesc, vblocks, lds, ws, st);
      return hipErrorInvalidValue;
    }
    return det_fused_batch_launch<N, GL>(desc, ndesc, vblocks, lds, ws, pair, ll == 2, st);
  }
};

// The batched elimination's matrices one by one: matrix i's primes are the virtual blocks from
// its block0 to the next descriptor's, rtiles * jtiles per prime.
template <int N, int GL>
struct EachDet {
  static hipError_t run(bool fixup, const BDet* desc, int ndesc, int64_t vblocks, uint8_t* ws,
                        hipStream_t st) {
    for (int i = 0; i < ndesc; ++i) {
      const BDet& d = desc[i];
      const int64_t end = i + 1 < ndesc ? desc[i + 1].block0 : vblocks;
      FusedDetArgs f;
      f.pre = (const uint32_t*)(ws + d.pre_off);
      f.detv = (uint32_t*)(ws + d.detv_off);
      f.denv = (uint32_t*)(ws + d.den_off);
      f.R = f.Rout = f.seg = d.R;
      f.off1 = f.off2 = 0;
      f.N0 = d.N0;
      f.m0 = d.m0;
      f.Q = d.Q;
      f.S = d.S;
      f.tw0 = d.tw0;
      f.tw_stride = d.tw_stride;
      f.pcs = d.pc;
      f.zero = d.zero;
      f.slot = d.slot;
      f.nslot = d.nslot;
      f.pn = (int)((end - d.block0) / (d.rtiles * d.jtiles));
      f.fixup = fixup;
      const hipError_t e = det_fused_launch<N, GL>(f, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// Calls F<N, GL>::run(args...) for the (order, lanes) pair if a kernel is compiled for it.
template <template <int, int> class F, int N, typename... A>
hipError_t det_dispatch_n(int lanes, A&&... args) {
  switch (lanes) {
    case 1:
      if constexpr (N <= 12) return F<N, 1>::run(std::forward<A>(args)...);
      break;
    case 2:
      if constexpr (N >= 2 && N <= 16) return F<N, 2>::run(std::forward<A>(args)...);
      break;
    case 4:
      if constexpr (N >= 4 && N <= 24) return F<N, 4>::run(std::forward<A>(args)...);
      break;
    case 8:
      if constexpr (N >= 8) return F<N, 8>::run(std::forward<A>(args)...);
      break;
    case 16:
      if constexpr (N >= 16) return F<N, 16>::run(std::forward<A>(args)...);
      break;
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <template <int, int> class F, int... Ns, typename... A>
hipError_t det_dispatch_seq(std::integer_sequence<int, Ns...>, int n, int lanes, A&&... args) {
  hipError_t r = hipErrorInvalidValue;
  ((n == Ns + 1 ? (r = det_dispatch_n<F, Ns + 1>(lanes, std::forward<A>(args)...), 0) : 0), ...);
  return r;
}

template <template <int, int> class F, typename... A>
hipError_t det_dispatch(int n, int lanes, A&&... args) {
  return det_dispatch_seq<F>(std::make_integer_sequence<int, kMaxN>{}, n, lanes,
                             std::forward<A>(args)...);
}

template <int PN>
hipError_t launch_garner_pn(const MatPlan& P, const uint32_t* coef, uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(garner_kernel<PN>, dim3(blocks_for(P.C)), dim3(kBlock), 0, st, coef, out, P.C,
                     P.pn, P.L, P.d_pc, P.d_gw, P.d_gc, P.d_mlimbs, P.d_hlimbs);
  return hipGetLastError();
}

template <int PN>
hipError_t launch_garner_batch(const BGarner* desc, int ndesc, int64_t vblocks, uint8_t* ws,
                               uint32_t* out, const int64_t* out_offsets, hipStream_t st) {
  hipLaunchKernelGGL(garner_batch_kernel<PN>, dim3(persistent_grid(vblocks)), dim3(kBlock), 0, st,
                     desc, ndesc, vblocks, ws, out, out_offsets);
  return hipGetLastError();
}

}  // namespace

bool det_config_supported(int n, int lanes) {
  if (n < 1 || n > kMaxN) return false;
  switch (lanes) {
    case 1: return n <= 12;
    case 2: return n >= 2 && n <= 16;
    case 4: return n >= 4 && n <= 24;
    case 8: return n >= 8;
    case 16: return n >= 16;
    default: return false;
  }
}

int expand_outputs_per_thread(int Nv, int64_t inner, int m) {
  // enough threads per line that a wave covers at least 64 consecutive outputs
  const int NJ = expand_jrange(Nv, m);
  int nJB = 1;
  while (nJB < NJ && nJB * inner < 64) nJB <<= 1;
  return NJ / nJB;
}

// Whether passes of 32-256 points along a contiguous axis take the register form
// (intt_reg_kernel); POLYDET_INTT_REGISTERS=0 keeps the LDS-staged form everywhere (for
// comparisons).
bool intt_register_form() {
  static const bool on = [] {
    const char* e = std::getenv("POLYDET_INTT_REGISTERS");
    return !(e && e[0] == '0');
  }();
  return on;
}

bool intt_register_pass(int Nv, int64_t inner) {
  return (Nv == 32 || Nv == 64 || Nv == 128 || Nv == 256) && inner >= kInttRegLines &&
         intt_register_form();
}

int intt_lines_per_block(int64_t lines, int Nv, int pn) {
  // as many lines as fit in kTileElems, fewer while that leaves under ~1024 blocks (W stays
  // a power of two, so it divides inner when inner >= W). Measured at the 12x12 trivariate
  // workload: targets of 512 and 2048 blocks were both slower.
  int W = kTileElems / Nv;
  while (W > 1 && ((lines + W - 1) / W) * pn < 1024) W >>= 1;
  return W;
}

hipError_t run_reduce(const MatPlan& P, const int64_t* coeffs, uint8_t* ws, hipStream_t st) {
  const int64_t count = P.nslot * P.T;
  if (count == 0) return hipSuccess;  // every entry is zero
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(count)), dim3(kBlock), 0, st, coeffs,
                     (uint32_t*)(ws + P.off_res), count, P.pn, P.T, P.d_slot_src, P.d_pc);
  return hipGetLastError();
}

// The evaluation passes over the variables v with vlo <= v <= vhi, from the last variable
// down (passes alternate tmpA, tmpB); with slab >= 0 the pass over variable 1 makes that slab
// only. With coeffs the first pass (over the last variable, which must be in the range and
// not sliced) reads the integer coefficients and reduces them itself (S1 in that launch).
hipError_t run_evaluate_passes(const MatPlan& P, uint8_t* ws, int vlo, int vhi, int slab,
                               hipStream_t st, const int64_t* coeffs = nullptr) {
  const uint32_t* in = (const uint32_t*)(ws + P.off_res);
  uint32_t* bufs[2] = {(uint32_t*)(ws + P.off_tmpA), (uint32_t*)(ws + P.off_tmpB)};
  int which = 0;
  const int last = P.fused ? 1 : 0;  // the fused kernel evaluates variable 0 itself
  for (int v = P.k - 1; v >= last; --v) {
    int64_t outer = 1, inner = 1;
    for (int u = 0; u < v; ++u) outer *= P.m[u];
    for (int u = v + 1; u < P.k; ++u) inner *= P.N[u];
    uint32_t* out = v == 0 ? (uint32_t*)(ws + P.off_eval) : bufs[which];
    if (v >= vlo && v <= vhi) {
      const SlabMap sm = slab_map(P, v == 1 ? slab : -1);
      hipError_t err = v == 1 && slab >= 0
                           ? launch_expand(P, in, out, outer, v, inner, st, sm.jbase, sm.Nout)
                           : launch_expand(P, in, out, outer, v, inner, st, 0, 0,
                                           v == P.k - 1 ? coeffs : nullptr);
      if (err != hipSuccess) return err;
    }
    in = out;
    which ^= 1;
  }
  return hipSuccess;
}

hipError_t run_evaluate(const MatPlan& P, uint8_t* ws, hipStream_t st) {
  if (P.k == 0) return hipSuccess;  // the residues are the values at the single point
  return run_evaluate_passes(P, ws, 0, P.k - 1, -1, st);
}

hipError_t run_reduce_evaluate(const MatPlan& P, const int64_t* coeffs, uint8_t* ws,
                               hipStream_t st) {
  // the residues themselves are the input of the elimination (no evaluation pass) or of
  // nothing (every entry zero): the reduction keeps its own launch
  const bool passes = P.k >= (P.fused ? 2 : 1);
  if (!passes || P.nslot * P.T == 0) {
    hipError_t err = run_reduce(P, coeffs, ws, st);
    return err != hipSuccess ? err : run_evaluate(P, ws, st);
  }
  return run_evaluate_passes(P, ws, 0, P.k - 1, -1, st, coeffs);
}

hipError_t run_evaluate_upper(const MatPlan& P, uint8_t* ws, hipStream_t st) {
  return run_evaluate_passes(P, ws, 2, P.k - 1, -1, st);  // variable 1 goes slab by slab
}

hipError_t run_evaluate_slab(const MatPlan& P, uint8_t* ws, int slab, hipStream_t st) {
  return run_evaluate_passes(P, ws, 1, 1, slab, st);
}

int64_t finalize_threads(int64_t G, int pn) {
  return (int64_t)pn * ((G + kFinalPoints - 1) / kFinalPoints);
}

hipError_t run_det(const MatPlan& P, uint8_t* ws, hipStream_t st) {
  return det_dispatch<SingleDet>(P.n, P.det_lanes, P, (const uint8_t*)ws,
                                 (uint32_t*)(ws + P.off_detv), -1, st);
}

hipError_t run_det_slab(const MatPlan& P, uint8_t* ws, int slab, hipStream_t st) {
  return det_dispatch<SingleDet>(P.n, P.det_lanes, P, (const uint8_t*)ws,
                                 (uint32_t*)(ws + P.off_detv), slab, st);
}

hipError_t run_finalize(const MatPlan& P, uint8_t* ws, hipStream_t st) {
  // with variables the first interpolation pass divides as it loads (intt_body)
  if (P.k > 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(finalize_threads(P.G, P.pn))), dim3(kBlock),
                     0, st, (const uint32_t*)(ws + P.off_detv), (const uint32_t*)(ws + P.off_den),
                     (uint32_t*)(ws + P.off_coef), P.G, P.pn, P.d_pc);
  return hipGetLastError();
}

// The interpolation passes over the variables 0 .. vhi in order (the first pass divides; the
// pass over variable v writes iA for even v and iB for odd v, the last variable's pass the
// coefficient region).
hipError_t run_interpolate_passes(const MatPlan& P, uint8_t* ws, int vhi, hipStream_t st) {
  const uint32_t* in = (const uint32_t*)(ws + P.off_detv);
  uint32_t* bufs[2] = {(uint32_t*)(ws + P.off_iA), (uint32_t*)(ws + P.off_iB)};
  int which = 0;
  for (int v = 0; v <= vhi; ++v) {
    int64_t outer = 1, inner = 1;
    for (int u = 0; u < v; ++u) outer *= P.D[u] + 1;
    for (int u = v + 1; u < P.k; ++u) inner *= P.N[u];
    uint32_t* out = v == P.k - 1 ? (uint32_t*)(ws + P.off_coef) : bufs[which];
    const int Nv = P.N[v];
    int logN = 0;
    while ((1 << logN) < Nv) ++logN;
    const int64_t lines = outer * inner;
    // the first pass also divides each point's numerator by its denominator
    const uint32_t* den = v == 0 ? (const uint32_t*)(ws + P.off_den) : nullptr;
    if (intt_register_pass(Nv, inner)) {
      const dim3 g((unsigned)(lines / kInttRegLines * P.pn));
      const int Dv1 = P.D[v] + 1;
      const uint32_t* itw = P.d_itw + P.tw_off[v];
      if (Nv == 32)
        hipLaunchKernelGGL(intt_reg_kernel<4>, g, dim3(kBlock), 0, st, in, out, outer, inner, Dv1,
                           itw, P.tw_stride, P.d_pc, den);
      else if (Nv == 64)
        hipLaunchKernelGGL(intt_reg_kernel<8>, g, dim3(kBlock), 0, st, in, out, outer, inner, Dv1,
                           itw, P.tw_stride, P.d_pc, den);
      else if (Nv == 128)
        hipLaunchKernelGGL(intt_reg_kernel<16>, g, dim3(kBlock), 0, st, in, out, outer, inner,
                           Dv1, itw, P.tw_stride, P.d_pc, den);
      else
        hipLaunchKernelGGL(intt_reg_kernel<32>, g, dim3(kBlock), 0, st, in, out, outer, inner,
                           Dv1, itw, P.tw_stride, P.d_pc, den);
      hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
      in = out;
      which ^= 1;
      continue;
    }
    int W = intt_lines_per_block(lines, Nv, P.pn);
    // the dividing first pass: enough lines that each thread has kFuseBatch points to invert
    // together (at 64^3 that halves the exponentiations; measured 2 us faster)
    if (v == 0)
      while (Nv * W < kFuseBatch * kBlock && Nv * (2 * W) <= kTileElems) W <<= 1;
    const int64_t tiles = (lines + W - 1) / W;
    const size_t lds = (size_t)(Nv * W + Nv / 2) * sizeof(uint32_t);
    hipLaunchKernelGGL(intt_kernel, dim3((unsigned)(tiles * P.pn)), dim3(kBlock), lds, st, in, out,
                       outer, Nv, logN, inner, P.D[v] + 1, W, P.d_itw + P.tw_off[v], P.tw_stride,
                       P.d_pc, den);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    in = out;
    which ^= 1;
  }
  return hipSuccess;
}

hipError_t run_interpolate(const MatPlan& P, uint8_t* ws, hipStream_t st) {
  if (P.k == 0) return hipSuccess;
  return run_interpolate_passes(P, ws, P.k - 1, st);
}

// Bytes of LDS for the tiles of intt_garner_kernel (every prime's W lines of N values and its
// N/2 twiddles) and the largest such size it takes.
constexpr size_t kInttGarnerLds = 40 * 1024;
size_t intt_garner_lds(int pn, int Nv, int W) {
  return (size_t)pn * ((size_t)Nv * W + Nv / 2) * sizeof(uint32_t);
}

template <int PN>
hipError_t launch_intt_garner(const MatPlan& P, const uint32_t* in, uint32_t* coef, uint32_t* out,
                              int64_t outer, int Nv, int logN, int W, hipStream_t st) {
  const int v = P.k - 1;
  const int64_t blocks = (outer + W - 1) / W;
  hipLaunchKernelGGL((intt_garner_kernel<PN>), dim3((unsigned)blocks), dim3(kBlock),
                     intt_garner_lds(P.pn, Nv, W), st, in, coef, out, outer, Nv, logN, P.D[v] + 1,
                     W, P.pn, P.L, P.d_itw + P.tw_off[v], P.tw_stride, P.d_pc, P.d_gw, P.d_gc,
                     P.d_mlimbs, P.d_hlimbs);
  return hipGetLastError();
}

hipError_t run_interpolate_reconstruct(const MatPlan& P, uint8_t* ws, uint32_t* out,
                                       hipStream_t st) {
  const int v = P.k - 1;
  // the last pass by itself: no variables, one variable (its pass also divides), or tiles
  // that do not fit
  if (P.k < 2 || intt_garner_lds(P.pn, P.N[v], 1) > kInttGarnerLds) {
    hipError_t err = run_interpolate(P, ws, st);
    return err != hipSuccess ? err : run_reconstruct(P, ws, out, st);
  }
  hipError_t err = run_interpolate_passes(P, ws, v - 1, st);
  if (err != hipSuccess) return err;
  int64_t outer = 1;
  for (int u = 0; u < v; ++u) outer *= P.D[u] + 1;
  const int Nv = P.N[v];
  int logN = 0;
  while ((1 << logN) < Nv) ++logN;
  // lines per block: a power of two, while at least 512 blocks remain and the tiles fit
  int W = 1;
  while (2 * W * Nv <= kTileElems && (outer + 2 * W - 1) / (2 * W) >= 512 &&
         intt_garner_lds(P.pn, Nv, 2 * W) <= kInttGarnerLds)
    W <<= 1;
  // input: the output of the pass over variable v - 1 (passes alternate iA, iB)
  const uint32_t* in = (const uint32_t*)(ws + ((v - 1) % 2 == 0 ? P.off_iA : P.off_iB));
  uint32_t* coef = (uint32_t*)(ws + P.off_coef);
  if (P.pn <= 8) return launch_intt_garner<8>(P, in, coef, out, outer, Nv, logN, W, st);
  if (P.pn <= 16) return launch_intt_garner<16>(P, in, coef, out, outer, Nv, logN, W, st);
  return launch_intt_garner<32>(P, in, coef, out, outer, Nv, logN, W, st);
}

hipError_t run_reconstruct(const MatPlan& P, uint8_t* ws, uint32_t* out, hipStream_t st) {
  const uint32_t* coef = (const uint32_t*)(ws + P.off_coef);
  if (P.pn <= 8) return launch_garner_pn<8>(P, coef, out, st);
  if (P.pn <= 16) return launch_garner_pn<16>(P, coef, out, st);
  return launch_garner_pn<32>(P, coef, out, st);
}

// ------------------------------------------------------------------------------------
// batched launches
// ------------------------------------------------------------------------------------
hipError_t batch_reduce(const BReduce* desc, int ndesc, int64_t vblocks, const int64_t* coeffs,
                        const int64_t* coeff_offsets, uint8_t* ws, hipStream_t st) {
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(persistent_grid(vblocks)), dim3(kBlock), 0, st,
                     desc, ndesc, vblocks, coeffs, coeff_offsets, ws);
  return hipGetLastError();
}

hipError_t batch_expand(const BExpand* desc, int ndesc, int64_t vblocks, uint8_t* ws,
                        hipStream_t st) {
  hipLaunchKernelGGL(expand_batch_kernel, dim3(persistent_grid(vblocks)), dim3(kBlock), 0, st,
                     desc, ndesc, vblocks, ws);
  return hipGetLastError();
}


hipError_t batch_intt(const BIntt* desc, int ndesc, int64_t vblocks, size_t lds, uint8_t* ws,
                      hipStream_t st) {
  hipLaunchKernelGGL(intt_batch_kernel, dim3(persistent_grid(vblocks)), dim3(kBlock), lds, st,
                     desc, ndesc, vblocks, ws);
  return hipGetLastError();
}

hipError_t batch_garner(const BGarner* desc, int ndesc, int64_t vblocks, int pnmax, uint8_t* ws,
                        uint32_t* out, const int64_t* out_offsets, hipStream_t st) {
  if (pnmax <= 8) return launch_garner_batch<8>(desc, ndesc, vblocks, ws, out, out_offsets, st);
  if (pnmax <= 16) return launch_garner_batch<16>(desc, ndesc, vblocks, ws, out, out_offsets, st);
  return launch_garner_batch<32>(desc, ndesc, vblocks, ws, out, out_offsets, st);
}

hipError_t batch_det(int n, int lanes, int ll, int pair, const BDet* desc, int ndesc,
                     int64_t vblocks, size_t lds, uint8_t* ws, hipStream_t st) {
  return det_dispatch<BatchDet>(n, lanes, ll, pair, desc, ndesc, vblocks, lds, ws, st);
}

hipError_t batch_det_each(int n, int lanes, bool fixup, const BDet* host_desc, int ndesc,
                          int64_t vblocks, uint8_t* ws, hipStream_t st) {
  return det_dispatch<EachDet>(n, lanes, fixup, host_desc, ndesc, vblocks, ws, st);
}

}  // namespace pd
