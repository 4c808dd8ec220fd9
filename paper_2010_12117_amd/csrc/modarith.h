// Modular arithmetic over Z/pZ for word-size primes p in (2^29, 2^30).
//
// Values are kept in Montgomery form x~ = x * R mod p with R = 2^32 (Montgomery 1985):
// the product of two representatives reduced by REDC is the representative of the product,
// so every stage (evaluation, elimination, interpolation) runs on representatives and only
// the reconstruction converts back. REDC(t) = (t + m p) / R with m = t * (-p^{-1}) mod R;
// for t < p R it returns a value below 2p, and one conditional subtraction finishes it.
// A sum of two products of reduced values stays below 2 p^2 < p R, which lets the
// elimination update fold two products into one reduction. Since p < 2^30, the sum may even
// have one factor of each product below 2p (then t < 4 p^2 < p R): the elimination keeps its
// entries unreduced in [0, 2p) and skips the conditional subtraction of most updates
// (mm2_lazy). Its two-step update sums three products, one of them with an unreduced factor,
// under one reduction: 2 p^2 + p^2 + p^2 = 4 p^2 < p R again (mm3_lazy).
//
// On gfx950 v_mad_u64_u32 and v_mul_lo_u32 issue at the fp64-FMA rate and plain 32-bit
// ALU ops at twice that, so one REDC costs one mul_lo, one mad_u64 and two plain ops.
#pragma once

#include <stdint.h>

#if defined(__HIP__)
#include <hip/hip_runtime.h>
#define PD_HD __host__ __device__ __forceinline__
#else
#define PD_HD inline
#endif

namespace pd {

PD_HD uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// r in [0, 2p) -> [0, p): when r < p, r - p wraps above r.
PD_HD uint32_t fold(uint32_t r, uint32_t p) { return umin32(r, r - p); }

// REDC for t + m p < 2^64 (holds for t < 2^63 since m p < 2^63).
PD_HD uint32_t redc(uint64_t t, uint32_t p, uint32_t pinv) {
  const uint32_t m = (uint32_t)t * pinv;
  const uint64_t u = t + (uint64_t)m * p;
  return fold((uint32_t)(u >> 32), p);
}

// Montgomery product a~ b~ / R; a < 2^32, b < p.
PD_HD uint32_t mm(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  return redc((uint64_t)a * b, p, pinv);
}

// (a b + c d) / R with every operand below p: one reduction for two products.
PD_HD uint32_t mm2(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t p, uint32_t pinv) {
  return redc((uint64_t)a * b + (uint64_t)c * d, p, pinv);
}

// (a b + c d + e f) / R with every operand below p: t < 3 p^2 < p R, one reduction.
PD_HD uint32_t mm3(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e, uint32_t f,
                   uint32_t p, uint32_t pinv) {
  return redc((uint64_t)a * b + (uint64_t)c * d + (uint64_t)e * f, p, pinv);
}

// (a b + c d) / R in [0, 2p) with a, c <= p and b, d < 2p (t < 4 p^2 < p R for p < 2^30).
PD_HD uint32_t mm2_lazy(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t p,
                        uint32_t pinv) {
  const uint64_t t = (uint64_t)a * b + (uint64_t)c * d;
  const uint32_t m = (uint32_t)t * pinv;
  // The mask changes nothing (the value is below 2p < 2^31) but keeps it a 32-bit value:
  // without it the compiler widens the next product's operand to the 64-bit shifted sum
  // (its high half known zero) and holds two registers per entry.
  return (uint32_t)((t + (uint64_t)m * p) >> 32) & 0x7FFFFFFFu;
}

// (a b + c d + e f) / R in [0, 2p) with b < 2p and every other operand <= p:
// t < 2 p^2 + 2 p^2 = 4 p^2 < p R, three products for one reduction.
PD_HD uint32_t mm3_lazy(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e, uint32_t f,
                        uint32_t p, uint32_t pinv) {
  const uint64_t t = (uint64_t)a * b + (uint64_t)c * d + (uint64_t)e * f;
  const uint32_t m = (uint32_t)t * pinv;
  return (uint32_t)((t + (uint64_t)m * p) >> 32) & 0x7FFFFFFFu;
}

PD_HD uint32_t addm(uint32_t a, uint32_t b, uint32_t p) { return fold(a + b, p); }

PD_HD uint32_t subm(uint32_t a, uint32_t b, uint32_t p) {
  const uint32_t d = a - b;
  return umin32(d, d + p);
}

PD_HD uint32_t negm(uint32_t a, uint32_t p) { return a ? p - a : 0u; }

// x~^e in Montgomery form (left-to-right binary powering from the top set bit of e, so a
// 30-bit exponent costs 29 squarings; e is uniform across a wave).
PD_HD uint32_t mpow(uint32_t x, uint32_t e, uint32_t one, uint32_t p, uint32_t pinv) {
  if (e == 0u) return one;
  uint32_t r = x;
  for (int b = 30 - __builtin_clz(e); b >= 0; --b) {
    r = mm(r, r, p, pinv);
    if ((e >> b) & 1u) r = mm(r, x, p, pinv);
  }
  return r;
}

// Inverse by Fermat's little theorem; 0 maps to 0.
PD_HD uint32_t minv(uint32_t x, uint32_t one, uint32_t p, uint32_t pinv) {
  return mpow(x, p - 2u, one, p, pinv);
}

// Per-prime constants, uploaded once per plan.
struct PrimeConst {
  uint32_t p;      // the prime
  uint32_t pinv;   // -p^{-1} mod 2^32
  uint32_t r1;     // R mod p: the representative of 1
  uint32_t r2;     // R^2 mod p: mm(x, r2) = x~
  uint32_t r3;     // R^3 mod p: mm(hi, r3) = (hi * 2^32)~
  uint32_t scale;  // prod_v N_v^{-1} mod p (plain): mm(c~, scale) = c / G, out of Montgomery form
  uint32_t pad0, pad1;
};

}  // namespace pd
