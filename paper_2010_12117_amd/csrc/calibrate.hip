// Vector-ALU throughput probes (include/polydet_calibrate.h). Each thread runs `iters`
// iterations of 8 independent chains; the probed instruction is written as inline assembly
// (register operands only) so that the compiler can neither fold the chains nor pick another
// instruction, except for the elimination update, which is the kernels' own mm2_lazy.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "modarith.h"
#include "polydet_calibrate.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 8;

// An odd modulus below 2^62 for the 64-bit probe (2^61 - 1, a Mersenne prime) and its
// -q^{-1} mod 2^64 by Newton's iteration (each step doubles the correct low bits).
constexpr uint64_t kProbePrime64 = (1ull << 61) - 1;
__host__ __device__ constexpr uint64_t probe_qinv64() {
  uint64_t inv = kProbePrime64;
  for (int it = 0; it < 6; ++it) inv *= 2u - kProbePrime64 * inv;
  return 0ull - inv;
}

template <int PROBE>
__global__ __launch_bounds__(kProbeBlock) void probe_kernel(uint32_t* out, int iters,
                                                            uint32_t seed, uint32_t p,
                                                            uint32_t pinv) {
  const uint32_t t = blockIdx.x * kProbeBlock + threadIdx.x;
  uint32_t res = 0;
  if constexpr (PROBE == POLYDET_PROBE_MAD_U64) {
    uint64_t acc[kChains];
    uint32_t x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      acc[c] = t + c;
      x[c] = seed + 3 * c + t;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        uint64_t carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0"
                     : "+v"(acc[c]), "=s"(carry)
                     : "v"(x[c]), "v"(seed));
      }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res ^= (uint32_t)acc[c] ^ (uint32_t)(acc[c] >> 32);
  } else if constexpr (PROBE == POLYDET_PROBE_MUL_LO || PROBE == POLYDET_PROBE_ADD) {
    uint32_t x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 5 * c + t;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if constexpr (PROBE == POLYDET_PROBE_MUL_LO)
          asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[c]) : "v"(seed));
        else
          asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(seed));
      }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res ^= x[c];
  } else if constexpr (PROBE == POLYDET_PROBE_UPDATE2) {
    // a_c <- (D a_c + f1 b_{c+1} + f0 b_{c+2}) / R with b = a / 2 (below p): the kernels'
    // two-step update (mm3_lazy) with both column factors changing every iteration, so that
    // no product is loop-invariant; one shift per update comes on top of the kernels' mix
    uint32_t a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = (seed + 7 * c + t) % p;
    const uint32_t D = (seed * 13u + 1u) % p, f1 = (seed * 17u + 3u) % p;
    const uint32_t f0 = (seed * 19u + 5u) % p;
    for (int i = 0; i < iters; ++i) {
      uint32_t b[kChains];
#pragma unroll
      for (int c = 0; c < kChains; ++c) b[c] = a[c] >> 1;
#pragma unroll
      for (int c = 0; c < kChains; ++c)
        a[c] = pd::mm3_lazy(D, a[c], f1, b[(c + 1) % kChains], f0, b[(c + 2) % kChains], p, pinv);
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res ^= a[c];
  } else if constexpr (PROBE == POLYDET_PROBE_UPDATE64) {
    // a_c <- (pi a_c + m a_{c+1}) / 2^64 mod q with q < 2^62 (Montgomery with R = 2^64): the
    // 128-bit sum of two products, m = t mod 2^64 * (-q^-1), (t + m q) / 2^64 in [0, 2q)
    const uint64_t q = kProbePrime64, qinv = probe_qinv64();
    uint64_t a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = ((uint64_t)seed * (7 * c + 1) + t) % q;
    const uint64_t piv = ((uint64_t)seed * 13u + 1u) % q, m = ((uint64_t)seed * 17u + 3u) % q;
    for (int i = 0; i < iters; ++i) {
      const uint64_t a0 = a[0];
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        const uint64_t b = c + 1 < kChains ? a[c + 1] : a0;
        const uint64_t l1 = piv * a[c], h1 = __umul64hi(piv, a[c]);
        const uint64_t l2 = m * b, h2 = __umul64hi(m, b);
        const uint64_t lo = l1 + l2;
        const uint64_t hi = h1 + h2 + (lo < l1 ? 1u : 0u);
        const uint64_t mm = lo * qinv;
        a[c] = hi + __umul64hi(mm, q) + (lo != 0 ? 1u : 0u);
      }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res ^= (uint32_t)a[c] ^ (uint32_t)(a[c] >> 32);
  } else if constexpr (PROBE == POLYDET_PROBE_UPDATE) {
    // a_c <- (pi a_c + m a_{c+1}) / R: the second product's operand changes every iteration,
    // as the pivot row's entries do in the elimination, so nothing is loop-invariant
    uint32_t a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = (seed + 7 * c + t) % p;
    const uint32_t piv = (seed * 13u + 1u) % p, m = (seed * 17u + 3u) % p;
    for (int i = 0; i < iters; ++i) {
      const uint32_t a0 = a[0];
#pragma unroll
      for (int c = 0; c < kChains; ++c)
        a[c] = pd::mm2_lazy(piv, a[c], m, c + 1 < kChains ? a[c + 1] : a0, p, pinv);
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res ^= a[c];
  } else {
    using F = typename std::conditional<PROBE == POLYDET_PROBE_FMA_F64, double, float>::type;
    F x[kChains];
    const F y = (F)1.0000001, z = (F)1e-7;
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (F)(t + c) * (F)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if constexpr (PROBE == POLYDET_PROBE_FMA_F64)
          asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(x[c]) : "v"(y), "v"(z));
        else
          asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x[c]) : "v"(y), "v"(z));
      }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res ^= (uint32_t)(int64_t)x[c];
  }
  out[t] = res;
}

template <int PROBE>
hipError_t launch_probe(uint32_t* out, int blocks, int iters, hipStream_t st) {
  const uint32_t p = 1073479681u;  // the largest prime of the library's table
  uint32_t inv = p;
  for (int it = 0; it < 5; ++it) inv *= 2u - p * inv;
  hipLaunchKernelGGL(probe_kernel<PROBE>, dim3(blocks), dim3(kProbeBlock), 0, st, out, iters,
                     0x9E3779B9u, p, 0u - inv);
  return hipGetLastError();
}

hipError_t launch(int probe, uint32_t* out, int blocks, int iters, hipStream_t st) {
  switch (probe) {
    case POLYDET_PROBE_MAD_U64: return launch_probe<POLYDET_PROBE_MAD_U64>(out, blocks, iters, st);
    case POLYDET_PROBE_MUL_LO: return launch_probe<POLYDET_PROBE_MUL_LO>(out, blocks, iters, st);
    case POLYDET_PROBE_ADD: return launch_probe<POLYDET_PROBE_ADD>(out, blocks, iters, st);
    case POLYDET_PROBE_UPDATE: return launch_probe<POLYDET_PROBE_UPDATE>(out, blocks, iters, st);
    case POLYDET_PROBE_FMA_F64: return launch_probe<POLYDET_PROBE_FMA_F64>(out, blocks, iters, st);
    case POLYDET_PROBE_UPDATE2: return launch_probe<POLYDET_PROBE_UPDATE2>(out, blocks, iters, st);
    case POLYDET_PROBE_UPDATE64:
      return launch_probe<POLYDET_PROBE_UPDATE64>(out, blocks, iters, st);
    default: return launch_probe<POLYDET_PROBE_FMA_F32>(out, blocks, iters, st);
  }
}

}  // namespace

extern "C" polydet_status polydet_calibrate_alu(int32_t probe, int32_t blocks, int32_t iters,
                                                double* ops_per_s, void* stream) {
  if (probe < 0 || probe >= POLYDET_PROBE_COUNT || blocks < 1 || iters < 1 || !ops_per_s)
    return POLYDET_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* out = nullptr;
  hipError_t e = hipMalloc((void**)&out, (size_t)blocks * kProbeBlock * sizeof(uint32_t));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? POLYDET_ENOMEM : POLYDET_EDEVICE;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0;
  if ((e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess &&
      (e = launch(probe, out, blocks, 1, st)) == hipSuccess &&  // warm-up
      (e = hipEventRecord(e0, st)) == hipSuccess &&
      (e = launch(probe, out, blocks, iters, st)) == hipSuccess &&
      (e = hipEventRecord(e1, st)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess) {
    e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (e != hipSuccess) return POLYDET_EDEVICE;
  *ops_per_s = (double)blocks * kProbeBlock * (double)iters * kChains / (ms * 1e-3);
  return POLYDET_OK;
}
