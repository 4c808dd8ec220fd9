/*
 * polydet calibration probes: the vector-ALU issue rates that bound the determinant kernels.
 *
 * The elimination of the DET stage (Wei & Chen, arXiv 2010.12117, Section 3.2) is bound by
 * integer vector arithmetic. Its roofline is derived from the chip's unit counts and clock;
 * these probes measure, on the GPU that is current, the throughput of the instructions that
 * make up one elimination update, and of the update itself, so that the derived peak can be
 * set beside a measured one.
 *
 * Each probe launches `blocks` blocks of 256 threads; every thread runs `iters` iterations of
 * 8 independent dependency chains of the probed operation, all operands in registers. The
 * result is the number of operations (lane operations; elimination updates for
 * POLYDET_PROBE_UPDATE) per second over the launch, timed with HIP events on `stream`.
 */
#ifndef POLYDET_CALIBRATE_H
#define POLYDET_CALIBRATE_H

#include <stdint.h>

#include "polydet.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum polydet_probe {
  POLYDET_PROBE_MAD_U64 = 0, /* v_mad_u64_u32: 32 x 32 -> 64-bit product plus a 64-bit addend */
  POLYDET_PROBE_MUL_LO = 1,  /* v_mul_lo_u32 */
  POLYDET_PROBE_ADD = 2,     /* v_add_u32 (a plain 32-bit ALU operation) */
  POLYDET_PROBE_UPDATE = 3,  /* one elimination update a <- (pi a + m b) / 2^32 mod p, as the
                              * kernels issue it: two products, one Montgomery reduction */
  POLYDET_PROBE_FMA_F64 = 4, /* v_fma_f64, the published fp64 vector rate */
  POLYDET_PROBE_FMA_F32 = 5, /* v_fma_f32 (unpacked) */
  POLYDET_PROBE_UPDATE2 = 6, /* one two-step elimination update a <- (D a + f1 u + f0 v) / 2^32
                              * mod p, as the kernels issue it: three products, one reduction */
  POLYDET_PROBE_UPDATE64 = 7, /* the single-step update with 64-bit residues (a prime below
                               * 2^62, R = 2^64): two 64 x 64-bit products, one reduction */
  POLYDET_PROBE_COUNT = 8
} polydet_probe;

/* Runs probe `probe` once and writes its rate to *ops_per_s. Synchronous: waits for the
 * launch. blocks >= 1, iters >= 1. Allocates and frees a small device buffer (one word per
 * thread) for the chains' results. EINVAL for an unknown probe or bad sizes; EDEVICE/ENOMEM
 * on HIP errors. */
polydet_status polydet_calibrate_alu(int32_t probe, int32_t blocks, int32_t iters,
                                     double* ops_per_s, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* POLYDET_CALIBRATE_H */
