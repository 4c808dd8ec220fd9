"""Exact determinants of multivariate integer-polynomial matrices on MI355X.

The modular method of Wei & Chen (arXiv 2010.12117, Algorithm 1) as hand-written HIP
kernels for gfx950 behind a C ABI (include/polydet.h); this package is the thin Python
binding (binding.py), the build script (build.py), the launch-mapping autotuner
(autotune.py), the calibration of the running-time prediction (calibrate.py) and a request
loop for serving (serving.py).
"""
from .binding import (DET_LANES_LOG2, FORCE_PN, HOST_ONLY, PRIME_OFFSET, STAGE_TIMING, STAGES,
                      UNFUSED_EVAL, BATCH_PLAIN, DET_LEFT_LOOKING, DET_EXCHANGE,
                      Plan, PolydetError,
                      coefficient_region, det, get_rates, get_tuning, limbs_to_ints, limits,
                      load_library, plan, plan_batch, reconstruct_device, set_rates, set_tuning,
                      solve_batch_device, solve_device, solve_primes_device, solve_stages_device)

__all__ = ["DET_LANES_LOG2", "FORCE_PN", "HOST_ONLY", "PRIME_OFFSET", "STAGE_TIMING", "STAGES",
           "UNFUSED_EVAL", "BATCH_PLAIN", "DET_LEFT_LOOKING", "DET_EXCHANGE",
           "Plan", "PolydetError",
           "coefficient_region", "det", "get_rates", "get_tuning", "limbs_to_ints", "limits",
           "load_library", "plan", "plan_batch", "reconstruct_device", "set_rates", "set_tuning",
           "solve_batch_device", "solve_device", "solve_primes_device", "solve_stages_device"]
