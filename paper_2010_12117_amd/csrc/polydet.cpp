// C-ABI of the library (include/polydet.h): plan construction, queries and the solve that
// enqueues the stages of Algorithm 1 (Wei & Chen, arXiv 2010.12117) on one stream.
#include "polydet.h"

#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "abi_internal.h"
#include "batch_plan.h"
#include "kernels.h"
#include "plan.h"

// Ring of event sets for POLYDET_STAGE_TIMING: a slot is read back (and its times added
// to the sums) only before it is reused or when the caller asks for the times.
struct StageTimer {
  static constexpr int kSlots = 256;
  static constexpr int kEvents = POLYDET_NUM_STAGES + 1;
  hipEvent_t ev[kSlots][kEvents] = {};
  bool pending[kSlots] = {};
  int64_t next = 0, solves = 0;
  double ms[POLYDET_NUM_STAGES] = {0};
  bool ready = false;
};

// POLYDET_STAGE_TIMING for batched solves: an event before and after every launch, read back
// (and added to the stage of the launch's kind) before the next solve records them again.
struct BatchTimer {
  std::vector<hipEvent_t> ev;  // [2 * launches]
  bool pending = false;
  int64_t solves = 0;
  double ms[POLYDET_NUM_STAGES] = {0};
};

// Device state of a batched solve: the descriptor tables and the offset arrays, and the extra
// streams on which a chunk's elimination launches run side by side.
struct BatchState {
  pd::BatchPlan bp;
  uint8_t* d_desc = nullptr;
  int64_t* d_offsets = nullptr;          // [2][count]: coefficient offsets, output offsets
  std::vector<int64_t> h_offsets;        // what d_offsets holds
  bool plain = false;
  BatchTimer* timer = nullptr;
  std::vector<hipStream_t> side;         // default-priority streams beside the caller's
  hipEvent_t fork = nullptr;             // recorded on the caller's stream before a fork
  std::vector<hipEvent_t> join;          // one per side stream, waited for at the join
  std::mutex mu;                         // one host thread at a time enqueues a solve
};

struct polydet_plan_s {
  pd::Plan plan;
  StageTimer* timer = nullptr;
  BatchState* batch = nullptr;
};

namespace {

thread_local std::string g_last_error;

polydet_status fail(polydet_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

polydet_status hip_fail(hipError_t err, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(err);
  return err == hipErrorOutOfMemory ? POLYDET_ENOMEM : POLYDET_EDEVICE;
}

polydet_status check_shape(const polydet_shape* s, pd::ShapeIn* out) {
  if (!s) return fail(POLYDET_EINVAL, "shape is NULL");
  out->n = s->n;
  out->k = s->nvars;
  out->coeff_bits = s->coeff_bits;
  if (s->nvars < 0 || s->nvars > POLYDET_MAX_VARS) return fail(POLYDET_EINVAL, "nvars must be in 0..8");
  for (int v = 0; v < POLYDET_MAX_VARS; ++v) out->deg[v] = v < s->nvars ? s->deg[v] : 0;
  return POLYDET_OK;
}

constexpr size_t kBatchBudget = size_t(16) << 30;  // default workspace per chunk of a batch
// Streams of a batched solve: 2 runs consecutive chunks side by side (each in its own half
// of the workspace, on the caller's stream and one of the plan's), so that a chunk's
// memory-bound passes overlap the next chunk's elimination; 1 runs every launch on the
// caller's stream, chunks of the whole budget.
constexpr int kBatchStreams = 2;

int batch_streams() {
  const char* v = std::getenv("POLYDET_BATCH_STREAMS");
  if (v && *v) {
    const int k = std::atoi(v);
    if (k == 1 || k == 2) return k;
  }
  return kBatchStreams;
}

size_t batch_budget() {
  const char* v = std::getenv("POLYDET_BATCH_BUDGET_MB");
  if (v && *v) {
    const long long mb = std::atoll(v);
    if (mb > 0) return (size_t)mb << 20;
  }
  return kBatchBudget;
}

polydet_status make_batch(polydet_plan_s* h, uint32_t flags) {
  BatchState* B = new (std::nothrow) BatchState();
  if (!B) return fail(POLYDET_ENOMEM, "host allocation failed");
  h->batch = B;
  B->plain = (flags & POLYDET_BATCH_PLAIN) != 0;
  if (B->plain) return POLYDET_OK;
  const int ns = batch_streams();
  std::string err = pd::build_batch(h->plan.mats, batch_budget(), ns == 2, &B->bp);
  if (!err.empty()) return fail(POLYDET_EINVAL, err);
  h->plan.ws_bytes = B->bp.ws_bytes;
  hipError_t e = hipMalloc((void**)&B->d_desc, std::max<size_t>(B->bp.desc_blob.size(), 256));
  if (e != hipSuccess) return hip_fail(e, "batch descriptors");
  if (!B->bp.desc_blob.empty()) {
    e = hipMemcpy(B->d_desc, B->bp.desc_blob.data(), B->bp.desc_blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch descriptors");
  }
  e = hipMalloc((void**)&B->d_offsets, 2 * sizeof(int64_t) * h->plan.mats.size());
  if (e != hipSuccess) return hip_fail(e, "batch offsets");
  if (flags & POLYDET_STAGE_TIMING) {
    B->timer = new (std::nothrow) BatchTimer();
    if (!B->timer) return fail(POLYDET_ENOMEM, "host allocation failed");
    B->timer->ev.assign(2 * B->bp.launches.size(), nullptr);
    for (auto& ev : B->timer->ev) {
      if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    return POLYDET_OK;  // timed solves keep every launch on the caller's stream, in order
  }
  if (B->bp.halves && B->bp.chunks > 1) {
    if ((e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreateWithFlags");
    hipStream_t sst = nullptr;
    hipEvent_t ev = nullptr;
    if ((e = hipStreamCreateWithFlags(&sst, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "hipStreamCreateWithFlags");
    B->side.push_back(sst);
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreateWithFlags");
    B->join.push_back(ev);
  }
  return POLYDET_OK;
}

polydet_status make_plan(const polydet_shape* shapes, int32_t count,
                         const int64_t* const* host_coeffs, uint32_t flags, bool batch,
                         size_t max_ws, polydet_plan_t* out) {
  if (!out) return fail(POLYDET_EINVAL, "output plan pointer is NULL");
  *out = nullptr;
  if (!shapes || count < 1) return fail(POLYDET_EINVAL, "need at least one shape");
  polydet_plan_s* h = new (std::nothrow) polydet_plan_s();
  if (!h) return fail(POLYDET_ENOMEM, "host allocation failed");
  h->plan.batch = batch;
  h->plan.mats.resize(count);
  for (int32_t i = 0; i < count; ++i) {
    pd::ShapeIn s;
    polydet_status st = check_shape(&shapes[i], &s);
    if (st != POLYDET_OK) {
      delete h;
      return st;
    }
    bool unsupported = false;
    const int64_t* hc = host_coeffs ? host_coeffs[i] : nullptr;
    std::string err = pd::build_matplan(s, hc, flags, max_ws, &h->plan.mats[i], &unsupported);
    if (err.empty() && (flags & POLYDET_STAGE_TIMING) &&
        (h->plan.mats[i].prime_group < h->plan.mats[i].pn || h->plan.mats[i].slabs > 1))
      err = "stage timing needs a plan that solves all primes at once (no workspace cap)";
    if (err.empty() && !pd::det_config_supported(s.n, h->plan.mats[i].det_lanes)) {
      unsupported = true;
      err = "no elimination kernel for this order and lane count";
    }
    if (!err.empty()) {
      delete h;
      return fail(unsupported ? POLYDET_EUNSUPPORTED : POLYDET_EINVAL,
                  (batch ? "matrix " + std::to_string(i) + ": " : std::string()) + err);
    }
    h->plan.ws_bytes = std::max(h->plan.ws_bytes, h->plan.mats[i].ws_bytes);
  }
  h->plan.host_only = (flags & POLYDET_HOST_ONLY) != 0;
  if (h->plan.host_only) {
    *out = h;
    g_last_error.clear();
    return POLYDET_OK;
  }
  hipError_t e = hipGetDevice(&h->plan.device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipGetDevice");
  }
  const int up = pd::upload_tables(&h->plan);
  if (up != 0) {
    delete h;
    return hip_fail((hipError_t)up, "uploading plan tables");
  }
  if (batch) {
    polydet_status bs = make_batch(h, flags);
    if (bs != POLYDET_OK) {
      polydet_plan_destroy(h);
      return bs;
    }
  }
  if ((flags & POLYDET_STAGE_TIMING) && !(h->batch && h->batch->timer)) {
    h->timer = new (std::nothrow) StageTimer();
    if (!h->timer) {
      polydet_plan_destroy(h);
      return fail(POLYDET_ENOMEM, "host allocation failed");
    }
    for (auto& slot : h->timer->ev) {
      for (auto& ev : slot) {
        hipError_t ee = hipEventCreate(&ev);
        if (ee != hipSuccess) {
          polydet_plan_destroy(h);
          return hip_fail(ee, "hipEventCreate");
        }
      }
    }
    h->timer->ready = true;
  }
  *out = h;
  g_last_error.clear();
  return POLYDET_OK;
}

hipError_t harvest(StageTimer* T, int slot) {
  if (!T->pending[slot]) return hipSuccess;
  hipError_t e = hipEventSynchronize(T->ev[slot][StageTimer::kEvents - 1]);
  if (e != hipSuccess) return e;
  for (int s = 0; s < POLYDET_NUM_STAGES; ++s) {
    float ms = 0;
    e = hipEventElapsedTime(&ms, T->ev[slot][s], T->ev[slot][s + 1]);
    if (e != hipSuccess) return e;
    T->ms[s] += ms;
  }
  T->pending[slot] = false;
  T->solves += 1;
  return hipSuccess;
}

int stage_of(pd::BLaunch::Kind k) {
  switch (k) {
    case pd::BLaunch::kReduce: return 0;
    case pd::BLaunch::kExpand: return 1;
    case pd::BLaunch::kDet: return 2;
    case pd::BLaunch::kIntt: return 4;
    default: return 5;
  }
}

hipError_t harvest_batch(BatchState* B) {
  BatchTimer* T = B->timer;
  if (!T || !T->pending) return hipSuccess;
  const size_t nl = B->bp.launches.size();
  if (nl == 0) {
    T->pending = false;
    T->solves += 1;
    return hipSuccess;
  }
  hipError_t e = hipEventSynchronize(T->ev[2 * nl - 1]);
  if (e != hipSuccess) return e;
  for (size_t i = 0; i < nl; ++i) {
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, T->ev[2 * i], T->ev[2 * i + 1])) != hipSuccess) return e;
    T->ms[stage_of(B->bp.launches[i].kind)] += ms;
  }
  T->pending = false;
  T->solves += 1;
  return hipSuccess;
}

// S1-S4 for primes [b, e), prime_group at a time; each group leaves its coefficient residues
// in the coefficient region.
polydet_status run_primes(const pd::MatPlan& P, const int64_t* d_coeffs, int b, int e,
                          uint8_t* ws, hipStream_t st) {
  hipError_t err;
  const int g = P.prime_group > 0 ? P.prime_group : P.pn;
  for (int lo = b; lo < e; lo += g) {
    const pd::MatPlan R = pd::prime_range_plan(P, lo, std::min(e, lo + g));
    if (R.slabs > 1) {
      if ((err = pd::run_reduce(R, d_coeffs, ws, st)) != hipSuccess) return hip_fail(err, "reduce");
      // one prime's grid in slabs along variable 1: the pre-tensor holds one slab at a time,
      // the determinants fill the whole grid
      if ((err = pd::run_evaluate_upper(R, ws, st)) != hipSuccess) return hip_fail(err, "evaluate");
      for (int b = 0; b < R.slabs; ++b) {
        if ((err = pd::run_evaluate_slab(R, ws, b, st)) != hipSuccess)
          return hip_fail(err, "evaluate");
        if ((err = pd::run_det_slab(R, ws, b, st)) != hipSuccess)
          return hip_fail(err, "determinants");
      }
    } else {
      if ((err = pd::run_reduce_evaluate(R, d_coeffs, ws, st)) != hipSuccess)
        return hip_fail(err, "reduce and evaluate");
      if ((err = pd::run_det(R, ws, st)) != hipSuccess) return hip_fail(err, "determinants");
    }
    if ((err = pd::run_finalize(R, ws, st)) != hipSuccess) return hip_fail(err, "finalize");
    if ((err = pd::run_interpolate(R, ws, st)) != hipSuccess) return hip_fail(err, "interpolate");
  }
  return POLYDET_OK;
}

// One stage of a solve: S1 reduce, S2 evaluate, S3 determinants (numerators and
// denominators), S3 end (finalize: the division, a launch of its own only without variables),
// S4 interpolate, S5 reconstruct.
hipError_t run_stage(const pd::MatPlan& P, int stage, const int64_t* d_coeffs, uint32_t* d_out,
                     uint8_t* ws, hipStream_t st) {
  switch (stage) {
    case 0: return pd::run_reduce(P, d_coeffs, ws, st);
    case 1: return pd::run_evaluate(P, ws, st);
    case 2: return pd::run_det(P, ws, st);
    case 3: return pd::run_finalize(P, ws, st);
    case 4: return pd::run_interpolate(P, ws, st);
    default: return pd::run_reconstruct(P, ws, d_out, st);
  }
}

const char* const kStageNames[POLYDET_NUM_STAGES] = {"reduce", "evaluate", "determinants",
                                                     "finalize", "interpolate", "reconstruct"};

// Stages [b, e) of the solve of P (all primes at once), with the plan's stage events if any.
polydet_status run_stages(const pd::MatPlan& P, int b, int e, const int64_t* d_coeffs,
                          uint32_t* d_out, uint8_t* ws, hipStream_t st, StageTimer* T) {
  hipError_t err;
  hipEvent_t* ev = nullptr;
  if (T) {
    const int slot = (int)(T->next++ % StageTimer::kSlots);
    if ((err = harvest(T, slot)) != hipSuccess) return hip_fail(err, "stage timing");
    ev = T->ev[slot];
    T->pending[slot] = true;
    // stages outside [b, e) read as zero: their two events are recorded back to back
    for (int s = 0; s <= b; ++s) {
      if ((err = hipEventRecord(ev[s], st)) != hipSuccess) return hip_fail(err, "stage timing");
    }
  }
  for (int s = b; s < e; ++s) {
    if (s == 0 && e >= 2 && !ev) {
      // S1 and S2 in one go: the first evaluation pass reduces the coefficients itself
      if ((err = pd::run_reduce_evaluate(P, d_coeffs, ws, st)) != hipSuccess)
        return hip_fail(err, "reduce and evaluate");
      s = 1;
      continue;
    }
    if (s == 4 && e == POLYDET_NUM_STAGES && !ev) {
      // S4 and S5 in one go: the last interpolation pass reconstructs the coefficients too
      if ((err = pd::run_interpolate_reconstruct(P, ws, d_out, st)) != hipSuccess)
        return hip_fail(err, "interpolate and reconstruct");
      break;
    }
    if ((err = run_stage(P, s, d_coeffs, d_out, ws, st)) != hipSuccess)
      return hip_fail(err, kStageNames[s]);
    if (ev && (err = hipEventRecord(ev[s + 1], st)) != hipSuccess)
      return hip_fail(err, "stage timing");
  }
  for (int s = e + 1; ev && s <= POLYDET_NUM_STAGES; ++s) {
    if ((err = hipEventRecord(ev[s], st)) != hipSuccess) return hip_fail(err, "stage timing");
  }
  return POLYDET_OK;
}

polydet_status run_one(const pd::MatPlan& P, const int64_t* d_coeffs, uint32_t* d_out,
                       uint8_t* ws, hipStream_t st, StageTimer* T) {
  if (P.prime_group < P.pn || P.slabs > 1) {  // capped: S1-S4 by prime groups (and slabs), S5
    polydet_status s = run_primes(P, d_coeffs, 0, P.pn, ws, st);
    if (s != POLYDET_OK) return s;
    hipError_t e = pd::run_reconstruct(P, ws, d_out, st);
    return e == hipSuccess ? POLYDET_OK : hip_fail(e, "reconstruct");
  }
  return run_stages(P, 0, POLYDET_NUM_STAGES, d_coeffs, d_out, ws, st, T);
}

polydet_status check_device(const pd::Plan& plan) {
  if (plan.host_only) return fail(POLYDET_EINVAL, "a host-only plan cannot be solved");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan.device) {
    return fail(POLYDET_EINVAL, "the current device differs from the plan's device " +
                                    std::to_string(plan.device));
  }
  return POLYDET_OK;
}

}  // namespace

polydet_status pd::abi_fail(polydet_status st, const std::string& msg) { return fail(st, msg); }

extern "C" {

polydet_status polydet_plan(const polydet_shape* shape, const int64_t* host_coeffs,
                            uint32_t flags, polydet_plan_t* out) {
  const int64_t* hc[1] = {host_coeffs};
  return make_plan(shape, 1, hc, flags, false, 0, out);
}

polydet_status polydet_plan_capped(const polydet_shape* shape, const int64_t* host_coeffs,
                                   uint32_t flags, size_t max_workspace_bytes,
                                   polydet_plan_t* out) {
  const int64_t* hc[1] = {host_coeffs};
  return make_plan(shape, 1, hc, flags, false, max_workspace_bytes, out);
}

polydet_status polydet_plan_batch(const polydet_shape* shapes, int32_t count,
                                  const int64_t* const* host_coeffs, uint32_t flags,
                                  polydet_plan_t* out) {
  return make_plan(shapes, count, host_coeffs, flags, true, 0, out);
}

polydet_status polydet_plan_query(polydet_plan_t plan, int32_t index, polydet_plan_info* out) {
  if (!plan || !out) return fail(POLYDET_EINVAL, "NULL plan or output");
  if (index < 0 || index >= (int32_t)plan->plan.mats.size()) return fail(POLYDET_EINVAL, "index out of range");
  const pd::MatPlan& P = plan->plan.mats[index];
  std::memset(out, 0, sizeof(*out));
  out->n = P.n;
  out->nvars = P.k;
  for (int v = 0; v < P.k; ++v) {
    out->deg[v] = P.deg[v];
    out->D[v] = P.D[v];
    out->N[v] = P.N[v];
  }
  out->G = P.G;
  out->ncoeff = P.C;
  out->nterms = P.T;
  out->pn = P.pn;
  out->limbs = P.L;
  out->det_lanes = P.det_lanes;
  out->det_sign = P.det_sign;
  for (int i = 0; i < P.n && i < 32; ++i) out->row_order[i] = (uint8_t)P.row_order[i];
  out->det_left_looking = P.det_ll ? 1 : 0;
  out->prime_group = P.prime_group;
  out->grid_slabs = P.slabs;
  out->coef_bytes = (size_t)P.pn * P.C * 4;
  out->in_bytes = P.in_bytes;
  out->out_bytes = P.out_bytes;
  out->workspace_bytes = plan->plan.batch ? plan->plan.ws_bytes : P.ws_bytes;
  out->off_eval = P.off_eval;
  out->off_detv = P.off_detv;
  out->off_coef = P.off_coef;
  out->off_den = P.off_den;
  out->nslots = P.nslot;
  out->predicted_ms = P.predicted_ms;
  return POLYDET_OK;
}

polydet_status polydet_plan_primes(polydet_plan_t plan, int32_t index, uint32_t* out,
                                   int32_t capacity) {
  if (!plan || !out) return fail(POLYDET_EINVAL, "NULL plan or output");
  if (index < 0 || index >= (int32_t)plan->plan.mats.size()) return fail(POLYDET_EINVAL, "index out of range");
  const pd::MatPlan& P = plan->plan.mats[index];
  if (capacity < P.pn) return fail(POLYDET_EINVAL, "capacity below the prime count");
  std::memcpy(out, P.primes.data(), 4 * P.pn);
  return POLYDET_OK;
}

polydet_status polydet_solve(polydet_plan_t plan, const int64_t* d_coeffs, uint32_t* d_out,
                             void* d_workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return fail(POLYDET_EINVAL, "NULL plan");
  if (plan->plan.batch) return fail(POLYDET_EINVAL, "batch plans are solved by polydet_solve_batch");
  if (!d_coeffs || !d_out || !d_workspace) return fail(POLYDET_EINVAL, "NULL buffer");
  const pd::MatPlan& P = plan->plan.mats[0];
  if (workspace_bytes < P.ws_bytes) return fail(POLYDET_EINVAL, "workspace too small");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(POLYDET_EINVAL, "workspace must be 256-byte aligned");
  polydet_status st = check_device(plan->plan);
  if (st != POLYDET_OK) return st;
  return run_one(P, d_coeffs, d_out, (uint8_t*)d_workspace, (hipStream_t)stream, plan->timer);
}

polydet_status polydet_solve_stages(polydet_plan_t plan, int32_t stage_begin, int32_t stage_end,
                                    const int64_t* d_coeffs, uint32_t* d_out, void* d_workspace,
                                    size_t workspace_bytes, void* stream) {
  if (!plan) return fail(POLYDET_EINVAL, "NULL plan");
  if (plan->plan.batch) return fail(POLYDET_EINVAL, "batch plans are solved by polydet_solve_batch");
  if (stage_begin < 0 || stage_end > POLYDET_NUM_STAGES || stage_begin >= stage_end)
    return fail(POLYDET_EINVAL, "stages must satisfy 0 <= begin < end <= POLYDET_NUM_STAGES");
  if (!d_workspace) return fail(POLYDET_EINVAL, "NULL workspace");
  if (stage_begin == 0 && !d_coeffs) return fail(POLYDET_EINVAL, "NULL coefficients");
  if (stage_end == POLYDET_NUM_STAGES && !d_out) return fail(POLYDET_EINVAL, "NULL output");
  const pd::MatPlan& P = plan->plan.mats[0];
  if (P.prime_group < P.pn || P.slabs > 1)
    return fail(POLYDET_EINVAL, "a capped plan runs by prime ranges (polydet_solve_primes)");
  if (workspace_bytes < P.ws_bytes) return fail(POLYDET_EINVAL, "workspace too small");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(POLYDET_EINVAL, "workspace must be 256-byte aligned");
  polydet_status st = check_device(plan->plan);
  if (st != POLYDET_OK) return st;
  return run_stages(P, stage_begin, stage_end, d_coeffs, d_out, (uint8_t*)d_workspace,
                    (hipStream_t)stream, plan->timer);
}

static polydet_status check_single(polydet_plan_t plan, void* d_workspace,
                                   size_t workspace_bytes) {
  if (!plan) return fail(POLYDET_EINVAL, "NULL plan");
  if (plan->plan.batch) return fail(POLYDET_EINVAL, "a batch plan cannot be solved by ranges");
  if (!d_workspace) return fail(POLYDET_EINVAL, "NULL workspace");
  if (workspace_bytes < plan->plan.mats[0].ws_bytes) return fail(POLYDET_EINVAL, "workspace too small");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(POLYDET_EINVAL, "workspace must be 256-byte aligned");
  return check_device(plan->plan);
}

polydet_status polydet_solve_primes(polydet_plan_t plan, const int64_t* d_coeffs,
                                    int32_t prime_begin, int32_t prime_end, void* d_workspace,
                                    size_t workspace_bytes, void* stream) {
  polydet_status st = check_single(plan, d_workspace, workspace_bytes);
  if (st != POLYDET_OK) return st;
  const pd::MatPlan& P = plan->plan.mats[0];
  if (!d_coeffs) return fail(POLYDET_EINVAL, "NULL coefficients");
  if (prime_begin < 0 || prime_end > P.pn || prime_begin >= prime_end)
    return fail(POLYDET_EINVAL, "prime range must satisfy 0 <= begin < end <= pn");
  return run_primes(P, d_coeffs, prime_begin, prime_end, (uint8_t*)d_workspace,
                    (hipStream_t)stream);
}

polydet_status polydet_reconstruct(polydet_plan_t plan, void* d_workspace,
                                   size_t workspace_bytes, uint32_t* d_out, void* stream) {
  polydet_status st = check_single(plan, d_workspace, workspace_bytes);
  if (st != POLYDET_OK) return st;
  if (!d_out) return fail(POLYDET_EINVAL, "NULL output");
  hipError_t e = pd::run_reconstruct(plan->plan.mats[0], (uint8_t*)d_workspace, d_out,
                                     (hipStream_t)stream);
  return e == hipSuccess ? POLYDET_OK : hip_fail(e, "reconstruct");
}

static polydet_status run_batched(polydet_plan_t plan, const int64_t* d_coeffs,
                           const int64_t* coeff_offsets, uint32_t* d_out,
                           const int64_t* out_offsets, uint8_t* ws, hipStream_t st) {
  BatchState* B = plan->batch;
  // the offsets, the timer and the fork/join events are the plan's: solves issued from
  // several host threads take turns
  std::lock_guard<std::mutex> lk(B->mu);
  const size_t count = plan->plan.mats.size();
  // device copies of the offsets, refreshed on the stream only when they change
  bool same = B->h_offsets.size() == 2 * count;
  for (size_t i = 0; same && i < count; ++i) {
    same = B->h_offsets[i] == coeff_offsets[i] && B->h_offsets[count + i] == out_offsets[i];
  }
  if (!same) {
    B->h_offsets.assign(coeff_offsets, coeff_offsets + count);
    B->h_offsets.insert(B->h_offsets.end(), out_offsets, out_offsets + count);
    // ordered after earlier work on the stream; waited for, since the host copy is
    // pageable and replaced by the next call with other offsets
    hipError_t e = hipMemcpyAsync(B->d_offsets, B->h_offsets.data(), 2 * count * sizeof(int64_t),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "batch offsets");
  }
  const int64_t* d_coff = B->d_offsets;
  const int64_t* d_ooff = B->d_offsets + count;
  BatchTimer* T = B->timer;
  if (T) {
    hipError_t e = harvest_batch(B);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
    T->pending = true;
  }
  const size_t nl = B->bp.launches.size();
  // chunks side by side: odd chunks on the plan's stream, forked from the caller's stream
  // after the offsets are in place and joined back before the matrices solved one by one
  const bool side = !B->side.empty() && !T;
  if (side) {
    hipError_t e = hipEventRecord(B->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(B->side[0], B->fork, 0);
    if (e != hipSuccess) return hip_fail(e, "batch fork");
  }
  for (size_t li = 0; li < nl; ++li) {
    const pd::BLaunch& L = B->bp.launches[li];
    const void* desc = B->d_desc + L.desc_off;
    hipError_t e = hipSuccess;
    const hipStream_t ls = side && (L.chunk % 2) ? B->side[0] : st;  // the launch's stream
    if (T && (e = hipEventRecord(T->ev[2 * li], ls)) != hipSuccess) return hip_fail(e, "stage timing");
    switch (L.kind) {
      case pd::BLaunch::kReduce:
        e = pd::batch_reduce((const pd::BReduce*)desc, L.ndesc, L.vblocks, d_coeffs, d_coff, ws, ls);
        break;
      case pd::BLaunch::kExpand:
        e = pd::batch_expand((const pd::BExpand*)desc, L.ndesc, L.vblocks, ws, ls);
        break;
      case pd::BLaunch::kDet:
        if (L.each) {
          e = pd::batch_det_each(L.n, L.lanes, L.ll == 2,
                                 (const pd::BDet*)(B->bp.desc_blob.data() + L.desc_off), L.ndesc,
                                 L.vblocks, ws, ls);
        } else {
          e = pd::batch_det(L.n, L.lanes, L.ll, L.pair, (const pd::BDet*)desc, L.ndesc,
                            L.vblocks, L.lds, ws, ls);
        }
        break;
      case pd::BLaunch::kIntt:
        e = pd::batch_intt((const pd::BIntt*)desc, L.ndesc, L.vblocks, L.lds, ws, ls);
        break;
      case pd::BLaunch::kGarner:
        e = pd::batch_garner((const pd::BGarner*)desc, L.ndesc, L.vblocks, L.pnmax, ws, d_out,
                             d_ooff, ls);
        break;
    }
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    if (T && (e = hipEventRecord(T->ev[2 * li + 1], ls)) != hipSuccess)
      return hip_fail(e, "stage timing");
  }
  if (side) {
    hipError_t e = hipEventRecord(B->join[0], B->side[0]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, B->join[0], 0);
    if (e != hipSuccess) return hip_fail(e, "batch join");
  }
  for (int i : B->bp.singles) {
    polydet_status r = run_one(plan->plan.mats[i], d_coeffs + coeff_offsets[i],
                               d_out + out_offsets[i], ws, st, nullptr);
    if (r != POLYDET_OK) return r;
  }
  return POLYDET_OK;
}

polydet_status polydet_solve_batch(polydet_plan_t plan, const int64_t* d_coeffs,
                                   const int64_t* coeff_offsets, uint32_t* d_out,
                                   const int64_t* out_offsets, void* d_workspace,
                                   size_t workspace_bytes, void* stream) {
  if (!plan) return fail(POLYDET_EINVAL, "NULL plan");
  if (!plan->plan.batch) return fail(POLYDET_EINVAL, "single-matrix plans are solved by polydet_solve");
  if (!d_coeffs || !d_out || !d_workspace || !coeff_offsets || !out_offsets)
    return fail(POLYDET_EINVAL, "NULL buffer or offsets");
  if (workspace_bytes < plan->plan.ws_bytes) return fail(POLYDET_EINVAL, "workspace too small");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(POLYDET_EINVAL, "workspace must be 256-byte aligned");
  for (size_t i = 0; i < plan->plan.mats.size(); ++i) {
    if (coeff_offsets[i] < 0 || out_offsets[i] < 0) return fail(POLYDET_EINVAL, "negative offset");
  }
  polydet_status st = check_device(plan->plan);
  if (st != POLYDET_OK) return st;
  if (plan->batch && !plan->batch->plain) {
    return run_batched(plan, d_coeffs, coeff_offsets, d_out, out_offsets, (uint8_t*)d_workspace,
                       (hipStream_t)stream);
  }
  for (size_t i = 0; i < plan->plan.mats.size(); ++i) {
    st = run_one(plan->plan.mats[i], d_coeffs + coeff_offsets[i], d_out + out_offsets[i],
                 (uint8_t*)d_workspace, (hipStream_t)stream, plan->timer);
    if (st != POLYDET_OK) return st;
  }
  return POLYDET_OK;
}

polydet_status polydet_stage_times(polydet_plan_t plan, double ms[POLYDET_NUM_STAGES],
                                   int64_t* solves) {
  if (!plan || !ms) return fail(POLYDET_EINVAL, "NULL plan or output");
  if (plan->batch && plan->batch->timer) {
    BatchTimer* BT = plan->batch->timer;
    hipError_t e = harvest_batch(plan->batch);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
    for (int s = 0; s < POLYDET_NUM_STAGES; ++s) {
      ms[s] = BT->ms[s];
      BT->ms[s] = 0;
    }
    if (solves) *solves = BT->solves;
    BT->solves = 0;
    return POLYDET_OK;
  }
  StageTimer* T = plan->timer;
  if (!T) return fail(POLYDET_EINVAL, "the plan was made without POLYDET_STAGE_TIMING");
  for (int slot = 0; slot < StageTimer::kSlots; ++slot) {
    hipError_t e = harvest(T, slot);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
  }
  for (int s = 0; s < POLYDET_NUM_STAGES; ++s) {
    ms[s] = T->ms[s];
    T->ms[s] = 0;
  }
  if (solves) *solves = T->solves;
  T->solves = 0;
  return POLYDET_OK;
}

void polydet_plan_destroy(polydet_plan_t plan) {
  if (!plan) return;
  if (plan->timer) {
    for (int slot = 0; slot < StageTimer::kSlots; ++slot) {
      if (plan->timer->pending[slot]) (void)hipEventSynchronize(plan->timer->ev[slot][StageTimer::kEvents - 1]);
      for (auto& ev : plan->timer->ev[slot]) {
        if (ev) (void)hipEventDestroy(ev);
      }
    }
    delete plan->timer;
  }
  if (plan->batch) {
    if (plan->batch->timer) {
      if (plan->batch->timer->pending && !plan->batch->timer->ev.empty())
        (void)hipEventSynchronize(plan->batch->timer->ev.back());
      for (auto& ev : plan->batch->timer->ev) {
        if (ev) (void)hipEventDestroy(ev);
      }
      delete plan->batch->timer;
    }
    for (hipStream_t sst : plan->batch->side) (void)hipStreamDestroy(sst);
    for (hipEvent_t ev : plan->batch->join) (void)hipEventDestroy(ev);
    if (plan->batch->fork) (void)hipEventDestroy(plan->batch->fork);
    if (plan->batch->d_desc) (void)hipFree(plan->batch->d_desc);
    if (plan->batch->d_offsets) (void)hipFree(plan->batch->d_offsets);
    delete plan->batch;
  }
  if (plan->plan.d_tables) (void)hipFree(plan->plan.d_tables);
  delete plan;
}

const char* polydet_status_string(polydet_status status) {
  switch (status) {
    case POLYDET_OK: return "ok";
    case POLYDET_EINVAL: return "invalid argument";
    case POLYDET_EUNSUPPORTED: return "beyond the library's limits";
    case POLYDET_ENOMEM: return "out of memory";
    case POLYDET_EDEVICE: return "device error";
    case POLYDET_ECANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* polydet_last_error(void) { return g_last_error.c_str(); }

static_assert(POLYDET_TUNE_ORDERS == pd::kMaxN + 1, "tuning table covers orders 0..kMaxN");

polydet_status polydet_set_tuning(const polydet_tuning* table) {
  pd::Tuning t;
  if (table) {
    for (int c = 0; c < 2; ++c) {
      for (int n = 0; n <= pd::kMaxN; ++n) {
        const int lanes = table->lanes[c][n], ll = table->left_looking[c][n];
        const int q = table->tile_points[c][n];
        const bool pow2q = q == 0 || q == 1 || q == 2 || q == 4 || q == 8 || q == 16;
        if (n == 0 && (lanes || ll || q)) return fail(POLYDET_EINVAL, "tuning: order 0 is unused");
        if (lanes != 0 && !pd::det_config_supported(n, lanes))
          return fail(POLYDET_EINVAL, "tuning: lanes per matrix not compiled for this order");
        if (ll < 0 || ll > 2 || (ll == 1 && n > pd::kLLMaxN))
          return fail(POLYDET_EINVAL, "tuning: left_looking must be 0, 1 (n <= 16) or 2");
        if (!pow2q) return fail(POLYDET_EINVAL, "tuning: tile_points must be 0, 1, 2, 4, 8 or 16");
        t.lanes[c][n] = lanes;
        t.left_looking[c][n] = ll;
        t.tile_points[c][n] = q;
      }
    }
  }
  pd::set_tuning(t);
  return POLYDET_OK;
}

polydet_status polydet_get_tuning(polydet_tuning* out) {
  if (!out) return fail(POLYDET_EINVAL, "tuning: null output");
  const pd::Tuning t = pd::get_tuning();
  for (int c = 0; c < 2; ++c) {
    for (int n = 0; n < POLYDET_TUNE_ORDERS; ++n) {
      out->lanes[c][n] = n <= pd::kMaxN ? t.lanes[c][n] : 0;
      out->left_looking[c][n] = n <= pd::kMaxN ? t.left_looking[c][n] : 0;
      out->tile_points[c][n] = n <= pd::kMaxN ? t.tile_points[c][n] : 0;
    }
  }
  return POLYDET_OK;
}

polydet_status polydet_set_rates(const polydet_rates* rates) {
  pd::Rates r;
  if (rates) {
    auto ok = [](double v) { return v >= 0 && v < 1e300; };
    for (int c = 0; c < 2; ++c) {
      for (int n = 0; n <= pd::kMaxN; ++n) {
        const double v = rates->det_updates_per_s[c][n];
        if (!ok(v)) return fail(POLYDET_EINVAL, "rates: negative or non-finite entry");
        if (v > 0) r.det_updates_per_s[c][n] = v;
      }
    }
    const double* scal[5] = {&rates->reduce_bytes_per_s, &rates->eval_bytes_per_s,
                             &rates->intt_bytes_per_s, &rates->garner_ops_per_s,
                             &rates->launch_us};
    double* dst[5] = {&r.reduce_bytes_per_s, &r.eval_bytes_per_s, &r.intt_bytes_per_s,
                      &r.garner_ops_per_s, &r.launch_us};
    for (int i = 0; i < 5; ++i) {
      if (!ok(*scal[i])) return fail(POLYDET_EINVAL, "rates: negative or non-finite entry");
      if (*scal[i] > 0) *dst[i] = *scal[i];
    }
  }
  pd::set_rates(r);
  return POLYDET_OK;
}

polydet_status polydet_get_rates(polydet_rates* out) {
  if (!out) return fail(POLYDET_EINVAL, "rates: null output");
  const pd::Rates r = pd::get_rates();
  std::memset(out, 0, sizeof(*out));
  for (int c = 0; c < 2; ++c) {
    for (int n = 0; n < POLYDET_TUNE_ORDERS; ++n) out->det_updates_per_s[c][n] = r.det_updates_per_s[c][n];
  }
  out->reduce_bytes_per_s = r.reduce_bytes_per_s;
  out->eval_bytes_per_s = r.eval_bytes_per_s;
  out->intt_bytes_per_s = r.intt_bytes_per_s;
  out->garner_ops_per_s = r.garner_ops_per_s;
  out->launch_us = r.launch_us;
  return POLYDET_OK;
}

void polydet_limits(int32_t* max_n, int32_t* max_vars, int32_t* max_grid_per_var,
                    int32_t* max_primes) {
  if (max_n) *max_n = pd::kMaxN;
  if (max_vars) *max_vars = pd::kMaxVars;
  if (max_grid_per_var) *max_grid_per_var = pd::kMaxGrid;
  if (max_primes) *max_primes = pd::kMaxPrimes;
}

}  // extern "C"
