// Host-side plan of the modular determinant (Algorithm 1 of Wei & Chen, arXiv 2010.12117):
// degree bound and power-of-two grid, coefficient bound and prime count (Section 2, after
// Algorithm 1, and equation "primes"), per-prime constants and root-of-unity tables,
// mixed-radix (Garner) tables of Section 3.4, and the workspace layout of one solve.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "modarith.h"

namespace pd {

constexpr int kMaxVars = 8;
constexpr int kMaxN = 32;          // largest matrix order with a compiled elimination kernel
constexpr int kMaxEntryDeg = 31;   // per-variable entry degree (evaluation kernel registers)
constexpr int kMaxGrid = 4096;     // per-variable grid (interpolation tile in LDS)
constexpr int kMaxPrimes = 32;     // reconstruction kernel registers
constexpr int kLLMaxN = 16;        // largest order with a left-looking elimination kernel
constexpr int kLLMaxM = 8;         // its limit on coefficients in the first variable

// Fused first-variable evaluation in pairs, for 2 <= m0 <= 6 coefficients in the first
// variable (its grid N0 is then even): lanes l and l + 32 of a wave take the points j0 and
// j0 + N0/2. Since w^{N0/2} = -1, f(w^{j0 + N0/2}) = E - O where f(w^{j0}) = E + O splits f
// into its even and odd terms; the lower lane sums the even terms, the upper lane the odd
// ones (fused_pair_terms of them, under one reduction), and they exchange the sums. A block
// then covers the first variable's grid index j0 in [0, N0/2) only, with half as many
// matrices per j-row.
PD_HD bool fused_paired(int m0) { return m0 >= 2 && m0 <= 6; }
PD_HD int fused_pair_terms(int m0) { return m0 <= 4 ? 2 : 3; }
// Class of the launch-mapping and rate tables (polydet_tuning, polydet_rates): 0 for a first
// variable with 2..4 coefficients, 1 for every other plan.
PD_HD int tune_class(int k, int m0) { return (k >= 1 && m0 >= 2 && m0 <= 4) ? 0 : 1; }
PD_HD int fused_jrange(int N0, int m0) { return fused_paired(m0) ? N0 / 2 : N0; }
// matrices (lane groups) in one j-row of a block of `block` lanes
PD_HD int fused_slots(int block, int lanes, int m0) {
  return (fused_paired(m0) ? block / 2 : block) / lanes;
}

// Evaluation passes (expand kernel) compute the outputs j and j + Nv/2 of a line together
// when the line has m >= 2 coefficients; their threads cover j in [0, expand_jrange).
PD_HD bool expand_paired(int Nv, int m) { return m >= 2 && Nv >= 2; }
PD_HD int expand_jrange(int Nv, int m) { return expand_paired(Nv, m) ? Nv / 2 : Nv; }

// LDS words of a fused elimination block's tile: m0 coefficient rows of Q points, each a
// matrix whose n rows are padded to a multiple of the lanes per matrix, with an odd stride.
PD_HD size_t fused_tile_words(int n, int lanes, int m0, int Q) {
  const int ncp = (n + lanes - 1) / lanes * lanes;
  return (size_t)((n * ncp) | 1) * m0 * Q;
}

// Launch-mapping table (polydet_tuning): [class][n], 0 = built-in choice. Class 0 is a first
// variable with 2..4 coefficients (paired evaluation), class 1 every other fused matrix.
struct Tuning {
  int lanes[2][kMaxN + 1] = {};
  int left_looking[2][kMaxN + 1] = {};
  int tile_points[2][kMaxN + 1] = {};
};
void set_tuning(const Tuning& t);
Tuning get_tuning();

// Rates of the running-time prediction (polydet_rates); the defaults are rough MI355X values
// used where no measured table is installed (0 entries of a table).
struct Rates {
  double det_updates_per_s[2][kMaxN + 1];
  double reduce_bytes_per_s = 1.0e12;
  double eval_bytes_per_s = 2.0e12;
  double intt_bytes_per_s = 1.2e12;
  double garner_ops_per_s = 2.0e12;
  double launch_us = 4.0;
  Rates() {
    for (auto& c : det_updates_per_s)
      for (auto& x : c) x = 3.5e12;
  }
};
void set_rates(const Rates& r);
Rates get_rates();

// The descending table of primes p in (2^29, 2^30) with p = 1 mod 2^16 (784 of them).
const std::vector<uint32_t>& prime_table();
uint32_t primitive_root(uint32_t p);
uint32_t powmod(uint32_t b, uint64_t e, uint32_t p);

struct MatPlan {
  int n = 0, k = 0;
  int deg[kMaxVars] = {0}, D[kMaxVars] = {0}, N[kMaxVars] = {0}, m[kMaxVars] = {0};
  int64_t G = 1, C = 1, T = 1, nent = 0;
  int pn = 0, L = 0, prime_off = 0, det_lanes = 1;
  int prime_group = 0;  // primes per S1-S4 pass (pn unless the workspace is capped)
  // Slabs of the grid along variable 1 (capped plans whose single prime does not fit): the
  // pass over variable 1 and the elimination run slab by slab on a pre-tensor of R / slabs
  // points; the determinants still fill the whole grid. 1 = the whole grid at once.
  int slabs = 1;
  std::vector<uint32_t> primes;
  std::vector<PrimeConst> pc;
  std::vector<uint8_t> entry_zero;  // empty when the plan was built without coefficients
  // Evaluated entries ("slots"): reduce and the evaluation passes run over nslot entries, slot
  // u holding input entry slot_src[u]; the elimination finds entry e (elimination order) at
  // slot entry_slot[e] (-1 for a zero entry). With coefficients and the fused evaluation the
  // slots are the distinct nonzero entries (equal coefficient boxes share one slot: the
  // replication of entries, e.g. in Sylvester matrices); otherwise every entry in elimination
  // order.
  int64_t nslot = 0;
  std::vector<int32_t> slot_src, entry_slot;
  // Rows in elimination order: row i of the matrix the kernels see is input row
  // row_order[i]. Chosen on the host from the zero pattern so that no pivot is structurally
  // zero; det_sign is the sign of that permutation.
  std::vector<int> row_order;
  int det_sign = 1;
  double log2_bound_sq = 0;         // upper estimate of log2(B^2)

  // device tables (inside the plan's single device allocation)
  const PrimeConst* d_pc = nullptr;
  const uint32_t* d_tw = nullptr;    // [pn][tw_stride]: forward w_v^t at tw_off[v] + t
  const uint32_t* d_itw = nullptr;   // same layout, w_v^{-t}
  int64_t tw_off[kMaxVars] = {0};
  int64_t tw_stride = 0;
  const uint32_t* d_gw = nullptr;    // [pn][pn] Garner weights (Montgomery): (p_0..p_{j-1}) mod p_i
  const uint32_t* d_gc = nullptr;    // [pn] (p_0..p_{i-1})^{-1} mod p_i (Montgomery)
  const uint32_t* d_mlimbs = nullptr;  // [L] M = p_0..p_{pn-1}
  const uint32_t* d_hlimbs = nullptr;  // [L] (M-1)/2
  const uint8_t* d_zero = nullptr;     // [nent] or null (in elimination row order)
  const int32_t* d_slot_src = nullptr;    // [nslot] input entry of each slot
  const int32_t* d_entry_slot = nullptr;  // [nent] slot of each entry (elimination order)
  const uint8_t* d_slot_zero = nullptr;   // zero flags by slot for the evaluation passes (or null)

  // fused first-variable evaluation + elimination (det_fused_kernel)
  bool fused = false;
  bool det_ll = false;  // left-looking elimination pass before the exchanging kernel
  int fuse_Q = 1, fuse_S = 1;
  size_t off_pre = 0;  // [pn][n*n][m0][R] input of the fused kernel

  // workspace layout (bytes, 256-aligned)
  size_t off_res = 0, off_tmpA = 0, off_tmpB = 0, off_eval = 0, off_detv = 0, off_den = 0,
         off_coef = 0,
         off_iA = 0, off_iB = 0, ws_bytes = 0;
  size_t in_bytes = 0, out_bytes = 0;
  double predicted_ms = 0;  // predict_ms with the rates installed when the plan was built
};

// Predicted device milliseconds of polydet_solve on plan P.
double predict_ms(const MatPlan& P, const Rates& r);

struct Plan {
  std::vector<MatPlan> mats;
  bool batch = false;
  bool host_only = false;
  int device = 0;
  void* d_tables = nullptr;  // one device allocation for every table of every matrix
  size_t ws_bytes = 0;       // workspace of one solve (a batch reuses it matrix by matrix)
};

struct ShapeIn {
  int n, k;
  int deg[kMaxVars];
  int coeff_bits;
};

// Fills everything host-side (no device work). max_ws > 0 caps the workspace of one solve
// (primes are then taken in groups of prime_group). Returns an empty string on success or an
// error message; *unsupported tells EUNSUPPORTED from EINVAL.
std::string build_matplan(const ShapeIn& s, const int64_t* host_coeffs, uint32_t flags,
                          size_t max_ws, MatPlan* out, bool* unsupported);

// The plan of primes [b, e) of P: the same tables offset to prime b, pn = e - b, the
// per-prime workspace regions of a group, and the coefficient residues written at prime b's
// slot of P's coefficient region. Only S1-S4 may run on it.
MatPlan prime_range_plan(const MatPlan& P, int b, int e);

// Serialises the device tables of every matrix, uploads them in one allocation and sets
// the d_* pointers. Returns a HIP error code (0 = success).
int upload_tables(Plan* plan);

}  // namespace pd
