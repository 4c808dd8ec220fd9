// Host-side plan: see plan.h.
#include "plan.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

namespace pd {

namespace {

std::mutex g_tuning_mu;
Tuning g_tuning;

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)((unsigned __int128)a * b % m);
}

// Deterministic Miller-Rabin for 32-bit integers (bases 2, 7, 61 cover all n < 4.7e9).
bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t q : {2u, 3u, 5u, 7u, 11u, 13u}) {
    if (n % q == 0) return n == q;
  }
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint32_t a : {2u, 7u, 61u}) {
    if (a % n == 0) continue;
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Little-endian multi-limb helpers for M = prod p_i.
void big_mul_small(std::vector<uint32_t>& a, uint32_t b) {
  uint64_t carry = 0;
  for (auto& x : a) {
    uint64_t t = (uint64_t)x * b + carry;
    x = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry) a.push_back((uint32_t)carry);
}

int big_bitlen(const std::vector<uint32_t>& a) {
  for (int i = (int)a.size() - 1; i >= 0; --i) {
    if (a[i]) return 32 * i + 32 - __builtin_clz(a[i]);
  }
  return 0;
}

}  // namespace

uint32_t powmod(uint32_t b, uint64_t e, uint32_t p) {
  uint64_t r = 1 % p, x = b % p;
  while (e) {
    if (e & 1) r = mulmod64(r, x, p);
    x = mulmod64(x, x, p);
    e >>= 1;
  }
  return (uint32_t)r;
}

const std::vector<uint32_t>& prime_table() {
  static const std::vector<uint32_t> table = [] {
    std::vector<uint32_t> t;
    const uint64_t step = 1ull << 16;
    for (uint64_t c = ((1ull << 30) - 1) / step; c * step + 1 > (1ull << 29); --c) {
      const uint64_t p = c * step + 1;
      if (p < (1ull << 30) && is_prime_u32((uint32_t)p)) t.push_back((uint32_t)p);
    }
    return t;
  }();
  return table;
}

uint32_t primitive_root(uint32_t p) {
  // p - 1 = c * 2^16: its prime factors are 2 and those of c.
  std::vector<uint32_t> qs;
  uint32_t m = p - 1;
  for (uint32_t f = 2; (uint64_t)f * f <= m; ++f) {
    if (m % f == 0) {
      qs.push_back(f);
      while (m % f == 0) m /= f;
    }
  }
  if (m > 1) qs.push_back(m);
  for (uint32_t g = 2;; ++g) {
    bool ok = true;
    for (uint32_t q : qs) {
      if (powmod(g, (p - 1) / q, p) == 1) { ok = false; break; }
    }
    if (ok) return g;
  }
}

static int default_det_lanes(int n) {
  if (n <= 12) return 1;
  if (n <= 16) return 2;
  if (n <= 24) return 4;
  return 8;
}

std::string build_matplan(const ShapeIn& s, const int64_t* host_coeffs, uint32_t flags,
                          size_t max_ws, MatPlan* out, bool* unsupported) {
  *unsupported = false;
  MatPlan P;
  if (s.n < 1) return "matrix order n must be >= 1";
  if (s.k < 0 || s.k > kMaxVars) return "nvars must be in 0..8";
  if (s.coeff_bits < 0 || s.coeff_bits > 63) return "coeff_bits must be in 0..63";
  for (int v = 0; v < s.k; ++v) {
    if (s.deg[v] < 0) return "degrees must be >= 0";
  }
  if (s.n > kMaxN) {
    *unsupported = true;
    return "matrix order above " + std::to_string(kMaxN) + " is not supported";
  }
  P.n = s.n;
  P.k = s.k;
  P.nent = (int64_t)s.n * s.n;
  P.G = P.C = P.T = 1;
  for (int v = 0; v < s.k; ++v) {
    if (s.deg[v] > kMaxEntryDeg) {
      *unsupported = true;
      return "entry degree above " + std::to_string(kMaxEntryDeg) + " is not supported";
    }
    P.deg[v] = s.deg[v];
    P.m[v] = s.deg[v] + 1;
    P.D[v] = s.n * s.deg[v];
    const int64_t Nv = next_pow2((int64_t)P.D[v] + 1);
    if (Nv > kMaxGrid) {
      *unsupported = true;
      return "grid size per variable above " + std::to_string(kMaxGrid) + " is not supported";
    }
    P.N[v] = (int)Nv;
    P.G *= Nv;
    P.C *= P.D[v] + 1;
    P.T *= P.m[v];
  }

  // Bound on the squared coefficients of det M (Hadamard on 1-norms), as log2 with a
  // margin that covers the rounding of the long-double sums many times over.
  long double log2b = 0;
  bool zero_bound = false;
  if (host_coeffs) {
    P.entry_zero.assign(P.nent, 0);
    std::vector<long double> norm(P.nent);
    for (int64_t e = 0; e < P.nent; ++e) {
      long double acc = 0;
      bool nz = false;
      const int64_t* c = host_coeffs + e * P.T;
      for (int64_t t = 0; t < P.T; ++t) {
        if (c[t]) {
          nz = true;
          acc += fabsl((long double)c[t]);
        }
      }
      norm[e] = acc;
      P.entry_zero[e] = nz ? 0 : 1;
    }
    long double rows = 0, cols = 0;
    bool rz = false, cz = false;
    for (int i = 0; i < s.n; ++i) {
      long double sr = 0, sc = 0;
      for (int j = 0; j < s.n; ++j) {
        sr += norm[i * s.n + j] * norm[i * s.n + j];
        sc += norm[j * s.n + i] * norm[j * s.n + i];
      }
      if (sr == 0) rz = true; else rows += log2l(sr);
      if (sc == 0) cz = true; else cols += log2l(sc);
    }
    if (rz || cz) zero_bound = true;
    log2b = std::min(rows, cols);
  } else {
    // every |c| <= 2^coeff_bits: |a_ij|_1 <= T 2^cb, so B^2 <= (n T^2 4^cb)^n
    log2b = (long double)s.n * (log2l((long double)s.n) + 2 * log2l((long double)P.T) +
                                2.0L * s.coeff_bits);
  }
  log2b += 1e-6L * (fabsl(log2b) + 1) + 1.0L;  // safety margin (may add one prime)
  P.log2_bound_sq = (double)log2b;

  const auto& table = prime_table();
  const int force_pn = (int)((flags >> 8) & 0xFFF);
  P.prime_off = (int)((flags >> 20) & 0x3FF);
  // least pn with sum log2 p_i > 1 + log2(B^2) / 2, i.e. M^2 > 4 B^2
  int need = 1;
  if (!zero_bound) {
    long double acc = 0;
    const long double target = 1.0L + log2b / 2;
    need = 0;
    while (acc <= target) {
      if (P.prime_off + need >= (int)table.size()) {
        *unsupported = true;
        return "the coefficient bound needs more primes than the table holds";
      }
      acc += log2l((long double)table[P.prime_off + need]) - 1e-12L;
      ++need;
    }
    need = std::max(need, 1);
  }
  if (force_pn) {
    if (force_pn < need) return "forced prime count is below what the bound needs";
    need = force_pn;
  }
  if (need > kMaxPrimes) {
    *unsupported = true;
    return "more than " + std::to_string(kMaxPrimes) + " primes are not supported";
  }
  if (P.prime_off + need > (int)table.size()) {
    *unsupported = true;
    return "prime offset and count exceed the prime table";
  }
  P.pn = need;
  P.primes.assign(table.begin() + P.prime_off, table.begin() + P.prime_off + need);

  std::vector<uint32_t> Mb{1};
  for (uint32_t p : P.primes) big_mul_small(Mb, p);
  P.L = std::max(1, (big_bitlen(Mb) + 31) / 32);

  // Structural pivoting: eliminate the zero pattern symbolically (an entry of the trailing
  // block becomes nonzero when it was nonzero or both its row's and its column's entries in
  // the pivot column and row were) and take, whenever the pivot is structurally zero, the
  // first lower row that is not. The kernels then meet a zero pivot only by accident
  // (probability about 1/p per step) and their runtime exchanges stay idle.
  P.row_order.resize(s.n);
  for (int i = 0; i < s.n; ++i) P.row_order[i] = i;
  P.det_sign = 1;
  if (!P.entry_zero.empty()) {
    std::vector<uint8_t> S(P.nent);
    for (int64_t e = 0; e < P.nent; ++e) S[e] = P.entry_zero[e] ? 0 : 1;
    for (int k = 0; k + 1 < s.n; ++k) {
      if (!S[k * s.n + k]) {
        int r = -1;
        for (int i = k + 1; i < s.n; ++i) {
          if (S[i * s.n + k]) { r = i; break; }
        }
        if (r < 0) continue;  // structurally singular column: the kernels find det 0
        for (int j = 0; j < s.n; ++j) std::swap(S[k * s.n + j], S[r * s.n + j]);
        std::swap(P.row_order[k], P.row_order[r]);
        P.det_sign = -P.det_sign;
      }
      for (int i = k + 1; i < s.n; ++i) {
        if (!S[i * s.n + k]) continue;
        for (int j = k + 1; j < s.n; ++j) S[i * s.n + j] |= S[k * s.n + j];
      }
    }
    std::vector<uint8_t> z(P.nent);
    for (int i = 0; i < s.n; ++i) {
      for (int j = 0; j < s.n; ++j) z[i * s.n + j] = P.entry_zero[P.row_order[i] * s.n + j];
    }
    P.entry_zero.swap(z);
  }

  // Slots: the distinct nonzero entries when the coefficients are known (see plan.h); the
  // layout below falls back to every entry when the elimination cannot evaluate the first
  // variable itself (the unfused path reads the full evaluation tensor by entry).
  auto identity_slots = [&]() {
    P.nslot = P.nent;
    P.slot_src.resize(P.nent);
    P.entry_slot.resize(P.nent);
    for (int i = 0; i < s.n; ++i) {
      for (int j = 0; j < s.n; ++j) {
        P.slot_src[i * s.n + j] = P.row_order[i] * s.n + j;
        P.entry_slot[i * s.n + j] = i * s.n + j;
      }
    }
  };
  identity_slots();
  if (host_coeffs && s.k >= 1 && !(flags & 1u)) {
    std::vector<int32_t> src, slot(P.nent, -1);
    std::unordered_map<uint64_t, std::vector<int32_t>> by_hash;  // box hash -> slots
    for (int64_t e = 0; e < P.nent; ++e) {
      if (P.entry_zero[e]) continue;
      const int64_t in_e = (int64_t)P.row_order[e / s.n] * s.n + e % s.n;
      const int64_t* box = host_coeffs + in_e * P.T;
      uint64_t h = 1469598103934665603ull;  // FNV-1a over the box's bytes
      const unsigned char* bytes = (const unsigned char*)box;
      for (size_t b = 0; b < sizeof(int64_t) * (size_t)P.T; ++b) h = (h ^ bytes[b]) * 1099511628211ull;
      auto& bucket = by_hash[h];
      int found = -1;
      for (int32_t u : bucket) {
        if (std::memcmp(host_coeffs + (int64_t)src[u] * P.T, box, sizeof(int64_t) * P.T) == 0) {
          found = u;
          break;
        }
      }
      if (found < 0) {
        found = (int)src.size();
        src.push_back((int32_t)in_e);
        bucket.push_back(found);
      }
      slot[e] = found;
    }
    P.nslot = (int64_t)src.size();
    P.slot_src.swap(src);
    P.entry_slot.swap(slot);
  }

  P.pc.resize(P.pn);
  for (int i = 0; i < P.pn; ++i) {
    const uint32_t p = P.primes[i];
    uint32_t inv = p;  // Newton iteration for p^{-1} mod 2^32
    for (int it = 0; it < 5; ++it) inv *= 2u - p * inv;
    PrimeConst c{};
    c.p = p;
    c.pinv = 0u - inv;
    c.r1 = (uint32_t)((1ull << 32) % p);
    c.r2 = (uint32_t)mulmod64(c.r1, c.r1, p);
    c.r3 = (uint32_t)mulmod64(c.r2, c.r1, p);
    c.scale = powmod((uint32_t)(P.G % p), p - 2, p);  // 1/G, times the row-order sign
    if (P.det_sign < 0) c.scale = c.scale ? p - c.scale : 0u;
    P.pc[i] = c;
  }

  // the measured launch-mapping table, where it has an entry for this order and class
  const Tuning tune = get_tuning();
  const int tclass = tune_class(s.k, P.m[0]);
  P.det_lanes = default_det_lanes(P.n);
  if (tune.lanes[tclass][P.n] > 0) P.det_lanes = tune.lanes[tclass][P.n];
  const int dl = (int)((flags >> 4) & 0xF);
  if (dl) {
    const int want = 1 << (dl - 1);
    if (want > 16) return "elimination lanes must be 1..16";
    P.det_lanes = want;
  }

  // Workspace layout for pg primes at a time: every per-prime region holds pg primes, the
  // coefficient residues (S4's output, S5's input) all pn. pg < pn only when the caller caps
  // the workspace (max_ws): S1-S4 then run group by group.
  auto layout = [&](size_t pg, int slabs) -> size_t {
  P.slabs = slabs;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  P.off_res = take(pg * std::max<int64_t>(P.nslot, 1) * P.T * 4);
  // forward passes run over the last variable first, writing tmpA, tmpB, tmpA, ... in turn;
  // the output of the pass over variable v has shape [pn*nent][prod_{u<v} m_u][prod_{u>=v} N_u]
  size_t interAB[2] = {0, 0};
  for (int v = s.k - 1; v >= 1; --v) {  // the pass over variable 0 writes off_eval or is fused
    int64_t sz = 1;
    for (int u = 0; u < v; ++u) sz *= P.m[u];
    for (int u = v; u < s.k; ++u) sz *= P.N[u];
    if (v == 1) sz /= slabs;  // one slab of the pre-tensor at a time
    const int which = (s.k - 1 - v) % 2;
    interAB[which] = std::max(interAB[which], (size_t)sz);
  }
  P.off_tmpA = take(pg * P.nslot * interAB[0] * 4);
  P.off_tmpB = take(pg * P.nslot * interAB[1] * 4);
  // Fused evaluation of the first variable inside the elimination kernel: a block stages
  // Q points of every entry (m0 coefficients each) in LDS, at most kFuseLds bytes, and
  // handles S values of the first variable's grid index.
  P.fused = s.k >= 1 && !(flags & 1u);
  if (P.fused) {
    constexpr size_t kFuseLds = 64 * 1024;
    const int64_t R = P.G / P.N[0] / slabs;  // points of the pre-tensor (one slab)
    const int per_block = fused_slots(256, P.det_lanes, P.m[0]);
    const int NJ = fused_jrange(P.N[0], P.m[0]);
    int Q = tune.tile_points[tclass][P.n] > 0 ? tune.tile_points[tclass][P.n] : 16;
    while (Q > 1 && (Q > per_block || Q > R ||
                     fused_tile_words(P.n, P.det_lanes, P.m[0], Q) * 4 > kFuseLds)) Q >>= 1;
    if (fused_tile_words(P.n, P.det_lanes, P.m[0], Q) * 4 > kFuseLds) {
      P.fused = false;  // the tile does not fit: evaluate in full, then eliminate
      if (P.nslot != P.nent) {  // the full evaluation tensor is indexed by entry
        identity_slots();
        P.off_res = 0;
        off = 0;
        P.off_res = take(pg * P.nslot * P.T * 4);
        P.off_tmpA = take(pg * P.nslot * interAB[0] * 4);
        P.off_tmpB = take(pg * P.nslot * interAB[1] * 4);
      }
    } else {
      const int J = per_block / Q;
      const int64_t base_blocks = (int64_t)pg * ((R + Q - 1) / Q);
      // enough blocks to fill 256 CUs several times; each block reuses its tile S / J times
      int iters = (int)std::max<int64_t>(1, (int64_t)NJ * base_blocks / (2048LL * J));
      iters = std::min(iters, std::max(1, (NJ + J - 1) / J));
      P.fuse_Q = Q;
      P.fuse_S = J * iters;
    }
  }
  // Left-looking elimination (one lane per matrix, pivot rows only in registers) on request
  // (flag bit 2) up to kLLMaxN, or where the table chose it; the exchanging kernel alone by
  // default and with flag bit 3.
  const bool want_ll = (flags & 4u) || (!(flags & 8u) && tune.left_looking[tclass][P.n] == 1);
  P.det_ll = P.fused && want_ll && !(flags & 8u) && s.n <= kLLMaxN && slabs == 1;
  if (P.fused) {
    // the pre-tensor is the output of the evaluation pass over variable 1 (pass index
    // k - 2 counting from the last variable; passes alternate tmpA, tmpB), or the residues
    P.off_pre = s.k == 1 ? P.off_res : ((s.k - 2) % 2 == 0 ? P.off_tmpA : P.off_tmpB);
    P.off_eval = SIZE_MAX;
  } else {
    P.off_eval = s.k == 0 ? P.off_res : take(pg * P.nent * P.G * 4);
  }
  P.off_detv = take(pg * P.G * 4);
  P.off_den = take(pg * P.G * 4);
  // interpolation passes run over the first variable first, trimming N_v to D_v + 1
  size_t iinter = 0;
  for (int v = 0; v + 1 < s.k; ++v) {
    int64_t sz = 1;
    for (int u = 0; u <= v; ++u) sz *= P.D[u] + 1;
    for (int u = v + 1; u < s.k; ++u) sz *= P.N[u];
    iinter = std::max(iinter, (size_t)sz);
  }
  P.off_iA = take(pg * iinter * 4);
  P.off_iB = take(pg * iinter * 4);
  P.off_coef = take((size_t)P.pn * P.C * 4);
  return std::max<size_t>(off, 256);
  };
  P.prime_group = P.pn;
  P.ws_bytes = layout(P.pn, 1);
  if (max_ws > 0 && P.ws_bytes > max_ws) {
    // the largest group of primes whose solve fits (integer matrices are never split: their
    // one point per prime costs nothing)
    int g = s.k == 0 ? 0 : P.pn - 1;
    while (g >= 1 && layout(g, 1) > max_ws) --g;
    if (g >= 1) {
      P.prime_group = g;
      P.ws_bytes = layout(g, 1);
    } else {
      // one prime at a time does not fit either: cut its grid into slabs along variable 1
      // (fused plans with two or more variables; a slab holds at least one pair of values)
      int sl = 2;
      const bool can = P.fused && s.k >= 2 && P.N[1] >= 4;
      while (can && sl < P.N[1] / 2 && layout(1, sl) > max_ws) sl *= 2;
      if (!can || layout(1, sl) > max_ws || !P.fused) {
        *unsupported = true;
        return can ? "the workspace cap is below the footprint of a solve one prime at a time, "
                     "even with its grid in slabs"
                   : "the workspace cap is below the footprint of a solve one prime at a time";
      }
      P.prime_group = 1;
      P.ws_bytes = layout(1, sl);
    }
  }
  P.in_bytes = (size_t)P.nent * P.T * 8;
  P.out_bytes = (size_t)P.C * P.L * 4;
  P.predicted_ms = predict_ms(P, get_rates());
  *out = std::move(P);
  return "";
}

MatPlan prime_range_plan(const MatPlan& P, int b, int e) {
  MatPlan R = P;
  R.pn = e - b;
  R.d_pc = P.d_pc + b;
  for (int v = 0; v < P.k; ++v) {
    R.tw_off[v] = P.tw_off[v] + (int64_t)b * P.tw_stride;
  }
  // the per-prime regions hold the group's primes from slot 0; the coefficient region holds
  // all pn primes (for an integer matrix, C = 1: the determinant residue of each prime)
  R.off_coef = P.off_coef + (size_t)b * P.C * 4;
  return R;
}

void set_tuning(const Tuning& t) {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning = t;
}

Tuning get_tuning() {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  return g_tuning;
}

int upload_tables(Plan* plan) {
  // layout per matrix: pc | tw | itw | gw | gc | mlimbs | hlimbs | zero
  std::vector<size_t> offs;
  size_t total = 0;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  struct Sizes { size_t pc, tw, gw, gc, ml, zero, ss, es; };
  std::vector<Sizes> sz;
  for (auto& P : plan->mats) {
    int64_t stride = 0;
    for (int v = 0; v < P.k; ++v) {
      P.tw_off[v] = stride;
      stride += P.N[v];
    }
    P.tw_stride = std::max<int64_t>(stride, 1);
    Sizes z;
    z.pc = al(sizeof(PrimeConst) * P.pn);
    z.tw = al(4 * P.pn * P.tw_stride);
    z.gw = al(4 * P.pn * P.pn);
    z.gc = al(4 * P.pn);
    z.ml = al(4 * P.L);
    z.zero = P.entry_zero.empty() ? 0 : al(P.nent);
    z.ss = al(4 * std::max<int64_t>(P.nslot, 1));
    z.es = al(4 * P.nent);
    sz.push_back(z);
    offs.push_back(total);
    total += z.pc + 2 * z.tw + z.gw + z.gc + 2 * z.ml + z.zero + z.ss + z.es;
  }
  std::vector<uint8_t> host(std::max<size_t>(total, 256), 0);
  for (size_t idx = 0; idx < plan->mats.size(); ++idx) {
    MatPlan& P = plan->mats[idx];
    const Sizes& z = sz[idx];
    uint8_t* base = host.data() + offs[idx];
    std::memcpy(base, P.pc.data(), sizeof(PrimeConst) * P.pn);
    uint32_t* tw = (uint32_t*)(base + z.pc);
    uint32_t* itw = (uint32_t*)(base + z.pc + z.tw);
    for (int i = 0; i < P.pn; ++i) {
      const uint32_t p = P.primes[i];
      const uint32_t g = primitive_root(p);
      for (int v = 0; v < P.k; ++v) {
        const uint32_t w = powmod(g, (p - 1) / (uint32_t)P.N[v], p);
        const uint32_t wi = powmod(w, p - 2, p);
        uint64_t a = P.pc[i].r1, b = P.pc[i].r1;  // Montgomery representatives of w^t
        for (int t = 0; t < P.N[v]; ++t) {
          tw[i * P.tw_stride + P.tw_off[v] + t] = (uint32_t)a;
          itw[i * P.tw_stride + P.tw_off[v] + t] = (uint32_t)b;
          a = mulmod64(a, w, p);
          b = mulmod64(b, wi, p);
        }
      }
    }
    uint32_t* gw = (uint32_t*)(base + z.pc + 2 * z.tw);
    uint32_t* gc = (uint32_t*)(base + z.pc + 2 * z.tw + z.gw);
    for (int i = 0; i < P.pn; ++i) {
      const uint32_t pi = P.primes[i];
      uint64_t mj = 1;  // (p_0 .. p_{j-1}) mod p_i
      for (int j = 0; j < P.pn; ++j) {
        gw[i * P.pn + j] = j < i ? (uint32_t)mulmod64(mj, P.pc[i].r1, pi) : 0u;
        if (j < i) mj = mulmod64(mj, P.primes[j] % pi, pi);
      }
      // here mj = (p_0 .. p_{i-1}) mod p_i
      const uint32_t ci = i == 0 ? 1u : powmod((uint32_t)mj, pi - 2, pi);
      gc[i] = (uint32_t)mulmod64(ci, P.pc[i].r1, pi);
    }
    std::vector<uint32_t> Mb{1};
    for (uint32_t p : P.primes) big_mul_small(Mb, p);
    Mb.resize(P.L, 0);
    std::vector<uint32_t> Hb(P.L, 0);  // (M - 1) / 2 = M >> 1 since M is odd
    for (int l = 0; l < P.L; ++l) {
      Hb[l] = (Mb[l] >> 1) | (l + 1 < P.L ? (Mb[l + 1] << 31) : 0u);
    }
    uint32_t* ml = (uint32_t*)(base + z.pc + 2 * z.tw + z.gw + z.gc);
    uint32_t* hl = (uint32_t*)(base + z.pc + 2 * z.tw + z.gw + z.gc + z.ml);
    std::memcpy(ml, Mb.data(), 4 * P.L);
    std::memcpy(hl, Hb.data(), 4 * P.L);
    if (z.zero) {
      std::memcpy(base + z.pc + 2 * z.tw + z.gw + z.gc + 2 * z.ml, P.entry_zero.data(), P.nent);
    }
    uint8_t* ss = base + z.pc + 2 * z.tw + z.gw + z.gc + 2 * z.ml + z.zero;
    if (P.nslot) std::memcpy(ss, P.slot_src.data(), 4 * P.nslot);
    std::memcpy(ss + z.ss, P.entry_slot.data(), 4 * P.nent);
  }
  void* d = nullptr;
  hipError_t err = hipMalloc(&d, host.size());
  if (err != hipSuccess) return (int)err;
  err = hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return (int)err;
  }
  plan->d_tables = d;
  for (size_t idx = 0; idx < plan->mats.size(); ++idx) {
    MatPlan& P = plan->mats[idx];
    const Sizes& z = sz[idx];
    uint8_t* base = (uint8_t*)d + offs[idx];
    P.d_pc = (const PrimeConst*)base;
    P.d_tw = (const uint32_t*)(base + z.pc);
    P.d_itw = (const uint32_t*)(base + z.pc + z.tw);
    P.d_gw = (const uint32_t*)(base + z.pc + 2 * z.tw);
    P.d_gc = (const uint32_t*)(base + z.pc + 2 * z.tw + z.gw);
    P.d_mlimbs = (const uint32_t*)(base + z.pc + 2 * z.tw + z.gw + z.gc);
    P.d_hlimbs = (const uint32_t*)(base + z.pc + 2 * z.tw + z.gw + z.gc + z.ml);
    P.d_zero = z.zero ? (const uint8_t*)(base + z.pc + 2 * z.tw + z.gw + z.gc + 2 * z.ml) : nullptr;
    P.d_slot_src = (const int32_t*)(base + z.pc + 2 * z.tw + z.gw + z.gc + 2 * z.ml + z.zero);
    P.d_entry_slot = (const int32_t*)((const uint8_t*)P.d_slot_src + z.ss);
    // the evaluation passes skip zero slots only when slots are entries (no dedup)
    P.d_slot_zero = P.nslot == P.nent ? P.d_zero : nullptr;
  }
  return 0;
}

}  // namespace pd
