// Host side of the batched solve (batch.h): chunking of the matrices by workspace budget,
// per-chunk workspace layout, the list of launches and their descriptor tables.
#include "batch_plan.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "kernels.h"

namespace pd {

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Elimination classes whose matrices run one by one on the single-matrix kernel inside a
// batched solve. At order 24 with 4 lanes and two-term pairing the batched kernel keeps more
// values in scratch memory than the single-matrix one (both at three waves per SIMD), and on
// the MI355X the class took 537 ms per solve of the 4096-matrix batch against 496 ms one by one;
// every other class runs at the single-matrix rate or faster batched.
bool det_each_class(int n, int lanes, int ll, int pair) {
  return n == 24 && lanes == 4 && ll == 0 && pair == 2;
}

// Workspace regions of one matrix inside a chunk (relative to the chunk's base). The fused
// path needs the residues, the evaluation passes before the first variable, the
// determinants, the interpolation ping-pong and the coefficients.
struct Regions {
  size_t res, tmpA, tmpB, pre, detv, den, iA, iB, coef, bytes;
};

Regions regions_of(const MatPlan& P, size_t base) {
  Regions r{};
  size_t off = base;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = al256(off + bytes);
    return o;
  };
  const size_t pn = P.pn;
  r.res = take(pn * std::max<int64_t>(P.nslot, 1) * P.T * 4);
  size_t interAB[2] = {0, 0};  // passes over variables k-1 .. 1 write tmpA, tmpB, ... in turn
  for (int v = P.k - 1; v >= 1; --v) {
    int64_t sz = 1;
    for (int u = 0; u < v; ++u) sz *= P.m[u];
    for (int u = v; u < P.k; ++u) sz *= P.N[u];
    const int which = (P.k - 1 - v) % 2;
    interAB[which] = std::max(interAB[which], (size_t)sz);
  }
  r.tmpA = take(pn * P.nslot * interAB[0] * 4);
  r.tmpB = take(pn * P.nslot * interAB[1] * 4);
  r.pre = P.k == 1 ? r.res : ((P.k - 2) % 2 == 0 ? r.tmpA : r.tmpB);
  r.detv = take(pn * P.G * 4);
  r.den = take(pn * P.G * 4);
  size_t iinter = 0;
  for (int v = 0; v + 1 < P.k; ++v) {
    int64_t sz = 1;
    for (int u = 0; u <= v; ++u) sz *= P.D[u] + 1;
    for (int u = v + 1; u < P.k; ++u) sz *= P.N[u];
    iinter = std::max(iinter, (size_t)sz);
  }
  r.iA = take(pn * iinter * 4);
  r.iB = take(pn * iinter * 4);
  r.coef = take(pn * P.C * 4);
  r.bytes = off - base;
  return r;
}

}  // namespace

bool batchable(const MatPlan& P) {
  if (!P.fused || P.k < 1) return false;
  for (int v = 1; v < P.k; ++v) {
    if (P.m[v] > kBatchMaxM) return false;
  }
  return true;
}

size_t batch_footprint(const MatPlan& P) { return regions_of(P, 0).bytes; }

std::string build_batch(const std::vector<MatPlan>& mats, size_t budget, bool halves,
                        BatchPlan* out) {
  BatchPlan B;
  B.halves = halves;
  if (halves) budget /= 2;  // two chunks in the workspace at once
  // order: batchable matrices grouped by order n (fewer elimination launches per chunk),
  // largest grids first within an order; the rest are solved one by one
  std::vector<int> order;
  for (int i = 0; i < (int)mats.size(); ++i) {
    if (batchable(mats[i])) order.push_back(i); else B.singles.push_back(i);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (mats[a].n != mats[b].n) return mats[a].n > mats[b].n;
    return mats[a].G * mats[a].pn > mats[b].G * mats[b].pn;
  });
  // greedy chunks under the budget
  std::vector<std::vector<int>> chunks;
  size_t used = 0;
  for (int i : order) {
    const size_t f = al256(batch_footprint(mats[i]));
    if (chunks.empty() || used + f > budget) {
      chunks.emplace_back();
      used = 0;
    }
    chunks.back().push_back(i);
    used += f;
  }
  size_t ws_need = 0;
  for (int i : B.singles) ws_need = std::max(ws_need, mats[i].ws_bytes);

  std::vector<uint8_t> blob;
  auto push = [&](const void* p, size_t bytes) {
    const size_t off = al256(blob.size());
    blob.resize(off + bytes);
    std::memcpy(blob.data() + off, p, bytes);
    return off;
  };

  // with halves, chunk c lives in half c mod 2 of the workspace (each half as large as the
  // largest chunk), so that consecutive chunks can run side by side
  size_t half = 0;
  for (const auto& chunk : chunks) {
    size_t sz = 0;
    for (int i : chunk) sz = al256(sz + regions_of(mats[i], 0).bytes);
    half = std::max(half, sz);
  }
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const auto& chunk = chunks[ci];
    const size_t base0 = halves ? (ci % 2) * half : 0;
    const size_t nb = B.launches.size();
    // layout
    std::vector<Regions> reg;
    size_t base = base0;
    for (int i : chunk) {
      reg.push_back(regions_of(mats[i], base));
      base = al256(base + reg.back().bytes);
    }
    ws_need = std::max(ws_need, base);

    // S1 reduce: one launch
    {
      std::vector<BReduce> d;
      int64_t vb = 0;
      for (size_t c = 0; c < chunk.size(); ++c) {
        const MatPlan& P = mats[chunk[c]];
        BReduce r{};
        r.block0 = vb;
        r.count = P.nslot * P.T;
        r.T = P.T;
        r.res_off = (int64_t)reg[c].res;
        r.mat = chunk[c];
        r.pn = P.pn;
        r.pc = P.d_pc;
        r.slot_src = P.d_slot_src;
        d.push_back(r);
        vb += (r.count + 255) / 256;
      }
      BLaunch L{};
      L.kind = BLaunch::kReduce;
      L.desc_off = push(d.data(), d.size() * sizeof(BReduce));
      L.ndesc = (int)d.size();
      L.vblocks = vb;
      B.launches.push_back(L);
    }
    // S2 evaluation passes (last variable first), stopping before the first variable;
    // pass s covers the matrices with at least s + 2 variables
    int maxk = 0;
    for (int i : chunk) maxk = std::max(maxk, mats[i].k);
    for (int s = 0; s + 1 < maxk; ++s) {
      std::vector<BExpand> d;
      int64_t vb = 0;
      for (size_t c = 0; c < chunk.size(); ++c) {
        const MatPlan& P = mats[chunk[c]];
        const int v = P.k - 1 - s;
        if (v < 1) continue;
        int64_t outer = 1, inner = 1;
        for (int u = 0; u < v; ++u) outer *= P.m[u];
        for (int u = v + 1; u < P.k; ++u) inner *= P.N[u];
        const size_t in_off = s == 0 ? reg[c].res : (s % 2 == 1 ? reg[c].tmpA : reg[c].tmpB);
        const size_t out_off = s % 2 == 0 ? reg[c].tmpA : reg[c].tmpB;
        BExpand e{};
        e.block0 = vb;
        e.in_off = (int64_t)in_off;
        e.out_off = (int64_t)out_off;
        e.B = (int64_t)P.pn * P.nslot;
        e.outer = outer;
        e.inner = inner;
        e.nent = P.nslot;
        e.tw_stride = P.tw_stride;
        e.m = P.m[v];
        e.Nv = P.N[v];
        e.JC = expand_outputs_per_thread(P.N[v], inner, P.m[v]);
        e.tw = P.d_tw + P.tw_off[v];
        e.pc = P.d_pc;
        e.zero = P.d_slot_zero;
        d.push_back(e);
        vb += (e.B * outer * (expand_jrange(e.Nv, e.m) / e.JC) * inner + 255) / 256;
      }
      if (d.empty()) continue;
      BLaunch L{};
      L.kind = BLaunch::kExpand;
      L.desc_off = push(d.data(), d.size() * sizeof(BExpand));
      L.ndesc = (int)d.size();
      L.vblocks = vb;
      B.launches.push_back(L);
    }
    // S3 elimination with the first variable's evaluation: one launch per (order, lanes,
    // elimination form, terms per lane of the paired evaluation or 0)
    std::map<std::tuple<int, int, int, int>, std::vector<size_t>> classes;
    for (size_t c = 0; c < chunk.size(); ++c) {
      const MatPlan& P = mats[chunk[c]];
      classes[{-P.n, P.det_lanes, P.det_ll ? 1 : 0,
               fused_paired(P.m[0]) ? fused_pair_terms(P.m[0]) : 0}].push_back(c);
    }
    for (auto& kv : classes) {
      std::vector<BDet> d;
      int64_t vb = 0;
      size_t lds = 0;
      for (size_t c : kv.second) {
        const MatPlan& P = mats[chunk[c]];
        BDet e{};
        e.block0 = vb;
        e.pre_off = (int64_t)reg[c].pre;
        e.detv_off = (int64_t)reg[c].detv;
        e.den_off = (int64_t)reg[c].den;
        e.R = P.G / P.N[0];
        e.tw_stride = P.tw_stride;
        e.rtiles = (e.R + P.fuse_Q - 1) / P.fuse_Q;
        e.jtiles = (fused_jrange(P.N[0], P.m[0]) + P.fuse_S - 1) / P.fuse_S;
        e.N0 = P.N[0];
        e.m0 = P.m[0];
        e.Q = P.fuse_Q;
        e.S = P.fuse_S;
        e.tw0 = P.d_tw + P.tw_off[0];
        e.pc = P.d_pc;
        e.zero = P.d_zero;
        e.slot = P.d_entry_slot;
        e.nslot = P.nslot;
        d.push_back(e);
        vb += (int64_t)P.pn * e.rtiles * e.jtiles;
        lds = std::max(lds, fused_tile_words(P.n, P.det_lanes, P.m[0], P.fuse_Q) * 4);
      }
      BLaunch L{};
      L.kind = BLaunch::kDet;
      L.desc_off = push(d.data(), d.size() * sizeof(BDet));
      L.ndesc = (int)d.size();
      L.vblocks = vb;
      L.n = -std::get<0>(kv.first);
      L.lanes = std::get<1>(kv.first);
      L.pair = std::get<3>(kv.first);
      L.each = det_each_class(L.n, L.lanes, std::get<2>(kv.first), L.pair);
      L.lds = lds;
      if (std::get<2>(kv.first)) {
        L.ll = 1;  // left-looking pass, then the repair pass of the exchanging kernel
        B.launches.push_back(L);
        L.ll = 2;
      }
      B.launches.push_back(L);
    }
    // S4 interpolation passes: pass v covers the matrices with more than v variables. The
    // first pass also divides each point's numerator by its denominator as it loads (S3's
    // end; every batched matrix has a variable), with enough lines per tile that a thread
    // inverts kFuseBatch denominators with one exponentiation.
    for (int v = 0; v < maxk; ++v) {
      std::vector<BIntt> d;
      int64_t vb = 0;
      size_t lds = 0;
      for (size_t c = 0; c < chunk.size(); ++c) {
        const MatPlan& P = mats[chunk[c]];
        if (v >= P.k) continue;
        int64_t outer = 1, inner = 1;
        for (int u = 0; u < v; ++u) outer *= P.D[u] + 1;
        for (int u = v + 1; u < P.k; ++u) inner *= P.N[u];
        const size_t in_off = v == 0 ? reg[c].detv : (v % 2 == 1 ? reg[c].iA : reg[c].iB);
        const size_t out_off = v == P.k - 1 ? reg[c].coef : (v % 2 == 0 ? reg[c].iA : reg[c].iB);
        const int Nv = P.N[v];
        int logN = 0;
        while ((1 << logN) < Nv) ++logN;
        const int64_t lines = outer * inner;
        // the register form up to 128 points (256 would raise the registers of every pass of
        // the batched kernel, which holds all forms)
        const bool reg_form = Nv <= 128 && intt_register_pass(Nv, inner);
        int W = reg_form ? kInttRegLines : intt_lines_per_block(lines, Nv, P.pn);
        if (v == 0 && !reg_form)
          while (Nv * W < kFuseBatch * 256 && Nv * (2 * W) <= kTileElems) W <<= 1;
        BIntt e{};
        e.block0 = vb;
        e.in_off = (int64_t)in_off;
        e.out_off = (int64_t)out_off;
        e.outer = outer;
        e.inner = inner;
        e.tw_stride = P.tw_stride;
        e.tiles = (lines + W - 1) / W;
        e.den_off = v == 0 ? (int64_t)reg[c].den : -1;
        e.pn = P.pn;
        e.Nv = Nv;
        e.logN = logN;
        e.Dv1 = P.D[v] + 1;
        e.W = W;
        e.reg = reg_form ? Nv / 8 : 0;
        e.itw = P.d_itw + P.tw_off[v];
        e.pc = P.d_pc;
        d.push_back(e);
        vb += e.tiles * P.pn;
        // tile and twiddles, or the register form's exchange rows
        lds = std::max(lds, reg_form ? (size_t)Nv * kInttRegLines * 4 : (size_t)(Nv * W + Nv / 2) * 4);
      }
      if (d.empty()) continue;
      BLaunch L{};
      L.kind = BLaunch::kIntt;
      L.desc_off = push(d.data(), d.size() * sizeof(BIntt));
      L.ndesc = (int)d.size();
      L.vblocks = vb;
      L.lds = lds;
      B.launches.push_back(L);
    }
    // S5 reconstruction: one launch
    {
      std::vector<BGarner> d;
      int64_t vb = 0;
      int pnmax = 1;
      for (size_t c = 0; c < chunk.size(); ++c) {
        const MatPlan& P = mats[chunk[c]];
        BGarner g{};
        g.block0 = vb;
        g.coef_off = (int64_t)reg[c].coef;
        g.C = P.C;
        g.mat = chunk[c];
        g.pn = P.pn;
        g.L = P.L;
        g.pc = P.d_pc;
        g.gw = P.d_gw;
        g.gc = P.d_gc;
        g.ml = P.d_mlimbs;
        g.hl = P.d_hlimbs;
        d.push_back(g);
        vb += (P.C + 255) / 256;
        pnmax = std::max(pnmax, P.pn);
      }
      BLaunch L{};
      L.kind = BLaunch::kGarner;
      L.desc_off = push(d.data(), d.size() * sizeof(BGarner));
      L.ndesc = (int)d.size();
      L.vblocks = vb;
      L.pnmax = pnmax;
      B.launches.push_back(L);
    }
    for (size_t li = nb; li < B.launches.size(); ++li) B.launches[li].chunk = (int32_t)ci;
  }
  B.desc_blob = std::move(blob);
  B.chunks = (int)chunks.size();
  B.ws_bytes = std::max<size_t>(ws_need, 256);
  *out = std::move(B);
  return "";
}

}  // namespace pd
