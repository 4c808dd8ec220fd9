// Running-time prediction of a solve (polydet_plan_info.predicted_ms).
//
// The paper predicts the time of a solve from the matrix's attributes (Section 5, equation
// predictRunningTime): primes x entries x the mean time to transform one entry, scaled by the
// replication factor mu (distinct entries / entries), leaving out the DET, IFFT and CRT stages,
// which weighed little on its GPU. Here the transforms are pruned and partly fused into the
// elimination, which dominates instead, so every stage gets a term, each the stage's work
// divided by a rate measured on the GPU (the package's calibration installs them with
// polydet_set_rates), plus a fixed cost per kernel launch:
//   reduce        (8 nslot T + 4 pn nslot T) bytes / reduce_bytes_per_s
//   evaluate      sum over the evaluation passes of 4 pn nslot (input box + output box) bytes
//                 / eval_bytes_per_s  (nslot = mu n^2: the paper's replication factor)
//   determinants  pn G sum_{m<n} m^2 elimination updates / det_updates_per_s[class][n]
//   interpolate   sum over the passes of 4 pn (input + output [+ denominators]) bytes
//                 / intt_bytes_per_s
//   reconstruct   ncoeff (pn (pn + 1) / 2 + pn L) products / garner_ops_per_s
#include <algorithm>
#include <mutex>

#include "plan.h"

namespace pd {

namespace {

std::mutex g_rates_mu;
Rates g_rates;

}  // namespace

void set_rates(const Rates& r) {
  std::lock_guard<std::mutex> lk(g_rates_mu);
  g_rates = r;
}

Rates get_rates() {
  std::lock_guard<std::mutex> lk(g_rates_mu);
  return g_rates;
}

double predict_ms(const MatPlan& P, const Rates& r) {
  const Rates def;  // built-in values for the entries the table leaves at 0
  auto pick = [](double v, double d) { return v > 0 ? v : d; };
  const double launch_s = pick(r.launch_us, def.launch_us) * 1e-6;
  const double pn = P.pn;
  const int groups = (P.pn + std::max(1, P.prime_group) - 1) / std::max(1, P.prime_group);
  double launches = 0, t = 0;
  // S1 reduce
  t += (8.0 * P.nslot * P.T + 4.0 * pn * P.nslot * P.T) / pick(r.reduce_bytes_per_s, def.reduce_bytes_per_s);
  launches += 1;
  // S2 evaluation passes (the last variable first; the first variable inside the elimination
  // when fused)
  double box_in = (double)P.T;  // current box: m_0 .. m_{v} then N_{v+1} ..
  double eval_bytes = 0;
  for (int v = P.k - 1; v >= (P.fused ? 1 : 0); --v) {
    const double box_out = box_in / P.m[v] * P.N[v];
    eval_bytes += 4.0 * pn * P.nslot * (box_in + box_out);
    box_in = box_out;
    launches += 1;
  }
  t += eval_bytes / pick(r.eval_bytes_per_s, def.eval_bytes_per_s);
  // S3 elimination
  const int cls = tune_class(P.k, P.m[0]);
  const double upd = (double)(P.n - 1) * P.n * (2.0 * P.n - 1) / 6.0;
  t += pn * (double)P.G * upd / pick(r.det_updates_per_s[cls][P.n], def.det_updates_per_s[cls][P.n]);
  launches += P.det_ll ? 2 : 1;
  if (P.k == 0) launches += 1;  // finalize
  // S4 interpolation passes (the first variable first, trimming N_v to D_v + 1)
  double intt_bytes = 0;
  double in = (double)P.G;
  for (int v = 0; v < P.k; ++v) {
    const double out = in / P.N[v] * (P.D[v] + 1);
    intt_bytes += 4.0 * pn * (in + out + (v == 0 ? in : 0.0));
    in = out;
    launches += 1;
  }
  t += intt_bytes / pick(r.intt_bytes_per_s, def.intt_bytes_per_s);
  // S5 reconstruction
  t += (double)P.C * (pn * (pn + 1) / 2 + pn * P.L) / pick(r.garner_ops_per_s, def.garner_ops_per_s);
  launches += 1;
  t += launch_s * (launches * groups - (groups - 1));  // the reconstruction runs once
  return t * 1e3;
}

}  // namespace pd
