// Precision planner of the mixed-precision PS scheme, compiled for host
// (ps_plan) and device (the per-matrix planning kernel), so a plan made on the
// GPU inside a captured graph and one made on the host from the same norms
// agree bit for bit.
//
// Rule (Liu, arXiv 2312.17396):
//  * Theorem 2.1 / eq. (choose-ui) with nu = 1: Horner product i may use unit
//    roundoff u_i = u ||B_0|| / (||B_i|| ||Y||^i).  Algorithms 2 and 3 print a
//    recursive form that also carries the i-th power of ||Y||; that is taken
//    as a misprint of the closed form.
//  * The framework needs u_r >= ... >= u_nu (section 2); the denominator is
//    replaced by its running maximum over j >= i, which leaves the closed form
//    unchanged whenever the decay condition (Bi-Xs-bnd) holds.
//  * nu = min{ i : u_i >= delta u }, else r + 1 (Algorithms 2 and 3,
//    delta = 10 by default, section 3.2); steps below nu keep the working
//    precision.
//  * IEEE-tier rounding (section 4.1.1): tier(i) is the lowest-precision
//    allowed tier whose unit roundoff does not exceed u_i.
//  * A zero denominator means every later product is exactly zero: u_i = inf.
#pragma once

#include <math.h>

#ifndef PS_HD
#if defined(__HIPCC__)
#define PS_HD __host__ __device__
#else
#define PS_HD
#endif
#endif

namespace psk {

// unit roundoff of tier t: FP64, FP32, BF16, FP8 (E4M3), and tier 4 =
// double-double (working precision only, 2^-106)
constexpr int kTierDD = 4;
PS_HD inline double tier_unit_roundoff(int t) {
  return t == 0 ? 0x1p-53 : t == 1 ? 0x1p-24 : t == 2 ? 0x1p-8 : t == 3 ? 0x1p-4 : 0x1p-106;
}
// the tiers below working tier w, highest precision first: w+1..3 (all of 0..3 below double-double)
PS_HD inline int first_lower_tier(int w) { return w == kTierDD ? 0 : w + 1; }

// normB[0..r], normY -> tier[0..r], u[0..r], *nu.  working_tier is 0 (FP64),
// 1 (FP32) or kTierDD.  mask bit t allows tier t (the working tier always allowed).
PS_HD inline void plan_tiers(int r, const double* normB, double normY, int working_tier,
                             unsigned mask, double delta, int* tier, double* u, int* nu_out) {
  const double uw = tier_unit_roundoff(working_tier);
  u[0] = uw;
  tier[0] = working_tier;
  double running = 0.0;
  for (int i = r; i >= 1; --i) {
    double yp = 1.0;
    for (int j = 0; j < i; ++j) yp *= normY;
    double term = normB[i] * yp;
    if (term > running || term != term) running = term;
    u[i] = (running == 0.0) ? INFINITY : uw * normB[0] / running;
  }
  int nu = r + 1;
  for (int i = 1; i <= r; ++i) {
    if (u[i] >= delta * uw) { nu = i; break; }
  }
  for (int i = 1; i <= r; ++i) {
    int best = working_tier;
    if (i >= nu) {
      for (int t = first_lower_tier(working_tier); t <= 3; ++t) {
        if (((mask >> t) & 1u) && tier_unit_roundoff(t) <= u[i]) best = t;
      }
    } else {
      u[i] = uw;
    }
    tier[i] = best;
  }
  *nu_out = nu;
}

}  // namespace psk
