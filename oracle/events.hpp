// Event-level steps after the matrix element (test infrastructure only):
// event weights and the cross-section sums, hit-or-miss unweighting, and the
// event-by-event random choice of a helicity configuration and a leading
// colour flow.  The paper lists cross-section calculation and unweighting
// among the serial tasks of the event generator that could move to the GPU
// (section 2), and names the helicity and leading-colour choice as the last
// feature added to the GPU workflow (section 5, Outlook); it gives no
// formulas for any of them, so the definitions below are the textbook ones.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace oracle {

// (hbar c)^2 = 0.3893793721 GeV^2 mb (PDG), in GeV^2 pb.
constexpr double kGeV2pb = 0.3893793721e9;

// Cross-section weight of an event of massless colliding partons at fixed
// sqrt(s): w = wgt |M|^2 / (2 s) in pb, wgt the phase-space weight (with the
// (2 pi)^(4-3n) convention), 2 s the flux factor.  The constant factor is
// formed first, then applied to the product wgt |M|^2.
inline double weight_factor(double sqrt_s) { return kGeV2pb / (2.0 * sqrt_s * sqrt_s); }

inline void event_weights(int64_t n, const double* wgt, const double* me, double sqrt_s, double* w) {
  const double k = weight_factor(sqrt_s);
  for (int64_t e = 0; e < n; ++e) w[e] = (wgt[e] * me[e]) * k;
}

// sum w, sum w^2 and max w, in event order; the sums accumulate in long
// double, so their own rounding stays below n 2^-64 relative.
inline void weight_stats(int64_t n, const double* w, double out[3]) {
  long double s = 0, s2 = 0;
  double mx = 0;
  for (int64_t e = 0; e < n; ++e) {
    s += w[e];
    s2 += (long double)w[e] * w[e];
    if (w[e] > mx) mx = w[e];
  }
  out[0] = (double)s;
  out[1] = (double)s2;
  out[2] = mx;
}

// Hit-or-miss: event e survives when r_e w_ref < w_e (r uniform in (0,1),
// w_ref at least the largest weight); survivors in increasing event order.
inline int64_t unweight(int64_t n, const double* w, const double* r, double w_ref, int64_t* idx) {
  int64_t k = 0;
  for (int64_t e = 0; e < n; ++e)
    if (r[e] * w_ref < w[e]) idx[k++] = e;
  return k;
}

// Inverse-CDF choice among non-negative weights taken in order: the first
// entry whose running sum exceeds r times the total.  When none does (the
// total is zero, or r is so close to 1 that r*total rounds to the total),
// the last entry with a non-zero weight, else entry 0.  `margin` receives the
// smallest distance of r*total to a running sum, relative to the total (how
// far the choice is from changing under rounding).
inline int choose(const std::vector<double>& wts, double r, double* margin) {
  double total = 0;
  for (double x : wts) total += x;
  const double t = r * total;
  double run = 0, m = INFINITY;
  int pick = -1;
  for (size_t i = 0; i < wts.size(); ++i) {
    run += wts[i];
    if (total > 0) m = std::fmin(m, std::fabs(run - t) / total);
    if (pick < 0 && run > t) pick = (int)i;
  }
  if (pick < 0) {
    pick = 0;
    for (size_t i = 0; i < wts.size(); ++i)
      if (wts[i] != 0) pick = (int)i;
  }
  if (margin) *margin = m;
  return pick;
}

}  // namespace oracle
