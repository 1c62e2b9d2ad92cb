// Choice of the scaling s and Taylor degree m for the scaled Taylor action
// exp(tau B) v = (T_m(tau B / s))^s v (section 2.2, where s and m are left to
// a "proper selection").
//
// Rule: with nu = tau * ||A||_1 choose integers s >= 1, 1 <= m <= 60 that
// minimise the cost s*m (ties to the smaller s) subject to
//   (i)  s * theta^(m+1) / (m+1)! <= tol      (theta = nu / s)
//   (ii) theta <= theta_max.
// A is symmetric negative semidefinite with spectral radius <= ||A||_1, so the
// Lagrange remainder of the degree-m Taylor polynomial of e^z on [-theta, 0]
// is at most theta^(m+1)/(m+1)! per factor; (ii) caps the growth of the
// partial sums (about e^theta) and with it the rounding error.
//
// m_min: a degree floor.  The augmented matrix that also carries phi2 (both
// columns of the omega block next to the nilpotent 2 x 2 block) reaches the
// phi2 vector only through (hB)^2 / 2, so schemes that need phi2 ask for m >= 2.

#include <cmath>

#include "plan.hpp"

namespace expint {

static double remainder_bound(int s, int m, double theta) {
  double t = static_cast<double>(s);
  for (int k = 1; k <= m + 1; ++k) t = t * (theta / static_cast<double>(k));
  return t;
}

bool choose_plan(double nu, double tol, double theta_max, int* s_out, int* m_out, int m_min) {
  if (!(nu >= 0.0) || std::isinf(nu) || !(tol > 0.0) || !(theta_max > 0.0)) return false;
  if (m_min < 1 || m_min > kPlanMaxDegree) return false;
  if (nu == 0.0) {
    *s_out = 1;
    *m_out = m_min;
    return true;
  }
  long s = static_cast<long>(std::ceil(nu / theta_max));
  if (s < 1) s = 1;
  while (nu / static_cast<double>(s) > theta_max) ++s;
  long best_cost = -1;
  int best_s = 0, best_m = 0;
  for (;; ++s) {
    if (s > 100000) return false;
    const double theta = nu / static_cast<double>(s);
    for (int m = m_min; m <= kPlanMaxDegree; ++m) {
      if (remainder_bound(static_cast<int>(s), m, theta) <= tol) {
        const long cost = s * m;
        if (best_cost < 0 || cost < best_cost) {
          best_cost = cost;
          best_s = static_cast<int>(s);
          best_m = m;
        }
        break;
      }
    }
    if (best_cost >= 0 && s >= best_cost) break;
  }
  *s_out = best_s;
  *m_out = best_m;
  return true;
}

void default_tolerances(expint_dtype dt, double* tol, double* theta_max) {
  if (dt == EXPINT_F64) {
    *tol = 1e-13;
    *theta_max = std::log(1024.0);
  } else {
    *tol = 1e-6;
    *theta_max = std::log(64.0);  // partial sums grow at most ~12.5x: ~1e-6 relative rounding
  }
}

}  // namespace expint
