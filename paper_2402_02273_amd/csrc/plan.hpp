#pragma once

#include "expint.h"

namespace expint {

constexpr int kPlanMaxDegree = 60;

// (s, m) for nu = tau * ||A||_1 with m >= m_min; false if nu, the tolerances
// or m_min are invalid.
bool choose_plan(double nu, double tol, double theta_max, int* s, int* m, int m_min = 1);
void default_tolerances(expint_dtype dt, double* tol, double* theta_max);

}  // namespace expint
