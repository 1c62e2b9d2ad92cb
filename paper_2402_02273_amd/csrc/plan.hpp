#pragma once

#include "expint.h"

namespace expint {

constexpr int kPlanMaxDegree = 60;

// (s, m) for nu = tau * ||A||_1; false if nu or the tolerances are invalid.
bool choose_plan(double nu, double tol, double theta_max, int* s, int* m);
void default_tolerances(expint_dtype dt, double* tol, double* theta_max);

}  // namespace expint
