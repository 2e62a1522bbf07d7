// Host helpers of the tabulated EAM potential (setfl form).
#pragma once
#include <cstdint>
#include <vector>

#include "ptamd.h"

namespace ptamd {

// Not-a-knot cubic spline through y[0..n-1] on knots k*h (n >= 4): per
// interval k the coefficients (a, b, c, d) of p(t) = a + t (b + t (c + t d)),
// t = x/h - k in [0, 1].  out gets 4 (n - 1) values.
void spline_coefficients(const double *y, int n, double h, std::vector<double> &out);

// Value and derivative of such a spline at x; past the last knot the end
// value continues with the end slope, before the first the first interval's
// cubic is used.
void spline_eval(const double *coef, int n, double h, double x, double *f, double *df);

// Checks a table; returns an empty string or what is wrong.
const char *check_table(const ptamd_eam_table *t);

}  // namespace ptamd
