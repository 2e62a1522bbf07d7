// Tabulated EAM potential: spline coefficients of the setfl tables, the setfl
// reader and host evaluation.  Host code only.
#include "eam_table.h"

#include <algorithm>
#include <cctype>
#include <cmath>
#include <fstream>
#include <sstream>
#include <string>

#pragma clang fp contract(off)

namespace ptamd {
void set_last_error(const std::string &msg);

void spline_coefficients(const double *y, int n, double h, std::vector<double> &out) {
  // Second derivatives M_k of the interpolant.  At interior knots
  //   M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1}) / h^2;
  // not-a-knot at knots 1 and n-2 on a uniform grid gives M_0 = 2 M_1 - M_2
  // and M_{n-1} = 2 M_{n-2} - M_{n-3}, which turns the equations of knots 1
  // and n-2 into 6 M_1 = d_1 and 6 M_{n-2} = d_{n-2}.  The knots between them
  // form a tridiagonal system (Thomas algorithm).
  std::vector<double> d(n, 0.0), M(n, 0.0);
  const double s = 6.0 / (h * h);
  for (int k = 1; k < n - 1; ++k) d[k] = s * (y[k - 1] - 2.0 * y[k] + y[k + 1]);
  M[1] = d[1] / 6.0;
  M[n - 2] = d[n - 2] / 6.0;
  const int lo = 2, hi = n - 3;  // unknowns M_lo..M_hi
  if (hi >= lo) {
    const int m = hi - lo + 1;
    std::vector<double> cp(m), dp(m);
    for (int q = 0; q < m; ++q) {
      const int k = lo + q;
      double rhs = d[k];
      if (k == lo) rhs -= M[1];
      if (k == hi) rhs -= M[n - 2];
      if (q == 0) {
        cp[q] = 1.0 / 4.0;
        dp[q] = rhs / 4.0;
      } else {
        const double den = 4.0 - cp[q - 1];
        cp[q] = 1.0 / den;
        dp[q] = (rhs - dp[q - 1]) / den;
      }
    }
    M[hi] = dp[m - 1];
    for (int q = m - 2; q >= 0; --q) M[lo + q] = dp[q] - cp[q] * M[lo + q + 1];
  }
  M[0] = 2.0 * M[1] - M[2];
  M[n - 1] = 2.0 * M[n - 2] - M[n - 3];
  out.assign((size_t)4 * (n - 1), 0.0);
  const double h2 = h * h;
  for (int k = 0; k < n - 1; ++k) {
    double *c = &out[(size_t)4 * k];
    c[0] = y[k];
    c[1] = (y[k + 1] - y[k]) - h2 * (2.0 * M[k] + M[k + 1]) / 6.0;
    c[2] = h2 * M[k] / 2.0;
    c[3] = h2 * (M[k + 1] - M[k]) / 6.0;
  }
}

void spline_eval(const double *coef, int n, double h, double x, double *f, double *df) {
  const double sx = x / h;
  const double fk = std::floor(sx);  // clamped before the conversion (NaN: below)
  int k = fk >= 0.0 ? (int)std::min(fk, (double)n) : -1;
  double t = sx - (double)k, over = 0.0;
  if (k < 0) {
    k = 0;
    t = sx;
  } else if (k > n - 2) {
    k = n - 2;
    t = 1.0;
    over = x - (double)(n - 1) * h;
  }
  const double *c = coef + (size_t)4 * k;
  *df = (c[1] + t * (2.0 * c[2] + 3.0 * t * c[3])) / h;
  *f = c[0] + t * (c[1] + t * (c[2] + t * c[3])) + over * *df;
}

const char *check_table(const ptamd_eam_table *t) {
  if (!t) return "table is NULL";
  if (t->nrho < 4 || t->nr < 4) return "need nrho >= 4 and nr >= 4";
  if (!(t->drho > 0.0) || !(t->dr > 0.0) || !std::isfinite(t->drho) || !std::isfinite(t->dr))
    return "need finite drho > 0 and dr > 0";
  if (!(t->rc > 0.0) || !(t->rc <= (t->nr - 1) * t->dr) || !(t->rc <= 12.0))
    return "need 0 < rc <= min((nr - 1) dr, 12 A)";
  if (!t->F || !t->rho || !t->rphi) return "table values are NULL";
  for (int k = 0; k < t->nrho; ++k)
    if (!std::isfinite(t->F[k])) return "non-finite F value";
  for (int k = 0; k < t->nr; ++k)
    if (!std::isfinite(t->rho[k]) || !std::isfinite(t->rphi[k])) return "non-finite rho or r*phi value";
  return "";
}

}  // namespace ptamd

using namespace ptamd;

namespace {

ptamd_status bad(ptamd_status st, const std::string &msg) {
  set_last_error(msg);
  return st;
}

// setfl files may write exponents with a Fortran 'D'
bool parse_double(std::string tok, double *v) {
  for (char &c : tok)
    if (c == 'D' || c == 'd') c = 'e';
  char *end = nullptr;
  *v = std::strtod(tok.c_str(), &end);
  return end && *end == '\0' && end != tok.c_str();
}

}  // namespace

extern "C" {

ptamd_status ptamd_read_setfl(const char *path, ptamd_eam_table *table, double *F, double *rho, double *rphi,
                              double *mass) {
  if (!path || !table) return bad(PTAMD_EINVAL, "path and table must not be NULL");
  std::ifstream in(path);
  if (!in) return bad(PTAMD_EINVAL, std::string("cannot open ") + path);
  std::string line;
  for (int k = 0; k < 3; ++k)
    if (!std::getline(in, line)) return bad(PTAMD_EINVAL, "setfl: missing comment lines");
  if (!std::getline(in, line)) return bad(PTAMD_EINVAL, "setfl: missing element line");
  {
    std::istringstream ss(line);
    int ne = 0;
    if (!(ss >> ne) || ne != 1) return bad(PTAMD_EINVAL, "setfl: only single-element files are read");
  }
  if (!std::getline(in, line)) return bad(PTAMD_EINVAL, "setfl: missing grid line");
  std::istringstream gs(line);
  std::string tok[5];
  for (auto &t : tok)
    if (!(gs >> t)) return bad(PTAMD_EINVAL, "setfl: grid line needs Nrho drho Nr dr cutoff");
  double v[5];
  for (int k = 0; k < 5; ++k)
    if (!parse_double(tok[k], &v[k])) return bad(PTAMD_EINVAL, "setfl: bad number on the grid line");
  if (!(v[0] >= 4 && v[2] >= 4 && v[0] < 1e8 && v[2] < 1e8)) return bad(PTAMD_EINVAL, "setfl: bad table sizes");
  table->nrho = (int32_t)v[0];
  table->drho = v[1];
  table->nr = (int32_t)v[2];
  table->dr = v[3];
  table->rc = v[4];
  if (!std::getline(in, line)) return bad(PTAMD_EINVAL, "setfl: missing element data line");
  {
    std::istringstream ss(line);
    std::string z, m;
    double mv = 0.0;
    if (!(ss >> z >> m) || !parse_double(m, &mv)) return bad(PTAMD_EINVAL, "setfl: bad element data line");
    if (mass) *mass = mv;
  }
  table->F = table->rho = table->rphi = nullptr;
  if (!F || !rho || !rphi) return PTAMD_OK;  // sizing call
  double *dst[3] = {F, rho, rphi};
  const int64_t cnt[3] = {table->nrho, table->nr, table->nr};
  std::string t;
  for (int a = 0; a < 3; ++a)
    for (int64_t k = 0; k < cnt[a]; ++k) {
      if (!(in >> t)) return bad(PTAMD_EINVAL, "setfl: file ends before all table values");
      if (!parse_double(t, &dst[a][k])) return bad(PTAMD_EINVAL, "setfl: bad table value '" + t + "'");
    }
  table->F = F;
  table->rho = rho;
  table->rphi = rphi;
  return PTAMD_OK;
}

ptamd_status ptamd_eam_table_eval(const ptamd_eam_table *table, int32_t which, int64_t n, const double *x,
                                  double *f, double *df) {
  const char *why = check_table(table);
  if (*why) return bad(PTAMD_EINVAL, why);
  if (which < 0 || which > 2 || n < 0 || (n > 0 && (!x || !f || !df))) return bad(PTAMD_EINVAL, "bad arguments");
  const double *y = which == 0 ? table->F : which == 1 ? table->rho : table->rphi;
  const int m = which == 0 ? table->nrho : table->nr;
  const double h = which == 0 ? table->drho : table->dr;
  std::vector<double> c;
  spline_coefficients(y, m, h, c);
  for (int64_t q = 0; q < n; ++q) spline_eval(c.data(), m, h, x[q], &f[q], &df[q]);
  return PTAMD_OK;
}

}  // extern "C"
