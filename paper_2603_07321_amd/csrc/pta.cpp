// PTA slow-time driver (Sec. 2.2 Steps 1-4, loading sequence of Sec. 2.4.2)
// on top of the converged averaging bursts.  Host code: three converged runs
// per slow step through the library's own entry points, then a few FP64
// operations per state function.  Formulas and readings are stated in
// include/ptamd.h beside the entry points.
#include <cmath>
#include <string>
#include <vector>

#include "ptamd.h"

#pragma clang fp contract(off)

namespace ptamd {
void set_last_error(const std::string &msg);
}

namespace {

ptamd_status invalid(const char *msg) {
  ptamd::set_last_error(msg);
  return PTAMD_EINVAL;
}

ptamd_status check_params(const ptamd_pta_params *p) {
  if (!p) return invalid("pta params are NULL");
  if (!std::isfinite(p->d_eps_h) || !(std::fabs(p->d_eps_h) < 0.05)) return invalid("need |d_eps_h| < 0.05");
  if (!(p->delta_over_h > 0.0) || !(p->delta_over_h <= 1.0)) return invalid("need 0 < delta_over_h <= 1");
  for (int f = 0; f < 4; ++f)
    if (!std::isfinite(p->tol_v[f]) || !std::isfinite(p->tol_j[f])) return invalid("tolerances must be finite");
  return PTAMD_OK;
}

// Simpson's rule over [t-Delta, t] with the runs at t-Delta, t-Delta/2, t (Eq. (simp)).
double simpson(double a, double b, double c) { return (a + 4.0 * b + c) / 6.0; }

// Three converged runs per replica: strain += d_first, run; += d_half, run;
// += d_half, run.  Each run starts from the state the one before left.
ptamd_status three_runs(ptamd_system *sys, const ptamd_pta_params *p, int nrep, double d_first, double d_half,
                        std::vector<double> &strain, std::vector<double> &R, std::vector<int64_t> &ns) {
  std::vector<double> inc(nrep), eps(nrep);
  std::vector<ptamd_averages> out(nrep);
  std::vector<int64_t> nc(nrep);
  strain.assign((size_t)3 * nrep, 0.0);
  R.assign((size_t)12 * nrep, 0.0);
  ns.assign((size_t)3 * nrep, 0);
  for (int k = 0; k < 3; ++k) {
    const double d = (k == 0) ? d_first : d_half;
    ptamd_status st;
    if (d != 0.0) {
      for (int r = 0; r < nrep; ++r) inc[r] = d;
      if ((st = ptamd_apply_strain_increments(sys, inc.data())) != PTAMD_OK) return st;
    }
    if ((st = ptamd_run_until_converged(sys, &p->conv, out.data(), nc.data())) != PTAMD_OK) return st;
    if ((st = ptamd_get_strain(sys, eps.data())) != PTAMD_OK) return st;
    for (int r = 0; r < nrep; ++r) {
      strain[(size_t)3 * r + k] = eps[r];
      double *row = &R[(size_t)12 * r + 4 * k];
      row[0] = out[r].ke;
      row[1] = out[r].pe;
      row[2] = out[r].szz;
      row[3] = out[r].tz;
      ns[(size_t)3 * r + k] = nc[r];
    }
  }
  return PTAMD_OK;
}

ptamd_status replicas(ptamd_system *sys, int *nrep) {
  ptamd_info inf;
  const ptamd_status st = ptamd_get_info(sys, &inf);
  if (st == PTAMD_OK) *nrep = inf.n_replicas;
  return st;
}

}  // namespace

extern "C" {

ptamd_status ptamd_pta_update(const ptamd_pta_params *prm, ptamd_pta_state *s, const double *R, const double *strains,
                              const int64_t *n_steps, ptamd_pta_record *rec) {
  ptamd_status st = check_params(prm);
  if (st != PTAMD_OK) return st;
  if (!s || !R || !strains || !n_steps || !rec) return invalid("NULL argument");
  const double h = 1.0;                        // slow time in units of the jump
  const double delta = prm->delta_over_h * h;  // Delta
  const bool first = s->n_jumps == 0;          // no R(t-h) yet
  for (int k = 0; k < 3; ++k) {
    rec->strain[k] = strains[k];
    rec->n_steps[k] = n_steps[k];
    for (int f = 0; f < 4; ++f) rec->R[k][f] = R[4 * k + f];
  }
  double vnew[4];
  int32_t jump_now[4];
  for (int f = 0; f < 4; ++f) {
    const double ra = R[f], rb = R[4 + f], rc = R[8 + f];
    const double dvdt = (s->R_t[f] - s->R_tmd[f]) / delta;        // Step 1, Eq. (dvdt_algo)
    const double vp = s->v[f] + h * dvdt;                         // Step 2, Eq. (pta_pred)
    const double vd = simpson(ra, rb, rc);                        // Step 3, Eq. (simp)
    const double ev = std::fabs((vp - vd) / vd);                  //         Eq. (rel_err)
    const double e1 = std::fabs((rc - s->R_t[f]) / s->R_t[f]);    //         Eq. (jump_err)
    const double e2 = first ? NAN : std::fabs((s->R_t[f] - s->R_prev[f]) / s->R_prev[f]);
    const bool second_form = first || s->jump_at_t[f] != 0;
    const bool jump = second_form ? (e1 >= prm->tol_j[f]) : (std::fabs(e1 / e2 - 1.0) >= prm->tol_j[f]);
    const int32_t status = (ev < prm->tol_v[f]) ? 0 : (jump ? 1 : 2);
    rec->v_pred[f] = vp;
    rec->v_d[f] = vd;
    rec->e_v[f] = ev;
    rec->e1[f] = e1;
    rec->e2[f] = e2;
    rec->status[f] = status;
    vnew[f] = (status == 0) ? vp : vd;
    rec->v[f] = vnew[f];
    jump_now[f] = status == 1;
  }
  for (int f = 0; f < 4; ++f) {
    s->R_prev[f] = s->R_t[f];
    s->R_tmd[f] = R[f];
    s->R_tmh[f] = R[4 + f];
    s->R_t[f] = R[8 + f];
    s->v[f] = vnew[f];
    s->jump_at_t[f] = jump_now[f];
  }
  s->strain = strains[2];
  s->n_jumps += 1;
  return PTAMD_OK;
}

ptamd_status ptamd_pta_start(ptamd_system *sys, const ptamd_pta_params *prm, ptamd_pta_state *state,
                             ptamd_pta_record *rec) {
  ptamd_status st = check_params(prm);
  if (st != PTAMD_OK) return st;
  if (!sys || !state || !rec) return invalid("NULL argument");
  int nrep = 0;
  if ((st = replicas(sys, &nrep)) != PTAMD_OK) return st;
  const double d_delta = prm->d_eps_h * prm->delta_over_h;
  std::vector<double> strain, R;
  std::vector<int64_t> ns;
  if ((st = three_runs(sys, prm, nrep, 0.0, 0.5 * d_delta, strain, R, ns)) != PTAMD_OK) return st;
  for (int r = 0; r < nrep; ++r) {
    ptamd_pta_state &s = state[r];
    ptamd_pta_record &c = rec[r];
    const double *Rr = &R[(size_t)12 * r];
    for (int k = 0; k < 3; ++k) {
      c.strain[k] = strain[(size_t)3 * r + k];
      c.n_steps[k] = ns[(size_t)3 * r + k];
      for (int f = 0; f < 4; ++f) c.R[k][f] = Rr[4 * k + f];
    }
    for (int f = 0; f < 4; ++f) {
      const double v = simpson(Rr[f], Rr[4 + f], Rr[8 + f]);
      s.R_tmd[f] = Rr[f];
      s.R_tmh[f] = Rr[4 + f];
      s.R_t[f] = Rr[8 + f];
      s.R_prev[f] = NAN;
      s.v[f] = v;
      s.jump_at_t[f] = 0;
      c.v_pred[f] = NAN;
      c.v_d[f] = v;
      c.v[f] = v;
      c.e_v[f] = c.e1[f] = c.e2[f] = NAN;
      c.status[f] = -1;
    }
    s.strain = c.strain[2];
    s.n_jumps = 0;
  }
  return PTAMD_OK;
}

ptamd_status ptamd_pta_jump(ptamd_system *sys, const ptamd_pta_params *prm, ptamd_pta_state *state,
                            ptamd_pta_record *rec) {
  ptamd_status st = check_params(prm);
  if (st != PTAMD_OK) return st;
  if (!sys || !state || !rec) return invalid("NULL argument");
  int nrep = 0;
  if ((st = replicas(sys, &nrep)) != PTAMD_OK) return st;
  const double d_delta = prm->d_eps_h * prm->delta_over_h;
  std::vector<double> strain, R;
  std::vector<int64_t> ns;
  if ((st = three_runs(sys, prm, nrep, prm->d_eps_h - d_delta, 0.5 * d_delta, strain, R, ns)) != PTAMD_OK) return st;
  for (int r = 0; r < nrep; ++r)
    if ((st = ptamd_pta_update(prm, &state[r], &R[(size_t)12 * r], &strain[(size_t)3 * r], &ns[(size_t)3 * r],
                               &rec[r])) != PTAMD_OK)
      return st;
  return PTAMD_OK;
}

}  // extern "C"
