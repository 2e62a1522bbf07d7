// Exercises the library's host-only C++ (the lattice builder, the spline and
// setfl code, the PTA arithmetic) under AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  The device entry
// points that pta.cpp also calls are stubs here that report no device.
// Prints "ok" and returns 0 when every check passes.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "eam_table.h"
#include "lattice.h"
#include "ptamd.h"

namespace ptamd {
static std::string g_last;
void set_last_error(const std::string &msg) { g_last = msg; }
}  // namespace ptamd

extern "C" {
ptamd_status ptamd_apply_strain_increments(ptamd_system *, const double *) { return PTAMD_ENODEV; }
ptamd_status ptamd_get_info(const ptamd_system *, ptamd_info *) { return PTAMD_ENODEV; }
ptamd_status ptamd_get_strain(const ptamd_system *, double *) { return PTAMD_ENODEV; }
ptamd_status ptamd_run_until_converged(ptamd_system *, const ptamd_conv_params *, ptamd_averages *, int64_t *) {
  return PTAMD_ENODEV;
}
}

static int fail(int code, const char *what) {
  std::printf("failed: %s (%s)\n", what, ptamd::g_last.c_str());
  return code;
}

int main(int argc, char **argv) {
  // lattice and velocities
  ptamd::HostState s;
  ptamd::build_cube(5, 4.05, true, 300.0, 11, s);
  if ((int64_t)s.x.size() != ptamd::fcc_atoms(5) || s.vx.size() != s.x.size()) return fail(2, "lattice sizes");
  ptamd::maxwell_boltzmann(s, 500.0, 12);

  // splines and tables
  const int nr = 64, nrho = 48;
  const double dr = 0.15, drho = 0.5;
  std::vector<double> F(nrho), rho(nr), rphi(nr);
  for (int k = 0; k < nrho; ++k) F[k] = -std::sqrt(k * drho + 1.0);
  for (int k = 0; k < nr; ++k) {
    const double r = k * dr + 0.5;
    rho[k] = std::exp(-r);
    rphi[k] = r * std::exp(-2.0 * r);
  }
  std::vector<double> coef;
  ptamd::spline_coefficients(rho.data(), nr, dr, coef);
  double f = 0.0, df = 0.0;
  ptamd::spline_eval(coef.data(), nr, dr, 3.3, &f, &df);
  ptamd::spline_eval(coef.data(), nr, dr, nr * dr + 1.0, &f, &df);  // past the last knot
  ptamd_eam_table t{nrho, drho, nr, dr, 8.0, F.data(), rho.data(), rphi.data()};
  if (*ptamd::check_table(&t)) return fail(3, "check_table");
  std::vector<double> xs = {-1.0, 0.0, 0.3, 7.9, 30.0, 1e3}, fv(xs.size()), dv(xs.size());
  for (int which = 0; which < 3; ++which)
    if (ptamd_eam_table_eval(&t, which, (int64_t)xs.size(), xs.data(), fv.data(), dv.data()) != PTAMD_OK)
      return fail(4, "eam_table_eval");
  ptamd_eam_table bad = t;
  bad.nr = 2;
  if (ptamd_eam_table_eval(&bad, 1, 1, xs.data(), fv.data(), dv.data()) == PTAMD_OK) return fail(5, "bad table accepted");

  // a setfl file: written, sized, read; and a truncated one
  const std::string dir = argc > 1 ? argv[1] : ".";
  const std::string path = dir + "/table.setfl", cut = dir + "/cut.setfl";
  {
    FILE *fp = std::fopen(path.c_str(), "w");
    FILE *fc = std::fopen(cut.c_str(), "w");
    if (!fp || !fc) return fail(6, "cannot write the test files");
    for (FILE *o : {fp, fc}) {
      std::fprintf(o, "c1\nc2\nc3\n1 Al\n%d %.17g %d %.17g %.17g\n13 26.98 4.05 fcc\n", nrho, drho, nr, dr, 8.0);
    }
    for (int k = 0; k < nrho; ++k) std::fprintf(fp, "%.17g\n", F[k]);
    for (int k = 0; k < nr; ++k) std::fprintf(fp, "%.17g\n", rho[k]);
    for (int k = 0; k < nr; ++k) std::fprintf(fp, "%.17g\n", rphi[k]);
    for (int k = 0; k < nrho / 2; ++k) std::fprintf(fc, "%.17g\n", F[k]);
    std::fclose(fp);
    std::fclose(fc);
  }
  ptamd_eam_table rt{};
  double mass = 0.0;
  if (ptamd_read_setfl(path.c_str(), &rt, nullptr, nullptr, nullptr, &mass) != PTAMD_OK) return fail(7, "setfl size");
  std::vector<double> F2(rt.nrho), rho2(rt.nr), rphi2(rt.nr);
  if (ptamd_read_setfl(path.c_str(), &rt, F2.data(), rho2.data(), rphi2.data(), &mass) != PTAMD_OK)
    return fail(8, "setfl read");
  if (F2 != F || rho2 != rho || rphi2 != rphi) return fail(9, "setfl values");
  if (ptamd_read_setfl(cut.c_str(), &rt, F2.data(), rho2.data(), rphi2.data(), &mass) == PTAMD_OK)
    return fail(10, "truncated setfl accepted");
  if (ptamd_read_setfl((dir + "/missing").c_str(), &rt, nullptr, nullptr, nullptr, nullptr) == PTAMD_OK)
    return fail(11, "missing file accepted");

  // the PTA arithmetic over a few slow steps, with a jump in the middle
  ptamd_pta_params prm{};
  prm.d_eps_h = 1e-3;
  prm.delta_over_h = 0.2;
  for (int q = 0; q < 4; ++q) {
    prm.tol_v[q] = 0.01;
    prm.tol_j[q] = 0.05;
  }
  ptamd_pta_state st{};
  ptamd_pta_record rec{};
  for (int step = 0; step < 6; ++step) {
    double R[12];
    for (int k = 0; k < 3; ++k)
      for (int q = 0; q < 4; ++q) R[4 * k + q] = 1.0 + 0.01 * (step + 0.1 * k) + (step == 3 ? 0.5 : 0.0) + q;
    const double strains[3] = {1e-3 * step, 1e-3 * step + 1e-4, 1e-3 * step + 2e-4};
    const int64_t ns[3] = {100, 120, 0};
    if (ptamd_pta_update(&prm, &st, R, strains, ns, &rec) != PTAMD_OK) return fail(12, "pta_update");
  }
  if (ptamd_pta_start(nullptr, &prm, &st, &rec) == PTAMD_OK) return fail(13, "pta_start without a system");
  std::printf("ok %zu atoms\n", s.x.size());
  return 0;
}
