// Host-side construction of the initial state: FCC cube, fixed boundary
// regions and Maxwell-Boltzmann velocities (Sec. 2.4.1 "Problem Setup" and
// Sec. 2.4.2 "Boundary conditions" of the paper).
#include "lattice.h"

#include <cmath>

namespace ptamd {

// Physical constants (CODATA 2018 values; the elementary charge is exact).
const double kBoltzmann = 8.617333262e-5;                         // eV/K
const double kMassAl = 26.9815385;                               // amu
const double kMvv2e = 1.66053906660e-27 * 1.0e10 / 1.602176634e-19;  // eV per amu A^2 / fs^2
const double kEvA3toGPa = 1.602176634e-19 / 1.0e-30 / 1.0e9;     // GPa per eV/A^3

// SplitMix64 of Steele, Lea and Flood (2014): output k of the stream seeded
// with `seed` is the finaliser applied to seed + (k + 1) * golden-gamma.
static inline uint64_t mix64(uint64_t seed, uint64_t k) {
  uint64_t v = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
  v ^= v >> 30;
  v *= 0xBF58476D1CE4E5B9ull;
  v ^= v >> 27;
  v *= 0x94D049BB133111EBull;
  v ^= v >> 31;
  return v;
}

// Standard normal number k of the stream: Box-Muller on the pair of
// uniforms (2*floor(k/2), 2*floor(k/2)+1); even k takes the cosine branch.
static inline double normal_k(uint64_t seed, uint64_t k) {
  const uint64_t pair = k >> 1;
  const double scale = 1.0 / 9007199254740992.0;  // 2^-53
  const double u1 = (double)((mix64(seed, 2 * pair) >> 11) + 1u) * scale;  // (0, 1]
  const double u2 = (double)(mix64(seed, 2 * pair + 1) >> 11) * scale;     // [0, 1)
  const double rad = std::sqrt(-2.0 * std::log(u1));
  const double ang = 6.283185307179586 * u2;
  return (k & 1) ? rad * std::sin(ang) : rad * std::cos(ang);
}

int64_t fcc_atoms(int32_t nc) { return 4ll * nc * nc * nc; }

void build_cube(int32_t nc, double a, bool fix_slabs, double T0, uint64_t seed, HostState &s) {
  const int64_t n = fcc_atoms(nc);
  s.x.resize(n); s.y.resize(n); s.z.resize(n);
  s.vx.assign(n, 0.0); s.vy.assign(n, 0.0); s.vz.assign(n, 0.0);
  s.group.assign(n, 0);
  // conventional cell: corner + three face centres, in half-lattice units
  const int off[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
  const double half = 0.5 * a;
  int64_t i = 0;
  for (int32_t cz = 0; cz < nc; ++cz)
    for (int32_t cy = 0; cy < nc; ++cy)
      for (int32_t cx = 0; cx < nc; ++cx)
        for (int b = 0; b < 4; ++b, ++i) {
          const int px = 2 * cx + off[b][0], py = 2 * cy + off[b][1], pz = 2 * cz + off[b][2];
          s.x[i] = (double)px * half;
          s.y[i] = (double)py * half;
          s.z[i] = (double)pz * half;
          // boundary regions: the three outermost atomic planes at each z face
          if (fix_slabs) s.group[i] = (pz < 3) ? 1 : ((pz > 2 * nc - 4) ? 2 : 0);
        }
  s.volume0 = (double)nc * nc * nc * a * a * a;
  s.area0 = ((double)nc * a) * ((double)nc * a);
  maxwell_boltzmann(s, T0, seed);
}

void maxwell_boltzmann(HostState &s, double T0, uint64_t seed) {
  const int64_t n = (int64_t)s.x.size();
  const double sigma = std::sqrt(kBoltzmann * T0 / (kMassAl * kMvv2e));
  double mean[3] = {0.0, 0.0, 0.0};
  int64_t nm = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (s.group[i] != 0) {
      s.vx[i] = s.vy[i] = s.vz[i] = 0.0;
      continue;
    }
    s.vx[i] = sigma * normal_k(seed, 3 * (uint64_t)i);
    s.vy[i] = sigma * normal_k(seed, 3 * (uint64_t)i + 1);
    s.vz[i] = sigma * normal_k(seed, 3 * (uint64_t)i + 2);
    mean[0] += s.vx[i];
    mean[1] += s.vy[i];
    mean[2] += s.vz[i];
    ++nm;
  }
  if (nm < 2) return;
  for (double &m : mean) m /= (double)nm;
  double sum2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (s.group[i] != 0) continue;
    s.vx[i] -= mean[0];
    s.vy[i] -= mean[1];
    s.vz[i] -= mean[2];
    sum2 += s.vx[i] * s.vx[i] + s.vy[i] * s.vy[i] + s.vz[i] * s.vz[i];
  }
  // temperature with 3 N_mob - 3 degrees of freedom, rescaled onto T0
  const double T = kMassAl * sum2 * kMvv2e / ((3.0 * (double)nm - 3.0) * kBoltzmann);
  if (T0 > 0.0 && T > 0.0) {
    const double f = std::sqrt(T0 / T);
    for (int64_t i = 0; i < n; ++i) {
      if (s.group[i] != 0) continue;
      s.vx[i] *= f;
      s.vy[i] *= f;
      s.vz[i] *= f;
    }
  }
}

}  // namespace ptamd
