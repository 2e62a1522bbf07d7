// Host-side initial state construction (FCC cube + Maxwell-Boltzmann).
#pragma once
#include <stdint.h>

#include <vector>

namespace ptamd {

extern const double kBoltzmann;
extern const double kMassAl;
extern const double kMvv2e;
extern const double kEvA3toGPa;

struct HostState {
  std::vector<double> x, y, z, vx, vy, vz;
  std::vector<uint8_t> group;  // 0 mobile, 1 bottom region, 2 top region
  double volume0 = 0.0, area0 = 0.0;
};

int64_t fcc_atoms(int32_t nc);
void build_cube(int32_t nc, double a, bool fix_slabs, double T0, uint64_t seed, HostState &s);
void maxwell_boltzmann(HostState &s, double T0, uint64_t seed);

}  // namespace ptamd
