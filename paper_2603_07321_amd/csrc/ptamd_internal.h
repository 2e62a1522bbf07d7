// Internal declarations shared by the device kernels and the host runtime.
// POD structs only: they are passed by value to kernels or live in device
// memory with the same layout on both sides.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptamd {

constexpr int kBlock = 256;     // threads per block for every kernel
constexpr int kTile = 256;      // atoms per replica tile (replica ranges are padded to this)
constexpr int kSlots = 64;      // spread factor of the fixed-point reduction slots
constexpr int kNQ = 8;          // reduced quantities per slot
constexpr int kSeriesCols = 6;  // K, U, sigma_zz, T, lambda, T_z
constexpr int kSEBlocks = 20;   // blocks of the standard-error estimate
constexpr uint8_t kPad = 255;   // group tag of padding atoms
constexpr double kFix = 68719476736.0;  // 2^36: fixed-point scale of global sums

// quantities reduced into the slots
enum : int {
  Q_MV2 = 0,   // sum_mob m v^2 (eV), after the second half kick, before lambda
  Q_MVZ2 = 1,  // sum_mob m v_z^2 (eV)
  Q_EPAIR = 2, // 1/2 sum_i sum_j V_s(r_ij) (eV)
  Q_WZZ = 3,   // W_zz = -1/2 sum_i sum_j g_ij dz^2 / r (eV)
  Q_RZ = 4,    // -sum_{top} F^int_z (eV/A)
  Q_EMB = 5,   // sum_i B(rhobar_i) (eV)
  Q_SPARE = 7
};

// error bits of Control::err
enum : int {
  E_NONFINITE = 1,
  E_ESCAPE = 2,
  E_OVERFLOW = 4,  // Verlet list capacity exceeded
  E_DRIFT = 8,     // an atom drifted beyond the binning margin before a list build
  E_STATE = 16,    // thermostat: T <= 0 or lambda^2 < 0
  E_SKIN = 32,     // an atom moved more than half the skin since the list build (a trigger was missed)
  E_PRUNE = 128    // an atom moved faster than the pruned lists allow (Control::vb2)
};

// Device-resident control block (one per system).
struct Control {
  int64_t base;      // absolute step index of the first step in the current chunk
  int32_t rebuild;   // set by a kick-drift that finds the lists too old; cleared by the next density pass
  int32_t err;       // error bits
  int64_t n_steps;   // steps of the current burst
  int64_t se_block;  // samples per standard-error block (n_steps / 20; lag / 10 when testing convergence)
  int64_t ncells;    // cells of all replicas (binning grid of the last sort)
  // convergence test of the running averages (0: fixed-length burst)
  int64_t conv_lag;       // k: checks at samples 2k, 3k, ..., each against the average k samples earlier
  double conv_tol[4];     // tolerance per state function (K, U, sigma_zz, T_z); <= 0: not tested
  double conv_floor[4];   // lower bound of the error's denominator (0: the plain relative error)
  int64_t nbuild;         // list builds triggered on the device (running count)
  uint64_t kt_first, kt_last;  // earliest start and latest end stamp of the last timed force launch
  // pruned lists (Params::inner): a pruning density pass keeps the entries
  // within rin of the atom; every kick checks |v|^2 <= vb2, which keeps each
  // atom within (rin - rc)/2 of where it was at the last pruning pass
  double rin2;
  double vb2;
};

constexpr int kStat = 16;  // u64 entries per statistics row
constexpr int kStatMom = 9;  // first of the six position-moment columns (sum of q and of q^2 per axis, q = rint(4 x))

// Per-replica constants and grid (device memory, read by kernels).
struct RepInfo {
  int64_t abeg, aend;   // padded atom range in the sorted arrays
  int64_t nreal;        // real atoms
  int64_t nmob;         // mobile atoms
  double T0, dof;       // thermostat target (K), 3 N_mob - 3
  double volume0, area0, strain;
  double origin[3];     // binning grid origin
  double inv_h;         // 1 / bin edge
  int32_t dims[3];
  int32_t pad1;
  // sorted order of the bins: axis ax[2] slowest, then ax[1], ax[0] fastest
  // (stencil rows run along ax[0]); the axis of widest spread goes slowest,
  // so that a bin layer holds as few atoms as the sample's shape allows
  int32_t ax[3];
  int32_t pad2;
  int64_t cell_off;     // offset of this replica's cells in the global cell arrays
  int64_t ncells;       // dims product (+1 virtual cell for padding atoms)
  double center[3];     // nominal cube centre (escape test)
};

// Per-replica burst accumulators (device memory).
// The running sums are kept twice, by the parity of the last sample they
// hold: the kick-drift launch that records sample s reads sum[(s-1)&1] and
// writes sum[s&1], so every block of that launch can read the sums through
// s-1 while the replica's first block adds sample s.  The checkpoint sums of
// the convergence test alternate the same way.
struct RepAcc {
  double sum[2][kSeriesCols];  // K, U, sigma_zz, T, lambda, T_z
  double blk[kSEBlocks][3];    // batch sums of K, U, sigma_zz
  double csum[2][4];           // sums of K, U, sigma_zz, T_z at the last two checkpoints
  int64_t nsamp;
  int64_t se_bs;               // samples per batch (doubles when 20 batches are full, convergence mode)
  int64_t conv_step;           // N_s once the averages converged (0 while running)
  double lam_last;
  double out[12];  // ke, pe, szz, tz, ke_se, pe_se, szz_se, temp, strain, n, spare...
};

// Values uniform over the launch, passed by value.
struct Params {
  // potential (FP64 master copies)
  double eps, a, rc, rc2, c_eps;
  int32_t n, m;        // integer exponents of V and rho
  double Vc, dVc, rhoc, drhoc;  // effective shift constants (0 where the mode has none)
  // lists and binning
  double rlist2;       // (rc + skin)^2
  float rlist2_lo, rlist2_hi;  // FP32 pre-filter band around rlist2 (0.1%)
  double cull2;        // (rc + skin + margin)^2: cells farther than this hold no list candidate
  double bin_h;        // binning cell edge: (rlist + 2 margin) / 2, searched with a 5^3 stencil
  double half_skin2;   // (skin/2)^2: displacement beyond which the lists are invalid
  double trig_v;       // rebuild trigger: |x - x_build| + trig_v |v| > trig_lim at a rebuild point
  double trig_lim;
  double margin2;      // binning margin^2
  double esc2;         // squared escape radius around the replica centre
  // integrator
  double dt, hdt_m, tau;
  int32_t thermostat;
  int32_t n_rep;
  double mvv2e_m;      // m * mvv2e (eV per (A/fs)^2)
  double kb, gpa;
  int64_t ntot;        // padded atoms, all replicas
  int64_t nbr_stride;  // ntot * lanes_per_atom
  int32_t cap_slots;   // list slots per lane (a multiple of kGroup)
  int32_t lpa;
  int32_t ktime;       // nonzero: the force kernel stamps per-block start/end times into Buffers::ktime
  int32_t conv;        // nonzero: replicas whose averages converged are skipped (Control::conv_lag > 0)
  int32_t top_free;    // nonzero: atoms of the top region (group 2) move along z (thermal relaxation)
  int32_t msum;        // nonzero: per-atom position sums of the burst's samples (Buffers::msx..msz)
  // tabulated potential (setfl form; used when tab != 0 instead of the Sutton-Chen functions)
  int32_t tab;
  int32_t tab_kmax;    // last interval of the r tables (nr - 2)
  double tab_inv_dr;   // 1 / dr
  double tab_inv_drho; // 1 / drho
  int32_t tab_nrho;
  int32_t fold;        // nonzero (mixed form): the density pass does the step's kick-drift (Buffers::pnext)
  int32_t inner;       // nonzero: the pair passes read the pruned lists (nbri, ncounti), which the
                       // density pass of each pruning step writes from the full ones
};

// Device buffers (pointers), passed by value.
struct Buffers {
  double *x, *y, *z, *vx, *vy, *vz, *fx, *fy, *fz;
  void *pos4;          // float4 or double4: x, y, z, B'
  void *pnext;         // mixed form: float4 x + dt (lp v + dt F / 2m), the position after the next step (lp: the last lambda)
  uint8_t *group;
  int32_t *orig;       // original global index of each sorted atom
  int32_t *cell;       // linear cell index (within the replica grid) at the last sort
  float *xs, *ys, *zs; // positions at the last sort
  float *xr, *yr, *zr; // positions at the last list build
  int32_t *nbr;        // Verlet lists, [slot][atom*lpa + lane]: per atom 16-bit steps or 32-bit indices (nwide)
  int32_t *ncount;     // list length per atom
  int32_t *nbase;      // 16-bit form: the index the atom's first steps count from (its smallest listed neighbour)
  uint8_t *nwide;      // 0: the atom's lists are 16-bit steps; 1, 2: 32-bit indices (2: their span needs them)
  int32_t *nbri;       // pruned lists (the layout of nbr)
  int32_t *ncounti;    // pruned list length per atom
  int32_t *nbasei;     // the base and form of each atom's pruned list, as they were at its pruning pass
  uint8_t *nwidei;     // (a full-list build before the next pruning pass may change nbase and nwide)
  double *eshift;      // Sutton-Chen: the pair-energy shift -n_c Vc - dVc (sum r - n_c rc) over the atom's
                       // pairs within rc, from the density pass (which sums r and n_c for rho's shift)
  int32_t *cell_start; // global cell arrays: [cell_off + c]
  int32_t *cell_count;
  int32_t *blk_rep;    // replica of each tile
  RepInfo *rep;
  RepAcc *acc;
  unsigned long long *slots;  // [2][n_rep][kSlots][kNQ]
  unsigned long long *stat;   // [n_rep][kSlots][kStat]: drift^2, v^2, bbox min/max keys, list displacement^2
  double *series;      // [n_rep][series_cap][kSeriesCols]
  unsigned long long *ktime;  // [blocks][2]: device wall-clock at block start and end (timed launches)
  double *msx, *msy, *msz;    // per-atom position sums over the burst's samples (null unless enabled)
  void *tab_r;     // per r interval: spline coefficients (a, b, c, d) of rho, then of r*phi (R precision)
  double *tab_F;   // per rhobar interval: (a, b, c, d) of F (FP64)
  int64_t series_cap;
  Control *ctl;
};

// Verlet-list layout.  Entry e of atom i belongs to lane l = e % lpa at slot
// s = e / lpa; slots are grouped in fours so that one 16-byte load fetches
// four indices, and consecutive (atom, lane) pairs are adjacent, so the 64
// lanes of a wave read 1 KiB contiguously.  stride = ntot * lpa.
constexpr int kGroup = 4;
// The pair kernels take 2 groups (8 slots) per lane and pass; every atom's
// list is padded with the sentinel index ntot up to a whole number of
// passes of all its lanes (8 * lanes entries), so the loops need no tail.
constexpr int kPass = 2 * kGroup;
__host__ __device__ inline size_t nbr_index(int64_t i, int e, int lpa, int64_t stride) {
  const int l = e % lpa, s = e / lpa;
  return ((size_t)(s / kGroup) * (size_t)stride + (size_t)i * lpa + l) * kGroup + (s % kGroup);
}

// The 16-bit form of an atom's lists: lane l of atom i holds its entries
// e = l, l + lpa, ... in increasing index order, each as the unsigned step
// from the lane's previous entry (the first from nbase[i], the smallest index
// in the atom's list).  The build keeps this form for every atom whose listed
// indices span less than 65,535 (all but a few evaporated atoms of the
// largest cubes: sorted order keeps an atom's neighbours within three or
// four bin layers of it); then every step between two of them fits, as do
// those of a pruned list.  Eight entries to a group per lane, so one 16-byte
// load gives a lane a whole pass and the pair kernels read half the bytes of
// 32-bit indices.  kOffSentinel (after a lane's last entry) stands for the
// sentinel index ntot.  The other atoms (Buffers::nwide) hold 32-bit indices
// (nbr_index) in the same buffer: columns are per atom, and the buffer has
// room for every atom in that form.
constexpr int kGroup16 = 8;
constexpr int kOffSentinel = 0xffff;
__host__ __device__ inline size_t nbr16_index(int64_t i, int e, int lpa, int64_t stride) {
  const int l = e % lpa, s = e / lpa;
  return ((size_t)(s / kGroup16) * (size_t)stride + (size_t)i * lpa + l) * kGroup16 + (s % kGroup16);
}

// ---- launch wrappers (kernels.hip) ----
void launch_burst_begin(const Params &p, const Buffers &b, int n_rep, hipStream_t s);
void launch_hold_group(const Buffers &b, int64_t ntot, int g, hipStream_t s);
void launch_kick_drift(const Params &p, const Buffers &b, int precision, int32_t k, int32_t mode, hipStream_t s);
void launch_pos4(const Params &p, const Buffers &b, int precision, hipStream_t s);
void launch_build(const Params &p, const Buffers &b, int precision, int lpa, hipStream_t s, int32_t cond = 0);
void launch_density(const Params &p, const Buffers &b, int precision, int lpa, int32_t k, hipStream_t s,
                    bool prune = false);
void launch_force(const Params &p, const Buffers &b, int precision, int lpa, int32_t k, int32_t mode,
                  hipStream_t s);
void launch_set_base(const Buffers &b, int64_t base, hipStream_t s);
void launch_set_ncells(const Buffers &b, int64_t n, hipStream_t s);
void launch_set_prune(const Buffers &b, double rin2, double vb2, hipStream_t s);
void launch_chunk_stats(const Params &p, const Buffers &b, hipStream_t s, int64_t n_stamps = 0);
void launch_snapshot(const Buffers &b, double *snap, unsigned long long *snap_slots, double *snap_acc, int restore,
                     int64_t ntot, int64_t nslots, int64_t nacc, hipStream_t s);
void launch_copy_back(const Params &p, const Buffers &b, const Buffers &scratch, int precision, hipStream_t s);
void launch_assign_count(const Params &p, const Buffers &b, int32_t *key, hipStream_t s);
// tiles of the cell scan for a replica of ncells cells; tsum holds tmax
// (the largest tile count of any replica) entries per replica
int scan_tiles(int64_t ncells);
void launch_scan_cells(const Params &p, const Buffers &b, int32_t *cursor, int32_t *tsum, int32_t tmax,
                       hipStream_t s);
void launch_scatter(const Params &p, const Buffers &b, const int32_t *key, int32_t *cursor, int32_t *tmp,
                    hipStream_t s);
void launch_cell_sort(const Params &p, const Buffers &b, const int32_t *tmp, int32_t *perm, int64_t ncells_tot,
                      hipStream_t s);
void launch_permute(const Params &p, const Buffers &b, const Buffers &scratch, const int32_t *perm,
                    const int32_t *key, int precision, hipStream_t s);
void launch_strain(const Params &p, const Buffers &b, const double *factor, hipStream_t s);
void launch_fill_i64(unsigned long long *ptr, int64_t n, unsigned long long v, hipStream_t s);
void launch_count_pairs(const Params &p, const Buffers &b, int precision, hipStream_t s);
// device probes: a streaming copy of bytes; FMA chains (returns the flops of one launch; out holds
// blocks * kBlock elements of the chosen type)
void launch_probe_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);
double launch_probe_fma(void *out, int fp64, int32_t blocks, int32_t iters, hipStream_t s);

}  // namespace ptamd
