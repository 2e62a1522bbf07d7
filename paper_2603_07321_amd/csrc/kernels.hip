// gfx950 kernels of the EAM molecular-dynamics burst.
//
// One MD step is three launches, captured in a HIP graph per chunk of steps
// (a chunk may start with a Verlet-list build, scheduled by the host):
//   kick_drift : Berendsen lambda of the previous step from the fixed-point
//                slot sums, v <- lambda v + dt/(2m) F, x <- x + dt v
//                (Eqs. (vv_algo_pos_pred_half), (vv_algo_pos_pred)); records
//                the previous step's sample (Eq. (R_m_t)).
//   density    : the host density rhobar_i and B'(rhobar_i) of Eq. (pe).
//   force      : F^int of Eq. (f_int), pair energy, virial W_zz, reaction;
//                second half kick (Eq. (vv_algo_vel_pred)); fixed-point
//                block sums into the slots.
// Fixed boundary atoms (v = 0, F = 0) are never kicked nor moved.
//
// Every global sum is a 64-bit fixed-point integer sum (scale 2^36) of
// per-atom values rounded once, so results do not depend on the block
// decomposition or the order of atomics.
#include "ptamd_internal.h"

#include <math.h>

#include <algorithm>

namespace ptamd {

template <class R> struct V4T;
template <> struct V4T<float> { using T = float4; };
template <> struct V4T<double> { using T = double4; };

__device__ __forceinline__ long long to_fix(double v) {
  // |v| < 1e8 keeps v * 2^36 inside int64; larger values are clamped (and flagged by callers)
  double s = v * kFix;
  s = fmin(fmax(s, -9.0e18), 9.0e18);
  return (long long)rint(s);
}

__device__ __forceinline__ long long shfl_xor_ll(long long v, int m) {
  int lo = (int)(unsigned)(v & 0xffffffffll);
  int hi = (int)(unsigned)((unsigned long long)v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

__device__ __forceinline__ double dist2_plain(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  // ((dx*dx + dy*dy) + dz*dz), no fused multiply-add: the same rounding as a
  // plain C evaluation, so list membership is decided identically everywhere.
  return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ double sub_plain(double a, double b) {
#pragma clang fp contract(off)
  return a - b;
}

template <class R> __device__ __forceinline__ R ipow(R x, int e) {
  R r = (R)1;
  while (e) {
    if (e & 1) r *= x;
    x *= x;
    e >>= 1;
  }
  return r;
}

// (a/r)^n and (a/r)^m.  NM = 1 is the Sutton-Chen aluminium pair n = 7,
// m = 6: t^6 = (t^2)^3, t^7 = t^6 t; NM = 0 takes any integer exponents.
template <class R, int NM>
__device__ __forceinline__ void sc_powers(R t, int n, int m, R *tn, R *tm) {
  if (NM == 1) {
    const R t2 = t * t;
    const R t6 = t2 * t2 * t2;
    *tm = t6;
    *tn = t6 * t;
  } else {
    *tm = ipow<R>(t, m);
    *tn = ipow<R>(t, n);
  }
}

template <class R, int NM> __device__ __forceinline__ R rho_pow(R t, int m) {
  if (NM == 1) {
    const R t2 = t * t;
    return t2 * t2 * t2;
  }
  return ipow<R>(t, m);
}

__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return rsqrt(x); }

// Slots per lane of an atom with cnt list entries, padded to whole passes.
template <int LPA> __device__ __forceinline__ int pass_slots(int cnt) {
  return (cnt + kPass * LPA - 1) / (kPass * LPA) * kPass;
}

__device__ __forceinline__ void set_err(const Buffers &b, int bits) { atomicOr(&b.ctl->err, bits); }

// Gather of one position entry: a uniform base plus a 32-bit byte offset
// (the global-load form with a scalar base), one shift per gather instead of
// 64-bit address arithmetic.  Indices stay below 2^27 (checked at creation).
template <class V4> __device__ __forceinline__ V4 gather(const V4 *base, int j) {
  const unsigned off = (unsigned)j * (unsigned)sizeof(V4);
  return *reinterpret_cast<const V4 *>(reinterpret_cast<const char *>(base) + off);
}

// The same, coordinates only (w undefined): the density passes need no B',
// and a 12-byte FP32 gather returns a quarter fewer bytes through the vector
// memory data path, which the pair passes keep busy.
template <class V4> __device__ __forceinline__ V4 gather_xyz(const V4 *base, int j) { return gather<V4>(base, j); }
template <> __device__ __forceinline__ float4 gather_xyz<float4>(const float4 *base, int j) {
  const unsigned off = (unsigned)j * (unsigned)sizeof(float4);
  const float3 v = *reinterpret_cast<const float3 *>(reinterpret_cast<const char *>(base) + off);
  return make_float4(v.x, v.y, v.z, 0.f);
}

// Origin of the pair kernels' gather copies (pos4, pnext) of a replica's
// positions: the FP32 copies of the mixed form hold coordinates relative to
// the cube's centre, so that their rounding (half an ulp of the coordinate)
// is set by the cube's half-size, not by where the cube sits; the FP64
// copies are absolute.  Only differences of these coordinates are used.
template <class R> __device__ __forceinline__ double gorigin(const RepInfo &rp, int d) {
  return sizeof(R) == sizeof(float) ? rp.center[d] : 0.0;
}

// One lane's walk over its padded list: passes of eight entries (two int4
// groups, eight independent gathers in flight).  The list entries of the
// next pass are loaded right after the current pass's gathers: loads return
// in order, so the arithmetic's waits for this pass's gathers never wait for
// them, and their latency (the list streams from HBM or the Infinity Cache)
// hides behind this pass's arithmetic.  The scheduling barriers keep that
// issue order.  (Gathering the next pass's positions ahead as well, into a
// second buffer, measured slower on the 62,500-atom cube.)  body(pj, jv)
// evaluates eight gathered entries (XYZ: coordinates only); jv holds their
// indices (the pruning density pass writes them into the pruned list).  An
// atom's list is in one of two forms (Buffers::nwide): 16-bit (w32 false),
// one 16-byte group of eight entries per pass, each entry the step from the
// lane's previous index (from the atom's base for its first), kOffSentinel
// the sentinel (only ever after the last real entry of a lane, so the
// running index may run on past it); or 32-bit indices, two groups of four
// per pass.  The lane holds nreal real entries.  Decoding takes one of three wave-uniform paths: no atom of
// the wavefront has 32-bit lists and every lane's pass is all real entries
// (every pass but the last one or two: no sentinel test); no 32-bit lists;
// or both forms.
template <bool XYZ, class V4, class Body>
__device__ __forceinline__ void pair_passes(const V4 *p4, const int4 *nb4, int64_t stride, int npl, int nreal,
                                            int base, bool w32, int sent, Body &&body) {
  V4 pj[8];
  int jv[8];
  int jp = base;
  const bool any_w32 = __ballot(w32) != 0ull;
  int4 la = nb4[0], lb = la;
  if (any_w32 && w32) lb = nb4[stride];
  for (int s = 0; s < npl; s += kPass) {
    const unsigned w[4] = {(unsigned)la.x, (unsigned)la.y, (unsigned)la.z, (unsigned)la.w};
    if (!any_w32 && __ballot(s + kPass > nreal) == 0ull) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        jp += (int)(w[u] & 0xffffu);
        jv[2 * u] = jp;
        jp += (int)(w[u] >> 16);
        jv[2 * u + 1] = jp;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned lo = w[u] & 0xffffu, hi = w[u] >> 16;
        jp += (int)lo;
        jv[2 * u] = lo == (unsigned)kOffSentinel ? sent : jp;
        jp += (int)hi;
        jv[2 * u + 1] = hi == (unsigned)kOffSentinel ? sent : jp;
      }
      if (any_w32 && w32) {
        jv[0] = la.x; jv[1] = la.y; jv[2] = la.z; jv[3] = la.w;
        jv[4] = lb.x; jv[5] = lb.y; jv[6] = lb.z; jv[7] = lb.w;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) pj[u] = XYZ ? gather_xyz<V4>(p4, jv[u]) : gather<V4>(p4, jv[u]);
    __builtin_amdgcn_sched_barrier(0);
    if (s + kPass < npl) {
      const size_t row = (size_t)((s + kPass) / kPass);  // the next pass
      if (any_w32 && w32) {
        la = nb4[(2 * row) * stride];
        lb = nb4[(2 * row + 1) * stride];
      } else {
        la = nb4[row * stride];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    body(pj, jv);
  }
}

// Real entries of lane `lane` of an atom with cnt list entries (entry e is
// at lane e % LPA).
template <int LPA> __device__ __forceinline__ int lane_entries(int cnt, int lane) {
  return cnt > lane ? (cnt - lane + LPA - 1) / LPA : 0;
}

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b % 8), and
// each XCD has an L2 of its own.  The pair kernels take their atoms by this
// remapped index, so that each XCD works through one contiguous eighth of
// the sorted atoms, whose neighbours' positions then stay in its L2, instead
// of every eighth block across the whole system.  A bijection on
// [0, gridDim.x) for any grid size.
constexpr unsigned kXcd = 8;
__device__ __forceinline__ int64_t xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned x = b % kXcd, q = nb / kXcd, r = nb % kXcd;
  return (int64_t)(x * q + min(x, r) + b / kXcd);
}

// Pruned lists.  The pruning density pass keeps, of every pass of the full
// list, the entries within rin of the atom, in the order they were met
// (pass, then slot, then lane), and deals them round-robin over the atom's
// lanes: kept entry e goes to lane e % LPA, slot e / LPA, so the lanes of an
// atom hold equal shares and the pruned list has the full list's layout.
// The kept indices of each pass go to a ring in LDS (16 LPA words per atom:
// what is not yet written out is less than two passes' worth); once a whole
// pass of the pruned list (8 LPA entries) is there, each lane reads its 8
// (stride LPA), forms its entries (16-bit form: steps from its previous
// index, the atom's base before the first; they fit, as every step between
// two indices of a 16-bit full list does) and stores them as one or two
// whole 16-byte groups.  The pruned list takes the full list's form.
template <int LPA>
struct PruneWriter {
  static constexpr int kWin = kPass * LPA;  // entries of one pass of all the atom's lanes
  static constexpr int kRing = 2 * kWin;    // a power of two
  int *ring;  // this atom's kRing words of LDS
  int cnt;    // entries kept so far (equal in the atom's lanes)
  int done;   // entries written out (a multiple of kWin)
  int last;   // 16-bit form: this lane's last index written
  bool w32;   // the atom's lists are 32-bit indices

  __device__ __forceinline__ void init(int *lds, int base, bool wide) {
    ring = lds + (int)(threadIdx.x / LPA) * kRing;
    cnt = done = 0;
    last = base;
    w32 = wide;
  }

  // one pass of the full list: keep[u], jv[u] of this lane's slot u
  __device__ __forceinline__ void pass(const Params &p, const Buffers &b, int64_t i, int lane, const bool (&keep)[8],
                                       const int (&jv)[8]) {
    const int lb = (int)(threadIdx.x & 63) & ~(LPA - 1);
    const unsigned below = (1u << lane) - 1u;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const unsigned m = (unsigned)(__ballot(keep[u]) >> lb) & (unsigned)((1ull << LPA) - 1ull);
      if (keep[u]) ring[(cnt + __popc(m & below)) & (kRing - 1)] = jv[u];
      cnt += __popc(m);
    }
    // (a wavefront's LDS accesses take effect in program order: only the
    // compiler is held back)
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    if (cnt - done >= kWin) flush(p, b, i, lane);
  }

  // writes entries done .. done + kWin - 1 (sentinels from cnt on)
  __device__ __forceinline__ void flush(const Params &p, const Buffers &b, int64_t i, int lane) {
    const int row = done / kWin;  // pass of the pruned list
    int v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int e = done + s * LPA + lane;
      if (e < cnt) {
        const int j = ring[e & (kRing - 1)];
        v[s] = w32 ? j : j - last;
        last = j;
      } else {
        v[s] = w32 ? (int)p.ntot : kOffSentinel;
      }
    }
    int4 *out = reinterpret_cast<int4 *>(b.nbri);
    if (!w32) {
      out[(size_t)row * p.nbr_stride + (size_t)i * LPA + lane] =
          make_int4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
    } else {
      out[(size_t)(2 * row) * p.nbr_stride + (size_t)i * LPA + lane] = make_int4(v[0], v[1], v[2], v[3]);
      out[(size_t)(2 * row + 1) * p.nbr_stride + (size_t)i * LPA + lane] = make_int4(v[4], v[5], v[6], v[7]);
    }
    done += kWin;
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  }

  // the last, partial pass
  __device__ __forceinline__ void finish(const Params &p, const Buffers &b, int64_t i, int lane, int base) {
    if (cnt > done) flush(p, b, i, lane);
    if (lane == 0) {
      b.ncounti[i] = cnt;
      b.nbasei[i] = base;
      b.nwidei[i] = w32 ? 1 : 0;
    }
  }
};

// Tabulated potential (NM = 2): interval and offset of r in the r tables.
// Pairs have r < rc <= (nr - 1) dr; the clamp keeps rounding at the last
// knot inside the table.
template <class R> __device__ __forceinline__ int tab_interval(const Params &p, R r, R *t) {
  const R sx = r * (R)p.tab_inv_dr;
  // r = 0 (coincident atoms) gives NaN here: index 0, the NaN propagates
  const int k = sx > (R)0 ? min((int)sx, p.tab_kmax) : 0;
  *t = sx - (R)k;
  return k;
}

// F(rhobar) and F'(rhobar) of the tabulated embedding function (FP64); past
// the last knot F continues linearly with its end slope.
__device__ __forceinline__ void tab_embed(const Params &p, const double *cF, double rb, double *F, double *dF) {
  const double sx = rb * p.tab_inv_drho;
  // below the first knot (a table with negative rho) or NaN: the first
  // interval, extrapolated; far above: clamped before the conversion
  int k = sx > 0.0 ? (int)fmin(sx, (double)p.tab_nrho) : 0;
  double t = sx - (double)k, over = 0.0;
  if (k > p.tab_nrho - 2) {
    k = p.tab_nrho - 2;
    t = 1.0;
    over = (sx - (double)(p.tab_nrho - 1)) / p.tab_inv_drho;
  }
  const double *c = cF + 4 * (size_t)k;
  *dF = (c[1] + t * (2.0 * c[2] + 3.0 * t * c[3])) * p.tab_inv_drho;
  *F = c[0] + t * (c[1] + t * (c[2] + t * c[3])) + over * *dF;
}

// Sum NQ int64 values over the block and add the totals into one slot row.
template <int NQ>
__device__ __forceinline__ void block_slot_add(long long (&v)[NQ], unsigned long long *row) {
  __shared__ long long sh[kBlock / 64][NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += shfl_xor_ll(v[q], o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[wid][q] = v[q];
  __syncthreads();
  if (threadIdx.x < NQ) {
    long long t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
    if (t != 0) atomicAdd(row + threadIdx.x, (unsigned long long)t);
  }
}

// Block sum of per-atom fixed-point values when one lane per atom holds
// them (APB atoms per block): through LDS instead of wavefront shuffles.
// Every atom's owner lane must call with owner = true (zeros for padding),
// so that all APB rows are written.
template <int NQ, int APB>
__device__ __forceinline__ void block_atoms_add(const long long (&v)[NQ], bool owner, int atom, unsigned long long *row) {
  __shared__ long long sh[APB][NQ];
  __shared__ long long part[NQ][8];
  if (owner)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[atom][q] = v[q];
  __syncthreads();
  if (threadIdx.x < NQ * 8) {
    const int q = threadIdx.x >> 3, p8 = threadIdx.x & 7;
    long long t = 0;
    for (int a = p8; a < APB; a += 8) t += sh[a][q];
    part[q][p8] = t;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    long long t = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += part[threadIdx.x][k];
    if (t != 0) atomicAdd(row + threadIdx.x, (unsigned long long)t);
  }
}

__device__ __forceinline__ unsigned long long *slot_row(const Buffers &b, int n_rep, int par, int r, int slot) {
  return b.slots + (((size_t)par * n_rep + r) * kSlots + slot) * kNQ;
}


// Atoms the integrator moves: mobile atoms (group 0) along x, y, z; during
// thermal relaxation the top region (group 2) along z only.  Every other
// atom is held (v = 0, F = 0).
__device__ __forceinline__ bool moves_z(const Params &p, uint8_t g) { return g == 0 || (p.top_free && g == 2); }

// ---------------------------------------------------------------------------
// burst start: zero accumulators, slots and errors
// ---------------------------------------------------------------------------
__global__ void k_burst_begin(Buffers b, int n_rep, int64_t ntot) {
  const size_t nslot = (size_t)2 * n_rep * kSlots * kNQ;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t t = t0; t < nslot; t += (size_t)gridDim.x * blockDim.x) b.slots[t] = 0ull;
  if (b.msx)
    for (size_t t = t0; t < (size_t)ntot; t += (size_t)gridDim.x * blockDim.x) b.msx[t] = b.msy[t] = b.msz[t] = 0.0;
  // accumulators zero; the last lambda 1 (no thermostat step taken yet)
  constexpr size_t kAccWords = sizeof(RepAcc) / sizeof(double);
  constexpr size_t kLamWord = offsetof(RepAcc, lam_last) / sizeof(double);
  const size_t nacc = (size_t)n_rep * kAccWords;
  double *acc = reinterpret_cast<double *>(b.acc);
  for (size_t t = t0; t < nacc; t += (size_t)gridDim.x * blockDim.x) acc[t] = (t % kAccWords == kLamWord) ? 1.0 : 0.0;
  if (t0 == 0) b.ctl->err = 0;
}

__global__ void k_set_base(Control *ctl, int64_t base) { ctl->base = base; }
__global__ void k_set_ncells(Control *ctl, int64_t n) { ctl->ncells = n; }
__global__ void k_set_prune(Control *ctl, double rin2, double vb2) {
  ctl->rin2 = rin2;
  ctl->vb2 = vb2;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// ---------------------------------------------------------------------------
// sampling of one completed step (thread 0 of the first block of a replica)
// ---------------------------------------------------------------------------
// State functions of one sample (after the thermostat's rescaling by lambda):
// m[0] = K, m[1] = U, m[2] = sigma_zz, m[3] = T_z, m[4] = T.  Every block of
// a kick-drift launch evaluates them with this one function, so all blocks of
// a replica agree bit for bit on what the replica's first block records.
__device__ void sample_values(const Params &p, const RepInfo &rp, const double *q, double lam, double *m) {
  const double l2 = lam * lam;
  const double mv2 = q[Q_MV2], mvz2 = q[Q_MVZ2];
  const double V = rp.volume0 * (1.0 + rp.strain);
  m[0] = 0.5 * l2 * mv2;
  m[1] = q[Q_EPAIR] + q[Q_EMB];
  m[2] = -(l2 * mvz2 + q[Q_WZZ]) / V * p.gpa;
  m[3] = (rp.area0 > 0.0) ? q[Q_RZ] / rp.area0 * p.gpa : 0.0;
  m[4] = (rp.dof > 0.0) ? l2 * mv2 / (rp.dof * p.kb) : 0.0;
}

// Column of the running sums that holds state function c (K, U, sigma_zz, T_z).
__device__ __forceinline__ int sum_col(int c) { return c == 3 ? 5 : c; }

// Sample s (1-based) of replica r: running sums, batch sums, series row.
__device__ void record_sample(const Params &p, const Buffers &b, const Control &c, const RepInfo &rp, RepAcc &A,
                              int r, int64_t s, const double *q, double lam) {
  double m[5];
  sample_values(p, rp, q, lam, m);
  const double *S0 = A.sum[(s - 1) & 1];
  double *S1 = A.sum[s & 1];
  S1[0] = S0[0] + m[0];
  S1[1] = S0[1] + m[1];
  S1[2] = S0[2] + m[2];
  S1[3] = S0[3] + m[4];
  S1[4] = S0[4] + lam;
  S1[5] = S0[5] + m[3];
  const int64_t bs0 = c.se_block;
  if (bs0 > 0) {
    int64_t bs = A.se_bs > 0 ? A.se_bs : bs0;
    int64_t bi = A.nsamp / bs;
    if (c.conv_lag > 0 && bi >= kSEBlocks) {
      // open-ended run: merge neighbouring batches, doubling their length
      for (int j = 0; j < kSEBlocks / 2; ++j)
        for (int c = 0; c < 3; ++c) A.blk[j][c] = A.blk[2 * j][c] + A.blk[2 * j + 1][c];
      for (int j = kSEBlocks / 2; j < kSEBlocks; ++j)
        for (int c = 0; c < 3; ++c) A.blk[j][c] = 0.0;
      bs *= 2;
      bi = A.nsamp / bs;
    }
    A.se_bs = bs;
    if (bi < kSEBlocks) {
      A.blk[bi][0] += m[0];
      A.blk[bi][1] += m[1];
      A.blk[bi][2] += m[2];
    }
  }
  if (s - 1 < b.series_cap) {
    double *row = b.series + ((size_t)r * b.series_cap + (s - 1)) * kSeriesCols;
    row[0] = m[0]; row[1] = m[1]; row[2] = m[2]; row[3] = m[4]; row[4] = lam; row[5] = m[3];
  }
  A.nsamp += 1;
  A.lam_last = lam;
  if (!isfinite(m[0]) || !isfinite(m[1]) || !isfinite(m[2])) set_err(b, E_NONFINITE);
}

// Convergence of the running averages at checkpoint i (a multiple of the
// lag k, i >= 2k): for every tested state function, the relative change of
// the running average over the last k samples, |R(i) - R(i-k)| / |R(i)|, is
// below its tolerance (the denominator bounded below by the function's
// floor).  m holds sample i, not yet added to the sums.
__device__ bool averages_converged(const Buffers &b, int r, int64_t i, int64_t lag, const double *m) {
  const RepAcc &A = b.acc[r];
  const Control &c = *b.ctl;
  const double *S = A.sum[(i - 1) & 1];
  const double *C = A.csum[((i / lag) - 1) & 1];
  for (int f = 0; f < 4; ++f) {
    const double tol = c.conv_tol[f];
    if (!(tol > 0.0)) continue;
    const double ri = (S[sum_col(f)] + m[f]) / (double)i;
    const double rk = C[f] / (double)(i - lag);
    const double den = fmax(fabs(ri), c.conv_floor[f]);
    const double e = fabs(ri - rk) / den;
    if (!(e < tol)) return false;
  }
  return true;
}


// Averages over the samples so far; batch standard errors from the complete
// batches (20 of n / 20 for a fixed-length burst, 10 to 20 for an open-ended one).
__device__ void write_averages(const Control &c, const RepInfo &rp, RepAcc &A) {
  const double n = (double)A.nsamp;
  const double *S = A.sum[A.nsamp & 1];
  A.out[0] = S[0] / n;
  A.out[1] = S[1] / n;
  A.out[2] = S[2] / n;
  A.out[3] = S[5] / n;
  const int64_t bs = A.se_bs;
  int64_t nb = 0;
  if (bs > 0) nb = (c.conv_lag > 0) ? min((int64_t)kSEBlocks, A.nsamp / bs) : (int64_t)kSEBlocks;
  for (int q = 0; q < 3; ++q) {
    double se = NAN;
    if (nb >= 2) {
      // two passes over the batch sums (no array of means: this code shares
      // its kernels' register budget)
      double mu = 0.0;
      for (int k = 0; k < nb; ++k) mu += A.blk[k][q] / (double)bs;
      mu /= (double)nb;
      double v = 0.0;
      for (int k = 0; k < nb; ++k) {
        const double d = A.blk[k][q] / (double)bs - mu;
        v += d * d;
      }
      se = sqrt(v / (double)(nb * (nb - 1)));
    }
    A.out[4 + q] = se;
  }
  A.out[7] = S[3] / n;
  A.out[8] = rp.strain;
  A.out[9] = n;
}

// ---------------------------------------------------------------------------
// start of a step, replica-wide: lambda of the previous step, the sample it
// completes and the convergence decision (shared by the kick-drift and the
// density pass that takes the kick-drift over in the mixed form)
// ---------------------------------------------------------------------------
// Berendsen's lambda from the replica's kinetic sum (fixed point, summed
// over the 64 slots): lambda^2 = 1 + (dt/tau)(T0/T - 1).  False (and
// lambda 1) where that needs T > 0 or gives a negative square.  Every path
// that takes lambda calls this one function, so they agree bit for bit.
__device__ __forceinline__ bool thermostat_lambda(const Params &p, const RepInfo &rp, long long qmv2, double *lam) {
  const double T = ((double)qmv2 / kFix) / (rp.dof * p.kb);
  const double l2 = 1.0 + (p.dt / p.tau) * (rp.T0 / T - 1.0);
  const bool ok = T > 0.0 && l2 >= 0.0;
  *lam = ok ? sqrt(l2) : 1.0;
  return ok;
}

struct StepStart {
  double lam;          // thermostat factor of the previous step (1 at step 1)
  int stop;            // the replica's averages converged at this step's sample
  const RepInfo *rep;  // the replica's data, staged in LDS
};

// Needs all kBlock threads of the block (two barriers).  While the first
// wavefront reduces the slots, the second stages in LDS what thread 0 needs
// afterwards: the replica's data, the control block and, in the replica's
// first block (which records the sample), the accumulators.  Thread 0 then
// works from LDS instead of a chain of dependent global loads; the
// accumulators go back at the end.  mode 1: finalize (the averages).
__device__ StepStart step_start(const Params &p, const Buffers &b, int r, int64_t step, bool first, int32_t mode) {
  __shared__ double s_lam;
  __shared__ int s_stop;
  __shared__ RepAcc s_acc;
  __shared__ RepInfo s_rep;
  __shared__ Control s_ctl;
  constexpr int kAccWords = (int)(sizeof(RepAcc) / sizeof(double));
  constexpr int kRepWords = (int)(sizeof(RepInfo) / sizeof(double));
  constexpr int kCtlWords = (int)(sizeof(Control) / sizeof(double));
  static_assert(sizeof(RepAcc) % 8 == 0 && sizeof(RepInfo) % 8 == 0 && sizeof(Control) % 8 == 0, "word copies");
  static_assert(kRepWords <= 64 && kCtlWords <= 64, "one word per lane of the staging wavefront");
  if (threadIdx.x >= 64 && threadIdx.x < 128) {
    const int t = (int)threadIdx.x - 64;
    if (t < kRepWords) reinterpret_cast<double *>(&s_rep)[t] = reinterpret_cast<const double *>(&b.rep[r])[t];
    if (t < kCtlWords) reinterpret_cast<double *>(&s_ctl)[t] = reinterpret_cast<const double *>(b.ctl)[t];
    if (first) {
      const double *src = reinterpret_cast<const double *>(&b.acc[r]);
      double *dst = reinterpret_cast<double *>(&s_acc);
      for (int u = t; u < kAccWords; u += 64) dst[u] = src[u];
    }
  }
  long long q[6];
  if (threadIdx.x < 64) {
    // lambda needs only the kinetic sum (Q_MV2, slot column 0); the sample's
    // other sums are reduced by the replica's first block, and by every
    // block at a convergence check (all of them take that decision)
    // Both parities' rows are loaded before the step index arrives.
    const unsigned long long *row0 = slot_row(b, p.n_rep, 0, r, threadIdx.x);
    const unsigned long long *row1 = slot_row(b, p.n_rep, 1, r, threadIdx.x);
    long long q0[6] = {0, 0, 0, 0, 0, 0}, q1[6] = {0, 0, 0, 0, 0, 0};
    q0[Q_MV2] = (long long)row0[Q_MV2];
    q1[Q_MV2] = (long long)row1[Q_MV2];
    if (first)
      for (int t = 1; t < 6; ++t) {
        q0[t] = (long long)row0[t];
        q1[t] = (long long)row1[t];
      }
    const bool odd = ((step - 1) & 1) != 0;
    const int64_t lag0 = p.conv ? b.ctl->conv_lag : 0;
    const bool check = lag0 > 0 && (step - 1) % lag0 == 0;
    if (check && !first)
      for (int t = 1; t < 6; ++t) {
        q0[t] = (long long)row0[t];
        q1[t] = (long long)row1[t];
      }
    const int nq = (first || check) ? 6 : 1;
#pragma unroll
    for (int t = 0; t < 6; ++t) q[t] = (step > 1) ? (odd ? q1[t] : q0[t]) : 0;
    if (step > 1)
      for (int t = 0; t < nq; ++t)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) q[t] += shfl_xor_ll(q[t], o);
  }
  __syncthreads();  // the staged copies are in LDS
  if (threadIdx.x == 0) {
    double lam = 1.0;
    int stop = 0;
    if (step > 1) {
      double qd[6];
      for (int t = 0; t < 6; ++t) qd[t] = (double)q[t] / kFix;
      const RepInfo &rp = s_rep;
      if (p.thermostat && !thermostat_lambda(p, rp, q[Q_MV2], &lam) && first) set_err(b, E_STATE);
      const int64_t smp = step - 1;  // the sample this launch completes
      const int64_t lag = p.conv ? s_ctl.conv_lag : 0;
      const bool check = lag > 0 && smp % lag == 0;
      if (check && smp >= 2 * lag) {
        // every block of the replica takes the same decision from the same data
        double m[5];
        sample_values(p, rp, qd, lam, m);
        stop = averages_converged(b, r, smp, lag, m) ? 1 : 0;
      }
      if (first) {
        RepAcc &A = s_acc;
        record_sample(p, b, s_ctl, rp, A, r, smp, qd, lam);
        if (check) {
          const double *S = A.sum[smp & 1];
          double *C = A.csum[(smp / lag) & 1];
          for (int f = 0; f < 4; ++f) C[f] = S[sum_col(f)];
        }
        if (stop) A.conv_step = smp;
        if (stop || mode == 1) write_averages(s_ctl, rp, A);
      }
    }
    s_lam = lam;
    s_stop = stop;
  }
  __syncthreads();
  if (first && step > 1 && threadIdx.x >= 64 && threadIdx.x < 128) {
    const double *src = reinterpret_cast<const double *>(&s_acc);
    double *dst = reinterpret_cast<double *>(&b.acc[r]);
    for (int t = (int)threadIdx.x - 64; t < kAccWords; t += 64) dst[t] = src[t];
  }
  return StepStart{s_lam, s_stop, &s_rep};
}

// A replica whose running averages converged in an earlier launch stays
// frozen (the whole block leaves together).  One that converges in this
// launch (at sample step - 1, written by its first block while others may
// still be starting) still takes this launch's lambda.
__device__ __forceinline__ bool frozen(const Params &p, const Buffers &b, int r, int64_t step) {
  if (!p.conv) return false;
  const int64_t cs = b.acc[r].conv_step;
  return cs != 0 && cs < step - 1;
}

// This lane's share of the replica's kinetic sum of the previous step (slot
// lane % 64 of its column), for start_lambda; loaded early by the caller.
__device__ __forceinline__ long long kinetic_slot(const Params &p, const Buffers &b, int r, int64_t step) {
  if (step <= 1 || !p.thermostat) return 0;
  return (long long)slot_row(b, p.n_rep, (int)((step - 1) & 1), r, (int)(threadIdx.x & 63))[Q_MV2];
}

// The start of a step for one block (uniform over it): the staged block
// path of step_start where the block records the sample (the replica's
// first block) or takes a convergence decision (every block at a
// checkpoint); elsewhere lambda only, summed by each wavefront from the
// slot values its lanes loaded (kinetic_slot), with neither barrier nor LDS.
__device__ __forceinline__ StepStart start_lambda(const Params &p, const Buffers &b, int r, int64_t step, bool first,
                                                  int32_t mode, long long qk) {
  const int64_t lag = p.conv ? b.ctl->conv_lag : 0;
  if (first || (lag > 0 && (step - 1) % lag == 0)) return step_start(p, b, r, step, first, mode);
  StepStart st{1.0, 0, &b.rep[r]};
  if (step > 1 && p.thermostat) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qk += shfl_xor_ll(qk, o);
    thermostat_lambda(p, *st.rep, qk, &st.lam);
  }
  return st;
}

// Per-atom state of the kick-drift (loaded early by the caller, so that the
// loads stay in flight while the slots are reduced).  Every array covers
// the padded range, so these loads need not wait for the group.
struct KickAtom {
  uint8_t grp;
  double x, y, z, vx, vy, vz, fx, fy, fz;
  float xr, yr, zr;
};

__device__ __forceinline__ KickAtom kick_load(const Buffers &b, int64_t i, bool full) {
  KickAtom a;
  a.grp = b.group[i];
  a.vx = b.vx[i];
  a.vy = b.vy[i];
  a.vz = b.vz[i];
  a.x = a.y = a.z = a.fx = a.fy = a.fz = 0.0;
  a.xr = a.yr = a.zr = 0.f;
  if (full) {
    a.fx = b.fx[i]; a.fy = b.fy[i]; a.fz = b.fz[i];
    a.x = b.x[i]; a.y = b.y[i]; a.z = b.z[i];
    a.xr = b.xr[i]; a.yr = b.yr[i]; a.zr = b.zr[i];
  }
  return a;
}

// v <- lambda v, then (step_on) v += dt/(2m) F and x += dt v for one atom;
// the escape and skin checks and the position sums.  point: a list rebuild
// point of the kick-drift graphs follows this step (the trigger test
// replaces the skin check).  store: this thread writes the atom back (the
// gather copy with w = 0 only when gather is set).  The updated state stays
// in a.
template <class R>
__device__ __forceinline__ void kick_atom(const Params &p, const Buffers &b, int64_t i, KickAtom &a, double lam,
                                          bool step_on, bool point, const RepInfo &rp, bool store, bool gather) {
  using V4 = typename V4T<R>::T;
  if (!moves_z(p, a.grp)) {  // fixed or padding atom: v = 0, never moves
    if (store && p.msum && step_on && a.grp != kPad) {
      b.msx[i] += a.x;
      b.msy[i] += a.y;
      b.msz[i] += a.z;
    }
    return;
  }
  a.vx *= lam;
  a.vy *= lam;
  a.vz *= lam;
  if (a.grp != 0) a.fx = a.fy = 0.0;  // a moving atom of the top region: along z only
  if (step_on) {
    a.vx += p.hdt_m * a.fx;
    a.vy += p.hdt_m * a.fy;
    a.vz += p.hdt_m * a.fz;
    a.x += p.dt * a.vx;
    a.y += p.dt * a.vy;
    a.z += p.dt * a.vz;
    if (store) {
      b.x[i] = a.x;
      b.y[i] = a.y;
      b.z[i] = a.z;
      if (gather) {
        // gather copy for the pair kernels; w (B') is rewritten by the density pass
        V4 v4;
        v4.x = (R)(a.x - gorigin<R>(rp, 0));
        v4.y = (R)(a.y - gorigin<R>(rp, 1));
        v4.z = (R)(a.z - gorigin<R>(rp, 2));
        v4.w = (R)0;
        reinterpret_cast<V4 *>(b.pos4)[i] = v4;
      }
      const double cx = a.x - rp.center[0], cy = a.y - rp.center[1], cz = a.z - rp.center[2];
      if (!(cx * cx + cy * cy + cz * cz <= p.esc2)) set_err(b, isfinite(a.x + a.y + a.z) ? E_ESCAPE : E_NONFINITE);
      const double ex = a.x - (double)a.xr, ey = a.y - (double)a.yr, ez = a.z - (double)a.zr;
      const double e2 = ex * ex + ey * ey + ez * ez;
      if (point) {
        // A rebuild point: the lists must last until the next one.  Rebuild
        // before this step's density pass if this atom's displacement since
        // the build, plus what its speed (with 50% headroom) adds over the
        // steps in between, reaches the limit (which also covers an atom
        // already past half the skin).
        if (sqrt(e2) + p.trig_v * sqrt(a.vx * a.vx + a.vy * a.vy + a.vz * a.vz) > p.trig_lim)
          atomicOr(&b.ctl->rebuild, 1);
      } else if (e2 > p.half_skin2) {
        set_err(b, E_SKIN);  // the lists this step will use are no longer valid
      }
      // pruned lists: no atom may outrun the speed they were pruned for
      if (p.inner && a.vx * a.vx + a.vy * a.vy + a.vz * a.vz > b.ctl->vb2) set_err(b, E_PRUNE);
      if (p.msum) {  // Eq. (mean_pos): this step's positions are sample s's
        b.msx[i] += a.x;
        b.msy[i] += a.y;
        b.msz[i] += a.z;
      }
    }
  }
  if (store) {
    b.vx[i] = a.vx;
    b.vy[i] = a.vy;
    b.vz[i] = a.vz;
  }
}

// Position of an atom after the next kick-drift, x + dt (lp v + dt/(2m) F),
// in the pair arithmetic's type, with lp a prediction of the next step's
// lambda: the last one taken (RepAcc::lam_last; 1 before the second step,
// where lambda is 1 exactly).  The mixed form's density pass forms its
// neighbours' positions from it.  The true step differs by (lambda - lp)
// dt v: lambda changes by (dt/tau) T0 dT / (2 T^2) per step, up to ~1e-4
// where a burst's start drains a tenth of the kinetic energy per 10 fs,
// ~1e-6 or less in equilibrium; times |v| dt ~ 0.015 A that is ~1e-6 A at
// most, below the FP32 resolution of the coordinates (7.6e-6 A at 100 A).
// (lp = 1 would be off by |lambda - 1| dt |v|, up to 1e-4 A early in a
// burst, where T is far from T0.)
template <class R>
__device__ __forceinline__ typename V4T<R>::T next_position(const Params &p, const RepInfo &rp, uint8_t g, double lp,
                                                            double x, double y, double z, double vx, double vy,
                                                            double vz, double fx, double fy, double fz) {
  typename V4T<R>::T n;
  if (moves_z(p, g)) {
    if (g != 0) fx = fy = 0.0;
    x += p.dt * (lp * vx + p.hdt_m * fx);
    y += p.dt * (lp * vy + p.hdt_m * fy);
    z += p.dt * (lp * vz + p.hdt_m * fz);
  }
  n.x = (R)(x - gorigin<R>(rp, 0));
  n.y = (R)(y - gorigin<R>(rp, 1));
  n.z = (R)(z - gorigin<R>(rp, 2));
  n.w = (R)0;
  return n;
}

// ---------------------------------------------------------------------------
// kick-drift (mode 0; mode 2: a list rebuild point follows) / finalize
// (mode 1).  The mixed form folds the kick-drift into the density pass and
// launches this kernel only to finalize.
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(kBlock) void k_kick_drift(Params p, Buffers b, int32_t k, int32_t mode) {
  const int64_t tile = blockIdx.x;
  const int r = (p.n_rep == 1) ? 0 : b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  KickAtom a = kick_load(b, i, mode != 1);
  const int64_t step = b.ctl->base + k;  // mode 0, 2: step being computed; mode 1: n_steps + 1
  if (frozen(p, b, r, step)) return;
  // (lambda per wavefront, as in the folded density pass, measured no
  // faster here: these blocks hold 256 atoms each, so there are few of them)
  const bool first = p.n_rep == 1 ? tile == 0 : (tile == 0 || b.blk_rep[tile - 1] != r);
  const StepStart st = step_start(p, b, r, step, first, mode);
  const bool step_on = mode != 1 && !st.stop;
  kick_atom<R>(p, b, i, a, st.lam, step_on, mode == 2, *st.rep, true, true);
}

// gather copy of positions (x, y, z, keep w) for the pair kernels, and in
// the mixed form the positions after the next drift (after a sort, a
// roll-back or new state: the state they derive from changed)
template <class R>
__global__ __launch_bounds__(kBlock) void k_pos4(Params p, Buffers b) {
  using V4 = typename V4T<R>::T;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint8_t g = b.group[i];
  if (g == kPad) return;
  V4 *p4 = reinterpret_cast<V4 *>(b.pos4);
  V4 v = p4[i];
  const double x = b.x[i], y = b.y[i], z = b.z[i];
  const int r = b.blk_rep[i / kTile];
  const RepInfo &rp = b.rep[r];
  v.x = (R)(x - gorigin<R>(rp, 0));
  v.y = (R)(y - gorigin<R>(rp, 1));
  v.z = (R)(z - gorigin<R>(rp, 2));
  p4[i] = v;
  if (p.fold) {
    // between the chunks of a burst: the same prediction the last force pass used
    reinterpret_cast<V4 *>(b.pnext)[i] = next_position<R>(p, rp, g, b.acc[r].lam_last, x, y, z, b.vx[i], b.vy[i],
                                                          b.vz[i], b.fx[i], b.fy[i], b.fz[i]);
  }
}

// ---------------------------------------------------------------------------
// density pass
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Verlet-list build
// ---------------------------------------------------------------------------
// Atom i's list holds every j != i within rlist.  Candidates come from the
// 5 x 5 x 5 bins around the bin i was sorted into: the bin edge is
// (rlist + 2 margin)/2, so the stencil reaches every atom within rlist while
// no atom has drifted more than the margin from its sorted position (checked
// here: E_DRIFT).  Bins of one stencil row (fixed y, z; consecutive x) are
// consecutive in the sorted order, so a row is one contiguous range of
// atoms.  Rows and bins whose box (open outward at the grid edge, where far
// atoms are clamped) lies farther than rlist + margin from atom i are
// skipped.  KB lanes share one atom; list positions come from a ballot
// prefix, so the order is fixed: rows in stencil order, atoms in sorted order.
constexpr int KB = 16;   // lanes per atom in the list build
constexpr int KCH = 4;   // candidates per lane per pass, loaded before use
constexpr int NRL = (25 + KB - 1) / KB;  // stencil rows per lane in phase 1

__device__ __forceinline__ double box_dist(double v, double o, double h, int n, int dim) {
  const double lo = (n == 0) ? -1e300 : o + n * h;
  const double hi = (n == dim - 1) ? 1e300 : o + (n + 1) * h;
  return fmax(fmax(lo - v, v - hi), 0.0);
}

template <class R> __device__ __forceinline__ float4 to_f4(typename V4T<R>::T v) {
  return make_float4((float)v.x, (float)v.y, (float)v.z, 0.f);
}

// Atom i's list in the 16-bit form (w32 false) or as 32-bit indices (w32).
// In the 16-bit form it returns false, having written nothing but list
// slots, if the listed indices span 65,535 or more (the caller then builds
// the 32-bit form): every step between two of them then fits 16 bits, and so
// do the steps of any subset, such as the pruned list.
// Phase 1 of a build: lane l of the atom's KB resolves stencil rows l,
// l + KB, ... into ranges of sorted atoms [rs, re), trimmed to the bins whose
// box lies within the culling radius of the atom (an empty range otherwise).
// Also checks the atom's drift since the sort against the margin.
template <class R>
__device__ __forceinline__ void stencil_rows(const Params &p, const Buffers &b, int64_t i, int lane,
                                             const RepInfo &rp, double xi, double yi, double zi, int (&rs)[NRL],
                                             int (&re)[NRL]) {
  if (lane == 0) {
    const double ex = xi - (double)b.xs[i], ey = yi - (double)b.ys[i], ez = zi - (double)b.zs[i];
    if (ex * ex + ey * ey + ez * ez > p.margin2) set_err(b, E_DRIFT);
  }
  // bins in sorted order: axis a2 slowest, a1, then a0 (the stencil rows)
  const int a0 = rp.ax[0], a1 = rp.ax[1], a2 = rp.ax[2];
  const int d0n = rp.dims[a0], d1n = rp.dims[a1], d2n = rp.dims[a2];
  const double pos[3] = {xi, yi, zi};
  const double p0 = pos[a0], p1 = pos[a1], p2 = pos[a2];
  const double o0 = rp.origin[a0], o1 = rp.origin[a1], o2 = rp.origin[a2];
  const double hb = p.bin_h;
  const int cl = b.cell[i];
  const int c0 = cl % d0n, c1 = (cl / d0n) % d1n, c2 = cl / (d0n * d1n);
#pragma unroll
  for (int h2 = 0; h2 < NRL; ++h2) {
    rs[h2] = re[h2] = 0;
    const int q = lane + h2 * KB;
    if (q >= 25) continue;
    const int n2 = c2 + q / 5 - 2, n1 = c1 + q % 5 - 2;
    if (n2 < 0 || n2 >= d2n || n1 < 0 || n1 >= d1n) continue;
    const double e2 = box_dist(p2, o2, hb, n2, d2n), e1 = box_dist(p1, o1, hb, n1, d1n);
    const double e12 = e1 * e1 + e2 * e2;
    if (e12 > p.cull2) continue;
    int lo = max(c0 - 2, 0), hi = min(c0 + 2, d0n - 1);
    while (lo <= hi) {
      const double d = box_dist(p0, o0, hb, lo, d0n);
      if (d * d + e12 <= p.cull2) break;
      ++lo;
    }
    while (hi >= lo) {
      const double d = box_dist(p0, o0, hb, hi, d0n);
      if (d * d + e12 <= p.cull2) break;
      --hi;
    }
    if (lo > hi) continue;
    const int64_t row = rp.cell_off + ((int64_t)n2 * d1n + n1) * d0n;
    rs[h2] = b.cell_start[row + lo];
    re[h2] = b.cell_start[row + hi] + b.cell_count[row + hi];
  }
}

// The rows' ranges of the q-th stencil row, from the lane that resolved it.
__device__ __forceinline__ void row_range(int q, int gbase, const int (&rs)[NRL], const int (&re)[NRL], int *s0,
                                          int *e0) {
  const int src = gbase + (q % KB);
  int rq = rs[0], eq = re[0];
#pragma unroll
  for (int h2 = 1; h2 < NRL; ++h2)
    if (q >= h2 * KB) {
      rq = rs[h2];
      eq = re[h2];
    }
  *s0 = __shfl(rq, src);
  *e0 = __shfl(eq, src);
}

template <class R, int LPA>
__device__ bool build_one(const Params &p, const Buffers &b, int64_t i, int lane, bool w32) {
  using V4 = typename V4T<R>::T;
  const int r = b.blk_rep[i / kTile];
  const V4 *p4 = reinterpret_cast<const V4 *>(b.pos4);
  const RepInfo &rp = b.rep[r];
  const double xi = b.x[i], yi = b.y[i], zi = b.z[i];
  // in the gather copies' coordinates (the FP32 prefilter)
  const float4 pi = make_float4((float)(R)(xi - gorigin<R>(rp, 0)), (float)(R)(yi - gorigin<R>(rp, 1)),
                                (float)(R)(zi - gorigin<R>(rp, 2)), 0.f);
  int rs[NRL], re[NRL];
  stencil_rows<R>(p, b, i, lane, rp, xi, yi, zi, rs, re);
  // phase 2: scan the rows in order, KB x KCH candidates per pass.  All
  // KCH positions are loaded before any is tested, and every lane tests its
  // candidates with the same FP32 arithmetic (no branch the compiler could
  // sink a load into: a load issued inside one would wait for all four);
  // only candidates in the band around rlist^2 take the FP64 decision.
  const int gbase = (threadIdx.x & 63) & ~(KB - 1);
  const unsigned long long gmask = (1ull << KB) - 1ull;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int cap = p.cap_slots * LPA;
  const int self = (int)i;
  // list slot of entry e (the layout of nbr_index, in unsigned arithmetic)
  const size_t slot_base = (size_t)self * (LPA * kGroup);
  const size_t group_stride = (size_t)p.nbr_stride * kGroup;
  int cnt = 0;
  int jmax = -1;  // this lane's last (largest) index kept
  // 16-bit form: each entry is the step from the entry LPA places before it
  // (the same lane's previous one), the first LPA from the atom's base, the
  // first index kept, which is the smallest (rows are met in increasing
  // sorted order, and each row's atoms in order).  ring (LDS, 64 words per
  // atom) holds the indices of the last kept entries by position: a ballot
  // keeps at most KB, and an entry looks back LPA <= KB places.
  int base = -1;
  __shared__ int ring[kBlock / KB][64];
  int *rg = ring[threadIdx.x / KB];
  for (int q = 0; q < 25; ++q) {
    int s0, e0;
    row_range(q, gbase, rs, re, &s0, &e0);
    for (int t = s0; t < e0; t += KB * KCH) {
      int jc[KCH];
      float4 qv[KCH];
#pragma unroll
      for (int u = 0; u < KCH; ++u) {
        jc[u] = t + u * KB + lane;
        qv[u] = to_f4<R>(p4[min(jc[u], e0 - 1)]);
      }
#pragma unroll
      for (int u = 0; u < KCH; ++u) {
        const int j = jc[u];
        const float dx = qv[u].x - pi.x, dy = qv[u].y - pi.y, dz = qv[u].z - pi.z;
        const float d2 = dx * dx + dy * dy + dz * dz;
        bool ok = (j < e0) & (j != self) & (d2 <= p.rlist2_hi);
        // near rlist the FP64 plain formula (no contraction) decides, with the
        // oracle's rounding; the FP32 copy settles candidates away from it
        if (ok && !(d2 < p.rlist2_lo))
          ok = dist2_plain(sub_plain(b.x[j], xi), sub_plain(b.y[j], yi), sub_plain(b.z[j], zi)) < p.rlist2;
        const unsigned long long m = (__ballot(ok) >> gbase) & gmask;
        // (uniform over the atom's lanes; the source lane is one of them)
        if (base < 0 && m != 0) base = __shfl(j, gbase + __ffsll((long long)m) - 1);
        if (ok) jmax = j;
        const unsigned pos = (unsigned)cnt + (unsigned)__popcll(m & below);
        int prev = base;
        if (!w32 && m != 0) {  // (most ballots keep nothing: uniform over the atom's lanes)
          // every kept entry's index first, then the one LPA places back
          // (this ballot's or an earlier one's); a wavefront's LDS accesses
          // take effect in program order, so only the compiler is held back
          if (ok) rg[pos & 63] = j;
          __builtin_amdgcn_wave_barrier();
          asm volatile("" ::: "memory");
          if (ok && pos >= (unsigned)LPA) prev = rg[(pos - LPA) & 63];
          __builtin_amdgcn_wave_barrier();
          asm volatile("" ::: "memory");
        }
        if (ok && pos < (unsigned)cap) {
          const unsigned l = pos % LPA, sl = pos / LPA;
          if (!w32) {
            // (a step of 65,535 or more is caught by the span test below,
            // which discards this attempt)
            reinterpret_cast<uint16_t *>(b.nbr)[(size_t)(sl / kGroup16) * (size_t)p.nbr_stride * kGroup16 +
                                                (size_t)self * (LPA * kGroup16) + l * kGroup16 + sl % kGroup16] =
                (uint16_t)(j - prev);
          } else {
            b.nbr[(size_t)(sl / kGroup) * group_stride + slot_base + l * kGroup + sl % kGroup] = j;
          }
        }
        cnt += __popcll(m);
      }
    }
  }
  // the span of the listed indices, equal in the atom's KB lanes
#pragma unroll
  for (int o = KB / 2; o > 0; o >>= 1) jmax = max(jmax, __shfl_xor(jmax, o));
  const bool wide = base >= 0 && jmax - base >= kOffSentinel;
  if (!w32 && wide) return false;
  const bool over = cnt > cap;  // cnt is the same in all KB lanes (ballot counts)
  if (over) cnt = cap;
  // pad to whole passes with the sentinel (cap is a multiple of kPass * LPA)
  const int padded = (cnt + kPass * LPA - 1) / (kPass * LPA) * (kPass * LPA);
  for (int e = cnt + lane; e < padded; e += KB) {
    if (!w32) reinterpret_cast<uint16_t *>(b.nbr)[nbr16_index(i, e, LPA, p.nbr_stride)] = (uint16_t)kOffSentinel;
    else b.nbr[nbr_index(i, e, LPA, p.nbr_stride)] = (int)p.ntot;
  }
  if (lane == 0) {
    if (over) set_err(b, E_OVERFLOW);
    b.ncount[i] = cnt;
    b.nbase[i] = base < 0 ? self : base;
    // 0: 16-bit; 32-bit indices: 1 where 16 bits would fit (the next build
    // tries them), 2 where they would not
    b.nwide[i] = w32 ? (wide ? 2 : 1) : 0;
    b.xr[i] = (float)xi;
    b.yr[i] = (float)yi;
    b.zr[i] = (float)zi;
  }
  return true;
}

// Grid-stride over atoms: KB lanes per atom.  cond != 0: a rebuild point
// inside a chunk, which builds only when the step before asked for it (its
// kick-drift, or in the mixed form the force pass before that).
template <class R, int LPA>
__global__ __launch_bounds__(kBlock) void k_build(Params p, Buffers b, int32_t cond) {
  if (cond) {
    if (b.ctl->rebuild == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long *>(&b.ctl->nbuild), 1ull);
  }
  const int lane = (int)(threadIdx.x & (KB - 1));
  const int64_t per_pass = (int64_t)gridDim.x * (kBlock / KB);
  for (int64_t i = (int64_t)blockIdx.x * (kBlock / KB) + threadIdx.x / KB; i < p.ntot; i += per_pass)
    if (b.group[i] != kPad) {  // a lane group skips together
      // the form the atom's last list took (2: 32-bit and wider than 16
      // bits) is tried first; a 16-bit attempt that does not fit is redone
      const bool w32 = b.nwide[i] == 2;
      if (!build_one<R, LPA>(p, b, i, lane, w32)) build_one<R, LPA>(p, b, i, lane, true);
    }
}

// Staged build.  The candidate scan only filters: each kept index goes, at
// its ballot-prefix position (the order of build_one), to the atom's buffer
// in LDS (Params::cap_slots * LPA words, the list's capacity).  Once the
// scan is over, the atom's lanes write the list from there in whole 16-byte
// groups, in the 16-bit form if the indices kept span less than 65,535 and
// as 32-bit indices otherwise; so no attempt is redone, and the per-candidate
// work is the filter, a ballot and at most one LDS store.  Same lists as
// build_one, entry for entry.
template <class R, int LPA>
__device__ void build_staged(const Params &p, const Buffers &b, int64_t i, int lane, int *buf, int *rowtab) {
  using V4 = typename V4T<R>::T;
  const int r = b.blk_rep[i / kTile];
  const V4 *p4 = reinterpret_cast<const V4 *>(b.pos4);
  const RepInfo &rp = b.rep[r];
  const double xi = b.x[i], yi = b.y[i], zi = b.z[i];
  const float4 pi = make_float4((float)(R)(xi - gorigin<R>(rp, 0)), (float)(R)(yi - gorigin<R>(rp, 1)),
                                (float)(R)(zi - gorigin<R>(rp, 2)), 0.f);
  int rs[NRL], re[NRL];
  stencil_rows<R>(p, b, i, lane, rp, xi, yi, zi, rs, re);
  const int gbase = (threadIdx.x & 63) & ~(KB - 1);
  const unsigned below = (1u << lane) - 1u;
  const int cap = p.cap_slots * LPA;
  const int self = (int)i;
  // The 25 row ranges as one sequence of candidates c = 0 .. T - 1: row q
  // holds c in [P_q, P_q+1) and candidate c of it is atom c + (rs_q - P_q).
  // The scan takes KB x KCH consecutive candidates per pass whatever rows
  // they fall in, instead of a pass per row (rows average fewer candidates
  // than a pass holds).  P and the offsets go to LDS (tab: P at 0 .. 25,
  // offsets at 32 .. 56); lane l resolved rows l and l + KB.
  int len[NRL];
#pragma unroll
  for (int h2 = 0; h2 < NRL; ++h2) len[h2] = re[h2] - rs[h2];
  int tot = 0;
  int *tab = rowtab + (threadIdx.x / KB) * 64;
#pragma unroll
  for (int h2 = 0; h2 < NRL; ++h2) {
    int incl = len[h2];
#pragma unroll
    for (int o = 1; o < KB; o <<= 1) {
      const int up = __shfl_up(incl, o, KB);
      if (lane >= o) incl += up;
    }
    const int q = lane + h2 * KB;
    const int start = tot + incl - len[h2];
    if (q < 25) {
      tab[q] = start;
      tab[32 + q] = rs[h2] - start;
    }
    tot += __shfl(incl, gbase + KB - 1);
  }
  if (lane == 0) tab[25] = tot;
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  // this lane's row, the next row's start and the offset (its candidates
  // only move forward)
  int k = 0, pn = tab[1], off = tab[32];
  int cnt = 0;
  for (int c0 = 0; c0 < tot; c0 += KB * KCH) {
    int jc[KCH];
    bool in[KCH];
#pragma unroll
    for (int u = 0; u < KCH; ++u) {
      const int c = c0 + u * KB + lane;
      while (k < 24 && c >= pn) {
        ++k;
        pn = tab[k + 1];
        off = tab[32 + k];
      }
      in[u] = c < tot;
      jc[u] = in[u] ? c + off : self;
    }
    float4 qv[KCH];
#pragma unroll
    for (int u = 0; u < KCH; ++u) qv[u] = to_f4<R>(gather<V4>(p4, jc[u]));
#pragma unroll
    for (int u = 0; u < KCH; ++u) {
      const int j = jc[u];
      const float dx = qv[u].x - pi.x, dy = qv[u].y - pi.y, dz = qv[u].z - pi.z;
      const float d2 = dx * dx + dy * dy + dz * dz;
      bool ok = in[u] & (j != self) & (d2 <= p.rlist2_hi);
      // near rlist the FP64 plain formula (no contraction) decides, with the
      // oracle's rounding; the FP32 copy settles candidates away from it
      if (ok && !(d2 < p.rlist2_lo))
        ok = dist2_plain(sub_plain(b.x[j], xi), sub_plain(b.y[j], yi), sub_plain(b.z[j], zi)) < p.rlist2;
      const unsigned m = (unsigned)(__ballot(ok) >> gbase) & ((1u << KB) - 1u);
      const int pos = cnt + __popc(m & below);
      if (ok && pos < cap) buf[pos] = j;
      cnt += __popc(m);
    }
  }
  // (a wavefront's LDS accesses take effect in program order: only the
  // compiler is held back)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  const bool over = cnt > cap;  // cnt is the same in all KB lanes (ballot counts)
  const int n = over ? cap : cnt;
  // kept in increasing index order: the span is the last minus the first
  const int base = n > 0 ? buf[0] : self;
  const bool w32 = n > 0 && buf[n - 1] - base >= kOffSentinel;
  const int padded = (n + kPass * LPA - 1) / (kPass * LPA) * (kPass * LPA);
  int4 *out = reinterpret_cast<int4 *>(b.nbr);
  if (!w32) {
    // group g: lane l = g % LPA of pass row = g / LPA, its eight entries
    for (int g = lane; g < padded / kGroup16; g += KB) {
      const int row = g / LPA, l = g % LPA;
      const int e0 = row * kGroup16 * LPA + l;
      int prev = row == 0 ? base : buf[e0 - LPA];
      unsigned v[kGroup16];
#pragma unroll
      for (int s = 0; s < kGroup16; ++s) {
        const int e = e0 + s * LPA;
        if (e < n) {
          const int j = buf[e];
          v[s] = (unsigned)(j - prev);
          prev = j;
        } else {
          v[s] = (unsigned)kOffSentinel;
        }
      }
      out[(size_t)row * p.nbr_stride + (size_t)i * LPA + l] =
          make_int4((int)(v[0] | (v[1] << 16)), (int)(v[2] | (v[3] << 16)), (int)(v[4] | (v[5] << 16)),
                    (int)(v[6] | (v[7] << 16)));
    }
  } else {
    // group g: lane l = g % LPA, slots 4 (g / LPA) .. 4 (g / LPA) + 3
    for (int g = lane; g < padded / kGroup; g += KB) {
      const int sg = g / LPA, l = g % LPA;
      int v[kGroup];
#pragma unroll
      for (int s = 0; s < kGroup; ++s) {
        const int e = (sg * kGroup + s) * LPA + l;
        v[s] = e < n ? buf[e] : (int)p.ntot;
      }
      out[(size_t)sg * p.nbr_stride + (size_t)i * LPA + l] = make_int4(v[0], v[1], v[2], v[3]);
    }
  }
  if (lane == 0) {
    if (over) set_err(b, E_OVERFLOW);
    b.ncount[i] = n;
    b.nbase[i] = base;
    b.nwide[i] = w32 ? 2 : 0;
    b.xr[i] = (float)xi;
    b.yr[i] = (float)yi;
    b.zr[i] = (float)zi;
  }
  // the buffer is reused by the atom's lanes for their next atom
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// The staged build's kernel: dynamic LDS of kBlock / KB buffers of
// Params::cap_slots * LPA words (launched where that fits kStageLdsMax,
// which leaves room for the row tables within a block's 64 KiB).
constexpr int kStageLdsMax = 60 * 1024;
template <class R, int LPA>
__global__ __launch_bounds__(kBlock) void k_build_staged(Params p, Buffers b, int32_t cond) {
  if (cond) {
    if (b.ctl->rebuild == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long *>(&b.ctl->nbuild), 1ull);
  }
  extern __shared__ int stage[];
  __shared__ int rowtab[(kBlock / KB) * 64];
  const int lane = (int)(threadIdx.x & (KB - 1));
  int *buf = stage + (size_t)(threadIdx.x / KB) * (size_t)(p.cap_slots * LPA);
  const int64_t per_pass = (int64_t)gridDim.x * (kBlock / KB);
  for (int64_t i = (int64_t)blockIdx.x * (kBlock / KB) + threadIdx.x / KB; i < p.ntot; i += per_pass)
    if (b.group[i] != kPad) build_staged<R, LPA>(p, b, i, lane, buf, rowtab);  // a lane group skips together
}

// In the mixed form (p.fold) the step's kick-drift is done here too.  The
// pair loop takes every position, the atom's own included, from
// Buffers::pnext, which the previous force pass wrote (the position after
// this step's drift, with the last lambda taken for this step's), so it
// needs neither lambda nor any other atom's update and starts at once.
// After it, every block takes lambda from the slot sums (start_lambda: the
// replica's first block also records the sample) and each atom's lanes
// update it exactly (lane 0 stores, the gather copy with its B').  One
// kernel boundary less per step.  Step 0 (forces at a burst's start) is
// the plain density pass.
// PR: a pruning pass (Params::inner): it walks the full list and writes the
// pruned one (the entries within rin, Control::rin2), which the pair passes
// of the following steps, up to the next pruning pass, read instead.
template <class R, int LPA, int NM, bool PR, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_density(Params p, Buffers b, int32_t k) {
  using V4 = typename V4T<R>::T;
  const int64_t blk = xcd_block();
  const int64_t gt = blk * kBlock + threadIdx.x;
  const int64_t i = gt / LPA;
  const int lane = (int)(gt & (LPA - 1));
  const int64_t tile = (blk * (kBlock / LPA)) / kTile;
  const int r = b.blk_rep[tile];
  const int64_t step = b.ctl->base + k;
  const int par = (int)(step & 1);
  const bool fold = FOLD && step >= 1;
  if (!FOLD) {
    // the slots of the other parity were consumed by this step's kick-drift
    // (in the mixed form the force pass clears them: this pass reads them)
    const size_t nz = (size_t)p.n_rep * kSlots * kNQ;
    unsigned long long *zp = b.slots + (size_t)(par ^ 1) * nz;
    for (size_t t = (size_t)gt; t < nz; t += (size_t)gridDim.x * kBlock) zp[t] = 0ull;
  }
  // every block of a conditional build has read the request: clear it
  if (gt == 0 && b.ctl->rebuild != 0) atomicAnd(&b.ctl->rebuild, 0);
  if (fold ? frozen(p, b, r, step) : (p.conv && b.acc[r].conv_step != 0)) return;  // converged replica: frozen
  const uint8_t g = b.group[i];
  const bool real = g != kPad;
  const V4 *p4 = reinterpret_cast<const V4 *>(b.pos4);
  const V4 *pn = fold ? reinterpret_cast<const V4 *>(b.pnext) : p4;  // positions of the pair terms
  V4 pi;
  if (real) pi = pn[i];
  // folded step: this lane's slot of the previous step's kinetic sum and
  // the atom's state, read ahead of the pair loop (the force pass that wrote
  // them has finished), so that the kick after it waits on no load.  The
  // registers this holds limit the kernel to 5 wavefronts per SIMD; the
  // folded sizes (up to 131,072 atoms) launch at most 8 at 4 lanes per atom
  // and 4 at 2, where the latency hidden outweighs the residency lost.
  const long long qk = fold ? kinetic_slot(p, b, r, step) : 0;
  KickAtom at{};
  if (fold) at = kick_load(b, i, true);
  // Sutton-Chen: sum of (a/r)^m, of r and the pair count; the shift
  // rho_s = (a/r)^m - rhoc - (r - rc) drhoc is applied once per atom.
  // Tables: the sum of the interpolated rho.
  R acc = (R)0, sr = (R)0;
  int np = 0;
  if (real) {
    const R rc2 = (R)p.rc2, a = (R)p.a;
    // the full list when pruning (or without pruned lists), else the pruned one
    const bool full = PR || !p.inner;
    // slots per lane: the list is padded with the far-away sentinel to whole
    // passes, so every slot of a pass holds a valid index
    const int cnt = (full ? b.ncount : b.ncounti)[i];
    const int npl = pass_slots<LPA>(cnt);
    const int base = full ? b.nbase[i] : b.nbasei[i];
    const bool w32 = (full ? b.nwide[i] : b.nwidei[i]) != 0;
    const int4 *nb4 = reinterpret_cast<const int4 *>(full ? b.nbr : b.nbri) + (size_t)i * LPA + lane;
    const R rin2 = PR ? (R)b.ctl->rin2 : (R)0;
    PruneWriter<LPA> pw;
    if (PR) {
      __shared__ int ring[PR ? 2 * kPass * kBlock : 1];
      pw.init(ring, base, w32);
    }
    pair_passes<true>(pn, nb4, p.nbr_stride, npl, lane_entries<LPA>(cnt, lane), base, w32, (int)p.ntot, [&](const V4(&pj)[8], const int(&jv)[8]) {
      bool keep[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const R dx = pj[u].x - pi.x, dy = pj[u].y - pi.y, dz = pj[u].z - pi.z;
        const R r2 = dx * dx + dy * dy + dz * dz;
        keep[u] = PR && r2 < rin2;
        if (r2 < rc2) {
          const R rinv = rsqrt_r(r2);
          if (NM == 2) {
            R t;
            const int kk = tab_interval<R>(p, r2 * rinv, &t);
            const V4 c = reinterpret_cast<const V4 *>(b.tab_r)[2 * kk];
            acc += c.x + t * (c.y + t * (c.z + t * c.w));
          } else {
            acc += rho_pow<R, NM>(a * rinv, p.m);
            sr += r2 * rinv;
            ++np;
          }
        }
      }
      if (PR) pw.pass(p, b, i, lane, keep, jv);
    });
    if (PR) pw.finish(p, b, i, lane, base);
  }
#pragma unroll
  for (int o = LPA / 2; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o);
    if (NM != 2) {
      sr += __shfl_xor(sr, o);
      np += __shfl_xor(np, o);
    }
  }
  if (fold) {
    const int64_t a0 = blk * (kBlock / LPA);  // the block's first atom
    const bool first = a0 % kTile == 0 && (tile == 0 || b.blk_rep[tile - 1] != r);
    const StepStart st = start_lambda(p, b, r, step, first, 0, qk);
    // a replica whose averages converged at this step's sample keeps its
    // state after lambda (no drift); the rest of this step is not needed
    kick_atom<R>(p, b, i, at, st.lam, !st.stop, false, *st.rep, lane == 0, false);
    if (st.stop) return;
    pi.x = (R)(at.x - gorigin<R>(*st.rep, 0));
    pi.y = (R)(at.y - gorigin<R>(*st.rep, 1));
    pi.z = (R)(at.z - gorigin<R>(*st.rep, 2));
  }
  long long q[1] = {0};
  if (lane == 0 && real) {
    double rb = (double)acc;
    if (NM != 2) {
      rb += -(double)np * p.rhoc - p.drhoc * ((double)sr - (double)np * p.rc);
      // the same pairs shift the pair energy, which the force pass adds
      b.eshift[i] = -(double)np * p.Vc - p.dVc * ((double)sr - (double)np * p.rc);
    }
    double Bp = 0.0, B = 0.0;
    if (NM == 2) {
      tab_embed(p, b.tab_F, rb, &B, &Bp);
    } else if (rb > 0.0) {
      const double sq = sqrt(rb);
      B = -p.c_eps * sq;
      Bp = -0.5 * p.c_eps / sq;
    }
    // the force pass reads B' (tables) or -m B' (Sutton-Chen, one product less per pair)
    const R wv = (R)(NM == 2 ? Bp : -(double)p.m * Bp);
    if (fold && moves_z(p, g)) {  // the gather copy of the moved atom, with its B'
      V4 v4 = pi;
      v4.w = wv;
      reinterpret_cast<V4 *>(b.pos4)[i] = v4;
    } else {
      reinterpret_cast<R *>(b.pos4)[4 * i + 3] = wv;
    }
    q[0] = to_fix(B);
  }
  block_atoms_add<1, kBlock / LPA>(q, lane == 0, threadIdx.x / LPA,
                                   slot_row(b, p.n_rep, par, r, blockIdx.x & (kSlots - 1)) + Q_EMB);
}

// ---------------------------------------------------------------------------
// force pass: mode 0 = step (second half kick + sums), 1 = forces only,
// 2 = step, and the next step is a list rebuild point of the mixed form
// ---------------------------------------------------------------------------
template <class R, int LPA, int NM, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_force(Params p, Buffers b, int32_t k, int32_t mode) {
  using V4 = typename V4T<R>::T;
  const unsigned long long t_begin = p.ktime ? wall_clock64() : 0ull;
  const int64_t blk = xcd_block();
  const int64_t gt = blk * kBlock + threadIdx.x;
  const int64_t i = gt / LPA;
  const int lane = (int)(gt & (LPA - 1));
  const int64_t tile = (blk * (kBlock / LPA)) / kTile;
  const int r = b.blk_rep[tile];
  const int64_t step = b.ctl->base + k;
  const int par = (int)(step & 1);
  if (FOLD) {
    // mixed form: the slots of the other parity were read by this step's
    // density pass (its kick-drift part); the next step's adds into them
    const size_t nz = (size_t)p.n_rep * kSlots * kNQ;
    unsigned long long *zp = b.slots + (size_t)(par ^ 1) * nz;
    for (size_t t = (size_t)gt; t < nz; t += (size_t)gridDim.x * kBlock) zp[t] = 0ull;
  }
  if (p.conv && b.acc[r].conv_step != 0) return;  // converged replica: frozen
  const uint8_t g = b.group[i];
  const bool real = g != kPad;
  // the state the epilogue needs, read ahead of the pair loop: z for the
  // virial, and in the mixed form what the next position takes
  double x = 0.0, y = 0.0, z = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
  if (real && lane == 0) {
    z = b.z[i];
    if (FOLD) {
      x = b.x[i]; y = b.y[i];
      vx = b.vx[i]; vy = b.vy[i]; vz = b.vz[i];
    }
  }
  const double eshift = (NM != 2 && real && lane == 0) ? b.eshift[i] : 0.0;  // read ahead too
  const double zc = b.rep[r].center[2];
  const V4 *p4 = reinterpret_cast<const V4 *>(b.pos4);
  // The virial W_zz = 1/2 sum_ij (z_i - z_j) F_ij,z equals sum_i z_i F_i,z
  // for these pair-antisymmetric internal forces, so it is formed per atom
  // after the loop instead of per pair; and since they sum to zero, as
  // sum_i (z_i - z_c) F_i,z about the cube's centre z_c, which weights each
  // force's rounding by at most the cube's half height.
  // Sutton-Chen, with w_j = -m B'_j from the density pass:
  //   dU/dr = [-n eps (a/r)^n + (w_i + w_j) (a/r)^m] / r - (dVc - (w_i + w_j) drhoc / m)
  // and the pair energy V - Vc - (r - rc) dVc summed as sum(-n V) here (as
  // sum (a/r)^n for n = 7, m = 6) and the shift, which the density pass
  // formed from its sums of r and of the pairs.  Tables: B' as is.
  R fx = 0, fy = 0, fz = 0, ep = 0;
  if (real) {
    const V4 pi = p4[i];
    const R rc2 = (R)p.rc2, a = (R)p.a;
    const R neps = -(R)p.n * (R)p.eps;
    const R dVc = (R)p.dVc, dm = (R)(p.drhoc / p.m);
    // slots per lane: the list is padded with the far-away sentinel to whole
    // passes, so every slot of a pass holds a valid index
    const int cnt = (p.inner ? b.ncounti : b.ncount)[i];
    const int npl = pass_slots<LPA>(cnt);
    const int base = p.inner ? b.nbasei[i] : b.nbase[i];
    const bool w32 = (p.inner ? b.nwidei[i] : b.nwide[i]) != 0;
    const int4 *nb4 = reinterpret_cast<const int4 *>(p.inner ? b.nbri : b.nbr) + (size_t)i * LPA + lane;
    pair_passes<false>(p4, nb4, p.nbr_stride, npl, lane_entries<LPA>(cnt, lane), base, w32, (int)p.ntot, [&](const V4(&pj)[8], const int(&)[8]) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const R dx = pj[u].x - pi.x, dy = pj[u].y - pi.y, dz = pj[u].z - pi.z;
        const R r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2) {
          const R rinv = rsqrt_r(r2);
          R f;
          if (NM == 2) {
            // setfl tables: V = (r phi)/r, V' = ((r phi)' - V)/r, rho' from its spline
            R t;
            const int kk = tab_interval<R>(p, r2 * rinv, &t);
            const V4 cr = reinterpret_cast<const V4 *>(b.tab_r)[2 * kk];
            const V4 cp = reinterpret_cast<const V4 *>(b.tab_r)[2 * kk + 1];
            const R idr = (R)p.tab_inv_dr;
            const R drho = (cr.y + t * ((R)2 * cr.z + (R)3 * t * cr.w)) * idr;
            const R rphi = cp.x + t * (cp.y + t * (cp.z + t * cp.w));
            const R drphi = (cp.y + t * ((R)2 * cp.z + (R)3 * t * cp.w)) * idr;
            const R V = rphi * rinv;
            f = ((drphi - V) * rinv + (pi.w + pj[u].w) * drho) * rinv;
            ep += V;
          } else if (NM == 1) {
            // n = m + 1: ws t^m - n eps t^n = (ws - n eps t) t^m, and the
            // energy sums t^n (eps applied once per atom)
            const R t = a * rinv, t2 = t * t;
            const R t6 = t2 * t2 * t2;
            const R ws = pi.w + pj[u].w;
            const R C = (neps * t + ws) * t6;
            const R D = dVc - ws * dm;
            f = (C * rinv - D) * rinv;
            ep += t6 * t;
          } else {
            R tn, tm;
            sc_powers<R, NM>(a * rinv, p.n, p.m, &tn, &tm);
            const R A = neps * tn;  // -n V
            const R ws = pi.w + pj[u].w;
            const R C = ws * tm + A;
            const R D = dVc - ws * dm;
            f = (C * rinv - D) * rinv;
            ep += A;
          }
          fx += f * dx;
          fy += f * dy;
          fz += f * dz;
        }
      }
    });
  }
#pragma unroll
  for (int o = LPA / 2; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o);
    fy += __shfl_xor(fy, o);
    fz += __shfl_xor(fz, o);
    ep += __shfl_xor(ep, o);
  }
  long long q[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (lane == 0 && real) {
    const double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
    b.fx[i] = Fx;
    b.fy[i] = Fy;
    b.fz[i] = Fz;
    if (!isfinite(Fx + Fy + Fz)) set_err(b, E_NONFINITE);
    if (moves_z(p, g)) {
      if (!FOLD) {
        vx = b.vx[i];
        vy = b.vy[i];
        vz = b.vz[i];
      }
      if (mode != 1) {
        if (g == 0) {
          vx += p.hdt_m * Fx;
          vy += p.hdt_m * Fy;
        }
        vz += p.hdt_m * Fz;
        b.vx[i] = vx;
        b.vy[i] = vy;
        b.vz[i] = vz;
      }
      q[Q_MV2] = to_fix(p.mvv2e_m * (vx * vx + vy * vy + vz * vz));
      q[Q_MVZ2] = to_fix(p.mvv2e_m * vz * vz);
    }
    if (FOLD) {
      // mixed form: where the next step's drift takes the atom, for the next
      // density pass (forces only: a burst's first step, lambda 1); and,
      // before a rebuild point, whether the lists last until the one after
      // it (from here, over m steps)
      const double lp = mode == 1 ? 1.0 : b.acc[r].lam_last;
      reinterpret_cast<V4 *>(b.pnext)[i] = next_position<R>(p, b.rep[r], g, lp, x, y, z, vx, vy, vz, Fx, Fy, Fz);
      if (mode == 2 && moves_z(p, g)) {
        const double ex = x - (double)b.xr[i], ey = y - (double)b.yr[i], ez = z - (double)b.zr[i];
        if (sqrt(ex * ex + ey * ey + ez * ez) + p.trig_v * sqrt(vx * vx + vy * vy + vz * vz) > p.trig_lim)
          atomicOr(&b.ctl->rebuild, 1);
      }
    }
    // pair energy of the atom: tables sum V; Sutton-Chen sums -n V (n = 7,
    // m = 6: (a/r)^n, that is V / eps), plus the shift
    const double epair = (NM == 2) ? (double)ep : (NM == 1 ? p.eps * (double)ep : -(double)ep / p.n) + eshift;
    q[Q_EPAIR] = to_fix(0.5 * epair);
    q[Q_WZZ] = to_fix((z - zc) * Fz);
    if (g == 2) q[Q_RZ] = to_fix(-Fz);
  }
  block_atoms_add<kNQ, kBlock / LPA>(q, lane == 0, threadIdx.x / LPA,
                                     slot_row(b, p.n_rep, par, r, blockIdx.x & (kSlots - 1)));
  if (p.ktime && threadIdx.x == 0) {
    // span of this block on the device wall clock (the host takes the
    // earliest start and the latest end over all blocks)
    b.ktime[2 * (size_t)blockIdx.x] = t_begin;
    b.ktime[2 * (size_t)blockIdx.x + 1] = wall_clock64();
  }

}

// ---------------------------------------------------------------------------
// chunk statistics: max drift since the last sort and max speed, per replica
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// order-preserving map of a double onto uint64 (for min/max atomics)
__device__ __forceinline__ unsigned long long okey(double v) {
  unsigned long long u = dbits(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// stat rows: [replica][slot][kStat] = drift^2, v^2 (max, double bits), min
// x,y,z and max x,y,z (order-preserving keys), displacement^2 since the list
// build (max, double bits)
// Block 0 also folds the per-block time stamps of a timed force launch
// (n_stamps start/end pairs) into Control::kt_first / kt_last.
__global__ void k_stat_init(unsigned long long *stat, int64_t rows, const unsigned long long *stamps,
                            int64_t n_stamps, Control *ctl) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * kStat;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % kStat);
    stat[t] = (c >= 2 && c < 5) ? ~0ull : 0ull;
  }
  if (blockIdx.x != 0 || n_stamps == 0) return;
  unsigned long long t0 = ~0ull, t1 = 0ull;
  for (int64_t q = threadIdx.x; q < n_stamps; q += blockDim.x) {
    t0 = min(t0, stamps[2 * q]);
    t1 = max(t1, stamps[2 * q + 1]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    t0 = min(t0, (unsigned long long)shfl_xor_ll((long long)t0, o));
    t1 = max(t1, (unsigned long long)shfl_xor_ll((long long)t1, o));
  }
  __shared__ unsigned long long sh[2][kBlock / 64];
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = t0;
    sh[1][threadIdx.x >> 6] = t1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      t0 = min(t0, sh[0][w]);
      t1 = max(t1, sh[1][w]);
    }
    ctl->kt_first = t0;
    ctl->kt_last = t1;
  }
}

// Chunk-end statistics per replica: max drift since the last sort, max
// speed and max displacement since the list build of the mobile atoms, and
// the bounding box of all real atoms (the grid of the next sort).
__global__ __launch_bounds__(kBlock) void k_chunk_stats(Params p, Buffers b) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  double d2 = 0.0, v2 = 0.0, l2 = 0.0;
  unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
  long long mom[6] = {0, 0, 0, 0, 0, 0};  // per axis: sum of q and of q^2, q = rint(4 x) (integers: order-free)
  const uint8_t g = b.group[i];
  if (g != kPad) {
    const double x = b.x[i], y = b.y[i], z = b.z[i];
    const double c[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
      mn[d] = mx[d] = okey(c[d]);
      // |x| < 1e4 A (the escape bound): q^2 < 1.6e9, far inside 64 bits over any atom count
      const long long q = isfinite(c[d]) ? (long long)rint(fmin(fmax(4.0 * c[d], -1e5), 1e5)) : 0;
      mom[d] = q;
      mom[3 + d] = q * q;
    }
    if (moves_z(p, g)) {
      const double ex = x - (double)b.xs[i], ey = y - (double)b.ys[i], ez = z - (double)b.zs[i];
      d2 = ex * ex + ey * ey + ez * ez;
      const double fx = x - (double)b.xr[i], fy = y - (double)b.yr[i], fz = z - (double)b.zr[i];
      l2 = fx * fx + fy * fy + fz * fz;
      v2 = b.vx[i] * b.vx[i] + b.vy[i] * b.vy[i] + b.vz[i] * b.vz[i];
    }
    if (!isfinite(x + y + z + d2 + v2 + l2)) {
      set_err(b, E_NONFINITE);
      d2 = v2 = l2 = 0.0;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 = fmax(d2, __shfl_xor(d2, o));
    v2 = fmax(v2, __shfl_xor(v2, o));
    l2 = fmax(l2, __shfl_xor(l2, o));
    for (int d = 0; d < 3; ++d) {
      mn[d] = min(mn[d], (unsigned long long)shfl_xor_ll((long long)mn[d], o));
      mx[d] = max(mx[d], (unsigned long long)shfl_xor_ll((long long)mx[d], o));
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) mom[d] += shfl_xor_ll(mom[d], o);
  }
  __shared__ unsigned long long sh[kBlock / 64][15];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid][0] = dbits(d2);
    sh[wid][1] = dbits(v2);
    for (int d = 0; d < 3; ++d) {
      sh[wid][2 + d] = mn[d];
      sh[wid][5 + d] = mx[d];
    }
    sh[wid][8] = dbits(l2);
    for (int d = 0; d < 6; ++d) sh[wid][kStatMom + d] = (unsigned long long)mom[d];
  }
  __syncthreads();
  if (threadIdx.x < kStatMom + 6) {
    const int c = threadIdx.x;
    unsigned long long v = sh[0][c];
    for (int w2 = 1; w2 < kBlock / 64; ++w2) {
      if (c >= kStatMom) v += sh[w2][c];  // two's-complement sums
      else v = (c >= 2 && c < 5) ? min(v, sh[w2][c]) : max(v, sh[w2][c]);
    }
    unsigned long long *dst = b.stat + ((size_t)r * kSlots + (blockIdx.x & (kSlots - 1))) * kStat + c;
    if (c >= kStatMom) atomicAdd(dst, v);
    else if (c >= 2 && c < 5) atomicMin(dst, v);
    else atomicMax(dst, v);
  }
}

__device__ __forceinline__ int cell_coord(double v, double o, double inv_h, int dim) {
  const double t = floor(sub_plain(v, o) * inv_h);
  if (!(t >= 0.0)) return 0;
  if (t >= (double)dim) return dim - 1;
  return (int)t;
}

__device__ __forceinline__ int atom_cell(const Buffers &b, const RepInfo &rp, int64_t i) {
  if (b.group[i] == kPad) return (int)(rp.ncells - 1);  // virtual last cell: padding sorts to the end
  int c[3];
  c[0] = cell_coord(b.x[i], rp.origin[0], rp.inv_h, rp.dims[0]);
  c[1] = cell_coord(b.y[i], rp.origin[1], rp.inv_h, rp.dims[1]);
  c[2] = cell_coord(b.z[i], rp.origin[2], rp.inv_h, rp.dims[2]);
  const int a0 = rp.ax[0], a1 = rp.ax[1], a2 = rp.ax[2];
  return (c[a2] * rp.dims[a1] + c[a1]) * rp.dims[a0] + c[a0];
}

// One atomic per distinct cell in a wave (atoms arrive nearly sorted, so a
// wave touches few cells).
__global__ __launch_bounds__(kBlock) void k_assign_count(Params p, Buffers b, int32_t *key) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  const RepInfo &rp = b.rep[r];
  const int c = atom_cell(b, rp, i);
  key[i] = c;
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(true);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lk = __shfl(c, leader);
    const unsigned long long m = __ballot(c == lk) & todo;
    if (lane == leader) atomicAdd(b.cell_count + rp.cell_off + lk, __popcll(m));
    todo &= ~m;
  }
}

// Exclusive scan of each replica's cell counts into cell_start (and the
// scatter cursors), starting at the replica's first sorted atom.  Three
// launches over tiles of kScanTile cells (grid: tiles x replicas, blocks
// past a replica's last tile leave at once): the tile sums; their scan per
// replica; each tile's scan from its base.  Every wavefront reads and
// writes contiguous runs.  (A single block per replica, each thread a run
// of its own, took 136 us on a 97,000-cell grid: its lanes read 64
// different cache lines per load through one compute unit.)  Counts stay
// below 2^27, so 32-bit sums suffice.
constexpr int kScanPer = 16;                    // cells per thread in a tile
constexpr int kScanTile = kBlock * kScanPer;    // 4096

// Sum over the block (all kBlock threads), returned to every thread.
__device__ __forceinline__ int block_sum_int(int v) {
  __shared__ int ws[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) t += ws[w];
  return t;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(Buffers b, int32_t *tsum, int32_t tmax) {
  const int r = blockIdx.y;
  const int64_t ncl = b.rep[r].ncells;
  const int64_t c0 = (int64_t)blockIdx.x * kScanTile;
  if (c0 >= ncl) return;  // uniform over the block
  const int32_t *cnt = b.cell_count + b.rep[r].cell_off + c0;
  const int n = (int)min<int64_t>(kScanTile, ncl - c0);
  int v[kScanPer];
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int k = u * kBlock + (int)threadIdx.x;  // contiguous over the block
    v[u] = k < n ? cnt[k] : 0;
  }
  int sum = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) sum += v[u];
  sum = block_sum_int(sum);
  if (threadIdx.x == 0) tsum[(size_t)r * tmax + blockIdx.x] = sum;
}

// one block per replica: tile sums -> tile bases (the replica's first atom
// plus the sums of the tiles before), in place
__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(Buffers b, int32_t *tsum, int32_t tmax) {
  __shared__ int ws[kBlock / 64];
  const int r = blockIdx.x;
  const int nt = (int)((b.rep[r].ncells + kScanTile - 1) / kScanTile);
  int32_t *t = tsum + (size_t)r * tmax;
  int carry = (int)b.rep[r].abeg;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k0 = 0; k0 < nt; k0 += kBlock) {
    const int k = k0 + (int)threadIdx.x;
    const int x = k < nt ? t[k] : 0;
    int v = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(v, o);
      if (lane >= o) v += y;
    }
    if (lane == 63) ws[wid] = v;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      before += w < wid ? ws[w] : 0;
      all += ws[w];
    }
    if (k < nt) t[k] = carry + before + v - x;
    carry += all;
    __syncthreads();  // ws is rewritten by the next round
  }
}

// each tile's exclusive scan from its base: thread t takes cells
// [t kScanPer, (t + 1) kScanPer) of the tile
__global__ __launch_bounds__(kBlock) void k_scan_write(Buffers b, const int32_t *tbase, int32_t tmax,
                                                       int32_t *cursor) {
  __shared__ int ws[kBlock / 64];
  const int r = blockIdx.y;
  const int64_t ncl = b.rep[r].ncells;
  const int64_t c0 = (int64_t)blockIdx.x * kScanTile;
  if (c0 >= ncl) return;  // uniform over the block
  const int64_t off = b.rep[r].cell_off + c0;
  const int n = (int)min<int64_t>(kScanTile, ncl - c0);
  const int k0 = (int)threadIdx.x * kScanPer;
  int v[kScanPer];
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) v[u] = k0 + u < n ? b.cell_count[off + k0 + u] : 0;
  int sum = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) sum += v[u];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) ws[wid] = incl;
  __syncthreads();
  int run = tbase[(size_t)r * tmax + blockIdx.x] + incl - sum;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) run += w < wid ? ws[w] : 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u)
    if (k0 + u < n) {
      b.cell_start[off + k0 + u] = run;
      cursor[off + k0 + u] = run;
      run += v[u];
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(Buffers b, const int32_t *key, int32_t *cursor, int32_t *tmp) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  const int64_t off = b.rep[r].cell_off;
  const int c = key[i];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long todo = __ballot(true);
  int pos = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lk = __shfl(c, leader);
    const unsigned long long m = __ballot(c == lk) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(cursor + off + lk, __popcll(m));
    base = __shfl(base, leader);
    if (c == lk) pos = base + __popcll(m & below);
    todo &= ~m;
  }
  tmp[pos] = (int32_t)i;
}

// Within each cell, order atoms by original index (padding atoms after, by
// position): a rank sort over unique keys.  The sorted order then depends on
// the positions only, not on the previous order nor on the order of atomics.
__device__ __forceinline__ long long sort_key(const Buffers &b, int v) {
  const int o = b.orig[v];
  return (o >= 0) ? (long long)o : ((1ll << 32) + (long long)v);
}

constexpr int kSortLds = 512;  // cells up to this size are ranked from LDS

__global__ __launch_bounds__(kBlock) void k_cell_sort(Buffers b, const int32_t *tmp, int32_t *perm, int64_t ncells_tot) {
  __shared__ long long keys[kBlock / 64][kSortLds];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * (kBlock / 64) + w;
  if (c >= ncells_tot) return;  // no block-wide barrier below: waves are independent
  const int start = b.cell_start[c], cnt = b.cell_count[c];
  if (cnt <= kSortLds) {
    for (int a = lane; a < cnt; a += 64) keys[w][a] = sort_key(b, tmp[start + a]);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int a = lane; a < cnt; a += 64) {
      const long long kv = keys[w][a];
      int rank = 0;
      for (int q = 0; q < cnt; ++q) rank += (keys[w][q] < kv) ? 1 : 0;
      perm[start + rank] = tmp[start + a];
    }
  } else {
    for (int a = lane; a < cnt; a += 64) {
      const int v = tmp[start + a];
      const long long kv = sort_key(b, v);
      int rank = 0;
      for (int q = 0; q < cnt; ++q) rank += (sort_key(b, tmp[start + q]) < kv) ? 1 : 0;
      perm[start + rank] = v;
    }
  }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_permute(Buffers b, Buffers sc, const int32_t *perm, const int32_t *key) {
  using V4 = typename V4T<R>::T;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t s = perm[i];
  const double x = b.x[s], y = b.y[s], z = b.z[s];
  sc.x[i] = x;
  sc.y[i] = y;
  sc.z[i] = z;
  sc.vx[i] = b.vx[s];
  sc.vy[i] = b.vy[s];
  sc.vz[i] = b.vz[s];
  sc.fx[i] = b.fx[s];
  sc.fy[i] = b.fy[s];
  sc.fz[i] = b.fz[s];
  sc.group[i] = b.group[s];
  sc.orig[i] = b.orig[s];
  sc.cell[i] = key[s];
  sc.nwide[i] = b.nwide[s];  // the form hint of the atom's next list build
  if (b.msx) {
    sc.msx[i] = b.msx[s];
    sc.msy[i] = b.msy[s];
    sc.msz[i] = b.msz[s];
  }
  sc.xs[i] = (float)x;
  sc.ys[i] = (float)y;
  sc.zs[i] = (float)z;
  const RepInfo &rp = b.rep[b.blk_rep[i / kTile]];
  V4 v;
  v.x = (R)(x - gorigin<R>(rp, 0));
  v.y = (R)(y - gorigin<R>(rp, 1));
  v.z = (R)(z - gorigin<R>(rp, 2));
  v.w = (R)0;
  reinterpret_cast<V4 *>(sc.pos4)[i] = v;
}

// state copy for roll-back: restore == 0 saves into the snapshot, 1 restores
__global__ __launch_bounds__(kBlock) void k_snapshot(Buffers b, double *snap, unsigned long long *snap_slots,
                                                     double *snap_acc, int restore, int64_t ntot, int64_t nslots,
                                                     int64_t nacc) {
  double *arr[12] = {b.x, b.y, b.z, b.vx, b.vy, b.vz, b.fx, b.fy, b.fz, b.msx, b.msy, b.msz};
  const int na = b.msx ? 12 : 9;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < ntot; t += stride) {
    for (int k = 0; k < na; ++k) {
      if (restore) arr[k][t] = snap[k * ntot + t];
      else snap[k * ntot + t] = arr[k][t];
    }
  }
  double *acc = reinterpret_cast<double *>(b.acc);
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nslots; t += stride) {
    if (restore) b.slots[t] = snap_slots[t];
    else snap_slots[t] = b.slots[t];
  }
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nacc; t += stride) {
    if (restore) acc[t] = snap_acc[t];
    else snap_acc[t] = acc[t];
  }
}

void launch_snapshot(const Buffers &b, double *snap, unsigned long long *snap_slots, double *snap_acc, int restore,
                     int64_t ntot, int64_t nslots, int64_t nacc, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>((ntot + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_snapshot, dim3(g), dim3(kBlock), 0, s, b, snap, snap_slots, snap_acc, restore, ntot, nslots,
                     nacc);
}

// v = 0 for every atom of group g (the top region is fixed again after relaxation)
__global__ __launch_bounds__(kBlock) void k_hold_group(Buffers b, int64_t ntot, uint8_t g) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < ntot && b.group[i] == g) b.vx[i] = b.vy[i] = b.vz[i] = 0.0;
}

void launch_hold_group(const Buffers &b, int64_t ntot, int g, hipStream_t s) {
  hipLaunchKernelGGL(k_hold_group, dim3((unsigned)((ntot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, b, ntot,
                     (uint8_t)g);
}

// copy the permuted arrays back into the primary buffers (one launch)
template <class R>
__global__ __launch_bounds__(kBlock) void k_copy_back(Buffers b, Buffers sc) {
  using V4 = typename V4T<R>::T;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  b.x[i] = sc.x[i]; b.y[i] = sc.y[i]; b.z[i] = sc.z[i];
  b.vx[i] = sc.vx[i]; b.vy[i] = sc.vy[i]; b.vz[i] = sc.vz[i];
  b.fx[i] = sc.fx[i]; b.fy[i] = sc.fy[i]; b.fz[i] = sc.fz[i];
  b.group[i] = sc.group[i];
  b.orig[i] = sc.orig[i];
  b.cell[i] = sc.cell[i];
  b.nwide[i] = sc.nwide[i];
  if (b.msx) {
    b.msx[i] = sc.msx[i];
    b.msy[i] = sc.msy[i];
    b.msz[i] = sc.msz[i];
  }
  b.xs[i] = sc.xs[i]; b.ys[i] = sc.ys[i]; b.zs[i] = sc.zs[i];
  reinterpret_cast<V4 *>(b.pos4)[i] = reinterpret_cast<const V4 *>(sc.pos4)[i];
}

__global__ __launch_bounds__(kBlock) void k_strain(Params p, Buffers b, const double *factor) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  if (b.group[i] == kPad) return;
  b.z[i] = b.z[i] * factor[r];
}

// pairs within rc (directed), list entries, pruned-list entries and atoms with 32-bit lists, summed into
// stat[r][slot][0..3]
template <class R>
__global__ __launch_bounds__(kBlock) void k_count_pairs(Params p, Buffers b) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  unsigned long long np = 0, ne = 0, nq = 0, nw = 0;
  if (b.group[i] != kPad) {
    const int cnt = b.ncount[i];
    const bool w32 = b.nwide[i] != 0;
    ne = cnt;
    nq = p.inner ? (unsigned long long)b.ncounti[i] : 0ull;
    nw = w32 ? 1 : 0;
    for (int l = 0; l < p.lpa; ++l) {
      int j = b.nbase[i];  // 16-bit form: steps from the lane's previous entry
      for (int e = l; e < cnt; e += p.lpa) {
        if (!w32) j += reinterpret_cast<const uint16_t *>(b.nbr)[nbr16_index(i, e, p.lpa, p.nbr_stride)];
        else j = b.nbr[nbr_index(i, e, p.lpa, p.nbr_stride)];
        const double d2 = dist2_plain(b.x[j] - b.x[i], b.y[j] - b.y[i], b.z[j] - b.z[i]);
        if (d2 < p.rc2) ++np;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    np += (unsigned long long)shfl_xor_ll((long long)np, o);
    ne += (unsigned long long)shfl_xor_ll((long long)ne, o);
    nq += (unsigned long long)shfl_xor_ll((long long)nq, o);
    nw += (unsigned long long)shfl_xor_ll((long long)nw, o);
  }
  if ((threadIdx.x & 63) == 0) {
    unsigned long long *row = b.stat + ((size_t)r * kSlots + (blockIdx.x & (kSlots - 1))) * kStat;
    atomicAdd(row, np);
    atomicAdd(row + 1, ne);
    atomicAdd(row + 2, nq);
    atomicAdd(row + 3, nw);
  }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned tiles(const Params &p) { return (unsigned)(p.ntot / kTile); }

void launch_burst_begin(const Params &p, const Buffers &b, int n_rep, hipStream_t s) {
  hipLaunchKernelGGL(k_burst_begin, dim3(64), dim3(kBlock), 0, s, b, n_rep, p.ntot);
}

void launch_set_base(const Buffers &b, int64_t base, hipStream_t s) {
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(1), 0, s, b.ctl, base);
}

void launch_set_ncells(const Buffers &b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ncells, dim3(1), dim3(1), 0, s, b.ctl, n);
}

void launch_set_prune(const Buffers &b, double rin2, double vb2, hipStream_t s) {
  hipLaunchKernelGGL(k_set_prune, dim3(1), dim3(1), 0, s, b.ctl, rin2, vb2);
}

void launch_fill_i64(unsigned long long *ptr, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kBlock), 0, s, ptr, n, v);
}

void launch_kick_drift(const Params &p, const Buffers &b, int precision, int32_t k, int32_t mode, hipStream_t s) {
  if (precision) hipLaunchKernelGGL(k_kick_drift<float>, dim3(tiles(p)), dim3(kBlock), 0, s, p, b, k, mode);
  else hipLaunchKernelGGL(k_kick_drift<double>, dim3(tiles(p)), dim3(kBlock), 0, s, p, b, k, mode);
}

void launch_pos4(const Params &p, const Buffers &b, int precision, hipStream_t s) {
  if (precision) hipLaunchKernelGGL(k_pos4<float>, dim3(tiles(p)), dim3(kBlock), 0, s, p, b);
  else hipLaunchKernelGGL(k_pos4<double>, dim3(tiles(p)), dim3(kBlock), 0, s, p, b);
}

// FOLD: the folded step (Params::fold), which exists in the mixed form only;
// its kernels are separate instances, so the others hold no registers for it.
template <class R, int NM, bool PR, bool FOLD>
static void density_lpa(const Params &p, const Buffers &b, int lpa, int32_t k, hipStream_t s) {
  const unsigned g = (unsigned)(p.ntot * lpa / kBlock);
  switch (lpa) {
    case 1: hipLaunchKernelGGL((k_density<R, 1, NM, PR, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    case 2: hipLaunchKernelGGL((k_density<R, 2, NM, PR, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    case 4: hipLaunchKernelGGL((k_density<R, 4, NM, PR, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    case 8: hipLaunchKernelGGL((k_density<R, 8, NM, PR, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    default: hipLaunchKernelGGL((k_density<R, 16, NM, PR, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
  }
}

template <class R, int NM>
static void density_form(const Params &p, const Buffers &b, int lpa, int32_t k, hipStream_t s, bool prune) {
  if constexpr (sizeof(R) == sizeof(float)) {
    if (p.fold) {
      (prune ? density_lpa<R, NM, true, true> : density_lpa<R, NM, false, true>)(p, b, lpa, k, s);
      return;
    }
  }
  (prune ? density_lpa<R, NM, true, false> : density_lpa<R, NM, false, false>)(p, b, lpa, k, s);
}

template <class R, int NM, bool FOLD>
static void force_fold(const Params &p, const Buffers &b, int lpa, int32_t k, int32_t mode, hipStream_t s) {
  const unsigned g = (unsigned)(p.ntot * lpa / kBlock);
  switch (lpa) {
    case 1: hipLaunchKernelGGL((k_force<R, 1, NM, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    case 2: hipLaunchKernelGGL((k_force<R, 2, NM, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    case 4: hipLaunchKernelGGL((k_force<R, 4, NM, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    case 8: hipLaunchKernelGGL((k_force<R, 8, NM, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    default: hipLaunchKernelGGL((k_force<R, 16, NM, FOLD>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
  }
}

template <class R, int NM>
static void force_lpa(const Params &p, const Buffers &b, int lpa, int32_t k, int32_t mode, hipStream_t s) {
  if constexpr (sizeof(R) == sizeof(float)) {
    if (p.fold) {
      force_fold<R, NM, true>(p, b, lpa, k, mode, s);
      return;
    }
  }
  force_fold<R, NM, false>(p, b, lpa, k, mode, s);
}

static bool is_al76(const Params &p) { return p.n == 7 && p.m == 6; }
// kernel form of the potential: 2 tables, 1 Sutton-Chen n = 7 / m = 6, 0 any Sutton-Chen
static int pot_form(const Params &p) { return p.tab ? 2 : (is_al76(p) ? 1 : 0); }

template <class R>
static void build_lpa(const Params &p, const Buffers &b, int lpa, int32_t cond, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>(p.ntot * KB / kBlock, 4096);
  const size_t lds = (size_t)(kBlock / KB) * (size_t)p.cap_slots * (size_t)lpa * sizeof(int);
  if (lds <= (size_t)kStageLdsMax) {
    switch (lpa) {
      case 1: hipLaunchKernelGGL((k_build_staged<R, 1>), dim3(g), dim3(kBlock), lds, s, p, b, cond); break;
      case 2: hipLaunchKernelGGL((k_build_staged<R, 2>), dim3(g), dim3(kBlock), lds, s, p, b, cond); break;
      case 4: hipLaunchKernelGGL((k_build_staged<R, 4>), dim3(g), dim3(kBlock), lds, s, p, b, cond); break;
      case 8: hipLaunchKernelGGL((k_build_staged<R, 8>), dim3(g), dim3(kBlock), lds, s, p, b, cond); break;
      default: hipLaunchKernelGGL((k_build_staged<R, 16>), dim3(g), dim3(kBlock), lds, s, p, b, cond); break;
    }
    return;
  }
  // lists too long to stage: the direct build
  switch (lpa) {
    case 1: hipLaunchKernelGGL((k_build<R, 1>), dim3(g), dim3(kBlock), 0, s, p, b, cond); break;
    case 2: hipLaunchKernelGGL((k_build<R, 2>), dim3(g), dim3(kBlock), 0, s, p, b, cond); break;
    case 4: hipLaunchKernelGGL((k_build<R, 4>), dim3(g), dim3(kBlock), 0, s, p, b, cond); break;
    case 8: hipLaunchKernelGGL((k_build<R, 8>), dim3(g), dim3(kBlock), 0, s, p, b, cond); break;
    default: hipLaunchKernelGGL((k_build<R, 16>), dim3(g), dim3(kBlock), 0, s, p, b, cond); break;
  }
}

void launch_build(const Params &p, const Buffers &b, int precision, int lpa, hipStream_t s, int32_t cond) {
  if (precision) build_lpa<float>(p, b, lpa, cond, s);
  else build_lpa<double>(p, b, lpa, cond, s);
}

void launch_density(const Params &p, const Buffers &b, int precision, int lpa, int32_t k, hipStream_t s,
                    bool prune) {
  prune = prune && p.inner;
  switch (pot_form(p) + 3 * (precision ? 1 : 0)) {
    case 0: density_form<double, 0>(p, b, lpa, k, s, prune); break;
    case 1: density_form<double, 1>(p, b, lpa, k, s, prune); break;
    case 2: density_form<double, 2>(p, b, lpa, k, s, prune); break;
    case 3: density_form<float, 0>(p, b, lpa, k, s, prune); break;
    case 4: density_form<float, 1>(p, b, lpa, k, s, prune); break;
    default: density_form<float, 2>(p, b, lpa, k, s, prune); break;
  }
}

void launch_force(const Params &p, const Buffers &b, int precision, int lpa, int32_t k, int32_t mode,
                  hipStream_t s) {
  switch (pot_form(p) + 3 * (precision ? 1 : 0)) {
    case 0: force_lpa<double, 0>(p, b, lpa, k, mode, s); break;
    case 1: force_lpa<double, 1>(p, b, lpa, k, mode, s); break;
    case 2: force_lpa<double, 2>(p, b, lpa, k, mode, s); break;
    case 3: force_lpa<float, 0>(p, b, lpa, k, mode, s); break;
    case 4: force_lpa<float, 1>(p, b, lpa, k, mode, s); break;
    default: force_lpa<float, 2>(p, b, lpa, k, mode, s); break;
  }
}

void launch_chunk_stats(const Params &p, const Buffers &b, hipStream_t s, int64_t n_stamps) {
  const int64_t rows = (int64_t)p.n_rep * kSlots;
  hipLaunchKernelGGL(k_stat_init, dim3((unsigned)std::min<int64_t>((rows * kStat + kBlock - 1) / kBlock, 1024)),
                     dim3(kBlock), 0, s, b.stat, rows, b.ktime, n_stamps, b.ctl);
  hipLaunchKernelGGL(k_chunk_stats, dim3(tiles(p)), dim3(kBlock), 0, s, p, b);
}

void launch_copy_back(const Params &p, const Buffers &b, const Buffers &scratch, int precision, hipStream_t s) {
  if (precision) hipLaunchKernelGGL(k_copy_back<float>, dim3(tiles(p)), dim3(kBlock), 0, s, b, scratch);
  else hipLaunchKernelGGL(k_copy_back<double>, dim3(tiles(p)), dim3(kBlock), 0, s, b, scratch);
}

void launch_assign_count(const Params &p, const Buffers &b, int32_t *key, hipStream_t s) {
  hipLaunchKernelGGL(k_assign_count, dim3(tiles(p)), dim3(kBlock), 0, s, p, b, key);
}

int scan_tiles(int64_t ncells) { return (int)((ncells + kScanTile - 1) / kScanTile); }

void launch_scan_cells(const Params &p, const Buffers &b, int32_t *cursor, int32_t *tsum, int32_t tmax,
                       hipStream_t s) {
  const dim3 grid((unsigned)tmax, (unsigned)p.n_rep);
  hipLaunchKernelGGL(k_scan_tiles, grid, dim3(kBlock), 0, s, b, tsum, tmax);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(p.n_rep), dim3(kBlock), 0, s, b, tsum, tmax);
  hipLaunchKernelGGL(k_scan_write, grid, dim3(kBlock), 0, s, b, tsum, tmax, cursor);
}

void launch_scatter(const Params &p, const Buffers &b, const int32_t *key, int32_t *cursor, int32_t *tmp,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(tiles(p)), dim3(kBlock), 0, s, b, key, cursor, tmp);
}

void launch_cell_sort(const Params &p, const Buffers &b, const int32_t *tmp, int32_t *perm, int64_t ncells_tot,
                      hipStream_t s) {
  const unsigned g = (unsigned)((ncells_tot + 3) / 4);
  hipLaunchKernelGGL(k_cell_sort, dim3(g), dim3(kBlock), 0, s, b, tmp, perm, ncells_tot);
}

void launch_permute(const Params &p, const Buffers &b, const Buffers &scratch, const int32_t *perm,
                         const int32_t *key, int precision, hipStream_t s) {
  if (precision) hipLaunchKernelGGL(k_permute<float>, dim3(tiles(p)), dim3(kBlock), 0, s, b, scratch, perm, key);
  else hipLaunchKernelGGL(k_permute<double>, dim3(tiles(p)), dim3(kBlock), 0, s, b, scratch, perm, key);
}

void launch_strain(const Params &p, const Buffers &b, const double *factor, hipStream_t s) {
  hipLaunchKernelGGL(k_strain, dim3(tiles(p)), dim3(kBlock), 0, s, p, b, factor);
}

void launch_count_pairs(const Params &p, const Buffers &b, int precision, hipStream_t s) {
  hipLaunchKernelGGL(k_count_pairs<double>, dim3(tiles(p)), dim3(kBlock), 0, s, p, b);
}

// ---------------------------------------------------------------------------
// device probes (achievable rates, for context next to the rooflines)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_probe_copy(const float4 *src, float4 *dst, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (int64_t)gridDim.x * kBlock)
    dst[t] = src[t];
}

// kProbeChains independent FMA chains per thread (one FMA per instruction:
// this code is built without packed FP32), their sum stored so that none
// is optimised away
constexpr int kProbeChains = 8;
template <class T>
__global__ __launch_bounds__(kBlock) void k_probe_fma(T *out, T mul, T add, int32_t iters) {
  T a[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) a[c] = (T)(threadIdx.x + c);
  for (int32_t it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) a[c] = fma(a[c], mul, add);
  T sum = (T)0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) sum += a[c];
  out[(size_t)blockIdx.x * kBlock + threadIdx.x] = sum;
}

void launch_probe_copy(const void *src, void *dst, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / (int64_t)sizeof(float4);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192));
  hipLaunchKernelGGL(k_probe_copy, dim3(g), dim3(kBlock), 0, s, static_cast<const float4 *>(src),
                     static_cast<float4 *>(dst), n);
}

double launch_probe_fma(void *out, int fp64, int32_t blocks, int32_t iters, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_probe_fma<double>, dim3(blocks), dim3(kBlock), 0, s, static_cast<double *>(out), 0.999999,
                       1e-7, iters);
  else
    hipLaunchKernelGGL(k_probe_fma<float>, dim3(blocks), dim3(kBlock), 0, s, static_cast<float *>(out), 0.999999f,
                       1e-7f, iters);
  return 2.0 * kProbeChains * (double)iters * (double)blocks * kBlock;  // flops
}

}  // namespace ptamd
