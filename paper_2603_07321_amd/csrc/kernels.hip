// gfx950 kernels of the EAM molecular-dynamics burst.
//
// One MD step is three launches, captured in a HIP graph per chunk of steps:
//   kick_drift : Berendsen lambda of the previous step from the fixed-point
//                slot sums, v <- lambda v + dt/(2m) F, x <- x + dt v
//                (Eqs. (vv_algo_pos_pred_half), (vv_algo_pos_pred)); records
//                the previous step's sample (Eq. (R_m_t)).
//   density    : rebuilds the Verlet lists when flagged, then the host
//                density rhobar_i and B'(rhobar_i) of Eq. (pe).
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

__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return rsqrt(x); }

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

__device__ __forceinline__ unsigned long long *slot_row(const Buffers &b, int n_rep, int par, int r, int slot) {
  return b.slots + (((size_t)par * n_rep + r) * kSlots + slot) * kNQ;
}

__device__ __forceinline__ void set_err(const Buffers &b, int bits) { atomicOr(&b.ctl->err, bits); }

// ---------------------------------------------------------------------------
// burst start: zero accumulators, slots and errors
// ---------------------------------------------------------------------------
__global__ void k_burst_begin(Buffers b, int n_rep) {
  const size_t nslot = (size_t)2 * n_rep * kSlots * kNQ;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t t = t0; t < nslot; t += (size_t)gridDim.x * blockDim.x) b.slots[t] = 0ull;
  const size_t nacc = (size_t)n_rep * (sizeof(RepAcc) / sizeof(double));
  double *acc = reinterpret_cast<double *>(b.acc);
  for (size_t t = t0; t < nacc; t += (size_t)gridDim.x * blockDim.x) acc[t] = 0.0;
  if (t0 == 0) b.ctl->err = 0;
}

__global__ void k_set_base(Control *ctl, int64_t base) { ctl->base = base; }

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// ---------------------------------------------------------------------------
// sampling of one completed step (thread 0 of the first block of a replica)
// ---------------------------------------------------------------------------
__device__ void record_sample(const Params &p, const Buffers &b, int r, int64_t s, const double *q, double lam) {
  const RepInfo &rp = b.rep[r];
  RepAcc &A = b.acc[r];
  const double l2 = lam * lam;
  const double mv2 = q[Q_MV2], mvz2 = q[Q_MVZ2];
  const double K = 0.5 * l2 * mv2;
  const double T = (rp.dof > 0.0) ? l2 * mv2 / (rp.dof * p.kb) : 0.0;
  const double U = q[Q_EPAIR] + q[Q_EMB];
  const double V = rp.volume0 * (1.0 + rp.strain);
  const double szz = -(l2 * mvz2 + q[Q_WZZ]) / V * p.gpa;
  const double tz = (rp.area0 > 0.0) ? q[Q_RZ] / rp.area0 * p.gpa : 0.0;
  A.sum[0] += K;
  A.sum[1] += U;
  A.sum[2] += szz;
  A.sum[3] += T;
  A.sum[4] += lam;
  A.sum[5] += tz;
  const int64_t bs = b.ctl->se_block;
  if (bs > 0) {
    const int64_t bi = (s - 1) / bs;
    if (bi < kSEBlocks) {
      A.blk[bi][0] += K;
      A.blk[bi][1] += U;
      A.blk[bi][2] += szz;
    }
  }
  if (s - 1 < b.series_cap) {
    double *row = b.series + ((size_t)r * b.series_cap + (s - 1)) * kSeriesCols;
    row[0] = K; row[1] = U; row[2] = szz; row[3] = T; row[4] = lam; row[5] = tz;
  }
  A.nsamp += 1;
  A.lam_last = lam;
  if (!isfinite(K) || !isfinite(U) || !isfinite(szz)) set_err(b, E_NONFINITE);
}

__device__ void write_averages(const Buffers &b, int r) {
  RepAcc &A = b.acc[r];
  const double n = (double)A.nsamp;
  A.out[0] = A.sum[0] / n;
  A.out[1] = A.sum[1] / n;
  A.out[2] = A.sum[2] / n;
  A.out[3] = A.sum[5] / n;
  const int64_t bs = b.ctl->se_block;
  for (int q = 0; q < 3; ++q) {
    double se = NAN;
    if (bs > 0) {
      double mu = 0.0, m[kSEBlocks];
      for (int k = 0; k < kSEBlocks; ++k) {
        m[k] = A.blk[k][q] / (double)bs;
        mu += m[k];
      }
      mu /= (double)kSEBlocks;
      double v = 0.0;
      for (int k = 0; k < kSEBlocks; ++k) v += (m[k] - mu) * (m[k] - mu);
      se = sqrt(v / (double)(kSEBlocks * (kSEBlocks - 1)));
    }
    A.out[4 + q] = se;
  }
  A.out[7] = A.sum[3] / n;
  A.out[8] = b.rep[r].strain;
  A.out[9] = n;
}

// ---------------------------------------------------------------------------
// kick-drift (mode 0) / finalize (mode 1)
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(kBlock) void k_kick_drift(Params p, Buffers b, int32_t k, int32_t mode) {
  using V4 = typename V4T<R>::T;
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t step = b.ctl->base + k;  // mode 0: step being computed; mode 1: n_steps + 1
  __shared__ double s_lam;
  if (threadIdx.x < 64) {
    long long q[6] = {0, 0, 0, 0, 0, 0};
    if (step > 1) {
      const unsigned long long *row = slot_row(b, p.n_rep, (int)((step - 1) & 1), r, threadIdx.x);
#pragma unroll
      for (int t = 0; t < 6; ++t) q[t] = (long long)row[t];
#pragma unroll
      for (int t = 0; t < 6; ++t)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) q[t] += shfl_xor_ll(q[t], o);
    }
    if (threadIdx.x == 0) {
      double lam = 1.0;
      if (step > 1) {
        double qd[6];
        for (int t = 0; t < 6; ++t) qd[t] = (double)q[t] / kFix;
        const RepInfo &rp = b.rep[r];
        if (p.thermostat) {
          const double T = qd[Q_MV2] / (rp.dof * p.kb);
          const double l2 = 1.0 + (p.dt / p.tau) * (rp.T0 / T - 1.0);
          if (!(T > 0.0) || !(l2 >= 0.0)) {
            if (tile == rp.abeg / kTile) set_err(b, E_STATE);
          } else {
            lam = sqrt(l2);
          }
        }
        if (tile == rp.abeg / kTile) {
          record_sample(p, b, r, step - 1, qd, lam);
          if (mode == 1) write_averages(b, r);
        }
      }
      s_lam = lam;
    }
  }
  __syncthreads();
  const double lam = s_lam;
  const int64_t i = tile * kTile + threadIdx.x;
  if (b.group[i] != 0) return;  // fixed or padding atom: v = 0, never moves
  double vx = b.vx[i] * lam, vy = b.vy[i] * lam, vz = b.vz[i] * lam;
  if (mode == 0) {
    vx += p.hdt_m * b.fx[i];
    vy += p.hdt_m * b.fy[i];
    vz += p.hdt_m * b.fz[i];
    const double x = b.x[i] + p.dt * vx;
    const double y = b.y[i] + p.dt * vy;
    const double z = b.z[i] + p.dt * vz;
    b.x[i] = x;
    b.y[i] = y;
    b.z[i] = z;
    // gather copy for the pair kernels; w (B') is rewritten by the density pass
    V4 v4;
    v4.x = (R)x;
    v4.y = (R)y;
    v4.z = (R)z;
    v4.w = (R)0;
    reinterpret_cast<V4 *>(b.pos4)[i] = v4;
    const RepInfo &rp = b.rep[r];
    const double cx = x - rp.center[0], cy = y - rp.center[1], cz = z - rp.center[2];
    if (!(cx * cx + cy * cy + cz * cz <= p.esc2)) set_err(b, isfinite(x + y + z) ? E_ESCAPE : E_NONFINITE);
    const double ex = x - (double)b.xr[i], ey = y - (double)b.yr[i], ez = z - (double)b.zr[i];
    if (ex * ex + ey * ey + ez * ez > p.half_skin2) b.ctl->rebuild = 1;
  }
  b.vx[i] = vx;
  b.vy[i] = vy;
  b.vz[i] = vz;
}

// gather copy of positions (x, y, z, keep w) for the pair kernels
template <class R>
__global__ __launch_bounds__(kBlock) void k_pos4(Buffers b) {
  using V4 = typename V4T<R>::T;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b.group[i] == kPad) return;
  V4 *p4 = reinterpret_cast<V4 *>(b.pos4);
  V4 v = p4[i];
  v.x = (R)b.x[i];
  v.y = (R)b.y[i];
  v.z = (R)b.z[i];
  p4[i] = v;
}

// ---------------------------------------------------------------------------
// density pass (+ Verlet-list rebuild when flagged)
// ---------------------------------------------------------------------------
template <int LPA>
__device__ void build_list(const Params &p, const Buffers &b, int64_t i, int lane, int r) {
  const RepInfo &rp = b.rep[r];
  const double xi = b.x[i], yi = b.y[i], zi = b.z[i];
  {
    const double ex = xi - (double)b.xs[i], ey = yi - (double)b.ys[i], ez = zi - (double)b.zs[i];
    if (lane == 0 && ex * ex + ey * ey + ez * ez > p.margin2) set_err(b, E_DRIFT);
  }
  const int dxn = rp.dims[0], dyn = rp.dims[1], dzn = rp.dims[2];
  const int cl = b.cell[i];
  const int cx = cl % dxn, cy = (cl / dxn) % dyn, cz = cl / (dxn * dyn);
  const int gbase = (threadIdx.x & 63) & ~(LPA - 1);
  const unsigned long long gmask = (LPA == 64) ? ~0ull : ((1ull << LPA) - 1ull);
  const unsigned long long below = (1ull << lane) - 1ull;
  int cnt = 0;
  const int cap = p.cap_slots * LPA;
  for (int oz = -1; oz <= 1; ++oz) {
    const int nz = cz + oz;
    if (nz < 0 || nz >= dzn) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      const int ny = cy + oy;
      if (ny < 0 || ny >= dyn) continue;
      for (int ox = -1; ox <= 1; ++ox) {
        const int nx = cx + ox;
        if (nx < 0 || nx >= dxn) continue;
        const int64_t c = rp.cell_off + ((int64_t)nz * dyn + ny) * dxn + nx;
        const int start = b.cell_start[c], count = b.cell_count[c];
        for (int t = 0; t < count; t += LPA) {
          const int jj = t + lane;
          bool ok = false;
          int j = 0;
          if (jj < count) {
            j = start + jj;
            if ((int64_t)j != i) {
              const double d2 = dist2_plain(sub_plain(b.x[j], xi), sub_plain(b.y[j], yi), sub_plain(b.z[j], zi));
              ok = d2 < p.rlist2;
            }
          }
          int pos, add;
          if (LPA == 1) {
            pos = cnt;
            add = ok ? 1 : 0;
          } else {
            const unsigned long long m = (__ballot(ok) >> gbase) & gmask;
            pos = cnt + __popcll(m & below);
            add = __popcll(m);
          }
          if (ok && pos < cap) b.nbr[(size_t)(pos / LPA) * p.nbr_stride + (size_t)i * LPA + (pos % LPA)] = j;
          cnt += add;
        }
      }
    }
  }
  if (lane == 0) {
    if (cnt > cap) {
      set_err(b, E_OVERFLOW);
      cnt = cap;
    }
    b.ncount[i] = cnt;
    b.xr[i] = (float)xi;
    b.yr[i] = (float)yi;
    b.zr[i] = (float)zi;
  }
}

template <class R, int LPA>
__global__ __launch_bounds__(kBlock) void k_density(Params p, Buffers b, int32_t k) {
  using V4 = typename V4T<R>::T;
  const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = gt / LPA;
  const int lane = (int)(gt & (LPA - 1));
  const int64_t tile = ((int64_t)blockIdx.x * (kBlock / LPA)) / kTile;
  const int r = b.blk_rep[tile];
  const int64_t step = b.ctl->base + k;
  const int par = (int)(step & 1);
  const bool rebuild = b.ctl->rebuild != 0;
  {
    // the slots of the other parity were consumed by this step's kick-drift
    const size_t nz = (size_t)p.n_rep * kSlots * kNQ;
    unsigned long long *zp = b.slots + (size_t)(par ^ 1) * nz;
    for (size_t t = (size_t)gt; t < nz; t += (size_t)gridDim.x * kBlock) zp[t] = 0ull;
  }
  const uint8_t g = b.group[i];
  const bool real = g != kPad;
  if (rebuild && real) build_list<LPA>(p, b, i, lane, r);
  const V4 *p4 = reinterpret_cast<const V4 *>(b.pos4);
  R acc = (R)0;
  if (real) {
    const V4 pi = p4[i];
    const R rc2 = (R)p.rc2, a = (R)p.a, rc = (R)p.rc, rhoc = (R)p.rhoc, drhoc = (R)p.drhoc;
    const int cnt = b.ncount[i];
    const int32_t *nb = b.nbr + (size_t)i * LPA + lane;
    for (int e = lane, s = 0; e < cnt; e += LPA, ++s) {
      const int j = nb[(size_t)s * p.nbr_stride];
      const V4 pj = p4[j];
      const R dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
      const R r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2) {
        const R rinv = rsqrt_r(r2);
        const R rr = r2 * rinv;
        const R rho = ipow<R>(a * rinv, p.m);
        acc += rho - rhoc - (rr - rc) * drhoc;
      }
    }
  }
#pragma unroll
  for (int o = LPA / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  long long q[1] = {0};
  if (lane == 0 && real) {
    const double rb = (double)acc;
    double Bp = 0.0, B = 0.0;
    if (rb > 0.0) {
      const double sq = sqrt(rb);
      B = -p.c_eps * sq;
      Bp = -0.5 * p.c_eps / sq;
    }
    reinterpret_cast<R *>(b.pos4)[4 * i + 3] = (R)Bp;
    q[0] = to_fix(B);
  }
  block_slot_add<1>(q, slot_row(b, p.n_rep, par, r, blockIdx.x & (kSlots - 1)) + Q_EMB);
}

// ---------------------------------------------------------------------------
// force pass: mode 0 = step (second half kick + sums), 1 = forces only
// ---------------------------------------------------------------------------
template <class R, int LPA>
__global__ __launch_bounds__(kBlock) void k_force(Params p, Buffers b, int32_t k, int32_t mode) {
  using V4 = typename V4T<R>::T;
  const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = gt / LPA;
  const int lane = (int)(gt & (LPA - 1));
  const int64_t tile = ((int64_t)blockIdx.x * (kBlock / LPA)) / kTile;
  const int r = b.blk_rep[tile];
  const int64_t step = b.ctl->base + k;
  const int par = (int)(step & 1);
  const uint8_t g = b.group[i];
  const bool real = g != kPad;
  const V4 *p4 = reinterpret_cast<const V4 *>(b.pos4);
  R fx = 0, fy = 0, fz = 0, ep = 0, w = 0;
  int npair = 0;
  if (real) {
    const V4 pi = p4[i];
    const R rc2 = (R)p.rc2, a = (R)p.a, rc = (R)p.rc, eps = (R)p.eps;
    const R nn = (R)p.n, mm = (R)p.m;
    const R Vc = (R)p.Vc, dVc = (R)p.dVc, drhoc = (R)p.drhoc;
    const int cnt = b.ncount[i];
    const int32_t *nb = b.nbr + (size_t)i * LPA + lane;
    for (int e = lane, s = 0; e < cnt; e += LPA, ++s) {
      const int j = nb[(size_t)s * p.nbr_stride];
      const V4 pj = p4[j];
      const R dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
      const R r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2) {
        const R rinv = rsqrt_r(r2);
        const R rr = r2 * rinv;
        const R t = a * rinv;
        const R V = eps * ipow<R>(t, p.n);
        const R rho = ipow<R>(t, p.m);
        const R dV = -nn * V * rinv;
        const R drho = -mm * rho * rinv;
        const R Vs = V - Vc - (rr - rc) * dVc;
        const R gg = (dV - dVc) + (pi.w + pj.w) * (drho - drhoc);
        const R f = gg * rinv;
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
        ep += Vs;
        w += f * dz * dz;
        ++npair;
      }
    }
  }
#pragma unroll
  for (int o = LPA / 2; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o);
    fy += __shfl_xor(fy, o);
    fz += __shfl_xor(fz, o);
    ep += __shfl_xor(ep, o);
    w += __shfl_xor(w, o);
    npair += __shfl_xor(npair, o);
  }
  long long q[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (lane == 0 && real) {
    const double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
    b.fx[i] = Fx;
    b.fy[i] = Fy;
    b.fz[i] = Fz;
    if (!isfinite(Fx + Fy + Fz)) set_err(b, E_NONFINITE);
    if (g == 0) {
      double vx = b.vx[i], vy = b.vy[i], vz = b.vz[i];
      if (mode == 0) {
        vx += p.hdt_m * Fx;
        vy += p.hdt_m * Fy;
        vz += p.hdt_m * Fz;
        b.vx[i] = vx;
        b.vy[i] = vy;
        b.vz[i] = vz;
      }
      q[Q_MV2] = to_fix(p.mvv2e_m * (vx * vx + vy * vy + vz * vz));
      q[Q_MVZ2] = to_fix(p.mvv2e_m * vz * vz);
    }
    q[Q_EPAIR] = to_fix(0.5 * (double)ep);
    q[Q_WZZ] = to_fix(-0.5 * (double)w);
    if (g == 2) q[Q_RZ] = to_fix(-Fz);
    q[Q_PAIRS] = npair;
  }
  block_slot_add<kNQ>(q, slot_row(b, p.n_rep, par, r, blockIdx.x & (kSlots - 1)));
  if (gt == 0 && b.ctl->rebuild) {
    b.ctl->list_builds += 1;
    b.ctl->rebuild = 0;
  }
}

// ---------------------------------------------------------------------------
// chunk statistics: max drift since the last sort and max speed, per replica
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

__global__ __launch_bounds__(kBlock) void k_chunk_stats(Params p, Buffers b) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  double d2 = 0.0, v2 = 0.0;
  if (b.group[i] == 0) {
    const double ex = b.x[i] - (double)b.xs[i], ey = b.y[i] - (double)b.ys[i], ez = b.z[i] - (double)b.zs[i];
    d2 = ex * ex + ey * ey + ez * ez;
    v2 = b.vx[i] * b.vx[i] + b.vy[i] * b.vy[i] + b.vz[i] * b.vz[i];
    if (!isfinite(d2 + v2)) {
      set_err(b, E_NONFINITE);
      d2 = v2 = 0.0;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 = fmax(d2, __shfl_xor(d2, o));
    v2 = fmax(v2, __shfl_xor(v2, o));
  }
  __shared__ double sh[kBlock / 64][2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid][0] = d2;
    sh[wid][1] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double m = 0.0;
    for (int w2 = 0; w2 < kBlock / 64; ++w2) m = fmax(m, sh[w2][threadIdx.x]);
    atomicMax(b.stat + ((size_t)r * kSlots + (blockIdx.x & (kSlots - 1))) * 4 + threadIdx.x, dbits(m));
  }
}

// ---------------------------------------------------------------------------
// spatial sort
// ---------------------------------------------------------------------------
// order-preserving map of a double onto uint64 (for min/max atomics)
__device__ __forceinline__ unsigned long long okey(double v) {
  unsigned long long u = dbits(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(kBlock) void k_bbox(Params p, Buffers b) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
  if (b.group[i] != kPad) {
    const double c[3] = {b.x[i], b.y[i], b.z[i]};
    for (int d = 0; d < 3; ++d) {
      mn[d] = okey(c[d]);
      mx[d] = mn[d];
    }
  }
  __shared__ unsigned long long sh[kBlock / 64][6];
  for (int d = 0; d < 3; ++d)
    for (int o = 32; o > 0; o >>= 1) {
      const long long a = shfl_xor_ll((long long)mn[d], o), c2 = shfl_xor_ll((long long)mx[d], o);
      mn[d] = min(mn[d], (unsigned long long)a);
      mx[d] = max(mx[d], (unsigned long long)c2);
    }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      sh[wid][d] = mn[d];
      sh[wid][3 + d] = mx[d];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    unsigned long long v = sh[0][d];
    for (int w2 = 1; w2 < kBlock / 64; ++w2) v = (d < 3) ? min(v, sh[w2][d]) : max(v, sh[w2][d]);
    unsigned long long *dst = b.stat + ((size_t)r * kSlots + (blockIdx.x & (kSlots - 1))) * 8 + d;
    if (d < 3) atomicMin(dst, v);
    else atomicMax(dst, v);
  }
}

__device__ __forceinline__ int cell_coord(double v, double o, double inv_h, int dim) {
  const double t = floor(sub_plain(v, o) * inv_h);
  if (!(t >= 0.0)) return 0;
  if (t >= (double)dim) return dim - 1;
  return (int)t;
}

__global__ __launch_bounds__(kBlock) void k_assign_count(Params p, Buffers b, int32_t *key) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  const RepInfo &rp = b.rep[r];
  int c;
  if (b.group[i] == kPad) {
    c = (int)(rp.ncells - 1);  // virtual last cell: padding sorts to the end
  } else {
    const int cx = cell_coord(b.x[i], rp.origin[0], rp.inv_h, rp.dims[0]);
    const int cy = cell_coord(b.y[i], rp.origin[1], rp.inv_h, rp.dims[1]);
    const int cz = cell_coord(b.z[i], rp.origin[2], rp.inv_h, rp.dims[2]);
    c = (cz * rp.dims[1] + cy) * rp.dims[0] + cx;
  }
  key[i] = c;
  atomicAdd(b.cell_count + rp.cell_off + c, 1);
}

// exclusive scan of one replica's cell counts (one block per replica)
__global__ __launch_bounds__(1024) void k_scan_cells(Params p, Buffers b, int32_t *cursor) {
  const int r = blockIdx.x;
  const RepInfo &rp = b.rep[r];
  const int64_t nc = rp.ncells;
  const int32_t *cnt = b.cell_count + rp.cell_off;
  int32_t *st = b.cell_start + rp.cell_off;
  int32_t *cur = cursor + rp.cell_off;
  __shared__ int64_t part[1024];
  const int64_t per = (nc + 1023) / 1024;
  const int64_t lo = threadIdx.x * per, hi = min(nc, lo + per);
  int64_t s = 0;
  for (int64_t c = lo; c < hi; ++c) s += cnt[c];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < 1024; ++t) {
      const int64_t v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = rp.abeg + part[threadIdx.x];
  for (int64_t c = lo; c < hi; ++c) {
    st[c] = (int32_t)run;
    cur[c] = (int32_t)run;
    run += cnt[c];
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(Buffers b, const int32_t *key, int32_t *cursor, int32_t *tmp) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  const int pos = atomicAdd(cursor + b.rep[r].cell_off + key[i], 1);
  tmp[pos] = (int32_t)i;
}

// Within each cell, order atoms by original index (padding atoms after, by
// position): a rank sort over unique keys.  The sorted order then depends on
// the positions only, not on the previous order nor on the order of atomics.
__device__ __forceinline__ long long sort_key(const Buffers &b, int v) {
  const int o = b.orig[v];
  return (o >= 0) ? (long long)o : ((1ll << 32) + (long long)v);
}

__global__ __launch_bounds__(kBlock) void k_cell_sort(Buffers b, const int32_t *tmp, int32_t *perm, int64_t ncells_tot) {
  const int64_t c = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (c >= ncells_tot) return;
  const int lane = threadIdx.x & 63;
  const int start = b.cell_start[c], cnt = b.cell_count[c];
  for (int a = lane; a < cnt; a += 64) {
    const int v = tmp[start + a];
    const long long kv = sort_key(b, v);
    int rank = 0;
    for (int q = 0; q < cnt; ++q) rank += (sort_key(b, tmp[start + q]) < kv) ? 1 : 0;
    perm[start + rank] = v;
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
  sc.xs[i] = (float)x;
  sc.ys[i] = (float)y;
  sc.zs[i] = (float)z;
  V4 v;
  v.x = (R)x;
  v.y = (R)y;
  v.z = (R)z;
  v.w = (R)0;
  reinterpret_cast<V4 *>(sc.pos4)[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_strain(Params p, Buffers b, const double *factor) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  if (b.group[i] == kPad) return;
  b.z[i] = b.z[i] * factor[r];
}

// pairs within rc (directed) and list entries, summed into stat[r][slot][0..1]
template <class R>
__global__ __launch_bounds__(kBlock) void k_count_pairs(Params p, Buffers b) {
  const int64_t tile = blockIdx.x;
  const int r = b.blk_rep[tile];
  const int64_t i = tile * kTile + threadIdx.x;
  unsigned long long np = 0, ne = 0;
  if (b.group[i] != kPad) {
    const int cnt = b.ncount[i];
    ne = cnt;
    for (int e = 0; e < cnt; ++e) {
      const int j = b.nbr[(size_t)(e / p.lpa) * p.nbr_stride + (size_t)i * p.lpa + (e % p.lpa)];
      const double d2 = dist2_plain(b.x[j] - b.x[i], b.y[j] - b.y[i], b.z[j] - b.z[i]);
      if (d2 < p.rc2) ++np;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    np += (unsigned long long)shfl_xor_ll((long long)np, o);
    ne += (unsigned long long)shfl_xor_ll((long long)ne, o);
  }
  if ((threadIdx.x & 63) == 0) {
    unsigned long long *row = b.stat + ((size_t)r * kSlots + (blockIdx.x & (kSlots - 1))) * 4;
    atomicAdd(row, np);
    atomicAdd(row + 1, ne);
  }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned tiles(const Params &p) { return (unsigned)(p.ntot / kTile); }

void launch_burst_begin(const Params &p, const Buffers &b, int n_rep, hipStream_t s) {
  hipLaunchKernelGGL(k_burst_begin, dim3(64), dim3(kBlock), 0, s, b, n_rep);
}

void launch_set_base(const Buffers &b, int64_t base, hipStream_t s) {
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(1), 0, s, b.ctl, base);
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
  if (precision) hipLaunchKernelGGL(k_pos4<float>, dim3(tiles(p)), dim3(kBlock), 0, s, b);
  else hipLaunchKernelGGL(k_pos4<double>, dim3(tiles(p)), dim3(kBlock), 0, s, b);
}

template <class R>
static void density_lpa(const Params &p, const Buffers &b, int lpa, int32_t k, hipStream_t s) {
  const unsigned g = (unsigned)(p.ntot * lpa / kBlock);
  switch (lpa) {
    case 1: hipLaunchKernelGGL((k_density<R, 1>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    case 2: hipLaunchKernelGGL((k_density<R, 2>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    case 4: hipLaunchKernelGGL((k_density<R, 4>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    case 8: hipLaunchKernelGGL((k_density<R, 8>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
    default: hipLaunchKernelGGL((k_density<R, 16>), dim3(g), dim3(kBlock), 0, s, p, b, k); break;
  }
}

template <class R>
static void force_lpa(const Params &p, const Buffers &b, int lpa, int32_t k, int32_t mode, hipStream_t s) {
  const unsigned g = (unsigned)(p.ntot * lpa / kBlock);
  switch (lpa) {
    case 1: hipLaunchKernelGGL((k_force<R, 1>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    case 2: hipLaunchKernelGGL((k_force<R, 2>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    case 4: hipLaunchKernelGGL((k_force<R, 4>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    case 8: hipLaunchKernelGGL((k_force<R, 8>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
    default: hipLaunchKernelGGL((k_force<R, 16>), dim3(g), dim3(kBlock), 0, s, p, b, k, mode); break;
  }
}

void launch_density(const Params &p, const Buffers &b, int precision, int lpa, int32_t k, hipStream_t s) {
  if (precision) density_lpa<float>(p, b, lpa, k, s);
  else density_lpa<double>(p, b, lpa, k, s);
}

void launch_force(const Params &p, const Buffers &b, int precision, int lpa, int32_t k, int32_t mode,
                  hipStream_t s) {
  if (precision) force_lpa<float>(p, b, lpa, k, mode, s);
  else force_lpa<double>(p, b, lpa, k, mode, s);
}

void launch_chunk_stats(const Params &p, const Buffers &b, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_stats, dim3(tiles(p)), dim3(kBlock), 0, s, p, b);
}

void launch_bbox(const Params &p, const Buffers &b, hipStream_t s) {
  hipLaunchKernelGGL(k_bbox, dim3(tiles(p)), dim3(kBlock), 0, s, p, b);
}

void launch_assign_count(const Params &p, const Buffers &b, int32_t *key, hipStream_t s) {
  hipLaunchKernelGGL(k_assign_count, dim3(tiles(p)), dim3(kBlock), 0, s, p, b, key);
}

void launch_scan_cells(const Params &p, const Buffers &b, int32_t *cursor, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_cells, dim3(p.n_rep), dim3(1024), 0, s, p, b, cursor);
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

}  // namespace ptamd
