/*
 * FP64 CPU oracle: the plain definition of one PTA averaging burst of
 * Sutton-Chen EAM molecular dynamics.  TEST INFRASTRUCTURE ONLY (see
 * oracle.h): the product library never links or calls it.
 *
 * Paper passages followed (sections and equation labels of the paper):
 *   - Sec. 2.3 "Molecular Dynamics": Eq. (pe) total energy, the host density
 *     rho^alpha, Eq. (f=ma), Eq. (f_int) internal force, and the three
 *     velocity-Verlet updates Eqs. (vv_algo_pos_pred_half), (vv_algo_pos_pred),
 *     (vv_algo_vel_pred).
 *   - Sec. 2.4.1 "Problem Setup": FCC sample, axes along <100>, fixed
 *     boundary regions, Eq. (state).
 *   - Sec. 2.4.2 "Boundary conditions": lattice positions + Maxwell-Boltzmann
 *     velocities at T0; boundary atoms fixed by v = 0, F = 0; load applied as
 *     a displacement, then held.
 *   - Sec. 2.4.3 "State functions": Eq. (state_variables) K, U, reaction
 *     stress; Sec. 2.2 Step 1 Eq. (R_m_t) running time average over
 *     r = 1..N_t.
 *   - Table 1: lattice parameter a = 4.05 A, MD time step 1 fs.
 * Readings where the paper is silent (potential form, thermostat, strain
 * mode, slab thickness, RNG, constants, virial stress) are the documented
 * ones of the design notes; each is restated at the code that uses it.
 *
 * Parity pinned by tests/test_oracle_*.py (closed forms, lattice sums, finite
 * differences, symmetry, invariants, integrator properties, brute force).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* constants                                                            */
/* ------------------------------------------------------------------ */

/* Al atomic mass (IUPAC standard atomic weight 26.9815385 u). */
double orc_mass_al(void) { return 26.9815385; }
/* Boltzmann constant in eV/K (CODATA 2018, exact). */
double orc_kb(void) { return 8.617333262e-5; }
/* 1 amu*A^2/fs^2 in eV: u = 1.66053906660e-27 kg, A^2/fs^2 = 1e10 m^2/s^2,
 * e = 1.602176634e-19 J (exact). */
double orc_mvv2e(void) { return 1.66053906660e-27 * 1.0e10 / 1.602176634e-19; }
/* 1 eV/A^3 = 1.602176634e-19 J / 1e-30 m^3 = 160.2176634 GPa. */
double orc_ev_a3_to_gpa(void) { return 1.602176634e-19 / 1.0e-30 / 1.0e9; }

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* random numbers                                                       */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), in the form Vigna
 * published: state advances by the golden-ratio increment, then a
 * xor-shift-multiply finaliser.  The k-th output of the stream seeded with
 * `seed` only depends on seed + (k+1)*increment, so it is counter based. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Box-Muller (1958): two uniforms -> two independent standard normals.
 * u1 in (0,1] (so the log is finite), u2 in [0,1). */
void orc_gaussians(uint64_t seed, int64_t count, double *out) {
    const double two53inv = 1.0 / 9007199254740992.0; /* 2^-53 */
    const double twopi = 6.283185307179586;
    for (int64_t k = 0; 2 * k < count; ++k) {
        uint64_t a = orc_splitmix64(seed, (uint64_t)(2 * k));
        uint64_t b = orc_splitmix64(seed, (uint64_t)(2 * k + 1));
        double u1 = (double)((a >> 11) + 1u) * two53inv;
        double u2 = (double)(b >> 11) * two53inv;
        double rad = sqrt(-2.0 * log(u1));
        double th = twopi * u2;
        out[2 * k] = rad * cos(th);
        if (2 * k + 1 < count) out[2 * k + 1] = rad * sin(th);
    }
}

/* ------------------------------------------------------------------ */
/* lattice: Sec. 2.4.1 and 2.4.2                                        */
/* ------------------------------------------------------------------ */

int64_t orc_fcc_count(int32_t nc) { return 4 * (int64_t)nc * nc * nc; }

/* FCC cube of nc^3 conventional cells with axes along [100],[010],[001]
 * (Problem setup).  Atom positions are integer plane indices times a/2; the
 * four-atom basis is (0,0,0),(1,1,0),(1,0,1),(0,1,1) in those units.  Order:
 * cell x fastest, then y, then z; basis atom innermost.
 * Boundary regions (Problem setup defines them as one lattice parameter
 * thick at each loaded face): read here as the three atomic planes
 * pz in {0,1,2} (bottom) and {2nc-3, 2nc-2, 2nc-1} (top), by integer plane
 * index, with the load axis along z. */
void orc_fcc_cube(int32_t nc, double a, int32_t fix_slabs,
                  double *x, double *y, double *z, uint8_t *group, int32_t *pz) {
    static const int bx[4] = {0, 1, 1, 0};
    static const int by[4] = {0, 1, 0, 1};
    static const int bz[4] = {0, 0, 1, 1};
    const double half = 0.5 * a;
    int64_t i = 0;
    for (int32_t iz = 0; iz < nc; ++iz)
        for (int32_t iy = 0; iy < nc; ++iy)
            for (int32_t ix = 0; ix < nc; ++ix)
                for (int b = 0; b < 4; ++b, ++i) {
                    int px = 2 * ix + bx[b], py = 2 * iy + by[b], qz = 2 * iz + bz[b];
                    x[i] = (double)px * half;
                    y[i] = (double)py * half;
                    z[i] = (double)qz * half;
                    if (pz) pz[i] = qz;
                    uint8_t g = 0;
                    if (fix_slabs) {
                        if (qz <= 2) g = 1;
                        else if (qz >= 2 * nc - 3) g = 2;
                    }
                    if (group) group[i] = g;
                }
}

/* Maxwell-Boltzmann velocities at T0 (Boundary conditions).  Each Cartesian
 * component of a mobile atom is N(0, kB T0 / m); the normals are the
 * counter-based stream above, three per atom in atom order (fixed atoms
 * consume theirs too and get v = 0).  The mean velocity of the mobile atoms
 * is removed and the set rescaled so that 2K / ((3 N_mob - 3) kB) = T0. */
int32_t orc_mb_velocities(int64_t n, const uint8_t *group, double T0, uint64_t seed,
                          double *vx, double *vy, double *vz) {
    const double m = orc_mass_al(), kb = orc_kb(), c = orc_mvv2e();
    double *g = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    if (!g) return -1;
    orc_gaussians(seed, 3 * n, g);
    const double sv = sqrt(kb * T0 / (m * c));
    int64_t nmob = 0;
    double sx = 0, sy = 0, sz = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (group[i] == 0) {
            vx[i] = sv * g[3 * i];
            vy[i] = sv * g[3 * i + 1];
            vz[i] = sv * g[3 * i + 2];
            sx += vx[i]; sy += vy[i]; sz += vz[i];
            ++nmob;
        } else {
            vx[i] = vy[i] = vz[i] = 0.0;
        }
    }
    free(g);
    if (nmob < 2) return -1;
    sx /= (double)nmob; sy /= (double)nmob; sz /= (double)nmob;
    double mv2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (group[i] != 0) continue;
        vx[i] -= sx; vy[i] -= sy; vz[i] -= sz;
        mv2 += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    }
    const double K = 0.5 * m * mv2 * c;
    const double dof = 3.0 * (double)nmob - 3.0;
    const double T = 2.0 * K / (dof * kb);
    if (T0 > 0.0 && T > 0.0) {
        const double s = sqrt(T0 / T);
        for (int64_t i = 0; i < n; ++i) {
            if (group[i] != 0) continue;
            vx[i] *= s; vy[i] *= s; vz[i] *= s;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* potential: Eq. (pe) with Sutton-Chen functions                       */
/* ------------------------------------------------------------------ */

static double sc_V(const orc_sc *p, double r) { return p->eps * pow(p->a / r, p->n); }
static double sc_dV(const orc_sc *p, double r) { return -p->n * p->eps * pow(p->a / r, p->n) / r; }
static double sc_rho(const orc_sc *p, double r) { return pow(p->a / r, p->m); }
static double sc_drho(const orc_sc *p, double r) { return -p->m * pow(p->a / r, p->m) / r; }

/* Value and derivative of a tabulated piecewise cubic at x (knots k*h,
 * k < n); past the last knot the end value continues with the end slope. */
static void tab_eval(const double *c, int32_t n, double h, double x, double *f, double *df) {
    double kk = floor(x / h);
    if (kk < 0.0) kk = 0.0;
    int64_t k = (int64_t)kk;
    double u = x - (double)k * h, over = 0.0;
    if (k > n - 2) {
        k = n - 2;
        u = h;
        over = x - (double)(n - 1) * h;
    }
    const double *q = c + 4 * k;
    *df = (3.0 * q[0] * u + 2.0 * q[1]) * u + q[2];
    *f = ((q[0] * u + q[1]) * u + q[2]) * u + q[3] + over * *df;
}

/* V_s, dV_s/dr, rho_s, drho_s/dr at separation r.  Zero for r >= rc. */
void orc_pair_terms(const orc_sc *p, double r, double *V, double *dV, double *rho, double *drho) {
    if (!(r < p->rc)) { *V = *dV = *rho = *drho = 0.0; return; }
    if (p->tab) {
        const orc_tab *t = p->tab;
        double rp, drp;
        tab_eval(t->rho, t->nr, t->dr, r, rho, drho);
        tab_eval(t->rphi, t->nr, t->dr, r, &rp, &drp);
        *V = rp / r;                 /* phi = (r phi) / r */
        *dV = (drp - *V) / r;        /* phi' = ((r phi)' - phi) / r */
        return;
    }
    double v = sc_V(p, r), dv = sc_dV(p, r), q = sc_rho(p, r), dq = sc_drho(p, r);
    if (p->shift == 1) {
        v -= sc_V(p, p->rc);
        q -= sc_rho(p, p->rc);
    } else if (p->shift == 2) {
        const double dvc = sc_dV(p, p->rc), dqc = sc_drho(p, p->rc);
        v = v - sc_V(p, p->rc) - (r - p->rc) * dvc;
        q = q - sc_rho(p, p->rc) - (r - p->rc) * dqc;
        dv -= dvc;
        dq -= dqc;
    }
    *V = v; *dV = dv; *rho = q; *drho = dq;
}

/* B(rhobar) = -c eps sqrt(rhobar); B(0) = 0. */
double orc_embed(const orc_sc *p, double rhobar) {
    if (p->tab) {
        double f, df;
        tab_eval(p->tab->F, p->tab->nrho, p->tab->drho, rhobar, &f, &df);
        return f;
    }
    if (!(rhobar > 0.0)) return 0.0;
    return -p->c * p->eps * sqrt(rhobar);
}

/* dB/drhobar = -c eps / (2 sqrt(rhobar)); taken as 0 at rhobar = 0 (an
 * isolated atom feels no embedding force). */
double orc_embed_deriv(const orc_sc *p, double rhobar) {
    if (p->tab) {
        double f, df;
        tab_eval(p->tab->F, p->tab->nrho, p->tab->drho, rhobar, &f, &df);
        return df;
    }
    if (!(rhobar > 0.0)) return 0.0;
    return -p->c * p->eps / (2.0 * sqrt(rhobar));
}

/* ------------------------------------------------------------------ */
/* energy and forces: Eq. (pe), host density, Eq. (f_int)               */
/* ------------------------------------------------------------------ */

double orc_atom_density(int64_t n, const double *x, const double *y, const double *z,
                        const orc_sc *p, int64_t i) {
    const double rc2 = p->rc * p->rc;
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2) {
            double V, dV, q, dq;
            orc_pair_terms(p, sqrt(r2), &V, &dV, &q, &dq);
            s += q;
        }
    }
    return s;
}

void orc_density(int64_t n, const double *x, const double *y, const double *z,
                 const orc_sc *p, double *rhobar) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) rhobar[i] = orc_atom_density(n, x, y, z, p, i);
}

/* Force on atom i:  F_i = -dU/dr_i = sum_j g_ij (r_j - r_i)/r_ij with
 * g_ij = V_s'(r_ij) + (B'(rhobar_i) + B'(rhobar_j)) rho_s'(r_ij). */
void orc_forces(int64_t n, const double *x, const double *y, const double *z,
                const uint8_t *group, const orc_sc *p,
                double *fx, double *fy, double *fz, double *e,
                double *U, double *Wzz, double *Rz) {
    const double rc2 = p->rc * p->rc;
    double *rb = (double *)malloc(sizeof(double) * (size_t)n);
    double *bp = (double *)malloc(sizeof(double) * (size_t)n);
    double *ea = (double *)malloc(sizeof(double) * (size_t)n);
    double *wa = (double *)malloc(sizeof(double) * (size_t)n);
    orc_density(n, x, y, z, p, rb);
    for (int64_t i = 0; i < n; ++i) bp[i] = orc_embed_deriv(p, rb[i]);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double f0 = 0.0, f1 = 0.0, f2 = 0.0, ep = 0.0, w = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double V, dV, q, dq;
            orc_pair_terms(p, r, &V, &dV, &q, &dq);
            double g = dV + (bp[i] + bp[j]) * dq;
            f0 += g * dx / r;
            f1 += g * dy / r;
            f2 += g * dz / r;
            ep += 0.5 * V;
            /* pair virial: 1/2 (z_i - z_j) F_ij,z = -1/2 g dz^2 / r */
            w += -0.5 * g * dz * dz / r;
        }
        fx[i] = f0; fy[i] = f1; fz[i] = f2;
        ea[i] = ep + orc_embed(p, rb[i]);
        wa[i] = w;
    }
    double u = 0.0, wz = 0.0, rz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        u += ea[i];
        wz += wa[i];
        if (group && group[i] == 2) rz -= fz[i];
        if (e) e[i] = ea[i];
    }
    *U = u; *Wzz = wz; *Rz = rz;
    free(rb); free(bp); free(ea); free(wa);
}

void orc_atom_force(int64_t n, const double *x, const double *y, const double *z,
                    const orc_sc *p, int64_t i, double f[3]) {
    const double rc2 = p->rc * p->rc;
    const double bpi = orc_embed_deriv(p, orc_atom_density(n, x, y, z, p, i));
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < rc2)) continue;
        double r = sqrt(r2);
        double V, dV, q, dq;
        orc_pair_terms(p, r, &V, &dV, &q, &dq);
        double bpj = orc_embed_deriv(p, orc_atom_density(n, x, y, z, p, j));
        double g = dV + (bpi + bpj) * dq;
        f0 += g * dx / r;
        f1 += g * dy / r;
        f2 += g * dz / r;
    }
    f[0] = f0; f[1] = f1; f[2] = f2;
}

/* ------------------------------------------------------------------ */
/* neighbour sets and cells                                             */
/* ------------------------------------------------------------------ */

int64_t orc_neighbors(int64_t n, const double *x, const double *y, const double *z,
                      double rlist, int64_t *offsets, int32_t *idx, int64_t cap) {
    const double rl2 = rlist * rlist;
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rl2) ++c;
        }
        cnt[i] = c;
    }
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + cnt[i];
    const int64_t total = offsets[n];
    if (idx) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t k = offsets[i];
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rl2) {
                    if (k < cap) idx[k] = (int32_t)j;
                    ++k;
                }
            }
        }
    }
    free(cnt);
    return total;
}

static int32_t cell_coord(double v, double o, double inv_h, int32_t dim) {
    double t = floor((v - o) * inv_h);
    if (!(t >= 0.0)) return 0;
    if (t >= (double)dim) return dim - 1;
    return (int32_t)t;
}

void orc_cell_assign(int64_t n, const double *x, const double *y, const double *z,
                     const double origin[3], double inv_h, const int32_t dims[3], int32_t *cxyz) {
    for (int64_t i = 0; i < n; ++i) {
        cxyz[3 * i] = cell_coord(x[i], origin[0], inv_h, dims[0]);
        cxyz[3 * i + 1] = cell_coord(y[i], origin[1], inv_h, dims[1]);
        cxyz[3 * i + 2] = cell_coord(z[i], origin[2], inv_h, dims[2]);
    }
}

/* ------------------------------------------------------------------ */
/* dynamics: velocity Verlet + constraints + Berendsen + sampling       */
/* ------------------------------------------------------------------ */

double orc_volume(const orc_state *s) { return s->volume0 * (1.0 + s->strain); }

/* Affine load step along z about z = 0 (the loaded-face displacement of
 * Boundary conditions, applied to all atoms): engineering strain is
 * additive, eps_k = eps_{k-1} + d_eps, and every z is scaled by
 * (1 + eps_k)/(1 + eps_{k-1}).  Velocities are unchanged. */
void orc_apply_strain(orc_state *s, double d_eps) {
    const double e_new = s->strain + d_eps;
    const double f = (1.0 + e_new) / (1.0 + s->strain);
    for (int64_t i = 0; i < s->n; ++i) s->z[i] *= f;
    s->strain = e_new;
}

/* Which atoms the integrator moves: mobile atoms (group 0) along x, y and z;
 * during thermal relaxation (Sec. 2.4.2) the top-region atoms (group 2) move
 * along the load axis z only; every other fixed atom keeps v = 0, F = 0. */
static int moves_xyz(uint8_t g) { return g == 0; }
static int moves_z(uint8_t g, const orc_md *md) { return g == 0 || (g == 2 && md->top_free_z); }

/* m v^2 and m v_z^2 summed over the atoms that move, and the degrees of
 * freedom of the thermostat: 3 N_mob - 3, plus one per top atom free in z. */
static void kinetic_sums(const orc_state *s, const orc_md *md, double *dof, double *mv2, double *mvz2) {
    const double m = orc_mass_al();
    double a = 0.0, b = 0.0;
    int64_t c = 0, t = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        if (!moves_z(s->group[i], md)) continue;
        a += m * (s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i] + s->vz[i] * s->vz[i]);
        b += m * s->vz[i] * s->vz[i];
        if (moves_xyz(s->group[i])) ++c; else ++t;
    }
    *dof = 3.0 * (double)c - 3.0 + (double)t;
    *mv2 = a; *mvz2 = b;
}

/* sigma_zz = -(1/V) (sum_mob m v_z^2 + W_zz), tension positive. */
static double stress_zz(const orc_state *s, double mvz2, double Wzz) {
    return -(mvz2 * orc_mvv2e() + Wzz) / orc_volume(s) * orc_ev_a3_to_gpa();
}

void orc_observables(const orc_state *s, const orc_sc *p, double *K, double *U, double *szz, double *tz) {
    const int64_t n = s->n;
    double *f = (double *)malloc(sizeof(double) * (size_t)(3 * n));
    double u, w, rz;
    orc_forces(n, s->x, s->y, s->z, s->group, p, f, f + n, f + 2 * n, NULL, &u, &w, &rz);
    const orc_md fixed_top = {1.0, 1.0, 0.0, 0, 0};
    double dof, mv2, mvz2;
    kinetic_sums(s, &fixed_top, &dof, &mv2, &mvz2);
    *K = 0.5 * mv2 * orc_mvv2e();
    *U = u;
    *szz = stress_zz(s, mvz2, w);
    *tz = (s->area0 > 0.0) ? rz / s->area0 * orc_ev_a3_to_gpa() : 0.0;
    free(f);
}

/* Standard error of the mean of a series (column col, every stride-th
 * value, n values) from 20 batch means of n / 20 samples each (the samples
 * beyond 20 (n / 20) are not used): sqrt(sum_b (m_b - mbar)^2 / (20 * 19)). */
void orc_block_se(const double *col, int64_t stride, int64_t n, double *se) {
    const int64_t nb = 20;
    if (n < nb) { *se = NAN; return; }
    const int64_t bs = n / nb;
    double means[20], mu = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        double s = 0.0;
        for (int64_t k = 0; k < bs; ++k) s += col[(b * bs + k) * stride];
        means[b] = s / (double)bs;
        mu += means[b];
    }
    mu /= (double)nb;
    double v = 0.0;
    for (int64_t b = 0; b < nb; ++b) v += (means[b] - mu) * (means[b] - mu);
    *se = sqrt(v / (double)(nb * (nb - 1)));
}

int32_t orc_run_burst(orc_state *s, const orc_sc *p, const orc_md *md, int64_t n_steps,
                      orc_averages *avg, double *series, double *pos_sum) {
    const int64_t n = s->n;
    const double m = orc_mass_al(), kb = orc_kb(), c = orc_mvv2e();
    /* acceleration = F/m in A/fs^2 with F in eV/A: divide by m * c. */
    const double hdt_m = 0.5 * md->dt / (m * c);
    double *fx = (double *)malloc(sizeof(double) * (size_t)n);
    double *fy = (double *)malloc(sizeof(double) * (size_t)n);
    double *fz = (double *)malloc(sizeof(double) * (size_t)n);
    double *ser = series;
    double *own = NULL;
    if (!ser) { own = (double *)malloc(sizeof(double) * (size_t)(n_steps * ORC_SER_NCOL)); ser = own; }
    int32_t status = 0;
    double U, W, Rz;

    /* forces at the burst start are recomputed from the positions; the
     * components along which an atom is held are zeroed (F = 0 of the
     * fixed regions) */
    orc_forces(n, s->x, s->y, s->z, s->group, p, fx, fy, fz, NULL, &U, &W, &Rz);
    for (int64_t i = 0; i < n; ++i) {
        if (!moves_xyz(s->group[i])) fx[i] = fy[i] = 0.0;
        if (!moves_z(s->group[i], md)) fz[i] = 0.0;
    }
    if (pos_sum)
        for (int64_t i = 0; i < 3 * n; ++i) pos_sum[i] = 0.0;

    double sk = 0.0, su = 0.0, ss = 0.0, st = 0.0, stz = 0.0;
    for (int64_t r = 1; r <= n_steps; ++r) {
        /* Eq. (vv_algo_pos_pred_half) and Eq. (vv_algo_pos_pred); fixed atoms
         * have v = 0 and F = 0 and therefore do not move. */
        for (int64_t i = 0; i < n; ++i) {
            if (moves_xyz(s->group[i])) {
                s->vx[i] += hdt_m * fx[i];
                s->vy[i] += hdt_m * fy[i];
                s->vz[i] += hdt_m * fz[i];
                s->x[i] += md->dt * s->vx[i];
                s->y[i] += md->dt * s->vy[i];
                s->z[i] += md->dt * s->vz[i];
            } else if (moves_z(s->group[i], md)) {
                s->vz[i] += hdt_m * fz[i];
                s->z[i] += md->dt * s->vz[i];
            }
        }
        /* new internal forces, energy, virial and reaction at r(sigma+dsigma) */
        orc_forces(n, s->x, s->y, s->z, s->group, p, fx, fy, fz, NULL, &U, &W, &Rz);
        for (int64_t i = 0; i < n; ++i) {
            if (!moves_xyz(s->group[i])) fx[i] = fy[i] = 0.0;
            if (!moves_z(s->group[i], md)) fz[i] = 0.0;
        }
        /* Eq. (vv_algo_vel_pred) */
        for (int64_t i = 0; i < n; ++i) {
            if (!moves_z(s->group[i], md)) continue;
            s->vx[i] += hdt_m * fx[i];
            s->vy[i] += hdt_m * fy[i];
            s->vz[i] += hdt_m * fz[i];
        }
        double dof, mv2, mvz2;
        kinetic_sums(s, md, &dof, &mv2, &mvz2);
        double lam = 1.0;
        if (md->thermostat) {
            /* Berendsen: lambda^2 = 1 + (dt/tau)(T0/T - 1), applied to the
             * mobile atoms at the end of the step. */
            const double T = mv2 * c / (dof * kb);
            const double l2 = 1.0 + (md->dt / md->tau) * (md->T0 / T - 1.0);
            if (!(T > 0.0) || !(l2 >= 0.0)) { status = -7; break; }
            lam = sqrt(l2);
            for (int64_t i = 0; i < n; ++i) {
                if (!moves_z(s->group[i], md)) continue;
                s->vx[i] *= lam; s->vy[i] *= lam; s->vz[i] *= lam;
            }
            kinetic_sums(s, md, &dof, &mv2, &mvz2);
        }
        /* Eq. (mean_pos): positions of sample r enter the per-atom sums */
        if (pos_sum)
            for (int64_t i = 0; i < n; ++i) {
                pos_sum[i] += s->x[i];
                pos_sum[n + i] += s->y[i];
                pos_sum[2 * n + i] += s->z[i];
            }
        /* state functions of Eq. (state_variables) after the full step */
        const double K = 0.5 * mv2 * c;
        const double T = (dof > 0.0) ? mv2 * c / (dof * kb) : 0.0;
        const double szz = stress_zz(s, mvz2, W);
        const double tz = (s->area0 > 0.0) ? Rz / s->area0 * orc_ev_a3_to_gpa() : 0.0;
        double *row = ser + (r - 1) * ORC_SER_NCOL;
        row[ORC_SER_K] = K; row[ORC_SER_U] = U; row[ORC_SER_SZZ] = szz;
        row[ORC_SER_T] = T; row[ORC_SER_LAMBDA] = lam; row[ORC_SER_TZ] = tz;
        sk += K; su += U; ss += szz; st += T; stz += tz;
    }
    if (status == 0 && avg) {
        /* Eq. (R_m_t): mean over the samples r = 1..N_t */
        const double inv = 1.0 / (double)n_steps;
        avg->ke = sk * inv; avg->pe = su * inv; avg->szz = ss * inv;
        avg->tz = stz * inv; avg->temp = st * inv;
        avg->n_samples = n_steps;
        orc_block_se(ser + ORC_SER_K, ORC_SER_NCOL, n_steps, &avg->ke_se);
        orc_block_se(ser + ORC_SER_U, ORC_SER_NCOL, n_steps, &avg->pe_se);
        orc_block_se(ser + ORC_SER_SZZ, ORC_SER_NCOL, n_steps, &avg->szz_se);
    }
    free(fx); free(fy); free(fz); free(own);
    return status;
}
