/*
 * FP64 CPU oracle for the EAM molecular-dynamics burst that Practical Time
 * Averaging (PTA) runs and averages (Baruah, Chatterjee, Acharya, Wang,
 * "Averaging Molecular Dynamics simulations to study the slow-strain-rate
 * behavior of metals").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no source, header, table or constant
 * with the GPU library: every definition below is written out here again from
 * the paper (and, where the paper is silent, from the documented reading).
 *
 * Plain, slow, obviously correct: all-pairs O(N^2) loops in original atom
 * order, full (both-direction) pair sums, every list rebuilt on every call,
 * FP64 throughout, compiled without floating-point contraction.
 *
 * Units: Angstrom, eV, fs, amu, K; stresses in GPa.
 */
#ifndef PTAMD_ORACLE_H
#define PTAMD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sutton-Chen form of the EAM energy of Eq. (pe):
 *   V(r) = eps (a/r)^n,  rho(r) = (a/r)^m,  B(rhobar) = -c eps sqrt(rhobar).
 * shift: 0 = truncated at rc, 1 = energy-shifted, 2 = shifted-force
 * (value and slope of V and rho both vanish at rc). */
/* Tabulated single-element EAM functions, the layout of a setfl file:
 * F(rhobar) on knots k*drho (k < nrho), rho(r) and r*phi(r) on knots k*dr
 * (k < nr).  Each is the piecewise cubic given by its coefficients per
 * interval k, highest power first, in u = x - x_k:
 *   f(x) = ((c[4k] u + c[4k+1]) u + c[4k+2]) u + c[4k+3].
 * Past the last knot F continues linearly with its end slope. */
typedef struct {
    int32_t nrho, nr;
    double drho, dr;
    const double *F;     /* 4*(nrho-1) */
    const double *rho;   /* 4*(nr-1) */
    const double *rphi;  /* 4*(nr-1) */
} orc_tab;

/* With tab != NULL the functions of Eq. (pe) are the tables instead:
 * V(r) = (r phi)(r) / r, rho(r), B = F; rc still bounds the pair sums and
 * shift is ignored. */
typedef struct {
    double eps, a, n, m, c, rc;
    int32_t shift;
    const orc_tab *tab;
} orc_sc;

typedef struct {
    double dt;        /* fs, the MD time step (Table 1: 1 fs) */
    double tau;       /* fs, Berendsen coupling time */
    double T0;        /* K, thermostat target */
    int32_t thermostat; /* 0 = NVE, 1 = Berendsen */
    int32_t top_free_z; /* 1: atoms of the top region (group 2) move along z only
                           (thermal relaxation, Sec. 2.4.2); 0: they are fixed */
} orc_md;

/* Physical constants (CODATA 2018 / exact SI).  Written here independently
 * of the GPU library. */
double orc_mass_al(void);      /* amu */
double orc_kb(void);           /* eV/K */
double orc_mvv2e(void);        /* eV per amu*A^2/fs^2 */
double orc_ev_a3_to_gpa(void); /* GPa per eV/A^3 */

/* ---- random numbers: counter-based SplitMix64 + Box-Muller ---- */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k);  /* k-th output (k >= 0) of the sequence seeded by seed */
void orc_gaussians(uint64_t seed, int64_t count, double *out);

/* ---- lattice (Problem setup / Boundary conditions) ---- */
int64_t orc_fcc_count(int32_t nc);
/* group: 0 mobile, 1 bottom slab (fixed), 2 top slab (fixed). pz: z plane index. */
void orc_fcc_cube(int32_t nc, double a, int32_t fix_slabs,
                  double *x, double *y, double *z, uint8_t *group, int32_t *pz);
/* Maxwell-Boltzmann velocities at T0 for mobile atoms, mean removed, rescaled
 * to T0 exactly with 3*N_mob-3 degrees of freedom.  Returns 0 or -1. */
int32_t orc_mb_velocities(int64_t n, const uint8_t *group, double T0, uint64_t seed,
                          double *vx, double *vy, double *vz);

/* ---- potential ---- */
void orc_pair_terms(const orc_sc *p, double r, double *V, double *dV, double *rho, double *drho);
double orc_embed(const orc_sc *p, double rhobar);
double orc_embed_deriv(const orc_sc *p, double rhobar);

/* ---- energy and forces ---- */
void orc_density(int64_t n, const double *x, const double *y, const double *z,
                 const orc_sc *p, double *rhobar);
/* Internal forces F^int (before any constraint), total U, virial
 * W_zz = sum_i z_i F_iz, reaction R_z = -sum_{group==2} F_iz.  Per-atom energy
 * e_i = 1/2 sum_j V_s(r_ij) + B(rhobar_i) is written if e != NULL. */
void orc_forces(int64_t n, const double *x, const double *y, const double *z,
                const uint8_t *group, const orc_sc *p,
                double *fx, double *fy, double *fz, double *e,
                double *U, double *Wzz, double *Rz);
/* The same quantities for one atom i, computed from scratch in O(N * nbar). */
double orc_atom_density(int64_t n, const double *x, const double *y, const double *z,
                        const orc_sc *p, int64_t i);
void orc_atom_force(int64_t n, const double *x, const double *y, const double *z,
                    const orc_sc *p, int64_t i, double f[3]);

/* ---- neighbour sets and cells ---- */
/* All j != i with dx*dx+dy*dy+dz*dz < rlist*rlist, dx = x_j - x_i, in ascending j.
 * offsets has n+1 entries.  Returns the total count (idx written only up to cap). */
int64_t orc_neighbors(int64_t n, const double *x, const double *y, const double *z,
                      double rlist, int64_t *offsets, int32_t *idx, int64_t cap);
/* Cell coordinates by the documented rule c_d = clamp(floor((x_d - o_d) * inv_h), 0, dims_d - 1). */
void orc_cell_assign(int64_t n, const double *x, const double *y, const double *z,
                     const double origin[3], double inv_h, const int32_t dims[3], int32_t *cxyz);

/* ---- dynamics ---- */
typedef struct {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz;
    const uint8_t *group;
    double volume0;   /* A^3 at zero strain */
    double area0;     /* A^2, cross-section for the reaction stress */
    double strain;    /* engineering strain along z */
} orc_state;

typedef struct {
    double ke, pe, szz, tz;        /* burst means: eV, eV, GPa, GPa */
    double ke_se, pe_se, szz_se;   /* 20-block standard errors (NaN if fewer than 20 samples) */
    double temp;                   /* mean temperature, K */
    int64_t n_samples;
} orc_averages;

/* Per-step series columns. */
enum { ORC_SER_K = 0, ORC_SER_U, ORC_SER_SZZ, ORC_SER_T, ORC_SER_LAMBDA, ORC_SER_TZ, ORC_SER_NCOL };

/* Run n_steps velocity-Verlet steps from the state; forces are recomputed at
 * the start.  series (n_steps x ORC_SER_NCOL, row major) may be NULL.
 * pos_sum (3n: x sums, then y, then z; may be NULL) receives the sum over the
 * samples r = 1..n_steps of every atom's position, the numerator of
 * Eq. (mean_pos).  Returns 0, or -7 if the thermostat meets T <= 0. */
/* Standard error of the mean from 20 batch means (NaN when n < 20). */
void orc_block_se(const double *col, int64_t stride, int64_t n, double *se);

int32_t orc_run_burst(orc_state *s, const orc_sc *p, const orc_md *md, int64_t n_steps,
                      orc_averages *avg, double *series, double *pos_sum);
/* eps_k = eps_{k-1} + d_eps; z <- z (1+eps_k)/(1+eps_{k-1}) for every atom. */
void orc_apply_strain(orc_state *s, double d_eps);
double orc_volume(const orc_state *s);

/* Instantaneous observables of a state (no time stepping). */
void orc_observables(const orc_state *s, const orc_sc *p, double *K, double *U, double *szz, double *tz);

int32_t orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
