/*
 * ptamd: MI355X (gfx950) library for the fast molecular-dynamics bursts of
 * Practical Time Averaging (PTA), after Baruah, Chatterjee, Acharya and Wang,
 * "Averaging Molecular Dynamics simulations to study the slow-strain-rate
 * behavior of metals".
 *
 * One call of ptamd_run_fast_md() is one PTA averaging burst: it holds the
 * load fixed, runs n velocity-Verlet steps of EAM dynamics of a free-surface
 * FCC aluminium cube and returns the running time averages of the kinetic
 * energy, the potential energy and the sigma_zz virial stress
 * (Sec. 2.2 Step 1, Eq. (R_m_t); state functions of Eq. (state_variables)).
 * ptamd_apply_strain_increment() moves the load between bursts (Sec. 2.4.2,
 * the loading sequence).
 *
 * Conventions for every entry point:
 *   - Units: Angstrom, eV, fs, amu, K; stresses in GPa (tension positive).
 *   - The load axis is z.  Arrays at the boundary are host arrays in the
 *     ORIGINAL atom order (the lattice order of ptamd_create_system, or the
 *     caller's order for ptamd_create_system_from_state); the library's
 *     internal spatial ordering is never visible.
 *   - The caller owns every host buffer it passes; each must hold at least
 *     the stated number of elements.  The library never keeps a host pointer
 *     after a call returns.  The library owns all device memory of a system.
 *   - Every function returns a ptamd_status; 0 is success.  On failure,
 *     ptamd_last_error() returns a message (thread local, valid until the
 *     next call on the same thread).  After an error other than
 *     PTAMD_EINVAL the system stays valid, but its state may be partly
 *     advanced: restore it with ptamd_set_state().
 *   - A system is not thread safe: one thread at a time per handle.
 *   - All device work is ordered on the system's HIP stream (the null
 *     stream unless ptamd_set_stream() names another).  Every call returns
 *     after its results are on the host.
 *   - There is no CPU fallback: without a usable gfx950 device every call
 *     that needs one returns PTAMD_ENODEV.
 */
#ifndef PTAMD_H
#define PTAMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptamd_system ptamd_system; /* opaque */

typedef enum {
    PTAMD_OK = 0,
    PTAMD_EINVAL = -1,     /* bad argument: nothing was changed */
    PTAMD_EDEVICE = -2,    /* a HIP runtime call failed */
    PTAMD_ENOMEM = -3,     /* device or host allocation failed */
    PTAMD_ENONFINITE = -4, /* a position, velocity or energy became NaN/Inf */
    PTAMD_EESCAPE = -5,    /* an atom left the allowed region around the cube */
    PTAMD_EOVERFLOW = -6,  /* an internal capacity could not be grown */
    PTAMD_ESTATE = -7,     /* thermostat met T <= 0, or lambda^2 < 0 */
    PTAMD_ENODEV = -8      /* no usable gfx950 device */
} ptamd_status;

/* Free-surface FCC cube of n_cells^3 conventional cells (4 atoms each) with
 * axes along [100],[010],[001] (Sec. 2.4.1 "Problem Setup").  Lattice
 * positions are integer plane indices times lattice_a/2.  Initial velocities
 * are Maxwell-Boltzmann at T0 (Sec. 2.4.2): normals from the counter-based
 * SplitMix64 stream of `seed` via Box-Muller, three per atom in atom order,
 * mobile atoms only, mean removed, rescaled to T0 with 3*N_mob-3 degrees of
 * freedom.  T0 is also the thermostat target.  With fix_slabs != 0 the
 * three lowest and three highest z planes are the fixed boundary regions
 * (v = 0, F = 0; Sec. 2.4.2); n_cells >= 4 then, else n_cells >= 1. */
typedef struct {
    int32_t n_cells;
    double lattice_a;
    double T0;
    uint64_t seed;
    int32_t fix_slabs;
} ptamd_lattice_desc;

/* Sutton-Chen functions in the EAM energy of Eq. (pe):
 *   V(r) = eps (a/r)^n,  rho(r) = (a/r)^m,  B(rhobar) = -c eps sqrt(rhobar),
 * cut at rc (strict r < rc).  shift: 0 truncated, 1 energy-shifted,
 * 2 shifted-force (value and slope of V and rho vanish at rc).
 * Requires eps >= 0, a > 0, n > 0, m > 0, c >= 0, 0 < rc <= 4a. */
typedef struct {
    double eps, a, n, m, c, rc;
    int32_t shift;
} ptamd_sc_params;

/* precision: 0 = FP64 everywhere; 1 = mixed (pair and density terms in FP32;
 * state, forces-to-velocity update and all global sums in FP64 / 64-bit fixed
 * point).  skin: Verlet-list skin in A (0 < skin <= 3).  lanes_per_atom:
 * lanes of a wavefront that share one atom's pair sums; 0 = chosen from the
 * atom count (ptamd_autotune() measures instead), else 1, 2, 4, 8 or 16.  thermostat: 0 = NVE,
 * 1 = Berendsen with coupling time tau_fs (> 0), applied to the mobile atoms
 * at the end of each step.  full_lists: 0 (default) = every 4 prune_every
 * steps (prune_every 1, 2 or 3; 0 = 1) the density pass prunes the Verlet
 * lists to the pairs within rc plus what the fastest atoms can close in the
 * steps until the next pruning, and the pair passes in between read those;
 * 1 = the pair passes read the full Verlet lists every step.  Results do not
 * depend on either beyond rounding (every pair term still tests r < rc). */
typedef struct {
    double dt_fs;
    double tau_fs;
    int32_t thermostat;
    int32_t precision;
    double skin;
    int32_t lanes_per_atom;
    int32_t full_lists;
    int32_t prune_every;
} ptamd_md_params;

/* Burst averages over the samples r = 1..n (Eq. (R_m_t)); *_se are
 * standard errors from 20 equal blocks (NaN below 20 samples); tz is the
 * reaction stress -sum_{top} F^int_z / area0 of Eq. (state_variables) read
 * along z; strain is the engineering strain at which the burst ran. */
typedef struct {
    double ke, pe, szz, tz;
    double ke_se, pe_se, szz_se;
    double temp;
    double strain;
    int64_t n_samples;
} ptamd_averages;

typedef struct {
    int64_t n_atoms;         /* all replicas */
    int32_t n_replicas;
    int32_t precision;
    int32_t lanes_per_atom;
    int32_t list_capacity;   /* per-atom Verlet-list capacity */
    int64_t list_builds;     /* since creation */
    int64_t sorts;           /* spatial re-sorts since creation */
    int64_t rollbacks;       /* chunks re-run after a failed bound */
    int64_t steps;           /* MD steps since creation */
    double skin;
    double bin_margin;
    int32_t list_index_bits; /* 16: list entries are 16-bit steps between a lane's consecutive
                                neighbour indices (atoms whose listed indices span 16 bits or more
                                hold 32-bit indices instead; ptamd_count_pairs counts them) */
    int32_t folded;          /* 1: each step's kick-drift runs inside its density pass (mixed form,
                                up to 131,072 padded atoms) */
    int32_t prune_every;     /* pruning passes every 4 prune_every steps; 0: full lists every step */
} ptamd_info;

/* ---- creation ---- */
ptamd_status ptamd_create_system(const ptamd_lattice_desc *desc, const ptamd_sc_params *sc,
                                 const ptamd_md_params *md, ptamd_system **out);
/* A system from an explicit state (n atoms; group[i]: 0 mobile, 1 fixed
 * bottom region, 2 fixed top region, whose internal z force is the
 * reaction).  volume0 (A^3, at zero strain) scales the virial stress,
 * area0 (A^2) the reaction stress; T0 is the thermostat target. */
ptamd_status ptamd_create_system_from_state(int64_t n, const double *x, const double *y, const double *z,
                                            const double *vx, const double *vy, const double *vz,
                                            const uint8_t *group, double volume0, double area0, double T0,
                                            const ptamd_sc_params *sc, const ptamd_md_params *md,
                                            ptamd_system **out);
/* R independent replicas in one system (one launch per kernel covers them
 * all).  Replica r is the cube of descs[r]; its thermostat target is
 * descs[r].T0.  Atoms are numbered replica by replica. */
ptamd_status ptamd_create_batch(int32_t n_replicas, const ptamd_lattice_desc *descs, const ptamd_sc_params *sc,
                                const ptamd_md_params *md, ptamd_system **out);
ptamd_status ptamd_destroy_system(ptamd_system *sys);

/* ---- tabulated EAM (the setfl form of the potential of Eq. (pe)) ----
 * The paper's runs use a tabulated aluminium EAM potential.  A table holds,
 * for one element, F(rhobar) at rhobar = k*drho (k < nrho), rho(r) and
 * r*phi(r) at r = k*dr (k < nr), as in a setfl file; V(r) = (r phi)(r) / r
 * is the pair term and F the embedding term B of Eq. (pe).  Between knots
 * each function is the not-a-knot cubic spline through its knots (the
 * unique C2 piecewise cubic whose third derivative is also continuous at the
 * second and the second-to-last knot); past the last knot F continues
 * linearly with its end slope.  Pairs count for r < rc.  Requires
 * nrho, nr >= 4, drho, dr > 0, 0 < rc <= min((nr-1) dr, 12 A), all values
 * finite.  The atomic mass stays the library's aluminium mass. */
typedef struct {
    int32_t nrho;
    double drho;
    int32_t nr;
    double dr;
    double rc;
    const double *F;     /* nrho values */
    const double *rho;   /* nr values */
    const double *rphi;  /* nr values: r * phi(r) */
} ptamd_eam_table;

/* Replaces the system's potential by the table (copied; the caller's arrays
 * may be freed afterwards).  Lists and cells are rebuilt at the next call;
 * the state is unchanged.  Every later evaluation uses the table. */
ptamd_status ptamd_set_eam_table(ptamd_system *sys, const ptamd_eam_table *table);
/* Reads a single-element setfl file (three comment lines; "1 <element>";
 * "Nrho drho Nr dr cutoff"; "Z mass a0 lattice"; then F, rho and r*phi as
 * whitespace-separated numbers).  Always sets the sizes and spacings of
 * *table and, if mass is not NULL, the file's mass; with F, rho and rphi
 * all non-NULL (holding nrho, nr and nr doubles) it also reads the values
 * into them and points the table at them.  Call once to size, once to read. */
ptamd_status ptamd_read_setfl(const char *path, ptamd_eam_table *table, double *F, double *rho, double *rphi,
                              double *mass);
/* The library's interpolation of one table function (which: 0 F, 1 rho,
 * 2 r*phi) at n arguments: values f and derivatives df.  Host only, no GPU
 * needed. */
ptamd_status ptamd_eam_table_eval(const ptamd_eam_table *table, int32_t which, int64_t n, const double *x,
                                  double *f, double *df);

/* ---- the hot path ---- */
/* Load step along z about z = 0 (Sec. 2.4.2 loading sequence, applied as an
 * affine strain of every atom): eps_k = eps_{k-1} + d_eps, every z scaled by
 * (1+eps_k)/(1+eps_{k-1}); velocities unchanged; fixed regions stay fixed at
 * their new positions.  |d_eps| < 0.05.  Applies to every replica. */
ptamd_status ptamd_apply_strain_increment(ptamd_system *sys, double d_eps);
/* Per-replica increments: d_eps has n_replicas entries. */
ptamd_status ptamd_apply_strain_increments(ptamd_system *sys, const double *d_eps);
/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same as
 * ptamd_apply_strain_increments, with the same results, but it allocates
 * nothing.  The per-replica scale factors go to a static device array of
 * the library, one per GPU, set up when the first system is created on it;
 * at most 4096 replicas per call (PTAMD_EINVAL beyond, with a message).
 * Every call on one GPU shares that array and overwrites it, so calls that
 * overlap on one GPU (systems driven from different threads or streams)
 * race; calls in sequence do not.  d_eps: caller-owned, n_replicas entries. */
ptamd_status ptamd_apply_strain_increments_noalloc(ptamd_system *sys, const double *d_eps);
/* One averaging burst of n_steps >= 1 steps (Sec. 2.3 velocity Verlet,
 * Eqs. (vv_algo_pos_pred_half), (vv_algo_pos_pred), (vv_algo_vel_pred), with
 * fixed regions and the optional Berendsen thermostat).  Forces are
 * recomputed from the positions at the start.  out has n_replicas entries. */
ptamd_status ptamd_run_fast_md(ptamd_system *sys, int64_t n_steps, ptamd_averages *out);

/* Convergence test of the running time averages (App. A, Eq. (R_m_conv)).
 * With R(i) the running average of a state function over samples 1..i, a
 * replica's burst ends at the first checkpoint i = j*lag, j >= 2, at which
 * every tested function f satisfies
 *     |R(i) - R(i-lag)| / max(|R(i)|, floor[f]) < tol[f].
 * Functions in the order K, U, sigma_zz, T_z; tol[f] <= 0 leaves f out (at
 * least one must be tested); floor[f] >= 0 (0 gives the plain relative
 * error of the appendix).  n_max is N_max: a replica not converged after
 * n_max samples stops there.  Table 1 gives tol 0.05 for K, U and the
 * reaction stress and N_max = 50000; the paper does not give the lag. */
typedef struct {
    int64_t lag;     /* >= 1 */
    int64_t n_max;   /* >= 2 * lag */
    double tol[4];
    double floor[4];
} ptamd_conv_params;

/* One averaging burst per replica whose length the convergence test sets
 * (Sec. 2.2 Step 1: N_t is the number of steps the running averages need to
 * converge).  Each replica stops at its own N_s, frozen from then on (its
 * final state is the state after sample N_s, the x^conv that Sec. 2.2 Step 4
 * carries to the next run), while the others go on in the same launches.
 * out[r] averages samples 1..N_s (n_samples = N_s); its standard errors come
 * from the complete batches of a batch-means scheme whose batches start at
 * max(1, lag/10) samples and double in length whenever 20 are full (NaN with
 * fewer than 2).  n_conv[r] = N_s, or 0 if replica r had not converged after
 * n_max samples (out[r] then averages all n_max).  Both arrays have
 * n_replicas entries. */
ptamd_status ptamd_run_until_converged(ptamd_system *sys, const ptamd_conv_params *conv, ptamd_averages *out,
                                       int64_t *n_conv);

/* ---- further observables of the paper ---- */
/* Per-atom mean positions of Eq. (mean_pos): with enable != 0 every later
 * burst also sums each atom's position over its samples r = 1..N_t (FP64,
 * 24 more bytes of device memory per atom; the sums follow the atoms through
 * re-sorts and roll-backs).  enable = 0 frees them. */
ptamd_status ptamd_set_mean_positions(ptamd_system *sys, int32_t enable);
/* Mean positions over the samples of the last burst (per replica its own
 * N_t: n_samples of its averages), original order, all replicas
 * concatenated.  PTAMD_ESTATE if switched off, or if no burst has run since
 * they were switched on or since another call evaluated forces. */
ptamd_status ptamd_get_mean_positions(ptamd_system *sys, double *x, double *y, double *z);

/* Thermal relaxation before loading (Sec. 2.4.2): the atoms of the top
 * region (group 2) move freely along z, each on its own, held along x and
 * y, while bursts of burst_steps run; the thermostat then also acts on
 * them, with one degree of freedom each.  It ends when the burst-averaged
 * reaction stress |T_z| of every replica is below tol_gpa, or after
 * max_bursts bursts; the top region is then held again where it stands
 * (v = 0).  The paper does not give a tolerance. */
typedef struct {
    int64_t burst_steps;   /* >= 1 */
    int64_t max_bursts;    /* >= 1 */
    double tol_gpa;        /* >= 0 */
} ptamd_relax_params;
/* out: the averages of the last burst, per replica; n_bursts: bursts run;
 * relaxed[r]: 1 if replica r met the tolerance in the last burst.  Every
 * replica needs a top region. */
ptamd_status ptamd_relax(ptamd_system *sys, const ptamd_relax_params *prm, ptamd_averages *out, int64_t *n_bursts,
                         int32_t *relaxed);

/* ---- the PTA slow-time driver (Sec. 2.2 Steps 1-4, Sec. 2.4.2) ----
 * One slow step t -> t+h takes three converged runs (ptamd_run_until_converged)
 * at the strains of slow times t+h-Delta, t+h-Delta/2 and t+h, each started
 * from the state the run before it left (Eq. (x_guess_step3)), so one
 * trajectory per replica carries through the whole sequence; between the
 * runs the load moves by affine strain increments.  Slow time is measured by
 * the applied strain: the first run of ptamd_pta_start is at the current
 * strain (slow time -Delta), and a jump h advances the strain by d_eps_h.
 * The slow variables v are the averaged K, U, sigma_zz and T_z (the paper's
 * are K, U and the reaction stress).  Per state function f:
 *   Step 1, Eq. (dvdt_algo): dv/dt = (R_t - R_{t-Delta}) / Delta
 *   Step 2, Eq. (pta_pred):  v_pred(t+h) = v(t) + h dv/dt
 *   Step 3, Eq. (simp):      v_d(t+h) = (R_{t+h-Delta} + 4 R_{t+h-Delta/2} + R_{t+h}) / 6
 *           Eq. (rel_err):   e_v = |(v_pred - v_d) / v_d|
 *   match (status 0) if e_v < tol_v[f]: v(t+h) = v_pred; otherwise the jump
 *   test of Eq. (jump_err), e1 = |(R_{t+h} - R_t)/R_t|, e2 = |(R_t - R_{t-h})/R_{t-h}|,
 *   flags a jump (status 1) if |e1/e2 - 1| >= tol_j[f], or if e1 >= tol_j[f]
 *   when a jump was flagged at t or there is no R_{t-h} yet (the first jump);
 *   with a jump, or with neither (status 2), v(t+h) = v_d.
 * All of it is FP64 host arithmetic exactly as written (IEEE: x/0 = inf,
 * comparisons with NaN are false).  Table 1: Delta = h/5; tol_v 1% K, 5% U,
 * 1% reaction; tol_j 8% K, 1% U, 5% reaction. */
typedef struct {
    double d_eps_h;             /* strain advanced per slow jump h (strain rate x h), |.| < 0.05 */
    double delta_over_h;        /* Delta / h, in (0, 1] */
    ptamd_conv_params conv;     /* how every running average is converged */
    double tol_v[4];            /* Eq. (rel_err) tolerance: K, U, sigma_zz, T_z */
    double tol_j[4];            /* Eq. (jump_err) tolerance */
} ptamd_pta_params;

/* Slow history of one replica, carried from one jump to the next (plain
 * data: the caller may store and restore it). */
typedef struct {
    double strain;              /* strain at slow time t */
    double R_tmd[4];            /* R(t - Delta) */
    double R_tmh[4];            /* R(t - Delta/2) */
    double R_t[4];              /* R(t) */
    double R_prev[4];           /* R(t - h), meaningful once n_jumps >= 1 */
    double v[4];                /* slow variables v(t) */
    int32_t jump_at_t[4];       /* a jump of the measure was flagged at t */
    int64_t n_jumps;            /* jumps taken since ptamd_pta_start */
} ptamd_pta_state;

/* What one slow step (or the start) did, per replica. */
typedef struct {
    double strain[3];           /* strains of the three runs */
    double R[3][4];             /* their converged running averages */
    int64_t n_steps[3];         /* N_s of each run (0: stopped at n_max unconverged) */
    double v_pred[4], v_d[4], v[4];
    double e_v[4], e1[4], e2[4];
    int32_t status[4];          /* 0 match, 1 jump, 2 neither, -1 start (no test) */
} ptamd_pta_record;

/* Slow time 0: runs at the current strain and after two increments of
 * Delta/2 (Sec. 2.4.2 steps 1-3); v(0) is their Simpson value.  state and
 * rec have n_replicas entries. */
ptamd_status ptamd_pta_start(ptamd_system *sys, const ptamd_pta_params *prm, ptamd_pta_state *state,
                             ptamd_pta_record *rec);
/* One slow step t -> t+h for every replica (Sec. 2.2 Steps 1-4). */
ptamd_status ptamd_pta_jump(ptamd_system *sys, const ptamd_pta_params *prm, ptamd_pta_state *state,
                            ptamd_pta_record *rec);
/* The arithmetic of one slow step alone (no device work): advances one
 * replica's state from t to t+h given the converged averages R[3][4] of the
 * three runs, their strains and N_s.  Host only; usable without a GPU. */
ptamd_status ptamd_pta_update(const ptamd_pta_params *prm, ptamd_pta_state *state, const double *R /* 3x4 */,
                              const double *strains /* 3 */, const int64_t *n_steps /* 3 */,
                              ptamd_pta_record *rec);

/* ---- state in and out (original order, all replicas concatenated) ---- */
ptamd_status ptamd_get_num_atoms(const ptamd_system *sys, int64_t *n);
ptamd_status ptamd_get_state(ptamd_system *sys, double *x, double *y, double *z, double *vx, double *vy,
                             double *vz);
ptamd_status ptamd_set_state(ptamd_system *sys, const double *x, const double *y, const double *z,
                             const double *vx, const double *vy, const double *vz);
ptamd_status ptamd_get_strain(const ptamd_system *sys, double *strain /* n_replicas */);

/* ---- inspection hooks for tests ---- */
/* Internal forces F^int of Eq. (f_int) before any constraint, at the current
 * positions, plus per-replica U (Eq. (pe)) and W_zz = sum_i z_i F_iz.
 * pe and wzz have n_replicas entries. */
ptamd_status ptamd_compute_forces(ptamd_system *sys, double *fx, double *fy, double *fz, double *pe,
                                  double *wzz);
/* The internal forces F^int of Eq. (f_int) (before any constraint) that the
 * device holds now: those of the last force pass, i.e. after a burst the
 * forces at its final positions as the burst's last step computed them
 * (in the mixed form from the folded step's density pass), without
 * recomputing anything.  fx, fy, fz: caller-owned, n_atoms each, original
 * atom order.  PTAMD_EINVAL on a null argument. */
ptamd_status ptamd_get_forces(ptamd_system *sys, double *fx, double *fy, double *fz);
/* Spatially sorts and rebuilds the Verlet list at the current positions and
 * returns it as CSR in original indices, each row ascending: offsets has
 * n+1 entries, idx has cap entries.  Returns PTAMD_EOVERFLOW (with
 * offsets filled) if cap is too small. */
ptamd_status ptamd_get_neighbors(ptamd_system *sys, int64_t *offsets, int32_t *idx, int64_t cap);
/* Cell coordinates (3 per atom, original order) of the last spatial sort,
 * and per replica its grid origin (3), 1/h and dims (3). */
ptamd_status ptamd_get_cells(ptamd_system *sys, int32_t *cxyz, double *origin, double *inv_h, int32_t *dims);
/* Per-step samples of the last burst for replica r, row major with 6
 * columns: K, U, sigma_zz, T, lambda, T_z.  cap = rows the buffer holds. */
ptamd_status ptamd_get_series(ptamd_system *sys, int32_t replica, double *buf, int64_t cap);
ptamd_status ptamd_get_info(const ptamd_system *sys, ptamd_info *info);

/* ---- streams and timing ---- */
/* Orders all later device work on stream (a hipStream_t, e.g. torch's
 * current stream on ROCm).  NULL selects the null stream. */
ptamd_status ptamd_set_stream(ptamd_system *sys, void *hip_stream);
/* Timing of the pair kernels (measurement hook).  The first call switches
 * timing on; from then on the first two steps of every burst chunk of at
 * least two steps are launched directly (the rest of the chunk stays a
 * graph; the first of them prunes the lists, the second is an ordinary
 * step).  The second step's density and force kernels are bracketed by HIP
 * events on the system's stream: their averages are density_event_ms and
 * avg_event_ms (each holds the dispatch latency of a direct launch, about a
 * microsecond).  The force kernel's blocks also stamp the device wall clock
 * at their start and end, and the launch's span (earliest start to latest
 * end) is averaged into avg_ms.  count = steps timed since the last reset.
 * Outputs may be NULL. */
ptamd_status ptamd_kernel_timing(ptamd_system *sys, double *avg_ms, double *avg_event_ms, double *density_event_ms,
                                 int64_t *count, int32_t reset);
/* Autotuner: times probe bursts of probe_steps (>= 10) steps from the
 * current state, in two stages: lanes per atom in {2, 4, 8, 16} x Verlet
 * skin in {1.0, 1.5, 2.0, 2.5} A, then (unless the system was created with
 * full_lists) the pruning interval: full lists or a pruning pass every 1, 2
 * or 3 rebuild points (4, 8 or 12 steps; prune_every 0, 1, 2, 3).  Each
 * candidate is probed twice and counts with its faster probe; the fastest
 * is kept (in the first stage, of the candidates within 3% of it, the one
 * with the largest skin: lists live shorter as a sample heats or
 * evaporates, which a probe from the current state does not see).  The
 * state is restored exactly (positions, velocities, atom order), and the
 * HIP graphs that bursts in the chosen configuration launch are built (with
 * the kernel timing as set by ptamd_kernel_timing).  With use_cache != 0 an
 * earlier choice for the same atom count, replica count, precision, cutoff
 * and list mode in this process is reused without probing.  The choice
 * changes summation order (hence rounding), never the computed quantities.
 * Outputs may be NULL. */
ptamd_status ptamd_autotune(ptamd_system *sys, int64_t probe_steps, int32_t use_cache, int32_t *lanes_per_atom,
                            double *skin, int32_t *prune_every, double *ms_per_step);
/* Unique pairs within rc at the current positions (for the algorithmic
 * flop count), summed over the replicas; list_entries: entries of the full
 * Verlet lists; pruned_entries (may be NULL): entries of the pruned lists
 * as the last pruning pass left them, 0 when the last chunk ran on full
 * lists; prune_radius (may be NULL): their radius in A (0 then); wide_atoms
 * (may be NULL): atoms whose lists hold 32-bit indices.  Sorts and rebuilds
 * the lists first if the state changed since the last burst. */
ptamd_status ptamd_count_pairs(ptamd_system *sys, int64_t *pairs_in_rc, int64_t *list_entries,
                               int64_t *pruned_entries, double *prune_radius, int64_t *wide_atoms);

/* Achievable rates of the current device, as context for the rooflines
 * (no part of the MD path): a streaming copy of bytes (a multiple of 16,
 * at least 1 MiB; float4 loads and stores; read plus write counted) in
 * GB/s, and independent FMA chains in FP32 (one FMA per instruction: the
 * library is built without packed FP32) and in FP64 in TFLOP/s, each the
 * best of reps (>= 1) launches timed with HIP events after one untimed
 * launch.  Allocates 2 x bytes of device memory for the copy and frees it
 * before returning.  Outputs may be NULL. */
ptamd_status ptamd_measure_device(int64_t bytes, int32_t reps, double *copy_gbs, double *fma32_tflops,
                                  double *fma64_tflops);

const char *ptamd_last_error(void);
const char *ptamd_version(void);

#ifdef __cplusplus
}
#endif
#endif
