/* Exercises the oracle's entry points on a small cube so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py)
 * sees every array access they make: lattice, velocities, densities and
 * forces, single-atom terms, neighbour sets (including a capacity smaller
 * than the count), cell assignment, a short burst with its series and
 * position sums, strain, observables and the block standard error.  Prints
 * "ok" and returns 0 when every result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int finite_all(const double *v, int64_t n) {
    for (int64_t k = 0; k < n; ++k)
        if (!isfinite(v[k])) return 0;
    return 1;
}

int main(void) {
    const int32_t nc = 4;
    const int64_t n = orc_fcc_count(nc);
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *vx = malloc(sizeof(double) * n), *vy = malloc(sizeof(double) * n), *vz = malloc(sizeof(double) * n);
    double *fx = malloc(sizeof(double) * n), *fy = malloc(sizeof(double) * n), *fz = malloc(sizeof(double) * n);
    double *e = malloc(sizeof(double) * n), *rho = malloc(sizeof(double) * n);
    uint8_t *group = malloc(n);
    int32_t *pz = malloc(sizeof(int32_t) * n);
    orc_fcc_cube(nc, 4.05, 1, x, y, z, group, pz);
    for (int64_t k = 0; k < n; ++k) x[k] += 0.01 * (double)((k * 7) % 11 - 5);  /* break the symmetry */
    if (orc_mb_velocities(n, group, 300.0, 7, vx, vy, vz) != 0) return 2;
    double g[9];
    orc_gaussians(3, 9, g);

    orc_sc p = {0.0033147, 4.05, 7.0, 6.0, 16.399, 8.1, 2, NULL};
    orc_density(n, x, y, z, &p, rho);
    double U = 0.0, W = 0.0, R = 0.0;
    orc_forces(n, x, y, z, group, &p, fx, fy, fz, e, &U, &W, &R);
    double f1[3];
    orc_atom_force(n, x, y, z, &p, n / 2, f1);
    const double r1 = orc_atom_density(n, x, y, z, &p, n / 3);
    double V, dV, rh, drh;
    orc_pair_terms(&p, 3.0, &V, &dV, &rh, &drh);
    const double b = orc_embed(&p, 10.0) + orc_embed_deriv(&p, 10.0) + orc_embed_deriv(&p, 0.0);

    int64_t *off = malloc(sizeof(int64_t) * (n + 1));
    const int64_t total = orc_neighbors(n, x, y, z, 9.1, off, NULL, 0);
    int32_t *idx = malloc(sizeof(int32_t) * (total > 0 ? total : 1));
    if (orc_neighbors(n, x, y, z, 9.1, off, idx, total / 2) != total) return 3;  /* short capacity */
    if (orc_neighbors(n, x, y, z, 9.1, off, idx, total) != total) return 3;
    const double origin[3] = {-8.0, -8.0, -8.0};
    const int32_t dims[3] = {3, 3, 3};
    int32_t *cxyz = malloc(sizeof(int32_t) * 3 * n);
    orc_cell_assign(n, x, y, z, origin, 1.0 / 9.0, dims, cxyz);

    orc_state s = {n, x, y, z, vx, vy, vz, group, pow(nc * 4.05, 3), pow(nc * 4.05, 2), 0.0};
    orc_md md = {1.0, 100.0, 300.0, 1, 0};
    const int64_t steps = 25;
    double *series = malloc(sizeof(double) * steps * ORC_SER_NCOL);
    double *pos = malloc(sizeof(double) * 3 * n);
    orc_averages avg;
    orc_apply_strain(&s, 1e-4);
    if (orc_run_burst(&s, &p, &md, steps, &avg, series, pos) != 0) return 4;
    double K, Uo, szz, tz;
    orc_observables(&s, &p, &K, &Uo, &szz, &tz);
    double se = 0.0;
    orc_block_se(series + ORC_SER_K, ORC_SER_NCOL, steps, &se);
    md.top_free_z = 1;
    if (orc_run_burst(&s, &p, &md, 3, &avg, NULL, NULL) != 0) return 4;

    const double sc[] = {U, W, R, f1[0], f1[1], f1[2], r1, V, dV, rh, drh, b, avg.ke, avg.pe, avg.szz, K, Uo, szz,
                         tz, se, orc_volume(&s)};
    if (!finite_all(fx, n) || !finite_all(rho, n) || !finite_all(e, n) || !finite_all(pos, 3 * n) ||
        !finite_all(series, steps * ORC_SER_NCOL) || !finite_all(sc, (int64_t)(sizeof sc / sizeof sc[0])))
        return 5;
    free(x); free(y); free(z); free(vx); free(vy); free(vz); free(fx); free(fy); free(fz);
    free(e); free(rho); free(group); free(pz); free(off); free(idx); free(cxyz); free(series); free(pos);
    printf("ok %lld atoms, %lld neighbour entries\n", (long long)n, (long long)total);
    return 0;
}
