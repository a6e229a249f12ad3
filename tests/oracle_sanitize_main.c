/*
 * Driver for the sanitised CPU build of the oracle (tests/test_oracle_sanitize.py):
 * creates lattices of every kind the oracle supports (periodic droplet, walled
 * jet with inlet and outflow, a closed box with no-slip and free-slip faces,
 * variable density with gravity, a one-plane lattice), steps them, reads every
 * output and frees them, so that AddressSanitizer and UndefinedBehaviorSanitizer
 * see all of the oracle's code paths.  Test infrastructure only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    int32_t bc[6];
    double nu, sigma, width, gamma, eps;
    double inlet_u, inlet_d, inlet_noise;
    uint64_t seed;
    int32_t vd;
    double rho_a, rho_b, nu_a, nu_b;
    double grav[3];
} orc_params;

typedef struct orc orc;
int orc_create(const orc_params *p, orc **out);
void orc_free(orc *o);
void orc_set_physical(orc *o, const double *rho, const double *u, const double *P, const double *phi, int64_t step);
void orc_step(orc *o, int64_t nsteps);
void orc_get_physical(orc *o, double *rho, double *u, double *P, double *phi);
void orc_get_raw(orc *o, double *drho, double *ub, double *Q, double *phi);
void orc_get_geometry(orc *o, double *G, double *n, double *kappa, double *F);
void orc_get_accel(orc *o, double *a, double *omega);
void orc_sums(orc *o, double *mass, double *phase);
void orc_get_populations(const orc *o, double *f, double *g);

static int run(const orc_params *p, int steps) {
    orc *o = NULL;
    if (orc_create(p, &o) != 0) return 1;
    const long N = (long)p->nx * p->ny * p->nz;
    double *rho = calloc(N, sizeof(double)), *u = calloc(3 * N, sizeof(double)), *P = calloc(6 * N, sizeof(double));
    double *phi = calloc(N, sizeof(double)), *G = calloc(3 * N, sizeof(double)), *n = calloc(3 * N, sizeof(double));
    double *k = calloc(N, sizeof(double)), *F = calloc(3 * N, sizeof(double)), *f = calloc(27 * N, sizeof(double));
    double *g = calloc(7 * N, sizeof(double)), *a = calloc(3 * N, sizeof(double)), *om = calloc(N, sizeof(double));
    if (!rho || !u || !P || !phi || !G || !n || !k || !F || !f || !g || !a || !om) return 2;
    for (long id = 0; id < N; ++id) {
        const int x = (int)(id % p->nx), y = (int)((id / p->nx) % p->ny), z = (int)(id / ((long)p->nx * p->ny));
        const double r = sqrt(pow(x - 0.5 * p->nx, 2) + pow(y - 0.5 * p->ny, 2) + pow(z - 0.5 * p->nz, 2));
        phi[id] = 0.5 * (1.0 - tanh(2.0 * (r - 0.25 * p->nx) / 3.0));
        rho[id] = 1.0;
        u[id] = 1e-3 * sin(0.3 * y);
    }
    orc_set_physical(o, rho, u, P, phi, 0);
    orc_step(o, steps);
    double m, ph;
    orc_get_physical(o, rho, u, P, phi);
    orc_get_raw(o, rho, u, P, phi);
    orc_get_geometry(o, G, n, k, F);
    orc_get_accel(o, a, om);
    orc_sums(o, &m, &ph);
    orc_get_populations(o, f, g);
    int bad = !isfinite(m) || !isfinite(ph);
    for (long id = 0; id < 3 * N; ++id) bad |= !isfinite(u[id]);
    free(rho); free(u); free(P); free(phi); free(G); free(n); free(k); free(F); free(f); free(g); free(a); free(om);
    orc_free(o);
    return bad ? 3 : 0;
}

int main(void) {
    orc_params base;
    memset(&base, 0, sizeof base);
    base.nu = 0.05; base.sigma = 0.01; base.width = 3.0; base.eps = 1e-4;
    int rc = 0;
    orc_params p = base;  /* periodic droplet */
    p.nx = 12; p.ny = 10; p.nz = 9;
    rc |= run(&p, 5);
    p = base;             /* jet: free-slip sides, inlet, outflow */
    p.nx = 10; p.ny = 9; p.nz = 12;
    p.bc[0] = p.bc[1] = p.bc[2] = p.bc[3] = 1; p.bc[4] = 2; p.bc[5] = 3;
    p.inlet_u = 0.05; p.inlet_d = 4.0; p.inlet_noise = 0.01; p.seed = 3;
    rc |= run(&p, 6) << 2;
    p = base;             /* closed box: no-slip x, free-slip y, periodic z */
    p.nx = 8; p.ny = 9; p.nz = 6;
    p.bc[0] = p.bc[1] = 4; p.bc[2] = p.bc[3] = 1;
    rc |= run(&p, 4) << 4;
    p = base;             /* variable density with gravity in a no-slip box */
    p.nx = 10; p.ny = 8; p.nz = 10;
    for (int s = 0; s < 6; ++s) p.bc[s] = 4;
    p.vd = 1; p.rho_a = 5.0; p.rho_b = 1.0; p.nu_a = 0.08; p.nu_b = 0.02; p.grav[2] = -1e-5;
    rc |= run(&p, 5) << 6;
    p = base;             /* one plane, periodic */
    p.nx = 16; p.ny = 1; p.nz = 1;
    rc |= run(&p, 3) << 8;
    printf("oracle sanitised run: rc=%d\n", rc);
    return rc;
}
