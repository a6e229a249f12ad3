/*
 * FP64 CPU oracle for the multicomponent thread-safe lattice Boltzmann (TSLB)
 * time step of Montessori, Hegele Jr. and Lauricella, "A high-performance
 * lattice Boltzmann model for multicomponent turbulent jet simulations"
 * (arXiv:2403.15773).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes.  The thread-safe step is an algebraic rewrite (Methodology,
 * Eqs. 5, 6 and 8) of a plain lattice BGK scheme whose non-equilibrium part is
 * regularised by Hermite projection.  The rewrite changes the storage (moments
 * instead of populations) and the streaming direction (rebuild from neighbours
 * instead of push), not the trajectory.  So the oracle is that plain scheme,
 * written in populations, with two population arrays (A/B) and push streaming:
 *
 *   hydrodynamics  D3Q27, f_i^post = f_i^eq (Eq. 16, third-order Hermite
 *                  equilibrium) + (1 - omega) f_i^neq (Eq. 7 plus Eq. 19,
 *                  regularised up to third order with a^3 built from a^2 and u
 *                  as in Eq. 18) + S_i / 2 (Guo's forcing source),
 *   phase field    D3Q7, g_k^post = g_k^eq(phi, u) + Lambda_k (Eqs. 23, 24),
 *   interface      n = grad(phi)/|grad(phi)|, kappa = div(n),
 *                  F = -sigma kappa grad(phi) (Eqs. 20, 21),
 *   boundaries     moments imposed on one-node boundary layers and the rest
 *                  copied from the nearest interior node (Eqs. 9, 10).
 *
 * Readings of passages the paper leaves open (each one is also listed with its
 * reason in the design notes of the repository):
 *   - Eq. 19 is printed without the weight w_i and with c c in place of the
 *     second Hermite polynomial; the oracle multiplies by w_i (as Eq. 7 does)
 *     and uses H2 = c c - c_s^2 I.
 *   - Eq. 18's grouping is read as a^3_abg = u_a a^2_bg + u_b a^2_ag + u_g a^2_ab.
 *   - How the surface-tension force enters the lattice is not stated; Guo's
 *     forcing is used: u = (j + F/2)/rho, and the non-equilibrium tensor fed to
 *     the regularisation is P = Pi - rho c_s^2 I - rho u u + (u F + F u)/2.
 *   - Eq. 21 is read as n = grad(phi)/(|grad(phi)| + eps) and kappa = div(n);
 *     both derivatives use the isotropic D3Q27 stencil
 *     d(.) = (1/c_s^2) sum_i w_i c_i (.)(y + c_i).
 *   - D3Q7 weights 1/4 (rest) and 1/8, c_sphi^2 = 1/4; the anti-diffusion sign
 *     follows Eq. 24 (interface sharpening) with n pointing up the gradient.
 *   - gamma = 2/W unless given.
 *
 * Pins.  The bulk step is pinned by moment identities, closed forms and
 * physical laws (Laplace, shear-wave decay, conservation) in the test suite.
 * The boundary rules (boundary_values, fill_boundaries) are pinned rule by rule (each imposes
 * what Eqs. 9-10 state and copies the rest), but a bounded flow as a whole,
 * the jet, has no closed form or printed value to compare with: jet physics
 * is parity unpinned (the GPU path is compared with this oracle only).
 *
 * Variable density and viscosity (the paper's future work: both components have
 * the same density and viscosity in its model).  Selected by params.vd = 1; the
 * equal-density scheme above is untouched.  The scheme is the velocity-based
 * phase-field lattice Boltzmann formulation for immiscible fluids of different
 * density (Fakhari, Mitchell, Leonardi and Bolster, Phys. Rev. E 96, 053301,
 * 2017), restated in the regularised Hermite form used here:
 *   - the populations carry the normalised pressure p* and the velocity:
 *     sum f = 1 + p*, sum f c = ubar, and the Hermite equilibrium and
 *     regularised parts take unit density in their velocity terms,
 *     f^eq/w = 1 + p* + c.u/c_s^2 + H2:uu/(2 c_s^4) + H3:uuu/(6 c_s^6);
 *   - rho(phi) = rho_b + phi (rho_a - rho_b) and nu(phi) = nu_b + phi (nu_a - nu_b)
 *     (phi clamped to [0, 1]), omega(phi) = 1/(3 nu(phi) + 1/2), per node;
 *   - the forcing is the acceleration a = (F_s + F_p + F_mu)/rho(phi) + g, with
 *     F_s = -sigma kappa grad(phi) (Eq. 20), the pressure force
 *     F_p = -p* c_s^2 grad(rho) and the viscous force
 *     F_mu = rho nu (grad u + grad u^T) . grad(rho) / rho, taken from the raw
 *     non-equilibrium stress as F_mu = -(1 - omega/2) Q . grad(rho) with
 *     Q = Pi - (1 + p*) c_s^2 I - ubar ubar; a = 0 on boundary layers;
 *   - Guo's forcing at unit density: u = ubar + a/2, P = Q + a a/4.
 * The pressure is p = rho(phi) p* c_s^2, so that at rest grad p = -sigma kappa
 * grad(phi) and a droplet keeps Laplace's pressure jump at any density ratio.
 *
 * Data layout: SoA, population i of node (x,y,z) at f[i*N + x + nx*(y + ny*z)].
 * Velocity i = (cx+1) + 3(cy+1) + 9(cz+1).  D3Q7 k = rest, +x, -x, +y, -y, +z, -z.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

enum { BC_PERIODIC = 0, BC_FREESLIP = 1, BC_INLET = 2, BC_OUTFLOW = 3, BC_NOSLIP = 4 };

typedef struct {
    int32_t nx, ny, nz;
    int32_t bc[6];          /* faces -x,+x,-y,+y,-z,+z */
    double nu;              /* kinematic viscosity; omega = 1/(3 nu + 1/2) */
    double sigma;           /* surface tension */
    double width;           /* interface width W */
    double gamma;           /* anti-diffusion constant; <= 0 means 2/W */
    double eps;             /* regulariser of |grad phi| */
    double inlet_u, inlet_d, inlet_noise;
    uint64_t seed;
    int32_t vd;             /* 1: variable density and viscosity (see the header) */
    double rho_a, rho_b;    /* densities of component A (phi = 1) and B (phi = 0) */
    double nu_a, nu_b;      /* their kinematic viscosities */
    double grav[3];         /* body acceleration g */
} orc_params;

typedef struct {
    orc_params p;
    long N;
    double omega, gamma;
    long step;
    int has_bnd;
    double *f, *fn, *g, *gn;                 /* populations, A/B */
    double *rho, *j, *Pi, *phi;             /* moments: rho, j (3N), Pi (6N: xx,yy,zz,xy,xz,yz), phi */
    double *G, *n, *kappa, *F;               /* geometry: G (3N), n (3N), kappa, F (3N) */
    double *acc, *om;                        /* variable density: acceleration a (3N), omega (N) */
} orc;

/* ---- lattices (Fig. of the D3Q27 set; D3Q7 of the interface equation) ---- */

static const double CS2 = 1.0 / 3.0;      /* c_s^2 of D3Q27 */
static const double CS2_PHI = 0.25;       /* c_s^2 of D3Q7 with weights 1/4, 1/8 */

static int C27[27][3];
static double W27[27];
static double H2T[27][3][3];              /* H2_ab(c_i) = c_a c_b - c_s^2 d_ab */
static double H3T[27][3][3][3];           /* H3_abg(c_i) = c_a c_b c_g - c_s^2 (c_g d_ab + c_a d_bg + c_b d_ag) */
/* nonzero entries of H3(c_i), listed once so the contractions below skip the zeros */
static int H3NZ[27];
static int H3IDX[27][27][3];
static const int C7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const double W7[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
static int lattice_ready = 0;

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

static void lattice_init(void) {
    if (lattice_ready) return;
    for (int i = 0; i < 27; ++i) {
        int c[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
        int s = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        for (int a = 0; a < 3; ++a) C27[i][a] = c[a];
        W27[i] = s == 0 ? 8.0 / 27.0 : s == 1 ? 2.0 / 27.0 : s == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                H2T[i][a][b] = c[a] * c[b] - CS2 * kd(a, b);
                for (int g = 0; g < 3; ++g)
                    H3T[i][a][b][g] = (double)(c[a] * c[b] * c[g]) -
                                      CS2 * (c[g] * kd(a, b) + c[a] * kd(b, g) + c[b] * kd(a, g));
            }
    }
    for (int i = 0; i < 27; ++i) {
        H3NZ[i] = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int g = 0; g < 3; ++g)
                    if (H3T[i][a][b][g] != 0.0) {
                        H3IDX[i][H3NZ[i]][0] = a; H3IDX[i][H3NZ[i]][1] = b; H3IDX[i][H3NZ[i]][2] = g;
                        H3NZ[i]++;
                    }
    }
    lattice_ready = 1;
}

/* symmetric 3x3 from the 6-vector xx,yy,zz,xy,xz,yz */
static void sym_expand(const double s[6], double m[3][3]) {
    m[0][0] = s[0]; m[1][1] = s[1]; m[2][2] = s[2];
    m[0][1] = m[1][0] = s[3];
    m[0][2] = m[2][0] = s[4];
    m[1][2] = m[2][1] = s[5];
}

static const int SYM_A[6] = {0, 1, 2, 0, 0, 1};
static const int SYM_B[6] = {0, 1, 2, 1, 2, 2};

/* ---- counter-based noise: SplitMix64 finaliser (Steele, Lea, Flood 2014) ---- */

static uint64_t splitmix_finalise(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* First SplitMix64 output of state s (state advanced by the golden gamma). */
uint64_t orc_splitmix64_next(uint64_t s) { return splitmix_finalise(s + 0x9e3779b97f4a7c15ULL); }

/* Uniform xi in [-1, 1) with 24 random bits, exact in binary32 and binary64.
 * counter = stream*2^62 + step*2^32 + node*4 + comp. */
double orc_noise(uint64_t seed, uint64_t stream, uint64_t step, uint64_t node, uint64_t comp) {
    uint64_t key = orc_splitmix64_next(seed);
    uint64_t ctr = (stream << 62) + (step << 32) + (node << 2) + comp;
    uint64_t h = splitmix_finalise(key ^ ctr);
    return (double)(h >> 40) * (1.0 / 8388608.0) - 1.0;
}

/* ---- single-node operators ---- */

/* Hydrodynamic post-collision populations at one node.
 *   f^eq   Eq. 16 (third-order Hermite equilibrium; a^n_eq = a^{n-1}_eq u, Eq. 15)
 *   f^neq  Eq. 7 + Eq. 19 with w_i and H2, a^2 = P, a^3 = u (x) P symmetrised (Eq. 18)
 *   S/2    half of Guo's source S_i = w_i [(c - u).F / c_s^2 + (c.u)(c.F) / c_s^4]
 * f^post = f^eq + (1 - omega) f^neq + S/2 is f^eq + (1-omega) Proj(f - f^eq)
 * + (1 - omega/2) S with Proj including the first-order part -F/2 of f - f^eq. */
void orc_collide(double rho, const double u[3], const double Ps[6], const double F[3], double omega,
                 double f[27]) {
    lattice_init();
    double P[3][3], a3[3][3][3];
    sym_expand(Ps, P);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int g = 0; g < 3; ++g) a3[a][b][g] = u[a] * P[b][g] + u[b] * P[a][g] + u[g] * P[a][b];
    const double cs4 = CS2 * CS2, cs6 = cs4 * CS2;
    for (int i = 0; i < 27; ++i) {
        const int *c = C27[i];
        double h1u = 0.0, h2uu = 0.0, h3uuu = 0.0, h2P = 0.0, h3a3 = 0.0, cF = 0.0, uF = 0.0, cu = 0.0;
        for (int a = 0; a < 3; ++a) {
            h1u += c[a] * u[a];
            cF += c[a] * F[a];
            uF += u[a] * F[a];
            for (int b = 0; b < 3; ++b) {
                h2uu += H2T[i][a][b] * u[a] * u[b];
                h2P += H2T[i][a][b] * P[a][b];
            }
        }
        for (int m = 0; m < H3NZ[i]; ++m) {
            int a = H3IDX[i][m][0], b = H3IDX[i][m][1], g = H3IDX[i][m][2];
            h3uuu += H3T[i][a][b][g] * u[a] * u[b] * u[g];
            h3a3 += H3T[i][a][b][g] * a3[a][b][g];
        }
        cu = h1u;
        double feq = W27[i] * rho * (1.0 + h1u / CS2 + h2uu / (2.0 * cs4) + h3uuu / (6.0 * cs6));
        double fneq = W27[i] * (h2P / (2.0 * cs4) + h3a3 / (6.0 * cs6));
        double S = W27[i] * ((cF - uF) / CS2 + cu * cF / cs4);
        f[i] = feq + (1.0 - omega) * fneq + 0.5 * S;
    }
}

/* The same collision with unit density in the velocity terms (variable-density
 * scheme): f^post = w [rho + c.u/c_s^2 + H2:uu/(2 c_s^4) + H3:uuu/(6 c_s^6)]
 * + (1 - omega) f^neq(P) + S(a)/2, rho = 1 + p*, a the acceleration. */
void orc_collide_vd(double rho, const double u[3], const double Ps[6], const double a[3], double omega,
                    double f[27]) {
    lattice_init();
    double P[3][3], a3[3][3][3];
    sym_expand(Ps, P);
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y)
            for (int z = 0; z < 3; ++z) a3[x][y][z] = u[x] * P[y][z] + u[y] * P[x][z] + u[z] * P[x][y];
    const double cs4 = CS2 * CS2, cs6 = cs4 * CS2;
    for (int i = 0; i < 27; ++i) {
        const int *c = C27[i];
        double h1u = 0.0, h2uu = 0.0, h3uuu = 0.0, h2P = 0.0, h3a3 = 0.0, ca = 0.0, ua = 0.0;
        for (int x = 0; x < 3; ++x) {
            h1u += c[x] * u[x];
            ca += c[x] * a[x];
            ua += u[x] * a[x];
            for (int y = 0; y < 3; ++y) {
                h2uu += H2T[i][x][y] * u[x] * u[y];
                h2P += H2T[i][x][y] * P[x][y];
            }
        }
        for (int m = 0; m < H3NZ[i]; ++m) {
            int x = H3IDX[i][m][0], y = H3IDX[i][m][1], z = H3IDX[i][m][2];
            h3uuu += H3T[i][x][y][z] * u[x] * u[y] * u[z];
            h3a3 += H3T[i][x][y][z] * a3[x][y][z];
        }
        double feq = W27[i] * (rho + h1u / CS2 + h2uu / (2.0 * cs4) + h3uuu / (6.0 * cs6));
        double fneq = W27[i] * (h2P / (2.0 * cs4) + h3a3 / (6.0 * cs6));
        double S = W27[i] * ((ca - ua) / CS2 + h1u * ca / cs4);
        f[i] = feq + (1.0 - omega) * fneq + 0.5 * S;
    }
}

/* Phase-field post-collision populations (Eqs. 23, 24): first-order equilibrium
 * w_k phi (1 + c_k.u / c_sphi^2), unit relaxation, plus Lambda_k = w_k gamma phi (1-phi) c_k.n. */
void orc_phase_collide(double phi, const double u[3], const double n[3], double gamma, double g[7]) {
    for (int k = 0; k < 7; ++k) {
        double cu = C7[k][0] * u[0] + C7[k][1] * u[1] + C7[k][2] * u[2];
        double cn = C7[k][0] * n[0] + C7[k][1] * n[1] + C7[k][2] * n[2];
        g[k] = W7[k] * phi * (1.0 + cu / CS2_PHI) + W7[k] * gamma * phi * (1.0 - phi) * cn;
    }
}

/* ---- lattice helpers ---- */

static long node_index(const orc *o, int x, int y, int z) {
    return x + (long)o->p.nx * (y + (long)o->p.ny * z);
}

static int axis_periodic(const orc *o, int axis) { return o->p.bc[2 * axis] == BC_PERIODIC; }

static int axis_len(const orc *o, int axis) { return axis == 0 ? o->p.nx : axis == 1 ? o->p.ny : o->p.nz; }

/* Neighbour coordinate on one axis: wrapped when periodic, clamped otherwise. */
static int coord_wrap_clamp(const orc *o, int axis, int v) {
    int n = axis_len(o, axis);  /* v is at most one node outside [0, n) */
    if (axis_periodic(o, axis)) return v < 0 ? v + n : v >= n ? v - n : v;
    return v < 0 ? 0 : v >= n ? n - 1 : v;
}

static int is_boundary(const orc *o, int x, int y, int z) {
    int v[3] = {x, y, z};
    for (int a = 0; a < 3; ++a)
        if (!axis_periodic(o, a) && (v[a] == 0 || v[a] == axis_len(o, a) - 1)) return 1;
    return 0;
}

/* ---- moments ---- */

static void node_moments(const orc *o, const double *f, const double *g, long id, double *rho, double j[3],
                         double Pi[6], double *phi) {
    double r = 0.0, jj[3] = {0, 0, 0}, pp[6] = {0, 0, 0, 0, 0, 0}, ph = 0.0;
    for (int i = 0; i < 27; ++i) {
        double fi = f[(long)i * o->N + id];
        r += fi;
        for (int a = 0; a < 3; ++a) jj[a] += fi * C27[i][a];
        for (int s = 0; s < 6; ++s) pp[s] += fi * C27[i][SYM_A[s]] * C27[i][SYM_B[s]];
    }
    for (int k = 0; k < 7; ++k) ph += g[(long)k * o->N + id];
    *rho = r;
    for (int a = 0; a < 3; ++a) j[a] = jj[a];
    for (int s = 0; s < 6; ++s) Pi[s] = pp[s];
    *phi = ph;
}

static void compute_moments(orc *o) {
    const int nx = o->p.nx, ny = o->p.ny, nz = o->p.nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = node_index(o, x, y, z);
                double r, j[3], Pi[6], ph;
                node_moments(o, o->f, o->g, id, &r, j, Pi, &ph);
                o->rho[id] = r;
                for (int a = 0; a < 3; ++a) o->j[3 * id + a] = j[a];
                for (int s = 0; s < 6; ++s) o->Pi[6 * id + s] = Pi[s];
                o->phi[id] = ph;
            }
}

/* Populations carrying exactly (rho, j, Pi): second-order Hermite projection
 * f_i = w_i [rho + c.j / c_s^2 + H2:(Pi - rho c_s^2 I) / (2 c_s^4)]. */
static void project_h2(double rho, const double j[3], const double Pis[6], double f[27]) {
    double Pi[3][3];
    sym_expand(Pis, Pi);
    for (int a = 0; a < 3; ++a) Pi[a][a] -= rho * CS2;
    for (int i = 0; i < 27; ++i) {
        double cj = 0.0, h2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            cj += C27[i][a] * j[a];
            for (int b = 0; b < 3; ++b) h2 += H2T[i][a][b] * Pi[a][b];
        }
        f[i] = W27[i] * (rho + cj / CS2 + h2 / (2.0 * CS2 * CS2));
    }
}

/* ---- interface geometry (Eqs. 20, 21) ---- */

static void compute_geometry(orc *o) {
    const int nx = o->p.nx, ny = o->p.ny, nz = o->p.nz;
    const double eps = o->p.eps;
    /* G = (1/c_s^2) sum_i w_i c_i phi(y + c_i), phi index clamped on walls */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = node_index(o, x, y, z);
                double G[3] = {0, 0, 0};
                for (int i = 0; i < 27; ++i) {
                    int xs = coord_wrap_clamp(o, 0, x + C27[i][0]);
                    int ys = coord_wrap_clamp(o, 1, y + C27[i][1]);
                    int zs = coord_wrap_clamp(o, 2, z + C27[i][2]);
                    double ph = o->phi[node_index(o, xs, ys, zs)];
                    for (int a = 0; a < 3; ++a) G[a] += W27[i] * C27[i][a] * ph / CS2;
                }
                double mag = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
                for (int a = 0; a < 3; ++a) {
                    o->G[3 * id + a] = G[a];
                    o->n[3 * id + a] = G[a] / (mag + eps);
                }
            }
    /* kappa = div n with the same stencil; F = -sigma kappa G; F = 0 on boundary layers */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = node_index(o, x, y, z);
                double k = 0.0;
                for (int i = 0; i < 27; ++i) {
                    int xs = coord_wrap_clamp(o, 0, x + C27[i][0]);
                    int ys = coord_wrap_clamp(o, 1, y + C27[i][1]);
                    int zs = coord_wrap_clamp(o, 2, z + C27[i][2]);
                    long s = node_index(o, xs, ys, zs);
                    for (int a = 0; a < 3; ++a) k += W27[i] * C27[i][a] * o->n[3 * s + a] / CS2;
                }
                o->kappa[id] = k;
                int bnd = is_boundary(o, x, y, z);
                for (int a = 0; a < 3; ++a) o->F[3 * id + a] = bnd ? 0.0 : -o->p.sigma * k * o->G[3 * id + a];
            }
}

/* ---- boundary layers (Eqs. 9, 10) ---- */

/* Smooth nozzle indicator s(r) = (1 - tanh(2 (r - D/2) / W)) / 2. */
static double nozzle_profile(const orc *o, int x, int y) {
    double dx = x - 0.5 * (o->p.nx - 1), dy = y - 0.5 * (o->p.ny - 1);
    double r = sqrt(dx * dx + dy * dy);
    return 0.5 * (1.0 - tanh(2.0 * (r - 0.5 * o->p.inlet_d) / o->p.width));
}

/* Which face rule governs a boundary node (z faces first, then y, then x). */
static int boundary_face(const orc *o, int x, int y, int z) {
    int v[3] = {x, y, z};
    for (int a = 2; a >= 0; --a) {
        if (axis_periodic(o, a)) continue;
        if (v[a] == 0) return 2 * a;
        if (v[a] == axis_len(o, a) - 1) return 2 * a + 1;
    }
    return -1;
}

/* Raw moments (rho, ubar = j/rho, Q = Pi - rho c_s^2 I - j j / rho, phi) imposed
 * on boundary node (x,y,z): the equilibrium part from the imposed rho and/or u,
 * the non-equilibrium part Q copied from the nearest interior node x_F. */
static void boundary_values(const orc *o, int x, int y, int z, double *rho, double ub[3], double Q[6],
                            double *phi) {
    int face = boundary_face(o, x, y, z);
    int axis = face / 2;
    int v[3] = {x, y, z};
    for (int a = 0; a < 3; ++a)
        if (!axis_periodic(o, a)) {
            int n = axis_len(o, a);
            v[a] = v[a] < 1 ? 1 : v[a] > n - 2 ? n - 2 : v[a];
        }
    long idF = node_index(o, v[0], v[1], v[2]);
    double r, j[3], Pi[6], ph;
    node_moments(o, o->f, o->g, idF, &r, j, Pi, &ph);
    const double dm = o->p.vd ? 1.0 : r;  /* density in the velocity terms */
    for (int a = 0; a < 3; ++a) ub[a] = j[a] / dm;
    for (int s = 0; s < 6; ++s)
        Q[s] = Pi[s] - (SYM_A[s] == SYM_B[s] ? r * CS2 : 0.0) - j[SYM_A[s]] * j[SYM_B[s]] / dm;
    *rho = r;
    *phi = ph;
    switch (o->p.bc[face]) {
    case BC_FREESLIP:
        ub[axis] = 0.0;
        for (int s = 3; s < 6; ++s)
            if (SYM_A[s] == axis || SYM_B[s] == axis) Q[s] = 0.0;
        break;
    case BC_NOSLIP:
        ub[0] = ub[1] = ub[2] = 0.0;
        break;
    case BC_OUTFLOW:
        *rho = 1.0;
        break;
    case BC_INLET: {
        double s = nozzle_profile(o, x, y);
        double xi = orc_noise(o->p.seed, 1, (uint64_t)o->step, (uint64_t)(x + (long)o->p.nx * y), 2);
        ub[0] = ub[1] = 0.0;
        ub[2] = o->p.inlet_u * s * (1.0 + o->p.inlet_noise * xi);
        *phi = s;
        break;
    }
    default:
        break;
    }
}

static void fill_boundaries(orc *o) {
    const int nx = o->p.nx, ny = o->p.ny, nz = o->p.nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!is_boundary(o, x, y, z)) continue;
                double r, ub[3], Q[6], ph, j[3], Pi[6], f[27];
                boundary_values(o, x, y, z, &r, ub, Q, &ph);
                const double dm = o->p.vd ? 1.0 : r;
                for (int a = 0; a < 3; ++a) j[a] = dm * ub[a];
                for (int s = 0; s < 6; ++s)
                    Pi[s] = Q[s] + (SYM_A[s] == SYM_B[s] ? r * CS2 : 0.0) + j[SYM_A[s]] * j[SYM_B[s]] / dm;
                project_h2(r, j, Pi, f);
                long id = node_index(o, x, y, z);
                for (int i = 0; i < 27; ++i) o->f[(long)i * o->N + id] = f[i];
                for (int k = 0; k < 7; ++k) o->g[(long)k * o->N + id] = W7[k] * ph;
            }
}

/* ---- the time step ---- */

/* Guo macroscopic velocity and forcing-corrected non-equilibrium tensor at a node. */
static void macroscopic(const orc *o, long id, double *rho, double u[3], double P[6]) {
    double r = o->rho[id];
    const double *j = o->j + 3 * id, *F = o->F + 3 * id, *Pi = o->Pi + 6 * id;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / r;
    for (int s = 0; s < 6; ++s) {
        int a = SYM_A[s], b = SYM_B[s];
        P[s] = Pi[s] - (a == b ? r * CS2 : 0.0) - r * u[a] * u[b] + 0.5 * (u[a] * F[b] + F[a] * u[b]);
    }
    *rho = r;
}

/* ---- variable density and viscosity ---- */

/* rho(phi), omega(phi) of the variable-density scheme (phi clamped to [0, 1]). */
static void vd_props(const orc *o, double phi, double *rho_phi, double *omega) {
    double c = phi < 0.0 ? 0.0 : phi > 1.0 ? 1.0 : phi;
    *rho_phi = o->p.rho_b + c * (o->p.rho_a - o->p.rho_b);
    double nu = o->p.nu_b + c * (o->p.nu_a - o->p.nu_b);
    *omega = 1.0 / (3.0 * nu + 0.5);
}

/* Acceleration of one interior node from its pressure p* = rho - 1, raw stress
 * Q, grad(phi) G and surface-tension force Fs:
 * a = (Fs - p* c_s^2 drho G - (1 - omega/2) drho Q.G) / rho(phi) + g. */
static void vd_accel(const orc *o, double pstar, const double Q[6], const double G[3], const double Fs[3],
                     double rho_phi, double omega, double a[3]) {
    const double drho = o->p.rho_a - o->p.rho_b;
    double Qm[3][3];
    sym_expand(Q, Qm);
    for (int x = 0; x < 3; ++x) {
        double QG = Qm[x][0] * G[0] + Qm[x][1] * G[1] + Qm[x][2] * G[2];
        double F = Fs[x] - pstar * CS2 * drho * G[x] - (1.0 - 0.5 * omega) * drho * QG;
        a[x] = F / rho_phi + o->p.grav[x];
    }
}

/* Per-node omega and acceleration of the current moments and geometry. */
static void compute_accel(orc *o) {
    const int nx = o->p.nx, ny = o->p.ny, nz = o->p.nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = node_index(o, x, y, z);
                double rp, om;
                vd_props(o, o->phi[id], &rp, &om);
                o->om[id] = om;
                double *a = o->acc + 3 * id;
                if (is_boundary(o, x, y, z)) {
                    a[0] = a[1] = a[2] = 0.0;
                    continue;
                }
                const double r = o->rho[id], *j = o->j + 3 * id, *Pi = o->Pi + 6 * id;
                double Q[6];
                for (int s = 0; s < 6; ++s)
                    Q[s] = Pi[s] - (SYM_A[s] == SYM_B[s] ? r * CS2 : 0.0) - j[SYM_A[s]] * j[SYM_B[s]];
                vd_accel(o, r - 1.0, Q, o->G + 3 * id, o->F + 3 * id, rp, om, a);
            }
}

/* Guo velocity and forcing-corrected tensor at unit density (variable density):
 * u = ubar + a/2, P = Pi - rho c_s^2 I - u u + (u a + a u)/2. */
static void macroscopic_vd(const orc *o, long id, double *rho, double u[3], double P[6]) {
    double r = o->rho[id];
    const double *j = o->j + 3 * id, *a = o->acc + 3 * id, *Pi = o->Pi + 6 * id;
    for (int x = 0; x < 3; ++x) u[x] = j[x] + 0.5 * a[x];
    for (int s = 0; s < 6; ++s) {
        int x = SYM_A[s], y = SYM_B[s];
        P[s] = Pi[s] - (x == y ? r * CS2 : 0.0) - u[x] * u[y] + 0.5 * (u[x] * a[y] + a[x] * u[y]);
    }
    *rho = r;
}

static void step_once(orc *o) {
    const int nx = o->p.nx, ny = o->p.ny, nz = o->p.nz;
    if (o->has_bnd) fill_boundaries(o);
    compute_moments(o);
    compute_geometry(o);
    if (o->p.vd) compute_accel(o);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = node_index(o, x, y, z);
                double r, u[3], P[6], fp[27], gp[7];
                if (o->p.vd) {
                    macroscopic_vd(o, id, &r, u, P);
                    orc_collide_vd(r, u, P, o->acc + 3 * id, o->om[id], fp);
                } else {
                    macroscopic(o, id, &r, u, P);
                    orc_collide(r, u, P, o->F + 3 * id, o->omega, fp);
                }
                orc_phase_collide(o->phi[id], u, o->n + 3 * id, o->gamma, gp);
                /* push: f_i(y + c_i, t+1) = f_i^post(y, t) (Eq. 6); interior destinations only */
                for (int i = 0; i < 27; ++i) {
                    int d[3] = {x + C27[i][0], y + C27[i][1], z + C27[i][2]};
                    int ok = 1;
                    for (int a = 0; a < 3; ++a) {
                        int n = axis_len(o, a);
                        if (axis_periodic(o, a)) d[a] = d[a] < 0 ? d[a] + n : d[a] >= n ? d[a] - n : d[a];
                        else if (d[a] < 1 || d[a] > n - 2) ok = 0;
                    }
                    if (ok) o->fn[(long)i * o->N + node_index(o, d[0], d[1], d[2])] = fp[i];
                }
                for (int k = 0; k < 7; ++k) {
                    int d[3] = {x + C7[k][0], y + C7[k][1], z + C7[k][2]};
                    int ok = 1;
                    for (int a = 0; a < 3; ++a) {
                        int n = axis_len(o, a);
                        if (axis_periodic(o, a)) d[a] = d[a] < 0 ? d[a] + n : d[a] >= n ? d[a] - n : d[a];
                        else if (d[a] < 1 || d[a] > n - 2) ok = 0;
                    }
                    if (ok) o->gn[(long)k * o->N + node_index(o, d[0], d[1], d[2])] = gp[k];
                }
            }
    double *t = o->f; o->f = o->fn; o->fn = t;
    t = o->g; o->g = o->gn; o->gn = t;
    o->step += 1;
}

/* ---- public entry points (ctypes) ---- */

void orc_lattice(int32_t c27[81], double w27[27], int32_t c7[21], double w7[7]) {
    lattice_init();
    for (int i = 0; i < 27; ++i) {
        for (int a = 0; a < 3; ++a) c27[3 * i + a] = C27[i][a];
        w27[i] = W27[i];
    }
    for (int k = 0; k < 7; ++k) {
        for (int a = 0; a < 3; ++a) c7[3 * k + a] = C7[k][a];
        w7[k] = W7[k];
    }
}

static int params_valid(const orc_params *p) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
    if (!(p->nu > 0.0) || !(p->sigma >= 0.0) || !(p->width > 0.0) || !(p->eps >= 0.0)) return 0;
    for (int a = 0; a < 3; ++a) {
        int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
        int n = a == 0 ? p->nx : a == 1 ? p->ny : p->nz;
        if ((lo == BC_PERIODIC) != (hi == BC_PERIODIC)) return 0;
        if (lo != BC_PERIODIC && n < 4) return 0;
        for (int s = 0; s < 2; ++s) {
            int b = p->bc[2 * a + s];
            if (b < 0 || b > 4) return 0;
            if (b == BC_INLET && !(a == 2 && s == 0)) return 0;
        }
    }
    double omega = 1.0 / (3.0 * p->nu + 0.5);
    if (p->vd) {
        if (p->vd != 1 || !(p->rho_a > 0.0) || !(p->rho_b > 0.0) || !(p->nu_a > 0.0) || !(p->nu_b > 0.0)) return 0;
        if (!(1.0 / (3.0 * p->nu_a + 0.5) < 2.0) || !(1.0 / (3.0 * p->nu_b + 0.5) < 2.0)) return 0;
        for (int a = 0; a < 3; ++a)
            if (!isfinite(p->grav[a])) return 0;
    }
    return omega < 2.0;
}

void orc_free(orc *o) {
    if (!o) return;
    free(o->f); free(o->fn); free(o->g); free(o->gn);
    free(o->rho); free(o->j); free(o->Pi); free(o->phi);
    free(o->G); free(o->n); free(o->kappa); free(o->F);
    free(o->acc); free(o->om);
    free(o);
}

int orc_create(const orc_params *p, orc **out) {
    lattice_init();
    *out = NULL;
    if (!params_valid(p)) return ORC_EINVAL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    if (!o) return ORC_ENOMEM;
    o->p = *p;
    o->N = (long)p->nx * p->ny * p->nz;
    o->omega = 1.0 / (3.0 * p->nu + 0.5);  /* nu = c_s^2 (1/omega - 1/2) */
    o->gamma = p->gamma > 0.0 ? p->gamma : 2.0 / p->width;
    o->has_bnd = 0;
    for (int s = 0; s < 6; ++s) o->has_bnd |= p->bc[s] != BC_PERIODIC;
    long N = o->N;
    o->f = malloc(sizeof(double) * 27 * N); o->fn = malloc(sizeof(double) * 27 * N);
    o->g = malloc(sizeof(double) * 7 * N); o->gn = malloc(sizeof(double) * 7 * N);
    o->rho = malloc(sizeof(double) * N); o->j = malloc(sizeof(double) * 3 * N);
    o->Pi = malloc(sizeof(double) * 6 * N); o->phi = malloc(sizeof(double) * N);
    o->G = malloc(sizeof(double) * 3 * N); o->n = malloc(sizeof(double) * 3 * N);
    o->kappa = malloc(sizeof(double) * N); o->F = malloc(sizeof(double) * 3 * N);
    o->acc = calloc(3 * (size_t)N, sizeof(double)); o->om = calloc((size_t)N, sizeof(double));
    if (!o->f || !o->fn || !o->g || !o->gn || !o->rho || !o->j || !o->Pi || !o->phi || !o->G || !o->n ||
        !o->kappa || !o->F || !o->acc || !o->om) {
        orc_free(o);
        return ORC_ENOMEM;
    }
    memset(o->fn, 0, sizeof(double) * 27 * N);
    memset(o->gn, 0, sizeof(double) * 7 * N);
    *out = o;
    return ORC_OK;
}

double orc_omega(const orc *o) { return o->omega; }
double orc_gamma(const orc *o) { return o->gamma; }
long orc_step_count(const orc *o) { return o->step; }

/* Initial state from physical fields (rho, u (3N, SoA), P (6N, SoA), phi):
 * F0 from phi; j = rho u - F0/2; Pi = P + rho c_s^2 I + rho u u - (u F0 + F0 u)/2;
 * f = Hermite-2 projection of (rho, j, Pi); g_k = w_k phi. */
void orc_set_physical(orc *o, const double *rho, const double *u, const double *P, const double *phi,
                      int64_t step) {
    const long N = o->N;
    memcpy(o->phi, phi, sizeof(double) * N);
    compute_geometry(o);
    if (o->p.vd) {
        /* variable density: rho = 1 + p*.  The acceleration depends on the raw
         * stress Q = P - a a/4 through F_mu, so (a, Q) is the fixed point of that
         * pair, reached to rounding in a few sweeps (a is small); then
         * ubar = u - a/2 and Pi = Q + rho c_s^2 I + ubar ubar. */
        const int nx = o->p.nx, ny = o->p.ny;
#pragma omp parallel for schedule(static)
        for (long id = 0; id < N; ++id) {
            const int x = (int)(id % nx), y = (int)((id / nx) % ny), z = (int)(id / ((long)nx * ny));
            double r = rho[id], uu[3], Q[6], a[3] = {0, 0, 0}, j[3], Pi[6], f[27], rp, om;
            for (int c = 0; c < 3; ++c) uu[c] = u[c * N + id];
            vd_props(o, phi[id], &rp, &om);
            const int bnd = is_boundary(o, x, y, z);
            for (int it = 0; it < 4; ++it) {
                for (int s = 0; s < 6; ++s) Q[s] = P[s * N + id] - 0.25 * a[SYM_A[s]] * a[SYM_B[s]];
                if (!bnd) vd_accel(o, r - 1.0, Q, o->G + 3 * id, o->F + 3 * id, rp, om, a);
            }
            for (int s = 0; s < 6; ++s) Q[s] = P[s * N + id] - 0.25 * a[SYM_A[s]] * a[SYM_B[s]];
            for (int c = 0; c < 3; ++c) j[c] = uu[c] - 0.5 * a[c];
            for (int s = 0; s < 6; ++s)
                Pi[s] = Q[s] + (SYM_A[s] == SYM_B[s] ? r * CS2 : 0.0) + j[SYM_A[s]] * j[SYM_B[s]];
            project_h2(r, j, Pi, f);
            for (int i = 0; i < 27; ++i) o->f[(long)i * N + id] = f[i];
            for (int k = 0; k < 7; ++k) o->g[(long)k * N + id] = W7[k] * phi[id];
        }
        o->step = step;
        return;
    }
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        double r = rho[id], uu[3], j[3], Pi[6], f[27];
        const double *F = o->F + 3 * id;
        for (int a = 0; a < 3; ++a) { uu[a] = u[a * N + id]; j[a] = r * uu[a] - 0.5 * F[a]; }
        for (int s = 0; s < 6; ++s) {
            int a = SYM_A[s], b = SYM_B[s];
            Pi[s] = P[s * N + id] + (a == b ? r * CS2 : 0.0) + r * uu[a] * uu[b] - 0.5 * (uu[a] * F[b] + F[a] * uu[b]);
        }
        project_h2(r, j, Pi, f);
        for (int i = 0; i < 27; ++i) o->f[(long)i * N + id] = f[i];
        for (int k = 0; k < 7; ++k) o->g[(long)k * N + id] = W7[k] * phi[id];
    }
    o->step = step;
}

void orc_step(orc *o, int64_t nsteps) {
    for (int64_t s = 0; s < nsteps; ++s) step_once(o);
}

/* Current state with boundary layers filled: moments and geometry refreshed. */
static void refresh(orc *o) {
    if (o->has_bnd) fill_boundaries(o);
    compute_moments(o);
    compute_geometry(o);
    if (o->p.vd) compute_accel(o);
}

/* Physical moments: rho, u = (j + F/2)/rho, P = Pi - rho c_s^2 I - rho u u + (uF + Fu)/2, phi. */
void orc_get_physical(orc *o, double *rho, double *u, double *P, double *phi) {
    refresh(o);
    const long N = o->N;
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        double r, uu[3], Ps[6];
        if (o->p.vd)
            macroscopic_vd(o, id, &r, uu, Ps);
        else
            macroscopic(o, id, &r, uu, Ps);
        if (rho) rho[id] = r;
        for (int a = 0; a < 3; ++a) if (u) u[a * N + id] = uu[a];
        for (int s = 0; s < 6; ++s) if (P) P[s * N + id] = Ps[s];
        if (phi) phi[id] = o->phi[id];
    }
}

/* Raw moments: rho - 1, ubar = j/rho, Q = Pi - rho c_s^2 I - j j / rho, phi (with
 * unit density in place of rho in ubar and Q in the variable-density scheme). */
void orc_get_raw(orc *o, double *drho, double *ub, double *Q, double *phi) {
    refresh(o);
    const long N = o->N;
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        double r = o->rho[id];
        const double *j = o->j + 3 * id, *Pi = o->Pi + 6 * id;
        const double dm = o->p.vd ? 1.0 : r;
        drho[id] = r - 1.0;
        for (int a = 0; a < 3; ++a) ub[a * N + id] = j[a] / dm;
        for (int s = 0; s < 6; ++s) {
            int a = SYM_A[s], b = SYM_B[s];
            Q[s * N + id] = Pi[s] - (a == b ? r * CS2 : 0.0) - j[a] * j[b] / dm;
        }
        phi[id] = o->phi[id];
    }
}

/* Geometry of the current state: G (3N), n (3N), kappa (N), F (3N), all SoA. */
void orc_get_geometry(orc *o, double *G, double *n, double *kappa, double *F) {
    refresh(o);
    const long N = o->N;
    for (long id = 0; id < N; ++id) {
        for (int a = 0; a < 3; ++a) {
            if (G) G[a * N + id] = o->G[3 * id + a];
            if (n) n[a * N + id] = o->n[3 * id + a];
            if (F) F[a * N + id] = o->F[3 * id + a];
        }
        if (kappa) kappa[id] = o->kappa[id];
    }
}

/* Variable-density acceleration a (3N, SoA) and omega (N) of the current state. */
void orc_get_accel(orc *o, double *a, double *omega) {
    refresh(o);
    const long N = o->N;
    for (long id = 0; id < N; ++id) {
        for (int c = 0; c < 3; ++c)
            if (a) a[c * N + id] = o->p.vd ? o->acc[3 * id + c] : 0.0;
        if (omega) omega[id] = o->p.vd ? o->om[id] : o->omega;
    }
}

/* Mass and phase sums of the current state (boundary layers filled). */
void orc_sums(orc *o, double *mass, double *phase) {
    refresh(o);
    double m = 0.0, ph = 0.0;
    for (long id = 0; id < o->N; ++id) { m += o->rho[id]; ph += o->phi[id]; }
    *mass = m;
    *phase = ph;
}

/* Raw populations, for tests: f (27N) and g (7N) of the current array. */
void orc_get_populations(const orc *o, double *f, double *g) {
    if (f) memcpy(f, o->f, sizeof(double) * 27 * o->N);
    if (g) memcpy(g, o->g, sizeof(double) * 7 * o->N);
}
