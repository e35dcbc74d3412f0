/*
 * lbm_oracle_3d.c -- plain, slow CPU reference of the TRT-R lattice Boltzmann model for the
 * convection-diffusion equation on the D3Q19 and D3Q27 lattices (the three-dimensional extension
 * that Sec. 2.2 of arXiv:2312.10316 calls straightforward).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may build, load or call it.  It
 * shares no code, header, table or constant with the HIP library and includes none of its files.
 *
 * The operations are those of the two-dimensional oracle with every index running over three
 * axes: Hermite tensors from e_i and the Kronecker delta, the full third-order Hermite equilibrium
 * (Eq. (6)), the TRT-R operator of Eq. (12) with the non-equilibrium moments of Eqs. (8) and (13),
 * the auxiliary term of Eq. (16) with central differences of the nodal u, the discrete source of
 * Eq. (3), and streaming on a lattice periodic in x, y and z (Eq. (14)).  Physical units (c = dx/dt).
 *
 * Readings where the paper is silent:
 *   - Velocities, in this order: 0:(0,0,0); 1,2:(+-1,0,0); 3,4:(0,+-1,0); 5,6:(0,0,+-1);
 *     7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0); 11:(1,0,1) 12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1);
 *     15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1) -- the D3Q19 set, weights 1/3, 1/18, 1/36 --
 *     and for D3Q27 also the corners 19:(1,1,1) 20:(-1,-1,-1) 21:(1,1,-1) 22:(-1,-1,1)
 *     23:(1,-1,1) 24:(-1,1,-1) 25:(-1,1,1) 26:(1,-1,-1), weights 8/27, 2/27, 1/54, 1/216
 *     (the tensor product of the one-dimensional weights 2/3, 1/6, 1/6); c_s^2 = c^2/3.
 *   - The third-order Hermite sum runs over all 27 index triples.  On both lattices H_xxx (and the
 *     like) vanish identically at every velocity; on D3Q19 H_xyz vanishes too, so only the
 *     xxy-type components contribute there, while D3Q27 keeps H_xyz.
 *   - Everything else as in the two-dimensional oracle (phi = sum g, fields at t_n and at the
 *     collision node, dS/dt supplied, u frozen within the step).
 */
#include <stdlib.h>
#include <string.h>

static const int EX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                           1, -1, 1, -1, 1, -1, -1, 1};
static const int EY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                           1, -1, 1, -1, -1, 1, 1, -1};
static const int EZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                           1, -1, -1, 1, 1, -1, 1, -1};
static const double W19[19] = {1.0 / 3.0,
                               1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double W27[27] = {8.0 / 27.0,
                               2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
                               1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
                               1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
                               1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0,
                               1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};

/* weights of the q-velocity lattice (q = 19 or 27) */
static const double *weights(int q) { return q == 27 ? W27 : W19; }

typedef struct orc3_problem {
    int nx, ny, nz;    /* periodic lattice, node (j, k, l) at index (l*ny + k)*nx + j */
    double dx, dt;     /* lattice spacing and time step; c = dx/dt */
    double lambda;     /* magic parameter Lambda = (tau1 - 1/2)(tau2 - 1/2) */
    double D_const;    /* kappa when no field is given */
    int aux;           /* 0: auxiliary term of Eq. (16); 2: none (1, the flux form, is two-dimensional only) */
    int q;             /* 19 (D3Q19) or 27 (D3Q27) */
} orc3_problem;

void orc3_lattice(int q, int *ex, int *ey, int *ez, double *w)
{
    const double *W = weights(q);
    for (int i = 0; i < q; ++i) { ex[i] = EX[i]; ey[i] = EY[i]; ez[i] = EZ[i]; w[i] = W[i]; }
}

static double ecomp(int i, int a, double c) { return c * (double)(a == 0 ? EX[i] : (a == 1 ? EY[i] : EZ[i])); }
static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }
static double herm2(int i, int a, int b, double c)
{
    double cs2 = c * c / 3.0;
    return ecomp(i, a, c) * ecomp(i, b, c) - cs2 * kd(a, b);
}
static double herm3(int i, int a, int b, int g, double c)
{
    double cs2 = c * c / 3.0;
    return ecomp(i, a, c) * ecomp(i, b, c) * ecomp(i, g, c)
         - cs2 * (ecomp(i, a, c) * kd(b, g) + ecomp(i, b, c) * kd(g, a) + ecomp(i, g, c) * kd(a, b));
}
static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Third-order Hermite equilibrium, Eq. (6), summed over all three axes. */
void orc3_equilibrium(int q, double phi, const double *u, double c, double *geq)
{
    const double *W = weights(q);
    double cs2 = c * c / 3.0;
    for (int i = 0; i < q; ++i) {
        double s1 = 0, s2 = 0, s3 = 0;
        for (int a = 0; a < 3; ++a) s1 += ecomp(i, a, c) * u[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) s2 += herm2(i, a, b, c) * u[a] * u[b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int g = 0; g < 3; ++g) s3 += herm3(i, a, b, g, c) * u[a] * u[b] * u[g];
        geq[i] = W[i] * phi * (1.0 + s1 / cs2 + s2 / (2.0 * cs2 * cs2) + s3 / (6.0 * cs2 * cs2 * cs2));
    }
}

/* TRT-R collision, Eq. (12), with B_a = sum_i H_a (g_i - g_eq_i) and B_ab = sum_i H_ab (g_i - g_eq_i). */
void orc3_collide(int q, const double *g, const double *u, double tau1, double tau2, double c, double *out)
{
    const double *W = weights(q);
    double cs2 = c * c / 3.0;
    double phi = 0;
    for (int i = 0; i < q; ++i) phi += g[i];
    double geq[27];
    orc3_equilibrium(q, phi, u, c, geq);
    double B1[3] = {0, 0, 0}, B2[3][3];
    memset(B2, 0, sizeof B2);
    for (int i = 0; i < q; ++i) {
        double gneq = g[i] - geq[i];
        for (int a = 0; a < 3; ++a) B1[a] += ecomp(i, a, c) * gneq;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) B2[a][b] += herm2(i, a, b, c) * gneq;
    }
    for (int i = 0; i < q; ++i) {
        double r1 = 0, r2 = 0;
        for (int a = 0; a < 3; ++a) r1 += ecomp(i, a, c) * B1[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) r2 += herm2(i, a, b, c) * B2[a][b];
        out[i] = geq[i] + (1.0 - 1.0 / tau1) * W[i] * r1 / cs2
                        + (1.0 - 1.0 / tau2) * W[i] * r2 / (2.0 * cs2 * cs2);
    }
}

/* g_i = g_eq_i(phi0, u) (the initial condition of Sec. 3).  u: [3][nz][ny][nx]. */
void orc3_init(const orc3_problem *p, const double *phi0, const double *u, double *g)
{
    size_t N = (size_t)p->nx * p->ny * p->nz;
    double c = p->dx / p->dt;
    for (size_t n = 0; n < N; ++n) {
        double un[3] = {u[n], u[N + n], u[2 * N + n]}, geq[27];
        orc3_equilibrium(p->q, phi0[n], un, c, geq);
        for (int i = 0; i < p->q; ++i) g[i * N + n] = geq[i];
    }
}

void orc3_phi(const orc3_problem *p, const double *g, double *phi)
{
    size_t N = (size_t)p->nx * p->ny * p->nz;
    for (size_t n = 0; n < N; ++n) {
        double s = 0;
        for (int i = 0; i < p->q; ++i) s += g[i * N + n];
        phi[n] = s;
    }
}

/* One step of Eq. (14) on the periodic lattice.  g_in / g_out: [q][nz][ny][nx]; u: [3][nz][ny][nx];
 * D, S, dSdt: [nz][ny][nx] or NULL. */
void orc3_step(const orc3_problem *p, const double *g_in, double *g_out, const double *u, const double *D,
               const double *S, const double *dSdt)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz, q = p->q;
    const double *W = weights(q);
    const size_t N = (size_t)nx * ny * nz;
    const double dx = p->dx, dt = p->dt, c = dx / dt, cs2 = c * c / 3.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = ((size_t)z * ny + y) * nx + x;
                double g[27], phi = 0;
                for (int i = 0; i < q; ++i) g[i] = g_in[i * N + n];
                for (int i = 0; i < q; ++i) phi += g[i];
                const double kappa = D ? D[n] : p->D_const;
                const double tau1 = 0.5 + kappa / (cs2 * dt);
                const double tau2 = 0.5 + p->lambda / (tau1 - 0.5);
                const double beta = 1.0 - 1.0 / (2.0 * tau1);
                const double un[3] = {u[n], u[N + n], u[2 * N + n]};
                double C[27];
                orc3_collide(q, g, un, tau1, tau2, c, C);

                /* Eq. (16): A_a = phi u_b d_b u_a, d_b the central difference of the nodal u */
                double A[3] = {0, 0, 0};
                if (p->aux == 0) {
                    size_t lo[3], hi[3];
                    lo[0] = ((size_t)z * ny + y) * nx + wrap(x - 1, nx);
                    hi[0] = ((size_t)z * ny + y) * nx + wrap(x + 1, nx);
                    lo[1] = ((size_t)z * ny + wrap(y - 1, ny)) * nx + x;
                    hi[1] = ((size_t)z * ny + wrap(y + 1, ny)) * nx + x;
                    lo[2] = ((size_t)wrap(z - 1, nz) * ny + y) * nx + x;
                    hi[2] = ((size_t)wrap(z + 1, nz) * ny + y) * nx + x;
                    for (int a = 0; a < 3; ++a) {
                        double s = 0;
                        for (int b = 0; b < 3; ++b)
                            s += un[b] * (u[a * N + hi[b]] - u[a * N + lo[b]]) / (2.0 * dx);
                        A[a] = phi * s;
                    }
                }
                const double src = S ? S[n] : 0.0, dsrc = dSdt ? dSdt[n] : 0.0;
                for (int i = 0; i < q; ++i) {
                    double eA = 0, eu = 0;
                    for (int a = 0; a < 3; ++a) {
                        eA += ecomp(i, a, c) * A[a];
                        eu += ecomp(i, a, c) * un[a];
                    }
                    const double G = W[i] * eA / cs2 * beta;                   /* Eq. (16) */
                    const double F = W[i] * src + beta * W[i] * eu / cs2 * src; /* Eq. (3) */
                    const double dF = W[i] * dsrc + beta * W[i] * eu / cs2 * dsrc;
                    const double P = C[i] + dt * G + dt * F + 0.5 * dt * dt * dF;
                    const size_t dst = ((size_t)wrap(z + EZ[i], nz) * ny + wrap(y + EY[i], ny)) * nx + wrap(x + EX[i], nx);
                    g_out[i * N + dst] = P;
                }
            }
}

void orc3_run(const orc3_problem *p, double *g, int nsteps, const double *u, const double *D, const double *S,
              const double *dSdt, double *work)
{
    size_t bytes = (size_t)p->q * p->nx * p->ny * p->nz * sizeof(double);
    for (int s = 0; s < nsteps; ++s) {
        orc3_step(p, g, work, u, D, S, dSdt);
        memcpy(g, work, bytes);
    }
}
