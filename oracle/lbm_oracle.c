/*
 * lbm_oracle.c -- plain, slow CPU reference of the TRT-R lattice Boltzmann model for the
 * convection-diffusion equation with variable coefficients
 * (Y. Yu, Z. Qin, H. Yuan, S. Shu, arXiv:2312.10316).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may build, load or call it.  It
 * shares no code, header, table or constant with the HIP library and includes none of its files.
 *
 * Everything is evaluated literally from the paper, node by node, in the order the paper states
 * it: the Hermite tensors are formed from e_i and the Kronecker delta, the equilibrium is the full
 * third-order Hermite sum, and the non-equilibrium moments are Hermite projections of g - g_eq
 * (no moment shortcuts, no fusion, no blocking).  Physical units throughout (c = dx/dt).
 *
 * The file is compiled twice: once with `real` = double (symbols orc_*), and once with
 * -DORC_COMPLEX, where `real` = double _Complex (symbols orc_z_*).  The complex build is the
 * complex-step derivative of the same code (Squire & Trapp, SIAM Review 1998): perturbing an input
 * by i*h gives d(output)/d(input) = Im(output)/h with no cancellation error.  Nothing else differs.
 *
 * The real build is also compiled a third time with -fopenmp (symbols unchanged, in their own
 * shared object): the node loop of a step is then split over host threads by rows.  Every node is
 * still evaluated by the same statements in the same order, and every destination is written by
 * exactly one node, so the results are bitwise those of one thread; that build exists only to time
 * the oracle on all host cores and to produce stored expected values of large cases.
 *
 * Readings where the paper is silent (each is listed in the design notes of the repository):
 *   - D2Q9 velocity order (the paper lists the set only): 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0)
 *     4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1), times c.
 *   - phi = sum_i g_i with no source correction (Sec. 2.2: the zeroth non-equilibrium moment
 *     vanishes; Sec. 2.4, first-order balance).
 *   - u, kappa and S are taken at the collision node and at time t_n.
 *   - the space derivative in the auxiliary term is the second-order central difference of the
 *     nodal u on the periodic lattice; the "flux" variant replaces phi u_b d_b u_a by
 *     d_b(phi u_a u_b) - u_a d_b(phi u_b) (equal by the product rule) with the same difference and
 *     phi = sum_i g_i at the neighbours at the same time level.
 *   - the time derivative of F_i uses the supplied dS/dt and a time-independent u within the step
 *     (Sec. 2.3 assumption).
 *   - the lattice is periodic in x and y, unless Dirichlet edges (non-equilibrium extrapolation)
 *     or walls (halfway anti-bounce-back) are selected; across such a boundary the difference of u
 *     in the auxiliary term is one-sided.
 *   - the anti-bounce-back wall value enters through the even part of the equilibrium at the wall
 *     value and the velocity of the boundary node, at the time the reflected population arrives.
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#define ORC_ROWS_PARALLEL _Pragma("omp parallel for schedule(static)")
#else
#define ORC_ROWS_PARALLEL
#endif

#ifdef ORC_COMPLEX
#include <complex.h>
typedef double _Complex real;
#define ORC(name) orc_z_##name
#else
typedef double real;
#define ORC(name) orc_##name
#endif

/* ---- D2Q9 lattice (Sec. 2.2, text after Eq. (3)) ------------------------------------------ */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Problem description shared by all oracle entry points (Sec. 2.1 problem statement plus the
 * lattice spacing, time step and magic parameter of Sec. 2.4). */
typedef struct orc_problem {
    int nx, ny;        /* periodic lattice, node (j, k) at index k*nx + j */
    double dx, dt;     /* lattice spacing and time step; c = dx/dt */
    double lambda;     /* magic parameter Lambda = (tau1 - 1/2)(tau2 - 1/2) */
    double D_const;    /* diffusion coefficient kappa when no field is given */
    int aux;           /* 0: auxiliary term of Eq. (16) with local phi; 1: flux-difference form;
                          2: no auxiliary term (ablation) */
    int boundary;      /* 0: periodic; 1: Dirichlet edges (the first and last rows and columns are
                          rebuilt by apply_nee before each step; across an edge the derivatives of
                          u in the auxiliary term are one-sided instead of wrapped); 2: walls at
                          y = -dx/2 and y = (ny - 1/2) dx by halfway anti-bounce-back, x periodic */
    double tau3;       /* MRT-R third-order relaxation time (Sec. 2.2, Eq. (11)); 0 or 1: TRT-R */
} orc_problem;

#ifndef ORC_COMPLEX
void orc_lattice(int *ex, int *ey, double *w)
{
    for (int i = 0; i < 9; ++i) { ex[i] = EX[i]; ey[i] = EY[i]; w[i] = W[i]; }
}
#endif

/* e_{i,a} (a = 0: x, a = 1: y) */
static double ecomp(int i, int a, double c) { return c * (double)(a == 0 ? EX[i] : EY[i]); }
static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* Hermite tensors, Sec. 2.2 text after Eq. (10):
 *   H_a = e_a,  H_ab = e_a e_b - cs2 delta_ab,
 *   H_abg = e_a e_b e_g - cs2 (e_a delta_bg + e_b delta_ga + e_g delta_ab). */
static double herm1(int i, int a, double c) { return ecomp(i, a, c); }
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

/* Third-order Hermite equilibrium, Sec. 2.2, Eq. (6):
 *   g_eq_i = w_i phi { 1 + H_a u_a / cs2 + H_ab u_a u_b / (2 cs2^2) + H_abg u_a u_b u_g / (6 cs2^3) } */
void ORC(equilibrium)(real phi, real ux, real uy, double c, real *geq)
{
    double cs2 = c * c / 3.0;
    real u[2] = {ux, uy};
    for (int i = 0; i < 9; ++i) {
        real s1 = 0, s2 = 0, s3 = 0;
        for (int a = 0; a < 2; ++a) s1 += herm1(i, a, c) * u[a];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) s2 += herm2(i, a, b, c) * u[a] * u[b];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int g = 0; g < 2; ++g) s3 += herm3(i, a, b, g, c) * u[a] * u[b] * u[g];
        geq[i] = W[i] * phi * (1.0 + s1 / cs2 + s2 / (2.0 * cs2 * cs2) + s3 / (6.0 * cs2 * cs2 * cs2));
    }
}

/* Relaxation pair.  kappa = (tau1 - 1/2) cs2 dt (Sec. 2.4, result of the Chapman-Enskog analysis)
 * and Lambda = (tau1 - 1/2)(tau2 - 1/2) (Sec. 2.4, magic parameter), each solved for its tau. */
void ORC(relaxation)(real kappa, double dx, double dt, double lambda, real *tau1, real *tau2)
{
    double c = dx / dt;
    double cs2 = c * c / 3.0;
    *tau1 = 0.5 + kappa / (cs2 * dt);
    *tau2 = 0.5 + lambda / (*tau1 - 0.5);
}

/* MRT-R collision operator, Sec. 2.2, Eq. (11), truncated after the third order, with the
 * non-equilibrium moments B_a = sum_i H_a (g_i - g_eq_i) (Eq. (8)), B_ab (Eq. (13)) and
 * B_abg = sum_i H_abg (g_i - g_eq_i):
 *   C_i = g_eq_i + (1 - 1/tau1) w_i H_a B_a / cs2 + (1 - 1/tau2) w_i H_ab B_ab / (2 cs2^2)
 *               + (1 - 1/tau3) w_i H_abg B_abg / (6 cs2^3).
 * tau3 = 1 drops the third-order non-equilibrium part: the TRT-R operator of Eq. (12).
 * phi is the zeroth moment sum_i g_i (Sec. 2.2: B_0^neq = 0). */
void ORC(collide_mrt)(const real *g, real ux, real uy, real tau1, real tau2, real tau3, double c, real *out)
{
    double cs2 = c * c / 3.0;
    real phi = 0;
    for (int i = 0; i < 9; ++i) phi += g[i];
    real geq[9];
    ORC(equilibrium)(phi, ux, uy, c, geq);
    real B1[2] = {0, 0};
    real B2[2][2] = {{0, 0}, {0, 0}};
    real B3[2][2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
    for (int i = 0; i < 9; ++i) {
        real gneq = g[i] - geq[i];  /* Eq. (5) */
        for (int a = 0; a < 2; ++a) B1[a] += herm1(i, a, c) * gneq;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) B2[a][b] += herm2(i, a, b, c) * gneq;
        if (tau3 != 1.0)  /* the third-order term vanishes for tau3 = 1 */
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int d = 0; d < 2; ++d) B3[a][b][d] += herm3(i, a, b, d, c) * gneq;
    }
    for (int i = 0; i < 9; ++i) {
        real r1 = 0, r2 = 0, r3 = 0;
        for (int a = 0; a < 2; ++a) r1 += herm1(i, a, c) * B1[a];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) r2 += herm2(i, a, b, c) * B2[a][b];
        if (tau3 != 1.0)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int d = 0; d < 2; ++d) r3 += herm3(i, a, b, d, c) * B3[a][b][d];
        out[i] = geq[i] + (1.0 - 1.0 / tau1) * W[i] * r1 / cs2
                        + (1.0 - 1.0 / tau2) * W[i] * r2 / (2.0 * cs2 * cs2)
                        + (1.0 - 1.0 / tau3) * W[i] * r3 / (6.0 * cs2 * cs2 * cs2);
    }
}

/* TRT-R collision operator, Sec. 2.2, Eq. (12): the MRT-R operator with tau3 = 1. */
void ORC(collide)(const real *g, real ux, real uy, real tau1, real tau2, double c, real *out)
{
    ORC(collide_mrt)(g, ux, uy, tau1, tau2, 1.0, c, out);
}

/* index of the velocity opposite to e_i */
static int opposite(int i)
{
    for (int j = 0; j < 9; ++j)
        if (EX[j] == -EX[i] && EY[j] == -EY[i]) return j;
    return -1;
}

static int wrap(int k, int n) { return ((k % n) + n) % n; }

/* Initial state, Sec. 3 (set-up of the benchmark): g_i = g_eq_i(phi0, u). */
void ORC(init)(const orc_problem *p, const real *phi0, const real *ux, const real *uy, real *g)
{
    size_t N = (size_t)p->nx * p->ny;
    double c = p->dx / p->dt;
    for (size_t n = 0; n < N; ++n) {
        real geq[9];
        ORC(equilibrium)(phi0[n], ux[n], uy[n], c, geq);
        for (int i = 0; i < 9; ++i) g[i * N + n] = geq[i];
    }
}

/* phi = sum_i g_i at every node. */
void ORC(phi)(const orc_problem *p, const real *g, real *phi)
{
    size_t N = (size_t)p->nx * p->ny;
    for (size_t n = 0; n < N; ++n) {
        real s = 0;
        for (int i = 0; i < 9; ++i) s += g[i * N + n];
        phi[n] = s;
    }
}

/* One time step of the TRT-R evolution equation, Sec. 2.2, Eq. (14):
 *   g_i(x + e_i dt, t + dt) = C_i + dt G_i + dt F_i + (dt^2 / 2) d_t F_i
 * with C_i of Eq. (12) (Eq. (11) when tau3 is set), F_i of Eq. (3), G_i of Eq. (16) (or the selected
 * reading), evaluated at every node x at time t_n and streamed to x + e_i dt on the periodic lattice.
 * With walls (boundary 2) a population that would cross y = -dx/2 or y = (ny - 1/2) dx returns to
 * its node reversed, by halfway anti-bounce-back for a Dirichlet value phi_w:
 *   g_opp(i)(x, t + dt) = -P_i(x) + 2 g_eq_i^+(phi_w, u(x)),  g_eq^+ = (g_eq_i + g_eq_opp(i)) / 2,
 * with phi_w = phi_b[x] of row 0 (bottom wall) or of row ny - 1 (top wall) at time t + dt.
 * g_in / g_out: [9][ny][nx].  D, S, dSdt may be NULL (constant D_const; no source); phi_b
 * ([ny][nx]) is read for walls only. */
void ORC(step)(const orc_problem *p, const real *g_in, real *g_out, const real *ux, const real *uy,
               const real *D, const real *S, const real *dSdt, const real *phi_b)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    const double dx = p->dx, dt = p->dt, c = dx / dt, cs2 = c * c / 3.0;

    real *phi_all = NULL;
    if (p->aux == 1) {  /* the flux form needs phi at the neighbours at the same time level */
        phi_all = (real *)malloc(N * sizeof(real));
        ORC(phi)(p, g_in, phi_all);
    }

    ORC_ROWS_PARALLEL
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t n = (size_t)y * nx + x;
            real g[9];
            for (int i = 0; i < 9; ++i) g[i] = g_in[i * N + n];
            real phi = 0;
            for (int i = 0; i < 9; ++i) phi += g[i];

            real kappa = D ? D[n] : (real)p->D_const;
            real tau1, tau2;
            ORC(relaxation)(kappa, dx, dt, p->lambda, &tau1, &tau2);
            real beta = 1.0 - 1.0 / (2.0 * tau1);

            real C[9];
            const real tau3 = p->tau3 == 0.0 ? 1.0 : p->tau3;
            ORC(collide_mrt)(g, ux[n], uy[n], tau1, tau2, tau3, c, C);

            /* neighbours along +/- x and +/- y */
            size_t nb[2][2];  /* nb[b][0] = x - e_b, nb[b][1] = x + e_b */
            nb[0][0] = (size_t)y * nx + wrap(x - 1, nx);
            nb[0][1] = (size_t)y * nx + wrap(x + 1, nx);
            nb[1][0] = (size_t)wrap(y - 1, ny) * nx + x;
            nb[1][1] = (size_t)wrap(y + 1, ny) * nx + x;
            const real *u[2] = {ux, uy};
            real un[2] = {ux[n], uy[n]};
            /* difference stencil d_b u ~ (u[hi] - u[lo]) / h: central, or one-sided at a Dirichlet edge */
            size_t lo[2] = {nb[0][0], nb[1][0]}, hi[2] = {nb[0][1], nb[1][1]};
            double h[2] = {2.0 * dx, 2.0 * dx};
            if (p->boundary == 1) {
                if (x == 0) { lo[0] = n; h[0] = dx; } else if (x == nx - 1) { hi[0] = n; h[0] = dx; }
            }
            if (p->boundary == 1 || p->boundary == 2) {
                if (y == 0) { lo[1] = n; h[1] = dx; } else if (y == ny - 1) { hi[1] = n; h[1] = dx; }
            }
            /* even part of the equilibrium at the wall value, for walls */
            real geq_w[9];
            const int wall_row = p->boundary == 2 && (y == 0 || y == ny - 1);
            if (wall_row) ORC(equilibrium)(phi_b[n], ux[n], uy[n], c, geq_w);

            /* A_a multiplies w_i e_ia / cs2 (1 - 1/(2 tau1)) in G_i */
            real A[2] = {0, 0};
            if (p->aux == 0) {
                /* Eq. (16): phi u_b d_b u_a, d_b by differences of the nodal u */
                for (int a = 0; a < 2; ++a) {
                    real s = 0;
                    for (int b = 0; b < 2; ++b) {
                        real dbua = (u[a][hi[b]] - u[a][lo[b]]) / h[b];
                        s += un[b] * dbua;
                    }
                    A[a] = phi * s;
                }
            } else if (p->aux == 1) {
                /* d_b(phi u_a u_b) - u_a d_b(phi u_b), same central difference */
                for (int a = 0; a < 2; ++a) {
                    real s = 0;
                    for (int b = 0; b < 2; ++b) {
                        size_t m = nb[b][0], q = nb[b][1];
                        real dflux = (phi_all[q] * u[a][q] * u[b][q] - phi_all[m] * u[a][m] * u[b][m]) / (2.0 * dx);
                        real dmass = (phi_all[q] * u[b][q] - phi_all[m] * u[b][m]) / (2.0 * dx);
                        s += dflux - un[a] * dmass;
                    }
                    A[a] = s;
                }
            }

            real src = S ? S[n] : (real)0.0;
            real dsrc = dSdt ? dSdt[n] : (real)0.0;

            for (int i = 0; i < 9; ++i) {
                real eA = 0, eu = 0;
                for (int a = 0; a < 2; ++a) {
                    eA += ecomp(i, a, c) * A[a];
                    eu += ecomp(i, a, c) * un[a];
                }
                /* Eq. (16) */
                real G = W[i] * eA / cs2 * beta;
                /* Eq. (3) and its time derivative (u, tau1 frozen within the step) */
                real F = W[i] * src + beta * W[i] * eu / cs2 * src;
                real dF = W[i] * dsrc + beta * W[i] * eu / cs2 * dsrc;
                real P = C[i] + dt * G + dt * F + 0.5 * dt * dt * dF;
                const int ty = y + EY[i];
                if (wall_row && (ty < 0 || ty >= ny)) {  /* halfway anti-bounce-back */
                    const int o = opposite(i);
                    g_out[o * N + n] = -P + (geq_w[i] + geq_w[o]);
                    continue;
                }
                size_t dst = (size_t)wrap(ty, ny) * nx + wrap(x + EX[i], nx);
                g_out[i * N + dst] = P;
            }
        }
    }
    free(phi_all);
}

/* Dirichlet edges by non-equilibrium extrapolation (Guo, Zheng and Shi, Chinese Physics 2002), the
 * boundary scheme of the benchmark of Sec. 3: the first and last rows and columns are boundary nodes;
 * at each boundary node x_b, with x_f its interior neighbour along the inward normal (the diagonal
 * neighbour at a corner),
 *   g_i(x_b) = g_eq_i(phi_b(x_b), u(x_b)) + [ g_i(x_f) - g_eq_i(phi(x_f), u(x_f)) ],  phi(x_f) = sum_i g_i(x_f).
 * Applied in place to the pre-collision state at t_n, before the step.  phi_b: [ny][nx] (only
 * boundary entries are read). */
void ORC(apply_nee)(const orc_problem *p, real *g, const real *ux, const real *uy, const real *phi_b)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    const double c = p->dx / p->dt;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            if (!(x == 0 || x == nx - 1 || y == 0 || y == ny - 1)) continue;
            const int xf = x + (x == 0) - (x == nx - 1), yf = y + (y == 0) - (y == ny - 1);
            const size_t b = (size_t)y * nx + x, f = (size_t)yf * nx + xf;
            real phif = 0;
            for (int i = 0; i < 9; ++i) phif += g[i * N + f];
            real geq_f[9], geq_b[9];
            ORC(equilibrium)(phif, ux[f], uy[f], c, geq_f);
            ORC(equilibrium)(phi_b[b], ux[b], uy[b], c, geq_b);
            for (int i = 0; i < 9; ++i) g[i * N + b] = geq_b[i] + (g[i * N + f] - geq_f[i]);
        }
    }
}

#ifndef ORC_COMPLEX
/* Host threads used by the row loop of a step in the OpenMP build (1 in the others); returns the
 * number in effect. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
#endif

/* nsteps repeated steps on g (in place); work holds 9*nx*ny values of scratch. */
void ORC(run)(const orc_problem *p, real *g, int nsteps, const real *ux, const real *uy,
              const real *D, const real *S, const real *dSdt, const real *phi_b, real *work)
{
    size_t bytes = (size_t)9 * p->nx * p->ny * sizeof(real);
    for (int s = 0; s < nsteps; ++s) {
        ORC(step)(p, g, work, ux, uy, D, S, dSdt, phi_b);
        memcpy(g, work, bytes);
    }
}
