/* Runs the D2Q9 oracle on the jobs of a binary file and writes the final populations, for the host
 * sanitizer test (tests/test_host_sanitizers.py): this translation unit includes the oracle's source,
 * so the whole oracle is compiled with AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Job (native endianness): int32 nx, ny, aux, boundary, nsteps, has_D, has_S, has_dSdt, has_phib;
 * double dx, dt, lambda, D_const, tau3; then double arrays g[9][ny][nx], ux[ny][nx], uy[ny][nx] and
 * the optional D, S, dSdt, phi_b ([ny][nx] each).  Output per job: g[9][ny][nx] after nsteps steps. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/lbm_oracle.c"

static double *read_doubles(FILE *f, size_t n)
{
    double *a = (double *)malloc(n * sizeof(double));
    if (!a || fread(a, sizeof(double), n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return a;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s jobs.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb"), *out = fopen(argv[2], "wb");
    if (!in || !out) return 2;
    int h[9];
    int jobs = 0;
    while (fread(h, sizeof(int), 9, in) == 9) {
        double d[5];
        if (fread(d, sizeof(double), 5, in) != 5) return 2;
        orc_problem p = {h[0], h[1], d[0], d[1], d[2], d[3], h[2], h[3], d[4]};
        const size_t n = (size_t)p.nx * p.ny;
        double *g = read_doubles(in, 9 * n), *ux = read_doubles(in, n), *uy = read_doubles(in, n);
        double *D = h[5] ? read_doubles(in, n) : NULL, *S = h[6] ? read_doubles(in, n) : NULL;
        double *dSdt = h[7] ? read_doubles(in, n) : NULL, *phib = h[8] ? read_doubles(in, n) : NULL;
        double *work = (double *)malloc(9 * n * sizeof(double));
        orc_run(&p, g, h[4], ux, uy, D, S, dSdt, phib, work);
        if (fwrite(g, sizeof(double), 9 * n, out) != 9 * n) return 2;
        free(g); free(ux); free(uy); free(D); free(S); free(dSdt); free(phib); free(work);
        ++jobs;
    }
    fclose(in);
    fclose(out);
    printf("%d jobs\n", jobs);
    return 0;
}
