/* Runs the D3Q19/D3Q27 oracle on the jobs of a binary file (host sanitizer test; this translation
 * unit includes the 3D oracle's source).
 *
 * Job: int32 nx, ny, nz, aux, q, nsteps, has_D; double dx, dt, lambda, D_const; then double arrays
 * g[q][nz][ny][nx], u[3][nz][ny][nx] and the optional D[nz][ny][nx].  Output per job: g after nsteps. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/lbm_oracle_3d.c"

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
    int h[7];
    int jobs = 0;
    while (fread(h, sizeof(int), 7, in) == 7) {
        double d[4];
        if (fread(d, sizeof(double), 4, in) != 4) return 2;
        orc3_problem p = {h[0], h[1], h[2], d[0], d[1], d[2], d[3], h[3], h[4]};
        const size_t n = (size_t)p.nx * p.ny * p.nz, q = (size_t)p.q;
        double *g = read_doubles(in, q * n), *u = read_doubles(in, 3 * n);
        double *D = h[6] ? read_doubles(in, n) : NULL;
        double *work = (double *)malloc(q * n * sizeof(double));
        orc3_run(&p, g, h[5], u, D, NULL, NULL, work);
        if (fwrite(g, sizeof(double), q * n, out) != q * n) return 2;
        free(g); free(u); free(D); free(work);
        ++jobs;
    }
    fclose(in);
    fclose(out);
    printf("%d jobs\n", jobs);
    return 0;
}
