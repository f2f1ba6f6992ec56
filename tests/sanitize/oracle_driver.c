/* Driver of the C oracle (oracle/csum.c) for the sanitizer build.  Reads a
 * field, positions and coefficient tables written by the test (raw binary64
 * arrays), runs the triple sum with and without gradient, and writes the
 * results; the test compares them with the numpy oracle.  Any out-of-bounds
 * access or undefined behaviour in the oracle aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_triple_sum(const void *field, int is_f32, int64_t N, const double *X, int64_t np, const double *coef,
                      const double *dcoef, int I, double *u, double *g);

static void *slurp(const char *path, size_t n)
{
    FILE *f = fopen(path, "rb");
    if (!f) { perror(path); exit(2); }
    void *p = malloc(n);
    if (fread(p, 1, n, f) != n) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 7) { fprintf(stderr, "usage: dir N np I out_u out_g\n"); return 2; }
    char path[4096];
    const int64_t N = atoll(argv[2]), np = atoll(argv[3]);
    const int I = atoi(argv[4]);
    snprintf(path, sizeof path, "%s/field.bin", argv[1]);
    double *field = slurp(path, (size_t)(N * N * N * 3) * sizeof(double));
    snprintf(path, sizeof path, "%s/X.bin", argv[1]);
    double *X = slurp(path, (size_t)np * 3 * sizeof(double));
    snprintf(path, sizeof path, "%s/coef.bin", argv[1]);
    double *coef = slurp(path, (size_t)(I * I) * sizeof(double));
    snprintf(path, sizeof path, "%s/dcoef.bin", argv[1]);
    double *dcoef = slurp(path, (size_t)(I * I) * sizeof(double));
    double *u = malloc((size_t)np * 3 * sizeof(double));
    double *g = malloc((size_t)np * 9 * sizeof(double));
    oracle_triple_sum(field, 0, N, X, np, coef, dcoef, I, u, g);
    FILE *fu = fopen(argv[5], "wb"), *fg = fopen(argv[6], "wb");
    if (!fu || !fg) return 2;
    fwrite(u, sizeof(double), (size_t)np * 3, fu);
    fwrite(g, sizeof(double), (size_t)np * 9, fg);
    fclose(fu);
    fclose(fg);
    free(field); free(X); free(coef); free(dcoef); free(u); free(g);
    return 0;
}
