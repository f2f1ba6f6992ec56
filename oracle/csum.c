/*
 * Oracle triple sum in plain C (TEST INFRASTRUCTURE ONLY: used by the tests as
 * a cross-check of the numpy oracle and by the benchmark to time the oracle on
 * host cores; the GPU library never links or calls it).
 *
 * Computes, per particle, steps 1-4 of the interpolation algorithm of Sec. 2.2
 * (wrap modulo 2*pi, grid cell, in-cell offset, Eq. "triple_sum") in binary64,
 * and optionally the velocity gradient through derivative kernels.  The
 * kernel polynomials come in as coefficient tables [I][I] (node j, power p,
 * ascending powers) computed by the Python oracle; weights are evaluated by
 * Horner.  Field layout u[x3][x2][x1][3]; positions X[p][3] = (x1, x2, x3);
 * gradient g[p][a][b] = d u_a / d x_b.  Plain loops, OpenMP over particles.
 *
 * Build with -ffp-contract=off: the wrap/cell sequence must round every
 * operation separately.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double kL = 6.283185307179586; /* fl64(2*pi) */

static void cell_offset(double x, int64_t N, double invd, int64_t *c, double *t)
{
    double q = floor(x / kL);
    double y = x - kL * q;
    if (y < 0.0) y = y + kL;
    if (y >= kL) y = 0.0;
    double s = y * invd;
    double cf = floor(s);
    *t = s - cf;
    *c = (int64_t)cf;
    if (*c >= N) { *c = 0; *t = 0.0; }
}

static double horner(const double *coef, int I, double t)
{
    double acc = coef[I - 1];
    for (int p = I - 2; p >= 0; --p) acc = acc * t + coef[p];
    return acc;
}

static double node_value(const void *field, int is_f32, int64_t idx)
{
    return is_f32 ? (double)((const float *)field)[idx] : ((const double *)field)[idx];
}

/* returns the number of OpenMP threads used */
int oracle_triple_sum(const void *field, int field_is_f32, int64_t N,
                      const double *X, int64_t Np,
                      const double *coef, const double *dcoef, int I,
                      double *u, double *grad)
{
    const double invd = (double)N / kL;
    int nthreads = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            nthreads = omp_get_num_threads();
#endif
        }
#pragma omp for schedule(static)
        for (int64_t p = 0; p < Np; ++p) {
            int64_t c[3];
            double t[3], w[3][16], dw[3][16];
            for (int d = 0; d < 3; ++d) {
                cell_offset(X[3 * p + d], N, invd, &c[d], &t[d]);
                for (int j = 0; j < I; ++j) {
                    w[d][j] = horner(coef + j * I, I, t[d]);
                    if (grad) dw[d][j] = horner(dcoef + j * I, I, t[d]) * invd;
                }
            }
            double acc[3] = {0.0, 0.0, 0.0};
            double g[3][3] = {{0.0}};
            for (int k3 = 0; k3 < I; ++k3) {
                int64_t z = ((c[2] + k3 - (I / 2 - 1)) % N + N) % N;
                for (int k2 = 0; k2 < I; ++k2) {
                    int64_t y = ((c[1] + k2 - (I / 2 - 1)) % N + N) % N;
                    for (int k1 = 0; k1 < I; ++k1) {
                        int64_t x = ((c[0] + k1 - (I / 2 - 1)) % N + N) % N;
                        int64_t base = ((z * N + y) * N + x) * 3;
                        double wv = w[0][k1] * w[1][k2] * w[2][k3];
                        for (int a = 0; a < 3; ++a) {
                            double f = node_value(field, field_is_f32, base + a);
                            acc[a] += wv * f;
                            if (grad) {
                                g[a][0] += dw[0][k1] * w[1][k2] * w[2][k3] * f;
                                g[a][1] += w[0][k1] * dw[1][k2] * w[2][k3] * f;
                                g[a][2] += w[0][k1] * w[1][k2] * dw[2][k3] * f;
                            }
                        }
                    }
                }
            }
            for (int a = 0; a < 3; ++a) {
                u[3 * p + a] = acc[a];
                if (grad)
                    for (int b = 0; b < 3; ++b) grad[9 * p + 3 * a + b] = g[a][b];
            }
        }
    }
    return nthreads;
}
