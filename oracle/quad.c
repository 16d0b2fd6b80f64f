/*
 * Oracle helper (test infrastructure only; never linked by the product library).
 *
 * Direct trapezoidal quadrature of the free-space potential at listed grid
 * nodes (Section 4, eq. TrapOrig2D and its 1D/3D analogues):
 *
 *     phi(x_t) ~= prod_i h_i * sum_{s interior} G(|x_t - x_s|) rho(x_s)
 *
 * with G(r) = r/2 (d=1), log(r)/(2 pi) (d=2), -1/(4 pi r) (d=3)  (Section 1).
 * Boundary nodes of the grid are excluded from the sum (the integrand
 * vanishes there, Section 4).  The target x_t may be any grid node whose
 * distance to every interior node with nonzero rho is positive.
 *
 * Interior nodes whose rho is exactly zero contribute exactly zero and are
 * skipped.  Each term is evaluated in double precision and accumulated in
 * long double (x87 extended precision): a sum of ~1e7 double terms rounded
 * step by step drifts by ~1e-12 relative, which is the size of the parity
 * bar, while the extended accumulator keeps the sum exact to ~1e-16.
 *
 * Layout: rho is row-major over n[0] x ... x n[d-1], last axis fastest.
 * targets holds ntargets * d node indices.  out receives ntargets values.
 * Returns 0 on success, -1 on an invalid argument, -2 if out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double green(int d, double r)
{
    const double pi = 3.14159265358979323846;
    if (d == 1) return 0.5 * r;
    if (d == 2) return log(r) / (2.0 * pi);
    return -1.0 / (4.0 * pi * r);
}

int oracle_boundary_direct(int d, const int64_t *n, const double *h,
                           const double *rho, int64_t ntargets,
                           const int64_t *targets, double *out)
{
    if (d < 1 || d > 3 || !n || !h || !rho || !targets || !out) return -1;
    int64_t nn[3] = {1, 1, 1};
    double hh[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d; ++a) {
        if (n[a] < 3 || !(h[a] > 0.0)) return -1;
        nn[3 - d + a] = n[a];
        hh[3 - d + a] = h[a];
    }
    /* gather the interior nodes with nonzero rho: (offsets along each axis, value) */
    int64_t cap = 1;
    for (int a = 0; a < 3; ++a) cap *= (nn[a] > 1 ? nn[a] - 2 : 1);
    double *sx = malloc(sizeof(double) * (size_t)cap * 4);
    if (!sx) return -2;
    int64_t ns = 0;
    int64_t lo0 = nn[0] > 1 ? 1 : 0, hi0 = nn[0] > 1 ? nn[0] - 1 : 1;
    int64_t lo1 = nn[1] > 1 ? 1 : 0, hi1 = nn[1] > 1 ? nn[1] - 1 : 1;
    for (int64_t i = lo0; i < hi0; ++i)
        for (int64_t j = lo1; j < hi1; ++j)
            for (int64_t k = 1; k < nn[2] - 1; ++k) {
                double v = rho[(i * nn[1] + j) * nn[2] + k];
                if (v != 0.0) {
                    sx[4 * ns + 0] = (double)i;
                    sx[4 * ns + 1] = (double)j;
                    sx[4 * ns + 2] = (double)k;
                    sx[4 * ns + 3] = v;
                    ++ns;
                }
            }
    double vol = 1.0;
    for (int a = 0; a < d; ++a) vol *= h[a];

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntargets; ++t) {
        double tx[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d; ++a) tx[3 - d + a] = (double)targets[t * d + a];
        long double acc = 0.0L;
        for (int64_t s = 0; s < ns; ++s) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double dx = (tx[a] - sx[4 * s + a]) * hh[a];
                r2 += dx * dx;
            }
            acc += (long double)(green(d, sqrt(r2)) * sx[4 * s + 3]);
        }
        out[t] = (double)acc * vol;
    }
    free(sx);
    return 0;
}

/*
 * Transpose of oracle_boundary_direct over the boundary nodes:
 *     out[s] = prod_i h_i * sum_{t} G(|x_t - x_s|) lam[t]      for every interior node s
 * where t runs over the listed target nodes with weights lam[t].  out has the
 * full grid's size; its boundary entries are set to 0.  Accumulated in long
 * double like oracle_boundary_direct.
 */
int oracle_boundary_adjoint(int d, const int64_t *n, const double *h, int64_t ntargets,
                            const int64_t *targets, const double *lam, double *out)
{
    if (d < 1 || d > 3 || !n || !h || !targets || !lam || !out) return -1;
    int64_t nn[3] = {1, 1, 1};
    double hh[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d; ++a) {
        if (n[a] < 3 || !(h[a] > 0.0)) return -1;
        nn[3 - d + a] = n[a];
        hh[3 - d + a] = h[a];
    }
    double vol = 1.0;
    for (int a = 0; a < d; ++a) vol *= h[a];
    double *tx = malloc(sizeof(double) * (size_t)(ntargets > 0 ? ntargets : 1) * 4);
    if (!tx) return -2;
    int64_t nt = 0;
    for (int64_t t = 0; t < ntargets; ++t) {
        if (lam[t] == 0.0) continue;
        double c[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d; ++a) c[3 - d + a] = (double)targets[t * d + a];
        tx[4 * nt + 0] = c[0];
        tx[4 * nt + 1] = c[1];
        tx[4 * nt + 2] = c[2];
        tx[4 * nt + 3] = lam[t];
        ++nt;
    }
    const int64_t total = nn[0] * nn[1] * nn[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t e = 0; e < total; ++e) {
        const int64_t k = e % nn[2], j = (e / nn[2]) % nn[1], i = e / (nn[1] * nn[2]);
        int interior = (k > 0 && k < nn[2] - 1);
        if (nn[1] > 1) interior = interior && j > 0 && j < nn[1] - 1;
        if (nn[0] > 1) interior = interior && i > 0 && i < nn[0] - 1;
        if (!interior) {
            out[e] = 0.0;
            continue;
        }
        const double s[3] = {(double)i, (double)j, (double)k};
        long double acc = 0.0L;
        for (int64_t t = 0; t < nt; ++t) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double dx = (tx[4 * t + a] - s[a]) * hh[a];
                r2 += dx * dx;
            }
            acc += (long double)(green(d, sqrt(r2)) * tx[4 * t + 3]);
        }
        out[e] = (double)acc * vol;
    }
    free(tx);
    return 0;
}
