/*
 * Oracle: plain float64 pair loop for the open-boundary RPY product
 * (U, Omega) = M(X) [F; T], matrix-free.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and by the benchmark's CPU
 * baseline, never by the HIP library, and sharing no code with it.
 *
 * Same mathematics as oracle/mobility.py (the generalised RPY tensors of
 * Rotne-Prager-Yamakawa and Wajnryb et al. that the paper's N-body solver
 * evaluates over all pairs, Sec. 3.5; block structure of eq.
 * (block_mobility)), written as the textbook double loop: one target at a
 * time, every source, no blocking, no vector intrinsics.  OpenMP splits the
 * targets across host threads; each target's sum runs over j = 0..N-1 in
 * order, so the result does not depend on the thread count.
 *
 * Layout: X, F, T, U, W are N x 3 row-major float64.  T and W may be NULL
 * (translational only).  F may be NULL when T is given (F = 0).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void coeffs(double r, double a, double eta, double *c1, double *c2,
                   double *d1, double *d2, double *f)
{
    const double pi = 3.14159265358979323846;
    const double mut = 1.0 / (6.0 * pi * eta * a);
    const double mur = 1.0 / (8.0 * pi * eta * a * a * a);
    if (r < 2.0 * a) {
        *c1 = mut * (1.0 - 9.0 * r / (32.0 * a));
        *c2 = mut * 3.0 * r / (32.0 * a);
        *d1 = mur * (1.0 - 27.0 * r / (32.0 * a) + 5.0 * r * r * r / (64.0 * a * a * a));
        *d2 = mur * (9.0 * r / (32.0 * a) - 3.0 * r * r * r / (64.0 * a * a * a));
        *f = (r / a - 3.0 * r * r / (8.0 * a * a)) / (16.0 * pi * eta * a * a);
    } else {
        *c1 = mut * (3.0 * a / (4.0 * r) + a * a * a / (2.0 * r * r * r));
        *c2 = mut * (3.0 * a / (4.0 * r) - 3.0 * a * a * a / (2.0 * r * r * r));
        *d1 = -1.0 / (16.0 * pi * eta * r * r * r);
        *d2 = 3.0 / (16.0 * pi * eta * r * r * r);
        *f = 1.0 / (8.0 * pi * eta * r * r);
    }
}

/* One target row i: accumulate over all sources. */
static void one_row(int64_t i, int64_t n, const double *x, const double *F,
                    const double *T, double a, double eta, double *u, double *w)
{
    double su[3] = {0, 0, 0}, sw[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
        double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double e[3] = {0, 0, 0};
        if (r > 0.0) { e[0] = d[0] / r; e[1] = d[1] / r; e[2] = d[2] / r; }
        double c1, c2, d1, d2, f;
        coeffs(r, a, eta, &c1, &c2, &d1, &d2, &f);
        double fj[3] = {0, 0, 0};
        if (F) { fj[0] = F[3 * j]; fj[1] = F[3 * j + 1]; fj[2] = F[3 * j + 2]; }
        double ef = e[0] * fj[0] + e[1] * fj[1] + e[2] * fj[2];
        for (int k = 0; k < 3; ++k) su[k] += c1 * fj[k] + c2 * ef * e[k];
        if (T) {
            double tj[3] = {T[3 * j], T[3 * j + 1], T[3 * j + 2]};
            double et = e[0] * tj[0] + e[1] * tj[1] + e[2] * tj[2];
            /* U_i += f T_j x e ;  Omega_i += f F_j x e + d1 T_j + d2 e (e.T_j) */
            su[0] += f * (tj[1] * e[2] - tj[2] * e[1]);
            su[1] += f * (tj[2] * e[0] - tj[0] * e[2]);
            su[2] += f * (tj[0] * e[1] - tj[1] * e[0]);
            sw[0] += f * (fj[1] * e[2] - fj[2] * e[1]) + d1 * tj[0] + d2 * et * e[0];
            sw[1] += f * (fj[2] * e[0] - fj[0] * e[2]) + d1 * tj[1] + d2 * et * e[1];
            sw[2] += f * (fj[0] * e[1] - fj[1] * e[0]) + d1 * tj[2] + d2 * et * e[2];
        }
    }
    u[0] = su[0]; u[1] = su[1]; u[2] = su[2];
    if (w) { w[0] = sw[0]; w[1] = sw[1]; w[2] = sw[2]; }
}

/* Full product: every target 0..n-1.  U (and W when T != NULL) are written. */
void oracle_rpy_mdot(int64_t n, const double *x, const double *F, const double *T,
                     double a, double eta, double *U, double *W)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        one_row(i, n, x, F, T, a, eta, U + 3 * i, (T && W) ? W + 3 * i : NULL);
}

/* Subset rows: targets rows[0..m-1]; output row k belongs to target rows[k]. */
void oracle_rpy_mdot_rows(int64_t n, const double *x, const double *F, const double *T,
                          double a, double eta, int64_t m, const int64_t *rows,
                          double *U, double *W)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < m; ++k)
        one_row(rows[k], n, x, F, T, a, eta, U + 3 * k, (T && W) ? W + 3 * k : NULL);
}

/* Number of OpenMP threads a parallel region uses (reported with timings). */
int oracle_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
