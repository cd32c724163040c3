/*
 * FP64 CPU oracle for network dynamics with a polynomial difference coupling
 * (App. A.3, difference form; Desai-Zwanzig model of App. A.5 with h(x) = x):
 *
 *   x_m' = omega_m + sum_{j=0..q} f_j x_m^j + (K/N) sum_l a_ml h(x_l - x_m),
 *   h(x) = sum_{a=0..p} h_a x^a.
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the product path may load or call it;
 * it shares no code with the HIP path.  The plain definition: every row sums
 * h over its adjacency (or over every l != m for complete graphs) in column
 * order, polynomials by Horner's rule, FP64; no moments, no expansion.
 */
#include <stdint.h>
#include <stdlib.h>

static double horner(int deg, const double *c, double x) {
    double v = c[deg];
    for (int j = deg - 1; j >= 0; j--) v = v * x + c[j];
    return v;
}

void oracle_poly_rhs(int64_t n, const int64_t *rp, const int32_t *col, int complete, const double *omega, double K,
                     int p, const double *h, int q, const double *f, const double *x, const int64_t *rows,
                     int64_t nrows, double *out) {
    const int64_t cnt = rows ? nrows : n;
    const double scale = K / (double)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        const int64_t m = rows ? rows[r] : r;
        double acc = 0.0;
        if (complete) {
            for (int64_t l = 0; l < n; l++)
                if (l != m) acc += horner(p, h, x[l] - x[m]);
        } else {
            for (int64_t e = rp[m]; e < rp[m + 1]; e++) acc += horner(p, h, x[col[e]] - x[m]);
        }
        out[r] = (omega ? omega[m] : 0.0) + (q >= 0 && f ? horner(q, f, x[m]) : 0.0) + scale * acc;
    }
}

/* Classical RK4 (stepper 0) or explicit Euler (1), x in place.
   Returns 0, or -1 when memory runs out. */
int oracle_poly_integrate(int64_t n, const int64_t *rp, const int32_t *col, int complete, const double *omega,
                          double K, int p, const double *h, int q, const double *f, double *x, double dt,
                          int64_t steps, int stepper) {
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    if (!k1 || !k2 || !k3 || !k4 || !tmp) {
        free(k1); free(k2); free(k3); free(k4); free(tmp);
        return -1;
    }
#define RHS(y, o) oracle_poly_rhs(n, rp, col, complete, omega, K, p, h, q, f, y, NULL, 0, o)
    for (int64_t s = 0; s < steps; s++) {
        RHS(x, k1);
        if (stepper == 1) {
            for (int64_t i = 0; i < n; i++) x[i] += dt * k1[i];
            continue;
        }
        for (int64_t i = 0; i < n; i++) tmp[i] = x[i] + 0.5 * dt * k1[i];
        RHS(tmp, k2);
        for (int64_t i = 0; i < n; i++) tmp[i] = x[i] + 0.5 * dt * k2[i];
        RHS(tmp, k3);
        for (int64_t i = 0; i < n; i++) tmp[i] = x[i] + dt * k3[i];
        RHS(tmp, k4);
        for (int64_t i = 0; i < n; i++) x[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
#undef RHS
    free(k1); free(k2); free(k3); free(k4); free(tmp);
    return 0;
}

/* General polynomial coupling (App. A.3, eq. PolyApprox): g(x, y) =
   sum_{a,b=0..p} c[a][b] x^a y^b for partner value x and own value y
   (row-major [(p+1)*(p+1)]), instead of h(x - y). */
static double g_poly(int p, const double *c, double x, double y) {
    double v = 0.0;
    double xa = 1.0;
    for (int a = 0; a <= p; a++) {
        double yb = 1.0;
        for (int b = 0; b <= p; b++) {
            v += c[a * (p + 1) + b] * xa * yb;
            yb *= y;
        }
        xa *= x;
    }
    return v;
}

void oracle_poly_rhs_general(int64_t n, const int64_t *rp, const int32_t *col, int complete, const double *omega,
                             double K, int p, const double *c, int q, const double *f, const double *x,
                             const int64_t *rows, int64_t nrows, double *out) {
    const int64_t cnt = rows ? nrows : n;
    const double scale = K / (double)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        const int64_t m = rows ? rows[r] : r;
        double acc = 0.0;
        if (complete) {
            for (int64_t l = 0; l < n; l++)
                if (l != m) acc += g_poly(p, c, x[l], x[m]);
        } else {
            for (int64_t e = rp[m]; e < rp[m + 1]; e++) acc += g_poly(p, c, x[col[e]], x[m]);
        }
        out[r] = (omega ? omega[m] : 0.0) + (q >= 0 && f ? horner(q, f, x[m]) : 0.0) + scale * acc;
    }
}

/* Two-component oscillators (Table 1 of the paper: van der Pol /
   FitzHugh-Nagumo with h(xi) = xi): for d = 0, 1
     x_{d,m}' = [d = 0] omega_m + f_d(x_{0,m}, x_{1,m})
                + (K/N) sum_l a_ml h(x_{d,l} - x_{d,m}),
   f_d(u, v) = sum_{i,j=0..3} F[d][i][j] u^i v^j, h as above (both components).
   x and out are [2][n] (rows: out[d][r]). */
static double f2_eval(const double *F, double u, double v) {
    double s = 0.0, ui = 1.0;
    for (int i = 0; i <= 3; i++) {
        double vj = 1.0;
        for (int j = 0; j <= 3; j++) {
            s += F[i * 4 + j] * ui * vj;
            vj *= v;
        }
        ui *= u;
    }
    return s;
}

void oracle_osc2_rhs(int64_t n, const int64_t *rp, const int32_t *col, int complete, const double *omega, double K,
                     int p, const double *h, const double *F, const double *x, const int64_t *rows, int64_t nrows,
                     double *out) {
    const int64_t cnt = rows ? nrows : n;
    const double scale = K / (double)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        const int64_t m = rows ? rows[r] : r;
        for (int d = 0; d < 2; d++) {
            const double *xd = x + d * n;
            double acc = 0.0;
            if (complete) {
                for (int64_t l = 0; l < n; l++)
                    if (l != m) acc += horner(p, h, xd[l] - xd[m]);
            } else {
                for (int64_t e = rp[m]; e < rp[m + 1]; e++) acc += horner(p, h, xd[col[e]] - xd[m]);
            }
            out[d * cnt + r] = (d == 0 && omega ? omega[m] : 0.0) + f2_eval(F + 16 * d, x[m], x[n + m]) + scale * acc;
        }
    }
}
