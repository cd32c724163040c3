/*
 * FP64 CPU oracle for the phase model on the two structured adjacencies of
 * App. B (extensions of step E1).  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path may load or call it; it shares no code with the HIP path.
 *
 *   theta_m' = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m),
 *   h(x) = dcos[0] + sum_{k=1..p} ( dsin[k] sin(k x) + dcos[k] cos(k x) ),
 *
 * with either
 *   rank one (App. B.1):  a_ml = alpha_m beta_l for every pair, l = m included;
 *   ring (App. B.2):      a_ml = 1 iff c_N(m, l) = min(|m - l|, N - |m - l|) <= k,
 *                         l = m included (c_N = 0).
 * The plain definitions: every row sums over all l in increasing order, libm
 * sin/cos, no observables, no window recurrences.  OpenMP splits rows only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double h_val(int p, const double *dsin, const double *dcos, double x) {
    double v = dcos[0];
    for (int k = 1; k <= p; k++) v += dsin[k] * sin(k * x) + dcos[k] * cos(k * x);
    return v;
}

static int64_t circ_dist(int64_t n, int64_t m, int64_t l) {
    const int64_t d = m > l ? m - l : l - m;
    return d < n - d ? d : n - d;
}

/* kind 0: rank one (alpha, beta used), kind 1: ring of half-width k.
   rows == NULL: all rows into out[m]; else out[r] = H_{rows[r]}. */
void oracle_structured_rhs(int kind, int64_t n, int64_t k, const double *alpha, const double *beta,
                           const double *omega, double K, int p, const double *dsin, const double *dcos,
                           const double *theta, const int64_t *rows, int64_t nrows, double *out) {
    const int64_t cnt = rows ? nrows : n;
    const double scale = K / (double)n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < cnt; r++) {
        const int64_t m = rows ? rows[r] : r;
        double acc = 0.0;
        for (int64_t l = 0; l < n; l++) {
            double a;
            if (kind == 0) a = alpha[m] * beta[l];
            else a = circ_dist(n, m, l) <= k ? 1.0 : 0.0;
            if (a != 0.0) acc += a * h_val(p, dsin, dcos, theta[l] - theta[m]);
        }
        out[r] = (omega ? omega[m] : 0.0) + scale * acc;
    }
}

static double order_param(int64_t n, const double *theta) {
    double c = 0.0, s = 0.0;
    for (int64_t l = 0; l < n; l++) { c += cos(theta[l]); s += sin(theta[l]); }
    return sqrt(c * c + s * s) / (double)n;
}

/* Classical RK4 (stepper 0) or explicit Euler (1), theta in place, optional
   r(t) trace at t_0..t_steps.  Returns 0, or -1 when memory runs out. */
int oracle_structured_integrate(int kind, int64_t n, int64_t k, const double *alpha, const double *beta,
                                const double *omega, double K, int p, const double *dsin, const double *dcos,
                                double *theta, double dt, int64_t steps, int stepper, double *r_trace) {
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    if (!k1 || !k2 || !k3 || !k4 || !tmp) {
        free(k1); free(k2); free(k3); free(k4); free(tmp);
        return -1;
    }
#define RHS(x, y) oracle_structured_rhs(kind, n, k, alpha, beta, omega, K, p, dsin, dcos, x, NULL, 0, y)
    if (r_trace) r_trace[0] = order_param(n, theta);
    for (int64_t s = 0; s < steps; s++) {
        RHS(theta, k1);
        if (stepper == 1) {
            for (int64_t i = 0; i < n; i++) theta[i] += dt * k1[i];
        } else {
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + 0.5 * dt * k1[i];
            RHS(tmp, k2);
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + 0.5 * dt * k2[i];
            RHS(tmp, k3);
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + dt * k3[i];
            RHS(tmp, k4);
            for (int64_t i = 0; i < n; i++) theta[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        }
        if (r_trace) r_trace[s + 1] = order_param(n, theta);
    }
#undef RHS
    free(k1); free(k2); free(k3); free(k4); free(tmp);
    return 0;
}
