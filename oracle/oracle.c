/*
 * FP64 CPU oracle for network dynamics of the form
 *     x_m' = f_m(x_m) + (1/N) sum_l a_ml g(x_l, x_m)            (eq. 2.1/2.2)
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load or call
 * this library; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP implementation.
 *
 * Everything here is the plain definition written out: direct summation over
 * the adjacency (or the hypergraph), libm sin/cos/pow, FP64 throughout, no
 * community structure, no Fourier observables, no phase wrapping.  OpenMP
 * splits rows only; every row is summed sequentially in column order, so the
 * result does not depend on the thread count.
 *
 * Models:
 *   phase (Sec. 2 eq. NetworkExample; Kuramoto and higher harmonics, App. A.4):
 *       theta_m' = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m),
 *       h(x) = dcos[0] + sum_{k=1..p} ( dsin[k] sin(k x) + dcos[k] cos(k x) )
 *       (real difference Fourier series, App. A.2).
 *   triadic (App. A.7 higher-order Kuramoto, on a hypergraph):
 *       theta_m' = omega_m + (K1/N) sum_l a_ml sin(theta_l - theta_m)
 *                + (K2/N^2) sum_{(j,k) ordered} B_mjk sin(theta_j + theta_k - 2 theta_m)
 *   Cucker-Smale (App. A.6, eq. Cucker_Smale):
 *       s_m' = v_m,
 *       v_m' = (1/N) sum_l a_ml K (sigma^2 + |s_l - s_m|^2)^(-beta) (v_l - v_m).
 * Time stepping (Sec. 3): classical four-stage Runge-Kutta, or explicit Euler.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* phase models                                                        */
/* ------------------------------------------------------------------ */

/* The coupling function h as its truncated real Fourier series. */
static double h_eval(int p, const double *dsin, const double *dcos, double x) {
    double v = dcos[0];
    for (int k = 1; k <= p; k++) v += dsin[k] * sin(k * x) + dcos[k] * cos(k * x);
    return v;
}

/*
 * Right-hand side H of the phase model.  complete != 0: a_ml = 1 for all
 * l != m (rp/col ignored).  rows == NULL: all rows, out[m]; otherwise
 * out[r] = H_{rows[r]}.
 */
void oracle_phase_rhs(int64_t n, const int64_t *rp, const int32_t *col, int complete,
                      const double *omega, double K, int p, const double *dsin,
                      const double *dcos, const double *theta, const int64_t *rows,
                      int64_t nrows, double *out) {
    int64_t cnt = rows ? nrows : n;
    double scale = K / (double)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        int64_t m = rows ? rows[r] : r;
        double acc = 0.0;
        if (complete) {
            for (int64_t l = 0; l < n; l++)
                if (l != m) acc += h_eval(p, dsin, dcos, theta[l] - theta[m]);
        } else {
            for (int64_t e = rp[m]; e < rp[m + 1]; e++)
                acc += h_eval(p, dsin, dcos, theta[col[e]] - theta[m]);
        }
        out[r] = (omega ? omega[m] : 0.0) + scale * acc;
    }
}

/* Global order parameter |(1/N) sum_l exp(i theta_l)| (App. A.4, r_1). */
double oracle_order_parameter(int64_t n, const double *theta) {
    double c = 0.0, s = 0.0;
    for (int64_t l = 0; l < n; l++) { c += cos(theta[l]); s += sin(theta[l]); }
    return sqrt(c * c + s * s) / (double)n;
}

/*
 * Integrate the phase model: stepper 0 = classical RK4, 1 = explicit Euler.
 * theta is updated in place; r_trace (optional) receives r at t_0..t_steps.
 * Returns 0, or -1 when memory runs out.
 */
int oracle_phase_integrate(int64_t n, const int64_t *rp, const int32_t *col, int complete,
                           const double *omega, double K, int p, const double *dsin,
                           const double *dcos, double *theta, double dt, int64_t steps,
                           int stepper, double *r_trace) {
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    if (!k1 || !k2 || !k3 || !k4 || !tmp) {
        free(k1); free(k2); free(k3); free(k4); free(tmp);
        return -1;
    }
    if (r_trace) r_trace[0] = oracle_order_parameter(n, theta);
    for (int64_t s = 0; s < steps; s++) {
        oracle_phase_rhs(n, rp, col, complete, omega, K, p, dsin, dcos, theta, NULL, 0, k1);
        if (stepper == 1) {
            for (int64_t i = 0; i < n; i++) theta[i] += dt * k1[i];
        } else {
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + 0.5 * dt * k1[i];
            oracle_phase_rhs(n, rp, col, complete, omega, K, p, dsin, dcos, tmp, NULL, 0, k2);
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + 0.5 * dt * k2[i];
            oracle_phase_rhs(n, rp, col, complete, omega, K, p, dsin, dcos, tmp, NULL, 0, k3);
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + dt * k3[i];
            oracle_phase_rhs(n, rp, col, complete, omega, K, p, dsin, dcos, tmp, NULL, 0, k4);
            for (int64_t i = 0; i < n; i++)
                theta[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        }
        if (r_trace) r_trace[s + 1] = oracle_order_parameter(n, theta);
    }
    free(k1); free(k2); free(k3); free(k4); free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* triadic (higher-order) phase model                                  */
/* ------------------------------------------------------------------ */

/* splitmix64 output for state x (Steele, Lea, Flood 2014): the hash that
   defines which intra-community triples are hyperedges. */
static uint64_t splitmix64_at(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t x) { return splitmix64_at(x); }

/* Is the triple {a,b,c} (distinct nodes of one community) a hyperedge? */
int oracle_triple_present(uint64_t seed, uint64_t threshold, int32_t a, int32_t b, int32_t c) {
    int32_t x = a, y = b, z = c, t;
    if (x > y) { t = x; x = y; y = t; }
    if (y > z) { t = y; y = z; z = t; }
    if (x > y) { t = x; x = y; y = t; }
    uint64_t key = (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
    return splitmix64_at(seed ^ key) < threshold;
}

/* probability p -> threshold on the 64-bit hash: floor(p * 2^64), saturating */
uint64_t oracle_triple_threshold(double p) {
    if (p <= 0.0) return 0;
    if (p >= 1.0) return UINT64_MAX;
    return (uint64_t)ldexp(p, 64);
}

typedef struct {
    int64_t n;
    const int32_t *labels;
    int64_t *memb_off;   /* community -> members (user ids) */
    int32_t *memb;
    int64_t *inc_off;    /* node -> incident cross triangles */
    int32_t *inc;        /* triangle index */
    int32_t ncomm;
} tri_index;

static void tri_index_build(tri_index *ix, int64_t n, const int32_t *labels, int64_t ntri,
                            const int32_t *tri) {
    ix->n = n; ix->labels = labels;
    int32_t nc = 0;
    for (int64_t i = 0; i < n; i++) if (labels[i] + 1 > nc) nc = labels[i] + 1;
    ix->ncomm = nc;
    ix->memb_off = calloc((size_t)nc + 1, sizeof(int64_t));
    ix->memb = malloc(sizeof(int32_t) * (n + 1));
    for (int64_t i = 0; i < n; i++) if (labels[i] >= 0) ix->memb_off[labels[i] + 1]++;
    for (int32_t c = 0; c < nc; c++) ix->memb_off[c + 1] += ix->memb_off[c];
    int64_t *pos = malloc(sizeof(int64_t) * ((size_t)nc + 1));
    memcpy(pos, ix->memb_off, sizeof(int64_t) * ((size_t)nc + 1));
    for (int64_t i = 0; i < n; i++) if (labels[i] >= 0) ix->memb[pos[labels[i]]++] = (int32_t)i;
    free(pos);
    ix->inc_off = calloc((size_t)n + 1, sizeof(int64_t));
    ix->inc = malloc(sizeof(int32_t) * (3 * ntri + 1));
    for (int64_t t = 0; t < ntri; t++)
        for (int k = 0; k < 3; k++) ix->inc_off[tri[3 * t + k] + 1]++;
    for (int64_t i = 0; i < n; i++) ix->inc_off[i + 1] += ix->inc_off[i];
    int64_t *ip = malloc(sizeof(int64_t) * (n + 1));
    memcpy(ip, ix->inc_off, sizeof(int64_t) * (n + 1));
    for (int64_t t = 0; t < ntri; t++)
        for (int k = 0; k < 3; k++) ix->inc[ip[tri[3 * t + k]]++] = (int32_t)t;
    free(ip);
}

static void tri_index_free(tri_index *ix) {
    free(ix->memb_off); free(ix->memb); free(ix->inc_off); free(ix->inc);
}

/*
 * Right-hand side of the triadic model.  Hyperedges: every triple of
 * distinct nodes of one community for which oracle_triple_present() holds,
 * plus the explicit list tri[ntri][3].  The sum over (j,k) runs over ordered
 * pairs, so each hyperedge {m,j,k} contributes twice to its centre m.
 */
void oracle_triadic_rhs(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *labels,
                        uint64_t tri_seed, double p_tri, int64_t ntri, const int32_t *tri,
                        const double *omega, double K1, double K2, const double *theta,
                        const int64_t *rows, int64_t nrows, double *out) {
    tri_index ix;
    tri_index_build(&ix, n, labels, ntri, tri);
    uint64_t thr = oracle_triple_threshold(p_tri);
    int64_t cnt = rows ? nrows : n;
    double s1 = K1 / (double)n, s2 = K2 / ((double)n * (double)n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < cnt; r++) {
        int64_t m = rows ? rows[r] : r;
        double pair = 0.0, triad = 0.0;
        for (int64_t e = rp[m]; e < rp[m + 1]; e++) pair += sin(theta[col[e]] - theta[m]);
        int32_t c = labels[m];
        if (c >= 0) {
            const int32_t *mem = ix.memb + ix.memb_off[c];
            int64_t lam = ix.memb_off[c + 1] - ix.memb_off[c];
            for (int64_t a = 0; a < lam; a++) {
                int32_t j = mem[a];
                if (j == m) continue;
                for (int64_t b = 0; b < lam; b++) {
                    int32_t k = mem[b];
                    if (k == m || k == j) continue;
                    if (oracle_triple_present(tri_seed, thr, (int32_t)m, j, k))
                        triad += sin(theta[j] + theta[k] - 2.0 * theta[m]);
                }
            }
        }
        for (int64_t q = ix.inc_off[m]; q < ix.inc_off[m + 1]; q++) {
            const int32_t *t = tri + 3 * (int64_t)ix.inc[q];
            int32_t o[2], w = 0;
            for (int k = 0; k < 3; k++) if (t[k] != m) o[w++] = t[k];
            /* ordered pairs (j,k) and (k,j) */
            triad += 2.0 * sin(theta[o[0]] + theta[o[1]] - 2.0 * theta[m]);
        }
        out[r] = (omega ? omega[m] : 0.0) + s1 * pair + s2 * triad;
    }
    tri_index_free(&ix);
}

int oracle_triadic_integrate(int64_t n, const int64_t *rp, const int32_t *col,
                             const int32_t *labels, uint64_t tri_seed, double p_tri,
                             int64_t ntri, const int32_t *tri, const double *omega, double K1,
                             double K2, double *theta, double dt, int64_t steps, int stepper,
                             double *r_trace) {
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    if (!k1 || !k2 || !k3 || !k4 || !tmp) {
        free(k1); free(k2); free(k3); free(k4); free(tmp);
        return -1;
    }
#define TRI_RHS(x, k) oracle_triadic_rhs(n, rp, col, labels, tri_seed, p_tri, ntri, tri, omega, K1, K2, x, NULL, 0, k)
    if (r_trace) r_trace[0] = oracle_order_parameter(n, theta);
    for (int64_t s = 0; s < steps; s++) {
        TRI_RHS(theta, k1);
        if (stepper == 1) {
            for (int64_t i = 0; i < n; i++) theta[i] += dt * k1[i];
        } else {
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + 0.5 * dt * k1[i];
            TRI_RHS(tmp, k2);
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + 0.5 * dt * k2[i];
            TRI_RHS(tmp, k3);
            for (int64_t i = 0; i < n; i++) tmp[i] = theta[i] + dt * k3[i];
            TRI_RHS(tmp, k4);
            for (int64_t i = 0; i < n; i++)
                theta[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        }
        if (r_trace) r_trace[s + 1] = oracle_order_parameter(n, theta);
    }
#undef TRI_RHS
    free(k1); free(k2); free(k3); free(k4); free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cucker-Smale                                                        */
/* ------------------------------------------------------------------ */

/*
 * State layout: s[d*n + i], v[d*n + i] for coordinate d < dim (planes).
 * Outputs sdot = v and vdot for the requested rows (same plane layout with
 * row count cnt).
 */
void oracle_cs_rhs(int64_t n, int dim, const int64_t *rp, const int32_t *col, int complete,
                   double K, double sigma, double beta, const double *s, const double *v,
                   const int64_t *rows, int64_t nrows, double *sdot, double *vdot) {
    int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        int64_t m = rows ? rows[r] : r;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int64_t e0 = complete ? 0 : rp[m], e1 = complete ? n : rp[m + 1];
        for (int64_t e = e0; e < e1; e++) {
            int64_t l = complete ? e : col[e];
            if (l == m) continue;
            double d2 = 0.0;
            for (int d = 0; d < dim; d++) {
                double dx = s[d * n + l] - s[d * n + m];
                d2 += dx * dx;
            }
            double w = K / pow(sigma * sigma + d2, beta);
            for (int d = 0; d < dim; d++) acc[d] += w * (v[d * n + l] - v[d * n + m]);
        }
        for (int d = 0; d < dim; d++) {
            if (sdot) sdot[d * cnt + r] = v[d * n + m];
            vdot[d * cnt + r] = acc[d] / (double)n;
        }
    }
}

int oracle_cs_integrate(int64_t n, int dim, const int64_t *rp, const int32_t *col, int complete,
                        double K, double sigma, double beta, double *s, double *v, double dt,
                        int64_t steps, int stepper) {
    int64_t sz = (int64_t)dim * n;
    double *ks[4], *kv[4];
    double *ts = malloc(sizeof(double) * sz), *tv = malloc(sizeof(double) * sz);
    int ok = ts && tv;
    for (int q = 0; q < 4; q++) {
        ks[q] = malloc(sizeof(double) * sz);
        kv[q] = malloc(sizeof(double) * sz);
        ok = ok && ks[q] && kv[q];
    }
    if (ok) {
        static const double a[4] = {0.0, 0.5, 0.5, 1.0};
        for (int64_t step = 0; step < steps; step++) {
            if (stepper == 1) {
                oracle_cs_rhs(n, dim, rp, col, complete, K, sigma, beta, s, v, NULL, 0, ks[0], kv[0]);
                for (int64_t i = 0; i < sz; i++) { s[i] += dt * ks[0][i]; v[i] += dt * kv[0][i]; }
                continue;
            }
            for (int q = 0; q < 4; q++) {
                if (q == 0) {
                    memcpy(ts, s, sizeof(double) * sz);
                    memcpy(tv, v, sizeof(double) * sz);
                } else {
                    for (int64_t i = 0; i < sz; i++) {
                        ts[i] = s[i] + a[q] * dt * ks[q - 1][i];
                        tv[i] = v[i] + a[q] * dt * kv[q - 1][i];
                    }
                }
                oracle_cs_rhs(n, dim, rp, col, complete, K, sigma, beta, ts, tv, NULL, 0, ks[q], kv[q]);
            }
            for (int64_t i = 0; i < sz; i++) {
                s[i] += dt / 6.0 * (ks[0][i] + 2.0 * ks[1][i] + 2.0 * ks[2][i] + ks[3][i]);
                v[i] += dt / 6.0 * (kv[0][i] + 2.0 * kv[1][i] + 2.0 * kv[2][i] + kv[3][i]);
            }
        }
    }
    free(ts); free(tv);
    for (int q = 0; q < 4; q++) { free(ks[q]); free(kv[q]); }
    return ok ? 0 : -1;
}

/* number of OpenMP threads the oracle runs with */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* phase model with a general (non-difference) coupling                */
/* ------------------------------------------------------------------ */

/*
 * g(x, y) as the real two-dimensional Fourier series of App. A.2 (eq.
 * FourierRealExpansion, period 2 pi): for partner phase x and own phase y,
 *   g = sum_{a,b=0..p} c11[a][b] cos(a x) cos(b y) + c12[a][b] cos(a x) sin(b y)
 *                    + c21[a][b] sin(a x) cos(b y) + c22[a][b] sin(a x) sin(b y),
 * coefficient arrays row-major [(p+1)*(p+1)].
 */
static double g_eval(int p, const double *c11, const double *c12, const double *c21, const double *c22,
                     double x, double y) {
    double v = 0.0;
    for (int a = 0; a <= p; a++)
        for (int b = 0; b <= p; b++) {
            const int i = a * (p + 1) + b;
            v += c11[i] * cos(a * x) * cos(b * y) + c12[i] * cos(a * x) * sin(b * y) +
                 c21[i] * sin(a * x) * cos(b * y) + c22[i] * sin(a * x) * sin(b * y);
        }
    return v;
}

/* H_m = omega_m + (K/N) sum_l a_ml g(theta_l, theta_m); complete != 0:
   a_ml = 1 for l != m. */
void oracle_phase_rhs_general(int64_t n, const int64_t *rp, const int32_t *col, int complete,
                              const double *omega, double K, int p, const double *c11, const double *c12,
                              const double *c21, const double *c22, const double *theta, const int64_t *rows,
                              int64_t nrows, double *out) {
    int64_t cnt = rows ? nrows : n;
    double scale = K / (double)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        int64_t m = rows ? rows[r] : r;
        double acc = 0.0;
        if (complete) {
            for (int64_t l = 0; l < n; l++)
                if (l != m) acc += g_eval(p, c11, c12, c21, c22, theta[l], theta[m]);
        } else {
            for (int64_t e = rp[m]; e < rp[m + 1]; e++)
                acc += g_eval(p, c11, c12, c21, c22, theta[col[e]], theta[m]);
        }
        out[r] = (omega ? omega[m] : 0.0) + scale * acc;
    }
}
