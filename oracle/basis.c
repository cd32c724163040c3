/*
 * FP64 CPU oracle, part 2: separable expansions of the Cucker-Smale weight.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as oracle.c: only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may call it; it shares no
 * code with the HIP implementation).
 *
 * The Cucker-Smale weight w(y) = K / (sigma^2 + |y|^2)^beta of App. A.6 is a
 * function of the position difference y = s_l - s_m.  Two separable stand-ins
 * for it are defined here:
 *
 *  Fourier (App. A.6, eq. Cucker_Smale_etaExpansion): on the cube [-L, L]^3
 *      w(y) ~ sum_{alpha in {-p..p}^3} c_alpha exp(i pi <alpha, y> / L),
 *      c_alpha = (2L)^-3 * integral over [-L, L]^3 of w(y) exp(-i pi <alpha, y>/L) dy.
 *    w is even in every coordinate, so c_alpha is real and depends only on
 *    (|alpha_1|, |alpha_2|, |alpha_3|), and the integral reduces to the
 *    product-cosine integral evaluated below with Gauss-Legendre quadrature.
 *
 *  Learned: a multilayer perceptron phi: R^3 -> R^R,
 *      u   = (2 s - lo - hi) / (hi - lo)           (per coordinate, box to [-1, 1])
 *      h1  = silu(W1 u + b1)                       (64)
 *      h2  = silu(W2 h1 + b2)                      (64)
 *      phi = W3 h2 + b3                            (R)
 *    silu(z) = z / (1 + exp(-z)), and the weight of a pair is the symmetric
 *    separable form  wt(a, b) = sum_r sgn_r phi_r(a) phi_r(b)  with fixed signs
 *    sgn_r, so wt(a, b) = wt(b, a) (antisymmetric coupling, conserved momentum).
 *    Parameter vector layout (floats or doubles, in this order):
 *      W1[64][3], b1[64], W2[64][64], b2[64], W3[R][64], b3[R], sgn[R].
 *    Training loss over pairs (a_k, b_k) with targets t_k:
 *      loss = (1/P) sum_k (wt(a_k, b_k) - t_k)^2;  sgn is not trained.
 *
 * The community-integration semantics (Sec. 3 with the S-neg correction of
 * App. A.1): the expanded weight replaces w on every present pair inside one
 * labelled community, the exact weight is used for every other pair.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HID 64

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes and weights on [-1, 1]                         */
/* ------------------------------------------------------------------ */

/* Newton iteration on P_m from the three-term recurrence
   (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1};  P_m' = m (x P_m - P_{m-1}) / (x^2 - 1). */
void oracle_gauss_legendre(int m, double *x, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < m; i++) {
        double z = cos(pi * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < m; k++) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            /* p1 = P_m(z), p0 = P_{m-1}(z) */
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ------------------------------------------------------------------ */
/* Fourier coefficients of the flock weight                            */
/* ------------------------------------------------------------------ */

static double cs_weight(double K, double sigma, double beta, double r2) {
    return K / pow(sigma * sigma + r2, beta);
}

/* c[(a1 * (p+1) + a2) * (p+1) + a3] = c_alpha for |alpha_l| = a_l in 0..p,
   by nq-point Gauss-Legendre quadrature per axis over [-L, L]. */
int oracle_cs_fourier_coeffs(double K, double sigma, double beta, double L, int p, int nq, double *c) {
    double *gx = malloc(sizeof(double) * nq), *gw = malloc(sizeof(double) * nq);
    double *f = malloc(sizeof(double) * nq * nq * nq);
    double *cs = malloc(sizeof(double) * nq * (p + 1));
    if (!gx || !gw || !f || !cs) { free(gx); free(gw); free(f); free(cs); return -1; }
    oracle_gauss_legendre(nq, gx, gw);
    const double pi = 3.14159265358979323846;
    int q = p + 1;
    /* weighted samples of w on the tensor grid, and the cosine factors */
    for (int i = 0; i < nq; i++)
        for (int j = 0; j < nq; j++)
            for (int k = 0; k < nq; k++) {
                double y1 = L * gx[i], y2 = L * gx[j], y3 = L * gx[k];
                f[((int64_t)i * nq + j) * nq + k] =
                    gw[i] * gw[j] * gw[k] * cs_weight(K, sigma, beta, y1 * y1 + y2 * y2 + y3 * y3);
            }
    for (int a = 0; a < q; a++)
        for (int i = 0; i < nq; i++) cs[a * nq + i] = cos(pi * a * gx[i]);
    for (int a1 = 0; a1 < q; a1++)
        for (int a2 = 0; a2 < q; a2++)
            for (int a3 = 0; a3 < q; a3++) {
                double sum = 0.0;
                for (int i = 0; i < nq; i++)
                    for (int j = 0; j < nq; j++)
                        for (int k = 0; k < nq; k++)
                            sum += f[((int64_t)i * nq + j) * nq + k] * cs[a1 * nq + i] * cs[a2 * nq + j] *
                                   cs[a3 * nq + k];
                /* dy = L^3 d(gx)^3 against the (2L)^-3 normalisation */
                c[(a1 * q + a2) * q + a3] = sum / 8.0;
            }
    free(gx);
    free(gw);
    free(f);
    free(cs);
    return 0;
}

/* The truncated series at a difference y: sum over alpha in {-p..p}^3. */
double oracle_cs_fourier_weight(const double *c, int p, double L, const double *y) {
    const double pi = 3.14159265358979323846;
    int q = p + 1;
    double sum = 0.0;
    for (int a1 = -p; a1 <= p; a1++)
        for (int a2 = -p; a2 <= p; a2++)
            for (int a3 = -p; a3 <= p; a3++) {
                double ca = c[(abs(a1) * q + abs(a2)) * q + abs(a3)];
                sum += ca * cos(pi * (a1 * y[0] + a2 * y[1] + a3 * y[2]) / L);
            }
    return sum;
}

/* ------------------------------------------------------------------ */
/* the learned basis                                                   */
/* ------------------------------------------------------------------ */

int64_t oracle_mlp_param_count(int R) { return HID * 3 + HID + HID * HID + HID + (int64_t)R * HID + 2 * R; }

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *sgn;
} mlp_view;

static mlp_view mlp_split(const double *p, int R) {
    mlp_view v;
    v.W1 = p;
    v.b1 = v.W1 + HID * 3;
    v.W2 = v.b1 + HID;
    v.b2 = v.W2 + HID * HID;
    v.W3 = v.b2 + HID;
    v.b3 = v.W3 + (int64_t)R * HID;
    v.sgn = v.b3 + R;
    return v;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
/* d silu / dz = sigma(z) (1 + z (1 - sigma(z))) */
static double silu_d(double z) {
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* forward pass of one point; keeps the pre-activations for backprop */
static void mlp_point(const mlp_view *m, int R, const double *lo, const double *hi, const double *x,
                      double *u, double *z1, double *h1, double *z2, double *h2, double *phi) {
    for (int d = 0; d < 3; d++) u[d] = (2.0 * x[d] - lo[d] - hi[d]) / (hi[d] - lo[d]);
    for (int o = 0; o < HID; o++) {
        double z = m->b1[o];
        for (int d = 0; d < 3; d++) z += m->W1[o * 3 + d] * u[d];
        z1[o] = z;
        h1[o] = silu(z);
    }
    for (int o = 0; o < HID; o++) {
        double z = m->b2[o];
        for (int k = 0; k < HID; k++) z += m->W2[o * HID + k] * h1[k];
        z2[o] = z;
        h2[o] = silu(z);
    }
    for (int r = 0; r < R; r++) {
        double z = m->b3[r];
        for (int k = 0; k < HID; k++) z += m->W3[r * HID + k] * h2[k];
        phi[r] = z;
    }
}

/* phi for n points given as planes x[d*n + i]; out[i*R + r] */
void oracle_mlp_forward(const double *params, int R, const double *lo, const double *hi, int64_t n,
                        const double *x, double *out) {
    mlp_view m = mlp_split(params, R);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double u[3], z1[HID], h1[HID], z2[HID], h2[HID], xi[3];
        for (int d = 0; d < 3; d++) xi[d] = x[d * n + i];
        mlp_point(&m, R, lo, hi, xi, u, z1, h1, z2, h2, out + i * R);
    }
}

/* loss and gradient over P pairs; a, b given as [P][3]; grad has the layout
   of params (the sgn entries get 0). */
int oracle_mlp_loss_grad(const double *params, int R, const double *lo, const double *hi, int64_t P,
                         const double *a, const double *b, const double *t, double *grad,
                         double *loss_out) {
    mlp_view m = mlp_split(params, R);
    int64_t np = oracle_mlp_param_count(R);
    memset(grad, 0, sizeof(double) * np);
    double *gW1 = grad, *gb1 = gW1 + HID * 3, *gW2 = gb1 + HID, *gb2 = gW2 + HID * HID, *gW3 = gb2 + HID,
           *gb3 = gW3 + (int64_t)R * HID;
    double *phiA = malloc(sizeof(double) * R), *phiB = malloc(sizeof(double) * R);
    double *d3 = malloc(sizeof(double) * R);
    if (!phiA || !phiB || !d3) { free(phiA); free(phiB); free(d3); return -1; }
    double loss = 0.0;
    for (int64_t k = 0; k < P; k++) {
        double uA[3], z1A[HID], h1A[HID], z2A[HID], h2A[HID];
        double uB[3], z1B[HID], h1B[HID], z2B[HID], h2B[HID];
        mlp_point(&m, R, lo, hi, a + 3 * k, uA, z1A, h1A, z2A, h2A, phiA);
        mlp_point(&m, R, lo, hi, b + 3 * k, uB, z1B, h1B, z2B, h2B, phiB);
        double wt = 0.0;
        for (int r = 0; r < R; r++) wt += m.sgn[r] * phiA[r] * phiB[r];
        double e = wt - t[k];
        loss += e * e;
        double g = 2.0 * e / (double)P; /* d loss / d wt */
        /* the two points of the pair, each backpropagated with the other's phi */
        for (int side = 0; side < 2; side++) {
            const double *u = side ? uB : uA, *z1 = side ? z1B : z1A, *h1 = side ? h1B : h1A;
            const double *z2 = side ? z2B : z2A, *h2 = side ? h2B : h2A, *other = side ? phiA : phiB;
            for (int r = 0; r < R; r++) d3[r] = g * m.sgn[r] * other[r];
            double d2[HID], d1[HID];
            for (int r = 0; r < R; r++) {
                gb3[r] += d3[r];
                for (int kk = 0; kk < HID; kk++) gW3[r * HID + kk] += d3[r] * h2[kk];
            }
            for (int kk = 0; kk < HID; kk++) {
                double s = 0.0;
                for (int r = 0; r < R; r++) s += m.W3[r * HID + kk] * d3[r];
                d2[kk] = s * silu_d(z2[kk]);
            }
            for (int o = 0; o < HID; o++) {
                gb2[o] += d2[o];
                for (int kk = 0; kk < HID; kk++) gW2[o * HID + kk] += d2[o] * h1[kk];
            }
            for (int kk = 0; kk < HID; kk++) {
                double s = 0.0;
                for (int o = 0; o < HID; o++) s += m.W2[o * HID + kk] * d2[o];
                d1[kk] = s * silu_d(z1[kk]);
            }
            for (int o = 0; o < HID; o++) {
                gb1[o] += d1[o];
                for (int d = 0; d < 3; d++) gW1[o * 3 + d] += d1[o] * u[d];
            }
        }
    }
    *loss_out = loss / (double)P;
    free(phiA);
    free(phiB);
    free(d3);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cucker-Smale right-hand side with a separable intra-community weight */
/* ------------------------------------------------------------------ */

/*
 * basis 1 = Fourier (coeffs c, order p, half-period L), 2 = learned (params, R,
 * lo, hi).  exact_comm (optional, indexed by label) marks communities whose
 * intra pairs use the exact weight.  Planes s[d*n+i], v[d*n+i]; outputs for
 * the requested rows as in oracle_cs_rhs.
 */
int oracle_cs_rhs_separable(int64_t n, const int64_t *rp, const int32_t *col, int complete,
                            const int32_t *labels, const uint8_t *exact_comm, double K, double sigma,
                            double beta, int basis, const double *c, int p, double L,
                            const double *params, int R, const double *lo, const double *hi,
                            const double *s, const double *v, const int64_t *rows, int64_t nrows,
                            double *sdot, double *vdot) {
    int64_t cnt = rows ? nrows : n;
    double *phi = NULL;
    const double *sgn = NULL;
    if (basis == 2) {
        phi = malloc(sizeof(double) * n * R);
        if (!phi) return -1;
        oracle_mlp_forward(params, R, lo, hi, n, s, phi);
        sgn = mlp_split(params, R).sgn;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < cnt; r++) {
        int64_t m = rows ? rows[r] : r;
        double acc[3] = {0, 0, 0};
        int64_t e0 = complete ? 0 : rp[m], e1 = complete ? n : rp[m + 1];
        int32_t cm = labels ? labels[m] : 0;
        for (int64_t e = e0; e < e1; e++) {
            int64_t l = complete ? e : col[e];
            if (l == m) continue;
            double y[3], d2 = 0.0;
            for (int d = 0; d < 3; d++) {
                y[d] = s[d * n + l] - s[d * n + m];
                d2 += y[d] * y[d];
            }
            int32_t cl = labels ? labels[l] : 0;
            int intra = cm >= 0 && cl == cm && !(exact_comm && exact_comm[cm]);
            double w;
            if (!intra) {
                w = K / pow(sigma * sigma + d2, beta);
            } else if (basis == 1) {
                w = oracle_cs_fourier_weight(c, p, L, y);
            } else {
                w = 0.0;
                for (int q = 0; q < R; q++) w += sgn[q] * phi[l * R + q] * phi[m * R + q];
            }
            for (int d = 0; d < 3; d++) acc[d] += w * (v[d * n + l] - v[d * n + m]);
        }
        for (int d = 0; d < 3; d++) {
            if (sdot) sdot[d * cnt + r] = v[d * n + m];
            vdot[d * cnt + r] = acc[d] / (double)n;
        }
    }
    free(phi);
    return 0;
}
