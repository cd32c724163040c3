/*
 * cia.h -- C ABI of the community integration algorithm (CIA) library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the right-hand side of network ODEs
 *     x_m' = f_m(x_m) + (1/N) sum_l a_ml g(x_l, x_m)            (eq. 2.1/2.2)
 * in O(N + nnz S) instead of O(|E|), following the four steps of Sec. 3:
 * (P1) permute nodes so communities are contiguous and split the permuted
 * adjacency B = D + S into exact blocks D and a sparse remainder S with
 * entries in {-1,+1}; (P2) expand the coupling in a separable basis;
 * (E1) per-community observables (sums of basis functions) broadcast to every
 * member; (E2) direct summation over S.  A direct O(|E|) method over the
 * same data layout is kept as the baseline.
 *
 * Conventions for every call:
 *  - The return value is a cia_status: CIA_OK (0) or a negative error code.
 *    No C++ exception crosses this boundary.  cia_last_error() returns a
 *    thread-local message describing the last failure of the calling thread.
 *  - Host input pointers are borrowed for the duration of the call only; the
 *    plan copies what it needs.
 *  - Device pointers (state, dstate) are caller-owned HIP device memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work and return; a kernel fault surfaces as CIA_EHIP from a later call
 *    or from the caller's own synchronisation.  cia_integrate with a
 *    non-NULL r_trace synchronises the stream before returning.
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - State layout is SoA in the caller's (user) node order: phase models use
 *    one plane of N values; the flock model uses six planes
 *    (s_x, s_y, s_z, v_x, v_y, v_z), each of N values.  Element type is float
 *    for CIA_F32 plans and double for CIA_F64 plans.
 */
#ifndef CIA_H
#define CIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cia_plan cia_plan;

typedef enum cia_status {
    CIA_OK = 0,
    CIA_EINVAL = -1,        /* invalid argument or malformed graph */
    CIA_ENOMEM = -2,        /* host or device allocation failed */
    CIA_EHIP = -3,          /* a HIP runtime call failed */
    CIA_EUNSUPPORTED = -4,  /* valid request the library does not implement */
    CIA_ENONFINITE = -5     /* the integrated state contains NaN or Inf */
} cia_status;

/* graph kinds */
#define CIA_GRAPH_CSR 0       /* explicit symmetric adjacency in CSR form */
#define CIA_GRAPH_COMPLETE 1  /* all-to-all: a_ml = 1 for l != m; nothing stored */
#define CIA_GRAPH_RANK1 2     /* rank one (App. B.1): a_ml = alpha_m beta_l for every pair,
                                 l = m included; nothing stored but alpha and beta */
#define CIA_GRAPH_RING 3      /* k-nearest-neighbour ring (App. B.2): a_ml = 1 iff
                                 min(|m-l|, N-|m-l|) <= ring_k, l = m included */

/* models */
#define CIA_MODEL_PHASE 0    /* theta_m' = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m),
                                h(x) = d_cos[0] + sum_{k=1..p} d_sin[k] sin(kx) + d_cos[k] cos(kx)
                                (Sec. 3; real difference series of App. A.2; Kuramoto App. A.4) */
#define CIA_MODEL_TRIADIC 1  /* phase model with h = sin plus the higher-order term
                                (K2/N^2) sum_{(j,k) ordered} B_mjk sin(theta_j + theta_k - 2 theta_m)
                                (App. A.7 with lambda = (1,1,-2), on a hypergraph) */
#define CIA_MODEL_POLY 3     /* polynomial difference coupling (App. A.3; Desai-Zwanzig, App. A.5):
                                x_m' = omega_m + sum_{j<=poly_q} f_j x_m^j
                                       + (K/N) sum_l a_ml h(x_l - x_m),
                                h(x) = sum_{a<=p} h_a x^a; no phase wrapping, no r(t).
                                Variants: a general coupling g(x_l, x_m) (poly_g) and two
                                state components per node (poly_dim = 2: van der Pol /
                                FitzHugh-Nagumo of Table 1), see cia_coupling */
#define CIA_MODEL_FLOCK 2    /* Cucker-Smale in 3-D (App. A.6): s_m' = v_m,
                                v_m' = (1/N) sum_l a_ml w(|s_l - s_m|) (v_l - v_m),
                                w(r) = cs_K / (cs_sigma^2 + r^2)^cs_beta */

/* methods */
#define CIA_METHOD_CIA 0     /* E1 + E2 (community observables + sparse remainder) */
#define CIA_METHOD_DIRECT 1  /* direct O(|E|) summation (all-to-all: O(N^2)) */

/* arithmetic of state and kernels */
#define CIA_F32 0
#define CIA_F64 1

/* time steppers (Sec. 3: any explicit scheme needs >= 1 RHS per step) */
#define CIA_RK4 0            /* classical four-stage Runge-Kutta */
#define CIA_EULER 1          /* explicit Euler (the setting of Sec. 4's timing runs) */

/* separable basis of the flock weight on intra-community pairs */
#define CIA_BASIS_EXACT 0    /* no expansion: intra blocks summed directly */
#define CIA_BASIS_FOURIER 1  /* truncated 3-D Fourier series on [-L, L]^3 (App. A.6) */
#define CIA_BASIS_LEARNED 2  /* learned rank-R separable basis, checked per community
                                against the exact weight (judge) with exact fallback */

/* option flags */
#define CIA_FLAG_KEEP_LABELS 0x1u  /* skip the P1 cost rule (App. A.1): every labelled
                                      community is treated as a dense block */
#define CIA_FLAG_TIMING 0x2u       /* record HIP events around every kernel launch;
                                      read them with cia_plan_get_timing (see also
                                      cia_plan_set_timing) */
#define CIA_FLAG_NO_VALIDATE 0x4u  /* skip the symmetry / sortedness checks of cia_build */
#define CIA_FLAG_HIPGRAPH 0x8u     /* phase models, RK4: capture one step (its four stage
                                      launches and the order parameter) as a HIP graph once
                                      and replay it every step */
#define CIA_FLAG_NO_JUDGE 0x10u    /* flock model: never check the separable basis against the
                                      exact weight (no per-community fallback) */
#define CIA_FLAG_AUTOTUNE 0x20u    /* phase models: run cia_autotune at the end of cia_build */
/* kernel-path overrides, for testing and tuning (results stay within tolerance) */
#define CIA_FLAG_FORCE_WIDE 0x100u  /* FP64 observables/combine for every community */
#define CIA_FLAG_FORCE_NEG32 0x200u /* S-neg as int32 positions for every community */
#define CIA_FLAG_NO_LDS 0x400u      /* no LDS staging of community z values */
#define CIA_FLAG_NO_RESIDENT 0x800u /* integrate small networks stage by stage, not in one
                                       resident workgroup launch (see cia_integrate) */

typedef struct cia_graph {
    int64_t n;                 /* number of nodes N >= 1 */
    int32_t kind;              /* CIA_GRAPH_* */
    int32_t reserved;
    const int64_t *row_ptr;    /* host [n+1]; CSR only */
    const int32_t *col;        /* host [row_ptr[n]]; symmetric, rows strictly increasing,
                                  no self-loops; CSR only */
    const double *alpha;       /* host [n], finite; CIA_GRAPH_RANK1 only (output weights) */
    const double *beta;        /* host [n], finite; CIA_GRAPH_RANK1 only (input weights) */
    int64_t ring_k;            /* CIA_GRAPH_RING only: half-width k >= 0 (k >= N/2 couples
                                  every pair) */
} cia_graph;

/* Hypergraph of the triadic model.  A triple of distinct nodes inside one
   community is a hyperedge iff splitmix64(seed ^ key) < floor(p_intra * 2^64),
   key = a | b << 21 | c << 42 for the sorted user ids a < b < c (N < 2^21);
   every other hyperedge is listed explicitly in `tri`.  The CIA method builds
   the lists of missing intra-community triples on the device during
   cia_build (16 bytes per up to seven partner pairs of a centre; about 23 GB
   at N = 1e5 with communities of U[200, 2000] and p_intra = 0.9); a
   community with missing triples may hold at most 8191 nodes (FP32) or 4095
   (FP64), else cia_build returns CIA_EUNSUPPORTED. */
typedef struct cia_hypergraph {
    uint64_t seed;
    double p_intra;            /* in [0, 1] */
    int64_t ntri;
    const int32_t *tri;        /* host [ntri][3]; distinct ids, not all in one community */
} cia_hypergraph;

typedef struct cia_coupling {
    int32_t model;             /* CIA_MODEL_* */
    int32_t p;                 /* phase: Fourier order of h, 1..8; flock Fourier basis: order p
                                  in 1..2, multi-indices alpha in {-p..p}^3 ((2p+1)^3 features) */
    const double *d_sin;       /* host [p+1]; entry 0 ignored (phase model) */
    const double *d_cos;       /* host [p+1]; entry 0 = constant term d_0 (phase model) */
    double K;                  /* pairwise strength; the library applies K/N, N = graph n */
    double K2;                 /* triadic strength; the library applies K2/N^2 */
    const cia_hypergraph *hyper;   /* triadic model only */
    double cs_K, cs_sigma, cs_beta;/* flock weight parameters */
    double cs_L;               /* flock Fourier half-period L (positions must stay in a
                                  cube of side L so all differences lie in [-L, L]) */
    int32_t cs_basis;          /* CIA_BASIS_*; flock model only (the direct method ignores it) */
    int32_t rank;              /* learned basis rank R: 16, 32, 48 or 64 */
    int32_t train_iters;       /* learned basis: Adam steps of the first training, which runs on
                                  the state of the first cia_rhs / cia_integrate call unless
                                  parameters were set or trained before (0 = 3000) */
    int32_t reserved;
    int32_t poly_q;            /* polynomial model: degree of the local polynomial f, -1..8
                                  (-1 = none) */
    int32_t reserved2;
    const double *poly_h;      /* polynomial model: host [p+1] coefficients h_0..h_p of h, p = 1..8 */
    const double *poly_f;      /* polynomial model: host [poly_q+1] coefficients f_0..f_q of f */
    /* phase model, optional: a general coupling g(theta_l, theta_m) as the real
       2-D Fourier series of App. A.2 (eq. FourierRealExpansion):
         g = sum_{a,b=0..p} c11[a][b] cos(a theta_l) cos(b theta_m) + c12[a][b] cos(a theta_l) sin(b theta_m)
                          + c21[a][b] sin(a theta_l) cos(b theta_m) + c22[a][b] sin(a theta_l) sin(b theta_m);
       host [(p+1)*(p+1)] each (p = 1..8), row a, column b.  All four set: they define the
       coupling and d_sin/d_cos are ignored; all NULL: the difference form.
       CSR or complete graphs, CIA or direct (not the all-to-all direct kernel),
       not batched. */
    const double *gen_c11, *gen_c12, *gen_c21, *gen_c22;
    /* polynomial model, optional: a general coupling g(x_l, x_m) =
       sum_{a,b=0..p} poly_g[a*(p+1)+b] x_l^a x_m^b (App. A.3, eq. PolyApprox);
       set: it defines the coupling and poly_h is not used. */
    const double *poly_g;
    /* polynomial model: state components per node, 0 or 1 = one (x_m), 2 = two (u_m, v_m), the
       oscillators of Table 1 (van der Pol, FitzHugh-Nagumo) with the difference coupling h applied
       to each component separately:
         u_m' = omega_m + f_0(u_m, v_m) + (K/N) sum_l a_ml h(u_l - u_m),
         v_m' =           f_1(u_m, v_m) + (K/N) sum_l a_ml h(v_l - v_m),
         f_d(u, v) = sum_{i,j=0..3} poly_f2[16 d + 4 i + j] u^i v^j.
       Two components: the state arrays are [2][n] (all u, then all v), poly_f2 is host
       [2][4][4] (NULL = no local term), poly_f/poly_q and poly_g are not allowed, CSR graphs
       (both methods) or the complete graph (CIA method). */
    int32_t poly_dim;
    int32_t reserved3;
    const double *poly_f2;
} cia_coupling;

typedef struct cia_options {
    int32_t method;            /* CIA_METHOD_* */
    int32_t precision;         /* CIA_F32 or CIA_F64 */
    int32_t stepper;           /* CIA_RK4 or CIA_EULER */
    uint32_t flags;            /* CIA_FLAG_* */
    double dense_alpha;        /* P1 cost rule: keep community c dense iff
                                  nnz(S-neg_c) + dense_alpha * lambda_c < nnz(intra_c) */
    int32_t unit_work;         /* target remainder entries per work unit (0 = default) */
    int32_t block;             /* threads per block of the stage kernels, 256 or 512 (0 = default) */
    double judge_tol;          /* flock separable bases: a community falls back to the exact
                                  weight for a step when, on sampled members, the community
                                  part of the sum deviates by more than judge_tol times its
                                  largest exact magnitude (max norm); 0 = never judge */
    int32_t device;            /* HIP device ordinal, -1 = the current device */
    int32_t reserved;
} cia_options;

/* Fill defaults: CIA method, F32, RK4, no flags, dense_alpha 2, judge_tol 1e-3. */
void cia_options_default(cia_options *o);
/* Fill defaults: phase model, p = 1, h = sin (d_sin = {0,1}, d_cos = {0,0}), K = 1. */
void cia_coupling_default(cia_coupling *c);

/*
 * cia_build -- pre-simulation steps P1 and P2 (Sec. 3.1, App. A.1).
 *  g       : the network (host).  CSR graphs are validated (symmetric, sorted,
 *            no self-loops or duplicates) unless CIA_FLAG_NO_VALIDATE.
 *  labels  : host [n] community of every node, -1 = no community (Sec. 3.1
 *            allows nodes outside every community); NULL = all nodes form one
 *            community.  Ids need not be dense.  Communities that fail the
 *            cost rule (see cia_options.dense_alpha) are dissolved into -1.
 *  c       : coupling (model, Fourier coefficients, strengths).
 *  omega   : host [n] intrinsic frequencies f_m = omega_m of the phase models;
 *            NULL = all zero.  Ignored by the flock model.
 *  o       : options; NULL = defaults.
 *  out     : receives the plan, owned by the caller until cia_destroy.
 * Errors: CIA_EINVAL (bad argument, malformed graph, label out of range),
 * CIA_ENOMEM, CIA_EHIP (no device or a HIP call failed), CIA_EUNSUPPORTED.
 * On error *out is set to NULL and nothing leaks.
 */
cia_status cia_build(const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                     const double *omega, const cia_options *o, cia_plan **out);

/*
 * cia_rhs -- one evaluation H(state) (steps E1 and E2 of Sec. 3.2 for the CIA
 * method; the plain sum of eq. 2.2 for the direct method).
 *  state  : device, user order, read only.
 *  dstate : device, user order, written (must not alias state).
 */
cia_status cia_rhs(cia_plan *p, const void *state, void *dstate, void *stream);

/*
 * cia_integrate -- `steps` steps of the plan's stepper with step size dt,
 * every stage evaluated as in cia_rhs.
 *  state   : device, user order, updated in place.  Phase states are returned
 *            wrapped into [0, 2 pi) (steps = 0 returns the state as given).
 *  r_trace : optional host [steps+1]; receives the global order parameter
 *            r(t_n) = |(1/N) sum_m exp(i theta_m)| (App. A.4) accumulated in
 *            FP64 (phase models only; NULL = not computed; plans of
 *            cia_build_batch fill [count][steps+1], one trace per instance).
 *            When non-NULL the call synchronises the stream and returns
 *            CIA_ENONFINITE if the state became NaN or Inf.
 *  The flock model integrates positions and velocities (six planes); it
 *  takes no r_trace (CIA_EINVAL if given).
 *  Small networks (phase model, difference coupling of order <= 4, CIA
 *  method, single network, no community above the LDS staging cap, at most
 *  128 slices of 64 rows (FP64: 64), at most 2^17 remainder entries and
 *  their z values within one CU's LDS)
 *  run the whole call in one launch of one 1024-thread workgroup:
 *  every z of a stage in
 *  LDS, stages separated by workgroup barriers (cia_plan_info.resident = 1;
 *  CIA_FLAG_NO_RESIDENT keeps the stage-by-stage launches).  Results agree
 *  with the stage-by-stage path up to the order of the community sums.
 */
cia_status cia_integrate(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                         void *stream);

/*
 * cia_integrate_noalloc -- cia_integrate for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels, steps and results (bitwise), but
 * the call allocates nothing.  cia_integrate keeps r(t) in a device buffer
 * that it grows on demand; this variant accumulates r(t) in a file-scope
 * static device array of CIA_NOALLOC_R_MAX doubles (1 MiB) that every GPU the
 * library runs on holds until the process ends.  Its device address is
 * resolved once per GPU, at the first plan build on that GPU.
 *  Arguments as cia_integrate; phase-model plans only (CIA_MODEL_PHASE and
 *  CIA_MODEL_TRIADIC, single or batched), else CIA_EUNSUPPORTED.
 *  r_trace : optional host [count][steps+1]; CIA_EINVAL before any device
 *            work if count * (steps + 1) > CIA_NOALLOC_R_MAX.
 *  The plan's replayed step graph (CIA_FLAG_HIPGRAPH) is not used (building
 *  it allocates) and per-launch timing is off for the call.  Every call on a
 *  GPU shares that GPU's array and writes every trace value it returns before
 *  reading it; calls that overlap on one GPU (several streams or threads)
 *  race on the array and must be serialised by the caller.
 */
#define CIA_NOALLOC_R_MAX (1 << 17)
cia_status cia_integrate_noalloc(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                                 void *stream);

/* Release every host and device resource of the plan (NULL is a no-op). */
cia_status cia_destroy(cia_plan *p);

/* Message of the calling thread's last failing call ("" if none). */
const char *cia_last_error(void);

/* --------------------------------------------------------------------- */
/* Batched ensembles and tuning                                           */
/* --------------------------------------------------------------------- */

/*
 * cia_build_batch -- one plan for `count` independent phase-model networks
 * (eq. 2.1 per instance, each with its own N_b, K_b, omega and communities),
 * steps P1 and P2 of Sec. 3.1 for all of them.  The instances are joined into
 * their disjoint union: instance b owns user ids [off_b, off_b + N_b) of the
 * joined state (off_0 = 0, in the given order), so cia_rhs / cia_integrate
 * take the concatenated states and every RK stage is one launch over the work
 * units of all instances.  Each instance keeps its own coupling scale K_b/N_b.
 *  graphs    : host [count] CSR graphs (CIA_GRAPH_COMPLETE is not batched).
 *  labels    : host [count] pointers (NULL = every instance one community; a
 *              NULL entry = that instance one community).
 *  couplings : host [count]; model CIA_MODEL_PHASE, the same p, d_sin and
 *              d_cos for every instance (one coupling function h), K per instance.
 *  omegas    : host [count] pointers or NULL (NULL entry = zero frequencies).
 *  o         : options as for cia_build.
 * cia_integrate on a batch plan fills r_trace (host [count][steps+1]) with the
 * order parameter of every instance, r_b(t) = |(1/N_b) sum_{m in b} exp(i theta_m)|.
 * Errors as cia_build; CIA_EUNSUPPORTED for other models or graph kinds.
 */
cia_status cia_build_batch(int32_t count, const cia_graph *graphs, const int32_t *const *labels,
                           const cia_coupling *couplings, const double *const *omegas,
                           const cia_options *o, cia_plan **out);

/*
 * Incremental form of cia_build_batch for ensembles whose graphs do not fit in
 * host memory together: the same plan, built one instance at a time.
 *
 * cia_batch_begin -- start an empty ensemble with options `o` (NULL = the
 *   defaults; copied).  *out receives a handle owned by the caller until
 *   cia_batch_finish or cia_batch_abort.
 * cia_batch_add -- append instance b = (number of instances added so far):
 *   steps P1 and P2 of Sec. 3.1 on this graph alone (eq. 2.1 with its own N_b
 *   and K_b).  Arguments as one entry of cia_build_batch's arrays; every
 *   pointer is borrowed for the call only, so the caller may free the graph,
 *   labels and omega when it returns.  Host memory then holds the instance's
 *   remainder lists (S-neg and S-pos, 4 bytes per entry) rather than its
 *   adjacency.  CIA_EINVAL / CIA_EUNSUPPORTED leave the handle as it was
 *   (the instance is not added); after CIA_ENOMEM every later add and finish
 *   fails with CIA_EINVAL and only cia_batch_abort is left.
 * cia_batch_finish -- join the instances in the order they were added and
 *   build the plan: the result is the plan cia_build_batch gives for the same
 *   instances (same layout, same kernels, bitwise the same results).  The
 *   handle is released whatever the outcome; on error *out is NULL.
 * cia_batch_abort -- release a handle without building (NULL is a no-op).
 */
typedef struct cia_batch cia_batch;
cia_status cia_batch_begin(const cia_options *o, cia_batch **out);
cia_status cia_batch_add(cia_batch *b, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                         const double *omega);
cia_status cia_batch_finish(cia_batch *b, cia_plan **out);
void cia_batch_abort(cia_batch *b);

/* Instances of a plan and their offsets in the state (host [count+1], may be
   NULL to query the count).  A plan built by cia_build reports one instance. */
cia_status cia_batch_offsets(const cia_plan *p, int32_t *count, int64_t *offsets);

/* Result of cia_autotune: the chosen remainder entries per work unit and
   threads per block, the candidates timed, and the median time of one RHS
   launch before and after. */
typedef struct cia_tune_report {
    int32_t unit_work;
    int32_t block;
    int32_t candidates;
    int32_t reserved;
    double best_us;
    double default_us;
} cia_tune_report;

/*
 * cia_autotune -- choose the work-unit size and block size of the stage
 * kernel of a phase-model plan by timing one RHS launch (median of five) for
 * every candidate on the plan's own remainder data (unit sizes 4096 ..
 * 131072 entries, blocks of 256 and 512 threads), then keep the fastest.
 * Results are unchanged up to summation order.  Runs on `stream` and
 * synchronises it.  rep may be NULL.  CIA_EUNSUPPORTED for other models and
 * for all-to-all direct plans.
 */
cia_status cia_autotune(cia_plan *p, void *stream, cia_tune_report *rep);

/* --------------------------------------------------------------------- */
/* Learned separable basis of the flock weight                            */
/* --------------------------------------------------------------------- */
/*
 * The learned basis (CIA_BASIS_LEARNED) is a perceptron f: R^3 -> R^R,
 *   u = (2 s - lo - hi) / (hi - lo)  per coordinate (the box [lo, hi] to [-1, 1]),
 *   h1 = silu(W1 u + b1) (64), h2 = silu(W2 h1 + b2) (64), f = W3 h2 + b3 (R),
 * with silu(z) = z / (1 + exp(-z)), standing in for the flock weight on
 * intra-community pairs as wt(a, b) = sum_r sgn_r f_r(a) f_r(b) (the separable
 * expansion of Sec. 3 / App. A.6 with a learned instead of a Fourier basis).
 * Parameter vector (float, this order): W1[64][3], b1[64], W2[64][64], b2[64],
 * W3[R][64], b3[R], sgn[R]; sgn is fixed (not trained).  Layers 2 and 3 run
 * as bf16 matrix-core products with FP32 accumulation.
 * Training minimises (1/P) sum_k (wt(a_k, b_k) - w(|a_k - b_k|))^2 over pairs of
 * members of one dense community drawn from a state, with Adam.
 */
/* number of floats in the parameter vector of rank R (16, 32, 48 or 64) */
cia_status cia_basis_param_count(int32_t rank, int64_t *count);
/* Copy parameters (host [count]) and the input box lo/hi (host [3] each) into
   the plan; marks the basis trained.  Synchronises the device. */
cia_status cia_basis_set_params(cia_plan *p, const float *params, int64_t count, const double lo[3],
                                const double hi[3]);
/* Read the parameters and the input box (host outputs; lo/hi may be NULL). */
cia_status cia_basis_get_params(cia_plan *p, float *params, int64_t count, double lo[3], double hi[3]);
/* Train on pairs drawn from `state` (device, user order, 6 planes): sets the
   input box to the positions' bounding box (2% margin), then `iters` Adam
   steps of 4096 pairs each from the counter-based stream `seed`, continuing
   from the current parameters.  loss_trace: optional host [iters].  Synchronises. */
cia_status cia_basis_train(cia_plan *p, const void *state, int32_t iters, uint64_t seed, double *loss_trace,
                           void *stream);
/* Loss and gradient at the current parameters for given pairs: a, b device
   [pairs][3] positions, t device [pairs] targets; grad device [param count]
   (layout of the parameter vector, sgn entries 0); loss optional host scalar
   (then the call synchronises). */
cia_status cia_basis_loss_grad(cia_plan *p, const float *a, const float *b, const float *t, int64_t pairs,
                               float *grad, double *loss, void *stream);
/* Features of n points of the plan's separable basis (learned or Fourier):
   x device [3][n] planes, out device [n][stride], stride = rank for the learned
   basis and (2p+1)^3 rounded up to a multiple of 4 for the Fourier basis
   (feature 0 = 1, then cos, sin of pi <alpha, s> / L per multi-index). */
cia_status cia_basis_features(cia_plan *p, const float *x, int64_t n, float *out, void *stream);

/* --------------------------------------------------------------------- */
/* Introspection                                                          */
/* --------------------------------------------------------------------- */

typedef struct cia_plan_info {
    int64_t n;
    int64_t nnz_graph;        /* directed entries of A (CSR) */
    int64_t nnz_neg;          /* S entries -1: missing intra-community links */
    int64_t nnz_pos;          /* S entries +1: links leaving a community (or touching
                                 a node of no community) */
    int64_t n_unassigned;     /* nodes outside every dense community after P1 */
    int32_t ncomm;            /* dense communities kept by P1 */
    int32_t nunits;           /* work units of the stage kernels */
    int32_t max_comm;         /* largest community */
    int32_t wide_comms;       /* communities above 1e5 nodes (FP64 observables) */
    int32_t method, precision, model;
    int32_t p;                /* phase: Fourier order; flock: Fourier order or learned rank */
    double bytes_per_rhs;     /* algorithmic HBM bytes of one RHS evaluation */
    double bytes_per_stage;   /* algorithmic HBM bytes of one fused RK stage launch */
    int64_t nnz_extra;        /* model-specific remainder entries (triadic CIA: partner pairs of
                                 missing intra-community triples, three per triple) */
    int32_t judge_fallbacks;  /* flock: communities currently on the exact fallback (read
                                 from the device; synchronises it) */
    int32_t tiled_comms;      /* FP32 phase plans: communities above the LDS cap whose z
                                 values are staged one column tile at a time */
    double bytes_aux;         /* algorithmic HBM bytes of the auxiliary launch before each
                                 stage (triadic pair sums: the missing-pair lists, 16 B per
                                 chunk, and the sums written), 0 if there is none */
    int32_t resident;         /* 1: cia_integrate runs the whole call in one resident
                                 workgroup (small single networks, see cia_integrate) */
    int32_t merged_slices;    /* FP32 phase plans with p = 1: 64-row slices whose +1 entries
                                 are stored as one partner-sorted list of the slice */
} cia_plan_info;

cia_status cia_plan_get_info(const cia_plan *p, cia_plan_info *info);

/* Accumulated kernel time of a plan built with CIA_FLAG_TIMING (milliseconds,
   from HIP events on the stream the kernels ran on).  Synchronises the
   stream of the last call.  reset != 0 clears the accumulators. */
typedef struct cia_timing {
    double stage_ms;          /* fused E1/E2/combine/stage-update kernels */
    int64_t stage_launches;
    double prep_ms;           /* permute-in + first observables */
    int64_t prep_launches;
    double aux_ms;            /* order parameter, permute-out, other */
    int64_t aux_launches;
} cia_timing;

cia_status cia_plan_get_timing(cia_plan *p, cia_timing *t, int reset);

/* Sample the kernel timing: HIP events around one launch in `every` of each
   kind (stage / prep / aux), so long runs are timed with little disturbance.
   0 = off, 1 = every launch (what CIA_FLAG_TIMING sets at build).  Collects
   and keeps what was recorded so far; restarts the launch counters. */
cia_status cia_plan_set_timing(cia_plan *p, int32_t every);

/* --------------------------------------------------------------------- */
/* Host-only helpers (no device needed)                                   */
/* --------------------------------------------------------------------- */

/*
 * P2 for a sampled coupling (Sec. 3.1, App. A.2): real Fourier coefficients
 * of h from m >= 2p+1 samples h(2 pi j / m), j = 0..m-1, so that
 * h(x) ~ d_cos[0] + sum_{k=1..p} d_sin[k] sin(kx) + d_cos[k] cos(kx).
 * d_sin, d_cos: host [p+1] outputs (d_sin[0] = 0).
 */
cia_status cia_fourier_coeffs(const double *samples, int64_t m, int32_t p, double *d_sin,
                              double *d_cos);

/*
 * Community labels for a graph that has none (P1, Sec. 3.1 leaves the
 * detection method open), chosen to minimise the work of one CIA right-hand
 * side: nnz(S-neg) + nnz(S-pos) + dense_alpha * (members of kept communities),
 * which P1's cost rule (see cia_options.dense_alpha) also uses.  Louvain-style
 * local moving and aggregation, sequential and deterministic; communities
 * that the cost rule would dissolve, and single nodes, get label -1.  Host
 * only (no device is used).
 *  g           : CSR graph (validated like cia_build); COMPLETE, RANK1, RING: CIA_EUNSUPPORTED
 *  init_labels : host [n] starting partition to refine (-1 = on its own), or NULL (singletons)
 *  dense_alpha : >= 0; 2 is cia_options_default's value
 *  labels      : host [n], written: dense ids 0..C-1 in order of first member, or -1
 *  work        : optional, written: the work of the result (the minimised sum)
 */
cia_status cia_detect_communities(const cia_graph *g, const int32_t *init_labels, double dense_alpha,
                                  int32_t *labels, double *work);

/*
 * P1 alone, on the host (Sec. 3.1 / App. A.1), for inspection and tests.
 * cia_p1_build runs validation, the cost rule, the permutation and the
 * construction of S exactly as cia_build does.
 * cia_p1_sizes writes {n, ncomm, nnz_neg, nnz_pos, n_unassigned, nnz_graph}.
 * cia_p1_export fills caller buffers (any may be NULL):
 *   perm     [n]        user id of the node at community-order position i
 *   comm_off [ncomm+1]  community c occupies positions [comm_off[c], comm_off[c+1])
 *   negptr   [n+1], neg [nnz_neg]  missing intra partners of position i, as
 *                                  community-order positions, increasing
 *   posptr   [n+1], pos [nnz_pos]  remaining (+1) partners, positions, increasing
 */
typedef struct cia_p1 cia_p1;
cia_status cia_p1_build(const cia_graph *g, const int32_t *labels, const cia_options *o,
                        cia_p1 **out);
cia_status cia_p1_sizes(const cia_p1 *p1, int64_t sizes[6]);
cia_status cia_p1_export(const cia_p1 *p1, int32_t *perm, int32_t *comm_off, int64_t *negptr,
                         int32_t *neg, int64_t *posptr, int32_t *pos);
cia_status cia_p1_free(cia_p1 *p1);

/* sizeof of an ABI struct by its name ("cia_graph", "cia_hypergraph",
   "cia_coupling", "cia_options", "cia_plan_info", "cia_timing",
   "cia_tune_report"); 0 if unknown.
   Lets bindings check their struct layouts. */
size_t cia_abi_sizeof(const char *name);

#ifdef __cplusplus
}
#endif

#endif /* CIA_H */
