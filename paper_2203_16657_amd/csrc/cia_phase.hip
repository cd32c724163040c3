// Phase-oscillator networks (Kuramoto and higher harmonics):
//     theta_m' = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m),
//     h(x) = d_0 + sum_{k=1..p} d_sin[k] sin(kx) + d_cos[k] cos(kx).
//
// CIA evaluation (Sec. 3.2, App. A.2 real difference series, App. A.4):
// with z_l = exp(i theta_l), the community observables (E1) are
//     Q_{c,k} = sum_{l in c} z_l^k                      (eq. PrecomputeQuantities)
// and the remainder sums over S (E2) are
//     T_{m,k} = sum_{l in S+(m)} z_l^k - sum_{l in S-(m)} z_l^k.
// Because h is separable, sum over l of h(theta_l - theta_m) collapses to
//     d_0 * count + sum_k Re[(Q_{c,k} + T_{m,k}) conj(z_m)^k (d_cos[k] - i d_sin[k])],
// so E1 and E2 add before the (eq. FastHdense) broadcast-combine.  The
// diagonal of the dense block (l = m) contributes h(0), removed analytically.
//
// Kernel structure on gfx950: one launch per RK stage.  A work unit (a block)
// owns a contiguous row range of one community.  It
//   1. sums the previous stage's per-unit partial observables of its
//      community in a fixed order (deterministic, no float atomics);
//   2. stages the community's z values in LDS (S-neg partners are local);
//   3. gathers T for a chunk of rows with a group of lanes per row;
//   4. combines, adds omega, applies the RK stage update, and computes the
//      next stage's z and its partial observables in the same pass.
// The direct method runs the same kernel with every node outside any
// community and the whole adjacency in the +1 list.
#include <cmath>
#include <cstring>

#include "plan.h"

namespace cia {

constexpr int PMAX = 8;
constexpr double WIDE_COMMUNITY = 1e5;     // FP64 observables above this size
constexpr size_t LDS_STAGE_BYTES = 64 * 1024;

// unit flag bits
constexpr int UF_STAGED = 1;   // community z staged in LDS
constexpr int UF_WIDE = 2;     // FP64 observables and combine (F32 plans)
constexpr int UF_NEG32 = 4;    // S-neg entries stored as int32 positions
constexpr int UF_LPR_SHIFT = 8;

struct alignas(16) Unit {
    int32_t r0, r1, comm, flags;
};

template <typename R>
struct cx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ void dsincos(float t, float *s, float *c) { sincosf(t, s, c); }
__device__ __forceinline__ void dsincos(double t, double *s, double *c) { sincos(t, s, c); }

// compensated accumulation (Knuth TwoSum)
__device__ __forceinline__ void tsum(float &s, float &c, float x) {
    float t = s + x;
    float bp = t - s;
    float e = (s - (t - bp)) + (x - bp);
    s = t;
    c += e;
}
__device__ __forceinline__ void tsum_pair(float &s, float &c, float s2, float c2) {
    float t = s + s2;
    float bp = t - s;
    float e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = c + c2 + e;
}

template <typename R>
__device__ __forceinline__ R wrap_2pi(R t);
template <>
__device__ __forceinline__ float wrap_2pi<float>(float t) {
    const float inv = 0.15915494309189535f;
    const float hi = 6.28318548202514648f;       // float(2 pi)
    const float lo = -1.7484555314695172e-7f;    // 2 pi - float(2 pi)
    float k = floorf(t * inv);
    float r = fmaf(-k, hi, t);
    r = fmaf(-k, lo, r);
    if (r < 0.f) r += hi;
    if (r >= hi) r -= hi;
    return r;
}
template <>
__device__ __forceinline__ double wrap_2pi<double>(double t) {
    const double twopi = 6.283185307179586;
    double r = t - twopi * floor(t / twopi);
    if (r < 0.0) r += twopi;
    if (r >= twopi) r -= twopi;
    return r;
}

enum Mode { M_PREP = 0, M_RHS = 1, M_RK4 = 2, M_EULER = 3 };

template <typename R>
struct PhaseArgs {
    const Unit *units;
    const int32_t *comm_off;
    const int32_t *cu_off;    // community -> range in cu_list
    const int32_t *cu_list;   // unit ids grouped by community
    const int64_t *negptr;
    const uint16_t *neg16;
    const int32_t *neg32;
    const int64_t *posptr;
    const int32_t *pos;
    const int32_t *perm;
    const R *omega;
    R *theta_n;               // theta at the start of the step (community order)
    R *acc;                   // RK4 accumulator
    const R *theta_cur;       // theta of the current stage (wide units only)
    R *theta_next;            // theta of the next stage (wide units only)
    const cx<R> *cs_in;       // z of the current stage
    cx<R> *cs_out;            // z of the next stage
    const double2 *q_in;      // [nunits][P] partial observables of the current stage
    double2 *q_out;
    double2 *r_part;          // [nunits] partial sum of z for the order parameter
    const R *state_in;        // user order (M_PREP)
    R *state_out;             // user order (M_RHS)
    R Kn, dt, d0, hzero;
    R dsin[PMAX + 1], dcos[PMAX + 1];
    int32_t stage, mode, want_r, lds_cap;
};

template <typename R, int P, int BLOCK>
__global__ __launch_bounds__(BLOCK) void phase_stage_kernel(PhaseArgs<R> a) {
    constexpr int NW = BLOCK / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R> *zsh = reinterpret_cast<cx<R> *>(smem);                         // [lds_cap]
    cx<R> *tsh = reinterpret_cast<cx<R> *>(smem + sizeof(cx<R>) * a.lds_cap);  // [BLOCK][P]
    __shared__ double2 qsh[P];
    __shared__ float red_s[NW][2 * P], red_c[NW][2 * P];
    __shared__ double red_d[NW][2 * P];
    __shared__ double2 red_r[NW];

    const Unit U = a.units[blockIdx.x];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int c = U.comm;
    const bool assigned = c >= 0;
    const bool staged = (U.flags & UF_STAGED) != 0;
    const bool wide = (U.flags & UF_WIDE) != 0;
    const bool neg32 = (U.flags & UF_NEG32) != 0;
    const int mode = a.mode;
    int off = 0, lam = 0;
    if (assigned) {
        off = a.comm_off[c];
        lam = a.comm_off[c + 1] - off;
    }

    // ---- 1. community observables of the current stage (E1, fixed order) ----
    if (mode != M_PREP && assigned) {
        if (wid == 0) {
            const int b = a.cu_off[c], e = a.cu_off[c + 1];
            for (int k = 0; k < P; k++) {
                double sx = 0.0, sy = 0.0;
                for (int j = b + lane; j < e; j += 64) {
                    double2 q = a.q_in[(size_t)a.cu_list[j] * P + k];
                    sx += q.x;
                    sy += q.y;
                }
                for (int o = 32; o > 0; o >>= 1) {
                    sx += __shfl_xor(sx, o);
                    sy += __shfl_xor(sy, o);
                }
                if (lane == 0) qsh[k] = make_double2(sx, sy);
            }
        }
        if (staged)
            for (int j = tid; j < lam; j += BLOCK) zsh[j] = a.cs_in[off + j];
    }
    __syncthreads();

    R qx[P], qy[P];
    double qdx[P], qdy[P];
    if (mode != M_PREP && assigned) {
#pragma unroll
        for (int k = 0; k < P; k++) {
            qdx[k] = qsh[k].x;
            qdy[k] = qsh[k].y;
            qx[k] = (R)qdx[k];
            qy[k] = (R)qdy[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < P; k++) qx[k] = qy[k] = (R)0, qdx[k] = qdy[k] = 0.0;
    }

    // partial observables of the next stage
    float ps[2 * P], pc[2 * P];
    double pd[2 * P];
#pragma unroll
    for (int k = 0; k < 2 * P; k++) ps[k] = pc[k] = 0.f, pd[k] = 0.0;
    double rx = 0.0, ry = 0.0;

    const int lpr_log = (U.flags >> UF_LPR_SHIFT) & 15;
    const int lpr = 1 << lpr_log;
    const int groups = BLOCK >> lpr_log;
    const int grp = tid >> lpr_log, gl = tid & (lpr - 1);

    for (int base = U.r0; base < U.r1; base += BLOCK) {
        const int nrows = min(BLOCK, U.r1 - base);
        // ---- 2. E2 gather: T_{m,k} over S for this chunk ----
        if (mode != M_PREP) {
            for (int rr = grp; rr < nrows; rr += groups) {
                const int i = base + rr;
                cx<R> T[P];
#pragma unroll
                for (int k = 0; k < P; k++) T[k].x = T[k].y = (R)0;
                const int64_t nb = a.negptr[i], ne = a.negptr[i + 1];
                for (int64_t e = nb + gl; e < ne; e += lpr) {
                    cx<R> z;
                    if (neg32) z = a.cs_in[a.neg32[e]];
                    else if (staged) z = zsh[a.neg16[e]];
                    else z = a.cs_in[off + (int)a.neg16[e]];
                    cx<R> zk = z;
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        T[k].x -= zk.x;
                        T[k].y -= zk.y;
                        if (k + 1 < P) zk = cmul(zk, z);
                    }
                }
                const int64_t pb = a.posptr[i], pe = a.posptr[i + 1];
                for (int64_t e = pb + gl; e < pe; e += lpr) {
                    cx<R> z = a.cs_in[a.pos[e]];
                    cx<R> zk = z;
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        T[k].x += zk.x;
                        T[k].y += zk.y;
                        if (k + 1 < P) zk = cmul(zk, z);
                    }
                }
                for (int o = lpr >> 1; o > 0; o >>= 1) {
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        T[k].x += __shfl_xor(T[k].x, o);
                        T[k].y += __shfl_xor(T[k].y, o);
                    }
                }
                if (gl == 0) {
#pragma unroll
                    for (int k = 0; k < P; k++) tsh[rr * P + k] = T[k];
                }
            }
            __syncthreads();
        }

        // ---- 3. combine (eq. FastHdense + E2), stage update, next z ----
        if (tid < nrows) {
            const int i = base + tid;
            R theta_new = (R)0;
            bool emit = true;
            if (mode == M_PREP) {
                theta_new = a.state_in[a.perm[i]];
                a.theta_n[i] = theta_new;
            } else {
                R H;
                const R om = a.omega ? a.omega[i] : (R)0;
                if (!wide) {
                    cx<R> z = staged ? zsh[i - off] : a.cs_in[i];
                    R s = (R)0;
                    if (a.d0 != (R)0) {
                        R cnt = (R)((a.posptr[i + 1] - a.posptr[i]) - (a.negptr[i + 1] - a.negptr[i]));
                        s = a.d0 * ((assigned ? (R)lam : (R)0) + cnt);
                    }
                    if (assigned) s -= a.hzero;
                    cx<R> zk = z;
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        cx<R> A = {qx[k] + tsh[tid * P + k].x, qy[k] + tsh[tid * P + k].y};
                        cx<R> zc = {zk.x, -zk.y};
                        cx<R> B = cmul(A, zc);
                        s += a.dcos[k + 1] * B.x + a.dsin[k + 1] * B.y;
                        if (k + 1 < P) zk = cmul(zk, z);
                    }
                    H = om + a.Kn * s;
                } else {
                    // FP64 observables and combine for very large communities
                    double t = (double)a.theta_cur[i];
                    double zs, zc0;
                    sincos(t, &zs, &zc0);
                    cx<double> z = {zc0, zs};
                    double s = 0.0;
                    if (a.d0 != (R)0) {
                        double cnt = (double)((a.posptr[i + 1] - a.posptr[i]) - (a.negptr[i + 1] - a.negptr[i]));
                        s = (double)a.d0 * ((double)lam + cnt);
                    }
                    s -= (double)a.hzero;
                    cx<double> zk = z;
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        cx<double> A = {qdx[k] + (double)tsh[tid * P + k].x, qdy[k] + (double)tsh[tid * P + k].y};
                        cx<double> B = cmul(A, cx<double>{zk.x, -zk.y});
                        s += (double)a.dcos[k + 1] * B.x + (double)a.dsin[k + 1] * B.y;
                        if (k + 1 < P) zk = cmul(zk, z);
                    }
                    H = (R)((double)om + (double)a.Kn * s);
                }
                const R tn = mode == M_RHS ? (R)0 : a.theta_n[i];
                if (mode == M_RHS) {
                    a.state_out[a.perm[i]] = H;
                    emit = false;
                } else if (mode == M_EULER) {
                    theta_new = wrap_2pi<R>(tn + a.dt * H);
                    a.theta_n[i] = theta_new;
                } else {
                    const int st = a.stage;
                    if (st == 0) {
                        a.acc[i] = H;
                        theta_new = tn + (R)0.5 * a.dt * H;
                    } else if (st == 1) {
                        a.acc[i] += (R)2 * H;
                        theta_new = tn + (R)0.5 * a.dt * H;
                    } else if (st == 2) {
                        a.acc[i] += (R)2 * H;
                        theta_new = tn + a.dt * H;
                    } else {
                        theta_new = wrap_2pi<R>(tn + a.dt / (R)6 * (a.acc[i] + H));
                        a.theta_n[i] = theta_new;
                    }
                }
            }
            // next-stage z, its partial observables, order parameter
            if (!emit) {
            } else if (wide) {
                double zs, zc0;
                sincos((double)theta_new, &zs, &zc0);
                a.cs_out[i] = cx<R>{(R)zc0, (R)zs};
                a.theta_next[i] = theta_new;
                cx<double> z = {zc0, zs}, zk = z;
#pragma unroll
                for (int k = 0; k < P; k++) {
                    pd[2 * k] += zk.x;
                    pd[2 * k + 1] += zk.y;
                    if (k + 1 < P) zk = cmul(zk, z);
                }
                rx += zc0;
                ry += zs;
            } else {
                R zs, zc0;
                dsincos(theta_new, &zs, &zc0);
                cx<R> z = {zc0, zs};
                a.cs_out[i] = z;
                if (assigned) {
                    cx<R> zk = z;
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        if constexpr (sizeof(R) == 4) {
                            tsum(ps[2 * k], pc[2 * k], (float)zk.x);
                            tsum(ps[2 * k + 1], pc[2 * k + 1], (float)zk.y);
                        } else {
                            pd[2 * k] += (double)zk.x;
                            pd[2 * k + 1] += (double)zk.y;
                        }
                        if (k + 1 < P) zk = cmul(zk, z);
                    }
                }
                rx += (double)zc0;
                ry += (double)zs;
            }
        }
        if (mode != M_PREP) __syncthreads();   // tsh is reused by the next chunk
    }
    if (mode == M_RHS) return;

    // ---- 4. unit partials: deterministic block reduction ----
    if (assigned) {
        if (sizeof(R) == 4 && !wide) {
#pragma unroll
            for (int k = 0; k < 2 * P; k++) {
                float s = ps[k], cc = pc[k];
                for (int o = 32; o > 0; o >>= 1) {
                    float s2 = __shfl_xor(s, o), c2 = __shfl_xor(cc, o);
                    tsum_pair(s, cc, s2, c2);
                }
                if (lane == 0) {
                    red_s[wid][k] = s;
                    red_c[wid][k] = cc;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 2 * P; k++) {
                double s = pd[k];
                for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
                if (lane == 0) red_d[wid][k] = s;
            }
        }
    }
    if (a.want_r) {
        for (int o = 32; o > 0; o >>= 1) {
            rx += __shfl_xor(rx, o);
            ry += __shfl_xor(ry, o);
        }
        if (lane == 0) red_r[wid] = make_double2(rx, ry);
    }
    __syncthreads();
    if (tid == 0) {
        if (assigned) {
            for (int k = 0; k < P; k++) {
                double vx, vy;
                if (sizeof(R) == 4 && !wide) {
                    float sx = red_s[0][2 * k], cxx = red_c[0][2 * k];
                    float sy = red_s[0][2 * k + 1], cyy = red_c[0][2 * k + 1];
                    for (int w = 1; w < NW; w++) {
                        tsum_pair(sx, cxx, red_s[w][2 * k], red_c[w][2 * k]);
                        tsum_pair(sy, cyy, red_s[w][2 * k + 1], red_c[w][2 * k + 1]);
                    }
                    vx = (double)sx + (double)cxx;
                    vy = (double)sy + (double)cyy;
                } else {
                    vx = red_d[0][2 * k];
                    vy = red_d[0][2 * k + 1];
                    for (int w = 1; w < NW; w++) {
                        vx += red_d[w][2 * k];
                        vy += red_d[w][2 * k + 1];
                    }
                }
                a.q_out[(size_t)blockIdx.x * P + k] = make_double2(vx, vy);
            }
        }
        if (a.want_r) {
            double2 r = red_r[0];
            for (int w = 1; w < NW; w++) {
                r.x += red_r[w].x;
                r.y += red_r[w].y;
            }
            a.r_part[blockIdx.x] = r;
        }
    }
}

// r(t) = |(1/N) sum z| from the unit partials, fixed order, one block.
__global__ __launch_bounds__(256) void order_reduce_kernel(const double2 *r_part, int nunits,
                                                           double invN, double *r_out) {
    __shared__ double sx[256], sy[256];
    double x = 0.0, y = 0.0;
    for (int j = threadIdx.x; j < nunits; j += 256) {
        x += r_part[j].x;
        y += r_part[j].y;
    }
    sx[threadIdx.x] = x;
    sy[threadIdx.x] = y;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sx[threadIdx.x] += sx[threadIdx.x + s];
            sy[threadIdx.x] += sy[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) r_out[0] = sqrt(sx[0] * sx[0] + sy[0] * sy[0]) * invN;
}

template <typename R>
__global__ void permute_out_kernel(int64_t n, const int32_t *perm, const R *src, R *dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

// Direct all-to-all sum for complete graphs (O(N^2)): T_m = sum_{l != m} z_l^k,
// z staged through LDS in tiles; then the same combine as above.
template <typename R, int P, int BLOCK>
__global__ __launch_bounds__(BLOCK) void all2all_kernel(int64_t n, const cx<R> *cs, const R *omega,
                                                        R Kn, R d0, const R *dsin, const R *dcos,
                                                        R *hout) {
    __shared__ cx<R> tile[BLOCK];
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    cx<R> T[P];
#pragma unroll
    for (int k = 0; k < P; k++) T[k].x = T[k].y = (R)0;
    for (int64_t t0 = 0; t0 < n; t0 += BLOCK) {
        int64_t j = t0 + threadIdx.x;
        tile[threadIdx.x] = j < n ? cs[j] : cx<R>{(R)0, (R)0};
        __syncthreads();
        const int lim = (int)min((int64_t)BLOCK, n - t0);
        for (int q = 0; q < lim; q++) {
            if (t0 + q == i) continue;
            cx<R> z = tile[q], zk = z;
#pragma unroll
            for (int k = 0; k < P; k++) {
                T[k].x += zk.x;
                T[k].y += zk.y;
                if (k + 1 < P) zk = cmul(zk, z);
            }
        }
        __syncthreads();
    }
    if (i < n) {
        cx<R> z = cs[i], zk = z;
        R s = d0 * (R)(n - 1);
#pragma unroll
        for (int k = 0; k < P; k++) {
            cx<R> B = cmul(T[k], cx<R>{zk.x, -zk.y});
            s += dcos[k + 1] * B.x + dsin[k + 1] * B.y;
            if (k + 1 < P) zk = cmul(zk, z);
        }
        hout[i] = (omega ? omega[i] : (R)0) + Kn * s;
    }
}

// Elementwise stage update from a precomputed H (used with the all-to-all
// direct kernel): same RK4 / Euler arithmetic as the fused kernel.
template <typename R>
__global__ void stage_update_kernel(int64_t n, int mode, int stage, R dt, const R *H, R *theta_n,
                                    R *acc, cx<R> *cs_out, const int32_t *perm, R *state_out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R h = H[i];
    if (mode == M_RHS) {
        state_out[perm[i]] = h;
        return;
    }
    R tn = theta_n[i], th;
    if (mode == M_EULER) {
        th = wrap_2pi<R>(tn + dt * h);
        theta_n[i] = th;
    } else if (stage == 0) {
        acc[i] = h;
        th = tn + (R)0.5 * dt * h;
    } else if (stage == 1) {
        acc[i] += (R)2 * h;
        th = tn + (R)0.5 * dt * h;
    } else if (stage == 2) {
        acc[i] += (R)2 * h;
        th = tn + dt * h;
    } else {
        th = wrap_2pi<R>(tn + dt / (R)6 * (acc[i] + h));
        theta_n[i] = th;
    }
    R s, c;
    dsincos(th, &s, &c);
    cs_out[i] = cx<R>{c, s};
}

template <typename R>
__global__ void z_from_theta_kernel(int64_t n, const int32_t *perm, const R *state, R *theta_n,
                                    cx<R> *cs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R t = state[perm[i]];
    theta_n[i] = t;
    R s, c;
    dsincos(t, &s, &c);
    cs[i] = cx<R>{c, s};
}

template <typename R>
__global__ void order_partial_kernel(int64_t n, const cx<R> *cs, double2 *part) {
    __shared__ double sx[256], sy[256];
    double x = 0.0, y = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        x += (double)cs[i].x;
        y += (double)cs[i].y;
    }
    sx[threadIdx.x] = x;
    sy[threadIdx.x] = y;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sx[threadIdx.x] += sx[threadIdx.x + s];
            sy[threadIdx.x] += sy[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sx[0], sy[0]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct PhaseState {
    int P = 1;
    bool f64 = false, direct = false, complete_direct = false;
    int block = 256;
    int32_t nunits = 0, ncomm = 0;
    int lds_cap = 0;
    size_t smem = 0;
    double K = 0, Kn = 0, d0 = 0, hzero = 0;
    double dsin[PMAX + 1] = {0}, dcos[PMAX + 1] = {0};
    // device
    Unit *units = nullptr;
    int32_t *comm_off = nullptr, *cu_off = nullptr, *cu_list = nullptr;
    int64_t *negptr = nullptr, *posptr = nullptr;
    uint16_t *neg16 = nullptr;
    int32_t *neg32 = nullptr, *pos = nullptr, *perm = nullptr;
    void *omega = nullptr, *theta_n = nullptr, *acc = nullptr, *theta_st[2] = {nullptr, nullptr};
    void *cs[2] = {nullptr, nullptr};
    double2 *q[2] = {nullptr, nullptr};
    double2 *r_part = nullptr;
    double *r_dev = nullptr;
    int64_t r_cap = 0;
    void *hbuf = nullptr;
    void *coef = nullptr;   // [2][PMAX+1] device copy of dsin/dcos (all-to-all kernel)
};

static int ilog2_ceil(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) l++;
    return l;
}

// Build the work units: contiguous row ranges of one community (or of the
// nodes outside every community), sized by remainder entries, ordered by
// decreasing work so the longest units start first.
static void make_units(const P1 &p1, const std::vector<int64_t> &negptr, const std::vector<int64_t> &posptr,
                       int64_t target, int block, int lds_cap, bool allow_stage, uint32_t flags,
                       std::vector<Unit> &units, std::vector<int32_t> &cu_off, std::vector<int32_t> &cu_list) {
    const int64_t n = p1.n;
    struct U2 {
        Unit u;
        int64_t work;
    };
    std::vector<U2> all;
    const uint32_t opt_flags = flags;
    auto row_work = [&](int64_t i) {
        return (negptr[i + 1] - negptr[i]) + (posptr[i + 1] - posptr[i]) + 8;
    };
    auto emit = [&](int64_t r0, int64_t r1, int32_t comm, int64_t lam) {
        // lanes per row from the mean remainder length of the range
        int64_t ent = 0;
        for (int64_t i = r0; i < r1; i++) ent += (negptr[i + 1] - negptr[i]) + (posptr[i + 1] - posptr[i]);
        double mean = (double)ent / (double)std::max<int64_t>(1, r1 - r0);
        int lg = ilog2_ceil((int64_t)std::ceil(mean / 2.0));
        lg = std::max(0, std::min(6, lg));
        int flags = lg << UF_LPR_SHIFT;
        if (comm >= 0) {
            if ((double)lam > WIDE_COMMUNITY || (opt_flags & CIA_FLAG_FORCE_WIDE)) flags |= UF_WIDE;
            if (lam > 65536 || (opt_flags & CIA_FLAG_FORCE_NEG32)) flags |= UF_NEG32;
            if (allow_stage && lam <= lds_cap && !(flags & (UF_WIDE | UF_NEG32))) flags |= UF_STAGED;
        }
        all.push_back({Unit{(int32_t)r0, (int32_t)r1, comm, flags}, ent + 8 * (r1 - r0)});
    };
    auto split = [&](int64_t b, int64_t e, int32_t comm, int64_t lam) {
        // at least ~block rows per unit unless the range is shorter
        int64_t r = b;
        while (r < e) {
            int64_t w = 0, r1 = r;
            while (r1 < e && (w < target || r1 - r < std::min<int64_t>(64, e - r))) {
                w += row_work(r1);
                r1++;
            }
            emit(r, r1, comm, lam);
            r = r1;
        }
    };
    for (int32_t c = 0; c < p1.ncomm; c++)
        split(p1.comm_off[c], p1.comm_off[c + 1], c, p1.comm_off[c + 1] - p1.comm_off[c]);
    split(p1.ncomm ? p1.comm_off[p1.ncomm] : 0, n, -1, 0);
    std::stable_sort(all.begin(), all.end(), [](const U2 &x, const U2 &y) { return x.work > y.work; });
    units.clear();
    for (auto &x : all) units.push_back(x.u);
    cu_off.assign(p1.ncomm + 1, 0);
    for (auto &u : units)
        if (u.comm >= 0) cu_off[u.comm + 1]++;
    for (int32_t c = 0; c < p1.ncomm; c++) cu_off[c + 1] += cu_off[c];
    cu_list.assign(cu_off[p1.ncomm], 0);
    std::vector<int32_t> fill(cu_off.begin(), cu_off.end());
    // units of one community listed in increasing row order (fixed summation order)
    std::vector<int32_t> ids(units.size());
    for (size_t k = 0; k < units.size(); k++) ids[k] = (int32_t)k;
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) { return units[x].r0 < units[y].r0; });
    for (int32_t k : ids)
        if (units[k].comm >= 0) cu_list[fill[units[k].comm]++] = k;
}

cia_status phase_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                       const double *omega, const cia_options *o) {
    PhaseState *s = new (std::nothrow) PhaseState();
    if (!s) return set_error(CIA_ENOMEM, "host allocation failed");
    p->phase = s;
    const bool f64 = o->precision == CIA_F64;
    s->f64 = f64;
    s->direct = o->method == CIA_METHOD_DIRECT;
    if (c->p < 1 || c->p > PMAX) return set_error(CIA_EINVAL, "coupling.p = %d; supported 1..%d", c->p, PMAX);
    if (!c->d_sin || !c->d_cos) return set_error(CIA_EINVAL, "coupling.d_sin/d_cos are NULL");
    s->P = c->p;
    s->K = c->K;
    s->Kn = c->K / (double)g->n;
    s->d0 = c->d_cos[0];
    s->hzero = c->d_cos[0];
    for (int k = 1; k <= c->p; k++) {
        s->dsin[k] = c->d_sin[k];
        s->dcos[k] = c->d_cos[k];
        s->hzero += c->d_cos[k];
    }
    if (!std::isfinite(s->Kn)) return set_error(CIA_EINVAL, "coupling.K is not finite");
    s->block = o->block == 512 ? 512 : 256;
    if (o->block != 0 && o->block != 256 && o->block != 512)
        return set_error(CIA_EINVAL, "options.block = %d; use 0, 256 or 512", o->block);
    const bool validate = (o->flags & CIA_FLAG_NO_VALIDATE) == 0;
    const bool keep = (o->flags & CIA_FLAG_KEEP_LABELS) != 0;
    const int64_t n = g->n;
    const size_t rs = f64 ? sizeof(double) : sizeof(float);

    P1 p1;
    std::vector<int64_t> negptr, posptr;
    std::vector<int32_t> poscol;
    std::vector<uint16_t> neg16;
    std::vector<int32_t> neg32;
    bool any_neg32 = false;
    try {
        if (!s->direct) {
            CIA_TRY(p1_build(g, labels, o->dense_alpha, keep, validate, true, p1));
            negptr.swap(p1.negptr);
            posptr.swap(p1.posptr);
            poscol.swap(p1.pos);
            for (int32_t cc = 0; cc < p1.ncomm; cc++)
                if (p1.comm_off[cc + 1] - p1.comm_off[cc] > 65536) any_neg32 = true;
            if (o->flags & CIA_FLAG_FORCE_NEG32) any_neg32 = true;
            neg16.resize(p1.neg_local.size());
            if (any_neg32) neg32.resize(p1.neg_local.size());
            for (int64_t i = 0; i < n; i++) {
                int32_t cc = p1.comm_of_pos[i];
                if (cc < 0) continue;
                for (int64_t e = negptr[i]; e < negptr[i + 1]; e++) {
                    neg16[e] = (uint16_t)p1.neg_local[e];
                    if (any_neg32) neg32[e] = p1.neg_local[e] + p1.comm_off[cc];
                }
            }
            std::vector<int32_t>().swap(p1.neg_local);
        } else {
            // direct method: community order for locality, no remainder split;
            // every node is "outside" and its whole row is the +1 list
            CIA_TRY(p1_build(g, labels, o->dense_alpha, true, validate, false, p1));
            if (g->kind == CIA_GRAPH_COMPLETE) {
                s->complete_direct = true;
            } else {
                CIA_TRY(p1_permuted_adjacency(g, p1, posptr, poscol));
                negptr.assign(n + 1, 0);
            }
        }
    } catch (const std::bad_alloc &) {
        return set_error(CIA_ENOMEM, "host allocation failed");
    }

    // LDS staging capacity (community z values)
    int64_t maxlam = 0;
    for (int32_t cc = 0; cc < p1.ncomm; cc++) maxlam = std::max<int64_t>(maxlam, p1.comm_off[cc + 1] - p1.comm_off[cc]);
    const int64_t zbytes = f64 ? 16 : 8;
    // total dynamic LDS (staging + per-chunk T values) stays within 64 KB
    const int64_t tsh_bytes = zbytes * s->block * s->P;
    int64_t cap = ((int64_t)LDS_STAGE_BYTES - tsh_bytes - 4096) / zbytes;
    if (cap < 0) cap = 0;
    if (s->direct) cap = 0;
    s->lds_cap = (int)std::min<int64_t>(cap, maxlam);

    // work units
    std::vector<Unit> units;
    std::vector<int32_t> cu_off, cu_list;
    if (!s->complete_direct) {
        P1 q = p1;
        if (s->direct) {
            q.ncomm = 0;
            q.comm_off.assign(1, 0);
        }
        int64_t target = o->unit_work > 0 ? o->unit_work : 16384;
        make_units(q, negptr, posptr, target, s->block, s->lds_cap,
                   !s->direct && !(o->flags & CIA_FLAG_NO_LDS), o->flags, units, cu_off, cu_list);
        s->ncomm = q.ncomm;
    }
    s->nunits = (int32_t)units.size();
    s->smem = (size_t)zbytes * s->lds_cap + (size_t)zbytes * s->block * s->P;
    if (s->smem > LDS_STAGE_BYTES) return set_error(CIA_EUNSUPPORTED, "LDS request too large");

    // info
    cia_plan_info &inf = p->info;
    inf.n = n;
    inf.nnz_graph = p1.nnz_graph;
    inf.nnz_neg = s->direct ? 0 : (int64_t)neg16.size();
    inf.nnz_pos = (int64_t)poscol.size();
    inf.n_unassigned = n - (p1.ncomm ? p1.comm_off[p1.ncomm] : 0);
    inf.ncomm = s->direct ? 0 : p1.ncomm;
    inf.nunits = s->nunits;
    inf.max_comm = (int32_t)maxlam;
    int wide = 0;
    for (int32_t cc = 0; cc < p1.ncomm; cc++)
        if ((double)(p1.comm_off[cc + 1] - p1.comm_off[cc]) > WIDE_COMMUNITY) wide++;
    inf.wide_comms = s->direct ? 0 : wide;
    inf.method = o->method;
    inf.precision = o->precision;
    inf.model = CIA_MODEL_PHASE;
    inf.p = c->p;
    // algorithmic bytes of one RHS: state in, omega, out, two row pointers
    // per node, remainder indices (2 B local / 4 B global) and, per node, its
    // z value written once and read once
    {
        double per_node = 3.0 * rs + 16.0 + 2.0 * 2 * rs;
        double idx = s->direct ? 4.0 * inf.nnz_pos : 2.0 * inf.nnz_neg + 4.0 * inf.nnz_pos;
        if (any_neg32) idx += 2.0 * inf.nnz_neg;
        inf.bytes_per_rhs = per_node * n + idx;
        // fused RK stage: theta_n, omega, acc in/out, z in/out, row pointers
        double stage_node = rs * 4 + 2.0 * 2 * rs + 16.0;
        inf.bytes_per_stage = stage_node * n + idx;
        if (s->complete_direct) inf.bytes_per_rhs = inf.bytes_per_stage = (double)n * (2 * 2 * rs + 2 * rs);
    }

    // ---- device upload ----
    std::vector<int32_t> perm32(p1.perm.begin(), p1.perm.end());
    CIA_TRY(dupload(p, &s->perm, perm32.data(), n));
    if (!s->complete_direct) {
        CIA_TRY(dupload(p, &s->units, units.data(), units.size()));
        std::vector<int32_t> coff(p1.comm_off.begin(), p1.comm_off.end());
        if (coff.empty()) coff.push_back(0);
        CIA_TRY(dupload(p, &s->comm_off, coff.data(), coff.size()));
        if (cu_off.empty()) cu_off.push_back(0);
        CIA_TRY(dupload(p, &s->cu_off, cu_off.data(), cu_off.size()));
        if (cu_list.empty()) cu_list.push_back(0);
        CIA_TRY(dupload(p, &s->cu_list, cu_list.data(), cu_list.size()));
        CIA_TRY(dupload(p, &s->negptr, negptr.data(), negptr.size()));
        CIA_TRY(dupload(p, &s->posptr, posptr.data(), posptr.size()));
        if (neg16.empty()) neg16.push_back(0);
        CIA_TRY(dupload(p, &s->neg16, neg16.data(), neg16.size()));
        if (any_neg32) CIA_TRY(dupload(p, &s->neg32, neg32.data(), neg32.size()));
        if (poscol.empty()) poscol.push_back(0);
        CIA_TRY(dupload(p, &s->pos, poscol.data(), poscol.size()));
    }
    {
        std::vector<int32_t>().swap(poscol);
        std::vector<uint16_t>().swap(neg16);
        std::vector<int32_t>().swap(neg32);
    }
    // omega in community order
    if (omega) {
        if (f64) {
            std::vector<double> om(n);
            for (int64_t i = 0; i < n; i++) om[i] = omega[p1.perm[i]];
            double *d;
            CIA_TRY(dupload(p, &d, om.data(), n));
            s->omega = d;
        } else {
            std::vector<float> om(n);
            for (int64_t i = 0; i < n; i++) om[i] = (float)omega[p1.perm[i]];
            float *d;
            CIA_TRY(dupload(p, &d, om.data(), n));
            s->omega = d;
        }
        for (int64_t i = 0; i < n; i++)
            if (!std::isfinite(omega[i])) return set_error(CIA_EINVAL, "omega[%lld] is not finite", (long long)i);
    }
    unsigned char *raw;
    CIA_TRY(dalloc(p, &raw, rs * n));
    s->theta_n = raw;
    CIA_TRY(dalloc(p, &raw, rs * n));
    s->acc = raw;
    for (int b = 0; b < 2; b++) {
        CIA_TRY(dalloc(p, &raw, 2 * rs * n));
        s->cs[b] = raw;
        if ((wide || (o->flags & CIA_FLAG_FORCE_WIDE)) && !f64) {
            CIA_TRY(dalloc(p, &raw, rs * n));
            s->theta_st[b] = raw;
        }
        CIA_TRY(dalloc(p, &s->q[b], (size_t)std::max(1, s->nunits) * s->P));
    }
    CIA_TRY(dalloc(p, &s->r_part, (size_t)std::max(1, s->nunits) + 1024));
    if (s->complete_direct) {
        CIA_TRY(dalloc(p, &raw, rs * n));
        s->hbuf = raw;
        if (f64) {
            double cf[2 * (PMAX + 1)];
            for (int k = 0; k <= PMAX; k++) cf[k] = s->dsin[k], cf[PMAX + 1 + k] = s->dcos[k];
            double *d;
            CIA_TRY(dupload(p, &d, cf, 2 * (PMAX + 1)));
            s->coef = d;
        } else {
            float cf[2 * (PMAX + 1)];
            for (int k = 0; k <= PMAX; k++) cf[k] = (float)s->dsin[k], cf[PMAX + 1 + k] = (float)s->dcos[k];
            float *d;
            CIA_TRY(dupload(p, &d, cf, 2 * (PMAX + 1)));
            s->coef = d;
        }
    }
    CIA_HIP(hipDeviceSynchronize());
    return CIA_OK;
}

void phase_free(cia_plan *p) {
    delete p->phase;
    p->phase = nullptr;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------

template <typename R>
static PhaseArgs<R> base_args(PhaseState *s) {
    PhaseArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.units = s->units;
    a.comm_off = s->comm_off;
    a.cu_off = s->cu_off;
    a.cu_list = s->cu_list;
    a.negptr = s->negptr;
    a.neg16 = s->neg16;
    a.neg32 = s->neg32;
    a.posptr = s->posptr;
    a.pos = s->pos;
    a.perm = s->perm;
    a.omega = static_cast<const R *>(s->omega);
    a.theta_n = static_cast<R *>(s->theta_n);
    a.acc = static_cast<R *>(s->acc);
    a.Kn = (R)s->Kn;
    a.d0 = (R)s->d0;
    a.hzero = (R)s->hzero;
    for (int k = 0; k <= PMAX; k++) {
        a.dsin[k] = (R)s->dsin[k];
        a.dcos[k] = (R)s->dcos[k];
    }
    a.lds_cap = s->lds_cap;
    return a;
}

template <typename R, int P>
static cia_status launch_stage_p(cia_plan *p, PhaseState *s, const PhaseArgs<R> &a, hipStream_t st, int kind) {
    if (s->nunits == 0) return CIA_OK;
    CIA_TRY(timing_begin(p, st, kind));
    if (s->block == 512)
        hipLaunchKernelGGL((phase_stage_kernel<R, P, 512>), dim3(s->nunits), dim3(512), s->smem, st, a);
    else
        hipLaunchKernelGGL((phase_stage_kernel<R, P, 256>), dim3(s->nunits), dim3(256), s->smem, st, a);
    CIA_HIP(hipGetLastError());
    return timing_end(p, st);
}

template <typename R>
static cia_status launch_stage(cia_plan *p, PhaseState *s, const PhaseArgs<R> &a, hipStream_t st, int kind) {
    switch (s->P) {
        case 1: return launch_stage_p<R, 1>(p, s, a, st, kind);
        case 2: return launch_stage_p<R, 2>(p, s, a, st, kind);
        case 3: return launch_stage_p<R, 3>(p, s, a, st, kind);
        case 4: return launch_stage_p<R, 4>(p, s, a, st, kind);
        case 5: return launch_stage_p<R, 5>(p, s, a, st, kind);
        case 6: return launch_stage_p<R, 6>(p, s, a, st, kind);
        case 7: return launch_stage_p<R, 7>(p, s, a, st, kind);
        default: return launch_stage_p<R, 8>(p, s, a, st, kind);
    }
}

template <typename R, int P>
static cia_status launch_all2all_p(cia_plan *p, PhaseState *s, hipStream_t st, const void *cs) {
    const int64_t n = p->n;
    const int64_t grid = (n + 255) / 256;
    const R *cf = static_cast<const R *>(s->coef);
    CIA_TRY(timing_begin(p, st, KK_STAGE));
    hipLaunchKernelGGL((all2all_kernel<R, P, 256>), dim3(grid), dim3(256), 0, st, n,
                       static_cast<const cx<R> *>(cs), static_cast<const R *>(s->omega), (R)s->Kn,
                       (R)s->d0, cf, cf + PMAX + 1, static_cast<R *>(s->hbuf));
    CIA_HIP(hipGetLastError());
    return timing_end(p, st);
}

template <typename R>
static cia_status launch_all2all(cia_plan *p, PhaseState *s, hipStream_t st, const void *cs) {
    switch (s->P) {
        case 1: return launch_all2all_p<R, 1>(p, s, st, cs);
        case 2: return launch_all2all_p<R, 2>(p, s, st, cs);
        case 3: return launch_all2all_p<R, 3>(p, s, st, cs);
        case 4: return launch_all2all_p<R, 4>(p, s, st, cs);
        case 5: return launch_all2all_p<R, 5>(p, s, st, cs);
        case 6: return launch_all2all_p<R, 6>(p, s, st, cs);
        case 7: return launch_all2all_p<R, 7>(p, s, st, cs);
        default: return launch_all2all_p<R, 8>(p, s, st, cs);
    }
}

static cia_status launch_order_reduce(cia_plan *p, PhaseState *s, hipStream_t st, int nparts, double *slot) {
    CIA_TRY(timing_begin(p, st, KK_AUX));
    hipLaunchKernelGGL(order_reduce_kernel, dim3(1), dim3(256), 0, st, s->r_part, nparts,
                       1.0 / (double)p->n, slot);
    CIA_HIP(hipGetLastError());
    return timing_end(p, st);
}

template <typename R>
static cia_status launch_order_partial(cia_plan *p, PhaseState *s, hipStream_t st, const void *cs, int *nparts) {
    const int64_t n = p->n;
    int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
    CIA_TRY(timing_begin(p, st, KK_AUX));
    hipLaunchKernelGGL((order_partial_kernel<R>), dim3(grid), dim3(256), 0, st, n,
                       static_cast<const cx<R> *>(cs), s->r_part);
    CIA_HIP(hipGetLastError());
    *nparts = grid;
    return timing_end(p, st);
}

template <typename R>
static cia_status rhs_impl(cia_plan *p, PhaseState *s, const void *state, void *dstate, hipStream_t st) {
    const int64_t n = p->n;
    if (s->complete_direct) {
        const int64_t grid = (n + 255) / 256;
        CIA_TRY(timing_begin(p, st, KK_PREP));
        hipLaunchKernelGGL((z_from_theta_kernel<R>), dim3(grid), dim3(256), 0, st, n, s->perm,
                           static_cast<const R *>(state), static_cast<R *>(s->theta_n),
                           static_cast<cx<R> *>(s->cs[0]));
        CIA_HIP(hipGetLastError());
        CIA_TRY(timing_end(p, st));
        CIA_TRY(launch_all2all<R>(p, s, st, s->cs[0]));
        CIA_TRY(timing_begin(p, st, KK_AUX));
        hipLaunchKernelGGL((stage_update_kernel<R>), dim3(grid), dim3(256), 0, st, n, (int)M_RHS, 0, (R)0,
                           static_cast<const R *>(s->hbuf), static_cast<R *>(s->theta_n),
                           static_cast<R *>(s->acc), static_cast<cx<R> *>(s->cs[1]), s->perm,
                           static_cast<R *>(dstate));
        CIA_HIP(hipGetLastError());
        return timing_end(p, st);
    }
    PhaseArgs<R> a = base_args<R>(s);
    a.mode = M_PREP;
    a.state_in = static_cast<const R *>(state);
    a.cs_out = static_cast<cx<R> *>(s->cs[0]);
    a.q_out = s->q[0];
    a.theta_next = static_cast<R *>(s->theta_st[0]);
    a.r_part = s->r_part;
    CIA_TRY(launch_stage<R>(p, s, a, st, KK_PREP));
    a = base_args<R>(s);
    a.mode = M_RHS;
    a.cs_in = static_cast<const cx<R> *>(s->cs[0]);
    a.q_in = s->q[0];
    a.theta_cur = static_cast<const R *>(s->theta_n);
    a.state_out = static_cast<R *>(dstate);
    return launch_stage<R>(p, s, a, st, KK_STAGE);
}

template <typename R>
static cia_status integrate_impl(cia_plan *p, PhaseState *s, void *state, double dt, int64_t steps,
                                 double *r_trace, hipStream_t st) {
    const int64_t n = p->n;
    const bool want_r = r_trace != nullptr;
    if (want_r && s->r_cap < steps + 1) {
        if (s->r_dev) {
            CIA_HIP(hipFree(s->r_dev));
            for (auto &q : p->dev_allocs)
                if (q == s->r_dev) q = nullptr;
            s->r_dev = nullptr;
        }
        CIA_TRY(dalloc(p, &s->r_dev, (size_t)steps + 1));
        s->r_cap = steps + 1;
    }
    const bool rk4 = p->stepper == CIA_RK4;
    const int64_t grid = (n + 255) / 256;
    int cur = 0;
    if (s->complete_direct) {
        CIA_TRY(timing_begin(p, st, KK_PREP));
        hipLaunchKernelGGL((z_from_theta_kernel<R>), dim3(grid), dim3(256), 0, st, n, s->perm,
                           static_cast<const R *>(state), static_cast<R *>(s->theta_n),
                           static_cast<cx<R> *>(s->cs[0]));
        CIA_HIP(hipGetLastError());
        CIA_TRY(timing_end(p, st));
        int np = 0;
        if (want_r) {
            CIA_TRY(launch_order_partial<R>(p, s, st, s->cs[0], &np));
            CIA_TRY(launch_order_reduce(p, s, st, np, s->r_dev));
        }
        for (int64_t k = 0; k < steps; k++) {
            const int nst = rk4 ? 4 : 1;
            for (int q = 0; q < nst; q++) {
                CIA_TRY(launch_all2all<R>(p, s, st, s->cs[cur]));
                CIA_TRY(timing_begin(p, st, KK_AUX));
                hipLaunchKernelGGL((stage_update_kernel<R>), dim3(grid), dim3(256), 0, st, n,
                                   (int)(rk4 ? M_RK4 : M_EULER), q, (R)dt, static_cast<const R *>(s->hbuf),
                                   static_cast<R *>(s->theta_n), static_cast<R *>(s->acc),
                                   static_cast<cx<R> *>(s->cs[cur ^ 1]), s->perm, static_cast<R *>(nullptr));
                CIA_HIP(hipGetLastError());
                CIA_TRY(timing_end(p, st));
                cur ^= 1;
            }
            if (want_r) {
                CIA_TRY(launch_order_partial<R>(p, s, st, s->cs[cur], &np));
                CIA_TRY(launch_order_reduce(p, s, st, np, s->r_dev + k + 1));
            }
        }
    } else {
        PhaseArgs<R> a = base_args<R>(s);
        a.mode = M_PREP;
        a.state_in = static_cast<const R *>(state);
        a.cs_out = static_cast<cx<R> *>(s->cs[0]);
        a.q_out = s->q[0];
        a.theta_next = static_cast<R *>(s->theta_st[0]);
        a.r_part = s->r_part;
        a.want_r = want_r;
        CIA_TRY(launch_stage<R>(p, s, a, st, KK_PREP));
        if (want_r) CIA_TRY(launch_order_reduce(p, s, st, s->nunits, s->r_dev));
        for (int64_t k = 0; k < steps; k++) {
            const int nst = rk4 ? 4 : 1;
            for (int q = 0; q < nst; q++) {
                a = base_args<R>(s);
                a.mode = rk4 ? M_RK4 : M_EULER;
                a.stage = q;
                a.dt = (R)dt;
                a.cs_in = static_cast<const cx<R> *>(s->cs[cur]);
                a.cs_out = static_cast<cx<R> *>(s->cs[cur ^ 1]);
                a.q_in = s->q[cur];
                a.q_out = s->q[cur ^ 1];
                a.theta_cur = static_cast<const R *>(q == 0 ? s->theta_n : s->theta_st[cur]);
                a.theta_next = static_cast<R *>(s->theta_st[cur ^ 1]);
                a.r_part = s->r_part;
                a.want_r = want_r && q == nst - 1;
                CIA_TRY(launch_stage<R>(p, s, a, st, KK_STAGE));
                cur ^= 1;
            }
            if (want_r) CIA_TRY(launch_order_reduce(p, s, st, s->nunits, s->r_dev + k + 1));
        }
    }
    CIA_TRY(timing_begin(p, st, KK_AUX));
    hipLaunchKernelGGL((permute_out_kernel<R>), dim3(grid), dim3(256), 0, st, n, s->perm,
                       static_cast<const R *>(s->theta_n), static_cast<R *>(state));
    CIA_HIP(hipGetLastError());
    CIA_TRY(timing_end(p, st));
    if (want_r) {
        CIA_HIP(hipMemcpyAsync(r_trace, s->r_dev, sizeof(double) * (steps + 1), hipMemcpyDeviceToHost, st));
        CIA_HIP(hipStreamSynchronize(st));
        for (int64_t k = 0; k <= steps; k++)
            if (!std::isfinite(r_trace[k]))
                return set_error(CIA_ENONFINITE, "state became non-finite (r(t_%lld) = %g)", (long long)k,
                                 r_trace[k]);
    }
    return CIA_OK;
}

cia_status phase_rhs(cia_plan *p, const void *state, void *dstate, hipStream_t st) {
    PhaseState *s = p->phase;
    return s->f64 ? rhs_impl<double>(p, s, state, dstate, st) : rhs_impl<float>(p, s, state, dstate, st);
}

cia_status phase_integrate(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                           hipStream_t st) {
    PhaseState *s = p->phase;
    return s->f64 ? integrate_impl<double>(p, s, state, dt, steps, r_trace, st)
                  : integrate_impl<float>(p, s, state, dt, steps, r_trace, st);
}

}  // namespace cia
