// Phase model on the structured adjacencies of App. B (extensions of step
// E1): rank-one coupling a_ml = alpha_m beta_l (App. B.1) and the
// k-nearest-neighbour ring a_ml = [min(|m-l|, N-|m-l|) <= k] (App. B.2), both
// with l = m included, and h as its real Fourier series (App. A.2):
//
//   theta_m' = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m).
//
// Each harmonic is treated on its own, as the paper suggests for h with
// several modes.  Nodes stay in user order; a block owns a tile of STILE
// consecutive nodes and writes FP64 tile sums of the next stage's z^k; a
// one-block launch between stages turns them into totals (and, for the
// ring, exclusive tile offsets), in a fixed order.
//
//  * rank one: R_k = sum_l beta_l z_l^k, then s_m = d0 sum beta +
//    sum_k (dsin_k Im + dcos_k Re)(R_k conj(z_m^k)) and H_m = omega_m +
//    (K/N) alpha_m s_m (eq. rank1fast);
//  * ring: the window sum F_{m,k} = sum_{l=m-k}^{m+k} z_l^k (indices mod N)
//    is Pc(m+k+1) - Pc(m-k) for the circular prefix sum Pc(x) =
//    floor(x/N) Tot_k + sum_{l < x mod N} z_l^k.  The paper's serial window
//    recurrence becomes, per block, two block scans over the block's two
//    shifted windows started from the tile offsets.
//
// The direct variants sum h over every coupled pair (O(N^2) for rank one,
// O(N k) for the ring) and share the stage update.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fastmath.h"
#include "plan.h"
#include "wave.h"

namespace cia {

namespace {

constexpr int SB = 256;            // threads per stage block
constexpr int SNPT = 4;            // consecutive nodes per thread (the vector helpers take 4)
constexpr int STILE = SB * SNPT;   // nodes per block
static_assert(STILE == 1 << 10, "ring_windows shifts by 10 for / STILE");
constexpr int SPMAX = 8;           // harmonics
constexpr int SCAN_CH = 256;       // most chunks of the tile-sum scan

enum SKind { SK_RANK1 = 0, SK_RING = 1, SK_RANK1_DIRECT = 2, SK_RING_DIRECT = 3 };
enum SMode { SM_PREP = 0, SM_RHS = 1, SM_RK4 = 2, SM_EULER = 3 };

template <typename R>
struct zc {
    R x, y;
};

template <typename R>
__device__ __forceinline__ zc<R> zmul(zc<R> a, zc<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ zc<R> zpow(zc<R> z, int k) {
    zc<R> r = z;
    for (int i = 1; i < k; i++) r = zmul(r, z);
    return r;
}
__device__ __forceinline__ void zsincos(float t, float *s, float *c) { fast_sincosf(t, s, c); }
__device__ __forceinline__ void zsincos(double t, double *s, double *c) { sincos(t, s, c); }

template <typename R>
__device__ __forceinline__ R wrap_phase(R t);
template <>
__device__ __forceinline__ float wrap_phase<float>(float t) {
    const float hi = 6.28318548202514648f;      // float(2 pi)
    const float lo = -1.7484555314695172e-7f;   // 2 pi - float(2 pi)
    const float k = floorf(t * 0.15915494309189535f);
    float r = fmaf(-k, lo, fmaf(-k, hi, t));
    if (r < 0.f) r += hi;
    if (r >= hi) r -= hi;
    return r;
}
template <>
__device__ __forceinline__ double wrap_phase<double>(double t) {
    const double twopi = 6.283185307179586;
    double r = t - twopi * floor(t / twopi);
    if (r < 0.0) r += twopi;
    if (r >= twopi) r -= twopi;
    return r;
}

__device__ __forceinline__ double2 d2add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Four consecutive entries from j0 (a multiple of 4, in a library-owned
// allocation, so full groups are aligned vector accesses); entries at or
// past n read as zero and are not written.
template <typename R>
__device__ __forceinline__ void load4(const R *p, int64_t j0, int64_t n, R (&v)[4]) {
    if (j0 + 4 <= n) {
        if constexpr (sizeof(R) == 4) {
            const float4 q = *reinterpret_cast<const float4 *>(p + j0);
            v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
        } else {
            const double2 q0 = *reinterpret_cast<const double2 *>(p + j0);
            const double2 q1 = *reinterpret_cast<const double2 *>(p + j0 + 2);
            v[0] = q0.x, v[1] = q0.y, v[2] = q1.x, v[3] = q1.y;
        }
    } else {
        for (int e = 0; e < 4; e++) v[e] = j0 + e < n ? p[j0 + e] : (R)0;
    }
}
template <typename R>
__device__ __forceinline__ void store4(R *p, int64_t j0, int64_t n, const R (&v)[4]) {
    if (j0 + 4 <= n) {
        if constexpr (sizeof(R) == 4) {
            *reinterpret_cast<float4 *>(p + j0) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
            *reinterpret_cast<double2 *>(p + j0) = make_double2(v[0], v[1]);
            *reinterpret_cast<double2 *>(p + j0 + 2) = make_double2(v[2], v[3]);
        }
    } else {
        for (int e = 0; e < 4; e++)
            if (j0 + e < n) p[j0 + e] = v[e];
    }
}
template <typename R>
__device__ __forceinline__ void load4z(const zc<R> *p, int64_t j0, int64_t n, zc<R> (&v)[4]) {
    if (j0 + 4 <= n) {
        if constexpr (sizeof(R) == 4) {
            const float4 q0 = *reinterpret_cast<const float4 *>(p + j0);
            const float4 q1 = *reinterpret_cast<const float4 *>(p + j0 + 2);
            v[0] = {q0.x, q0.y}, v[1] = {q0.z, q0.w}, v[2] = {q1.x, q1.y}, v[3] = {q1.z, q1.w};
        } else {
            for (int e = 0; e < 4; e++) {
                const double2 q = *reinterpret_cast<const double2 *>(p + j0 + e);
                v[e] = {q.x, q.y};
            }
        }
    } else {
        for (int e = 0; e < 4; e++) v[e] = j0 + e < n ? p[j0 + e] : zc<R>{(R)0, (R)0};
    }
}
template <typename R>
__device__ __forceinline__ void store4z(zc<R> *p, int64_t j0, int64_t n, const zc<R> (&v)[4]) {
    if (j0 + 4 <= n) {
        if constexpr (sizeof(R) == 4) {
            *reinterpret_cast<float4 *>(p + j0) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
            *reinterpret_cast<float4 *>(p + j0 + 2) = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
        } else {
            for (int e = 0; e < 4; e++) *reinterpret_cast<double2 *>(p + j0 + e) = make_double2(v[e].x, v[e].y);
        }
    } else {
        for (int e = 0; e < 4; e++)
            if (j0 + e < n) p[j0 + e] = v[e];
    }
}

// Block sum of one double2 per thread (fixed order), broadcast to all threads.
template <int NT>
__device__ __forceinline__ double2 block_sum(double2 v, double2 *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double2 r = sh[0];
    for (int w = 1; w < NT / 64; w++) r = d2add(r, sh[w]);
    return r;
}

// Batched block sums and scans, one barrier pair for all: sv[m] (m < MS)
// become their block sums, xv[m] (m < MX) their exclusive scans in thread
// order, with the block totals in xt[m].  The order of every sum is fixed.
// sh holds NT / 64 * (MS + MX) double2.
template <int NT, int MS, int MX>
__device__ __forceinline__ void block_sums_scans(double2 (&sv)[MS], double2 (&xv)[MX], double2 (&xt)[MX],
                                                 double2 *sh) {
    constexpr int M = MS + MX;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < MS; m++) sv[m] = wave_sum(sv[m]);
    double2 ex[MX], wt[MX];
#pragma unroll
    for (int m = 0; m < MX; m++) {
        const double2 inc = wave_incl_scan(xv[m]);
        ex[m] = wave_shr1(inc);
        wt[m] = make_double2(lane63(inc.x), lane63(inc.y));
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < MS; m++) sh[wid * M + m] = sv[m];
#pragma unroll
        for (int m = 0; m < MX; m++) sh[wid * M + MS + m] = wt[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MS; m++) {
        double2 r = sh[m];
        for (int w = 1; w < NT / 64; w++) r = d2add(r, sh[w * M + m]);
        sv[m] = r;
    }
#pragma unroll
    for (int m = 0; m < MX; m++) {
        double2 off = make_double2(0.0, 0.0), tot = make_double2(0.0, 0.0);
        for (int w = 0; w < NT / 64; w++) {
            const double2 q = sh[w * M + MS + m];
            if (w < wid) off = d2add(off, q);
            tot = d2add(tot, q);
        }
        xt[m] = tot;
        xv[m] = d2add(off, ex[m]);
    }
}

// Block sums of M double2 per thread in one barrier pair (fixed order);
// sh holds NT / 64 * M double2.
template <int NT, int M>
__device__ __forceinline__ void block_sums(double2 (&v)[M], double2 *sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < M; m++) v[m] = wave_sum(v[m]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < M; m++) sh[wid * M + m] = v[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; m++) {
        double2 r = sh[m];
        for (int w = 1; w < NT / 64; w++) r = d2add(r, sh[w * M + m]);
        v[m] = r;
    }
}

template <typename R>
struct SArgs {
    int64_t n, kw;                      // nodes; ring half-width
    int32_t ntiles, mode, stage;
    int32_t tcols;                      // ring: the window shift in tiles, at least 1
    R dt, Kn, d0w;                      // d0w: dcos[0] times the row weight (sum beta, or 2 kw + 1)
    R dsin[SPMAX + 1], dcos[SPMAX + 1];
    const R *omega, *alpha, *beta;      // [n]; alpha, beta for rank one only
    const R *state_in;                  // prep: theta in user order
    R *state_out;                       // rhs: H
    R *theta_n, *acc;                   // theta at the step start; RK4 accumulator
    const zc<R> *z_in;                  // z of the current stage
    zc<R> *z_out;                       // z of the next stage
    const double2 *tot;                 // scan output: [P+1] totals, then ring tile offsets [(ntiles+1)][P]
    double2 *part;                      // [ntiles][P+1]: tile sums of w z^k, k = 1..P, then of z
};

// Ring window sums for this thread's nodes j = a0 + SNPT t + e, harmonic by
// harmonic, added into s as (dsin_k Im + dcos_k Re)(F_{j,k} conj(z_j^k)).
// Every z the block needs (the start tile of each shifted window up to the
// window start, and the two windows) is loaded at once; per harmonic, the
// two partial-tile sums and the two window scans share one barrier pair.
template <typename R, int P>
__device__ __forceinline__ void ring_windows(const SArgs<R> &a, int64_t a0, const zc<R> (&zj)[SNPT], R (&s)[SNPT],
                                             double2 *sh) {
    const int t = threadIdx.x;
    const int64_t n = a.n, kw = a.kw;
    const double2 *off = a.tot + (P + 1);
    int64_t q[2], tl[2];
    zc<R> zt[2][SNPT], zw[2][SNPT];
    bool in_t[2][SNPT];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        // 0 <= a0 < n and 0 <= kw < n / 2, so the window start st wraps at
        // most once: q = floor(st / n) is -1 or 0 (r = 0), 0 or 1 (r = 1)
        const int64_t st = r == 0 ? a0 - kw : a0 + kw + 1;
        q[r] = st < 0 ? -1 : (st >= n ? 1 : 0);
        const int64_t sp = st - q[r] * n;   // in [0, n)
        tl[r] = sp >> 10;                   // sp / STILE
#pragma unroll
        for (int u = 0; u < SNPT; u++) {
            const int64_t i = tl[r] * STILE + t + (int64_t)u * SB;
            in_t[r][u] = i < sp;
            zt[r][u] = i < sp ? a.z_in[i] : zc<R>{(R)0, (R)0};
        }
        const int64_t x0 = sp + (int64_t)SNPT * t;   // reduced mod n below
#pragma unroll
        for (int e = 0; e < SNPT; e++) {
            int64_t x = x0 + e;
            while (x >= n) x -= n;
            zw[r][e] = a.z_in[x];
        }
    }
#pragma unroll 1
    for (int k = 1; k <= P; k++) {
        // per window: the start tile's sum of z^k up to the window start
        // (block sum) and this thread's window sum (block scan); powers by
        // the recurrence of zpow
        double2 pt[2], ts[2], btot[2];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            double2 v = make_double2(0.0, 0.0), w = make_double2(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < SNPT; u++)
                if (in_t[r][u]) {
                    const zc<R> z = zpow(zt[r][u], k);
                    v.x += (double)z.x;
                    v.y += (double)z.y;
                }
#pragma unroll
            for (int e = 0; e < SNPT; e++) {
                const zc<R> z = zpow(zw[r][e], k);
                w.x += (double)z.x;
                w.y += (double)z.y;
            }
            pt[r] = v;
            ts[r] = w;
        }
        block_sums_scans<SB, 2, 2>(pt, ts, btot, sh);
        const double2 Tot = off[(int64_t)a.ntiles * P + (k - 1)];
        double2 pc[2][SNPT];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const double2 o = off[tl[r] * P + (k - 1)];
            const double2 base =
                make_double2((double)q[r] * Tot.x + o.x + pt[r].x, (double)q[r] * Tot.y + o.y + pt[r].y);
            double2 run = d2add(base, ts[r]);
#pragma unroll
            for (int e = 0; e < SNPT; e++) {
                pc[r][e] = run;
                const zc<R> z = zpow(zw[r][e], k);
                run.x += (double)z.x;
                run.y += (double)z.y;
            }
        }
#pragma unroll
        for (int e = 0; e < SNPT; e++) {
            const R fx = (R)(pc[1][e].x - pc[0][e].x), fy = (R)(pc[1][e].y - pc[0][e].y);
            // F conj(z_j^k)
            const zc<R> zjk = zpow(zj[e], k);
            const R wr = fx * zjk.x + fy * zjk.y, wi = fy * zjk.x - fx * zjk.y;
            s[e] += a.dsin[k] * wi + a.dcos[k] * wr;
        }
    }
}

// Tile of block i for the ring.  Workgroups are dealt to the 8 XCDs in turn
// (block i runs on XCD i mod 8, in increasing i), so XCD x is given a
// contiguous run of an order that lists tile T = q D + c (D = tcols) column
// by column: c outer, q inner (tcols = 1: the natural order, so each XCD
// holds a contiguous run of tiles).  A block of tile T reads z from its own
// tile and from T - D - 1, T - D, T + D and T + D + 1, all in columns
// c - 1 .. c + 1, so the five readers of a tile run on one XCD within about
// 2 N / (D STILE) blocks of each other and share its lines in that XCD's L2
// (the plain block order puts them on different XCDs, each fetching the
// tile on its own).
__device__ __forceinline__ int64_t ring_tile(uint32_t i, uint32_t nb, uint32_t D) {
    constexpr uint32_t X = 8;
    const uint32_t x = i % X, j = i / X;
    const uint32_t base = nb / X, extra = nb % X;
    const uint32_t pos = x * base + (x < extra ? x : extra) + j;
    const uint32_t Q = nb / D, rem = nb % D;
    uint32_t c, q;
    if (pos < rem * (Q + 1)) {
        c = pos / (Q + 1);
        q = pos - c * (Q + 1);
    } else {
        const uint32_t p2 = pos - rem * (Q + 1);
        c = rem + p2 / Q;
        q = p2 - (c - rem) * Q;
    }
    return (int64_t)q * D + c;
}

// h(theta_l - theta_j) from z_l and z_j (powers by recurrence)
template <typename R, int P>
__device__ __forceinline__ R h_pair(const SArgs<R> &a, zc<R> zl, zc<R> zj) {
    // e^{i(theta_l - theta_j)} = z_l conj(z_j)
    const zc<R> d = {zl.x * zj.x + zl.y * zj.y, zl.y * zj.x - zl.x * zj.y};
    R v = a.dcos[0];
    zc<R> dk = d;
#pragma unroll
    for (int k = 1; k <= P; k++) {
        v += a.dsin[k] * dk.y + a.dcos[k] * dk.x;
        if (k < P) dk = zmul(dk, d);
    }
    return v;
}

template <typename R, int P, int KIND>
__global__ __launch_bounds__(SB) void struct_stage_kernel(SArgs<R> a) {
    constexpr bool RANK1 = KIND == SK_RANK1 || KIND == SK_RANK1_DIRECT;
    __shared__ double2 sh[SB / 64 * (4 > P + 1 ? 4 : P + 1)];   // block_sums_scans<SB, 2, 2>, block_sums<SB, P + 1>
    __shared__ zc<R> zst[SB];
    __shared__ R bst[SB];
    const int t = threadIdx.x;
    const int64_t n = a.n;
    const int64_t tile = KIND == SK_RING ? ring_tile(blockIdx.x, (uint32_t)a.ntiles, (uint32_t)a.tcols)
                                         : (int64_t)blockIdx.x;
    const int64_t a0 = tile * STILE;
    const int64_t j0 = a0 + (int64_t)SNPT * t;
    const int mode = a.mode;

    R tn[SNPT], om[SNPT], av[SNPT], s[SNPT], al[SNPT];
    zc<R> zj[SNPT];
#pragma unroll
    for (int e = 0; e < SNPT; e++) {
        tn[e] = om[e] = av[e] = s[e] = (R)0;
        al[e] = (R)1;
        zj[e] = zc<R>{(R)0, (R)0};
    }
    if (mode == SM_PREP) {
#pragma unroll
        for (int e = 0; e < SNPT; e++)
            if (j0 + e < n) tn[e] = a.state_in[j0 + e];   // caller's buffer: no alignment assumed
    } else {
        if (mode != SM_RHS) load4(a.theta_n, j0, n, tn);
        if (a.omega) load4(a.omega, j0, n, om);
        if (mode == SM_RK4 && a.stage > 0) load4(a.acc, j0, n, av);
        if (RANK1) load4(a.alpha, j0, n, al);
        load4z(a.z_in, j0, n, zj);
    }

    if (mode != SM_PREP) {
        // ---- s_j = sum_l a_jl h(theta_l - theta_j), without the factor alpha_j ----
        if constexpr (KIND == SK_RANK1) {
            zc<R> zk[SNPT];
#pragma unroll
            for (int e = 0; e < SNPT; e++) {
                s[e] = a.d0w;
                zk[e] = zj[e];
            }
#pragma unroll
            for (int k = 1; k <= P; k++) {
                const double2 Rk = a.tot[k - 1];
                const R rx = (R)Rk.x, ry = (R)Rk.y;
#pragma unroll
                for (int e = 0; e < SNPT; e++) {
                    const R wr = rx * zk[e].x + ry * zk[e].y, wi = ry * zk[e].x - rx * zk[e].y;
                    s[e] += a.dsin[k] * wi + a.dcos[k] * wr;
                    if (k < P) zk[e] = zmul(zk[e], zj[e]);
                }
            }
        } else if constexpr (KIND == SK_RING) {
#pragma unroll
            for (int e = 0; e < SNPT; e++) s[e] = a.d0w;
            ring_windows<R, P>(a, a0, zj, s, sh);
        } else if constexpr (KIND == SK_RANK1_DIRECT) {
            // every partner l, staged SB at a time; FP32 sums per stage chunk, FP64 across
            double sd[SNPT] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t l0 = 0; l0 < n; l0 += SB) {
                __syncthreads();
                const int64_t l = l0 + t;
                zst[t] = l < n ? a.z_in[l] : zc<R>{(R)0, (R)0};
                bst[t] = l < n ? a.beta[l] : (R)0;
                __syncthreads();
                const int cnt = (int)(n - l0 < SB ? n - l0 : SB);
                R sf[SNPT] = {(R)0, (R)0, (R)0, (R)0};
                for (int u = 0; u < cnt; u++) {
                    const zc<R> zl = zst[u];
                    const R b = bst[u];
#pragma unroll
                    for (int e = 0; e < SNPT; e++) sf[e] += b * h_pair<R, P>(a, zl, zj[e]);
                }
#pragma unroll
                for (int e = 0; e < SNPT; e++) sd[e] += (double)sf[e];
            }
#pragma unroll
            for (int e = 0; e < SNPT; e++) s[e] = (R)sd[e];
        } else {
            // ring, direct: the 2 kw + 1 partners of each node (2 kw + 1 < n)
#pragma unroll
            for (int e = 0; e < SNPT; e++) {
                const int64_t j = j0 + e;
                if (j >= n) continue;
                double sd = 0.0;
                for (int64_t d0 = -a.kw; d0 <= a.kw; d0 += SB) {
                    const int64_t d1 = d0 + SB - 1 < a.kw ? d0 + SB - 1 : a.kw;
                    R sf = (R)0;
                    for (int64_t d = d0; d <= d1; d++) {
                        int64_t l = (j + d) % n;
                        if (l < 0) l += n;
                        sf += h_pair<R, P>(a, a.z_in[l], zj[e]);
                    }
                    sd += (double)sf;
                }
                s[e] = (R)sd;
            }
        }
    }

    // ---- combine, stage update, next z and its tile sums ----
    R tnew[SNPT], H[SNPT];
#pragma unroll
    for (int e = 0; e < SNPT; e++) {
        H[e] = om[e] + a.Kn * al[e] * s[e];
        tnew[e] = tn[e];
    }
    if (mode == SM_RHS) {
#pragma unroll
        for (int e = 0; e < SNPT; e++)
            if (j0 + e < n) a.state_out[j0 + e] = H[e];
        return;
    }
    if (mode == SM_PREP) {
        store4(a.theta_n, j0, n, tn);
    } else if (mode == SM_EULER) {
#pragma unroll
        for (int e = 0; e < SNPT; e++) tnew[e] = wrap_phase<R>(tn[e] + a.dt * H[e]);
        store4(a.theta_n, j0, n, tnew);
    } else if (a.stage < 3) {
        R acc[SNPT];
        const R c = a.stage == 2 ? a.dt : (R)0.5 * a.dt;
#pragma unroll
        for (int e = 0; e < SNPT; e++) {
            acc[e] = a.stage == 0 ? H[e] : av[e] + (R)2 * H[e];
            tnew[e] = tn[e] + c * H[e];
        }
        store4(a.acc, j0, n, acc);
    } else {
#pragma unroll
        for (int e = 0; e < SNPT; e++) tnew[e] = wrap_phase<R>(tn[e] + a.dt / (R)6 * (av[e] + H[e]));
        store4(a.theta_n, j0, n, tnew);
    }
    zc<R> zn[SNPT];
    R wt[SNPT];
    if (KIND == SK_RANK1) load4(a.beta, j0, n, wt);
#pragma unroll
    for (int e = 0; e < SNPT; e++) {
        R sn, c0;
        zsincos(tnew[e], &sn, &c0);
        const bool ok = j0 + e < n;
        zn[e] = ok ? zc<R>{c0, sn} : zc<R>{(R)0, (R)0};
        if (KIND != SK_RANK1) wt[e] = (R)1;
    }
    store4z(a.z_out, j0, n, zn);
    // tile sums: slot k-1 of w z^k (k = 1..P; the E1 variants), slot P of z
    if constexpr (KIND == SK_RANK1 || KIND == SK_RING) {
        double2 v[P + 1];
        zc<R> zk[SNPT];
#pragma unroll
        for (int e = 0; e < SNPT; e++) zk[e] = zn[e];
#pragma unroll
        for (int k = 1; k <= P; k++) {
            v[k - 1] = make_double2(0.0, 0.0);
#pragma unroll
            for (int e = 0; e < SNPT; e++) {
                v[k - 1].x += (double)(wt[e] * zk[e].x);
                v[k - 1].y += (double)(wt[e] * zk[e].y);
            }
            if (k < P) {
#pragma unroll
                for (int e = 0; e < SNPT; e++) zk[e] = zmul(zk[e], zn[e]);
            }
        }
        v[P] = make_double2(0.0, 0.0);
#pragma unroll
        for (int e = 0; e < SNPT; e++) {
            v[P].x += (double)zn[e].x;
            v[P].y += (double)zn[e].y;
        }
        block_sums<SB, P + 1>(v, sh);
        if (t == 0) {
#pragma unroll
            for (int m = 0; m <= P; m++) a.part[(size_t)tile * (P + 1) + m] = v[m];
        }
    } else {
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int e = 0; e < SNPT; e++) {
            v.x += (double)zn[e].x;
            v.y += (double)zn[e].y;
        }
        v = block_sum<SB>(v, sh);
        if (t == 0) a.part[(size_t)tile * (P + 1) + P] = v;
    }
}

// Totals of the tile sums (every slot) and, for the ring, exclusive tile
// offsets of slots 0..P-1, in two launches spread over the CUs (a single
// block cannot pull the tile sums of a large network fast enough).  The
// tiles form nch <= SCAN_CH chunks of ct consecutive tiles; one 64-lane
// block per chunk.  The order of every sum is fixed.

// Launch 1: chunk sums csum[c][sl] of every slot (lane-strided over the
// chunk's tiles, then a wave sum).
template <int P>
__global__ __launch_bounds__(64) void struct_chunk_kernel(const double2 *part, int32_t ntiles, int32_t ct,
                                                          double2 *csum) {
    const int l = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * ct, t1 = t0 + ct < ntiles ? t0 + ct : ntiles;
    double2 v[P + 1];
#pragma unroll
    for (int sl = 0; sl <= P; sl++) v[sl] = make_double2(0.0, 0.0);
    for (int64_t T = t0 + l; T < t1; T += 64)
#pragma unroll
        for (int sl = 0; sl <= P; sl++) v[sl] = d2add(v[sl], part[T * (P + 1) + sl]);
#pragma unroll
    for (int sl = 0; sl <= P; sl++) {
        v[sl] = wave_sum(v[sl]);
        if (l == 0) csum[(int64_t)blockIdx.x * (P + 1) + sl] = v[sl];
    }
}

// Launch 2: for the ring, block c adds the chunk sums before it (its chunk
// offset) and writes the exclusive offsets of its tiles (wave scans of 64
// tiles at a time); the last chunk's block also writes the totals (tot, the
// ring's final offset slot) and r_out = |total of slot P| / n.  Without the
// ring one block does only the last part.
template <int P>
__global__ __launch_bounds__(64) void struct_offsets_kernel(const double2 *part, const double2 *csum, int32_t ntiles,
                                                            int32_t ct, int32_t nch, int ring, double invN,
                                                            double2 *tot, double *r_out) {
    const int l = threadIdx.x;
    const int c = ring ? (int)blockIdx.x : nch - 1;
    double2 o[P + 1];
#pragma unroll
    for (int sl = 0; sl <= P; sl++) o[sl] = make_double2(0.0, 0.0);
    for (int c2 = l; c2 < c; c2 += 64)
#pragma unroll
        for (int sl = 0; sl <= P; sl++) o[sl] = d2add(o[sl], csum[(int64_t)c2 * (P + 1) + sl]);
#pragma unroll
    for (int sl = 0; sl <= P; sl++) o[sl] = wave_sum(o[sl]);
    double2 *off = tot + (P + 1);
    if (ring) {
        const int64_t t0 = (int64_t)c * ct, t1 = t0 + ct < ntiles ? t0 + ct : ntiles;
        double2 run[P];
#pragma unroll
        for (int sl = 0; sl < P; sl++) run[sl] = o[sl];
        for (int64_t b = t0; b < t1; b += 64) {
            const int64_t T = b + l;
#pragma unroll
            for (int sl = 0; sl < P; sl++) {
                const double2 inc = wave_incl_scan(T < t1 ? part[T * (P + 1) + sl] : make_double2(0.0, 0.0));
                if (T < t1) off[T * P + sl] = d2add(run[sl], wave_shr1(inc));
                run[sl] = d2add(run[sl], make_double2(lane63(inc.x), lane63(inc.y)));
            }
        }
    }
    if (c == nch - 1 && l == 0) {
#pragma unroll
        for (int sl = 0; sl <= P; sl++) {
            const double2 T = d2add(o[sl], csum[(int64_t)c * (P + 1) + sl]);
            tot[sl] = T;
            if (ring && sl < P) off[(int64_t)ntiles * P + sl] = T;
            if (sl == P && r_out) r_out[0] = sqrt(T.x * T.x + T.y * T.y) * invN;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct StructState {
    int kind = SK_RANK1;
    int P = 1;
    bool f64 = false;
    double Kn = 0, d0w = 0;
    double dsin[SPMAX + 1] = {0}, dcos[SPMAX + 1] = {0};
    int64_t kw = 0;
    int32_t ntiles = 0;
    int32_t ct = 0, nch = 0;            // tiles per scan chunk, chunks (<= SCAN_CH)
    void *omega = nullptr, *alpha = nullptr, *beta = nullptr;
    void *theta_n = nullptr, *acc = nullptr, *z[2] = {nullptr, nullptr};
    double2 *part[2] = {nullptr, nullptr};
    double2 *tot = nullptr;
    double2 *csum = nullptr;            // [nch][P+1] chunk sums
    double *r_dev = nullptr;
    int64_t r_cap = 0;
};

template <typename R>
static cia_status upload_as(cia_plan *p, void **dst, const double *src, int64_t n) {
    std::vector<R> h(n);
    for (int64_t i = 0; i < n; i++) h[i] = (R)src[i];
    R *d;
    CIA_TRY(dupload(p, &d, h.data(), (size_t)n));
    *dst = d;
    return CIA_OK;
}

cia_status struct_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                        const double *omega, const cia_options *o) {
    if (c->model != CIA_MODEL_PHASE)
        return set_error(CIA_EUNSUPPORTED, "rank-one and ring graphs take the phase model only");
    if (labels) return set_error(CIA_EINVAL, "rank-one and ring graphs take no community labels (pass NULL)");
    if (c->gen_c11 || c->gen_c12 || c->gen_c21 || c->gen_c22)
        return set_error(CIA_EUNSUPPORTED, "rank-one and ring graphs take the difference form of the coupling");
    if (c->p < 1 || c->p > SPMAX) return set_error(CIA_EINVAL, "coupling.p = %d; supported 1..%d", c->p, SPMAX);
    if (!c->d_sin || !c->d_cos) return set_error(CIA_EINVAL, "coupling.d_sin/d_cos are NULL");
    for (int k = 0; k <= c->p; k++)
        if (!std::isfinite(c->d_sin[k]) || !std::isfinite(c->d_cos[k]))
            return set_error(CIA_EINVAL, "coupling coefficients must be finite");
    const int64_t n = g->n;
    if (n > ((int64_t)1 << 40)) return set_error(CIA_EUNSUPPORTED, "n = %lld is too large", (long long)n);
    StructState *s = new (std::nothrow) StructState();
    if (!s) return set_error(CIA_ENOMEM, "host allocation failed");
    p->structd = s;
    s->f64 = o->precision == CIA_F64;
    s->P = c->p;
    for (int k = 0; k <= c->p; k++) {
        s->dsin[k] = c->d_sin[k];
        s->dcos[k] = c->d_cos[k];
    }
    s->Kn = c->K / (double)n;
    if (!std::isfinite(s->Kn)) return set_error(CIA_EINVAL, "coupling.K is not finite");
    if (omega)
        for (int64_t i = 0; i < n; i++)
            if (!std::isfinite(omega[i])) return set_error(CIA_EINVAL, "omega[%lld] is not finite", (long long)i);

    // rank one, or a ring; a ring of 2k + 1 >= n couples every pair (rank one
    // with unit weights)
    std::vector<double> ones;
    const double *alpha = g->alpha, *beta = g->beta;
    bool rank1 = g->kind == CIA_GRAPH_RANK1;
    if (g->kind == CIA_GRAPH_RING) {
        if (g->ring_k < 0) return set_error(CIA_EINVAL, "graph.ring_k = %lld < 0", (long long)g->ring_k);
        s->kw = g->ring_k;
        if (2 * g->ring_k + 1 >= n || g->ring_k >= n) {
            rank1 = true;
            ones.assign(n, 1.0);
            alpha = beta = ones.data();
        }
    }
    if (rank1) {
        if (!alpha || !beta) return set_error(CIA_EINVAL, "rank-one graph: alpha/beta is NULL");
        double sb = 0.0;
        for (int64_t i = 0; i < n; i++) {
            if (!std::isfinite(alpha[i]) || !std::isfinite(beta[i]))
                return set_error(CIA_EINVAL, "rank-one graph: alpha/beta[%lld] is not finite", (long long)i);
            sb += beta[i];
        }
        s->d0w = c->d_cos[0] * sb;
        s->kind = o->method == CIA_METHOD_DIRECT ? SK_RANK1_DIRECT : SK_RANK1;
    } else {
        s->d0w = c->d_cos[0] * (double)(2 * s->kw + 1);
        s->kind = o->method == CIA_METHOD_DIRECT ? SK_RING_DIRECT : SK_RING;
    }
    const int64_t ntiles = (n + STILE - 1) / STILE;
    if (ntiles > INT32_MAX) return set_error(CIA_EUNSUPPORTED, "n = %lld is too large", (long long)n);
    s->ntiles = (int32_t)ntiles;

    const size_t rs = s->f64 ? sizeof(double) : sizeof(float);
    if (s->f64) {
        if (omega) CIA_TRY(upload_as<double>(p, &s->omega, omega, n));
        if (rank1) {
            CIA_TRY(upload_as<double>(p, &s->alpha, alpha, n));
            CIA_TRY(upload_as<double>(p, &s->beta, beta, n));
        }
    } else {
        if (omega) CIA_TRY(upload_as<float>(p, &s->omega, omega, n));
        if (rank1) {
            CIA_TRY(upload_as<float>(p, &s->alpha, alpha, n));
            CIA_TRY(upload_as<float>(p, &s->beta, beta, n));
        }
    }
    unsigned char *raw;
    CIA_TRY(dalloc(p, &raw, rs * n));
    s->theta_n = raw;
    CIA_TRY(dalloc(p, &raw, rs * n));
    s->acc = raw;
    for (int b = 0; b < 2; b++) {
        CIA_TRY(dalloc(p, &raw, 2 * rs * n));
        s->z[b] = raw;
        CIA_TRY(dalloc(p, &s->part[b], (size_t)ntiles * (s->P + 1)));
        CIA_HIP(hipMemset(s->part[b], 0, sizeof(double2) * (size_t)ntiles * (s->P + 1)));
    }
    CIA_TRY(dalloc(p, &s->tot, (size_t)(s->P + 1) + (size_t)(ntiles + 1) * s->P));
    s->ct = (int32_t)((ntiles + SCAN_CH - 1) / SCAN_CH);
    s->nch = (int32_t)((ntiles + s->ct - 1) / s->ct);
    CIA_TRY(dalloc(p, &s->csum, (size_t)s->nch * (s->P + 1)));

    cia_plan_info &inf = p->info;
    inf.n = n;
    inf.nnz_graph = rank1 ? n * n : n * (2 * s->kw + 1);
    inf.method = o->method;
    inf.precision = o->precision;
    inf.model = CIA_MODEL_PHASE;
    inf.p = s->P;
    inf.nunits = s->ntiles;
    inf.ncomm = 1;
    inf.max_comm = (int32_t)std::min<int64_t>(n, INT32_MAX);
    // algorithmic bytes per node: theta_n, omega, acc in and out, z read and
    // written once, and for rank one alpha and beta
    const double per_node = (4.0 + 2.0 * 2.0) * rs + (rank1 ? 2.0 * rs : 0.0);
    inf.bytes_per_stage = per_node * (double)n;
    inf.bytes_per_rhs = (4.0 * rs + 2.0 * rs + (rank1 ? 2.0 * rs : 0.0)) * (double)n;
    return CIA_OK;
}

void struct_free(cia_plan *p) {
    delete p->structd;
    p->structd = nullptr;
}

template <typename R, int P>
static void launch_stage_kind(const StructState *s, const SArgs<R> &a, hipStream_t st) {
    const dim3 g(s->ntiles), b(SB);
    switch (s->kind) {
        case SK_RANK1: hipLaunchKernelGGL((struct_stage_kernel<R, P, SK_RANK1>), g, b, 0, st, a); break;
        case SK_RING: hipLaunchKernelGGL((struct_stage_kernel<R, P, SK_RING>), g, b, 0, st, a); break;
        case SK_RANK1_DIRECT: hipLaunchKernelGGL((struct_stage_kernel<R, P, SK_RANK1_DIRECT>), g, b, 0, st, a); break;
        default: hipLaunchKernelGGL((struct_stage_kernel<R, P, SK_RING_DIRECT>), g, b, 0, st, a); break;
    }
}

template <typename R>
static cia_status launch_stage(cia_plan *p, const StructState *s, const SArgs<R> &a, hipStream_t st, int kind) {
    CIA_TRY(timing_begin(p, st, kind));
    switch (s->P) {
        case 1: launch_stage_kind<R, 1>(s, a, st); break;
        case 2: launch_stage_kind<R, 2>(s, a, st); break;
        case 3: launch_stage_kind<R, 3>(s, a, st); break;
        case 4: launch_stage_kind<R, 4>(s, a, st); break;
        case 5: launch_stage_kind<R, 5>(s, a, st); break;
        case 6: launch_stage_kind<R, 6>(s, a, st); break;
        case 7: launch_stage_kind<R, 7>(s, a, st); break;
        default: launch_stage_kind<R, 8>(s, a, st); break;
    }
    CIA_HIP(hipGetLastError());
    return timing_end(p, st);
}

// totals / offsets of the tile sums in part[b]; r_out optional
template <int P>
static void launch_scan_p(const StructState *s, int b, double invN, double *r_out, hipStream_t st) {
    const int ring = s->kind == SK_RING ? 1 : 0;
    hipLaunchKernelGGL(struct_chunk_kernel<P>, dim3(s->nch), dim3(64), 0, st, s->part[b], s->ntiles, s->ct, s->csum);
    hipLaunchKernelGGL(struct_offsets_kernel<P>, dim3(ring ? s->nch : 1), dim3(64), 0, st, s->part[b], s->csum,
                       s->ntiles, s->ct, s->nch, ring, invN, s->tot, r_out);
}
static cia_status launch_scan(cia_plan *p, const StructState *s, int b, double *r_out, hipStream_t st) {
    CIA_TRY(timing_begin(p, st, KK_AUX));
    const double invN = 1.0 / (double)p->n;
    switch (s->P) {
        case 1: launch_scan_p<1>(s, b, invN, r_out, st); break;
        case 2: launch_scan_p<2>(s, b, invN, r_out, st); break;
        case 3: launch_scan_p<3>(s, b, invN, r_out, st); break;
        case 4: launch_scan_p<4>(s, b, invN, r_out, st); break;
        case 5: launch_scan_p<5>(s, b, invN, r_out, st); break;
        case 6: launch_scan_p<6>(s, b, invN, r_out, st); break;
        case 7: launch_scan_p<7>(s, b, invN, r_out, st); break;
        default: launch_scan_p<8>(s, b, invN, r_out, st); break;
    }
    CIA_HIP(hipGetLastError());
    return timing_end(p, st);
}

template <typename R>
static SArgs<R> base_args(cia_plan *p, const StructState *s) {
    SArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.n = p->n;
    a.kw = s->kw;
    a.ntiles = s->ntiles;
    // column order when the window shift is large against one XCD's share of
    // the tiles; otherwise tcols = 1, each XCD a contiguous run of tiles
    const int64_t D = std::max<int64_t>(1, s->kw / STILE);
    a.tcols = 4 * (D + 1) <= s->ntiles / 8 ? 1 : (int32_t)D;
    a.Kn = (R)s->Kn;
    a.d0w = (R)s->d0w;
    for (int k = 0; k <= SPMAX; k++) {
        a.dsin[k] = (R)s->dsin[k];
        a.dcos[k] = (R)s->dcos[k];
    }
    a.omega = static_cast<const R *>(s->omega);
    a.alpha = static_cast<const R *>(s->alpha);
    a.beta = static_cast<const R *>(s->beta);
    a.theta_n = static_cast<R *>(s->theta_n);
    a.acc = static_cast<R *>(s->acc);
    a.tot = s->tot;
    return a;
}

template <typename R>
static cia_status prep(cia_plan *p, const StructState *s, const void *state, hipStream_t st) {
    SArgs<R> a = base_args<R>(p, s);
    a.mode = SM_PREP;
    a.state_in = static_cast<const R *>(state);
    a.z_out = static_cast<zc<R> *>(s->z[0]);
    a.part = s->part[0];
    return launch_stage<R>(p, s, a, st, KK_PREP);
}

static bool needs_scan(const StructState *s) { return s->kind == SK_RANK1 || s->kind == SK_RING; }

template <typename R>
static cia_status rhs_impl(cia_plan *p, StructState *s, const void *state, void *dstate, hipStream_t st) {
    CIA_TRY(prep<R>(p, s, state, st));
    if (needs_scan(s)) CIA_TRY(launch_scan(p, s, 0, nullptr, st));
    SArgs<R> a = base_args<R>(p, s);
    a.mode = SM_RHS;
    a.z_in = static_cast<const zc<R> *>(s->z[0]);
    a.state_out = static_cast<R *>(dstate);
    return launch_stage<R>(p, s, a, st, KK_STAGE);
}

template <typename R>
static cia_status integrate_impl(cia_plan *p, StructState *s, void *state, double dt, int64_t steps,
                                 double *r_trace, hipStream_t st) {
    const bool want_r = r_trace != nullptr;
    if (want_r && s->r_cap < steps + 1) {
        if (s->r_dev) {
            CIA_HIP(hipFree(s->r_dev));
            for (auto &q : p->dev_allocs)
                if (q == s->r_dev) q = nullptr;
            s->r_dev = nullptr;
        }
        CIA_TRY(dalloc(p, &s->r_dev, (size_t)(steps + 1)));
        s->r_cap = steps + 1;
    }
    const bool rk4 = p->stepper == CIA_RK4;
    CIA_TRY(prep<R>(p, s, state, st));
    int cur = 0;
    for (int64_t k = 0; k < steps; k++) {
        const int nst = rk4 ? 4 : 1;
        for (int q = 0; q < nst; q++) {
            // the scan before a step's first stage also gives r(t_k)
            double *r_out = want_r && q == 0 ? s->r_dev + k : nullptr;
            if (needs_scan(s) || r_out) CIA_TRY(launch_scan(p, s, cur, r_out, st));
            SArgs<R> a = base_args<R>(p, s);
            a.mode = rk4 ? SM_RK4 : SM_EULER;
            a.stage = q;
            a.dt = (R)dt;
            a.z_in = static_cast<const zc<R> *>(s->z[cur]);
            a.z_out = static_cast<zc<R> *>(s->z[cur ^ 1]);
            a.part = s->part[cur ^ 1];
            CIA_TRY(launch_stage<R>(p, s, a, st, KK_STAGE));
            cur ^= 1;
        }
    }
    if (want_r) CIA_TRY(launch_scan(p, s, cur, s->r_dev + steps, st));
    CIA_HIP(hipMemcpyAsync(state, s->theta_n, (s->f64 ? sizeof(double) : sizeof(float)) * (size_t)p->n,
                           hipMemcpyDeviceToDevice, st));
    if (want_r) {
        CIA_HIP(hipMemcpyAsync(r_trace, s->r_dev, sizeof(double) * (size_t)(steps + 1), hipMemcpyDeviceToHost, st));
        CIA_HIP(hipStreamSynchronize(st));
        for (int64_t k = 0; k <= steps; k++)
            if (!std::isfinite(r_trace[k]))
                return set_error(CIA_ENONFINITE, "state became non-finite (r(t_%lld) = %g)", (long long)k,
                                 r_trace[k]);
    }
    return CIA_OK;
}

cia_status struct_rhs(cia_plan *p, const void *state, void *dstate, hipStream_t st) {
    StructState *s = p->structd;
    return s->f64 ? rhs_impl<double>(p, s, state, dstate, st) : rhs_impl<float>(p, s, state, dstate, st);
}

cia_status struct_integrate(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace, hipStream_t st) {
    StructState *s = p->structd;
    return s->f64 ? integrate_impl<double>(p, s, state, dt, steps, r_trace, st)
                  : integrate_impl<float>(p, s, state, dt, steps, r_trace, st);
}

}  // namespace cia
