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
// Data layout in HBM (sliced ELLPACK with one wavefront per slice): inside
// every community the rows are ordered by decreasing remainder length (the
// order inside a community is free in step P1), and cut into slices of 64
// consecutive rows.  A slice stores chunk k (16 bytes) of all 64 rows
// contiguously, so lane l of a wavefront owns row l of the slice, streams its
// list with fully coalesced 1 KiB loads and accumulates in registers: no
// segmented reduction and no barrier inside the gather.  Rows of communities
// whose z values are staged in LDS store uint16 indices local to the
// community (8 per chunk, pad = lambda, an LDS slot holding 0); all other rows
// store int32 positions (4 per chunk, pad = N, a z slot holding 0).
//
// Kernel structure on gfx950: one launch per RK stage.  A block owns a run
// of slices of one community.  It
//   1. sums the previous stage's per-unit partial observables of its
//      community in a fixed order (deterministic, no float atomics) and
//      stages the community's z values in LDS (S-neg partners are local);
//   2. each wavefront takes slices in turn: gather T over S-neg (LDS) and
//      S-pos (global), then combine, add omega, apply the RK stage update and
//      compute the next stage's z and its partial observables, per lane;
//   3. reduces the partial observables of the block in a fixed order.
// The direct method runs the same kernel with every node outside any
// community and the whole adjacency in the +1 list.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <type_traits>

#include "fastmath.h"
#include "plan.h"
#include "wave.h"

namespace cia {

constexpr int PMAX = 8;
constexpr double WIDE_COMMUNITY = 1e5;   // FP64 observables above this size
constexpr size_t LDS_BYTES = 64 * 1024;  // dynamic LDS budget of a stage block
constexpr int GEN_PMAX = 8;              // largest order of the general (non-difference) coupling
constexpr int SLICE = 64;                // rows per slice = lanes per wavefront

// unit flag bits
constexpr int UF_STAGED = 1;   // community z staged in LDS, S-neg as uint16 local indices
constexpr int UF_WIDE = 2;     // FP64 observables and combine (F32 plans)
constexpr int UF_ASSIGNED = 4; // rows of a dense community (E1 applies)
constexpr int UF_TILED = 8;    // community above the LDS cap: z staged tile by tile, S-neg per tile

// 64 rows of one community; chunk k of lane l of stream q sits at
// beg[q] + 64 k + l.  Streams: 0 = S-neg, 1 = S-pos (pairwise remainder),
// 2 = missing intra-community hyperedges, 3 = hyperedges across communities
// (triadic model; each entry a partner pair).
struct alignas(16) Slice {
    int32_t row0, rows;   // first row (community order), number of rows (1..64)
    uint32_t beg[4];      // first 16-byte chunk of each stream's block
    int32_t w[4];         // chunks per lane of each stream
    int32_t tw;           // tiled communities: first entry of this slice's per-tile S-neg widths
    int32_t sflags;       // SF_* (keeps the descriptor at 48 bytes)
};

// slice flag bits
// SF_MERGED: the S-pos entries of the slice's rows form one stream sorted by
// partner, each 32-bit entry the partner's position | (lane of the row << 26);
// entry e sits in word (e % 256) / 64 of chunk e / 256 of lane e % 64, so the
// 64 lanes of one gather read 64 consecutive partners.  Padding: the word n.
constexpr int SF_MERGED = 1;
constexpr int MERGE_ROW_SHIFT = 26;

// A work unit (one block): a run of slices of one community or of the rows
// outside every community, with everything needed to start in one load.
struct alignas(16) Unit {
    int32_t s0, s1;      // slices [s0, s1)
    int32_t flags;       // UF_*
    int32_t off, lam;    // community rows [off, off + lam); lam = 0 outside communities
    int32_t qslot;       // slot of this unit's partial observables
    int32_t qbeg, qend;  // slots of every unit of the community, in increasing row order
};

template <typename R>
struct cx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// key of a triple of user ids: sorted a < b < c packed as a | b << 21 | c << 42
__host__ __device__ static inline uint64_t triple_key(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return (uint64_t)a | ((uint64_t)b << 21) | ((uint64_t)c << 42);
}

__device__ __forceinline__ void dsincos(float t, float *s, float *c) { fast_sincosf(t, s, c); }
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
// TwoSum-compensated wavefront sum of (s, c) pairs over the DPP lane moves
// of wave_incl_scan (a lane without a source adds (0, 0), which changes
// nothing); lane 63's pair, the total, ends in every lane.
__device__ __forceinline__ void wave_tsum(float &s, float &c) {
#define CIA_STEP(C, M) tsum_pair(s, c, dpp_f<C, M>(s), dpp_f<C, M>(c));
    CIA_WAVE_SCAN_STEPS(CIA_STEP)
#undef CIA_STEP
    s = lane63(s);
    c = lane63(c);
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
    const Slice *slices;
    const uint4 *negdata;     // S-neg slice blocks
    const uint4 *posdata;     // S-pos slice blocks
    const void *tri_m;        // triadic CIA: per row, sum over missing intra pairs of z_j z_k (cx<R>)
    const uint4 *tposdata;    // hyperedges across communities (triadic)
    const cx<R> *h_extra;     // direct triadic: sum over present intra pairs of z_j z_k
    const int32_t *cnt;       // [n] |S+| - |S-| per row (only when d_0 != 0)
    const int32_t *perm;      // community order -> user order
    const R *omega;
    R *theta_n;               // theta at the start of the step (community order)
    R *acc;                   // RK4 accumulator
    const R *th_in;           // theta of the current stage, [n+1] (random gathers, FP64 path)
    R *th_out;                // theta of the next stage
    const cx<R> *cs_in;       // z of the current stage, [n+1], z[n] = 0
    cx<R> *cs_out;            // z of the next stage
    const double2 *q_in;      // [slots][P] partial observables of the current stage
    double2 *q_out;
    double2 *r_part;          // [nunits] partial sum of z for the order parameter
    // the previous launch's order-parameter partials, summed at kernel start by
    // one wavefront of the last block into r_prev_out (+ *r_prev_slot)
    const double2 *r_prev_part;
    double *r_prev_out;
    const int64_t *r_prev_slot;
    int32_t r_prev_n;
    double invN;
    const R *state_in;        // user order (M_PREP)
    R *state_out;             // user order (M_RHS)
    const R *kn;              // batched ensembles: K_b / N_b per node (community order), else NULL
    R Kn, dt, d0, hzero;
    R K2n;                    // triadic strength K2 / N^2
    R dsin[PMAX + 1], dcos[PMAX + 1];
    double ph[PMAX + 1], pf[PMAX + 1];   // polynomial model: h and f coefficients
    const R *gen;             // general coupling: c11, c12, c21, c22, each [(P+1)^2]; NULL = difference form
    const double *pgen;       // polynomial model, general coupling c[a][b] [(P+1)^2]; NULL = h(x_l - x_m)
    double pf2[32];           // polynomial model with two components: F[d][i][j], f_d = sum F u^i v^j
    int32_t pq;
    int32_t stage, mode, want_r, lds_cap;
    uint32_t pad_pos;         // position whose z is 0 (= n): target of padded int32 entries
    const int32_t *tile_w;    // tiled communities: S-neg chunks per lane of every (slice, tile)
    int32_t tile_cap;         // largest tile of a tiled community (nodes)
};

// The remainder streams are read once per stage: non-temporal loads keep
// them from evicting the z values that the gathers reuse from L2.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4 *p) {
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

template <typename R, int P>
__device__ __forceinline__ void acc_z(cx<R> (&T)[P], cx<R> z, R sign) {
    cx<R> zk = z;
#pragma unroll
    for (int k = 0; k < P; k++) {
        T[k].x += sign * zk.x;
        T[k].y += sign * zk.y;
        if (k + 1 < P) zk = cmul(zk, z);
    }
}

// z of the staged community at a byte offset (local index * sizeof(z)):
// staged local indices are stored pre-scaled, so the address needs no shift
// r(t) = |(1/N) sum z| from the unit partials: one wavefront, lane-strided
// FP64 sums then a DPP wave sum, so the order is fixed.  Used by the
// stage kernel (folded into the next launch) and by order_reduce_kernel.
__device__ __forceinline__ void reduce_r_wave(const double2 *part, int n, double invN, double *out) {
    const int lane = threadIdx.x & 63;
    double x = 0.0, y = 0.0;
#pragma unroll 8
    for (int j = lane; j < n; j += 64) {
        const double2 v = part[j];
        x += v.x;
        y += v.y;
    }
    x = wave_sum(x);
    y = wave_sum(y);
    if (lane == 0) *out = sqrt(x * x + y * y) * invN;
}

template <typename R>
struct alignas(2 * sizeof(R)) cx_aligned {
    R x, y;
};
template <typename R>
__device__ __forceinline__ cx<R> zat(const cx<R> *zsh, uint32_t byte_off) {
    // the aligned type keeps the access a single 8- (16-) byte LDS read
    const cx_aligned<R> v =
        *reinterpret_cast<const cx_aligned<R> *>(reinterpret_cast<const unsigned char *>(zsh) + byte_off);
    return cx<R>{v.x, v.y};
}

// Stream `w` chunks of one lane's row (stride 64 chunks, U per batch): 4
// int32 global positions per chunk, double-buffered (batch j+1's loads are
// in flight while batch j's partners are gathered), as z (GATHER_Z) or as
// theta with z recomputed.
template <typename R, int P, int U, bool GATHER_Z>
__device__ __forceinline__ void gather_rows(cx<R> (&T)[P], const uint4 *__restrict__ col, int w,
                                            const cx<R> *__restrict__ cs, const R *__restrict__ th, uint32_t pad,
                                            R sign, uint4 padv) {
    if (w <= 0) return;
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) v[u] = u < w ? ld_stream(col + (size_t)u * SLICE) : padv;
    for (int k = 0; k < w; k += U) {
        uint4 vn[U];
#pragma unroll
        for (int u = 0; u < U; u++) vn[u] = k + U + u < w ? ld_stream(col + (size_t)(k + U + u) * SLICE) : padv;
        cx<R> z[U][4];
        if (GATHER_Z) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                z[u][0] = cs[v[u].x];
                z[u][1] = cs[v[u].y];
                z[u][2] = cs[v[u].z];
                z[u][3] = cs[v[u].w];
            }
        } else {
            // theta gathers (half the footprint of z), z recomputed; the
            // padding position contributes 0
            R t[U][4];
#pragma unroll
            for (int u = 0; u < U; u++) {
                t[u][0] = th[v[u].x];
                t[u][1] = th[v[u].y];
                t[u][2] = th[v[u].z];
                t[u][3] = th[v[u].w];
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t q4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    R sn, cs0;
                    dsincos(t[u][q], &sn, &cs0);
                    const bool ok = q4[q] != pad;
                    z[u][q] = cx<R>{ok ? cs0 : (R)0, ok ? sn : (R)0};
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int q = 0; q < 4; q++) acc_z<R, P>(T, z[u][q], sign);
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = vn[u];
    }
}

// Staged rows: the S-neg chunks gathered from LDS and the S-pos chunks by
// theta gathers, with the first S-pos batch's index loads issued beside the
// S-neg loads and its theta gathers in flight while the LDS gathers run.
template <typename R, int P, int UL, int UG>
__device__ __forceinline__ void gather_staged_rows(cx<R> (&T)[P], const uint4 *__restrict__ neg, int wn,
                                                   const uint4 *__restrict__ pos, int wp, const cx<R> *zsh,
                                                   const cx<R> *__restrict__ cs, const R *__restrict__ th,
                                                   uint32_t pad, uint4 padl, uint4 padp) {
    uint4 nv[UL], pv[UG];
#pragma unroll
    for (int u = 0; u < UL; u++) nv[u] = u < wn ? ld_stream(neg + (size_t)u * SLICE) : padl;
#pragma unroll
    for (int u = 0; u < UG; u++) pv[u] = u < wp ? ld_stream(pos + (size_t)u * SLICE) : padp;
    R t[UG][4];
#pragma unroll
    for (int u = 0; u < UG; u++) {
        t[u][0] = th[pv[u].x];
        t[u][1] = th[pv[u].y];
        t[u][2] = th[pv[u].z];
        t[u][3] = th[pv[u].w];
    }
    for (int k = 0; k < wn; k += UL) {
        if (k > 0) {
#pragma unroll
            for (int u = 0; u < UL; u++) nv[u] = k + u < wn ? ld_stream(neg + (size_t)(k + u) * SLICE) : padl;
        }
#pragma unroll
        for (int u = 0; u < UL; u++) {
            const uint32_t q4[4] = {nv[u].x, nv[u].y, nv[u].z, nv[u].w};
            cx<R> z[8];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                z[2 * q] = zat(zsh, q4[q] & 0xffffu);
                z[2 * q + 1] = zat(zsh, q4[q] >> 16);
            }
#pragma unroll
            for (int q = 0; q < 8; q++) acc_z<R, P>(T, z[q], (R)-1);
        }
    }
#pragma unroll
    for (int u = 0; u < UG; u++) {
        const uint32_t q4[4] = {pv[u].x, pv[u].y, pv[u].z, pv[u].w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            R sn, c0;
            dsincos(t[u][q], &sn, &c0);
            const bool ok = q4[q] != pad;
            acc_z<R, P>(T, cx<R>{ok ? c0 : (R)0, ok ? sn : (R)0}, (R)1);
        }
    }
    if (wp > UG)
        gather_rows<R, P, UG, false>(T, pos + (size_t)UG * SLICE, wp - UG, cs, th, pad, (R)1, padp);
}

// S-pos of a slice stored merged (SF_MERGED): the wavefront walks the
// partner-sorted stream of all its rows, so the 64 lanes of one gather read
// neighbouring partners and share cache lines, and each lane adds its z into
// the sum of the entry's row in LDS (acc: [64] x sums then [64] y sums) as a
// 64-bit fixed-point integer in units of 2^-40.  Integer sums do not depend on
// the order of the additions, so the result is deterministic; |cos|, |sin| <= 1
// keeps a row of up to 2^23 entries from overflowing.  Lane l then adds row l's
// sum to T.  Every lane of the wavefront takes part (uniform w).
template <int U>
__device__ __forceinline__ void merged_pos_sum(cx<float> &T, const uint4 *__restrict__ col, int w,
                                               const float *__restrict__ th, uint32_t pad,
                                               unsigned long long *acc) {
    const int lane = threadIdx.x & 63;
    constexpr uint32_t MASK = (1u << MERGE_ROW_SHIFT) - 1;
    __hip_atomic_store(acc + lane, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    __hip_atomic_store(acc + 64 + lane, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    __builtin_amdgcn_wave_barrier();
    const uint4 padv = make_uint4(pad, pad, pad, pad);
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) v[u] = u < w ? ld_stream(col + (size_t)u * SLICE) : padv;
    for (int k = 0; k < w; k += U) {
        uint4 vn[U];
#pragma unroll
        for (int u = 0; u < U; u++) vn[u] = k + U + u < w ? ld_stream(col + (size_t)(k + U + u) * SLICE) : padv;
        float t[U][4];
#pragma unroll
        for (int u = 0; u < U; u++) {
            t[u][0] = th[v[u].x & MASK];
            t[u][1] = th[v[u].y & MASK];
            t[u][2] = th[v[u].z & MASK];
            t[u][3] = th[v[u].w & MASK];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t q4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                float sn, c0;
                dsincos(t[u][q], &sn, &c0);
                if (q4[q] != pad) {
                    const int row = (int)(q4[q] >> MERGE_ROW_SHIFT);
                    const long long fx = (long long)__builtin_rintf(c0 * 0x1p40f);
                    const long long fy = (long long)__builtin_rintf(sn * 0x1p40f);
                    __hip_atomic_fetch_add(acc + row, (unsigned long long)fx, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                    __hip_atomic_fetch_add(acc + 64 + row, (unsigned long long)fy, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = vn[u];
    }
    __builtin_amdgcn_wave_barrier();
    const long long sx = (long long)__hip_atomic_load(acc + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const long long sy = (long long)__hip_atomic_load(acc + 64 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    T.x += (float)sx * 0x1p-40f;
    T.y += (float)sy * 0x1p-40f;
}

// S-neg chunks of one lane gathered from the staged z in LDS: 8 uint16 byte
// offsets per chunk, UL chunks per batch (a tile of a tiled community).
template <typename R, int P, int UL>
__device__ __forceinline__ void gather_lds_rows(cx<R> (&T)[P], const uint4 *__restrict__ neg, int wn,
                                                const cx<R> *zsh, uint4 padl) {
    for (int k = 0; k < wn; k += UL) {
        uint4 nv[UL];
#pragma unroll
        for (int u = 0; u < UL; u++) nv[u] = k + u < wn ? ld_stream(neg + (size_t)(k + u) * SLICE) : padl;
#pragma unroll
        for (int u = 0; u < UL; u++) {
            const uint32_t q4[4] = {nv[u].x, nv[u].y, nv[u].z, nv[u].w};
            cx<R> z[8];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                z[2 * q] = zat(zsh, q4[q] & 0xffffu);
                z[2 * q + 1] = zat(zsh, q4[q] >> 16);
            }
#pragma unroll
            for (int q = 0; q < 8; q++) acc_z<R, P>(T, z[q], (R)-1);
        }
    }
}

// Stream a lane's list of partner pairs (j, k) and return sum z_j z_k:
// 2 pairs of int32 positions per chunk, gathered as z (GATHER_Z) or as
// theta with z recomputed; the pad position contributes 0.
template <typename R, int U, bool GATHER_Z>
__device__ __forceinline__ cx<R> gather_pairs(const uint4 *__restrict__ col, int w, const cx<R> *__restrict__ cs,
                                              const R *__restrict__ th, uint32_t pad, uint4 padv) {
    cx<R> M = {(R)0, (R)0};
    auto zof = [&](uint32_t j) -> cx<R> {
        if (GATHER_Z) return cs[j];
        R sn, c0;
        dsincos(th[j], &sn, &c0);
        return j != pad ? cx<R>{c0, sn} : cx<R>{(R)0, (R)0};
    };
    for (int k = 0; k < w; k += U) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = k + u < w ? ld_stream(col + (size_t)(k + u) * SLICE) : padv;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const cx<R> p0 = cmul(zof(v[u].x), zof(v[u].y));
            const cx<R> p1 = cmul(zof(v[u].z), zof(v[u].w));
            M.x += p0.x + p1.x;
            M.y += p0.y + p1.y;
        }
    }
    return M;
}

// General coupling (App. A.2, eq. FourierRealExpansion): sum over partners
// of g(theta_l, theta_m) from the partner harmonics C_a = sum cos(a theta_l),
// S_a = sum sin(a theta_l) (C_0 = M0, the partner count) and this node's
// cos/sin(b theta_m); for an assigned row the l = m term that the community
// sums include is removed.
template <typename T, int P>
__device__ __forceinline__ T gen_sum(const float *gf, const double *gd, const T (&C)[P + 1], const T (&Sn)[P + 1],
                                     cx<T> z, bool self) {
    constexpr int NP = (P + 1) * (P + 1);
    T cb[P + 1], sb[P + 1];
    cb[0] = (T)1;
    sb[0] = (T)0;
    cx<T> zk = z;
#pragma unroll
    for (int b = 1; b <= P; b++) {
        cb[b] = zk.x;
        sb[b] = zk.y;
        if (b < P) zk = cmul(zk, z);
    }
    T s = (T)0, own = (T)0;
#pragma unroll
    for (int a = 0; a <= P; a++)
#pragma unroll
        for (int b = 0; b <= P; b++) {
            const int i = a * (P + 1) + b;
            const T c11 = gf ? (T)gf[i] : (T)gd[i], c12 = gf ? (T)gf[NP + i] : (T)gd[NP + i];
            const T c21 = gf ? (T)gf[2 * NP + i] : (T)gd[2 * NP + i], c22 = gf ? (T)gf[3 * NP + i] : (T)gd[3 * NP + i];
            s += (c11 * C[a] + c21 * Sn[a]) * cb[b] + (c12 * C[a] + c22 * Sn[a]) * sb[b];
            if (self) own += (c11 * cb[a] + c21 * sb[a]) * cb[b] + (c12 * cb[a] + c22 * sb[a]) * sb[b];
        }
    return s - own;
}
template <typename R>
__device__ __forceinline__ const float *gen_f(const R *g) {
    if constexpr (sizeof(R) == 4) return reinterpret_cast<const float *>(g);
    else return nullptr;
}
template <typename R>
__device__ __forceinline__ const double *gen_d(const R *g) {
    if constexpr (sizeof(R) == 8) return reinterpret_cast<const double *>(g);
    else return nullptr;
}

// DIRECT: every row is an outside row with its whole adjacency in the +1
// list (no observables, no staging).  WIDE: the FP64 path of very large
// communities is compiled in (F32 plans that have such communities).
// TRI: the triadic term of the higher-order model (P = 2 observables give
// S1 = sum z and S2 = sum z^2 per community).
// MERGE: FP32 plans with P = 1 whose S-pos has slices stored merged.
template <typename R, int P, int BLOCK, bool DIRECT, bool WIDE, bool TRI, bool GEN = false, bool MERGE = false>
__global__ __launch_bounds__(BLOCK) void phase_stage_kernel(PhaseArgs<R> a) {
    constexpr int NW = BLOCK / 64;
    constexpr bool MG = MERGE && sizeof(R) == 4 && P == 1 && !DIRECT && !TRI && !GEN;
    constexpr int UL = P >= 4 ? 2 : 8 / P;  // chunks per batch, LDS-gathered rows
    constexpr int UG = P >= 2 ? 1 : 2;      // chunks per batch, global-gathered rows (two in flight)
    constexpr int UM = 4;                   // chunks per batch of a merged S-pos slice (16 gathers per lane)
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R> *zsh = reinterpret_cast<cx<R> *>(smem);   // [lds_cap + 1]
    __shared__ double2 qsh[P];
    __shared__ float red_s[NW][2 * P], red_c[NW][2 * P];
    __shared__ double red_d[NW][2 * P];
    __shared__ double2 red_r[NW];
    __shared__ unsigned long long macc[MG ? NW : 1][128];   // merged S-pos row sums, per wavefront

    const Unit Un = a.units[blockIdx.x];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    // r(t) of the previous step from its partials (the kernel boundary makes
    // them visible), by the first block, which starts before all others
    if (a.r_prev_out && blockIdx.x == 0 && wid == 0)
        reduce_r_wave(a.r_prev_part, a.r_prev_n, a.invN, a.r_prev_out + (a.r_prev_slot ? *a.r_prev_slot : 0));
    const bool assigned = !DIRECT && (Un.flags & UF_ASSIGNED) != 0;
    const bool staged = !DIRECT && (Un.flags & UF_STAGED) != 0;
    const bool wide = WIDE && (Un.flags & UF_WIDE) != 0;
    const int mode = a.mode;
    const bool gather = mode != M_PREP;
    const int off = Un.off, lam = Un.lam;

    // ---- 1. unit start: the community's z in LDS and its observables (E1,
    //      fixed order over the units of the community) ----
    if (gather && assigned) {
        if (staged) {
            // eight loads in flight per thread before the LDS writes
            constexpr int US = 8;
            for (int j0 = tid; j0 < lam; j0 += BLOCK * US) {
                cx<R> v[US];
#pragma unroll
                for (int u = 0; u < US; u++)
                    if (j0 + u * BLOCK < lam) v[u] = a.cs_in[off + j0 + u * BLOCK];
#pragma unroll
                for (int u = 0; u < US; u++)
                    if (j0 + u * BLOCK < lam) zsh[j0 + u * BLOCK] = v[u];
            }
            if (tid == 0) zsh[lam] = cx<R>{(R)0, (R)0};   // slot of the padding index
        }
        if (wid == NW - 1) {
            for (int k = 0; k < P; k++) {
                double sx = 0.0, sy = 0.0;
                for (int j = Un.qbeg + lane; j < Un.qend; j += 64) {
                    double2 q = a.q_in[(size_t)j * P + k];
                    sx += q.x;
                    sy += q.y;
                }
                sx = wave_sum(sx);
                sy = wave_sum(sy);
                if (lane == 0) qsh[k] = make_double2(sx, sy);
            }
        }
    }
    __syncthreads();

    R qx[P], qy[P];
    double qdx[P], qdy[P];
    if (gather && assigned) {
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

    // ---- 1b. communities above the LDS cap (WIDE instantiations only): the
    //      S-neg sums of this wavefront's slices, the community's z staged
    //      one column tile at a time ----
    constexpr int SMAX = P <= 2 ? 4 : (P <= 4 ? 2 : 1);   // slices per wavefront of a tiled unit
    const bool tiled = WIDE && gather && (Un.flags & UF_TILED) != 0;
    cx<R> Tn[SMAX][P];
#pragma unroll
    for (int j = 0; j < SMAX; j++)
#pragma unroll
        for (int k = 0; k < P; k++) Tn[j][k].x = Tn[j][k].y = (R)0;
    if (WIDE && tiled) {
        const int nt = (lam + a.tile_cap - 1) / a.tile_cap;
        const int ts = (lam + nt - 1) / nt;
        const uint32_t tb = (uint32_t)ts * (uint32_t)sizeof(cx<R>);   // pad: the zero slot zsh[ts]
        const uint4 padt = make_uint4(tb | (tb << 16), tb | (tb << 16), tb | (tb << 16), tb | (tb << 16));
        int toff[SMAX];
#pragma unroll
        for (int j = 0; j < SMAX; j++) toff[j] = 0;
        constexpr int ULT = P >= 4 ? 2 : 8 / P;
        for (int t = 0; t < nt; t++) {
            const int t0 = t * ts, len = min(ts, lam - t0);
            if (t > 0) __syncthreads();   // the previous tile's gathers are done
            for (int j0 = tid; j0 < len; j0 += BLOCK * 8) {
                cx<R> v[8];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (j0 + u * BLOCK < len) v[u] = a.cs_in[off + t0 + j0 + u * BLOCK];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (j0 + u * BLOCK < len) zsh[j0 + u * BLOCK] = v[u];
            }
            if (tid == 0) zsh[ts] = cx<R>{(R)0, (R)0};
            __syncthreads();
#pragma unroll
            for (int j = 0; j < SMAX; j++) {
                const int sl = Un.s0 + wid + j * NW;
                if (sl < Un.s1) {
                    const Slice S = a.slices[sl];
                    const int w = a.tile_w[S.tw + t];
                    gather_lds_rows<R, P, ULT>(Tn[j], a.negdata + S.beg[0] + (size_t)toff[j] * SLICE + lane, w, zsh,
                                               padt);
                    toff[j] += w;
                }
            }
        }
    }

    // partial observables of the next stage
    float ps[2 * P], pc[2 * P];
    double pd[2 * P];
#pragma unroll
    for (int k = 0; k < 2 * P; k++) ps[k] = pc[k] = 0.f, pd[k] = 0.0;
    double rx = 0.0, ry = 0.0;

    const uint32_t padb = (uint32_t)lam * (uint32_t)sizeof(cx<R>);
    const uint32_t pad16 = padb | (padb << 16);
    const uint4 padl = make_uint4(pad16, pad16, pad16, pad16);
    const uint4 padp = make_uint4(a.pad_pos, a.pad_pos, a.pad_pos, a.pad_pos);

    // ---- 2. slices, one wavefront each, one row per lane ----
    // each slice's descriptor is loaded one slice ahead, so its scalar load is
    // in flight while the previous slice is gathered
    Slice Snext;
    if (Un.s0 + wid < Un.s1) Snext = a.slices[Un.s0 + wid];
    int jsl = 0;   // this wavefront's slice count (tiled units: index into Tn)
    for (int sl = Un.s0 + wid; sl < Un.s1; sl += NW, jsl++) {
        const Slice S = Snext;
        if (sl + NW < Un.s1) Snext = a.slices[sl + NW];
        const bool mine = lane < S.rows;
        const int i = S.row0 + lane;
        // operands of the combine / stage update, loaded before the gather
        R tn = (R)0, om = (R)0, av = (R)0, thc = (R)0, knv = a.Kn;
        int cv = 0;
        if (mine) {
            if (mode == M_PREP) {
                tn = a.state_in[a.perm[i]];
            } else {
                if (mode != M_RHS) tn = a.theta_n[i];
                if (a.omega) om = a.omega[i];
                if (a.kn) knv = a.kn[i];
                if (mode == M_RK4 && a.stage > 0) av = a.acc[i];
                if (a.d0 != (R)0) cv = a.cnt[i];
                if (WIDE && wide) thc = a.th_in[i];
            }
        }
        cx<R> T[P];
#pragma unroll
        for (int k = 0; k < P; k++) T[k].x = T[k].y = (R)0;
        const bool merged = MG && (S.sflags & SF_MERGED) != 0;
        const int wpos = merged ? 0 : S.w[1];
        if (gather) {
            if (!DIRECT && staged) {
                gather_staged_rows<R, P, UL, UG>(T, a.negdata + S.beg[0] + lane, S.w[0], a.posdata + S.beg[1] + lane,
                                                 wpos, zsh, a.cs_in, a.th_in, a.pad_pos, padl, padp);
            } else {
                if (WIDE && tiled) {
                    // S-neg summed tile by tile above (static indexing keeps Tn in registers)
#pragma unroll
                    for (int j = 0; j < SMAX; j++)
                        if (j == jsl)
#pragma unroll
                            for (int k = 0; k < P; k++) T[k].x += Tn[j][k].x, T[k].y += Tn[j][k].y;
                } else if (!DIRECT)
                    gather_rows<R, P, UG, false>(T, a.negdata + S.beg[0] + lane, S.w[0], a.cs_in, a.th_in, a.pad_pos, (R)-1, padp);
                gather_rows<R, P, UG, DIRECT>(T, a.posdata + S.beg[1] + lane, wpos, a.cs_in, a.th_in, a.pad_pos, (R)1, padp);
            }
            if constexpr (MG) {
                if (merged)
                    merged_pos_sum<UM>(T[0], a.posdata + S.beg[1] + lane, S.w[1], a.th_in, a.pad_pos, macc[wid]);
            }
        }
        cx<R> Mt = {(R)0, (R)0}, Xt = {(R)0, (R)0};   // missing intra / cross hyperedge pair sums
        if (TRI && gather) {
            if (!DIRECT && assigned && mine && a.tri_m) Mt = static_cast<const cx<R> *>(a.tri_m)[i];
            Xt = gather_pairs<R, 2, DIRECT>(a.tposdata + S.beg[3] + lane, S.w[3], a.cs_in, a.th_in, a.pad_pos, padp);
        }

        // ---- combine (eq. FastHdense + E2), stage update, next z ----
        if (mine) {
            R theta_new = (R)0;
            bool emit = true;
            if (mode == M_PREP) {
                theta_new = tn;
                a.theta_n[i] = theta_new;
            } else {
                R H;
                if (!wide) {
                    cx<R> z = staged ? zsh[i - off] : a.cs_in[i];
                    R s = (R)0;
                    if constexpr (GEN) {
                        R Cg[P + 1], Sg[P + 1];
                        Cg[0] = (assigned ? (R)lam : (R)0) + (R)cv;
                        Sg[0] = (R)0;
#pragma unroll
                        for (int k = 0; k < P; k++) {
                            Cg[k + 1] = qx[k] + T[k].x;
                            Sg[k + 1] = qy[k] + T[k].y;
                        }
                        s = gen_sum<R, P>(gen_f(a.gen), gen_d(a.gen), Cg, Sg, z, assigned);
                    } else {
                        if (a.d0 != (R)0) s = a.d0 * ((assigned ? (R)lam : (R)0) + (R)cv);
                        if (assigned) s -= a.hzero;
                        cx<R> zk = z;
#pragma unroll
                        for (int k = 0; k < P; k++) {
                            cx<R> A = {qx[k] + T[k].x, qy[k] + T[k].y};
                            cx<R> B = cmul(A, cx<R>{zk.x, -zk.y});
                            s += a.dcos[k + 1] * B.x + a.dsin[k + 1] * B.y;
                            if (k + 1 < P) zk = cmul(zk, z);
                        }
                    }
                    H = om + knv * s;
                    if constexpr (TRI && P >= 2) {
                        // sum over ordered distinct partner pairs of z_j z_k, then
                        // Im(conj(z_m)^2 * .) (App. A.7 with lambda = (1,1,-2))
                        const cx<R> z2 = cmul(z, z);
                        cx<R> D;
                        if (DIRECT) {
                            const cx<R> E = a.h_extra[i];
                            D = cx<R>{(R)2 * (E.x + Xt.x), (R)2 * (E.y + Xt.y)};
                        } else {
                            D = cx<R>{(R)0, (R)0};
                            if (assigned) {
                                const cx<R> A1 = {qx[0] - z.x, qy[0] - z.y};
                                const cx<R> A2 = {qx[1] - z2.x, qy[1] - z2.y};
                                const cx<R> A11 = cmul(A1, A1);
                                D = cx<R>{A11.x - A2.x, A11.y - A2.y};
                            }
                            D.x += (R)2 * (Xt.x - Mt.x);
                            D.y += (R)2 * (Xt.y - Mt.y);
                        }
                        H += a.K2n * cmul(D, cx<R>{z2.x, -z2.y}).y;
                    }
                } else {
                    // FP64 observables and combine for very large communities
                    double zs, zc0;
                    sincos((double)thc, &zs, &zc0);
                    cx<double> z = {zc0, zs};
                    double s = 0.0;
                    if constexpr (GEN) {
                        double Cg[P + 1], Sg[P + 1];
                        Cg[0] = (double)lam + (double)cv;
                        Sg[0] = 0.0;
#pragma unroll
                        for (int k = 0; k < P; k++) {
                            Cg[k + 1] = qdx[k] + (double)T[k].x;
                            Sg[k + 1] = qdy[k] + (double)T[k].y;
                        }
                        s = gen_sum<double, P>(gen_f(a.gen), gen_d(a.gen), Cg, Sg, z, true);
                    } else {
                        if (a.d0 != (R)0) s = (double)a.d0 * ((double)lam + (double)cv);
                        s -= (double)a.hzero;
                        cx<double> zk = z;
#pragma unroll
                        for (int k = 0; k < P; k++) {
                            cx<double> A = {qdx[k] + (double)T[k].x, qdy[k] + (double)T[k].y};
                            cx<double> B = cmul(A, cx<double>{zk.x, -zk.y});
                            s += (double)a.dcos[k + 1] * B.x + (double)a.dsin[k + 1] * B.y;
                            if (k + 1 < P) zk = cmul(zk, z);
                        }
                    }
                    H = (R)((double)om + (double)knv * s);
                }
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
                        a.acc[i] = av + (R)2 * H;
                        theta_new = tn + (R)0.5 * a.dt * H;
                    } else if (st == 2) {
                        a.acc[i] = av + (R)2 * H;
                        theta_new = tn + a.dt * H;
                    } else {
                        theta_new = wrap_2pi<R>(tn + a.dt / (R)6 * (av + H));
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
                a.th_out[i] = theta_new;
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
                if (!DIRECT) a.th_out[i] = theta_new;
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
    }
    if (mode == M_RHS) return;

    // ---- 3. unit partials: deterministic block reduction ----
    if (assigned) {
        if (sizeof(R) == 4 && !wide) {
#pragma unroll
            for (int k = 0; k < 2 * P; k++) {
                float s = ps[k], cc = pc[k];
                wave_tsum(s, cc);
                if (lane == 0) {
                    red_s[wid][k] = s;
                    red_c[wid][k] = cc;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 2 * P; k++) {
                const double s = wave_sum(pd[k]);
                if (lane == 0) red_d[wid][k] = s;
            }
        }
    }
    if (a.want_r) {
        rx = wave_sum(rx);
        ry = wave_sum(ry);
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
                a.q_out[(size_t)Un.qslot * P + k] = make_double2(vx, vy);
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

// ---------------------------------------------------------------------------
// small networks: the whole integration in one launch of one workgroup
// ---------------------------------------------------------------------------
// For a network whose z values fit one workgroup's LDS, every step and stage
// of cia_integrate runs inside one 1024-thread workgroup: all z of the
// current stage sit in LDS, so the S-neg and S-pos partners of a row are both
// LDS reads, stages are separated by workgroup barriers instead of kernel
// launches, and theta_n, the RK4 accumulator and omega of a row stay in its
// lane's registers for the whole call.  Same layout (slices, remainder
// streams, padding) as the stage kernel; E1 observables and r(t) from
// per-slice FP64 partials summed in a fixed order.
constexpr int RES_PMAX = 4;
constexpr size_t RES_LDS_BYTES = 160 * 1024;   // LDS of one CU
constexpr int64_t RES_MAX_REMAINDER = 1 << 17; // S-neg + S-pos entries
// 1024 threads (128 VGPRs per lane).  A lane keeps theta_n, the
// accumulator, omega and H of one row per slice of its wavefront in
// registers: 8 slices in FP32, 4 in FP64 (twice the registers per row), and
// loads RES_UB (FP64: half as many) remainder chunks of each stream at once.
template <typename R>
__host__ __device__ constexpr int res_block() { return 1024; }
template <typename R>
__host__ __device__ constexpr int res_slices() { return sizeof(R) == 8 ? 4 : 8; }
template <typename R>
__host__ __device__ constexpr int res_ub() { return sizeof(R) == 8 ? 2 : 4; }

template <typename R>
struct ResArgs {
    const Slice *slices;
    const uint4 *negdata, *posdata;
    const int32_t *slice_comm;   // [nslices] community of each slice, -1 = rows of no community
    const int32_t *slice_flags;  // [nslices] UF_STAGED: S-neg as uint16 local byte offsets
    const int32_t *comm_off;     // [ncomm + 1]
    const int32_t *comm_slice0;  // [ncomm + 1] first slice of each community (slices of one community are contiguous)
    const int32_t *cnt;          // [n] |S+| - |S-| (only when d0 != 0)
    const int32_t *perm;
    const R *omega;
    const R *state_in;           // user order
    R *state_out;                // user order
    double *r_out;               // [steps + 1] or NULL
    int32_t n, nslices, ncomm, mode;   // mode: M_RK4 or M_EULER
    int64_t steps;
    R dt, Kn, d0, hzero;
    R dsin[PMAX + 1], dcos[PMAX + 1];
};

// LDS of the resident kernel: z of every node and the zero slot (rounded up
// to 16 bytes), the slice partials and the community sums
template <typename R>
__host__ __device__ constexpr size_t res_zbytes(int64_t n) { return (sizeof(cx<R>) * (size_t)(n + 1) + 15) & ~(size_t)15; }
template <typename R>
__host__ __device__ constexpr size_t res_smem(int64_t n, int64_t nslices, int64_t ncomm, int P) {
    // z | slice partials | community sums | slice descriptors | slice
    // community and flags | community offsets and first slices | omega and
    // |S+| - |S-| per row
    // (the 8-byte omega array sits before the 4-byte arrays, so it stays aligned)
    return res_zbytes<R>(n) + sizeof(double2) * (size_t)(nslices * (P + 1) + ncomm * P) +
           sizeof(Slice) * (size_t)nslices + sizeof(R) * (size_t)n +
           sizeof(int32_t) * (size_t)(2 * nslices + 2 * (ncomm + 1) + n);
}

template <typename R, int P>
__global__ __launch_bounds__(res_block<R>()) void resident_integrate_kernel(ResArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R> *zsh = reinterpret_cast<cx<R> *>(smem);                                   // [n + 1]
    double2 *part = reinterpret_cast<double2 *>(smem + res_zbytes<R>(a.n));          // [nslices][P + 1]
    double2 *Q = part + (size_t)a.nslices * (P + 1);                                 // [ncomm][P]
    Slice *ssh = reinterpret_cast<Slice *>(Q + (size_t)a.ncomm * P);                 // [nslices]
    R *om_sh = reinterpret_cast<R *>(ssh + a.nslices);                                // [n]
    int32_t *scomm = reinterpret_cast<int32_t *>(om_sh + a.n);                        // [nslices]
    int32_t *sflag = scomm + a.nslices;                                               // [nslices]
    int32_t *coff = sflag + a.nslices;                                                // [ncomm + 1]
    int32_t *cs0 = coff + (a.ncomm + 1);                                              // [ncomm + 1]
    int32_t *cnt_sh = cs0 + (a.ncomm + 1);                                            // [n]
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nst = a.mode == M_RK4 ? 4 : 1;
    constexpr int RES_BLOCK = res_block<R>();
    constexpr int RES_WAVES = RES_BLOCK / 64;
    constexpr int RES_SLICES = res_slices<R>();
    constexpr int UB = res_ub<R>();   // remainder chunks per batch of loads (S-neg and S-pos issued together)

    // descriptors read every stage: into LDS once
    for (int t = threadIdx.x; t < a.nslices; t += RES_BLOCK) {
        ssh[t] = a.slices[t];
        scomm[t] = a.slice_comm[t];
        sflag[t] = a.slice_flags[t];
    }
    for (int t = threadIdx.x; t <= a.ncomm; t += RES_BLOCK) {
        coff[t] = a.comm_off[t];
        cs0[t] = a.comm_slice0[t];
    }
    for (int i = threadIdx.x; i < a.n; i += RES_BLOCK) {
        om_sh[i] = a.omega ? a.omega[i] : (R)0;
        cnt_sh[i] = a.d0 != (R)0 ? a.cnt[i] : 0;
    }
    __syncthreads();

    // this lane's rows: one per slice of its wavefront
    R tn[RES_SLICES], acc[RES_SLICES], H[RES_SLICES];
#pragma unroll
    for (int j = 0; j < RES_SLICES; j++) {
        tn[j] = acc[j] = H[j] = (R)0;
        const int sl = wid + j * RES_WAVES;
        if (sl < a.nslices) {
            const Slice S = ssh[sl];
            if (lane < S.rows) tn[j] = a.state_in[a.perm[S.row0 + lane]];
        }
    }
    if (threadIdx.x == 0) zsh[a.n] = cx<R>{(R)0, (R)0};   // target of padded S-pos entries

    // z of the stage state th, the slice partials of z^k (k = 1..P) and of z,
    // then the community sums and r
    auto publish = [&](const R (&th)[RES_SLICES], int64_t rslot) {
#pragma unroll
        for (int j = 0; j < RES_SLICES; j++) {
            const int sl = wid + j * RES_WAVES;
            if (sl >= a.nslices) continue;
            const Slice S = ssh[sl];
            double2 pk[P + 1];
#pragma unroll
            for (int k = 0; k <= P; k++) pk[k] = make_double2(0.0, 0.0);
            if (lane < S.rows) {
                R sn, c0;
                dsincos(th[j], &sn, &c0);
                const cx<R> z = {c0, sn};
                zsh[S.row0 + lane] = z;
                cx<R> zk = z;
#pragma unroll
                for (int k = 0; k < P; k++) {
                    pk[k] = make_double2((double)zk.x, (double)zk.y);
                    if (k + 1 < P) zk = cmul(zk, z);
                }
                pk[P] = make_double2((double)z.x, (double)z.y);
            }
#pragma unroll
            for (int k = 0; k <= P; k++) pk[k] = wave_sum(pk[k]);
            if (lane == 0)
#pragma unroll
                for (int k = 0; k <= P; k++) part[(size_t)sl * (P + 1) + k] = pk[k];
        }
        __syncthreads();
        // community sums of z^k over their slices, in slice order; r over all slices
        for (int t = threadIdx.x; t < a.ncomm * P + 1; t += RES_BLOCK) {
            if (t < a.ncomm * P) {
                const int c = t / P, k = t % P;
                double2 q = make_double2(0.0, 0.0);
                for (int sl = cs0[c]; sl < cs0[c + 1]; sl++) {
                    const double2 v = part[(size_t)sl * (P + 1) + k];
                    q.x += v.x;
                    q.y += v.y;
                }
                Q[t] = q;
            } else if (a.r_out && rslot >= 0) {
                double x = 0.0, y = 0.0;
                for (int sl = 0; sl < a.nslices; sl++) {
                    const double2 v = part[(size_t)sl * (P + 1) + P];
                    x += v.x;
                    y += v.y;
                }
                a.r_out[rslot] = sqrt(x * x + y * y) / (double)a.n;
            }
        }
        __syncthreads();
    };

    publish(tn, 0);
    for (int64_t step = 0; step < a.steps; step++) {
        for (int st = 0; st < nst; st++) {
            // right-hand side of every row from the z values in LDS
#pragma unroll
            for (int j = 0; j < RES_SLICES; j++) {
                const int sl = wid + j * RES_WAVES;
                if (sl >= a.nslices) continue;
                const Slice S = ssh[sl];
                const int c = scomm[sl];
                const bool st16 = (sflag[sl] & UF_STAGED) != 0;
                const uint32_t cbase = c >= 0 ? (uint32_t)coff[c] * (uint32_t)sizeof(cx<R>) : 0u;
                // staged pads are lambda * sizeof(z): the next community's first z
                // (or the zero slot), skipped by value
                const uint32_t padb = c >= 0 ? (uint32_t)(coff[c + 1] - coff[c]) * (uint32_t)sizeof(cx<R>) : 0u;
                cx<R> T[P];
#pragma unroll
                for (int k = 0; k < P; k++) T[k].x = T[k].y = (R)0;
                const uint4 *neg = a.negdata + S.beg[0] + lane;
                const uint4 *pos = a.posdata + S.beg[1] + lane;
                for (int q0 = 0; q0 < S.w[0] || q0 < S.w[1]; q0 += UB) {
                    // both streams' next UB chunks in flight together
                    uint4 nv[UB], pv[UB];
#pragma unroll
                    for (int u = 0; u < UB; u++) {
                        nv[u] = q0 + u < S.w[0] ? neg[(size_t)(q0 + u) * SLICE] : make_uint4(padb | (padb << 16), padb | (padb << 16), padb | (padb << 16), padb | (padb << 16));
                        pv[u] = q0 + u < S.w[1] ? pos[(size_t)(q0 + u) * SLICE] : make_uint4(a.n, a.n, a.n, a.n);
                    }
#pragma unroll
                    for (int u = 0; u < UB; u++) {
                        if (q0 + u >= S.w[0]) continue;
                        const uint32_t q4[4] = {nv[u].x, nv[u].y, nv[u].z, nv[u].w};
                        if (st16) {
#pragma unroll
                            for (int e = 0; e < 4; e++) {
                                const uint32_t lo = q4[e] & 0xffffu, hi = q4[e] >> 16;
                                cx<R> z0 = zat(zsh, cbase + lo), z1 = zat(zsh, cbase + hi);
                                if (lo == padb) z0 = cx<R>{(R)0, (R)0};
                                if (hi == padb) z1 = cx<R>{(R)0, (R)0};
                                acc_z<R, P>(T, z0, (R)-1);
                                acc_z<R, P>(T, z1, (R)-1);
                            }
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; e++) acc_z<R, P>(T, zsh[q4[e]], (R)-1);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < UB; u++) {
                        acc_z<R, P>(T, zsh[pv[u].x], (R)1);
                        acc_z<R, P>(T, zsh[pv[u].y], (R)1);
                        acc_z<R, P>(T, zsh[pv[u].z], (R)1);
                        acc_z<R, P>(T, zsh[pv[u].w], (R)1);
                    }
                }
                if (lane < S.rows) {
                    const int i = S.row0 + lane;
                    const cx<R> z = zsh[i];
                    const bool assigned = c >= 0;
                    const R lam = assigned ? (R)(coff[c + 1] - coff[c]) : (R)0;
                    R s = (R)0;
                    if (a.d0 != (R)0) s = a.d0 * (lam + (R)cnt_sh[i]);
                    if (assigned) s -= a.hzero;
                    cx<R> zk = z;
#pragma unroll
                    for (int k = 0; k < P; k++) {
                        const double2 q = assigned ? Q[c * P + k] : make_double2(0.0, 0.0);
                        const cx<R> A = {(R)q.x + T[k].x, (R)q.y + T[k].y};
                        const cx<R> B = cmul(A, cx<R>{zk.x, -zk.y});
                        s += a.dcos[k + 1] * B.x + a.dsin[k + 1] * B.y;
                        if (k + 1 < P) zk = cmul(zk, z);
                    }
                    H[j] = om_sh[i] + a.Kn * s;
                }
            }
            __syncthreads();   // every z of this stage has been read
            // stage update and the next stage's z
            R th[RES_SLICES];
#pragma unroll
            for (int j = 0; j < RES_SLICES; j++) {
                if (a.mode == M_EULER) {
                    tn[j] = wrap_2pi<R>(tn[j] + a.dt * H[j]);
                    th[j] = tn[j];
                } else if (st == 0) {
                    acc[j] = H[j];
                    th[j] = tn[j] + (R)0.5 * a.dt * H[j];
                } else if (st == 1) {
                    acc[j] += (R)2 * H[j];
                    th[j] = tn[j] + (R)0.5 * a.dt * H[j];
                } else if (st == 2) {
                    acc[j] += (R)2 * H[j];
                    th[j] = tn[j] + a.dt * H[j];
                } else {
                    tn[j] = wrap_2pi<R>(tn[j] + a.dt / (R)6 * (acc[j] + H[j]));
                    th[j] = tn[j];
                }
            }
            publish(th, st == nst - 1 ? step + 1 : -1);
        }
    }
#pragma unroll
    for (int j = 0; j < RES_SLICES; j++) {
        const int sl = wid + j * RES_WAVES;
        if (sl >= a.nslices) continue;
        const Slice S = ssh[sl];
        if (lane < S.rows) a.state_out[a.perm[S.row0 + lane]] = tn[j];
    }
}

// ---------------------------------------------------------------------------
// polynomial difference coupling (App. A.3; Desai-Zwanzig, App. A.5)
// ---------------------------------------------------------------------------
// The stage kernel of the polynomial model on the same units, slices and
// remainder streams as the phase model; the staged and gathered value is x
// itself.  E1: per-community moments W_k = sum_{l in c} x_l^k (FP64 unit
// partials, summed in a fixed order).  E2: per row, the partners' moments
// T_k = sum_{S+} x_l^k - sum_{S-} x_l^k.  Combine (eq. PolyDifferenceRHSfast
// by Taylor coefficients): with M_k = W_k + T_k and M_0 = lambda_c + |S+| -
// |S-|, sum_l a_ml h(x_l - x_m) = sum_k M_k g_k(x_m) - h(0), where g_k(x) =
// sum_{a>=k} C(a,k) h_a (-x)^(a-k) are the coefficients of h(y - x) in y,
// and h(0) removes the l = m term that the community sum includes.  The
// direct variant evaluates h(x_l - x_m) on every edge.

// value staged in LDS at a byte offset
template <typename R>
__device__ __forceinline__ R xat(const R *xsh, uint32_t byte_off) {
    return *reinterpret_cast<const R *>(reinterpret_cast<const unsigned char *>(xsh) + byte_off);
}

template <typename R, int P>
__device__ __forceinline__ void acc_pow(R (&T)[P], R x, R sign) {
    R xk = x;
#pragma unroll
    for (int k = 0; k < P; k++) {
        T[k] += sign * xk;
        xk *= x;
    }
}

// The D values of one node, from an array of D-vectors (index v) or from
// LDS at a byte offset: one 4/8/16-byte load.
template <typename R, int D>
__device__ __forceinline__ void ldv(const R *p, uint32_t v, R (&out)[D]) {
    if constexpr (D == 1) {
        out[0] = p[v];
    } else {
        using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
        const V2 t = reinterpret_cast<const V2 *>(p)[v];
        out[0] = t.x;
        out[1] = t.y;
    }
}

template <typename R, int D>
__device__ __forceinline__ void ldsv(const R *xsh, uint32_t byte_off, R (&out)[D]) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(xsh) + byte_off;
    if constexpr (D == 1) {
        out[0] = *reinterpret_cast<const R *>(b);
    } else {
        using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
        const V2 t = *reinterpret_cast<const V2 *>(b);
        out[0] = t.x;
        out[1] = t.y;
    }
}

// D state components (1, or 2 for the two-component oscillators of the
// paper's Table 1): component d of position i lives at d * n + i in theta_n
// and acc, and the stage values are D-vectors, [n + 1][D] with a zero vector
// at n, so one load gathers every component of a partner; LDS holds the
// community's values the same way, [lambda + 1][D], and one byte offset of
// the S-neg stream reaches the whole vector; the unit moments of component d
// go to the .x (d = 0) and .y (d = 1) halves of the partials.
template <typename R, int P, int BLOCK, bool DIRECT, int D>
__global__ __launch_bounds__(BLOCK) void poly_stage_kernel(PhaseArgs<R> a) {
    constexpr int NW = BLOCK / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    R *xsh = reinterpret_cast<R *>(smem);   // [lds_cap + 1][D]
    __shared__ double qsh[D][P];
    __shared__ double red[NW][D][P];

    const Unit Un = a.units[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool assigned = !DIRECT && (Un.flags & UF_ASSIGNED) != 0;
    const bool staged = !DIRECT && (Un.flags & UF_STAGED) != 0;
    const int mode = a.mode;
    const bool gather = mode != M_PREP;
    const int off = Un.off, lam = Un.lam;
    const int64_t n = a.pad_pos;          // nodes; stage arrays have a zero slot at n

    // ---- unit start: the community's values in LDS and its moments ----
    if (gather && assigned) {
        if (staged) {
            constexpr int US = 8;   // loads in flight per thread before the LDS writes
            const int nv = lam * D;
            for (int j0 = tid; j0 < nv; j0 += BLOCK * US) {
                R v[US];
#pragma unroll
                for (int u = 0; u < US; u++)
                    if (j0 + u * BLOCK < nv) v[u] = a.th_in[(int64_t)off * D + j0 + u * BLOCK];
#pragma unroll
                for (int u = 0; u < US; u++)
                    if (j0 + u * BLOCK < nv) xsh[j0 + u * BLOCK] = v[u];
            }
            if (tid < D) xsh[lam * D + tid] = (R)0;
        }
        if (wid == NW - 1) {
            for (int k = 0; k < P; k++) {
                double sx = 0.0, sy = 0.0;
                for (int j = Un.qbeg + lane; j < Un.qend; j += 64) {
                    const double2 q = a.q_in[(size_t)j * P + k];
                    sx += q.x;
                    sy += q.y;
                }
                sx = wave_sum(sx);
                sy = wave_sum(sy);
                if (lane == 0) {
                    qsh[0][k] = sx;
                    if (D == 2) qsh[D - 1][k] = sy;
                }
            }
        }
    }
    __syncthreads();
    double W[D][P], pd[D][P];
#pragma unroll
    for (int d = 0; d < D; d++)
#pragma unroll
        for (int k = 0; k < P; k++) {
            W[d][k] = (gather && assigned) ? qsh[d][k] : 0.0;
            pd[d][k] = 0.0;
        }

    const uint32_t padb = (uint32_t)lam * (uint32_t)(D * sizeof(R));
    const uint32_t pad16 = padb | (padb << 16);
    const uint4 padl = make_uint4(pad16, pad16, pad16, pad16);
    const uint32_t pad = a.pad_pos;
    const uint4 padp = make_uint4(pad, pad, pad, pad);

    for (int sl = Un.s0 + wid; sl < Un.s1; sl += NW) {
        const Slice S = a.slices[sl];
        const bool mine = lane < S.rows;
        const int i = S.row0 + lane;
        R tn[D], av[D], xm[D];
        R om = (R)0, knv = a.Kn;
        int cv = 0;
#pragma unroll
        for (int d = 0; d < D; d++) tn[d] = av[d] = xm[d] = (R)0;
        if (mine) {
            if (mode == M_PREP) {
#pragma unroll
                for (int d = 0; d < D; d++) tn[d] = a.state_in[d * n + a.perm[i]];
            } else {
                if (a.omega) om = a.omega[i];
                if (a.kn) knv = a.kn[i];
                cv = a.cnt[i];
#pragma unroll
                for (int d = 0; d < D; d++) {
                    if (mode != M_RHS) tn[d] = a.theta_n[d * n + i];
                    if (mode == M_RK4 && a.stage > 0) av[d] = a.acc[d * n + i];
                }
                if (staged) ldv<R, D>(xsh, (uint32_t)(i - off), xm);
                else ldv<R, D>(a.th_in, (uint32_t)i, xm);
            }
        }
        R T[D][P];
#pragma unroll
        for (int d = 0; d < D; d++)
#pragma unroll
            for (int k = 0; k < P; k++) T[d][k] = (R)0;
        double Eh[D];   // direct: sum of h(x_l - x_m), or of g(x_l, x_m)
#pragma unroll
        for (int d = 0; d < D; d++) Eh[d] = 0.0;
        // direct with a general coupling (one component): g(x_l, x_m) = sum_a x_l^a B_a
        R Bg[P + 1];
        if (DIRECT && D == 1 && a.pgen) {
#pragma unroll
            for (int q = 0; q <= P; q++) {
                double v = 0.0, xb = 1.0;
                for (int b = 0; b <= P; b++) {
                    v += a.pgen[q * (P + 1) + b] * xb;
                    xb *= (double)xm[0];
                }
                Bg[q] = (R)v;
            }
        }
        if (gather) {
            if (!DIRECT) {
                // S-neg: up to UN chunks in flight (LDS gathers), or UGL (global gathers)
                const uint4 *col = a.negdata + S.beg[0] + lane;
                if (staged) {
                    constexpr int UN = D == 1 ? 8 : 4;
                    for (int k = 0; k < S.w[0]; k += UN) {
                        uint4 v[UN];
#pragma unroll
                        for (int u = 0; u < UN; u++) v[u] = k + u < S.w[0] ? ld_stream(col + (size_t)(k + u) * SLICE) : padl;
#pragma unroll
                        for (int u = 0; u < UN; u++) {
                            const uint32_t q4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                            for (int q = 0; q < 4; q++) {
                                R xa[D], xb[D];
                                ldsv<R, D>(xsh, q4[q] & 0xffffu, xa);
                                ldsv<R, D>(xsh, q4[q] >> 16, xb);
#pragma unroll
                                for (int d = 0; d < D; d++) {
                                    acc_pow<R, P>(T[d], xa[d], (R)-1);
                                    acc_pow<R, P>(T[d], xb[d], (R)-1);
                                }
                            }
                        }
                    }
                } else {
                    constexpr int UGL = 4;
                    for (int k = 0; k < S.w[0]; k += UGL) {
                        uint4 v[UGL];
#pragma unroll
                        for (int u = 0; u < UGL; u++) v[u] = k + u < S.w[0] ? ld_stream(col + (size_t)(k + u) * SLICE) : padp;
                        R xl[UGL][4][D];
#pragma unroll
                        for (int u = 0; u < UGL; u++) {
                            ldv<R, D>(a.th_in, v[u].x, xl[u][0]);
                            ldv<R, D>(a.th_in, v[u].y, xl[u][1]);
                            ldv<R, D>(a.th_in, v[u].z, xl[u][2]);
                            ldv<R, D>(a.th_in, v[u].w, xl[u][3]);
                        }
#pragma unroll
                        for (int u = 0; u < UGL; u++)
#pragma unroll
                            for (int q = 0; q < 4; q++)
#pragma unroll
                                for (int d = 0; d < D; d++) acc_pow<R, P>(T[d], xl[u][q][d], (R)-1);
                    }
                }
            }
            // S-pos (the whole adjacency for the direct method): UGP chunks in flight
            constexpr int UGP = 4;
            const uint4 *col = a.posdata + S.beg[1] + lane;
            for (int k = 0; k < S.w[1]; k += UGP) {
                uint4 v[UGP];
#pragma unroll
                for (int u = 0; u < UGP; u++) v[u] = k + u < S.w[1] ? ld_stream(col + (size_t)(k + u) * SLICE) : padp;
                R xl[UGP][4][D];   // the padding position holds 0
#pragma unroll
                for (int u = 0; u < UGP; u++) {
                    ldv<R, D>(a.th_in, v[u].x, xl[u][0]);
                    ldv<R, D>(a.th_in, v[u].y, xl[u][1]);
                    ldv<R, D>(a.th_in, v[u].z, xl[u][2]);
                    ldv<R, D>(a.th_in, v[u].w, xl[u][3]);
                }
#pragma unroll
                for (int d = 0; d < D; d++) {
#pragma unroll
                    for (int u = 0; u < UGP; u++) {
                        const uint32_t q4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            if (DIRECT) {
                                if (q4[q] != pad) {
                                    R hv;
                                    if (D == 1 && a.pgen) {
                                        hv = Bg[P];
#pragma unroll
                                        for (int e = P - 1; e >= 0; e--) hv = hv * xl[u][q][d] + Bg[e];
                                    } else {
                                        const R dd = xl[u][q][d] - xm[d];
                                        hv = (R)a.ph[P];
#pragma unroll
                                        for (int e = P - 1; e >= 0; e--) hv = hv * dd + (R)a.ph[e];
                                    }
                                    Eh[d] += (double)hv;
                                }
                            } else {
                                acc_pow<R, P>(T[d], xl[u][q][d], (R)1);
                            }
                        }
                    }
                }
            }
        }
        if (mine) {
            R xnew[D];
            if (mode == M_PREP) {
#pragma unroll
                for (int d = 0; d < D; d++) {
                    xnew[d] = tn[d];
                    a.theta_n[d * n + i] = tn[d];
                }
            } else {
                // local term: f(x) (one component, Horner) or f_d(x_0, x_1)
                double fl[D];
                if (D == 1) {
                    double f = 0.0;
                    for (int j = a.pq; j >= 0; j--) f = f * (double)xm[0] + a.pf[j];
                    fl[0] = f;
                } else {
#pragma unroll
                    for (int d = 0; d < D; d++) {
                        double f = 0.0, ui = 1.0;
#pragma unroll
                        for (int ii = 0; ii <= 3; ii++) {
                            double vj = 1.0;
#pragma unroll
                            for (int jj = 0; jj <= 3; jj++) {
                                f += a.pf2[d * 16 + ii * 4 + jj] * ui * vj;
                                vj *= (double)xm[D - 1];
                            }
                            ui *= (double)xm[0];
                        }
                        fl[d] = f;
                    }
                }
#pragma unroll
                for (int d = 0; d < D; d++) {
                    double s;
                    if (DIRECT) {
                        s = Eh[d];
                    } else if (D == 1 && a.pgen) {
                        // general coupling: sum_b x_m^b sum_a c[a][b] M_a, minus g(x_m, x_m)
                        double M[P + 1];
                        M[0] = (assigned ? (double)lam : 0.0) + (double)cv;
#pragma unroll
                        for (int k = 1; k <= P; k++) M[k] = W[d][k - 1] + (double)T[d][k - 1];
                        const double x = (double)xm[d];
                        double xp[2 * P + 1];
                        xp[0] = 1.0;
#pragma unroll
                        for (int k = 1; k <= 2 * P; k++) xp[k] = xp[k - 1] * x;
                        s = 0.0;
                        double own = 0.0;
#pragma unroll
                        for (int q = 0; q <= P; q++)
#pragma unroll
                            for (int b = 0; b <= P; b++) {
                                const double cab = a.pgen[q * (P + 1) + b];
                                s += cab * M[q] * xp[b];
                                own += cab * xp[q + b];
                            }
                        if (assigned) s -= own;
                    } else {
                        // g_k(x_m): Taylor shift of h by -x_m (repeated synthetic division)
                        double g[P + 1];
#pragma unroll
                        for (int k = 0; k <= P; k++) g[k] = a.ph[k];
                        const double c = -(double)xm[d];
#pragma unroll
                        for (int k = 0; k < P; k++)
#pragma unroll
                            for (int j = P - 1; j >= k; j--) g[j] += c * g[j + 1];
                        s = g[0] * ((assigned ? (double)lam : 0.0) + (double)cv);
#pragma unroll
                        for (int k = 1; k <= P; k++) s += g[k] * (W[d][k - 1] + (double)T[d][k - 1]);
                        if (assigned) s -= a.ph[0];
                    }
                    const R H = (R)((d == 0 ? (double)om : 0.0) + fl[d] + (double)knv * s);
                    if (mode == M_RHS) {
                        a.state_out[d * n + a.perm[i]] = H;
                        xnew[d] = (R)0;
                    } else if (mode == M_EULER) {
                        xnew[d] = tn[d] + a.dt * H;
                        a.theta_n[d * n + i] = xnew[d];
                    } else if (a.stage == 0) {
                        a.acc[d * n + i] = H;
                        xnew[d] = tn[d] + (R)0.5 * a.dt * H;
                    } else if (a.stage == 1) {
                        a.acc[d * n + i] = av[d] + (R)2 * H;
                        xnew[d] = tn[d] + (R)0.5 * a.dt * H;
                    } else if (a.stage == 2) {
                        a.acc[d * n + i] = av[d] + (R)2 * H;
                        xnew[d] = tn[d] + a.dt * H;
                    } else {
                        xnew[d] = tn[d] + a.dt / (R)6 * (av[d] + H);
                        a.theta_n[d * n + i] = xnew[d];
                    }
                }
            }
            if (mode != M_RHS) {
                if constexpr (D == 1) {
                    a.th_out[i] = xnew[0];
                } else {
                    using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
                    V2 t;
                    t.x = xnew[0];
                    t.y = xnew[D - 1];
                    reinterpret_cast<V2 *>(a.th_out)[i] = t;
                }
#pragma unroll
                for (int d = 0; d < D; d++) {
                    if (assigned) {
                        double xk = (double)xnew[d];
#pragma unroll
                        for (int k = 0; k < P; k++) {
                            pd[d][k] += xk;
                            xk *= (double)xnew[d];
                        }
                    }
                }
            }
        }
    }
    if (mode == M_RHS || !assigned) return;
    // ---- unit moments of the next stage: fixed-order block reduction ----
#pragma unroll
    for (int d = 0; d < D; d++)
#pragma unroll
        for (int k = 0; k < P; k++) {
            const double v = wave_sum(pd[d][k]);
            if (lane == 0) red[wid][d][k] = v;
        }
    __syncthreads();
    if (tid == 0)
        for (int k = 0; k < P; k++) {
            double v[D];
            for (int d = 0; d < D; d++) {
                v[d] = red[0][d][k];
                for (int w = 1; w < NW; w++) v[d] += red[w][d][k];
            }
            a.q_out[(size_t)Un.qslot * P + k] = make_double2(v[0], D == 2 ? v[D - 1] : 0.0);
        }
}

// ---------------------------------------------------------------------------
// triadic model: intra-community hyperedges (App. A.7 on a hypergraph)
// ---------------------------------------------------------------------------
// A triple {m, j, k} of one community is a hyperedge iff
// splitmix64(seed ^ key(m, j, k)) < thr.  The kernels below take a block of
// up to TRI_ROWS centres of one community, stage the community's user ids
// (and z) in LDS and give each wavefront one centre at a time; the centre's
// partner pairs (x, y), x < y, are walked x-major with the 64 lanes over y.

// splitmix64 output for state x (Steele, Lea, Flood, OOPSLA 2014)
__host__ __device__ static inline uint64_t splitmix64_out(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

constexpr int TRI_ROWS = 16;   // centres per enumeration block (4 wavefronts)
constexpr int TRI_RUN = 7;     // partners per chunk of a missing-pair list

struct alignas(16) TriBlock {
    int32_t off, lam, row0, rows;
};

// lanes below the calling lane whose bit is set in m
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Pairs (x, y), x < y < lam, x != me != y, of centre `me`: group(x, y, ok,
// miss) for every 64 consecutive y of an x (ok: y is a partner; miss: the
// triple is not a hyperedge), then run_end(x).  Wave-uniform control flow.
template <typename G, typename E>
__device__ __forceinline__ void tri_walk(const uint32_t *us, int lam, int me, uint64_t seed, uint64_t thr,
                                         G &&group, E &&run_end) {
    const int lane = threadIdx.x & 63;
    const uint32_t ui = us[me];
    for (int x = 0; x < lam - 1; x++) {
        if (x == me) continue;
        const uint32_t ux = us[x];
        for (int y0 = x + 1; y0 < lam; y0 += 64) {
            const int y = y0 + lane;
            const bool ok = y < lam && y != me;
            bool miss = false;
            if (ok) miss = splitmix64_out(seed ^ triple_key(ui, ux, us[y])) >= thr;
            group(x, y, ok, miss);
        }
        run_end(x);
    }
}

// Missing-pair lists, pass 1: per centre, the number of missing partner
// pairs and of list chunks (a chunk holds one x and up to TRI_RUN of its y).
__global__ __launch_bounds__(256) void tri_count_kernel(const TriBlock *blocks, const int32_t *perm, uint64_t seed,
                                                        uint64_t thr, int32_t *nchunk, int32_t *npair) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *us = reinterpret_cast<uint32_t *>(smem);
    const TriBlock B = blocks[blockIdx.x];
    for (int j = threadIdx.x; j < B.lam; j += 256) us[j] = (uint32_t)perm[B.off + j];
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int r = wid; r < B.rows; r += 4) {
        const int i = B.row0 + r;
        int c = 0, chunks = 0, pairs = 0;
        tri_walk(
            us, B.lam, i - B.off, seed, thr,
            [&](int, int, bool ok, bool miss) { c += __popcll(__ballot(ok && miss)); },
            [&](int) {
                chunks += (c + TRI_RUN - 1) / TRI_RUN;
                pairs += c;
                c = 0;
            });
        if (lane == 0) {
            nchunk[i] = chunks;
            npair[i] = pairs;
        }
    }
}

// Pass 2: write the lists.  Centre i owns chunks [cptr[i], cptr[i+1]); a
// chunk is 8 uint16 LDS byte offsets (x, then y_1..y_7, unused slots at the
// zero slot lam).  Writes past the centre's range are dropped; written[i]
// (chunks produced) lets the host check the two passes agree.
__global__ __launch_bounds__(256) void tri_fill_kernel(const TriBlock *blocks, const int32_t *perm, uint64_t seed,
                                                       uint64_t thr, uint32_t zb, const int64_t *cptr, uint16_t *out,
                                                       int32_t *written) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *us = reinterpret_cast<uint32_t *>(smem);
    const TriBlock B = blocks[blockIdx.x];
    for (int j = threadIdx.x; j < B.lam; j += 256) us[j] = (uint32_t)perm[B.off + j];
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint16_t pad = (uint16_t)((uint32_t)B.lam * zb);
    for (int r = wid; r < B.rows; r += 4) {
        const int i = B.row0 + r;
        const int64_t lim = cptr[i + 1];
        int64_t base = cptr[i];
        int c = 0;
        tri_walk(
            us, B.lam, i - B.off, seed, thr,
            [&](int, int y, bool ok, bool miss) {
                const bool m = ok && miss;
                const uint64_t mask = __ballot(m);
                if (m) {
                    const int pos = c + lanes_below(mask);
                    const int64_t ch = base + pos / TRI_RUN;
                    if (ch < lim) out[ch * 8 + 1 + pos % TRI_RUN] = (uint16_t)((uint32_t)y * zb);
                }
                c += __popcll(mask);
            },
            [&](int x) {
                const int nch = (c + TRI_RUN - 1) / TRI_RUN;
                for (int q = lane; q < nch * 8; q += 64) {
                    const int j = q >> 3, sl = q & 7;
                    if (base + j >= lim) break;
                    if (sl == 0) out[(base + j) * 8] = (uint16_t)((uint32_t)x * zb);
                    else if (j * TRI_RUN + sl - 1 >= c) out[(base + j) * 8 + sl] = pad;
                }
                base += nch;
                c = 0;
            });
        if (lane == 0) written[i] = (int32_t)(base - cptr[i]);
    }
}

// CIA: per centre, M = sum over its missing partner pairs of z_x z_y, one
// wavefront per centre streaming its chunks (x z_x times the sum of the
// run's z_y).  Units: centres [c0, c1) of one community, z staged in LDS.
struct alignas(16) TriUnit {
    int32_t off, lam, c0, c1;
};

template <typename R>
__global__ __launch_bounds__(256) void tri_missing_kernel(const TriUnit *units, const cx<R> *cs, const int64_t *cptr,
                                                          const uint4 *chunks, cx<R> *M) {
    constexpr int U = 4;   // chunks in flight per lane
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R> *zsh = reinterpret_cast<cx<R> *>(smem);
    const TriUnit T = units[blockIdx.x];
    for (int j = threadIdx.x; j < T.lam; j += 256) zsh[j] = cs[T.off + j];
    if (threadIdx.x == 0) zsh[T.lam] = cx<R>{(R)0, (R)0};
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t padb = (uint32_t)T.lam * (uint32_t)sizeof(cx<R>);
    const uint32_t pad16 = padb | (padb << 16);
    const uint4 padv = make_uint4(pad16, pad16, pad16, pad16);
    for (int i = T.c0 + wid; i < T.c1; i += 4) {
        const int64_t e = cptr[i + 1];
        cx<R> acc = {(R)0, (R)0};
        for (int64_t k = cptr[i] + lane; k < e; k += 64 * U) {
            uint4 v[U];
#pragma unroll
            for (int u = 0; u < U; u++) v[u] = k + 64 * u < e ? ld_stream(chunks + k + 64 * u) : padv;
#pragma unroll
            for (int u = 0; u < U; u++) {
                const cx<R> zx = zat(zsh, v[u].x & 0xffffu);
                const uint32_t ys[7] = {v[u].x >> 16, v[u].y & 0xffffu, v[u].y >> 16, v[u].z & 0xffffu,
                                        v[u].z >> 16, v[u].w & 0xffffu, v[u].w >> 16};
                cx<R> S = zat(zsh, ys[0]);
#pragma unroll
                for (int q = 1; q < 7; q++) {
                    const cx<R> zy = zat(zsh, ys[q]);
                    S.x += zy.x;
                    S.y += zy.y;
                }
                const cx<R> p = cmul(zx, S);
                acc.x += p.x;
                acc.y += p.y;
            }
        }
        acc.x = wave_sum(acc.x);
        acc.y = wave_sum(acc.y);
        if (lane == 0) M[i] = acc;
    }
}

// Direct triadic baseline: per centre, the sum of z_x z_y over the PRESENT
// intra-community hyperedges {m, x, y}, x < y, found by evaluating the
// hyperedge predicate for every pair of the community (O(lambda^2) per
// centre); one wavefront per centre, lanes over y.
template <typename R>
__global__ __launch_bounds__(256) void triadic_present_kernel(const TriBlock *blocks, const int32_t *perm,
                                                              const cx<R> *cs, uint64_t seed, uint64_t thr,
                                                              cx<R> *out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const TriBlock B = blocks[blockIdx.x];
    cx<R> *zs = reinterpret_cast<cx<R> *>(smem);
    uint32_t *us = reinterpret_cast<uint32_t *>(smem + sizeof(cx<R>) * B.lam);
    for (int j = threadIdx.x; j < B.lam; j += 256) {
        zs[j] = cs[B.off + j];
        us[j] = (uint32_t)perm[B.off + j];
    }
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int r = wid; r < B.rows; r += 4) {
        const int i = B.row0 + r;
        cx<R> E = {(R)0, (R)0}, S = {(R)0, (R)0};
        tri_walk(
            us, B.lam, i - B.off, seed, thr,
            [&](int, int y, bool ok, bool miss) {
                if (ok && !miss) {
                    const cx<R> zy = zs[y];
                    S.x += zy.x;
                    S.y += zy.y;
                }
            },
            [&](int x) {
                const cx<R> p = cmul(zs[x], S);
                E.x += p.x;
                E.y += p.y;
                S = cx<R>{(R)0, (R)0};
            });
        E.x = wave_sum(E.x);
        E.y = wave_sum(E.y);
        if (lane == 0) out[i] = E;
    }
}

// standalone reduction (one wavefront); with slot_ctr (replayed graphs) the
// output slot is r_out + *slot_ctr
__global__ __launch_bounds__(64) void order_reduce_kernel(const double2 *r_part, int nunits, double invN,
                                                          double *r_out, const int64_t *slot_ctr) {
    reduce_r_wave(r_part, nunits, invN, r_out + (slot_ctr ? *slot_ctr : 0));
}

// Batched ensembles: r_b(t) = |(1/N_b) sum over the nodes of instance b of z|,
// one block per instance over its positions (grouped, increasing), FP64,
// fixed order.  Output r_out[b * stride + slot (+ *slot_ctr)].
template <typename R>
__global__ __launch_bounds__(256) void order_grouped_kernel(const cx<R> *cs, const int32_t *grp_idx,
                                                            const int64_t *grp_off, double *r_out, int64_t stride,
                                                            int64_t slot, const int64_t *slot_ctr) {
    __shared__ double sx[256], sy[256];
    const int b = blockIdx.x;
    const int64_t e0 = grp_off[b], e1 = grp_off[b + 1];
    double x = 0.0, y = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const cx<R> z = cs[grp_idx[e]];
        x += (double)z.x;
        y += (double)z.y;
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
    if (threadIdx.x == 0) {
        const double inv = e1 > e0 ? 1.0 / (double)(e1 - e0) : 0.0;
        r_out[(int64_t)b * stride + slot + (slot_ctr ? *slot_ctr : 0)] =
            sqrt(sx[0] * sx[0] + sy[0] * sy[0]) * inv;
    }
}

// advances the slot counter of replayed step graphs (one thread; vector store)
__global__ void counter_kernel(int64_t *ctr, int64_t set, int add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] = add ? ctr[0] + set : set;
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
            acc_z<R, P>(T, tile[q], (R)1);
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
    bool has_wide = false;   // F32 plan with a community beyond the LDS cap (FP64 observables or tiled)
    bool merged = false;     // some S-pos slices stored merged (SF_MERGED)
    bool tri = false;        // triadic model
    bool poly = false;       // polynomial difference coupling
    void *gen = nullptr;     // general coupling coefficients on the device (R), or NULL
    double *pgen = nullptr;  // polynomial model: general coupling coefficients, or NULL
    int pq = -1;             // degree of the local polynomial f (-1: none)
    int pdim = 1;            // polynomial model: state components per node (1 or 2)
    double ph[PMAX + 1] = {0}, pf[PMAX + 1] = {0};   // coefficients of h and f
    double pf2[32] = {0};    // two components: local polynomials F[d][i][j]
    double K2n = 0;
    uint64_t tri_seed = 0, tri_thr = 0;
    TriBlock *tri_blocks = nullptr;   // direct triadic: (community, centres) blocks
    int32_t ntri_blocks = 0;
    size_t tri_smem = 0;
    TriUnit *tri_units = nullptr;     // CIA triadic: missing-pair sum units
    int32_t tri_nunits = 0;
    size_t tri_msmem = 0;
    int64_t *tri_cptr = nullptr;      // [n+1] chunk offsets of the missing-pair lists
    uint4 *tri_chunks = nullptr;
    void *tri_m = nullptr;            // [n] missing-pair sums (cx<R>)
    void *h_extra = nullptr;
    int32_t nunits = 0, ncomm = 0;
    int lds_cap = 0;
    size_t smem = 0;
    double K = 0, Kn = 0, d0 = 0, hzero = 0;
    double dsin[PMAX + 1] = {0}, dcos[PMAX + 1] = {0};
    // device
    Unit *units = nullptr;
    Slice *slices = nullptr;
    uint4 *negdata = nullptr, *posdata = nullptr, *tposdata = nullptr;
    int32_t *tile_w = nullptr;   // per (slice, tile) S-neg widths of tiled communities
    int32_t tile_cap = 0;        // tile capacity (nodes) of tiled communities
    // small networks: the whole integration in one resident workgroup
    bool resident = false;
    size_t res_smem = 0;
    int32_t nslices = 0;
    int32_t *res_slice_comm = nullptr, *res_slice_flags = nullptr, *res_comm_off = nullptr, *res_comm_slice0 = nullptr;
    int32_t *cnt = nullptr, *perm = nullptr;
    void *omega = nullptr, *theta_n = nullptr, *acc = nullptr, *th[2] = {nullptr, nullptr};
    void *cs[2] = {nullptr, nullptr};
    double2 *q[2] = {nullptr, nullptr};
    double2 *r_part = nullptr;
    double *r_dev = nullptr;
    int64_t r_cap = 0;
    void *hbuf = nullptr;
    void *coef = nullptr;   // [2][PMAX+1] device copy of dsin/dcos (all-to-all kernel)
    // batched ensembles
    int32_t batch = 0;            // instances (0: a single network)
    int32_t *grp_idx = nullptr;   // positions grouped by instance
    int64_t *grp_off = nullptr;   // [batch+1]
    void *kn = nullptr;           // K_b / N_b per position
    // capacities of the unit-dependent buffers (the autotuner rebuilds units)
    size_t units_cap = 0, q_cap = 0, rpart_cap = 0;
    // host inputs of make_units, kept for the autotuner
    std::vector<Slice> h_slices;
    std::vector<int32_t> h_seg_off, h_comm_off;
    std::vector<char> h_staged;
    int32_t h_ncomm = 0;
    uint32_t h_flags = 0;
    int64_t unit_work = 32768;
    void *tune_in = nullptr, *tune_out = nullptr;
    // replayed RK4 step graph
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double g_dt = 0.0;
    int64_t g_stride = 0;
    bool g_want_r = false;
    double *g_r = nullptr;
    int64_t *r_ctr = nullptr;
    ~PhaseState() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto &e : gev)
            if (e) (void)hipEventDestroy(e);
        if (gstream) (void)hipStreamDestroy(gstream);
    }
};

// Row lists handed to the packer: old-order CSR lists of up to four streams.
// Stream entries are either local indices inside the row's community
// (`local`) or old positions; pair streams hold two ints per entry.
struct StreamIn {
    const std::vector<int64_t> *ptr = nullptr;   // [n+1] in entries (null: empty stream)
    const int32_t *val = nullptr;
    int32_t *mut = nullptr;   // S-neg of tiled communities: val, rewritten in place by build_sell
    bool local = false;
    bool pair = false;
};

struct Sell {
    std::vector<int32_t> newpos;          // old position -> new position
    std::vector<Slice> slices;
    std::vector<int32_t> tile_w;          // tiled communities: S-neg width of every (slice, tile)
    std::vector<int32_t> seg_slice_off;   // segment -> first slice
    std::vector<uint4> data[4];
};

// Order rows inside every segment by decreasing remainder work (globally
// gathered chunks first, then LDS-gathered chunks), cut the
// segments into 64-row slices and pack the sliced blocks of every stream.
// Segments are the communities [comm_off[c], comm_off[c+1]) and the tail of
// rows outside every community.  In segments with seg_staged[c], local
// entries are stored as uint16 indices (8 per chunk, pairs 4 per chunk, pad
// lambda), pre-multiplied by zscale = sizeof(z) so they are LDS byte
// offsets; everything else as int32 new positions (4 per chunk, pairs 2 per
// chunk, pad n).
// Segments with seg_staged[c] == SEG_TILED hold a community above the LDS
// cap: its S-neg (stream 0) is split by column tile (ntiles = ceil(lambda /
// tile_cap) tiles of TS = ceil(lambda / ntiles) nodes), every tile stored as
// its own sliced block of uint16 in-tile byte offsets (pad TS * zscale), the
// blocks of a slice one after another; out.tile_w holds every (slice, tile)
// width and Slice::tw the slice's first.
constexpr char SEG_STAGED = 1, SEG_TILED = 2;
static inline void tile_shape(int64_t lam, int64_t tile_cap, int64_t &nt, int64_t &ts) {
    nt = (lam + tile_cap - 1) / tile_cap;
    ts = (lam + nt - 1) / nt;
}

static cia_status build_sell(int64_t n, const std::vector<int32_t> &comm_off, int32_t ncomm,
                             const std::vector<char> &seg_staged, const StreamIn (&S)[4], uint32_t zscale,
                             Sell &out, int64_t tile_cap = 0, bool merge_pos = false) {
    const int32_t nseg = ncomm + 1;
    std::vector<int64_t> sb(nseg + 1);
    for (int32_t c = 0; c <= ncomm; c++) sb[c] = c < ncomm ? comm_off[c] : (ncomm ? comm_off[ncomm] : 0);
    sb[nseg] = n;
    auto len = [&](int q, int64_t i) -> int64_t { return S[q].ptr ? (*S[q].ptr)[i + 1] - (*S[q].ptr)[i] : 0; };
    auto tiled = [&](int q, int32_t c) -> bool { return q == 0 && c < ncomm && seg_staged[c] == SEG_TILED; };
    // entries per 16-byte chunk of stream q in segment c
    auto per = [&](int q, int32_t c) -> int64_t {
        const bool st = c < ncomm && seg_staged[c] && S[q].local;
        const int64_t eb = (st ? 2 : 4) * (S[q].pair ? 2 : 1);
        return 16 / eb;
    };
    // entries of row i (old position) of a tiled segment in column tile t:
    // once rewritten to new local indices and sorted, each tile is one range
    auto tile_range = [&](int32_t c, int64_t i, int64_t t, int64_t ts, int64_t &e0, int64_t &e1) {
        const int32_t *v = S[0].val + (*S[0].ptr)[i];
        const int64_t m = len(0, i);
        e0 = std::lower_bound(v, v + m, (int32_t)(t * ts)) - v;
        e1 = std::lower_bound(v, v + m, (int32_t)((t + 1) * ts)) - v;
    };
    // (for a tiled S-neg this is the untiled count: it only orders the rows)
    auto chunks = [&](int q, int32_t c, int64_t i) -> int64_t { return (len(q, i) + per(q, c) - 1) / per(q, c); };
    out.newpos.resize(n);
    std::vector<int32_t> oldpos(n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < nseg; c++) {
        const int64_t b = sb[c], e = sb[c + 1];
        std::vector<int64_t> key(e - b);
        // globally gathered streams (1, 3: a partner phase and its sincos per
        // slot) first, LDS-gathered streams (0, 2) second, so every slice is
        // nearly uniform in both and few padded slots are evaluated
        for (int64_t k = 0; k < e - b; k++)
            key[k] = ((chunks(1, c, b + k) + chunks(3, c, b + k)) << 32) + chunks(0, c, b + k) + chunks(2, c, b + k);
        std::vector<int32_t> idx(e - b);
        for (int64_t k = 0; k < e - b; k++) idx[k] = (int32_t)k;
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return key[x] > key[y]; });
        for (int64_t k = 0; k < e - b; k++) {
            oldpos[b + k] = (int32_t)(b + idx[k]);
            out.newpos[b + idx[k]] = (int32_t)(b + k);
        }
    }
    // tiled segments: S-neg entries rewritten to new local indices (the
    // staging order) and sorted per row, so tiles are ranges of each row
    for (int32_t c = 0; c < ncomm; c++) {
        if (seg_staged[c] != SEG_TILED || !S[0].ptr) continue;
        if (!S[0].mut) return set_error(CIA_EINVAL, "internal: tiled S-neg needs a writable list");
        const int64_t b = sb[c], e = sb[c + 1];
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = b; i < e; i++) {
            int32_t *v = S[0].mut + (*S[0].ptr)[i];
            const int64_t m = len(0, i);
            for (int64_t k = 0; k < m; k++) v[k] = out.newpos[b + v[k]] - (int32_t)b;
            std::sort(v, v + m);
        }
    }
    // S-pos slices stored merged (SF_MERGED, FP32 plans with P = 1): those
    // whose partners are dense enough that 64 consecutive ones of the sorted
    // stream share cache lines (on average at most MERGE_SPAN nodes apart:
    // 64 4-byte theta values within 64 lines of 128 bytes, mostly far fewer),
    // and long enough that the padding to 256 entries is small
    constexpr int64_t MERGE_MIN = 256, MERGE_SPAN = 32;
    std::vector<int64_t> sl_first(nseg + 1, 0);
    for (int32_t c = 0; c < nseg; c++) sl_first[c + 1] = sl_first[c] + (sb[c + 1] - sb[c] + SLICE - 1) / SLICE;
    std::vector<int64_t> mcount;   // merged S-pos entries per slice, 0 = one row per lane
    if (merge_pos && S[1].ptr && n < ((int64_t)1 << MERGE_ROW_SHIFT)) {
        mcount.assign(sl_first[nseg], 0);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < sl_first[nseg]; k++) {
            const int32_t c = (int32_t)(std::upper_bound(sl_first.begin(), sl_first.end(), k) - sl_first.begin()) - 1;
            const int64_t r = sb[c] + (k - sl_first[c]) * SLICE, rows = std::min<int64_t>(SLICE, sb[c + 1] - r);
            int64_t tot = 0, longest = 0;
            int32_t lo = INT32_MAX, hi = -1;
            for (int64_t l = 0; l < rows; l++) {
                const int64_t o = oldpos[r + l];
                for (int64_t e = (*S[1].ptr)[o]; e < (*S[1].ptr)[o + 1]; e++) {
                    const int32_t pn = out.newpos[S[1].val[e]];
                    lo = std::min(lo, pn);
                    hi = std::max(hi, pn);
                }
                tot += len(1, o);
                longest = std::max(longest, len(1, o));
            }
            // a row's fixed-point sum holds at most 2^23 entries of magnitude <= 2^40
            if (tot >= MERGE_MIN && longest < ((int64_t)1 << 23) && (int64_t)hi - lo + 1 <= MERGE_SPAN * tot)
                mcount[k] = tot;
        }
    }
    // slices and their widths
    out.slices.clear();
    out.tile_w.clear();
    out.seg_slice_off.assign(nseg + 1, 0);
    uint64_t tot[4] = {0, 0, 0, 0};
    for (int32_t c = 0; c < nseg; c++) {
        out.seg_slice_off[c] = (int32_t)out.slices.size();
        for (int64_t r = sb[c]; r < sb[c + 1]; r += SLICE) {
            Slice Sl{};
            Sl.row0 = (int32_t)r;
            Sl.rows = (int32_t)std::min<int64_t>(SLICE, sb[c + 1] - r);
            for (int q = 0; q < 4; q++) {
                int64_t w = 0;
                if (tiled(q, c)) {
                    // per-tile widths, the tile blocks one after another
                    int64_t nt, ts;
                    tile_shape(sb[c + 1] - sb[c], tile_cap, nt, ts);
                    Sl.tw = (int32_t)out.tile_w.size();
                    for (int64_t t = 0; t < nt; t++) {
                        int64_t wt = 0;
                        for (int l = 0; l < Sl.rows; l++) {
                            int64_t e0, e1;
                            tile_range(c, oldpos[r + l], t, ts, e0, e1);
                            wt = std::max(wt, (e1 - e0 + 7) / 8);
                        }
                        out.tile_w.push_back((int32_t)wt);
                        w += wt;
                    }
                } else if (q == 1 && !mcount.empty() && mcount[out.slices.size()] > 0) {
                    // merged: 256 entries per chunk row (4 per lane)
                    w = (mcount[out.slices.size()] + 4 * SLICE - 1) / (4 * SLICE);
                    Sl.sflags |= SF_MERGED;
                } else {
                    for (int l = 0; l < Sl.rows; l++) w = std::max(w, chunks(q, c, oldpos[r + l]));
                }
                Sl.beg[q] = (uint32_t)tot[q];
                Sl.w[q] = (int32_t)w;
                tot[q] += (uint64_t)w * SLICE;
                if (tot[q] > 0xffffffffULL) return set_error(CIA_EUNSUPPORTED, "remainder stream above 64 GiB");
            }
            out.slices.push_back(Sl);
        }
    }
    out.seg_slice_off[nseg] = (int32_t)out.slices.size();
    try {
        for (int q = 0; q < 4; q++) out.data[q].resize(std::max<uint64_t>(tot[q], 1));
    } catch (const std::bad_alloc &) {
        return set_error(CIA_ENOMEM, "host allocation of the sliced remainder failed");
    }
    const int64_t nsl = (int64_t)out.slices.size();
    std::vector<int32_t> seg_of_slice(nsl);
    for (int32_t c = 0; c < nseg; c++)
        for (int32_t k = out.seg_slice_off[c]; k < out.seg_slice_off[c + 1]; k++) seg_of_slice[k] = c;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nsl; k++) {
        const Slice &Sl = out.slices[k];
        const int32_t c = seg_of_slice[k];
        const int64_t off = sb[c], lam = sb[c + 1] - sb[c];
        for (int q = 0; q < 4; q++) {
            if (!S[q].ptr || Sl.w[q] == 0) continue;
            if (tiled(q, c)) {
                // tile t's block: its width's chunks of in-tile offsets, pad TS
                int64_t nt, ts;
                tile_shape(lam, tile_cap, nt, ts);
                uint16_t *w16 = reinterpret_cast<uint16_t *>(out.data[q].data() + Sl.beg[q]);
                int64_t base = 0;   // chunks of the earlier tiles, per lane
                for (int64_t t = 0; t < nt; t++) {
                    const int64_t wt = out.tile_w[Sl.tw + t];
                    for (int l = 0; l < SLICE; l++) {
                        const int64_t o = l < Sl.rows ? oldpos[Sl.row0 + l] : -1;
                        int64_t e0 = 0, e1 = 0;
                        if (o >= 0) tile_range(c, o, t, ts, e0, e1);
                        const int32_t *src = o >= 0 ? S[q].val + (*S[q].ptr)[o] : nullptr;
                        for (int64_t e = 0; e < wt * 8; e++) {
                            const int64_t chunk = base + e / 8, slot = e % 8;
                            uint16_t v = (uint16_t)(ts * zscale);
                            if (e < e1 - e0) v = (uint16_t)((src[e0 + e] - t * ts) * zscale);
                            w16[(chunk * SLICE + l) * 8 + slot] = v;
                        }
                    }
                    base += wt;
                }
                continue;
            }
            if (q == 1 && (Sl.sflags & SF_MERGED)) {
                // every row's partners, sorted by (new position, lane)
                std::vector<uint64_t> ent;
                ent.reserve((size_t)Sl.w[q] * 4 * SLICE);
                for (int l = 0; l < Sl.rows; l++) {
                    const int64_t o = oldpos[Sl.row0 + l];
                    for (int64_t e = (*S[q].ptr)[o]; e < (*S[q].ptr)[o + 1]; e++)
                        ent.push_back(((uint64_t)out.newpos[S[q].val[e]] << 6) | (uint64_t)l);
                }
                std::sort(ent.begin(), ent.end());
                uint32_t *w32 = reinterpret_cast<uint32_t *>(out.data[q].data() + Sl.beg[q]);
                for (int64_t e = 0; e < (int64_t)Sl.w[q] * 4 * SLICE; e++) {
                    const int64_t chunk = e / (4 * SLICE), word = (e % (4 * SLICE)) / SLICE, l = e % SLICE;
                    uint32_t v = (uint32_t)n;
                    if (e < (int64_t)ent.size())
                        v = (uint32_t)(ent[e] >> 6) | ((uint32_t)(ent[e] & 63) << MERGE_ROW_SHIFT);
                    w32[(chunk * SLICE + l) * 4 + word] = v;
                }
                continue;
            }
            const int64_t pc = per(q, c);
            const bool st16 = c < ncomm && seg_staged[c] && S[q].local;
            const int ne = S[q].pair ? 2 : 1;   // ints per entry
            uint16_t *w16 = reinterpret_cast<uint16_t *>(out.data[q].data() + Sl.beg[q]);
            uint32_t *w32 = reinterpret_cast<uint32_t *>(out.data[q].data() + Sl.beg[q]);
            for (int l = 0; l < SLICE; l++) {
                const int64_t o = l < Sl.rows ? oldpos[Sl.row0 + l] : -1;
                const int64_t nn = o >= 0 ? len(q, o) : 0;
                const int32_t *src = o >= 0 ? S[q].val + (*S[q].ptr)[o] * ne : nullptr;
                for (int64_t e = 0; e < (int64_t)Sl.w[q] * pc; e++) {
                    const int64_t chunk = e / pc, slot = e % pc;
                    for (int t = 0; t < ne; t++) {
                        const int64_t word = ((chunk * SLICE + l) * pc + slot) * ne + t;
                        if (st16) {
                            uint16_t v = (uint16_t)(lam * zscale);
                            if (e < nn) v = (uint16_t)((out.newpos[off + src[e * ne + t]] - off) * zscale);
                            w16[word] = v;
                        } else {
                            uint32_t v = (uint32_t)n;
                            if (e < nn) {
                                const int64_t old = S[q].local ? off + src[e * ne + t] : src[e * ne + t];
                                v = (uint32_t)out.newpos[old];
                            }
                            w32[word] = v;
                        }
                    }
                }
            }
        }
    }
    return CIA_OK;
}

// Slices a tiled community's unit may hold: SMAX per wavefront of the stage
// kernel (SMAX = 4, 2, 1 for P <= 2, <= 4, above).
static int tiled_slices(int P, int block) { return (P <= 2 ? 4 : (P <= 4 ? 2 : 1)) * (block / 64); }
static cia_status check_tiled_units(const std::vector<Unit> &units, int P, int block) {
    for (const Unit &u : units)
        if ((u.flags & UF_TILED) && u.s1 - u.s0 > tiled_slices(P, block))
            return set_error(CIA_EINVAL, "internal: tiled unit of %d slices", u.s1 - u.s0);
    return CIA_OK;
}

// Build the work units and their launch order.
//  - a unit is a run of slices of one community (or of the rows outside every
//    community), sized by slice chunks;
//  - communities are assigned whole to one of the 8 XCDs (workgroup ids are
//    dispatched round-robin over the XCDs), largest first onto the least
//    loaded XCD, so a community's staged z values are read through one L2;
//  - inside an XCD the longest units start first; the launch order
//    interleaves the 8 XCD queues (padding with empty units);
//  - partial-observable slots are numbered community by community in
//    increasing row order, so a community sums a contiguous slot range in a
//    fixed order.  Returns the number of slots.
static int32_t make_units(const Sell &sell, const std::vector<int32_t> &comm_off, int32_t ncomm,
                          int64_t target_chunks, int min_slices, const std::vector<char> &comm_staged,
                          uint32_t opt_flags, std::vector<Unit> &units, int max_tiled_slices = 16) {
    const int NX = 8;
    struct U2 {
        Unit u;
        int64_t work;
        int32_t comm;
    };
    // cost of a slice in chunk units: its chunks plus a fixed cost for the
    // combine operands and the row-order round trips
    auto sw = [&](int32_t k) -> int64_t {
        const Slice &S = sell.slices[k];
        return (int64_t)(S.w[0] + S.w[1] + S.w[2] + S.w[3] + 16) * SLICE;
    };
    std::vector<std::vector<U2>> groups;
    auto make_group = [&](int32_t k0, int32_t k1, int32_t comm, int64_t off, int64_t lam) {
        std::vector<U2> g;
        int32_t k = k0;
        // a tiled community's unit holds at most max_tiled_slices slices (its
        // wavefronts keep the S-neg sums of every slice across the tiles)
        const bool tl = comm >= 0 && comm_staged[comm] == SEG_TILED;
        while (k < k1) {
            int64_t w = 0;
            int32_t e = k;
            while (e < k1 && (w < target_chunks || e - k < std::min(min_slices, k1 - k)) &&
                   (!tl || e - k < max_tiled_slices)) {
                w += sw(e);
                e++;
            }
            int flags = 0;
            if (comm >= 0) {
                flags |= UF_ASSIGNED;
                if ((double)lam > WIDE_COMMUNITY || (opt_flags & CIA_FLAG_FORCE_WIDE)) flags |= UF_WIDE;
                if (comm_staged[comm] == SEG_STAGED) flags |= UF_STAGED;
                if (tl) flags |= UF_TILED;
            }
            Unit u{k, e, flags, (int32_t)(comm >= 0 ? off : 0), (int32_t)(comm >= 0 ? lam : 0), 0, 0, 0};
            g.push_back({u, w, comm});
            k = e;
        }
        groups.push_back(std::move(g));
    };
    for (int32_t c = 0; c < ncomm; c++)
        make_group(sell.seg_slice_off[c], sell.seg_slice_off[c + 1], c, comm_off[c], comm_off[c + 1] - comm_off[c]);
    {
        make_group(sell.seg_slice_off[ncomm], sell.seg_slice_off[ncomm + 1], -1, 0, 0);
        std::vector<U2> rest = std::move(groups.back());
        groups.pop_back();
        for (auto &u : rest) groups.push_back(std::vector<U2>{u});
    }
    int32_t slot = 0;
    for (auto &g : groups) {
        if (g.empty() || g[0].comm < 0) continue;
        int32_t qb = slot;
        for (auto &u : g) u.u.qslot = slot++;
        for (auto &u : g) {
            u.u.qbeg = qb;
            u.u.qend = slot;
        }
    }
    std::vector<int64_t> gw(groups.size(), 0);
    for (size_t k = 0; k < groups.size(); k++)
        for (auto &u : groups[k]) gw[k] += u.work;
    std::vector<size_t> order(groups.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return gw[x] > gw[y]; });
    std::vector<std::vector<U2>> xq(NX);
    std::vector<int64_t> xl(NX, 0);
    for (size_t k : order) {
        int best = 0;
        for (int x = 1; x < NX; x++)
            if (xl[x] < xl[best]) best = x;
        for (auto &u : groups[k]) xq[best].push_back(u);
        xl[best] += gw[k];
    }
    size_t depth = 0;
    for (int x = 0; x < NX; x++) {
        std::stable_sort(xq[x].begin(), xq[x].end(), [](const U2 &a, const U2 &b) { return a.work > b.work; });
        depth = std::max(depth, xq[x].size());
    }
    units.clear();
    for (size_t j = 0; j < depth; j++)
        for (int x = 0; x < NX; x++)
            units.push_back(j < xq[x].size() ? xq[x][j].u : Unit{0, 0, 0, 0, 0, 0, 0, 0});
    while (!units.empty() && units.back().s0 == units.back().s1) units.pop_back();
    return slot;
}

// ---------------------------------------------------------------------------
// triadic model: hyperedge lists per centre (App. A.7 on a hypergraph)
// ---------------------------------------------------------------------------

static uint64_t triple_threshold(double p) {
    if (p <= 0.0) return 0;
    if (p >= 1.0) return UINT64_MAX;
    return (uint64_t)std::ldexp(p, 64);
}

// For every centre, the partner pairs of the explicit cross-community
// hyperedges (old positions), in P1's (old) position order.  The
// intra-community triples are given by the predicate and listed on the GPU.
static cia_status triadic_cross_lists(const P1 &p1, const cia_hypergraph *h, std::vector<int64_t> &xptr,
                                      std::vector<int32_t> &xval) {
    const int64_t n = p1.n;
    // explicit hyperedges, three centres each
    xptr.assign(n + 1, 0);
    const int32_t *t = h->tri;
    if (h->ntri > 0 && !t) return set_error(CIA_EINVAL, "hypergraph: tri is NULL");
    for (int64_t q = 0; q < h->ntri; q++) {
        const int32_t a = t[3 * q], b = t[3 * q + 1], d = t[3 * q + 2];
        if (a < 0 || b < 0 || d < 0 || a >= n || b >= n || d >= n || a == b || b == d || a == d)
            return set_error(CIA_EINVAL, "hypergraph: triangle %lld is not three distinct nodes", (long long)q);
        const int32_t ca = p1.comm_of_pos[p1.inv[a]], cb = p1.comm_of_pos[p1.inv[b]], cd = p1.comm_of_pos[p1.inv[d]];
        if (ca >= 0 && ca == cb && cb == cd)
            return set_error(CIA_EINVAL, "hypergraph: triangle %lld lies inside one community "
                                         "(such triples are given by the predicate)", (long long)q);
        xptr[p1.inv[a] + 1]++;
        xptr[p1.inv[b] + 1]++;
        xptr[p1.inv[d] + 1]++;
    }
    for (int64_t i = 0; i < n; i++) xptr[i + 1] += xptr[i];
    xval.assign(2 * std::max<int64_t>(xptr[n], 1), 0);
    std::vector<int64_t> fill(xptr.begin(), xptr.end() - 1);
    for (int64_t q = 0; q < h->ntri; q++) {
        const int32_t v[3] = {p1.inv[t[3 * q]], p1.inv[t[3 * q + 1]], p1.inv[t[3 * q + 2]]};
        for (int r = 0; r < 3; r++) {
            const int64_t at = fill[v[r]]++;
            xval[2 * at] = v[(r + 1) % 3];
            xval[2 * at + 1] = v[(r + 2) % 3];
        }
    }
    return CIA_OK;
}

// Device scratch of one build step, freed on every exit path.
struct DevTmp {
    void *p = nullptr;
    DevTmp() = default;
    DevTmp(const DevTmp &) = delete;
    DevTmp &operator=(const DevTmp &) = delete;
    ~DevTmp() {
        if (p) (void)hipFree(p);
    }
    cia_status alloc(size_t bytes) {
        hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return set_error(e == hipErrorOutOfMemory ? CIA_ENOMEM : CIA_EHIP, "hipMalloc of %zu bytes failed: %s",
                             bytes, hipGetErrorString(e));
        }
        return CIA_OK;
    }
};

// Enumeration blocks (community, up to TRI_ROWS centres) of every community
// with at least three members.
static std::vector<TriBlock> tri_blocks(const std::vector<int32_t> &comm_off, int32_t ncomm, int32_t &maxl) {
    std::vector<TriBlock> tb;
    maxl = 0;
    for (int32_t cc = 0; cc < ncomm; cc++) {
        const int32_t off = comm_off[cc], lam = comm_off[cc + 1] - off;
        if (lam < 3) continue;
        maxl = std::max(maxl, lam);
        for (int32_t r = 0; r < lam; r += TRI_ROWS) tb.push_back(TriBlock{off, lam, off + r, std::min(TRI_ROWS, lam - r)});
    }
    return tb;
}

// CIA triadic: the missing-pair lists of every centre, built on the device
// (count pass, offsets on the host, fill pass), and the units of the
// per-stage missing-pair sum, centres of one community with about equal
// list length.  npairs: missing partner pairs over all centres (three per
// missing triple); nchunks: list chunks of 16 bytes.
static cia_status tri_build_missing(cia_plan *p, PhaseState *s, const std::vector<int32_t> &comm_off, int32_t ncomm,
                                    int64_t n, uint32_t zb, int64_t &npairs, int64_t &nchunks) {
    npairs = nchunks = 0;
    if (s->tri_thr == UINT64_MAX) return CIA_OK;   // every intra triple is a hyperedge
    int32_t maxl = 0;
    const std::vector<TriBlock> tb = tri_blocks(comm_off, ncomm, maxl);
    if (tb.empty()) return CIA_OK;
    if ((int64_t)maxl * zb > 65535)
        return set_error(CIA_EUNSUPPORTED,
                         "triadic model: community of %d nodes; missing-pair lists cover communities of up to %d nodes",
                         maxl, (int)(65535 / zb));
    DevTmp dblk, dcnt, dpair;
    CIA_TRY(dblk.alloc(sizeof(TriBlock) * tb.size()));
    CIA_TRY(dcnt.alloc(sizeof(int32_t) * n));
    CIA_TRY(dpair.alloc(sizeof(int32_t) * n));
    CIA_HIP(hipMemcpy(dblk.p, tb.data(), sizeof(TriBlock) * tb.size(), hipMemcpyHostToDevice));
    CIA_HIP(hipMemset(dcnt.p, 0, sizeof(int32_t) * n));
    CIA_HIP(hipMemset(dpair.p, 0, sizeof(int32_t) * n));
    const auto *blk = static_cast<const TriBlock *>(dblk.p);
    hipLaunchKernelGGL(tri_count_kernel, dim3((unsigned)tb.size()), dim3(256), (size_t)maxl * 4, nullptr, blk, s->perm,
                       (uint64_t)s->tri_seed, (uint64_t)s->tri_thr, static_cast<int32_t *>(dcnt.p),
                       static_cast<int32_t *>(dpair.p));
    CIA_HIP(hipGetLastError());
    std::vector<int32_t> cnt(n), pairs(n);
    CIA_HIP(hipMemcpy(cnt.data(), dcnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    CIA_HIP(hipMemcpy(pairs.data(), dpair.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    std::vector<int64_t> cptr(n + 1, 0);
    for (int64_t i = 0; i < n; i++) {
        cptr[i + 1] = cptr[i] + cnt[i];
        npairs += pairs[i];
    }
    nchunks = cptr[n];
    CIA_TRY(dupload(p, &s->tri_cptr, cptr.data(), cptr.size()));
    CIA_TRY(dalloc(p, &s->tri_chunks, (size_t)std::max<int64_t>(nchunks, 1)));
    hipLaunchKernelGGL(tri_fill_kernel, dim3((unsigned)tb.size()), dim3(256), (size_t)maxl * 4, nullptr, blk, s->perm,
                       (uint64_t)s->tri_seed, (uint64_t)s->tri_thr, zb, s->tri_cptr,
                       reinterpret_cast<uint16_t *>(s->tri_chunks), static_cast<int32_t *>(dpair.p));
    CIA_HIP(hipGetLastError());
    std::vector<int32_t> wrote(n);
    CIA_HIP(hipMemcpy(wrote.data(), dpair.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (const TriBlock &b : tb)
        for (int32_t r = 0; r < b.rows; r++)
            if (wrote[b.row0 + r] != cnt[b.row0 + r])
                return set_error(CIA_EHIP, "triadic lists: fill pass wrote %d chunks for centre %d, count pass %d",
                                 wrote[b.row0 + r], b.row0 + r, cnt[b.row0 + r]);

    // units: cut a community's centres every TRI_ROWS / 4 * 4 centres once
    // the unit holds `target` chunks (four wavefronts share a unit)
    const int64_t target = std::max<int64_t>(nchunks / 2048, 1024);
    std::vector<TriUnit> units;
    std::vector<int64_t> work;
    for (int32_t cc = 0; cc < ncomm; cc++) {
        const int32_t off = comm_off[cc], lam = comm_off[cc + 1] - off;
        if (lam < 3) continue;
        int32_t c0 = off;
        int64_t w = 0;
        for (int32_t i = off; i < off + lam; i++) {
            w += cnt[i];
            if ((w >= target && (i + 1 - c0) % 4 == 0) || i + 1 == off + lam) {
                units.push_back(TriUnit{off, lam, c0, i + 1});
                work.push_back(w);
                c0 = i + 1;
                w = 0;
            }
        }
    }
    // longest units first
    std::vector<int32_t> ord(units.size());
    for (size_t k = 0; k < ord.size(); k++) ord[k] = (int32_t)k;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    std::vector<TriUnit> sorted(units.size());
    for (size_t k = 0; k < ord.size(); k++) sorted[k] = units[ord[k]];
    s->tri_nunits = (int32_t)sorted.size();
    CIA_TRY(dupload(p, &s->tri_units, sorted.data(), sorted.size()));
    s->tri_msmem = (size_t)(maxl + 1) * zb;
    if (s->tri_msmem > LDS_BYTES) return set_error(CIA_EUNSUPPORTED, "triadic model: LDS request too large");
    unsigned char *raw;
    CIA_TRY(dalloc(p, &raw, (size_t)zb * n));
    CIA_HIP(hipMemset(raw, 0, (size_t)zb * n));
    s->tri_m = raw;
    return CIA_OK;
}

// Whether the plan's integration runs in one resident workgroup: a single
// network of the phase model with the difference coupling (order <= 4), the
// CIA method, every community staged whole, at most 128 slices and LDS for
// all z values, slice partials and community sums.
template <typename R, int P>
static bool res_attr(size_t bytes) {
    const hipError_t e = hipFuncSetAttribute((const void *)resident_integrate_kernel<R, P>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) (void)hipGetLastError();
    return e == hipSuccess;
}
template <typename R>
static bool res_attr_p(int P, size_t bytes) {
    switch (P) {
        case 1: return res_attr<R, 1>(bytes);
        case 2: return res_attr<R, 2>(bytes);
        case 3: return res_attr<R, 3>(bytes);
        default: return res_attr<R, 4>(bytes);
    }
}

static cia_status resident_setup(cia_plan *p, PhaseState *s, const cia_options *o) {
    s->resident = false;
    if (s->direct || s->complete_direct || s->tri || s->poly || s->gen || s->batch > 0 || s->has_wide) return CIA_OK;
    if ((o->flags & CIA_FLAG_NO_RESIDENT) || s->P > RES_PMAX || s->h_slices.empty() || s->merged) return CIA_OK;
    // one CU's LDS serves every remainder gather of a stage: beyond about
    // 1.3e5 entries the stage-by-stage launches over all CUs are faster
    // (measured: 34K entries 1.6x faster resident, 280K equal, 2.5M 4x slower)
    if (p->info.nnz_neg + p->info.nnz_pos > RES_MAX_REMAINDER) return CIA_OK;
    const int64_t nsl = (int64_t)s->h_slices.size();
    if (nsl > (int64_t)(s->f64 ? res_block<double>() / 64 * res_slices<double>()
                               : res_block<float>() / 64 * res_slices<float>())) return CIA_OK;
    for (const Slice &S : s->h_slices)
        if (S.w[2] || S.w[3]) return CIA_OK;
    const int32_t nc = s->h_ncomm;
    const size_t bytes = s->f64 ? res_smem<double>(p->n, nsl, nc, s->P) : res_smem<float>(p->n, nsl, nc, s->P);
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess) {
        (void)hipGetLastError();
        lds_max = 64 * 1024;
    }
    if (bytes > std::min<size_t>(RES_LDS_BYTES, (size_t)lds_max)) return CIA_OK;
    // a device that refuses the LDS size keeps the stage-by-stage path
    if (!(s->f64 ? res_attr_p<double>(s->P, bytes) : res_attr_p<float>(s->P, bytes))) return CIA_OK;
    std::vector<int32_t> scomm(nsl, -1), sflags(nsl, 0);
    for (int32_t c = 0; c < nc; c++)
        for (int32_t k = s->h_seg_off[c]; k < s->h_seg_off[c + 1]; k++) {
            scomm[k] = c;
            sflags[k] = s->h_staged[c] == SEG_STAGED ? UF_STAGED : 0;
        }
    std::vector<int32_t> cs0(s->h_seg_off.begin(), s->h_seg_off.begin() + nc + 1);
    CIA_TRY(dupload(p, &s->res_slice_comm, scomm.data(), scomm.size()));
    CIA_TRY(dupload(p, &s->res_slice_flags, sflags.data(), sflags.size()));
    CIA_TRY(dupload(p, &s->res_comm_off, s->h_comm_off.data(), s->h_comm_off.size()));
    CIA_TRY(dupload(p, &s->res_comm_slice0, cs0.data(), cs0.size()));
    s->nslices = (int32_t)nsl;
    s->res_smem = bytes;
    s->resident = true;
    p->info.resident = 1;
    return CIA_OK;
}

cia_status phase_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                       const double *omega, const cia_options *o, const BatchSpec *bs, P1 *pre) {
    PhaseState *s = new (std::nothrow) PhaseState();
    if (!s) return set_error(CIA_ENOMEM, "host allocation failed");
    p->phase = s;
    const bool f64 = o->precision == CIA_F64;
    s->f64 = f64;
    s->direct = o->method == CIA_METHOD_DIRECT;
    if (c->model == CIA_MODEL_POLY) {
        if (c->p < 1 || c->p > PMAX) return set_error(CIA_EINVAL, "coupling.p = %d; supported 1..%d", c->p, PMAX);
        if (!c->poly_h && !c->poly_g) return set_error(CIA_EINVAL, "polynomial model: coupling.poly_h is NULL");
        if (c->poly_q < -1 || c->poly_q > PMAX)
            return set_error(CIA_EINVAL, "coupling.poly_q = %d; supported -1..%d", c->poly_q, PMAX);
        if (c->poly_q >= 0 && !c->poly_f) return set_error(CIA_EINVAL, "polynomial model: coupling.poly_f is NULL");
        if (c->poly_g) {
            const int np = (c->p + 1) * (c->p + 1);
            for (int k = 0; k < np; k++)
                if (!std::isfinite(c->poly_g[k])) return set_error(CIA_EINVAL, "coupling.poly_g must be finite");
            CIA_TRY(dupload(p, &s->pgen, c->poly_g, (size_t)np));
        } else {
            for (int k = 0; k <= c->p; k++)
                if (!std::isfinite(c->poly_h[k])) return set_error(CIA_EINVAL, "coupling.poly_h must be finite");
        }
        for (int k = 0; k <= c->poly_q; k++)
            if (!std::isfinite(c->poly_f[k])) return set_error(CIA_EINVAL, "coupling.poly_f must be finite");
        if (c->poly_dim < 0 || c->poly_dim > 2)
            return set_error(CIA_EINVAL, "coupling.poly_dim = %d; supported 0..2", c->poly_dim);
        if (c->poly_dim == 2) {
            if (c->poly_g || c->poly_q >= 0)
                return set_error(CIA_EUNSUPPORTED, "two components: poly_g and poly_f/poly_q are not supported");
            if (bs) return set_error(CIA_EUNSUPPORTED, "two components: batched ensembles are not supported");
            if (c->poly_f2)
                for (int k = 0; k < 32; k++) {
                    if (!std::isfinite(c->poly_f2[k])) return set_error(CIA_EINVAL, "coupling.poly_f2 must be finite");
                    s->pf2[k] = c->poly_f2[k];
                }
            s->pdim = 2;
        }
        if (g->kind == CIA_GRAPH_COMPLETE && o->method == CIA_METHOD_DIRECT)
            return set_error(CIA_EUNSUPPORTED, "polynomial model: the direct method needs an explicit CSR graph");
        s->poly = true;
        s->P = c->p;
        s->pq = c->poly_q;
        if (!c->poly_g)
            for (int k = 0; k <= c->p; k++) s->ph[k] = c->poly_h[k];
        for (int k = 0; k <= c->poly_q; k++) s->pf[k] = c->poly_f[k];
        // the zeroth moment of every row's partners (|S+| - |S-|) is always needed
        s->d0 = 1.0;
    }
    const bool gen = c->model == CIA_MODEL_PHASE && (c->gen_c11 || c->gen_c12 || c->gen_c21 || c->gen_c22);
    if (c->model == CIA_MODEL_PHASE) {
        if (c->p < 1 || c->p > PMAX) return set_error(CIA_EINVAL, "coupling.p = %d; supported 1..%d", c->p, PMAX);
        if (!gen) {
            if (!c->d_sin || !c->d_cos) return set_error(CIA_EINVAL, "coupling.d_sin/d_cos are NULL");
            for (int k = 0; k <= c->p; k++)
                if (!std::isfinite(c->d_sin[k]) || !std::isfinite(c->d_cos[k]))
                    return set_error(CIA_EINVAL, "coupling coefficients must be finite");
            s->d0 = c->d_cos[0];
            s->hzero = c->d_cos[0];
            for (int k = 1; k <= c->p; k++) {
                s->dsin[k] = c->d_sin[k];
                s->dcos[k] = c->d_cos[k];
                s->hzero += c->d_cos[k];
            }
        }
        s->P = c->p;
        if (gen) {
            if (c->p > GEN_PMAX)
                return set_error(CIA_EUNSUPPORTED, "general coupling: order p = %d; supported 1..%d", c->p, GEN_PMAX);
            if (!c->gen_c11 || !c->gen_c12 || !c->gen_c21 || !c->gen_c22)
                return set_error(CIA_EINVAL, "general coupling: set all of gen_c11, gen_c12, gen_c21, gen_c22");
            const int np = (c->p + 1) * (c->p + 1);
            for (int i = 0; i < np; i++)
                if (!std::isfinite(c->gen_c11[i]) || !std::isfinite(c->gen_c12[i]) || !std::isfinite(c->gen_c21[i]) ||
                    !std::isfinite(c->gen_c22[i]))
                    return set_error(CIA_EINVAL, "general coupling coefficients must be finite");
            if (g->kind == CIA_GRAPH_COMPLETE && o->method == CIA_METHOD_DIRECT)
                return set_error(CIA_EUNSUPPORTED, "general coupling: the direct method needs an explicit CSR graph");
            if (bs) return set_error(CIA_EUNSUPPORTED, "general coupling: ensembles are not batched");
            std::vector<double> gh(4 * (size_t)np);
            for (int i = 0; i < np; i++) {
                gh[i] = c->gen_c11[i];
                gh[np + i] = c->gen_c12[i];
                gh[2 * np + i] = c->gen_c21[i];
                gh[3 * np + i] = c->gen_c22[i];
            }
            if (o->precision == CIA_F64) {
                double *d;
                CIA_TRY(dupload(p, &d, gh.data(), gh.size()));
                s->gen = d;
            } else {
                std::vector<float> gf(gh.begin(), gh.end());
                float *d;
                CIA_TRY(dupload(p, &d, gf.data(), gf.size()));
                s->gen = d;
            }
            s->d0 = 1.0;   // the partner counts are always needed
        }
    }
    s->K = c->K;
    s->Kn = c->K / (double)g->n;
    if (!std::isfinite(s->Kn)) return set_error(CIA_EINVAL, "coupling.K is not finite");
    if (c->model == CIA_MODEL_TRIADIC) {
        const cia_hypergraph *h = c->hyper;
        if (!h) return set_error(CIA_EINVAL, "triadic model: coupling.hyper is NULL");
        if (!(h->p_intra >= 0.0 && h->p_intra <= 1.0)) return set_error(CIA_EINVAL, "hypergraph: p_intra outside [0,1]");
        if (h->ntri < 0) return set_error(CIA_EINVAL, "hypergraph: ntri < 0");
        if (g->n >= (int64_t(1) << 21)) return set_error(CIA_EUNSUPPORTED, "triadic model: n must be below 2^21");
        if (g->kind != CIA_GRAPH_CSR) return set_error(CIA_EUNSUPPORTED, "triadic model: the pairwise graph must be CSR");
        if (!std::isfinite(c->K2)) return set_error(CIA_EINVAL, "coupling.K2 is not finite");
        s->tri = true;
        s->K2n = c->K2 / ((double)g->n * (double)g->n);
        s->tri_seed = h->seed;
        s->tri_thr = triple_threshold(h->p_intra);
        // pairwise part h = sin, evaluated with order-2 observables (S1, S2)
        s->P = 2;
        for (int k = 0; k <= PMAX; k++) s->dsin[k] = s->dcos[k] = 0.0;
        s->dsin[1] = 1.0;
        s->d0 = s->hzero = 0.0;
    }
    if (o->block != 0 && o->block != 256 && o->block != 512)
        return set_error(CIA_EINVAL, "options.block = %d; use 0, 256 or 512", o->block);
    s->block = o->block == 512 ? 512 : 256;
    if (omega)
        for (int64_t i = 0; i < g->n; i++)
            if (!std::isfinite(omega[i])) return set_error(CIA_EINVAL, "omega[%lld] is not finite", (long long)i);
    const bool validate = (o->flags & CIA_FLAG_NO_VALIDATE) == 0;
    const bool keep = (o->flags & CIA_FLAG_KEEP_LABELS) != 0;
    const int64_t n = g->n;
    const size_t rs = f64 ? sizeof(double) : sizeof(float);
    // bytes per staged value: z for the phase models, x for the polynomial one
    const int64_t zbytes = s->poly ? (int64_t)rs * s->pdim : (f64 ? 16 : 8);

    // LDS staging capacity (community z values, plus one zero slot); uint16
    // local indices also bound it (the padding index lambda must fit)
    int64_t cap = (int64_t)LDS_BYTES / zbytes - 1;
    if (s->direct || (o->flags & (CIA_FLAG_NO_LDS | CIA_FLAG_FORCE_NEG32))) cap = 0;
    cap = std::min<int64_t>(cap, 65535);

    P1 p1;
    Sell sell;
    std::vector<int32_t> cnt_old;
    std::vector<char> comm_staged;
    int64_t nnz_neg = 0, nnz_pos = 0, nnz_neg_staged = 0, nnz_tri = 0;
    try {
        std::vector<int64_t> xptr;
        std::vector<int32_t> xval;
        if (!s->direct) {
            // triadic hyperedges are defined on the given communities: keep them all
            if (pre) p1 = std::move(*pre);   // batched ensembles: P1 of every instance, joined
            else CIA_TRY(p1_build(g, labels, o->dense_alpha, keep || s->tri, validate, true, p1));
            nnz_neg = (int64_t)p1.neg_local.size();
            nnz_pos = (int64_t)p1.pos.size();
            comm_staged.assign(p1.ncomm, 0);
            for (int32_t cc = 0; cc < p1.ncomm; cc++) {
                int64_t lam = p1.comm_off[cc + 1] - p1.comm_off[cc];
                bool wide = (double)lam > WIDE_COMMUNITY || (o->flags & CIA_FLAG_FORCE_WIDE);
                if (s->tri && wide) return set_error(CIA_EUNSUPPORTED, "triadic model: community above 1e5 nodes");
                // above the LDS cap, FP32 phase plans (difference coupling) stage
                // the community's z tile by tile; other plans gather int32 positions
                const bool tile_ok = !f64 && !s->poly && !s->tri && !gen && cap > 0;
                comm_staged[cc] = wide ? 0 : (lam <= cap ? SEG_STAGED : (tile_ok ? SEG_TILED : 0));
                if (comm_staged[cc]) nnz_neg_staged += p1.negptr[p1.comm_off[cc + 1]] - p1.negptr[p1.comm_off[cc]];
            }
            StreamIn S[4];
            S[0].ptr = &p1.negptr;
            S[0].val = p1.neg_local.data();
            S[0].mut = p1.neg_local.data();
            S[0].local = true;
            S[1].ptr = &p1.posptr;
            S[1].val = p1.pos.data();
            if (s->tri) {
                CIA_TRY(triadic_cross_lists(p1, c->hyper, xptr, xval));
                S[3].ptr = &xptr;
                S[3].val = xval.data();
                S[3].pair = true;
            }
            // merged S-pos slices: FP32, p = 1, and not for single networks small
            // enough for the resident integrator, whose kernel reads one row per lane
            const bool merge_pos = !f64 && !s->poly && !s->tri && !gen && s->P == 1 &&
                                   (pre || (o->flags & CIA_FLAG_NO_RESIDENT) || nnz_neg + nnz_pos > RES_MAX_REMAINDER);
            CIA_TRY(build_sell(n, p1.comm_off, p1.ncomm, comm_staged, S, (uint32_t)zbytes, sell, cap, merge_pos));
            s->tile_cap = (int32_t)cap;
            if (s->d0 != 0.0) {
                // |S+| - |S-| per row (all zero for a complete graph)
                cnt_old.resize(n);
                for (int64_t i = 0; i < n; i++)
                    cnt_old[i] = (int32_t)((p1.posptr[i + 1] - p1.posptr[i]) - (p1.negptr[i + 1] - p1.negptr[i]));
            }
            std::vector<int32_t>().swap(p1.neg_local);
            std::vector<int32_t>().swap(p1.pos);
        } else {
            // direct method: community order for locality, no remainder split;
            // every node is "outside" and its whole row is the +1 list
            if (!pre) CIA_TRY(p1_build(g, labels, o->dense_alpha, true, validate, false, p1));
            if (g->kind == CIA_GRAPH_COMPLETE) {
                s->complete_direct = true;
            } else {
                std::vector<int64_t> arp;
                std::vector<int32_t> acol;
                if (pre) {
                    // batched ensembles: the joined permuted adjacency is the +1 list
                    p1 = std::move(*pre);
                    arp.swap(p1.posptr);
                    acol.swap(p1.pos);
                } else {
                    CIA_TRY(p1_permuted_adjacency(g, p1, arp, acol));
                }
                nnz_pos = arp[n];
                // rows sorted by degree inside each community segment
                StreamIn S[4];
                S[1].ptr = &arp;
                S[1].val = acol.data();
                if (s->tri) {
                    CIA_TRY(triadic_cross_lists(p1, c->hyper, xptr, xval));
                    S[3].ptr = &xptr;
                    S[3].val = xval.data();
                    S[3].pair = true;
                }
                std::vector<char> none(p1.ncomm, 0);
                CIA_TRY(build_sell(n, p1.comm_off, p1.ncomm, none, S, (uint32_t)zbytes, sell));
                if (s->d0 != 0.0) {
                    cnt_old.resize(n);
                    for (int64_t i = 0; i < n; i++) cnt_old[i] = (int32_t)(arp[i + 1] - arp[i]);
                }
            }
        }
    } catch (const std::bad_alloc &) {
        return set_error(CIA_ENOMEM, "host allocation failed");
    }

    // final node order: P1 permutation refined by the in-community sort
    std::vector<int32_t> perm2(n);
    if (!s->complete_direct) {
        for (int64_t i = 0; i < n; i++) perm2[sell.newpos[i]] = p1.perm[i];
    } else {
        for (int64_t i = 0; i < n; i++) perm2[i] = p1.perm[i];
    }
    std::vector<int32_t> cnt;
    if (!cnt_old.empty()) {
        cnt.resize(n);
        for (int64_t i = 0; i < n; i++) cnt[sell.newpos[i]] = cnt_old[i];
    }

    int64_t maxlam = 0, maxstaged = 0;
    for (int32_t cc = 0; cc < p1.ncomm; cc++) {
        int64_t lam = p1.comm_off[cc + 1] - p1.comm_off[cc];
        maxlam = std::max<int64_t>(maxlam, lam);
        if (!s->direct && comm_staged[cc] == SEG_STAGED) maxstaged = std::max<int64_t>(maxstaged, lam);
        if (!s->direct && comm_staged[cc] == SEG_TILED) {
            int64_t nt, ts;
            tile_shape(lam, cap, nt, ts);
            maxstaged = std::max<int64_t>(maxstaged, ts);
        }
    }
    s->lds_cap = (int)maxstaged;

    // work units
    std::vector<Unit> units;
    int32_t nslots = 0;
    if (!s->complete_direct) {
        const int32_t nc = s->direct ? 0 : p1.ncomm;
        s->unit_work = o->unit_work > 0 ? o->unit_work : 32768;
        s->h_slices = sell.slices;
        for (const Slice &Sl : sell.slices)
            if (Sl.sflags & SF_MERGED) s->merged = true;
        s->h_flags = o->flags;
        s->h_staged = comm_staged;
        if (s->direct) {
            // the direct path has one segment per community too; treat all as outside rows
            s->h_seg_off = {0, (int32_t)sell.slices.size()};
            s->h_comm_off = {0};
            s->h_ncomm = 0;
        } else {
            s->h_seg_off = sell.seg_slice_off;
            s->h_comm_off = p1.comm_off;
            s->h_ncomm = nc;
        }
        Sell view;
        view.slices = s->h_slices;
        view.seg_slice_off = s->h_seg_off;
        nslots = make_units(view, s->h_comm_off, s->h_ncomm, s->unit_work, 4, s->h_staged, s->h_flags, units,
                            tiled_slices(s->P, s->block));
        CIA_TRY(check_tiled_units(units, s->P, s->block));
        s->ncomm = nc;
    }
    if (f64)
        for (Unit &u : units) u.flags &= ~UF_WIDE;   // FP64 plans compute everything in FP64
    if (s->poly)
        for (Unit &u : units) u.flags &= ~UF_WIDE;   // the polynomial moments are FP64 throughout
    for (const Unit &u : units)
        if (u.flags & (UF_WIDE | UF_TILED)) s->has_wide = true;
    s->nunits = (int32_t)units.size();
    s->smem = (size_t)zbytes * (s->lds_cap + 1);
    if (s->smem > LDS_BYTES) return set_error(CIA_EUNSUPPORTED, "LDS request too large");

    // info
    cia_plan_info &inf = p->info;
    inf.n = n;
    inf.nnz_graph = p1.nnz_graph;
    inf.nnz_neg = nnz_neg;
    inf.nnz_pos = nnz_pos;
    inf.n_unassigned = s->direct ? n : n - (p1.ncomm ? p1.comm_off[p1.ncomm] : 0);
    inf.ncomm = s->direct ? 0 : p1.ncomm;
    inf.nunits = s->nunits;
    inf.max_comm = (int32_t)maxlam;
    int wide = 0;
    for (int32_t cc = 0; cc < p1.ncomm; cc++)
        if ((double)(p1.comm_off[cc + 1] - p1.comm_off[cc]) > WIDE_COMMUNITY) wide++;
    inf.wide_comms = s->direct ? 0 : wide;
    int tiledc = 0;
    for (int32_t cc = 0; cc < p1.ncomm; cc++)
        if (!s->direct && comm_staged[cc] == SEG_TILED) tiledc++;
    inf.tiled_comms = tiledc;
    inf.merged_slices = 0;
    for (const Slice &Sl : s->h_slices)
        if (Sl.sflags & SF_MERGED) inf.merged_slices++;
    inf.method = o->method;
    inf.precision = o->precision;
    inf.model = s->tri ? CIA_MODEL_TRIADIC : (s->poly ? CIA_MODEL_POLY : CIA_MODEL_PHASE);
    inf.p = s->P;
    inf.nnz_extra = nnz_tri;
    {
        // Algorithmic bytes (no padding).  Per node and RHS: theta in, omega,
        // H out, its z written once and read once; per remainder entry its
        // index (2 B local for LDS-staged communities, else 4 B).  The fused
        // RK stage replaces "theta in / H out" by theta_n in plus acc in and
        // out.
        double idx = 2.0 * (double)nnz_neg_staged + 4.0 * (double)(nnz_neg - nnz_neg_staged) + 4.0 * (double)nnz_pos;
        double zb = s->poly ? (double)rs : 2.0 * rs;   // staged and gathered value: z, or x
        if (s->poly && s->pdim == 2) {
            // two components: every per-node stream and every gathered value doubles
            // (omega, counts and indices do not)
            inf.bytes_per_rhs = 2.0 * (2.0 * rs + 2.0 * zb) * (double)n + rs * (double)n + idx;
            inf.bytes_per_stage = 2.0 * (3.0 * rs + 2.0 * zb) * (double)n + rs * (double)n + idx;
        } else {
            inf.bytes_per_rhs = (3.0 * rs + 2.0 * zb) * (double)n + idx;
            inf.bytes_per_stage = (4.0 * rs + 2.0 * zb) * (double)n + idx;
        }
        if (s->complete_direct) inf.bytes_per_rhs = inf.bytes_per_stage = (double)n * (2 * zb + 2 * rs);
    }

    // ---- device upload ----
    CIA_TRY(dupload(p, &s->perm, perm2.data(), n));
    if (!s->complete_direct) {
        if (units.empty()) units.push_back(Unit{0, 0, 0, 0, 0, 0, 0, 0});
        CIA_TRY(dupload(p, &s->units, units.data(), units.size()));
        s->units_cap = units.size();
        if (sell.slices.empty()) sell.slices.push_back(Slice{});
        CIA_TRY(dupload(p, &s->slices, sell.slices.data(), sell.slices.size()));
        CIA_TRY(dupload(p, &s->negdata, sell.data[0].data(), sell.data[0].size()));
        CIA_TRY(dupload(p, &s->posdata, sell.data[1].data(), sell.data[1].size()));
        CIA_TRY(dupload(p, &s->tposdata, sell.data[3].data(), sell.data[3].size()));
        if (sell.tile_w.empty()) sell.tile_w.push_back(0);
        CIA_TRY(dupload(p, &s->tile_w, sell.tile_w.data(), sell.tile_w.size()));
        // the kernels read cnt[i] only when d_0 != 0, and then it holds n entries
        if (s->d0 != 0.0 && (int64_t)cnt.size() != n)
            return set_error(CIA_EINVAL, "internal: row counts missing for d_0 != 0");
        if (!cnt.empty()) CIA_TRY(dupload(p, &s->cnt, cnt.data(), cnt.size()));
        else CIA_TRY(dalloc(p, &s->cnt, 1));
    }
    for (int q = 0; q < 4; q++) std::vector<uint4>().swap(sell.data[q]);
    // omega in community order
    if (omega) {
        if (f64) {
            std::vector<double> om(n);
            for (int64_t i = 0; i < n; i++) om[i] = omega[perm2[i]];
            double *d;
            CIA_TRY(dupload(p, &d, om.data(), n));
            s->omega = d;
        } else {
            std::vector<float> om(n);
            for (int64_t i = 0; i < n; i++) om[i] = (float)omega[perm2[i]];
            float *d;
            CIA_TRY(dupload(p, &d, om.data(), n));
            s->omega = d;
        }
    }
    unsigned char *raw;
    const int64_t nd = s->pdim;   // state components per node
    CIA_TRY(dalloc(p, &raw, rs * n * nd));
    s->theta_n = raw;
    CIA_TRY(dalloc(p, &raw, rs * n * nd));
    s->acc = raw;
    for (int b = 0; b < 2; b++) {
        // z arrays carry one extra zero slot at position n (the padding target)
        CIA_TRY(dalloc(p, &raw, 2 * rs * (n + 1)));
        CIA_HIP(hipMemset(raw + 2 * rs * n, 0, 2 * rs));
        s->cs[b] = raw;
        // stage theta (random S-pos gathers and the FP64 path): nd values per
        // node, node-major, and a zero entry at node n
        CIA_TRY(dalloc(p, &raw, rs * (n + 1) * nd));
        CIA_HIP(hipMemset(raw + rs * n * nd, 0, rs * nd));
        s->th[b] = raw;
        CIA_TRY(dalloc(p, &s->q[b], (size_t)std::max(1, nslots) * s->P));
    }
    s->q_cap = (size_t)std::max(1, nslots) * s->P;
    CIA_TRY(dalloc(p, &s->r_part, (size_t)std::max(1, s->nunits) + 1024));
    s->rpart_cap = (size_t)std::max(1, s->nunits) + 1024;
    if (bs) {
        // instance of every position, positions grouped by instance, K_b / N_b
        s->batch = bs->count;
        std::vector<int64_t> goff(bs->count + 1, 0);
        std::vector<int32_t> inst(n), gidx(n);
        for (int64_t i = 0; i < n; i++) {
            const int64_t u = perm2[i];
            inst[i] = (int32_t)(std::upper_bound(bs->offsets, bs->offsets + bs->count + 1, u) - bs->offsets - 1);
            goff[inst[i] + 1]++;
        }
        for (int32_t b = 0; b < bs->count; b++) goff[b + 1] += goff[b];
        std::vector<int64_t> fill(goff.begin(), goff.end() - 1);
        for (int64_t i = 0; i < n; i++) gidx[fill[inst[i]]++] = (int32_t)i;
        CIA_TRY(dupload(p, &s->grp_idx, gidx.data(), n));
        CIA_TRY(dupload(p, &s->grp_off, goff.data(), goff.size()));
        if (f64) {
            std::vector<double> k(n);
            for (int64_t i = 0; i < n; i++) k[i] = bs->kn[perm2[i]];
            double *d;
            CIA_TRY(dupload(p, &d, k.data(), n));
            s->kn = d;
        } else {
            std::vector<float> k(n);
            for (int64_t i = 0; i < n; i++) k[i] = (float)bs->kn[perm2[i]];
            float *d;
            CIA_TRY(dupload(p, &d, k.data(), n));
            s->kn = d;
        }
    }
    if (s->tri && s->direct) {
        // present-pair enumeration blocks: up to TRI_ROWS centres of one community each
        int32_t maxl = 0;
        std::vector<TriBlock> tb = tri_blocks(p1.comm_off, p1.ncomm, maxl);
        s->tri_smem = (size_t)maxl * (2 * rs + 4);
        if (s->tri_smem > LDS_BYTES)
            return set_error(CIA_EUNSUPPORTED, "direct triadic: community of %d nodes does not fit in LDS", maxl);
        s->ntri_blocks = (int32_t)tb.size();
        if (tb.empty()) tb.push_back(TriBlock{0, 0, 0, 0});
        CIA_TRY(dupload(p, &s->tri_blocks, tb.data(), tb.size()));
        CIA_TRY(dalloc(p, &raw, 2 * rs * n));
        CIA_HIP(hipMemset(raw, 0, 2 * rs * n));
        s->h_extra = raw;
    }
    if (s->tri && !s->direct) {
        int64_t npairs = 0, nchunks = 0;
        CIA_TRY(tri_build_missing(p, s, p1.comm_off, p1.ncomm, n, (uint32_t)zbytes, npairs, nchunks));
        inf.nnz_extra = npairs;
        // per stage: the pair-sum launch reads every chunk once and writes one
        // sum per community row, which the stage launch reads
        const double rows = (double)(p1.ncomm ? p1.comm_off[p1.ncomm] : 0);
        inf.bytes_aux = 16.0 * (double)nchunks + (double)zbytes * rows;
        inf.bytes_per_stage += (double)zbytes * rows;
        inf.bytes_per_rhs += inf.bytes_aux + (double)zbytes * rows;
    }
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
    CIA_TRY(resident_setup(p, s, o));
    // device address of this GPU's scratch array for the allocation-free
    // entry point, resolved at set-up with the plan's device current
    double *scr = nullptr;
    CIA_TRY(noalloc_scratch(p->device, &scr));
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
static PhaseArgs<R> base_args(cia_plan *p, PhaseState *s) {
    PhaseArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.units = s->units;
    a.slices = s->slices;
    a.negdata = s->negdata;
    a.posdata = s->posdata;
    a.tri_m = s->tri_m;
    a.tposdata = s->tposdata;
    a.h_extra = static_cast<const cx<R> *>(s->h_extra);
    a.K2n = (R)s->K2n;
    for (int k = 0; k <= PMAX; k++) {
        a.ph[k] = s->ph[k];
        a.pf[k] = s->pf[k];
    }
    a.pq = s->pq;
    for (int k = 0; k < 32; k++) a.pf2[k] = s->pf2[k];
    a.gen = static_cast<const R *>(s->gen);
    a.pgen = s->pgen;
    a.cnt = s->cnt;
    a.perm = s->perm;
    a.omega = static_cast<const R *>(s->omega);
    a.kn = static_cast<const R *>(s->kn);
    a.invN = 1.0 / (double)p->n;
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
    a.tile_w = s->tile_w;
    a.tile_cap = s->tile_cap;
    a.pad_pos = (uint32_t)p->n;
    return a;
}

template <typename R, int P, int BLOCK>
static void launch_stage_v(PhaseState *s, const PhaseArgs<R> &a, hipStream_t st) {
    const dim3 g(s->nunits), b(BLOCK);
    if (s->poly) {
        if (s->pdim == 2) {
            if (s->direct) hipLaunchKernelGGL((poly_stage_kernel<R, P, BLOCK, true, 2>), g, b, s->smem, st, a);
            else hipLaunchKernelGGL((poly_stage_kernel<R, P, BLOCK, false, 2>), g, b, s->smem, st, a);
        } else {
            if (s->direct) hipLaunchKernelGGL((poly_stage_kernel<R, P, BLOCK, true, 1>), g, b, s->smem, st, a);
            else hipLaunchKernelGGL((poly_stage_kernel<R, P, BLOCK, false, 1>), g, b, s->smem, st, a);
        }
        return;
    }
    if (s->tri) {
        if constexpr (P == 2) {
            if (s->direct) hipLaunchKernelGGL((phase_stage_kernel<R, 2, BLOCK, true, false, true>), g, b, s->smem, st, a);
            else hipLaunchKernelGGL((phase_stage_kernel<R, 2, BLOCK, false, false, true>), g, b, s->smem, st, a);
        }
        return;
    }
    if constexpr (P <= GEN_PMAX) {
      if (s->gen) {
        // general (non-difference) coupling: its own instantiations, so the
        // difference form keeps its register budget
        if (s->direct)
            hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, true, false, false, true>), g, b, s->smem, st, a);
        else if (sizeof(R) == 4 && s->has_wide)
            hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, false, true, false, true>), g, b, s->smem, st, a);
        else
            hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, false, false, false, true>), g, b, s->smem, st, a);
        return;
      }
    }
    if constexpr (sizeof(R) == 4 && P == 1) {
        if (s->merged) {
            // plans with merged S-pos slices (built for FP32, P = 1 only)
            if (s->has_wide)
                hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, false, true, false, false, true>), g, b, s->smem, st,
                                   a);
            else
                hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, false, false, false, false, true>), g, b, s->smem,
                                   st, a);
            return;
        }
    }
    if (s->direct)
        hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, true, false, false>), g, b, s->smem, st, a);
    else if (sizeof(R) == 4 && s->has_wide)
        hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, false, true, false>), g, b, s->smem, st, a);
    else
        hipLaunchKernelGGL((phase_stage_kernel<R, P, BLOCK, false, false, false>), g, b, s->smem, st, a);
}

template <typename R, int BLOCK>
static void launch_stage_v_any(PhaseState *s, const PhaseArgs<R> &a, hipStream_t st) {
    switch (s->P) {
        case 1: launch_stage_v<R, 1, BLOCK>(s, a, st); break;
        case 2: launch_stage_v<R, 2, BLOCK>(s, a, st); break;
        case 3: launch_stage_v<R, 3, BLOCK>(s, a, st); break;
        case 4: launch_stage_v<R, 4, BLOCK>(s, a, st); break;
        case 5: launch_stage_v<R, 5, BLOCK>(s, a, st); break;
        case 6: launch_stage_v<R, 6, BLOCK>(s, a, st); break;
        case 7: launch_stage_v<R, 7, BLOCK>(s, a, st); break;
        default: launch_stage_v<R, 8, BLOCK>(s, a, st); break;
    }
}

// The triadic model's launch before each gathering stage: the pair sums
// its stage reads (CIA: missing intra pairs; direct: present intra pairs).
template <typename R>
static bool has_tri_aux(const PhaseState *s, const PhaseArgs<R> &a) {
    return s->tri && a.mode != M_PREP && (s->direct ? s->ntri_blocks : s->tri_nunits) > 0;
}
template <typename R>
static void launch_tri_aux(PhaseState *s, const PhaseArgs<R> &a, hipStream_t st) {
    if (!has_tri_aux<R>(s, a)) return;
    if (s->direct)
        hipLaunchKernelGGL((triadic_present_kernel<R>), dim3(s->ntri_blocks), dim3(256), s->tri_smem, st,
                           s->tri_blocks, s->perm, a.cs_in, (uint64_t)s->tri_seed, (uint64_t)s->tri_thr,
                           static_cast<cx<R> *>(s->h_extra));
    else
        hipLaunchKernelGGL((tri_missing_kernel<R>), dim3(s->tri_nunits), dim3(256), s->tri_msmem, st, s->tri_units,
                           a.cs_in, s->tri_cptr, s->tri_chunks, static_cast<cx<R> *>(s->tri_m));
}

template <typename R, int P>
static cia_status launch_stage_p(cia_plan *p, PhaseState *s, const PhaseArgs<R> &a, hipStream_t st, int kind) {
    if (s->nunits == 0) return CIA_OK;
    if (has_tri_aux<R>(s, a)) {
        CIA_TRY(timing_begin(p, st, KK_AUX));
        launch_tri_aux<R>(s, a, st);
        CIA_HIP(hipGetLastError());
        CIA_TRY(timing_end(p, st));
    }
    CIA_TRY(timing_begin(p, st, kind));
    if (s->block == 512) launch_stage_v<R, P, 512>(s, a, st);
    else launch_stage_v<R, P, 256>(s, a, st);
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
    hipLaunchKernelGGL(order_reduce_kernel, dim3(1), dim3(64), 0, st, s->r_part, nparts,
                       1.0 / (double)p->n, slot, (const int64_t *)nullptr);
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
    PhaseArgs<R> a = base_args<R>(p, s);
    a.mode = M_PREP;
    a.state_in = static_cast<const R *>(state);
    a.cs_out = static_cast<cx<R> *>(s->cs[0]);
    a.q_out = s->q[0];
    a.th_out = static_cast<R *>(s->th[0]);
    a.r_part = s->r_part;
    CIA_TRY(launch_stage<R>(p, s, a, st, KK_PREP));
    a = base_args<R>(p, s);
    a.mode = M_RHS;
    a.cs_in = static_cast<const cx<R> *>(s->cs[0]);
    a.q_in = s->q[0];
    a.th_in = static_cast<const R *>(s->th[0]);
    a.state_out = static_cast<R *>(dstate);
    return launch_stage<R>(p, s, a, st, KK_STAGE);
}

// r(t) of the current z: the global order parameter from the unit partials,
// or per instance for batched ensembles.  slot: index in the trace; ctr:
// slot counter of replayed graphs (then `slot` is the base).
template <typename R>
static cia_status launch_order(cia_plan *p, PhaseState *s, hipStream_t st, double *rb, const void *cs, int64_t slot,
                               int64_t stride, const int64_t *ctr, bool timed) {
    if (timed) CIA_TRY(timing_begin(p, st, KK_AUX));
    if (s->batch > 0) {
        hipLaunchKernelGGL((order_grouped_kernel<R>), dim3(s->batch), dim3(256), 0, st,
                           static_cast<const cx<R> *>(cs), s->grp_idx, s->grp_off, rb, stride, slot, ctr);
    } else {
        hipLaunchKernelGGL(order_reduce_kernel, dim3(1), dim3(64), 0, st, s->r_part, s->nunits,
                           1.0 / (double)p->n, rb + slot, ctr);
    }
    CIA_HIP(hipGetLastError());
    return timed ? timing_end(p, st) : CIA_OK;
}

template <typename R>
static PhaseArgs<R> stage_args(cia_plan *p, PhaseState *s, bool rk4, int q, double dt, int cur, bool want_r) {
    PhaseArgs<R> a = base_args<R>(p, s);
    a.mode = rk4 ? M_RK4 : M_EULER;
    a.stage = q;
    a.dt = (R)dt;
    a.cs_in = static_cast<const cx<R> *>(s->cs[cur]);
    a.cs_out = static_cast<cx<R> *>(s->cs[cur ^ 1]);
    a.q_in = s->q[cur];
    a.q_out = s->q[cur ^ 1];
    a.th_in = static_cast<const R *>(s->th[cur]);
    a.th_out = static_cast<R *>(s->th[cur ^ 1]);
    a.r_part = s->r_part;
    a.want_r = want_r;
    return a;
}

// single networks, RK4: the first stage of a step sums the order-parameter
// partials that the previous launch (prep pass or last stage) left, into
// `slot` (+ *ctr)
template <typename R>
static void fold_order(PhaseState *s, PhaseArgs<R> &a, double *slot, const int64_t *ctr) {
    a.r_prev_part = s->r_part;
    a.r_prev_out = slot;
    a.r_prev_slot = ctr;
    a.r_prev_n = s->nunits;
}

template <typename R>
static cia_status integrate_impl(cia_plan *p, PhaseState *s, void *state, double dt, int64_t steps,
                                 double *r_trace, hipStream_t st, double *r_ext = nullptr) {
    const int64_t n = p->n;
    const bool want_r = r_trace != nullptr;
    const int64_t nr = s->batch > 0 ? s->batch : 1;   // traces
    const int64_t stride = steps + 1;
    if (want_r && !r_ext && s->r_cap < nr * stride) {
        // at least 4096 slots per trace, and at least double the old size, so
        // calls of up to 4095 steps never reallocate after the first one
        const int64_t cap = std::max(nr * stride, std::max(2 * s->r_cap, nr * (int64_t)4096));
        if (s->r_dev) {
            CIA_HIP(hipFree(s->r_dev));
            for (auto &q : p->dev_allocs)
                if (q == s->r_dev) q = nullptr;
            s->r_dev = nullptr;
        }
        CIA_TRY(dalloc(p, &s->r_dev, (size_t)cap));
        s->r_cap = cap;
    }
    // device trace of r(t): the plan's own buffer, or the caller-provided one
    // of the allocation-free entry point
    double *const rb = r_ext ? r_ext : s->r_dev;
    if (s->resident && (p->stepper == CIA_RK4 || p->stepper == CIA_EULER)) {
        ResArgs<R> ra{};
        ra.slices = s->slices;
        ra.negdata = s->negdata;
        ra.posdata = s->posdata;
        ra.slice_comm = s->res_slice_comm;
        ra.slice_flags = s->res_slice_flags;
        ra.comm_off = s->res_comm_off;
        ra.comm_slice0 = s->res_comm_slice0;
        ra.cnt = s->cnt;
        ra.perm = s->perm;
        ra.omega = static_cast<const R *>(s->omega);
        ra.state_in = static_cast<const R *>(state);
        ra.state_out = static_cast<R *>(state);
        ra.r_out = want_r ? rb : nullptr;
        ra.n = (int32_t)n;
        ra.nslices = s->nslices;
        ra.ncomm = s->h_ncomm;
        ra.mode = p->stepper == CIA_RK4 ? M_RK4 : M_EULER;
        ra.steps = steps;
        ra.dt = (R)dt;
        ra.Kn = (R)s->Kn;
        ra.d0 = (R)s->d0;
        ra.hzero = (R)s->hzero;
        for (int k = 0; k <= PMAX; k++) {
            ra.dsin[k] = (R)s->dsin[k];
            ra.dcos[k] = (R)s->dcos[k];
        }
        CIA_TRY(timing_begin(p, st, KK_STAGE, (int)std::min<int64_t>(INT32_MAX, std::max<int64_t>(1, steps * (p->stepper == CIA_RK4 ? 4 : 1)))));
        switch (s->P) {
            case 1: hipLaunchKernelGGL((resident_integrate_kernel<R, 1>), dim3(1), dim3(res_block<R>()), s->res_smem, st, ra); break;
            case 2: hipLaunchKernelGGL((resident_integrate_kernel<R, 2>), dim3(1), dim3(res_block<R>()), s->res_smem, st, ra); break;
            case 3: hipLaunchKernelGGL((resident_integrate_kernel<R, 3>), dim3(1), dim3(res_block<R>()), s->res_smem, st, ra); break;
            default: hipLaunchKernelGGL((resident_integrate_kernel<R, 4>), dim3(1), dim3(res_block<R>()), s->res_smem, st, ra); break;
        }
        CIA_HIP(hipGetLastError());
        CIA_TRY(timing_end(p, st));
        if (want_r) {
            CIA_HIP(hipMemcpyAsync(r_trace, rb, sizeof(double) * (steps + 1), hipMemcpyDeviceToHost, st));
            CIA_HIP(hipStreamSynchronize(st));
            for (int64_t k = 0; k <= steps; k++)
                if (!std::isfinite(r_trace[k]))
                    return set_error(CIA_ENONFINITE, "state became non-finite (r(t_%lld) = %g)", (long long)k,
                                     r_trace[k]);
        }
        return CIA_OK;
    }
    const bool rk4 = p->stepper == CIA_RK4;
    const int64_t grid = (n + 255) / 256;
    int cur = 0;
    // the unit partials of r are produced by the stage kernel for single
    // networks; ensembles reduce per instance from z instead
    const bool part_r = want_r && s->batch == 0;
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
            CIA_TRY(launch_order_reduce(p, s, st, np, rb));
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
                CIA_TRY(launch_order_reduce(p, s, st, np, rb + k + 1));
            }
        }
    } else {
        // (the direct triadic path launches an extra kernel per stage: no graph)
        // (the allocation-free entry point never builds a graph: its set-up allocates)
        const bool replay = (p->flags & CIA_FLAG_HIPGRAPH) && rk4 && steps > 0 && !(s->tri && s->direct) && !r_ext;
        hipStream_t ws = st;   // stream the steps run on
        if (replay) {
            if (!s->gstream) {
                CIA_HIP(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));
                CIA_HIP(hipEventCreateWithFlags(&s->gev[0], hipEventDisableTiming));
                CIA_HIP(hipEventCreateWithFlags(&s->gev[1], hipEventDisableTiming));
                CIA_TRY(dalloc(p, &s->r_ctr, 1));
            }
            CIA_HIP(hipEventRecord(s->gev[0], st));
            CIA_HIP(hipStreamWaitEvent(s->gstream, s->gev[0], 0));
            ws = s->gstream;
        }
        PhaseArgs<R> a = base_args<R>(p, s);
        a.mode = M_PREP;
        a.state_in = static_cast<const R *>(state);
        a.cs_out = static_cast<cx<R> *>(s->cs[0]);
        a.q_out = s->q[0];
        a.th_out = static_cast<R *>(s->th[0]);
        a.r_part = s->r_part;
        a.want_r = part_r;
        CIA_TRY(launch_stage<R>(p, s, a, ws, KK_PREP));
        // r(t_0): with RK4 on single networks it is folded into the first
        // stage of the first step (or reduced below when steps == 0)
        const bool fold = part_r && rk4;
        if (want_r && !fold) CIA_TRY(launch_order<R>(p, s, ws, rb, s->cs[0], 0, stride, nullptr, true));
        if (replay) {
            // one RK4 step (four stage launches, r(t) and its slot counter) as a
            // graph, instantiated once per (dt, trace) and replayed every step
            if (!s->gexec || s->g_dt != dt || s->g_want_r != want_r || s->g_r != s->r_dev ||
                s->g_stride != stride) {
                if (s->gexec) CIA_HIP(hipGraphExecDestroy(s->gexec));
                if (s->graph) CIA_HIP(hipGraphDestroy(s->graph));
                s->gexec = nullptr;
                s->graph = nullptr;
                CIA_HIP(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
                for (int q = 0; q < 4; q++) {
                    PhaseArgs<R> b = stage_args<R>(p, s, true, q, dt, q & 1, part_r && q == 3);
                    if (fold && q == 0) fold_order<R>(s, b, rb, s->r_ctr);
                    if (s->nunits > 0) launch_tri_aux<R>(s, b, ws);
                    if (s->block == 512) launch_stage_v_any<R, 512>(s, b, ws);
                    else launch_stage_v_any<R, 256>(s, b, ws);
                }
                if (want_r) {
                    if (!fold) CIA_TRY(launch_order<R>(p, s, ws, rb, s->cs[0], 1, stride, s->r_ctr, false));
                    hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, ws, s->r_ctr, (int64_t)1, 1);
                }
                hipGraph_t gr = nullptr;
                const hipError_t ec = hipStreamEndCapture(ws, &gr);
                if (ec != hipSuccess) return set_error(CIA_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
                s->graph = gr;
                CIA_HIP(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
                s->g_dt = dt;
                s->g_stride = stride;
                s->g_want_r = want_r;
                s->g_r = s->r_dev;
            }
            if (want_r) hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, ws, s->r_ctr, (int64_t)0, 0);
            CIA_HIP(hipGetLastError());
            for (int64_t k = 0; k < steps; k++) {
                CIA_TRY(timing_begin(p, ws, KK_STAGE, 4));
                CIA_HIP(hipGraphLaunch(s->gexec, ws));
                CIA_TRY(timing_end(p, ws));
            }
        } else {
            for (int64_t k = 0; k < steps; k++) {
                const int nst = rk4 ? 4 : 1;
                for (int q = 0; q < nst; q++) {
                    a = stage_args<R>(p, s, rk4, q, dt, cur, part_r && q == nst - 1);
                    if (fold && q == 0) fold_order<R>(s, a, rb + k, nullptr);
                    CIA_TRY(launch_stage<R>(p, s, a, ws, KK_STAGE));
                    cur ^= 1;
                }
                if (want_r && !fold) CIA_TRY(launch_order<R>(p, s, ws, rb, s->cs[cur], k + 1, stride, nullptr, true));
            }
        }
        // the last step's r(t) (its partials were left by the final stage)
        if (fold) CIA_TRY(launch_order<R>(p, s, ws, rb, nullptr, steps, stride, nullptr, true));
        CIA_TRY(timing_begin(p, ws, KK_AUX));
        for (int d = 0; d < s->pdim; d++)
            hipLaunchKernelGGL((permute_out_kernel<R>), dim3(grid), dim3(256), 0, ws, n, s->perm,
                               static_cast<const R *>(s->theta_n) + d * n, static_cast<R *>(state) + d * n);
        CIA_HIP(hipGetLastError());
        CIA_TRY(timing_end(p, ws));
        if (replay) {
            CIA_HIP(hipEventRecord(s->gev[1], ws));
            CIA_HIP(hipStreamWaitEvent(st, s->gev[1], 0));
        }
        if (want_r) {
            CIA_HIP(hipMemcpyAsync(r_trace, rb, sizeof(double) * nr * stride, hipMemcpyDeviceToHost, st));
            CIA_HIP(hipStreamSynchronize(st));
            for (int64_t k = 0; k < nr * stride; k++)
                if (!std::isfinite(r_trace[k]))
                    return set_error(CIA_ENONFINITE, "state became non-finite (r trace entry %lld = %g)",
                                     (long long)k, r_trace[k]);
        }
        return CIA_OK;
    }
    CIA_TRY(timing_begin(p, st, KK_AUX));
    for (int d = 0; d < s->pdim; d++)
        hipLaunchKernelGGL((permute_out_kernel<R>), dim3(grid), dim3(256), 0, st, n, s->perm,
                           static_cast<const R *>(s->theta_n) + d * n, static_cast<R *>(state) + d * n);
    CIA_HIP(hipGetLastError());
    CIA_TRY(timing_end(p, st));
    if (want_r) {
        CIA_HIP(hipMemcpyAsync(r_trace, rb, sizeof(double) * (steps + 1), hipMemcpyDeviceToHost, st));
        CIA_HIP(hipStreamSynchronize(st));
        for (int64_t k = 0; k <= steps; k++)
            if (!std::isfinite(r_trace[k]))
                return set_error(CIA_ENONFINITE, "state became non-finite (r(t_%lld) = %g)", (long long)k,
                                 r_trace[k]);
    }
    return CIA_OK;
}

// ---------------------------------------------------------------------------
// autotuner: unit size and block size, timed on the plan's own data
// ---------------------------------------------------------------------------

// Make the units for `target` and upload them (growing the unit-dependent
// buffers when needed).
static cia_status apply_units(cia_plan *p, PhaseState *s, int64_t target) {
    Sell view;
    view.slices = s->h_slices;
    view.seg_slice_off = s->h_seg_off;
    std::vector<Unit> units;
    const int32_t nslots = make_units(view, s->h_comm_off, s->h_ncomm, target, 4, s->h_staged, s->h_flags, units,
                                      tiled_slices(s->P, s->block));
    CIA_TRY(check_tiled_units(units, s->P, s->block));
    if (units.empty()) units.push_back(Unit{0, 0, 0, 0, 0, 0, 0, 0});
    if (units.size() > s->units_cap) {
        CIA_TRY(dalloc(p, &s->units, units.size()));
        s->units_cap = units.size();
    }
    CIA_HIP(hipMemcpy(s->units, units.data(), sizeof(Unit) * units.size(), hipMemcpyHostToDevice));
    const size_t qneed = (size_t)std::max(1, nslots) * s->P;
    if (qneed > s->q_cap) {
        for (int b = 0; b < 2; b++) CIA_TRY(dalloc(p, &s->q[b], qneed));
        s->q_cap = qneed;
    }
    if (units.size() + 1024 > s->rpart_cap) {
        CIA_TRY(dalloc(p, &s->r_part, units.size() + 1024));
        s->rpart_cap = units.size() + 1024;
    }
    s->nunits = (int32_t)units.size();
    s->unit_work = target;
    // a captured step graph holds the old launch shape
    if (s->gexec) {
        CIA_HIP(hipGraphExecDestroy(s->gexec));
        s->gexec = nullptr;
    }
    if (s->graph) {
        CIA_HIP(hipGraphDestroy(s->graph));
        s->graph = nullptr;
    }
    return CIA_OK;
}

template <typename R>
static cia_status tune_impl(cia_plan *p, PhaseState *s, hipStream_t st, cia_tune_report *rep) {
    const int64_t n = p->n;
    if (!s->tune_in) {
        unsigned char *raw;
        CIA_TRY(dalloc(p, &raw, sizeof(R) * n * s->pdim));
        CIA_HIP(hipMemset(raw, 0, sizeof(R) * n * s->pdim));
        s->tune_in = raw;
        CIA_TRY(dalloc(p, &raw, sizeof(R) * n * s->pdim));
        s->tune_out = raw;
    }
    hipEvent_t e0, e1;
    CIA_HIP(hipEventCreate(&e0));
    CIA_HIP(hipEventCreate(&e1));
    // time of one RHS launch (median of 5 after 2 warm-up launches); the
    // triadic pair-sum launch does not depend on the units and is not timed
    // (its stale sums only feed the discarded output)
    auto measure = [&](double *us) -> cia_status {
        PhaseArgs<R> a = base_args<R>(p, s);
        a.mode = M_PREP;
        a.state_in = static_cast<const R *>(s->tune_in);
        a.cs_out = static_cast<cx<R> *>(s->cs[0]);
        a.q_out = s->q[0];
        a.th_out = static_cast<R *>(s->th[0]);
        a.r_part = s->r_part;
        if (s->block == 512) launch_stage_v_any<R, 512>(s, a, st);
        else launch_stage_v_any<R, 256>(s, a, st);
        a = base_args<R>(p, s);
        a.mode = M_RHS;
        a.cs_in = static_cast<const cx<R> *>(s->cs[0]);
        a.q_in = s->q[0];
        a.th_in = static_cast<const R *>(s->th[0]);
        a.state_out = static_cast<R *>(s->tune_out);
        std::vector<float> t;
        for (int k = 0; k < 7; k++) {
            CIA_HIP(hipEventRecord(e0, st));
            if (s->block == 512) launch_stage_v_any<R, 512>(s, a, st);
            else launch_stage_v_any<R, 256>(s, a, st);
            CIA_HIP(hipEventRecord(e1, st));
            CIA_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            CIA_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (k >= 2) t.push_back(ms);
        }
        CIA_HIP(hipGetLastError());
        std::sort(t.begin(), t.end());
        *us = 1e3 * t[t.size() / 2];
        return CIA_OK;
    };
    const int64_t def_work = s->unit_work;
    const int def_block = s->block;
    double def_us = 0.0;
    CIA_TRY(measure(&def_us));
    double best_us = def_us;
    int64_t best_work = def_work;
    int best_block = def_block;
    int ncand = 0;
    static const int64_t works[] = {4096, 8192, 16384, 32768, 65536, 131072};
    static const int blocks[] = {256, 512};
    for (int bl : blocks)
        for (int64_t w : works) {
            s->block = bl;
            CIA_TRY(apply_units(p, s, w));
            double us = 0.0;
            CIA_TRY(measure(&us));
            ncand++;
            if (us < best_us) {
                best_us = us;
                best_work = w;
                best_block = bl;
            }
        }
    s->block = best_block;
    CIA_TRY(apply_units(p, s, best_work));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->info.nunits = s->nunits;
    if (rep) {
        rep->unit_work = (int32_t)best_work;
        rep->block = best_block;
        rep->candidates = ncand;
        rep->reserved = 0;
        rep->best_us = best_us;
        rep->default_us = def_us;
    }
    return CIA_OK;
}

cia_status phase_autotune(cia_plan *p, hipStream_t st, cia_tune_report *rep) {
    PhaseState *s = p->phase;
    if (s->complete_direct || s->h_slices.empty())
        return set_error(CIA_EUNSUPPORTED, "nothing to tune on an all-to-all direct plan");
    return s->f64 ? tune_impl<double>(p, s, st, rep) : tune_impl<float>(p, s, st, rep);
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

// ---------------------------------------------------------------------------
// allocation-free integration: the r(t) trace in a static device array
// ---------------------------------------------------------------------------
// One copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (in host code it only names the symbol); it uses
// the device address that hipGetSymbolAddress returns with that GPU current.
static __device__ __align__(256) double scratch[NOALLOC_R_MAX];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};
}  // namespace

// Device address of this GPU's scratch array; the caller has made `dev`
// current.  Resolved once per device (at plan build, or at the first
// allocation-free call on the device).
cia_status noalloc_scratch(int dev, double **out) {
    *out = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(CIA_EUNSUPPORTED, "device %d: above %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) {
            (void)hipGetLastError();
            return set_error(CIA_EHIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
        }
        g_scratch[dev] = static_cast<double *>(q);
    }
    *out = g_scratch[dev];
    return CIA_OK;
}

cia_status phase_integrate_noalloc(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                                   hipStream_t st) {
    PhaseState *s = p->phase;
    const int64_t nr = s->batch > 0 ? s->batch : 1;
    if (r_trace && (steps + 1) > NOALLOC_R_MAX / nr)
        return set_error(CIA_EINVAL, "allocation-free integration: %lld trace values (%lld instances x %lld) exceed "
                         "the %lld-value scratch array", (long long)(nr * (steps + 1)), (long long)nr,
                         (long long)(steps + 1), (long long)NOALLOC_R_MAX);
    double *rb = nullptr;
    CIA_TRY(noalloc_scratch(p->device, &rb));
    // per-launch timing creates events: off for this call
    const int32_t every = p->timing_every;
    p->timing_every = 0;
    const cia_status r = s->f64 ? integrate_impl<double>(p, s, state, dt, steps, r_trace, st, rb)
                                : integrate_impl<float>(p, s, state, dt, steps, r_trace, st, rb);
    p->timing_every = every;
    return r;
}

}  // namespace cia
