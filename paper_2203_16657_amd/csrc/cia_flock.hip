// Cucker-Smale flocking in 3-D (App. A.6) with the community integration
// algorithm: per-community observables of a separable expansion of the
// weight (E1), signed corrections over the sparse remainder S (E2), and an
// exact per-community fallback.
//
//   s_m' = v_m,   v_m' = (1/N) sum_l a_ml w(s_l - s_m) (v_l - v_m),
//   w(y) = K / (sigma^2 + |y|^2)^beta.
//
// Inside a dense community c the weight is replaced by a symmetric separable
// form  wt(a, b) = sum_r sgn_r f_r(a) f_r(b)  so that
//   sum_{l in c} wt(s_l, s_m) (v_l - v_m) = sum_r sgn_r f_r(s_m) (V_cr - v_m P_cr),
//   P_cr = sum_{l in c} f_r(s_l),  V_cr = sum_{l in c} f_r(s_l) v_l           (E1),
// the missing intra pairs S-neg are subtracted with the same wt and the pairs
// S-pos (leaving the community) are added with the exact w (E2, App. A.1).
// The self pair contributes wt (v_m - v_m) = 0.
//
// Feature maps f:
//  * Fourier (eq. Cucker_Smale_etaExpansion): the truncated series on [-L, L]^3
//    in real form, f = {1} u {cos, sin}(pi <alpha, s> / L) over the half set of
//    multi-indices alpha in {-p..p}^3 with alpha > 0 (first nonzero entry
//    positive), sgn = {c_0, 2 c_alpha, 2 c_alpha}.
//  * learned: a 3-64-64-R SiLU perceptron evaluated with bf16 MFMA tiles and
//    FP32 accumulation, trained on intra-community pair samples of the current
//    state (hand-written forward, backward and Adam kernels).  A judge checks
//    each community on sampled members against the exact weight once per
//    step and switches failing communities to the exact fallback.
//  * exact: every community uses the fallback: the all-pairs sum over the
//    community minus S-neg, with the exact weight.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "fastmath.h"
#include "plan.h"
#include "wave.h"

namespace cia {

namespace {

constexpr int HID = 64;            // hidden width of the learned basis
constexpr int TPR = 2;             // threads per row in the stage kernel
constexpr int CHUNK_ROWS = 256;    // rows per chunk of the stage kernel
constexpr int FBLOCK = CHUNK_ROWS * TPR;
constexpr int EXACT_RT = 2;        // lanes per row of flock_exact_kernel
static_assert(TPR == EXACT_RT, "both stage kernels read the same S-neg slices");
constexpr int JUDGE_SAMPLES = 16;  // sampled members per community and step
constexpr int TRAIN_PAIRS = 4096;  // pairs per optimiser step
constexpr int TILE_PTS = 64;       // points per MFMA tile (32 pairs in training)
constexpr int HS = 68;             // padded LDS row of bf16 tiles (K = 64)
constexpr int MLP_GRID = 1024;     // most blocks of mlp_features_kernel
constexpr size_t STAGE_LDS_CAP = 96 * 1024;

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

struct FlockChunk {
    int32_t row0, rows, comm, staged;
    int32_t sbase;   // flock_exact_kernel: first S-neg slice of the chunk, -1 if none
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

__host__ __device__ inline uint16_t to_bf16(float f) {
    uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
    u = __float_as_uint(f);
#else
    std::memcpy(&u, &f, 4);
#endif
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                            // nearest even
    return (uint16_t)(u >> 16);
}

__device__ inline float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_grad(float z) {
    float sg = 1.0f / (1.0f + __expf(-z));
    return sg * (1.0f + z * (1.0f - sg));
}

// w = K (s2 + r2)^(-beta) as K 2^(-beta log2(s2 + r2)) on the hardware base-2
// logarithm and exponential (v_log_f32, v_exp_f32, about one ulp each).  The
// argument is clamped below at the smallest normal float: those instructions
// do not take denormal inputs, and s2 + r2 is at least s2 for every pair.
__device__ inline float cs_weight(float r2, float K, float s2, float beta) {
    const float x = fmaxf(s2 + r2, 1.17549435e-38f);
    return K * __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(x));
}

__host__ __device__ inline uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// One 16x16 tile C += A * B^T over K (a multiple of 16) with bf16 MFMA and
// FP32 accumulation.  Element (m, k) of A is A[m*am + k*ak] and element
// (n, k) of B is B[n*bn + k*bk] (tile origins already applied), so any
// operand orientation in LDS is read in place.  Each 32-wide k block is one
// gfx950 16x16x32 step (lane l supplies row m = l%16 and k = 8*(l/16)..+7 of
// the block), a last 16-wide block one 16x16x16 step (k = 4*(l/16)..+3); the
// result element t of lane l is C[4*(l/16) + t][l%16].
__device__ inline f4v mma16(const uint16_t *A, int am, int ak, const uint16_t *B, int bn, int bk, int K,
                            f4v acc) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    int k0 = 0;
    for (; k0 + 32 <= K; k0 += 32) {
        const int kq = k0 + (lane >> 4) * 8;
        bf8v a, b;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            a[t] = __builtin_bit_cast(__bf16, A[r * am + (kq + t) * ak]);
            b[t] = __builtin_bit_cast(__bf16, B[r * bn + (kq + t) * bk]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    if (k0 < K) {
        const int kq = k0 + (lane >> 4) * 4;
        s4v a, b;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            a[t] = (short)A[r * am + (kq + t) * ak];
            b[t] = (short)B[r * bn + (kq + t) * bk];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// offsets of the parameter vector W1[64][3], b1[64], W2[64][64], b2[64],
// W3[R][64], b3[R], sgn[R]
struct ParamOffsets {
    int W1, b1, W2, b2, W3, b3, sgn, total;
};
__host__ __device__ inline ParamOffsets param_offsets(int R) {
    ParamOffsets o;
    o.W1 = 0;
    o.b1 = o.W1 + HID * 3;
    o.W2 = o.b1 + HID;
    o.b2 = o.W2 + HID * HID;
    o.W3 = o.b2 + HID;
    o.b3 = o.W3 + R * HID;
    o.sgn = o.b3 + R;
    o.total = o.sgn + R;
    return o;
}

// --------------------------------------------------------------------------
// state permutation (user order <-> community order), 6 planes
// --------------------------------------------------------------------------

__global__ void flock_permute_in(const float *__restrict__ user, const int32_t *__restrict__ perm, int64_t n,
                                 float *__restrict__ Y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t u = perm[i];
#pragma unroll
    for (int d = 0; d < 6; d++) Y[d * n + i] = user[d * n + u];
}

__global__ void flock_permute_out(const float *__restrict__ Y, const int32_t *__restrict__ perm, int64_t n,
                                  float *__restrict__ user) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t u = perm[i];
#pragma unroll
    for (int d = 0; d < 6; d++) user[d * n + u] = Y[d * n + i];
}

// --------------------------------------------------------------------------
// feature maps
// --------------------------------------------------------------------------

// Fourier features of every point (one thread per point): F[i][0] = 1,
// F[i][1+2h] = cos(pi <alpha_h, s_i> / L), F[i][2+2h] = sin(...), zero padding.
__global__ void fourier_features_kernel(const float *__restrict__ X, int64_t n, const int4 *__restrict__ alpha,
                                        int nh, float pi_over_L, int Rp, const int32_t *__restrict__ comm_of,
                                        const int32_t *__restrict__ fb, float *__restrict__ F) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (comm_of) {  // only members of communities on the separable path need features
        const int c = comm_of[i];
        if (c < 0 || (fb && fb[c])) return;
    }
    float x0 = X[i], x1 = X[n + i], x2 = X[2 * n + i];
    float *f = F + i * Rp;
    f[0] = 1.0f;
    for (int h = 0; h < nh; h++) {
        int4 a = alpha[h];
        float th = pi_over_L * ((float)a.x * x0 + (float)a.y * x1 + (float)a.z * x2);
        float sn, cs;
        fast_sincosf(th, &sn, &cs);
        f[1 + 2 * h] = cs;
        f[2 + 2 * h] = sn;
    }
    for (int r = 1 + 2 * nh; r < Rp; r++) f[r] = 0.0f;
}

struct MlpArgs {
    const int32_t *comm_of;   // optional: skip tiles without a member of a separable-path community
    const int32_t *fb;        //   (with fb: communities on the exact fallback count as not needing)
    const float *params;   // FP32 master parameters (W1, b1, b2, b3 read from here)
    const uint16_t *w2b;   // bf16 W2 [64][64]
    const uint16_t *w3b;   // bf16 W3 [R][64]
    float scale[3], shift[3];  // u = s * scale + shift maps the training box to [-1, 1]
    int R;
};

// Learned features, 64 points per tile: layer 1 on the VALU, layers 2 and 3
// as 16x16x16 bf16 MFMA tiles (wave w owns points 16w..16w+15).  A block
// stages the weights once and takes every gridDim.x-th tile.
__global__ __launch_bounds__(256) void mlp_features_kernel(const float *__restrict__ X, int64_t n, MlpArgs m,
                                                           float *__restrict__ F) {
    __shared__ uint16_t sW2[HID * HS], sW3[HID * HS], sH1[TILE_PTS * HS], sH2[TILE_PTS * HS];
    __shared__ float sW1[HID * 3], sb1[HID], sb2[HID], sb3[HID];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int R = m.R;
    const ParamOffsets po = param_offsets(R);
    for (int q = t; q < HID * HID; q += 256) sW2[(q >> 6) * HS + (q & 63)] = m.w2b[q];
    for (int q = t; q < R * HID; q += 256) sW3[(q >> 6) * HS + (q & 63)] = m.w3b[q];
    for (int q = t; q < HID * 3; q += 256) sW1[q] = m.params[po.W1 + q];
    if (t < HID) {
        sb1[t] = m.params[po.b1 + t];
        sb2[t] = m.params[po.b2 + t];
    }
    if (t < R) sb3[t] = m.params[po.b3 + t];
    const int64_t ntiles = (n + TILE_PTS - 1) / TILE_PTS;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * TILE_PTS;
        if (m.comm_of) {
            const int64_t p = p0 + (t >> 2);
            int need = 0;
            if (p < n) {
                const int c = m.comm_of[p];
                need = c >= 0 && !(m.fb && m.fb[c]);
            }
            if (!__syncthreads_or(need)) continue;  // the whole block skips the tile
        }
        {
            // layer 1: thread t -> point t/4, hidden units 16*(t%4) .. +15
            const int pl = t >> 2, g = (t & 3) * 16;
            const int64_t p = p0 + pl;
            float u0 = 0.f, u1 = 0.f, u2 = 0.f;
            if (p < n) {
                u0 = X[p] * m.scale[0] + m.shift[0];
                u1 = X[n + p] * m.scale[1] + m.shift[1];
                u2 = X[2 * n + p] * m.scale[2] + m.shift[2];
            }
            __syncthreads();  // weights in LDS; the previous tile's layer 2 is done with sH1
            for (int o = g; o < g + 16; o++) {
                float z = sb1[o] + sW1[o * 3] * u0 + sW1[o * 3 + 1] * u1 + sW1[o * 3 + 2] * u2;
                sH1[pl * HS + o] = to_bf16(silu_f(z));
            }
        }
        __syncthreads();
        // layer 2: H2 = silu(H1 W2^T + b2)
        const int mrow = 16 * w;
        for (int nt = 0; nt < HID / 16; nt++) {
            f4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(sH1 + mrow * HS, HS, 1, sW2 + nt * 16 * HS, HS, 1, HID, acc);
            const int col = nt * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int row = mrow + (lane >> 4) * 4 + q;
                sH2[row * HS + col] = to_bf16(silu_f(acc[q] + sb2[col]));
            }
        }
        __syncthreads();
        // layer 3: F = H2 W3^T + b3
        for (int nt = 0; nt < R / 16; nt++) {
            f4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(sH2 + mrow * HS, HS, 1, sW3 + nt * 16 * HS, HS, 1, HID, acc);
            const int col = nt * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int64_t p = p0 + mrow + (lane >> 4) * 4 + q;
                if (p < n) F[p * R + col] = acc[q] + sb3[col];
            }
        }
        __syncthreads();  // layer 3 is done with sH2 before the next tile's layer 2
    }
}

// --------------------------------------------------------------------------
// E1: per-community sums P_cr = sum f_r, V_cr = sum f_r v (FP64 accumulation)
// --------------------------------------------------------------------------

constexpr int E1_BLOCK = 1024;   // threads of flock_e1_kernel (G of them per item)
__global__ __launch_bounds__(E1_BLOCK) void flock_e1_kernel(const float *__restrict__ F, const float *__restrict__ Y,
                                                       int64_t n, const int32_t *__restrict__ comm_off, int Rp,
                                                       const int32_t *__restrict__ fb, float *__restrict__ Q) {
    __shared__ double part[E1_BLOCK];
    const int c = blockIdx.x, t = threadIdx.x;
    if (fb && fb[c]) return;  // exact fallback: no observables needed (whole block)
    const int c0 = comm_off[c], c1 = comm_off[c + 1];
    const int items = Rp * 4;
    // G threads share an item and take every G-th row; four independent
    // accumulators keep several loads in flight
    const int G = items >= E1_BLOCK ? 1 : E1_BLOCK / items;
    for (int base = 0; base < items; base += E1_BLOCK / G) {
        const int item = base + t % (E1_BLOCK / G), ph = t / (E1_BLOCK / G);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (item < items && ph < G) {
            const int r = item >> 2, q = item & 3;
            const float *vq = Y + (int64_t)(2 + q) * n;  // q = 1..3 -> v planes 3..5
            int j = c0 + ph;
            for (; j + 3 * G < c1; j += 4 * G) {
                const float f0 = F[(int64_t)j * Rp + r], f1 = F[(int64_t)(j + G) * Rp + r];
                const float f2 = F[(int64_t)(j + 2 * G) * Rp + r], f3 = F[(int64_t)(j + 3 * G) * Rp + r];
                if (q == 0) {
                    s0 += f0; s1 += f1; s2 += f2; s3 += f3;
                } else {
                    s0 += (double)f0 * vq[j];
                    s1 += (double)f1 * vq[j + G];
                    s2 += (double)f2 * vq[j + 2 * G];
                    s3 += (double)f3 * vq[j + 3 * G];
                }
            }
            for (; j < c1; j += G) {
                const float f = F[(int64_t)j * Rp + r];
                s0 += q == 0 ? (double)f : (double)f * vq[j];
            }
        }
        part[t] = (s0 + s1) + (s2 + s3);
        __syncthreads();
        if (ph == 0 && item < items) {
            double v = part[t];
            for (int g = 1; g < G; g++) v += part[t + g * (E1_BLOCK / G)];
            Q[((int64_t)c * Rp + (item >> 2)) * 4 + (item & 3)] = (float)v;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// the fused stage kernel: E1 broadcast + E2 + exact fallback + stepper update
// --------------------------------------------------------------------------

struct FlockArgs {
    const FlockChunk *chunks;
    const int32_t *comm_off;
    const int64_t *negptr;
    const int32_t *neg;  // partner index inside the community
    const int64_t *posptr;
    const int32_t *pos;  // partner position
    const int64_t *arp;  // direct method: adjacency in community order
    const int32_t *acol;
    const float *F;
    const float *sgn;
    const float *Q;
    const int32_t *fb;   // per community: 1 = exact fallback
    const float *Ys;     // stage state (6 planes, community order)
    float *Ynext;        // next stage state (RK4 stages 0-2, Euler)
    float *Y0;           // step base state (RK4; updated at stage 3)
    float *acc;          // RK4 accumulator (6 planes)
    float *out;          // RHS mode: dstate in user order
    const int32_t *perm;
    int64_t n;
    float invN, K, s2, beta;
    float cdt;           // RK4: c_{s+1} dt of the next stage; Euler: dt
    float dt6;           // RK4: dt / 6
    int stage;           // RK4 stage 0..3
    int mode;            // 0 = RHS, 1 = RK4 stage, 2 = Euler step
    int Rp;
    int exact_lds;       // flock_exact_kernel: dynamic LDS bytes of the launch
    // flock_exact_kernel: S-neg of staged chunks as slices of 64 / EXACT_RT
    // rows (one wavefront), entry k of every row of a slice stored together
    // (community-local indices; past a row's length, 0)
    const uint16_t *sneg;
    const int64_t *sneg_off;   // per slice: first entry
    const int32_t *sneg_w;     // per slice: entries per row (the longest row's)
    const uint8_t *srow;       // per row of a sliced chunk: the chunk row its thread slot takes
                               // (rows by decreasing S-neg length, so a slice's rows are alike)
    int plain;           // s2 >= the smallest normal float and s2^(-beta) finite: no clamp, and the
                         // self pair adds exactly 0 (flock_exact_kernel)
};

__device__ inline void flock_emit(const FlockArgs &a, int64_t i, const float k[6]) {
    const int64_t n = a.n;
    if (a.mode == 0) {
        const int64_t u = a.perm[i];
#pragma unroll
        for (int d = 0; d < 6; d++) a.out[d * n + u] = k[d];
        return;
    }
    if (a.mode == 2) {
#pragma unroll
        for (int d = 0; d < 6; d++) a.Ynext[d * n + i] = a.Ys[d * n + i] + a.cdt * k[d];
        return;
    }
    const float b = (a.stage == 1 || a.stage == 2) ? 2.0f : 1.0f;
#pragma unroll
    for (int d = 0; d < 6; d++) {
        const int64_t q = d * n + i;
        const float ac = a.stage == 0 ? k[d] : a.acc[q] + b * k[d];
        if (a.stage < 3) {
            a.acc[q] = ac;
            a.Ynext[q] = a.Y0[q] + a.cdt * k[d];
        } else {
            a.Y0[q] = a.Y0[q] + a.dt6 * ac;
        }
    }
}

// Chunks of the communities on a basis (the expansion of the weight, E1 and
// E2 of App. A.6): two lanes per row (each takes every other partner, then
// the row's sums are combined across the pair); the block covers up to 256
// rows of one community.  Staged chunks copy the community's state planes and
// features into LDS first.  The S-neg pairs come from the slices of
// flock_exact_kernel where the chunk has them (rows in the slices' order).
// RP > 0 fixes the feature stride at compile time (own features held in
// registers); RP == 0 reads it from the arguments.  Chunks on the exact path
// (fallback communities, rows of no community) are flock_exact_kernel's.
template <int RP>
__global__ __launch_bounds__(FBLOCK) void flock_stage_kernel(FlockArgs a) {
    extern __shared__ float lds[];
    const FlockChunk ch = a.chunks[blockIdx.x];
    const int64_t n = a.n;
    const int c = ch.comm;
    const int Rp = RP > 0 ? RP : a.Rp;
    int64_t c0 = 0;
    int lam = 0;
    bool fb = true;
    if (c >= 0) {
        c0 = a.comm_off[c];
        lam = a.comm_off[c + 1] - (int)c0;
        fb = a.fb[c] != 0;
    }
    if (fb) return;   // an exact-path chunk; before any barrier
    const bool staged = ch.staged != 0 && c >= 0;
    float *sY = lds;                       // [6][lam]
    float *sF = lds + ((6 * lam + 3) & ~3);  // [lam][Rp], 16-byte aligned
    if (staged) {
        // eight loads in flight per thread before the LDS writes
        constexpr int US = 8;
        const int ny = 6 * lam;
        for (int q0 = threadIdx.x; q0 < ny; q0 += FBLOCK * US) {
            float v[US];
#pragma unroll
            for (int u = 0; u < US; u++) {
                const int q = q0 + u * FBLOCK;
                if (q < ny) {
                    const int d = q / lam, j = q - d * lam;
                    v[u] = a.Ys[d * n + c0 + j];
                }
            }
#pragma unroll
            for (int u = 0; u < US; u++)
                if (q0 + u * FBLOCK < ny) sY[q0 + u * FBLOCK] = v[u];
        }
        if (!fb) {
            const int nf = lam * Rp;
            for (int q0 = threadIdx.x; q0 < nf; q0 += FBLOCK * US) {
                float v[US];
#pragma unroll
                for (int u = 0; u < US; u++)
                    if (q0 + u * FBLOCK < nf) v[u] = a.F[c0 * Rp + q0 + u * FBLOCK];
#pragma unroll
                for (int u = 0; u < US; u++)
                    if (q0 + u * FBLOCK < nf) sF[q0 + u * FBLOCK] = v[u];
            }
        }
    }
    __syncthreads();
    // TPR consecutive lanes share a row (a row's group never straddles a
    // wavefront); whole groups past the chunk leave together
    const int rloc = (int)threadIdx.x / TPR, sub = (int)threadIdx.x % TPR;
    if (rloc >= ch.rows) return;  // no barrier below
    // chunks with S-neg slices take their rows in the slices' order
    const bool sliced = ch.sbase >= 0;
    const int64_t i = ch.row0 + (sliced ? (int)a.srow[ch.row0 + rloc] : rloc);
    float xi[3], vi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        xi[d] = a.Ys[d * n + i];
        vi[d] = a.Ys[(3 + d) * n + i];
    }
    // community member j (local index): position and velocity
    auto member = [&](int jl, float xj[3], float vj[3]) {
        if (staged) {
#pragma unroll
            for (int d = 0; d < 3; d++) {
                xj[d] = sY[d * lam + jl];
                vj[d] = sY[(3 + d) * lam + jl];
            }
        } else {
#pragma unroll
            for (int d = 0; d < 3; d++) {
                xj[d] = a.Ys[d * n + c0 + jl];
                vj[d] = a.Ys[(3 + d) * n + c0 + jl];
            }
        }
    };
    float acc[3] = {0.f, 0.f, 0.f};
    const int64_t e0 = a.negptr[i], e1 = a.negptr[i + 1];
    // E1 broadcast: sum_r sgn_r f_r(s_i) (V_cr - v_i P_cr), by the
    // first lane of the row's group
    const float *fi = staged ? sF + (i - c0) * Rp : a.F + i * Rp;
    const float4 *Qc = reinterpret_cast<const float4 *>(a.Q) + (int64_t)c * Rp;
    float g[RP > 0 ? RP : 1];
    float sP = 0.f, sV0 = 0.f, sV1 = 0.f, sV2 = 0.f;
    for (int r = 0; r < Rp; r++) {
        const float gr = a.sgn[r] * fi[r];
        if (RP > 0) g[RP > 0 ? r : 0] = gr;
        if (sub == 0) {
            const float4 q = Qc[r];
            sP += gr * q.x;
            sV0 += gr * q.y;
            sV1 += gr * q.z;
            sV2 += gr * q.w;
        }
    }
    acc[0] = sV0 - vi[0] * sP;
    acc[1] = sV1 - vi[1] * sP;
    acc[2] = sV2 - vi[2] * sP;
    // E2, S-neg: subtract the expanded weight of the missing intra pairs
    auto sneg_pair = [&](int jl, bool in) {
        const float *fj = staged ? sF + (int64_t)jl * Rp : a.F + (c0 + jl) * Rp;
        float wt = 0.f;
        if (RP > 0) {
#pragma unroll
            for (int r = 0; r < (RP > 0 ? RP : 1); r += 4) {
                const float4 f4 = *reinterpret_cast<const float4 *>(fj + r);
                wt += g[r] * f4.x + g[r + 1] * f4.y + g[r + 2] * f4.z + g[r + 3] * f4.w;
            }
        } else {
            for (int r = 0; r < Rp; r++) wt += a.sgn[r] * fi[r] * fj[r];
        }
        wt = in ? wt : 0.f;
        float xj[3], vj[3];
        member(jl, xj, vj);
#pragma unroll
        for (int d = 0; d < 3; d++) acc[d] -= wt * (vj[d] - vi[d]);
    };
    if (sliced) {
        // the wavefront's slice: entry k of its rows in one coalesced load
        constexpr int SR = 64 / TPR;
        const int sl = ch.sbase + rloc / SR, rs = rloc % SR;
        const uint16_t *sp = a.sneg + a.sneg_off[sl];
        const int sw = a.sneg_w[sl], len = (int)(e1 - e0);
        for (int k = sub; k < sw; k += TPR) sneg_pair(sp[(int64_t)k * SR + rs], k < len);
    } else {
        for (int64_t e = e0 + sub; e < e1; e += TPR) sneg_pair(a.neg[e], true);
    }
    // E2, S-pos: exact weight on the pairs leaving the community
    for (int64_t e = a.posptr[i] + sub, e1 = a.posptr[i + 1]; e < e1; e += TPR) {
        const int64_t j = a.pos[e];
        const float d0 = a.Ys[j] - xi[0], d1 = a.Ys[n + j] - xi[1], d2 = a.Ys[2 * n + j] - xi[2];
        const float w = cs_weight(d0 * d0 + d1 * d1 + d2 * d2, a.K, a.s2, a.beta);
#pragma unroll
        for (int d = 0; d < 3; d++) acc[d] += w * (a.Ys[(3 + d) * n + j] - vi[d]);
    }
    // the row's partial sums, combined in a fixed order across its group
#pragma unroll
    for (int d = 0; d < 3; d++)
        for (int o = 1; o < TPR; o <<= 1) acc[d] += __shfl_xor(acc[d], o);
    if (sub == 0) {
        const float k[6] = {vi[0], vi[1], vi[2], acc[0] * a.invN, acc[1] * a.invN, acc[2] * a.invN};
        flock_emit(a, i, k);
    }
}

// Exact community path: the community sums of App. A.6 eq. (Cucker_Smale)
// taken pair by pair, with RT lanes per row.  The community's state is staged
// in LDS as three pair planes {s_x, s_y}, {s_z, v_x}, {v_y, v_z}.  The dense
// sum runs over every member of the row's community four members at a time,
// two 16-byte LDS broadcasts per pair plane (every lane of a row group takes
// the same members);
// where s2 is a normal float and s2^(-beta) finite it sums w v_j and w and
// subtracts v_i times the weight sum once (the self pair then adds exactly
// 0), otherwise the self pair is masked and the clamp of cs_weight applies.
// The S-neg pairs are then subtracted: a staged chunk's rows run in order of
// decreasing S-neg length, and the S-neg of the 64 / RT rows of a wavefront
// is a slice whose k-th entries lie together (one coalesced load of 16-bit
// member indices per step, each member three 8-byte LDS gathers).  Last the
// S-pos pairs are added.  Rows of no community take only their S-pos pairs.
// Weights are taken without K, which multiplies the row's total.  Chunks of
// communities on a basis are left to flock_stage_kernel.
template <int RT>
__global__ __launch_bounds__(CHUNK_ROWS * RT) void flock_exact_kernel(FlockArgs a) {
    extern __shared__ float lds[];
    const FlockChunk ch = a.chunks[blockIdx.x];
    const int64_t n = a.n;
    const int c = ch.comm;
    int64_t c0 = 0;
    int lam = 0;
    bool fb = true;
    if (c >= 0) {
        c0 = a.comm_off[c];
        lam = a.comm_off[c + 1] - (int)c0;
        fb = a.fb[c] != 0;
    }
    if (!fb) return;   // before any barrier
    const int lamp = (lam + 3) & ~3;   // plane stride, a multiple of 4 floats
    const bool staged = c >= 0 && (int64_t)6 * lamp * (int64_t)sizeof(float) <= (int64_t)a.exact_lds;
    // the state as three pair planes [3][lamp] of {s_x, s_y}, {s_z, v_x},
    // {v_y, v_z} (state dimension d is component d mod 2 of plane d / 2),
    // pad entries 0
    float *sY = lds;
    if (staged) {
        constexpr int US = 8;          // loads in flight per thread before the LDS writes
        const int ny = 6 * lamp;
        for (int q0 = threadIdx.x; q0 < ny; q0 += CHUNK_ROWS * RT * US) {
            float v[US];
#pragma unroll
            for (int u = 0; u < US; u++) {
                const int q = q0 + u * CHUNK_ROWS * RT;
                const int d = q / lamp, j = q - d * lamp;
                v[u] = q < ny && j < lam ? a.Ys[d * n + c0 + j] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < US; u++) {
                const int q = q0 + u * CHUNK_ROWS * RT;
                const int d = q / lamp, j = q - d * lamp;
                if (q < ny) sY[(d >> 1) * 2 * lamp + 2 * j + (d & 1)] = v[u];
            }
        }
    }
    const float2 *PP = reinterpret_cast<const float2 *>(sY);   // PP[p * lamp + j]
    __syncthreads();
    const int rloc = (int)threadIdx.x / RT, sub = (int)threadIdx.x % RT;
    if (rloc >= ch.rows) return;   // no barrier below
    const bool sliced = staged && ch.sbase >= 0;
    const int64_t i = ch.row0 + (sliced ? (int)a.srow[ch.row0 + rloc] : rloc);
    float xi[3], vi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        xi[d] = a.Ys[d * n + i];
        vi[d] = a.Ys[(3 + d) * n + i];
    }
    const float s2 = a.s2, nbeta = -a.beta;
    // (s2 + r2)^(-beta) on the hardware base-2 log and exp (as cs_weight)
    auto wt = [&](float d0, float d1, float d2) {
        const float x = fmaxf(s2 + (d0 * d0 + d1 * d1 + d2 * d2), 1.17549435e-38f);
        return __builtin_amdgcn_exp2f(nbeta * __builtin_amdgcn_logf(x));
    };
    // the same where s2 is a normal float (s2 + r2 >= s2: no clamp)
    auto wt_plain = [&](float d0, float d1, float d2) {
        const float x = fmaf(d2, d2, fmaf(d1, d1, fmaf(d0, d0, s2)));
        return __builtin_amdgcn_exp2f(nbeta * __builtin_amdgcn_logf(x));
    };
    float acc[3] = {0.f, 0.f, 0.f};
    if (c >= 0) {
        const int il = (int)(i - c0);
        if (staged) {
            // whole groups of four members, two 16-byte LDS broadcasts per
            // pair plane
            const float4 *P4 = reinterpret_cast<const float4 *>(sY);   // P4[p * lamp / 2 + 2 g + h]
            const int h4 = lamp >> 1, gfull = lam >> 2;
            // plain: sum w v_j and w, and take v_i times the weight sum once
            float aw[4] = {0.f, 0.f, 0.f, 0.f};
            auto groups = [&](auto plain) {
#pragma unroll 2
                for (int g = sub; g < gfull; g += RT) {
                    float4 Q[3][2];
#pragma unroll
                    for (int p = 0; p < 3; p++) {
                        Q[p][0] = P4[p * h4 + 2 * g];
                        Q[p][1] = P4[p * h4 + 2 * g + 1];
                    }
                    // member u: dimension 2p + e is component 2 (u & 1) + e of Q[p][u >> 1]
                    const float xs[3][4] = {{Q[0][0].x, Q[0][0].z, Q[0][1].x, Q[0][1].z},
                                            {Q[0][0].y, Q[0][0].w, Q[0][1].y, Q[0][1].w},
                                            {Q[1][0].x, Q[1][0].z, Q[1][1].x, Q[1][1].z}};
                    const float vs[3][4] = {{Q[1][0].y, Q[1][0].w, Q[1][1].y, Q[1][1].w},
                                            {Q[2][0].x, Q[2][0].z, Q[2][1].x, Q[2][1].z},
                                            {Q[2][0].y, Q[2][0].w, Q[2][1].y, Q[2][1].w}};
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        if constexpr (decltype(plain)::value) {
                            // the self pair adds w(0) (v_i - v_i), finite w(0)
                            const float w = wt_plain(xs[0][u] - xi[0], xs[1][u] - xi[1], xs[2][u] - xi[2]);
#pragma unroll
                            for (int d = 0; d < 3; d++) aw[d] = fmaf(w, vs[d][u], aw[d]);
                            aw[3] += w;
                        } else {
                            float w = wt(xs[0][u] - xi[0], xs[1][u] - xi[1], xs[2][u] - xi[2]);
                            w = 4 * g + u == il ? 0.f : w;
#pragma unroll
                            for (int d = 0; d < 3; d++) acc[d] += w * (vs[d][u] - vi[d]);
                        }
                    }
                }
            };
            if (a.plain) {
                groups(std::integral_constant<bool, true>());
#pragma unroll
                for (int d = 0; d < 3; d++) acc[d] = fmaf(-vi[d], aw[3], aw[d]);
            } else {
                groups(std::integral_constant<bool, false>());
            }
            // the last lam mod 4 members
            for (int j = 4 * gfull + sub; j < lam; j += RT) {
                if (j == il) continue;
                const float2 A = PP[j], B = PP[lamp + j], C = PP[2 * lamp + j];
                const float w = wt(A.x - xi[0], A.y - xi[1], B.x - xi[2]);
                acc[0] += w * (B.y - vi[0]);
                acc[1] += w * (C.x - vi[1]);
                acc[2] += w * (C.y - vi[2]);
            }
        } else {
            for (int j = sub; j < lam; j += RT) {
                if (j == il) continue;
                const int64_t q = c0 + j;
                const float w = wt(a.Ys[q] - xi[0], a.Ys[n + q] - xi[1], a.Ys[2 * n + q] - xi[2]);
#pragma unroll
                for (int d = 0; d < 3; d++) acc[d] += w * (a.Ys[(3 + d) * n + q] - vi[d]);
            }
        }
        // S-neg: the missing intra pairs (never the self pair)
        if (sliced) {
            // this row's slice: one coalesced load of entry k for the
            // wavefront's rows, members gathered from LDS
            constexpr int SR = 64 / RT;
            const int sl = ch.sbase + rloc / SR, rs = rloc % SR;
            const uint16_t *sp = a.sneg + a.sneg_off[sl];
            const int sw = a.sneg_w[sl];
            const int len = (int)(a.negptr[i + 1] - a.negptr[i]);
            auto sneg = [&](auto plain) {
#pragma unroll 4
                for (int k = sub; k < sw; k += RT) {
                    const int jl = sp[(int64_t)k * SR + rs];
                    const float2 A = PP[jl], B = PP[lamp + jl], C = PP[2 * lamp + jl];
                    const float d0 = A.x - xi[0], d1 = A.y - xi[1], d2 = B.x - xi[2];
                    float w = decltype(plain)::value ? wt_plain(d0, d1, d2) : wt(d0, d1, d2);
                    w = k < len ? w : 0.f;
                    acc[0] -= w * (B.y - vi[0]);
                    acc[1] -= w * (C.x - vi[1]);
                    acc[2] -= w * (C.y - vi[2]);
                }
            };
            if (a.plain)
                sneg(std::integral_constant<bool, true>());
            else
                sneg(std::integral_constant<bool, false>());
        } else {
            // a community above the staging cap (no slices): members from
            // global memory
            for (int64_t e = a.negptr[i] + sub, e1 = a.negptr[i + 1]; e < e1; e += RT) {
                const int jl = a.neg[e];
                float xj[3], vj[3];
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    xj[d] = a.Ys[d * n + c0 + jl];
                    vj[d] = a.Ys[(3 + d) * n + c0 + jl];
                }
                const float w = wt(xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]);
#pragma unroll
                for (int d = 0; d < 3; d++) acc[d] -= w * (vj[d] - vi[d]);
            }
        }
    }
    // S-pos: the pairs leaving the community
    for (int64_t e = a.posptr[i] + sub, e1 = a.posptr[i + 1]; e < e1; e += RT) {
        const int64_t j = a.pos[e];
        const float w = wt(a.Ys[j] - xi[0], a.Ys[n + j] - xi[1], a.Ys[2 * n + j] - xi[2]);
#pragma unroll
        for (int d = 0; d < 3; d++) acc[d] += w * (a.Ys[(3 + d) * n + j] - vi[d]);
    }
    // the row's partial sums, combined in a fixed order across its group
#pragma unroll
    for (int d = 0; d < 3; d++)
        for (int o = 1; o < RT; o <<= 1) acc[d] += __shfl_xor(acc[d], o);
    if (sub == 0) {
        const float kn = a.K * a.invN;
        const float k[6] = {vi[0], vi[1], vi[2], acc[0] * kn, acc[1] * kn, acc[2] * kn};
        flock_emit(a, i, k);
    }
}

// Direct method: one wavefront per row of the adjacency in community order.
__global__ __launch_bounds__(256) void flock_direct_kernel(FlockArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t n = a.n;
    if (i >= n) return;  // whole wavefront leaves together
    float xi[3], vi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        xi[d] = a.Ys[d * n + i];
        vi[d] = a.Ys[(3 + d) * n + i];
    }
    float acc[3] = {0.f, 0.f, 0.f};
    for (int64_t e = a.arp[i] + lane, e1 = a.arp[i + 1]; e < e1; e += 64) {
        const int64_t j = a.acol[e];
        const float d0 = a.Ys[j] - xi[0], d1 = a.Ys[n + j] - xi[1], d2 = a.Ys[2 * n + j] - xi[2];
        const float w = cs_weight(d0 * d0 + d1 * d1 + d2 * d2, a.K, a.s2, a.beta);
#pragma unroll
        for (int d = 0; d < 3; d++) acc[d] += w * (a.Ys[(3 + d) * n + j] - vi[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; d++) acc[d] = wave_sum(acc[d]);
    if (lane == 0) {
        const float k[6] = {vi[0], vi[1], vi[2], acc[0] * a.invN, acc[1] * a.invN, acc[2] * a.invN};
        flock_emit(a, i, k);
    }
}

// --------------------------------------------------------------------------
// judge: sampled members of every community, expanded vs exact weight
// --------------------------------------------------------------------------

struct JudgeArgs {
    const int32_t *comm_off;
    const int64_t *negptr;
    const int32_t *neg;
    const float *F, *sgn, *Q, *Y;
    float2 *es;          // [ncomm][JUDGE_SAMPLES]: (error, scale) of every sample
    int64_t n;
    float K, s2, beta;
    int Rp;
    uint64_t seed;
};

// One 64-lane block per (community, sample).  For the sampled member i the
// community part of its sum is computed twice: exactly (all pairs minus
// S-neg, exact weight) and as the method does (E1 broadcast minus S-neg with
// the expanded weight); the block writes max_d |approx - exact| (NaN kept)
// and max_d |exact|.  flock_judge_decide then takes every community's
// maximum over its samples.
__global__ __launch_bounds__(64) void flock_judge_kernel(JudgeArgs a) {
    extern __shared__ float gsh[];   // [Rp]: sgn_r f_r(s_i)
    const int c = blockIdx.x / JUDGE_SAMPLES, smp = blockIdx.x % JUDGE_SAMPLES, lane = threadIdx.x;
    const int64_t n = a.n;
    const int64_t c0 = a.comm_off[c];
    const int lam = a.comm_off[c + 1] - (int)c0;
    const int Rp = a.Rp;
    if (lam <= 0) {  // the whole block leaves together
        if (lane == 0) a.es[blockIdx.x] = make_float2(0.f, 0.f);
        return;
    }
    const int64_t i = c0 + (int64_t)(mix64(a.seed ^ ((uint64_t)c << 20) ^ (uint64_t)smp) % (uint64_t)lam);
    float xi[3], vi[3];
    for (int d = 0; d < 3; d++) {
        xi[d] = a.Y[d * n + i];
        vi[d] = a.Y[(3 + d) * n + i];
    }
    for (int r = lane; r < Rp; r += 64) gsh[r] = a.sgn[r] * a.F[i * Rp + r];
    __syncthreads();
    float ex[3] = {0.f, 0.f, 0.f}, ap[3] = {0.f, 0.f, 0.f};
    for (int64_t j = c0 + lane; j < c0 + lam; j += 64) {
        if (j == i) continue;
        const float d0 = a.Y[j] - xi[0], d1 = a.Y[n + j] - xi[1], d2 = a.Y[2 * n + j] - xi[2];
        const float wx = cs_weight(d0 * d0 + d1 * d1 + d2 * d2, a.K, a.s2, a.beta);
        for (int d = 0; d < 3; d++) ex[d] += wx * (a.Y[(3 + d) * n + j] - vi[d]);
    }
    const float4 *g4 = reinterpret_cast<const float4 *>(gsh);
    for (int64_t e = a.negptr[i] + lane; e < a.negptr[i + 1]; e += 64) {
        const int64_t j = c0 + a.neg[e];
        const float d0 = a.Y[j] - xi[0], d1 = a.Y[n + j] - xi[1], d2 = a.Y[2 * n + j] - xi[2];
        const float wx = cs_weight(d0 * d0 + d1 * d1 + d2 * d2, a.K, a.s2, a.beta);
        const float4 *fj = reinterpret_cast<const float4 *>(a.F + j * Rp);   // Rp is a multiple of 4
        float wt = 0.f;
        for (int r = 0; r < Rp / 4; r++) {
            const float4 f = fj[r], g = g4[r];
            wt += g.x * f.x + g.y * f.y + g.z * f.z + g.w * f.w;
        }
        for (int d = 0; d < 3; d++) {
            const float dv = a.Y[(3 + d) * n + j] - vi[d];
            ex[d] -= wx * dv;
            ap[d] -= wt * dv;
        }
    }
    // E1 broadcast, lane-strided over the features
    float sP = 0.f, sV[3] = {0.f, 0.f, 0.f};
    for (int r = lane; r < Rp; r += 64) {
        const float g = gsh[r];
        const float4 q = reinterpret_cast<const float4 *>(a.Q)[(int64_t)c * Rp + r];
        sP += g * q.x;
        sV[0] += g * q.y;
        sV[1] += g * q.z;
        sV[2] += g * q.w;
    }
    sP = wave_sum(sP);
    float e_ = 0.f, s_ = 0.f;
    for (int d = 0; d < 3; d++) {
        const float exd = wave_sum(ex[d]);
        const float apd = wave_sum(ap[d]) + wave_sum(sV[d]) - vi[d] * sP;
        const float diff = fabsf(apd - exd);
        e_ = (diff > e_ || diff != diff) ? diff : e_;  // NaN propagates
        s_ = fmaxf(s_, fabsf(exd));
    }
    if (lane == 0) a.es[blockIdx.x] = make_float2(e_, s_);
}

// A community falls back to the exact path when
//   max_i |approx_i - exact_i|_inf > tol * max_i |exact_i|_inf
// over its sampled members, or when any of it is not finite.
__global__ void flock_judge_decide(const float2 *__restrict__ es, int ncomm, float tol, int32_t *__restrict__ fb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncomm) return;
    float e_ = 0.f, s_ = 0.f;
    for (int q = 0; q < JUDGE_SAMPLES; q++) {
        const float2 v = es[(int64_t)c * JUDGE_SAMPLES + q];
        e_ = (v.x > e_ || v.x != v.x) ? v.x : e_;
        s_ = fmaxf(s_, v.y);
    }
    const bool ok = (e_ <= tol * s_) && isfinite(e_) && isfinite(s_);
    fb[c] = ok ? 0 : 1;
}

// --------------------------------------------------------------------------
// training of the learned basis
// --------------------------------------------------------------------------

// Pair samples from the current state: a uniformly drawn member i of a dense
// community and a uniformly drawn other member j of the same community; the
// target is the exact weight.  Counter-based (splitmix64) so every sample is
// reproducible from (seed, index).
__global__ void flock_sample_pairs(const float *__restrict__ Y, int64_t n, const int32_t *__restrict__ comm_of,
                                   const int32_t *__restrict__ comm_off, int64_t nassigned, uint64_t seed,
                                   int P, float K, float s2, float beta, float *__restrict__ pa,
                                   float *__restrict__ pb, float *__restrict__ pt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const uint64_t h1 = mix64(seed ^ (2ull * (uint64_t)k));
    const uint64_t h2 = mix64(seed ^ (2ull * (uint64_t)k + 1ull));
    const int64_t i = (int64_t)(h1 % (uint64_t)nassigned);
    const int c = comm_of[i];
    const int64_t c0 = comm_off[c];
    const int64_t lam = comm_off[c + 1] - c0;
    int64_t j = i;
    if (lam > 1) {
        j = c0 + (int64_t)(h2 % (uint64_t)(lam - 1));
        if (j >= i) j++;
    }
    float r2 = 0.f;
    for (int d = 0; d < 3; d++) {
        const float xa = Y[d * n + i], xb = Y[d * n + j];
        pa[3 * k + d] = xa;
        pb[3 * k + d] = xb;
        r2 += (xb - xa) * (xb - xa);
    }
    pt[k] = cs_weight(r2, K, s2, beta);
}

struct TrainArgs {
    const float *params;
    const uint16_t *w2b, *w3b;
    const float *pa, *pb, *pt;
    int P;          // pairs
    int R;
    float scale[3], shift[3];
    float *gpart;   // [gridDim.x][total params]
    double *lpart;  // [gridDim.x]
};

// Forward and backward of the pair loss (1/P) sum (wt(a,b) - t)^2 over tiles
// of 32 pairs (64 points: point 2k = a_k, 2k+1 = b_k).  Every GEMM is a bf16
// MFMA tile product with FP32 accumulation; bias and first-layer gradients
// are VALU sums.  Each block accumulates its tiles' gradients and writes one
// partial gradient vector (summed in fixed order by flock_grad_reduce).
__global__ __launch_bounds__(256) void flock_train_kernel(TrainArgs a) {
    __shared__ uint16_t sW2[HID * HS], sW3[HID * HS];
    __shared__ uint16_t sH1[TILE_PTS * HS], sH2[TILE_PTS * HS], sD3[TILE_PTS * HS], sD2[TILE_PTS * HS];
    __shared__ float sZ1[TILE_PTS * HID], sZ2[TILE_PTS * HID], sPhi[TILE_PTS * HID], sD3f[TILE_PTS * HID];
    __shared__ float sW1[HID * 3], sb1[HID], sb2[HID], sb3[HID], sSg[HID], sU[TILE_PTS * 3], sG[TILE_PTS / 2];
    __shared__ double sL[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int R = a.R;
    const ParamOffsets po = param_offsets(R);
    for (int q = t; q < HID * HID; q += 256) sW2[(q >> 6) * HS + (q & 63)] = a.w2b[q];
    for (int q = t; q < R * HID; q += 256) sW3[(q >> 6) * HS + (q & 63)] = a.w3b[q];
    for (int q = t; q < HID * 3; q += 256) sW1[q] = a.params[po.W1 + q];
    if (t < HID) {
        sb1[t] = a.params[po.b1 + t];
        sb2[t] = a.params[po.b2 + t];
    }
    if (t < R) {
        sb3[t] = a.params[po.b3 + t];
        sSg[t] = a.params[po.sgn + t];
    }
    // gradient accumulators: dW2 rows 16w.. (4 column tiles), dW3 columns 16w..
    // (R/16 row tiles), dW1/db1 (thread t: unit t/4, column t%4 with 3 = bias),
    // db2 (t < 64), db3 (t < R)
    f4v gW2[4], gW3[4];
    for (int q = 0; q < 4; q++) {
        gW2[q] = f4v{0.f, 0.f, 0.f, 0.f};
        gW3[q] = f4v{0.f, 0.f, 0.f, 0.f};
    }
    float g1 = 0.f, gb2 = 0.f, gb3 = 0.f;
    double lsum = 0.0;
    const int ntiles = (a.P + TILE_PTS / 2 - 1) / (TILE_PTS / 2);
    const float gscale = 2.0f / (float)a.P;
    const int mrow = 16 * w;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();  // weights loaded / previous tile consumed
        if (t < TILE_PTS) {
            const int k = tile * (TILE_PTS / 2) + (t >> 1);
            const float *src = (t & 1) ? a.pb : a.pa;
            for (int d = 0; d < 3; d++) sU[t * 3 + d] = k < a.P ? src[3 * k + d] * a.scale[d] + a.shift[d] : 0.f;
        }
        __syncthreads();
        {   // layer 1
            const int pl = t >> 2, g = (t & 3) * 16;
            const float u0 = sU[pl * 3], u1 = sU[pl * 3 + 1], u2 = sU[pl * 3 + 2];
            for (int o = g; o < g + 16; o++) {
                const float z = sb1[o] + sW1[o * 3] * u0 + sW1[o * 3 + 1] * u1 + sW1[o * 3 + 2] * u2;
                sZ1[pl * HID + o] = z;
                sH1[pl * HS + o] = to_bf16(silu_f(z));
            }
        }
        __syncthreads();
        for (int nt = 0; nt < 4; nt++) {  // layer 2
            f4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(sH1 + mrow * HS, HS, 1, sW2 + nt * 16 * HS, HS, 1, HID, acc);
            const int col = nt * 16 + (lane & 15);
            for (int q = 0; q < 4; q++) {
                const int row = mrow + (lane >> 4) * 4 + q;
                const float z = acc[q] + sb2[col];
                sZ2[row * HID + col] = z;
                sH2[row * HS + col] = to_bf16(silu_f(z));
            }
        }
        __syncthreads();
        for (int nt = 0; nt < R / 16; nt++) {  // layer 3
            f4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(sH2 + mrow * HS, HS, 1, sW3 + nt * 16 * HS, HS, 1, HID, acc);
            const int col = nt * 16 + (lane & 15);
            for (int q = 0; q < 4; q++) sPhi[(mrow + (lane >> 4) * 4 + q) * HID + col] = acc[q] + sb3[col];
        }
        __syncthreads();
        if (t < TILE_PTS / 2) {  // pair residuals
            const int k = tile * (TILE_PTS / 2) + t;
            float wt = 0.f;
            for (int r = 0; r < R; r++) wt += sSg[r] * sPhi[(2 * t) * HID + r] * sPhi[(2 * t + 1) * HID + r];
            const float e = k < a.P ? wt - a.pt[k] : 0.f;
            lsum += (double)e * (double)e;
            sG[t] = gscale * e;
        }
        __syncthreads();
        // delta3[p][r] = g_pair * sgn_r * phi_partner[r]
        for (int q = t; q < TILE_PTS * R; q += 256) {
            const int p = q / R, r = q - p * R;
            const float d3 = sG[p >> 1] * sSg[r] * sPhi[(p ^ 1) * HID + r];
            sD3f[p * HID + r] = d3;
            sD3[p * HS + r] = to_bf16(d3);
        }
        __syncthreads();
        // delta2 = (delta3 W3) * silu'(z2), in place of z2
        for (int nt = 0; nt < 4; nt++) {
            f4v acc = {0.f, 0.f, 0.f, 0.f};
            // B element (n = hidden unit, k = r) is W3[r][n]
            acc = mma16(sD3 + mrow * HS, HS, 1, sW3 + nt * 16, 1, HS, R, acc);
            const int col = nt * 16 + (lane & 15);
            for (int q = 0; q < 4; q++) {
                const int row = mrow + (lane >> 4) * 4 + q;
                const float d2 = acc[q] * silu_grad(sZ2[row * HID + col]);
                sZ2[row * HID + col] = d2;
                sD2[row * HS + col] = to_bf16(d2);
            }
        }
        __syncthreads();
        // delta1 = (delta2 W2) * silu'(z1), in place of z1
        for (int nt = 0; nt < 4; nt++) {
            f4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(sD2 + mrow * HS, HS, 1, sW2 + nt * 16, 1, HS, HID, acc);
            const int col = nt * 16 + (lane & 15);
            for (int q = 0; q < 4; q++) {
                const int row = mrow + (lane >> 4) * 4 + q;
                sZ1[row * HID + col] = acc[q] * silu_grad(sZ1[row * HID + col]);
            }
        }
        // weight gradients over the tile's 64 points (k = point index)
        for (int nt = 0; nt < 4; nt++)  // dW2[o][k] += sum_p delta2[p][o] h1[p][k]
            gW2[nt] = mma16(sD2 + mrow, 1, HS, sH1 + nt * 16, 1, HS, TILE_PTS, gW2[nt]);
        for (int mt = 0; mt < R / 16; mt++)  // dW3[r][k] += sum_p delta3[p][r] h2[p][k]
            gW3[mt] = mma16(sD3 + mt * 16, 1, HS, sH2 + mrow, 1, HS, TILE_PTS, gW3[mt]);
        __syncthreads();  // delta1 complete
        {
            const int o = t >> 2, col = t & 3;
            float s = 0.f;
            for (int p = 0; p < TILE_PTS; p++) s += sZ1[p * HID + o] * (col < 3 ? sU[p * 3 + col] : 1.0f);
            g1 += s;
        }
        if (t < HID) {
            float s = 0.f;
            for (int p = 0; p < TILE_PTS; p++) s += sZ2[p * HID + t];
            gb2 += s;
        }
        if (t < R) {
            float s = 0.f;
            for (int p = 0; p < TILE_PTS; p++) s += sD3f[p * HID + t];
            gb3 += s;
        }
    }
    // write this block's partial gradient in parameter layout
    float *gp = a.gpart + (int64_t)blockIdx.x * po.total;
    {
        const int o = t >> 2, col = t & 3;
        if (col < 3) gp[po.W1 + o * 3 + col] = g1;
        else gp[po.b1 + o] = g1;
    }
    if (t < HID) gp[po.b2 + t] = gb2;
    if (t < R) {
        gp[po.b3 + t] = gb3;
        gp[po.sgn + t] = 0.f;
    }
    for (int nt = 0; nt < 4; nt++)
        for (int q = 0; q < 4; q++) {
            const int o = mrow + (lane >> 4) * 4 + q, k = nt * 16 + (lane & 15);
            gp[po.W2 + o * HID + k] = gW2[nt][q];
        }
    for (int mt = 0; mt < R / 16; mt++)
        for (int q = 0; q < 4; q++) {
            const int r = mt * 16 + (lane >> 4) * 4 + q, k = mrow + (lane & 15);
            gp[po.W3 + r * HID + k] = gW3[mt][q];
        }
    // loss partial (threads 0..31 hold residual sums)
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) sL[w] = lsum;
    __syncthreads();
    if (t == 0) a.lpart[blockIdx.x] = sL[0] + sL[1] + sL[2] + sL[3];
}

// grad[q] = sum over blocks of the partials, in block order; loss = sum / P
__global__ void flock_grad_reduce(const float *__restrict__ gpart, const double *__restrict__ lpart, int nblk,
                                  int total, int P, float *__restrict__ grad, double *__restrict__ loss) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < total) {
        float s = 0.f;
        for (int b = 0; b < nblk; b++) s += gpart[(int64_t)b * total + q];
        grad[q] = s;
    }
    if (q == 0 && loss) {
        double l = 0.0;
        for (int b = 0; b < nblk; b++) l += lpart[b];
        *loss = l / (double)P;
    }
}

// Adam step on every trained parameter (the signs are fixed), then the bf16
// copies of W2 and W3 used by the MFMA kernels.
__global__ void flock_adam(float *__restrict__ params, float *__restrict__ m1, float *__restrict__ m2,
                           const float *__restrict__ grad, int R, float lr, float b1, float b2, float c1,
                           float c2, float eps, uint16_t *__restrict__ w2b, uint16_t *__restrict__ w3b) {
    const ParamOffsets po = param_offsets(R);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= po.sgn) return;
    const float g = grad[q];
    const float a = b1 * m1[q] + (1.f - b1) * g;
    const float b = b2 * m2[q] + (1.f - b2) * g * g;
    m1[q] = a;
    m2[q] = b;
    const float p = params[q] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    params[q] = p;
    if (q >= po.W2 && q < po.b2) w2b[q - po.W2] = to_bf16(p);
    if (q >= po.W3 && q < po.b3) w3b[q - po.W3] = to_bf16(p);
}

__global__ void flock_bf16_copies(const float *__restrict__ params, int R, uint16_t *__restrict__ w2b,
                                  uint16_t *__restrict__ w3b) {
    const ParamOffsets po = param_offsets(R);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < HID * HID) w2b[q] = to_bf16(params[po.W2 + q]);
    if (q < R * HID) w3b[q] = to_bf16(params[po.W3 + q]);
}

__global__ void flock_fill_i32(int32_t *p, int64_t count, int32_t v) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = v;
}

inline unsigned grid_for(int64_t count, int block) { return (unsigned)((count + block - 1) / block); }

}  // namespace

// ==========================================================================
// host side
// ==========================================================================

struct FlockState {
    int basis = CIA_BASIS_EXACT;
    int R = 0, Rp = 0;       // features and their stride (Rp = R rounded up to 4)
    int fp = 0;              // Fourier order
    double L = 0.0;
    float K = 1.f, s2 = 1.f, beta = 0.f;
    float judge_tol = 0.f;
    bool judge = false;
    bool trained = false;
    int train_iters = 0;
    uint64_t judge_seed = 0x5EEDull;
    int32_t ncomm = 0;
    int64_t nassigned = 0;
    // graph in community order
    int32_t *perm = nullptr, *comm_off = nullptr, *comm_of = nullptr;
    int64_t *negptr = nullptr, *posptr = nullptr, *arp = nullptr;
    int32_t *neg = nullptr, *pos = nullptr, *acol = nullptr;
    FlockChunk *chunks = nullptr;
    int nchunks = 0;
    uint16_t *sneg = nullptr;           // flock_exact_kernel's sliced S-neg
    uint8_t *srow = nullptr;
    int64_t *sneg_off = nullptr;
    int32_t *sneg_w = nullptr;
    size_t lds_bytes = 0;
    size_t lds_exact = 0;   // LDS of the exact-path launch (state planes only)
    // state and E1
    float *Y[3] = {nullptr, nullptr, nullptr};
    float *acc = nullptr;
    float *F = nullptr, *sgn = nullptr, *Q = nullptr;
    int32_t *fb = nullptr;
    float2 *judge_es = nullptr;         // [ncomm][JUDGE_SAMPLES] per-sample judge results
    int4 *alpha = nullptr;
    int nh = 0;
    // learned basis
    float *params = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    uint16_t *w2b = nullptr, *w3b = nullptr;
    float scale[3] = {1, 1, 1}, shift[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    int64_t adam_t = 0;
    // training scratch (allocated on first use)
    float *pa = nullptr, *pb = nullptr, *pt = nullptr, *gpart = nullptr;
    double *lpart = nullptr, *losses = nullptr, *loss1 = nullptr;
    int train_blocks = 0;
    int64_t losses_cap = 0;
};

namespace {

// Gauss-Legendre rule on [-1, 1] (roots of P_m by Newton's method from the
// Chebyshev-like initial guess, weights 2 / ((1 - x^2) P_m'(x)^2)).
void legendre_rule(int m, std::vector<double> &x, std::vector<double> &w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; i++) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5)), d = 1.0;
        for (int it = 0; it < 64; it++) {
            double pk = z, pkm1 = 1.0;
            for (int k = 2; k <= m; k++) {
                const double pn = ((2 * k - 1) * z * pk - (k - 1) * pkm1) / k;
                pkm1 = pk;
                pk = pn;
            }
            d = m * (pkm1 - z * pk) / (1.0 - z * z);
            const double step = pk / d;
            z -= step;
            if (std::fabs(step) < 1e-15) break;
        }
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * d * d);
    }
}

// c_alpha for |alpha| in {0..p}^3 of w on [-L, L]^3 (App. A.6), by a 64-point
// Gauss-Legendre product rule; w is even per coordinate, so only the cosine
// parts survive and c depends on (|a1|, |a2|, |a3|).
std::vector<double> fourier_coefficients(double K, double s2, double beta, double L, int p) {
    const int m = 64, q = p + 1;
    std::vector<double> x, wq;
    legendre_rule(m, x, wq);
    std::vector<double> cosv((size_t)q * m);
    for (int a = 0; a < q; a++)
        for (int i = 0; i < m; i++) cosv[(size_t)a * m + i] = std::cos(M_PI * a * x[i]);
    // partial sums over the last two axes for every (i, a2, a3)
    std::vector<double> part((size_t)m * q * q, 0.0);
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++)
            for (int k = 0; k < m; k++) {
                const double y2 = L * L * (x[i] * x[i] + x[j] * x[j] + x[k] * x[k]);
                const double f = wq[j] * wq[k] * K * std::pow(s2 + y2, -beta);
                for (int a2 = 0; a2 < q; a2++)
                    for (int a3 = 0; a3 < q; a3++)
                        part[((size_t)i * q + a2) * q + a3] += f * cosv[(size_t)a2 * m + j] * cosv[(size_t)a3 * m + k];
            }
    std::vector<double> c((size_t)q * q * q, 0.0);
    for (int a1 = 0; a1 < q; a1++)
        for (int a2 = 0; a2 < q; a2++)
            for (int a3 = 0; a3 < q; a3++) {
                double s = 0.0;
                for (int i = 0; i < m; i++) s += wq[i] * cosv[(size_t)a1 * m + i] * part[((size_t)i * q + a2) * q + a3];
                c[((size_t)a1 * q + a2) * q + a3] = s / 8.0;  // (L^3 from dy) / (2L)^3
            }
    return c;
}

// default initial parameters: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) per
// layer from a counter-based generator, signs +1 (w is a positive-definite
// kernel, so a sum of squares is the natural separable form)
std::vector<float> initial_params(int R, uint64_t seed) {
    const ParamOffsets po = param_offsets(R);
    std::vector<float> p(po.total);
    uint64_t ctr = 0;
    auto uni = [&](double bound) {
        const uint64_t h = mix64(seed ^ (ctr++ * 0xD1B54A32D192ED03ull));
        return (float)(bound * (2.0 * ((h >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
    };
    for (int q = po.W1; q < po.W2; q++) p[q] = uni(1.0 / std::sqrt(3.0));
    for (int q = po.W2; q < po.W3; q++) p[q] = uni(1.0 / std::sqrt((double)HID));
    for (int q = po.W3; q < po.sgn; q++) p[q] = uni(1.0 / std::sqrt((double)HID));
    for (int q = po.sgn; q < po.total; q++) p[q] = 1.0f;
    return p;
}

FlockArgs base_args(cia_plan *p) {
    FlockState *f = p->flock;
    FlockArgs a{};
    a.chunks = f->chunks;
    a.comm_off = f->comm_off;
    a.negptr = f->negptr;
    a.neg = f->neg;
    a.sneg = f->sneg;
    a.sneg_off = f->sneg_off;
    a.sneg_w = f->sneg_w;
    a.srow = f->srow;
    a.posptr = f->posptr;
    a.pos = f->pos;
    a.arp = f->arp;
    a.acol = f->acol;
    a.F = f->F;
    a.sgn = f->sgn;
    a.Q = f->Q;
    a.fb = f->fb;
    a.perm = f->perm;
    a.n = p->n;
    a.invN = (float)(1.0 / (double)p->n);
    a.K = f->K;
    a.s2 = f->s2;
    a.beta = f->beta;
    a.Rp = f->Rp;
    return a;
}

MlpArgs mlp_args(FlockState *f) {
    MlpArgs m{};
    m.params = f->params;
    m.w2b = f->w2b;
    m.w3b = f->w3b;
    for (int d = 0; d < 3; d++) {
        m.scale[d] = f->scale[d];
        m.shift[d] = f->shift[d];
    }
    m.R = f->R;
    return m;
}

void set_box(FlockState *f, const double lo[3], const double hi[3]) {
    for (int d = 0; d < 3; d++) {
        f->lo[d] = lo[d];
        f->hi[d] = hi[d];
        f->scale[d] = (float)(2.0 / (hi[d] - lo[d]));
        f->shift[d] = (float)(-(hi[d] + lo[d]) / (hi[d] - lo[d]));
    }
}

// features of the stage state X (community order) into f->F
// features of the points X into F; with comm_of (a stage state in community
// order) only members of communities that need them are computed: every
// separable-path community, or with fb those not on the exact fallback
cia_status run_features(cia_plan *p, const float *X, int64_t n, float *F, hipStream_t s,
                        const int32_t *comm_of = nullptr, const int32_t *fb = nullptr) {
    FlockState *f = p->flock;
    if (f->basis == CIA_BASIS_FOURIER) {
        fourier_features_kernel<<<grid_for(n, 256), 256, 0, s>>>(X, n, f->alpha, f->nh, (float)(M_PI / f->L),
                                                                 f->Rp, comm_of, fb, F);
    } else if (f->basis == CIA_BASIS_LEARNED) {
        MlpArgs m = mlp_args(f);
        m.comm_of = comm_of;
        m.fb = fb;
        // about four blocks per CU, each staging the weights once
        const int64_t ntiles = (n + TILE_PTS - 1) / TILE_PTS;
        mlp_features_kernel<<<(int)std::min<int64_t>(ntiles, MLP_GRID), 256, 0, s>>>(X, n, m, F);
    }
    CIA_HIP(hipGetLastError());
    return CIA_OK;
}

// features + E1 (+ judge) for the stage state Ys
cia_status run_observables(cia_plan *p, const float *Ys, bool judge, hipStream_t s) {
    FlockState *f = p->flock;
    if (p->method != CIA_METHOD_CIA || f->basis == CIA_BASIS_EXACT || f->ncomm == 0) return CIA_OK;
    CIA_TRY(timing_begin(p, s, KK_PREP));
    // the judged stage needs every community's features and observables; the
    // other stages skip communities held on the exact fallback
    const int32_t *skip = (judge && f->judge) ? nullptr : f->fb;
    CIA_TRY(run_features(p, Ys, p->n, f->F, s, f->comm_of, skip));
    flock_e1_kernel<<<f->ncomm, E1_BLOCK, 0, s>>>(f->F, Ys, p->n, f->comm_off, f->Rp, skip, f->Q);
    CIA_HIP(hipGetLastError());
    if (judge && f->judge) {
        JudgeArgs j{};
        j.comm_off = f->comm_off;
        j.negptr = f->negptr;
        j.neg = f->neg;
        j.F = f->F;
        j.sgn = f->sgn;
        j.Q = f->Q;
        j.Y = Ys;
        j.es = f->judge_es;
        j.n = p->n;
        j.K = f->K;
        j.s2 = f->s2;
        j.beta = f->beta;
        j.Rp = f->Rp;
        j.seed = mix64(f->judge_seed++);
        flock_judge_kernel<<<f->ncomm * JUDGE_SAMPLES, 64, (size_t)f->Rp * sizeof(float), s>>>(j);
        CIA_HIP(hipGetLastError());
        flock_judge_decide<<<grid_for(f->ncomm, 256), 256, 0, s>>>(f->judge_es, f->ncomm, f->judge_tol, f->fb);
        CIA_HIP(hipGetLastError());
    }
    CIA_TRY(timing_end(p, s));
    return CIA_OK;
}

cia_status launch_stage(cia_plan *p, const FlockArgs &a0, hipStream_t s) {
    FlockState *f = p->flock;
    CIA_TRY(timing_begin(p, s, KK_STAGE));
    if (p->method == CIA_METHOD_DIRECT) {
        flock_direct_kernel<<<grid_for(p->n, 4), 256, 0, s>>>(a0);
    } else if (f->nchunks > 0) {
        FlockArgs a = a0;
        // exact-path chunks (communities on the exact fallback, rows of no
        // community) in their own kernel; then, with a basis, the others
        a.exact_lds = (int)f->lds_exact;
        {
            const double w0 = std::pow((double)f->s2, -(double)f->beta);   // the largest weight
            a.plain = f->s2 >= FLT_MIN && std::isfinite(w0) && w0 < 1e38 ? 1 : 0;
        }
        flock_exact_kernel<EXACT_RT><<<f->nchunks, CHUNK_ROWS * EXACT_RT, f->lds_exact, s>>>(a);
        if (f->basis == CIA_BASIS_EXACT) {
            CIA_HIP(hipGetLastError());
            CIA_TRY(timing_end(p, s));
            return CIA_OK;
        }
        const size_t lds = f->lds_bytes;
        switch (f->Rp) {
            case 16: flock_stage_kernel<16><<<f->nchunks, FBLOCK, lds, s>>>(a); break;
            case 28: flock_stage_kernel<28><<<f->nchunks, FBLOCK, lds, s>>>(a); break;
            case 32: flock_stage_kernel<32><<<f->nchunks, FBLOCK, lds, s>>>(a); break;
            case 48: flock_stage_kernel<48><<<f->nchunks, FBLOCK, lds, s>>>(a); break;
            // 64 features cached in registers would cost too many of them
            default: flock_stage_kernel<0><<<f->nchunks, FBLOCK, lds, s>>>(a); break;
        }
    }
    CIA_HIP(hipGetLastError());
    CIA_TRY(timing_end(p, s));
    return CIA_OK;
}

cia_status ensure_train_buffers(cia_plan *p, int64_t pairs) {
    FlockState *f = p->flock;
    const ParamOffsets po = param_offsets(f->R);
    if (!f->pa) {
        CIA_TRY(dalloc(p, &f->pa, (size_t)3 * TRAIN_PAIRS));
        CIA_TRY(dalloc(p, &f->pb, (size_t)3 * TRAIN_PAIRS));
        CIA_TRY(dalloc(p, &f->pt, (size_t)TRAIN_PAIRS));
        f->train_blocks = 128;
        CIA_TRY(dalloc(p, &f->gpart, (size_t)f->train_blocks * po.total));
        CIA_TRY(dalloc(p, &f->lpart, (size_t)f->train_blocks));
        CIA_TRY(dalloc(p, &f->loss1, 1));
    }
    (void)pairs;
    return CIA_OK;
}

// loss and gradient of P pairs (device buffers a, b: [P][3]; t: [P])
cia_status loss_grad(cia_plan *p, const float *pa, const float *pb, const float *pt, int P, float *grad,
                     double *loss_dev, hipStream_t s) {
    FlockState *f = p->flock;
    const ParamOffsets po = param_offsets(f->R);
    TrainArgs t{};
    t.params = f->params;
    t.w2b = f->w2b;
    t.w3b = f->w3b;
    t.pa = pa;
    t.pb = pb;
    t.pt = pt;
    t.P = P;
    t.R = f->R;
    for (int d = 0; d < 3; d++) {
        t.scale[d] = f->scale[d];
        t.shift[d] = f->shift[d];
    }
    t.gpart = f->gpart;
    t.lpart = f->lpart;
    const int ntiles = (P + TILE_PTS / 2 - 1) / (TILE_PTS / 2);
    const int nblk = std::max(1, std::min(f->train_blocks, ntiles));
    flock_train_kernel<<<nblk, 256, 0, s>>>(t);
    CIA_HIP(hipGetLastError());
    flock_grad_reduce<<<grid_for(po.total, 256), 256, 0, s>>>(f->gpart, f->lpart, nblk, po.total, P, grad,
                                                               loss_dev);
    CIA_HIP(hipGetLastError());
    return CIA_OK;
}

// Train the learned basis on pair samples of the community-order state Y.
cia_status train(cia_plan *p, const float *Y, int iters, uint64_t seed, double *loss_trace, hipStream_t s) {
    FlockState *f = p->flock;
    if (f->nassigned == 0) return set_error(CIA_EINVAL, "no dense community to train the basis on");
    CIA_TRY(ensure_train_buffers(p, TRAIN_PAIRS));
    // input box from the positions, 2% margin
    std::vector<float> hx((size_t)3 * p->n);
    CIA_HIP(hipMemcpyAsync(hx.data(), Y, sizeof(float) * 3 * p->n, hipMemcpyDeviceToHost, s));
    CIA_HIP(hipStreamSynchronize(s));
    double lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        double a = INFINITY, b = -INFINITY;
        for (int64_t i = 0; i < p->n; i++) {
            const double v = hx[(size_t)d * p->n + i];
            a = std::min(a, v);
            b = std::max(b, v);
        }
        if (!std::isfinite(a) || !std::isfinite(b)) return set_error(CIA_ENONFINITE, "state holds NaN or Inf");
        const double mid = 0.5 * (a + b), half = std::max(0.5 * (b - a) * 1.02, 1e-3);
        lo[d] = mid - half;
        hi[d] = mid + half;
    }
    set_box(f, lo, hi);
    if (iters > f->losses_cap) {
        CIA_TRY(dalloc(p, &f->losses, (size_t)iters));
        f->losses_cap = iters;
    }
    const ParamOffsets po = param_offsets(f->R);
    const float b1 = 0.9f, b2 = 0.999f;
    for (int it = 0; it < iters; it++) {
        flock_sample_pairs<<<grid_for(TRAIN_PAIRS, 256), 256, 0, s>>>(
            Y, p->n, f->comm_of, f->comm_off, f->nassigned, mix64(seed ^ ((uint64_t)it << 24)), TRAIN_PAIRS,
            f->K, f->s2, f->beta, f->pa, f->pb, f->pt);
        CIA_HIP(hipGetLastError());
        CIA_TRY(loss_grad(p, f->pa, f->pb, f->pt, TRAIN_PAIRS, f->grad, f->losses + it, s));
        f->adam_t++;
        const double lr = it < iters / 2 ? 3e-3 : (it < (5 * iters) / 6 ? 1e-3 : 3e-4);
        const float c1 = (float)(1.0 - std::pow((double)b1, (double)f->adam_t));
        const float c2 = (float)(1.0 - std::pow((double)b2, (double)f->adam_t));
        flock_adam<<<grid_for(po.sgn, 256), 256, 0, s>>>(f->params, f->m1, f->m2, f->grad, f->R, (float)lr, b1, b2,
                                                          c1, c2, 1e-8f, f->w2b, f->w3b);
        CIA_HIP(hipGetLastError());
    }
    if (loss_trace && iters > 0) {
        CIA_HIP(hipMemcpyAsync(loss_trace, f->losses, sizeof(double) * iters, hipMemcpyDeviceToHost, s));
        CIA_HIP(hipStreamSynchronize(s));
    }
    f->trained = true;
    return CIA_OK;
}

cia_status ensure_trained(cia_plan *p, const float *Y, hipStream_t s) {
    FlockState *f = p->flock;
    if (f->basis != CIA_BASIS_LEARNED || f->trained || p->method != CIA_METHOD_CIA) return CIA_OK;
    return train(p, Y, f->train_iters, 0x7A1Bull, nullptr, s);
}

FlockState *flock_of(cia_plan *p) { return p ? p->flock : nullptr; }

}  // namespace

cia_status flock_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                       const cia_options *o) {
    if (o->precision != CIA_F32)
        return set_error(CIA_EUNSUPPORTED, "the flock model runs in FP32 only (precision = %d)", o->precision);
    if (!(c->cs_sigma > 0.0) || !std::isfinite(c->cs_sigma) || !std::isfinite(c->cs_K) || !std::isfinite(c->cs_beta))
        return set_error(CIA_EINVAL, "flock weight needs finite cs_K, cs_beta and cs_sigma > 0");
    const int basis = c->cs_basis;
    if (basis != CIA_BASIS_EXACT && basis != CIA_BASIS_FOURIER && basis != CIA_BASIS_LEARNED)
        return set_error(CIA_EINVAL, "coupling.cs_basis = %d", basis);
    if (basis == CIA_BASIS_FOURIER && (c->p < 1 || c->p > 2))
        return set_error(CIA_EINVAL, "Fourier flock basis needs p in 1..2 (p = %d)", c->p);
    if (basis == CIA_BASIS_FOURIER && !(c->cs_L > 0.0))
        return set_error(CIA_EINVAL, "Fourier flock basis needs cs_L > 0");
    if (basis == CIA_BASIS_LEARNED && (c->rank < 16 || c->rank > 64 || c->rank % 16))
        return set_error(CIA_EINVAL, "learned basis rank must be 16, 32, 48 or 64 (rank = %d)", c->rank);
    if (o->judge_tol < 0.0 || !std::isfinite(o->judge_tol))
        return set_error(CIA_EINVAL, "options.judge_tol = %g", o->judge_tol);
    if (g->n > INT32_MAX) return set_error(CIA_EINVAL, "n too large");

    auto *f = new (std::nothrow) FlockState();
    if (!f) return set_error(CIA_ENOMEM, "host allocation failed");
    p->flock = f;
    f->basis = p->method == CIA_METHOD_CIA ? basis : CIA_BASIS_EXACT;
    f->K = (float)c->cs_K;
    f->s2 = (float)(c->cs_sigma * c->cs_sigma);
    f->beta = (float)c->cs_beta;
    f->judge_tol = (float)o->judge_tol;
    f->judge = f->basis != CIA_BASIS_EXACT && !(o->flags & CIA_FLAG_NO_JUDGE) && o->judge_tol > 0.0;
    f->train_iters = c->train_iters > 0 ? c->train_iters : 3000;

    const bool cia_method = p->method == CIA_METHOD_CIA;
    P1 p1;
    CIA_TRY(p1_build(g, labels, o->dense_alpha, (o->flags & CIA_FLAG_KEEP_LABELS) != 0,
                     !(o->flags & CIA_FLAG_NO_VALIDATE), cia_method, p1));
    const int64_t n = p1.n;
    f->ncomm = p1.ncomm;
    f->nassigned = p1.ncomm ? p1.comm_off[p1.ncomm] : 0;
    CIA_TRY(dupload(p, &f->perm, p1.perm.data(), n));
    CIA_TRY(dupload(p, &f->comm_off, p1.comm_off.data(), p1.comm_off.size()));
    CIA_TRY(dupload(p, &f->comm_of, p1.comm_of_pos.data(), n));
    for (int q = 0; q < 3; q++) CIA_TRY(dalloc(p, &f->Y[q], (size_t)6 * n));
    CIA_TRY(dalloc(p, &f->acc, (size_t)6 * n));

    cia_plan_info &info = p->info;
    info.n = n;
    info.nnz_graph = p1.nnz_graph;
    info.method = p->method;
    info.precision = p->precision;
    info.model = CIA_MODEL_FLOCK;
    info.ncomm = p1.ncomm;
    info.n_unassigned = n - f->nassigned;
    int32_t maxc = 0;
    for (int32_t q = 0; q < p1.ncomm; q++) maxc = std::max(maxc, p1.comm_off[q + 1] - p1.comm_off[q]);
    info.max_comm = maxc;

    if (!cia_method) {
        std::vector<int64_t> rp;
        std::vector<int32_t> col;
        CIA_TRY(p1_permuted_adjacency(g, p1, rp, col));
        CIA_TRY(dupload(p, &f->arp, rp.data(), rp.size()));
        CIA_TRY(dupload(p, &f->acol, col.data(), col.size()));
        info.nnz_pos = (int64_t)col.size();
        info.nunits = (int32_t)grid_for(n, 4);
        // CSR row pointers and indices, 6 state planes read per row plus the
        // gathered partner (6 floats), 6 planes written
        info.bytes_per_rhs = (double)n * (8 + 24 + 24) + (double)col.size() * (4 + 24);
        info.bytes_per_stage = info.bytes_per_rhs + (double)n * 24 * 2;
        return CIA_OK;
    }

    info.nnz_neg = (int64_t)p1.neg_local.size();
    info.nnz_pos = (int64_t)p1.pos.size();
    CIA_TRY(dupload(p, &f->negptr, p1.negptr.data(), p1.negptr.size()));
    CIA_TRY(dupload(p, &f->neg, p1.neg_local.data(), p1.neg_local.size()));
    CIA_TRY(dupload(p, &f->posptr, p1.posptr.data(), p1.posptr.size()));
    CIA_TRY(dupload(p, &f->pos, p1.pos.data(), p1.pos.size()));

    // basis
    std::vector<float> sg;
    if (f->basis == CIA_BASIS_FOURIER) {
        const int pf = c->p, q = pf + 1;
        f->fp = pf;
        f->L = c->cs_L;
        const std::vector<double> cf = fourier_coefficients(c->cs_K, c->cs_sigma * c->cs_sigma, c->cs_beta, c->cs_L, pf);
        std::vector<int4> al;
        sg.push_back((float)cf[0]);
        for (int a1 = -pf; a1 <= pf; a1++)
            for (int a2 = -pf; a2 <= pf; a2++)
                for (int a3 = -pf; a3 <= pf; a3++) {
                    const bool positive = a1 > 0 || (a1 == 0 && (a2 > 0 || (a2 == 0 && a3 > 0)));
                    if (!positive) continue;
                    al.push_back(int4{a1, a2, a3, 0});
                    const float w2 = (float)(2.0 * cf[((size_t)std::abs(a1) * q + std::abs(a2)) * q + std::abs(a3)]);
                    sg.push_back(w2);
                    sg.push_back(w2);
                }
        f->nh = (int)al.size();
        f->R = 1 + 2 * f->nh;
        f->Rp = (f->R + 3) / 4 * 4;
        sg.resize(f->Rp, 0.0f);
        CIA_TRY(dupload(p, &f->alpha, al.data(), al.size()));
    } else if (f->basis == CIA_BASIS_LEARNED) {
        f->R = f->Rp = c->rank;
        const ParamOffsets po = param_offsets(f->R);
        const std::vector<float> init = initial_params(f->R, 0xC1A0ull);
        CIA_TRY(dupload(p, &f->params, init.data(), init.size()));
        CIA_TRY(dalloc(p, &f->m1, po.total));
        CIA_TRY(dalloc(p, &f->m2, po.total));
        CIA_TRY(dalloc(p, &f->grad, po.total));
        CIA_HIP(hipMemset(f->m1, 0, sizeof(float) * po.total));
        CIA_HIP(hipMemset(f->m2, 0, sizeof(float) * po.total));
        CIA_TRY(dalloc(p, &f->w2b, (size_t)HID * HID));
        CIA_TRY(dalloc(p, &f->w3b, (size_t)f->R * HID));
        flock_bf16_copies<<<grid_for(HID * HID, 256), 256>>>(f->params, f->R, f->w2b, f->w3b);
        CIA_HIP(hipGetLastError());
        f->sgn = f->params + po.sgn;  // signs live in the parameter vector
        const double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        set_box(f, lo, hi);
    }
    if (f->basis == CIA_BASIS_FOURIER) CIA_TRY(dupload(p, &f->sgn, sg.data(), sg.size()));
    if (f->basis != CIA_BASIS_EXACT) {
        CIA_TRY(dalloc(p, &f->F, (size_t)n * f->Rp));
        CIA_TRY(dalloc(p, &f->Q, (size_t)std::max(1, f->ncomm) * f->Rp * 4));
    }
    CIA_TRY(dalloc(p, &f->fb, (size_t)std::max(1, f->ncomm)));
    if (f->judge) CIA_TRY(dalloc(p, &f->judge_es, (size_t)std::max(1, f->ncomm) * JUDGE_SAMPLES));
    if (f->ncomm > 0) {
        flock_fill_i32<<<grid_for(f->ncomm, 256), 256>>>(f->fb, f->ncomm, f->basis == CIA_BASIS_EXACT ? 1 : 0);
        CIA_HIP(hipGetLastError());
    }

    // chunks: <= 256 rows of one community, staged in LDS when it fits
    int dev_lds = 0;
    CIA_HIP(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
    const size_t cap = std::min(STAGE_LDS_CAP, (size_t)dev_lds);
    std::vector<FlockChunk> ch;
    size_t lds = 0, lds_ex = 0;
    constexpr int32_t SR = 64 / EXACT_RT;   // rows of an S-neg slice (one wavefront)
    static_assert(CHUNK_ROWS <= 256, "chunk rows are numbered by uint8_t");
    std::vector<uint16_t> sneg;
    std::vector<int64_t> sneg_off;
    std::vector<int32_t> sneg_w;
    std::vector<uint8_t> srow(n, 0);
    for (int32_t q = 0; q < p1.ncomm; q++) {
        const int32_t c0 = p1.comm_off[q], lam = p1.comm_off[q + 1] - c0;
        const size_t planes = (((size_t)6 * lam + 3) & ~(size_t)3) * sizeof(float);
        const size_t planes_e = (size_t)6 * (((size_t)lam + 3) & ~(size_t)3) * sizeof(float);   // exact kernel
        const size_t need = planes + (size_t)lam * (f->basis == CIA_BASIS_EXACT ? 0 : f->Rp) * sizeof(float);
        const int staged = need <= cap ? 1 : 0;
        if (staged) lds = std::max(lds, need);
        const bool staged_e = planes_e <= cap;   // flock_exact_kernel stages the planes
        if (staged_e) lds_ex = std::max(lds_ex, planes_e);
        for (int32_t r = 0; r < lam; r += CHUNK_ROWS) {
            const int32_t rows = std::min(CHUNK_ROWS, lam - r);
            int32_t sbase = -1;
            if (staged_e) {
                // the chunk's rows by decreasing S-neg length (stable), then
                // S-neg slices of SR of them: entry k of the slice's rows together
                const int64_t rw0 = (int64_t)c0 + r;
                auto len = [&](int32_t t) { return p1.negptr[rw0 + t + 1] - p1.negptr[rw0 + t]; };
                std::vector<int32_t> ord(rows);
                std::iota(ord.begin(), ord.end(), 0);
                std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return len(x) > len(y); });
                for (int32_t t = 0; t < rows; t++) srow[rw0 + t] = (uint8_t)ord[t];
                sbase = (int32_t)sneg_w.size();
                for (int32_t s0 = 0; s0 < rows; s0 += SR) {
                    const int32_t rs = std::min(SR, rows - s0);
                    int64_t w = 0;
                    for (int32_t u = 0; u < rs; u++) w = std::max(w, len(ord[s0 + u]));
                    sneg_off.push_back((int64_t)sneg.size());
                    sneg_w.push_back((int32_t)w);
                    for (int64_t k = 0; k < w; k++)
                        for (int32_t u = 0; u < SR; u++) {
                            const bool in = u < rs && k < len(ord[s0 + u]);
                            sneg.push_back(in ? (uint16_t)p1.neg_local[p1.negptr[rw0 + ord[s0 + u]] + k] : (uint16_t)0);
                        }
                }
            }
            ch.push_back(FlockChunk{c0 + r, rows, q, staged, sbase});
        }
    }
    for (int64_t r = f->nassigned; r < n; r += CHUNK_ROWS)
        ch.push_back(FlockChunk{(int32_t)r, (int32_t)std::min<int64_t>(CHUNK_ROWS, n - r), -1, 0, -1});
    if (!sneg_w.empty()) {
        if (sneg.empty()) sneg.push_back(0);   // every slice of width 0
        CIA_TRY(dupload(p, &f->sneg, sneg.data(), sneg.size()));
        CIA_TRY(dupload(p, &f->sneg_off, sneg_off.data(), sneg_off.size()));
        CIA_TRY(dupload(p, &f->sneg_w, sneg_w.data(), sneg_w.size()));
        CIA_TRY(dupload(p, &f->srow, srow.data(), srow.size()));
    }
    f->nchunks = (int)ch.size();
    f->lds_bytes = lds;
    f->lds_exact = lds_ex;
    if (!ch.empty()) CIA_TRY(dupload(p, &f->chunks, ch.data(), ch.size()));
    // the limit is raised to the staging cap (not to this plan's need), so
    // plans of other sizes never lower it for one another
    if (lds > 64 * 1024 || lds_ex > 64 * 1024) {
        hipError_t e = hipSuccess;
        switch (f->Rp) {
            case 16: e = hipFuncSetAttribute((const void *)flock_stage_kernel<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap); break;
            case 28: e = hipFuncSetAttribute((const void *)flock_stage_kernel<28>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap); break;
            case 32: e = hipFuncSetAttribute((const void *)flock_stage_kernel<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap); break;
            case 48: e = hipFuncSetAttribute((const void *)flock_stage_kernel<48>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap); break;
            default: break;
        }
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)flock_stage_kernel<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)flock_exact_kernel<EXACT_RT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(CIA_EHIP, "cannot raise the LDS limit of the flock stage kernel to %zu bytes", cap);
        }
    }
    info.nunits = f->nchunks;
    info.p = f->basis == CIA_BASIS_FOURIER ? f->fp : f->R;
    // algorithmic bytes: 6 planes read and written, row pointers, S entries,
    // the features written and read once, the E1 sums
    const double feat = f->basis == CIA_BASIS_EXACT ? 0.0 : (double)n * f->Rp * 4 * 2;
    info.bytes_per_rhs = (double)n * (24 + 24 + 16) + 4.0 * (info.nnz_neg + info.nnz_pos) + feat;
    info.bytes_per_stage = info.bytes_per_rhs + (double)n * 24 * 2;
    CIA_HIP(hipDeviceSynchronize());
    return CIA_OK;
}

cia_status flock_rhs(cia_plan *p, const void *state, void *dstate, hipStream_t s) {
    FlockState *f = p->flock;
    const int64_t n = p->n;
    CIA_TRY(timing_begin(p, s, KK_AUX));
    flock_permute_in<<<grid_for(n, 256), 256, 0, s>>>(static_cast<const float *>(state), f->perm, n, f->Y[0]);
    CIA_HIP(hipGetLastError());
    CIA_TRY(timing_end(p, s));
    CIA_TRY(ensure_trained(p, f->Y[0], s));
    CIA_TRY(run_observables(p, f->Y[0], true, s));
    FlockArgs a = base_args(p);
    a.Ys = f->Y[0];
    a.out = static_cast<float *>(dstate);
    a.mode = 0;
    return launch_stage(p, a, s);
}

cia_status flock_integrate(cia_plan *p, void *state, double dt, int64_t steps, hipStream_t s) {
    FlockState *f = p->flock;
    const int64_t n = p->n;
    CIA_TRY(timing_begin(p, s, KK_AUX));
    flock_permute_in<<<grid_for(n, 256), 256, 0, s>>>(static_cast<const float *>(state), f->perm, n, f->Y[0]);
    CIA_HIP(hipGetLastError());
    CIA_TRY(timing_end(p, s));
    CIA_TRY(ensure_trained(p, f->Y[0], s));
    FlockArgs a = base_args(p);
    int cur = 0;  // Euler: index of the current state buffer
    for (int64_t step = 0; step < steps; step++) {
        if (p->stepper == CIA_EULER) {
            a.Ys = f->Y[cur];
            a.Ynext = f->Y[cur ^ 1];
            a.mode = 2;
            a.cdt = (float)dt;
            CIA_TRY(run_observables(p, a.Ys, true, s));
            CIA_TRY(launch_stage(p, a, s));
            cur ^= 1;
            continue;
        }
        static const float cnext[3] = {0.5f, 0.5f, 1.0f};
        for (int st = 0; st < 4; st++) {
            a.Ys = st == 0 ? f->Y[0] : (st == 2 ? f->Y[2] : f->Y[1]);
            a.Ynext = st == 0 ? f->Y[1] : (st == 1 ? f->Y[2] : f->Y[1]);
            if (st == 3) a.Ynext = nullptr;
            a.Y0 = f->Y[0];
            a.acc = f->acc;
            a.stage = st;
            a.mode = 1;
            a.cdt = st < 3 ? (float)(cnext[st] * dt) : 0.f;
            a.dt6 = (float)(dt / 6.0);
            CIA_TRY(run_observables(p, a.Ys, st == 0, s));
            CIA_TRY(launch_stage(p, a, s));
        }
    }
    CIA_TRY(timing_begin(p, s, KK_AUX));
    flock_permute_out<<<grid_for(n, 256), 256, 0, s>>>(f->Y[p->stepper == CIA_EULER ? cur : 0], f->perm, n,
                                                       static_cast<float *>(state));
    CIA_HIP(hipGetLastError());
    CIA_TRY(timing_end(p, s));
    return CIA_OK;
}

void flock_free(cia_plan *p) {
    delete p->flock;
    p->flock = nullptr;
}

// ---- learned-basis entry points ----

static cia_status need_learned(cia_plan *p) {
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    if (p->model != CIA_MODEL_FLOCK || !p->flock || p->flock->basis == CIA_BASIS_EXACT)
        return set_error(CIA_EINVAL, "plan has no separable flock basis");
    return CIA_OK;
}

cia_status flock_judge_count(cia_plan *p, int32_t *count) {
    *count = 0;
    FlockState *f = p->flock;
    if (!f || f->ncomm == 0 || !f->fb) return CIA_OK;
    std::vector<int32_t> h(f->ncomm);
    CIA_HIP(hipDeviceSynchronize());
    CIA_HIP(hipMemcpy(h.data(), f->fb, sizeof(int32_t) * f->ncomm, hipMemcpyDeviceToHost));
    for (int32_t v : h) *count += v != 0;
    return CIA_OK;
}

cia_status flock_basis_features(cia_plan *p, const float *x, int64_t n, float *out, hipStream_t s) {
    CIA_TRY(need_learned(p));
    if (n < 0) return set_error(CIA_EINVAL, "n = %lld", (long long)n);
    if (n == 0) return CIA_OK;
    if (!x || !out) return set_error(CIA_EINVAL, "x/out is NULL");
    return run_features(p, x, n, out, s);
}

cia_status flock_basis_set_params(cia_plan *p, const float *params, int64_t count, const double lo[3],
                                  const double hi[3]) {
    CIA_TRY(need_learned(p));
    FlockState *f = p->flock;
    if (f->basis != CIA_BASIS_LEARNED) return set_error(CIA_EINVAL, "plan's basis is not learned");
    const ParamOffsets po = param_offsets(f->R);
    if (!params || count != po.total)
        return set_error(CIA_EINVAL, "params: need %d values, got %lld", po.total, (long long)count);
    for (int d = 0; d < 3; d++)
        if (!(hi[d] > lo[d]) || !std::isfinite(lo[d]) || !std::isfinite(hi[d]))
            return set_error(CIA_EINVAL, "input box: need lo < hi in every coordinate");
    CIA_HIP(hipDeviceSynchronize());
    CIA_HIP(hipMemcpy(f->params, params, sizeof(float) * po.total, hipMemcpyHostToDevice));
    CIA_HIP(hipMemset(f->m1, 0, sizeof(float) * po.total));
    CIA_HIP(hipMemset(f->m2, 0, sizeof(float) * po.total));
    f->adam_t = 0;
    flock_bf16_copies<<<grid_for(HID * HID, 256), 256>>>(f->params, f->R, f->w2b, f->w3b);
    CIA_HIP(hipGetLastError());
    CIA_HIP(hipDeviceSynchronize());
    set_box(f, lo, hi);
    f->trained = true;
    return CIA_OK;
}

cia_status flock_basis_get_params(cia_plan *p, float *params, int64_t count, double lo[3], double hi[3]) {
    CIA_TRY(need_learned(p));
    FlockState *f = p->flock;
    if (f->basis != CIA_BASIS_LEARNED) return set_error(CIA_EINVAL, "plan's basis is not learned");
    const ParamOffsets po = param_offsets(f->R);
    if (!params || count != po.total)
        return set_error(CIA_EINVAL, "params: need %d values, got %lld", po.total, (long long)count);
    CIA_HIP(hipDeviceSynchronize());
    CIA_HIP(hipMemcpy(params, f->params, sizeof(float) * po.total, hipMemcpyDeviceToHost));
    for (int d = 0; d < 3; d++) {
        if (lo) lo[d] = f->lo[d];
        if (hi) hi[d] = f->hi[d];
    }
    return CIA_OK;
}

cia_status flock_basis_train(cia_plan *p, const void *state, int32_t iters, uint64_t seed, double *loss_trace,
                             hipStream_t s) {
    CIA_TRY(need_learned(p));
    FlockState *f = p->flock;
    if (f->basis != CIA_BASIS_LEARNED) return set_error(CIA_EINVAL, "plan's basis is not learned");
    if (!state) return set_error(CIA_EINVAL, "state is NULL");
    if (iters < 0) return set_error(CIA_EINVAL, "iters = %d", iters);
    flock_permute_in<<<grid_for(p->n, 256), 256, 0, s>>>(static_cast<const float *>(state), f->perm, p->n, f->Y[0]);
    CIA_HIP(hipGetLastError());
    return train(p, f->Y[0], iters, seed, loss_trace, s);
}

cia_status flock_basis_loss_grad(cia_plan *p, const float *a, const float *b, const float *t, int64_t P,
                                 float *grad, double *loss, hipStream_t s) {
    CIA_TRY(need_learned(p));
    FlockState *f = p->flock;
    if (f->basis != CIA_BASIS_LEARNED) return set_error(CIA_EINVAL, "plan's basis is not learned");
    if (P < 1 || P > (int64_t)1 << 24) return set_error(CIA_EINVAL, "pairs = %lld", (long long)P);
    if (!a || !b || !t || !grad) return set_error(CIA_EINVAL, "NULL buffer");
    CIA_TRY(ensure_train_buffers(p, P));
    CIA_TRY(loss_grad(p, a, b, t, (int)P, grad, f->loss1, s));
    if (loss) {
        CIA_HIP(hipMemcpyAsync(loss, f->loss1, sizeof(double), hipMemcpyDeviceToHost, s));
        CIA_HIP(hipStreamSynchronize(s));
    }
    return CIA_OK;
}

int64_t flock_param_count(int32_t rank) { return param_offsets(rank).total; }

}  // namespace cia
