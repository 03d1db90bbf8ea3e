/*
 * IPPO actor-critic kernels for gfx950: policy forward with sampling, GAE, and the fused
 * clipped-PPO forward + backward with activation recomputation.
 *
 * Each agent type has its own network (arXiv 2511.02136, Sec. 4.2: independent PPO with
 * separate weights per type): an MLP 40 -> 256 -> 256 -> (9 logits + 1 value), tanh,
 * fp32.  The dense products run on MFMA (v_mfma_f32_16x16x4f32): a wavefront computes
 * 16x16 output tiles; for lane l, the A operand is A[l%16][k0 + l/16], the B operand
 * B[k0 + l/16][l%16], and accumulator element i is C[4*(l/16) + i][l%16].
 *
 * Parameter layout (flat fp32): W1 [40][256] (input-major), b1 [256], W2 [256][256],
 * b2 [256], W3 [256][10], b3 [10]  (78,858 values).
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "lob.h"
#include "lob_device.h"

#pragma clang fp contract(off)

namespace ippo {

using lobk::hash4;
using lobk::uni;

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int IN = LOB_OBS_DIM, HID = 256, OUT = 10, OUTP = 16;
constexpr int O_W1 = 0, O_B1 = O_W1 + IN * HID, O_W2 = O_B1 + HID, O_B2 = O_W2 + HID * HID, O_W3 = O_B2 + HID,
              O_B3 = O_W3 + HID * OUT, NPARAM = O_B3 + OUT;
static_assert(NPARAM == 78858, "parameter count");
constexpr int PW = NPARAM + 6; /* per-workgroup partial: gradient, the 4 loss sums, 2 floats of padding
                                  (a multiple of 4 floats: partials are summed in 16-byte loads) */
constexpr int PPO_WGS = 256; /* workgroups of the fused PPO kernel */
constexpr int64_t PARAM_COPY_BYTES = NPARAM * 4 + 16; /* workspace room for an aligned parameter copy */
constexpr int64_t W2T_BYTES = (int64_t)HID * HID * 4 + 16;  /* workspace room for W2 transposed (aligned) */

constexpr int TR = 64;          /* samples per workgroup tile */
/* waves per workgroup: four per SIMD (the LDS tile allows one workgroup per CU), so the
 * address arithmetic and loads of some waves overlap the MFMAs of others (one wave per
 * SIMD left the matrix pipe idle 60% of the time; two per SIMD took the fused call from
 * 1.14 to 1.02 ms, four to 1.00 ms) */
constexpr int NW = 16, NTH = 64 * NW;
constexpr int CW = HID / NW, CT = CW / 16; /* hidden columns per wave, in 16-wide tiles */
constexpr int RT = CT;                     /* 16-row tiles per wave over the 256 hidden rows */
constexpr int XS = 52;          /* LDS row stride of the input tile (cols 40..51 zero) */
constexpr int IN1 = 48;         /* layer-1 depth: IN rounded up to a multiple of 16 */
constexpr int HS = 260;         /* LDS row stride of hidden tiles */
constexpr int OS = 17;          /* LDS row stride of the output tile */
constexpr int LDS_FLOATS = TR * XS + 2 * TR * HS + TR * OS;
constexpr int TRP = 32;         /* samples per workgroup tile of the policy forward */
constexpr int LDS_FLOATS_P = TRP * XS + 2 * TRP * HS + TRP * OS;
constexpr uint64_t DOM_POLICY = 0x504F4C4943ULL; /* "POLIC" */

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 zero4() { return floatx4{0.f, 0.f, 0.f, 0.f}; }

/* acc[mt][nt] += A[r0+16mt .. +16][0..K) * B[0..K)[c0+16nt .. +16]; A(i, k), B(k, j) are
 * accessors; K a multiple of 4.  Software-pipelined GEMM_DEPTH steps deep: the operands
 * of step k + 4 GEMM_DEPTH are loaded right after the MFMAs of step k are issued, so
 * their latency (LDS, or L2 for weights) is covered by the MFMAs of the steps between,
 * even with one wave per SIMD; loads past the end re-read the last step (in bounds). */
constexpr int GEMM_DEPTH = 2;
template <int MT, int NT, class FA, class FB>
__device__ __forceinline__ void gemm(floatx4 (&acc)[MT][NT], int K, int r0, int c0, FA A, FB B) {
    constexpr int D = GEMM_DEPTH;
    const int l = (int)(threadIdx.x & 63);
    const int li = l & 15, lk = l >> 4;
    const int kl = K - 4; /* the last step */
    float a[D][MT], b[D][NT];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        const int k = min(4 * s, kl);
#pragma unroll
        for (int m = 0; m < MT; ++m) a[s][m] = A(r0 + 16 * m + li, k + lk);
#pragma unroll
        for (int n = 0; n < NT; ++n) b[s][n] = B(k + lk, c0 + 16 * n + li);
    }
    for (int k0 = 0; k0 < K; k0 += 4 * D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            if (k0 + 4 * s < K) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n) acc[m][n] = mfma(a[s][m], b[s][n], acc[m][n]);
                const int kn = min(k0 + 4 * s + 4 * D, kl);
#pragma unroll
                for (int m = 0; m < MT; ++m) a[s][m] = A(r0 + 16 * m + li, kn + lk);
#pragma unroll
                for (int n = 0; n < NT; ++n) b[s][n] = B(kn + lk, c0 + 16 * n + li);
            }
        }
    }
}

/* The same product with K a multiple of 16 and k permuted inside each block of 16: in
 * MFMA step t of the block at k0, lane l supplies k = k0 + 4(l/16) + t for both operands
 * (only the order of the additions changes).  A lane's four k values are then
 * consecutive, so an operand stored k-contiguous arrives in one 16-byte load.
 * A4(i, kb) / B4(kb, j) return the operand at k = kb .. kb+3; one block is prefetched. */
template <int MT, int NT, class FA, class FB>
__device__ __forceinline__ void gemm16(floatx4 (&acc)[MT][NT], int K, int r0, int c0, FA A4, FB B4) {
    const int l = (int)(threadIdx.x & 63);
    const int li = l & 15, kq = 4 * (l >> 4);
    floatx4 a[MT], b[NT];
#pragma unroll
    for (int m = 0; m < MT; ++m) a[m] = A4(r0 + 16 * m + li, kq);
#pragma unroll
    for (int n = 0; n < NT; ++n) b[n] = B4(kq, c0 + 16 * n + li);
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int kn = min(k0 + 16, K - 16) + kq; /* past the end: the last block again */
        floatx4 an[MT], bn[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) an[m] = A4(r0 + 16 * m + li, kn);
#pragma unroll
        for (int n = 0; n < NT; ++n) bn[n] = B4(kn, c0 + 16 * n + li);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[m][n] = mfma(a[m][t], b[n][t], acc[m][n]);
#pragma unroll
        for (int m = 0; m < MT; ++m) a[m] = an[m];
#pragma unroll
        for (int n = 0; n < NT; ++n) b[n] = bn[n];
    }
}

/* gemm16 with PF blocks of 16 k in flight: a lane's operands for the next PF blocks are
 * loaded while the current block's MFMAs run, so a weight operand read from L2 (the
 * recurrent network's per-step products) waits once per PF blocks rather than once per
 * block.  K a multiple of 16. */
template <int MT, int NT, int PF, class FA, class FB>
__device__ __forceinline__ void gemm16p(floatx4 (&acc)[MT][NT], int K, int r0, int c0, FA A4, FB B4) {
    const int l = (int)(threadIdx.x & 63);
    const int li = l & 15, kq = 4 * (l >> 4);
    const int nb = K / 16;
    floatx4 a[PF][MT], b[PF][NT];
#pragma unroll
    for (int s = 0; s < PF; ++s) {
        const int kb = 16 * min(s, nb - 1) + kq;
#pragma unroll
        for (int m = 0; m < MT; ++m) a[s][m] = A4(r0 + 16 * m + li, kb);
#pragma unroll
        for (int n = 0; n < NT; ++n) b[s][n] = B4(kb, c0 + 16 * n + li);
    }
    for (int blk = 0; blk < nb; blk += PF) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            if (blk + s < nb) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int m = 0; m < MT; ++m)
#pragma unroll
                        for (int n = 0; n < NT; ++n) acc[m][n] = mfma(a[s][m][t], b[s][n][t], acc[m][n]);
                const int kn = 16 * min(blk + s + PF, nb - 1) + kq; /* past the end: the last block again */
#pragma unroll
                for (int m = 0; m < MT; ++m) a[s][m] = A4(r0 + 16 * m + li, kn);
#pragma unroll
                for (int n = 0; n < NT; ++n) b[s][n] = B4(kn, c0 + 16 * n + li);
            }
        }
    }
}

/* acc[m][n] += A[rows][0..K) * B[0..K)[c0+16n ..] for the 64 rows from r0 with the rows of
 * the four tiles interleaved: row li of tile m is r0 + 4 li + m.  The four tiles' A
 * operands at one k are then consecutive, so an A stored row-contiguous arrives in one
 * 16-byte load: A4(i0, k) returns A(i0 .. i0+3, k).  Two steps are prefetched. */
template <int NT, class FA, class FB>
__device__ __forceinline__ void gemm_rows4(floatx4 (&acc)[4][NT], int K, int r0, int c0, FA A4, FB B) {
    const int l = (int)(threadIdx.x & 63);
    const int li = l & 15, lk = l >> 4;
    const int kl = K - 4;
    floatx4 a[2];
    float b[2][NT];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        a[s] = A4(r0 + 4 * li, 4 * s + lk);
#pragma unroll
        for (int n = 0; n < NT; ++n) b[s][n] = B(4 * s + lk, c0 + 16 * n + li);
    }
    for (int k0 = 0; k0 < K; k0 += 8) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[m][n] = mfma(a[s][m], b[s][n], acc[m][n]);
            const int kn = min(k0 + 4 * s + 8, kl) + lk;
            a[s] = A4(r0 + 4 * li, kn);
#pragma unroll
            for (int n = 0; n < NT; ++n) b[s][n] = B(kn, c0 + 16 * n + li);
        }
    }
}

__device__ __forceinline__ floatx4 lds4(const float *p) { return *(const floatx4 *)p; }

/* tanh from the exponential, tanh x = 1 - 2 / (e^(2x) + 1), on the hardware 2^x and
 * reciprocal instructions (about 1 ulp each): absolute error about 1e-7 over the whole
 * range (+-1 at the ends: e^(2x) overflows to inf or underflows to 0), against some
 * thirty instructions for the library's tanhf.  The activations enter the backward as
 * 1 - h^2 and the outputs through 256-term sums, so an absolute error of this size
 * stays far inside the kernels' tolerances. */
__device__ __forceinline__ float tanh_exp(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f); /* 2 x log2(e) */
    return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

#define GLOBAL __attribute__((address_space(1)))
#define LOCAL __attribute__((address_space(3)))

/* row / column of accumulator element i of a 16x16 tile held by this lane */
__device__ __forceinline__ int acc_row(int i) { return 4 * ((int)(threadIdx.x & 63) >> 4) + i; }
__device__ __forceinline__ int acc_col() { return (int)(threadIdx.x & 15); }

/* the policy's input scaling of observation feature c (xs null: none) */
__device__ __forceinline__ float obs_in(const float *__restrict__ obs, const float *__restrict__ xs, int64_t i, int c) {
    return xs ? obs[i] * xs[c] : obs[i];
}

/* ---- forward of a tile of R samples (R a multiple of 16, at most 64) into LDS: X (the
 * observations times the input scales xs, when given), H1 = tanh(X W1 + b1),
 * H2 = tanh(H1 W2 + b2), O = H2 W3 + b3 (O cols 10..15 zero) ---- */
template <int R, bool W2T>
__device__ __forceinline__ void forward_tile(const float *__restrict__ P, const float *__restrict__ obs,
                                             const float *__restrict__ xs, int rows, float *X, float *H1, float *H2,
                                             float *O, const float *__restrict__ w2t) {
    constexpr int MT = R / 16; /* 16-row tiles per wave */
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < R * XS; i += blockDim.x) {
        const int r = i / XS, c = i % XS;
        X[i] = (r < rows && c < IN) ? obs_in(obs, xs, (int64_t)r * IN + c, c) : 0.f;
    }
    __syncthreads();
    /* layer 1: each wave computes R rows x CW cols */
    {
        floatx4 acc[MT][CT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < CT; ++n) acc[m][n] = zero4();
        /* K = 48: X columns 40..47 are zero and the W1 rows past 40 read as zero */
        gemm16<MT, CT>(acc, IN1, 0, CW * wave, [&](int i, int kb) { return lds4(X + i * XS + kb); },
                      [&](int kb, int j) {
                          floatx4 v;
#pragma unroll
                          for (int t = 0; t < 4; ++t) v[t] = kb + t < IN ? P[O_W1 + (kb + t) * HID + j] : 0.f;
                          return v;
                      });
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < CT; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * m + acc_row(i), c = CW * wave + 16 * n + acc_col();
                    H1[r * HS + c] = tanh_exp(acc[m][n][i] + P[O_B1 + c]);
                }
    }
    __syncthreads();
    /* layer 2 */
    {
        floatx4 acc[MT][CT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < CT; ++n) acc[m][n] = zero4();
        if constexpr (W2T) {
            /* W2 transposed (w2t[j][k]): a lane's four k values in one 16-byte load */
            gemm16<MT, CT>(acc, HID, 0, CW * wave, [&](int i, int kb) { return lds4(H1 + i * HS + kb); },
                          [&](int kb, int j) { return *(const floatx4 *)(w2t + j * HID + kb); });
        } else {
            gemm16<MT, CT>(acc, HID, 0, CW * wave, [&](int i, int kb) { return lds4(H1 + i * HS + kb); },
                          [&](int kb, int j) {
                              floatx4 v;
#pragma unroll
                              for (int t = 0; t < 4; ++t) v[t] = P[O_W2 + (kb + t) * HID + j];
                              return v;
                          });
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < CT; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * m + acc_row(i), c = CW * wave + 16 * n + acc_col();
                    H2[r * HS + c] = tanh_exp(acc[m][n][i] + P[O_B2 + c]);
                }
    }
    __syncthreads();
    /* layer 3: wave w < R/16 computes rows 16w..16w+15, cols 0..15, k permuted in blocks
     * of 16 as in gemm16.  The lane's whole W3 column is loaded first, so the weight loads
     * (from L2) wait once rather than once per block. */
    if (wave < R / 16) {
        const int li = tid & 15, kq = 4 * ((tid & 63) >> 4);
        floatx4 bw[HID / 16];
#pragma unroll
        for (int s = 0; s < HID / 16; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t) bw[s][t] = li < OUT ? P[O_W3 + (16 * s + kq + t) * OUT + li] : 0.f;
        floatx4 acc = zero4();
        const float *hr = H2 + (16 * wave + li) * HS + kq;
#pragma unroll
        for (int s = 0; s < HID / 16; ++s) {
            const floatx4 av = lds4(hr + 16 * s);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma(av[t], bw[s][t], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * wave + acc_row(i), c = acc_col();
            O[r * OS + c] = c < OUT ? acc[i] + P[O_B3 + c] : 0.f;
        }
    }
    __syncthreads();
}

/* ------------------------------------------------------------------------------
 * Policy forward for the rollout: logits, value, a sampled action (Gumbel-max on a
 * counter hash) and its log-probability.  grid (ceil(n/TRP), n_agents), NTH threads.
 * Tiles of 32 samples: the rollout's 4096 envs x 2 agents then give 256 workgroups, one
 * per CU (64-sample tiles left half of the CUs idle).
 * ---------------------------------------------------------------------------- */
/* One sample's head: the first nact of the outputs z are the policy logits, z[9] the
 * value.  Samples an action by Gumbel-max with noise from the counter hash of (seed,
 * agent, action, t, row) and writes it, its log-probability and the value (and the ten
 * outputs when logits is given). */
__device__ __forceinline__ void sample_head(const float *z, int nact, uint64_t seed, int ag, int t, int e,
                                            int32_t *action, float *logp, float *value, float *logits) {
    float m = z[0];
    for (int j = 1; j < nact; ++j) m = fmaxf(m, z[j]);
    float s = 0.f;
    for (int j = 0; j < nact; ++j) s += expf(z[j] - m);
    const float lse = m + logf(s);
    int best = 0;
    float bv = -INFINITY;
    for (int j = 0; j < nact; ++j) {
        const uint64_t h = hash4(seed, DOM_POLICY, (uint64_t)ag << 8 | (uint64_t)j, (uint64_t)t, (uint64_t)e);
        const float u = ((float)(uint32_t)(h >> 40) + 0.5f) * (1.0f / 16777216.0f);
        const float g = -logf(-logf(u));
        const float v = z[j] + g;
        if (v > bv) { bv = v; best = j; }
    }
    *action = best;
    *logp = z[best] - lse;
    *value = z[9];
    if (logits)
        for (int j = 0; j < OUT; ++j) logits[j] = z[j];
}

struct FwdArgs {
    const float *params; /* [A][NPARAM] */
    const float *obs;    /* [A][n][40] */
    const float *obs_scale; /* [40] or null */
    int32_t n, n_agents;
    int32_t n_act[LOB_MAX_AGENTS];
    uint64_t seed;
    const uint64_t *epoch; /* device counter mixed into the seed, or null */
    int32_t t;
    float *logits; /* [A][n][10] or null */
    int32_t *actions;
    float *logp, *value; /* [A][n] */
};

__global__ void __launch_bounds__(NTH) k_policy_forward(FwdArgs a) {
    extern __shared__ float sm[];
    float *X = sm, *H1 = X + TRP * XS, *H2 = H1 + TRP * HS, *O = H2 + TRP * HS;
    const int ag = (int)blockIdx.y;
    const int row0 = (int)blockIdx.x * TRP;
    const int rows = min(TRP, a.n - row0);
    const float *P = a.params + (int64_t)ag * NPARAM;
    forward_tile<TRP, false>(P, a.obs + ((int64_t)ag * a.n + row0) * IN, a.obs_scale, rows, X, H1, H2, O, nullptr);
    const int tid = (int)threadIdx.x;
    if (tid < rows) {
        const uint64_t seed = a.epoch ? a.seed + 0x9E3779B97F4A7C15ULL * a.epoch[0] : a.seed;
        const int64_t o = (int64_t)ag * a.n + row0 + tid;
        sample_head(O + tid * OS, a.n_act[ag], seed, ag, a.t, row0 + tid, a.actions + o, a.logp + o, a.value + o,
                    a.logits ? a.logits + o * OUT : nullptr);
    }
}

/* ------------------------------------------------------------------------------
 * GAE over [T][n]: one thread per column, reverse scan over time.
 * ---------------------------------------------------------------------------- */
__global__ void k_gae(const float *__restrict__ r, const float *__restrict__ v, const uint8_t *__restrict__ d,
                      const float *__restrict__ last_v, int T, int n, float gamma, float lam, float *adv, float *ret) {
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= n) return;
    float nv = last_v[c], na = 0.f;
    for (int t = T - 1; t >= 0; --t) {
        const int64_t i = (int64_t)t * n + c;
        const float nd = d[i] ? 0.f : 1.f;
        const float delta = r[i] + gamma * nv * nd - v[i];
        na = delta + gamma * lam * nd * na;
        adv[i] = na;
        ret[i] = na + v[i];
        nv = v[i];
    }
}

/* ------------------------------------------------------------------------------
 * Fused clipped-PPO loss forward + backward for one minibatch of one network.
 * For each tile of TR samples, a workgroup recomputes the forward in LDS, forms the
 * per-sample gradient of the loss w.r.t. the outputs and back-propagates through the MLP
 * in LDS.  A fixed grid of PPO_WGS workgroups (one per compute unit) strides over the
 * tiles, each summing its tiles' parameter gradients and loss sums into one partial of
 * PW floats: 256 partials (80 MB, within the last-level cache) for any minibatch size,
 * rather than one per tile.
 * ---------------------------------------------------------------------------- */
struct PpoArgs {
    const float *params;
    const float *obs;
    const float *obs_scale; /* [40] or null */
    const int32_t *act;
    const float *logp_old, *adv, *ret, *v_old;
    int32_t m, n_act;
    float clip, c_v, c_e, scale; /* scale = 1 / m */
    float *partial;              /* [grid][PW]: gradient, then loss sums (total, policy, value, entropy) */
    const float *w2t;            /* W2 transposed, [256][256] (workspace) */
};

/* W2 transposed, w2t[j][k] = W2[k][j], for the forward's 16-byte operand loads */
__global__ void k_w2t(const float *__restrict__ P, float *__restrict__ w2t) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < HID * HID) w2t[(i % HID) * HID + i / HID] = P[O_W2 + i];
}

/* One sample's clipped-PPO loss terms from its ten outputs z (logits, then the value) and
 * their gradient w.r.t. z, scaled by `scale` (1 / minibatch samples): policy -min(r A,
 * clip(r, 1-clip, 1+clip) A) with r = exp(logp - logp_old), value 0.5 max((V-R)^2,
 * (V_old + clip(V - V_old) - R)^2), entropy H; lsum = {total, policy, value, entropy}.
 * An action outside [0, nact) counts as action 0, as the env step takes it. */
__device__ __forceinline__ void loss_head(const float *z, int nact, int act, float logp_old, float A, float R,
                                          float vo, float clip, float c_v, float c_e, float scale, float *dz,
                                          float *lsum) {
    float mx = z[0];
    for (int j = 1; j < nact; ++j) mx = fmaxf(mx, z[j]);
    float se = 0.f;
    for (int j = 0; j < nact; ++j) se += expf(z[j] - mx);
    const float lse = mx + logf(se);
    float H = 0.f;
    for (int j = 0; j < nact; ++j) {
        const float lp = z[j] - lse;
        H -= expf(lp) * lp;
    }
    if ((unsigned)act >= (unsigned)nact) act = 0;
    const float logp = z[act] - lse;
    const float ratio = expf(logp - logp_old);
    const float s1 = ratio * A;
    const float rc = fminf(fmaxf(ratio, 1.f - clip), 1.f + clip);
    const float s2 = rc * A;
    const float pol = -fminf(s1, s2);
    const float dlogp = s1 <= s2 ? -A * ratio : 0.f;
    const float v = z[9];
    const float dvv = v - vo;
    const float vc = vo + fminf(fmaxf(dvv, -clip), clip);
    const float l1 = (v - R) * (v - R), l2 = (vc - R) * (vc - R);
    const float val = 0.5f * fmaxf(l1, l2);
    const float dval = l1 >= l2 ? (v - R) : (fabsf(dvv) < clip ? (vc - R) : 0.f);
    for (int j = 0; j < nact; ++j) {
        const float lp = z[j] - lse;
        const float p = expf(lp);
        const float dlp = (j == act ? 1.f : 0.f) - p;
        dz[j] = scale * (dlogp * dlp + c_e * p * (lp + H));
    }
    dz[9] = scale * c_v * dval;
    lsum[0] = pol + c_v * val - c_e * H;
    lsum[1] = pol;
    lsum[2] = val;
    lsum[3] = H;
}

/* One tile of the fused kernel.  first: write the partial G, else add to it (each element
 * is read and rewritten by the lane that wrote it).  A function of its own, not inlined:
 * inside the kernel's tile loop the compiler keeps the per-lane LDS addresses of every
 * unrolled load live across tiles and spills. */
__device__ __noinline__ void ppo_tile(const PpoArgs &a, const GLOBAL float *Pg, GLOBAL float *Gg, const GLOBAL float *obs_g,
                                      LOCAL float *sm, int tile, bool first) {
    /* pointers to global memory and LDS arrive as such (a generic pointer parameter would
     * make every access a flat one, which waits on both the memory and the LDS counter) */
    const float *__restrict__ P = (const float *)Pg;
    float *__restrict__ G = (float *)Gg;
    float *X = (float *)sm, *H1 = X + TR * XS, *H2 = H1 + TR * HS, *O = H2 + TR * HS;
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    {
        const int row0 = tile * TR;
        const int rows = min(TR, a.m - row0);
        auto put = [&](int i, float v) { G[i] = first ? v : G[i] + v; };
        forward_tile<TR, true>(P, (const float *)obs_g + (int64_t)row0 * IN, a.obs_scale, rows, X, H1, H2, O, a.w2t);

        /* per-sample loss and its gradient w.r.t. the 10 outputs (scaled by 1/m) */
        float lsum[4] = {0.f, 0.f, 0.f, 0.f};
        if (tid < TR) {
            float *z = O + tid * OS;
            float dz[OUT];
#pragma unroll
            for (int j = 0; j < OUT; ++j) dz[j] = 0.f;
            if (tid < rows) {
                const int s = row0 + tid;
                loss_head(z, a.n_act, a.act[s], a.logp_old[s], a.adv[s], a.ret[s], a.v_old[s], a.clip, a.c_v, a.c_e,
                          a.scale, dz, lsum);
            }
            /* the output tile now holds dOut (cols 10..15 stay zero) */
            for (int j = 0; j < OUT; ++j) z[j] = dz[j];
        }
        /* loss sums of the tile: wave 0 reduces its 64 lanes */
        if (wave == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v = lsum[q];
                for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
                if (tid == 0) put(NPARAM + q, v);
            }
        }
        __syncthreads();

        /* dW3 = H2^T dOut (256 x 16, cols < 10 kept), db3 = column sums of dOut */
        {
            floatx4 acc[RT][1];
#pragma unroll
            for (int m = 0; m < RT; ++m) acc[m][0] = zero4();
            gemm<RT, 1>(acc, TR, CW * wave, 0, [&](int i, int k) { return H2[k * HS + i]; },
                        [&](int k, int j) { return O[k * OS + j]; });
#pragma unroll
            for (int m = 0; m < RT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = CW * wave + 16 * m + acc_row(i), c = acc_col();
                    if (c < OUT) put(O_W3 + r * OUT + c, acc[m][0][i]);
                }
            if (tid < OUT) {
                float s = 0.f;
                for (int r = 0; r < TR; ++r) s += O[r * OS + tid];
                put(O_B3 + tid, s);
            }
        }
        __syncthreads();
        /* dH2 = (dOut W3^T) * (1 - H2^2), in place of H2 */
        {
            floatx4 acc[4][CT];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n) acc[m][n] = zero4();
            gemm16<4, CT>(acc, OUTP, 0, CW * wave,
                          [&](int i, int kb) {
                              floatx4 v;
#pragma unroll
                              for (int t = 0; t < 4; ++t) v[t] = O[i * OS + kb + t];
                              return v;
                          },
                          [&](int kb, int j) {
                              floatx4 v;
#pragma unroll
                              for (int t = 0; t < 4; ++t) v[t] = kb + t < OUT ? P[O_W3 + j * OUT + kb + t] : 0.f;
                              return v;
                          });
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * m + acc_row(i), c = CW * wave + 16 * n + acc_col();
                        const float h = H2[r * HS + c];
                        H2[r * HS + c] = acc[m][n][i] * (1.f - h * h);
                    }
        }
        __syncthreads();
        /* dW2 = H1^T dH2 (256 x 256) in four passes of 64 x CW per wave; db2 */
        for (int pass = 0; pass < 4; ++pass) {
            floatx4 acc[4][CT];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n) acc[m][n] = zero4();
            const int r0 = 64 * pass, c0 = CW * wave;
            /* the partial of the earlier tiles, loaded before the product so that the
             * MFMAs cover the load latency */
            float prev[4][CT][4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        prev[m][n][i] = first ? 0.f : G[O_W2 + (r0 + 4 * acc_row(i) + m) * HID + c0 + 16 * n + acc_col()];
            gemm_rows4<CT>(acc, TR, r0, c0, [&](int i0, int k) { return lds4(H1 + k * HS + i0); },
                           [&](int k, int j) { return H2[k * HS + j]; });
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = r0 + 4 * acc_row(i) + m, c = c0 + 16 * n + acc_col();
                        G[O_W2 + r * HID + c] = first ? acc[m][n][i] : prev[m][n][i] + acc[m][n][i];
                    }
        }
        if (tid < HID) {
            float s = 0.f;
            for (int r = 0; r < TR; ++r) s += H2[r * HS + tid];
            put(O_B2 + tid, s);
        }
        __syncthreads();
        /* dH1 = (dH2 W2^T) * (1 - H1^2), in place of H1 */
        {
            floatx4 acc[4][CT];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n) acc[m][n] = zero4();
            /* W2 read transposed: a lane's four k values are consecutive in memory (the
             * parameters are 16-byte aligned) */
            gemm16<4, CT>(acc, HID, 0, CW * wave, [&](int i, int kb) { return lds4(H2 + i * HS + kb); },
                          [&](int kb, int j) { return *(const floatx4 *)(P + O_W2 + j * HID + kb); });
            /* each element of H1 is read and rewritten by the lane that owns it */
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * m + acc_row(i), c = CW * wave + 16 * n + acc_col();
                        const float h = H1[r * HS + c];
                        H1[r * HS + c] = acc[m][n][i] * (1.f - h * h);
                    }
        }
        __syncthreads();
        /* dW1 = X^T dH1 (40 x 256, computed as 48 x 256 with zero rows), db1 */
        {
            floatx4 acc[3][CT];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n) acc[m][n] = zero4();
            gemm<3, CT>(acc, TR, 0, CW * wave, [&](int i, int k) { return X[k * XS + i]; },
                        [&](int k, int j) { return H1[k * HS + j]; });
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int n = 0; n < CT; ++n)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * m + acc_row(i), c = CW * wave + 16 * n + acc_col();
                        if (r < IN) put(O_W1 + r * HID + c, acc[m][n][i]);
                    }
            if (tid < HID) {
                float s = 0.f;
                for (int r = 0; r < TR; ++r) s += H1[r * HS + tid];
                put(O_B1 + tid, s);
            }
        }
        __syncthreads(); /* the next tile's forward overwrites the LDS tiles */
    }
}

__global__ void __launch_bounds__(NTH) k_ppo_fwd_bwd(PpoArgs a) {
    extern __shared__ float sm[];
    float *G = a.partial + (int64_t)blockIdx.x * PW;
    const int ntile = (a.m + TR - 1) / TR;
    for (int tile = (int)blockIdx.x; tile < ntile; tile += (int)gridDim.x)
        ppo_tile(a, (const GLOBAL float *)a.params, (GLOBAL float *)G, (const GLOBAL float *)a.obs, (LOCAL float *)sm,
                 tile, tile == (int)blockIdx.x);
}

/* Sum of the per-workgroup partials in a fixed order (deterministic), in two levels:
 * chunk c of RCH consecutive workgroups is summed in workgroup order into sums[c], then
 * the chunk sums in chunk order.  Level 1 keeps 8 loads in flight per thread. */
constexpr int RCH = 64;
__global__ void k_reduce_chunks(const floatx4 *__restrict__ partial, int nwg, int width4, floatx4 *__restrict__ sums) {
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= width4) return;
    const int w0 = (int)blockIdx.y * RCH, w1 = min(nwg, w0 + RCH);
    floatx4 s = zero4();
    int w = w0;
    for (; w + 8 <= w1; w += 8) {
        floatx4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(w + u) * width4 + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; w < w1; ++w) s += partial[(int64_t)w * width4 + j];
    sums[(int64_t)blockIdx.y * width4 + j] = s;
}
/* columns [0, NPARAM) go to grad, the next 4 to loss (the padding is not summed) */
__global__ void k_reduce_final(const float *__restrict__ sums, int nch, float *grad, float *loss) {
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= NPARAM + 4) return;
    float s = 0.f;
    for (int c = 0; c < nch; ++c) s += sums[(int64_t)c * PW + j];
    if (j < NPARAM) grad[j] = s;
    else loss[j - NPARAM] = s;
}

/* ==============================================================================
 * Recurrent (GRU) actor-critic.  The paper trains its agents with a GRU-based network
 * (Sec. 5.2.1), one per agent type (Sec. 4.2); the sizes are a reading:
 *   e_t = tanh(x_t W_e + b_e)                                   40 -> 128
 *   r_t = sigmoid(e_t W_ir + b_ir + h_{t-1} W_hr + b_hr)
 *   u_t = sigmoid(e_t W_iz + b_iz + h_{t-1} W_hz + b_hz)
 *   n_t = tanh(e_t W_in + b_in + r_t * (h_{t-1} W_hn + b_hn))
 *   h_t = (1 - u_t) n_t + u_t h_{t-1}                           hidden state 128
 *   out_t = h_t W_o + b_o                                       9 logits + value
 * with h_{t-1} = 0 at an episode's first step.  Flat parameters: W_e [40][128], b_e,
 * W_i [128][384] (gate columns r | u | n), b_i, W_h [128][384], b_h, W_o [128][10], b_o.
 * Tiles of 16 rows (envs) run every product on v_mfma_f32_16x16x4f32.
 * ============================================================================ */
constexpr int GHD = 128, G3 = 3 * GHD, GIN = 40, GINP = 48;
constexpr int GO_WE = 0, GO_BE = GO_WE + GIN * GHD, GO_WI = GO_BE + GHD, GO_BI = GO_WI + GHD * G3,
              GO_WH = GO_BI + G3, GO_BH = GO_WH + GHD * G3, GO_WO = GO_BH + G3, GO_BO = GO_WO + GHD * OUT,
              GNP = GO_BO + OUT;
static_assert(GNP == LOB_GRU_PARAMS, "GRU parameter count");
constexpr int GPW = GNP + 2;  /* per-workgroup gradient partial, a multiple of 4 floats */
constexpr int TG = 16;        /* rows (envs) per tile */
constexpr int HSG = GHD + 4;  /* LDS row strides */
constexpr int GS = G3 + 4;
constexpr int GRU_STEP_TH = 512, GRU_SEQ_TH = 512, GRU_DW_TH = 1024;
constexpr int GRU_DW_WGS = 256; /* workgroups of the weight-gradient kernel */

__device__ __forceinline__ float sigmoid_exp(float x) {
    /* 1 / (1 + e^-x) on the hardware 2^x and reciprocal instructions */
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-x * 1.4426950408889634f));
}

/* the gates and the new state: HN = (1 - u) n + u HP; with keep, GI's three column
 * blocks are overwritten by r, u and n */
__device__ __forceinline__ void gru_update(float *GI, const float *GH, const float *HP, float *HN, int tid, int nth,
                                           bool keep, int nrow = TG) {
    for (int i = tid; i < nrow * GHD; i += nth) {
        const int r = i / GHD, j = i % GHD;
        const float *gi = GI + r * GS, *gh = GH + r * GS;
        const float rr = sigmoid_exp(gi[j] + gh[j]);
        const float u = sigmoid_exp(gi[GHD + j] + gh[GHD + j]);
        const float nn = tanh_exp(gi[2 * GHD + j] + rr * gh[2 * GHD + j]);
        HN[r * HSG + j] = (1.f - u) * nn + u * HP[r * HSG + j];
        if (keep) {
            GI[r * GS + j] = rr;
            GI[r * GS + GHD + j] = u;
            GI[r * GS + 2 * GHD + j] = nn;
        }
    }
}

/* The sequence kernel's weights, prepared in its workspace so that every product reads
 * its weight operand k-contiguous in 16-byte loads: W_e^T [128][48] (k >= 40 zero),
 * W_i^T and W_h^T [384][128] (the gate products), W_i and W_h [128][384] (the backward
 * products, 16-byte aligned copies), W_o^T [16][128] and W_o [128][16] (cols >= 10 zero). */
struct GruW {
    const float *WeT, *WiT, *WhT, *Wi, *Wh, *WoT, *WoP;
};
constexpr int GW_WET = 0, GW_WIT = GW_WET + GHD * GINP, GW_WHT = GW_WIT + G3 * GHD, GW_WI = GW_WHT + G3 * GHD,
              GW_WH = GW_WI + GHD * G3, GW_WOT = GW_WH + GHD * G3, GW_WOP = GW_WOT + 16 * GHD,
              GW_FLOATS = GW_WOP + GHD * 16;
static_assert(GW_FLOATS % 4 == 0, "prepared weights keep 16-byte alignment");

__global__ void k_gru_prep(const float *__restrict__ P, float *W) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < GHD * GINP) {
        const int j = i / GINP, k = i % GINP;
        W[GW_WET + i] = k < GIN ? P[GO_WE + k * GHD + j] : 0.f;
    }
    if (i < G3 * GHD) {
        const int g = i / GHD, e = i % GHD; /* W^T[g][e] = W[e][g] */
        W[GW_WIT + i] = P[GO_WI + e * G3 + g];
        W[GW_WHT + i] = P[GO_WH + e * G3 + g];
        W[GW_WI + i] = P[GO_WI + i];
        W[GW_WH + i] = P[GO_WH + i];
    }
    if (i < 16 * GHD) {
        const int j = i / GHD, k = i % GHD;
        W[GW_WOT + i] = j < OUT ? P[GO_WO + k * OUT + j] : 0.f;
        const int jj = i / 16, kk = i % 16;
        W[GW_WOP + i] = kk < OUT ? P[GO_WO + jj * OUT + kk] : 0.f;
    }
}

constexpr int GPF = 4; /* 16-k blocks in flight in the sequence kernel's products */

__device__ __forceinline__ floatx4 gload4(const float *p) { return *(const floatx4 *)p; }

/* ---- one step of the rollout: grid (ceil(n / 32), n_agents), GRU_STEP_TH threads.  A
 * workgroup takes 32 envs of one agent (two row tiles), so every weight it streams from
 * the caches serves 32 rows; the state products on v_mfma_f32_16x16x4f32, the cell, the
 * head and the sampling. ---- */
struct GruStepArgs {
    const float *params;  /* [A][GNP] */
    const float *obs;     /* [A][n][40] */
    const float *obs_scale; /* [40] or null */
    const float *h_in;    /* [A][n][128] */
    float *h_out;         /* [A][n][128], may be h_in */
    const uint8_t *start; /* [n] or null: 1 = the episode starts at this step (h_{t-1} = 0) */
    int32_t n;
    int32_t n_act[LOB_MAX_AGENTS];
    uint64_t seed;
    const uint64_t *epoch;
    int32_t t;
    float *logits;
    int32_t *actions;
    float *logp, *value;
};
constexpr int TS = 32; /* envs per workgroup of the rollout step */
constexpr int GRU_STEP_LDS = TS * (XS + 3 * HSG + 2 * GS + OS);
static_assert(GRU_STEP_TH == 512, "8 waves: 8 column tiles of 128, 48 of the two gate products");

__global__ void __launch_bounds__(GRU_STEP_TH) k_gru_step(GruStepArgs a) {
    extern __shared__ float sm[];
    float *X = sm, *E = X + TS * XS, *HP = E + TS * HSG, *HN = HP + TS * HSG, *GI = HN + TS * HSG,
          *GH = GI + TS * GS, *O = GH + TS * GS;
    const int ag = (int)blockIdx.y, row0 = (int)blockIdx.x * TS, rows = min(TS, a.n - row0);
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    const float *P = a.params + (int64_t)ag * GNP;
    const int64_t base = (int64_t)ag * a.n + row0;
    for (int i = tid; i < TS * XS; i += GRU_STEP_TH) {
        const int r = i / XS, c = i % XS;
        X[i] = (r < rows && c < GIN) ? obs_in(a.obs, a.obs_scale, (base + r) * GIN + c, c) : 0.f;
    }
    for (int i = tid; i < TS * GHD; i += GRU_STEP_TH) {
        const int r = i / GHD, c = i % GHD;
        const bool zero = r >= rows || (a.start && a.start[row0 + r]);
        HP[r * HSG + c] = zero ? 0.f : a.h_in[(base + r) * GHD + c];
    }
    __syncthreads();
    {
        /* E = tanh(X W_e + b_e): column tile `wave` of both row tiles */
        floatx4 acc[2][1] = {{zero4()}, {zero4()}};
        gemm<2, 1>(acc, GINP, 0, 16 * wave, [&](int i, int k) { return X[i * XS + k]; },
                   [&](int k, int j) { return k < GIN ? P[GO_WE + k * GHD + j] : 0.f; });
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * mt + acc_row(i), c = 16 * wave + acc_col();
                E[r * HSG + c] = tanh_exp(acc[mt][0][i] + P[GO_BE + c]);
            }
    }
    __syncthreads();
    /* GI = E W_i + b_i and GH = HP W_h + b_h: column tiles 6 wave .. 6 wave + 5 of the 48
     * (24 of each product; a wave's tiles never straddle the two), three at a time */
    for (int c3 = 0; c3 < 6; c3 += 3) {
        const int ct0 = 6 * wave + c3;
        const bool hh = ct0 >= G3 / 16;
        const int c0 = 16 * (hh ? ct0 - G3 / 16 : ct0);
        const float *A = hh ? HP : E;
        const float *W = P + (hh ? GO_WH : GO_WI);
        floatx4 acc[2][3];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int n = 0; n < 3; ++n) acc[mt][n] = zero4();
        gemm<2, 3>(acc, GHD, 0, c0, [&](int i, int k) { return A[i * HSG + k]; },
                   [&](int k, int j) { return W[k * G3 + j]; });
        float *D = hh ? GH : GI;
        const float *bias = P + (hh ? GO_BH : GO_BI);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int n = 0; n < 3; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * mt + acc_row(i), c = c0 + 16 * n + acc_col();
                    D[r * GS + c] = acc[mt][n][i] + bias[c];
                }
    }
    __syncthreads();
    gru_update(GI, GH, HP, HN, tid, GRU_STEP_TH, false, TS);
    __syncthreads();
    for (int i = tid; i < TS * GHD; i += GRU_STEP_TH) {
        const int r = i / GHD, c = i % GHD;
        if (r < rows) a.h_out[(base + r) * GHD + c] = HN[r * HSG + c];
    }
    if (wave < 2) {
        /* O = HN W_o + b_o (cols 10..15 zero): row tile `wave` */
        floatx4 acc[1][1] = {{zero4()}};
        gemm<1, 1>(acc, GHD, 16 * wave, 0, [&](int i, int k) { return HN[i * HSG + k]; },
                   [&](int k, int j) { return j < OUT ? P[GO_WO + k * OUT + j] : 0.f; });
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * wave + acc_row(i), c = acc_col();
            O[r * OS + c] = c < OUT ? acc[0][0][i] + P[GO_BO + c] : 0.f;
        }
    }
    __syncthreads();
    if (tid < rows) {
        const uint64_t seed = a.epoch ? a.seed + 0x9E3779B97F4A7C15ULL * a.epoch[0] : a.seed;
        const int64_t o = base + tid;
        sample_head(O + tid * OS, a.n_act[ag], seed, ag, a.t, row0 + tid, a.actions + o, a.logp + o, a.value + o,
                    a.logits ? a.logits + o * OUT : nullptr);
    }
}

/* ---- clipped-PPO loss over whole sequences, forward and backward through time ----
 * Only the recurrence h_{t-1} -> h_t is sequential; everything that does not depend on
 * the previous state runs as batched products over all T m samples (s = t m + env):
 *   k_gru_in   E = tanh(X W_e + b_e) and GI = E W_i + b_i of every sample;
 *   k_gru_fwd  one workgroup per tile of 16 sequences: GH = h_{t-1} W_h + b_h and the
 *              cell, t = 0 .. T-1, keeping only the hidden states (HS [T+1][m][128],
 *              HS[0] = h0, HS[t] = h_{t-1} as stored before an episode start zeroes it);
 *   k_gru_head the outputs h_t W_o + b_o, the per-sample loss terms and their gradient dO;
 *   k_gru_bwd  one workgroup per tile: t = T-1 .. 0, GH recomputed from h_{t-1}, dh
 *              (carried from step t+1, plus dO W_o^T) taken back through the cell into the
 *              gate pre-activation gradients DGI, DGH (DGI overwrites the sample's GI),
 *              and dh_{t-1} = u dh + DGH W_h^T;
 *   k_gru_de   the embedding pre-activation gradient DE = (DGI W_i^T) (1 - E^2);
 * then k_gru_dw forms the weight gradients over all samples. */
struct GruSeqArgs {
    const float *params, *obs;  /* obs [T][m][40] */
    const float *obs_scale;     /* [40] or null */
    const uint8_t *start;       /* [T][m] */
    const float *h0;            /* [m][128] */
    const int32_t *act;
    const float *logp_old, *adv, *ret, *v_old; /* [T][m] */
    int32_t T, m, n_act;
    float clip, c_v, c_e, scale; /* scale = 1 / (T m) */
    float *HS, *E, *DGI, *DGH, *DE, *DO, *LS; /* workspace */
    GruW w;                     /* prepared weights (workspace) */
};
constexpr int TI = 64;          /* samples per workgroup of the batched kernels */
constexpr int GRU_IN_TH = 512, GRU_HEAD_TH = 256;
constexpr int GRU_IN_LDS = TI * (XS + HSG);                   /* X and E tiles */
constexpr int GRU_FWD_LDS = TG * (HSG + 3 * GS);               /* HP, GH, two GI buffers */
constexpr int GRU_BWD_LDS = TG * (4 * HSG + 4 * GS + 32) + 2 * TG; /* DH, DHO, GH, DGH; two of HP, GI, dO, ST */
constexpr int GRU_HEAD_LDS = TI * (OS + 4);                    /* outputs, loss terms */
constexpr int DES = G3 + 4;                                    /* LDS row stride of k_gru_de's DGI tile */
constexpr int GRU_DE_LDS = TI * DES;
static_assert(GRU_IN_TH == 512 && GRU_SEQ_TH == 512, "8 waves: 8 column tiles of 128, 24 of 384");

/* E and GI of the 64 samples from s0 = 64 blockIdx.x (the last workgroup may have fewer) */
__global__ void __launch_bounds__(GRU_IN_TH) k_gru_in(GruSeqArgs a) {
    extern __shared__ float sm[];
    float *X = sm, *E = X + TI * XS;
    const int64_t S = (int64_t)a.T * a.m, s0 = (int64_t)blockIdx.x * TI;
    const int rows = (int)min((int64_t)TI, S - s0);
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < TI * XS; i += GRU_IN_TH) {
        const int r = i / XS, c = i % XS;
        X[i] = (r < rows && c < GIN) ? obs_in(a.obs, a.obs_scale, (s0 + r) * GIN + c, c) : 0.f;
    }
    __syncthreads();
    {
        /* E: column tile `wave` of the four row tiles */
        floatx4 acc[4][1] = {{zero4()}, {zero4()}, {zero4()}, {zero4()}};
        gemm16p<4, 1, 3>(acc, GINP, 0, 16 * wave, [&](int i, int kb) { return lds4(X + i * XS + kb); },
                         [&](int kb, int j) { return gload4(a.w.WeT + j * GINP + kb); });
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * mt + acc_row(i), c = 16 * wave + acc_col();
                const float e = tanh_exp(acc[mt][0][i] + a.params[GO_BE + c]);
                E[r * HSG + c] = e;
                if (r < rows) a.E[(s0 + r) * GHD + c] = e;
            }
    }
    __syncthreads();
    {
        /* GI: column tiles 3 wave .. 3 wave + 2 of the four row tiles */
        floatx4 acc[4][3];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int n = 0; n < 3; ++n) acc[mt][n] = zero4();
        gemm16p<4, 3, 2>(acc, GHD, 0, 48 * wave, [&](int i, int kb) { return lds4(E + i * HSG + kb); },
                         [&](int kb, int j) { return gload4(a.w.WiT + j * GHD + kb); });
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int n = 0; n < 3; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * mt + acc_row(i), c = 48 * wave + 16 * n + acc_col();
                    if (r < rows) a.DGI[(s0 + r) * G3 + c] = acc[mt][n][i] + a.params[GO_BI + c];
                }
    }
}

/* The weights of a wave's three GH column tiles (48 wave .. 48 wave + 47), held in
 * registers for a whole recurrence: lane l keeps W_h^T rows 48 wave + 16 n + l % 16 at
 * k = 16 blk + 4 (l / 16) .. + 3, the operands of every MFMA step of the product, and
 * the three bias values of its column. */
struct GhRegs {
    floatx4 w[GHD / 16][3];
    float b[3];
};
__device__ __forceinline__ void gh_regs_load(GhRegs &g, const float *__restrict__ P, const GruW &w, int wave) {
    const int l = (int)(threadIdx.x & 63), li = l & 15, kq = 4 * (l >> 4);
#pragma unroll
    for (int blk = 0; blk < GHD / 16; ++blk)
#pragma unroll
        for (int n = 0; n < 3; ++n) g.w[blk][n] = gload4(w.WhT + (48 * wave + 16 * n + li) * GHD + 16 * blk + kq);
#pragma unroll
    for (int n = 0; n < 3; ++n) g.b[n] = P[GO_BH + 48 * wave + 16 * n + li];
}
/* GH = HP W_h + b_h for a tile from the register-resident weights: only HP is read */
__device__ __forceinline__ void gru_gh_regs(const GhRegs &g, const float *HP, float *GH, int wave) {
    const int l = (int)(threadIdx.x & 63), li = l & 15, kq = 4 * (l >> 4);
    floatx4 av[GHD / 16];
#pragma unroll
    for (int blk = 0; blk < GHD / 16; ++blk) av[blk] = lds4(HP + li * HSG + 16 * blk + kq);
    floatx4 acc[3] = {zero4(), zero4(), zero4()};
#pragma unroll
    for (int blk = 0; blk < GHD / 16; ++blk)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int n = 0; n < 3; ++n) acc[n] = mfma(av[blk][t], g.w[blk][n][t], acc[n]);
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int i = 0; i < 4; ++i) GH[acc_row(i) * GS + 48 * wave + 16 * n + acc_col()] = acc[n][i] + g.b[n];
}

/* A step's GI rows (three float4 per thread) and the episode-start flags of the rows a
 * thread handles are loaded into registers ahead of their step, so that no step waits on
 * device memory. */
constexpr int GRU_GE = TG * G3 / 4 / GRU_SEQ_TH, GRU_HE = TG * GHD / GRU_SEQ_TH;
static_assert(TG * G3 % (4 * GRU_SEQ_TH) == 0 && TG * GHD % GRU_SEQ_TH == 0, "whole elements per thread");

/* Two barriers per step: GH = HP W_h + b_h, then the cell, which also writes the next
 * step's input state (HP, zeroed at an episode start; each thread its own elements) and
 * stores the next step's GI rows into the other of two GI buffers. */
__global__ void __launch_bounds__(GRU_SEQ_TH) k_gru_fwd(GruSeqArgs a) {
    extern __shared__ float sm[];
    float *HP = sm, *GH = HP + TG * HSG, *GIb = GH + TG * GS; /* GIb: two buffers */
    const int row0 = (int)blockIdx.x * TG, rows = min(TG, a.m - row0);
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    const int T = a.T, m = a.m;
    GhRegs gr;
    gh_regs_load(gr, a.params, a.w, wave);
    floatx4 gv[GRU_GE];
    uint8_t sv[GRU_HE];
    auto load = [&](int t) {
#pragma unroll
        for (int k = 0; k < GRU_GE; ++k) {
            const int q = tid + k * GRU_SEQ_TH, r = q / (G3 / 4), c = 4 * (q % (G3 / 4));
            gv[k] = r < rows ? gload4(a.DGI + ((int64_t)t * m + row0 + r) * G3 + c) : zero4();
        }
#pragma unroll
        for (int k = 0; k < GRU_HE; ++k) {
            const int r = (tid + k * GRU_SEQ_TH) / GHD;
            sv[k] = r < rows ? a.start[(int64_t)t * m + row0 + r] : 1;
        }
    };
    auto store_gi = [&](float *GI) {
#pragma unroll
        for (int k = 0; k < GRU_GE; ++k) {
            const int q = tid + k * GRU_SEQ_TH, r = q / (G3 / 4), c = 4 * (q % (G3 / 4));
            *(floatx4 *)(GI + r * GS + c) = gv[k];
        }
    };
    load(0);
    store_gi(GIb);
#pragma unroll
    for (int k = 0; k < GRU_HE; ++k) {
        const int i = tid + k * GRU_SEQ_TH, r = i / GHD, c = i % GHD;
        const float v = r < rows ? a.h0[(int64_t)(row0 + r) * GHD + c] : 0.f;
        if (r < rows) a.HS[(int64_t)(row0 + r) * GHD + c] = v;
        HP[r * HSG + c] = sv[k] ? 0.f : v;
    }
    if (T > 1) load(1);
    __syncthreads();
    for (int t = 0; t < T; ++t) {
        gru_gh_regs(gr, HP, GH, wave);
        __syncthreads();
        const float *GI = GIb + (t & 1) * TG * GS;
#pragma unroll
        for (int k = 0; k < GRU_HE; ++k) {
            const int i = tid + k * GRU_SEQ_TH, r = i / GHD, j = i % GHD;
            const float *gi = GI + r * GS, *gh = GH + r * GS;
            const float rr = sigmoid_exp(gi[j] + gh[j]);
            const float u = sigmoid_exp(gi[GHD + j] + gh[GHD + j]);
            const float nn = tanh_exp(gi[2 * GHD + j] + rr * gh[2 * GHD + j]);
            const float hn = (1.f - u) * nn + u * HP[r * HSG + j];
            if (r < rows) a.HS[((int64_t)(t + 1) * m + row0 + r) * GHD + j] = hn;
            HP[r * HSG + j] = sv[k] ? 0.f : hn; /* sv: the start flags of step t + 1 */
        }
        if (t + 1 < T) {
            store_gi(GIb + ((t + 1) & 1) * TG * GS);
            if (t + 2 < T) load(t + 2);
        }
        __syncthreads();
    }
}

/* the outputs of the 64 samples from s0 = 64 blockIdx.x (h_t of sample s is HS[s + m]),
 * their loss terms and dO (scaled by 1 / (T m)); the workgroup's loss sums in sample
 * order */
__global__ void __launch_bounds__(GRU_HEAD_TH) k_gru_head(GruSeqArgs a) {
    extern __shared__ float sm[];
    float *O = sm, *LT = O + TI * OS;
    const int64_t S = (int64_t)a.T * a.m, s0 = (int64_t)blockIdx.x * TI;
    const int rows = (int)min((int64_t)TI, S - s0);
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    {
        /* row tile `wave` */
        floatx4 acc[1][1] = {{zero4()}};
        const int r0 = 16 * wave;
        gemm16p<1, 1, GPF>(acc, GHD, 0, 0,
                           [&](int i, int kb) {
                               return r0 + i < rows ? gload4(a.HS + (s0 + r0 + i + a.m) * GHD + kb) : zero4();
                           },
                           [&](int kb, int j) { return gload4(a.w.WoT + j * GHD + kb); });
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + acc_row(i), c = acc_col();
            O[r * OS + c] = c < OUT ? acc[0][0][i] + a.params[GO_BO + c] : 0.f;
        }
    }
    __syncthreads();
    if (tid < TI) {
        float dz[OUT], ls[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < OUT; ++j) dz[j] = 0.f;
        if (tid < rows) {
            const int64_t s = s0 + tid;
            loss_head(O + tid * OS, a.n_act, a.act[s], a.logp_old[s], a.adv[s], a.ret[s], a.v_old[s], a.clip, a.c_v,
                      a.c_e, a.scale, dz, ls);
#pragma unroll
            for (int j = 0; j < 16; ++j) a.DO[s * 16 + j] = j < OUT ? dz[j] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) LT[tid * 4 + q] = ls[q];
    }
    __syncthreads();
    if (tid < 4) {
        float v = 0.f;
        for (int r = 0; r < TI; ++r) v += LT[r * 4 + tid];
        a.LS[(int64_t)blockIdx.x * 4 + tid] = v;
    }
}

/* Two barriers per step, software-pipelined: the product phase after the cell of step
 * t + 1 forms dh_t = u dh + DGH_{t+1} W_h^T together with step t's GH (recomputed from
 * h_{t-1}) and dO_t W_o^T; then the cell of step t.  A step's inputs (GI rows, h_{t-1},
 * start flags, dO) go into one of two buffers by the parity of t, loaded into registers
 * two steps ahead. */
__global__ void __launch_bounds__(GRU_SEQ_TH) k_gru_bwd(GruSeqArgs a) {
    extern __shared__ float sm[];
    float *DH = sm, *DHO = DH + TG * HSG, *GH = DHO + TG * HSG, *DGH = GH + TG * GS;
    float *HPb = DGH + TG * GS;        /* [2][TG][HSG] */
    float *GIb = HPb + 2 * TG * HSG;   /* [2][TG][GS] */
    float *DOb = GIb + 2 * TG * GS;    /* [2][TG][16] */
    float *STb = DOb + 2 * TG * 16;    /* [2][TG] */
    const int row0 = (int)blockIdx.x * TG, rows = min(TG, a.m - row0);
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    const int T = a.T, m = a.m;
    GhRegs gr;
    gh_regs_load(gr, a.params, a.w, wave);
    floatx4 gv[GRU_GE], dov = zero4();
    float hv[GRU_HE];
    uint8_t sv[GRU_HE];
    auto load = [&](int t) {
#pragma unroll
        for (int k = 0; k < GRU_GE; ++k) {
            const int q = tid + k * GRU_SEQ_TH, r = q / (G3 / 4), c = 4 * (q % (G3 / 4));
            gv[k] = r < rows ? gload4(a.DGI + ((int64_t)t * m + row0 + r) * G3 + c) : zero4();
        }
#pragma unroll
        for (int k = 0; k < GRU_HE; ++k) {
            const int i = tid + k * GRU_SEQ_TH, r = i / GHD, c = i % GHD;
            sv[k] = r < rows ? a.start[(int64_t)t * m + row0 + r] : 1;
            hv[k] = r < rows ? a.HS[((int64_t)t * m + row0 + r) * GHD + c] : 0.f;
        }
        if (tid < TG * 4) {
            const int r = tid / 4, c = 4 * (tid % 4);
            dov = r < rows ? gload4(a.DO + ((int64_t)t * m + row0 + r) * 16 + c) : zero4();
        }
    };
    auto stage = [&](int t) { /* the registers (step t) into the buffers of t's parity */
        const int p = t & 1;
        float *GI = GIb + p * TG * GS, *HP = HPb + p * TG * HSG;
#pragma unroll
        for (int k = 0; k < GRU_GE; ++k) {
            const int q = tid + k * GRU_SEQ_TH, r = q / (G3 / 4), c = 4 * (q % (G3 / 4));
            *(floatx4 *)(GI + r * GS + c) = gv[k];
        }
#pragma unroll
        for (int k = 0; k < GRU_HE; ++k) {
            const int i = tid + k * GRU_SEQ_TH, r = i / GHD, c = i % GHD;
            HP[r * HSG + c] = sv[k] ? 0.f : hv[k];
            if (c == 0) STb[p * TG + r] = sv[k] ? 1.f : 0.f;
        }
        if (tid < TG * 4) *(floatx4 *)(DOb + p * TG * 16 + (tid / 4) * 16 + 4 * (tid % 4)) = dov;
    };
    /* GH of step t (from h_{t-1}) and dO_t W_o^T (column tile `wave`, K = 16, rows 10..15
     * of W_o^T zero) */
    auto gates_and_out = [&](int t) {
        const int p = t & 1;
        gru_gh_regs(gr, HPb + p * TG * HSG, GH, wave);
        floatx4 acc[1][1] = {{zero4()}};
        const float *DOt = DOb + p * TG * 16;
        gemm16p<1, 1, 1>(acc, 16, 0, 16 * wave, [&](int i, int kb) { return lds4(DOt + i * 16 + kb); },
                         [&](int kb, int j) { return gload4(a.w.WoP + j * 16 + kb); });
#pragma unroll
        for (int i = 0; i < 4; ++i) DHO[acc_row(i) * HSG + 16 * wave + acc_col()] = acc[0][0][i];
    };
    for (int i = tid; i < TG * HSG; i += GRU_SEQ_TH) DH[i] = 0.f;
    load(T - 1);
    stage(T - 1);
    if (T > 1) load(T - 2);
    __syncthreads();
    gates_and_out(T - 1);
    __syncthreads();
    for (int t = T - 1; t >= 0; --t) {
        const int p = t & 1;
        const float *GI = GIb + p * TG * GS, *HP = HPb + p * TG * HSG;
        /* the cell again and back through it: gate pre-activation gradients (to the
         * workspace, DGI over the sample's GI); DH keeps the direct part u dh of dh_{t-1} */
#pragma unroll
        for (int k = 0; k < GRU_HE; ++k) {
            const int i = tid + k * GRU_SEQ_TH, r = i / GHD, j = i % GHD;
            const float *gi = GI + r * GS, *gh = GH + r * GS;
            const float rr = sigmoid_exp(gi[j] + gh[j]);
            const float u = sigmoid_exp(gi[GHD + j] + gh[GHD + j]);
            const float ghn = gh[2 * GHD + j];
            const float nn = tanh_exp(gi[2 * GHD + j] + rr * ghn);
            const float hp = HP[r * HSG + j];
            const float dh = DH[r * HSG + j] + DHO[r * HSG + j];
            const float dnp = dh * (1.f - u) * (1.f - nn * nn);
            const float dup = dh * (hp - nn) * u * (1.f - u);
            const float drp = dnp * ghn * rr * (1.f - rr);
            DGH[r * GS + j] = drp;
            DGH[r * GS + GHD + j] = dup;
            DGH[r * GS + 2 * GHD + j] = dnp * rr;
            DH[r * HSG + j] = dh * u;
            if (r < rows) {
                const int64_t s = ((int64_t)t * m + row0 + r) * G3;
                a.DGI[s + j] = drp;
                a.DGI[s + GHD + j] = dup;
                a.DGI[s + 2 * GHD + j] = dnp;
                a.DGH[s + j] = drp;
                a.DGH[s + GHD + j] = dup;
                a.DGH[s + 2 * GHD + j] = dnp * rr;
            }
        }
        if (t == 0) break;
        /* step t - 1's inputs into the other buffers (their step t + 1 readers are done) */
        stage(t - 1);
        if (t >= 2) load(t - 2);
        __syncthreads();
        /* dh_{t-1} = u dh + DGH W_h^T (column tile `wave`, K = 384), zero at an episode
         * start of step t (also set for rows past the last sequence); with step t - 1's
         * GH and dO W_o^T */
        {
            floatx4 acc[1][1] = {{zero4()}};
            gemm16p<1, 1, 2 * GPF>(acc, G3, 0, 16 * wave, [&](int i, int kb) { return lds4(DGH + i * GS + kb); },
                                   [&](int kb, int j) { return gload4(a.w.Wh + j * G3 + kb); });
            const float *ST = STb + p * TG;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = acc_row(i), c = 16 * wave + acc_col();
                DH[r * HSG + c] = ST[r] != 0.f ? 0.f : DH[r * HSG + c] + acc[0][0][i];
            }
        }
        gates_and_out(t - 1);
        __syncthreads();
    }
}

/* DE = (DGI W_i^T) (1 - E^2) of the 64 samples from s0 = 64 blockIdx.x: column tile
 * `wave` of the four row tiles */
__global__ void __launch_bounds__(GRU_IN_TH) k_gru_de(GruSeqArgs a) {
    extern __shared__ float sm[];
    float *D = sm; /* the 64 samples' DGI rows, read from memory once for all eight waves */
    const int64_t S = (int64_t)a.T * a.m, s0 = (int64_t)blockIdx.x * TI;
    const int rows = (int)min((int64_t)TI, S - s0);
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    for (int q = tid; q < TI * G3 / 4; q += GRU_IN_TH) {
        const int r = q / (G3 / 4), c = 4 * (q % (G3 / 4));
        *(floatx4 *)(D + r * DES + c) = r < rows ? gload4(a.DGI + (s0 + r) * G3 + c) : zero4();
    }
    __syncthreads();
    floatx4 acc[4][1] = {{zero4()}, {zero4()}, {zero4()}, {zero4()}};
    gemm16p<4, 1, GPF>(acc, G3, 0, 16 * wave, [&](int i, int kb) { return lds4(D + i * DES + kb); },
                       [&](int kb, int j) { return gload4(a.w.Wi + j * G3 + kb); });
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * mt + acc_row(i), c = 16 * wave + acc_col();
            if (r < rows) {
                const float e = a.E[(s0 + r) * GHD + c];
                a.DE[(s0 + r) * GHD + c] = acc[mt][0][i] * (1.f - e * e);
            }
        }
}

/* ---- weight gradients over all T m samples: workgroup w takes a contiguous range of
 * samples (s = t m + env) and writes one partial of every parameter; the partials are
 * then summed in a fixed order.  The range is staged through LDS DWK samples at a time
 * (every operand read from memory once per workgroup), in two passes:
 *   1. dW_i = E^T DGI and dW_h = HP^T DGH (HP zero at an episode start): 8 x 24 tiles
 *      each, in blocks of 4 x 6 tiles, one block per wave; the bias sums of DGI, DGH;
 *   2. dW_e = X^T DE (3 x 8 tiles, rows 40..47 dropped) and dW_o = HN^T DO (8 tiles),
 *      two tiles per wave; the bias sums of DE and DO.
 * The sample index is the MFMA k index: lane l supplies sample k0 + l / 16 of a row
 * tile's column l % 16.  LDS rows are padded to 16 mod 64 words, so the four sample rows
 * one MFMA step reads fall on disjoint banks. ---- */
struct GruDwArgs {
    const float *obs;          /* [S][40] */
    const float *obs_scale;    /* [40] or null */
    const uint8_t *start;      /* [S] */
    const float *HS, *E, *DGI, *DGH, *DE, *DO;
    int64_t S, m;
    float *partial;            /* [grid][GPW] */
};
constexpr int DWK = 16;                                    /* samples per staged chunk */
constexpr int DSH = GHD + 16, DSG = G3 + 16, DSX = 80, DSO = 16;
constexpr int DW_LDS = DWK * (2 * DSH + 2 * DSG);           /* floats (pass 1; pass 2 needs less) */
static_assert(DWK * (DSX + 2 * DSH + DSO) <= DW_LDS, "pass 2 fits in pass 1's LDS");
static_assert(GRU_DW_TH == 1024 && DWK % 4 == 0, "16 waves: the 16 blocks of pass 1, 32 tiles of pass 2");

__global__ void __launch_bounds__(GRU_DW_TH) k_gru_dw(GruDwArgs a) {
    extern __shared__ float sm[];
    const int64_t s0 = a.S * (int64_t)blockIdx.x / gridDim.x, s1 = a.S * (int64_t)(blockIdx.x + 1) / gridDim.x;
    const int len = (int)(s1 - s0);
    float *G = a.partial + (int64_t)blockIdx.x * GPW;
    const int tid = (int)threadIdx.x, wave = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;

    /* pass 1 */
    {
        float *sE = sm, *sHP = sE + DWK * DSH, *sGI = sHP + DWK * DSH, *sGH = sGI + DWK * DSG;
        const bool hh = wave >= 8; /* waves 0..7: dW_i, 8..15: dW_h */
        const int r0 = 64 * ((wave >> 2) & 1), c0 = 96 * (wave & 3);
        const float *sA = hh ? sHP : sE, *sB = hh ? sGH : sGI;
        floatx4 acc[4][6];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 6; ++n) acc[m][n] = zero4();
        float bsum = 0.f; /* threads below 768: column tid of [DGI | DGH] */
        for (int k0 = 0; k0 < len; k0 += DWK) {
            const int kc = min(DWK, len - k0);
            __syncthreads();
            for (int q = tid; q < DWK * (GHD / 4); q += GRU_DW_TH) {
                const int r = q / (GHD / 4), c = 4 * (q % (GHD / 4));
                floatx4 e = zero4(), h = zero4();
                if (r < kc) {
                    const int64_t sa = s0 + k0 + r;
                    e = gload4(a.E + sa * GHD + c);
                    if (!a.start[sa]) h = gload4(a.HS + sa * GHD + c);
                }
                *(floatx4 *)(sE + r * DSH + c) = e;
                *(floatx4 *)(sHP + r * DSH + c) = h;
            }
            for (int q = tid; q < DWK * (G3 / 4); q += GRU_DW_TH) {
                const int r = q / (G3 / 4), c = 4 * (q % (G3 / 4));
                floatx4 gi = zero4(), gh = zero4();
                if (r < kc) {
                    const int64_t sa = s0 + k0 + r;
                    gi = gload4(a.DGI + sa * G3 + c);
                    gh = gload4(a.DGH + sa * G3 + c);
                }
                *(floatx4 *)(sGI + r * DSG + c) = gi;
                *(floatx4 *)(sGH + r * DSG + c) = gh;
            }
            __syncthreads();
            if (tid < 2 * G3) {
                const float *col = tid < G3 ? sGI + tid : sGH + (tid - G3);
                for (int r = 0; r < kc; ++r) bsum += col[r * DSG];
            }
            for (int kk = 0; kk < kc; kk += 4) {
                float av[4], bv[6];
#pragma unroll
                for (int m = 0; m < 4; ++m) av[m] = sA[(kk + lk) * DSH + r0 + 16 * m + li];
#pragma unroll
                for (int n = 0; n < 6; ++n) bv[n] = sB[(kk + lk) * DSG + c0 + 16 * n + li];
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < 6; ++n) acc[m][n] = mfma(av[m], bv[n], acc[m][n]);
            }
        }
        float *W = G + (hh ? GO_WH : GO_WI);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 6; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    W[(r0 + 16 * m + acc_row(i)) * G3 + c0 + 16 * n + acc_col()] = acc[m][n][i];
        if (tid < G3) G[GO_BI + tid] = bsum;
        else if (tid < 2 * G3) G[GO_BH + tid - G3] = bsum;
    }

    /* pass 2: waves 0..11 two dW_e tiles (row tile wave / 4, column tiles 2 (wave % 4) and
     * the next), waves 12..15 two dW_o tiles (row tiles 2 (wave - 12) and the next) */
    {
        float *sX = sm, *sDE = sX + DWK * DSX, *sHN = sDE + DWK * DSH, *sDO = sHN + DWK * DSH;
        const bool wo = wave >= 12;
        const float *sA0, *sA1, *sB0, *sB1;
        int sa_, sb_;
        if (!wo) {
            const int rt = wave >> 2, ct = 2 * (wave & 3);
            sA0 = sA1 = sX + 16 * rt; sB0 = sDE + 16 * ct; sB1 = sDE + 16 * (ct + 1);
            sa_ = DSX; sb_ = DSH;
        } else {
            const int rt = 2 * (wave - 12);
            sA0 = sHN + 16 * rt; sA1 = sHN + 16 * (rt + 1); sB0 = sB1 = sDO;
            sa_ = DSH; sb_ = DSO;
        }
        floatx4 acc[2] = {zero4(), zero4()};
        float bsum = 0.f; /* threads below 128 + 10: column tid of [DE | DO] */
        for (int k0 = 0; k0 < len; k0 += DWK) {
            const int kc = min(DWK, len - k0);
            __syncthreads();
            for (int q = tid; q < DWK * DSX; q += GRU_DW_TH) {
                const int r = q / DSX, c = q % DSX;
                sX[q] = (r < kc && c < GIN) ? obs_in(a.obs, a.obs_scale, (s0 + k0 + r) * GIN + c, c) : 0.f;
            }
            for (int q = tid; q < DWK * (GHD / 4); q += GRU_DW_TH) {
                const int r = q / (GHD / 4), c = 4 * (q % (GHD / 4));
                floatx4 d = zero4(), h = zero4();
                if (r < kc) {
                    const int64_t sa = s0 + k0 + r;
                    d = gload4(a.DE + sa * GHD + c);
                    h = gload4(a.HS + (sa + a.m) * GHD + c);
                }
                *(floatx4 *)(sDE + r * DSH + c) = d;
                *(floatx4 *)(sHN + r * DSH + c) = h;
            }
            for (int q = tid; q < DWK * 4; q += GRU_DW_TH) {
                const int r = q / 4, c = 4 * (q % 4);
                *(floatx4 *)(sDO + r * DSO + c) = r < kc ? gload4(a.DO + (s0 + k0 + r) * 16 + c) : zero4();
            }
            __syncthreads();
            if (tid < GHD + OUT) {
                const float *col = tid < GHD ? sDE + tid : sDO + (tid - GHD);
                const int st = tid < GHD ? DSH : DSO;
                for (int r = 0; r < kc; ++r) bsum += col[r * st];
            }
            for (int kk = 0; kk < kc; kk += 4) {
                const float a0 = sA0[(kk + lk) * sa_ + li], a1 = sA1[(kk + lk) * sa_ + li];
                const float b0 = sB0[(kk + lk) * sb_ + li], b1 = sB1[(kk + lk) * sb_ + li];
                acc[0] = mfma(a0, b0, acc[0]);
                acc[1] = mfma(a1, b1, acc[1]);
            }
        }
        if (!wo) {
            const int rt = wave >> 2, ct = 2 * (wave & 3);
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * rt + acc_row(i);
                    if (r < GIN) G[GO_WE + r * GHD + 16 * (ct + n) + acc_col()] = acc[n][i];
                }
        } else {
            const int rt = 2 * (wave - 12);
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (acc_col() < OUT) G[GO_WO + (16 * (rt + n) + acc_row(i)) * OUT + acc_col()] = acc[n][i];
        }
        if (tid < GHD) G[GO_BE + tid] = bsum;
        else if (tid < GHD + OUT) G[GO_BO + tid - GHD] = bsum;
    }
    if (tid < GPW - GNP) G[GNP + tid] = 0.f;
}

/* columns [0, width) of the chunk sums summed in chunk order into out */
__global__ void k_reduce_out(const float *__restrict__ sums, int nch, int pitch, int width, float *out) {
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= width) return;
    float s = 0.f;
    for (int c = 0; c < nch; ++c) s += sums[(int64_t)c * pitch + j];
    out[j] = s;
}

/* the workgroups' loss sums in a fixed order: thread i adds the contiguous run of entries
 * [i n / 256, (i + 1) n / 256) in order, then those 256 sums are added in thread order */
constexpr int GRU_LOSS_TH = 256;
__global__ void __launch_bounds__(GRU_LOSS_TH) k_gru_loss(const float *__restrict__ LS, int n, float *loss) {
    __shared__ float part[GRU_LOSS_TH][4];
    const int tid = (int)threadIdx.x;
    const int lo = (int)((int64_t)n * tid / GRU_LOSS_TH), hi = (int)((int64_t)n * (tid + 1) / GRU_LOSS_TH);
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = lo; i < hi; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += LS[(int64_t)i * 4 + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) part[tid][q] = v[q];
    __syncthreads();
    if (tid < 4) {
        float sum = 0.f;
        for (int i = 0; i < GRU_LOSS_TH; ++i) sum += part[i][tid];
        loss[tid] = sum;
    }
}

__global__ void k_bump(uint64_t *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c[0] += 1;
}

} // namespace ippo

using namespace ippo;

namespace {
bool lds_opt_in() {
    static bool done = false;
    if (!done) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_policy_forward),
                                hipFuncAttributeMaxDynamicSharedMemorySize, LDS_FLOATS_P * 4) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_ppo_fwd_bwd),
                                hipFuncAttributeMaxDynamicSharedMemorySize, LDS_FLOATS * 4) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_gru_step),
                                hipFuncAttributeMaxDynamicSharedMemorySize, GRU_STEP_LDS * 4) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_gru_fwd),
                                hipFuncAttributeMaxDynamicSharedMemorySize, GRU_FWD_LDS * 4) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_gru_bwd),
                                hipFuncAttributeMaxDynamicSharedMemorySize, GRU_BWD_LDS * 4) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_gru_dw),
                                hipFuncAttributeMaxDynamicSharedMemorySize, DW_LDS * 4) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_gru_de),
                                hipFuncAttributeMaxDynamicSharedMemorySize, GRU_DE_LDS * 4) != hipSuccess)
            return false;
        done = true;
    }
    return true;
}
/* the GRU loss workspace, in floats from its start (every part a multiple of 4 floats) */
struct GruWs {
    int64_t hs, e, dgi, dgh, de, dout, ls, wts, part, sums, total;
    int ntile, nin, nwg, nch;
};
GruWs gru_ws(int32_t T, int32_t m) {
    GruWs w{};
    const int64_t S = (int64_t)T * m;
    w.ntile = (m + TG - 1) / TG;
    w.nin = (int)((S + TI - 1) / TI);
    w.nwg = (int)std::min<int64_t>(GRU_DW_WGS, (S + 63) / 64);
    w.nch = (w.nwg + RCH - 1) / RCH;
    int64_t o = 0;
    w.hs = o; o += (int64_t)(T + 1) * m * GHD;
    w.e = o; o += S * GHD;
    w.dgi = o; o += S * G3;
    w.dgh = o; o += S * G3;
    w.de = o; o += S * GHD;
    w.dout = o; o += S * 16;
    w.ls = o; o += (int64_t)w.nin * 4;
    w.wts = o; o += GW_FLOATS;
    w.part = o; o += (int64_t)w.nwg * GPW;
    w.sums = o; o += (int64_t)w.nch * GPW;
    w.total = o;
    return w;
}

int64_t ppo_workspace_bytes(int32_t m) {
    const int64_t nwg = std::min<int64_t>((m + TR - 1) / TR, PPO_WGS), nch = (nwg + RCH - 1) / RCH;
    return (nwg + nch) * PW * 4 + PARAM_COPY_BYTES + W2T_BYTES;
}

int ppo_launch(const float *params, const float *obs, const float *obs_scale, const int32_t *act, const float *logp_old,
               const float *adv,
               const float *ret, const float *v_old, int32_t m, int32_t n_actions, float clip, float c_v, float c_e,
               float *workspace, int64_t workspace_bytes, float *loss, float *grad, void *stream) {
    if (!params || !obs || !act || !logp_old || !adv || !ret || !v_old || !workspace || !loss || !grad)
        return LOB_EINVAL;
    if (m <= 0 || n_actions < 1 || n_actions > 9 || !(clip > 0.f)) return LOB_EINVAL;
    const int nwg = std::min((m + TR - 1) / TR, PPO_WGS);
    const int nch = (nwg + RCH - 1) / RCH;
    const int64_t part_bytes = (int64_t)(nwg + nch) * PW * 4;
    if (workspace_bytes < part_bytes + PARAM_COPY_BYTES + W2T_BYTES || ((uintptr_t)workspace & 15)) return LOB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    /* the kernel reads W2 in 16-byte loads: parameters that are not 16-byte aligned (a
     * row of a [networks][LOB_PPO_PARAMS] array) are first copied into the workspace */
    if ((uintptr_t)params & 15) {
        float *copy = (float *)(((uintptr_t)workspace + part_bytes + 15) & ~(uintptr_t)15);
        if (hipMemcpyAsync(copy, params, (size_t)NPARAM * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return LOB_EHIP;
        params = copy;
    }
    PpoArgs a;
    a.params = params; a.obs = obs; a.obs_scale = obs_scale; a.act = act; a.logp_old = logp_old; a.adv = adv;
    a.ret = ret; a.v_old = v_old;
    a.m = m; a.n_act = n_actions; a.clip = clip; a.c_v = c_v; a.c_e = c_e; a.scale = 1.0f / (float)m;
    a.partial = workspace;
    float *w2t = (float *)(((uintptr_t)workspace + part_bytes + PARAM_COPY_BYTES + 15) & ~(uintptr_t)15);
    a.w2t = w2t;
    if (!lds_opt_in()) return LOB_EHIP;
    hipLaunchKernelGGL(k_w2t, dim3((unsigned)(HID * HID / 256)), dim3(256), 0, st, params, w2t);
    hipLaunchKernelGGL(k_ppo_fwd_bwd, dim3((unsigned)nwg), dim3(NTH), LDS_FLOATS * 4, st, a);
    float *sums = workspace + (int64_t)nwg * PW;
    hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((PW / 4 + 255) / 256), (unsigned)nch), dim3(256), 0, st,
                       (const floatx4 *)a.partial, nwg, PW / 4, (floatx4 *)sums);
    hipLaunchKernelGGL(k_reduce_final, dim3((unsigned)((PW + 255) / 256)), dim3(256), 0, st, (const float *)sums, nch,
                       grad, loss);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

/* The fixed scratch of lob_ppo_fwd_bwd_noalloc: the workspace of the largest call (256
 * workgroup partials, the first reduction level's chunk sums, room for an aligned
 * parameter copy and for W2 transposed), one copy per GPU for the life of the process.  In host code `scratch`
 * only names the symbol: its device address on the current GPU comes from
 * hipGetSymbolAddress, taken once per device and kept. */
constexpr int64_t PPO_SCRATCH_BYTES =
    ((int64_t)PPO_WGS + (PPO_WGS + RCH - 1) / RCH) * PW * 4 + PARAM_COPY_BYTES + W2T_BYTES;
static __device__ __align__(256) float scratch[(PPO_SCRATCH_BYTES + 3) / 4];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_dev[MAX_DEVICES] = {};

/* the current device's address of `scratch` (resolved on the first call on a device) */
int scratch_ptr(float **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LOB_EHIP;
    if (dev < 0 || dev >= MAX_DEVICES) return LOB_EUNSUPPORTED;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LOB_EHIP;
        scratch_dev[dev] = static_cast<float *>(p);
    }
    *out = scratch_dev[dev];
    return LOB_OK;
}

} // namespace

extern "C" {

int lob_policy_forward(const float *params, const float *obs, const float *obs_scale, int32_t n_agents, int32_t n,
                       const int32_t *n_actions,
                       uint64_t seed, const uint64_t *epoch, int32_t t, float *logits, int32_t *actions, float *logp,
                       float *value, void *stream) {
    if (!params || !obs || !n_actions || !actions || !logp || !value) return LOB_EINVAL;
    if (n_agents < 1 || n_agents > LOB_MAX_AGENTS || n <= 0) return LOB_EINVAL;
    FwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = params; a.obs = obs; a.obs_scale = obs_scale; a.n = n; a.n_agents = n_agents;
    for (int i = 0; i < n_agents; ++i) {
        if (n_actions[i] < 1 || n_actions[i] > 9) return LOB_EINVAL;
        a.n_act[i] = n_actions[i];
    }
    a.seed = seed; a.epoch = epoch; a.t = t; a.logits = logits; a.actions = actions; a.logp = logp; a.value = value;
    if (!lds_opt_in()) return LOB_EHIP;
    const dim3 grid((unsigned)((n + TRP - 1) / TRP), (unsigned)n_agents);
    hipLaunchKernelGGL(k_policy_forward, grid, dim3(NTH), LDS_FLOATS_P * 4, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

int lob_gru_step(const float *params, const float *obs, const float *obs_scale, const float *h_in, float *h_out,
                 const uint8_t *start,
                 int32_t n_agents, int32_t n, const int32_t *n_actions, uint64_t seed, const uint64_t *epoch, int32_t t,
                 float *logits, int32_t *actions, float *logp, float *value, void *stream) {
    if (!params || !obs || !h_in || !h_out || !n_actions || !actions || !logp || !value) return LOB_EINVAL;
    if (n_agents < 1 || n_agents > LOB_MAX_AGENTS || n <= 0) return LOB_EINVAL;
    GruStepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = params; a.obs = obs; a.obs_scale = obs_scale; a.h_in = h_in; a.h_out = h_out; a.start = start; a.n = n;
    for (int i = 0; i < n_agents; ++i) {
        if (n_actions[i] < 1 || n_actions[i] > 9) return LOB_EINVAL;
        a.n_act[i] = n_actions[i];
    }
    a.seed = seed; a.epoch = epoch; a.t = t; a.logits = logits; a.actions = actions; a.logp = logp; a.value = value;
    if (!lds_opt_in()) return LOB_EHIP;
    hipLaunchKernelGGL(k_gru_step, dim3((unsigned)((n + TS - 1) / TS), (unsigned)n_agents), dim3(GRU_STEP_TH),
                       GRU_STEP_LDS * 4, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

int64_t lob_gru_ppo_workspace_bytes(int32_t T, int32_t m) {
    if (T <= 0 || m <= 0) return LOB_EINVAL;
    return gru_ws(T, m).total * 4;
}

int lob_gru_ppo_fwd_bwd(const float *params, const float *obs, const float *obs_scale, const uint8_t *start,
                        const float *h0,
                        const int32_t *act, const float *logp_old, const float *adv, const float *ret,
                        const float *v_old, int32_t T, int32_t m, int32_t n_actions, float clip, float c_v, float c_e,
                        float *workspace, int64_t workspace_bytes, float *loss, float *grad, void *stream) {
    if (!params || !obs || !start || !h0 || !act || !logp_old || !adv || !ret || !v_old || !workspace || !loss || !grad)
        return LOB_EINVAL;
    if (T <= 0 || m <= 0 || n_actions < 1 || n_actions > 9 || !(clip > 0.f)) return LOB_EINVAL;
    if ((int64_t)T * m > ((int64_t)1 << 31) / G3) return LOB_EUNSUPPORTED;
    const GruWs w = gru_ws(T, m);
    if (workspace_bytes < w.total * 4 || ((uintptr_t)workspace & 15)) return LOB_EINVAL;
    if (!lds_opt_in()) return LOB_EHIP;
    hipStream_t st = (hipStream_t)stream;
    float *ws = workspace;
    hipLaunchKernelGGL(k_gru_prep, dim3((GHD * G3 + 255) / 256), dim3(256), 0, st, params, ws + w.wts);
    GruSeqArgs a;
    a.params = params; a.obs = obs; a.obs_scale = obs_scale; a.start = start; a.h0 = h0; a.act = act; a.logp_old = logp_old; a.adv = adv;
    a.ret = ret; a.v_old = v_old; a.T = T; a.m = m; a.n_act = n_actions; a.clip = clip; a.c_v = c_v; a.c_e = c_e;
    a.scale = 1.0f / (float)((int64_t)T * m);
    a.HS = ws + w.hs; a.E = ws + w.e; a.DGI = ws + w.dgi; a.DGH = ws + w.dgh; a.DE = ws + w.de; a.DO = ws + w.dout;
    a.LS = ws + w.ls;
    const float *W = ws + w.wts;
    a.w = GruW{W + GW_WET, W + GW_WIT, W + GW_WHT, W + GW_WI, W + GW_WH, W + GW_WOT, W + GW_WOP};
    hipLaunchKernelGGL(k_gru_in, dim3((unsigned)w.nin), dim3(GRU_IN_TH), GRU_IN_LDS * 4, st, a);
    hipLaunchKernelGGL(k_gru_fwd, dim3((unsigned)w.ntile), dim3(GRU_SEQ_TH), GRU_FWD_LDS * 4, st, a);
    hipLaunchKernelGGL(k_gru_head, dim3((unsigned)w.nin), dim3(GRU_HEAD_TH), GRU_HEAD_LDS * 4, st, a);
    hipLaunchKernelGGL(k_gru_bwd, dim3((unsigned)w.ntile), dim3(GRU_SEQ_TH), GRU_BWD_LDS * 4, st, a);
    hipLaunchKernelGGL(k_gru_de, dim3((unsigned)w.nin), dim3(GRU_IN_TH), GRU_DE_LDS * 4, st, a);
    GruDwArgs d;
    d.obs = obs; d.obs_scale = obs_scale; d.start = start; d.HS = a.HS; d.E = a.E; d.DGI = a.DGI; d.DGH = a.DGH; d.DE = a.DE; d.DO = a.DO;
    d.S = (int64_t)T * m; d.m = m; d.partial = ws + w.part;
    hipLaunchKernelGGL(k_gru_dw, dim3((unsigned)w.nwg), dim3(GRU_DW_TH), DW_LDS * 4, st, d);
    hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((GPW / 4 + 255) / 256), (unsigned)w.nch), dim3(256), 0, st,
                       (const floatx4 *)(ws + w.part), w.nwg, GPW / 4, (floatx4 *)(ws + w.sums));
    hipLaunchKernelGGL(k_reduce_out, dim3((unsigned)((GNP + 255) / 256)), dim3(256), 0, st, (const float *)(ws + w.sums),
                       w.nch, GPW, GNP, grad);
    hipLaunchKernelGGL(k_gru_loss, dim3(1), dim3(GRU_LOSS_TH), 0, st, (const float *)(ws + w.ls), w.nin, loss);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

int lob_counter_bump(uint64_t *counter, void *stream) {
    if (!counter) return LOB_EINVAL;
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, (hipStream_t)stream, counter);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

int lob_gae(const float *reward, const float *value, const uint8_t *done, const float *last_value, int32_t T,
            int32_t n, float gamma, float lam, float *adv, float *ret, void *stream) {
    if (!reward || !value || !done || !last_value || !adv || !ret || T <= 0 || n <= 0) return LOB_EINVAL;
    hipLaunchKernelGGL(k_gae, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, reward, value,
                       done, last_value, T, n, gamma, lam, adv, ret);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

int64_t lob_ppo_workspace_bytes(int32_t m) {
    if (m <= 0) return LOB_EINVAL;
    return ppo_workspace_bytes(m);
}

int lob_ppo_fwd_bwd(const float *params, const float *obs, const float *obs_scale, const int32_t *act,
                    const float *logp_old,
                    const float *adv, const float *ret, const float *v_old, int32_t m, int32_t n_actions, float clip,
                    float c_v, float c_e, float *workspace, int64_t workspace_bytes, float *loss, float *grad,
                    void *stream) {
    return ppo_launch(params, obs, obs_scale, act, logp_old, adv, ret, v_old, m, n_actions, clip, c_v, c_e, workspace,
                      workspace_bytes, loss, grad, stream);
}

int lob_ppo_fwd_bwd_noalloc(const float *params, const float *obs, const float *obs_scale, const int32_t *act,
                            const float *logp_old,
                            const float *adv, const float *ret, const float *v_old, int32_t m, int32_t n_actions,
                            float clip, float c_v, float c_e, float *loss, float *grad, void *stream) {
    /* argument checks before any device call */
    if (!params || !obs || !act || !logp_old || !adv || !ret || !v_old || !loss || !grad) return LOB_EINVAL;
    if (m <= 0 || n_actions < 1 || n_actions > 9 || !(clip > 0.f)) return LOB_EINVAL;
    if (ppo_workspace_bytes(m) > PPO_SCRATCH_BYTES) return LOB_EINVAL; /* beyond the fixed scratch */
    float *ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc != LOB_OK) return rc;
    return ppo_launch(params, obs, obs_scale, act, logp_old, adv, ret, v_old, m, n_actions, clip, c_v, c_e, ws,
                      PPO_SCRATCH_BYTES, loss, grad, stream);
}

} // extern "C"
