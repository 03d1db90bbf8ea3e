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

/* ---- forward of a tile of R samples (R a multiple of 16, at most 64) into LDS: X,
 * H1 = tanh(X W1 + b1), H2 = tanh(H1 W2 + b2), O = H2 W3 + b3 (O cols 10..15 zero) ---- */
template <int R>
__device__ __forceinline__ void forward_tile(const float *__restrict__ P, const float *__restrict__ obs, int rows,
                                             float *X, float *H1, float *H2, float *O) {
    constexpr int MT = R / 16; /* 16-row tiles per wave */
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < R * XS; i += blockDim.x) {
        const int r = i / XS, c = i % XS;
        X[i] = (r < rows && c < IN) ? obs[(int64_t)r * IN + c] : 0.f;
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
        gemm16<MT, CT>(acc, HID, 0, CW * wave, [&](int i, int kb) { return lds4(H1 + i * HS + kb); },
                      [&](int kb, int j) {
                          floatx4 v;
#pragma unroll
                          for (int t = 0; t < 4; ++t) v[t] = P[O_W2 + (kb + t) * HID + j];
                          return v;
                      });
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
struct FwdArgs {
    const float *params; /* [A][NPARAM] */
    const float *obs;    /* [A][n][40] */
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
    forward_tile<TRP>(P, a.obs + ((int64_t)ag * a.n + row0) * IN, rows, X, H1, H2, O);
    const int tid = (int)threadIdx.x;
    if (tid < rows) {
        const int nact = a.n_act[ag];
        const int e = row0 + tid;
        const uint64_t seed = a.epoch ? a.seed + 0x9E3779B97F4A7C15ULL * a.epoch[0] : a.seed;
        const float *z = O + tid * OS;
        float m = z[0];
        for (int j = 1; j < nact; ++j) m = fmaxf(m, z[j]);
        float s = 0.f;
        for (int j = 0; j < nact; ++j) s += expf(z[j] - m);
        const float lse = m + logf(s);
        int best = 0;
        float bv = -INFINITY;
        for (int j = 0; j < nact; ++j) {
            const uint64_t h = hash4(seed, DOM_POLICY, (uint64_t)ag << 8 | (uint64_t)j, (uint64_t)a.t, (uint64_t)e);
            const float u = ((float)(uint32_t)(h >> 40) + 0.5f) * (1.0f / 16777216.0f);
            const float g = -logf(-logf(u));
            const float v = z[j] + g;
            if (v > bv) { bv = v; best = j; }
        }
        const int64_t o = (int64_t)ag * a.n + e;
        a.actions[o] = best;
        a.logp[o] = z[best] - lse;
        a.value[o] = z[9];
        if (a.logits)
            for (int j = 0; j < OUT; ++j) a.logits[o * OUT + j] = z[j];
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
    const int32_t *act;
    const float *logp_old, *adv, *ret, *v_old;
    int32_t m, n_act;
    float clip, c_v, c_e, scale; /* scale = 1 / m */
    float *partial;              /* [grid][PW]: gradient, then loss sums (total, policy, value, entropy) */
};

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
        forward_tile<TR>(P, (const float *)obs_g + (int64_t)row0 * IN, rows, X, H1, H2, O);

        /* per-sample loss and its gradient w.r.t. the 10 outputs (scaled by 1/m) */
        float lsum[4] = {0.f, 0.f, 0.f, 0.f};
        if (tid < TR) {
            float *z = O + tid * OS;
            float dz[OUT];
#pragma unroll
            for (int j = 0; j < OUT; ++j) dz[j] = 0.f;
            if (tid < rows) {
                const int s = row0 + tid;
                const int nact = a.n_act;
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
                /* an action outside [0, nact) counts as action 0, as the env step takes it */
                int act = a.act[s];
                if ((unsigned)act >= (unsigned)nact) act = 0;
                const float logp = z[act] - lse;
                const float ratio = expf(logp - a.logp_old[s]);
                const float A = a.adv[s];
                const float s1 = ratio * A;
                const float rc = fminf(fmaxf(ratio, 1.f - a.clip), 1.f + a.clip);
                const float s2 = rc * A;
                const float pol = -fminf(s1, s2);
                const float dlogp = s1 <= s2 ? -A * ratio : 0.f;
                const float v = z[9], R = a.ret[s], vo = a.v_old[s];
                const float dvv = v - vo;
                const float vc = vo + fminf(fmaxf(dvv, -a.clip), a.clip);
                const float l1 = (v - R) * (v - R), l2 = (vc - R) * (vc - R);
                const float val = 0.5f * fmaxf(l1, l2);
                const float dval = l1 >= l2 ? (v - R) : (fabsf(dvv) < a.clip ? (vc - R) : 0.f);
                for (int j = 0; j < nact; ++j) {
                    const float lp = z[j] - lse;
                    const float p = expf(lp);
                    const float dlp = (j == act ? 1.f : 0.f) - p;
                    dz[j] = a.scale * (dlogp * dlp + a.c_e * p * (lp + H));
                }
                dz[9] = a.scale * a.c_v * dval;
                lsum[0] = pol + a.c_v * val - a.c_e * H;
                lsum[1] = pol;
                lsum[2] = val;
                lsum[3] = H;
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
                                hipFuncAttributeMaxDynamicSharedMemorySize, LDS_FLOATS * 4) != hipSuccess)
            return false;
        done = true;
    }
    return true;
}
int64_t ppo_workspace_bytes(int32_t m) {
    const int64_t nwg = std::min<int64_t>((m + TR - 1) / TR, PPO_WGS), nch = (nwg + RCH - 1) / RCH;
    return (nwg + nch) * PW * 4 + PARAM_COPY_BYTES;
}

int ppo_launch(const float *params, const float *obs, const int32_t *act, const float *logp_old, const float *adv,
               const float *ret, const float *v_old, int32_t m, int32_t n_actions, float clip, float c_v, float c_e,
               float *workspace, int64_t workspace_bytes, float *loss, float *grad, void *stream) {
    if (!params || !obs || !act || !logp_old || !adv || !ret || !v_old || !workspace || !loss || !grad)
        return LOB_EINVAL;
    if (m <= 0 || n_actions < 1 || n_actions > 9 || !(clip > 0.f)) return LOB_EINVAL;
    const int nwg = std::min((m + TR - 1) / TR, PPO_WGS);
    const int nch = (nwg + RCH - 1) / RCH;
    const int64_t part_bytes = (int64_t)(nwg + nch) * PW * 4;
    if (workspace_bytes < part_bytes + PARAM_COPY_BYTES || ((uintptr_t)workspace & 15)) return LOB_EINVAL;
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
    a.params = params; a.obs = obs; a.act = act; a.logp_old = logp_old; a.adv = adv; a.ret = ret; a.v_old = v_old;
    a.m = m; a.n_act = n_actions; a.clip = clip; a.c_v = c_v; a.c_e = c_e; a.scale = 1.0f / (float)m;
    a.partial = workspace;
    if (!lds_opt_in()) return LOB_EHIP;
    hipLaunchKernelGGL(k_ppo_fwd_bwd, dim3((unsigned)nwg), dim3(NTH), LDS_FLOATS * 4, st, a);
    float *sums = workspace + (int64_t)nwg * PW;
    hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((PW / 4 + 255) / 256), (unsigned)nch), dim3(256), 0, st,
                       (const floatx4 *)a.partial, nwg, PW / 4, (floatx4 *)sums);
    hipLaunchKernelGGL(k_reduce_final, dim3((unsigned)((PW + 255) / 256)), dim3(256), 0, st, (const float *)sums, nch,
                       grad, loss);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

/* The fixed scratch of lob_ppo_fwd_bwd_noalloc: the workspace of the largest call (256
 * workgroup partials, the first reduction level's chunk sums and room for an aligned
 * parameter copy), one copy per GPU for the life of the process.  In host code `scratch`
 * only names the symbol: its device address on the current GPU comes from
 * hipGetSymbolAddress, taken once per device and kept. */
constexpr int64_t PPO_SCRATCH_BYTES =
    ((int64_t)PPO_WGS + (PPO_WGS + RCH - 1) / RCH) * PW * 4 + PARAM_COPY_BYTES;
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

int lob_policy_forward(const float *params, const float *obs, int32_t n_agents, int32_t n, const int32_t *n_actions,
                       uint64_t seed, const uint64_t *epoch, int32_t t, float *logits, int32_t *actions, float *logp,
                       float *value, void *stream) {
    if (!params || !obs || !n_actions || !actions || !logp || !value) return LOB_EINVAL;
    if (n_agents < 1 || n_agents > LOB_MAX_AGENTS || n <= 0) return LOB_EINVAL;
    FwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = params; a.obs = obs; a.n = n; a.n_agents = n_agents;
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

int lob_ppo_fwd_bwd(const float *params, const float *obs, const int32_t *act, const float *logp_old,
                    const float *adv, const float *ret, const float *v_old, int32_t m, int32_t n_actions, float clip,
                    float c_v, float c_e, float *workspace, int64_t workspace_bytes, float *loss, float *grad,
                    void *stream) {
    return ppo_launch(params, obs, act, logp_old, adv, ret, v_old, m, n_actions, clip, c_v, c_e, workspace,
                      workspace_bytes, loss, grad, stream);
}

int lob_ppo_fwd_bwd_noalloc(const float *params, const float *obs, const int32_t *act, const float *logp_old,
                            const float *adv, const float *ret, const float *v_old, int32_t m, int32_t n_actions,
                            float clip, float c_v, float c_e, float *loss, float *grad, void *stream) {
    /* argument checks before any device call */
    if (!params || !obs || !act || !logp_old || !adv || !ret || !v_old || !loss || !grad) return LOB_EINVAL;
    if (m <= 0 || n_actions < 1 || n_actions > 9 || !(clip > 0.f)) return LOB_EINVAL;
    if (ppo_workspace_bytes(m) > PPO_SCRATCH_BYTES) return LOB_EINVAL; /* beyond the fixed scratch */
    float *ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc != LOB_OK) return rc;
    return ppo_launch(params, obs, act, logp_old, adv, ret, v_old, m, n_actions, clip, c_v, c_e, ws,
                      PPO_SCRATCH_BYTES, loss, grad, stream);
}

} // extern "C"
