// Learned surrogate of the rollout cost on gfx950: a 3-layer network
// (n_in -> 256 -> 256 -> 1, GELU) on BF16 MFMA with FP32 accumulation.
//
//   u = (x - mu) * inv_sigma,  h1 = gelu(W1 u + b1),  h2 = gelu(W2 h1 + b2),
//   y = w3 . h2 + b3  (y predicts log(1 + C))
//
// Layers 1 and 2 and every backward contraction run on
// v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+7] and
// B[8(l/16)..+7][l%16] (8 bf16 each) and receives D[4(l/16)+j][l%16], j < 4.
// Weights are read as BF16 working copies in both orientations (W and W^T),
// so every B operand is one contiguous 16-byte load.  Layer 3 (one output)
// and the GELUs are FP32 VALU work.
//
// Inference (k_mlp_infer): a workgroup of eight waves takes 64 samples and the
// waves split the neurons of every layer; it runs forward, the output dot, and
// the input gradient
//   dy/dx = ((w3 * gelu'(z2)) W2 * gelu'(z1)) W1 * inv_sigma
// with gelu'(z1) kept in registers from the forward.
// Training (k_mlp_train_fb, k_mlp_wgrad, k_mlp_adam): the same forward with
// the loss gradient, activations written feature-major for the weight
// gradients dW = delta^T act (MFMA with the samples as K), per-tile bias
// partial sums reduced in a fixed order, then Adam on FP32 master weights and
// a refresh of the BF16 copies.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace stamp {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

constexpr int kIn = kMlpIn;    // padded input width
constexpr int kW = kMlpWidth;  // hidden width
constexpr int kTrainRows = 16;  // samples per training workgroup (one partial-sum tile)
constexpr int kLdU = kIn + 8;  // LDS row strides (bf16), padded against bank conflicts
constexpr int kLdH = kW + 8;

// GELU z Phi(z) and its derivative Phi(z) + z phi(z) from one exponential:
// erf by Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7, far below the BF16
// rounding of the activations), erf(x) = 1 - t (a1 + t (a2 + ... a5 t)) e^{-x^2},
// t = 1 / (1 + p x), x = |z| / sqrt 2, so that e^{-x^2} = e^{-z^2/2} is also
// sqrt(2 pi) phi(z).
__device__ __forceinline__ void gelu_pair(float z, float& g, float& gp) {
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = hw_rcp(fmaf(0.3275911f, x, 1.0f));
    const float e = hw_exp2(-0.72134752044448170f * z * z);  // e^{-z^2/2}
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    const float erf_abs = fmaf(-q * t, e, 1.0f);
    const float Phi = 0.5f + 0.5f * copysignf(erf_abs, z);
    g = z * Phi;
    gp = fmaf(z * 0.39894228040143268f, e, Phi);
}
__device__ __forceinline__ float gelu(float z) {
    float g, gp;
    gelu_pair(z, g, gp);
    return g;
}
__device__ __forceinline__ float gelu_grad(float z) {
    float g, gp;
    gelu_pair(z, g, gp);
    return gp;
}


// For acc += A B with A 16 rows x K (LDS, row stride lda) and B[k][n] =
// Bt[n][k] (global, rows of ldb bf16): the B fragments of the 16 columns that
// start at Bt row n0, every k-step of K, loaded ahead of their products.
template <int K>
__device__ __forceinline__ void load_wfrag(bf16x8 (&w)[K / 32], const __bf16* __restrict__ Bt, int ldb, int n0) {
    const int l = threadIdx.x & 63;
    const __bf16* b = Bt + (int64_t)(n0 + (l & 15)) * ldb + 8 * (l >> 4);
#pragma unroll
    for (int k = 0; k < K / 32; ++k) w[k] = *reinterpret_cast<const bf16x8*>(b + 32 * k);
}

// The product itself, k-steps in order, from the fragments in registers.
template <int K>
__device__ __forceinline__ f4 mma_rows_w(const __bf16* A, int lda, const bf16x8 (&w)[K / 32], f4 acc) {
    const int l = threadIdx.x & 63;
    const __bf16* a = A + (l & 15) * lda + 8 * (l >> 4);
#pragma unroll
    for (int k = 0; k < K / 32; ++k)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(a + 32 * k), w[k], acc, 0, 0, 0);
    return acc;
}

// Sum over the 16 lanes that share l/16 (they hold the 16 columns of a block).
__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}
// Sum over the 4 lane groups l/16 (the 4 row quarters of a block).
__device__ __forceinline__ float sum_groups(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

struct MlpPtrs {
    const float* mu;
    const float* isig;
    const float* b1;
    const float* b2;
    const float* w3;
    float b3;
    const __bf16* W1;   // [256][64]   (out, in)
    const __bf16* W1T;  // [64][256]   (in, out)
    const __bf16* W2;   // [256][256]  (out, in)
    const __bf16* W2T;  // [256][256]  (in, out)
};

__device__ __forceinline__ MlpPtrs mlp_ptrs(const float* P, const __bf16* Wb) {
    MlpPtrs m;
    m.mu = P + kMlpOffMu;
    m.isig = P + kMlpOffIsig;
    m.b1 = P + kMlpOffB1;
    m.b2 = P + kMlpOffB2;
    m.w3 = P + kMlpOffW3;
    m.b3 = P[kMlpOffB3];
    m.W1 = Wb + kMlpBfW1;
    m.W1T = Wb + kMlpBfW1T;
    m.W2 = Wb + kMlpBfW2;
    m.W2T = Wb + kMlpBfW2T;
    return m;
}

// Stage this wave's 16 standardised input rows into U (bf16).  Input sample i:
// x_mode 0: X[src * n_in + f] with src = idx ? idx[i] : i (d unused);
// x_mode 1: f < d from X[f * M + i] (structure of arrays), f >= d from enc[f - d].
// One lane's share of a 16-sample block's standardised inputs, loaded but not
// yet stored (lane l takes features l / 16 + 4 q of sample l % 16).
struct StageVals {
    float xv[kIn / 4], mu[kIn / 4], is[kIn / 4];
};

__device__ __forceinline__ void stage_load(StageVals& v, const MlpPtrs& m, const float* __restrict__ X, int x_mode,
                                           int M, int n_in, int d, const float* __restrict__ enc, int row0,
                                           const int* __restrict__ src_row = nullptr) {
    const int l = threadIdx.x & 63;
    const int r = l & 15;
    const int i = row0 + r;
    const int ic = min(i, M - 1);
    const int64_t src = (src_row && i < M) ? src_row[r] : ic;
    // every load is issued before the first use (addresses clamped into
    // range, out-of-range values replaced when stored): global loads complete
    // in order, so a load-use chain per feature would wait once per feature
#pragma unroll
    for (int q = 0; q < kIn / 4; ++q) {
        const int f = (l >> 4) + 4 * q, fc = min(f, n_in - 1);
        const float* p = x_mode == 0 ? X + src * n_in + fc : (fc < d ? X + (int64_t)fc * M + ic : enc + (fc - d));
        v.xv[q] = *p;
        v.mu[q] = m.mu[fc];
        v.is[q] = m.isig[fc];
    }
}

__device__ __forceinline__ void stage_store(__bf16* U, const StageVals& v, int M, int n_in, int row0) {
    const int l = threadIdx.x & 63;
    const int r = l & 15;
    const int i = row0 + r;
#pragma unroll
    for (int q = 0; q < kIn / 4; ++q) {
        const int f = (l >> 4) + 4 * q;
        const float x = (i < M && f < n_in) ? v.xv[q] : 0.0f;
        const float u = f < n_in ? (x - v.mu[q]) * v.is[q] : 0.0f;
        U[r * kLdU + f] = (__bf16)u;
    }
}

__device__ __forceinline__ void stage_inputs(__bf16* U, const MlpPtrs& m, const float* __restrict__ X, int x_mode,
                                             int M, int n_in, int d, const float* __restrict__ enc, int row0,
                                             const int* __restrict__ src_row = nullptr) {
    StageVals v;
    stage_load(v, m, X, x_mode, M, n_in, d, enc, row0, src_row);
    stage_store(U, v, M, n_in, row0);
}

// Exact bound term of the plan cost, added to the network's prediction of
// the rollout part: wb * sum_k relu(|o_k| - o_max)^2 + relu(-D_k)^2 +
// relu(D_k - d_max)^2 over the H pushes (o_k = x_{6k+4}, D_k = x_{6k+5}).
struct BoundTerm {
    int H;  // 0: no bound term
    float wb, omax, dmax;
};

__device__ __forceinline__ float x_raw(const float* __restrict__ X, int x_mode, int M, int n_in, int i, int f) {
    return x_mode == 0 ? X[(int64_t)i * n_in + f] : X[(int64_t)f * M + i];
}

__device__ __forceinline__ float bound_cost(const BoundTerm& bt, const float* __restrict__ X, int x_mode, int M,
                                            int n_in, int i) {
    float L = 0.0f;
    for (int k = 0; k < bt.H; ++k) {
        const float o = x_raw(X, x_mode, M, n_in, i, 6 * k + 4);
        const float D = x_raw(X, x_mode, M, n_in, i, 6 * k + 5);
        const float a = fmaxf(fabsf(o) - bt.omax, 0.0f);
        const float b1 = fmaxf(-D, 0.0f);
        const float b2 = fmaxf(D - bt.dmax, 0.0f);
        L += a * a + b1 * b1 + b2 * b2;
    }
    return bt.wb * L;
}

// d(bound term)/dx_f for the raw input value x of coordinate f.
__device__ __forceinline__ float bound_grad(const BoundTerm& bt, int f, float x) {
    if (f >= 6 * bt.H) return 0.0f;
    const int r = f % 6;
    if (r == 4) {
        const float a = fmaxf(fabsf(x) - bt.omax, 0.0f);
        const float sg = x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f);
        return bt.wb * 2.0f * a * sg;
    }
    if (r == 5) return bt.wb * (2.0f * fmaxf(x - bt.dmax, 0.0f) - 2.0f * fmaxf(-x, 0.0f));
    return 0.0f;
}

// ---------------------------------------------------------------------------
// Inference: y (and cost = expm1 y) and grad_out[f][i] = scale * e^y * dy/dx_f
// for f < d (structure of arrays, the SVGD gradient layout; grad_out holds
// exactly d rows of M, in either input layout).
//
// A workgroup of NW waves takes 16 SB samples; the waves split the 256
// neurons of each layer (TN = 16 / NW tiles of 16 each), so every weight
// fragment is read once per workgroup and all four SIMDs of a CU work.  The
// products are taken transposed, Z^T = W U^T: the weights are the A operand
// (rows of W, one 16-byte load a lane), the activations the B operand (rows
// of the sample-major LDS buffers), and a lane receives four consecutive
// neurons of one sample, which it writes to LDS as one 8-byte store.  The
// biases start the accumulators.  gelu'(z1) stays in registers from the
// forward for the input gradient (same layout as the backward product).
template <int NW>
struct InferShape {
    static constexpr int TN = 16 / NW;  // 16-neuron tiles per wave
};

// Fragment of A = rows n0..n0+15 of a row-major bf16 matrix with ld columns,
// k-step kk (32 columns).
__device__ __forceinline__ bf16x8 a_frag(const __bf16* __restrict__ W, int ld, int n0, int kk) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const bf16x8*>(W + (int64_t)(n0 + (l & 15)) * ld + 32 * kk + 8 * (l >> 4));
}
// Fragment of B = activations of samples s0..s0+15 (sample-major LDS, row stride ld), k-step kk.
__device__ __forceinline__ bf16x8 b_frag(const __bf16* S, int ld, int s0, int kk) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const bf16x8*>(S + (s0 + (l & 15)) * ld + 32 * kk + 8 * (l >> 4));
}
// Four bf16 values as one 8-byte LDS store.
__device__ __forceinline__ void store4(__bf16* p, float a, float b, float c, float d) {
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
    bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
    *reinterpret_cast<bf16x4*>(p) = v;
}

template <int NW, int SB>
__global__ __launch_bounds__(64 * NW) void k_mlp_infer(const float* __restrict__ P, const __bf16* __restrict__ Wb,
                                                       const float* __restrict__ X, int x_mode, int M, int n_in, int d,
                                                       const float* __restrict__ enc, BoundTerm bt,
                                                       float* __restrict__ y_out, float* __restrict__ cost_out,
                                                       float* __restrict__ grad_out, float grad_scale) {
    constexpr int TN = InferShape<NW>::TN;
    constexpr int S = 16 * SB;  // samples per workgroup
    constexpr int K1 = kIn / 32, K2 = kW / 32;
    __shared__ __align__(16) __bf16 sU[S * kLdU];
    __shared__ __align__(16) __bf16 sH[S * kLdH];  // h1, then delta1
    __shared__ __align__(16) __bf16 sD[S * kLdH];  // delta2
    __shared__ __align__(16) float sB1[kW], sB2[kW], sW3[kW], sIs[kIn];
    __shared__ float sYp[NW][S];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63, col = l & 15, kq = l >> 4;
    const int row0 = blockIdx.x * S;
    const int n0 = wave * 16 * TN;  // the wave's first neuron
    const MlpPtrs m = mlp_ptrs(P, Wb);
    const bool want_grad = grad_out != nullptr;

    // Loads complete in order, so what the first barrier waits for is issued
    // first: the inputs (a 16-sample block per wave, NW >= SB) and the
    // constants; then this wave's weight fragments of both forward layers
    // (layer 1's first), which stay in flight through the barrier.
    static_assert(NW >= SB && 64 * NW >= kW, "one input block and one constant per thread at most");
    StageVals sv;
    if (wave < SB) stage_load(sv, m, X, x_mode, M, n_in, d, enc, row0 + 16 * wave);
    float cb1 = 0.f, cb2 = 0.f, cw3 = 0.f, cis = 0.f;
    if (threadIdx.x < kW) {
        cb1 = m.b1[threadIdx.x];
        cb2 = m.b2[threadIdx.x];
        cw3 = m.w3[threadIdx.x];
    }
    if (threadIdx.x < kIn) cis = m.isig[threadIdx.x];
    bf16x8 a1[TN][K1], a2[TN][K2];
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
        for (int k = 0; k < K1; ++k) a1[a][k] = a_frag(m.W1, kIn, n0 + 16 * a, k);
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
        for (int k = 0; k < K2; ++k) a2[a][k] = a_frag(m.W2, kW, n0 + 16 * a, k);
    if (wave < SB) stage_store(sU + wave * 16 * kLdU, sv, M, n_in, row0 + 16 * wave);
    if (threadIdx.x < kW) {
        sB1[threadIdx.x] = cb1;
        sB2[threadIdx.x] = cb2;
        sW3[threadIdx.x] = cw3;
    }
    if (threadIdx.x < kIn) sIs[threadIdx.x] = cis;
    __syncthreads();

    // layer 1: z1^T = W1 u^T + b1; h1 to LDS, gelu'(z1) kept
    float gp1[TN][SB][4];
    {
        f4 acc[TN][SB];
#pragma unroll
        for (int a = 0; a < TN; ++a) {
            const f4 bias = *reinterpret_cast<const f4*>(sB1 + n0 + 16 * a + 4 * kq);
#pragma unroll
            for (int b = 0; b < SB; ++b) acc[a][b] = bias;
        }
#pragma unroll
        for (int k = 0; k < K1; ++k) {
            bf16x8 bu[SB];
#pragma unroll
            for (int b = 0; b < SB; ++b) bu[b] = b_frag(sU, kLdU, 16 * b, k);
#pragma unroll
            for (int a = 0; a < TN; ++a)
#pragma unroll
                for (int b = 0; b < SB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[a][k], bu[b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < TN; ++a)
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                float h[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) gelu_pair(acc[a][b][t], h[t], gp1[a][b][t]);
                store4(sH + (16 * b + col) * kLdH + n0 + 16 * a + 4 * kq, h[0], h[1], h[2], h[3]);
            }
    }
    __syncthreads();

    // layer 2, the output dot and delta2 = w3 gelu'(z2)
    {
        f4 acc[TN][SB];
#pragma unroll
        for (int a = 0; a < TN; ++a) {
            const f4 bias = *reinterpret_cast<const f4*>(sB2 + n0 + 16 * a + 4 * kq);
#pragma unroll
            for (int b = 0; b < SB; ++b) acc[a][b] = bias;
        }
#pragma unroll
        for (int k = 0; k < K2; ++k) {
            bf16x8 bh[SB];
#pragma unroll
            for (int b = 0; b < SB; ++b) bh[b] = b_frag(sH, kLdH, 16 * b, k);
#pragma unroll
            for (int a = 0; a < TN; ++a)
#pragma unroll
                for (int b = 0; b < SB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[a][k], bh[b], acc[a][b], 0, 0, 0);
        }
        // the backward's weight fragments (W2^T rows of the same neurons) load
        // while the activations are evaluated
        if (want_grad) {
#pragma unroll
            for (int a = 0; a < TN; ++a)
#pragma unroll
                for (int k = 0; k < K2; ++k) a2[a][k] = a_frag(m.W2T, kW, n0 + 16 * a, k);
        }
        float yp[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) yp[b] = 0.0f;
#pragma unroll
        for (int a = 0; a < TN; ++a) {
            const f4 w3 = *reinterpret_cast<const f4*>(sW3 + n0 + 16 * a + 4 * kq);
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                float dl[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    float g, gp;
                    gelu_pair(acc[a][b][t], g, gp);
                    yp[b] = fmaf(w3[t], g, yp[b]);
                    dl[t] = w3[t] * gp;
                }
                if (want_grad) store4(sD + (16 * b + col) * kLdH + n0 + 16 * a + 4 * kq, dl[0], dl[1], dl[2], dl[3]);
            }
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const float v = sum_groups(yp[b]);
            if (kq == 0) sYp[wave][16 * b + col] = v;
        }
    }
    __syncthreads();

    if (want_grad) {
        // the input gradient's first item of this wave (items go to the waves
        // in turn): its W1^T fragments and raw inputs load during the backward
        const int ft = min((d + 15) / 16, kIn / 16);
        bf16x8 aw0[K2];
        float xr0[4] = {0.f, 0.f, 0.f, 0.f};
        if (wave < ft * SB) {
            const int f0 = 16 * (wave / SB), i = row0 + 16 * (wave % SB) + col;
#pragma unroll
            for (int k = 0; k < K2; ++k) aw0[k] = a_frag(m.W1T, kW, f0, k);
            if (bt.H && i < M)
#pragma unroll
                for (int t = 0; t < 4; ++t) xr0[t] = x_raw(X, x_mode, M, n_in, i, min(f0 + 4 * kq + t, d - 1));
        }
        // delta1^T = (W2^T delta2^T) * gelu'(z1), to LDS over h1 (every wave is
        // past layer 2)
        f4 acc[TN][SB];
#pragma unroll
        for (int a = 0; a < TN; ++a)
#pragma unroll
            for (int b = 0; b < SB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < K2; ++k) {
            bf16x8 bd[SB];
#pragma unroll
            for (int b = 0; b < SB; ++b) bd[b] = b_frag(sD, kLdH, 16 * b, k);
#pragma unroll
            for (int a = 0; a < TN; ++a)
#pragma unroll
                for (int b = 0; b < SB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[a][k], bd[b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < TN; ++a)
#pragma unroll
            for (int b = 0; b < SB; ++b)
                store4(sH + (16 * b + col) * kLdH + n0 + 16 * a + 4 * kq, acc[a][b][0] * gp1[a][b][0],
                       acc[a][b][1] * gp1[a][b][1], acc[a][b][2] * gp1[a][b][2], acc[a][b][3] * gp1[a][b][3]);
        __syncthreads();
        // dy/dx^T = W1^T delta1^T on (16-input tile, sample block) items taken
        // by the waves in turn, then the chain through the standardisation
        // (only the first d inputs are asked for)
        for (int it = wave; it < ft * SB; it += NW) {
            const int f0 = 16 * (it / SB), b = it % SB;
            const int s = 16 * b + col, i = row0 + s;
            bf16x8 aw[K2];
            float xr[4] = {0.f, 0.f, 0.f, 0.f};
            if (it == wave) {
#pragma unroll
                for (int k = 0; k < K2; ++k) aw[k] = aw0[k];
#pragma unroll
                for (int t = 0; t < 4; ++t) xr[t] = xr0[t];
            } else {
#pragma unroll
                for (int k = 0; k < K2; ++k) aw[k] = a_frag(m.W1T, kW, f0, k);
                if (bt.H && i < M)
#pragma unroll
                    for (int t = 0; t < 4; ++t) xr[t] = x_raw(X, x_mode, M, n_in, i, min(f0 + 4 * kq + t, d - 1));
            }
            float y = m.b3;
            for (int w = 0; w < NW; ++w) y += sYp[w][s];
            const float ey = expf(y);
            f4 g = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < K2; ++k) g = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[k], b_frag(sH, kLdH, 16 * b, k), g, 0, 0, 0);
            if (i < M) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int f = f0 + 4 * kq + t;
                    if (f < d) {
                        float gi = ey * g[t] * sIs[f];
                        if (bt.H) gi += bound_grad(bt, f, xr[t]);
                        grad_out[(int64_t)f * M + i] = grad_scale * gi;
                    }
                }
            }
        }
    }
    for (int s = threadIdx.x; s < S; s += 64 * NW) {
        const int i = row0 + s;
        if (i < M) {
            float y = m.b3;
            for (int w = 0; w < NW; ++w) y += sYp[w][s];
            if (y_out) y_out[i] = y;
            if (cost_out) cost_out[i] = expm1f(y) + (bt.H ? bound_cost(bt, X, x_mode, M, n_in, i) : 0.0f);
        }
    }
}
constexpr int kInfWaves = 8;    // waves per workgroup
constexpr int kInfBlocks = 4;   // 16-sample blocks per workgroup
constexpr int kInfRows = 16 * kInfBlocks;

// Training forward + backward of a minibatch (M a multiple of 64, inputs AoS):
// sample i is dataset row src = idx ? idx[i] : i of X [n_rows][n_in], its
// target log(1 + cost[src]).  An index outside [0, n_rows) reads row 0 and
// sets STAMP_STATUS_BAD_INDEX.
// A workgroup of four waves takes kTrainRows = 16 samples and each wave 64 of
// every layer's 256 neurons (four 16-neuron blocks), the activations passing
// between the waves through LDS; every block's weight fragments load while
// the previous block computes.
// Writes feature-major BF16 activations for the weight gradients and per-tile
// partial sums: part[tile][0..255] = sum delta1, [256..511] = sum delta2,
// [512..767] = sum delta3 * h2, [768] = sum delta3, [769] = sum (y - t)^2 / M.
__global__ __launch_bounds__(256) void k_mlp_train_fb(const float* __restrict__ P, const __bf16* __restrict__ Wb,
                                                      const float* __restrict__ X, const float* __restrict__ cost,
                                                      const int* __restrict__ idx, int n_rows, int M, int n_in,
                                                      uint32_t* __restrict__ status, __bf16* __restrict__ UT,
                                                      __bf16* __restrict__ H1T, __bf16* __restrict__ D2T,
                                                      __bf16* __restrict__ D1T, float* __restrict__ part) {
    static_assert(kTrainRows == 16, "one 16-row block per workgroup");
    constexpr int NB = kW / 16 / 4;  // 16-neuron blocks per wave
    __shared__ __bf16 sU[16 * kLdU];
    __shared__ __bf16 sH[16 * kLdH];
    __shared__ __bf16 sD[16 * kLdH];
    __shared__ float sRed[kMlpPartStride];
    __shared__ float sY[4][16];
    __shared__ int sSrc[16];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int kq = l >> 4, col = l & 15;
    const int row0 = blockIdx.x * kTrainRows;
    const int nb0 = wave * NB;  // the wave's first neuron block
    const MlpPtrs m = mlp_ptrs(P, Wb);
    const float inv_m = 1.0f / (float)M;

    if (threadIdx.x < 16) {
        int src = idx ? idx[row0 + threadIdx.x] : row0 + threadIdx.x;
        if (src < 0 || src >= n_rows) {
            if (status) atomicOr(status, (uint32_t)STAMP_STATUS_BAD_INDEX);
            src = 0;
        }
        sSrc[threadIdx.x] = src;
    }
    __syncthreads();
    if (wave == 0) stage_inputs(sU, m, X, 0, M, n_in, 0, nullptr, row0, sSrc);
    __syncthreads();
    // U^T for dW1
    for (int e = threadIdx.x; e < kIn * 16; e += 256) {
        const int f = e >> 4, r = e & 15;
        UT[(int64_t)f * M + row0 + r] = sU[r * kLdU + f];
    }
    // layer 1 on the wave's neurons: z1 kept for delta1, h1 to LDS
    f4 z1[NB];
    float b1v[NB];
    {
        bf16x8 w0[kIn / 32], w1[kIn / 32];
        b1v[0] = m.b1[nb0 * 16 + col];
        load_wfrag<kIn>(w0, m.W1, kIn, nb0 * 16);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const int cb = nb0 + a;
            if (a + 1 < NB) {
                load_wfrag<kIn>(w1, m.W1, kIn, (cb + 1) * 16);
                b1v[a + 1] = m.b1[(cb + 1) * 16 + col];
            }
            z1[a] = mma_rows_w<kIn>(sU, kLdU, w0, f4{0.f, 0.f, 0.f, 0.f});
            const int c = cb * 16 + col;
            for (int j = 0; j < 4; ++j) {
                const __bf16 h = (__bf16)gelu(z1[a][j] + b1v[a]);
                sH[(4 * kq + j) * kLdH + c] = h;
                H1T[(int64_t)c * M + row0 + 4 * kq + j] = h;
            }
#pragma unroll
            for (int k = 0; k < kIn / 32; ++k) w0[k] = w1[k];
        }
    }
    __syncthreads();
    // layer 2 on the wave's neurons and their part of y
    f4 z2[NB];
    float w3v[NB];
    float yp[4] = {0.f, 0.f, 0.f, 0.f};
    {
        bf16x8 v0[kW / 32], v1[kW / 32];
        float b20 = m.b2[nb0 * 16 + col], b21 = 0.0f;
        w3v[0] = m.w3[nb0 * 16 + col];
        load_wfrag<kW>(v0, m.W2, kW, nb0 * 16);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const int cb = nb0 + a;
            if (a + 1 < NB) {
                load_wfrag<kW>(v1, m.W2, kW, (cb + 1) * 16);
                b21 = m.b2[(cb + 1) * 16 + col];
                w3v[a + 1] = m.w3[(cb + 1) * 16 + col];
            }
            f4 acc = mma_rows_w<kW>(sH, kLdH, v0, f4{0.f, 0.f, 0.f, 0.f});
            for (int j = 0; j < 4; ++j) {
                acc[j] += b20;
                yp[j] += w3v[a] * gelu(acc[j]);
            }
            z2[a] = acc;
#pragma unroll
            for (int k = 0; k < kW / 32; ++k) v0[k] = v1[k];
            b20 = b21;
        }
    }
    for (int j = 0; j < 4; ++j) {
        const float v = sum16(yp[j]);
        if (col == 0) sY[wave][4 * kq + j] = v;
    }
    __syncthreads();
    // delta3 = dL/dy = 2 (y - t) / M, y from the waves' parts in wave order
    float d3[4];
    float lsum = 0.0f;
    for (int j = 0; j < 4; ++j) {
        const int r = 4 * kq + j;
        const float y = (((sY[0][r] + sY[1][r]) + sY[2][r]) + sY[3][r]) + m.b3;
        const float e = y - log1pf(cost[sSrc[r]]);
        d3[j] = 2.0f * e * inv_m;
        lsum += e * e * inv_m;
    }
    // delta2 = delta3 w3 gelu'(z2) on the wave's neurons; partial sums of
    // delta2 and delta3 h2
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int c = (nb0 + a) * 16 + col;
        float s2 = 0.0f, s3 = 0.0f;
        for (int j = 0; j < 4; ++j) {
            const float dz = d3[j] * w3v[a] * gelu_grad(z2[a][j]);
            const __bf16 db = (__bf16)dz;
            sD[(4 * kq + j) * kLdH + c] = db;
            D2T[(int64_t)c * M + row0 + 4 * kq + j] = db;
            s2 += dz;
            s3 += d3[j] * gelu(z2[a][j]);
        }
        s2 = sum_groups(s2);
        s3 = sum_groups(s3);
        if (kq == 0) {
            sRed[256 + c] = s2;
            sRed[512 + c] = s3;
        }
    }
    if (wave == 0) {
        float s = d3[0] + d3[1] + d3[2] + d3[3];
        s = sum_groups(s);
        const float ls = sum_groups(lsum);
        if (l == 0) {
            sRed[768] = s;
            sRed[769] = ls;
        }
    }
    __syncthreads();
    // delta1 = (delta2 W2) gelu'(z1) on the wave's neurons
    {
        bf16x8 t0[kW / 32], t1[kW / 32];
        load_wfrag<kW>(t0, m.W2T, kW, nb0 * 16);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const int kb = nb0 + a;
            if (a + 1 < NB) load_wfrag<kW>(t1, m.W2T, kW, (kb + 1) * 16);
            const f4 t = mma_rows_w<kW>(sD, kLdH, t0, f4{0.f, 0.f, 0.f, 0.f});
            const int k = kb * 16 + col;
            float s1 = 0.0f;
            for (int j = 0; j < 4; ++j) {
                const float dz = t[j] * gelu_grad(z1[a][j] + b1v[a]);
                D1T[(int64_t)k * M + row0 + 4 * kq + j] = (__bf16)dz;
                s1 += dz;
            }
            s1 = sum_groups(s1);
            if (kq == 0) sRed[k] = s1;
#pragma unroll
            for (int q = 0; q < kW / 32; ++q) t0[q] = t1[q];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kMlpPartStride; e += 256)
        part[(int64_t)blockIdx.x * kMlpPartStride + e] = e < 770 ? sRed[e] : 0.0f;
}

// Weight-gradient partials of a minibatch split in `splits` sample ranges:
// part[q][c][k] = sum over the samples s of range q of AT[c][s] BT[k][s]
// (AT [nc][M], BT [nk][M], BF16 feature-major; nc, nk multiples of 64).  A
// workgroup of four waves takes a 64 x 64 output tile of one range, each wave
// a 32 x 32 quarter as 2 x 2 MFMA tiles; Adam adds the ranges in order.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const __bf16* __restrict__ AT, const __bf16* __restrict__ BT,
                                                   int M, int nc, int nk, int per, float* __restrict__ part) {
    const int tk = nk / 64;
    const int c0 = (int)(blockIdx.x / tk) * 64, k0 = (int)(blockIdx.x % tk) * 64;
    const int q = blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int r = l & 15, kq = l >> 4;
    const int cw = c0 + 32 * (wave >> 1), kw = k0 + 32 * (wave & 1);
    const int s0 = q * per;
    const __bf16* a0 = AT + (int64_t)(cw + r) * M + 8 * kq;
    const __bf16* b0 = BT + (int64_t)(kw + r) * M + 8 * kq;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int s = s0; s < s0 + per; s += 32) {
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = *reinterpret_cast<const bf16x8*>(a0 + (int64_t)16 * i * M + s);
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = *reinterpret_cast<const bf16x8*>(b0 + (int64_t)16 * j * M + s);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    float* out = part + (int64_t)q * nc * nk;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) out[(int64_t)(cw + 16 * i + 4 * kq + t) * nk + kw + 16 * j + r] = acc[i][j][t];
}

// Sample ranges of the weight gradients: the largest power of two up to 32
// whose ranges are whole 32-sample MFMA steps.
__host__ __device__ __forceinline__ int wgrad_splits(int M) {
    int q = 32;
    while (q > 1 && M % (32 * q)) q >>= 1;
    return q;
}

// Adam on the trained tensors (FP32 master weights): the weight gradients add
// their sample ranges in range order, the bias and output-weight gradients
// the training workgroups' partial sums in workgroup order (32 loads in
// flight).  Element 0 (mu, not trained) writes the loss instead when asked.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ P, float* __restrict__ mom,
                                                  float* __restrict__ vel, const float* __restrict__ dW1,
                                                  const float* __restrict__ dW2, int splits,
                                                  const float* __restrict__ part, int tiles, int n_in, int t,
                                                  float lr, float b1, float b2, float eps, float* loss) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kMlpParams) return;
    // the range sum (stride bytes between ranges) or the workgroup sum
    auto sum = [&](const float* base, int64_t stride, int n) {
        constexpr int F = 32;  // loads in flight (the 16-row tiles of a large batch are many)
        float g = 0.0f;
        for (int q0 = 0; q0 < n; q0 += F) {
            float u[F];
#pragma unroll
            for (int k = 0; k < F; ++k) u[k] = base[(int64_t)min(q0 + k, n - 1) * stride];
#pragma unroll
            for (int k = 0; k < F; ++k)
                if (q0 + k < n) g += u[k];
        }
        return g;
    };
    if (e == 0 && loss) *loss = sum(part + 769, kMlpPartStride, tiles);
    float g;
    if (e >= kMlpOffW1 && e < kMlpOffB1) {
        const int k = (e - kMlpOffW1) / kIn, f = (e - kMlpOffW1) % kIn;
        g = f < n_in ? sum(dW1 + k * kIn + f, (int64_t)kW * kIn, splits) : 0.0f;
    } else if (e >= kMlpOffW2 && e < kMlpOffB2) {
        g = sum(dW2 + (e - kMlpOffW2), (int64_t)kW * kW, splits);
    } else {
        int idx;
        if (e >= kMlpOffB1 && e < kMlpOffW2) idx = e - kMlpOffB1;              // sum delta1
        else if (e >= kMlpOffB2 && e < kMlpOffW3) idx = 256 + (e - kMlpOffB2);  // sum delta2
        else if (e >= kMlpOffW3 && e < kMlpOffB3) idx = 512 + (e - kMlpOffW3);  // sum delta3 h2
        else if (e == kMlpOffB3) idx = 768;                                     // sum delta3
        else return;  // mu, inv_sigma and padding are not trained
        g = sum(part + idx, kMlpPartStride, tiles);
    }
    const float mm = b1 * mom[e] + (1.0f - b1) * g;
    const float vv = b2 * vel[e] + (1.0f - b2) * g * g;
    mom[e] = mm;
    vel[e] = vv;
    const float mhat = mm / (1.0f - powf(b1, (float)t));
    const float vhat = vv / (1.0f - powf(b2, (float)t));
    P[e] = P[e] - lr * mhat / (sqrtf(vhat) + eps);
}

// BF16 working copies of W1, W1^T, W2, W2^T from the FP32 parameters.
__global__ __launch_bounds__(256) void k_mlp_prepare(const float* __restrict__ P, __bf16* __restrict__ Wb) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < kW * kIn) {
        const int k = e / kIn, f = e % kIn;
        const __bf16 w = (__bf16)P[kMlpOffW1 + e];
        Wb[kMlpBfW1 + e] = w;
        Wb[kMlpBfW1T + f * kW + k] = w;
    }
    if (e < kW * kW) {
        const int c = e / kW, k = e % kW;
        const __bf16 w = (__bf16)P[kMlpOffW2 + e];
        Wb[kMlpBfW2 + e] = w;
        Wb[kMlpBfW2T + k * kW + c] = w;
    }
}

// mu and inv_sigma from the data: mean and population standard deviation of
// each input over the M rows of X [M][n_in] (FP64 sums, two passes, one
// workgroup: 16 row lanes x 64 features, summed in a fixed order).
// inv_sigma = 1 / max(sigma, 1e-3); padded inputs get mu 0, inv_sigma 1.
// With cost, b3 = mean log(1 + cost) (the mean training target).
__global__ __launch_bounds__(1024) void k_mlp_standardize(const float* __restrict__ X, const float* __restrict__ cost,
                                                          int M, int n_in, float* __restrict__ P) {
    __shared__ double red[16][kIn];
    __shared__ double mean[kIn];
    __shared__ double tsum[1024];
    const int f = threadIdx.x & 63, r = threadIdx.x >> 6;
    double s = 0.0;
    if (f < n_in)
        for (int64_t i = r; i < M; i += 16) s += (double)X[i * n_in + f];
    red[r][f] = s;
    __syncthreads();
    if (r == 0) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += red[q][f];
        mean[f] = t / (double)M;
    }
    __syncthreads();
    const double mu = mean[f];
    s = 0.0;
    if (f < n_in)
        for (int64_t i = r; i < M; i += 16) {
            const double e = (double)X[i * n_in + f] - mu;
            s += e * e;
        }
    __syncthreads();
    red[r][f] = s;
    __syncthreads();
    if (r == 0) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += red[q][f];
        const double sd = sqrt(t / (double)M);
        P[kMlpOffMu + f] = f < n_in ? (float)mu : 0.0f;
        P[kMlpOffIsig + f] = f < n_in ? (float)(1.0 / fmax(sd, 1e-3)) : 1.0f;
    }
    if (cost) {
        double t = 0.0;
        for (int64_t i = threadIdx.x; i < M; i += 1024) t += log1p((double)cost[i]);
        tsum[threadIdx.x] = t;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) tsum[threadIdx.x] += tsum[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) P[kMlpOffB3] = (float)(tsum[0] / (double)M);
    }
}

// Training rows from particles: Xo[i][f] = theta[f][i] for f < d, enc[f - d] after.
__global__ void k_mlp_pack_rows(const float* __restrict__ theta, int N, int d, const float* __restrict__ enc,
                                int n_in, float* __restrict__ Xo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * n_in) return;
    const int i = (int)(e / n_in), f = (int)(e % n_in);
    Xo[e] = f < d ? theta[(int64_t)f * N + i] : enc[f - d];
}

// Surrogate check: out[p] = mean_i |log(1 + c_sur_i) - log(1 + c_true_i)| over
// problem p's particles (one workgroup per problem, fixed-order tree sum).
__global__ __launch_bounds__(256) void k_log_err(const ProblemDesc* __restrict__ descs, const float* __restrict__ c_true,
                                                 const float* __restrict__ c_sur, float* __restrict__ out) {
    __shared__ float red[256];
    const int p = blockIdx.x;
    const int N = descs[p].N;
    const int64_t off = descs[p].cost_off;
    float s = 0.0f;
    for (int i = threadIdx.x; i < N; i += 256) s += fabsf(log1pf(c_sur[off + i]) - log1pf(c_true[off + i]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = red[0] / (float)N;
}


}  // namespace

hipError_t launch_mlp_prepare(const float* P, __bf16* Wb, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_prepare, dim3((kW * kW + 255) / 256), dim3(256), 0, st, P, Wb);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* P, const __bf16* Wb, const float* X, int x_mode, int M, int n_in, int d,
                            const float* enc, int bound_H, float wb, float omax, float dmax, float* y_out,
                            float* cost_out, float* grad_out, float grad_scale, hipStream_t st) {
    const BoundTerm bt{bound_H, wb, omax, dmax};
    hipLaunchKernelGGL((k_mlp_infer<kInfWaves, kInfBlocks>), dim3((M + kInfRows - 1) / kInfRows), dim3(64 * kInfWaves), 0,
                       st, P, Wb, X,
                       x_mode, M, n_in, d, enc, bt, y_out, cost_out, grad_out, grad_scale);
    return hipGetLastError();
}

hipError_t launch_log_err(const ProblemDesc* descs, int n_problems, const float* c_true, const float* c_sur,
                          float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_log_err, dim3(n_problems), dim3(256), 0, st, descs, c_true, c_sur, out);
    return hipGetLastError();
}

hipError_t launch_mlp_standardize(const float* X, const float* cost, int M, int n_in, float* P, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_standardize, dim3(1), dim3(1024), 0, st, X, cost, M, n_in, P);
    return hipGetLastError();
}

hipError_t launch_mlp_pack_rows(const float* theta, int N, int d, const float* enc, int n_in, float* Xo,
                                hipStream_t st) {
    const int64_t n = (int64_t)N * n_in;
    hipLaunchKernelGGL(k_mlp_pack_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, N, d, enc, n_in,
                       Xo);
    return hipGetLastError();
}

MlpTrainLayout mlp_train_layout(int M) {
    MlpTrainLayout L{};
    const size_t act = (size_t)M * 2;  // bytes per feature row of a bf16 activation
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    L.ut = take(act * kIn);
    L.h1t = take(act * kW);
    L.d2t = take(act * kW);
    L.d1t = take(act * kW);
    L.dw1 = take((size_t)wgrad_splits(M) * kW * kIn * 4);
    L.dw2 = take((size_t)wgrad_splits(M) * kW * kW * 4);
    L.part = take((size_t)(M / kTrainRows) * kMlpPartStride * 4);
    L.total = off;
    return L;
}

hipError_t launch_mlp_train_step(float* P, __bf16* Wb, float* mom, float* vel, int t, float lr, float b1, float b2,
                                 float eps, const float* X, const float* cost, const int* idx, int n_rows, int M,
                                 int n_in, float* loss_out, uint32_t* status, char* ws, const MlpTrainLayout& L,
                                 hipStream_t st) {
    __bf16* UT = reinterpret_cast<__bf16*>(ws + L.ut);
    __bf16* H1T = reinterpret_cast<__bf16*>(ws + L.h1t);
    __bf16* D2T = reinterpret_cast<__bf16*>(ws + L.d2t);
    __bf16* D1T = reinterpret_cast<__bf16*>(ws + L.d1t);
    float* dW1 = reinterpret_cast<float*>(ws + L.dw1);
    float* dW2 = reinterpret_cast<float*>(ws + L.dw2);
    float* part = reinterpret_cast<float*>(ws + L.part);
    const int tiles = M / kTrainRows;
    const int splits = wgrad_splits(M), per = M / splits;
    hipLaunchKernelGGL(k_mlp_train_fb, dim3(tiles), dim3(256), 0, st, P, Wb, X, cost, idx, n_rows, M, n_in, status,
                       UT, H1T, D2T, D1T, part);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((kW / 64) * (kW / 64), splits), dim3(256), 0, st, D2T, H1T, M, kW, kW, per,
                       dW2);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((kW / 64) * (kIn / 64), splits), dim3(256), 0, st, D1T, UT, M, kW, kIn, per,
                       dW1);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, P, mom, vel, dW1, dW2, splits,
                       part, tiles, n_in, t, lr, b1, b2, eps, loss_out);
    hipLaunchKernelGGL(k_mlp_prepare, dim3((kW * kW + 255) / 256), dim3(256), 0, st, P, Wb);
    return hipGetLastError();
}

}  // namespace stamp
