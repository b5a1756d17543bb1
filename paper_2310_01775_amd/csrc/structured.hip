// SVGD direction under the structured pusher kernel (Appendix E-C):
//
//   K(theta, theta') = sum_k [ alpha_g exp(-|g_k - g_k'|^2 / h_g)
//                             + alpha_z exp(-|s_k - s_k'|^2 / h_z),  s_k = softmax(a_k)
//                             + alpha_p exp(kappa (cos(p_k - p_k') - 1)) ]
//   phi_i = (1/N) sum_j w_j [ K(theta_j, theta_i) g_j + grad_{theta_j} K(theta_j, theta_i) ]
//
// with the per-pair kernel gradient written out term by term:
//   RBF on g:       (2 alpha_g / h_g) (g_i - g_j) e_g
//   RBF on softmax: J(a_j) (2 alpha_z / h_z) (s_i - s_j) e_z,  J = diag(s_j) - s_j s_j^T,
//                   so J u = s_j (u - s_j . u)
//   von Mises:      alpha_p kappa sin(p_i - p_j) e_p,  the angle difference from
//                   the cosines and sines of both angles.
//
// Layouts: push = per action [a_k (4 logits), o_k, D_k] with g_k = (o_k, D_k)
// and no angle (d = 6K); pose = [a_1..a_K, (x, y, phi)_1..K] with g_k = (x, y)
// and p_k = phi (d = 7K).  Bandwidths: per component, the median heuristic on
// the features of every action, h_c = max(m2_c / ln N, 1e-12) / K (the exact
// lower median from median.hip), unless the caller fixes them.
//
// Data flow: a prep kernel writes the features in structure-of-arrays form
// (rows 4k+c: softmax; 4K+2k+c: g; 6K+2k, 6K+2k+1: cos p, sin p); the two
// medians run on the softmax and g rows, each into its own selection state,
// which the contraction reads; the contraction (one thread per row
// i, columns staged through LDS, the layout fixed at compile time so every
// accumulator index is a constant) writes per-chunk partial sums that the
// plain step's reduce kernel sums in a fixed order.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace stamp {

namespace {

template <int LAYOUT>
struct Lay;

template <>
struct Lay<kStructPush> {
    static constexpr int per = 6, angles = 0;
    __host__ __device__ static constexpr int a(int, int k, int c) { return 6 * k + c; }
    __host__ __device__ static constexpr int g(int, int k, int c) { return 6 * k + 4 + c; }
    __host__ __device__ static constexpr int p(int, int) { return -1; }
};

template <>
struct Lay<kStructPose> {
    static constexpr int per = 7, angles = 1;
    __host__ __device__ static constexpr int a(int, int k, int c) { return 4 * k + c; }
    __host__ __device__ static constexpr int g(int K, int k, int c) { return 4 * K + 3 * k + c; }
    __host__ __device__ static constexpr int p(int K, int k) { return 4 * K + 3 * k + 2; }
};

// ---- features, one thread per particle -----------------------------------------
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_struct_prep(int N, int K, const float* __restrict__ theta,
                                                     float* __restrict__ feat) {
    using L = Lay<LAYOUT>;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    for (int k = 0; k < K; ++k) {
        float a[4], m = -INFINITY;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            a[c] = theta[(int64_t)L::a(K, k, c) * N + i];
            m = fmaxf(m, a[c]);
        }
        float e[4], s = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            e[c] = expf(a[c] - m);
            s += e[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) feat[(int64_t)(4 * k + c) * N + i] = e[c] / s;
#pragma unroll
        for (int c = 0; c < 2; ++c) feat[(int64_t)(4 * K + 2 * k + c) * N + i] = theta[(int64_t)L::g(K, k, c) * N + i];
        if constexpr (L::angles != 0) {
            const float p = theta[(int64_t)L::p(K, k) * N + i];
            feat[(int64_t)(6 * K + 2 * k) * N + i] = cosf(p);
            feat[(int64_t)(6 * K + 2 * k + 1) * N + i] = sinf(p);
        }
    }
}

// Bandwidth c: the fixed value, or the median heuristic's m2 / ln N (floored)
// over K, from that component's own median state.
struct StructBw {
    const SelState* sel[2];  // g, softmax
    float fixed[2];
    int K;
    __device__ __forceinline__ float h(int c) const { return fixed[c] > 0.0f ? fixed[c] : sel[c]->h / (float)K; }
};

// N = 1: phi = g
__global__ void k_struct_single(int d, const float* __restrict__ g, float* __restrict__ phi) {
    for (int l = threadIdx.x; l < d; l += blockDim.x) phi[l] = g[l];
}

// the bandwidths for the caller (a lone particle reports the fixed ones, else 1)
__global__ void k_struct_hout(StructBw bw, int N, float* __restrict__ h_out) {
    if (threadIdx.x < 2) {
        const int c = threadIdx.x;
        h_out[c] = N > 1 ? bw.h(c) : (bw.fixed[c] > 0.0f ? bw.fixed[c] : 1.0f);
    }
}

struct StructArgs {
    int N, chunk;
    float alpha_g, alpha_z, alpha_p, kappa;
    const float* feat;
    const float* grad;
    const float* wts;
    StructBw bw;
    float* partial;
};

// ---- contraction: partial sums over the columns of one chunk --------------------
template <int KA, int LAYOUT>
__global__ __launch_bounds__(256) void k_struct_partial(StructArgs a) {
    using L = Lay<LAYOUT>;
    constexpr int NA = L::angles;
    constexpr int NF = KA * (6 + 2 * NA);  // staged features per column
    constexpr int D = KA * L::per;         // coordinates
    constexpr int JT = 64;
    constexpr float kLog2e = 1.44269504088896341f;
    __shared__ float fj[JT][NF];
    __shared__ float gj[JT][D];
    __shared__ float wj[JT];
    const int N = a.N;
    const int split = blockIdx.y;
    const int j0 = split * a.chunk, j1 = min(j0 + a.chunk, N);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ii = min(i, N - 1);
    const float hg = a.bw.h(0), hz = a.bw.h(1);
    const float cg = -kLog2e / hg, cz = -kLog2e / hz, cp = a.kappa * kLog2e;
    const float rg0 = 2.0f * a.alpha_g / hg, rz0 = 2.0f * a.alpha_z / hz, rp0 = a.alpha_p * a.kappa;
    float fi[NF], acc[D];
#pragma unroll
    for (int f = 0; f < NF; ++f) fi[f] = a.feat[(int64_t)f * N + ii];
#pragma unroll
    for (int l = 0; l < D; ++l) acc[l] = 0.0f;
    for (int jb = j0; jb < j1; jb += JT) {
        const int njc = min(JT, j1 - jb);
        __syncthreads();
        for (int e = threadIdx.x; e < JT * NF; e += blockDim.x) {  // consecutive threads, consecutive columns
            const int jj = e % JT, f = e / JT;
            fj[jj][f] = jj < njc ? a.feat[(int64_t)f * N + jb + jj] : 0.0f;
        }
        for (int e = threadIdx.x; e < JT * D; e += blockDim.x) {
            const int jj = e % JT, l = e / JT;
            gj[jj][l] = jj < njc ? a.grad[(int64_t)l * N + jb + jj] : 0.0f;
        }
        for (int jj = threadIdx.x; jj < JT; jj += blockDim.x) wj[jj] = (a.wts && jj < njc) ? a.wts[jb + jj] : 1.0f;
        __syncthreads();
        for (int jj = 0; jj < njc; ++jj) {
            const float w = wj[jj];
            const float rz1 = rz0 * w, rg1 = rg0 * w, rp1 = rp0 * w;
            float ksum = 0.0f;
#pragma unroll
            for (int k = 0; k < KA; ++k) {
                // RBF on softmax(a_k), its gradient through the softmax at a_j
                float u[4], dz = 0.0f, su = 0.0f;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    u[c] = fi[4 * k + c] - fj[jj][4 * k + c];
                    dz = fmaf(u[c], u[c], dz);
                    su = fmaf(fj[jj][4 * k + c], u[c], su);
                }
                const float ez = hw_exp2(cz * dz);
                const float rz = rz1 * ez;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[L::a(KA, k, c)] = fmaf(rz * fj[jj][4 * k + c], u[c] - su, acc[L::a(KA, k, c)]);
                // RBF on g_k
                const float v0 = fi[4 * KA + 2 * k] - fj[jj][4 * KA + 2 * k];
                const float v1 = fi[4 * KA + 2 * k + 1] - fj[jj][4 * KA + 2 * k + 1];
                const float eg = hw_exp2(cg * fmaf(v0, v0, v1 * v1));
                const float rg = rg1 * eg;
                acc[L::g(KA, k, 0)] = fmaf(rg, v0, acc[L::g(KA, k, 0)]);
                acc[L::g(KA, k, 1)] = fmaf(rg, v1, acc[L::g(KA, k, 1)]);
                ksum = fmaf(a.alpha_z, ez, fmaf(a.alpha_g, eg, ksum));
                if constexpr (NA != 0) {  // von Mises on p_k
                    const float ci = fi[6 * KA + 2 * k], si = fi[6 * KA + 2 * k + 1];
                    const float cj = fj[jj][6 * KA + 2 * k], sj = fj[jj][6 * KA + 2 * k + 1];
                    const float cd = fmaf(ci, cj, si * sj);   // cos(p_i - p_j)
                    const float sd = fmaf(si, cj, -ci * sj);  // sin(p_i - p_j)
                    const float ep = hw_exp2(cp * (cd - 1.0f));
                    acc[L::p(KA, k)] = fmaf(rp1 * ep, sd, acc[L::p(KA, k)]);
                    ksum = fmaf(a.alpha_p, ep, ksum);
                }
            }
            const float kw = ksum * w;
#pragma unroll
            for (int l = 0; l < D; ++l) acc[l] = fmaf(kw, gj[jj][l], acc[l]);
        }
    }
    if (i < N) {
        float* out = a.partial + (int64_t)split * D * N;
#pragma unroll
        for (int l = 0; l < D; ++l) out[(int64_t)l * N + i] = acc[l];
    }
}

template <int LAYOUT>
void launch_partial(int K, dim3 grid, const StructArgs& a, hipStream_t st) {
    switch (K) {
        case 1: hipLaunchKernelGGL((k_struct_partial<1, LAYOUT>), grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_struct_partial<2, LAYOUT>), grid, dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_struct_partial<3, LAYOUT>), grid, dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_struct_partial<4, LAYOUT>), grid, dim3(256), 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_struct_partial<5, LAYOUT>), grid, dim3(256), 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_struct_partial<6, LAYOUT>), grid, dim3(256), 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_struct_partial<7, LAYOUT>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_struct_partial<8, LAYOUT>), grid, dim3(256), 0, st, a); break;
    }
}

}  // namespace

namespace {

struct StructView {
    float* feat;
    SvgdLayout Lg;  // the layout of the g median: its selection state in the structured region
    StructBw bw;
};

StructView struct_view(void* ws, const SvgdLayout& L, const StructKernel& sk) {
    char* base = static_cast<char*>(ws);
    StructView v;
    v.feat = reinterpret_cast<float*>(base + L.sfeat_off);
    v.Lg = L;
    v.Lg.sel_off = L.sh_off;
    v.bw.sel[0] = reinterpret_cast<const SelState*>(base + v.Lg.sel_off);
    v.bw.sel[1] = reinterpret_cast<const SelState*>(base + L.sel_off);
    v.bw.fixed[0] = sk.h_g;
    v.bw.fixed[1] = sk.h_z;
    v.bw.K = sk.K;
    return v;
}

}  // namespace

// features and the two medians: the g rows (2K) and the softmax rows (4K),
// each into its own selection state
hipError_t launch_struct_bandwidth(int N, const float* theta, const StructKernel& sk, void* ws, const SvgdLayout& L,
                                   hipStream_t st) {
    if (N < 2) return hipSuccess;
    const StructView v = struct_view(ws, L, sk);
    const int K = sk.K;
    hipError_t e;
    if (sk.layout == kStructPush)
        hipLaunchKernelGGL(k_struct_prep<kStructPush>, dim3((N + 255) / 256), dim3(256), 0, st, N, K, theta, v.feat);
    else
        hipLaunchKernelGGL(k_struct_prep<kStructPose>, dim3((N + 255) / 256), dim3(256), 0, st, N, K, theta, v.feat);
    if (!(sk.h_g > 0.0f) &&
        (e = launch_median(N, 2 * K, v.feat + (int64_t)4 * K * N, 0.0f, 1, ws, v.Lg, nullptr, st)) != hipSuccess)
        return e;
    if (!(sk.h_z > 0.0f) && (e = launch_median(N, 4 * K, v.feat, 0.0f, 1, ws, L, nullptr, st)) != hipSuccess)
        return e;
    return hipGetLastError();
}

// the contraction from the features and bandwidths the workspace holds
hipError_t launch_struct_direction(int N, int d, const float* grad, const float* wts, const StructKernel& sk,
                                   float* phi, float* h_out, void* ws, const SvgdLayout& L, uint32_t* status,
                                   hipStream_t st) {
    const StructView v = struct_view(ws, L, sk);
    hipError_t e;
    if (N == 1) {
        hipLaunchKernelGGL(k_struct_single, dim3(1), dim3(64), 0, st, d, grad, phi);
    } else {
        StructArgs a;
        a.N = N;
        a.chunk = (N + L.splits - 1) / L.splits;
        a.alpha_g = sk.alpha_g;
        a.alpha_z = sk.alpha_z;
        a.alpha_p = sk.alpha_p;
        a.kappa = sk.kappa;
        a.feat = v.feat;
        a.grad = grad;
        a.wts = wts;
        a.bw = v.bw;
        a.partial = reinterpret_cast<float*>(static_cast<char*>(ws) + L.part_off);
        const dim3 grid((N + 255) / 256, L.splits);
        if (sk.layout == kStructPush) launch_partial<kStructPush>(sk.K, grid, a, st);
        else launch_partial<kStructPose>(sk.K, grid, a, st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_phi_reduce(N, d, L.splits, a.partial, phi, status, st)) != hipSuccess) return e;
    }
    if (h_out) hipLaunchKernelGGL(k_struct_hout, dim3(1), dim3(64), 0, st, v.bw, N, h_out);
    return hipGetLastError();
}

hipError_t launch_svgd_structured(int N, int d, const float* theta, const float* grad, const float* wts,
                                  const StructKernel& sk, float* phi, float* h_out, void* ws, const SvgdLayout& L,
                                  uint32_t* status, hipStream_t st) {
    hipError_t e = launch_struct_bandwidth(N, theta, sk, ws, L, st);
    if (e != hipSuccess) return e;
    return launch_struct_direction(N, d, grad, wts, sk, phi, h_out, ws, L, status, st);
}

}  // namespace stamp
