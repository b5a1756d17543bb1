// SVGD step on gfx950: median-heuristic bandwidth and the direction of Eq. (1).
//
//   D_ij = sum_l (theta_il - theta_jl)^2           (direct differences, FP32)
//   m2   = exact lower median of D over i < j      (Appendix D-B median heuristic)
//   h    = max(m2 / ln N, 1e-12)
//   phi_i = (1/N) sum_j exp(-D_ij/h) [ g_j + (2/h)(theta_i - theta_j) ]
//
// The median is an exact order statistic found by radix selection over the
// FP32 bit patterns of D (non-negative floats order like unsigned integers):
// pass 0 writes D for every 64x64 tile pair I <= J and histograms bits 30..20,
// passes 1 and 2 histogram bits 19..9 and 8..0 of the survivors.  Per-block
// histograms live in LDS and are flushed with integer atomics (exact, so the
// result does not depend on scheduling).  The contraction recomputes D in
// 256-row x chunk tiles with theta_j and g_j staged through LDS, writes
// per-chunk partial sums, and a second kernel reduces them in a fixed order.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace stamp {

namespace {

constexpr int kTile = 64;          // rows/cols of a distance tile
constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr int kBins0 = 2048, kBins1 = 2048, kBins2 = 512;

struct SelState {
    uint32_t prefix;  // selected high bits so far
    uint32_t rank;    // 1-based rank still to find inside the current prefix
    float h;          // resulting bandwidth
    float m2;         // the median
};

__global__ __launch_bounds__(256) void k_dist_hist0(int N, int d, int nt, const float* __restrict__ theta,
                                                    uint32_t* __restrict__ dist, uint32_t* __restrict__ hist) {
    const int I = blockIdx.y, J = blockIdx.x;
    if (I > J) return;
    __shared__ float ti[64][kTile + 1];
    __shared__ float tj[64][kTile + 1];
    __shared__ uint32_t lh[kBins0];
    const int tid = threadIdx.x;
    for (int b = tid; b < kBins0; b += 256) lh[b] = 0;
    // stage both tiles (d <= 64)
    for (int e = tid; e < d * kTile; e += 256) {
        const int l = e / kTile, r = e % kTile;
        const int gi = I * kTile + r, gj = J * kTile + r;
        ti[l][r] = gi < N ? theta[(int64_t)l * N + gi] : 0.0f;
        tj[l][r] = gj < N ? theta[(int64_t)l * N + gj] : 0.0f;
    }
    __syncthreads();
    const int64_t tile_id = (int64_t)I * nt - (int64_t)I * (I - 1) / 2 + (J - I);
    uint32_t* out = dist + tile_id * (kTile * kTile);
    const int jj = tid & (kTile - 1);
    const int gj = J * kTile + jj;
    for (int q = 0; q < kTile / 4; ++q) {
        const int ii = (tid >> 6) + 4 * q;
        const int gi = I * kTile + ii;
        uint32_t bits = kInvalid;
        if (gi < gj && gj < N) {
            float acc = 0.0f;
            for (int l = 0; l < d; ++l) {
                const float df = ti[l][ii] - tj[l][jj];
                acc = fmaf(df, df, acc);
            }
            bits = __float_as_uint(acc);
            atomicAdd(&lh[bits >> 20], 1u);
        }
        out[ii * kTile + jj] = bits;
    }
    __syncthreads();
    for (int b = tid; b < kBins0; b += 256)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// Histogram of bits [shift, shift+nbits) of the survivors whose bits above
// shift+nbits equal the selected prefix.
template <int NB>
__global__ __launch_bounds__(256) void k_hist_pass(const uint32_t* __restrict__ dist, int64_t n, int shift,
                                                   const SelState* __restrict__ sel, uint32_t* __restrict__ hist) {
    __shared__ uint32_t lh[NB];
    for (int b = threadIdx.x; b < NB; b += 256) lh[b] = 0;
    __syncthreads();
    const uint32_t want = sel->prefix;
    const int hi = shift + __builtin_ctz(NB);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const uint32_t b = dist[e];
        if (b != kInvalid && (b >> hi) == want) atomicAdd(&lh[(b >> shift) & (NB - 1)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NB; b += 256)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// Find the bin holding the remaining rank; extend the prefix.  One block.
template <int NB>
__global__ __launch_bounds__(256) void k_select(const uint32_t* __restrict__ hist, SelState* sel, int first,
                                                int last, int N, float* h_out) {
    constexpr int PER = NB / 256;
    __shared__ uint32_t part[256];
    const int tid = threadIdx.x;
    uint32_t loc[PER];
    uint32_t sum = 0;
    for (int q = 0; q < PER; ++q) {
        loc[q] = hist[tid * PER + q];
        sum += loc[q];
    }
    part[tid] = sum;
    __syncthreads();
    // exclusive prefix of the per-thread sums (serial over 256 values by lane 0
    // is 256 adds; a Hillis-Steele scan keeps it parallel)
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const uint32_t incl = part[tid];
    const uint32_t excl = incl - sum;
    uint32_t rank;
    uint32_t prefix;
    if (first) {
        // rank = ceil(P/2), P = N(N-1)/2
        const uint64_t P = (uint64_t)N * (uint64_t)(N - 1) / 2;
        rank = (uint32_t)((P + 1) / 2);
        prefix = 0;
    } else {
        rank = sel->rank;
        prefix = sel->prefix;
    }
    __syncthreads();
    if (excl < rank && rank <= incl) {
        uint32_t c = excl;
        for (int q = 0; q < PER; ++q) {
            if (c < rank && rank <= c + loc[q]) {
                const uint32_t bin = (uint32_t)(tid * PER + q);
                const uint32_t np = (prefix << __builtin_ctz(NB)) | bin;
                const uint32_t nr = rank - c;
                sel->prefix = np;
                sel->rank = nr;
                if (last) {
                    const float m2 = __uint_as_float(np);
                    float h = m2 / logf((float)N);
                    h = fmaxf(h, 1e-12f);
                    sel->m2 = m2;
                    sel->h = h;
                    if (h_out) *h_out = h;
                }
                break;
            }
            c += loc[q];
        }
    }
}

__global__ void k_set_h(SelState* sel, float h, float* h_out) {
    sel->h = h;
    sel->m2 = -1.0f;
    if (h_out) *h_out = h;
}

// partial[split][l][i] = sum_{j in chunk} K_ij (g_jl + (2/h)(theta_il - theta_jl))
template <int DP>
__global__ __launch_bounds__(256) void k_phi_partial(int N, int d, int chunk, const float* __restrict__ theta,
                                                     const float* __restrict__ g, const SelState* __restrict__ sel,
                                                     float* __restrict__ partial) {
    constexpr int JT = 64;  // columns staged per round
    __shared__ float tj[JT][DP];
    __shared__ float gj[JT][DP];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int split = blockIdx.y;
    const int j0 = split * chunk, j1 = min(j0 + chunk, N);
    const float h = sel->h;
    const float inv_h = 1.0f / h;
    const float c2 = 2.0f * inv_h;
    const int ii = min(i, N - 1);
    float ti[DP], acc[DP];
#pragma unroll
    for (int l = 0; l < DP; ++l) {
        ti[l] = l < d ? theta[(int64_t)l * N + ii] : 0.0f;
        acc[l] = 0.0f;
    }
    for (int jb = j0; jb < j1; jb += JT) {
        const int nj = min(JT, j1 - jb);
        __syncthreads();
        for (int e = threadIdx.x; e < JT * DP; e += 256) {
            const int jj = e / DP, l = e % DP;
            const bool ok = jj < nj && l < d;
            tj[jj][l] = ok ? theta[(int64_t)l * N + jb + jj] : 0.0f;
            gj[jj][l] = ok ? g[(int64_t)l * N + jb + jj] : 0.0f;
        }
        __syncthreads();
        for (int jj = 0; jj < nj; ++jj) {
            float D = 0.0f;
#pragma unroll
            for (int l = 0; l < DP; ++l) {
                const float df = ti[l] - tj[jj][l];
                D = fmaf(df, df, D);
            }
            const float k = expf(-D * inv_h);
#pragma unroll
            for (int l = 0; l < DP; ++l) acc[l] = fmaf(k, fmaf(c2, ti[l] - tj[jj][l], gj[jj][l]), acc[l]);
        }
    }
    if (i < N) {
        float* out = partial + (int64_t)split * d * N;
        for (int l = 0; l < d; ++l) out[(int64_t)l * N + i] = acc[l];
    }
}

__global__ __launch_bounds__(256) void k_phi_reduce(int N, int d, int splits, const float* __restrict__ partial,
                                                    float* __restrict__ phi, uint32_t* status) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)d * N;
    if (e >= n) return;
    float s = 0.0f;
    for (int q = 0; q < splits; ++q) s += partial[(int64_t)q * n + e];
    const float r = s / (float)N;
    phi[e] = r;
    if (status && !isfinite(r)) atomicOr(status, STAMP_STATUS_NONFINITE_PHI);
}

__global__ void k_copy(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) b[e] = a[e];
}

__global__ __launch_bounds__(256) void k_update(int64_t n, float* __restrict__ theta, const float* __restrict__ phi,
                                                float* __restrict__ m, float* __restrict__ v, int t0,
                                                const int* __restrict__ t_dev, float lr, float b1, float b2,
                                                float eps, int use_adam) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float f = phi[e];
    if (!use_adam) {
        theta[e] = theta[e] + lr * f;
        return;
    }
    const int t = t_dev ? t0 + *t_dev + 1 : t0;
    const float gr = -f;
    const float mm = b1 * m[e] + (1.0f - b1) * gr;
    const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    const float mhat = mm / (1.0f - powf(b1, (float)t));
    const float vhat = vv / (1.0f - powf(b2, (float)t));
    theta[e] = theta[e] - lr * mhat / (sqrtf(vhat) + eps);
}

__global__ void k_modes(int N, int H, const float* __restrict__ theta, int32_t* __restrict__ modes) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)N * H) return;
    const int k = (int)(e / N), i = (int)(e % N);
    int best = 0;
    float bv = theta[(int64_t)(6 * k) * N + i];
    for (int s = 1; s < kModes; ++s) {
        const float a = theta[(int64_t)(6 * k + s) * N + i];
        if (a > bv) {
            bv = a;
            best = s;
        }
    }
    modes[e] = best;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void k_incr(int* p) { *p += 1; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <int DP>
hipError_t launch_phi_partial(int N, int d, int chunk, int splits, const float* theta, const float* g,
                              const SelState* sel, float* partial, hipStream_t st) {
    dim3 grid((N + 255) / 256, splits);
    hipLaunchKernelGGL(k_phi_partial<DP>, grid, dim3(256), 0, st, N, d, chunk, theta, g, sel, partial);
    return hipGetLastError();
}

}  // namespace

SvgdLayout svgd_workspace_layout(int N, int d) {
    SvgdLayout L{};
    const int nt = (N + kTile - 1) / kTile;
    L.tiles = nt;
    L.dist_floats = (size_t)nt * (nt + 1) / 2 * kTile * kTile;
    const int rowblocks = (N + 255) / 256;
    int splits = 2048 / rowblocks;
    const int maxs = (N + 15) / 16;
    if (splits > maxs) splits = maxs;
    if (splits < 1) splits = 1;
    L.splits = splits;
    L.part_floats = (size_t)splits * d * N;
    size_t off = 0;
    L.dist_off = off;
    off = align256(off + (N >= 2 ? L.dist_floats * 4 : 0));
    L.hist_off = off;
    off = align256(off + (kBins0 + kBins1 + kBins2) * 4);
    L.sel_off = off;
    off = align256(off + sizeof(SelState));
    L.h_off = L.sel_off;
    L.part_off = off;
    off = align256(off + L.part_floats * 4);
    L.total = off;
    return L;
}

hipError_t launch_svgd(int N, int d, const float* theta, const float* grad_logp, float bandwidth, float* phi,
                       float* h_out, void* ws, const SvgdLayout& L, uint32_t* status, hipStream_t st) {
    char* base = static_cast<char*>(ws);
    SelState* sel = reinterpret_cast<SelState*>(base + L.sel_off);
    hipError_t e;
    if (N == 1) {  // phi = g
        hipLaunchKernelGGL(k_set_h, dim3(1), dim3(1), 0, st, sel, 1.0f, h_out);
        hipLaunchKernelGGL(k_copy, dim3((d + 255) / 256), dim3(256), 0, st, grad_logp, phi, (int64_t)d);
        return hipGetLastError();
    }
    if (bandwidth > 0.0f) {
        hipLaunchKernelGGL(k_set_h, dim3(1), dim3(1), 0, st, sel, bandwidth, h_out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        uint32_t* dist = reinterpret_cast<uint32_t*>(base + L.dist_off);
        uint32_t* h0 = reinterpret_cast<uint32_t*>(base + L.hist_off);
        uint32_t* h1 = h0 + kBins0;
        uint32_t* h2 = h1 + kBins1;
        const int nt = L.tiles;
        hipLaunchKernelGGL(k_fill_u32, dim3((kBins0 + kBins1 + kBins2 + 255) / 256), dim3(256), 0, st, h0, 0u,
                           (int64_t)(kBins0 + kBins1 + kBins2));
        hipLaunchKernelGGL(k_dist_hist0, dim3(nt, nt), dim3(256), 0, st, N, d, nt, theta, dist, h0);
        hipLaunchKernelGGL(k_select<kBins0>, dim3(1), dim3(256), 0, st, h0, sel, 1, 0, N, h_out);
        const int64_t n = (int64_t)L.dist_floats;
        int blocks = (int)((n + 255) / 256);
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_hist_pass<kBins1>, dim3(blocks), dim3(256), 0, st, dist, n, 9, sel, h1);
        hipLaunchKernelGGL(k_select<kBins1>, dim3(1), dim3(256), 0, st, h1, sel, 0, 0, N, h_out);
        hipLaunchKernelGGL(k_hist_pass<kBins2>, dim3(blocks), dim3(256), 0, st, dist, n, 0, sel, h2);
        hipLaunchKernelGGL(k_select<kBins2>, dim3(1), dim3(256), 0, st, h2, sel, 0, 1, N, h_out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    float* partial = reinterpret_cast<float*>(base + L.part_off);
    const int chunk = (N + L.splits - 1) / L.splits;
    if (d <= 8) e = launch_phi_partial<8>(N, d, chunk, L.splits, theta, grad_logp, sel, partial, st);
    else if (d <= 16) e = launch_phi_partial<16>(N, d, chunk, L.splits, theta, grad_logp, sel, partial, st);
    else if (d <= 24) e = launch_phi_partial<24>(N, d, chunk, L.splits, theta, grad_logp, sel, partial, st);
    else if (d <= 32) e = launch_phi_partial<32>(N, d, chunk, L.splits, theta, grad_logp, sel, partial, st);
    else if (d <= 48) e = launch_phi_partial<48>(N, d, chunk, L.splits, theta, grad_logp, sel, partial, st);
    else e = launch_phi_partial<64>(N, d, chunk, L.splits, theta, grad_logp, sel, partial, st);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)d * N;
    hipLaunchKernelGGL(k_phi_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, d, L.splits,
                       partial, phi, status);
    return hipGetLastError();
}

hipError_t launch_update(int64_t n, float* theta, const float* phi, float* m, float* v, int t0, const int* t_dev,
                         float lr, float b1, float b2, float eps, int use_adam, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, theta, phi, m, v, t0,
                       t_dev, lr, b1, b2, eps, use_adam);
    return hipGetLastError();
}

hipError_t launch_modes(int N, int H, const float* theta, int32_t* modes, hipStream_t st) {
    const int64_t n = (int64_t)N * H;
    hipLaunchKernelGGL(k_modes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, H, theta, modes);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_incr(int* p, hipStream_t st) {
    hipLaunchKernelGGL(k_incr, dim3(1), dim3(1), 0, st, p);
    return hipGetLastError();
}

}  // namespace stamp
