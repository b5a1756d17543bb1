// SVGD step on gfx950: median-heuristic bandwidth and the direction of Eq. (1).
//
//   D_ij = sum_l (theta_il - theta_jl)^2           (direct differences, FP32)
//   m2   = exact lower median of D over i < j      (Appendix D-B median heuristic)
//   h    = max(m2 / ln N, 1e-12)
//   phi_i = (1/N) sum_j exp(-D_ij/h) [ g_j + (2/h)(theta_i - theta_j) ]
//
// The median (median.hip) is the exact order statistic of the FP32 distances,
// found by an interval select seeded from a sample of pairs.  The contraction
// runs on the FP32 matrix cores (phi32.hip).  This file holds the workspace
// layout, the step's launchers, the split-sum reduce that the structured
// kernel's contraction shares, the importance weights of Eq. (4), the update
// and small helpers.
//
// Each stage has a single-problem kernel and a batched kernel over a work list
// of many problems; both call the same device body.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace stamp {

namespace {


// ---- bodies -----------------------------------------------------------------

// phi[e] = (sum over splits of partial[q][e], in split order) / N
__device__ __forceinline__ void phi_reduce_elem(int64_t e, int64_t n, int N, int splits,
                                                const float* __restrict__ partial, float* __restrict__ phi,
                                                uint32_t* status) {
    float s = 0.0f;
    for (int q0 = 0; q0 < splits; q0 += 16) {  // 16 independent loads in flight
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = q0 + u < splits ? partial[(int64_t)(q0 + u) * n + e] : 0.0f;
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
    }
    const float r = s / (float)N;
    phi[e] = r;
    if (status && !isfinite(r)) atomicOr(status, STAMP_STATUS_NONFINITE_PHI);
}

// ---- single-problem kernels ---------------------------------------------------

__global__ __launch_bounds__(256) void k_phi_reduce(int N, int d, int splits, const float* __restrict__ partial,
                                                    float* __restrict__ phi, uint32_t* status) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)d * N;
    if (e < n) phi_reduce_elem(e, n, N, splits, partial, phi, status);
}

// ---- batched kernels ----------------------------------------------------------
// Work-list entries are int4 (problem, a, b, c) with a stage-specific meaning.

__device__ __forceinline__ char* svgd_base(const ProblemDesc& D, char* ws) { return ws + D.svgd_off; }

// Importance weights of Eq. (4) for one problem (one workgroup of 256):
// w_j proportional to exp(C_disc,j - C_rel,j), the relaxed over the discrete
// plan's likelihood, scaled to mean 1 (max-subtracted; a non-finite log-weight
// gives weight 0; all non-finite gives equal weights).
__device__ void dsvgd_weights_body(int N, const float* __restrict__ c_rel, const float* __restrict__ c_disc,
                                   float* __restrict__ w) {
    __shared__ float red[256];
    const int tid = threadIdx.x;
    float m = -INFINITY;
    for (int j = tid; j < N; j += 256) {
        const float lw = c_disc[j] - c_rel[j];
        if (isfinite(lw)) m = fmaxf(m, lw);
    }
    red[tid] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    m = red[0];
    __syncthreads();
    if (!isfinite(m)) {
        for (int j = tid; j < N; j += 256) w[j] = 1.0f;
        return;
    }
    double sum = 0.0;
    for (int j = tid; j < N; j += 256) {
        const float lw = c_disc[j] - c_rel[j];
        sum += isfinite(lw) ? (double)expf(lw - m) : 0.0;
    }
    __shared__ double rs[256];
    rs[tid] = sum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) rs[tid] += rs[tid + s];
        __syncthreads();
    }
    const float scale = (float)((double)N / rs[0]);
    for (int j = tid; j < N; j += 256) {
        const float lw = c_disc[j] - c_rel[j];
        w[j] = isfinite(lw) ? expf(lw - m) * scale : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_dsvgd_weights(int N, const float* c_rel, const float* c_disc, float* w) {
    dsvgd_weights_body(N, c_rel, c_disc, w);
}

__global__ __launch_bounds__(256) void k_dsvgd_weights_batched(const ProblemDesc* __restrict__ descs,
                                                               const float* c_rel, const float* c_disc, float* w) {
    const ProblemDesc& D = descs[blockIdx.x];
    dsvgd_weights_body(D.N, c_rel + D.cost_off, c_disc + D.cost_off, w + D.cost_off);
}

__global__ __launch_bounds__(256) void k_update(int64_t n, const float* __restrict__ phi, UpdateArgs u) {
    __shared__ float den[2];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    ElemOut o{};
    if (e < n) o = pass_elem(phi, nullptr, e, u, true);
    block_denominators(u, den);
    if (o.ok) update_apply(u, den, o.ue, o.in, o.r);
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

}  // namespace

SvgdLayout svgd_workspace_layout(int N, int d) {
    SvgdLayout L{};
    const int nt = (N + kTile - 1) / kTile;
    L.tiles = nt;
    {
        const uint64_t P = (uint64_t)N * (uint64_t)(N > 0 ? N - 1 : 0) / 2;
        // the sample bracket holds about 6.6% of the pairs: P/8 leaves room for
        // uneven segments (an overflow falls back to passes over every pair)
        uint64_t cap = P / 8 + (uint64_t)kCandSegs * kCandSegMin;
        cap = (cap + kCandSegs - 1) / kCandSegs * kCandSegs;
        L.cand_cap = (uint32_t)(cap < 0xffff0000ull ? cap : 0xffff0000ull);
        L.med_rows = N > 4096 ? 256 : 64;  // small problems: more, smaller items
        L.med_rb = (N + L.med_rows - 1) / L.med_rows;
        L.med_cc = (N + kMedCols - 1) / kMedCols;
    }
    // column chunks: about 2048 (256-row block x chunk) tiles, >= 16 columns,
    // at most 64 chunks; depends on N only, so every launch shape sums in the
    // same order
    const int rowblocks = (N + 255) / 256;
    int splits = 2048 / rowblocks;
    const int maxs = (N + 15) / 16;
    if (splits > maxs) splits = maxs;
    if (splits > 64) splits = 64;
    if (splits < 1) splits = 1;
    L.splits = splits;
    // FP32 matrix-core form: rows padded to the 256-row block; column splits
    // of a multiple of 16 columns: about 2048 (64-row wave x split) items, but
    // at least 64 columns per split, so that small problems do not pay for many
    // partial sums in the reduce
    L.npad = (N + kRows16 - 1) / kRows16 * kRows16;
    L.ks32 = phi32_ks(d);
    L.ot32 = phi32_ot(d);
    L.split3 = d <= kPhi3MaxD ? 1 : 0;
    if (L.split3) {
        // split form: 64-row workgroups whose 4 waves take quarters of a
        // split (so a split is a multiple of 128 columns); about one full
        // round of resident workgroups (2 per CU: register bound)
        const int rowblocks = L.npad / 64;
        int s3 = (512 + rowblocks / 2) / rowblocks;
        if (s3 > L.npad / 128) s3 = L.npad / 128;
        if (s3 > 32) s3 = 32;
        if (s3 < 1) s3 = 1;
        const int chunk = ((L.npad + s3 - 1) / s3 + 127) / 128 * 128;
        L.splits32 = (L.npad + chunk - 1) / chunk;
        L.chunk32 = chunk;
    } else {
        const int waves = L.npad / 64;
        int s32 = (2048 + waves - 1) / waves;
        if (s32 > L.npad / 64) s32 = L.npad / 64;
        if (s32 < 1) s32 = 1;
        const int chunk = ((L.npad + s32 - 1) / s32 + 15) / 16 * 16;
        L.splits32 = (L.npad + chunk - 1) / chunk;
        L.chunk32 = chunk;
    }
    // the partial sums of both contractions share one region: the FP32
    // matrix-core form's [splits32][16 ot][npad] and the structured kernel's
    // [splits][d][N]
    L.part_floats = std::max((size_t)splits * d * N, (size_t)L.splits32 * 16 * L.ot32 * L.npad);
    size_t off = 0;
    L.cand_off = off;
    off = align256(off + (N >= 2 ? (size_t)L.cand_cap * 4 : 0));
    L.hist_off = off;
    off = align256(off + kMedBins * 4);
    L.cnt_off = off;
    off = align256(off + (size_t)L.med_rb * L.med_cc * 2 * 4);
    L.sel_off = off;
    off = align256(off + sizeof(SelState));
    L.part_off = off;
    off = align256(off + L.part_floats * 4);
    L.x32_off = off;
    off = align256(off + (size_t)L.npad * 4 * L.ks32 * 4);
    L.n32_off = off;
    off = align256(off + (size_t)L.npad * 4);
    L.v32_off = off;
    off = align256(off + (L.split3 ? 0 : (size_t)L.npad * 16 * L.ot32 * 4));
    L.xs3_off = off;
    off = align256(off + (L.split3 ? (size_t)L.npad * 3 * 32 * 2 : 0));
    L.vs3_off = off;
    off = align256(off + (L.split3 ? (size_t)3 * L.npad * 16 * L.ot32 * 2 : 0));
    // BF16 matrix-core form
    L.kd = d <= 30 ? 32 : d <= 62 ? 64 : 96;  // the rows and two more Gram columns for e_i
    L.vc = d <= 30 ? 32 : d <= 62 ? 64 : 80;  // V = [g - (2/h) x | 1 | 0]: d + 1 columns, padded
    {
        // one full round of resident workgroups (3 per CU at 32 Gram
        // columns, 2 at 64, 1 at 96: register bound), not a round and a partial one;
        // a split gives each of its workgroup's 4 waves at least 32 columns
        const int resident = (L.kd == 32 ? 3 : L.kd == 64 ? 2 : 1) * 256;
        const int rowblocks = L.npad / kTile16;
        int s16 = (resident + rowblocks / 2) / rowblocks;
        if (s16 > L.npad / 128) s16 = L.npad / 128;
        if (s16 > 32) s16 = 32;
        if (s16 < 1) s16 = 1;
        const int chunk = ((L.npad + s16 - 1) / s16 + 127) / 128 * 128;
        L.splits16 = (L.npad + chunk - 1) / chunk;
        L.chunk16 = chunk;
    }
    L.smp_off = off;
    off = align256(off + (size_t)kMedSample * 4);
    L.ctr_off = off;
    off = align256(off + 64 * 4);
    L.nrm_off = off;
    off = align256(off + (size_t)L.npad * 4);
    L.xb_off = off;
    off = align256(off + (size_t)L.npad * L.kd * 2);
    L.xc_off = off;
    off = align256(off + (size_t)L.npad * L.kd * 2);
    L.vt_off = off;
    off = align256(off + (size_t)L.vc * L.npad * 2);
    L.p16_off = off;
    off = align256(off + (size_t)L.splits16 * L.vc * L.npad * 4);
    L.sfeat_off = off;
    off = align256(off + (size_t)2 * d * N * 4);
    L.sh_off = off;
    off = align256(off + sizeof(SelState));
    L.total = off;
    return L;
}

hipError_t launch_svgd(int N, int d, const float* theta, const float* grad_logp, float bandwidth, float* phi,
                       float* h_out, void* ws, const SvgdLayout& L, int phi_rows, uint32_t* status, hipStream_t st,
                       const float* wts) {
    hipError_t e = launch_svgd_bandwidth(N, d, theta, bandwidth, h_out, ws, L, st);
    if (e != hipSuccess) return e;
    return launch_svgd_direction(N, d, theta, grad_logp, phi, ws, L, phi_rows, status, st, wts);
}

hipError_t launch_svgd_bandwidth(int N, int d, const float* theta, float bandwidth, float* h_out, void* ws,
                                 const SvgdLayout& L, hipStream_t st) {
    hipError_t e = launch_operands32(N, d, theta, ws, L, st);
    if (e != hipSuccess) return e;
    return launch_median(N, d, theta, bandwidth, 1, ws, L, h_out, st, 1);
}

hipError_t launch_svgd_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, const float* grad,
                               float* phi, char* ws, uint32_t* status, hipStream_t st, const float* wts) {
    hipError_t e = launch_svgd_bandwidth_batched(P, descs, theta, 1, ws, st);
    if (e != hipSuccess) return e;
    return launch_svgd_direction_batched(P, descs, theta, grad, phi, ws, status, st, wts);
}

hipError_t launch_svgd_bandwidth_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, int exact,
                                         char* ws, hipStream_t st, int* step) {
    // the theta-only operands of the FP32 form (exact median, whose all-pairs
    // passes read them) or of the BF16 form (sampled median)
    if (!exact) return launch_bandwidth16_batched(P, descs, theta, ws, st, step);
    hipError_t e;
    if ((e = launch_operands32_batched(P, descs, theta, ws, st, step)) != hipSuccess) return e;
    return launch_median_batched(P, descs, theta, 1, ws, st);
}

hipError_t launch_phi_reduce(int N, int d, int splits, const float* partial, float* phi, uint32_t* status,
                             hipStream_t st) {
    const int64_t n = (int64_t)d * N;
    hipLaunchKernelGGL(k_phi_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, d, splits, partial, phi,
                       status);
    return hipGetLastError();
}

hipError_t launch_dsvgd_weights(int N, const float* c_rel, const float* c_disc, float* w, hipStream_t st) {
    hipLaunchKernelGGL(k_dsvgd_weights, dim3(1), dim3(256), 0, st, N, c_rel, c_disc, w);
    return hipGetLastError();
}

hipError_t launch_dsvgd_weights_batched(int n_problems, const ProblemDesc* descs, const float* c_rel,
                                        const float* c_disc, float* w, hipStream_t st) {
    hipLaunchKernelGGL(k_dsvgd_weights_batched, dim3(n_problems), dim3(256), 0, st, descs, c_rel, c_disc, w);
    return hipGetLastError();
}

hipError_t launch_update(int64_t n, float* theta, const float* phi, float* m, float* v, int t0, const int* t_dev,
                         float lr, float b1, float b2, float eps, int use_adam, hipStream_t st) {
    const UpdateArgs u{theta, m, v, t0, t_dev, lr, b1, b2, eps, use_adam};
    hipLaunchKernelGGL(k_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, phi, u);
    return hipGetLastError();
}

hipError_t launch_modes(int N, int H, const float* theta, int32_t* modes, hipStream_t st) {
    const int64_t n = (int64_t)N * H;
    hipLaunchKernelGGL(k_modes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, H, theta, modes);
    return hipGetLastError();
}

// The discrete plan as a particle: logits 40 e_Gamma - 20 per push (Gamma the
// argmax side, lowest index on ties), offsets and depths copied.
__global__ void k_onehot(int N, int H, const float* __restrict__ theta, float* __restrict__ out) {
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
    for (int s = 0; s < kModes; ++s) out[(int64_t)(6 * k + s) * N + i] = s == best ? 20.0f : -20.0f;
    out[(int64_t)(6 * k + 4) * N + i] = theta[(int64_t)(6 * k + 4) * N + i];
    out[(int64_t)(6 * k + 5) * N + i] = theta[(int64_t)(6 * k + 5) * N + i];
}

hipError_t launch_onehot(int N, int H, const float* theta, float* out, hipStream_t st) {
    const int64_t n = (int64_t)N * H;
    hipLaunchKernelGGL(k_onehot, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, H, theta, out);
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
