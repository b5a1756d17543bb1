// SVGD step on the BF16 matrix cores (the direction of Eq. (1) in reduced
// precision, for iterations whose gradients are approximate anyway).
//
//   bandwidth: h = max(m2 / ln N, 1e-12) with m2 the lower median of the
//     squared distances of a fixed sample of kMedSample particle pairs (all
//     N(N-1)/2 pairs when there are at most that many: then m2 is exact;
//     median.hip, sampled mode);
//   x_i = theta_i - mean theta, x^_i = bf16(sqrt(m) x_i), m = 2 log2(e) / h
//     (centring shrinks the Gram cancellation)
//   K_ij = exp(-max(D_ij, 0) / h) with D_ij = |x_i - x_j|^2, so
//   log2 K_ij = x^_i . x^_j + e_i + e_j, e = -|x^|^2 / 2   (Gram on MFMA, FP32 accumulate)
// e_i rides in two more Gram columns of the row operand (a BF16 hi/lo pair
// against ones in the column operand) and e_j is the Gram accumulator's
// starting value (bf16_operands.h), so the Gram MFMA gives log2 K itself: one
// exponential per element, whose clamp to [0, 1] is the max(D, 0).
//   V_j = bf16[ g_j - (2/h) x_j | 1 | 0 ]
//   A_i = sum_j bf16(K_ij) V_j                   (MFMA, FP32 accumulate)
//   phi_i = (A_i[0..d) + (2/h) x_i A_i[d]) / N
// which is Eq. (1) with theta_i - theta_j = x_i - x_j.
//
// Contraction tiling: a workgroup owns 64 rows (4 row tiles of 16) and one
// column split, whose columns its 4 waves take in consecutive quarters (each
// wave holds all 64 rows' operands); the waves' sums for those rows are added
// through LDS in wave order before the split's partial is stored, so the
// partials, and the reduce that reads them, are a quarter of what a
// workgroup of 4 x 64 rows would write.  Per 32 columns a wave issues, per row tile, two Gram
// MFMAs (16x16x32) giving S^T for 2 x 16 columns, turns them into K in
// registers (one multiply-add, one exponential per element, one conversion
// per pair) and feeds K as the A operand of the K.V MFMAs.  The S^T output
// layout (lane holds columns j = 4(l/16)+t of row l%16) is exactly an A
// operand whose k index is permuted; V is stored chunk by chunk in that same
// permuted order, so no data moves between the two products and every lane
// reads its 8 V values with one 16-byte load.  V has d + 1 columns rounded up
// to the 16-column tile: 32 for d < 32, 64 for d < 64, 80 for d = 64.
#include <math.h>

#include "bf16_operands.h"
#include "common.h"
#include "internal.h"

namespace stamp {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

struct View16 {  // one problem's BF16-form workspace
    float* smp;
    float* ctr;
    float* nrm;  // e_i = -|x^_i|^2 / 2
    __bf16* xb;  // the Gram's row operand [x^ | e hi | e lo | 0]
    __bf16* xc;  // its column operand [x^ | 1 | 1 | 0]
    __bf16* vt;  // V by 32-particle chunk: [npad / 32][vc][32], particles in MFMA k order
    float* p16;
    SelState* sel;
};

__device__ __forceinline__ View16 view16(const SvgdLayout& L, char* base) {
    View16 v;
    v.smp = reinterpret_cast<float*>(base + L.smp_off);
    v.ctr = reinterpret_cast<float*>(base + L.ctr_off);
    v.nrm = reinterpret_cast<float*>(base + L.nrm_off);
    v.xb = reinterpret_cast<__bf16*>(base + L.xb_off);
    v.xc = reinterpret_cast<__bf16*>(base + L.xc_off);
    v.vt = reinterpret_cast<__bf16*>(base + L.vt_off);
    v.p16 = reinterpret_cast<float*>(base + L.p16_off);
    v.sel = reinterpret_cast<SelState*>(base + L.sel_off);
    return v;
}

// Layout of V within a 32-particle chunk q: column c occupies the 32 values
// at (q vc + c) 32; lane group kq of the K.V MFMA holds k slots 8 kq ..
// 8 kq + 7, which are the chunk's particles 4 kq .. 4 kq + 3 and then
// 16 + 4 kq .. 16 + 4 kq + 3.

// ---- operands: the scaled rows x^ and e need h, V needs g and h; both are
// packed after the bandwidth (bf16_operands.h for the rows).  A workgroup
// takes 64 padded rows (blockIdx.y picks them within a 256-row chunk, so the
// grid fills more of the chip).
// V: a thread per (32-particle chunk, column, lane group kq) makes one
// 16-byte store, the 8 values that lane group of the K.V product reads.
__device__ void pack16_v_rows(int N, int d, int kd, int vc, int row0, const float* __restrict__ theta,
                              const float* __restrict__ g, const View16& w) {
    const float c2 = 2.0f / w.sel->h;
    const int per = 4 * vc;  // stores per chunk
    row0 += 64 * blockIdx.y;
    pack16_theta_rows(N, d, kd, row0, threadIdx.x, theta, w.ctr, sqrtf(2.0f * 1.44269504088896341f / w.sel->h),
                      w.xb, w.xc, w.nrm);
    for (int o = threadIdx.x; o < 2 * per; o += 256) {
        const int q = (row0 >> 5) + o / per, c = (o >> 2) % vc, kq = o & 3;
        const float ctr = c < d ? w.ctr[c] : 0.0f;
        bf16x8 v;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int i = 32 * q + 4 * kq + (s & 3) + (s >= 4 ? 16 : 0);
            float x = 0.0f;
            if (i < N) x = c < d ? fmaf(-c2, theta[(int64_t)c * N + i] - ctr, g[(int64_t)c * N + i]) : (c == d ? 1.0f : 0.0f);
            v[s] = (__bf16)x;
        }
        *reinterpret_cast<bf16x8*>(w.vt + ((int64_t)q * vc + c) * 32 + 8 * kq) = v;
    }
}

// ---- contraction: partial sums of K V over columns [j0, j1) ----------------------
// Operands of one 32-column chunk, as this lane holds them.
template <int KS, int OT>
struct Chunk16 {
    bf16x8 xj[2][KS];  // A of the Gram (column operand): rows j = jc + 16 sub + (l % 16)
    f4 nj[2];          // e_j for j = jc + 16 sub + 4 (l / 16) + t: the Gram accumulator's start
    bf16x8 vb[OT];     // B of K.V: V[j][16 o + l % 16], j in the permuted order
};

template <int KD, int VC>
__device__ __forceinline__ void load_chunk(Chunk16<KD / 32, VC / 16>& c, const View16& w, int npad, int jc, int col,
                                           int kq) {
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
        const int j = jc + 16 * sub + col;
#pragma unroll
        for (int ks = 0; ks < KD / 32; ++ks)
            c.xj[sub][ks] = *reinterpret_cast<const bf16x8*>(w.xc + (int64_t)j * KD + 32 * ks + 8 * kq);
        c.nj[sub] = *reinterpret_cast<const f4*>(w.nrm + jc + 16 * sub + 4 * kq);
    }
    const __bf16* vch = w.vt + ((int64_t)(jc >> 5) * VC + col) * 32 + 8 * kq;
#pragma unroll
    for (int o = 0; o < VC / 16; ++o) c.vb[o] = *reinterpret_cast<const bf16x8*>(vch + 16 * o * 32);
}

// One 32-column chunk for the wave's 4 row tiles: the 8 Gram MFMAs first,
// then K for every row tile (VALU), then the K.V MFMAs, so the VALU work of a
// row tile overlaps the MFMAs still in flight for the next ones.
template <int KD, int VC>
__device__ __forceinline__ void chunk16_compute(const Chunk16<KD / 32, VC / 16>& cur, const bf16x8 (&xi)[4][KD / 32],
                                                f4 (&acc)[4][VC / 16]) {
    constexpr int KS = KD / 32;
    constexpr int OT = VC / 16;
    f4 s[4][2];  // log2 K: x^_i . x^_j + e_i + e_j
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        s[r][0] = cur.nj[0];
        s[r][1] = cur.nj[1];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            s[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.xj[0][ks], xi[r][ks], s[r][0], 0, 0, 0);
            s[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.xj[1][ks], xi[r][ks], s[r][1], 0, 0, 0);
        }
    }
    bf16x8 ka[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float kv[8];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            kv[t] = unit_clamp(hw_exp2(s[r][0][t]));
            kv[4 + t] = unit_clamp(hw_exp2(s[r][1][t]));
        }
        ka[r] = bf16x8{(__bf16)kv[0], (__bf16)kv[1], (__bf16)kv[2], (__bf16)kv[3],
                       (__bf16)kv[4], (__bf16)kv[5], (__bf16)kv[6], (__bf16)kv[7]};
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o) acc[r][o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[r], cur.vb[o], acc[r][o], 0, 0, 0);
}

template <int KD, int VC>
__device__ void phi16_body(int npad, int row0, int j0, int j1, int split, const View16& w) {
    constexpr int KS = KD / 32;   // Gram k-steps
    constexpr int OT = VC / 16;   // output column tiles
    __shared__ f4 red[3][4 * OT][64];  // waves 1..3's sums, as their lanes hold them
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int rbase = row0;
    {  // this wave's quarter of the split (a multiple of 32 columns)
        const int q = (j1 - j0) >> 2;
        j0 += wave * q;
        j1 = j0 + q;
    }
    bf16x8 xi[4][KS];  // B of the Gram (row operand)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = rbase + 16 * r + col;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xi[r][ks] = *reinterpret_cast<const bf16x8*>(w.xb + (int64_t)i * KD + 32 * ks + 8 * kq);
    }
    f4 acc[4][OT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o) acc[r][o] = f4{0.f, 0.f, 0.f, 0.f};

    // the next chunk's operands load while this one computes: at kd = 32 two
    // buffers in turn, so no operand is copied between them; the wider Grams
    // copy the next chunk into the current one instead (two live buffers in
    // the unrolled loop would take them past 256 registers, one wave per SIMD)
    Chunk16<KS, OT> c0, c1;
    if (j0 < j1) load_chunk<KD, VC>(c0, w, npad, j0, col, kq);
    if constexpr (KD == 32) {
        for (int jc = j0; jc < j1; jc += 64) {
            if (jc + 32 < j1) load_chunk<KD, VC>(c1, w, npad, jc + 32, col, kq);
            chunk16_compute<KD, VC>(c0, xi, acc);
            if (jc + 32 >= j1) break;
            if (jc + 64 < j1) load_chunk<KD, VC>(c0, w, npad, jc + 64, col, kq);
            chunk16_compute<KD, VC>(c1, xi, acc);
        }
    } else {
        for (int jc = j0; jc < j1; jc += 32) {
            if (jc + 32 < j1) load_chunk<KD, VC>(c1, w, npad, jc + 32, col, kq);
            chunk16_compute<KD, VC>(c0, xi, acc);
            c0 = c1;
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 0; o < OT; ++o) red[wave - 1][r * OT + o][lane] = acc[r][o];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 0; o < OT; ++o) acc[r][o] += red[u][r * OT + o][lane];
    float* out = w.p16 + (int64_t)split * VC * npad;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o)
            *reinterpret_cast<f4*>(out + (int64_t)(16 * o + col) * npad + rbase + 16 * r + 4 * kq) = acc[r][o];
}

// ---- phi from the split sums (fixed split order) ---------------------------
// One thread per element (l, i) adds rows l and d of every split in split
// order, eight loads in flight (indices clamped, so no load is predicated).
__device__ __forceinline__ void split_sums(const float* __restrict__ pl, const float* __restrict__ pd,
                                           int64_t sstride, int splits, float& sl, float& sd) {
    sl = 0.0f;
    sd = 0.0f;
    for (int q0 = 0; q0 < splits; q0 += 4) {
        float a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = min(q0 + u, splits - 1) * sstride;
            a[u] = pl[k];
            b[u] = pd[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u < splits) {
                sl += a[u];
                sd += b[u];
            }
    }
}

// phi (stored when phi is not null) and, with upd, the operands of the
// update of Algorithm 1 on element uoff + l N + i
__device__ ElemOut reduce16_elem(int N, int d, int npad, int vc, int splits, int l, int i, const float* theta,
                                 float* phi, const View16& w, uint32_t* status, const UpdateArgs& upd, bool apply,
                                 int64_t uoff) {
    ElemOut o{true, 0.0f, uoff + (int64_t)l * N + i, {}};
    if (apply) o.in = update_load(upd, o.ue);  // issued with the sums' loads
    float sv, s1;
    split_sums(w.p16 + (int64_t)l * npad + i, w.p16 + (int64_t)d * npad + i, (int64_t)vc * npad, splits, sv, s1);
    const float x = theta[(int64_t)l * N + i] - w.ctr[l];
    o.r = fmaf(2.0f / w.sel->h * x, s1, sv) / (float)N;
    if (phi) phi[(int64_t)l * N + i] = o.r;
    if (status && !isfinite(o.r)) atomicOr(status, STAMP_STATUS_NONFINITE_PHI);
    return o;
}

// ---- single-problem kernels -----------------------------------------------------
struct One16 {
    int N, d;
    SvgdLayout L;
    float fixed_h;
};

__global__ __launch_bounds__(kCentreThreads) void k_center(One16 a, const float* theta, char* ws) {
    particle_mean_body<kCentreThreads>(a.N, blockIdx.x, theta, view16(a.L, ws).ctr);
}

__global__ __launch_bounds__(256) void k_pack16_v(One16 a, const float* theta, const float* g, char* ws) {
    pack16_v_rows(a.N, a.d, a.L.kd, a.L.vc, blockIdx.x * 256, theta, g, view16(a.L, ws));
}

template <int KD, int VC>
__global__ __launch_bounds__(256) void k_phi16(One16 a, char* ws) {
    const int split = blockIdx.y;
    const int j0 = split * a.L.chunk16, j1 = min(j0 + a.L.chunk16, a.L.npad);
    phi16_body<KD, VC>(a.L.npad, blockIdx.x * kTile16, j0, j1, split, view16(a.L, ws));
}

// upd.use_adam < 0: no update
__global__ __launch_bounds__(256) void k_reduce16(One16 a, const float* theta, const float* g, float* phi, char* ws,
                                                  uint32_t* status, UpdateArgs upd) {
    __shared__ float den[2];
    const bool apply = upd.use_adam >= 0;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    ElemOut o{};
    if (e < (int64_t)a.d * a.N) {
        if (a.N == 1) o = pass_elem(g, phi, e, upd, apply);
        else o = reduce16_elem(a.N, a.d, a.L.npad, a.L.vc, a.L.splits16, (int)e / a.N, (int)e % a.N, theta, phi,
                               view16(a.L, ws), status, upd, apply, 0);
    }
    if (apply) {
        block_denominators(upd, den);
        if (o.ok) update_apply(upd, den, o.ue, o.in, o.r);
    }
}

// ---- batched kernels (work-list entries as in svgd.hip) ---------------------------
__device__ __forceinline__ char* base_of(const ProblemDesc& D, char* ws) { return ws + D.svgd_off; }

__global__ __launch_bounds__(256) void k_pack16_v_batched(const ProblemDesc* __restrict__ descs,
                                                          const int4* __restrict__ work, const float* theta,
                                                          const float* grad, char* ws) {
    const int4 e = work[blockIdx.x];
    const ProblemDesc& D = descs[e.x];
    if (D.N < 2) return;
    pack16_v_rows(D.N, D.d, D.sv.kd, D.sv.vc, e.y, theta + D.theta_off, grad + D.theta_off,
                  view16(D.sv, base_of(D, ws)));
}

// entry = (problem, row block, split, -)
template <int KD, int VC>
__global__ __launch_bounds__(256) void k_phi16_batched(const ProblemDesc* __restrict__ descs,
                                                       const int4* __restrict__ work, char* ws) {
    const int4 e = work[blockIdx.x];
    const ProblemDesc& D = descs[e.x];
    const int j0 = e.z * D.sv.chunk16, j1 = min(j0 + D.sv.chunk16, D.sv.npad);
    phi16_body<KD, VC>(D.sv.npad, e.y * kTile16, j0, j1, e.z, view16(D.sv, base_of(D, ws)));
}

// entry = (problem, first element, end element, -) of the problem's d*N block
__global__ __launch_bounds__(256) void k_reduce16_batched(const ProblemDesc* __restrict__ descs,
                                                          const int4* __restrict__ work, const float* theta,
                                                          const float* grad, float* phi, char* ws, uint32_t* status,
                                                          UpdateArgs upd) {
    __shared__ float den[2];
    const bool apply = upd.use_adam >= 0;
    const int4 w = work[blockIdx.x];
    const ProblemDesc& D = descs[w.x];
    const int64_t e = w.y + threadIdx.x;
    ElemOut o{};
    if (e < w.z) {
        if (D.N == 1) o = pass_elem(grad, phi, D.theta_off + e, upd, apply);
        else o = reduce16_elem(D.N, D.d, D.sv.npad, D.sv.vc, D.sv.splits16, (int)e / D.N, (int)e % D.N,
                               theta + D.theta_off, phi ? phi + D.theta_off : nullptr, view16(D.sv, base_of(D, ws)),
                               status, upd, apply, D.theta_off);
    }
    if (apply) {
        block_denominators(upd, den);
        if (o.ok) update_apply(upd, den, o.ue, o.in, o.r);
    }
}

}  // namespace

hipError_t launch_operands16(int N, int d, const float* theta, void* ws, const SvgdLayout& L, hipStream_t st) {
    if (N < 2) return hipSuccess;
    One16 a{N, d, L, 0.0f};
    char* b = static_cast<char*>(ws);
    hipLaunchKernelGGL(k_center, dim3(d), dim3(kCentreThreads), 0, st, a, theta, b);
    return hipGetLastError();
}

hipError_t launch_svgd16_direction(int N, int d, const float* theta, const float* grad, float* phi, void* ws,
                                   const SvgdLayout& L, uint32_t* status, hipStream_t st, const UpdateArgs* upd) {
    One16 a{N, d, L, 0.0f};
    char* b = static_cast<char*>(ws);
    if (N >= 2) {
        hipLaunchKernelGGL(k_pack16_v, dim3(L.npad / 256, 4), dim3(256), 0, st, a, theta, grad, b);
        const dim3 grid(L.npad / kTile16, L.splits16);
        if (L.kd == 32) hipLaunchKernelGGL((k_phi16<32, 32>), grid, dim3(256), 0, st, a, b);
        else if (L.kd == 64) hipLaunchKernelGGL((k_phi16<64, 64>), grid, dim3(256), 0, st, a, b);
        else hipLaunchKernelGGL((k_phi16<96, 80>), grid, dim3(256), 0, st, a, b);
    }
    UpdateArgs u{};
    u.use_adam = -1;
    if (upd) u = *upd;
    const int64_t n = (int64_t)d * N;
    hipLaunchKernelGGL(k_reduce16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, theta, grad, phi, b, status,
                       u);
    return hipGetLastError();
}

hipError_t launch_svgd16(int N, int d, const float* theta, const float* grad, float bandwidth, float* phi,
                         float* h_out, void* ws, const SvgdLayout& L, uint32_t* status, hipStream_t st) {
    hipError_t e = launch_median(N, d, theta, bandwidth, 0, ws, L, h_out, st);
    if (e != hipSuccess) return e;
    if ((e = launch_operands16(N, d, theta, ws, L, st)) != hipSuccess) return e;
    return launch_svgd16_direction(N, d, theta, grad, phi, ws, L, status, st, nullptr);
}

hipError_t launch_svgd16_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, const float* grad,
                                 float* phi, char* ws, uint32_t* status, hipStream_t st) {
    hipError_t e = launch_bandwidth16_batched(P, descs, theta, ws, st);
    if (e != hipSuccess) return e;
    return launch_svgd16_direction_batched(P, descs, theta, grad, phi, ws, status, st, nullptr);
}

hipError_t launch_svgd16_direction_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta,
                                           const float* grad, float* phi, char* ws, uint32_t* status,
                                           hipStream_t st, const UpdateArgs* upd) {
    if (P.n_row16)
        hipLaunchKernelGGL(k_pack16_v_batched, dim3(P.n_row16, 4), dim3(256), 0, st, descs, P.row16_work, theta, grad,
                           ws);
    // a solve's problems have d = 6H <= 48: V takes the padded dimension's width
    if (P.n_phi16[0])
        hipLaunchKernelGGL((k_phi16_batched<32, 32>), dim3(P.n_phi16[0]), dim3(256), 0, st, descs, P.phi16_work[0], ws);
    if (P.n_phi16[1])
        hipLaunchKernelGGL((k_phi16_batched<64, 64>), dim3(P.n_phi16[1]), dim3(256), 0, st, descs, P.phi16_work[1],
                           ws);
    UpdateArgs u{};
    u.use_adam = -1;
    if (upd) u = *upd;
    hipLaunchKernelGGL(k_reduce16_batched, dim3(P.n_red), dim3(256), 0, st, descs, P.red_work, theta, grad, phi, ws,
                       status, u);
    return hipGetLastError();
}

}  // namespace stamp
