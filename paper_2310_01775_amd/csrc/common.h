// Shared device-side definitions of the STAMP hot path (gfx950).
//
// Lane mapping of the rollout kernels: one lane per (particle i, push side s,
// block b), lane = 4 SL i + SL s + b, where SL = 1, 2 or 4 block slots (B
// rounded up; slots b >= B are idle copies of block 0) hold the blocks of the
// sub-rollout of side s (North, East, South, West = 0..3).  The blocks of a
// sub-rollout exchange positions (and, in the reverse sweep, force adjoints)
// by quad_perm DPP moves within their quad; the four sides of a particle meet
// only at phase boundaries, where the phase mixture
// S_{k+1} = sum_s softmax(a_k)_s X_s and the adjoint's per-particle sums are
// cross-lane DPP adds over the particle's 4 SL lanes (no LDS, no barrier).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stamp.h"

namespace stamp {

constexpr int kModes = STAMP_MODES;
constexpr int kMaxBlocks = STAMP_MAX_BLOCKS;
constexpr int kMaxPushes = STAMP_MAX_PUSHES;

// Scene and cost constants in the form the kernels use, derived once on the
// host from stamp_scene / stamp_cost_w (Sec. III-B model, Appendix E-B cost).
struct SimConst {
    int H, B, T;
    float dt;
    float inv_m[kMaxBlocks];   // 1 / m_b
    float inv_I[kMaxBlocks];   // 1 / I_b, I_b = m_b (2 h_b)^2 / 6
    float cf[kMaxBlocks];      // mu_b m_b g           (sliding friction)
    float cr[kMaxBlocks];      // mu_b m_b g rho_b     (spin friction)
    float ev2[kMaxBlocks];     // eps_v^2
    float ew2[kMaxBlocks];     // eps_w^2
    float dtm[kMaxBlocks];     // dt / m_b
    float dtI[kMaxBlocks];     // dt / I_b
    float crw2[kMaxBlocks];    // cr_b eps_w^2 (spin friction derivative)
    float pose0[kMaxBlocks][3];
    float hsum[kMaxBlocks][kMaxBlocks];  // h_b + h_c
    float h0;                  // half size of the pushed block
    float h0d;                 // h0 + standoff
    float kp, kb, beta, inv_beta, er2;
    float beta_log2e;          // beta * log2(e): exp(-beta|z|) = 2^(-beta_log2e |z|)
    float ln2_over_beta;       // log1p(u)/beta = log2(1+u) * ln2/beta
    // cost (Appendix E-B)
    float goal[3], tol;
    float wt, wr, wtr, wb, omax, dmax, ea2;
    // 1: the adjoint returns the gradient of the per-phase split of the cost
    // (each push's parameters follow their own phase's term; no adjoint crosses
    // a phase boundary); 0: the gradient of C
    int per_phase;
};

// Layout of the rollout tape (floats), lane-contiguous so that each lane moves
// its 6B-float state with 3B dwordx2 accesses and a wave touches one contiguous
// 64*24B*B span per entry:
//   entries [n_entries][4N][6B] : pre-step states (every step, or checkpoints)
//   ends    [H][4N][6B]         : sub-rollout states after each phase's last step
//   state order per block b: x, y, phi, vx, vy, omega
struct TapeGeom {
    int64_t lanes;      // 4N
    int64_t n_entries;  // T, or sum_k ceil(L_k / K)
    int64_t ends_off;   // n_entries * 6B * 4N
    int ckpt;           // 0 = full tape
};

// ---- SVGD step layout ---------------------------------------------------------
constexpr int kTile = 64;        // rows/cols of a distance tile
constexpr int kMedBins = 2048;   // bins of one interval-select pass
constexpr int kMedCols = 64;     // columns of an all-pairs work item (rows: med_rows)
constexpr int kCandSegs = 64;    // candidate buffer segments (one counter each)
constexpr int kCandParts = 4;    // workgroups per segment of a candidate pass
constexpr uint32_t kCandSegMin = 16384;  // candidate slots per segment at least

// Median select state (one per problem): the interval [lo, hi] of FP32 bit
// patterns known to hold the median, its rank inside, the pass bookkeeping,
// and the resulting bandwidth.
struct SelState {
    uint32_t lo, hi;     // inclusive interval of bit patterns
    uint32_t rank;       // 1-based rank of the median among the values in it
    uint32_t shift;      // histogram bin = (bits - lo) >> shift
    uint32_t mode;       // 0 done, 1 pass 0 pending, 2 candidate passes, 3 all-pairs passes
    uint32_t overflow;   // pass 0: a candidate segment overflowed
    uint32_t seg[kCandSegs];  // pass 0: slots used in each candidate segment
    float h;             // resulting bandwidth
    float m2;            // the median
};

// Byte offsets inside one problem's SVGD workspace.
struct SvgdLayout {
    size_t cand_off;                // bracket values of the median select (uint32 bit patterns)
    uint32_t cand_cap;              // their capacity: kCandSegs segments of cand_cap / kCandSegs
    size_t cnt_off;                 // per all-pairs item: pairs under, over the bracket
    int med_rows;                   // rows (one per thread) of an all-pairs item: 64 or 256
    int med_rb, med_cc;             // all-pairs items: row blocks x column chunks
    size_t hist_off;                // kMedBins histogram of the median select
    size_t sel_off;                 // SelState
    size_t part_off, part_floats;   // phi partial sums [splits][d][N]
    int splits;                     // column chunks of the phi contraction
    int tiles;                      // 64-row tiles
    // BF16 matrix-core form (sampled median, centred Gram distances)
    int npad;                       // N rounded up to the 256-row block
    // FP32 direction (phi32.hip): on the FP32 matrix cores, or for d <= 31 in
    // split form (every operand as three BF16 parts on the BF16 matrix cores)
    int ks32, ot32;                 // Gram k-steps (4 coordinates each), 16-column tiles of V
    int split3;                     // 1: the split form runs the contraction
    int splits32, chunk32;          // column splits and their width (a multiple of 16; of 128 in split form)
    size_t x32_off;                 // npad x 4 ks32 floats: centred rows in MFMA operand order
    size_t n32_off;                 // npad floats: their squared norms
    size_t v32_off;                 // npad x 16 ot32 floats: V = w [g - (2/h) x | 1 | 0], tiled
    size_t xs3_off;                 // split form: npad x 3 x 32 bf16, the centred rows' three parts (slot 31: -|x|^2/2)
    size_t vs3_off;                 // split form: 3 x npad x 16 ot32 bf16, V's three parts, chunked
    int kd, vc;                     // Gram width (d + 2 rounded up to 32) and V columns (d + 1 rounded up)
    int splits16, chunk16;          // column splits of its contraction and their width
    size_t smp_off;                 // kMedSample floats: the sampled distances
    size_t ctr_off;                 // 64 floats: particle mean
    size_t nrm_off;                 // npad floats: e_i = -|x^_i|^2 / 2
    size_t xb_off;                  // npad x kd bf16: scaled centred rows [x^ | e hi | e lo | 0], the Gram's row operand
    size_t xc_off;                  // npad x kd bf16: the same rows as [x^ | 1 | 1 | 0], its column operand
    size_t vt_off;                  // vc x npad bf16: V = [g - (2/h) x | 1 | 0], chunked
    size_t p16_off;                 // splits16 x vc x npad floats: partial sums
    // structured kernel: per-particle features (at most 2d rows of N floats)
    // and the selection state of its second median
    size_t sfeat_off, sh_off;
    size_t total;
};

// The structured pusher kernel (Appendix E-C), as the caller configures it.
constexpr int kStructPush = 0;  // per action [a_k (4), o_k, D_k]; d = 6K
constexpr int kStructPose = 1;  // [a_1..a_K, (x, y, phi)_1..K]; d = 7K
constexpr int kStructMaxK = 8;
struct StructKernel {
    int layout, K;
    float alpha_g, alpha_z, alpha_p;
    float h_g, h_z;  // > 0 fixed, else the per-component median heuristic
    float kappa;
};

constexpr int kMedSample = 8192;  // distances drawn for the sampled median
constexpr int kRows16 = 256;      // row padding unit of both matrix-core forms
constexpr int kTile16 = 64;       // rows per workgroup of the BF16 contraction

// One problem of a batched solve, resident in device memory.
struct ProblemDesc {
    SimConst c;
    TapeGeom g;
    SvgdLayout sv;
    int N, d;
    float fixed_h;     // > 0: fixed bandwidth
    int pad;
    int64_t theta_off;  // floats into the packed theta / m / v / grad / phi arrays
    int64_t cost_off;   // floats into the packed cost array
    int64_t tape_off;   // floats into the tape region
    int64_t seg_off;    // floats into the segment replay region
    int64_t svgd_off;   // bytes into the SVGD region
};

// Shape classes of the FP32 direction's contraction: the split form for
// d <= 31 (classes 0 and 1: one or two 16-column tiles of V = [.. d .. | 1]),
// then the FP32 matrix-core form by Gram k-steps (an even count of
// 4-coordinate steps) and 16-column tiles of V.
constexpr int kPhi32Classes = 9;
constexpr int kPhi3MaxD = 31;  // the split form's Gram is 32 coordinates wide, V 32 columns
__host__ __device__ inline int phi32_ks(int d) { return 2 * ((d + 7) / 8); }
__host__ __device__ inline int phi32_ot(int d) { return (d + 16) / 16; }

// Device work lists of one batched SVGD step (built once per solve).
// Padded dimension of the median's all-pairs items, and the class of an item
// shape (padded dimension, rows) as a bit index 0..5.
__host__ __device__ inline int med_dp(int d) { return d <= 16 ? 16 : d <= 32 ? 32 : 64; }
__host__ __device__ inline int med_class(int dp, int rows) { return (dp == 16 ? 0 : dp == 32 ? 2 : 4) + (rows == 256); }
// Work lists of the median's all-pairs items, one per item shape: 6 direct
// shapes (med_class), then 16 Gram-form shapes (ks32, rows) of the problems
// above 2^20 pairs, then 2 of the split-form Gram (ks32 = 0: d <= 31, the
// rows as three BF16 parts).
constexpr int kMedLists = 6 + 16 + 2;
__host__ __device__ inline int med_gram_list(int ks32, int rows) {
    return (ks32 == 0 ? 22 : 6 + 2 * (ks32 / 2 - 1)) + (rows == 256);
}

struct BatchPlan {
    int n_problems;
    const int4* dist_work;  int n_dist;   // (p, row block, column chunk, -) of the median passes,
    int dist_start[kMedLists];            // sorted by item shape: list c = entries
    int dist_n[kMedLists];                //   [dist_start[c], dist_start[c] + dist_n[c])
    const int4* cand_work;  int n_cand;   // (p, segment, part, -) of the median's candidate passes
                                          //   (problems above 2^20 pairs)
    const int4* fin_work;   int n_fin;    // (p, -, -, -): problems of 2^20 pairs at most, whose select
                                          //   ends in one workgroup after pass 0
    const int4* phi_work[kPhi32Classes];  // (p, row block, split, -) per contraction class
    int n_phi[kPhi32Classes];
    // BF16 matrix-core form: (problem, coordinate), (problem, 256-row chunk),
    // and (problem, row block, split) per padded dimension 32 / 64
    const int4* ctr_work;
    int n_ctr;
    const int4* row16_work;
    int n_row16;
    const int4* phi16_work[2];
    int n_phi16[2];
    int phi_rows;                         // rows per contraction workgroup
    const int4* red_work;   int n_red;    // (p, first elem, end elem, -)
};

// Mean of coordinate l over N particles ([d][N] layout), one workgroup of
// kMeanThreads: four independent partial sums per thread keep four loads in
// flight; a fixed tree adds the threads' sums (same order on every launch).
constexpr int kMeanThreads = 1024;
template <int NT = kMeanThreads>
__device__ __forceinline__ void particle_mean_body(int N, int l, const float* __restrict__ theta,
                                                   float* __restrict__ ctr) {
    constexpr int kMeanThreads = NT;
    __shared__ float red[kMeanThreads];
    const float* t = theta + (int64_t)l * N;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    int i = threadIdx.x;
    for (; i + 3 * kMeanThreads < N; i += 4 * kMeanThreads) {
        s0 += t[i];
        s1 += t[i + kMeanThreads];
        s2 += t[i + 2 * kMeanThreads];
        s3 += t[i + 3 * kMeanThreads];
    }
    for (; i < N; i += kMeanThreads) s0 += t[i];
    red[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int w = kMeanThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) ctr[l] = red[0] / (float)N;
}

// The update of Algorithm 1 on one element: Adam minimising -phi with the
// bias-correction denominators den = (1 - b1^t, 1 - b2^t), or theta += lr phi.
struct UpdateArgs {
    float* theta;
    float* m;
    float* v;
    int t0;
    const int* t_dev;  // non-null: step t = t0 + *t_dev + 1 (graph replay), else t = t0
    float lr, b1, b2, eps;
    int use_adam;
    int t_pre;         // 1: this iteration's first kernel already advanced *t_dev, so t = t0 + *t_dev
};

// The bias-correction denominators den[0..1] of the workgroup: thread 0
// computes them into LDS.  Every thread calls this, after issuing its element
// loads, so that the counter's load and the powers overlap those loads.
__device__ __forceinline__ void block_denominators(const UpdateArgs& u, float* den) {
    if (u.use_adam && threadIdx.x == 0) {
        const int t = u.t_dev ? u.t0 + *u.t_dev + (u.t_pre ? 0 : 1) : u.t0;
        den[0] = 1.0f - powf(u.b1, (float)t);
        den[1] = 1.0f - powf(u.b2, (float)t);
    }
    __syncthreads();
}

// The update of element e from its loaded theta, m and v (the loads can be
// issued with the kernel's other loads).
struct UpdateIn {
    float theta, m, v;
};
__device__ __forceinline__ UpdateIn update_load(const UpdateArgs& u, int64_t e) {
    UpdateIn in{u.theta[e], 0.0f, 0.0f};
    if (u.use_adam) {
        in.m = u.m[e];
        in.v = u.v[e];
    }
    return in;
}
__device__ __forceinline__ void update_apply(const UpdateArgs& u, const float* den, int64_t e, const UpdateIn& in,
                                             float f) {
    if (!u.use_adam) {
        u.theta[e] = in.theta + u.lr * f;
        return;
    }
    const float gr = -f;
    const float mm = u.b1 * in.m + (1.0f - u.b1) * gr;
    const float vv = u.b2 * in.v + (1.0f - u.b2) * gr * gr;
    u.m[e] = mm;
    u.v[e] = vv;
    const float mhat = mm / den[0];
    const float vhat = vv / den[1];
    u.theta[e] = in.theta - u.lr * mhat / (sqrtf(vhat) + u.eps);
}

// One element's direction r and, for the update, its index and loaded operands.
struct ElemOut {
    bool ok;
    float r;
    int64_t ue;
    UpdateIn in;
};
// a single particle: phi = g
// (the update's arguments by reference with a flag: a pointer to a kernel
// argument would place the argument in scratch memory)
__device__ __forceinline__ ElemOut pass_elem(const float* g, float* phi, int64_t e, const UpdateArgs& upd,
                                             bool apply) {
    ElemOut o{true, g[e], e, {}};
    if (phi) phi[e] = o.r;
    if (apply) o.in = update_load(upd, e);
    return o;
}

// Phase k of a T-step, H-push rollout: steps [t_k, t_{k+1}), t_k = ceil(kT/H).
__host__ __device__ inline int phase_start(int k, int T, int H) { return (k * T + H - 1) / H; }

// ---- quad (4-lane) exchange by DPP quad_perm -------------------------------
__device__ __forceinline__ float quad_xor1(float v) {
    // quad_perm [1,0,3,2]
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_xor2(float v) {
    // quad_perm [2,3,0,1]
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
}
// Sum over the 4 lanes of a quad; (v0+v1)+(v2+v3) on every lane, bit-identical.
__device__ __forceinline__ float quad_sum(float v) {
    v = v + quad_xor1(v);
    return v + quad_xor2(v);
}

// ---- hardware transcendentals (v_rsq/v_rcp/v_exp/v_log, ~1 ulp) -------------
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
// min(max(x, 0), 1): becomes the clamp bit of the instruction producing x
__device__ __forceinline__ float unit_clamp(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// ---- smooth penalty ---------------------------------------------------------
// sp(z) = log(1 + exp(beta z)) / beta = max(z,0) + log1p(exp(-beta|z|)) / beta.
// log1p(u) is taken as log2(1+u) ln2: for u below FP32 resolution this drops a
// term of size u/beta (< 1e-10 m at beta = 1000), far under the step's rounding.
__device__ __forceinline__ float softplus_u(float z, float beta_log2e) {
    return hw_exp2(-beta_log2e * fabsf(z));
}
__device__ __forceinline__ float softplus(float z, float beta_log2e, float ln2_over_beta) {
    const float u = softplus_u(z, beta_log2e);
    return fmaf(hw_log2(1.0f + u), ln2_over_beta, fmaxf(z, 0.0f));
}
// d sp / dz = 1 / (1 + exp(-beta z)), from u = exp(-beta|z|) without overflow
__device__ __forceinline__ float softplus_grad(float z, float beta_log2e) {
    const float u = softplus_u(z, beta_log2e);
    const float r = hw_rcp(1.0f + u);
    return z >= 0.0f ? r : u * r;
}

__device__ __forceinline__ float relu(float x) { return fmaxf(x, 0.0f); }

// Quintic time scaling of a push: s(tau) = 10 tau^3 - 15 tau^4 + 6 tau^5.
__device__ __forceinline__ float push_profile(float tau) {
    const float t3 = tau * tau * tau;
    return t3 * fmaf(fmaf(6.0f, tau, -15.0f), tau, 10.0f);
}


// ---------------------------------------------------------------------------
// Surrogate network (n_in -> 256 -> 256 -> 1).  FP32 parameter vector, floats:
constexpr int kMlpIn = STAMP_MLP_IN_PAD;     // padded input width
constexpr int kMlpWidth = STAMP_MLP_WIDTH;   // hidden width
constexpr int kMlpOffMu = 0;                                   // [kMlpIn]
constexpr int kMlpOffIsig = kMlpOffMu + kMlpIn;                // [kMlpIn]
constexpr int kMlpOffW1 = kMlpOffIsig + kMlpIn;                // [256][kMlpIn]
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpWidth * kMlpIn;      // [256]
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpWidth;               // [256][256]
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpWidth * kMlpWidth;   // [256]
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpWidth;               // [256]
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpWidth;               // [1]
constexpr int kMlpParams = kMlpOffB3 + 1;
static_assert(kMlpParams == STAMP_MLP_PARAMS, "parameter layout");
// BF16 working copies, elements: W1, W1^T, W2, W2^T
constexpr int kMlpBfW1 = 0;
constexpr int kMlpBfW1T = kMlpBfW1 + kMlpWidth * kMlpIn;
constexpr int kMlpBfW2 = kMlpBfW1T + kMlpWidth * kMlpIn;
constexpr int kMlpBfW2T = kMlpBfW2 + kMlpWidth * kMlpWidth;
constexpr int kMlpBfTotal = kMlpBfW2T + kMlpWidth * kMlpWidth;
static_assert(kMlpBfTotal == STAMP_MLP_BF16_WEIGHTS, "bf16 layout");
constexpr int kMlpPartStride = 772;  // per-tile partial sums of a training step

}  // namespace stamp
