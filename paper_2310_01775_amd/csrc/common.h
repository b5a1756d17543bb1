// Shared device-side definitions of the STAMP hot path (gfx950).
//
// Lane mapping of the rollout kernels: lane 4*i + s runs particle i's
// sub-rollout of push side s (North, East, South, West = 0..3).  The four
// lanes of a particle are one DPP quad, so the phase mixture
// S_{k+1} = sum_s softmax(a_k)_s X_s and every per-particle reduction of the
// adjoint are two quad_perm DPP moves, no LDS and no barrier.
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
    float pose0[kMaxBlocks][3];
    float hsum[kMaxBlocks][kMaxBlocks];  // h_b + h_c
    float h0;                  // half size of the pushed block
    float h0d;                 // h0 + standoff
    float kp, kb, beta, inv_beta, er2;
    // cost (Appendix E-B)
    float goal[3], tol;
    float wt, wr, wtr, wb, omax, dmax, ea2;
};

// Layout of the rollout tape (floats):
//   entries [n_entries][6B][4N] : pre-step states (every step, or checkpoints)
//   ends    [H][6B][4N]         : sub-rollout states after each phase's last step
struct TapeGeom {
    int64_t lanes;      // 4N
    int64_t n_entries;  // T, or sum_k ceil(L_k / K)
    int64_t ends_off;   // n_entries * 6B * 4N
    int ckpt;           // 0 = full tape
};

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

// ---- smooth penalty ---------------------------------------------------------
// sp(z) = log(1 + exp(beta z)) / beta = max(z,0) + log1p(exp(-beta|z|)) / beta
__device__ __forceinline__ float softplus(float z, float beta, float inv_beta) {
    return fmaxf(z, 0.0f) + log1pf(expf(-beta * fabsf(z))) * inv_beta;
}
// d sp / dz = 1 / (1 + exp(-beta z)), evaluated without overflow
__device__ __forceinline__ float softplus_grad(float z, float beta) {
    float e = expf(-beta * fabsf(z));
    float r = 1.0f / (1.0f + e);
    return z >= 0.0f ? r : e * r;
}

__device__ __forceinline__ float relu(float x) { return fmaxf(x, 0.0f); }

// Quintic time scaling of a push: s(tau) = 10 tau^3 - 15 tau^4 + 6 tau^5.
__device__ __forceinline__ float push_profile(float tau) {
    return tau * tau * tau * (10.0f + tau * (-15.0f + 6.0f * tau));
}

}  // namespace stamp
