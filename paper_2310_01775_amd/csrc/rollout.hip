// Relaxed block-pushing rollout and its adjoint on gfx950.
//
// Model (Sec. III-B: semi-implicit Euler with spring-based penalty contacts;
// Sec. IV-A and Appendix E: pushing from the N/E/S/W faces of block 0).
// Push phase k runs once per side s from the shared phase-start state S_k; the
// next phase starts from S_{k+1} = sum_s softmax(a_k)_s X_s(t_{k+1}).
//
// Lanes: one per (particle i, side s, block b).  The SL = 1, 2 or 4 block
// slots of a (particle, side) sub-rollout sit in one DPP quad (SL = B rounded
// up; slots b >= B are idle copies), so a lane integrates one block and reads
// the other blocks' positions (and, in the reverse, force adjoints) by
// quad_perm moves each step; the sides of a particle meet only at phase
// boundaries.  A step thus costs one block's friction and integration, B-1
// pair terms and the pusher per lane, instead of all blocks' work.
//
// The adjoint is the exact reverse of the forward arithmetic (Sec. III-B:
// gradients back-propagated through the whole trajectory), either from a full
// tape of pre-step states or by replaying checkpointed segments of <= K steps
// into a scratch buffer and reversing each.
#include "common.h"
#include "internal.h"

namespace stamp {

// One wave per workgroup: a small particle set spreads over as many CUs as it
// has waves instead of stacking four waves on one CU.
constexpr int kRolloutBlock = 64;

// Block slots per (particle, side) sub-rollout, and lanes per particle.
template <int B>
struct Slots {
    static constexpr int SL = B == 1 ? 1 : (B == 2 ? 2 : 4);
    static constexpr int LANES = 4 * SL;
};

// State of one block: position, angle, velocities.
struct Blk {
    float x, y, ph, vx, vy, om;
};

// Fixed data of one lane during one push phase.  The pusher of side s sits at
// A + R(A)[(h0 + standoff) n_s + o t_s - D sig n_s] (anchor A = block-0 pose at
// the phase start), i.e. at P0 + sig V with P0 = A + R(A)((h0 + standoff) n_s
// + o t_s) and V = -D R(A) n_s, both fixed over the phase.
struct Push {
    float nx, ny, tx, ty;  // face normal n_s and tangent t_s (block frame)
    float P0x, P0y;        // pusher position at sig = 0 (world frame)
    float Vx, Vy;          // pusher travel over the phase (world frame)
};

// Anchor-frame quantities of a phase, kept for the adjoint.
struct Anchor {
    float cA, sA;          // rotation of the anchor
    float q0x, q0y;        // (h0 + standoff) n_s + o t_s (block frame)
};

// sin and cos by Cody-Waite reduction x = r + k pi/2 (pi/2 in two parts,
// fused multiply-adds), |r| <= pi/4, and Taylor polynomials in r^2 (sin to
// r^9, cos to r^10: truncation below 3e-9 on the reduced range); about one
// FP32 ulp over the block angles a push produces.
__device__ __forceinline__ void sincos_rd(float x, float& s, float& c) {
    const float k = rintf(x * 0.636619772f);  // 2/pi
    float r = fmaf(-k, 1.57079637f, x);       // pi/2 rounded to FP32
    r = fmaf(-k, -4.37113883e-8f, r);         // pi/2 minus that
    const float r2 = r * r;
    float ps = fmaf(r2, 2.75573192e-6f, -1.98412698e-4f);  // 1/9!, -1/7!
    ps = fmaf(r2, ps, 8.33333333e-3f);                     // 1/5!
    ps = fmaf(r2, ps, -1.66666667e-1f);                    // -1/3!
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -2.75573192e-7f, 2.48015873e-5f);  // -1/10!, 1/8!
    pc = fmaf(r2, pc, -1.38888889e-3f);                    // -1/6!
    pc = fmaf(r2, pc, 4.16666667e-2f);                     // 1/4!
    pc = fmaf(r2, pc, -0.5f);
    const float cr = fmaf(r2, pc, 1.0f);
    const int q = (int)k & 3;  // sin(r + q pi/2), cos(r + q pi/2)
    const float ss = (q & 1) ? cr : sr;
    const float cc = (q & 1) ? sr : cr;
    s = (q & 2) ? -ss : ss;
    c = ((q + 1) & 2) ? -cc : cc;
}

// The phase's pusher data from the anchor pose (Ax, Ay, Aph) and (o, D); the
// forward pass and the adjoint both build it here, so replays match bit for bit.
__device__ __forceinline__ void phase_push(const SimConst& c, float Ax, float Ay, float Aph, float o, float D,
                                           Push& p, Anchor& a) {
    sincos_rd(Aph, a.sA, a.cA);
    a.q0x = fmaf(c.h0d, p.nx, o * p.tx);
    a.q0y = fmaf(c.h0d, p.ny, o * p.ty);
    p.P0x = Ax + fmaf(a.cA, a.q0x, -(a.sA * a.q0y));
    p.P0y = Ay + fmaf(a.sA, a.q0x, a.cA * a.q0y);
    p.Vx = -D * fmaf(a.cA, p.nx, -(a.sA * p.ny));
    p.Vy = -D * fmaf(a.sA, p.nx, a.cA * p.ny);
}


// Tape entries hold, per (particle, side) sub-rollout, its blocks' states one
// after another: block b of sub-rollout 4i+s is slot (4i+s)B+b, 6 floats
// (x, y, phi, vx, vy, omega).
__device__ __forceinline__ void load_blk(Blk& X, const float* __restrict__ entry, int64_t slot) {
    const float2* p = reinterpret_cast<const float2*>(entry + slot * 6);
    const float2 a = p[0], c = p[1], e = p[2];
    X.x = a.x;
    X.y = a.y;
    X.ph = c.x;
    X.vx = c.y;
    X.vy = e.x;
    X.om = e.y;
}

// The same at a 32-bit float offset from a wave-uniform entry pointer (a
// scalar base plus a vector offset in the memory instruction).
__device__ __forceinline__ void load_blk_at(Blk& X, const float* __restrict__ entry, uint32_t off) {
    const float2* p = reinterpret_cast<const float2*>(entry + off);
    const float2 a = p[0], c = p[1], e = p[2];
    X.x = a.x;
    X.y = a.y;
    X.ph = c.x;
    X.vx = c.y;
    X.vy = e.x;
    X.om = e.y;
}

__device__ __forceinline__ void store_blk(const Blk& X, float* __restrict__ entry, int64_t slot) {
    float2* p = reinterpret_cast<float2*>(entry + slot * 6);
    p[0] = make_float2(X.x, X.y);
    p[1] = make_float2(X.ph, X.vx);
    p[2] = make_float2(X.vy, X.om);
}

__device__ __forceinline__ void store_blk_at(const Blk& X, float* __restrict__ entry, uint32_t off) {
    float2* p = reinterpret_cast<float2*>(entry + off);
    p[0] = make_float2(X.x, X.y);
    p[1] = make_float2(X.ph, X.vx);
    p[2] = make_float2(X.vy, X.om);
}

// Push profile s((j + 1) / L) of step j of a phase: the wave evaluates 64
// consecutive steps at once (one per lane) and each step reads its value back
// with readlane, so a step costs one instruction instead of the polynomial.
// Every pass (forward, replay, reverse) takes the same per-lane expression.
struct Profile {
    float invL;
    int base;
    float v;
    __device__ __forceinline__ void reset(float inv) {
        invL = inv;
        base = -1;
    }
    __device__ __forceinline__ float at(int j) {
        const int b0 = j & ~63;
        if (b0 != base) {
            base = b0;
            v = push_profile((float)(b0 + 1 + (int)__lane_id()) * invL);
        }
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j & 63));
    }
};

// Index of the K-th block other than b (increasing order).
__host__ __device__ constexpr int other_block(int K, int b) { return K < b ? K : K + 1; }

// quad_perm control that hands lane slot b the value of slot other_block(K, b)
// of its own group of SL slots.
template <int SL, int K>
constexpr int other_sel() {
    int sel = 0;
    for (int p = 0; p < 4; ++p) {
        const int b = p % SL, base = p - b;
        int q = other_block(K, b);
        if (q >= SL) q = 0;
        sel |= (base + q) << (2 * p);
    }
    return sel;
}

template <int SL, int K>
__device__ __forceinline__ float from_other_k(float v) {
    constexpr int sel = other_sel<SL, K>();
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), sel, 0xF, 0xF, false));
}

// K is a constant of an unrolled loop (0..2).
template <int SL>
__device__ __forceinline__ float from_other(float v, int K) {
    if (K == 0) return from_other_k<SL, 0>(v);
    if (K == 1) return from_other_k<SL, 1>(v);
    return from_other_k<SL, 2>(v);
}

// Sum over the four sides of a particle (lanes SL apart): (v0+v1)+(v2+v3) on
// every lane, bit-identical.
template <int SL>
__device__ __forceinline__ float side_sum(float v) {
    if constexpr (SL == 1) {
        return quad_sum(v);
    } else {
        v = v + __shfl_xor(v, SL);
        return v + __shfl_xor(v, 2 * SL);
    }
}

// Sum over the block slots of a sub-rollout.
template <int SL>
__device__ __forceinline__ float slot_sum(float v) {
    if constexpr (SL >= 2) v = v + quad_xor1(v);
    if constexpr (SL == 4) v = v + quad_xor2(v);
    return v;
}

// Constants of this lane's block b (slots b >= B take block 0's).
template <int B>
struct BlkConst {
    float cf, cr, ev2, ew2, dtm, dtI, crw2;
    float hs[B > 1 ? B - 1 : 1];  // h_b + h_q of the other blocks, increasing q
    float x0, y0, ph0;            // initial pose
};

template <int B>
__device__ __forceinline__ float pick(const float* a, int b) {
    float v = a[0];
#pragma unroll
    for (int q = 1; q < B; ++q) v = (b == q) ? a[q] : v;
    return v;
}

template <int B>
__device__ __forceinline__ BlkConst<B> blk_const(const SimConst& c, int b) {
    BlkConst<B> k;
    k.cf = pick<B>(c.cf, b);
    k.cr = pick<B>(c.cr, b);
    k.ev2 = pick<B>(c.ev2, b);
    k.ew2 = pick<B>(c.ew2, b);
    k.dtm = pick<B>(c.dtm, b);
    k.dtI = pick<B>(c.dtI, b);
    k.crw2 = pick<B>(c.crw2, b);
    float px[kMaxBlocks], py[kMaxBlocks], pp[kMaxBlocks];
#pragma unroll
    for (int q = 0; q < kMaxBlocks; ++q) {
        px[q] = c.pose0[q][0];
        py[q] = c.pose0[q][1];
        pp[q] = c.pose0[q][2];
    }
    k.x0 = pick<B>(px, b);
    k.y0 = pick<B>(py, b);
    k.ph0 = pick<B>(pp, b);
#pragma unroll
    for (int K = 0; K < (B > 1 ? B - 1 : 1); ++K) {
        float v = 0.0f;
#pragma unroll
        for (int bb = 0; bb < B; ++bb) v = (b == bb && B > 1) ? c.hsum[bb][other_block(K, bb)] : v;
        k.hs[K] = v;
    }
    return k;
}

// One semi-implicit Euler step of block b of the sub-rollout (pusher of this
// lane's side on block 0).  Products that feed a sum are fused (fmaf); the
// reverse below differentiates the same expressions.  Forces on a block sum in
// the order friction, pairs by increasing partner, pusher.
template <int B>
__device__ __forceinline__ void step_forward(const SimConst& c, const BlkConst<B>& k, int b, Blk& X, const Push& p,
                                             float sig) {
    constexpr int SL = Slots<B>::SL;
    constexpr int NO = B - 1;
    float ox[NO > 0 ? NO : 1], oy[NO > 0 ? NO : 1];
#pragma unroll
    for (int K = 0; K < NO; ++K) {
        ox[K] = from_other<SL>(X.x, K);
        oy[K] = from_other<SL>(X.y, K);
    }
    // regularised Coulomb friction
    const float inv = hw_rsq(fmaf(X.vx, X.vx, fmaf(X.vy, X.vy, k.ev2)));
    const float kf = k.cf * inv;
    float Fx = -kf * X.vx;
    float Fy = -kf * X.vy;
    const float invw = hw_rsq(fmaf(X.om, X.om, k.ew2));
    float Tq = -(k.cr * invw) * X.om;
    // block-block penalty on the inscribed disks, central force
#pragma unroll
    for (int K = 0; K < NO; ++K) {
        const float dx = X.x - ox[K], dy = X.y - oy[K];
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, c.er2));
        const float rinv = hw_rsq(d2);
        const float pen = fmaf(-d2, rinv, k.hs[K]);  // h_b + h_q - r
        const float fr = c.kb * softplus(pen, c.beta_log2e, c.ln2_over_beta) * rinv;
        Fx = fmaf(fr, dx, Fx);
        Fy = fmaf(fr, dy, Fy);
    }
    // the virtual pusher of this side, on block 0: contact normal e = R(phi0) n
    {
        const float relx = fmaf(sig, p.Vx, p.P0x) - X.x;
        const float rely = fmaf(sig, p.Vy, p.P0y) - X.y;
        float s0, c0;
        sincos_rd(X.ph, s0, c0);
        const float ex = fmaf(c0, p.nx, -(s0 * p.ny)), ey = fmaf(s0, p.nx, c0 * p.ny);
        const float pen = c.h0 - fmaf(ex, relx, ey * rely);
        const float f = c.kp * softplus(pen, c.beta_log2e, c.ln2_over_beta);
        if (b == 0) {
            Fx = fmaf(-f, ex, Fx);
            Fy = fmaf(-f, ey, Fy);
            Tq = fmaf(-f, fmaf(relx, ey, -(rely * ex)), Tq);  // rel x (-f e)
        }
    }
    // semi-implicit Euler: velocities, then positions with the new velocities
    X.vx = fmaf(k.dtm, Fx, X.vx);
    X.vy = fmaf(k.dtm, Fy, X.vy);
    X.om = fmaf(k.dtI, Tq, X.om);
    X.x = fmaf(c.dt, X.vx, X.x);
    X.y = fmaf(c.dt, X.vy, X.y);
    X.ph = fmaf(c.dt, X.om, X.ph);
}

// Reverse of step_forward at pre-step state X of block b.  On entry L is the
// adjoint of the block's post-step state; on exit that of its pre-step state.
// Adjoints of the phase's pusher data (P0, V) are accumulated on block 0.
template <int B>
__device__ __forceinline__ void step_reverse(const SimConst& c, const BlkConst<B>& k, int b, const Blk& X, Blk& L,
                                             const Push& p, float sig, float& P0xb, float& P0yb, float& Vxb,
                                             float& Vyb) {
    constexpr int SL = Slots<B>::SL;
    constexpr int NO = B - 1;
    // integrator: x' = x + dt v', v' = v + (dt/m) F
    L.vx = fmaf(c.dt, L.x, L.vx);
    L.vy = fmaf(c.dt, L.y, L.vy);
    L.om = fmaf(c.dt, L.ph, L.om);
    const float Fxb = k.dtm * L.vx;
    const float Fyb = k.dtm * L.vy;
    const float Tqb = k.dtI * L.om;
    float ox[NO > 0 ? NO : 1], oy[NO > 0 ? NO : 1], ofx[NO > 0 ? NO : 1], ofy[NO > 0 ? NO : 1];
#pragma unroll
    for (int K = 0; K < NO; ++K) {
        ox[K] = from_other<SL>(X.x, K);
        oy[K] = from_other<SL>(X.y, K);
        ofx[K] = from_other<SL>(Fxb, K);
        ofy[K] = from_other<SL>(Fyb, K);
    }
    // pusher
    {
        const float relx = fmaf(sig, p.Vx, p.P0x) - X.x;
        const float rely = fmaf(sig, p.Vy, p.P0y) - X.y;
        float s0, c0;
        sincos_rd(X.ph, s0, c0);
        const float ex = fmaf(c0, p.nx, -(s0 * p.ny)), ey = fmaf(s0, p.nx, c0 * p.ny);
        const float cross = fmaf(relx, ey, -(rely * ex));
        const float pen = c.h0 - fmaf(ex, relx, ey * rely);
        const float u = softplus_u(pen, c.beta_log2e);
        const float f = c.kp * fmaf(hw_log2(1.0f + u), c.ln2_over_beta, fmaxf(pen, 0.0f));
        const float rr = hw_rcp(1.0f + u);
        const float spg = pen >= 0.0f ? rr : u * rr;  // sp'(pen)
        // F0 += -f e, T0 += -f cross
        const float fb = -fmaf(cross, Tqb, fmaf(ex, Fxb, ey * Fyb));
        const float crossb = -f * Tqb;
        const float penb = fb * c.kp * spg;
        // cross = relx ey - rely ex, pen = h0 - (ex relx + ey rely)
        const float exb = fmaf(-f, Fxb, -fmaf(crossb, rely, penb * relx));
        const float eyb = fmaf(-f, Fyb, fmaf(crossb, relx, -(penb * rely)));
        const float relxb = fmaf(crossb, ey, -(penb * ex));
        const float relyb = -fmaf(crossb, ex, penb * ey);
        // e = (c0 nx - s0 ny, s0 nx + c0 ny)
        const float c0b = fmaf(exb, p.nx, eyb * p.ny);
        const float s0b = fmaf(eyb, p.nx, -(exb * p.ny));
        if (b == 0) {
            L.ph += fmaf(c0, s0b, -(s0 * c0b));
            // rel = P0 + sig V - x0
            L.x -= relxb;
            L.y -= relyb;
            P0xb += relxb;
            P0yb += relyb;
            Vxb = fmaf(sig, relxb, Vxb);
            Vyb = fmaf(sig, relyb, Vyb);
        }
    }
    // block-block contacts: F_b += f u with u = Delta / r, Delta = x_b - x_q
#pragma unroll
    for (int K = 0; K < NO; ++K) {
        const float dx = X.x - ox[K], dy = X.y - oy[K];
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, c.er2));
        const float rinv = hw_rsq(d2);
        const float pen = fmaf(-d2, rinv, k.hs[K]);
        const float u = softplus_u(pen, c.beta_log2e);
        const float fr = c.kb * fmaf(hw_log2(1.0f + u), c.ln2_over_beta, fmaxf(pen, 0.0f)) * rinv;
        const float rr = hw_rcp(1.0f + u);
        const float fp = c.kb * (pen >= 0.0f ? rr : u * rr);  // f'(pen)
        const float gx = Fxb - ofx[K], gy = Fyb - ofy[K];
        const float gu = fmaf(gx, dx, gy * dy) * rinv;  // adjoint of f
        // d(f u)/dDelta = f/r (I - u u^T) + f'(pen)(-u) u^T
        const float k2 = (fr + fp) * gu * rinv;  // coefficient of Delta
        L.x += fmaf(fr, gx, -(k2 * dx));
        L.y += fmaf(fr, gy, -(k2 * dy));
    }
    // friction
    const float inv = hw_rsq(fmaf(X.vx, X.vx, fmaf(X.vy, X.vy, k.ev2)));
    const float kf = k.cf * inv;
    const float kd = kf * inv * inv * fmaf(Fxb, X.vx, Fyb * X.vy);
    L.vx = fmaf(kd, X.vx, fmaf(-kf, Fxb, L.vx));
    L.vy = fmaf(kd, X.vy, fmaf(-kf, Fyb, L.vy));
    const float invw = hw_rsq(fmaf(X.om, X.om, k.ew2));
    L.om = fmaf(-(k.crw2 * (invw * invw * invw)), Tqb, L.om);
}

__device__ __forceinline__ void side_frame(int s, Push& p) {
    p.nx = (s == 1) ? 1.0f : ((s == 3) ? -1.0f : 0.0f);
    p.ny = (s == 0) ? 1.0f : ((s == 2) ? -1.0f : 0.0f);
    p.tx = -p.ny;
    p.ty = p.nx;
}

// softmax(a_k)_s of this lane's side (max-subtracted, Eq. 5's relaxation)
__device__ __forceinline__ float side_weight(const float* __restrict__ theta, int N, int i, int k, int s) {
    float a0 = theta[(int64_t)(6 * k + 0) * N + i];
    float a1 = theta[(int64_t)(6 * k + 1) * N + i];
    float a2 = theta[(int64_t)(6 * k + 2) * N + i];
    float a3 = theta[(int64_t)(6 * k + 3) * N + i];
    float m = fmaxf(fmaxf(a0, a1), fmaxf(a2, a3));
    float e0 = expf(a0 - m), e1 = expf(a1 - m), e2 = expf(a2 - m), e3 = expf(a3 - m);
    float es = (s == 0) ? e0 : (s == 1) ? e1 : (s == 2) ? e2 : e3;
    return es / (((e0 + e1) + e2) + e3);
}

__device__ __forceinline__ float smooth_abs(float u, float ea2) { return sqrtf(u * u + ea2); }

// ---------------------------------------------------------------------------
// Forward rollout of one lane: particle i, side s, block slot b.  Every lane of
// the wave runs it (cross-lane moves and readlane need all lanes): lanes past
// the last particle repeat particle N-1 and write nothing.
template <int B>
__device__ __forceinline__ void rollout_fwd_lane(const SimConst& c, int N, const float* __restrict__ theta,
                                                 float* __restrict__ cost, float* __restrict__ tape,
                                                 const TapeGeom& g, uint32_t* status, int64_t lane) {
    constexpr int SL = Slots<B>::SL;
    const int64_t iw = lane / (4 * SL);
    const bool live = iw < N;
    const int i = live ? (int)iw : N - 1;
    const int r = (int)(lane % (4 * SL));
    const int s = r / SL, b = r % SL;
    const bool real = b < B && live;  // writes its block's states
    const int64_t slot = ((int64_t)4 * i + s) * B + b;
    const uint32_t off = (uint32_t)(slot * 6);  // within an entry (< 2^32 floats)
    const int64_t stride = 6 * B * g.lanes;  // floats per tape entry
    const int H = c.H, T = c.T;
    const BlkConst<B> k = blk_const<B>(c, b);

    Blk S;
    S.x = k.x0;
    S.y = k.y0;
    S.ph = k.ph0;
    S.vx = S.vy = S.om = 0.0f;
    float Px[kMaxPushes + 1], Py[kMaxPushes + 1];  // block 0's, on slot 0
    float Lbound = 0.0f;
    Push p;
    side_frame(s, p);
    int64_t entry = 0;
    for (int kk = 0; kk < H; ++kk) {
        const int tk = phase_start(kk, T, H), tk1 = phase_start(kk + 1, T, H);
        const float invL = 1.0f / (float)(tk1 - tk);
        Px[kk] = S.x;
        Py[kk] = S.y;
        const float z = side_weight(theta, N, i, kk, s);
        const float o = theta[(int64_t)(6 * kk + 4) * N + i];
        const float D = theta[(int64_t)(6 * kk + 5) * N + i];
        Anchor an;
        phase_push(c, S.x, S.y, S.ph, o, D, p, an);  // block 0's anchor on slot 0
        Lbound += relu(fabsf(o) - c.omax) * relu(fabsf(o) - c.omax) + relu(-D) * relu(-D) +
                  relu(D - c.dmax) * relu(D - c.dmax);
        Blk X = S;
        Profile prof;
        prof.reset(invL);
        const int nst = tk1 - tk;
        if (tape && g.ckpt == 0) {
            float* e = tape + (int64_t)tk * stride;
            for (int j = 0; j < nst; ++j, e += stride) {
                if (real) store_blk_at(X, e, off);
                step_forward<B>(c, k, b, X, p, prof.at(j));
            }
        } else {
            int until = 0;  // steps to the next checkpoint
            for (int j = 0; j < nst; ++j) {
                if (tape && until == 0) {
                    if (real) store_blk_at(X, tape + entry * stride, off);
                    ++entry;
                    until = g.ckpt;
                }
                --until;
                step_forward<B>(c, k, b, X, p, prof.at(j));
            }
        }
        if (tape && real) store_blk_at(X, tape + g.ends_off + (int64_t)kk * stride, off);
        // phase mixture over the sides
        S.x = side_sum<SL>(z * X.x);
        S.y = side_sum<SL>(z * X.y);
        S.ph = side_sum<SL>(z * X.ph);
        S.vx = side_sum<SL>(z * X.vx);
        S.vy = side_sum<SL>(z * X.vy);
        S.om = side_sum<SL>(z * X.om);
    }
    Px[H] = S.x;
    Py[H] = S.y;
    if (s != 0 || b != 0 || !live) return;
    // cost (Appendix E-B), on slot 0 of side 0
    const float dxg = fabsf(Px[H] - c.goal[0]) - c.tol, dyg = fabsf(Py[H] - c.goal[1]) - c.tol;
    const float Ltarget = relu(dxg) * relu(dxg) + relu(dyg) * relu(dyg);
    const float Lrot = 1.0f - cosf(S.ph - c.goal[2]);
    float Ltraj = 0.0f;
    for (int kk = 1; kk <= H; ++kk) {
        Ltraj += smooth_abs(Px[kk - 1] - Px[kk], c.ea2) + smooth_abs(Py[kk - 1] - Py[kk], c.ea2);
        Ltraj += smooth_abs(Px[kk] - Px[H], c.ea2) + smooth_abs(Py[kk] - Py[H], c.ea2);
        Ltraj -= smooth_abs(Px[kk - 1] - Px[H], c.ea2) + smooth_abs(Py[kk - 1] - Py[H], c.ea2);
    }
    const float C = c.wt * Ltarget + c.wr * Lrot + c.wtr * Ltraj + c.wb * Lbound;
    cost[i] = C;
    if (status && !isfinite(C)) atomicOr(status, STAMP_STATUS_NONFINITE_COST);
}

// ---------------------------------------------------------------------------
// Reverse sweep of one lane; cost_bar (or cb_scalar when null) scales dC/dtheta.
template <int B>
__device__ __forceinline__ void rollout_adj_lane(const SimConst& c, int N, const float* __restrict__ theta,
                                                 const float* __restrict__ tape, const TapeGeom& g,
                                                 const float* __restrict__ cost_bar, float cb_scalar,
                                                 float* __restrict__ grad, float* __restrict__ seg,
                                                 uint32_t* status, int64_t lane) {
    constexpr int SL = Slots<B>::SL;
    const int64_t iw = lane / (4 * SL);
    const bool live = iw < N;  // lanes past the last particle repeat particle N-1, write nothing
    const int i = live ? (int)iw : N - 1;
    const int r = (int)(lane % (4 * SL));
    const int s = r / SL, b = r % SL;
    const bool blk = b < B;        // a block slot (not an idle one)
    const bool real = blk && live;  // writes scratch and results
    const int64_t slot = ((int64_t)4 * i + s) * B + b;
    const int64_t slot0 = ((int64_t)4 * i + s) * B;  // block 0 of this sub-rollout
    const int64_t lslot = blk ? slot : slot0;         // idle slots read block 0's data
    const uint32_t off = (uint32_t)(slot * 6), loff = (uint32_t)(lslot * 6);
    const int H = c.H, T = c.T;
    const int64_t stride = 6 * B * g.lanes;  // floats per tape entry
    const BlkConst<B> k = blk_const<B>(c, b);

    // entry index of each phase start
    int ent[kMaxPushes];
    {
        int e = 0;
        for (int kk = 0; kk < H; ++kk) {
            const int tk = phase_start(kk, T, H), tk1 = phase_start(kk + 1, T, H);
            ent[kk] = (g.ckpt == 0) ? tk : e;
            if (g.ckpt) e += (tk1 - tk + g.ckpt - 1) / g.ckpt;
        }
    }
    // phase-start positions P_k and the final block-0 pose
    float Px[kMaxPushes + 1], Py[kMaxPushes + 1];
    for (int kk = 0; kk < H; ++kk) {
        Px[kk] = tape[ent[kk] * stride + slot0 * 6 + 0];
        Py[kk] = tape[ent[kk] * stride + slot0 * 6 + 1];
    }
    float phT;
    {
        const float z = side_weight(theta, N, i, H - 1, s);
        const float* e = tape + g.ends_off + (int64_t)(H - 1) * stride + slot0 * 6;
        Px[H] = side_sum<SL>(z * e[0]);
        Py[H] = side_sum<SL>(z * e[1]);
        phT = side_sum<SL>(z * e[2]);
    }
    const float cb = cost_bar ? cost_bar[i] : cb_scalar;

    // dC/dP_k and dC/dphi_T, scaled by cost_bar
    float Pxb[kMaxPushes + 1], Pyb[kMaxPushes + 1];
    for (int kk = 0; kk <= H; ++kk) Pxb[kk] = Pyb[kk] = 0.0f;
    {
        const float ux = Px[H] - c.goal[0], uy = Py[H] - c.goal[1];
        Pxb[H] += cb * c.wt * 2.0f * relu(fabsf(ux) - c.tol) * copysignf(1.0f, ux);
        Pyb[H] += cb * c.wt * 2.0f * relu(fabsf(uy) - c.tol) * copysignf(1.0f, uy);
    }
    const float phTb = cb * c.wr * sinf(phT - c.goal[2]);
    const float wtr = cb * c.wtr;
    if (!c.per_phase) {
        for (int kk = 1; kk <= H; ++kk) {
            float u, dd;
            u = Px[kk - 1] - Px[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk - 1] += dd; Pxb[kk] -= dd;
            u = Py[kk - 1] - Py[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk - 1] += dd; Pyb[kk] -= dd;
            u = Px[kk] - Px[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk] += dd;     Pxb[H] -= dd;
            u = Py[kk] - Py[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk] += dd;     Pyb[H] -= dd;
            u = Px[kk - 1] - Px[H];   dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk - 1] -= dd; Pxb[H] += dd;
            u = Py[kk - 1] - Py[H];   dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk - 1] -= dd; Pyb[H] += dd;
        }
    } else {
        // Per-phase split: term kk of L_traj is phase kk-1's and reaches only
        // that phase's end P_kk (its start P_{kk-1} and the final P_H are other
        // phases' constants); the last term, MH(P_H, P_H) = 2 eps_a, has no
        // gradient.  The target and rotation terms stay on the last phase.
        for (int kk = 1; kk < H; ++kk) {
            float u, dd;
            u = Px[kk - 1] - Px[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk] -= dd;
            u = Py[kk - 1] - Py[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk] -= dd;
            u = Px[kk] - Px[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk] += dd;
            u = Py[kk] - Py[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk] += dd;
        }
    }

    // adjoint of S_H (block 0 carries the cost's terms)
    Blk Ls;
    Ls.x = Ls.y = Ls.ph = Ls.vx = Ls.vy = Ls.om = 0.0f;
    if (b == 0) {
        Ls.x = Pxb[H];
        Ls.y = Pyb[H];
        Ls.ph = phTb;
    }

    Push p;
    side_frame(s, p);
    bool bad = false;
    for (int kk = H - 1; kk >= 0; --kk) {
        const int tk = phase_start(kk, T, H), tk1 = phase_start(kk + 1, T, H);
        const float invL = 1.0f / (float)(tk1 - tk);
        const float z = side_weight(theta, N, i, kk, s);
        const float o = theta[(int64_t)(6 * kk + 4) * N + i];
        const float D = theta[(int64_t)(6 * kk + 5) * N + i];
        // phase end: S_{k+1} = sum_s z_s X_s
        Blk Xe, L;
        load_blk_at(Xe, tape + g.ends_off + (int64_t)kk * stride, loff);
        const float zp = Ls.x * Xe.x + Ls.y * Xe.y + Ls.ph * Xe.ph + Ls.vx * Xe.vx + Ls.vy * Xe.vy + Ls.om * Xe.om;
        const float zb = slot_sum<SL>(blk ? zp : 0.0f);
        L.x = z * Ls.x;
        L.y = z * Ls.y;
        L.ph = z * Ls.ph;
        L.vx = z * Ls.vx;
        L.vy = z * Ls.vy;
        L.om = z * Ls.om;
        const float ab = z * (zb - side_sum<SL>(z * zb));  // softmax VJP
        // anchor of the phase (block 0's pose, on slot 0)
        Blk A;
        load_blk_at(A, tape + ent[kk] * stride, loff);
        Anchor an;
        phase_push(c, A.x, A.y, A.ph, o, D, p, an);
        float P0xb = 0.0f, P0yb = 0.0f, Vxb = 0.0f, Vyb = 0.0f;
        Profile prof;
        prof.reset(invL);
        if (g.ckpt == 0) {
            // reverse sweep over the full tape; the states of the next two
            // (earlier) steps are in flight while a step is reversed.  The
            // loads are unconditional (indices clamped at entry 0, whose
            // extra copies go unused): with a load on some paths only, the
            // compiler waits for every load in flight at the loop head.
            const float* base = tape + (int64_t)tk * stride;  // step j's entry: base + j stride
            int j = tk1 - tk - 1;
            Blk XA, XB;
            load_blk_at(XA, base + (int64_t)j * stride, loff);
            load_blk_at(XB, base + (int64_t)max(j - 1, 0) * stride, loff);
            for (; j >= 1; j -= 2) {
                Blk X = XA;
                load_blk_at(XA, base + (int64_t)max(j - 2, 0) * stride, loff);
                step_reverse<B>(c, k, b, X, L, p, prof.at(j), P0xb, P0yb, Vxb, Vyb);
                X = XB;
                load_blk_at(XB, base + (int64_t)max(j - 3, 0) * stride, loff);
                step_reverse<B>(c, k, b, X, L, p, prof.at(j - 1), P0xb, P0yb, Vxb, Vyb);
            }
            if (j == 0) step_reverse<B>(c, k, b, XA, L, p, prof.at(0), P0xb, P0yb, Vxb, Vyb);
        } else {
            const int nseg = (tk1 - tk + g.ckpt - 1) / g.ckpt;
            for (int q = nseg - 1; q >= 0; --q) {
                const int js = q * g.ckpt;
                const int je = min(js + g.ckpt, tk1 - tk);
                Blk X;
                load_blk_at(X, tape + (int64_t)(ent[kk] + q) * stride, loff);
                for (int j = js; j < je; ++j) {  // replay the segment
                    if (real) store_blk_at(X, seg + (int64_t)(j - js) * stride, off);
                    step_forward<B>(c, k, b, X, p, prof.at(j));
                }
                for (int j = je - 1; j >= js; --j) {
                    if (real) load_blk_at(X, seg + (int64_t)(j - js) * stride, off);  // a lane reads its own writes
                    step_reverse<B>(c, k, b, X, L, p, prof.at(j), P0xb, P0yb, Vxb, Vyb);
                }
            }
        }
        // back to the anchor and (o, D): P0 = A + R(A) q0, q0 = (h0 + standoff) n + o t,
        // V = -D e_A, e_A = R(A) n (meaningful on slot 0, zero elsewhere)
        const float eAx = fmaf(an.cA, p.nx, -(an.sA * p.ny)), eAy = fmaf(an.sA, p.nx, an.cA * p.ny);
        const float Db = -fmaf(Vxb, eAx, Vyb * eAy);
        const float eAxb = -D * Vxb, eAyb = -D * Vyb;
        const float cAb = fmaf(eAxb, p.nx, eAyb * p.ny) + fmaf(P0xb, an.q0x, P0yb * an.q0y);
        const float sAb = fmaf(eAyb, p.nx, -(eAxb * p.ny)) + fmaf(P0yb, an.q0x, -(P0xb * an.q0y));
        const float q0xb = fmaf(an.cA, P0xb, an.sA * P0yb), q0yb = fmaf(an.cA, P0yb, -(an.sA * P0xb));
        const float ob = fmaf(q0xb, p.tx, q0yb * p.ty);
        const float Aphb = fmaf(an.cA, sAb, -(an.sA * cAb));
        // adjoint of S_k: the four sub-rollouts share it
        Ls.x = side_sum<SL>(L.x);
        Ls.y = side_sum<SL>(L.y);
        Ls.ph = side_sum<SL>(L.ph);
        Ls.vx = side_sum<SL>(L.vx);
        Ls.vy = side_sum<SL>(L.vy);
        Ls.om = side_sum<SL>(L.om);
        const float Axs = side_sum<SL>(P0xb), Ays = side_sum<SL>(P0yb), Aphs = side_sum<SL>(Aphb);
        const float obs = side_sum<SL>(ob), Dbs = side_sum<SL>(Db);
        if (c.per_phase) {
            // S_k is the previous phase's output: its adjoint stops here, and
            // the previous phase starts from its own term's seed on P_k
            Ls.x = Ls.y = Ls.ph = Ls.vx = Ls.vy = Ls.om = 0.0f;
        }
        if (b == 0) {
            if (c.per_phase) {
                Ls.x = Pxb[kk];
                Ls.y = Pyb[kk];
            } else {
                Ls.x += Axs + Pxb[kk];
                Ls.y += Ays + Pyb[kk];
                Ls.ph += Aphs;
            }
            // bound loss on o_k, D_k
            const float wb2 = 2.0f * cb * c.wb;
            const float obt = obs + wb2 * relu(fabsf(o) - c.omax) * copysignf(1.0f, o);
            const float Dbt = Dbs + wb2 * (relu(D - c.dmax) - relu(-D));
            if (live) {
                grad[(int64_t)(6 * kk + s) * N + i] = ab;
                if (s == 0) grad[(int64_t)(6 * kk + 4) * N + i] = obt;
                if (s == 1) grad[(int64_t)(6 * kk + 5) * N + i] = Dbt;
                bad = bad || !isfinite(ab) || !isfinite(obt) || !isfinite(Dbt);
            }
        }
    }
    if (status && bad) atomicOr(status, STAMP_STATUS_NONFINITE_GRAD);
}

// ---------------------------------------------------------------------------
// Packed lanes: one lane per (particle i, side s) sub-rollout, holding all B
// blocks (lane = 4i + s).  A step then costs B frictions, B(B-1)/2 pair terms
// (each once) and one pusher per lane, with no cross-lane moves, instead of
// 4 SL lanes per particle that repeat every pair term twice and the pusher on
// every block slot (at B = 3 one slot in four idles).  It rounds exactly as
// the block-per-lane form: each block's forces add in the same order
// (friction, partners by increasing index, pusher), the higher block of a
// pair takes the lower block's term with Delta negated (negation is exact),
// and the sides and blocks meet in the same sums.  Same tape layout.

// One semi-implicit Euler step of all B blocks of a sub-rollout.
template <int B>
__device__ __forceinline__ void step_forward_packed(const SimConst& c, Blk (&X)[B], const Push& p, float sig) {
    float Fx[B], Fy[B], Tq[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float inv = hw_rsq(fmaf(X[b].vx, X[b].vx, fmaf(X[b].vy, X[b].vy, c.ev2[b])));
        const float kf = c.cf[b] * inv;
        Fx[b] = -kf * X[b].vx;
        Fy[b] = -kf * X[b].vy;
        const float invw = hw_rsq(fmaf(X[b].om, X[b].om, c.ew2[b]));
        Tq[b] = -(c.cr[b] * invw) * X[b].om;
    }
    // pair terms, once per pair b < q: Delta = x_b - x_q, force fr Delta on b
    float pdx[B][B], pdy[B][B], pfr[B][B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = b + 1; q < B; ++q) {
            const float dx = X[b].x - X[q].x, dy = X[b].y - X[q].y;
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, c.er2));
            const float rinv = hw_rsq(d2);
            const float pen = fmaf(-d2, rinv, c.hsum[b][q]);
            pdx[b][q] = dx;
            pdy[b][q] = dy;
            pfr[b][q] = c.kb * softplus(pen, c.beta_log2e, c.ln2_over_beta) * rinv;
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = 0; q < B; ++q) {
            if (q == b) continue;
            const float fr = q > b ? pfr[b][q] : pfr[q][b];
            const float dx = q > b ? pdx[b][q] : -pdx[q][b];
            const float dy = q > b ? pdy[b][q] : -pdy[q][b];
            Fx[b] = fmaf(fr, dx, Fx[b]);
            Fy[b] = fmaf(fr, dy, Fy[b]);
        }
    }
    // the virtual pusher of this side, on block 0: contact normal e = R(phi0) n
    {
        const float relx = fmaf(sig, p.Vx, p.P0x) - X[0].x;
        const float rely = fmaf(sig, p.Vy, p.P0y) - X[0].y;
        float s0, c0;
        sincos_rd(X[0].ph, s0, c0);
        const float ex = fmaf(c0, p.nx, -(s0 * p.ny)), ey = fmaf(s0, p.nx, c0 * p.ny);
        const float pen = c.h0 - fmaf(ex, relx, ey * rely);
        const float f = c.kp * softplus(pen, c.beta_log2e, c.ln2_over_beta);
        Fx[0] = fmaf(-f, ex, Fx[0]);
        Fy[0] = fmaf(-f, ey, Fy[0]);
        Tq[0] = fmaf(-f, fmaf(relx, ey, -(rely * ex)), Tq[0]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        X[b].vx = fmaf(c.dtm[b], Fx[b], X[b].vx);
        X[b].vy = fmaf(c.dtm[b], Fy[b], X[b].vy);
        X[b].om = fmaf(c.dtI[b], Tq[b], X[b].om);
        X[b].x = fmaf(c.dt, X[b].vx, X[b].x);
        X[b].y = fmaf(c.dt, X[b].vy, X[b].y);
        X[b].ph = fmaf(c.dt, X[b].om, X[b].ph);
    }
}

// Reverse of step_forward_packed at pre-step states X; L: post-step adjoints
// on entry, pre-step adjoints on exit; pusher adjoints accumulate as in
// step_reverse (block 0).
template <int B>
__device__ __forceinline__ void step_reverse_packed(const SimConst& c, const Blk (&X)[B], Blk (&L)[B], const Push& p,
                                                    float sig, float& P0xb, float& P0yb, float& Vxb, float& Vyb) {
    float Fxb[B], Fyb[B], Tqb[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        L[b].vx = fmaf(c.dt, L[b].x, L[b].vx);
        L[b].vy = fmaf(c.dt, L[b].y, L[b].vy);
        L[b].om = fmaf(c.dt, L[b].ph, L[b].om);
        Fxb[b] = c.dtm[b] * L[b].vx;
        Fyb[b] = c.dtm[b] * L[b].vy;
        Tqb[b] = c.dtI[b] * L[b].om;
    }
    // pusher (block 0)
    {
        const float relx = fmaf(sig, p.Vx, p.P0x) - X[0].x;
        const float rely = fmaf(sig, p.Vy, p.P0y) - X[0].y;
        float s0, c0;
        sincos_rd(X[0].ph, s0, c0);
        const float ex = fmaf(c0, p.nx, -(s0 * p.ny)), ey = fmaf(s0, p.nx, c0 * p.ny);
        const float cross = fmaf(relx, ey, -(rely * ex));
        const float pen = c.h0 - fmaf(ex, relx, ey * rely);
        const float u = softplus_u(pen, c.beta_log2e);
        const float f = c.kp * fmaf(hw_log2(1.0f + u), c.ln2_over_beta, fmaxf(pen, 0.0f));
        const float rr = hw_rcp(1.0f + u);
        const float spg = pen >= 0.0f ? rr : u * rr;
        const float fb = -fmaf(cross, Tqb[0], fmaf(ex, Fxb[0], ey * Fyb[0]));
        const float crossb = -f * Tqb[0];
        const float penb = fb * c.kp * spg;
        const float exb = fmaf(-f, Fxb[0], -fmaf(crossb, rely, penb * relx));
        const float eyb = fmaf(-f, Fyb[0], fmaf(crossb, relx, -(penb * rely)));
        const float relxb = fmaf(crossb, ey, -(penb * ex));
        const float relyb = -fmaf(crossb, ex, penb * ey);
        const float c0b = fmaf(exb, p.nx, eyb * p.ny);
        const float s0b = fmaf(eyb, p.nx, -(exb * p.ny));
        L[0].ph += fmaf(c0, s0b, -(s0 * c0b));
        L[0].x -= relxb;
        L[0].y -= relyb;
        P0xb += relxb;
        P0yb += relyb;
        Vxb = fmaf(sig, relxb, Vxb);
        Vyb = fmaf(sig, relyb, Vyb);
    }
    // block-block contacts, once per pair b < q; each block adds its partners
    // in increasing order
    float pdx[B][B], pdy[B][B], pfr[B][B], pk2[B][B], pgx[B][B], pgy[B][B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = b + 1; q < B; ++q) {
            const float dx = X[b].x - X[q].x, dy = X[b].y - X[q].y;
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, c.er2));
            const float rinv = hw_rsq(d2);
            const float pen = fmaf(-d2, rinv, c.hsum[b][q]);
            const float u = softplus_u(pen, c.beta_log2e);
            const float fr = c.kb * fmaf(hw_log2(1.0f + u), c.ln2_over_beta, fmaxf(pen, 0.0f)) * rinv;
            const float rr = hw_rcp(1.0f + u);
            const float fp = c.kb * (pen >= 0.0f ? rr : u * rr);
            const float gx = Fxb[b] - Fxb[q], gy = Fyb[b] - Fyb[q];
            const float gu = fmaf(gx, dx, gy * dy) * rinv;
            pdx[b][q] = dx;
            pdy[b][q] = dy;
            pfr[b][q] = fr;
            pk2[b][q] = (fr + fp) * gu * rinv;
            pgx[b][q] = gx;
            pgy[b][q] = gy;
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = 0; q < B; ++q) {
            if (q == b) continue;
            const int lo = q > b ? b : q, hi = q > b ? q : b;
            const float sg = q > b ? 1.0f : -1.0f;  // the higher block sees Delta and g negated
            const float fr = pfr[lo][hi], k2 = pk2[lo][hi];
            const float dx = sg * pdx[lo][hi], dy = sg * pdy[lo][hi];
            const float gx = sg * pgx[lo][hi], gy = sg * pgy[lo][hi];
            L[b].x += fmaf(fr, gx, -(k2 * dx));
            L[b].y += fmaf(fr, gy, -(k2 * dy));
        }
    }
    // friction
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float inv = hw_rsq(fmaf(X[b].vx, X[b].vx, fmaf(X[b].vy, X[b].vy, c.ev2[b])));
        const float kf = c.cf[b] * inv;
        const float kd = kf * inv * inv * fmaf(Fxb[b], X[b].vx, Fyb[b] * X[b].vy);
        L[b].vx = fmaf(kd, X[b].vx, fmaf(-kf, Fxb[b], L[b].vx));
        L[b].vy = fmaf(kd, X[b].vy, fmaf(-kf, Fyb[b], L[b].vy));
        const float invw = hw_rsq(fmaf(X[b].om, X[b].om, c.ew2[b]));
        L[b].om = fmaf(-(c.crw2[b] * (invw * invw * invw)), Tqb[b], L[b].om);
    }
}

template <int B>
__device__ __forceinline__ void load_blks(Blk (&X)[B], const float* __restrict__ entry, uint32_t off) {
#pragma unroll
    for (int b = 0; b < B; ++b) load_blk_at(X[b], entry, off + 6 * b);
}

template <int B>
__device__ __forceinline__ void store_blks(const Blk (&X)[B], float* __restrict__ entry, uint32_t off) {
#pragma unroll
    for (int b = 0; b < B; ++b) store_blk_at(X[b], entry, off + 6 * b);
}

// Sum over the block slots in the block-per-lane form's order: (v0+v1)+(v2+v3),
// an absent fourth slot adding zero.
template <int B>
__device__ __forceinline__ float blocks_sum(const float (&v)[B]) {
    if constexpr (B == 1) return v[0];
    else if constexpr (B == 2) return v[0] + v[1];
    else if constexpr (B == 3) return (v[0] + v[1]) + (v[2] + 0.0f);
    else return (v[0] + v[1]) + (v[2] + v[3]);
}

// Orders a wave's LDS writes before its later LDS reads by other lanes of the
// same wave (and those reads before later writes): LDS instructions of one
// wave execute in issue order; the fences keep the compiler from moving them
// and wait for the writes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int B>
__device__ __forceinline__ void stage_blks(const Blk (&X)[B], float* stage, int lw) {
    float2* q = reinterpret_cast<float2*>(stage + lw * 6 * B);
#pragma unroll
    for (int b = 0; b < B; ++b) {
        q[3 * b + 0] = make_float2(X[b].x, X[b].y);
        q[3 * b + 1] = make_float2(X[b].ph, X[b].vx);
        q[3 * b + 2] = make_float2(X[b].vy, X[b].om);
    }
}

// Forward rollout of one packed lane (particle i, side s); as rollout_fwd_lane.
// WAVES: waves per workgroup (each stages its tape stores in its own LDS region).
template <int B, int WAVES>
__device__ __forceinline__ void rollout_fwd_packed(const SimConst& c, int N, const float* __restrict__ theta,
                                                   float* __restrict__ cost, float* __restrict__ tape,
                                                   const TapeGeom& g, uint32_t* status, int64_t lane) {
    const int64_t iw = lane / 4;
    const bool live = iw < N;
    const int i = live ? (int)iw : N - 1;
    const int s = (int)(lane % 4);
    const uint32_t off = (uint32_t)(((int64_t)4 * i + s) * B * 6);
    const int64_t stride = 6 * B * g.lanes;
    const int H = c.H, T = c.T;
    // the wave's span of a tape entry: its live lanes' 6B floats each, from
    // the first lane's slot on (a multiple of 4 floats: lanes come in
    // particles of 4)
    __shared__ __align__(16) float stage_all[WAVES][64 * 6 * B];  // one region per wave of a workgroup
    float* stage = stage_all[WAVES == 1 ? 0 : (threadIdx.x >> 6) % WAVES];
    const int lw = (int)(lane & 63);
    const int64_t lane0 = lane - lw;
    const int64_t wave_off = lane0 * 6 * B;
    const int span4 = (int)(min((int64_t)64, (int64_t)4 * N - lane0) * 6 * B / 4);
    Blk S[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        S[b].x = c.pose0[b][0];
        S[b].y = c.pose0[b][1];
        S[b].ph = c.pose0[b][2];
        S[b].vx = S[b].vy = S[b].om = 0.0f;
    }
    float Px[kMaxPushes + 1], Py[kMaxPushes + 1];
    float Lbound = 0.0f;
    Push p;
    side_frame(s, p);
    int64_t entry = 0;
    for (int kk = 0; kk < H; ++kk) {
        const int tk = phase_start(kk, T, H), tk1 = phase_start(kk + 1, T, H);
        const float invL = 1.0f / (float)(tk1 - tk);
        Px[kk] = S[0].x;
        Py[kk] = S[0].y;
        const float z = side_weight(theta, N, i, kk, s);
        const float o = theta[(int64_t)(6 * kk + 4) * N + i];
        const float D = theta[(int64_t)(6 * kk + 5) * N + i];
        Anchor an;
        phase_push(c, S[0].x, S[0].y, S[0].ph, o, D, p, an);
        Lbound += relu(fabsf(o) - c.omax) * relu(fabsf(o) - c.omax) + relu(-D) * relu(-D) +
                  relu(D - c.dmax) * relu(D - c.dmax);
        Blk X[B];
#pragma unroll
        for (int b = 0; b < B; ++b) X[b] = S[b];
        Profile prof;
        prof.reset(invL);
        const int nst = tk1 - tk;
        if (tape && g.ckpt == 0) {
            // Each step's states go through LDS so that the wave writes its
            // contiguous span of the entry with 16-byte stores of consecutive
            // lanes (a lane's own 6B floats would make every store
            // instruction touch B times the cache lines).
            float* e = tape + (int64_t)tk * stride + wave_off;
            for (int j = 0; j < nst; ++j, e += stride) {
                stage_blks<B>(X, stage, lw);
                wave_lds_sync();
                for (int k = lw; k < span4; k += 64)
                    *reinterpret_cast<float4*>(e + 4 * k) = *reinterpret_cast<const float4*>(stage + 4 * k);
                wave_lds_sync();
                step_forward_packed<B>(c, X, p, prof.at(j));
            }
        } else {
            int until = 0;
            for (int j = 0; j < nst; ++j) {
                if (tape && until == 0) {
                    if (live) store_blks<B>(X, tape + entry * stride, off);
                    ++entry;
                    until = g.ckpt;
                }
                --until;
                step_forward_packed<B>(c, X, p, prof.at(j));
            }
        }
        if (tape && live) store_blks<B>(X, tape + g.ends_off + (int64_t)kk * stride, off);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            S[b].x = side_sum<1>(z * X[b].x);
            S[b].y = side_sum<1>(z * X[b].y);
            S[b].ph = side_sum<1>(z * X[b].ph);
            S[b].vx = side_sum<1>(z * X[b].vx);
            S[b].vy = side_sum<1>(z * X[b].vy);
            S[b].om = side_sum<1>(z * X[b].om);
        }
    }
    Px[H] = S[0].x;
    Py[H] = S[0].y;
    if (s != 0 || !live) return;
    const float dxg = fabsf(Px[H] - c.goal[0]) - c.tol, dyg = fabsf(Py[H] - c.goal[1]) - c.tol;
    const float Ltarget = relu(dxg) * relu(dxg) + relu(dyg) * relu(dyg);
    const float Lrot = 1.0f - cosf(S[0].ph - c.goal[2]);
    float Ltraj = 0.0f;
    for (int kk = 1; kk <= H; ++kk) {
        Ltraj += smooth_abs(Px[kk - 1] - Px[kk], c.ea2) + smooth_abs(Py[kk - 1] - Py[kk], c.ea2);
        Ltraj += smooth_abs(Px[kk] - Px[H], c.ea2) + smooth_abs(Py[kk] - Py[H], c.ea2);
        Ltraj -= smooth_abs(Px[kk - 1] - Px[H], c.ea2) + smooth_abs(Py[kk - 1] - Py[H], c.ea2);
    }
    const float C = c.wt * Ltarget + c.wr * Lrot + c.wtr * Ltraj + c.wb * Lbound;
    cost[i] = C;
    if (status && !isfinite(C)) atomicOr(status, STAMP_STATUS_NONFINITE_COST);
}

// Reverse sweep of one packed lane; as rollout_adj_lane.
template <int B>
__device__ __forceinline__ void rollout_adj_packed(const SimConst& c, int N, const float* __restrict__ theta,
                                                   const float* __restrict__ tape, const TapeGeom& g,
                                                   const float* __restrict__ cost_bar, float cb_scalar,
                                                   float* __restrict__ grad, float* __restrict__ seg,
                                                   uint32_t* status, int64_t lane) {
    const int64_t iw = lane / 4;
    const bool live = iw < N;
    const int i = live ? (int)iw : N - 1;
    const int s = (int)(lane % 4);
    const int64_t slot0 = ((int64_t)4 * i + s) * B;
    const uint32_t off = (uint32_t)(slot0 * 6);
    const int H = c.H, T = c.T;
    const int64_t stride = 6 * B * g.lanes;

    int ent[kMaxPushes];
    {
        int e = 0;
        for (int kk = 0; kk < H; ++kk) {
            const int tk = phase_start(kk, T, H), tk1 = phase_start(kk + 1, T, H);
            ent[kk] = (g.ckpt == 0) ? tk : e;
            if (g.ckpt) e += (tk1 - tk + g.ckpt - 1) / g.ckpt;
        }
    }
    float Px[kMaxPushes + 1], Py[kMaxPushes + 1];
    for (int kk = 0; kk < H; ++kk) {
        Px[kk] = tape[ent[kk] * stride + slot0 * 6 + 0];
        Py[kk] = tape[ent[kk] * stride + slot0 * 6 + 1];
    }
    float phT;
    {
        const float z = side_weight(theta, N, i, H - 1, s);
        const float* e = tape + g.ends_off + (int64_t)(H - 1) * stride + slot0 * 6;
        Px[H] = side_sum<1>(z * e[0]);
        Py[H] = side_sum<1>(z * e[1]);
        phT = side_sum<1>(z * e[2]);
    }
    const float cb = cost_bar ? cost_bar[i] : cb_scalar;
    float Pxb[kMaxPushes + 1], Pyb[kMaxPushes + 1];
    for (int kk = 0; kk <= H; ++kk) Pxb[kk] = Pyb[kk] = 0.0f;
    {
        const float ux = Px[H] - c.goal[0], uy = Py[H] - c.goal[1];
        Pxb[H] += cb * c.wt * 2.0f * relu(fabsf(ux) - c.tol) * copysignf(1.0f, ux);
        Pyb[H] += cb * c.wt * 2.0f * relu(fabsf(uy) - c.tol) * copysignf(1.0f, uy);
    }
    const float phTb = cb * c.wr * sinf(phT - c.goal[2]);
    const float wtr = cb * c.wtr;
    if (!c.per_phase) {
        for (int kk = 1; kk <= H; ++kk) {
            float u, dd;
            u = Px[kk - 1] - Px[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk - 1] += dd; Pxb[kk] -= dd;
            u = Py[kk - 1] - Py[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk - 1] += dd; Pyb[kk] -= dd;
            u = Px[kk] - Px[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk] += dd;     Pxb[H] -= dd;
            u = Py[kk] - Py[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk] += dd;     Pyb[H] -= dd;
            u = Px[kk - 1] - Px[H];   dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk - 1] -= dd; Pxb[H] += dd;
            u = Py[kk - 1] - Py[H];   dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk - 1] -= dd; Pyb[H] += dd;
        }
    } else {
        for (int kk = 1; kk < H; ++kk) {
            float u, dd;
            u = Px[kk - 1] - Px[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk] -= dd;
            u = Py[kk - 1] - Py[kk];  dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk] -= dd;
            u = Px[kk] - Px[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pxb[kk] += dd;
            u = Py[kk] - Py[H];       dd = wtr * u / smooth_abs(u, c.ea2);  Pyb[kk] += dd;
        }
    }
    Blk Ls[B];
#pragma unroll
    for (int b = 0; b < B; ++b) Ls[b].x = Ls[b].y = Ls[b].ph = Ls[b].vx = Ls[b].vy = Ls[b].om = 0.0f;
    Ls[0].x = Pxb[H];
    Ls[0].y = Pyb[H];
    Ls[0].ph = phTb;

    Push p;
    side_frame(s, p);
    bool bad = false;
    for (int kk = H - 1; kk >= 0; --kk) {
        const int tk = phase_start(kk, T, H), tk1 = phase_start(kk + 1, T, H);
        const float invL = 1.0f / (float)(tk1 - tk);
        const float z = side_weight(theta, N, i, kk, s);
        const float o = theta[(int64_t)(6 * kk + 4) * N + i];
        const float D = theta[(int64_t)(6 * kk + 5) * N + i];
        Blk Xe[B], L[B];
        load_blks<B>(Xe, tape + g.ends_off + (int64_t)kk * stride, off);
        float zpb[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            zpb[b] = Ls[b].x * Xe[b].x + Ls[b].y * Xe[b].y + Ls[b].ph * Xe[b].ph + Ls[b].vx * Xe[b].vx +
                     Ls[b].vy * Xe[b].vy + Ls[b].om * Xe[b].om;
            L[b].x = z * Ls[b].x;
            L[b].y = z * Ls[b].y;
            L[b].ph = z * Ls[b].ph;
            L[b].vx = z * Ls[b].vx;
            L[b].vy = z * Ls[b].vy;
            L[b].om = z * Ls[b].om;
        }
        const float zb = blocks_sum<B>(zpb);
        const float ab = z * (zb - side_sum<1>(z * zb));  // softmax VJP
        Blk A;
        load_blk_at(A, tape + ent[kk] * stride, off);  // block 0's pose: the anchor
        Anchor an;
        phase_push(c, A.x, A.y, A.ph, o, D, p, an);
        float P0xb = 0.0f, P0yb = 0.0f, Vxb = 0.0f, Vyb = 0.0f;
        Profile prof;
        prof.reset(invL);
        if (g.ckpt == 0) {
            const float* base = tape + (int64_t)tk * stride;
            int j = tk1 - tk - 1;
            Blk XA[B], XB[B];
            load_blks<B>(XA, base + (int64_t)j * stride, off);
            load_blks<B>(XB, base + (int64_t)max(j - 1, 0) * stride, off);
            for (; j >= 1; j -= 2) {
                Blk X[B];
#pragma unroll
                for (int b = 0; b < B; ++b) X[b] = XA[b];
                load_blks<B>(XA, base + (int64_t)max(j - 2, 0) * stride, off);
                step_reverse_packed<B>(c, X, L, p, prof.at(j), P0xb, P0yb, Vxb, Vyb);
#pragma unroll
                for (int b = 0; b < B; ++b) X[b] = XB[b];
                load_blks<B>(XB, base + (int64_t)max(j - 3, 0) * stride, off);
                step_reverse_packed<B>(c, X, L, p, prof.at(j - 1), P0xb, P0yb, Vxb, Vyb);
            }
            if (j == 0) step_reverse_packed<B>(c, XA, L, p, prof.at(0), P0xb, P0yb, Vxb, Vyb);
        } else {
            const int nseg = (tk1 - tk + g.ckpt - 1) / g.ckpt;
            for (int q = nseg - 1; q >= 0; --q) {
                const int js = q * g.ckpt;
                const int je = min(js + g.ckpt, tk1 - tk);
                Blk X[B];
                load_blks<B>(X, tape + (int64_t)(ent[kk] + q) * stride, off);
                for (int j = js; j < je; ++j) {
                    if (live) store_blks<B>(X, seg + (int64_t)(j - js) * stride, off);
                    step_forward_packed<B>(c, X, p, prof.at(j));
                }
                for (int j = je - 1; j >= js; --j) {
                    if (live) load_blks<B>(X, seg + (int64_t)(j - js) * stride, off);
                    step_reverse_packed<B>(c, X, L, p, prof.at(j), P0xb, P0yb, Vxb, Vyb);
                }
            }
        }
        const float eAx = fmaf(an.cA, p.nx, -(an.sA * p.ny)), eAy = fmaf(an.sA, p.nx, an.cA * p.ny);
        const float Db = -fmaf(Vxb, eAx, Vyb * eAy);
        const float eAxb = -D * Vxb, eAyb = -D * Vyb;
        const float cAb = fmaf(eAxb, p.nx, eAyb * p.ny) + fmaf(P0xb, an.q0x, P0yb * an.q0y);
        const float sAb = fmaf(eAyb, p.nx, -(eAxb * p.ny)) + fmaf(P0yb, an.q0x, -(P0xb * an.q0y));
        const float q0xb = fmaf(an.cA, P0xb, an.sA * P0yb), q0yb = fmaf(an.cA, P0yb, -(an.sA * P0xb));
        const float ob = fmaf(q0xb, p.tx, q0yb * p.ty);
        const float Aphb = fmaf(an.cA, sAb, -(an.sA * cAb));
#pragma unroll
        for (int b = 0; b < B; ++b) {
            Ls[b].x = side_sum<1>(L[b].x);
            Ls[b].y = side_sum<1>(L[b].y);
            Ls[b].ph = side_sum<1>(L[b].ph);
            Ls[b].vx = side_sum<1>(L[b].vx);
            Ls[b].vy = side_sum<1>(L[b].vy);
            Ls[b].om = side_sum<1>(L[b].om);
        }
        const float Axs = side_sum<1>(P0xb), Ays = side_sum<1>(P0yb), Aphs = side_sum<1>(Aphb);
        const float obs = side_sum<1>(ob), Dbs = side_sum<1>(Db);
        if (c.per_phase) {
#pragma unroll
            for (int b = 0; b < B; ++b) Ls[b].x = Ls[b].y = Ls[b].ph = Ls[b].vx = Ls[b].vy = Ls[b].om = 0.0f;
            Ls[0].x = Pxb[kk];
            Ls[0].y = Pyb[kk];
        } else {
            Ls[0].x += Axs + Pxb[kk];
            Ls[0].y += Ays + Pyb[kk];
            Ls[0].ph += Aphs;
        }
        const float wb2 = 2.0f * cb * c.wb;
        const float obt = obs + wb2 * relu(fabsf(o) - c.omax) * copysignf(1.0f, o);
        const float Dbt = Dbs + wb2 * (relu(D - c.dmax) - relu(-D));
        if (live) {
            grad[(int64_t)(6 * kk + s) * N + i] = ab;
            if (s == 0) grad[(int64_t)(6 * kk + 4) * N + i] = obt;
            if (s == 1) grad[(int64_t)(6 * kk + 5) * N + i] = Dbt;
            bad = bad || !isfinite(ab) || !isfinite(obt) || !isfinite(Dbt);
        }
    }
    if (status && bad) atomicOr(status, STAMP_STATUS_NONFINITE_GRAD);
}

template <int B>
__global__ __launch_bounds__(kRolloutBlock) void k_rollout_fwd_packed(SimConst c, int N,
                                                                      const float* __restrict__ theta,
                                                                      float* __restrict__ cost,
                                                                      float* __restrict__ tape, TapeGeom g,
                                                                      uint32_t* status) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    rollout_fwd_packed<B, 1>(c, N, theta, cost, tape, g, status, lane);
}

template <int B>
__global__ __launch_bounds__(kRolloutBlock) void k_rollout_adj_packed(SimConst c, int N,
                                                                      const float* __restrict__ theta,
                                                                      const float* __restrict__ tape, TapeGeom g,
                                                                      const float* __restrict__ cost_bar,
                                                                      float cb_scalar, float* __restrict__ grad,
                                                                      float* __restrict__ seg, uint32_t* status) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    rollout_adj_packed<B>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, lane);
}

// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kRolloutBlock) void k_rollout_fwd(SimConst c, int N, const float* __restrict__ theta,
                                                               float* __restrict__ cost, float* __restrict__ tape,
                                                               TapeGeom g, uint32_t* status) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    rollout_fwd_lane<B>(c, N, theta, cost, tape, g, status, lane);
}

template <int B>
__global__ __launch_bounds__(kRolloutBlock) void k_rollout_adj(SimConst c, int N, const float* __restrict__ theta,
                                                               const float* __restrict__ tape, TapeGeom g,
                                                               const float* __restrict__ cost_bar, float cb_scalar,
                                                               float* __restrict__ grad, float* __restrict__ seg,
                                                               uint32_t* status) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    rollout_adj_lane<B>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, lane);
}

// ---------------------------------------------------------------------------
// Batched rollouts: one launch over the wave tiles of many problems.  Tile t is
// (problem p, first particle i0) and covers 64 lanes: 64 / (4 SL) particles
// (rollout_tile_particles); each wave takes tiles in a grid-stride loop.  The
// block count B of the problem selects the compiled body at run time.
template <int B, bool PK>
__device__ __forceinline__ void fwd_tile(const ProblemDesc& D, int i0, int l, const float* theta, float* cost,
                                         float* tape, uint32_t* status) {
    const int64_t lane = (int64_t)(PK ? 4 : Slots<B>::LANES) * i0 + l;
    if constexpr (PK)
        rollout_fwd_packed<B, 4>(D.c, D.N, theta + D.theta_off, cost + D.cost_off, tape ? tape + D.tape_off : nullptr,
                              D.g, status, lane);
    else
        rollout_fwd_lane<B>(D.c, D.N, theta + D.theta_off, cost + D.cost_off, tape ? tape + D.tape_off : nullptr,
                            D.g, status, lane);
}

template <int B, bool PK>
__device__ __forceinline__ void adj_tile(const ProblemDesc& D, int i0, int l, const float* theta, const float* tape,
                                         float cb_scalar, float* grad, float* seg, uint32_t* status) {
    const int64_t lane = (int64_t)(PK ? 4 : Slots<B>::LANES) * i0 + l;
    if constexpr (PK)
        rollout_adj_packed<B>(D.c, D.N, theta + D.theta_off, tape + D.tape_off, D.g, nullptr, cb_scalar,
                              grad + D.theta_off, seg + D.seg_off, status, lane);
    else
        rollout_adj_lane<B>(D.c, D.N, theta + D.theta_off, tape + D.tape_off, D.g, nullptr, cb_scalar,
                            grad + D.theta_off, seg + D.seg_off, status, lane);
}

template <bool PK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PK ? 2 : 4))) void k_rollout_fwd_batched(const ProblemDesc* __restrict__ descs,
                                                             const int2* __restrict__ tiles, int ntiles,
                                                             const float* __restrict__ theta, float* __restrict__ cost,
                                                             float* __restrict__ tape, uint32_t* status) {
    const int waves = blockDim.x >> 6;
    // the wave index is uniform across the wave: readfirstlane lets the tile,
    // its problem descriptor and the scene constants live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    for (int t = blockIdx.x * waves + wave; t < ntiles; t += gridDim.x * waves) {
        const int2 tl = tiles[t];
        const ProblemDesc& D = descs[tl.x];
        switch (D.c.B) {
            case 1: fwd_tile<1, PK>(D, tl.y, l, theta, cost, tape, status); break;
            case 2: fwd_tile<2, PK>(D, tl.y, l, theta, cost, tape, status); break;
            case 3: fwd_tile<3, PK>(D, tl.y, l, theta, cost, tape, status); break;
            default: fwd_tile<4, PK>(D, tl.y, l, theta, cost, tape, status); break;
        }
    }
}

template <bool PK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PK ? 2 : 4))) void k_rollout_adj_batched(const ProblemDesc* __restrict__ descs,
                                                             const int2* __restrict__ tiles, int ntiles,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ tape, float cb_scalar,
                                                             float* __restrict__ grad, float* __restrict__ seg,
                                                             uint32_t* status) {
    const int waves = blockDim.x >> 6;
    // the wave index is uniform across the wave: readfirstlane lets the tile,
    // its problem descriptor and the scene constants live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    for (int t = blockIdx.x * waves + wave; t < ntiles; t += gridDim.x * waves) {
        const int2 tl = tiles[t];
        const ProblemDesc& D = descs[tl.x];
        switch (D.c.B) {
            case 1: adj_tile<1, PK>(D, tl.y, l, theta, tape, cb_scalar, grad, seg, status); break;
            case 2: adj_tile<2, PK>(D, tl.y, l, theta, tape, cb_scalar, grad, seg, status); break;
            case 3: adj_tile<3, PK>(D, tl.y, l, theta, tape, cb_scalar, grad, seg, status); break;
            default: adj_tile<4, PK>(D, tl.y, l, theta, tape, cb_scalar, grad, seg, status); break;
        }
    }
}

int rollout_tile_particles(int B, bool packed) { return packed ? 16 : 64 / (4 * (B == 1 ? 1 : (B == 2 ? 2 : 4))); }

hipError_t launch_rollout_fwd_batched(const ProblemDesc* descs, const int2* tiles, int ntiles, int block,
                                      int grid, const float* theta, float* cost, float* tape, uint32_t* status,
                                      hipStream_t st, bool packed) {
    if (packed)
        hipLaunchKernelGGL(k_rollout_fwd_batched<true>, dim3(grid), dim3(block), 0, st, descs, tiles, ntiles, theta,
                           cost, tape, status);
    else
        hipLaunchKernelGGL(k_rollout_fwd_batched<false>, dim3(grid), dim3(block), 0, st, descs, tiles, ntiles, theta,
                           cost, tape, status);
    return hipGetLastError();
}

hipError_t launch_rollout_adj_batched(const ProblemDesc* descs, const int2* tiles, int ntiles, int block,
                                      int grid, const float* theta, const float* tape, float cb_scalar,
                                      float* grad, float* seg, uint32_t* status, hipStream_t st, bool packed) {
    if (packed)
        hipLaunchKernelGGL(k_rollout_adj_batched<true>, dim3(grid), dim3(block), 0, st, descs, tiles, ntiles, theta,
                           tape, cb_scalar, grad, seg, status);
    else
        hipLaunchKernelGGL(k_rollout_adj_batched<false>, dim3(grid), dim3(block), 0, st, descs, tiles, ntiles, theta,
                           tape, cb_scalar, grad, seg, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int B>
static hipError_t launch_fwd_b(const SimConst& c, int N, const float* theta, float* cost, float* tape,
                               const TapeGeom& g, uint32_t* status, hipStream_t st, bool packed) {
    // one block: both layouts are the same lanes; the block-per-lane kernel runs it
    const bool pk = packed && B > 1;
    const int64_t lanes = (int64_t)(pk ? 4 : Slots<B>::LANES) * N;
    const unsigned grid = (unsigned)((lanes + kRolloutBlock - 1) / kRolloutBlock);
    if (pk)
        hipLaunchKernelGGL(k_rollout_fwd_packed<B>, dim3(grid), dim3(kRolloutBlock), 0, st, c, N, theta, cost, tape,
                           g, status);
    else
        hipLaunchKernelGGL(k_rollout_fwd<B>, dim3(grid), dim3(kRolloutBlock), 0, st, c, N, theta, cost, tape, g,
                           status);
    return hipGetLastError();
}

template <int B>
static hipError_t launch_adj_b(const SimConst& c, int N, const float* theta, const float* tape,
                               const TapeGeom& g, const float* cost_bar, float cb_scalar, float* grad,
                               float* seg, uint32_t* status, hipStream_t st, bool packed) {
    const bool pk = packed && B > 1;
    const int64_t lanes = (int64_t)(pk ? 4 : Slots<B>::LANES) * N;
    const unsigned grid = (unsigned)((lanes + kRolloutBlock - 1) / kRolloutBlock);
    if (pk)
        hipLaunchKernelGGL(k_rollout_adj_packed<B>, dim3(grid), dim3(kRolloutBlock), 0, st, c, N, theta, tape, g,
                           cost_bar, cb_scalar, grad, seg, status);
    else
        hipLaunchKernelGGL(k_rollout_adj<B>, dim3(grid), dim3(kRolloutBlock), 0, st, c, N, theta, tape, g, cost_bar,
                           cb_scalar, grad, seg, status);
    return hipGetLastError();
}

hipError_t launch_rollout_fwd(const SimConst& c, int N, const float* theta, float* cost, float* tape,
                              const TapeGeom& g, uint32_t* status, hipStream_t st, bool packed) {
    switch (c.B) {
        case 1: return launch_fwd_b<1>(c, N, theta, cost, tape, g, status, st, packed);
        case 2: return launch_fwd_b<2>(c, N, theta, cost, tape, g, status, st, packed);
        case 3: return launch_fwd_b<3>(c, N, theta, cost, tape, g, status, st, packed);
        case 4: return launch_fwd_b<4>(c, N, theta, cost, tape, g, status, st, packed);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rollout_adj(const SimConst& c, int N, const float* theta, const float* tape,
                              const TapeGeom& g, const float* cost_bar, float cb_scalar, float* grad,
                              float* seg, uint32_t* status, hipStream_t st, bool packed) {
    switch (c.B) {
        case 1: return launch_adj_b<1>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st, packed);
        case 2: return launch_adj_b<2>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st, packed);
        case 3: return launch_adj_b<3>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st, packed);
        case 4: return launch_adj_b<4>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st, packed);
    }
    return hipErrorInvalidValue;
}

}  // namespace stamp
