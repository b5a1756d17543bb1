// Relaxed block-pushing rollout and its adjoint on gfx950.
//
// Model (Sec. III-B: semi-implicit Euler with spring-based penalty contacts;
// Sec. IV-A and Appendix E: pushing from the N/E/S/W faces of block 0).
// Push phase k runs once per side s from the shared phase-start state S_k; the
// next phase starts from S_{k+1} = sum_s softmax(a_k)_s X_s(t_{k+1}).  One lane
// per (particle, side): lane 4i+s integrates X_s of particle i in registers;
// the quad of a particle meets only at phase boundaries (DPP).
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

template <int B>
struct State {
    float x[B], y[B], ph[B], vx[B], vy[B], om[B];
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

// Entry e of the tape holds, for every lane, its 6B-float state contiguously.
template <int B>
__device__ __forceinline__ void load_state(State<B>& X, const float* __restrict__ entry, int64_t lane) {
    const float2* p = reinterpret_cast<const float2*>(entry + lane * (6 * B));
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float2 a = p[3 * b + 0], c = p[3 * b + 1], e = p[3 * b + 2];
        X.x[b] = a.x;
        X.y[b] = a.y;
        X.ph[b] = c.x;
        X.vx[b] = c.y;
        X.vy[b] = e.x;
        X.om[b] = e.y;
    }
}

template <int B>
__device__ __forceinline__ void store_state(const State<B>& X, float* __restrict__ entry, int64_t lane) {
    float2* p = reinterpret_cast<float2*>(entry + lane * (6 * B));
#pragma unroll
    for (int b = 0; b < B; ++b) {
        p[3 * b + 0] = make_float2(X.x[b], X.y[b]);
        p[3 * b + 1] = make_float2(X.ph[b], X.vx[b]);
        p[3 * b + 2] = make_float2(X.vy[b], X.om[b]);
    }
}

// One semi-implicit Euler step of the sub-rollout (pusher of this lane's side).
// Products that feed a sum are fused (fmaf); the reverse below differentiates
// the same expressions.
template <int B>
__device__ __forceinline__ void step_forward(const SimConst& c, State<B>& X, const Push& p, float sig) {
    float Fx[B], Fy[B], Tq[B];
    // regularised Coulomb friction, every block
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float inv = hw_rsq(fmaf(X.vx[b], X.vx[b], fmaf(X.vy[b], X.vy[b], c.ev2[b])));
        const float k = c.cf[b] * inv;
        Fx[b] = -k * X.vx[b];
        Fy[b] = -k * X.vy[b];
        const float invw = hw_rsq(fmaf(X.om[b], X.om[b], c.ew2[b]));
        Tq[b] = -(c.cr[b] * invw) * X.om[b];
    }
    // block-block penalty on the inscribed disks, central force
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = b + 1; q < B; ++q) {
            const float dx = X.x[b] - X.x[q], dy = X.y[b] - X.y[q];
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, c.er2));
            const float rinv = hw_rsq(d2);
            const float pen = fmaf(-d2, rinv, c.hsum[b][q]);  // h_b + h_c - r
            const float fr = c.kb * softplus(pen, c.beta_log2e, c.ln2_over_beta) * rinv;
            Fx[b] = fmaf(fr, dx, Fx[b]);
            Fy[b] = fmaf(fr, dy, Fy[b]);
            Fx[q] = fmaf(-fr, dx, Fx[q]);
            Fy[q] = fmaf(-fr, dy, Fy[q]);
        }
    }
    // the virtual pusher of this side, on block 0: contact normal e = R(phi0) n
    {
        const float relx = fmaf(sig, p.Vx, p.P0x) - X.x[0];
        const float rely = fmaf(sig, p.Vy, p.P0y) - X.y[0];
        float s0, c0;
        sincos_rd(X.ph[0], s0, c0);
        const float ex = fmaf(c0, p.nx, -(s0 * p.ny)), ey = fmaf(s0, p.nx, c0 * p.ny);
        const float pen = c.h0 - fmaf(ex, relx, ey * rely);
        const float f = c.kp * softplus(pen, c.beta_log2e, c.ln2_over_beta);
        Fx[0] = fmaf(-f, ex, Fx[0]);
        Fy[0] = fmaf(-f, ey, Fy[0]);
        Tq[0] = fmaf(-f, fmaf(relx, ey, -(rely * ex)), Tq[0]);  // rel x (-f e)
    }
    // semi-implicit Euler: velocities, then positions with the new velocities
#pragma unroll
    for (int b = 0; b < B; ++b) {
        X.vx[b] = fmaf(c.dtm[b], Fx[b], X.vx[b]);
        X.vy[b] = fmaf(c.dtm[b], Fy[b], X.vy[b]);
        X.om[b] = fmaf(c.dtI[b], Tq[b], X.om[b]);
        X.x[b] = fmaf(c.dt, X.vx[b], X.x[b]);
        X.y[b] = fmaf(c.dt, X.vy[b], X.y[b]);
        X.ph[b] = fmaf(c.dt, X.om[b], X.ph[b]);
    }
}

// Reverse of step_forward at pre-step state X.  On entry L is the adjoint of the
// post-step state; on exit the adjoint of the pre-step state.  Adjoints of the
// phase's pusher data (P0, V) are accumulated.
template <int B>
__device__ __forceinline__ void step_reverse(const SimConst& c, const State<B>& X, State<B>& L, const Push& p,
                                             float sig, float& P0xb, float& P0yb, float& Vxb, float& Vyb) {
    float Fxb[B], Fyb[B], Tqb[B];
    // integrator: x' = x + dt v', v' = v + (dt/m) F
#pragma unroll
    for (int b = 0; b < B; ++b) {
        L.vx[b] = fmaf(c.dt, L.x[b], L.vx[b]);
        L.vy[b] = fmaf(c.dt, L.y[b], L.vy[b]);
        L.om[b] = fmaf(c.dt, L.ph[b], L.om[b]);
        Fxb[b] = c.dtm[b] * L.vx[b];
        Fyb[b] = c.dtm[b] * L.vy[b];
        Tqb[b] = c.dtI[b] * L.om[b];
    }
    // pusher
    {
        const float relx = fmaf(sig, p.Vx, p.P0x) - X.x[0];
        const float rely = fmaf(sig, p.Vy, p.P0y) - X.y[0];
        float s0, c0;
        sincos_rd(X.ph[0], s0, c0);
        const float ex = fmaf(c0, p.nx, -(s0 * p.ny)), ey = fmaf(s0, p.nx, c0 * p.ny);
        const float cross = fmaf(relx, ey, -(rely * ex));
        const float pen = c.h0 - fmaf(ex, relx, ey * rely);
        const float u = softplus_u(pen, c.beta_log2e);
        const float f = c.kp * fmaf(hw_log2(1.0f + u), c.ln2_over_beta, fmaxf(pen, 0.0f));
        const float rr = hw_rcp(1.0f + u);
        const float spg = pen >= 0.0f ? rr : u * rr;  // sp'(pen)
        // F0 += -f e, T0 += -f cross
        const float fb = -fmaf(cross, Tqb[0], fmaf(ex, Fxb[0], ey * Fyb[0]));
        const float crossb = -f * Tqb[0];
        const float penb = fb * c.kp * spg;
        // cross = relx ey - rely ex, pen = h0 - (ex relx + ey rely)
        const float exb = fmaf(-f, Fxb[0], -fmaf(crossb, rely, penb * relx));
        const float eyb = fmaf(-f, Fyb[0], fmaf(crossb, relx, -(penb * rely)));
        const float relxb = fmaf(crossb, ey, -(penb * ex));
        const float relyb = -fmaf(crossb, ex, penb * ey);
        // e = (c0 nx - s0 ny, s0 nx + c0 ny)
        const float c0b = fmaf(exb, p.nx, eyb * p.ny);
        const float s0b = fmaf(eyb, p.nx, -(exb * p.ny));
        L.ph[0] += fmaf(c0, s0b, -(s0 * c0b));
        // rel = P0 + sig V - x0
        L.x[0] -= relxb;
        L.y[0] -= relyb;
        P0xb += relxb;
        P0yb += relyb;
        Vxb = fmaf(sig, relxb, Vxb);
        Vyb = fmaf(sig, relyb, Vyb);
    }
    // block-block contacts: F_b += f u, F_c -= f u with u = Delta / r
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int q = b + 1; q < B; ++q) {
            const float dx = X.x[b] - X.x[q], dy = X.y[b] - X.y[q];
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, c.er2));
            const float rinv = hw_rsq(d2);
            const float pen = fmaf(-d2, rinv, c.hsum[b][q]);
            const float u = softplus_u(pen, c.beta_log2e);
            const float fr = c.kb * fmaf(hw_log2(1.0f + u), c.ln2_over_beta, fmaxf(pen, 0.0f)) * rinv;
            const float rr = hw_rcp(1.0f + u);
            const float fp = c.kb * (pen >= 0.0f ? rr : u * rr);  // f'(pen)
            const float gx = Fxb[b] - Fxb[q], gy = Fyb[b] - Fyb[q];
            const float gu = fmaf(gx, dx, gy * dy) * rinv;   // adjoint of f
            // d(f u)/dDelta = f/r (I - u u^T) + f'(pen)(-u) u^T
            const float k2 = (fr + fp) * gu * rinv;  // coefficient of Delta
            const float dxb = fmaf(fr, gx, -(k2 * dx));
            const float dyb = fmaf(fr, gy, -(k2 * dy));
            L.x[b] += dxb;
            L.x[q] -= dxb;
            L.y[b] += dyb;
            L.y[q] -= dyb;
        }
    }
    // friction
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const float inv = hw_rsq(fmaf(X.vx[b], X.vx[b], fmaf(X.vy[b], X.vy[b], c.ev2[b])));
        const float k = c.cf[b] * inv;
        const float kd = k * inv * inv * fmaf(Fxb[b], X.vx[b], Fyb[b] * X.vy[b]);
        L.vx[b] = fmaf(kd, X.vx[b], fmaf(-k, Fxb[b], L.vx[b]));
        L.vy[b] = fmaf(kd, X.vy[b], fmaf(-k, Fyb[b], L.vy[b]));
        const float invw = hw_rsq(fmaf(X.om[b], X.om[b], c.ew2[b]));
        L.om[b] = fmaf(-(c.crw2[b] * (invw * invw * invw)), Tqb[b], L.om[b]);
    }
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
// Forward rollout of one lane (particle i = lane/4, side s = lane%4).  The four
// lanes of a quad must all run it (phase mixture by DPP).
template <int B>
__device__ __forceinline__ void rollout_fwd_lane(const SimConst& c, int N, const float* __restrict__ theta,
                                                 float* __restrict__ cost, float* __restrict__ tape,
                                                 const TapeGeom& g, uint32_t* status, int64_t lane) {
    const int i = (int)(lane >> 2);
    const int s = (int)(lane & 3);
    const int H = c.H, T = c.T;

    State<B> S;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        S.x[b] = c.pose0[b][0];
        S.y[b] = c.pose0[b][1];
        S.ph[b] = c.pose0[b][2];
        S.vx[b] = S.vy[b] = S.om[b] = 0.0f;
    }
    float Px[kMaxPushes + 1], Py[kMaxPushes + 1];
    float Lbound = 0.0f;
    Push p;
    side_frame(s, p);
    int64_t entry = 0;
    for (int k = 0; k < H; ++k) {
        const int tk = phase_start(k, T, H), tk1 = phase_start(k + 1, T, H);
        const float invL = 1.0f / (float)(tk1 - tk);
        Px[k] = S.x[0];
        Py[k] = S.y[0];
        const float z = side_weight(theta, N, i, k, s);
        const float o = theta[(int64_t)(6 * k + 4) * N + i];
        const float D = theta[(int64_t)(6 * k + 5) * N + i];
        Anchor an;
        phase_push(c, S.x[0], S.y[0], S.ph[0], o, D, p, an);
        Lbound += relu(fabsf(o) - c.omax) * relu(fabsf(o) - c.omax) + relu(-D) * relu(-D) +
                  relu(D - c.dmax) * relu(D - c.dmax);
        State<B> X = S;
        for (int t = tk; t < tk1; ++t) {
            if (tape) {
                if (g.ckpt == 0) {
                    store_state(X, tape + (int64_t)t * 6 * B * g.lanes, lane);
                } else if ((t - tk) % g.ckpt == 0) {
                    store_state(X, tape + entry * 6 * B * g.lanes, lane);
                    ++entry;
                }
            }
            step_forward<B>(c, X, p, push_profile((float)(t - tk + 1) * invL));
        }
        if (tape) store_state(X, tape + g.ends_off + (int64_t)k * 6 * B * g.lanes, lane);
        // phase mixture
#pragma unroll
        for (int b = 0; b < B; ++b) {
            S.x[b] = quad_sum(z * X.x[b]);
            S.y[b] = quad_sum(z * X.y[b]);
            S.ph[b] = quad_sum(z * X.ph[b]);
            S.vx[b] = quad_sum(z * X.vx[b]);
            S.vy[b] = quad_sum(z * X.vy[b]);
            S.om[b] = quad_sum(z * X.om[b]);
        }
    }
    Px[H] = S.x[0];
    Py[H] = S.y[0];
    // cost (Appendix E-B)
    const float dxg = fabsf(Px[H] - c.goal[0]) - c.tol, dyg = fabsf(Py[H] - c.goal[1]) - c.tol;
    const float Ltarget = relu(dxg) * relu(dxg) + relu(dyg) * relu(dyg);
    const float Lrot = 1.0f - cosf(S.ph[0] - c.goal[2]);
    float Ltraj = 0.0f;
    for (int k = 1; k <= H; ++k) {
        Ltraj += smooth_abs(Px[k - 1] - Px[k], c.ea2) + smooth_abs(Py[k - 1] - Py[k], c.ea2);
        Ltraj += smooth_abs(Px[k] - Px[H], c.ea2) + smooth_abs(Py[k] - Py[H], c.ea2);
        Ltraj -= smooth_abs(Px[k - 1] - Px[H], c.ea2) + smooth_abs(Py[k - 1] - Py[H], c.ea2);
    }
    const float C = c.wt * Ltarget + c.wr * Lrot + c.wtr * Ltraj + c.wb * Lbound;
    if (s == 0) {
        cost[i] = C;
        if (status && !isfinite(C)) atomicOr(status, STAMP_STATUS_NONFINITE_COST);
    }
}

// ---------------------------------------------------------------------------
// Reverse sweep of one lane; cost_bar (or cb_scalar when null) scales dC/dtheta.
template <int B>
__device__ __forceinline__ void rollout_adj_lane(const SimConst& c, int N, const float* __restrict__ theta,
                                                 const float* __restrict__ tape, const TapeGeom& g,
                                                 const float* __restrict__ cost_bar, float cb_scalar,
                                                 float* __restrict__ grad, float* __restrict__ seg,
                                                 uint32_t* status, int64_t lane) {
    const int i = (int)(lane >> 2);
    const int s = (int)(lane & 3);
    const int H = c.H, T = c.T;
    const int64_t stride = 6 * B * g.lanes;  // floats per tape entry

    // entry index of each phase start
    int ent[kMaxPushes];
    {
        int e = 0;
        for (int k = 0; k < H; ++k) {
            const int tk = phase_start(k, T, H), tk1 = phase_start(k + 1, T, H);
            ent[k] = (g.ckpt == 0) ? tk : e;
            if (g.ckpt) e += (tk1 - tk + g.ckpt - 1) / g.ckpt;
        }
    }
    // phase-start positions P_k and the final block-0 pose
    float Px[kMaxPushes + 1], Py[kMaxPushes + 1];
    for (int k = 0; k < H; ++k) {
        Px[k] = tape[ent[k] * stride + lane * 6 * B + 0];
        Py[k] = tape[ent[k] * stride + lane * 6 * B + 1];
    }
    float phT;
    {
        const float z = side_weight(theta, N, i, H - 1, s);
        const float* e = tape + g.ends_off + (int64_t)(H - 1) * stride + lane * 6 * B;
        Px[H] = quad_sum(z * e[0]);
        Py[H] = quad_sum(z * e[1]);
        phT = quad_sum(z * e[2]);
    }
    const float cb = cost_bar ? cost_bar[i] : cb_scalar;

    // dC/dP_k and dC/dphi_T, scaled by cost_bar
    float Pxb[kMaxPushes + 1], Pyb[kMaxPushes + 1];
    for (int k = 0; k <= H; ++k) Pxb[k] = Pyb[k] = 0.0f;
    {
        const float ux = Px[H] - c.goal[0], uy = Py[H] - c.goal[1];
        Pxb[H] += cb * c.wt * 2.0f * relu(fabsf(ux) - c.tol) * copysignf(1.0f, ux);
        Pyb[H] += cb * c.wt * 2.0f * relu(fabsf(uy) - c.tol) * copysignf(1.0f, uy);
    }
    const float phTb = cb * c.wr * sinf(phT - c.goal[2]);
    const float wtr = cb * c.wtr;
    for (int k = 1; k <= H; ++k) {
        float u, d;
        u = Px[k - 1] - Px[k];  d = wtr * u / smooth_abs(u, c.ea2);  Pxb[k - 1] += d; Pxb[k] -= d;
        u = Py[k - 1] - Py[k];  d = wtr * u / smooth_abs(u, c.ea2);  Pyb[k - 1] += d; Pyb[k] -= d;
        u = Px[k] - Px[H];      d = wtr * u / smooth_abs(u, c.ea2);  Pxb[k] += d;     Pxb[H] -= d;
        u = Py[k] - Py[H];      d = wtr * u / smooth_abs(u, c.ea2);  Pyb[k] += d;     Pyb[H] -= d;
        u = Px[k - 1] - Px[H];  d = wtr * u / smooth_abs(u, c.ea2);  Pxb[k - 1] -= d; Pxb[H] += d;
        u = Py[k - 1] - Py[H];  d = wtr * u / smooth_abs(u, c.ea2);  Pyb[k - 1] -= d; Pyb[H] += d;
    }

    // adjoint of S_H
    State<B> Ls;
#pragma unroll
    for (int b = 0; b < B; ++b) Ls.x[b] = Ls.y[b] = Ls.ph[b] = Ls.vx[b] = Ls.vy[b] = Ls.om[b] = 0.0f;
    Ls.x[0] = Pxb[H];
    Ls.y[0] = Pyb[H];
    Ls.ph[0] = phTb;

    Push p;
    side_frame(s, p);
    bool bad = false;
    for (int k = H - 1; k >= 0; --k) {
        const int tk = phase_start(k, T, H), tk1 = phase_start(k + 1, T, H);
        const float invL = 1.0f / (float)(tk1 - tk);
        const float z = side_weight(theta, N, i, k, s);
        const float o = theta[(int64_t)(6 * k + 4) * N + i];
        const float D = theta[(int64_t)(6 * k + 5) * N + i];
        // phase end: S_{k+1} = sum_s z_s X_s
        State<B> Xe, L;
        load_state(Xe, tape + g.ends_off + (int64_t)k * stride, lane);
        float zb = 0.0f;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            zb += Ls.x[b] * Xe.x[b] + Ls.y[b] * Xe.y[b] + Ls.ph[b] * Xe.ph[b] + Ls.vx[b] * Xe.vx[b] +
                  Ls.vy[b] * Xe.vy[b] + Ls.om[b] * Xe.om[b];
            L.x[b] = z * Ls.x[b];
            L.y[b] = z * Ls.y[b];
            L.ph[b] = z * Ls.ph[b];
            L.vx[b] = z * Ls.vx[b];
            L.vy[b] = z * Ls.vy[b];
            L.om[b] = z * Ls.om[b];
        }
        const float ab = z * (zb - quad_sum(z * zb));  // softmax VJP
        // anchor of the phase
        const float* ea = tape + ent[k] * stride + lane * 6 * B;
        Anchor an;
        phase_push(c, ea[0], ea[1], ea[2], o, D, p, an);
        float P0xb = 0.0f, P0yb = 0.0f, Vxb = 0.0f, Vyb = 0.0f;
        if (g.ckpt == 0) {
            // reverse sweep over the full tape; the next (earlier) state is
            // fetched while the current step is reversed
            State<B> Xn;
            load_state(Xn, tape + (int64_t)(tk1 - 1) * stride, lane);
            for (int t = tk1 - 1; t >= tk; --t) {
                const State<B> X = Xn;
                if (t > tk) load_state(Xn, tape + (int64_t)(t - 1) * stride, lane);
                step_reverse<B>(c, X, L, p, push_profile((float)(t - tk + 1) * invL), P0xb, P0yb, Vxb, Vyb);
            }
        } else {
            const int nseg = (tk1 - tk + g.ckpt - 1) / g.ckpt;
            for (int j = nseg - 1; j >= 0; --j) {
                const int ts = tk + j * g.ckpt;
                const int te = min(ts + g.ckpt, tk1);
                State<B> X;
                load_state(X, tape + (int64_t)(ent[k] + j) * stride, lane);
                for (int t = ts; t < te; ++t) {  // replay the segment
                    store_state(X, seg + (int64_t)(t - ts) * stride, lane);
                    step_forward<B>(c, X, p, push_profile((float)(t - tk + 1) * invL));
                }
                for (int t = te - 1; t >= ts; --t) {
                    load_state(X, seg + (int64_t)(t - ts) * stride, lane);
                    step_reverse<B>(c, X, L, p, push_profile((float)(t - tk + 1) * invL), P0xb, P0yb, Vxb,
                                    Vyb);
                }
            }
        }
        // back to the anchor and (o, D): P0 = A + R(A) q0, q0 = (h0 + standoff) n + o t,
        // V = -D e_A, e_A = R(A) n
        const float eAx = fmaf(an.cA, p.nx, -(an.sA * p.ny)), eAy = fmaf(an.sA, p.nx, an.cA * p.ny);
        const float Db = -fmaf(Vxb, eAx, Vyb * eAy);
        const float eAxb = -D * Vxb, eAyb = -D * Vyb;
        const float cAb = fmaf(eAxb, p.nx, eAyb * p.ny) + fmaf(P0xb, an.q0x, P0yb * an.q0y);
        const float sAb = fmaf(eAyb, p.nx, -(eAxb * p.ny)) + fmaf(P0yb, an.q0x, -(P0xb * an.q0y));
        const float q0xb = fmaf(an.cA, P0xb, an.sA * P0yb), q0yb = fmaf(an.cA, P0yb, -(an.sA * P0xb));
        const float ob = fmaf(q0xb, p.tx, q0yb * p.ty);
        const float Axb = P0xb, Ayb = P0yb;
        const float Aphb = fmaf(an.cA, sAb, -(an.sA * cAb));
        // adjoint of S_k: the four sub-rollouts share it
#pragma unroll
        for (int b = 0; b < B; ++b) {
            Ls.x[b] = quad_sum(L.x[b]);
            Ls.y[b] = quad_sum(L.y[b]);
            Ls.ph[b] = quad_sum(L.ph[b]);
            Ls.vx[b] = quad_sum(L.vx[b]);
            Ls.vy[b] = quad_sum(L.vy[b]);
            Ls.om[b] = quad_sum(L.om[b]);
        }
        Ls.x[0] += quad_sum(Axb) + Pxb[k];
        Ls.y[0] += quad_sum(Ayb) + Pyb[k];
        Ls.ph[0] += quad_sum(Aphb);
        // bound loss on o_k, D_k
        const float wb2 = 2.0f * cb * c.wb;
        const float obt = quad_sum(ob) + wb2 * relu(fabsf(o) - c.omax) * copysignf(1.0f, o);
        const float Dbt = quad_sum(Db) + wb2 * (relu(D - c.dmax) - relu(-D));
        grad[(int64_t)(6 * k + s) * N + i] = ab;
        if (s == 0) grad[(int64_t)(6 * k + 4) * N + i] = obt;
        if (s == 1) grad[(int64_t)(6 * k + 5) * N + i] = Dbt;
        bad = bad || !isfinite(ab) || !isfinite(obt) || !isfinite(Dbt);
    }
    if (status && bad) atomicOr(status, STAMP_STATUS_NONFINITE_GRAD);
}

// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kRolloutBlock) void k_rollout_fwd(SimConst c, int N, const float* __restrict__ theta,
                                                               float* __restrict__ cost, float* __restrict__ tape,
                                                               TapeGeom g, uint32_t* status) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((lane >> 2) >= N) return;  // whole quads leave together
    rollout_fwd_lane<B>(c, N, theta, cost, tape, g, status, lane);
}

template <int B>
__global__ __launch_bounds__(kRolloutBlock) void k_rollout_adj(SimConst c, int N, const float* __restrict__ theta,
                                                               const float* __restrict__ tape, TapeGeom g,
                                                               const float* __restrict__ cost_bar, float cb_scalar,
                                                               float* __restrict__ grad, float* __restrict__ seg,
                                                               uint32_t* status) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((lane >> 2) >= N) return;
    rollout_adj_lane<B>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, lane);
}

// ---------------------------------------------------------------------------
// Batched rollouts: one launch over the wave tiles of many problems.  Tile t is
// (problem p, first particle i0) and covers particles i0..i0+15 (64 lanes); each
// wave takes tiles in a grid-stride loop.  The block count B of the problem
// selects the compiled body at run time.
__global__ __launch_bounds__(256) void k_rollout_fwd_batched(const ProblemDesc* __restrict__ descs,
                                                             const int2* __restrict__ tiles, int ntiles,
                                                             const float* __restrict__ theta, float* __restrict__ cost,
                                                             float* __restrict__ tape, uint32_t* status) {
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int t = blockIdx.x * waves + wave; t < ntiles; t += gridDim.x * waves) {
        const int2 tl = tiles[t];
        const ProblemDesc& D = descs[tl.x];
        const int64_t lane = 4 * (int64_t)tl.y + l;
        if ((lane >> 2) >= D.N) continue;
        const float* th = theta + D.theta_off;
        float* co = cost + D.cost_off;
        float* tp = tape ? tape + D.tape_off : nullptr;
        switch (D.c.B) {
            case 1: rollout_fwd_lane<1>(D.c, D.N, th, co, tp, D.g, status, lane); break;
            case 2: rollout_fwd_lane<2>(D.c, D.N, th, co, tp, D.g, status, lane); break;
            case 3: rollout_fwd_lane<3>(D.c, D.N, th, co, tp, D.g, status, lane); break;
            default: rollout_fwd_lane<4>(D.c, D.N, th, co, tp, D.g, status, lane); break;
        }
    }
}

__global__ __launch_bounds__(256) void k_rollout_adj_batched(const ProblemDesc* __restrict__ descs,
                                                             const int2* __restrict__ tiles, int ntiles,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ tape, float cb_scalar,
                                                             float* __restrict__ grad, float* __restrict__ seg,
                                                             uint32_t* status) {
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int t = blockIdx.x * waves + wave; t < ntiles; t += gridDim.x * waves) {
        const int2 tl = tiles[t];
        const ProblemDesc& D = descs[tl.x];
        const int64_t lane = 4 * (int64_t)tl.y + l;
        if ((lane >> 2) >= D.N) continue;
        const float* th = theta + D.theta_off;
        const float* tp = tape + D.tape_off;
        float* gr = grad + D.theta_off;
        float* sg = seg + D.seg_off;
        switch (D.c.B) {
            case 1: rollout_adj_lane<1>(D.c, D.N, th, tp, D.g, nullptr, cb_scalar, gr, sg, status, lane); break;
            case 2: rollout_adj_lane<2>(D.c, D.N, th, tp, D.g, nullptr, cb_scalar, gr, sg, status, lane); break;
            case 3: rollout_adj_lane<3>(D.c, D.N, th, tp, D.g, nullptr, cb_scalar, gr, sg, status, lane); break;
            default: rollout_adj_lane<4>(D.c, D.N, th, tp, D.g, nullptr, cb_scalar, gr, sg, status, lane); break;
        }
    }
}

hipError_t launch_rollout_fwd_batched(const ProblemDesc* descs, const int2* tiles, int ntiles, int block,
                                      int grid, const float* theta, float* cost, float* tape, uint32_t* status,
                                      hipStream_t st) {
    hipLaunchKernelGGL(k_rollout_fwd_batched, dim3(grid), dim3(block), 0, st, descs, tiles, ntiles, theta, cost,
                       tape, status);
    return hipGetLastError();
}

hipError_t launch_rollout_adj_batched(const ProblemDesc* descs, const int2* tiles, int ntiles, int block,
                                      int grid, const float* theta, const float* tape, float cb_scalar,
                                      float* grad, float* seg, uint32_t* status, hipStream_t st) {
    hipLaunchKernelGGL(k_rollout_adj_batched, dim3(grid), dim3(block), 0, st, descs, tiles, ntiles, theta, tape,
                       cb_scalar, grad, seg, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int B>
static hipError_t launch_fwd_b(const SimConst& c, int N, const float* theta, float* cost, float* tape,
                               const TapeGeom& g, uint32_t* status, hipStream_t st) {
    const int64_t lanes = 4 * (int64_t)N;
    const unsigned grid = (unsigned)((lanes + kRolloutBlock - 1) / kRolloutBlock);
    hipLaunchKernelGGL(k_rollout_fwd<B>, dim3(grid), dim3(kRolloutBlock), 0, st, c, N, theta, cost, tape, g,
                       status);
    return hipGetLastError();
}

template <int B>
static hipError_t launch_adj_b(const SimConst& c, int N, const float* theta, const float* tape,
                               const TapeGeom& g, const float* cost_bar, float cb_scalar, float* grad,
                               float* seg, uint32_t* status, hipStream_t st) {
    const int64_t lanes = 4 * (int64_t)N;
    const unsigned grid = (unsigned)((lanes + kRolloutBlock - 1) / kRolloutBlock);
    hipLaunchKernelGGL(k_rollout_adj<B>, dim3(grid), dim3(kRolloutBlock), 0, st, c, N, theta, tape, g, cost_bar,
                       cb_scalar, grad, seg, status);
    return hipGetLastError();
}

hipError_t launch_rollout_fwd(const SimConst& c, int N, const float* theta, float* cost, float* tape,
                              const TapeGeom& g, uint32_t* status, hipStream_t st) {
    switch (c.B) {
        case 1: return launch_fwd_b<1>(c, N, theta, cost, tape, g, status, st);
        case 2: return launch_fwd_b<2>(c, N, theta, cost, tape, g, status, st);
        case 3: return launch_fwd_b<3>(c, N, theta, cost, tape, g, status, st);
        case 4: return launch_fwd_b<4>(c, N, theta, cost, tape, g, status, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rollout_adj(const SimConst& c, int N, const float* theta, const float* tape,
                              const TapeGeom& g, const float* cost_bar, float cb_scalar, float* grad,
                              float* seg, uint32_t* status, hipStream_t st) {
    switch (c.B) {
        case 1: return launch_adj_b<1>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st);
        case 2: return launch_adj_b<2>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st);
        case 3: return launch_adj_b<3>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st);
        case 4: return launch_adj_b<4>(c, N, theta, tape, g, cost_bar, cb_scalar, grad, seg, status, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stamp
