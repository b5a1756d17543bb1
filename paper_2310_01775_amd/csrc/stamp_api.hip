// C ABI of libstamp.so: argument checks, derived constants, workspace carving
// and kernel launches.  See include/stamp.h for the contract of every call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"
#include "stamp.h"

struct stamp_ctx {
    int device = 0;
    int clock_khz = 100000;  // wall-clock counter rate of the device
    std::string err;
};

namespace stamp {
namespace {

int fail(stamp_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(stamp_ctx* ctx, int code, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int hip_fail(stamp_ctx* ctx, hipError_t e, const char* where) {
    return fail(ctx, STAMP_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

// Validate a scene + weights and derive the kernels' constants.
int derive(stamp_ctx* ctx, const stamp_scene* s, const stamp_cost_w* w, SimConst* c) {
    if (!s || !w) return fail(ctx, STAMP_EINVAL, "null scene or cost weights");
    if (s->H < 1 || s->H > kMaxPushes) return fail(ctx, STAMP_EINVAL, "H=%d not in [1,%d]", s->H, kMaxPushes);
    if (s->M != kModes) return fail(ctx, STAMP_EINVAL, "M=%d, only 4 push sides are modelled", s->M);
    if (s->B < 1 || s->B > kMaxBlocks) return fail(ctx, STAMP_EINVAL, "B=%d not in [1,%d]", s->B, kMaxBlocks);
    if (s->T < s->H) return fail(ctx, STAMP_EINVAL, "T=%d < H=%d", s->T, s->H);
    if (!finite_pos(s->dt)) return fail(ctx, STAMP_EINVAL, "dt must be finite and > 0");
    if (!finite_pos(s->sp_beta)) return fail(ctx, STAMP_EINVAL, "sp_beta must be > 0");
    if (!(isfinite(s->k_push) && s->k_push >= 0 && isfinite(s->k_block) && s->k_block >= 0))
        return fail(ctx, STAMP_EINVAL, "stiffness must be finite and >= 0");
    if (!(isfinite(s->g) && s->g >= 0 && isfinite(s->eps_v_scale) && s->eps_v_scale >= 0 &&
          isfinite(s->eps_r) && isfinite(s->standoff) && isfinite(s->goal_tol)))
        return fail(ctx, STAMP_EINVAL, "non-finite model constant");
    for (int b = 0; b < s->B; ++b) {
        if (!finite_pos(s->half[b]) || !finite_pos(s->mass[b]) || !(isfinite(s->mu[b]) && s->mu[b] >= 0))
            return fail(ctx, STAMP_EINVAL, "block %d: half and mass must be > 0, mu >= 0", b);
        for (int q = 0; q < 3; ++q)
            if (!isfinite(s->pose0[b][q])) return fail(ctx, STAMP_EINVAL, "block %d: non-finite pose", b);
    }
    const float wv[7] = {w->target, w->rot, w->traj, w->bound, w->o_max, w->d_max, w->traj_eps};
    for (float v : wv)
        if (!isfinite(v)) return fail(ctx, STAMP_EINVAL, "non-finite cost weight");
    memset(c, 0, sizeof *c);
    c->H = s->H;
    c->B = s->B;
    c->T = s->T;
    c->dt = s->dt;
    const double rho_sq = (sqrt(2.0) + log(1.0 + sqrt(2.0))) / 6.0;  // mean |r| of a unit square
    for (int b = 0; b < s->B; ++b) {
        const double h = s->half[b], m = s->mass[b], mu = s->mu[b], g = s->g;
        const double I = m * (2.0 * h) * (2.0 * h) / 6.0;
        const double rho = 2.0 * h * rho_sq;
        const double ev = std::max((double)s->eps_v_scale * (double)s->dt * mu * g, 1e-6);
        const double ew = ev * m * rho / I;
        c->inv_m[b] = (float)(1.0 / m);
        c->inv_I[b] = (float)(1.0 / I);
        c->cf[b] = (float)(mu * m * g);
        c->cr[b] = (float)(mu * m * g * rho);
        c->ev2[b] = (float)(ev * ev);
        c->ew2[b] = (float)(ew * ew);
        for (int q = 0; q < 3; ++q) c->pose0[b][q] = s->pose0[b][q];
        for (int q = 0; q < s->B; ++q) c->hsum[b][q] = (float)((double)s->half[b] + (double)s->half[q]);
    }
    c->h0 = s->half[0];
    c->h0d = (float)((double)s->half[0] + (double)s->standoff);
    c->kp = s->k_push;
    c->kb = s->k_block;
    c->beta = s->sp_beta;
    c->inv_beta = (float)(1.0 / (double)s->sp_beta);
    c->er2 = (float)((double)s->eps_r * (double)s->eps_r);
    c->beta_log2e = (float)((double)s->sp_beta / log(2.0));
    c->ln2_over_beta = (float)(log(2.0) / (double)s->sp_beta);
    for (int q = 0; q < 3; ++q) c->goal[q] = s->goal[q];
    c->tol = s->goal_tol;
    c->wt = w->target;
    c->wr = w->rot;
    c->wtr = w->traj;
    c->wb = w->bound;
    c->omax = w->o_max;
    c->dmax = w->d_max;
    c->ea2 = (float)((double)w->traj_eps * (double)w->traj_eps);
    return STAMP_OK;
}

TapeGeom tape_geom(const stamp_scene* s, int N, int K) {
    TapeGeom g{};
    g.lanes = 4 * (int64_t)N;
    g.ckpt = K;
    if (K == 0) {
        g.n_entries = s->T;
    } else {
        int64_t e = 0;
        for (int k = 0; k < s->H; ++k) {
            const int L = phase_start(k + 1, s->T, s->H) - phase_start(k, s->T, s->H);
            e += (L + K - 1) / K;
        }
        g.n_entries = e;
    }
    g.ends_off = g.n_entries * 6 * s->B * g.lanes;
    return g;
}

size_t tape_floats(const stamp_scene* s, int N, int K) {
    const TapeGeom g = tape_geom(s, N, K);
    return (size_t)(g.ends_off + (int64_t)s->H * 6 * s->B * g.lanes);
}

size_t adj_ws_bytes(const stamp_scene* s, int N, int K) {
    return K > 0 ? (size_t)K * 6 * s->B * 4 * (size_t)N * sizeof(float) : 0;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool scene_ok(const stamp_scene* s) {
    return s && s->H >= 1 && s->H <= kMaxPushes && s->B >= 1 && s->B <= kMaxBlocks && s->T >= s->H &&
           s->M == kModes;
}

constexpr int kMaxSvgdDim = 64;
constexpr int kMaxSvgdN = 65536;

// Per-problem workspace of the solve: tape, gradient, phi, cost, replay and
// SVGD scratch, step counter.
struct SolveLayout {
    size_t tape_off, grad_off, phi_off, cost_off, seg_off, svgd_off, ctr_off, total;
    SvgdLayout svgd;
};

// The solve workspace starts with the per-problem clock pairs, then one
// problem region (problems run one after another and reuse it).
size_t clock_header_bytes(int n_problems) { return align256((size_t)n_problems * 2 * sizeof(uint64_t)); }

SolveLayout solve_layout(const stamp_scene* s, int N, int K) {
    SolveLayout L{};
    const int d = 6 * s->H;
    size_t off = 0;
    L.tape_off = off;
    off = align256(off + tape_floats(s, N, K) * 4);
    L.grad_off = off;
    off = align256(off + (size_t)d * N * 4);
    L.phi_off = off;
    off = align256(off + (size_t)d * N * 4);
    L.cost_off = off;
    off = align256(off + (size_t)N * 4);
    L.seg_off = off;
    off = align256(off + adj_ws_bytes(s, N, K));
    L.svgd = svgd_workspace_layout(N, d);
    L.svgd_off = off;
    off = align256(off + L.svgd.total);
    L.ctr_off = off;
    off = align256(off + 256);
    L.total = off;
    return L;
}

__global__ void k_stamp_clock(uint64_t* dst) { *dst = wall_clock64(); }

__global__ void k_clock_to_us(const uint64_t* clk, int n, float us_per_tick, float* out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[p] = (float)(clk[2 * p + 1] - clk[2 * p]) * us_per_tick;
}

}  // namespace
}  // namespace stamp

using namespace stamp;

extern "C" {

const char* stamp_version(void) { return "stamp-mi355x 0.1 (gfx950)"; }

int32_t stamp_create(stamp_ctx** ctx, int32_t device) {
    if (!ctx) return STAMP_EINVAL;
    *ctx = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return STAMP_EHIP;
    if (device < 0 || device >= n) return STAMP_EINVAL;
    if ((e = hipSetDevice(device)) != hipSuccess) return STAMP_EHIP;
    stamp_ctx* c = new stamp_ctx();
    c->device = device;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->clock_khz = khz;
    *ctx = c;
    return STAMP_OK;
}

void stamp_destroy(stamp_ctx* ctx) { delete ctx; }

const char* stamp_last_error(const stamp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t stamp_tape_floats(const stamp_scene* scene, int32_t N, int32_t ckpt_every) {
    if (!scene_ok(scene) || N < 1 || ckpt_every < 0) return 0;
    return tape_floats(scene, N, ckpt_every);
}

size_t stamp_adj_workspace_bytes(const stamp_scene* scene, int32_t N, int32_t ckpt_every) {
    if (!scene_ok(scene) || N < 1 || ckpt_every < 0) return 0;
    return adj_ws_bytes(scene, N, ckpt_every);
}

size_t stamp_svgd_workspace_bytes(int32_t N, int32_t d) {
    if (N < 1 || d < 1 || d > kMaxSvgdDim || N > kMaxSvgdN) return 0;
    return svgd_workspace_layout(N, d).total;
}

size_t stamp_solve_workspace_bytes(int32_t n_problems, const stamp_scene* scenes, const int32_t* N,
                                   const stamp_solver_cfg* cfg) {
    if (n_problems < 1 || !scenes || !N || !cfg || cfg->ckpt_every < 0) return 0;
    size_t m = 0;
    for (int p = 0; p < n_problems; ++p) {
        if (!scene_ok(&scenes[p]) || N[p] < 1) return 0;
        m = std::max(m, solve_layout(&scenes[p], N[p], cfg->ckpt_every).total);
    }
    return clock_header_bytes(n_problems) + m;
}

int32_t stamp_rollout_fwd(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                          const float* theta, float* cost, float* tape, int32_t ckpt_every, uint32_t* status,
                          void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !cost) return fail(ctx, STAMP_EINVAL, "null theta or cost");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    if (ckpt_every < 0) return fail(ctx, STAMP_EINVAL, "ckpt_every < 0");
    SimConst c;
    int r = derive(ctx, scene, w, &c);
    if (r) return r;
    const TapeGeom g = tape_geom(scene, N, ckpt_every);
    hipError_t e = launch_rollout_fwd(c, N, theta, cost, tape, g, status, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "rollout_fwd");
}

int32_t stamp_rollout_adj(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                          const float* theta, const float* tape, int32_t ckpt_every, const float* cost_bar,
                          float* grad, void* workspace, size_t ws_bytes, uint32_t* status, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !tape || !grad) return fail(ctx, STAMP_EINVAL, "null theta, tape or grad");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    if (ckpt_every < 0) return fail(ctx, STAMP_EINVAL, "ckpt_every < 0");
    SimConst c;
    int r = derive(ctx, scene, w, &c);
    if (r) return r;
    const size_t need = adj_ws_bytes(scene, N, ckpt_every);
    if (need && (!workspace || ws_bytes < need))
        return fail(ctx, STAMP_ENOSPACE, "adjoint workspace %zu < %zu bytes", ws_bytes, need);
    const TapeGeom g = tape_geom(scene, N, ckpt_every);
    hipError_t e = launch_rollout_adj(c, N, theta, tape, g, cost_bar, 1.0f, grad, (float*)workspace, status,
                                      (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "rollout_adj");
}

int32_t stamp_svgd_step(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, const float* grad_logp,
                        float bandwidth, float* phi, float* h_out, void* workspace, size_t ws_bytes,
                        void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !grad_logp || !phi) return fail(ctx, STAMP_EINVAL, "null theta, grad_logp or phi");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    if (d > kMaxSvgdDim || N > kMaxSvgdN)
        return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports d <= %d, N <= %d", kMaxSvgdDim, kMaxSvgdN);
    if (!isfinite(bandwidth)) return fail(ctx, STAMP_EINVAL, "non-finite bandwidth");
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "svgd workspace %zu < %zu bytes", ws_bytes, L.total);
    hipError_t e = launch_svgd(N, d, theta, grad_logp, bandwidth, phi, h_out, workspace, L, nullptr,
                               (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_step");
}

int32_t stamp_adam_step(stamp_ctx* ctx, int64_t n, float* theta, const float* phi, float* m, float* v, int32_t t,
                        float lr, float beta1, float beta2, float eps, int32_t use_adam, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !phi || (use_adam && (!m || !v))) return fail(ctx, STAMP_EINVAL, "null pointer");
    if (n < 1) return fail(ctx, STAMP_EINVAL, "n < 1");
    if (use_adam && t < 1) return fail(ctx, STAMP_EINVAL, "Adam step t=%d < 1", t);
    if (!isfinite(lr) || (use_adam && !(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps >= 0)))
        return fail(ctx, STAMP_EINVAL, "bad Adam hyper-parameters");
    hipError_t e = launch_update(n, theta, phi, m, v, t, nullptr, lr, beta1, beta2, eps, use_adam,
                                 (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "adam_step");
}

int32_t stamp_solve(stamp_ctx* ctx, int32_t n_problems, const stamp_scene* scenes, const stamp_cost_w* w,
                    const int32_t* N, const stamp_solver_cfg* cfg, float* theta, float* adam_m, float* adam_v,
                    float* cost_out, int32_t* modes_out, float* solve_time_us, void* workspace,
                    size_t ws_bytes, uint32_t* status, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (n_problems < 1 || !scenes || !w || !N || !cfg) return fail(ctx, STAMP_EINVAL, "null problem arrays");
    if (!theta || !cost_out) return fail(ctx, STAMP_EINVAL, "null theta or cost_out");
    if (cfg->iters < 0 || cfg->ckpt_every < 0 || cfg->t0 < 0) return fail(ctx, STAMP_EINVAL, "bad solver cfg");
    if (cfg->use_adam && (!adam_m || !adam_v)) return fail(ctx, STAMP_EINVAL, "Adam needs m and v");
    if (!isfinite(cfg->lr) || !isfinite(cfg->bandwidth)) return fail(ctx, STAMP_EINVAL, "non-finite lr/bandwidth");
    if (cfg->use_adam && !(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1 &&
                           cfg->adam_eps >= 0))
        return fail(ctx, STAMP_EINVAL, "bad Adam hyper-parameters");
    std::vector<SimConst> consts(n_problems);
    size_t need = 0;
    for (int p = 0; p < n_problems; ++p) {
        int r = derive(ctx, &scenes[p], &w[p], &consts[p]);
        if (r) return r;
        if (N[p] < 1) return fail(ctx, STAMP_EINVAL, "problem %d: N=%d < 1", p, N[p]);
        if (6 * scenes[p].H > kMaxSvgdDim || N[p] > kMaxSvgdN)
            return fail(ctx, STAMP_EUNSUPPORTED, "problem %d too large for the svgd step", p);
        need = std::max(need, solve_layout(&scenes[p], N[p], cfg->ckpt_every).total);
    }
    need += clock_header_bytes(n_problems);
    if (!workspace || ws_bytes < need) return fail(ctx, STAMP_ENOSPACE, "solve workspace %zu < %zu", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    uint64_t* clk = (uint64_t*)workspace;
    char* base = (char*)workspace + clock_header_bytes(n_problems);
    hipError_t e = hipSuccess;
    int64_t th_off = 0, n_off = 0, m_off = 0;
    for (int p = 0; p < n_problems && e == hipSuccess; ++p) {
        const stamp_scene* s = &scenes[p];
        const SimConst& c = consts[p];
        const int n = N[p], d = 6 * s->H, K = cfg->ckpt_every;
        const SolveLayout L = solve_layout(s, n, K);
        float* tape = (float*)(base + L.tape_off);
        float* grad = (float*)(base + L.grad_off);
        float* phi = (float*)(base + L.phi_off);
        float* cost = (float*)(base + L.cost_off);
        float* seg = (float*)(base + L.seg_off);
        void* sws = base + L.svgd_off;
        int* ctr = (int*)(base + L.ctr_off);
        float* th = theta + th_off;
        float* mm = adam_m ? adam_m + th_off : nullptr;
        float* vv = adam_v ? adam_v + th_off : nullptr;
        const TapeGeom g = tape_geom(s, n, K);
        if (solve_time_us) hipLaunchKernelGGL(k_stamp_clock, dim3(1), dim3(1), 0, st, clk + 2 * p);
        for (int it = 0; it < cfg->iters && e == hipSuccess; ++it) {
            if ((e = launch_rollout_fwd(c, n, th, cost, tape, g, status, st)) != hipSuccess) break;
            // grad = -dC/dtheta = grad log rho
            if ((e = launch_rollout_adj(c, n, th, tape, g, nullptr, -1.0f, grad, seg, status, st)) != hipSuccess)
                break;
            if ((e = launch_svgd(n, d, th, grad, cfg->bandwidth, phi, nullptr, sws, L.svgd, status, st)) !=
                hipSuccess)
                break;
            e = launch_update((int64_t)d * n, th, phi, mm, vv, cfg->t0 + it + 1, nullptr, cfg->lr, cfg->beta1,
                              cfg->beta2, cfg->adam_eps, cfg->use_adam, st);
        }
        if (e == hipSuccess) e = launch_rollout_fwd(c, n, th, cost_out + n_off, nullptr, g, status, st);
        if (e == hipSuccess && modes_out) e = launch_modes(n, s->H, th, modes_out + m_off, st);
        if (e == hipSuccess && solve_time_us) hipLaunchKernelGGL(k_stamp_clock, dim3(1), dim3(1), 0, st, clk + 2 * p + 1);
        (void)ctr;
        th_off += (int64_t)d * n;
        n_off += n;
        m_off += (int64_t)s->H * n;
    }
    if (e == hipSuccess && solve_time_us) {
        hipLaunchKernelGGL(k_clock_to_us, dim3((n_problems + 63) / 64), dim3(64), 0, st, clk, n_problems,
                           1000.0f / (float)ctx->clock_khz, solve_time_us);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "solve");
    return STAMP_OK;
}

}  // extern "C"
