// C ABI of libstamp.so: argument checks, derived constants, workspace carving
// and kernel launches.  See include/stamp.h for the contract of every call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"
#include "stamp.h"

// Launch shapes picked by the autotuner for one batch signature.
struct StampTune {
    int roll_block = 64;  // threads per rollout workgroup (64, 128, 256)
    int roll_grid = 0;    // rollout workgroups (0: one wave per tile)
    int phi_rows = 256;   // rows per contraction workgroup
};

struct stamp_ctx {
    int device = 0;
    int clock_khz = 100000;  // wall-clock counter rate of the device
    int num_cus = 256;
    std::string err;
    hipStream_t stream = nullptr;  // library stream: solves are captured and replayed here
    hipStream_t side = nullptr;    // the bandwidth stage runs here, beside the rollout
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join = nullptr;
    std::map<std::string, StampTune> tune;  // autotune cache, keyed by batch signature
    int autotune = 1;
    int rollout_layout = STAMP_LAYOUT_AUTO;  // block per lane, or all blocks of a sub-rollout per lane
    StampTune pinned;                        // used when pinned.roll_block > 0
    int is_pinned = 0;
    // Instantiated graphs of an iteration kind (SVGD, surrogate phase, SGD
    // refinement) for one solve: one iteration, and kGraphUnroll iterations in
    // one graph (consecutive launches of a graph leave a gap of several
    // microseconds on the queue; inside one graph the iterations follow each
    // other directly).  Kept per kind and batch, so that the classes of a
    // class-scheduled solve each keep theirs.
    struct IterGraphs {
        hipGraphExec_t one = nullptr, many = nullptr;
        std::string key_one, key_many;
        void destroy() {
            if (one) (void)hipGraphExecDestroy(one);
            if (many) (void)hipGraphExecDestroy(many);
            one = many = nullptr;
        }
    };
    std::map<std::string, IterGraphs> graphs;
    static constexpr size_t kMaxGraphSlots = 48;
    // the slot of `kind` for the batch `key`; the cache is emptied (after the
    // library stream has drained) when it would outgrow kMaxGraphSlots
    IterGraphs& graph_slot(const std::string& kind, const std::string& key) {
        const std::string k = kind + "#" + key;
        auto it = graphs.find(k);
        if (it != graphs.end()) return it->second;
        if (graphs.size() >= kMaxGraphSlots) destroy_graphs();
        return graphs[k];
    }
    void destroy_graphs() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto& g : graphs) g.second.destroy();
        graphs.clear();
    }
    void* scratch = nullptr;  // this device's copy of the no-alloc scratch array (device address)
};

// Scratch memory of stamp_svgd_step_noalloc: a file-scope device array that
// each GPU holds from the library's load until the process ends.  Host code
// never uses the array's name (a host-side stand-in, not a device address):
// stamp_create looks up each device's address with hipGetSymbolAddress, with
// that device current, and every launch takes that pointer.
static __device__ __align__(256) unsigned char scratch[STAMP_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up once).
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}
}  // namespace

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
        c->dtm[b] = (float)((double)s->dt / m);
        c->dtI[b] = (float)((double)s->dt / I);
        c->crw2[b] = (float)(mu * m * g * rho * ew * ew);
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

// Lanes of the block-per-lane rollout layout (4 sides x SL block slots per particle).
int64_t block_lanes(int N, int B) { return (int64_t)4 * (B == 1 ? 1 : (B == 2 ? 2 : 4)) * N; }

// Automatic layout.  The block-per-lane form keeps more waves in flight,
// which pays while a rollout is latency-bound (few waves per SIMD: at N = 1024
// or 4096 particles of 3 blocks it is 1.3-1.6x faster).  Once its lanes fill
// the chip (kPackedAutoLanes), one lane per sub-rollout issues about half the
// instructions per particle and wins: N = 16384, B = 3, forward 177 vs 236 us,
// adjoint 178 vs 336 us; the 64-problem batch 1.88 vs 2.12 ms per iteration.
// The tape layout is the same, and so are the results, bit for bit.  (The
// forward and the adjoint take the rule separately, so either may be chosen
// on its own.)
constexpr int64_t kPackedAutoLanes = (int64_t)2 * 64 * 1024;
bool packed_for(const stamp_ctx* ctx, int64_t lanes, bool adjoint) {
    (void)adjoint;
    if (ctx->rollout_layout == STAMP_LAYOUT_BLOCKS) return false;
    if (ctx->rollout_layout == STAMP_LAYOUT_PACKED) return true;
    return lanes >= kPackedAutoLanes;
}

constexpr int kGraphUnroll = 4;  // iterations per unrolled graph
constexpr int kMaxSvgdDim = 64;
constexpr int kMaxSvgdN = 65536;

// Workspace of a solve over n problems, all resident at once:
//   clock pairs | descriptors | work lists | step counter |
//   tapes | segment buffers | grad | phi | cost scratch | per-problem SVGD regions
struct SolvePlan {
    std::vector<stamp::ProblemDesc> descs;
    std::vector<int2> roll_tiles, adj_tiles;  // forward and adjoint rollout tiles (their layouts may differ)
    std::vector<int4> dist_work, cand_work, fin_work, red_work;
    std::vector<int4> phi_work[kPhi32Classes];
    std::vector<int4> ctr_work, row16_work, phi16_work[2];  // BF16 form
    int phi_rows = 256;
    int dist_start[kMedLists] = {}, dist_n[kMedLists] = {};  // dist_work sorted by item shape
    size_t clk_off = 0, desc_off = 0, roll_off = 0, adj_tiles_off = 0, dist_off = 0, cand_off = 0, fin_off = 0,
           red_off = 0;
    size_t ctr16_off = 0, row16_off = 0, phi16_off[2] = {};
    size_t phi_off[kPhi32Classes] = {};
    size_t ctr_off = 0, err_off = 0, tape_off = 0, seg_off = 0, grad_off = 0, phi_vec_off = 0, cost_off = 0,
           cdisc_off = 0, wts_off = 0, svgd_off = 0;
    size_t total = 0;
    int64_t n_theta = 0, n_part = 0;
    std::string key;  // batch signature (sizes only)
};

constexpr int kRedChunk = 256;    // elements per workgroup of the phi reduction

// Lay out the workspace and build the work lists.  phi_rows fixes the row
// blocks of the contraction work list.
void build_plan(int n, const stamp_scene* scenes, const int32_t* N, int K, float bandwidth, int phi_rows,
                const std::vector<stamp::SimConst>* consts, SolvePlan& P, bool packed_fwd = false,
                bool packed_adj = false) {
    P = SolvePlan{};  // rebuilt from scratch: appending twice would repeat work items
    P.phi_rows = phi_rows;
    P.descs.resize(n);
    int64_t th = 0, co = 0, tp = 0, sg = 0;
    size_t sv = 0;
    char buf[64];
    P.key.clear();
    std::vector<int4> dist_lists[kMedLists];
    for (int p = 0; p < n; ++p) {
        ProblemDesc& D = P.descs[p];
        memset(&D, 0, sizeof D);
        if (consts) D.c = (*consts)[p];
        const stamp_scene* s = &scenes[p];
        D.N = N[p];
        D.d = 6 * s->H;
        D.g = tape_geom(s, N[p], K);
        D.sv = svgd_workspace_layout(N[p], D.d);
        D.fixed_h = bandwidth > 0.0f ? bandwidth : 0.0f;
        D.theta_off = th;
        D.cost_off = co;
        D.tape_off = tp;
        D.seg_off = sg;
        D.svgd_off = (int64_t)sv;
        th += (int64_t)D.d * D.N;
        co += D.N;
        tp += (int64_t)((tape_floats(s, N[p], K) + 63) & ~size_t(63));
        sg += (int64_t)((adj_ws_bytes(s, N[p], K) / 4 + 63) & ~size_t(63));
        sv += align256(D.sv.total);
        snprintf(buf, sizeof buf, "%d/%d/%d/%d;", N[p], s->H, s->B, s->T);
        P.key += buf;
        for (int i0 = 0; i0 < D.N; i0 += rollout_tile_particles(s->B, packed_fwd))
            P.roll_tiles.push_back(make_int2(p, i0));
        for (int i0 = 0; i0 < D.N; i0 += rollout_tile_particles(s->B, packed_adj))
            P.adj_tiles.push_back(make_int2(p, i0));
        // median passes over all pairs, for problems whose pairs exceed the sample:
        // every (row block, column chunk) item (items without a pair i < j write
        // zero counts), and (segment, part) of the candidate passes
        if (D.N >= 2 && !(bandwidth > 0.0f) && (uint64_t)D.N * (uint64_t)(D.N - 1) / 2 > (uint64_t)kMedSample) {
            // problems above 2^20 pairs take the Gram form (median.hip)
            const bool gram = (uint64_t)D.N * (uint64_t)(D.N - 1) / 2 > (1ull << 20);
            const int c = gram ? med_gram_list(D.sv.split3 ? 0 : D.sv.ks32, D.sv.med_rows)
                               : med_class(med_dp(D.d), D.sv.med_rows);
            for (int rb = 0; rb < D.sv.med_rb; ++rb)
                for (int cc = 0; cc < D.sv.med_cc; ++cc) dist_lists[c].push_back(make_int4(p, rb, cc, 0));
            if (gram) {
                for (int g = 0; g < kCandSegs; ++g)
                    for (int q = 0; q < kCandParts; ++q) P.cand_work.push_back(make_int4(p, g, q, 0));
            } else {
                P.fin_work.push_back(make_int4(p, 0, 0, 0));
            }
        }
        if (D.N >= 2) {
            const int c = phi32_class(D.d);
            const int rows = D.sv.split3 ? 64 : phi_rows;  // the split form's workgroups take 64 rows
            for (int rb = 0; rb * rows < D.sv.npad; ++rb)
                for (int q = 0; q < D.sv.splits32; ++q) P.phi_work[c].push_back(make_int4(p, rb, q, 0));
        }
        // BF16 form: its lists do not depend on the row block of the FP32 form
        for (int r0 = 0; r0 < D.N; r0 += kRows16) P.row16_work.push_back(make_int4(p, r0, 0, 0));
        if (D.N >= 2) {
            for (int l = 0; l < D.d; ++l) P.ctr_work.push_back(make_int4(p, l, 0, 0));
            static_assert(6 * kMaxPushes <= 62, "a solve's problems take the 32- or 64-wide BF16 Gram");
            const int c16 = D.sv.kd == 32 ? 0 : 1;
            for (int rb = 0; rb < D.sv.npad / kTile16; ++rb)
                for (int q = 0; q < D.sv.splits16; ++q) P.phi16_work[c16].push_back(make_int4(p, rb, q, 0));
        }
        const int64_t ne = (int64_t)D.d * D.N;
        for (int64_t e = 0; e < ne; e += kRedChunk)
            P.red_work.push_back(make_int4(p, (int)e, (int)std::min<int64_t>(e + kRedChunk, ne), 0));
    }
    P.n_theta = th;
    for (int c = 0; c < kMedLists; ++c) {
        P.dist_start[c] = (int)P.dist_work.size();
        P.dist_n[c] = (int)dist_lists[c].size();
        P.dist_work.insert(P.dist_work.end(), dist_lists[c].begin(), dist_lists[c].end());
    }
    // The contraction lists get the room of their longest form (64-row
    // blocks), so that no region of the workspace moves when the row block
    // changes: pointers into it stay valid across every launch shape.
    size_t phi_cap[kPhi32Classes] = {};
    for (int p = 0; p < n; ++p) {
        const ProblemDesc& D = P.descs[p];
        if (D.N < 2) continue;
        phi_cap[phi32_class(D.d)] += (size_t)(D.sv.npad / 64) * D.sv.splits32;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    P.clk_off = take((size_t)n * 2 * sizeof(uint64_t));
    P.desc_off = take(P.descs.size() * sizeof(ProblemDesc));
    P.roll_off = take(P.roll_tiles.size() * sizeof(int2));
    P.adj_tiles_off = take(P.adj_tiles.size() * sizeof(int2));
    P.dist_off = take(P.dist_work.size() * sizeof(int4));
    P.cand_off = take(P.cand_work.size() * sizeof(int4));
    P.fin_off = take(P.fin_work.size() * sizeof(int4));
    P.red_off = take(P.red_work.size() * sizeof(int4));
    for (int c = 0; c < kPhi32Classes; ++c) P.phi_off[c] = take(phi_cap[c] * sizeof(int4));
    P.ctr16_off = take(P.ctr_work.size() * sizeof(int4));
    P.row16_off = take(P.row16_work.size() * sizeof(int4));
    for (int c = 0; c < 2; ++c) P.phi16_off[c] = take(P.phi16_work[c].size() * sizeof(int4));
    P.ctr_off = take(256);
    P.err_off = take((size_t)n * sizeof(float));
    P.tape_off = take((size_t)tp * 4);
    P.seg_off = take((size_t)sg * 4);
    P.grad_off = take((size_t)th * 4);
    P.phi_vec_off = take((size_t)th * 4);
    P.cost_off = take((size_t)co * 4);
    P.cdisc_off = take((size_t)co * 4);  // discrete-plan costs (importance weights)
    P.wts_off = take((size_t)co * 4);    // importance weights
    P.svgd_off = take(sv);
    P.total = off;
}

// Workspace of a solve (the same for every phi row choice of the autotuner).
size_t plan_bytes(int n, const stamp_scene* scenes, const int32_t* N, int K, float bandwidth) {
    SolvePlan P;
    build_plan(n, scenes, N, K, bandwidth, 256, nullptr, P);
    return P.total;
}

// ---- class-scheduled solve --------------------------------------------------
// With cfg->classes = C > 1 the problems are ordered by a prediction of their
// device time per iteration and cut into min(C, n) classes of consecutive
// cost and about equal predicted work, each solved as a batch of its own, the
// cheapest first, so a cheap problem is done when its class is instead of
// when the most expensive one is.  The prediction adds the rollout's block steps (4 sides x B blocks x
// (T + H) steps per particle) and the pairwise stages' pairs scaled by the
// dimension; at N = 16384, B = 3, d = 30 one block step costs about 9.4 ps
// and one ordered pair about 2.4 ps, hence the weight 0.26 of a pair at d = 30.
struct ClassPlan {
    std::vector<int> order;                       // problems by predicted cost, ascending
    std::vector<int> first;                       // class c: order[first[c] .. first[c + 1])
    std::vector<int64_t> th_off, co_off, mo_off;  // each problem's place in the packed arrays
    size_t clk_off = 0, th_off_s = 0, m_off_s = 0, v_off_s = 0, cost_off_s = 0, modes_off_s = 0, plan_off = 0;
    size_t plan_bytes = 0, total = 0;
};

bool class_plan(int n, const stamp_scene* scenes, const int32_t* N, const stamp_solver_cfg* cfg, ClassPlan& L) {
    const int C = std::min(cfg->classes, n);
    std::vector<double> cost(n);
    L.th_off.assign(n, 0);
    L.co_off.assign(n, 0);
    L.mo_off.assign(n, 0);
    int64_t th = 0, co = 0, mo = 0;
    for (int p = 0; p < n; ++p) {
        const stamp_scene& sc = scenes[p];
        const double d = 6.0 * sc.H, np = N[p];
        cost[p] = 4.0 * sc.B * (double)(sc.T + sc.H) * np + 0.26 * (d / 30.0) * np * np;
        L.th_off[p] = th;
        L.co_off[p] = co;
        L.mo_off[p] = mo;
        th += (int64_t)6 * sc.H * N[p];
        co += N[p];
        mo += (int64_t)sc.H * N[p];
    }
    L.order.resize(n);
    for (int p = 0; p < n; ++p) L.order[p] = p;
    std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) { return cost[a] < cost[b]; });
    // classes of equal predicted work: class c ends at the first problem whose
    // running sum reaches (c + 1) / C of the total, and holds at least one
    // problem (a class of many cheap problems costs one iteration's launch
    // latency per iteration, as a class of one does)
    double total = 0.0;
    for (int p = 0; p < n; ++p) total += cost[p];
    L.first.assign(1, 0);
    double run = 0.0;
    for (int q = 0; q < n; ++q) {
        run += cost[L.order[q]];
        const int c = (int)L.first.size() - 1;  // the open class
        const int left = n - (q + 1);             // problems after this one
        const int need = C - (c + 1);             // classes still to open after this one
        if ((run >= total * (c + 1) / C && left >= need && need > 0) || left == need) L.first.push_back(q + 1);
        if ((int)L.first.size() == C + 1) break;
    }
    while ((int)L.first.size() < C + 1) L.first.push_back(n);
    int64_t fmax = 0, nmax = 0, hmax = 0;
    for (int c = 0; c < C; ++c) {
        int64_t f = 0, k = 0, h = 0;
        std::vector<stamp_scene> sc;
        std::vector<int32_t> nn;
        for (int q = L.first[c]; q < L.first[c + 1]; ++q) {
            const int p = L.order[q];
            f += (int64_t)6 * scenes[p].H * N[p];
            k += N[p];
            h += (int64_t)scenes[p].H * N[p];
            sc.push_back(scenes[p]);
            nn.push_back(N[p]);
        }
        fmax = std::max(fmax, f);
        nmax = std::max(nmax, k);
        hmax = std::max(hmax, h);
        const size_t b = plan_bytes((int)sc.size(), sc.data(), nn.data(), cfg->ckpt_every, cfg->bandwidth);
        if (!b) return false;
        L.plan_bytes = std::max(L.plan_bytes, b);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    L.clk_off = take((size_t)2 * n * sizeof(uint64_t));
    L.th_off_s = take((size_t)fmax * 4);
    L.m_off_s = take((size_t)fmax * 4);
    L.v_off_s = take((size_t)fmax * 4);
    L.cost_off_s = take((size_t)nmax * 4);
    L.modes_off_s = take((size_t)hmax * 4);
    L.plan_off = take(L.plan_bytes);
    L.total = off;
    return true;
}

// True when two plans place every workspace region at the same offset.
bool same_layout(const SolvePlan& a, const SolvePlan& b) {
    bool ok = a.total == b.total && a.clk_off == b.clk_off && a.desc_off == b.desc_off && a.roll_off == b.roll_off &&
              a.adj_tiles_off == b.adj_tiles_off &&
              a.dist_off == b.dist_off && a.cand_off == b.cand_off && a.fin_off == b.fin_off &&
              a.red_off == b.red_off &&
              a.ctr_off == b.ctr_off && a.err_off == b.err_off && a.tape_off == b.tape_off && a.seg_off == b.seg_off &&
              a.grad_off == b.grad_off && a.phi_vec_off == b.phi_vec_off && a.cost_off == b.cost_off &&
              a.cdisc_off == b.cdisc_off && a.wts_off == b.wts_off && a.svgd_off == b.svgd_off;
    for (int c = 0; c < kPhi32Classes; ++c) ok = ok && a.phi_off[c] == b.phi_off[c];
    ok = ok && a.ctr16_off == b.ctr16_off && a.row16_off == b.row16_off && a.phi16_off[0] == b.phi16_off[0] &&
         a.phi16_off[1] == b.phi16_off[1];
    return ok;
}

__global__ void k_stamp_clock(uint64_t* dst) { *dst = wall_clock64(); }

__global__ void k_clock_to_us(const uint64_t* clk, int n, float us_per_tick, float* out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[p] = (float)(clk[2 * p + 1] - clk[2 * p]) * us_per_tick;
}

hipError_t launch_clock(uint64_t* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_stamp_clock, dim3(1), dim3(1), 0, st, dst);
    return hipGetLastError();
}

hipError_t launch_clock_to_us(const uint64_t* clk, int n, float us_per_tick, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_clock_to_us, dim3((n + 63) / 64), dim3(64), 0, st, clk, n, us_per_tick, out);
    return hipGetLastError();
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
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, device) == hipSuccess && v > 0) c->clock_khz = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0) c->num_cus = v;
    // default-priority stream of our own: solves are captured into graphs here
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
        scratch_address(device, &c->scratch) != hipSuccess) {
        stamp_destroy(c);
        return STAMP_EHIP;
    }
    *ctx = c;
    return STAMP_OK;
}

void stamp_destroy(stamp_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    ctx->destroy_graphs();
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int32_t stamp_set_autotune(stamp_ctx* ctx, int32_t enable) {
    if (!ctx) return STAMP_EINVAL;
    ctx->autotune = enable ? 1 : 0;
    return STAMP_OK;
}

int32_t stamp_set_rollout_layout(stamp_ctx* ctx, int32_t layout) {
    if (!ctx) return STAMP_EINVAL;
    if (layout != STAMP_LAYOUT_AUTO && layout != STAMP_LAYOUT_BLOCKS && layout != STAMP_LAYOUT_PACKED)
        return fail(ctx, STAMP_EINVAL, "layout %d is not STAMP_LAYOUT_AUTO, _BLOCKS or _PACKED", layout);
    ctx->rollout_layout = layout;
    return STAMP_OK;
}

int32_t stamp_set_launch_shape(stamp_ctx* ctx, int32_t roll_block, int32_t roll_grid, int32_t phi_rows) {
    if (!ctx) return STAMP_EINVAL;
    if (roll_block == 0 && roll_grid == 0 && phi_rows == 0) {
        ctx->is_pinned = 0;
        return STAMP_OK;
    }
    if (!(roll_block == 64 || roll_block == 128 || roll_block == 256) || roll_grid < 0 ||
        !(phi_rows == 64 || phi_rows == 128 || phi_rows == 256))
        return fail(ctx, STAMP_EINVAL, "launch shape: roll_block and phi_rows in {64,128,256}, roll_grid >= 0");
    ctx->pinned.roll_block = roll_block;
    ctx->pinned.roll_grid = roll_grid;
    ctx->pinned.phi_rows = phi_rows;
    ctx->is_pinned = 1;
    return STAMP_OK;
}

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
    for (int p = 0; p < n_problems; ++p)
        if (!scene_ok(&scenes[p]) || N[p] < 1 || N[p] > kMaxSvgdN) return 0;
    if (cfg->classes > 1 && n_problems > 1) {
        ClassPlan L;
        return class_plan(n_problems, scenes, N, cfg, L) ? L.total : 0;
    }
    return plan_bytes(n_problems, scenes, N, cfg->ckpt_every, cfg->bandwidth);
}

int32_t stamp_rollout_fwd(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                          const float* theta, float* cost, float* tape, size_t tape_len, int32_t ckpt_every,
                          uint32_t* status, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !cost) return fail(ctx, STAMP_EINVAL, "null theta or cost");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    if (ckpt_every < 0) return fail(ctx, STAMP_EINVAL, "ckpt_every < 0");
    SimConst c;
    int r = derive(ctx, scene, w, &c);
    if (r) return r;
    if (tape && tape_len < tape_floats(scene, N, ckpt_every))
        return fail(ctx, STAMP_ENOSPACE, "tape %zu < %zu floats", tape_len, tape_floats(scene, N, ckpt_every));
    const TapeGeom g = tape_geom(scene, N, ckpt_every);
    hipError_t e = launch_rollout_fwd(c, N, theta, cost, tape, g, status, (hipStream_t)stream,
                                      packed_for(ctx, block_lanes(N, c.B), false));
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "rollout_fwd");
}

int32_t stamp_dsvgd_weights(stamp_ctx* ctx, int32_t N, const float* cost_relaxed, const float* cost_discrete,
                            float* weights, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!cost_relaxed || !cost_discrete || !weights) return fail(ctx, STAMP_EINVAL, "null cost or weights");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    hipError_t e = launch_dsvgd_weights(N, cost_relaxed, cost_discrete, weights, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "dsvgd_weights");
}

size_t stamp_readout_workspace_bytes(const stamp_scene* scene, int32_t N) {
    if (!scene || N < 1 || scene->H < 1 || scene->H > kMaxPushes) return 0;
    return (size_t)6 * scene->H * N * sizeof(float);
}

int32_t stamp_plan_readout(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                           const float* theta, int32_t* modes, float* cost, void* workspace, size_t ws_bytes,
                           uint32_t* status, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !modes || !cost) return fail(ctx, STAMP_EINVAL, "null theta, modes or cost");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    SimConst c;
    int r = derive(ctx, scene, w, &c);
    if (r) return r;
    const size_t need = stamp_readout_workspace_bytes(scene, N);
    if (!workspace || ws_bytes < need) return fail(ctx, STAMP_ENOSPACE, "read-out workspace %zu < %zu", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    float* plan = (float*)workspace;
    hipError_t e = launch_modes(N, scene->H, theta, modes, st);
    if (e == hipSuccess) e = launch_onehot(N, scene->H, theta, plan, st);
    if (e == hipSuccess)
        e = launch_rollout_fwd(c, N, plan, cost, nullptr, tape_geom(scene, N, 0), status, st,
                               packed_for(ctx, block_lanes(N, c.B), false));
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "plan_readout");
}

static int32_t rollout_adj_impl(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                                const float* theta, const float* tape, size_t tape_len, int32_t ckpt_every,
                                const float* cost_bar, float* grad, void* workspace, size_t ws_bytes,
                                uint32_t* status, void* stream, int per_phase) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !tape || !grad) return fail(ctx, STAMP_EINVAL, "null theta, tape or grad");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    if (ckpt_every < 0) return fail(ctx, STAMP_EINVAL, "ckpt_every < 0");
    SimConst c;
    int r = derive(ctx, scene, w, &c);
    if (r) return r;
    if (tape_len < tape_floats(scene, N, ckpt_every))
        return fail(ctx, STAMP_ENOSPACE, "tape %zu < %zu floats", tape_len, tape_floats(scene, N, ckpt_every));
    const size_t need = adj_ws_bytes(scene, N, ckpt_every);
    if (need && (!workspace || ws_bytes < need))
        return fail(ctx, STAMP_ENOSPACE, "adjoint workspace %zu < %zu bytes", ws_bytes, need);
    const TapeGeom g = tape_geom(scene, N, ckpt_every);
    c.per_phase = per_phase;
    hipError_t e = launch_rollout_adj(c, N, theta, tape, g, cost_bar, 1.0f, grad, (float*)workspace, status,
                                      (hipStream_t)stream, packed_for(ctx, block_lanes(N, c.B), true));
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "rollout_adj");
}

int32_t stamp_rollout_adj(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                          const float* theta, const float* tape, size_t tape_len, int32_t ckpt_every,
                          const float* cost_bar, float* grad, void* workspace, size_t ws_bytes, uint32_t* status,
                          void* stream) {
    return rollout_adj_impl(ctx, scene, w, N, theta, tape, tape_len, ckpt_every, cost_bar, grad, workspace,
                            ws_bytes, status, stream, 0);
}

int32_t stamp_rollout_adj_phases(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                                 const float* theta, const float* tape, size_t tape_len, int32_t ckpt_every,
                                 const float* cost_bar, float* grad, void* workspace, size_t ws_bytes,
                                 uint32_t* status, void* stream) {
    return rollout_adj_impl(ctx, scene, w, N, theta, tape, tape_len, ckpt_every, cost_bar, grad, workspace,
                            ws_bytes, status, stream, 1);
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
    hipError_t e = launch_svgd(N, d, theta, grad_logp, bandwidth, phi, h_out, workspace, L, 0, nullptr,
                               (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_step");
}

int32_t stamp_svgd_step_noalloc(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, const float* grad_logp,
                                float bandwidth, float* phi, float* h_out, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !grad_logp || !phi) return fail(ctx, STAMP_EINVAL, "null theta, grad_logp or phi");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    if (d > kMaxSvgdDim || N > kMaxSvgdN)
        return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports d <= %d, N <= %d", kMaxSvgdDim, kMaxSvgdN);
    if (!isfinite(bandwidth)) return fail(ctx, STAMP_EINVAL, "non-finite bandwidth");
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (L.total > (size_t)STAMP_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, STAMP_ENOSPACE, "N=%d, d=%d needs %zu bytes of scratch; the no-alloc step holds %zu "
                                         "(use stamp_svgd_step with a workspace)",
                    N, d, L.total, (size_t)STAMP_NOALLOC_SCRATCH_BYTES);
    if (!ctx->scratch) return fail(ctx, STAMP_EHIP, "no scratch address on device %d", ctx->device);
    hipError_t e = launch_svgd(N, d, theta, grad_logp, bandwidth, phi, h_out, ctx->scratch, L, 0, nullptr,
                               (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_step_noalloc");
}

int32_t stamp_svgd_bandwidth(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, float bandwidth, float* h_out,
                             void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta) return fail(ctx, STAMP_EINVAL, "null theta");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    if (d > kMaxSvgdDim || N > kMaxSvgdN)
        return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports d <= %d, N <= %d", kMaxSvgdDim, kMaxSvgdN);
    if (!isfinite(bandwidth)) return fail(ctx, STAMP_EINVAL, "non-finite bandwidth");
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "svgd workspace %zu < %zu bytes", ws_bytes, L.total);
    hipError_t e = launch_svgd_bandwidth(N, d, theta, bandwidth, h_out, workspace, L, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_bandwidth");
}

int32_t stamp_svgd_direction(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, const float* grad_logp,
                             const float* weights, float* phi, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !grad_logp || !phi) return fail(ctx, STAMP_EINVAL, "null theta, grad_logp or phi");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    if (d > kMaxSvgdDim || N > kMaxSvgdN)
        return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports d <= %d, N <= %d", kMaxSvgdDim, kMaxSvgdN);
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "svgd workspace %zu < %zu bytes", ws_bytes, L.total);
    hipError_t e = launch_svgd_direction(N, d, theta, grad_logp, phi, workspace, L, 0, nullptr, (hipStream_t)stream,
                                         weights);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_direction");
}

int32_t stamp_svgd_update(stamp_ctx* ctx, int32_t N, int32_t d, float* theta, const float* grad_logp,
                          const float* weights, float* phi, float* m, float* v, int32_t t, float lr, float beta1,
                          float beta2, float eps, int32_t use_adam, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !grad_logp) return fail(ctx, STAMP_EINVAL, "null theta or grad_logp");
    if (use_adam && (!m || !v)) return fail(ctx, STAMP_EINVAL, "Adam needs m and v");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    if (d > kMaxSvgdDim || N > kMaxSvgdN)
        return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports d <= %d, N <= %d", kMaxSvgdDim, kMaxSvgdN);
    if (use_adam && t < 1) return fail(ctx, STAMP_EINVAL, "Adam step t=%d < 1", t);
    if (!isfinite(lr) || (use_adam && !(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps >= 0)))
        return fail(ctx, STAMP_EINVAL, "bad Adam hyper-parameters");
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "svgd workspace %zu < %zu bytes", ws_bytes, L.total);
    const UpdateArgs u{theta, m, v, t, nullptr, lr, beta1, beta2, eps, use_adam ? 1 : 0};
    hipError_t e = launch_svgd_direction(N, d, theta, grad_logp, phi, workspace, L, 0, nullptr, (hipStream_t)stream,
                                         weights, &u);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_update");
}

int32_t stamp_svgd_step_weighted(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, const float* grad_logp,
                                 const float* weights, float bandwidth, float* phi, float* h_out, void* workspace,
                                 size_t ws_bytes, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !grad_logp || !phi || !weights)
        return fail(ctx, STAMP_EINVAL, "null theta, grad_logp, weights or phi");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    if (d > kMaxSvgdDim || N > kMaxSvgdN)
        return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports d <= %d, N <= %d", kMaxSvgdDim, kMaxSvgdN);
    if (!isfinite(bandwidth)) return fail(ctx, STAMP_EINVAL, "non-finite bandwidth");
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "svgd workspace %zu < %zu bytes", ws_bytes, L.total);
    hipError_t e = launch_svgd(N, d, theta, grad_logp, bandwidth, phi, h_out, workspace, L, 0, nullptr,
                               (hipStream_t)stream, weights);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_step_weighted");
}

// validates a caller's structured kernel for particles of dimension d
static int32_t check_struct(stamp_ctx* ctx, const stamp_struct_kernel* k, int d, StructKernel* out) {
    if (!k) return fail(ctx, STAMP_EINVAL, "null structured kernel");
    if (k->layout != STAMP_KERNEL_PUSH && k->layout != STAMP_KERNEL_POSE)
        return fail(ctx, STAMP_EINVAL, "unknown kernel layout %d", k->layout);
    if (k->K < 1 || k->K > kStructMaxK) return fail(ctx, STAMP_EINVAL, "kernel K=%d outside 1..%d", k->K, kStructMaxK);
    const int want = (k->layout == STAMP_KERNEL_PUSH ? 6 : 7) * k->K;
    if (d != want) return fail(ctx, STAMP_EINVAL, "d=%d, the kernel layout needs %d", d, want);
    const float v[] = {k->alpha_g, k->alpha_z, k->alpha_p, k->kappa};
    for (float x : v)
        if (!isfinite(x) || x < 0.0f) return fail(ctx, STAMP_EINVAL, "kernel weights and kappa must be finite, >= 0");
    if (!isfinite(k->h_g) || !isfinite(k->h_z)) return fail(ctx, STAMP_EINVAL, "non-finite kernel bandwidth");
    *out = StructKernel{k->layout, k->K, k->alpha_g, k->alpha_z, k->alpha_p, k->h_g, k->h_z, k->kappa};
    return STAMP_OK;
}

int32_t stamp_svgd_step_structured(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta,
                                   const float* grad_logp, const float* weights, const stamp_struct_kernel* kernel,
                                   float* phi, float* h_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !grad_logp || !phi) return fail(ctx, STAMP_EINVAL, "null theta, grad_logp or phi");
    if (N < 1 || d < 1) return fail(ctx, STAMP_EINVAL, "N=%d, d=%d must be >= 1", N, d);
    StructKernel sk;
    int32_t r = check_struct(ctx, kernel, d, &sk);
    if (r) return r;
    if (N > kMaxSvgdN) return fail(ctx, STAMP_EUNSUPPORTED, "svgd step supports N <= %d", kMaxSvgdN);
    const SvgdLayout L = svgd_workspace_layout(N, d);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "svgd workspace %zu < %zu bytes", ws_bytes, L.total);
    hipError_t e = launch_svgd_structured(N, d, theta, grad_logp, weights, sk, phi, h_out, workspace, L, nullptr,
                                          (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_step_structured");
}

int32_t stamp_svgd_step_bf16(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, const float* grad_logp,
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
    hipError_t e = launch_svgd16(N, d, theta, grad_logp, bandwidth, phi, h_out, workspace, L, nullptr,
                                 (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "svgd_step_bf16");
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

}  // extern "C"

// Algorithm 1's loop over a batch of problems; sur (may be null) adds the
// surrogate phase in front of the true iterations.
static int32_t solve_impl(stamp_ctx* ctx, int32_t n_problems, const stamp_scene* scenes, const stamp_cost_w* w,
                          const int32_t* N, const stamp_solver_cfg* cfg, const stamp_surrogate* sur, float* theta,
                          float* adam_m, float* adam_v, float* cost_out, int32_t* modes_out, float* solve_time_us,
                          stamp_surrogate_report* rep, void* workspace, size_t ws_bytes, uint32_t* status,
                          void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (n_problems < 1 || !scenes || !w || !N || !cfg) return fail(ctx, STAMP_EINVAL, "null problem arrays");
    if (!theta || !cost_out) return fail(ctx, STAMP_EINVAL, "null theta or cost_out");
    if (cfg->iters < 0 || cfg->ckpt_every < 0 || cfg->t0 < 0 || cfg->sgd_iters < 0 || cfg->dsvgd < 0 ||
        cfg->dsvgd > 1)
        return fail(ctx, STAMP_EINVAL, "bad solver cfg");
    if (cfg->dsvgd && sur) return fail(ctx, STAMP_EINVAL, "importance weights apply to the simulator iterations only");
    if (cfg->per_phase < 0 || cfg->per_phase > 1) return fail(ctx, STAMP_EINVAL, "cfg->per_phase must be 0 or 1");
    // structured kernel: the push layout with K = each problem's H
    std::vector<StructKernel> skern;
    if (cfg->kernel) {
        if (cfg->kernel->layout != STAMP_KERNEL_PUSH)
            return fail(ctx, STAMP_EINVAL, "the solve's particles take the push kernel layout");
        if (sur && sur->phi_bf16) return fail(ctx, STAMP_EINVAL, "the structured kernel has no BF16 form");
        skern.resize(n_problems);
        for (int p = 0; p < n_problems; ++p) {
            stamp_struct_kernel k = *cfg->kernel;
            k.K = scenes[p].H;
            int32_t r = check_struct(ctx, &k, 6 * scenes[p].H, &skern[p]);
            if (r) return r;
        }
    }
    if (cfg->use_adam && (!adam_m || !adam_v)) return fail(ctx, STAMP_EINVAL, "Adam needs m and v");
    if (!isfinite(cfg->lr) || !isfinite(cfg->bandwidth)) return fail(ctx, STAMP_EINVAL, "non-finite lr/bandwidth");
    if (cfg->use_adam && !(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1 &&
                           cfg->adam_eps >= 0))
        return fail(ctx, STAMP_EINVAL, "bad Adam hyper-parameters");
    std::vector<SimConst> consts(n_problems);
    for (int p = 0; p < n_problems; ++p) {
        int r = derive(ctx, &scenes[p], &w[p], &consts[p]);
        if (r) return r;
        consts[p].per_phase = cfg->per_phase;
        if (N[p] < 1) return fail(ctx, STAMP_EINVAL, "problem %d: N=%d < 1", p, N[p]);
        if (6 * scenes[p].H > kMaxSvgdDim || N[p] > kMaxSvgdN)
            return fail(ctx, STAMP_EUNSUPPORTED, "problem %d too large for the svgd step", p);
    }
    const int K = cfg->ckpt_every;
    const size_t need = plan_bytes(n_problems, scenes, N, K, cfg->bandwidth);
    if (!workspace || ws_bytes < need) return fail(ctx, STAMP_ENOSPACE, "solve workspace %zu < %zu", ws_bytes, need);

    hipStream_t caller = (hipStream_t)stream;
    hipStream_t st = ctx->stream;
    hipError_t e;
#define STAMP_TRY(x, what)                              \
    do {                                                \
        if ((e = (x)) != hipSuccess) return hip_fail(ctx, e, what); \
    } while (0)
    // order our stream after the caller's pending work on its inputs
    STAMP_TRY(hipEventRecord(ctx->ev_in, caller), "event record");
    STAMP_TRY(hipStreamWaitEvent(st, ctx->ev_in, 0), "stream wait");

    // launch shapes: tuned once per batch signature
    // rollout layout of the whole batch, by its block-per-lane lane count
    int64_t all_lanes = 0;
    for (int p = 0; p < n_problems; ++p) all_lanes += block_lanes(N[p], scenes[p].B);
    const bool packed = packed_for(ctx, all_lanes, false), packed_adj = packed_for(ctx, all_lanes, true);
    SolvePlan P;
    build_plan(n_problems, scenes, N, K, cfg->bandwidth, 256, &consts, P, packed, packed_adj);
    // Every rebuild below (another row block) must keep the regions where the
    // pointers derived next point: the layout reserves the longest lists.
    const SolvePlan layout0 = P;
    auto rebuild = [&](int rows) -> bool {
        build_plan(n_problems, scenes, N, K, cfg->bandwidth, rows, &consts, P, packed, packed_adj);
        return same_layout(P, layout0);
    };
    const std::string tkey = P.key + "K" + std::to_string(K) + (cfg->bandwidth > 0 ? "fixed" : "median");
    StampTune tune;
    auto it_t = ctx->tune.find(tkey);
    const bool have_tune = ctx->is_pinned || it_t != ctx->tune.end();
    if (ctx->is_pinned) tune = ctx->pinned;
    else if (have_tune) tune = it_t->second;
    if (tune.phi_rows != 256 && !rebuild(tune.phi_rows))
        return fail(ctx, STAMP_EINVAL, "internal: workspace layout depends on the row block");

    char* ws = (char*)workspace;
    ProblemDesc* d_desc = (ProblemDesc*)(ws + P.desc_off);
    int2* d_roll = (int2*)(ws + P.roll_off);
    int2* d_adj_tiles = (int2*)(ws + P.adj_tiles_off);
    int* d_ctr = (int*)(ws + P.ctr_off);
    uint64_t* d_clk = (uint64_t*)(ws + P.clk_off);
    float* d_tape = (float*)(ws + P.tape_off);
    float* d_seg = (float*)(ws + P.seg_off);
    float* d_grad = (float*)(ws + P.grad_off);
    float* d_phi = (float*)(ws + P.phi_vec_off);
    char* d_svgd = ws + P.svgd_off;
    auto upload = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    auto upload_lists = [&]() -> hipError_t {
        hipError_t r;
        if ((r = upload(P.desc_off, P.descs.data(), P.descs.size() * sizeof(ProblemDesc))) != hipSuccess) return r;
        if ((r = upload(P.roll_off, P.roll_tiles.data(), P.roll_tiles.size() * sizeof(int2))) != hipSuccess) return r;
        if ((r = upload(P.adj_tiles_off, P.adj_tiles.data(), P.adj_tiles.size() * sizeof(int2))) != hipSuccess)
            return r;
        if ((r = upload(P.dist_off, P.dist_work.data(), P.dist_work.size() * sizeof(int4))) != hipSuccess) return r;
        if ((r = upload(P.cand_off, P.cand_work.data(), P.cand_work.size() * sizeof(int4))) != hipSuccess) return r;
        if ((r = upload(P.fin_off, P.fin_work.data(), P.fin_work.size() * sizeof(int4))) != hipSuccess) return r;
        if ((r = upload(P.red_off, P.red_work.data(), P.red_work.size() * sizeof(int4))) != hipSuccess) return r;
        for (int c = 0; c < kPhi32Classes; ++c)
            if ((r = upload(P.phi_off[c], P.phi_work[c].data(), P.phi_work[c].size() * sizeof(int4))) != hipSuccess)
                return r;
        if ((r = upload(P.ctr16_off, P.ctr_work.data(), P.ctr_work.size() * sizeof(int4))) != hipSuccess) return r;
        if ((r = upload(P.row16_off, P.row16_work.data(), P.row16_work.size() * sizeof(int4))) != hipSuccess) return r;
        for (int c = 0; c < 2; ++c)
            if ((r = upload(P.phi16_off[c], P.phi16_work[c].data(), P.phi16_work[c].size() * sizeof(int4))) !=
                hipSuccess)
                return r;
        return hipStreamSynchronize(st);  // host lists may go out of scope after this
    };
    STAMP_TRY(upload_lists(), "upload work lists");
    const int ntiles = (int)P.roll_tiles.size(), nadj = (int)P.adj_tiles.size();
    auto batch_plan = [&]() {
        BatchPlan B{};
        B.n_problems = n_problems;
        B.dist_work = (const int4*)(ws + P.dist_off);
        B.n_dist = (int)P.dist_work.size();
        for (int c = 0; c < kMedLists; ++c) {
            B.dist_start[c] = P.dist_start[c];
            B.dist_n[c] = P.dist_n[c];
        }
        B.cand_work = (const int4*)(ws + P.cand_off);
        B.fin_work = (const int4*)(ws + P.fin_off);
        B.n_fin = (int)P.fin_work.size();
        B.n_cand = (int)P.cand_work.size();
        for (int c = 0; c < kPhi32Classes; ++c) {
            B.phi_work[c] = (const int4*)(ws + P.phi_off[c]);
            B.n_phi[c] = (int)P.phi_work[c].size();
        }
        B.phi_rows = P.phi_rows;
        B.red_work = (const int4*)(ws + P.red_off);
        B.n_red = (int)P.red_work.size();
        B.ctr_work = (const int4*)(ws + P.ctr16_off);
        B.n_ctr = (int)P.ctr_work.size();
        B.row16_work = (const int4*)(ws + P.row16_off);
        B.n_row16 = (int)P.row16_work.size();
        for (int c = 0; c < 2; ++c) {
            B.phi16_work[c] = (const int4*)(ws + P.phi16_off[c]);
            B.n_phi16[c] = (int)P.phi16_work[c].size();
        }
        return B;
    };
    auto roll_grid = [&](const StampTune& t, int tiles) {
        const int waves = t.roll_block / 64;
        const int full = (tiles + waves - 1) / waves;
        return t.roll_grid > 0 ? std::min(t.roll_grid, full) : full;
    };

    if (!have_tune && ctx->autotune && cfg->iters + cfg->sgd_iters > 0) {
        {
            // time the rollout shapes and the contraction row blocks on this batch
            hipEvent_t a, b;
            STAMP_TRY(hipEventCreate(&a), "event");
            STAMP_TRY(hipEventCreate(&b), "event");
            auto timed = [&](auto&& fn) -> float {
                fn();  // warm-up
                (void)hipEventRecord(a, st);
                fn();
                (void)hipEventRecord(b, st);
                (void)hipEventSynchronize(b);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, a, b);
                return ms;
            };
            float best = 1e30f;
            StampTune cand;
            const int persist = ctx->num_cus * 4;
            for (int block : {64, 128, 256}) {
                if (n_problems == 1) break;  // a single problem takes the per-call rollout kernels
                for (int grid : {0, persist}) {
                    cand.roll_block = block;
                    cand.roll_grid = grid;
                    const float ms = timed([&] {
                        (void)launch_rollout_fwd_batched(d_desc, d_roll, ntiles, block, roll_grid(cand, ntiles), theta,
                                                         d_phi, d_tape, nullptr, st, packed);
                        (void)launch_rollout_adj_batched(d_desc, d_adj_tiles, nadj, block, roll_grid(cand, nadj), theta,
                                                         d_tape, -1.0f, d_grad, d_seg, nullptr, st, packed_adj);
                    });
                    if (ms < best) {
                        best = ms;
                        tune.roll_block = block;
                        tune.roll_grid = grid;
                    }
                }
            }
            best = 1e30f;
            for (int rows : {64, 128, 256}) {
                if (!rebuild(rows)) return fail(ctx, STAMP_EINVAL, "internal: workspace layout depends on the row block");
                STAMP_TRY(upload_lists(), "upload work lists");
                const BatchPlan B = batch_plan();
                const float ms =
                    timed([&] { (void)launch_svgd_batched(B, d_desc, theta, d_grad, d_phi, d_svgd, nullptr, st); });
                if (ms < best) {
                    best = ms;
                    tune.phi_rows = rows;
                }
            }
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (P.phi_rows != tune.phi_rows) {
                if (!rebuild(tune.phi_rows))
                    return fail(ctx, STAMP_EINVAL, "internal: workspace layout depends on the row block");
                STAMP_TRY(upload_lists(), "upload work lists");
            }
        }
        ctx->tune[tkey] = tune;
    }
    const BatchPlan B = batch_plan();
    const int rgrid = roll_grid(tune, ntiles);
    // Rollouts of the batch.  A single problem takes the per-call kernels,
    // compiled for its block count (fewer registers than the batched kernel,
    // which holds every block count's body: at 16 384 particles of 3 blocks the
    // adjoint fits four waves per SIMD instead of three).
    const bool single = n_problems == 1;
    auto roll_fwd = [&](const float* th, float* cost, float* tape, uint32_t* stat) -> hipError_t {
        if (single) {
            const ProblemDesc& D = P.descs[0];
            return launch_rollout_fwd(D.c, D.N, th + D.theta_off, cost + D.cost_off, tape ? tape + D.tape_off : nullptr,
                                      D.g, stat, st, packed);
        }
        return launch_rollout_fwd_batched(d_desc, d_roll, ntiles, tune.roll_block, rgrid, th, cost, tape, stat, st,
                                          packed);
    };
    auto roll_adj = [&](uint32_t* stat) -> hipError_t {
        if (single) {
            const ProblemDesc& D = P.descs[0];
            return launch_rollout_adj(D.c, D.N, theta + D.theta_off, d_tape + D.tape_off, D.g, nullptr, -1.0f,
                                      d_grad + D.theta_off, d_seg + D.seg_off, stat, st, packed_adj);
        }
        return launch_rollout_adj_batched(d_desc, d_adj_tiles, nadj, tune.roll_block, roll_grid(tune, nadj), theta,
                                          d_tape, -1.0f, d_grad, d_seg, stat, st, packed_adj);
    };

    // one SVGD iteration over every problem, captured once and replayed; with
    // importance weights (Eq. 4) each particle's discrete plan is rolled out
    // too (its one-hot particle built in the phi buffer, which the step
    // overwrites afterwards)
    float* d_cdisc = (float*)(ws + P.cdisc_off);
    float* d_wts = (float*)(ws + P.wts_off);
    // The SVGD step in two halves.  The bandwidth stage (medians, and the
    // structured kernel's features) depends on theta only, so it runs on the
    // side stream while the rollout produces the gradient; the direction stage
    // joins it.  exact = 0: the BF16 form's sampled median.
    auto bandwidth_stage = [&](hipStream_t s, int exact, int* step = nullptr) -> hipError_t {
        if (skern.empty()) return launch_svgd_bandwidth_batched(B, d_desc, theta, exact, d_svgd, s, step);
        for (int p = 0; p < n_problems; ++p) {
            const ProblemDesc& D = P.descs[p];
            hipError_t r = launch_struct_bandwidth(D.N, theta + D.theta_off, skern[p], d_svgd + D.svgd_off, D.sv, s);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    };
    // fork_at marks the point the bandwidth stage depends on; branch launches
    // it on the side stream (after the main stream's next work when that work
    // should lead the graph).  One side stream only: every stream a process
    // creates takes one of its few hardware queues, and two streams sharing a
    // queue run one after the other.
    auto fork_at = [&]() -> hipError_t { return hipEventRecord(ctx->ev_fork, st); };
    auto branch = [&](int exact, int* step = nullptr) -> hipError_t {
        hipError_t r;
        if ((r = hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0)) != hipSuccess) return r;
        if ((r = bandwidth_stage(ctx->side, exact, step)) != hipSuccess) return r;
        return hipEventRecord(ctx->ev_join, ctx->side);
    };
    auto fork = [&](int exact, int* step = nullptr) -> hipError_t {
        hipError_t r = fork_at();
        return r == hipSuccess ? branch(exact, step) : r;
    };
    auto join = [&]() -> hipError_t { return hipStreamWaitEvent(st, ctx->ev_join, 0); };
    const UpdateArgs upd{theta, adam_m, adam_v, cfg->t0, d_ctr, cfg->lr, cfg->beta1, cfg->beta2, cfg->adam_eps,
                         cfg->use_adam};
    auto direction_stage = [&](const float* wts) -> hipError_t {
        if (skern.empty()) return launch_svgd_direction_batched(B, d_desc, theta, d_grad, d_phi, d_svgd, status, st, wts);
        for (int p = 0; p < n_problems; ++p) {
            const ProblemDesc& D = P.descs[p];
            hipError_t r = launch_struct_direction(D.N, D.d, d_grad + D.theta_off, wts ? wts + D.cost_off : nullptr,
                                                   skern[p], d_phi + D.theta_off, nullptr, d_svgd + D.svgd_off, D.sv,
                                                   status, st);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    };
    // the direction and the update in one pass (the FP32 form's reduce
    // applies the update), or the direction then the update
    auto direction_update_stage = [&](const float* wts, const UpdateArgs& u) -> hipError_t {
        if (skern.empty())
            return launch_svgd_direction_batched(B, d_desc, theta, d_grad, nullptr, d_svgd, status, st, wts, &u);
        hipError_t r = direction_stage(wts);
        if (r != hipSuccess) return r;
        return launch_update(P.n_theta, theta, d_phi, adam_m, adam_v, cfg->t0, d_ctr, cfg->lr, cfg->beta1,
                             cfg->beta2, cfg->adam_eps, cfg->use_adam, st);
    };
    // the bandwidth stage's first launch advances the step counter when it
    // has one (the particle mean of some problem with N >= 2): the update
    // then reads the counter already advanced, and no counter kernel ends the
    // iteration
    const bool ctr_in_mean = skern.empty() && B.n_ctr > 0;
    UpdateArgs upd_pre = upd;
    upd_pre.t_pre = 1;
    auto iteration = [&]() -> hipError_t {
        hipError_t r;
        if ((r = fork(1, ctr_in_mean ? d_ctr : nullptr)) != hipSuccess) return r;
        if ((r = roll_fwd(theta, (float*)(ws + P.cost_off), d_tape, status)) != hipSuccess) return r;
        if ((r = roll_adj(status)) != hipSuccess) return r;
        if (cfg->dsvgd) {
            for (int p = 0; p < n_problems; ++p) {
                const ProblemDesc& D = P.descs[p];
                if ((r = launch_onehot(D.N, scenes[p].H, theta + D.theta_off, d_phi + D.theta_off, st)) != hipSuccess)
                    return r;
            }
            if ((r = roll_fwd(d_phi, d_cdisc, nullptr, status)) != hipSuccess) return r;
            if ((r = launch_dsvgd_weights_batched(n_problems, d_desc, (const float*)(ws + P.cost_off), d_cdisc,
                                                  d_wts, st)) != hipSuccess)
                return r;
        }
        if ((r = join()) != hipSuccess) return r;
        if (ctr_in_mean) return direction_update_stage(cfg->dsvgd ? d_wts : nullptr, upd_pre);
        if ((r = direction_update_stage(cfg->dsvgd ? d_wts : nullptr, upd)) != hipSuccess) return r;
        return launch_incr(d_ctr, st);
    };
    // one SGD refinement iteration: the update takes phi = grad log rho
    auto sgd_iteration = [&]() -> hipError_t {
        hipError_t r;
        if ((r = roll_fwd(theta, (float*)(ws + P.cost_off), d_tape, status)) != hipSuccess) return r;
        if ((r = roll_adj(status)) != hipSuccess) return r;
        if ((r = launch_update(P.n_theta, theta, d_grad, adam_m, adam_v, cfg->t0, d_ctr, cfg->lr, cfg->beta1,
                               cfg->beta2, cfg->adam_eps, cfg->use_adam, st)) != hipSuccess)
            return r;
        return launch_incr(d_ctr, st);
    };
    // the surrogate-phase iteration: the network's cost gradient (exact bound
    // term included) replaces rollout + adjoint, every other stage unchanged
    const int s_iters = sur ? sur->iters : 0;
    std::vector<int64_t> enc_off(n_problems, 0);
    if (sur)
        for (int p = 1; p < n_problems; ++p) enc_off[p] = enc_off[p - 1] + (sur->n_in - 6 * scenes[p - 1].H);
    auto sur_infer = [&](int p, float* cost, float* grad, float scale) -> hipError_t {
        const ProblemDesc& D = P.descs[p];
        const float* enc = sur->n_in > D.d ? sur->enc + enc_off[p] : nullptr;
        return launch_mlp_infer(sur->params, (const __bf16*)sur->wbf16, theta + D.theta_off, 1, D.N, sur->n_in, D.d,
                                enc, scenes[p].H, w[p].bound, w[p].o_max, w[p].d_max, nullptr,
                                cost ? cost + D.cost_off : nullptr, grad ? grad + D.theta_off : nullptr, scale, st);
    };
    auto sur_iteration = [&]() -> hipError_t {
        hipError_t r;
        if (sur->phi_bf16) {
            // The sampled median and the BF16 operands take ~15 us when they
            // have the chip to themselves, but beside the network's inference
            // their single-workgroup select waits for its workgroups to drain,
            // and the fork and join cost ~10 us each: they run first, on the
            // same stream (and advance the step counter on the way).
            if (skern.empty()) {
                if ((r = launch_bandwidth16_batched(B, d_desc, theta, d_svgd, st, d_ctr)) != hipSuccess) return r;
            } else if ((r = bandwidth_stage(st, 0)) != hipSuccess) {
                return r;
            }
            for (int p = 0; p < n_problems; ++p)
                if ((r = sur_infer(p, nullptr, d_grad, -1.0f)) != hipSuccess) return r;
        } else {
            // the network's gradient is the longest branch: it leads the graph
            if ((r = fork_at()) != hipSuccess) return r;
            for (int p = 0; p < n_problems; ++p)
                if ((r = sur_infer(p, nullptr, d_grad, -1.0f)) != hipSuccess) return r;
            if ((r = branch(1)) != hipSuccess) return r;
            if ((r = join()) != hipSuccess) return r;
        }
        if (sur->phi_bf16 && skern.empty()) {  // the counter was advanced at the start
            UpdateArgs u = upd;
            u.t_pre = 1;
            return launch_svgd16_direction_batched(B, d_desc, theta, d_grad, nullptr, d_svgd, status, st, &u);
        }
        if (sur->phi_bf16) {
            if ((r = launch_svgd16_direction_batched(B, d_desc, theta, d_grad, nullptr, d_svgd, status, st, &upd)) !=
                hipSuccess)
                return r;
        } else if ((r = direction_update_stage(nullptr, upd)) != hipSuccess) {
            return r;
        }
        return launch_incr(d_ctr, st);
    };
    char gkey[512];
    snprintf(gkey, sizeof gkey, "|%p|%p|%p|%p|%p|%d|%d|%.9g|%.9g|%.9g|%.9g|%d|%d|%d|%d|", (void*)ws, (void*)theta,
             (void*)adam_m, (void*)adam_v, (void*)status, cfg->t0, cfg->use_adam, cfg->lr, cfg->beta1, cfg->beta2,
             cfg->adam_eps, tune.roll_block, rgrid, tune.phi_rows, cfg->dsvgd);
    std::string full_key = tkey + gkey;
    {  // every problem's constants (scene, cost weights, split): the single-problem
       // rollout launches take them by value, so the captured graph holds them
        uint64_t hsh = 1469598103934665603ull;  // FNV-1a over the bytes
        const unsigned char* b = reinterpret_cast<const unsigned char*>(consts.data());
        for (size_t i = 0; i < consts.size() * sizeof(SimConst); ++i) hsh = (hsh ^ b[i]) * 1099511628211ull;
        snprintf(gkey, sizeof gkey, "c%016llx|", (unsigned long long)hsh);
        full_key += gkey;
    }
    if (cfg->kernel) {  // the kernel's parameters are arguments of the captured launches
        const stamp_struct_kernel& k = *cfg->kernel;
        snprintf(gkey, sizeof gkey, "struct|%.9g|%.9g|%.9g|%.9g|%.9g|%.9g|", k.alpha_g, k.alpha_z, k.alpha_p, k.h_g,
                 k.h_z, k.kappa);
        full_key += gkey;
    }
    // capture `body` into `graph` unless the cached one was made for `key`
    auto ensure_graph = [&](hipGraphExec_t& graph, std::string& have_key, const std::string& key,
                            auto&& body) -> int32_t {
        if (graph && have_key == key) return STAMP_OK;
        if (graph) {
            STAMP_TRY(hipStreamSynchronize(st), "sync");
            (void)hipGraphExecDestroy(graph);
            graph = nullptr;
        }
        hipGraph_t g = nullptr;
        STAMP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
        const hipError_t ce = body();
        const hipError_t ee = hipStreamEndCapture(st, &g);
        if (ce != hipSuccess) return hip_fail(ctx, ce, "capture iteration");
        if (ee != hipSuccess) return hip_fail(ctx, ee, "end capture");
        e = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            graph = nullptr;
            return hip_fail(ctx, e, "graph instantiate");
        }
        have_key = key;
        return STAMP_OK;
    };
    // `count` iterations of `body`: the unrolled graph as often as it fits,
    // the one-iteration graph for the rest
    auto run_iterations = [&](stamp_ctx::IterGraphs& G, const std::string& key, int count, auto&& body) -> int32_t {
        if (count >= kGraphUnroll) {
            int32_t r = ensure_graph(G.many, G.key_many, key + "|unrolled", [&]() -> hipError_t {
                for (int u = 0; u < kGraphUnroll; ++u) {
                    const hipError_t e2 = body();
                    if (e2 != hipSuccess) return e2;
                }
                return hipSuccess;
            });
            if (r) return r;
        }
        if (count % kGraphUnroll) {
            int32_t r = ensure_graph(G.one, G.key_one, key, body);
            if (r) return r;
        }
        int it = 0;
        for (; it + kGraphUnroll <= count; it += kGraphUnroll) STAMP_TRY(hipGraphLaunch(G.many, st), "graph launch");
        for (; it < count; ++it) STAMP_TRY(hipGraphLaunch(G.one, st), "graph launch");
        return STAMP_OK;
    };
    STAMP_TRY(launch_fill_u32((uint32_t*)d_ctr, 0u, 1, st), "counter");
    if (solve_time_us)
        for (int p = 0; p < n_problems; ++p) STAMP_TRY(launch_clock(d_clk + 2 * p, st), "clock");
    // surrogate phase, judged against the rollout at each check
    int run = 0, checks = 0, fell_back = 0;
    float last_err = 0.0f;
    if (s_iters > 0) {
        // the network's pointers and each problem's bound weights are kernel
        // arguments of the captured graph, so they are part of its key
        char skey[160];
        snprintf(skey, sizeof skey, "sur|%p|%p|%p|%d|%d|", (const void*)sur->params, sur->wbf16,
                 (const void*)sur->enc, sur->n_in, sur->phi_bf16);
        std::string sk = full_key + skey;
        for (int p = 0; p < n_problems; ++p) {
            snprintf(skey, sizeof skey, "%.9g/%.9g/%.9g;", w[p].bound, w[p].o_max, w[p].d_max);
            sk += skey;
        }
        float* d_err = (float*)(ws + P.err_off);
        float* c_true = (float*)(ws + P.cost_off);
        std::vector<float> h_err(n_problems);
        while (run < s_iters) {
            const int chunk = sur->check_every > 0 ? std::min(sur->check_every, s_iters - run) : s_iters - run;
            int32_t r = run_iterations(ctx->graph_slot("sur", sk), sk, chunk, sur_iteration);
            if (r) return r;
            run += chunk;
            STAMP_TRY(roll_fwd(theta, c_true, nullptr, status), "check rollout");
            for (int p = 0; p < n_problems; ++p) STAMP_TRY(sur_infer(p, d_phi, nullptr, 1.0f), "check network");
            STAMP_TRY(launch_log_err(d_desc, n_problems, c_true, d_phi, d_err, st), "check error");
            STAMP_TRY(hipMemcpyAsync(h_err.data(), d_err, n_problems * sizeof(float), hipMemcpyDeviceToHost, st),
                      "check copy");
            STAMP_TRY(hipStreamSynchronize(st), "check sync");
            ++checks;
            last_err = 0.0f;
            for (float v : h_err) last_err = (v > last_err || !(v == v)) ? v : last_err;
            if (sur->max_log_err > 0.0f && !(last_err <= sur->max_log_err) && run < s_iters) {
                fell_back = 1;
                break;
            }
        }
    }
    if (rep) {
        rep->iters_run = run;
        rep->fell_back = fell_back;
        rep->checks = checks;
        rep->log_err = last_err;
    }
    if (cfg->iters - run > 0) {
        int32_t r = run_iterations(ctx->graph_slot("svgd", full_key), full_key, cfg->iters - run, iteration);
        if (r) return r;
    }
    if (cfg->sgd_iters > 0) {  // refinement: the step counter runs on
        int32_t r = run_iterations(ctx->graph_slot("sgd", full_key), full_key, cfg->sgd_iters, sgd_iteration);
        if (r) return r;
    }
    // final true cost and discrete plan of every particle
    STAMP_TRY(roll_fwd(theta, cost_out, nullptr, status), "final rollout");
    if (modes_out) {
        int64_t m_off = 0;
        for (int p = 0; p < n_problems; ++p) {
            STAMP_TRY(launch_modes(N[p], scenes[p].H, theta + P.descs[p].theta_off, modes_out + m_off, st), "modes");
            m_off += (int64_t)scenes[p].H * N[p];
        }
    }
    if (solve_time_us) {
        for (int p = 0; p < n_problems; ++p)
            STAMP_TRY(launch_clock(d_clk + 2 * p + 1, st), "clock");
        STAMP_TRY(launch_clock_to_us(d_clk, n_problems, 1000.0f / (float)ctx->clock_khz, solve_time_us, st),
                  "clock");
    }
    // the caller's stream waits for the solve
    STAMP_TRY(hipEventRecord(ctx->ev_out, st), "event record");
    STAMP_TRY(hipStreamWaitEvent(caller, ctx->ev_out, 0), "stream wait");
#undef STAMP_TRY
    return STAMP_OK;
}

static int32_t solve_classes(stamp_ctx* ctx, int32_t n, const stamp_scene* scenes, const stamp_cost_w* w,
                             const int32_t* N, const stamp_solver_cfg* cfg, float* theta, float* adam_m,
                             float* adam_v, float* cost_out, int32_t* modes_out, float* solve_time_us,
                             void* workspace, size_t ws_bytes, uint32_t* status, void* stream) {
    if (!scenes || !w || !N) return fail(ctx, STAMP_EINVAL, "null problem arrays");
    if (!theta || !cost_out) return fail(ctx, STAMP_EINVAL, "null theta or cost_out");
    for (int p = 0; p < n; ++p)
        if (!scene_ok(&scenes[p]) || N[p] < 1 || N[p] > kMaxSvgdN)
            return fail(ctx, STAMP_EINVAL, "problem %d: bad scene or N=%d", p, N[p]);
    ClassPlan L;
    if (!class_plan(n, scenes, N, cfg, L)) return fail(ctx, STAMP_EINVAL, "bad solver cfg");
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "class-scheduled solve workspace %zu < %zu", ws_bytes, L.total);
    hipStream_t caller = (hipStream_t)stream;
    char* ws = (char*)workspace;
    uint64_t* d_clk = (uint64_t*)(ws + L.clk_off);
    float* s_th = (float*)(ws + L.th_off_s);
    float* s_m = (float*)(ws + L.m_off_s);
    float* s_v = (float*)(ws + L.v_off_s);
    float* s_cost = (float*)(ws + L.cost_off_s);
    int32_t* s_modes = (int32_t*)(ws + L.modes_off_s);
    stamp_solver_cfg one = *cfg;
    one.classes = 0;
    hipError_t e;
#define STAMP_TRY(x, what)                                          \
    do {                                                            \
        if ((e = (x)) != hipSuccess) return hip_fail(ctx, e, what); \
    } while (0)
    // a problem's [off, off + count) elements between the packed array and the class's
    auto move = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, caller) : hipSuccess;
    };
    if (solve_time_us)
        for (int p = 0; p < n; ++p) STAMP_TRY(launch_clock(d_clk + 2 * p, caller), "clock");
    for (size_t c = 0; c + 1 < L.first.size(); ++c) {
        std::vector<stamp_scene> sc;
        std::vector<stamp_cost_w> wc;
        std::vector<int32_t> nc;
        int64_t f = 0, k = 0, h = 0;
        for (int q = L.first[c]; q < L.first[c + 1]; ++q) {  // the class's inputs, packed in its order
            const int p = L.order[q];
            sc.push_back(scenes[p]);
            wc.push_back(w[p]);
            nc.push_back(N[p]);
            const size_t fb = (size_t)6 * scenes[p].H * N[p] * 4;
            STAMP_TRY(move(s_th + f, theta + L.th_off[p], fb), "pack theta");
            if (adam_m) STAMP_TRY(move(s_m + f, adam_m + L.th_off[p], fb), "pack m");
            if (adam_v) STAMP_TRY(move(s_v + f, adam_v + L.th_off[p], fb), "pack v");
            f += (int64_t)6 * scenes[p].H * N[p];
        }
        const int32_t r = solve_impl(ctx, (int32_t)sc.size(), sc.data(), wc.data(), nc.data(), &one, nullptr, s_th,
                                     adam_m ? s_m : nullptr, adam_v ? s_v : nullptr, s_cost,
                                     modes_out ? s_modes : nullptr, nullptr, nullptr, ws + L.plan_off, L.plan_bytes,
                                     status, stream);
        if (r) return r;
        f = 0;
        for (int q = L.first[c]; q < L.first[c + 1]; ++q) {  // and back to their places
            const int p = L.order[q];
            const size_t fb = (size_t)6 * scenes[p].H * N[p] * 4;
            STAMP_TRY(move(theta + L.th_off[p], s_th + f, fb), "unpack theta");
            if (adam_m) STAMP_TRY(move(adam_m + L.th_off[p], s_m + f, fb), "unpack m");
            if (adam_v) STAMP_TRY(move(adam_v + L.th_off[p], s_v + f, fb), "unpack v");
            STAMP_TRY(move(cost_out + L.co_off[p], s_cost + k, (size_t)N[p] * 4), "unpack cost");
            if (modes_out)
                STAMP_TRY(move(modes_out + L.mo_off[p], s_modes + h, (size_t)scenes[p].H * N[p] * 4), "unpack modes");
            if (solve_time_us) STAMP_TRY(launch_clock(d_clk + 2 * p + 1, caller), "clock");
            f += (int64_t)6 * scenes[p].H * N[p];
            k += N[p];
            h += (int64_t)scenes[p].H * N[p];
        }
    }
    if (solve_time_us)
        STAMP_TRY(launch_clock_to_us(d_clk, n, 1000.0f / (float)ctx->clock_khz, solve_time_us, caller), "clock");
#undef STAMP_TRY
    return STAMP_OK;
}

extern "C" {

int32_t stamp_solve(stamp_ctx* ctx, int32_t n_problems, const stamp_scene* scenes, const stamp_cost_w* w,
                    const int32_t* N, const stamp_solver_cfg* cfg, float* theta, float* adam_m, float* adam_v,
                    float* cost_out, int32_t* modes_out, float* solve_time_us, void* workspace, size_t ws_bytes,
                    uint32_t* status, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!cfg) return fail(ctx, STAMP_EINVAL, "null cfg");
    if (cfg->classes < 0) return fail(ctx, STAMP_EINVAL, "cfg->classes=%d < 0", cfg->classes);
    if (cfg->classes > 1 && n_problems > 1)
        return solve_classes(ctx, n_problems, scenes, w, N, cfg, theta, adam_m, adam_v, cost_out, modes_out,
                             solve_time_us, workspace, ws_bytes, status, stream);
    return solve_impl(ctx, n_problems, scenes, w, N, cfg, nullptr, theta, adam_m, adam_v, cost_out, modes_out,
                      solve_time_us, nullptr, workspace, ws_bytes, status, stream);
}

int32_t stamp_solve_surrogate(stamp_ctx* ctx, int32_t n_problems, const stamp_scene* scenes, const stamp_cost_w* w,
                              const int32_t* N, const stamp_solver_cfg* cfg, const stamp_surrogate* sur, float* theta,
                              float* adam_m, float* adam_v, float* cost_out, int32_t* modes_out, float* solve_time_us,
                              stamp_surrogate_report* report, void* workspace, size_t ws_bytes, uint32_t* status,
                              void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!sur || !cfg || !scenes || n_problems < 1) return fail(ctx, STAMP_EINVAL, "null surrogate, cfg or scenes");
    if (cfg->classes > 1) return fail(ctx, STAMP_EINVAL, "class scheduling applies to stamp_solve");
    if (sur->iters < 0 || sur->iters > cfg->iters)
        return fail(ctx, STAMP_EINVAL, "surrogate iters=%d not in [0, iters=%d]", sur->iters, cfg->iters);
    if (sur->n_in < 1 || sur->n_in > kMlpIn) return fail(ctx, STAMP_EINVAL, "n_in=%d not in [1,%d]", sur->n_in, kMlpIn);
    if (!sur->params || !sur->wbf16) return fail(ctx, STAMP_EINVAL, "null network parameters");
    if (sur->check_every < 0 || !isfinite(sur->max_log_err)) return fail(ctx, STAMP_EINVAL, "bad check settings");
    for (int p = 0; p < n_problems; ++p) {
        const int d = 6 * scenes[p].H;
        if (scenes[p].H < 1 || d > sur->n_in)
            return fail(ctx, STAMP_EINVAL, "problem %d: d=%d exceeds the network's n_in=%d", p, d, sur->n_in);
        if (d < sur->n_in && !sur->enc) return fail(ctx, STAMP_EINVAL, "null scene encodings");
    }
    return solve_impl(ctx, n_problems, scenes, w, N, cfg, sur, theta, adam_m, adam_v, cost_out, modes_out,
                      solve_time_us, report, workspace, ws_bytes, status, stream);
}

// ---- learned cost surrogate --------------------------------------------------

int32_t stamp_mlp_prepare(stamp_ctx* ctx, const float* params, void* wbf16, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!params || !wbf16) return fail(ctx, STAMP_EINVAL, "null params or wbf16");
    hipError_t e = launch_mlp_prepare(params, (__bf16*)wbf16, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "mlp_prepare");
}

int32_t stamp_mlp_standardize(stamp_ctx* ctx, int32_t M, int32_t n_in, const float* x, const float* cost,
                              float* params, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!x || !params) return fail(ctx, STAMP_EINVAL, "null x or params");
    if (M < 1) return fail(ctx, STAMP_EINVAL, "M=%d < 1", M);
    if (n_in < 1 || n_in > kMlpIn) return fail(ctx, STAMP_EINVAL, "n_in=%d not in [1,%d]", n_in, kMlpIn);
    hipError_t e = launch_mlp_standardize(x, cost, M, n_in, params, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "mlp_standardize");
}

int32_t stamp_mlp_label(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                        const float* theta, int32_t n_in, const float* enc, float* x, float* cost, uint32_t* status,
                        void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!theta || !x || !cost) return fail(ctx, STAMP_EINVAL, "null theta, x or cost");
    if (N < 1) return fail(ctx, STAMP_EINVAL, "N=%d < 1", N);
    if (!w || !scene) return fail(ctx, STAMP_EINVAL, "null scene or cost weights");
    stamp_cost_w w_roll = *w;
    w_roll.bound = 0.0f;  // the network learns the rollout part only
    SimConst c;
    int r = derive(ctx, scene, &w_roll, &c);
    if (r) return r;
    const int d = 6 * scene->H;
    if (n_in < d || n_in > kMlpIn) return fail(ctx, STAMP_EINVAL, "n_in=%d not in [d=%d, %d]", n_in, d, kMlpIn);
    if (n_in > d && !enc) return fail(ctx, STAMP_EINVAL, "null scene encoding");
    const TapeGeom g = tape_geom(scene, N, 0);
    hipError_t e = launch_rollout_fwd(c, N, theta, cost, nullptr, g, status, (hipStream_t)stream,
                                      packed_for(ctx, block_lanes(N, c.B), false));
    if (e == hipSuccess) e = launch_mlp_pack_rows(theta, N, d, enc, n_in, x, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "mlp_label");
}

int32_t stamp_mlp_forward(stamp_ctx* ctx, int32_t M, int32_t n_in, int32_t d, const float* params, const void* wbf16,
                          const float* x, int32_t x_layout, const float* enc, const stamp_cost_w* w, float* y,
                          float* cost, float* grad, float grad_scale, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!params || !wbf16 || !x) return fail(ctx, STAMP_EINVAL, "null params, wbf16 or x");
    if (M < 1) return fail(ctx, STAMP_EINVAL, "M=%d < 1", M);
    if (n_in < 1 || n_in > kMlpIn) return fail(ctx, STAMP_EINVAL, "n_in=%d not in [1,%d]", n_in, kMlpIn);
    if (d < 1 || d > n_in) return fail(ctx, STAMP_EINVAL, "d=%d not in [1,n_in]", d);
    if (x_layout != 0 && x_layout != 1) return fail(ctx, STAMP_EINVAL, "x_layout=%d not 0 or 1", x_layout);
    if (x_layout == 1 && d < n_in && !enc) return fail(ctx, STAMP_EINVAL, "null scene encoding");
    if (w && d % 6) return fail(ctx, STAMP_EINVAL, "bound term needs plan inputs (d=%d not a multiple of 6)", d);
    if (w && (!isfinite(w->bound) || !isfinite(w->o_max) || !isfinite(w->d_max)))
        return fail(ctx, STAMP_EINVAL, "non-finite bound weights");
    if (!isfinite(grad_scale)) return fail(ctx, STAMP_EINVAL, "non-finite grad_scale");
    hipError_t e = launch_mlp_infer(params, (const __bf16*)wbf16, x, x_layout, M, n_in, d, enc, w ? d / 6 : 0,
                                    w ? w->bound : 0.0f, w ? w->o_max : 0.0f, w ? w->d_max : 0.0f, y, cost, grad,
                                    grad_scale, (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "mlp_forward");
}

size_t stamp_mlp_train_workspace_bytes(int32_t M) {
    if (M < 64 || M % 64) return 0;
    return mlp_train_layout(M).total;
}

int32_t stamp_mlp_train_step(stamp_ctx* ctx, int32_t M, int32_t n_in, const float* x, const float* cost,
                             const int32_t* idx, int32_t n_rows, float* params, void* wbf16, float* adam_m,
                             float* adam_v, int32_t t, float lr, float beta1, float beta2, float eps, float* loss,
                             uint32_t* status, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (!x || !cost || !params || !wbf16 || !adam_m || !adam_v) return fail(ctx, STAMP_EINVAL, "null pointer");
    if (M < 64 || M % 64) return fail(ctx, STAMP_EINVAL, "M=%d must be a positive multiple of 64", M);
    if (n_in < 1 || n_in > kMlpIn) return fail(ctx, STAMP_EINVAL, "n_in=%d not in [1,%d]", n_in, kMlpIn);
    if (n_rows < 1 || (!idx && n_rows < M))
        return fail(ctx, STAMP_EINVAL, "n_rows=%d too small for a minibatch of %d", n_rows, M);
    if (t < 1) return fail(ctx, STAMP_EINVAL, "Adam step t=%d < 1", t);
    if (!isfinite(lr) || !(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps >= 0))
        return fail(ctx, STAMP_EINVAL, "bad Adam hyper-parameters");
    const MlpTrainLayout L = mlp_train_layout(M);
    if (!workspace || ws_bytes < L.total)
        return fail(ctx, STAMP_ENOSPACE, "mlp train workspace %zu < %zu bytes", ws_bytes, L.total);
    hipError_t e = launch_mlp_train_step(params, (__bf16*)wbf16, adam_m, adam_v, t, lr, beta1, beta2, eps, x, cost,
                                         idx, n_rows, M, n_in, loss, status, (char*)workspace, L,
                                         (hipStream_t)stream);
    return e == hipSuccess ? STAMP_OK : hip_fail(ctx, e, "mlp_train_step");
}

int32_t stamp_mlp_train_steps(stamp_ctx* ctx, int32_t n_steps, int32_t M, int32_t n_in, const float* x,
                              const float* cost, const int32_t* idx, int32_t n_rows, float* params, void* wbf16,
                              float* adam_m, float* adam_v, int32_t t0, const float* lr, float beta1, float beta2,
                              float eps, float* loss, uint32_t* status, void* workspace, size_t ws_bytes,
                              void* stream) {
    if (!ctx) return STAMP_EINVAL;
    if (n_steps < 1 || !idx || !lr || t0 < 0) return fail(ctx, STAMP_EINVAL, "n_steps < 1, null idx or lr, or t0 < 0");
    for (int s = 0; s < n_steps; ++s)
        if (!isfinite(lr[s])) return fail(ctx, STAMP_EINVAL, "lr[%d] is not finite", s);
    // the checks of one step cover every step
    const int32_t r = stamp_mlp_train_step(ctx, M, n_in, x, cost, idx, n_rows, params, wbf16, adam_m, adam_v, t0 + 1,
                                           lr[0], beta1, beta2, eps, loss, status, workspace, ws_bytes, stream);
    if (r) return r;
    const MlpTrainLayout L = mlp_train_layout(M);
    for (int s = 1; s < n_steps; ++s) {
        const hipError_t e = launch_mlp_train_step(params, (__bf16*)wbf16, adam_m, adam_v, t0 + s + 1, lr[s], beta1,
                                                   beta2, eps, x, cost, idx + (int64_t)s * M, n_rows, M, n_in,
                                                   loss ? loss + s : nullptr, status, (char*)workspace, L,
                                                   (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train_steps");
    }
    return STAMP_OK;
}

}  // extern "C"
