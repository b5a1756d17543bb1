/*
 * stamp.h -- C ABI of the MI355X (gfx950) STAMP SVGD hot path.
 *
 * STAMP (Lee et al., arXiv 2310.01775) samples task-and-motion plans with Stein
 * variational gradient descent.  Each particle is a relaxed discrete action
 * sequence plus continuous push parameters; its log-posterior gradient comes from
 * a differentiable rigid-body pushing rollout.  This library runs one SVGD
 * iteration (and loops of them) on the GPU:
 *
 *   rollout forward  (Sec. III-B; Sec. IV-A; Appendix E-B)  stamp_rollout_fwd
 *   rollout adjoint  (Sec. III-B, back-propagation through the trajectory)
 *                                                            stamp_rollout_adj
 *   median bandwidth + SVGD direction (Eq. 1; Appendix D-B) stamp_svgd_step
 *   update (Algorithm 1's step, or Adam)                     stamp_adam_step
 *   the loop of Algorithm 1 (SVGD phase)                     stamp_solve
 *
 * Conventions shared by every call
 * --------------------------------
 * - Particle arrays are structure-of-arrays, particle index fastest:
 *   theta[l * N + i] is coordinate l of particle i, d = 6 * H coordinates.
 *   For push k: l = 6k+0..6k+3 are the side logits a_k (North, East, South,
 *   West), l = 6k+4 the contact offset o_k (m), l = 6k+5 the push depth D_k (m).
 * - All array arguments are DEVICE pointers to float32 (or int32/uint32 where
 *   typed so), owned by the caller, contiguous, 4-byte aligned.  Scene, cost and
 *   solver structs are HOST pointers, read during the call only.
 * - Every compute call is asynchronous on `stream` (a hipStream_t passed as
 *   void*; NULL = the null stream) and returns once its kernels are enqueued.
 *   No compute call allocates memory; scratch comes in through `workspace`,
 *   sized by the matching *_bytes call.
 * - Return value: STAMP_OK or a negative STAMP_E* code.  Argument errors are
 *   detected on the host before anything is enqueued.  STAMP_EHIP means a HIP
 *   runtime call failed; stamp_last_error() returns its text.
 * - Asynchronous numerical faults (a non-finite cost, state or gradient) set
 *   bits in the caller's device word `status` (may be NULL to skip), which the
 *   caller reads after synchronising.  The library never clears it.
 * - One stamp_ctx per thread that issues calls; a context is not thread-safe.
 */
#ifndef STAMP_H
#define STAMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STAMP_OK 0
#define STAMP_EINVAL (-1)       /* null pointer, size or parameter out of range */
#define STAMP_ENOSPACE (-2)     /* workspace or tape smaller than required */
#define STAMP_EHIP (-3)         /* HIP runtime error; see stamp_last_error */
#define STAMP_EUNSUPPORTED (-4) /* valid request this build does not implement */

#define STAMP_MODES 4       /* push sides N, E, S, W (Sec. V-A) */
#define STAMP_MAX_BLOCKS 4  /* blocks per scene */
#define STAMP_MAX_PUSHES 8  /* H, pushes per plan */

/* learned cost surrogate (stamp_mlp_*) */
#define STAMP_MLP_WIDTH 256          /* hidden width of both hidden layers */
#define STAMP_MLP_IN_PAD 64          /* input width the weights are stored at */
#define STAMP_MLP_PARAMS 82817       /* floats of the parameter vector */
#define STAMP_MLP_BF16_WEIGHTS 163840 /* bf16 elements of the working copies */
#define STAMP_SCENE_ENC 24           /* floats of the scene encoding */

/* scratch bytes each GPU holds for stamp_svgd_step_noalloc */
#define STAMP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* bits of the device status word */
#define STAMP_STATUS_NONFINITE_COST 1u
#define STAMP_STATUS_NONFINITE_GRAD 2u
#define STAMP_STATUS_NONFINITE_PHI 4u
#define STAMP_STATUS_BAD_INDEX 8u     /* a training index outside the dataset */

typedef struct stamp_ctx stamp_ctx;

/* Planar pushing scene (Sec. IV-A "Block-Pushing", Appendix E-A).  Block 0 is
 * the pushed block; blocks 1..B-1 are free obstacles it can collide with.
 * T is the total number of integration steps, split into H push phases of
 * floor/ceil(T/H) steps; dt the step (s).  The model constants parameterise the
 * spring-based penalty contacts and regularised Coulomb friction of Sec. III-B:
 *   k_push, k_block  penalty stiffness (N/m) of pusher and block-block contact
 *   sp_beta          sharpness (1/m) of the softplus penalty log(1+e^{beta z})/beta
 *   standoff         distance (m) outside the face where each push starts
 *   g                gravity (m/s^2); eps_v_scale: eps_v = eps_v_scale*dt*mu*g
 *   eps_r            regulariser (m) of the block-centre distance */
typedef struct stamp_scene {
    int32_t H, M, B, T; /* pushes (1..8), modes (must be 4), blocks (1..4), steps (>= H) */
    float dt;
    float half[STAMP_MAX_BLOCKS];  /* half side length (m) */
    float mass[STAMP_MAX_BLOCKS];  /* kg */
    float mu[STAMP_MAX_BLOCKS];    /* ground friction coefficient */
    float pose0[STAMP_MAX_BLOCKS][3]; /* initial x, y (m), phi (rad) */
    float goal[3];                 /* goal x, y, phi of block 0 */
    float goal_tol;                /* dead-zone half-width of the target loss (m) */
    float k_push, k_block, sp_beta, standoff, g, eps_v_scale, eps_r;
} stamp_scene;

/* Cost weights (Appendix E-B): C = target*L_target + rot*L_rot + traj*L_traj
 * + bound*L_bound; o_max/d_max bound the offset and depth; traj_eps smooths the
 * Manhattan distance of L_traj.  log rho = -C. */
typedef struct stamp_cost_w {
    float target, rot, traj, bound, o_max, d_max, traj_eps;
} stamp_cost_w;

/* Solver settings (Algorithm 1: an SVGD phase, then an SGD refinement phase,
 * each a fixed number of iterations). */
typedef struct stamp_solver_cfg {
    int32_t iters;     /* SVGD iterations (>= 0) */
    int32_t t0;        /* Adam steps already taken (resume); step t = t0+1.. */
    float lr;          /* Adam lr, or epsilon of the plain step theta += lr*phi */
    float beta1, beta2, adam_eps;
    int32_t use_adam;  /* 1: Adam on -phi; 0: plain step */
    float bandwidth;   /* > 0: fixed h; <= 0: median heuristic every iteration */
    int32_t ckpt_every;/* tape mode inside the solve: 0 full tape, K>0 checkpoints */
    int32_t sgd_iters; /* SGD refinement iterations after the SVGD ones (>= 0; Algorithm 1's
                          second phase, Sec. III-C): the update takes phi = grad log rho of
                          each particle alone, with the same step rule and step counter */
    int32_t dsvgd;     /* 1: weight the SVGD sum by the importance weights of Eq. (4)
                          (stamp_dsvgd_weights of the relaxed and the discrete plan's cost,
                          one extra rollout per particle and iteration); 0: w_j = 1 */
    int32_t per_phase; /* 1: every simulator iteration takes the gradient of the per-phase split
                          of the cost (stamp_rollout_adj_phases); 0: the gradient of C */
    int32_t classes;   /* stamp_solve over several problems: 0 or 1, one batch in which the
                          problems advance in lockstep; C > 1, the problems are ordered by
                          their predicted cost per iteration and solved in min(C, n_problems)
                          classes of consecutive cost and about equal predicted work,
                          cheapest class first, each class one batch of its own (same
                          results, bit for bit), so that a cheap problem is done when its
                          class is */
    const struct stamp_struct_kernel* kernel; /* NULL: the RBF kernel on theta; else the
                          structured kernel (push layout; K is taken from each scene's H,
                          the field itself is ignored) in every SVGD iteration */
} stamp_solver_cfg;

/* ---- context ----------------------------------------------------------- */

/* Create a context bound to HIP device `device` (made current).  Returns
 * STAMP_EINVAL for a null ctx or a bad device, STAMP_EHIP on runtime errors. */
int32_t stamp_create(stamp_ctx** ctx, int32_t device);
void stamp_destroy(stamp_ctx* ctx);
/* Text of the last error recorded in ctx ("" if none); valid until the next call. */
const char* stamp_last_error(const stamp_ctx* ctx);
/* Library version string. */
const char* stamp_version(void);
/* Enable (default) or disable the launch-shape autotuner of stamp_solve.  When
 * enabled, the first solve of a batch signature (sizes of every problem, tape
 * mode, bandwidth mode) times candidate rollout workgroup sizes and grids and
 * contraction row blocks on the real data, synchronously, and caches the
 * fastest in ctx; the candidates differ only in launch shape, not in the
 * arithmetic, so results do not depend on the choice. */
int32_t stamp_set_autotune(stamp_ctx* ctx, int32_t enable);
/* Pin the launch shapes of stamp_solve instead of tuning them: rollout
 * workgroup size roll_block (64, 128 or 256 threads), rollout workgroup count
 * roll_grid (0 = one wave per 16-particle tile, else a persistent grid of at
 * most that many workgroups), contraction rows per workgroup phi_rows (64, 128
 * or 256).  All three 0 returns to the autotuned shapes. */
int32_t stamp_set_launch_shape(stamp_ctx* ctx, int32_t roll_block, int32_t roll_grid, int32_t phi_rows);

/* ---- sizing (host only, no GPU work) ------------------------------------- */

/* Rollout lane layout (results are the same bit for bit; only speed differs):
 * STAMP_LAYOUT_BLOCKS gives each block of a (particle, side) sub-rollout its
 * own lane (more waves: faster while the rollout is latency-bound on a small
 * particle set), STAMP_LAYOUT_PACKED one lane per sub-rollout holding all its
 * blocks (about half the instructions per particle), for the forward and the
 * adjoint alike.  STAMP_LAYOUT_AUTO (default): packed once the block-per-lane
 * form would need 2^17 lanes (two waves per SIMD), e.g. from 8192 particles of
 * 3 or 4 blocks, or a whole batch of that many lanes.  Applies to every rollout
 * of the context's later calls.  STAMP_EINVAL for another value. */
#define STAMP_LAYOUT_AUTO 0
#define STAMP_LAYOUT_BLOCKS 1
#define STAMP_LAYOUT_PACKED 2
int32_t stamp_set_rollout_layout(stamp_ctx* ctx, int32_t layout);

/* Floats of the rollout tape for N particles.  ckpt_every = 0 keeps the full
 * trajectory; K > 0 keeps a checkpoint every K steps inside each push phase.
 * Layout: [n_entries][4N][6B] then the phase-end block [H][4N][6B]: lane
 * 4i+s holds particle i's sub-rollout of side s, its state of block b at
 * 6b + (x, y, phi, vx, vy, omega).  Returns 0 on bad arguments. */
size_t stamp_tape_floats(const stamp_scene* scene, int32_t N, int32_t ckpt_every);
/* Workspace bytes of stamp_rollout_adj (segment replay buffer when K > 0). */
size_t stamp_adj_workspace_bytes(const stamp_scene* scene, int32_t N, int32_t ckpt_every);
/* Workspace bytes of stamp_svgd_step for N particles of dimension d. */
size_t stamp_svgd_workspace_bytes(int32_t N, int32_t d);
/* Workspace bytes of stamp_solve over n_problems problems (host arrays). */
size_t stamp_solve_workspace_bytes(int32_t n_problems, const stamp_scene* scenes,
                                   const int32_t* N, const stamp_solver_cfg* cfg);

/* ---- hot path ------------------------------------------------------------ */

/* Roll N particles through the relaxed pushing simulation (Sec. III-B, IV-A):
 * each push phase runs once per side from the shared phase-start state and the
 * next phase starts from the softmax(a_k)-weighted mixture of the outcomes.
 *   theta [d][N] in; cost [N] out (C of Appendix E-B);
 *   tape  out, or NULL when no adjoint follows; tape_floats is its length in
 *         floats (ignored when tape is NULL) and must be at least
 *         stamp_tape_floats(scene, N, ckpt_every).
 * Errors: STAMP_EINVAL for null ctx/scene/w/theta/cost, N < 1, H not in 1..8,
 * M != 4, B not in 1..4, T < H, dt <= 0, ckpt_every < 0; STAMP_ENOSPACE when
 * tape_floats is too small (nothing is enqueued). */
int32_t stamp_rollout_fwd(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w,
                          int32_t N, const float* theta, float* cost, float* tape, size_t tape_floats,
                          int32_t ckpt_every, uint32_t* status, void* stream);

/* Reverse sweep of the rollout (back-propagation through the trajectory,
 * Sec. III-B): grad[l*N+i] = cost_bar[i] * dC_i/dtheta_{l,i}.
 *   tape from stamp_rollout_fwd with the same theta and ckpt_every, of
 *         tape_floats floats (>= stamp_tape_floats(scene, N, ckpt_every));
 *   cost_bar [N] or NULL (= all ones); pass cost_bar = -1 to get grad log rho.
 *   workspace >= stamp_adj_workspace_bytes (may be NULL when that is 0).
 * Errors as stamp_rollout_fwd (tape may not be NULL here); STAMP_ENOSPACE if
 * tape_floats or ws_bytes is too small. */
int32_t stamp_rollout_adj(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w,
                          int32_t N, const float* theta, const float* tape, size_t tape_floats,
                          int32_t ckpt_every, const float* cost_bar, float* grad, void* workspace,
                          size_t ws_bytes, uint32_t* status, void* stream);

/* The adjoint of the per-phase split of the cost (appendix "Exploding Gradient
 * Issues": a cost that is a sum of per-action terms C = sum_k C_k lets each
 * action be optimised against its own term, so no gradient has to cross the
 * whole horizon).  The pushing cost splits by the phase whose end state a term
 * reads: push k's bound term to phase k; L_traj's term j = MH(P_{j-1}, P_j) +
 * MH(P_j, P_H) - MH(P_{j-1}, P_H) to phase j-1 (whose end is P_j); L_target and
 * L_rot to the last phase.  Inside C_k the positions other phases produce (its
 * start P_k and, for k < H-1, the final P_H) are constants and the rollout's
 * adjoint stops at the phase start, so
 *   grad[l*N+i] = cost_bar[i] * dC_{k(l),i}/dtheta_{l,i},   k(l) = l / 6.
 * The costs still sum to C (the value stamp_rollout_fwd returns).  Arguments,
 * layouts and errors as stamp_rollout_adj; one push (H = 1) gives its result. */
int32_t stamp_rollout_adj_phases(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w,
                                 int32_t N, const float* theta, const float* tape, size_t tape_floats,
                                 int32_t ckpt_every, const float* cost_bar, float* grad, void* workspace,
                                 size_t ws_bytes, uint32_t* status, void* stream);

/* SVGD direction of Eq. (1) with the RBF kernel K_ij = exp(-|theta_i-theta_j|^2/h):
 *   phi_i = (1/N) sum_j K_ij [ grad_logp_j + (2/h)(theta_i - theta_j) ].
 * bandwidth > 0 fixes h; otherwise h = max(m2 / ln N, 1e-12) with m2 the exact
 * lower median (the ceil(P/2)-th smallest) of the P = N(N-1)/2 squared distances
 * over i < j (median heuristic, Appendix D-B), as FP32 computes them: by direct
 * differences when P <= 2^20, in the Gram form |x_i|^2 + |x_j|^2 - 2 x_i.x_j of
 * the centred particles (matrix cores, clamped at 0) above.  The contraction
 * takes distances in that Gram form throughout.  For d <= 31 both Gram forms
 * and the contraction run on the BF16 matrix cores with every FP32 operand as
 * three BF16 parts (six part products per FP32 product, FP32 accumulation):
 * results of FP32 accuracy, not bit-equal to an FP32 matrix product.
 * N = 1 gives phi = grad_logp.
 *   theta, grad_logp, phi: [d][N]; h_out: one device float (may be NULL).
 * Errors: STAMP_EINVAL for null pointers, N < 1, d < 1; STAMP_ENOSPACE. */
int32_t stamp_svgd_step(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta,
                        const float* grad_logp, float bandwidth, float* phi, float* h_out,
                        void* workspace, size_t ws_bytes, void* stream);

/* stamp_svgd_step without a workspace argument, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The step's scratch (median select state and candidates,
 * operand tiles, partial sums) lives in a device array of
 * STAMP_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on holds
 * from the library's load until the process ends; the call allocates nothing.
 * Results equal stamp_svgd_step's for the same arguments bit for bit (the
 * same kernels).  The array is shared by every call on a GPU and keeps the last
 * call's contents (nothing in it needs to start at zero): calls that overlap
 * on one GPU -- from two streams or two contexts -- race and give undefined
 * results; serialise them.
 * Errors as stamp_svgd_step; STAMP_ENOSPACE when stamp_svgd_workspace_bytes(N, d)
 * exceeds the array (it fits N <= 4096 particles at d <= 36, e.g. 4096 x 30). */
int32_t stamp_svgd_step_noalloc(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta,
                                const float* grad_logp, float bandwidth, float* phi, float* h_out,
                                void* stream);

/* stamp_svgd_step in two halves, for callers that overlap the bandwidth with
 * the rollout (it depends on theta only):
 *   stamp_svgd_bandwidth: h (median heuristic, or bandwidth if > 0) into the
 *     workspace (and h_out if not NULL);
 *   stamp_svgd_direction: phi from theta, grad_logp and the h that the
 *     workspace holds, i.e. from the last stamp_svgd_bandwidth call on this
 *     workspace for the same theta; weights [N] device or NULL (Eq. (4)).
 * The caller orders the two calls (same stream, or an event between streams)
 * and must not run another call on the same workspace in between.  Arguments,
 * layouts and errors as stamp_svgd_step. */
int32_t stamp_svgd_bandwidth(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, float bandwidth,
                             float* h_out, void* workspace, size_t ws_bytes, void* stream);
int32_t stamp_svgd_direction(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta, const float* grad_logp,
                             const float* weights, float* phi, void* workspace, size_t ws_bytes, void* stream);
/* stamp_svgd_direction followed by stamp_adam_step in one pass: phi from the
 * bandwidth the workspace holds, then the update of Algorithm 1 applied to
 * theta in place (Adam at step t >= 1 with moments m, v, or theta += lr phi
 * when use_adam = 0); phi [d][N] is also stored when not NULL.  Bit for bit
 * the two calls' result.  Errors: those of both calls. */
int32_t stamp_svgd_update(stamp_ctx* ctx, int32_t N, int32_t d, float* theta, const float* grad_logp,
                          const float* weights, float* phi, float* m, float* v, int32_t t, float lr, float beta1,
                          float beta2, float eps, int32_t use_adam, void* workspace, size_t ws_bytes, void* stream);

/* The SVGD direction of stamp_svgd_step in reduced precision on the BF16
 * matrix cores, for iterations whose gradients are approximate anyway (the
 * surrogate phase).  Differences from stamp_svgd_step:
 *   - the median heuristic uses a fixed sample of 8192 particle pairs (all
 *     pairs when N(N-1)/2 <= 8192, then it is exact), distances in FP32;
 *   - the particles are centred on their mean, scaled by sqrt(2 log2(e) / h)
 *     and rounded to BF16 (x^); log2 K_ij comes from the Gram form
 *     x^_i.x^_j - |x^_i|^2/2 - |x^_j|^2/2 (MFMA, FP32 accumulation), so the
 *     distance is clamped at 0 by clamping K_ij to [0, 1];
 *   - K_ij is rounded to BF16 and K V, V_j = [g_j - (2/h) x_j | 1] rounded to
 *     BF16 (x_j the centred FP32 particle), is accumulated on MFMA in FP32;
 *     phi_i = (K V)_i[0..d) + (2/h) x_i (K V)_i[d], over N.
 * Same arguments, layouts and workspace (stamp_svgd_workspace_bytes). */
int32_t stamp_svgd_step_bf16(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta,
                             const float* grad_logp, float bandwidth, float* phi, float* h_out,
                             void* workspace, size_t ws_bytes, void* stream);

/* The SVGD direction of Eq. (4) with importance weights: as stamp_svgd_step,
 * phi_i = (1/N) sum_j w_j k(theta_j, theta_i) [g_j + (2/h)(theta_i - theta_j)]
 * for weights [N] (device, non-negative, mean 1 so that w_j / N = w_j / sum w);
 * the bandwidth is the unweighted median heuristic.  Errors: as
 * stamp_svgd_step; STAMP_EINVAL for null weights. */
int32_t stamp_svgd_step_weighted(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta,
                                 const float* grad_logp, const float* weights, float bandwidth, float* phi,
                                 float* h_out, void* workspace, size_t ws_bytes, void* stream);

/* The structured pusher kernel of Appendix E-C, a sum over actions k of
 *   alpha_g exp(-|g_k - g_k'|^2 / h_g)                 (RBF on the continuous part)
 * + alpha_z exp(-|softmax(a_k) - softmax(a_k')|^2 / h_z) (RBF on the relaxed action)
 * + alpha_p exp(kappa (cos(p_k - p_k') - 1))          (von Mises on an angle)
 * over one of two particle layouts:
 *   STAMP_KERNEL_PUSH: per action [a_k (4 logits), o_k, D_k], g_k = (o_k, D_k),
 *                      no angle; d = 6K (the rollout's particle layout);
 *   STAMP_KERNEL_POSE: [a_1..a_K, (x, y, phi)_1..K], g_k = (x, y), p_k = phi;
 *                      d = 7K (the paper's goal-pose particles).
 * h_g, h_z <= 0 select the median heuristic per component: h_c = max(m2_c /
 * ln N, 1e-12) / K with m2_c the exact lower median over pairs i < j of
 * sum_k |c_ik - c_jk|^2 on that component's features (softmax(a_k) or g_k). */
#define STAMP_KERNEL_PUSH 0
#define STAMP_KERNEL_POSE 1
typedef struct stamp_struct_kernel {
    int32_t layout;   /* STAMP_KERNEL_PUSH or STAMP_KERNEL_POSE */
    int32_t K;        /* actions, 1..8 */
    float alpha_g, alpha_z, alpha_p;  /* term weights (finite, >= 0) */
    float h_g, h_z;   /* RBF bandwidths: > 0 fixed, <= 0 median heuristic */
    float kappa;      /* von Mises concentration (finite, >= 0) */
} stamp_struct_kernel;

/* The SVGD direction of Eq. (1) (Eq. (4) with weights) under the structured
 * kernel: phi_i = (1/N) sum_j w_j [ K(theta_j, theta_i) grad_logp_j
 * + grad_{theta_j} K(theta_j, theta_i) ], the softmax term differentiated
 * through the softmax.  theta, grad_logp, phi: [d][N] device; weights: [N]
 * device or NULL (all 1); h_out: two device floats (h_g, h_z) or NULL.  N = 1
 * gives phi = grad_logp.  Workspace: stamp_svgd_workspace_bytes(N, d).
 * Errors: STAMP_EINVAL for null pointers, N < 1, a bad layout or K, d not
 * matching the layout, or negative / non-finite term weights, kappa or bandwidths;
 * STAMP_EUNSUPPORTED for N > 65536; STAMP_ENOSPACE. */
int32_t stamp_svgd_step_structured(stamp_ctx* ctx, int32_t N, int32_t d, const float* theta,
                                   const float* grad_logp, const float* weights,
                                   const stamp_struct_kernel* kernel, float* phi, float* h_out,
                                   void* workspace, size_t ws_bytes, void* stream);

/* Importance weights of Eq. (4) (discrete SVGD): the relaxed plan's likelihood
 * over the discrete plan's, w_j proportional to exp(-C_relaxed,j) /
 * exp(-C_discrete,j), scaled to mean 1 (max-subtracted in the exponent; a
 * non-finite cost gives weight 0; if every one is non-finite, all weights are
 * 1).  cost_relaxed from stamp_rollout_fwd, cost_discrete from
 * stamp_plan_readout; all device [N].  Errors: STAMP_EINVAL for null arrays
 * or N < 1. */
int32_t stamp_dsvgd_weights(stamp_ctx* ctx, int32_t N, const float* cost_relaxed, const float* cost_discrete,
                            float* weights, void* stream);

/* Update of Algorithm 1 on n = d*N floats, in place:
 *   use_adam = 1: Adam minimising -phi at step t (>= 1), bias-corrected;
 *   use_adam = 0: theta += lr * phi (m, v untouched, may be NULL). */
int32_t stamp_adam_step(stamp_ctx* ctx, int64_t n, float* theta, const float* phi, float* m,
                        float* v, int32_t t, float lr, float beta1, float beta2, float eps,
                        int32_t use_adam, void* stream);

/* Algorithm 1 for cfg->iters SVGD iterations (rollout -> adjoint -> bandwidth
 * -> phi -> update), then cfg->sgd_iters SGD iterations (rollout -> adjoint ->
 * update with phi = grad log rho), over n_problems independent problems.
 * Problem p has N[p] particles and scene scenes[p]; its particles, Adam moments
 * and outputs are packed one after another:
 *   theta, adam_m, adam_v: sum_p 6*H_p*N_p floats, problem p's block [d_p][N_p];
 *   cost_out: sum_p N_p (final true cost); modes_out: sum_p H_p*N_p int32,
 *   problem p's block [H_p][N_p] = argmax side per push (Gamma, Eq. 5), or NULL;
 *   solve_time_us: n_problems floats or NULL: device time from the solve's first
 *   kernel to the last kernel of the problem's own batch (cfg->classes <= 1: the
 *   problems advance in lockstep and the values coincide; cfg->classes > 1: the
 *   end of the problem's class).
 * cfg->classes > 1: the workspace holds each class's packed inputs and outputs
 * beside the largest class's batch (stamp_solve_workspace_bytes with the same
 * cfg); the classes run one after another on the context's stream.
 * adam_m/adam_v may be NULL only when use_adam = 0; m and v are not cleared.
 * Every stage of an iteration is one kernel over all problems (work lists of
 * (problem, tile)); the iteration is captured once into a HIP graph on the
 * context's own stream and replayed cfg->iters times; the caller's stream is
 * joined by events on entry and exit.  The call blocks the host while it
 * uploads the work lists (and while the autotuner runs, on first use).  The
 * result is bit-identical to running stamp_rollout_fwd, stamp_rollout_adj
 * (cost_bar = -1), stamp_svgd_step and stamp_adam_step per problem. */
int32_t stamp_solve(stamp_ctx* ctx, int32_t n_problems, const stamp_scene* scenes,
                    const stamp_cost_w* w, const int32_t* N, const stamp_solver_cfg* cfg,
                    float* theta, float* adam_m, float* adam_v, float* cost_out,
                    int32_t* modes_out, float* solve_time_us, void* workspace,
                    size_t ws_bytes, uint32_t* status, void* stream);


/* Plan read-out (Algorithm 1's result, Eq. 5): the discrete plan Gamma of
 * each particle (argmax side per push, lowest index on ties) into modes [H][N]
 * int32, and the cost of executing that discrete plan with the particle's
 * offsets and depths into cost [N]: the rollout of theta with each push's
 * logits replaced by 40 e_Gamma - 20, whose softmax weight of the chosen side
 * is 1 in FP32.  workspace (>= stamp_readout_workspace_bytes floats' bytes)
 * holds that plan vector.  Errors: as stamp_rollout_fwd; STAMP_EINVAL for
 * null modes or cost; STAMP_ENOSPACE if ws_bytes is too small. */
size_t stamp_readout_workspace_bytes(const stamp_scene* scene, int32_t N);
int32_t stamp_plan_readout(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                           const float* theta, int32_t* modes, float* cost, void* workspace, size_t ws_bytes,
                           uint32_t* status, void* stream);

/* ---- learned cost surrogate ------------------------------------------------
 * A network that predicts the rollout part of a plan's cost from the plan and
 * a scene encoding, so that early SVGD iterations can take its gradient in
 * place of the adjoint's.  It extends the method (the paper differentiates the
 * simulator throughout, Sec. III-B); the true rollout stays the judge and the
 * fallback.
 *
 *   x = [theta (d), scene encoding (n_in - d)],  n_in <= 64
 *   u = (x - mu) * inv_sigma
 *   h1 = gelu(W1 u + b1), h2 = gelu(W2 h1 + b2)       (width 256, exact erf GELU)
 *   y = w3 . h2 + b3                                    (y predicts log(1 + C_roll))
 *   C_hat = exp(y) - 1 + bound * L_bound(theta)
 * C_roll is the cost of Appendix E-B without its bound term; L_bound (a closed
 * form in theta, no rollout) is added exactly, with its gradient.
 *
 * Parameter vector `params` (STAMP_MLP_PARAMS floats, FP32 master copy):
 *   [0,64) mu, [64,128) inv_sigma, [128, 16512) W1 as [256][64] (row = output,
 *   columns n_in..63 zero), [16512,16768) b1, [16768, 82304) W2 as [256][256],
 *   [82304,82560) b2, [82560,82816) w3, [82816] b3.
 * `wbf16` (STAMP_MLP_BF16_WEIGHTS bf16 = 2 bytes each, device) holds the BF16
 * copies the matrix cores read: W1, W1^T, W2, W2^T.  stamp_mlp_prepare fills it
 * from params; stamp_mlp_train_step refreshes it after each update.
 * Arithmetic: BF16 inputs to the matrix products, FP32 accumulation, FP32
 * biases, GELU, output layer, bound term and Adam. */

/* Fill wbf16 from params.  Errors: STAMP_EINVAL for null pointers. */
int32_t stamp_mlp_prepare(stamp_ctx* ctx, const float* params, void* wbf16, void* stream);

/* Set mu and inv_sigma of params from training inputs x [M][n_in]: the mean
 * and population standard deviation of each input (inv_sigma = 1/max(sd,
 * 1e-3)); inputs n_in..63 get mu 0, inv_sigma 1.  With cost [M] (device, may
 * be NULL) the output bias b3 starts at the mean target, mean log(1 + cost).
 * Other entries untouched.
 * Errors: STAMP_EINVAL for null x or params, M < 1, n_in not in 1..64. */
int32_t stamp_mlp_standardize(stamp_ctx* ctx, int32_t M, int32_t n_in, const float* x, const float* cost,
                              float* params, void* stream);

/* Label training plans with the simulator: roll the N particles theta [d][N]
 * forward (as stamp_rollout_fwd, without the bound term of w) into cost [N],
 * and write their network inputs x [N][n_in] = [theta_i, enc] with enc the
 * n_in - d floats of the scene encoding (device).
 * Errors: as stamp_rollout_fwd; STAMP_EINVAL if n_in < d or n_in > 64, or enc
 * is NULL while n_in > d. */
int32_t stamp_mlp_label(stamp_ctx* ctx, const stamp_scene* scene, const stamp_cost_w* w, int32_t N,
                        const float* theta, int32_t n_in, const float* enc, float* x, float* cost,
                        uint32_t* status, void* stream);

/* Evaluate the network on M samples.
 *   x_layout 0: x is [M][n_in] (sample-major), enc ignored;
 *   x_layout 1: x is [d][M] (the particle layout), enc [n_in - d] device floats
 *               shared by all samples.
 *   w: NULL, or cost weights whose bound term (weight, o_max, d_max) is added
 *      to cost and grad; then d must be a multiple of 6 (plan inputs).
 *   y [M] (the network output), cost [M] (C_hat) and grad [d][M] =
 *   grad_scale * dC_hat/dx over the first d inputs are each optional (NULL skips).
 * Errors: STAMP_EINVAL for null params/wbf16/x, M < 1, n_in not in 1..64,
 * d not in 1..n_in, x_layout not 0 or 1, enc NULL with x_layout 1 and d < n_in,
 * or w given with d not a multiple of 6. */
int32_t stamp_mlp_forward(stamp_ctx* ctx, int32_t M, int32_t n_in, int32_t d, const float* params,
                          const void* wbf16, const float* x, int32_t x_layout, const float* enc,
                          const stamp_cost_w* w, float* y, float* cost, float* grad, float grad_scale,
                          void* stream);

/* Workspace bytes of stamp_mlp_train_step for a minibatch of M samples. */
size_t stamp_mlp_train_workspace_bytes(int32_t M);

/* One Adam step (step count t >= 1, bias-corrected) of the mean squared error
 * (1/M) sum_i (y_i - log(1 + cost[r_i]))^2 over a minibatch of M dataset rows
 * r_i = idx[i] (idx: M device int32, or NULL for rows 0..M-1) of the dataset
 * x [n_rows][n_in], cost [n_rows] (stamp_mlp_label writes both).  Updates W1,
 * b1, W2, b2, w3, b3 of params in place (mu, inv_sigma fixed) with the Adam
 * moments adam_m, adam_v (STAMP_MLP_PARAMS floats each, zero before step 1),
 * then refreshes wbf16.  loss (one device float, may be NULL) receives the
 * loss of the weights before the step.  An index outside [0, n_rows) reads
 * row 0 and sets STAMP_STATUS_BAD_INDEX in status (may be NULL).
 * Errors: STAMP_EINVAL for null pointers, M < 64 or not a multiple of 64, n_in
 * not in 1..64, n_rows < 1 (or < M without idx), t < 1; STAMP_ENOSPACE if
 * ws_bytes is too small. */
int32_t stamp_mlp_train_step(stamp_ctx* ctx, int32_t M, int32_t n_in, const float* x, const float* cost,
                             const int32_t* idx, int32_t n_rows, float* params, void* wbf16, float* adam_m,
                             float* adam_v, int32_t t, float lr, float beta1, float beta2, float eps, float* loss,
                             uint32_t* status, void* workspace, size_t ws_bytes, void* stream);

/* n_steps consecutive Adam steps of stamp_mlp_train_step in one call, the
 * kernels launched back to back by the library: step s (0-based) is Adam step
 * t0 + s + 1 on the minibatch rows idx[s * M .. s * M + M) (idx: n_steps * M
 * device int32, not NULL) with learning rate lr[s] (lr: n_steps host floats);
 * loss (n_steps device floats, may be NULL) receives each step's loss before
 * its update.  The result equals n_steps calls of stamp_mlp_train_step bit for
 * bit.  Same workspace (stamp_mlp_train_workspace_bytes(M)).
 * Errors: those of stamp_mlp_train_step; STAMP_EINVAL for n_steps < 1, a null
 * idx or lr, t0 < 0 or a non-finite lr[s]. */
int32_t stamp_mlp_train_steps(stamp_ctx* ctx, int32_t n_steps, int32_t M, int32_t n_in, const float* x,
                              const float* cost, const int32_t* idx, int32_t n_rows, float* params, void* wbf16,
                              float* adam_m, float* adam_v, int32_t t0, const float* lr, float beta1, float beta2,
                              float eps, float* loss, uint32_t* status, void* workspace, size_t ws_bytes,
                              void* stream);

/* Surrogate phase of stamp_solve_surrogate. */
typedef struct stamp_surrogate {
    int32_t iters;        /* leading iterations that take the network's gradient (0..cfg->iters) */
    int32_t n_in;         /* network inputs; problem p's encoding has n_in - d_p floats */
    int32_t check_every;  /* > 0: judge the network against the rollout every so many
                             surrogate iterations; the phase always ends with one check */
    float max_log_err;    /* > 0: leave the surrogate phase early when a check finds the
                             mean |log(1+C_hat) - log(1+C)| of any problem above it */
    int32_t phi_bf16;     /* 1: the surrogate iterations take the SVGD direction of
                             stamp_svgd_step_bf16; 0: that of stamp_svgd_step */
    int32_t reserved;
    const float* params;  /* device, STAMP_MLP_PARAMS floats */
    const void* wbf16;    /* device, STAMP_MLP_BF16_WEIGHTS bf16 (stamp_mlp_prepare) */
    const float* enc;     /* device, the problems' scene encodings one after another */
} stamp_surrogate;

/* What the surrogate phase did (host struct, filled before the call returns). */
typedef struct stamp_surrogate_report {
    int32_t iters_run;    /* surrogate iterations actually taken */
    int32_t fell_back;    /* 1 if a check ended the phase early */
    int32_t checks;       /* checks made */
    float log_err;        /* mean |log(1+C_hat) - log(1+C)| at the last check, max over problems */
} stamp_surrogate_report;

/* stamp_solve with a surrogate phase: the first sur->iters iterations use the
 * network's cost gradient (exact bound term included) in place of the
 * rollout adjoint, every other stage unchanged; the remaining iterations are
 * the true iterations of stamp_solve, continuing the same Adam step count.
 * The surrogate iteration is captured once into its own HIP graph and
 * replayed in chunks of check_every.  Each check rolls the particles forward
 * through the simulator, compares its cost with the network's and may end the
 * phase (fallback to the simulator).  The call blocks the host at each check.
 * Workspace: stamp_solve_workspace_bytes (the same plan).  report may be NULL.
 * Errors: as stamp_solve; STAMP_EINVAL for a null sur, sur->iters outside
 * [0, cfg->iters], n_in outside [max d_p, 64], null params/wbf16, or a null
 * enc while some problem has n_in > d_p. */
int32_t stamp_solve_surrogate(stamp_ctx* ctx, int32_t n_problems, const stamp_scene* scenes,
                              const stamp_cost_w* w, const int32_t* N, const stamp_solver_cfg* cfg,
                              const stamp_surrogate* sur, float* theta, float* adam_m, float* adam_v,
                              float* cost_out, int32_t* modes_out, float* solve_time_us,
                              stamp_surrogate_report* report, void* workspace, size_t ws_bytes,
                              uint32_t* status, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STAMP_H */
