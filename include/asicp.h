/*
 * asicp.h -- C ABI of the MI355X (gfx950) batched Annealed Stein ICP grasp
 * solver: "Grasping by Parallel Shape Matching" (arXiv 2412.08346).
 *
 * The solver takes the inputs of the paper's Algorithm 1 -- the gripper's
 * contact (inner-surface) cloud S per preshape, the object cloud R, the
 * collision cloud C, the gripper's signed distance field (built from the
 * complete gripper cloud G), the initial particles Theta_0, k_stein and
 * k_max (Sec. IV-A, Algorithm 1 inputs) -- and returns, per object, the pose
 * theta that minimises the grasp loss among collision-free particles
 * (Algorithm 1 return; Sec. VI-A).  Every iteration of every particle runs in
 * hand-written HIP kernels on the stream the caller passes.
 *
 * Conventions (all calls)
 *   - Units are metres.  A pose theta is (tx, ty, tz, qw, qx, qy, qz): the
 *     translation and a unit quaternion, scalar first (Sec. III-A).  A pose
 *     maps gripper-frame points into the object frame: s' = R(q) s + t.
 *   - Device arrays are float32 structure-of-arrays unless stated; "device"
 *     means memory of the current HIP device, "host" ordinary CPU memory.
 *   - Particle numbering: i = ((o * n_preshapes) + p) * K + j for object o,
 *     preshape p, particle j < K.  A group (o, p) is one Stein population.
 *   - Streams are passed as void* holding a hipStream_t (NULL = the null
 *     stream).  create / step / solve only enqueue work; result synchronises.
 *   - Status: ASICP_OK (0) or a negative code; on error asicp_last_error()
 *     returns a message (thread-local, valid until the next call on the same
 *     thread).  No C++ exception crosses this boundary.
 *   - The library never allocates device memory: the caller provides one
 *     workspace of asicp_workspace_bytes() bytes, aligned to 256 bytes.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef ASICP_H
#define ASICP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t asicp_status;
#define ASICP_OK 0
#define ASICP_E_INVALID (-1) /* bad argument; detected on the host, no device work done */
#define ASICP_E_STATE (-2)   /* call not allowed in the context's current state           */
#define ASICP_E_HIP (-3)     /* a HIP runtime call or kernel launch failed                 */
#define ASICP_E_NUMERIC (-4) /* a pose, cost or gradient became NaN / Inf on the device    */
#define ASICP_E_HOST (-5)    /* host-side failure (out of host memory); no C++ exception    */
                             /* ever crosses this interface                               */

/* Preconditioner A of the SGD-ICP update, eq. (3). */
#define ASICP_PRECOND_GN_DIAG 0  /* 1/(1+lambda) on t, 3/(2(rho^2 + lambda |TCP|^2)) on rotation */
#define ASICP_PRECOND_IDENTITY 1
/* Annealing. */
#define ASICP_SCHED_GEOMETRIC 0    /* gamma = 1, repulsion tau_k = T0 (T1/T0)^(k/(k_max-1))     */
#define ASICP_SCHED_PAPER_CYCLIC 1 /* eq. (11): gamma = (mod(k, k_max/C)/(k_max/C))^p, tau = 1 */
/* Combination of the translation RBF kernel (eq. 9) and the rotation kernel (eq. 10). */
#define ASICP_KERNEL_PRODUCT 0
#define ASICP_KERNEL_BLOCK 1
/* RBF bandwidth h of eq. (9). */
#define ASICP_BW_MEDIAN 0 /* lower median of |t_i - t_j|^2 over pairs / ln K, floored at h_min */
#define ASICP_BW_FIXED 1
/* Flags. */
#define ASICP_FLAG_DEBUG 1u  /* record per-point forward and reverse NN indices (needs more workspace) */
#define ASICP_FLAG_TIMING 2u /* record HIP events around every forward-NN launch                     */
#define ASICP_FLAG_NO_PRUNE 4u /* visit every object chunk in the forward NN (plain brute force); by    */
                               /* default chunks whose bounding box is provably farther than every     */
                               /* query's current best are skipped (same nearest-neighbour values)     */

/* Signed distance grid of one preshape (Sec. IV-C): value at node (i, j, k)
 * is the signed distance of origin + cell * (i, j, k) to the complete
 * gripper, negative inside.  A point collides when it lies inside the node box
 * and its trilinear interpolant is strictly negative. */
typedef struct {
  const float* values; /* device, [nz][ny][nx], x fastest; borrowed */
  int32_t nx, ny, nz;  /* >= 2 each */
  float origin[3];
  float cell;          /* > 0 */
} asicp_sdf;

/* One batch: n_objects objects x n_preshapes preshapes x K particles.  All
 * device pointers are borrowed: the caller keeps them alive and unmodified
 * until asicp_destroy.  Host arrays are read during asicp_create only. */
typedef struct {
  int32_t n_objects;           /* >= 1                                               */
  int32_t n_preshapes;         /* >= 1                                               */
  int32_t particles_per_group; /* K, 1 .. 1024                                       */
  const float* rx;             /* device, object clouds R concatenated (SoA)         */
  const float* ry;
  const float* rz;
  const int32_t* r_off;        /* host [n_objects+1]; every object has >= 1 point    */
  const float* cx;             /* device, collision clouds C concatenated (SoA);     */
  const float* cy;             /*   may alias rx/ry/rz; an object may have 0 points  */
  const float* cz;
  const int32_t* c_off;        /* host [n_objects+1]                                 */
  const float* sx;             /* device, contact clouds S concatenated, gripper     */
  const float* sy;             /*   frame                                            */
  const float* sz;
  const int32_t* s_off;        /* host [n_preshapes+1]; every preshape >= 1 point    */
  const asicp_sdf* sdf;        /* host [n_preshapes]                                 */
  const float* theta0;         /* device [7][Ktot] initial particles                 */
  const float* prev_cost;      /* device [Ktot] or NULL: resume state (cost of the   */
  const int32_t* converged;    /*   previous iteration, converged flags)             */
  int32_t k_start;             /* first iteration to run (0 .. k_max)                */
  const float* prior;          /* HOST, optional (NULL: none), [n_objects*n_preshapes][9]
                                  per group, Sec. III-C / eq. (8): mean translation
                                  mu_t[3], translation precision w_t = 1/sigma^2
                                  (>= 0), mean rotation mu_q[4] (w, x, y, z; unit
                                  within 1e-3, normalised on use), von Mises
                                  concentration kappa (>= 0).  Log prior
                                  -w_t/2 |t - mu_t|^2 + kappa tr(R(mu_q)^T R(q)), in the
                                  cost's units (m^2): the cost stands for a likelihood
                                  variance times a negative log likelihood, so w_t and
                                  kappa carry that variance.  The prior's gradient joins
                                  the Stein driving term only (the SGD phase of eq. (3)
                                  has none).  Copied during create. */
} asicp_problem;

/* Iteration settings.  Table I of the paper: k_max 40, k_stein 15, cyclic
 * annealing C 5 p 2, eta 1, cost weights 1 (lambda 1), convergence 2e-4. */
typedef struct {
  int32_t k_max;        /* iterations, >= 1                                          */
  int32_t k_stein;      /* iterations with the Stein update, 0 .. k_max; SGD after   */
  float eta;            /* learning rate, > 0                                        */
  float lambda;         /* weight of the TCP-CoM loss (eq. 13), >= 0                 */
  int32_t precond;      /* ASICP_PRECOND_*                                           */
  int32_t schedule;     /* ASICP_SCHED_*                                             */
  float T0, T1;         /* geometric schedule, > 0                                   */
  float cyc_C, cyc_p;   /* cyclic schedule, > 0                                      */
  int32_t kernel_mode;  /* ASICP_KERNEL_*                                            */
  int32_t bw_mode;      /* ASICP_BW_*                                                */
  float h_fixed;        /* bandwidth for ASICP_BW_FIXED, > 0                         */
  float h_min;          /* floor of the median bandwidth, > 0                        */
  float conv_tol;       /* relative cost change counted as converged, >= 0           */
  float w_pen;          /* weight of an optional SDF penetration term added to C:    */
                        /*   w_pen / M_c * sum over colliding points of phi^2; 0     */
                        /*   gives the paper's cost (not in the paper; for the       */
                        /*   adjoint of asicp_cost_grad)                             */
  int32_t minibatch;    /* 0: the whole object cloud; 1: a mini-batch per iteration  */
                        /*   of size M min(k, 2 k_max/3) / (2 k_max/3) (>= 1),       */
                        /*   Table I, drawn by a keyed permutation from `seed`       */
  uint64_t seed;        /* mini-batch seed                                           */
  uint32_t flags;       /* ASICP_FLAG_*                                              */
} asicp_config;

/* Outputs.  Every pointer may be NULL.  Host arrays hold n_objects entries
 * (best_theta 7 per object); device arrays use Ktot = n_objects*n_preshapes*K,
 * G = n_objects*n_preshapes, Nmax = largest preshape, Mcmax = largest
 * collision cloud.  Per-particle values are those of the last evaluation:
 * after asicp_step, the evaluation that the last update used; after
 * asicp_solve, the final evaluation at theta_{k_max}. */
typedef struct {
  /* host */
  int32_t* best_particle;   /* [n_objects] particle index i of the returned grasp       */
  int32_t* best_free;       /* [n_objects] 1 if it is collision free, 0 if none was     */
  float* best_theta;        /* [7*n_objects]                                            */
  float* best_cost;         /* [n_objects]                                              */
  int32_t iterations_done;  /* out: the next iteration to run                           */
  int32_t final_evaluated;  /* out: 1 once asicp_solve has run the final evaluation     */
  /* device */
  float* theta;             /* [7][Ktot] current poses                                  */
  float* cost;              /* [Ktot] C = 1/2 (L_ct + lambda L_com), eqs. (13)-(15)     */
  float* col_cost;          /* [Ktot] 1/2 L_col of eq. (18); 0 without collision        */
  int32_t* ncol;            /* [Ktot] colliding points                                  */
  int32_t* converged;       /* [Ktot]                                                   */
  float* prev_cost;         /* [Ktot]                                                   */
  float* grad;              /* [6][Ktot] gradient used: (g_t, g_w), collision if ncol>0 */
  float* grad_ct;           /* [6][Ktot] gradient of C                                  */
  float* grad_col;          /* [6][Ktot] gradient of 1/2 L_col                          */
  float* phi;               /* [6][Ktot] last update direction (Stein phi, or -A g)     */
  float* h;                 /* [G] last bandwidth (0 in the SGD phase)                  */
  int32_t* nn_idx;          /* [Ktot][Nmax] forward NN index per contact point (DEBUG)  */
  int32_t* rev_idx;         /* [Ktot][Mcmax] reverse NN index, -1 if the point does not */
                            /*   collide (DEBUG)                                        */
} asicp_result_t;

typedef struct asicp_ctx_s* asicp_ctx;

/* Workspace size for this problem and config (host only, no device work). */
asicp_status asicp_workspace_bytes(const asicp_problem* pb, const asicp_config* cfg, size_t* bytes);

/* Validate everything on the host (ASICP_E_INVALID before any device work),
 * carve the workspace and enqueue the per-object / per-preshape set-up on
 * `stream`: centre of mass of each object cloud, tool centre point (centroid
 * of each contact cloud), preconditioner, MFMA-ready copies of the clouds,
 * and the particle state from theta0 (and the resume arrays).  `*out` is
 * library-owned host memory released by asicp_destroy.  The workspace is
 * borrowed like the problem's device arrays. */
asicp_status asicp_create(const asicp_problem* pb, const asicp_config* cfg, void* workspace,
                          size_t workspace_bytes, void* stream, asicp_ctx* out);

/* Enqueue the set-up again from the borrowed inputs (which the caller may
 * have rewritten in place: a new object of the same size, new initial
 * particles) and return the context to the state asicp_create left it in:
 * the next iteration is k_start, no final evaluation.  Launch choices and
 * timing records are kept.  Reusing one context this way keeps its side
 * stream and avoids creating contexts per solve. */
asicp_status asicp_reset(asicp_ctx ctx, void* stream);

/* Enqueue n_iters iterations of Algorithm 1 (n_iters >= 0).  Running past
 * k_max, or stepping after the final evaluation, is ASICP_E_STATE. */
asicp_status asicp_step(asicp_ctx ctx, int32_t n_iters, void* stream);

/* Enqueue the remaining iterations, the final evaluation at theta_{k_max} and
 * the selection of the returned grasp per object. */
asicp_status asicp_solve(asicp_ctx ctx, void* stream);

/* Gradient forms of asicp_cost_grad. */
#define ASICP_GRAD_TANGENT 0 /* [6][Ktot]: d/dt, then d/dw for the world rotation vector w  */
                             /*   about the gripper origin (q <- Exp(w) q), eqs. (16)-(17)  */
#define ASICP_GRAD_POSE 1    /* [7][Ktot]: d/dt, then d/dq with the cost a function of the  */
                             /*   unit quaternion q / |q|: 2 M(q) g_w, M(q) = [-q_v^T ;     */
                             /*   q_w I - [q_v]x] (the tangent of unit quaternions, eq. 17) */

/* Per-particle cost and its gradient at arbitrary poses: the adjoint of the
 * iteration's cost with respect to each pose.  `theta` (device [7][Ktot])
 * replaces the context's poses; the cost C = 1/2 (L_ct + lambda L_com) of
 * eqs. (13)-(15), plus the penetration term when w_pen > 0, and its gradient
 * in the form `grad_form` (ASICP_GRAD_*), with nearest-neighbour pairs and
 * gate decisions held at `theta`, go to cost_out (device [Ktot]) and grad_out
 * (device, [6][Ktot] or [7][Ktot]); either may be NULL.  Enqueued on
 * `stream`. */
asicp_status asicp_cost_grad(asicp_ctx ctx, const float* theta, float* cost_out, float* grad_out,
                             int32_t grad_form, void* stream);

/* Vector-Jacobian product of the per-particle costs for reverse-mode
 * differentiation: dtheta[a][i] = gout[i] * grad[a][i] for a < 7 (device
 * arrays; grad from asicp_cost_grad with ASICP_GRAD_POSE, gout [Ktot], dtheta
 * [7][Ktot], which may alias grad).  ktot >= 0.  Enqueued on `stream`. */
asicp_status asicp_pose_vjp(const float* grad, const float* gout, float* dtheta, int32_t ktot, void* stream);

/* Run the whole solve again as one HIP graph on `stream`: set-up from the
 * borrowed inputs (which the caller may have rewritten in place: a new object
 * of the same size, new initial particles), iterations k_start .. k_max-1,
 * the final evaluation and the selection.  The graph is captured on the first
 * call (on private streams kept with the graph; `stream` may be the null
 * stream) and replayed after, so repeated solves pay no per-kernel launch
 * cost.  Afterwards the context is in the state
 * asicp_solve leaves it in.  Not available with ASICP_FLAG_DEBUG
 * (ASICP_E_STATE); ASICP_FLAG_TIMING events are not recorded inside the graph. */
asicp_status asicp_replay(asicp_ctx ctx, void* stream);

/* Launch choices that change no result: how work is placed on the XCDs, how
 * much provably useless work the pruned nearest-neighbour search skips, and
 * the forward NN's shape (queries per wavefront, points per pruning chunk).
 * Every choice returns bit-identical outputs; only the speed differs. */
typedef struct {
  int32_t xcd_map;       /* 0: forward NN: whole particles' work dealt round-robin   */
                         /*    over the XCDs (each particle in one L2, every XCD a    */
                         /*    mix of near and far particles); collision gate: each   */
                         /*    XCD takes a contiguous range of its work;              */
                         /* 1: dispatch order (consecutive work on different XCDs).   */
                         /*    Default 1.                                             */
  int32_t fine;          /* forward NN: test each candidate chunk against every      */
                         /*    query's own bound (1) or only the query block's (0).   */
                         /*    Default 1.                                             */
  int32_t query_blocks;  /* forward NN: blocks of 16 contact points per wavefront,    */
                         /*    1, 2 or 4 (fewer: more wavefronts for small problems). */
                         /*    Default 4.                                             */
  int32_t chunk_points;  /* forward NN: object points per pruning chunk, 64 or 128.   */
                         /*    Default 128.                                           */
} asicp_launch_t;

/* Number of launch choices, and the index of one in asicp_autotune's ms_out:
 * ((qi * 2 + (chunk_points == 128)) * 2 + xcd_map) * 2 + fine, with qi = 0, 1,
 * 2 for query_blocks = 1, 2, 4. */
#define ASICP_LAUNCH_CHOICES 24

/* Read or set the launch choices of a context (set: xcd_map and fine 0 or 1,
 * query_blocks 1, 2 or 4, chunk_points 64 or 128, else ASICP_E_INVALID).
 * Setting them discards a captured asicp_replay graph. */
asicp_status asicp_get_launch(asicp_ctx ctx, asicp_launch_t* out);
asicp_status asicp_set_launch(asicp_ctx ctx, const asicp_launch_t* in);

/* Time every launch choice on the context's current poses (`reps`
 * evaluations each after one warm-up, HIP events on `stream`; an evaluation
 * runs the forward NN on `stream` beside the bandwidth select, in the Stein
 * phase, and the collision kernel on the context's side stream, as an
 * iteration does), keep the fastest and return it in `chosen` (may be
 * NULL); ms_out (host, may be NULL, ASICP_LAUNCH_CHOICES floats) receives the
 * average time per evaluation of each choice at the index given above.
 * Synchronises `stream`.  The solve's state is left as it was (tuning
 * launches are not counted by asicp_kernel_time); a captured asicp_replay
 * graph is discarded.  Results never depend on the choice, so tuning cannot
 * change what a solve returns. */
asicp_status asicp_autotune(asicp_ctx ctx, int32_t reps, void* stream, asicp_launch_t* chosen,
                            float* ms_out);

/* Synchronise `stream`, then fill `out` (see asicp_result_t).  Device outputs
 * are copied on `stream` before it is synchronised.  Returns ASICP_E_HIP for
 * an asynchronous HIP error and ASICP_E_NUMERIC if the device flagged a
 * non-finite pose, cost or gradient (the outputs are still written). */
asicp_status asicp_result(asicp_ctx ctx, asicp_result_t* out, void* stream);

/* With ASICP_FLAG_TIMING: total time and count of the forward-NN kernel
 * launches enqueued so far by asicp_step / asicp_solve / asicp_cost_grad,
 * from HIP events recorded on the launch stream
 * around each launch, and (nn_pairs, may be NULL) the number of (contact
 * point, object point) distances those launches evaluated (each forward
 * wave counts into a slot of its own, summed here on the host).
 * Synchronises on the events. */
asicp_status asicp_kernel_time(asicp_ctx ctx, double* total_ms, int32_t* launches, double* nn_pairs);

/* Release the context (host memory and HIP events only). NULL is a no-op. */
void asicp_destroy(asicp_ctx ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* asicp_last_error(void);

/* ---------------------------------------------------------------------------
 * Learned grasp proposal (seeds for the iteration above).  The paper points to
 * learned priors and data-driven seeding as the way to need fewer
 * initialisations (Sec. V, the ablation; Sec. VII); this network and its training
 * are the library's own.  A max-pooled point encoder, 3 -> 64 -> 128 -> 256
 * per point (BF16 matrix products, FP32 accumulation) and a 256 -> 256 -> 256
 * -> n_pre * n_seed * 7 head, maps each object cloud to n_seed seed poses per
 * preshape: t = mean(cloud) + 0.1 o[0:3] (metres), q = o[3:7] / |o[3:7]|.
 *
 * Parameters: one FP32 device array of asicp_pn_param_count() floats in the
 * order W1 (64x3), b1, W2 (128x64), b2, W3 (256x128), b3, W4 (256x256), b4,
 * W5 (256x256), b5, W6 (O x 256), b6, O = n_pre * n_seed * 7, matrices
 * row-major (output index first).  Clouds: device SoA x, y, z, concatenated;
 * off (HOST) [n_obj + 1] point offsets, off[0] = 0, 1..4194304 points each.
 * The workspace (device, caller-owned, asicp_pn_workspace_bytes) holds every
 * intermediate; nothing is allocated.  All calls are enqueued on `stream`.
 * Errors: ASICP_E_INVALID (arguments, checked on the host), ASICP_E_HIP
 * (launch failures); message in asicp_pn_last_error(). */

/* Parameter floats for n_pre preshapes and n_seed seeds (-1 if
 * n_pre * n_seed * 7 is not in 7..1024). */
int64_t asicp_pn_param_count(int32_t n_pre, int32_t n_seed);

/* Workspace bytes for n_obj objects (1..65536). */
asicp_status asicp_pn_workspace_bytes(int32_t n_obj, int32_t n_pre, int32_t n_seed, size_t* bytes);

/* Forward pass.  seeds (device, may be NULL): [7][n_obj * n_pre * n_seed]
 * poses (tx ty tz qw qx qy qz, q_w >= 0), particle order (object, preshape,
 * seed) -- the layout of asicp_problem.theta0 -- each backed off by
 * `retract` metres along its approach axis (the gripper's +z, R(q) e_z), so
 * that a seed predicted on the surface starts clear of it.  raw (device,
 * may be NULL): [n_obj][n_pre * n_seed * 7] network outputs. */
asicp_status asicp_pn_forward(const float* params, int32_t n_pre, int32_t n_seed, int32_t n_obj,
                              const int32_t* off, const float* x, const float* y, const float* z,
                              float retract, float* seeds, float* raw, void* workspace, size_t ws_bytes,
                              void* stream);

/* asicp_pn_forward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results as
 * asicp_pn_forward; every intermediate lives in a device array inside the
 * library instead (1 MiB per device, held by each device the library runs
 * on until the process ends).  Nothing is allocated: no hipMalloc, hipFree
 * or allocating library routine.  Limit: at most 64 objects per call
 * (ASICP_E_INVALID beyond it, checked on the host before any device work).
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (the pass clears what it accumulates into): calls that
 * overlap on one device -- on different streams or host threads without
 * ordering between them -- race and give undefined results. */
asicp_status asicp_pn_forward_noalloc(const float* params, int32_t n_pre, int32_t n_seed, int32_t n_obj,
                                      const int32_t* off, const float* x, const float* y, const float* z,
                                      float retract, float* seeds, float* raw, void* stream);

/* Set loss per object against targets (device [n_obj][n_pre][n_targets][7]
 * poses, unit q): per preshape the symmetric Chamfer distance
 * (1/T) sum_g min_a d + (1/S) sum_a min_g d with
 * d = |t_a - t_g|^2 / 0.01 + (1 - (q_a . q_g)^2), averaged over preshapes ->
 * loss (device [n_obj]).  grad (device, param_count floats) receives the
 * gradient of the mean loss over the objects, summed in a fixed order. */
asicp_status asicp_pn_loss_grad(const float* params, int32_t n_pre, int32_t n_seed, int32_t n_obj,
                                const int32_t* off, const float* x, const float* y, const float* z,
                                const float* targets, int32_t n_targets, float* loss, float* grad,
                                void* workspace, size_t ws_bytes, void* stream);

/* One Adam step (Kingma and Ba, 2015) on `count` parameters, step >= 1 (bias
 * corrections 1 - beta^step); m and v are the caller's moment buffers. */
asicp_status asicp_pn_adam(float* params, float* m, float* v, const float* grad, int64_t count, float lr,
                           float beta1, float beta2, float eps, int32_t step, void* stream);

/* Message of the last failed asicp_pn_* call on this thread. */
const char* asicp_pn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ASICP_H */
