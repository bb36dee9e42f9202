/*
 * cadmm.h -- C ABI of the MI355X (gfx950) ADMM collision-avoidance library.
 *
 * Method: "GPU-Accelerated Optimization-Based Collision Avoidance"
 * (arXiv 2406.07048). Robot = union of convex polytope parts {x : A_i x <= b_i}
 * posed by the state through R(s), rho(s) (Sec. IV-A); obstacles = union of
 * polytopes {y : C_j y <= d_j} (Sec. IV-A); collision-free constraint from the
 * dual of the scale LP (Sec. III-B, eq. poly_colli_free_conts); MPC problem
 * (Sec. IV-A, eq. MPC_opt_origin) split by ADMM (Sec. IV-B) into
 *   (1) one small QP per (time step t, part i, obstacle j)  (eq. ADMM_dual_updates,
 *       in the form of Sec. IV-C eq. const_least_square),
 *   (2) one trajectory QP with R(s), rho(s) linearised at the current iterate
 *       (eq. ADMM_state_updates, one SQP step per iteration),
 *   (3) the scaled-multiplier update (eq. ADMM_residue_updates),
 * stopped by the sums of squared changes of Sec. IV-B.
 *
 * Readings fixed by this library where the paper is silent:
 *  - The dual-update QP carries a proximal term (eps/2) sum_l D_l (y_l - yhat_l)^2
 *    with yhat the previous iterate and D_l = ||row_l K||^2, which makes every
 *    sub-problem solution unique and vanishes at ADMM fixed points.
 *  - Each robot part i is scaled about its own centre o_i (body frame);
 *    world pose of part i: y = R(s)(x + o_i) + rho(s). Requires b_i > 0.
 *  - Collision pairs exist for t = 1..N (x_0 is fixed data); cost
 *    F = sum_{t=1..N} (x_t - xref_t)^T Q_s (x_t - xref_t) + sum_{t=0..N-1} u_t^T Q_u u_t.
 *  - Dynamics (Sec. IV-A eq. system_eqn, s_{t+1} = s_t + f(s_t, u_t)) are either
 *    given already linearised, x_{t+1} = A_t x_t + B_t u_t + c_t (time-invariant,
 *    per step or per scenario and step), or one of the built-in nonlinear f
 *    (kinematic bicycle, quadrotor), linearised about the current iterate at
 *    every ADMM iteration: the one SQP step per iteration of Sec. IV-B.
 *  - Initial iterate: obstacle-free LQ trajectory; zeta = xi = 0;
 *    y = (lam*, mu*, max(alpha* - 1, 0)) from the scale LP.
 *
 * Conventions
 *  - All functions return an int status (CADMM_OK = 0 on success); no
 *    exception or abort crosses the ABI. cadmm_strerror(code) gives the
 *    meaning, cadmm_last_error() the detail of the last failure.
 *  - Device memory always belongs to the caller (workspace and every I/O
 *    buffer). The library allocates host memory for handles only.
 *  - Computation is FP32 on the device. Host descriptors are FP64.
 *  - A handle is bound to one stream and is not thread-safe.
 *
 * Canonical pair layout (used by every state buffer below)
 *  - Pair blocks b enumerate (scenario s, part i, obstacle j) in that nesting
 *    order (j runs over the scenario's obstacles). Block b holds the N pairs
 *    t = 1..N and has n_b = n_r,i + n_o,j + 1 dual rows (lambda, mu, gamma).
 *  - y: block b occupies n_b * N floats starting at y_off(b) =
 *    N * sum_{b' < b} n_b', row-major [row][t-1].
 *  - zeta[b*N + t-1]; xi[(b*dim + c)*N + t-1]; alpha[b*N + t-1].
 *  - x[(s*(N+1) + t)*n_s + k] for t = 0..N; u[(s*N + t)*n_u + k] for t = 0..N-1.
 */
#ifndef CADMM_H
#define CADMM_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CADMM_OK = 0,
    CADMM_INVALID = 1,        /* bad descriptor: sizes, b_i <= 0, non-finite, zero normal, ... */
    CADMM_DEVICE = 2,         /* a HIP call failed (detail in cadmm_last_error) */
    CADMM_WORKSPACE = 3,      /* workspace too small or misaligned */
    CADMM_NOT_CONVERGED = 4   /* warning from admm_solve: outputs are written */
};

enum { CADMM_ATT_YAW = 0, CADMM_ATT_EULER_ZYX = 1 };

/* Dynamics models (cadmm_desc.model). */
enum { CADMM_MODEL_LINEAR = 0, CADMM_MODEL_BICYCLE = 1, CADMM_MODEL_QUADROTOR = 2 };

/* Limits of this build. */
#define CADMM_MAX_N 64           /* horizon */
#define CADMM_MAX_NS 16          /* state size */
#define CADMM_MAX_NU 8           /* input size */
#define CADMM_MAX_PART_FACES 8   /* faces of one robot part */
#define CADMM_MAX_OBS_FACES 32   /* faces of one obstacle */
#define CADMM_MAX_ACTIVE_BOUNDS 64   /* bounds active at once in one scenario's trajectory QP */

/*
 * Problem descriptor. Host pointers, read only during collision_admm_setup.
 *  dim           spatial dimension, 2 (planar, attitude = yaw) or 3 (ZYX Euler)
 *  n_s, n_u, N   state size, input size, horizon (1..CADMM_MAX_N)
 *  n_parts, part_face_ptr[n_parts+1], part_A[F_r*dim], part_b[F_r] (> 0),
 *      part_off[n_parts*dim]        robot parts {x : A_i x <= b_i}, centre o_i
 *                                   (1 <= n_parts <= 32767)
 *  n_scen, obs_ptr[n_scen+1]        obstacles of scenario s: obs_ptr[s]..obs_ptr[s+1]-1
 *  obs_face_ptr[M+1], obs_C[F_o*dim], obs_d[F_o]   obstacles {y : C_j y <= d_j}
 *  A_dyn[n_models*n_s*n_s], B_dyn[n_models*n_s*n_u], c_dyn[n_models*n_s]
 *                 linear models x_{t+1} = A x_t + B u_t + c (row-major); step t
 *                 (0..N-1) of scenario s uses model s*dyn_s_stride + t*dyn_t_stride,
 *                 n_models = (n_scen-1)*dyn_s_stride + (N-1)*dyn_t_stride + 1
 *                 (both strides 0: one time-invariant model)
 *  pos_idx[dim], att_idx[1|3], att_kind            state indices of rho(s) and attitude
 *  Q_s[n_s*n_s], Q_u[n_u*n_u] (symmetric), x_ref[n_scen*(N+1)*n_s], x0[n_scen*n_s]
 *  sigma (ADMM penalty), eps_prox (proximal weight), eps_pri, eps_dual (stop test;
 *                 a negative value never holds, so every iteration runs)
 *  max_sweeps     Newton sweep budget of each pair QP (0 = default 24)
 *  waves_per_group  pair blocks per workgroup of the pair kernels (0 = autotune, else 1..8)
 *  lanes_per_pair   lanes that share one pair QP in the pair phase (0 = autotune, else 1, 2, 4);
 *                   a block then spans ceil(N / (64 / lanes_per_pair)) waves, and
 *                   waves_per_group times that may not exceed 8
 *  dyn_t_stride, dyn_s_stride   model strides (>= 0), see A_dyn
 *  model          CADMM_MODEL_LINEAR: the linear models above are the dynamics.
 *                 CADMM_MODEL_BICYCLE (dim 2, n_s 4 = (p_x, p_y, theta, v), n_u 2 =
 *                 (a, delta); model_par = (dt, wheelbase)) or CADMM_MODEL_QUADROTOR
 *                 (dim 3, n_s 12 = (p, v, phi theta psi, body rates), n_u 4 =
 *                 (thrust change, torques); model_par = (dt, mass, J_x, J_y, J_z, g)):
 *                 s_{t+1} = s_t + dt f_c(s_t, u_t) with that f_c, linearised about
 *                 the current iterate at every ADMM iteration (the SQP step of
 *                 Sec. IV-B); the linear models then only give the initial
 *                 (obstacle-free) trajectory. The reverse pass (admm_record,
 *                 admm_backward) needs CADMM_MODEL_LINEAR.
 *  model_par[8]   parameters of the nonlinear model (unused for CADMM_MODEL_LINEAR)
 *  s_min[n_s], s_max[n_s], u_min[n_u], u_max[n_u]
 *                 state and input bounds of Sec. IV-A eq. MPC_opt_origin (its state
 *                 and control rows), s_min <= x_t <= s_max for t = 1..N and
 *                 u_min <= u_t <= u_max for t = 0..N-1, in every scenario; each
 *                 array may be NULL and each entry +-INFINITY (no bound); min <= max
 *                 required. With any finite bound the trajectory QP of every
 *                 iteration (and the initial obstacle-free trajectory) is the
 *                 bounded QP, solved to the bounded minimiser (the indicator IC_0 of
 *                 Sec. IV-B eq. ADMM_Lagrangian); needs n_s <= 12, n_u <= 4, at most
 *                 CADMM_MAX_ACTIVE_BOUNDS bounds active at once per scenario
 *                 (cadmm_result.active_bounds reports -2 beyond), and no reverse pass.
 */
typedef struct cadmm_desc {
    int dim, n_s, n_u, N;
    int n_parts;
    const int* part_face_ptr;
    const double* part_A;
    const double* part_b;
    const double* part_off;
    int n_scen;
    const int* obs_ptr;
    const int* obs_face_ptr;
    const double* obs_C;
    const double* obs_d;
    const double* A_dyn;
    const double* B_dyn;
    const double* c_dyn;
    const int* pos_idx;
    const int* att_idx;
    int att_kind;
    const double* Q_s;
    const double* Q_u;
    const double* x_ref;
    const double* x0;
    double sigma, eps_prox, eps_pri, eps_dual;
    int max_sweeps;
    int waves_per_group;
    int lanes_per_pair;
    int dyn_t_stride, dyn_s_stride;
    int model;
    double model_par[8];
    const double* s_min;
    const double* s_max;
    const double* u_min;
    const double* u_max;
} cadmm_desc;

typedef struct cadmm_handle cadmm_handle;

/* Per-scenario outcome of admm_solve (host struct, one per scenario). */
typedef struct cadmm_result {
    int iters;                 /* iterations this scenario ran */
    int converged;             /* 1 if the stopping test of Sec. IV-B held */
    float r_pri, r_dual;       /* last sums of squared multiplier / dual changes */
    float cost;                /* tracking cost F of the final trajectory */
    float min_alpha;           /* min scale alpha* over the scenario's pairs at the final trajectory */
    int unconverged_pairs;     /* pair QPs that hit the sweep budget in the last iteration */
    int active_bounds;         /* bounds active in the last trajectory QP (0 without bounds);
                                  -1: no point met the bounds (the iterate then breaks some),
                                  -2: more than CADMM_MAX_ACTIVE_BOUNDS were needed,
                                  -3: the active-set step cap was reached */
} cadmm_result;

/* Size info of a descriptor: bytes of device workspace, number of pair
 * blocks, number of pairs, and floats of y (canonical layout). Any output
 * pointer may be NULL. Validates the descriptor (CADMM_INVALID). */
int cadmm_workspace_size(const cadmm_desc* desc, size_t* bytes, int* n_blocks,
                         long long* n_pairs, long long* y_floats);

/* Validates desc, uploads it into the caller's device workspace d_ws
 * (bytes >= cadmm_workspace_size, 256-byte aligned), builds the work lists,
 * captures the iteration as a HIP graph and initialises the iterate (obstacle-
 * free LQ trajectory, scale-LP certificates, zero multipliers) on stream.
 * On success *out receives a handle owned by the caller (free with
 * collision_admm_destroy). The workspace must outlive the handle. */
int collision_admm_setup(const cadmm_desc* desc, void* d_ws, size_t bytes,
                         hipStream_t stream, cadmm_handle** out);

/* Enqueue n_iters ADMM iterations (Sec. IV-B: pair QPs, trajectory QP,
 * multiplier update, residuals) on the handle's stream. No host sync.
 * Scenarios whose stopping test has held are left unchanged. */
int admm_iterate(cadmm_handle* h, int n_iters);

/* Iterate until every scenario met the stopping test or max_iters
 * iterations; reads the device convergence flags every check_every
 * iterations (the only device-to-host syncs; check_every <= 0 means 8).
 * The next chunk of iterations is queued before the flags of the previous
 * one are read, so one more chunk may run after every scenario stopped; it
 * changes nothing (stopped scenarios are left unchanged) and the total never
 * exceeds max_iters. Fills out[n_scen] and returns CADMM_OK, or
 * CADMM_NOT_CONVERGED (outputs still written). */
int admm_solve(cadmm_handle* h, int max_iters, int check_every, cadmm_result* out);

/* Reset the iterate to the initial one of setup (same device work as setup). */
int admm_reset(cadmm_handle* h);

/* Copy the iterate out of (get) or into (set) caller-owned DEVICE buffers in
 * the canonical layout; any pointer may be NULL to skip that part. Enqueued on
 * the handle's stream. set also clears the per-scenario stop flags. */
int admm_get_state(cadmm_handle* h, float* x, float* u, float* y, float* zeta, float* xi);
int admm_set_state(cadmm_handle* h, const float* x, const float* u, const float* y,
                   const float* zeta, const float* xi);

/* Residual history: host buffers of max_iters*n_scen floats receive r_pri and
 * r_dual per iteration (row k, column s; NaN where a scenario had stopped).
 * Returns the number of rows written. Syncs the stream. */
int admm_get_history(cadmm_handle* h, int max_rows, float* r_pri, float* r_dual);

/* Scale alpha* of every pair at the current trajectory (Sec. III-A eq.
 * scale_opt), written to a caller DEVICE buffer alpha[n_pairs] (canonical). */
int admm_scales(cadmm_handle* h, float* alpha);

/* Profiling: run n_iters iterations with eager (non-graph) launches and
 * events recorded around each kernel's own execution (hipExtLaunchKernel)
 * on the handle's stream, one set per iteration, read after one
 * synchronisation at the end; ms_out[4] receives the mean milliseconds of
 * (pair QPs + contributions, trajectory QP, multiplier update, residual
 * test). The durations include the dispatch overhead the events carry (a
 * few microseconds above a profiler's kernel times). Advances the iterate.
 * Syncs. */
int admm_phase_times(cadmm_handle* h, int n_iters, float* ms_out);

/* Launch shape chosen at setup (autotuned unless fixed in the descriptor):
 * pair blocks per workgroup, number of workgroups and lanes per pair QP of
 * the pair phase. Any output pointer may be NULL. */
int admm_launch_config(cadmm_handle* h, int* waves_per_group, int* n_workgroups, int* lanes_per_pair);

/* Replace the obstacle face offsets d (host FP64, F_o values in obs_face_ptr
 * order) and/or the initial states x0 (host FP64, n_scen*n_s); NULL keeps the
 * current values. The iterate is not touched: call admm_reset (or
 * admm_record) to start from the new data. Syncs the stream. */
int admm_set_params(cadmm_handle* h, const double* obs_d, const double* x0);

/* Restart the pair iterate at the current trajectory: y = (lam*, mu*,
 * max(alpha* - 1, 0)) from the scale LP of every pair (Sec. III-B eq.
 * scale_opt_dual) at the handle's current x, zeta = xi = 0, stop flags
 * cleared; x and u are kept. The initialisation of setup, applied to a
 * trajectory set with admm_set_state (a warm start). Enqueued on the
 * handle's stream. */
int admm_reset_duals(cadmm_handle* h);

/* Replace the reference trajectory x_ref (host FP64, n_scen*(N+1)*n_s, as in
 * the descriptor) for the following iterations; the iterate is not touched.
 * With admm_set_params (new x0) and admm_set_state (a shifted warm start)
 * this moves a handle from one receding-horizon cycle to the next. Syncs the
 * stream. */
int admm_set_reference(cadmm_handle* h, const double* x_ref);

/* One step of a built-in nonlinear model on the host, in FP64:
 * s_next = s + dt f_c(s, u) (Sec. IV-A eq. system_eqn; the models and
 * model_par as in cadmm_desc.model); the plant of a simulated closed loop.
 * s, s_next: n_s values, u: n_u values (host). CADMM_INVALID for
 * CADMM_MODEL_LINEAR or non-finite input. */
int cadmm_model_step(int model, const double* model_par, const double* s, const double* u, double* s_next);

/*
 * Differentiation through the unrolled iteration. The differentiated map is
 *     L(d, x0) = sum_s F_s(x^K, u^K),
 * the tracking cost (Sec. IV-A eq. navigation_cost) after exactly K
 * iterations of Sec. IV-B (no stopping test) from s^0 = the obstacle-free LQ
 * trajectory of x0, zeta^0 = xi^0 = 0 and the dual iterate y^0 that the handle
 * holds when admm_record is called (after admm_reset: the scale-LP
 * certificates at s^0). y^0 is held fixed: its dependence on (d, x0) is not
 * differentiated. Each pair QP is differentiated on its free set
 * {l : y_l > 0}; where a dual is exactly zero with a zero multiplier the
 * map has a kink and the one-sided derivative of that active set is taken.
 *
 * admm_grad_workspace_size: bytes of the caller-owned DEVICE gradient
 *   workspace for K = n_iters iterations with a checkpoint of the iterate
 *   (x, u, y, zeta, xi) every ckpt_every iterations; it grows like
 *   (K / ckpt_every + ckpt_every) iterates.
 * admm_record: runs the K iterations on the handle's stream (graph replay),
 *   keeping the checkpoints in d_gws (256-byte aligned, >= the size above),
 *   and leaves the handle at iterate K; cost_out (DEVICE, n_scen floats, may
 *   be NULL) receives F_s(x^K, u^K). No host sync.
 * admm_backward: the reverse pass over the run recorded in d_gws (same
 *   pointer): each segment of ckpt_every iterations is replayed from its
 *   checkpoint (bitwise identical to the recorded run) and reversed step by
 *   step. Writes dL_scale * dL/dd to grad_d[F_o] and dL_scale * dL/dx0 to
 *   grad_x0[n_scen*n_s] (DEVICE FP32, overwritten). Leaves the handle at
 *   iterate K. No host sync. CADMM_INVALID if nothing was recorded in d_gws.
 * All three return CADMM_INVALID for a nonlinear model (desc.model != 0) or
 * with state or input bounds.
 */
int admm_grad_workspace_size(cadmm_handle* h, int n_iters, int ckpt_every, size_t* bytes);
int admm_record(cadmm_handle* h, int n_iters, int ckpt_every, void* d_gws, size_t bytes, float* cost_out);
int admm_backward(cadmm_handle* h, void* d_gws, size_t bytes, float dL_scale, float* grad_d, float* grad_x0);

void collision_admm_destroy(cadmm_handle* h);

/* Solvers of the stateless pair-QP batch (cadmm_pair_batch.solver). */
enum { CADMM_PAIR_NEWTON = 0, CADMM_PAIR_LEMKE = 1 };

/*
 * Stateless batch of dual-update QPs (Sec. IV-C eq. const_least_square with
 * the proximal term): for each pair p with rows l in row_ptr[p]..row_ptr[p+1]-1
 *     min_y 1/2 ||K^T y + bhat||^2 + eps/2 sum_l ||K_l||^2 (y_l - yhat_l)^2
 *     s.t.  kappa^T y = 1,  y >= 0.
 * All pointers are DEVICE pointers, caller-owned:
 *   row_ptr[n_pairs+1] (int), K[rows*(dim+1)] row-major, kappa[rows] (>= 0, at
 *   least one > 0 per pair), yhat[rows], bhat[n_pairs*(dim+1)]
 *   outputs y[rows], r[n_pairs*(dim+1)] = K^T y + bhat, nu[n_pairs] (the
 *   multiplier of kappa^T y = 1 in the stationarity condition
 *   K r + eps D (y - yhat) - nu kappa - w = 0, w >= 0, w^T y = 0), status[n_pairs]
 *   (sweeps used, -1 if the sweep budget ran out, -3 if the pair holds more
 *   rows than the solver's row tile).
 * A pair may hold at most CADMM_MAX_PART_FACES + CADMM_MAX_OBS_FACES + 1 rows.
 * solver: CADMM_PAIR_NEWTON, the dual semismooth Newton method in the
 *   (dim+2)-dimensional dual (one lane per pair; max_sweeps 0 = 24); or
 *   CADMM_PAIR_LEMKE, the route of Sec. IV-C: the equality variable with the
 *   largest kappa eliminated (eq. const_least_square_ineq), the KKT
 *   conditions as an LCP (eq. linear_complementarity_problem, the proximal
 *   term carried through the elimination) solved by Lemke's complementary
 *   pivoting, one wavefront per pair; max_sweeps then bounds the pivots
 *   (0 = 200), status holds the pivots used or -1 (secondary ray), -2 (pivot
 *   budget), -3 (rows outside 2..CADMM_MAX_PART_FACES + CADMM_MAX_OBS_FACES + 1).
 * work, work_bytes: optional caller-owned DEVICE workspace (256-byte aligned,
 *   work_bytes >= pair_qp_batch_workspace_size) for the dual Newton solver's
 *   two-launch form: a wavefront runs as long as its slowest pair, so the
 *   first launch stops every solve after three sweeps and queues the
 *   unfinished ones, which a second launch resumes one per lane. The outputs
 *   are bitwise those of the one-launch form (NULL work). Ignored by Lemke.
 */
typedef struct cadmm_pair_batch {
    int n_pairs, dim;
    const int* row_ptr;
    const float* K;
    const float* kappa;
    const float* yhat;
    const float* bhat;
    float eps;
    int max_sweeps;
    float* y;
    float* r;
    float* nu;
    int* status;
    int solver;
    void* work;
    size_t work_bytes;
} cadmm_pair_batch;

int pair_qp_batch(const cadmm_pair_batch* b, hipStream_t stream);

/* Bytes of the workspace of pair_qp_batch's two-launch form for n_pairs pairs
 * (a counter and one queue entry per pair). */
int pair_qp_batch_workspace_size(int n_pairs, size_t* bytes);

/* Largest batch of pair_qp_batch_noalloc. */
#define CADMM_NOALLOC_MAX_PAIRS (1 << 19)

/*
 * pair_qp_batch (dual Newton solver, two-launch form) with the library's own
 * device buffer in place of b->work, for callers that cannot allocate device
 * memory (code under HIP-graph capture, tight serving loops): it calls no
 * allocating routine. The buffer is a static device array of 24 MB, one per
 * GPU, held until the process ends; its address is looked up on the first
 * call on each device. Every call on a GPU shares that GPU's buffer, so calls
 * that overlap on one GPU (other streams, other threads) race; calls on one
 * stream do not. b->work, b->work_bytes and b->solver are ignored. Returns
 * CADMM_INVALID for more than CADMM_NOALLOC_MAX_PAIRS pairs (and as
 * pair_qp_batch), CADMM_DEVICE if the buffer's address cannot be found.
 */
int pair_qp_batch_noalloc(const cadmm_pair_batch* b, hipStream_t stream);

/*
 * Stateless batch of scale LPs (Sec. III-A eq. scale_opt and its dual Sec.
 * III-B eq. scale_opt_dual) in the robot part's frame:
 *     alpha* = min alpha  s.t.  A x <= alpha b,  Cp x <= dp.
 * DEVICE pointers: a_ptr[n_pairs+1], A[ra*dim], b[ra] (> 0);
 *   o_ptr[n_pairs+1], Cp[ro*dim], dp[ro]; outputs alpha[n_pairs],
 *   lam[ra], mu[ro] (the dual certificate), status[n_pairs] (0 ok).
 */
typedef struct cadmm_scale_batch {
    int n_pairs, dim;
    const int* a_ptr;
    const float* A;
    const float* b;
    const int* o_ptr;
    const float* Cp;
    const float* dp;
    float* alpha;
    float* lam;
    float* mu;
    int* status;
} cadmm_scale_batch;

int pair_scale_batch(const cadmm_scale_batch* b, hipStream_t stream);

const char* cadmm_strerror(int code);
const char* cadmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CADMM_H */
