/*
 * cord.h - C ABI of libcord: batched, differentiable rope and cloth
 * simulation with smoothed contact on AMD Instinct MI355X (gfx950).
 *
 * The operations follow the simulator of "Robustness without Wrinkles:
 * Parallel Simulation and Robust MPC for Certified Deformable Manipulation"
 * (CORD-SLS):
 *   - Sec. 3, Problem 1 / eq. (dynamics_sim): the planner dynamics
 *     q_{k+1} = f(q_k, u_k) with configuration q and control u;
 *   - Sec. 4.1, eqs. (dynamics), (holonomic-constraint), (contact-constraint),
 *     (dynamics-first-stage), (dynamics-second-stage): the two-stage step;
 *   - Sec. 4.1 "Contact Smoothing": complementarity relaxed to gap*lam = kappa;
 *   - Sec. 4.1 "Differentiating Through Simulation", eq. (diff-sim): the
 *     implicit-function backward pass;
 *   - Sec. 4.2 (output-feedback SLS program): the linearizations A(z,v),
 *     B(z,v) along a nominal trajectory.
 *
 * Conventions shared by every call
 *   - Every call returns an int: CORD_OK (0) or one of the CORD_E* codes.
 *     Nothing throws, aborts or exits across this ABI.  cord_last_error()
 *     returns a thread-local, NUL-terminated message for the last failure
 *     on the calling thread (valid until the next call on that thread).
 *   - Buffers named s0, u, traj, A, Bm, ... are DEVICE pointers owned by the
 *     caller (e.g. torch.Tensor.data_ptr() of a cuda tensor), FP32, never
 *     aliased with each other.  Descriptors passed by pointer are HOST
 *     memory and are copied before the call returns.
 *   - Work is enqueued on the caller's HIP stream (`stream`, a hipStream_t;
 *     NULL = the default stream) without any hidden synchronisation; the
 *     call returns once the work is enqueued.  A cord_sim may be used from
 *     one stream at a time.
 *   - Device-side solver outcomes are written per instance into
 *     `inst_status` (device int32[n_inst], may be NULL); read them after
 *     synchronising the stream.  A non-OK status never stops other
 *     instances.
 *
 * State layout of one instance with n nodes and n_grip grippers
 *   s = [x_0 .. x_{n-1} | v_0 .. v_{n-1}]   (xyz interleaved), n_s = 6 n
 *   u = [u_0 | .. | u_{n_grip-1}]           (gripper velocities), n_u = 3 n_grip
 * Grasp modes (cord_instance_desc.grip_mode):
 *   CORD_GRIP_DIRICHLET  grippers hold their node rigidly (the D -> infinity
 *                        limit of the holonomic penalty of eq.
 *                        (dynamics-first-stage)): x+_j = x_j + dt u_k,
 *                        v+_j = u_k.
 *   CORD_GRIP_PENALTY    the penalty of eq. (dynamics-first-stage) with the
 *                        smoothed activation of Sec. 4.1 "Contact Smoothing":
 *                        gripper positions join the state,
 *                        s = [x | v | g_0 .. g_{n_grip-1}], n_s = 6 n + 3 n_grip,
 *                        g+_k = g_k + dt u_k; node j of gripper k stays free
 *                        and is pulled towards g+_k with stiffness
 *                        D_k = D_max exp(-|x_j - g_k| / kappa_h)
 *                        (kappa_h = 0: D_max if |x_j - g_k| <= r_g, else 0),
 *                        which also enters P of eq. (dynamics-second-stage).
 *
 * Batches may be ragged (different n, T per instance).  Every I/O buffer is
 * the concatenation of per-instance blocks in instance order; the block
 * sizes are given with each call below and cord_sim_offsets() returns the
 * float offset of every block.  For a uniform batch the layout is simply
 * [B][...].
 */
#ifndef CORD_H
#define CORD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define CORD_OK            0
#define CORD_EINVAL        1   /* invalid argument or descriptor            */
#define CORD_ENOMEM        2   /* device or host allocation failed          */
#define CORD_EHIP          3   /* a HIP runtime call failed (see message)   */
#define CORD_EUNSUPPORTED  4   /* valid but not supported (e.g. too many obstacles) */
#define CORD_EAGAIN        5   /* queue full, try again                     */
#define CORD_ETOOBIG       6   /* request larger than the memory budget     */

/* per-instance device status (inst_status[]) */
#define CORD_ST_OK             0
#define CORD_ST_NEWTON_NOCONV  1   /* stage-1 Newton hit its iteration cap       */
#define CORD_ST_NOT_PD         2   /* a solve met non-positive curvature         */
#define CORD_ST_QP_NOCONV      3   /* stage-2 interior point hit its cap         */
#define CORD_ST_NONFINITE      4   /* NaN/Inf in inputs or iterates              */

#define CORD_MAX_GRIP    4
#define CORD_MAX_SPHERE  4
#define CORD_MAX_BOX     2
#define CORD_MAX_OBST    4   /* ground + spheres + boxes, per instance          */

#define CORD_ROPE   0
#define CORD_CLOTH  1

#define CORD_GRIP_DIRICHLET 0
#define CORD_GRIP_PENALTY   1

/*
 * Physical parameters of one instance.
 *   dt        time step [s], > 0
 *   gamma     velocity damping in [0, 1]: the stage-1 inertial term is
 *             M (q* - x_hat)/dt^2 with x_hat = x + dt (1 - gamma) v.
 *             gamma = 1 is the paper's quasi-static eq. (dynamics).
 *   gravity   [m/s^2], part of tau(u) in eq. (dynamics)
 *   kappa_fwd contact relaxation of rollouts [J]; 0 = hard contact
 *             (eq. contact-constraint)
 *   kappa_bwd contact relaxation of the derivatives [J], > 0.  kappa_fwd = 0
 *             < kappa_bwd is the paper's surrogate-gradient mode.
 *   mu        friction coefficient of the cone F_mu = {lam : |lam_t| <=
 *             mu lam_n} of eq. (contact-constraint), >= 0.  With mu > 0 the
 *             constraint value of a contact pair is [phi + n.D ; the
 *             tangential part of the node's displacement over the step],
 *             held in the dual cone {y_n >= mu |y_t|} (Anitescu's
 *             relaxation); smoothed it is the central point y . lam = kappa
 *             of the cone's barrier.  Friction needs kappa_fwd > 0
 *             (otherwise CORD_EUNSUPPORTED).  Dense A_t/B_t of such
 *             instances use the row-by-row kernel.
 */
typedef struct {
    float dt;
    float gamma;
    float gravity[3];
    float kappa_fwd;
    float kappa_bwd;
    float mu;
} cord_params;

/*
 * One rope or cloth instance (Sec. 4.1: a nodal system with stretching and
 * bending energy).
 *   kind      CORD_ROPE: nx nodes in a chain (ny must be 1), stretch springs
 *             between neighbours (stiffness k_struct, rest h) and a
 *             discrete-curvature bending term 1/2 k_bend |x_a - 2x_b + x_c|^2.
 *             1 <= nx <= 256 (nx = 1: a single particle).
 *             CORD_CLOTH: nx*ny grid, node (ix, iy) has index iy*nx + ix;
 *             structural (k_struct, rest h), shear (k_shear, rest h*sqrt 2)
 *             and bend springs two nodes apart (k_bend, rest 2h).
 *             nx, ny >= 2 and nx*ny <= 2304.  Larger instances:
 *             CORD_EUNSUPPORTED.
 *   T         horizon (number of steps), >= 1
 *   mass      lumped mass of every node [kg], > 0
 *   grip_node node held by gripper k, distinct, in [0, n)
 *   ground    nonzero: the plane z = 0 is an obstacle
 *   sphere    (cx, cy, cz, r) with r > 0
 *   box       (cx, cy, cz, hx, hy, hz, rho): axis-aligned box of half
 *             extents h with edges rounded by rho, 0 <= rho < min(h)
 *   grip_mode CORD_GRIP_DIRICHLET or CORD_GRIP_PENALTY (see the state layout)
 *   D_max     penalty mode: grasp stiffness at full activation [N/m], > 0
 *   kappa_h   penalty mode: activation length [m], >= 0 (0: hard activation)
 *   r_g       penalty mode: hard activation radius [m], > 0 when kappa_h = 0
 */
typedef struct {
    int32_t kind;
    int32_t nx, ny;
    int32_t T;
    float h;
    float mass;
    float k_struct, k_shear, k_bend;
    int32_t n_grip;
    int32_t grip_node[CORD_MAX_GRIP];
    int32_t ground;
    int32_t n_sphere;
    float sphere[CORD_MAX_SPHERE][4];
    int32_t n_box;
    float box[CORD_MAX_BOX][7];
    cord_params params;
    int32_t grip_mode;
    float D_max;
    float kappa_h;
    float r_g;
} cord_instance_desc;

typedef struct cord_sim cord_sim;

/*
 * Create a simulator for n_inst instances (Sec. 4.1).  The descriptors are
 * validated and copied; static per-instance data is uploaded to the
 * current HIP device.
 * Errors: CORD_EINVAL (n_inst < 1, dt <= 0, gamma outside [0,1], rope with
 * ny != 1, cloth with nx or ny < 2, n < 1, bad grip/obstacle data, T < 1,
 * kappa_bwd <= 0 or kappa_fwd < 0, mass <= 0, h <= 0, negative stiffness,
 * mu < 0 or not finite),
 * CORD_EUNSUPPORTED (mu > 0 with kappa_fwd = 0, more than CORD_MAX_OBST obstacles, a node
 * count no kernel configuration covers: ropes up to 256 nodes, cloths up
 * to 2304 nodes), CORD_ENOMEM, CORD_EHIP.  *out is set only on success.
 */
int cord_sim_create(const cord_instance_desc* inst, int32_t n_inst, cord_sim** out);

/* Free a simulator and its device memory (NULL is a no-op).  The caller
 * must have synchronised every stream that still uses it. */
int cord_sim_destroy(cord_sim* sim);

/* Sizes, in floats, of the whole-batch buffers. */
typedef struct {
    int64_t n_inst;
    int64_t s_floats;      /* sum n_s           : s0, s0_bar, final states */
    int64_t u_floats;      /* sum T n_u         : u, u_bar                 */
    int64_t traj_floats;   /* sum (T+1) n_s     : full trajectory          */
    int64_t A_floats;      /* sum T n_s^2       : dense A_t                */
    int64_t B_floats;      /* sum T n_s n_u     : dense B_t                */
    int32_t max_n;         /* largest node count                          */
    int32_t max_T;         /* longest horizon                             */
    int64_t aux_floats;    /* sum 14 T n        : step internals (cord_sim_set_aux) */
} cord_sim_info_t;

int cord_sim_info(const cord_sim* sim, cord_sim_info_t* out);

/*
 * Keep the internals of every solved step so the derivatives need not
 * re-solve it.  The adjoint and the linearizations of eq. (diff-sim) are
 * evaluated at the step's stage-1 solution q*, its stage-2 correction and
 * contact multipliers (Sec. 4.1, "Differentiating Through Simulation");
 * without them each step is solved again from its stored state.
 *   aux  device buffer of info.aux_floats floats, owned by the caller, or
 *        NULL to stop using one.  Per instance and step: the stage-1
 *        increment q* - x and the stage-2 correction (3 floats per node
 *        each) and, per obstacle slot, the contact multiplier and gap.
 * While a buffer is set, cord_rollout with FULL storage writes the
 * internals of every step, and cord_rollout_backward with FULL storage and
 * cord_linearize read them instead of solving the step again.  This applies
 * to instances with kappa_fwd == kappa_bwd (the others are always solved
 * again).  The caller must pass to cord_rollout_backward / cord_linearize
 * the trajectory written by the last such rollout.  The derivatives are
 * then evaluated at exactly the state the rollout solved; without the
 * buffer the step is solved again (in the adjoint kernel with the same
 * arithmetic, in the linearization kernels up to FP32 rounding).  One
 * buffer may be set on several simulators created from the same instance
 * descriptors: one simulator's rollout then feeds the others' adjoint or
 * linearization, e.g. on another stream; the caller orders those calls
 * (the readers after the rollout, the next rollout after the readers).
 * Errors: CORD_EINVAL (NULL sim).
 */
int cord_sim_set_aux(cord_sim* sim, float* aux);

/*
 * Float offsets of every instance's block (host arrays of n_inst + 1
 * entries; any pointer may be NULL).  ckpt_every selects the checkpoint
 * layout of ckpt_off (see cord_rollout_opts); pass 0 if unused.
 */
int cord_sim_offsets(const cord_sim* sim, int32_t ckpt_every, int64_t* s_off,
                     int64_t* u_off, int64_t* traj_off, int64_t* ckpt_off,
                     int64_t* A_off, int64_t* B_off);

/* ---------------------------------------------------------------- rollout */
#define CORD_STORE_FULL   0   /* traj holds s_0 .. s_T: (T+1) n_s per instance          */
#define CORD_STORE_CKPT   1   /* traj holds s_0, s_K, s_2K, .. and s_T:                  */
                              /*   (ceil(T/K) + 1) n_s per instance                        */
#define CORD_STORE_FINAL  2   /* traj holds s_T only: n_s per instance                     */

typedef struct {
    int32_t store;        /* CORD_STORE_*                                         */
    int32_t ckpt_every;   /* K >= 1 for CORD_STORE_CKPT                          */
    int32_t use_kappa_bwd;/* nonzero: roll out f with kappa_bwd instead of kappa_fwd */
    int32_t reserved;
    uint32_t* counters;   /* optional device uint32[n_inst][4], added to: Newton
                             iterations, conjugate-gradient iterations (all solves),
                             interior-point iterations, solved steps                */
    float* final_state;   /* optional device [n_s] per instance: s_T, in any store mode */
} cord_rollout_opts;

/*
 * Forward rollout s_{t+1} = f(s_t, u_t), t < T (eq. dynamics_sim), with the
 * two-stage step of Sec. 4.1 at kappa_fwd.
 *   s0   [n_s] per instance            u  [T][n_u] per instance
 *   traj written per opts->store (see CORD_STORE_*)
 * opts may be NULL (= FULL storage).  Errors: CORD_EINVAL (NULL buffer,
 * bad opts), CORD_EHIP (launch failure).
 */
int cord_rollout(cord_sim* sim, const float* s0, const float* u, float* traj,
                 int32_t* inst_status, const cord_rollout_opts* opts, void* stream);

typedef struct {
    int32_t store;        /* how `traj` was written: CORD_STORE_FULL or _CKPT   */
    int32_t ckpt_every;   /* K used by the forward pass                        */
    int32_t use_kappa_bwd;/* the forward pass ran with kappa_bwd (recompute uses it) */
    int32_t reserved;
    const float* sT_bar;  /* device [n_s] per instance, used when traj_bar is NULL */
    uint32_t* counters;   /* optional device uint32[n_inst][4] as in cord_rollout */
} cord_backward_opts;

/*
 * Reverse-mode gradient of a rollout (eq. diff-sim): for every step, in
 * reverse order, the step is re-solved at kappa_bwd from the stored or
 * recomputed state s_t, then the adjoint solves with the stage-2 KKT
 * matrix and with dF/dq* are applied.
 *   u         [T][n_u] per instance (the controls of the forward pass)
 *   traj      written by cord_rollout with opts->store (FULL or CKPT)
 *   traj_bar  [T+1][n_s] per instance, cotangent of every state, or NULL
 *             (then opts->sT_bar is the cotangent of s_T)
 *   s0_bar    [n_s] per instance (output)
 *   u_bar     [T][n_u] per instance (output)
 * With CKPT storage the states inside each segment are recomputed from its
 * checkpoint with the same kernel configuration as the forward pass, so
 * they are bitwise equal to a FULL rollout.  The library keeps a device
 * workspace for the recomputed segment (grown on demand: CORD_ENOMEM if
 * that fails).
 */
int cord_rollout_backward(cord_sim* sim, const float* u, const float* traj,
                          const float* traj_bar, float* s0_bar, float* u_bar,
                          int32_t* inst_status, const cord_backward_opts* opts, void* stream);

/*
 * cord_rollout_backward without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * cord_rollout_backward, bitwise the same outputs, except:
 *   - the checkpoint offsets and the workspace of the recomputed segments
 *     (CORD_STORE_CKPT) live in a static device array of the library,
 *     64 MiB on every GPU it runs on, held until the process ends; a call
 *     needing more (8 n_inst bytes of table rounded up to a multiple of
 *     256, plus 4 ckpt_every sum(n_s) bytes) returns CORD_ETOOBIG;
 *   - the kernels are launched one per size class on `stream`, whatever
 *     the simulator's launch mode (the persistent and graph modes would
 *     create streams, queues and graphs);
 *   - every call on one GPU shares that array: calls that overlap on one
 *     GPU (other streams, other threads, other simulators) race and must be
 *     ordered by the caller.
 * No hipMalloc, hipFree or allocating library call is made.  CORD_EHIP if
 * the device address of the array could not be obtained when the simulator
 * was created.
 */
int cord_rollout_backward_noalloc(cord_sim* sim, const float* u, const float* traj,
                                  const float* traj_bar, float* s0_bar, float* u_bar,
                                  int32_t* inst_status, const cord_backward_opts* opts, void* stream);

/* Tangents for cord_linearize's JVP mode: per step t, k tangent pairs
 * (ds_t, du_t) map to ds_{t+1} = A_t ds_t + B_t du_t (steps independent). */
typedef struct {
    int32_t k;            /* tangents per step, >= 1                          */
    const float* ds;      /* device [T][k][n_s] per instance, or NULL (= 0)   */
    const float* du;      /* device [T][k][n_u] per instance, or NULL (= 0)   */
    float* out;           /* device [T][k][n_s] per instance                  */
} cord_jvp;

/*
 * Linearizations along a trajectory (Sec. 4.2, A(z,v), B(z,v)): for every
 * t < T, A_t = ds_{t+1}/ds_t and B_t = ds_{t+1}/du_t of f at kappa_bwd,
 * evaluated at the stored states traj (FULL storage) and controls u.
 *   A   [T][n_s][n_s] row-major per instance, or NULL
 *   Bm  [T][n_s][n_u] row-major per instance, or NULL
 *   jvp JVP mode (may be NULL); may be combined with A/Bm.
 * For ropes of up to 128 particles with a Dirichlet grasp, A/Bm come from
 * the banded direct kernel; the simulator then keeps a device scratch table
 * for it (allocated on the first such call: 302 MB for the 64-particle
 * class on MI355X, of which the resident workgroups touch 151 MB; if that
 * allocation fails the kernel works without it, at lower speed, with
 * bitwise the same results).  Linearize calls on one
 * simulator share that table: calls on different streams must not overlap.
 * Environment: CORD_LINEARIZE_NO_SCRATCH=1 (read at every call) runs the
 * direct kernel without the table (bitwise the same results);
 * CORD_LINEARIZE_ITERATIVE=1 (read once per process) uses the row-by-row
 * kernel for every instance (the same derivatives up to FP32 rounding).
 * Errors: CORD_EINVAL if A, Bm and jvp are all NULL.
 */
int cord_linearize(cord_sim* sim, const float* traj, const float* u, float* A, float* Bm,
                   const cord_jvp* jvp, int32_t* inst_status, void* stream);

/*
 * Counters of the dense rope linearization since the simulator was created
 * (host array of 2): out2[0] steps whose scratch slot was found shared
 * by two workgroups resident at the same time (each such step is done
 * again by the row-by-row kernel, so A_t stays exact; nonzero would mean
 * the hardware slot key does not separate resident workgroups), out2[1]
 * steps done again by that kernel for any reason (a non-positive pivot
 * of a band factor, an indefinite dF/dq* of Sec. 4.1 "Differentiating
 * Through Simulation", or a shared slot).  Synchronizes the device.
 * Errors: CORD_EINVAL, CORD_EHIP.
 */
int cord_sim_lin_stats(cord_sim* sim, int64_t* out2);

/*
 * Sizes in bytes of the public structs, for bindings that mirror them:
 * out[0] cord_params, out[1] cord_instance_desc, out[2] cord_sim_info_t,
 * out[3] cord_rollout_opts, out[4] cord_backward_opts, out[5] cord_jvp.
 * Writes min(n, 6) entries of the host array out; returns CORD_EINVAL if
 * out is NULL.
 */
int cord_abi_sizes(int64_t* out, int32_t n);

/* ---------------------------------------------------------------- launch */
/*
 * How cord_rollout and cord_rollout_backward are launched.  Instances are
 * grouped into size classes (ropes with n <= 32, 64, 128, 256 nodes; cloths
 * with n <= 64, 128, 256, 512, 1024 nodes); each class has one kernel
 * configuration (threads per workgroup x particles per thread), chosen by
 * default or by cord_autotune.  Results of an instance depend only on its
 * class configuration, never on the rest of the batch or on the launch mode.
 *   CORD_LAUNCH_GROUPED       one launch per class, one workgroup per instance
 *   CORD_LAUNCH_PER_INSTANCE  one launch per instance (the plain launch)
 *   CORD_LAUNCH_PERSISTENT    one persistent launch per class, each on its own
 *                             stream forked from the caller's; workgroups pull
 *                             instances (longest n*T first) from a device work
 *                             queue until it is empty
 *   CORD_LAUNCH_GRAPH         the persistent multi-stream sequence captured
 *                             once into a hipGraph per set of buffers and then
 *                             replayed with a single hipGraphLaunch
 */
#define CORD_LAUNCH_GROUPED       0
#define CORD_LAUNCH_PER_INSTANCE  1
#define CORD_LAUNCH_PERSISTENT    2
#define CORD_LAUNCH_GRAPH         3

/* Select the launch mode (default CORD_LAUNCH_GROUPED).  CORD_EINVAL for an
 * unknown mode.  Changing the mode drops cached graphs. */
int cord_sim_set_launch(cord_sim* sim, int32_t mode);

/*
 * Autotuner: for every size class, time each kernel configuration that covers
 * the class (a forward rollout of up to `sample` instances of the class, with
 * the caller's s0 and u, FINAL storage, median of 3 after a warm-up), keep
 * the fastest and regroup.  cache_path (may be NULL) is a JSON file of
 * previous choices, read first (classes found there are not re-timed) and
 * rewritten afterwards.  Synchronises `stream`; allocates temporary device
 * buffers.  Errors: CORD_EINVAL, CORD_ENOMEM, CORD_EHIP.
 */
int cord_autotune(cord_sim* sim, const float* s0, const float* u, int32_t sample, const char* cache_path,
                  void* stream);

/* Size classes in use: writes up to `cap` entries of topology (CORD_ROPE /
 * CORD_CLOTH), largest node count of the class, threads per workgroup,
 * particles per thread, and instance count; *count = number of classes. */
int cord_sim_classes(const cord_sim* sim, int32_t* topo, int32_t* nmax, int32_t* nt, int32_t* ppt,
                     int32_t* n_inst, int32_t cap, int32_t* count);

/* ---------------------------------------------------------------- conformal calibration */
/*
 * Conformal calibration of the one-step model error (Sec. 4.4,
 * "Calibrated Reachability Guarantees via Conformal Prediction").  A
 * calibration set of n perceived-state transitions (q_i, u_i, q_i+) is a
 * simulator of n instances with T = 1 (the geometry, material and
 * obstacles of each pair; quasi-static gamma = 1 is the paper's model).
 *
 * cord_cp_scores: the nonconformity scores s_i = |q_i+ - f(q_i, u_i)|_2 over
 * the node positions, f being one step of the simulator (at kappa_fwd).
 *   s_bar   device [n_s] per instance: the perceived state (positions used;
 *           the velocity block is the step's input velocity)
 *   u       device [n_u] per instance
 *   s_next  device [n_s] per instance: the perceived next state (only the
 *           position block is read)
 *   scores  device float[n_inst] (output)
 * The library keeps a device buffer for the predictions (allocated on the
 * first call).  Errors: CORD_EINVAL (NULL buffer, an instance with T != 1),
 * CORD_ENOMEM, CORD_EHIP.
 *
 * cord_cp_radius: for a trajectory-level miscoverage delta over `horizon`
 * steps, the radius r_CP = s_(k), the k-th smallest score with
 * k = ceil((n + 1)(1 - delta / horizon)) evaluated in double precision
 * with a margin of 1e-9 (so that a decimal delta whose exact product is an
 * integer does not round k up), or +infinity if k > n.  Ties are ordered
 * by index and a NaN score after every number.
 *   scores  device float[n], 1 <= n <= 65536
 *   radius  device float (output);  index  device int32 (output, may be
 *           NULL): the calibration pair whose score is the radius, -1 for
 *           +infinity
 * Errors: CORD_EINVAL (NULL scores or radius, n < 1, horizon < 1,
 * delta / horizon outside (0, 1)), CORD_EUNSUPPORTED (n > 65536), CORD_EHIP.
 */
int cord_cp_scores(cord_sim* sim, const float* s_bar, const float* u, const float* s_next, float* scores,
                   int32_t* inst_status, void* stream);
int cord_cp_radius(const float* scores, int32_t n, double delta, int32_t horizon, float* radius,
                   int32_t* index, void* stream);

/* ---------------------------------------------------------------- planning service */
/*
 * Gradient-based trajectory planning (the nominal (z, v) of Sec. 4.2, stage
 * (1); "gradient-based trajectory optimization", Sec. 1 and Table 1), served
 * with continuous batching.
 *
 * One request plans for one rope or cloth: n_cand candidate control
 * sequences over the instance's horizon T are improved together by
 * `iters` projected-gradient steps
 *     u <- clip(u - step * dJ/du, -u_max, u_max),
 *     J(u) = |x_T[goal_node] - goal|^2 + u_reg * sum_t |u_t|^2,
 * each step being a batched forward rollout and adjoint of all candidates
 * (cord_rollout / cord_rollout_backward).  Candidate 0 starts from u_warm,
 * candidate c > 0 from u_warm + sigma * N(0, 1) unless u_init gives all
 * starts explicitly.  The normal values come from SplitMix64 seeded with
 * `seed`, two outputs per value, candidate by candidate and then in u's
 * order: each output maps to a = ((x >> 11) + 1/2) 2^-53 in (0, 1), and
 * z = sqrt(-2 ln a1) cos(2 pi a2) (Box-Muller, in double), rounded to
 * float; the start is the float sum u_warm + sigma * z.  After the last step the
 * candidates are rolled out once more, the lowest J wins (ties: lowest
 * index), and for want_AB the dense A_t, B_t along the winner are computed
 * (cord_linearize).  All of this runs on the device without host round trips;
 * the winner's controls, trajectory and Jacobians stay on the device until the
 * request completes, then are copied to host buffers owned by the server.
 */
typedef struct {
    cord_instance_desc inst;   /* the object, its parameters and horizon T             */
    const float* s0;           /* HOST [n_s] initial state                             */
    const float* u_warm;       /* HOST [T][n_u] warm start, or NULL (zeros)            */
    const float* u_init;       /* HOST [n_cand][T][n_u] explicit starts, or NULL       */
    int32_t goal_node;         /* node whose final position is steered                 */
    float goal[3];
    uint64_t seed;
    int32_t n_cand;            /* candidates, >= 1                                     */
    int32_t iters;             /* gradient steps, >= 0                                 */
    float step;                /* step size                                            */
    float u_max;               /* |u| bound per component, > 0                         */
    float sigma;               /* std of the candidate perturbation                    */
    float u_reg;               /* control regularisation weight, >= 0                  */
    int32_t want_AB;           /* nonzero: dense A_t, B_t along the winner             */
    int32_t reserved;
} cord_plan_request;

typedef struct {
    int32_t status;            /* CORD_OK, or the error code of a failed request       */
    int32_t sim_status;        /* worst per-candidate solver status (CORD_ST_*)        */
    int32_t best;              /* winning candidate                                    */
    int32_t T, n_s, n_u, n_cand;
    float cost;                /* J of the winner                                      */
    const float* u;            /* HOST [T][n_u] winner controls                        */
    const float* traj;         /* HOST [T+1][n_s] winner trajectory                    */
    const float* A;            /* HOST [T][n_s][n_s] or NULL                           */
    const float* B;            /* HOST [T][n_s][n_u] or NULL                           */
    const float* costs;        /* HOST [n_cand] final J of every candidate             */
    double t_submit, t_admit, t_done;   /* seconds on the server's steady clock        */
} cord_plan_result;

typedef struct cord_server cord_server;

/*
 * Start a planning server on `device`: one scheduler thread and `max_slots`
 * device streams.  Requests are admitted in arrival order (a request that
 * does not fit may be overtaken by at most 8 later ones) when a slot is free
 * and its device footprint fits in what remains of `hbm_budget` bytes;
 * admitted requests run concurrently, one per slot stream.  max_slots = 1 is
 * the one-request-at-a-time server.  Errors: CORD_EINVAL, CORD_EHIP, CORD_ENOMEM.
 */
int cord_server_create(int32_t device, size_t hbm_budget, int32_t max_slots, int32_t queue_cap,
                       cord_server** out);

/* Stop accepting, finish or cancel queued work, join the thread, free all
 * memory (including unreleased results). */
int cord_server_destroy(cord_server* srv);

/*
 * Submit a request (copied; host pointers may be reused on return).  Never
 * blocks.  Errors: CORD_EINVAL (bad request), CORD_EUNSUPPORTED (as
 * cord_sim_create), CORD_EAGAIN (queue full), CORD_ETOOBIG (footprint above
 * the whole budget).  *ticket identifies the request.
 */
int cord_plan_submit(cord_server* srv, const cord_plan_request* req, uint64_t* ticket);

/* CORD_OK and *out filled if the request is done (its status field tells
 * success), CORD_EAGAIN if still queued or running, CORD_EINVAL for an
 * unknown ticket. */
int cord_plan_poll(cord_server* srv, uint64_t ticket, cord_plan_result* out);

/* As cord_plan_poll but waits up to timeout_ms (< 0: forever). */
int cord_plan_wait(cord_server* srv, uint64_t ticket, int32_t timeout_ms, cord_plan_result* out);

/* Free a finished request's result buffers; the ticket becomes unknown. */
int cord_plan_release(cord_server* srv, uint64_t ticket);

/* Server counters: submitted, admitted, completed, failed, queued now,
 * running now, peak queue depth, bytes in use (host array of 8 int64). */
int cord_server_stats(cord_server* srv, int64_t* out8);

/* ---------------------------------------------------------------- output-feedback SLS */
/*
 * Stage 3 of the output-feedback SLS decomposition (Sec. 4.2,
 * "Simulator-Informed GPU-Parallel Output Feedback SLS") for a batch of B
 * nominal trajectories of N steps, state size n, input size m, with the
 * perception returning the full state (C = I, Sec. 4.4).  Conventions:
 * x_{j+1} = A_j x_j + B_j u_j + E_j w_j and y_{j+1} = x_j + F_j e_j (the
 * measurement of x_j has index j + 1).  All buffers are device memory,
 * row-major, instance-major, owned by the caller:
 *   A, E, F      float[B][N][n][n]   (A as written by cord_linearize for
 *                                     instances of equal n_s and T = N)
 *   Bm           float[B][N][n][m]   K  float[B][N+1][m][n]
 *   Xi           float[B][n][n]      initial uncertainty
 *   Pi           float[B][N+1][n][n] L  float[B][N][n][n], L[j] = L_{j+1}
 *   horizon operators: dense float[B][(N+1) r][(N+1) n] with block (k, j)
 *   at rows k r, columns j n, where r = n for state rows and m for input
 *   rows; the blocks right of the block diagonal are written as zeros.
 * Calls are stream-ordered on `stream` (NULL = default stream); calls on one
 * handle share its workspace and must not overlap.
 *
 * cord_sls_create: a handle for (B, N, n, m) and its device workspace
 * (about 2 B (N+1)^2 n^2 + 12 B (N+1) n^2 floats).  Errors: CORD_EINVAL,
 * CORD_EUNSUPPORTED (n > 1024), CORD_ETOOBIG (one horizon operator above
 * 64 GiB), CORD_ENOMEM.
 *
 * cord_sls_kalman: the Kalman recursion (eq. kalman_recursions),
 * Pi_0 = Xi Xi^T, L_{j+1} = -(F_j F_j^T + Pi_j)^{-1} Pi_j A_j^T,
 * Pi_{j+1} = E_j E_j^T + A_j Pi_j A_j^T + A_j Pi_j L_{j+1}, either
 * CORD_SLS_SERIAL (one workgroup per instance steps through the horizon,
 * each step in the scan elements' form Pi' = E E^T + W^T Pi A^T with
 * W = (I + (F F^T)^{-1} Pi)^{-1} A^T, L = W - A^T, which is the same
 * recursion without the subtraction that FP32 cannot resolve when the
 * measurements are accurate) or
 * CORD_SLS_SCAN (the associative scan of eqs. combination_rules and
 * initialization, ceil(log2(N+1)) rounds, then all gains at once).
 * status: device int32[B], CORD_ST_NOT_PD where a solve met a zero or
 * non-finite pivot.  Errors: CORD_EINVAL, CORD_EHIP.
 *
 * cord_sls_observer: the observer responses (eq. backward_propagations):
 * Phx[k][j] = Ahat_{k-1} .. Ahat_j with Ahat_j = A_j + L_{j+1}^T, Phx[k][k]
 * = I, and Phy[k][j] = Phx[k][j] L_j^T for 1 <= j <= k (column block 0 is
 * zero); both (N+1) n x (N+1) n.  The products are formed by doubling along
 * the block diagonals: one GEMM per block, 2 ceil(log2 N) launches.
 *
 * cord_sls_state_feedback: the responses of u_j = K_j x_j, Pbx = (I - Z(A +
 * B K))^{-1} ((N+1) n square) and Pbu = blkdiag(K) Pbx ((N+1) m x (N+1) n):
 * a stand-in for stage 2 of the decomposition (GPU-SLS, prior work the paper
 * builds on), with the same kernels as cord_sls_observer.
 *
 * cord_sls_assemble: with M = I - ZA, the closed-loop responses
 * Pxw = Pbx + Phx - Pbx M Phx,  Puw = Pbu (I - M Phx),
 * Pxe = Phy - Pbx M Phy,        Pue = -Pbu M Phy,
 * as block-triangular GEMMs (only the nonzero block range of each output
 * tile is summed).
 *
 * cord_sls_tubes: the tube widths of the tightening constraints (eq.
 * of_optimization) for unit-ball w_j and e_j,
 * tau[k] = sum_{j<k} rownorm(Pxw[k][j+1] E_j) + rownorm(Pxe[k][j+1] F_j)
 * (float[B][N+1][n]; tau[0] = 0), and likewise tau_u from Puw and Pue
 * (float[B][N+1][m]) when tau_u is not NULL.  Errors: CORD_EINVAL,
 * CORD_EHIP.
 */
typedef struct cord_sls cord_sls;
#define CORD_SLS_SERIAL 0
#define CORD_SLS_SCAN   1
int cord_sls_create(int32_t batch, int32_t horizon, int32_t n, int32_t n_u, cord_sls** out);
int cord_sls_destroy(cord_sls* sls);
int cord_sls_kalman(cord_sls* sls, const float* A, const float* E, const float* F, const float* Xi, int32_t mode,
                    float* Pi, float* L, int32_t* status, void* stream);
int cord_sls_observer(cord_sls* sls, const float* A, const float* L, float* Phx, float* Phy, void* stream);
int cord_sls_state_feedback(cord_sls* sls, const float* A, const float* Bm, const float* K, float* Pbx, float* Pbu,
                            void* stream);
int cord_sls_assemble(cord_sls* sls, const float* A, const float* Pbx, const float* Pbu, const float* Phx,
                      const float* Phy, float* Pxw, float* Puw, float* Pxe, float* Pue, void* stream);
int cord_sls_tubes(cord_sls* sls, const float* Pxw, const float* Pxe, const float* Puw, const float* Pue,
                   const float* E, const float* F, float* tau_x, float* tau_u, void* stream);

/* Thread-local message of the last error on this thread ("" if none). */
const char* cord_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CORD_H */
