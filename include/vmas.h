/*
 * vmas.h -- C boundary of the MI355X (gfx950) batched 2D physics step.
 *
 * The method is the world step of VMAS (Bettini et al., 2022), Sec. 3 "Core":
 *   Eq. (1)  f_i = f^a_i + m_i g + sum_{j != i} f^e_ij ;
 *            xdot_i(t+1) = (1 - zeta) xdot_i(t) + f_i / m_i dt ;
 *            x_i(t+1)    = x_i(t) + xdot_i(t+1) dt
 *   Eq. (2)  f^e_ij = c * x_ij/|x_ij| * k * log(1 + exp(-(|x_ij| - d_min)/k))
 *            if |x_ij| <= d_min, else 0 ; x_ij joins the closest points
 *   Eq. (3)  tau_i = sum_j r_ij x f^e_ij (signed), then the same update on
 *            (theta, omega) with moment of inertia I_i.
 * for every entity of every environment of a batch, all environments at once.
 *
 * Readings where the paper is silent (all fixed by this library):
 *   - shapes: a sphere's core is its centre (radius enters d_min), a line is
 *     a segment along its local x axis of length L, a box a solid lx x ly
 *     rectangle; |x_ij| is the signed distance between cores (negative when
 *     they overlap, by the separating-axis test), d_min = rho_i + rho_j +
 *     min_dist with rho = r for spheres and 0 otherwise;
 *   - the torque of Eq. (3) is the signed 2D cross product of the arm
 *     (contact point - centre) with the force;
 *   - flags: immovable entities keep x and v (no gravity), non-rotatable ones
 *     keep theta and omega, non-collidable ones take part in no pair; a pair
 *     where neither entity can move or rotate is skipped;
 *   - the action of an agent is a force at its centre (no torque);
 *   - the max speed clamps |v| after the velocity update, keeping direction;
 *   - default moments of inertia: disc m r^2/2, rectangle m (lx^2+ly^2)/12,
 *     rod m L^2/12;
 *   - a joint is a linear spring of stiffness joint_stiffness between two
 *     body-frame anchor points (rest length: given, or the anchor distance in
 *     the initial state); by default the two jointed entities do not collide.
 *   - the contact decision |x_ij| <= d_min (inclusive) is taken in FP32;
 *     between two spheres it is fma(dx, dx, fl(dy*dy)) <= fl(d_min*d_min)
 *     (one fused multiply-add) with dx = fl(x_i - x_j), dy = fl(y_i - y_j),
 *     d_min = fl(fl(r_i + r_j) + min_dist); other pairs compare the FP32
 *     signed distance with the FP32 d_min. An exact evaluation can decide
 *     differently only for pairs within FP32 rounding of d_min.
 *
 * Memory. Every state, action, mask, force and gradient buffer passed to the
 * step calls is DEVICE memory owned by the caller; the library never frees
 * or retains those pointers after a call returns. The handle owns its own
 * device copies of the static description (shapes, masses, joints, launch
 * plans, checkpoint workspace); vmas_destroy_batch frees them.
 *
 * Layouts.
 *   state    float32 [6][N], field-major: x, y, vx, vy, theta, omega; the
 *            entities of an environment are contiguous, environments in order.
 *   actions  float32 [A][2] per step ([T][A][2] for rollouts): one row per
 *            agent; the agents of environment b are its first n_agents[b]
 *            entities, rows in environment order.
 *   mask     uint8 [P], P = sum_b n_b (n_b - 1) / 2: one byte per pair slot,
 *            environments in order, pairs (a < c) of local indices in
 *            lexicographic order; 1 when the pair is in contact (Eq. 2 active),
 *            0 otherwise (also for pairs that are not eligible).
 *   forces   float32 [3][N]: total force x, y and torque on each entity that
 *            can move or rotate (Eq. 1 first row, Eq. 3 first row); 0 for the
 *            others.
 *
 * Streams and errors. All device work is enqueued on the caller's stream
 * (a hipStream_t passed as void*, NULL = the default stream) and the calls
 * return after enqueue; only vmas_create_batch blocks. Arguments are checked
 * on the host before any device work: a bad argument returns
 * VMAS_ERR_INVALID_ARGUMENT, a HIP failure VMAS_ERR_DEVICE, a state that went
 * non-finite under VMAS_DEBUG_NONFINITE VMAS_ERR_NONFINITE (on the next call);
 * the reason is in
 * vmas_last_error() (thread-local, valid until the next call on that thread).
 * A handle must not be used from two threads at once; calls on different
 * handles are independent. Calls that overlap on one stream are ordered by it.
 */
#ifndef VMAS_H
#define VMAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VMAS_OK = 0,
  VMAS_ERR_INVALID_ARGUMENT = 1,
  VMAS_ERR_OUT_OF_MEMORY = 2,
  VMAS_ERR_DEVICE = 3,
  VMAS_ERR_UNSUPPORTED = 4,
  VMAS_ERR_NONFINITE = 5
} vmas_status;

typedef enum { VMAS_SHAPE_SPHERE = 0, VMAS_SHAPE_BOX = 1, VMAS_SHAPE_LINE = 2 } vmas_shape;

/* Entity flag bits (Sec. 3 "Core": movable, rotatable, collidable). */
enum { VMAS_MOVABLE = 1, VMAS_ROTATABLE = 2, VMAS_COLLIDABLE = 4 };

/* World parameters (Sec. 3: dt, zeta, g; Eq. 2: c, k, d_min). */
typedef struct {
  float dt;               /* integration step delta t > 0 */
  float drag;             /* velocity damping zeta in [0, 1] */
  float gravity[2];       /* g */
  float contact_force;    /* c >= 0 */
  float contact_margin;   /* k > 0 */
  float min_dist;         /* added to every pair's d_min (>= 0) */
  float joint_stiffness;  /* spring constant of every joint (>= 0) */
  uint32_t flags;         /* 0 or VMAS_DEBUG_NONFINITE; other bits are rejected */
} vmas_world_params;

/* World flag bits.
 * VMAS_DEBUG_NONFINITE: after the work of every call that advances the state
 *   (vmas_step, vmas_rollout, vmas_rollout_graph, vmas_step_surrogate) the
 *   library enqueues a check of the output state on the same stream: an
 *   environment one of whose entities holds a NaN or an infinity (a blown-up
 *   simulation, e.g. beyond the stability bound of the penalty spring) is
 *   marked on the device and counted the first time it is seen. The next call
 *   on the handle (any step, rollout or adjoint call) first synchronises its
 *   stream, reads the count and, when environments were marked since the last
 *   report, returns VMAS_ERR_NONFINITE with the counts in vmas_last_error()
 *   and enqueues no work; the call after it proceeds. vmas_nonfinite_envs
 *   lists the marked environments. Costs one pass over the state per call and
 *   one stream synchronisation per call; off by default. */
enum { VMAS_DEBUG_NONFINITE = 1 };

/* Static description of a batch. All pointers are HOST memory, read during
 * vmas_create_batch only. N = total entities, A = total agents, J = joints. */
typedef struct {
  int32_t n_envs;                 /* >= 1 */
  const int32_t* env_offset;      /* [n_envs+1] entity offsets, or NULL: uniform */
  int32_t n_per_env;              /* entities per environment when env_offset is NULL */
  const int32_t* n_agents;        /* [n_envs], 0 <= n_agents[b] <= n_b */
  const uint8_t* shape;           /* [N] vmas_shape */
  const float* dims;              /* [N][2]: sphere (r, -), box (lx, ly), line (L, -); > 0 */
  const float* mass;              /* [N] > 0 for entities that can move or rotate */
  const float* inertia;           /* [N] or NULL; <= 0 selects the textbook default */
  const float* max_speed;         /* [N] or NULL; <= 0: no clamp */
  const uint8_t* flags;           /* [N] VMAS_MOVABLE | VMAS_ROTATABLE | VMAS_COLLIDABLE */
  int32_t n_joints;               /* J >= 0 */
  const int32_t* joint_a;         /* [J] global entity ids, both in one environment */
  const int32_t* joint_b;         /* [J] */
  const float* joint_anchor_a;    /* [J][2] body-frame anchor on a */
  const float* joint_anchor_b;    /* [J][2] body-frame anchor on b */
  const float* joint_rest;        /* [J] rest length; < 0: the anchor distance in init_state,
                                     evaluated with the step's own FP32 arithmetic (so the
                                     joint exerts exactly no force in that state) */
  const uint8_t* joint_collide;   /* [J] or NULL: 0 = the jointed pair does not collide */
  const float* init_state;        /* [6][N] host state, needed only when a rest length is < 0 */
} vmas_batch_desc;

typedef struct vmas_batch vmas_batch; /* opaque handle */
typedef struct vmas_mlp vmas_mlp;     /* opaque handle of the contact surrogate */

typedef struct {
  int32_t n_envs;
  int32_t n_entities;    /* N */
  int32_t n_agents;      /* A */
  int32_t n_joints;      /* J */
  int64_t n_pair_slots;  /* P */
  int32_t schedule;      /* current launch plan id (see vmas_set_schedule) */
  int32_t n_schedules;   /* number of launch plans available */
  int32_t max_env_size;  /* largest n_b */
  int32_t tune_cached;   /* 1: the last vmas_autotune took its choice from the cache */
} vmas_batch_info;

/* Creates a batch on HIP device `device`: validates the description, copies
 * it to the device and builds the launch plans. Blocks until the upload is
 * done. On success *out owns device memory until vmas_destroy_batch. */
vmas_status vmas_create_batch(const vmas_world_params* params, const vmas_batch_desc* desc,
                              int device, vmas_batch** out);

/* Frees the handle and all device memory it owns (NULL is accepted). The
 * caller must make sure no work that uses the handle is still running. */
vmas_status vmas_destroy_batch(vmas_batch* batch);

vmas_status vmas_batch_get_info(const vmas_batch* batch, vmas_batch_info* info);

/* One step (Eq. 1-3) of every environment, state updated in place.
 *   state    device float32 [6][N] (in/out)
 *   actions  device float32 [A][2] (may be NULL only when A == 0)
 *   mask     device uint8 [P] or NULL: contact mask of this step
 *   forces   device float32 [3][N] or NULL: forces and torques of this step */
vmas_status vmas_step(vmas_batch* batch, float* state, const float* actions, uint8_t* mask,
                      float* forces, void* stream);

/* T consecutive steps in one persistent launch; the state stays on chip
 * between steps and only the actions stream in.
 *   state       device float32 [6][N] (in/out): state at t0 in, at t0+T out
 *   actions     device float32 [T][A][2], or NULL: the actions are drawn in
 *               the kernel, uniform in [-1, 1)^2, from the counter-based
 *               SplitMix64 stream (seed = action_seed, stream 2, element
 *               ((t0 + t) * A + agent) * 2 + comp; u = (draw >> 40) 2^-24,
 *               a = 2u - 1)
 *   t0          step index of the first step (only used for drawn actions)
 *   T           number of steps, >= 0
 *   traj        device float32 [T+1][6][N] or NULL: the state after every step
 *               (index 0 = input state)
 *   final_mask  device uint8 [P] or NULL: contact mask of the last step
 * Splitting a rollout (T = k + (T - k), same actions) gives bitwise the same
 * final state. */
vmas_status vmas_rollout(vmas_batch* batch, float* state, const float* actions,
                         uint64_t action_seed, int32_t t0, int32_t T, float* traj,
                         uint8_t* final_mask, void* stream);

/* Reverse-mode derivative of one vmas_step (hand-written adjoint; contact
 * decisions and the branches of the closest-point routines are held fixed).
 *   state_t          device float32 [6][N]: the state the step started from
 *   actions_t        device float32 [A][2]
 *   grad_state_next  device float32 [6][N]: dL/d state_{t+1}
 *   grad_state_t     device float32 [6][N] (out): dL/d state_t
 *   grad_actions_t   device float32 [A][2] (out) or NULL: dL/d actions_t */
vmas_status vmas_step_backward(vmas_batch* batch, const float* state_t, const float* actions_t,
                               const float* grad_state_next, float* grad_state_t,
                               float* grad_actions_t, void* stream);

/* Reverse-mode derivative of a T-step rollout with checkpointing: the
 * forward pass is replayed from checkpoints stored every `ckpt_every` steps
 * (workspace owned by the handle, ceil(T / ckpt_every) + ckpt_every + 1 states),
 * so memory is O(T / k + k) states instead of O(T); the reverse steps of a
 * segment run in one launch, each computing what vmas_step_backward computes
 * (the same bits). Sphere batches in which every entity moves and none has
 * a speed cap need only positions in the reverse step (a third of a state):
 * in the same workspace a window over the last segments then gets the
 * positions of one forward launch and is not replayed. Every ckpt_every
 * gives the same bits.
 *   state0        device float32 [6][N]: initial state
 *   actions       device float32 [T][A][2]
 *   grad_state_T  device float32 [6][N]: dL/d state_T
 *   grad_state0   device float32 [6][N] (out) or NULL
 *   grad_actions  device float32 [T][A][2] (out) or NULL */
vmas_status vmas_rollout_backward(vmas_batch* batch, const float* state0, const float* actions,
                                  int32_t T, int32_t ckpt_every, const float* grad_state_T,
                                  float* grad_state0, float* grad_actions, void* stream);

/* vmas_rollout_backward for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and kernels, but the checkpoint
 * workspace lives in a fixed 64 MiB device array inside the library (one
 * per device, held until the process ends) instead of memory the handle
 * allocates; the call itself allocates nothing. The workspace needs
 * 6 N (ceil(T / k) + k + 3) floats (k = min(ckpt_every, T)); a larger need
 * returns VMAS_ERR_INVALID_ARGUMENT before any device work. All calls on one
 * device share that array and leave their data in it: calls that overlap in
 * time on one device (different streams, threads or handles) race and must
 * be serialised by the caller. With VMAS_DEBUG_NONFINITE the call
 * synchronises its stream first, like every call of such a batch. */
vmas_status vmas_rollout_backward_noalloc(vmas_batch* batch, const float* state0,
                                          const float* actions, int32_t T, int32_t ckpt_every,
                                          const float* grad_state_T, float* grad_state0,
                                          float* grad_actions, void* stream);

/* Launch plans. Plan ids are 0 .. n_schedules-1 (see vmas_schedule_name);
 * every plan computes the same results bit for bit. Names:
 * "entity-lane/<block>/<natural|size-sorted>" (a lane per entity that moves
 * or rotates, whole environments per workgroup of <block> lanes, in natural
 * or size order), "pair-queue/<block>/<order>" (batches with boxes or
 * segments, environments of at most 32 entities: every pair tested and
 * evaluated once from LDS queues), "pair-queue/<block>/natural/even" (the
 * same with a whole number of workgroups per compute unit, each filled to an
 * equal share of the lanes), "quad/256" (sphere batches with at most 4
 * movers and 4 static collidable entities per environment),
 * "quad-ordered/64" (the same when the movers are the first entities of
 * every environment), "bucketed/<lo>-<hi>:<plan>/..." (sphere batches whose
 * environment sizes span several of the buckets 1-4, 5-8, 9-16, 17-32,
 * 33-64, 65-: every bucket runs its own plan, chosen per bucket, and the
 * buckets' launches run at the same time on side streams of the handle,
 * joined back into the caller's stream); "" for an id whose plan does not
 * fit the batch. vmas_autotune first times, for every size bucket, each
 * candidate plan on that bucket alone and chooses per bucket, then times
 * each plan on a T-step rollout of a scratch copy of `state` (state itself
 * is not modified) with the given actions (device float32 [T][A][2]; NULL:
 * actions drawn in the kernel, seed 12345): about 20 ms of warm-up on the
 * current plan, then three rounds over all plans with two timed runs each;
 * a plan's time is its fastest run, and a later plan replaces the current
 * choice only when it is at least 3 % faster. The choice is cached in the
 * process, keyed by the device architecture, the histogram of environment
 * shapes (size, movers, static collidables) and the rollout length rounded
 * up to a power of two; a later batch of the same key takes it without
 * timing (vmas_batch_info.tune_cached). With the environment variable
 * VMAS_AUTOTUNE_CACHE naming a file, the cache is also read from and
 * appended to that file. Returns the plan id in *chosen (and makes it
 * current). It synchronises the stream; it allocates one state-sized scratch
 * buffer for the duration of the call. */
vmas_status vmas_set_schedule(vmas_batch* batch, int32_t schedule);
vmas_status vmas_autotune(vmas_batch* batch, const float* state, const float* actions, int32_t T,
                          void* stream, int32_t* chosen);
const char* vmas_schedule_name(const vmas_batch* batch, int32_t schedule);

/* Rollout through a cached hipGraph: the first call builds a graph that
 * holds the rollout kernel as its one node (built explicitly, not captured,
 * so any stream works); later calls with the same T, the same plan and
 * actions given or drawn alike rebind the kernel arguments and launch the
 * graph on `stream`. Calls with traj or final_mask, or T <= 0, run
 * vmas_rollout. Same arguments and results as vmas_rollout. */
vmas_status vmas_rollout_graph(vmas_batch* batch, float* state, const float* actions,
                               uint64_t action_seed, int32_t t0, int32_t T, float* traj,
                               uint8_t* final_mask, void* stream);

/* ---- Learned contact surrogate -------------------------------------------
 * A 12 -> 128 -> 128 -> 2 MLP with tanh hidden layers mapping pair features
 * to the Eq. (2) contact force, with hand-written forward, backward and Adam
 * kernels: products on the matrix cores with BF16 operands and FP32
 * accumulation, everything else FP32. This is an addition to the paper's
 * method (which has no learned component). Parameters are one FP32 vector
 * in the order W1 [128][12], b1 [128], W2 [128][128], b2 [128], W3 [2][128],
 * b3 [2] (row-major, output index first). Training minimises the mean
 * squared error L = sum((y - t)^2) / (2 n). The handle owns its parameters,
 * Adam moments (beta1 0.9, beta2 0.999, eps 1e-8) and workspaces; calls on
 * one handle must not overlap. X, Y, dY, targets, grad and dX are DEVICE
 * arrays owned by the caller: X [n][12], Y / dY / target [n][2]. */
/* Number of parameters (18434). */
int32_t vmas_mlp_num_params(void);

/* params: host FP32 [num_params], or NULL for a uniform(-1/sqrt(fan_in),
 * 1/sqrt(fan_in)) initialisation drawn from `seed`. Blocks. */
vmas_status vmas_mlp_create(const float* params, uint64_t seed, int device, vmas_mlp** out);
vmas_status vmas_mlp_destroy(vmas_mlp* mlp);

/* Copies the FP32 parameters to host memory out [num_params]; synchronises `stream`. */
vmas_status vmas_mlp_get_params(const vmas_mlp* mlp, float* out, void* stream);

/* Y = f(X). */
vmas_status vmas_mlp_forward(vmas_mlp* mlp, const float* X, int64_t n, float* Y, void* stream);

/* Given dL/dY, the gradients dL/dparams (device [num_params], or NULL) and
 * dL/dX (device [n][12], or NULL). Deterministic: the batch is reduced in a
 * fixed order, no float atomics. */
vmas_status vmas_mlp_backward(vmas_mlp* mlp, const float* X, int64_t n, const float* dY,
                              float* grad, float* dX, void* stream);

/* One Adam step on the mean squared error of the batch; loss (device [1] or
 * NULL) receives the loss before the step. */
vmas_status vmas_mlp_train_step(vmas_mlp* mlp, const float* X, const float* target, int64_t n,
                                float lr, float* loss, void* stream);

/* Surrogate inputs and targets. For the pair slots listed in `slots`
 * (device int64 [m], mask order; NULL: all P slots, m = P) writes, for the
 * pair (i, j), i < j, in the pair frame e = (c_i - c_j)/|c_i - c_j| of angle phi:
 *   features  device float32 [m][12]: min(max(g / Lk, -16), 16), g / L with
 *             g = |c_i - c_j| - R_i - R_j (bounding radii: sphere r, box half
 *             diagonal, line L/2), cos and sin of (theta_i - phi), cos and sin
 *             of (theta_j - phi) (1 and 0 for spheres), dims_i / L, dims_j / L,
 *             shape codes of i and j (sphere 0, box 0.5, line 1); L = 0.1,
 *             Lk = 0.001;
 *   targets   device float32 [m][2] or NULL: the exact Eq. (2) force on i along
 *             e and along its left normal, divided by c * 0.02 (0 when not in
 *             contact or not a candidate);
 *   flags     device uint8 [m]: bit 0 network candidate (eligible pair without
 *             a segment, g <= band), bit 1 candidate in contact (exact FP32
 *             decision). Pairs with a segment are never candidates: the
 *             surrogate step gives them the exact narrow phase. */
vmas_status vmas_pair_features(vmas_batch* batch, const float* state, float band,
                               const int64_t* slots, int64_t m, float* features, float* targets,
                               uint8_t* flags, void* stream);

/* One step whose contact forces come from the surrogate network for every
 * candidate pair (bit 0 above), read through Eq. (2): a pair whose predicted
 * penetration k log(expm1(|f|/(c k))) exceeds fallback_frac times its half
 * size (sphere r; box half of the smaller side) takes the exact narrow phase
 * and Eq. (2) force; otherwise f is replaced by the nearest force Eq. (2) can
 * produce: 0 when |f| < F0/2, else f scaled up to at least F0 = c k ln 2 (the
 * force at zero penetration). Pairs
 * with a segment always take the exact narrow phase; joints are exact. The
 * surrogate gives no torque. forces: device [3][N] or NULL; n_fallback:
 * device int32 counter or NULL (incremented by the number of fallback pair
 * sides). The first call allocates a workspace of P x 60 bytes. Errors:
 * VMAS_ERR_INVALID_ARGUMENT (NULL handles, band < 0, 2^31 or more pair slots). */
vmas_status vmas_step_surrogate(vmas_batch* batch, vmas_mlp* mlp, float* state,
                                const float* actions, float band, float fallback_frac,
                                float* forces, int32_t* n_fallback, void* stream);

/* VMAS_DEBUG_NONFINITE batches only: synchronises `stream`, then writes
 * marks (host uint8 [n_envs], or NULL): 1 for every environment that has held
 * a non-finite state since creation or the last clear, and count (host, or
 * NULL): their number. clear != 0 then unmarks all environments.
 * VMAS_ERR_INVALID_ARGUMENT for a batch created without the flag. */
vmas_status vmas_nonfinite_envs(vmas_batch* batch, uint8_t* marks, int32_t* count, int32_t clear,
                                void* stream);

/* Reason for the last failure on this thread ("" if none). */
const char* vmas_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VMAS_H */
