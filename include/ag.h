/*
 * ag.h -- C ABI of the batched multirotor step on MI355X (gfx950).
 *
 * The operation behind every call is the per-vehicle step of the parallel
 * SE(3) geometric controller of Kulkarni, Forgaard and Alexis, "Aerial Gym --
 * Isaac Gym Simulator for Aerial Robots" (arXiv 2305.16510):
 *   - controller, Sec. IV: attitude mode (Sec. IV-A, eqs. (1)-(5)), velocity
 *     mode (Sec. IV-B, eqs. (6)-(9)), position mode (named in Sec. I), plus a
 *     wrench pass-through test mode;
 *   - allocation of (f, M) to clamped rotor thrusts (the paper applies f and M
 *     directly; Sec. II motivates modelling the rotor reaction torque);
 *   - rigid-body Newton-Euler dynamics with quaternion integration (the part
 *     the paper hands to its physics engine, Sec. I and end of Sec. IV-B).
 * Vehicles are independent (data parallel over the batch, Sec. III and VI).
 *
 * Conventions.  All device arrays are structure-of-arrays with a common
 * leading dimension `ld` (elements, ld >= n): row r of an array with R rows
 * starts at element r*ld.  Vehicle i's state is
 *   state[r*ld + i], r = 0..12: x(3) [m], v(3) [m/s], q(4) = (w, x, y, z)
 *   Hamilton unit quaternion body->inertial, Omega(3) [rad/s] in the body frame.
 * The inertial frame is z-up, gravity is -g e3, rotor thrust acts along +b3.
 * mode[i] (int8) selects the command held in target[r*ld + i], r = 0..3:
 *   0 position : (x_d, y_d, z_d, psi_d)              in the inertial frame
 *   1 velocity : (v_d x, y, z in the vehicle frame V, psidot_d)   (eqs. (6)-(9))
 *   2 attitude : (phi_d, theta_d, psidot_d, f)                   (eqs. (1)-(5))
 *   3 wrench   : (f, M_x, M_y, M_z) passed to allocation (test mode)
 *   other      : zero wrench command
 * vparams (optional) rows: m, J1, J2, J3, 10 gains
 *   (kx_xy, kx_z, kv_xy, kv_z, kR_x, kR_y, kR_z, kW_x, kW_y, kW_z), arm, u_max.
 *
 * Ownership.  The caller owns every device buffer (state, mode, target,
 * vparams, outputs, workspaces) and keeps them alive while the handle uses
 * them.  The library never allocates device memory; it owns only host-side
 * bookkeeping and HIP graph objects.  All work is enqueued on cfg.stream.
 *
 * Errors.  Arguments are checked synchronously (AG_E_INVALID).  Device and
 * launch failures are sticky: the failing call and every later call on the
 * handle return AG_E_HIP until ag_destroy; ag_last_error gives the text.
 * Non-finite vehicles are not errors: they are flagged per vehicle.
 * A handle is not thread safe.
 */
#ifndef AG_H
#define AG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AG_STATE_DIM 13
#define AG_TARGET_DIM 4
#define AG_VPARAM_DIM 16
#define AG_NGAINS 10
#define AG_MAX_ROTORS 8
#define AG_WRENCH_DIM 8
#define AG_MAX_GROUPS 4096

typedef struct ag_sim* ag_handle;

typedef enum {
    AG_OK = 0,
    AG_E_INVALID = 1,     /* bad argument; nothing was enqueued */
    AG_E_HIP = 2,         /* HIP runtime or launch failure (sticky) */
    AG_E_NOMEM = 3,       /* a caller workspace is too small */
    AG_E_STATE = 4,       /* call not valid in the handle's current state */
    AG_E_UNSUPPORTED = 5  /* feature combination not implemented */
} ag_status;

/* Mode 4 (AG_MODE_TRACK) is the full geometric tracking law of Lee et al.,
 * the reference the paper adapts (Sec. IV): desired frame from the force
 * direction and a heading b1d = (cos psi_d, sin psi_d, 0), and the moment's
 * feed-forward term -J (hat(Omega) R^T R_d Omega_d - R^T R_d dOmega_d) that the
 * paper drops after eq. (5) restored.  It reads cfg.traj (16 rows per vehicle:
 * x_d(3), v_d(3), a_d(3), psi_d, Omega_d(3), dOmega_d(3)); without cfg.traj a
 * mode-4 vehicle gets a zero wrench.  Commands and trajectory rows are read
 * once per launch and held for the steps of that launch. */
#define AG_TRAJ_DIM 16
enum { AG_MODE_POSITION = 0, AG_MODE_VELOCITY = 1, AG_MODE_ATTITUDE = 2, AG_MODE_WRENCH = 3, AG_MODE_TRACK = 4 };

/* Per-vehicle flag bits written to cfg.flags_out at the end of each ag_step. */
enum { AG_FLAG_NONFINITE = 1, AG_FLAG_SATURATED = 2, AG_FLAG_RESET = 4 };

/* A contiguous range of vehicles sharing a rotor layout and default
 * parameters.  Rotor layout (n_rotors in {4, 6, 8}): rotors at angles
 * pi/n + 2 pi i/n in the body x-y plane at `arm`, spin (-1)^i, yaw torque
 * c_tau per newton of thrust; thrusts are clamped to [u_min, u_max]. */
typedef struct {
    int64_t first, count;
    int32_t n_rotors;
    float arm, c_tau, u_min, u_max;
    float mass;
    float inertia[3];
    float gains[AG_NGAINS];
} ag_group_desc;

typedef struct {
    int64_t n;              /* vehicles, 1 .. 2^31-1 */
    int64_t ld;             /* leading dimension of every SoA array, >= n */
    float dt;               /* step [s] */
    float g;                /* gravity [m/s^2] */
    uint64_t seed;          /* key of the counter-based reset generator */
    int64_t index_base;     /* global index of vehicle 0 (reset counters), index_base + n <= 2^32 */
    void* stream;           /* hipStream_t; graphs are used only on a non-null stream */
    int32_t n_groups;       /* 1 .. AG_MAX_GROUPS, covering [0, n) in order */
    const ag_group_desc* groups;   /* host array, copied by ag_create */
    float* state;           /* device [13][ld], read and written by ag_step / ag_reset */
    int8_t* mode;           /* device [ld] */
    float* target;          /* device [4][ld]; ag_reset and automatic resets rewrite goals */
    const float* vparams;   /* device [16][ld] or NULL (group defaults) */
    float* wrench_out;      /* device [8][ld] or NULL: commanded f, M and applied f', M' of the last step */
    float* rotor_out;       /* device [8][ld] or NULL: clamped rotor thrusts of the last step (zero-padded) */
    uint8_t* flags_out;     /* device [ld] or NULL: AG_FLAG_* bits of the last ag_step call */
    float reset_prob;       /* probability of the counter-based reset mask (per vehicle and step) */
    int32_t auto_reset;     /* 1: ag_step resets masked vehicles before every step */
    float reset_lo[3];      /* box of redrawn positions and goals [m] */
    float reset_hi[3];
    int32_t collect_stats;  /* 1: ag_step accumulates the ag_stats counters and final-state sums */
    int32_t autotune_scratch;  /* 1: workspace holds scratch state so ag_autotune leaves results untouched */
    const float* traj;      /* device [16][ld] or NULL: trajectory rows of mode 4 (see AG_MODE_TRACK) */
    float* goal;            /* device [3][ld] or NULL: goal of the goal-reaching task (ag_observe);
                               every reset (explicit or automatic) redraws it for the reset vehicles */
} ag_config;

/* Execution policy of ag_step.  kind 0: one launch of the per-step kernel per
 * step (plain launches, one vehicle per lane).  kind 1: fused kernel keeping
 * state in registers for k steps per launch, vpl vehicles per lane, a grid-
 * stride loop over tiles of block*vpl vehicles (grid 0 = one block per tile),
 * replayed from a cached HIP graph when use_graph is 1 and the stream is not
 * null.  Every policy gives bitwise identical states.  With automatic resets
 * a fused launch first finds, lists and redraws the resets of its k steps
 * (k <= 64 then) in dense kernels, holding up to one event per vehicle in
 * the workspace; events beyond that are redrawn in the step loop.
 * kind 2: the fused kernel in work-queue form (block 64, vpl 1; a single
 * vehicle group and no observers, trajectories, per-vehicle parameters or
 * automatic resets, else AG_E_INVALID): a grid of grid wavefronts (0: as
 * many as the chip holds at once; rounded down to a multiple of 32, at
 * least 32) takes tiles of 64 vehicles on demand from 32 queues in the
 * workspace and copies the next tile's rows into LDS while it steps the
 * current one.
 * Launches of one handle share the queues, so they must not overlap (they
 * are ordered on the handle's stream). */
typedef struct {
    int32_t kind, block, vpl, k, grid, use_graph;
} ag_exec;

/* Batch statistics since the last clear.  Counters: saturated rotor commands
 * (rotor-steps with the raw command outside [u_min, u_max]), automatic
 * resets, invalid mode codes seen by ag_set_targets, steps taken.  Final-
 * state values describe the state after the last ag_step. */
typedef struct {
    int64_t steps;
    int64_t n_saturated;
    int64_t n_resets;
    int64_t n_invalid_mode;
    int64_t n_nonfinite;    /* vehicles with a non-finite state */
    int64_t n_finite;
    int64_t n_position;     /* finite position-mode vehicles */
    double pos_err_sum;     /* sum of |x - x_d| over finite position-mode vehicles */
    double omega_sum;       /* sum of |Omega| over finite vehicles */
} ag_stats;

/* Device workspace (bytes) that ag_create needs for this configuration. */
ag_status ag_workspace_size(const ag_config* cfg, size_t* bytes);

/* Create a batch of cfg->n independent vehicles (Sec. III: many environments
 * simulated in parallel, one robot each; Sec. VI: the throughput is that of the
 * whole batch).  Validate cfg, build the per-group tables (rotor allocation
 * matrix and its min-norm pseudo-inverse, inverse mass and inertia) in FP64 on
 * the host, round them to FP32 and upload them into `workspace` (device, >=
 * the size from ag_workspace_size, 256-byte aligned; owned by the caller,
 * which keeps it alive until ag_destroy).  Enqueues on cfg->stream and waits
 * for it.  AG_E_INVALID: cfg fails validation (message on stderr) or a rotor
 * layout's tables lack the structure the kernels assume; AG_E_NOMEM:
 * workspace too small; AG_E_HIP: a copy or launch failed.  *out is NULL on
 * failure. */
ag_status ag_create(const ag_config* cfg, void* workspace, size_t workspace_bytes, ag_handle* out);

/* Wait for the handle's stream, then release the host-side handle and its
 * graphs (device buffers stay with the caller).  The handle is freed even
 * when the wait reports a device error (returned as AG_E_HIP). */
ag_status ag_destroy(ag_handle h);

/* New commands for vehicles [first, first+count) (Sec. IV: the high-level
 * position, velocity or attitude commands a user gives each vehicle; Sec. III:
 * the per-environment action of a Gym-style step): copies mode_src[i] and
 * target_src[r*src_ld + i] (device pointers; NULL = keep the bound buffers'
 * contents) into the bound buffers and checks the mode codes; invalid codes
 * are counted in ag_stats.n_invalid_mode (such vehicles get a zero wrench).
 * Call it over any range of the bound mode or target buffers written
 * directly, so that data the handle derives from the commands is renewed. */
ag_status ag_set_targets(ag_handle h, int64_t first, int64_t count, const int8_t* mode_src,
                         const float* target_src, int64_t src_ld);

/* Advance every vehicle by n_steps steps (controller, allocation, clamping,
 * integration; with auto_reset, the counter-based reset before each step),
 * asynchronously on the handle's stream, with the current execution policy.
 * Operation: one step is the map of Sec. IV (command of the vehicle's mode,
 * desired attitude and rate, eqs. (1)-(2), errors and moment, eqs. (3)-(5);
 * velocity mode eqs. (6)-(9)) followed by allocation and the rigid-body
 * update the paper delegates to its physics engine (Sec. I, end of Sec. IV-B);
 * the batch is stepped in lock step, as the environments of Sec. III.
 * Fused launches with one vehicle per lane, no trajectory buffer, no
 * observers and no automatic resets run the vehicles of each group in an
 * order by command mode within segments of 4,096 (workspace), so that
 * wavefronts of one mode run that mode's copy of the step loop.  The order is
 * computed by the first such call of 32 or more steps (or by ag_prepare or
 * ag_autotune) and kept until ag_set_targets or ag_apply_actions changes the
 * commands; a call shorter than 32 steps with no current order runs without
 * it.  The order decides only which lanes share a wavefront: results are
 * bitwise those of any other policy, also when the mode buffer was written
 * directly (the order is then merely stale; ag_set_targets over the written
 * range renews it). */
ag_status ag_step(ag_handle h, int32_t n_steps);

/* Prepare ag_step(h, n_steps) under the current execution policy without
 * stepping: build, cache and upload to the device the HIP graph it will
 * replay (when the policy uses graphs), and compute the mode order when the
 * policy's fused launches use one and it is not current (one launch on the
 * handle's stream).  A prepared call of any length then runs in mode order. */
ag_status ag_prepare(ag_handle h, int32_t n_steps);

ag_status ag_set_exec(ag_handle h, const ag_exec* e);
ag_status ag_get_exec(ag_handle h, ag_exec* e);

/* Choose the fused policy for calls of probe_steps steps: time candidate
 * fused policies (block 64..512, vehicles per lane 1 or 2, k the powers of
 * two from 4 to 1024 up to probe_steps and probe_steps itself, grid one block
 * per tile or a persistent multiple of the CU count) on probe_steps-step
 * calls and keep the fastest; synchronises the stream.  With
 * autotune_scratch the probes write scratch buffers, so the state is
 * untouched; without it the call returns AG_E_STATE.  The choice is cached
 * for the process, and appended to the text file named by the environment
 * variable AG_AUTOTUNE_CACHE when it is set (read once per process), under a
 * key of the device architecture and CU count, n, the group layout (counts and
 * rotor counts), the kernel class (rotor class, per-vehicle parameters,
 * automatic resets, observers, trajectories, graphs) and probe_steps; a later
 * call with the same key takes the cached policy without timing.  Every
 * policy gives bitwise identical results. */
ag_status ag_autotune(ag_handle h, int32_t probe_steps, ag_exec* chosen);

/* Reset vehicles before global step `step` (Sec. III: environments are reset
 * individually, Gym-style; Sec. V: the asset manager randomises at reset, here
 * the vehicle's state and goal): the mask is mask_in (device uint8[n], nonzero
 * = reset) or, if NULL, the counter-based mask for that step (Philox4x32-10
 * keyed by cfg.seed, one draw per global vehicle index and step, reset when
 * the first word is below floor(reset_prob 2^32)).  Reset vehicles get a
 * redrawn state and, in position mode, goal.  Optionally writes mask_out
 * (uint8[n]), the ascending indices of reset vehicles (indices_out, int32[n])
 * and their number (count_out, int32[1]); all outputs are device pointers.
 * Asynchronous on the handle's stream; AG_E_INVALID for step < 0. */
ag_status ag_reset(ag_handle h, const uint8_t* mask_in, int64_t step, uint8_t* mask_out,
                   int32_t* indices_out, int32_t* count_out);

/* Obstacle poses at environment reset (Sec. V, asset manager): every
 * environment (one per vehicle, index i) holds n_obs obstacle slots.  For each
 * environment in env_mask (device uint8[n], nonzero = reset; NULL = all), slot
 * k gets a position lo + (hi - lo) * frac with frac_a in [frac_lo_a, frac_hi_a]
 * of the environment box (env_lo/env_hi device [3][ld] per environment, or
 * NULL to use box_lo/box_hi for all) and an attitude from Z-Y-X Euler angles
 * (roll, pitch, yaw) in [eul_lo, eul_hi]; dimensions whose lock bit is set
 * take lock_val (a fraction for x, y, z, an angle for roll, pitch, yaw).
 * slots: device [n_obs][20] floats = frac_lo(3), frac_hi(3), eul_lo(3),
 * eul_hi(3), lock bits (x, y, z, roll, pitch, yaw as bits 0-5, stored as a
 * float), lock_val(6), unused(1).  Output obstacle i*n_obs + k as rows
 * (x, y, z, qw, qx, qy, qz) of out (device [7][out_ld], out_ld >= n*n_obs);
 * rows of environments not reset are left untouched.  Draws come from the
 * handle's counter-based generator at step `step` (0 <= step < 2^32). */
ag_status ag_randomize_obstacles(ag_handle h, int32_t n_obs, const float* slots, const float* env_lo,
                                 const float* env_hi, const float* box_lo, const float* box_hi,
                                 const uint8_t* env_mask, int64_t step, float* out, int64_t out_ld);

/* Pinhole depth camera mounted on each vehicle (Sec. III: cameras with a
 * configurable pose on the robot; Sec. I and VII: ray casting for depth).
 * Camera frame: x forward, y left, z up; pixel (u, v) of a width x height
 * image looks along normalize(1, -(u + 1/2 - W/2)/f, -(v + 1/2 - H/2)/f) with
 * f = (W/2) / tan(hfov/2). */
typedef struct {
    int32_t width, height;
    float hfov;             /* horizontal field of view [rad], in (0, pi) */
    float max_depth;        /* [m]: value of pixels with no hit or a deeper hit */
    float floor_z;          /* floor plane z [m] seen from above; NaN = no floor */
    float mount_pos[3];     /* camera position in the body frame [m] */
    float mount_quat[4];    /* camera attitude in the body frame (w, x, y, z), unit */
} ag_camera;

/* Depth images of vehicles [first, first + count): depth[(i - first)][v][u]
 * (device, count * height * width floats) is the distance along the optical
 * axis to the first entry of the ray into an obstacle of vehicle i's
 * environment or into the floor (the exit when the camera is inside an
 * obstacle), or max_depth.  Obstacles: n_obs (<= 256) per environment with
 * poses in rows (x, y, z, qw, qx, qy, qz) of obst (device [7][obst_ld],
 * obstacle i*n_obs + k, the layout of ag_randomize_obstacles) and shapes
 * (device [n_obs][8]): type 0 box (half extents x, y, z), 1 sphere (radius),
 * 2 cylinder along its z axis (radius, half height). */
ag_status ag_render_depth(ag_handle h, const ag_camera* cam, int32_t n_obs, const float* shapes, const float* obst,
                          int64_t obst_ld, int64_t first, int64_t count, float* depth);

/* Goal-reaching task of a Gym-style vectorised environment (Sec. III:
 * Gym-style interfaces; Sec. I: goal reaching with attitude and velocity
 * commands).  Actions (device [4][act_ld], one column per vehicle) are
 * clamped to [-1, 1] and mapped to commands target = offset + scale * a
 * (row-wise, 4 rows) for every vehicle, whose mode is set to `mode`.
 * Observation, reward and termination after a step, per vehicle:
 *   obs    = (goal - x, v, q, Omega)            rows of obs (device [13][obs_ld])
 *   reward = -|goal - x| - w_v |v| - w_omega |Omega| + bonus if |goal - x| < r_goal
 *   done   = episode >= max_steps or |goal - x| > r_far or a non-finite state
 * with goal = cfg.goal (or target rows 0-2 when cfg.goal is NULL) and the
 * per-vehicle episode counter (device int32[n]) incremented first and reset to
 * 0 for finished vehicles.  Non-finite vehicles get a zero observation and
 * reward.  With advance = 0 only obs is written (no counter, reward or done),
 * e.g. after resetting the finished vehicles with ag_reset(done mask). */
typedef struct {
    float w_v, w_omega, bonus, r_goal, r_far;
    int32_t max_steps;
} ag_task;

ag_status ag_apply_actions(ag_handle h, const float* actions, int64_t act_ld, int32_t mode, const float* scale,
                           const float* offset);
ag_status ag_observe(ag_handle h, const ag_task* task, int32_t advance, float* obs, int64_t obs_ld, float* reward,
                     uint8_t* done, int32_t* episode);

/* Synchronise and read the statistics (clear = 1 zeroes the counters). */
ag_status ag_get_stats(ag_handle h, ag_stats* out, int32_t clear);

/* Global step counter (number of steps taken; used by automatic resets). */
ag_status ag_get_step(ag_handle h, int64_t* step);
ag_status ag_set_step(ag_handle h, int64_t step);

/* Differentiable rollout of the tracking loss
 *   L = (1/n) sum_i sum_{t=1..T} ( |x_{i,t} - x_goal,i|^2 + w_omega |Omega_{i,t}|^2 )
 * over post-step states, x_goal = the position-mode target.  The paper trains
 * controllers and policies on the batched simulator (Sec. I, III); this
 * differentiates the controller-plus-dynamics rollout of Sec. IV with respect
 * to each vehicle's ten gains (eq. (5)'s k_R, k_Omega and the position and
 * velocity gains of eqs. (6)-(7), layout of cfg.vparams rows 4..13) and its
 * initial state.  Requires position or wrench modes and per-vehicle vparams.
 *   x0     device [13][ld] starting state, or NULL: the bound state (not modified)
 *   gains  device [10][ld] gains of the rollout, or NULL: vparams rows 4..13
 *          (the other vparams rows are always taken from cfg.vparams)
 * Forward: steps every vehicle n_steps times from x0, keeping the state every
 * ckpt_every steps in `ws`.  Outputs (device, each optional): loss_out [n],
 * vehicle i's sum over t (without 1/n); batch_loss [1], L itself, summed in
 * FP64 in a fixed order (per 64 vehicles, then over those partials), so that
 * equal inputs give a bitwise equal L; final_state [13][ld].
 * Adjoint: recomputes each checkpoint segment (into one of two tape buffers
 * in `ws`, overlapped with the reverse sweep of the later segment) and sweeps
 * it backwards, writing dL/dgains (dgains [10][ld]) and dL/dx0 (dx0 [13][ld])
 * multiplied by seed_grad and, when seed_dev (device float [1]) is not NULL,
 * by *seed_dev read on the device (an upstream gradient that need not be
 * copied to the host).  The adjoint reads the checkpoints of the forward call:
 * both calls take the same x0, gains, n_steps, ckpt_every, w_omega and
 * workspace, and the buffers they read must not change in between.
 * Workspace (caller-owned, 256-byte aligned, size from
 * ag_rollout_workspace_size): n_ckpt + 2 ckpt_every states of 13 floats per
 * vehicle, n_ckpt = ceil(n_steps / ckpt_every), and ceil(n / 64) doubles of
 * loss partials, each part 256-byte aligned.  Asynchronous on the handle's
 * stream.  AG_E_NOMEM: workspace missing, misaligned or small; AG_E_UNSUPPORTED:
 * no vparams, or a trajectory buffer is bound; AG_E_INVALID: n_steps or
 * ckpt_every < 1, non-finite w_omega, missing dgains or dx0. */
ag_status ag_rollout_workspace_size(ag_handle h, int32_t n_steps, int32_t ckpt_every, size_t* bytes);
ag_status ag_rollout_forward(ag_handle h, const float* x0, const float* gains, int32_t n_steps,
                             int32_t ckpt_every, float w_omega, void* ws, size_t ws_bytes, float* loss_out,
                             float* batch_loss, float* final_state);
ag_status ag_rollout_adjoint(ag_handle h, const float* x0, const float* gains, int32_t n_steps,
                             int32_t ckpt_every, float w_omega, float seed_grad, const float* seed_dev,
                             void* ws, size_t ws_bytes, float* dgains, float* dx0);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * forward and adjoint of the differentiable rollout above in one call,
 * ag_rollout_forward (per-vehicle and batch loss) followed by
 * ag_rollout_adjoint (seed_grad, no device factor), with the checkpoints,
 * tapes and loss partials in the library's own static device scratch instead
 * of a caller workspace.  Allocates nothing.  The scratch holds 192 MiB per
 * GPU (the 65,536-vehicle, 200-step, 20-step-checkpoint rollout needs 171 MB):
 * a rollout whose ag_rollout_workspace_size exceeds it is rejected with
 * AG_E_NOMEM and a message, nothing enqueued.  Every call on one GPU shares
 * that GPU's scratch (from any handle), so calls that overlap on one GPU
 * (different streams, threads or handles) race; calls on one stream do not.
 * Other arguments, outputs and errors as for the two calls it combines. */
ag_status ag_rollout_grad_noalloc(ag_handle h, const float* x0, const float* gains, int32_t n_steps,
                                  int32_t ckpt_every, float w_omega, float seed_grad, float* loss_out,
                                  float* batch_loss, float* dgains, float* dx0);

/* Wait for the handle's stream; returns a sticky error if one occurred. */
ag_status ag_sync(ag_handle h);
const char* ag_last_error(ag_handle h);
const char* ag_status_string(ag_status s);

#ifdef __cplusplus
}
#endif
#endif /* AG_H */
