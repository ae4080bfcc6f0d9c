// ag_internal.h -- kernel argument blocks and kernel lookup shared by the
// kernel translation unit and the host runtime (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ag {

// Statistics slot written by one block of a step launch (64 bytes).
struct StatSlot {
    long long n_saturated;   // accumulated over launches until folded
    long long n_resets;      // accumulated over launches until folded
    long long n_nonfinite;   // final state of the launch
    long long n_finite;
    long long n_position;
    double pos_err_sum;
    double omega_sum;
    double pad;
};

// Cumulative statistics kept on the device.
struct StatAcc {
    long long steps, n_saturated, n_resets, n_invalid_mode;
    long long n_nonfinite, n_finite, n_position;
    double pos_err_sum, omega_sum;
};

// Reset events of one fused launch (steps tb .. tb + k - 1, k <= 64), found
// and redrawn before the launch by dense kernels, so that the step loop only
// copies a redrawn state: bits[i] has bit j set when vehicle i resets before
// step tb + j; off[i] is the index of its first event in vehicle-major order;
// list[e] = (i << 6) | j; data is [16][cap] (13 state rows, 3 goal rows).
// Events with index >= cap are redrawn in the step loop itself.
struct EvBufs {
    unsigned long long* bits;  // [n]
    int32_t* off;              // [n]
    long long* block_counts;   // [nblocks of 256 vehicles] (counts, then exclusive offsets)
    long long* total;          // [1]
    long long* list;           // [cap]
    float* data;               // [16][cap]
    long long cap;
};

// Work-queue kernel: kQueueSub queues per XCD, each with a ticket counter and
// a done count in a line of kQueueLine words of its own.
constexpr int kQueueSub = 4;
constexpr int kQueueLine = 64;
constexpr int kQueueWords = 8 * kQueueSub * kQueueLine;

struct StepArgs {
    float* state;              // [13][ld] (read and written in place)
    const int8_t* mode;        // [ld]
    float* target;             // [4][ld] (goals rewritten by resets)
    const float* vparams;      // [16][ld] or null
    const float* traj;         // [16][ld] or null (tracking mode)
    const float* gtab;         // [n_groups][GSTRIDE]
    const int32_t* goff;       // [n_groups + 1]
    float* wrench_out;         // [8][ld] or null
    float* rotor_out;          // [8][ld] or null
    uint8_t* flags_out;        // [ld] or null
    float* goal;               // [3][ld] or null: redrawn for reset vehicles
    StatSlot* slots;           // [grid] or null
    const long long* d_step;   // device step counter (graph launches) or null
    long long t0;              // first global step when d_step is null
    long long t_off;           // added to *d_step
    long long n, ld;
    int32_t n_groups;
    int32_t span;              // max groups overlapping one tile (LDS entries)
    int32_t k;                 // steps per launch
    int32_t flags_accumulate;  // OR flags into flags_out instead of overwriting
    float dt, g;
    uint32_t key0, key1;       // reset generator key
    unsigned long long thr;    // reset threshold (word < thr)
    uint32_t index_base;
    float lo[3], hi[3];
    EvBufs ev;                 // reset events (RESET kernels)
    const int32_t* perm;       // [n] vehicle of each lane position (fused kernels), or null: identity
    unsigned* queue;           // [kQueueWords] tile queues of the work-queue kernel (zero between launches)
    int32_t ev_stage;          // event-fed kernels: the launch's LDS holds the per-wavefront event copies
};

struct ResetArgs {
    float* state;
    const int8_t* mode;
    float* target;
    const uint8_t* mask_in;    // or null: counter-based mask
    float* goal;               // [3][ld] or null
    uint8_t* mask_out;         // [n]
    int32_t* block_counts;     // [nblocks]
    long long n, ld;
    long long t;
    uint32_t key0, key1;
    unsigned long long thr;
    uint32_t index_base;
    float lo[3], hi[3];
};

struct RolloutArgs {
    const float* x0;           // [13][ld]
    const int8_t* mode;
    const float* target;
    const float* vparams;      // required
    const float* gtab;
    const int32_t* goff;
    float* ckpt;               // [n_ckpt][13][n]
    float* tape;               // [m][13][n]
    float* loss_out;           // [n] or null
    double* loss_part;         // [ceil(n / 64)] FP64 loss sums of 64 vehicles, or null
    float* final_state;        // [13][ld] or null
    const float* gains;        // [10][ld] gains of the rollout, or null: vparams rows
    const float* seed_dev;     // [1] device factor of the gradients, or null
    float* dgains;             // [10][ld]
    float* dx0;                // [13][ld]
    long long n, ld;
    int32_t n_groups, span;
    int32_t T, m, n_ckpt;
    float dt, g, w_omega, seed_grad;
    float inv_n;               // 1/n in FP32 (the batch mean's factor)
};

constexpr int kMaxSpanLds = 160;   // groups per tile that fit the LDS budget

// Kernel lookup (defined in ag_kernels.hip).  nr_class: 4, 6 or 8 rotors in
// every group, or 0 for a launch mixing rotor counts.  rst: 0 no resets; 1
// resets (a fused launch takes them from the event kernels and redraws events
// past the buffer itself); 2 fused launch whose events all fit the buffer.
// A fused launch with resets runs the rst = 2 and rst = 1 kernels in turn;
// each leaves at once unless the launch's event count selects it.
const void* step_kernel(int nr_class, bool vp, int rst, int vpl, bool one_step, bool obs, bool trk);
// The work-queue form of the fused kernel (exec kind 2: single group, no
// observers, resets, trajectories or per-vehicle parameters, one vehicle per
// lane, blocks of 64) and its dynamic LDS.
const void* step_queue_kernel(int nr_class);
size_t step_queue_lds_bytes();
const void* fold_kernel();
const void* advance_kernel();
const void* set_step_kernel();
const void* set_targets_kernel();
const void* reset_mask_kernel();
const void* reset_scan_kernel();
const void* reset_scatter_kernel();
const void* clear_slots_kernel();
const void* rollout_fwd_kernel(int nr_class);
const void* rollout_adj_kernel(int nr_class);

// Batch loss: fixed-order FP64 sum of the per-64-vehicle partials, times 1/n.
struct LossFoldArgs {
    const double* part;
    int32_t nparts;
    double inv_n;
    float* out;                // [1]
};
const void* loss_fold_kernel();

struct FoldArgs {
    StatSlot* slots;
    int32_t nslots;
    StatAcc* acc;
    long long steps;
    int32_t has_final;
};

struct SetTargetsArgs {
    int8_t* mode_dst;
    float* target_dst;
    const int8_t* mode_src;
    const float* target_src;
    long long ld, src_ld, first, count;
    StatAcc* acc;
};

struct ScanArgs {
    int32_t* block_counts;     // in: counts, out: exclusive offsets
    int32_t nblocks;
    int32_t* count_out;        // or null
};

struct ScatterArgs {
    const uint8_t* mask;
    const int32_t* offsets;
    int32_t* indices;
    long long n;
};

struct CounterArgs {
    long long* d_step;
    long long value;
};

struct ClearArgs {
    StatSlot* slots;
    int32_t nslots;
};

constexpr int kResetBlock = 256;

struct ObstArgs {
    const float* slots;        // [n_obs][20]
    const float* env_lo;       // [3][ld] or null (box_lo for every env)
    const float* env_hi;
    const uint8_t* mask;       // [n_env] or null (all)
    float* out;                // [7][out_ld]
    long long n_env, ld, out_ld, t;
    int32_t n_obs;
    uint32_t key0, key1, index_base;
    float box_lo[3], box_hi[3];
};

const void* obstacles_kernel();

struct CameraArgs {
    const float* state;        // [13][ld] vehicle poses
    const float* shapes;       // [n_obs][8]
    const float* obst;         // [7][obst_ld]
    float* depth;              // [count][H][W]
    long long ld, obst_ld, first;
    int32_t n_obs, W, H, has_floor;
    float inv_f, max_depth, floor_z;
    float mount_p[3], mount_q[4];
};

const void* depth_kernel();

struct ActArgs {
    const float* actions;      // [4][act_ld]
    float* target;             // [4][ld]
    int8_t* mode;
    long long n, ld, act_ld;
    int32_t new_mode;
    float scale[4], offset[4];
};

struct TaskArgs {
    const float* state;        // [13][ld]
    const float* goal;         // [3][goal_ld]
    float* obs;                // [13][obs_ld]
    float* reward;             // [n] or null
    uint8_t* done;             // [n] or null
    int32_t* episode;          // [n] or null
    long long n, ld, goal_ld, obs_ld;
    int32_t advance, max_steps;
    float w_v, w_omega, bonus, r_goal, r_far;
};

const void* actions_kernel();
const void* observe_kernel();

// Reset events of a fused launch: mask (bits and per-block counts), scan,
// scatter (per-vehicle offsets and the event list), redraw (one lane per
// event).  They take the launch's StepArgs (steps, keys, threshold, bounds, ev).
const void* ev_mask_kernel();
const void* ev_scan_kernel();
const void* ev_scatter_kernel();
const void* ev_redraw_kernel();

// Mode order of a fused launch: in every segment of kOrderSeg consecutive
// vehicles, the vehicles of each group are listed stably by command mode
// (0, 1, 2, then every other code), so that wavefronts hold one mode; each
// vehicle stays in its segment and its group.  A segment split by more than
// kOrderPieces groups is listed in index order.
constexpr int kOrderSeg = 4096;
constexpr int kOrderPieces = 8;
constexpr int kOrderBlock = 256;
// fused launches of at least this many steps per call use the order
constexpr int kOrderMinSteps = 32;
struct OrderArgs {
    const int8_t* mode;
    const int32_t* goff;
    int32_t* perm;
    long long n;
    int32_t n_groups;
};
const void* mode_order_kernel();

}  // namespace ag
