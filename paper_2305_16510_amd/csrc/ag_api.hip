// ag_api.hip -- host runtime behind the C ABI of include/ag.h.
//
// Owns only host-side bookkeeping: validated configuration, workspace
// layout, the per-group tables (built in FP64, rounded to FP32 and copied
// into the caller's workspace), the step counter mirror, cached HIP graphs
// of fused rollouts and the autotuner.  Every device buffer belongs to the
// caller.  No hipMalloc anywhere.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ag.h"
#include "ag_internal.h"
#include "ag_step.h"

using namespace ag;

// Scratch of ag_rollout_grad_noalloc: checkpoints, tapes and loss partials of
// one differentiable rollout, in the code object's own device memory (each
// GPU the library is loaded on holds a copy until the process ends).  Host
// code never uses this name as an address: ag_create looks up each device's
// copy with hipGetSymbolAddress and keeps that pointer.
constexpr size_t kNoAllocScratchBytes = (size_t)192 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr size_t kAlign = 256;
constexpr int kRolloutBlock = 64;     // vehicles per block of the rollout kernels

// Device address of `scratch` on each device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// With device `dev` current: the address of its copy of `scratch` (null if
// the lookup failed; *err then says why).
void* device_scratch(int dev, hipError_t* err) {
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
        g_scratch_err[dev] = e;
        g_scratch_done[dev] = true;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct WsLayout {
    size_t gtab, goff, d_step, acc, slots, block_counts, mask, scratch, total;
    size_t ev_bits, ev_off, ev_bc, ev_total, ev_list, ev_data;
    size_t perm, queue;
    long long nslots, nblocks, ev_cap;
};

WsLayout ws_layout(const ag_config* c) {
    WsLayout L{};
    size_t off = 0;
    L.gtab = off; off = align_up(off + (size_t)c->n_groups * GSTRIDE * sizeof(float));
    L.goff = off; off = align_up(off + (size_t)(c->n_groups + 1) * sizeof(int32_t));
    L.d_step = off; off = align_up(off + sizeof(long long));
    L.acc = off; off = align_up(off + sizeof(StatAcc));
    L.nslots = (c->n + 63) / 64;
    L.slots = off; off = align_up(off + (size_t)L.nslots * sizeof(StatSlot));
    L.nblocks = (c->n + kResetBlock - 1) / kResetBlock;
    L.block_counts = off; off = align_up(off + (size_t)L.nblocks * sizeof(int32_t));
    L.mask = off; off = align_up(off + (size_t)c->n);
    L.perm = off; off = align_up(off + (size_t)c->n * sizeof(int32_t));
    L.queue = off; off = align_up(off + (size_t)kQueueWords * sizeof(unsigned));
    L.scratch = off;
    if (c->autotune_scratch) off = align_up(off + (size_t)(AG_STATE_DIM + AG_TARGET_DIM) * c->ld * sizeof(float));
    // reset events of fused launches (automatic resets): room for n events per
    // launch, i.e. one per vehicle; further events are redrawn in the step loop
    L.ev_cap = (c->auto_reset && c->reset_prob > 0.0f) ? c->n : 0;
    if (L.ev_cap > 0) {
        L.ev_bits = off; off = align_up(off + (size_t)c->n * sizeof(unsigned long long));
        L.ev_off = off; off = align_up(off + (size_t)c->n * sizeof(int32_t));
        L.ev_bc = off; off = align_up(off + (size_t)L.nblocks * sizeof(long long));
        L.ev_total = off; off = align_up(off + sizeof(long long));
        L.ev_list = off; off = align_up(off + (size_t)L.ev_cap * sizeof(long long));
        L.ev_data = off; off = align_up(off + (size_t)16 * L.ev_cap * sizeof(float));
    }
    L.total = off;
    return L;
}

struct ExecKey {
    int kind, block, vpl, k, grid, use_graph;
    bool operator==(const ExecKey& o) const {
        return kind == o.kind && block == o.block && vpl == o.vpl && k == o.k && grid == o.grid &&
               use_graph == o.use_graph;
    }
};

struct GraphEntry {
    int n_steps;
    bool ordered;      // fused launches read the mode order (kept in the workspace)
    ExecKey key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    unsigned long long stamp;
};

}  // namespace

struct ag_sim {
    ag_config cfg;
    std::vector<ag_group_desc> groups;
    std::vector<int32_t> goff_host;
    hipStream_t stream;
    char* ws;
    WsLayout L;
    float* gtab;
    int32_t* goff;
    long long* d_step;
    StatAcc* acc;
    StatSlot* slots;
    int32_t* perm;          // mode order of fused launches
    unsigned* queue;        // tile queues of the work-queue kernel (zero between launches)
    int q_occ;              // its wavefronts per CU (0: not yet queried, -1: query failed)
    bool order_valid;       // perm was computed since the last change of commands
    int32_t* block_counts;
    uint8_t* mask_buf;
    float* scratch;
    int nr_class;
    bool vp;
    bool reset_on;
    uint32_t key0, key1;
    unsigned long long thr;
    ag_exec exec;
    long long t;
    bool dev_step_dirty;
    std::vector<GraphEntry> graphs;
    unsigned long long stamp;
    ag_status sticky;
    std::string err;
    int num_cus;
    std::vector<std::pair<long long, int>> span_cache;
    EvBufs ev;
    void* noalloc_scratch;        // this device's copy of `scratch`, or null
    hipError_t noalloc_err;       // why the lookup failed
};

namespace {

ag_status set_err(ag_handle h, ag_status s, const std::string& msg) {
    if (h) {
        h->err = msg;
        if (s == AG_E_HIP) h->sticky = AG_E_HIP;
    }
    return s;
}

ag_status hip_fail(ag_handle h, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_err(h, AG_E_HIP, m);
}

#define AG_HIP(h, call)                                   \
    do {                                                  \
        hipError_t e__ = (call);                          \
        if (e__ != hipSuccess) return hip_fail(h, e__, #call); \
    } while (0)

#define AG_CHECK_HANDLE(h)                                \
    do {                                                  \
        if (!(h)) return AG_E_INVALID;                    \
        if ((h)->sticky != AG_OK) return (h)->sticky;     \
    } while (0)

// ---- FP64 group tables -------------------------------------------------------
// Rotor layout: n rotors at pi/n + 2 pi i/n, spin (-1)^i.  Unit-arm allocation
// columns (1, sin a, -cos a, s c_tau); pseudo-inverse A^T (A A^T)^{-1}.
bool invert4(double m[4][4], double inv[4][4]) {
    double a[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) a[i][j] = j < 4 ? m[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
        int p = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
        if (std::fabs(a[p][c]) < 1e-300) return false;
        for (int j = 0; j < 8; ++j) std::swap(a[c][j], a[p][j]);
        const double d = a[c][c];
        for (int j = 0; j < 8; ++j) a[c][j] /= d;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            for (int j = 0; j < 8; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) inv[i][j] = a[i][j + 4];
    return true;
}

bool build_group_entry(const ag_group_desc& g, float* e) {
    const int n = g.n_rotors;
    double A[4][8] = {};
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        const double al = pi / n + 2.0 * pi * i / n;
        const double s = (i % 2 == 0) ? 1.0 : -1.0;
        // sines and cosines that are zero in exact arithmetic (cos of 90 and
        // 270 degrees) come out of the library as ~1e-16: take them as zero
        double sa = std::sin(al), ca = std::cos(al);
        if (std::fabs(sa) < 1e-12) sa = 0.0;
        if (std::fabs(ca) < 1e-12) ca = 0.0;
        A[0][i] = 1.0;
        A[1][i] = sa;
        A[2][i] = -ca;
        A[3][i] = s * (double)g.c_tau;
    }
    double G[4][4] = {}, Gi[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            for (int i = 0; i < n; ++i) G[r][c] += A[r][i] * A[c][i];
    if (!invert4(G, Gi)) return false;
    for (int k = 0; k < GSTRIDE; ++k) e[k] = 0.0f;
    double pinv[8][4], cmax[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i) {
        for (int r = 0; r < 4; ++r) {
            double p = 0.0;
            for (int c = 0; c < 4; ++c) p += A[c][i] * Gi[c][r];
            pinv[i][r] = p;
            cmax[r] = std::max(cmax[r], std::fabs(p));
        }
    }
    for (int i = 0; i < n; ++i) {
        for (int r = 0; r < 4; ++r) {
            // entries that vanish in exact arithmetic come out of the FP64
            // inverse about 1e-16 times the column's largest entry
            const double p = std::fabs(pinv[i][r]) < 1e-12 * cmax[r] ? 0.0 : pinv[i][r];
            e[G_APINV + 4 * i + r] = (float)p;
            e[G_ACOL + 4 * i + r] = (float)A[r][i];
        }
    }
    e[G_UMIN] = g.u_min;
    e[G_UMAX] = g.u_max;
    e[G_ARM] = g.arm;
    e[G_INV_ARM] = (float)(1.0 / (double)g.arm);
    e[G_MASS] = g.mass;
    e[G_INV_MASS] = (float)(1.0 / (double)g.mass);
    for (int k = 0; k < 3; ++k) {
        e[G_J + k] = g.inertia[k];
        e[G_JINV + k] = (float)(1.0 / (double)g.inertia[k]);
    }
    for (int k = 0; k < AG_NGAINS; ++k) e[G_GAINS + k] = g.gains[k];
    e[G_NR] = (float)n;
    if (n == 4) {
        // the kernels' quad butterflies assume that every row of the FP32
        // tables is one magnitude with the signs of the X layout
        static const float sx[4] = {1, 1, -1, -1}, sy[4] = {-1, 1, 1, -1}, sz[4] = {1, -1, 1, -1};
        const float* p0 = e + G_APINV;
        const float* c0 = e + G_ACOL;
        for (int i = 0; i < 4; ++i) {
            const float* p = p0 + 4 * i;
            const float* c = c0 + 4 * i;
            if (p[0] != p0[0] || p[1] != sx[i] * p0[1] || p[2] != sy[i] * p0[1] || p[3] != sz[i] * p0[3] ||
                c[0] != 1.0f || c[1] != sx[i] * c0[1] || c[2] != sy[i] * c0[1] || c[3] != sz[i] * c0[3])
                return false;
        }
        e[G_Q_F] = p0[0];
        e[G_Q_XY] = p0[1];
        e[G_Q_Z] = p0[3];
        e[G_Q_S] = c0[1];
        e[G_Q_CT] = c0[3];
    } else {
        // hexa and octo: the kernels' pair form assumes that rotor i + n/2
        // has rotor i's rows with the x-y terms negated and the yaw term
        // times (-1)^(n/2), and that the yaw terms alternate in sign
        const int h = n / 2;
        const float so = (h % 2) ? -1.0f : 1.0f;
        for (int k = 0; k < 2; ++k) {
            const float* t = e + (k == 0 ? G_APINV : G_ACOL);
            for (int i = 0; i < n; ++i) {
                const float* r = t + 4 * i;
                if (r[0] != t[0] || r[3] != ((i % 2) ? -t[3] : t[3])) return false;
                if (i < h) {
                    const float* o = t + 4 * (i + h);
                    if (o[1] != -r[1] || o[2] != -r[2] || o[3] != so * r[3]) return false;
                }
            }
        }
    }
    return true;
}

std::string validate(const ag_config* c) {
    if (!c) return "cfg is null";
    if (c->n < 1 || c->n > 2147483647LL) return "n must be in [1, 2^31-1]";
    if (c->ld < c->n) return "ld must be >= n";
    if (!(c->dt > 0.0f) || !std::isfinite(c->dt)) return "dt must be positive and finite";
    if (!std::isfinite(c->g)) return "g must be finite";
    if (c->index_base < 0 || c->index_base + c->n > 4294967296LL) return "index_base + n must be <= 2^32";
    if (!c->state || !c->mode || !c->target) return "state, mode and target buffers are required";
    if (c->n_groups < 1 || c->n_groups > AG_MAX_GROUPS || !c->groups) return "n_groups must be in [1, AG_MAX_GROUPS]";
    long long expect = 0;
    for (int g = 0; g < c->n_groups; ++g) {
        const ag_group_desc& d = c->groups[g];
        if (d.first != expect || d.count < 1) return "groups must be non-empty, contiguous and in order";
        expect += d.count;
        if (d.n_rotors != 4 && d.n_rotors != 6 && d.n_rotors != 8) return "n_rotors must be 4, 6 or 8";
        if (!(d.arm > 0) || !(d.c_tau > 0) || !(d.mass > 0)) return "arm, c_tau and mass must be positive";
        if (!(d.inertia[0] > 0) || !(d.inertia[1] > 0) || !(d.inertia[2] > 0)) return "inertia must be positive";
        if (!(d.u_min <= d.u_max)) return "u_min must be <= u_max";
    }
    if (expect != c->n) return "groups must cover [0, n)";
    if (!(c->reset_prob >= 0.0f && c->reset_prob <= 1.0f)) return "reset_prob must be in [0, 1]";
    for (int k = 0; k < 3; ++k)
        if (!(c->reset_lo[k] <= c->reset_hi[k])) return "reset_lo must be <= reset_hi";
    return "";
}

// Largest number of groups that any tile of `tile` consecutive vehicles overlaps.
int tile_span(ag_handle h, long long tile) {
    for (auto& p : h->span_cache)
        if (p.first == tile) return p.second;
    const long long n = h->cfg.n;
    const int G = h->cfg.n_groups;
    int best = 1, g = 0;
    for (long long base = 0; base < n; base += tile) {
        const long long end = std::min(base + tile, n) - 1;
        while (g + 1 < G && h->goff_host[g + 1] <= base) ++g;
        int gh = g;
        while (gh + 1 < G && h->goff_host[gh + 1] <= end) ++gh;
        best = std::max(best, gh - g + 1);
    }
    h->span_cache.push_back({tile, best});
    return best;
}

size_t lds_bytes(int span) { return (size_t)span * GSTRIDE * sizeof(float) + (size_t)(span + 1) * sizeof(int32_t); }

StepArgs base_args(ag_handle h) {
    StepArgs a{};
    a.state = h->cfg.state;
    a.mode = h->cfg.mode;
    a.target = h->cfg.target;
    a.vparams = h->cfg.vparams;
    a.traj = h->cfg.traj;
    a.goal = h->cfg.goal;
    a.gtab = h->gtab;
    a.goff = h->goff;
    a.wrench_out = h->cfg.wrench_out;
    a.rotor_out = h->cfg.rotor_out;
    a.flags_out = h->cfg.flags_out;
    a.slots = h->cfg.collect_stats ? h->slots : nullptr;
    a.n = h->cfg.n;
    a.ld = h->cfg.ld;
    a.n_groups = h->cfg.n_groups;
    a.dt = h->cfg.dt;
    a.g = h->cfg.g;
    a.key0 = h->key0;
    a.key1 = h->key1;
    a.thr = h->thr;
    a.index_base = (uint32_t)h->cfg.index_base;
    for (int k = 0; k < 3; ++k) {
        a.lo[k] = h->cfg.reset_lo[k];
        a.hi[k] = h->cfg.reset_hi[k];
    }
    a.ev = h->ev;
    a.queue = h->queue;
    return a;
}

// Whether fused launches of the current handle take their resets from the
// event kernels.
bool uses_events(ag_handle h, const ag_exec& e) { return h->reset_on && e.kind == 1 && h->ev.cap > 0; }

// Whether the policy's fused launches can run in mode order (their kernels
// have the mode-specialised step loops).
bool order_policy(ag_handle h, const ag_exec& e) {
    const bool obs = h->cfg.wrench_out || h->cfg.rotor_out || h->cfg.flags_out || h->cfg.collect_stats;
    return (e.kind == 1 || e.kind == 2) && e.vpl == 1 && h->cfg.traj == nullptr && !obs && !h->reset_on;
}

// Whether the fused launches of an ag_step of n_steps steps run in mode order.
// The order is computed once and kept until the commands change; a stale
// order costs one pass over the modes, which short calls skip.  (Any order
// within groups gives the same results: it only decides which lanes share a
// wavefront.)
bool uses_order(ag_handle h, const ag_exec& e, int n_steps) {
    return order_policy(h, e) && (h->order_valid || n_steps >= kOrderMinSteps);
}

OrderArgs order_args(ag_handle h) {
    return OrderArgs{h->cfg.mode, h->goff, h->perm, h->cfg.n, h->cfg.n_groups};
}

dim3 order_grid(ag_handle h) { return dim3((unsigned)((h->cfg.n + kOrderSeg - 1) / kOrderSeg)); }

ag_status launch(ag_handle h, const void* fn, dim3 grid, dim3 block, size_t shmem, void* args);

// Compute the mode order into the workspace unless it is current.
ag_status ensure_order(ag_handle h) {
    if (h->order_valid) return AG_OK;
    OrderArgs o = order_args(h);
    ag_status st = launch(h, mode_order_kernel(), order_grid(h), dim3(kOrderBlock), 0, &o);
    if (st == AG_OK) h->order_valid = true;
    return st;
}

// The event kernels of one launch, in order (they take the launch's arguments).
struct EvKernels {
    const void* fn[4];
    dim3 grid[4], block[4];
};

EvKernels event_kernels(ag_handle h) {
    const unsigned nb = (unsigned)h->L.nblocks;
    const unsigned nr = (unsigned)((h->ev.cap + 255) / 256);
    return EvKernels{{ev_mask_kernel(), ev_scan_kernel(), ev_scatter_kernel(), ev_redraw_kernel()},
                     {dim3(nb), dim3(1), dim3(nb), dim3(nr)},
                     {dim3(kResetBlock), dim3(1024), dim3(kResetBlock), dim3(256)}};
}

struct LaunchShape {
    const void* fn;
    const void* fn_fb;   // fused launches with resets: the variant for overfull event buffers, run after fn
    dim3 grid, block;
    size_t shmem;
    int span;
    bool ev_stage;       // the LDS holds a copy of each wavefront's reset events
};

// Launch shape of the work-queue kernel (exec kind 2).
std::string queue_shape(ag_handle h, const ag_exec& e, LaunchShape& s) {
    if (e.block != 64) return "exec kind 2 needs block 64";
    if (e.vpl != 1) return "exec kind 2 needs vpl 1";
    if (e.k < 1) return "exec.k must be >= 1";
    if (e.grid < 0) return "exec.grid must be >= 0";
    const bool obs = h->cfg.wrench_out || h->cfg.rotor_out || h->cfg.flags_out || h->cfg.collect_stats;
    if (h->cfg.n_groups != 1 || h->vp || obs || h->cfg.traj || h->reset_on)
        return "exec kind 2 needs one vehicle group and no observers, trajectories, per-vehicle parameters "
               "or automatic resets";
    s.fn = step_queue_kernel(h->nr_class);
    s.fn_fb = nullptr;
    s.shmem = step_queue_lds_bytes();
    if (!s.fn) return "no kernel for this combination of policy and configuration";
    if (h->q_occ == 0) {
        int occ = 0;
        h->q_occ = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, s.fn, 64, s.shmem) == hipSuccess && occ > 0
                       ? occ : -1;
    }
    if (h->q_occ < 0 && e.grid == 0) return "exec kind 2: occupancy query failed (give exec.grid)";
    // as many wavefronts as run at once, a multiple of the queue count (every
    // queue served by as many wavefronts), and no more than the tiles need
    const long long nq = 8LL * kQueueSub;
    const long long ntiles = (h->cfg.n + 63) / 64;
    long long grid = e.grid > 0 ? e.grid : (long long)h->num_cus * h->q_occ;
    grid = std::min(grid / nq * nq, (ntiles + nq - 1) / nq * nq);
    s.grid = dim3((unsigned)std::max(grid, nq));
    s.block = dim3(64);
    s.span = 1;
    s.ev_stage = false;
    return "";
}

std::string shape_for(ag_handle h, const ag_exec& e, LaunchShape& s) {
    if (e.kind == 2) return queue_shape(h, e, s);
    if (e.kind != 0 && e.kind != 1) return "exec.kind must be 0 (per-step), 1 (fused) or 2 (fused, work queue)";
    if (e.block < 64 || e.block > 512 || e.block % 64) return "exec.block must be a multiple of 64 in [64, 512]";
    const bool one = e.kind == 0;
    const int vpl = one ? 1 : e.vpl;
    if (vpl != 1 && vpl != 2) return "exec.vpl must be 1 or 2";
    if (!one && e.k < 1) return "exec.k must be >= 1";
    if (e.grid < 0) return "exec.grid must be >= 0";
    const long long tile = (long long)e.block * vpl;
    const int span = tile_span(h, tile);
    if (span > kMaxSpanLds) return "vehicle groups too small for this tile size (too many groups per tile)";
    const long long ntiles = (h->cfg.n + tile - 1) / tile;
    long long grid = (one || e.grid == 0) ? ntiles : std::min<long long>(e.grid, ntiles);
    if (grid > h->L.nslots) grid = h->L.nslots;
    if (grid > 2147483647LL) return "grid too large";
    if (h->reset_on && !one && e.k > 64) return "with automatic resets exec.k must be <= 64";
    const bool obs = h->cfg.wrench_out || h->cfg.rotor_out || h->cfg.flags_out || h->cfg.collect_stats;
    const bool trk = h->cfg.traj != nullptr;
    if (trk && vpl != 1) return "with a trajectory buffer exec.vpl must be 1";
    const bool events = h->reset_on && !one && h->ev.cap > 0;
    s.fn = step_kernel(h->nr_class, h->vp, events ? 2 : (h->reset_on ? 1 : 0), vpl, one, obs, trk);
    s.fn_fb = events ? step_kernel(h->nr_class, h->vp, 1, vpl, one, obs, trk) : nullptr;
    if (!s.fn || (events && !s.fn_fb)) return "no kernel for this combination of policy and configuration";
    s.grid = dim3((unsigned)grid);
    s.block = dim3((unsigned)e.block);
    s.span = span;
    s.shmem = lds_bytes(span);
    // event-fed launches of one vehicle per lane also copy each wavefront's
    // events into LDS when that fits 64 KiB with the group entries (the
    // overflow variant launched after them gets the same shape)
    const size_t staged = ev_stage_offset(span) * sizeof(float) + (size_t)(e.block / 64) * 16 * kEvStage * sizeof(float);
    s.ev_stage = events && vpl == 1 && staged <= 65536;
    if (s.ev_stage) s.shmem = staged;
    return "";
}

ag_status launch(ag_handle h, const void* fn, dim3 grid, dim3 block, size_t shmem, void* args) {
    void* params[] = {args};
    AG_HIP(h, hipLaunchKernel(fn, grid, block, params, shmem, h->stream));
    return AG_OK;
}

ag_status launch_fold(ag_handle h, int nslots, long long steps) {
    FoldArgs f{h->slots, nslots, h->acc, steps, 1};
    return launch(h, fold_kernel(), dim3(1), dim3(256), 0, &f);
}

// Direct (non-graph) launches of n steps with exec e on the given buffers.
ag_status run_direct(ag_handle h, const ag_exec& e, int n_steps, StepArgs a, bool fold) {
    LaunchShape s;
    std::string m = shape_for(h, e, s);
    if (!m.empty()) return set_err(h, AG_E_INVALID, m);
    a.span = s.span;
    a.ev_stage = s.ev_stage ? 1 : 0;
    a.d_step = nullptr;
    a.perm = nullptr;
    if (uses_order(h, e, n_steps)) {
        ag_status st = ensure_order(h);
        if (st != AG_OK) return st;
        a.perm = h->perm;
    }
    const int k = e.kind == 0 ? 1 : e.k;
    for (int done = 0, j = 0; done < n_steps; done += k, ++j) {
        a.t0 = h->t + done;
        a.k = std::min(k, n_steps - done);
        a.flags_accumulate = done > 0;
        if (uses_events(h, e)) {
            const EvKernels ek = event_kernels(h);
            for (int q = 0; q < 4; ++q) {
                ag_status st = launch(h, ek.fn[q], ek.grid[q], ek.block[q], 0, &a);
                if (st != AG_OK) return st;
            }
        }
        ag_status st = launch(h, s.fn, s.grid, s.block, s.shmem, &a);
        if (st == AG_OK && s.fn_fb) st = launch(h, s.fn_fb, s.grid, s.block, s.shmem, &a);
        if (st != AG_OK) return st;
    }
    if (fold && a.slots) return launch_fold(h, (int)s.grid.x, n_steps);
    return AG_OK;
}

ag_status add_node(ag_handle h, hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t* dep, const void* fn,
                   dim3 grid, dim3 block, size_t shmem, void* args) {
    hipKernelNodeParams p{};
    void* params[] = {args};
    p.func = const_cast<void*>(fn);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = (unsigned)shmem;
    p.kernelParams = params;
    p.extra = nullptr;
    AG_HIP(h, hipGraphAddKernelNode(node, g, dep, dep ? 1 : 0, &p));
    return AG_OK;
}

// Graph of the fused or per-step launches of ag_step(n_steps); `ordered`:
// the launches read the mode order (computed outside the graph).
ag_status build_graph(ag_handle h, int n_steps, bool ordered, GraphEntry& ge) {
    LaunchShape s;
    std::string m = shape_for(h, h->exec, s);
    if (!m.empty()) return set_err(h, AG_E_INVALID, m);
    hipGraph_t g;
    AG_HIP(h, hipGraphCreate(&g, 0));
    StepArgs a = base_args(h);
    a.span = s.span;
    a.ev_stage = s.ev_stage ? 1 : 0;
    a.d_step = h->d_step;
    const int k = h->exec.kind == 0 ? 1 : h->exec.k;
    hipGraphNode_t prev = nullptr, node = nullptr;
    a.perm = ordered ? h->perm : nullptr;
    for (int done = 0; done < n_steps; done += k) {
        a.t_off = done;
        a.k = std::min(k, n_steps - done);
        a.flags_accumulate = done > 0;
        if (uses_events(h, h->exec)) {
            const EvKernels ek = event_kernels(h);
            for (int q = 0; q < 4; ++q) {
                ag_status st = add_node(h, g, &node, prev ? &prev : nullptr, ek.fn[q], ek.grid[q], ek.block[q], 0, &a);
                if (st != AG_OK) { (void)hipGraphDestroy(g); return st; }
                prev = node;
            }
        }
        ag_status st = add_node(h, g, &node, prev ? &prev : nullptr, s.fn, s.grid, s.block, s.shmem, &a);
        if (st != AG_OK) { (void)hipGraphDestroy(g); return st; }
        prev = node;
        if (s.fn_fb) {
            st = add_node(h, g, &node, &prev, s.fn_fb, s.grid, s.block, s.shmem, &a);
            if (st != AG_OK) { (void)hipGraphDestroy(g); return st; }
            prev = node;
        }
    }
    if (a.slots) {
        FoldArgs f{h->slots, (int)s.grid.x, h->acc, n_steps, 1};
        ag_status st = add_node(h, g, &node, &prev, fold_kernel(), dim3(1), dim3(256), 0, &f);
        if (st != AG_OK) { (void)hipGraphDestroy(g); return st; }
        prev = node;
    }
    CounterArgs c{h->d_step, n_steps};
    ag_status st = add_node(h, g, &node, &prev, advance_kernel(), dim3(1), dim3(64), 0, &c);
    if (st != AG_OK) { (void)hipGraphDestroy(g); return st; }
    hipGraphExec_t ex;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(h, e, "hipGraphInstantiate"); }
    ge.n_steps = n_steps;
    ge.ordered = ordered;
    ge.key = {h->exec.kind, h->exec.block, h->exec.vpl, h->exec.k, h->exec.grid, h->exec.use_graph};
    ge.graph = g;
    ge.exec = ex;
    ge.stamp = ++h->stamp;
    return AG_OK;
}

void drop_graphs(ag_handle h) {
    for (auto& ge : h->graphs) {
        (void)hipGraphExecDestroy(ge.exec);
        (void)hipGraphDestroy(ge.graph);
    }
    h->graphs.clear();
}

}  // namespace

extern "C" {

const char* ag_status_string(ag_status s) {
    switch (s) {
        case AG_OK: return "ok";
        case AG_E_INVALID: return "invalid argument";
        case AG_E_HIP: return "HIP error";
        case AG_E_NOMEM: return "workspace too small";
        case AG_E_STATE: return "invalid state";
        case AG_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown";
}

ag_status ag_workspace_size(const ag_config* cfg, size_t* bytes) {
    if (!bytes) return AG_E_INVALID;
    std::string m = validate(cfg);
    if (!m.empty()) return AG_E_INVALID;
    *bytes = ws_layout(cfg).total;
    return AG_OK;
}

ag_status ag_create(const ag_config* cfg, void* workspace, size_t workspace_bytes, ag_handle* out) {
    if (!out) return AG_E_INVALID;
    *out = nullptr;
    std::string m = validate(cfg);
    if (!m.empty()) {
        std::fprintf(stderr, "ag_create: %s\n", m.c_str());
        return AG_E_INVALID;
    }
    WsLayout L = ws_layout(cfg);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return AG_E_INVALID;
    if (workspace_bytes < L.total) return AG_E_NOMEM;

    ag_sim* h = new ag_sim();
    h->cfg = *cfg;
    h->groups.assign(cfg->groups, cfg->groups + cfg->n_groups);
    h->cfg.groups = nullptr;
    h->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    h->ws = static_cast<char*>(workspace);
    h->L = L;
    h->gtab = reinterpret_cast<float*>(h->ws + L.gtab);
    h->goff = reinterpret_cast<int32_t*>(h->ws + L.goff);
    h->d_step = reinterpret_cast<long long*>(h->ws + L.d_step);
    h->acc = reinterpret_cast<StatAcc*>(h->ws + L.acc);
    h->slots = reinterpret_cast<StatSlot*>(h->ws + L.slots);
    h->perm = reinterpret_cast<int32_t*>(h->ws + L.perm);
    h->queue = reinterpret_cast<unsigned*>(h->ws + L.queue);
    h->q_occ = 0;
    h->block_counts = reinterpret_cast<int32_t*>(h->ws + L.block_counts);
    h->mask_buf = reinterpret_cast<uint8_t*>(h->ws + L.mask);
    h->scratch = cfg->autotune_scratch ? reinterpret_cast<float*>(h->ws + L.scratch) : nullptr;
    h->ev = EvBufs{};
    if (L.ev_cap > 0) {
        h->ev.bits = reinterpret_cast<unsigned long long*>(h->ws + L.ev_bits);
        h->ev.off = reinterpret_cast<int32_t*>(h->ws + L.ev_off);
        h->ev.block_counts = reinterpret_cast<long long*>(h->ws + L.ev_bc);
        h->ev.total = reinterpret_cast<long long*>(h->ws + L.ev_total);
        h->ev.list = reinterpret_cast<long long*>(h->ws + L.ev_list);
        h->ev.data = reinterpret_cast<float*>(h->ws + L.ev_data);
        h->ev.cap = L.ev_cap;
    }
    int maxr = 4;
    for (auto& g : h->groups) maxr = std::max(maxr, g.n_rotors);
    bool uniform = true;
    for (auto& g : h->groups) uniform = uniform && g.n_rotors == h->groups[0].n_rotors;
    h->nr_class = uniform ? h->groups[0].n_rotors : 0;   // 0: mixed rotor counts
    (void)maxr;
    h->vp = cfg->vparams != nullptr;
    h->reset_on = cfg->auto_reset != 0 && cfg->reset_prob > 0.0f;
    h->key0 = (uint32_t)(cfg->seed & 0xFFFFFFFFull);
    h->key1 = (uint32_t)(cfg->seed >> 32);
    const double thr = std::floor((double)cfg->reset_prob * 4294967296.0);
    h->thr = (unsigned long long)std::min(std::max(thr, 0.0), 4294967296.0);
    h->t = 0;
    h->dev_step_dirty = true;
    h->order_valid = false;
    h->stamp = 0;
    h->sticky = AG_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        h->num_cus = 256;
    h->noalloc_err = hipSuccess;
    h->noalloc_scratch = hipGetDevice(&dev) == hipSuccess ? device_scratch(dev, &h->noalloc_err) : nullptr;
    if (!h->noalloc_scratch && h->noalloc_err == hipSuccess) h->noalloc_err = hipErrorInvalidDevice;
    h->exec = {1, 256, 1, 16, 0, h->stream != nullptr ? 1 : 0};

    std::vector<float> tab((size_t)cfg->n_groups * GSTRIDE);
    h->goff_host.resize(cfg->n_groups + 1);
    for (int g = 0; g < cfg->n_groups; ++g) {
        if (!build_group_entry(h->groups[g], &tab[(size_t)g * GSTRIDE])) {
            delete h;
            return AG_E_INVALID;
        }
        h->goff_host[g] = (int32_t)h->groups[g].first;
    }
    h->goff_host[cfg->n_groups] = (int32_t)cfg->n;
    tile_span(h, kRolloutBlock);   // cached now: rollout calls then allocate no host memory
    StatAcc zero{};
    hipError_t e = hipMemcpyAsync(h->gtab, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->goff, h->goff_host.data(), h->goff_host.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->acc, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream);
    static const unsigned qzero[kQueueWords] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(h->queue, qzero, sizeof(qzero), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        CounterArgs c{h->d_step, 0};
        void* p1[] = {&c};
        e = hipLaunchKernel(set_step_kernel(), dim3(1), dim3(64), p1, 0, h->stream);
    }
    if (e == hipSuccess) {
        ClearArgs ca{h->slots, (int)L.nslots};
        void* p2[] = {&ca};
        e = hipLaunchKernel(clear_slots_kernel(), dim3((unsigned)((L.nslots + 255) / 256)), dim3(256), p2, 0,
                            h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        std::fprintf(stderr, "ag_create: %s\n", hipGetErrorString(e));
        delete h;
        return AG_E_HIP;
    }
    h->dev_step_dirty = false;
    *out = h;
    return AG_OK;
}

ag_status ag_destroy(ag_handle h) {
    if (!h) return AG_E_INVALID;
    // let launches and graph replays still queued on the stream finish before
    // their executable graphs are destroyed
    const hipError_t e = hipStreamSynchronize(h->stream);
    drop_graphs(h);
    delete h;
    return e == hipSuccess ? AG_OK : AG_E_HIP;
}

ag_status ag_set_targets(ag_handle h, int64_t first, int64_t count, const int8_t* mode_src,
                         const float* target_src, int64_t src_ld) {
    AG_CHECK_HANDLE(h);
    if (first < 0 || count < 0 || first + count > h->cfg.n) return set_err(h, AG_E_INVALID, "range out of bounds");
    if (target_src && src_ld < count) return set_err(h, AG_E_INVALID, "src_ld must be >= count");
    if (count == 0) return AG_OK;
    SetTargetsArgs a{h->cfg.mode, h->cfg.target, mode_src, target_src, h->cfg.ld, src_ld, first, count, h->acc};
    h->order_valid = false;
    return launch(h, set_targets_kernel(), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, &a);
}

ag_status ag_set_exec(ag_handle h, const ag_exec* e) {
    AG_CHECK_HANDLE(h);
    if (!e) return AG_E_INVALID;
    LaunchShape s;
    std::string m = shape_for(h, *e, s);
    if (!m.empty()) return set_err(h, AG_E_INVALID, m);
    if (e->use_graph && !h->stream) return set_err(h, AG_E_INVALID, "graphs need a non-null stream");
    h->exec = *e;
    return AG_OK;
}

ag_status ag_get_exec(ag_handle h, ag_exec* e) {
    if (!h || !e) return AG_E_INVALID;
    *e = h->exec;
    return AG_OK;
}

}  // extern "C"

namespace {

// Find or build the cached graph for n_steps under the current policy.
ag_status cached_graph(ag_handle h, int n_steps, bool ordered, GraphEntry** out) {
    const ag_exec& e = h->exec;
    ExecKey key{e.kind, e.block, e.vpl, e.k, e.grid, e.use_graph};
    for (auto& g : h->graphs)
        if (g.n_steps == n_steps && g.ordered == ordered && g.key == key) {
            g.stamp = ++h->stamp;
            *out = &g;
            return AG_OK;
        }
    GraphEntry ng;
    ag_status st = build_graph(h, n_steps, ordered, ng);
    if (st != AG_OK) return st;
    if (h->graphs.size() >= 8) {
        auto old = std::min_element(h->graphs.begin(), h->graphs.end(),
                                    [](const GraphEntry& a, const GraphEntry& b) { return a.stamp < b.stamp; });
        (void)hipGraphExecDestroy(old->exec);
        (void)hipGraphDestroy(old->graph);
        h->graphs.erase(old);
    }
    h->graphs.push_back(ng);
    *out = &h->graphs.back();
    return AG_OK;
}

bool uses_graph(ag_handle h, int n_steps) {
    const ag_exec& e = h->exec;
    const int k = e.kind == 0 ? 1 : e.k;
    return e.use_graph && h->stream && (n_steps + k - 1) / k >= 2;
}

}  // namespace

extern "C" {

ag_status ag_prepare(ag_handle h, int32_t n_steps) {
    AG_CHECK_HANDLE(h);
    if (n_steps < 0) return set_err(h, AG_E_INVALID, "n_steps must be >= 0");
    if (n_steps == 0) return AG_OK;
    // a call that is prepared for will run in mode order whatever its length
    if (order_policy(h, h->exec)) {
        ag_status st = ensure_order(h);
        if (st != AG_OK) return st;
    }
    if (!uses_graph(h, n_steps)) return AG_OK;
    GraphEntry* ge = nullptr;
    ag_status st = cached_graph(h, n_steps, uses_order(h, h->exec, n_steps), &ge);
    if (st != AG_OK) return st;
    // move the executable graph to the device now, not at its first launch
    AG_HIP(h, hipGraphUpload(ge->exec, h->stream));
    return AG_OK;
}

ag_status ag_step(ag_handle h, int32_t n_steps) {
    AG_CHECK_HANDLE(h);
    if (n_steps < 0) return set_err(h, AG_E_INVALID, "n_steps must be >= 0");
    if (n_steps == 0) return AG_OK;
    if (!uses_graph(h, n_steps)) {
        ag_status st = run_direct(h, h->exec, n_steps, base_args(h), true);
        if (st != AG_OK) return st;
        h->t += n_steps;
        h->dev_step_dirty = true;
        return AG_OK;
    }
    const bool ordered = uses_order(h, h->exec, n_steps);
    GraphEntry* ge = nullptr;
    ag_status st = cached_graph(h, n_steps, ordered, &ge);
    if (st != AG_OK) return st;
    if (ordered) {
        st = ensure_order(h);
        if (st != AG_OK) return st;
    }
    if (h->dev_step_dirty) {
        CounterArgs c{h->d_step, h->t};
        st = launch(h, set_step_kernel(), dim3(1), dim3(64), 0, &c);
        if (st != AG_OK) return st;
        h->dev_step_dirty = false;
    }
    AG_HIP(h, hipGraphLaunch(ge->exec, h->stream));
    h->t += n_steps;
    return AG_OK;
}

}  // extern "C"

namespace {

// ---- autotune cache ------------------------------------------------------------
// Chosen policies, per process and optionally in a text file (one line per
// key: "<key> kind block vpl k grid use_graph"), keyed by everything the
// timing depends on: device, n, group layout, kernel class and call length.
std::mutex g_tune_mu;
std::vector<std::pair<std::string, ag_exec>> g_tune;
bool g_tune_file_read = false;

const char* tune_file() {
    const char* f = std::getenv("AG_AUTOTUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

void tune_read_file_locked() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = tune_file();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[512];
    ag_exec e{};
    while (std::fscanf(f, "%511s %d %d %d %d %d %d", key, &e.kind, &e.block, &e.vpl, &e.k, &e.grid,
                       &e.use_graph) == 7)
        g_tune.push_back({key, e});
    std::fclose(f);
}

bool tune_lookup(const std::string& key, ag_exec* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_read_file_locked();
    for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
        if (it->first == key) {
            *out = it->second;
            return true;
        }
    return false;
}

void tune_store(const std::string& key, const ag_exec& e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_read_file_locked();
    g_tune.push_back({key, e});
    if (const char* path = tune_file()) {
        if (FILE* f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), e.kind, e.block, e.vpl, e.k, e.grid, e.use_graph);
            std::fclose(f);
        }
    }
}

std::string tune_key(ag_handle h, int probe_steps) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        for (char& c : arch)
            if (c == ':' || c == ' ') c = '.';
    }
    // group layout: FNV-1a over (count, rotor count) of every group
    unsigned long long fh = 1469598103934665603ull;
    auto mix = [&](long long v) {
        for (int b = 0; b < 8; ++b) {
            fh ^= (unsigned long long)((v >> (8 * b)) & 0xff);
            fh *= 1099511628211ull;
        }
    };
    for (const auto& g : h->groups) {
        mix(g.count);
        mix(g.n_rotors);
    }
    const bool obs = h->cfg.wrench_out || h->cfg.rotor_out || h->cfg.flags_out || h->cfg.collect_stats;
    char buf[384];
    std::snprintf(buf, sizeof buf, "%s/cu%d/n%lld/g%d.%016llx/nr%d/vp%d/rst%d.%d/obs%d/trk%d/graph%d/L%d",
                  arch.c_str(), h->num_cus, (long long)h->cfg.n, h->cfg.n_groups, fh, h->nr_class, h->vp ? 1 : 0,
                  h->reset_on ? 1 : 0, h->ev.cap > 0 ? 1 : 0, obs ? 1 : 0, h->cfg.traj ? 1 : 0,
                  h->exec.use_graph, probe_steps);
    return buf;
}

}  // namespace

extern "C" {

ag_status ag_autotune(ag_handle h, int32_t probe_steps, ag_exec* chosen) {
    AG_CHECK_HANDLE(h);
    if (!h->scratch) return set_err(h, AG_E_STATE, "autotune needs cfg.autotune_scratch = 1");
    if (probe_steps < 1) return set_err(h, AG_E_INVALID, "probe_steps must be >= 1");
    const std::string key = tune_key(h, probe_steps);
    ag_exec cached{};
    LaunchShape cs;
    if (tune_lookup(key, &cached) && shape_for(h, cached, cs).empty()) {
        h->exec = cached;
        if (chosen) *chosen = cached;
        return AG_OK;
    }
    // trials run in mode order whenever the tuned calls will
    if (order_policy(h, ag_exec{1, 64, 1, 1, 0, 0})) {
        ag_status st = ensure_order(h);
        if (st != AG_OK) return st;
    }
    const long long ld = h->cfg.ld;
    float* s_state = h->scratch;
    float* s_target = h->scratch + (size_t)AG_STATE_DIM * ld;
    StepArgs a = base_args(h);
    a.state = s_state;
    a.target = s_target;
    a.wrench_out = nullptr;
    a.rotor_out = nullptr;
    a.flags_out = nullptr;
    a.goal = nullptr;          // trials on scratch copies leave the caller's goals alone
    hipEvent_t e0, e1;
    AG_HIP(h, hipEventCreate(&e0));
    AG_HIP(h, hipEventCreate(&e1));
    int occ_blocks_per_cu = 0;
    const int blocks[] = {64, 128, 256, 512};
    const int vpls[] = {1, 2};
    // powers of two up to the call length, and the call length itself (one
    // launch per call)
    std::vector<int> ks = {4, 8, 16, 32, 64, 128, 256, 512, 1024};
    if (probe_steps <= 1024 && std::find(ks.begin(), ks.end(), probe_steps) == ks.end()) ks.push_back(probe_steps);
    // short trials are noisier: more repetitions (the first is not counted;
    // a 20-step call of 1M vehicles varies by a few per cent between calls,
    // about the difference between the two fused forms)
    const int reps = probe_steps >= 256 ? 3 : probe_steps >= 64 ? 7 : 15;
    ag_exec best = h->exec;
    float best_ms = 1e30f;
    const long long saved_t = h->t;
    // the candidates: fused launches of every block, vpl and k, each on one
    // block per tile and on a persistent grid, and the work-queue form
    std::vector<ag_exec> cands;
    for (int b : blocks)
        for (int v : vpls)
            for (int k : ks) {
                if (k > probe_steps && k != 4) continue;
                for (int gmode = 0; gmode < 2; ++gmode) {
                    ag_exec cand{1, b, v, k, 0, h->exec.use_graph};
                    LaunchShape s;
                    if (!shape_for(h, cand, s).empty()) continue;
                    if (gmode == 1) {
                        // a persistent grid: as many blocks as fit on the chip at once
                        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_blocks_per_cu, s.fn, b, s.shmem) !=
                                hipSuccess || occ_blocks_per_cu < 1)
                            continue;
                        long long gp = (long long)h->num_cus * occ_blocks_per_cu;
                        gp = (gp + 7) / 8 * 8;
                        if (gp >= (long long)s.grid.x) continue;
                        cand.grid = (int)gp;
                    }
                    cands.push_back(cand);
                }
            }
    for (int k : ks) {
        if (k > probe_steps && k != 4) continue;
        ag_exec cand{2, 64, 1, k, 0, h->exec.use_graph};
        LaunchShape s;
        if (shape_for(h, cand, s).empty()) cands.push_back(cand);
    }
    for (const ag_exec& cand : cands) {
        float ms_min = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            AG_HIP(h, hipMemcpy2DAsync(s_state, ld * sizeof(float), h->cfg.state, ld * sizeof(float),
                                       h->cfg.n * sizeof(float), AG_STATE_DIM, hipMemcpyDeviceToDevice, h->stream));
            AG_HIP(h, hipMemcpy2DAsync(s_target, ld * sizeof(float), h->cfg.target, ld * sizeof(float),
                                       h->cfg.n * sizeof(float), AG_TARGET_DIM, hipMemcpyDeviceToDevice,
                                       h->stream));
            AG_HIP(h, hipEventRecord(e0, h->stream));
            ag_status st = run_direct(h, cand, probe_steps, a, false);
            if (st != AG_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return st;
            }
            AG_HIP(h, hipEventRecord(e1, h->stream));
            AG_HIP(h, hipEventSynchronize(e1));
            float ms = 0.0f;
            AG_HIP(h, hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) ms_min = std::min(ms_min, ms);
        }
        if (ms_min < best_ms) {
            best_ms = ms_min;
            best = cand;
        }
    }
    h->t = saved_t;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ClearArgs ca{h->slots, (int)h->L.nslots};
    ag_status st = launch(h, clear_slots_kernel(), dim3((unsigned)((h->L.nslots + 255) / 256)), dim3(256), 0, &ca);
    if (st != AG_OK) return st;
    AG_HIP(h, hipStreamSynchronize(h->stream));
    h->exec = best;
    tune_store(key, best);
    if (chosen) *chosen = best;
    return AG_OK;
}

ag_status ag_reset(ag_handle h, const uint8_t* mask_in, int64_t step, uint8_t* mask_out, int32_t* indices_out,
                   int32_t* count_out) {
    AG_CHECK_HANDLE(h);
    if (step < 0) return set_err(h, AG_E_INVALID, "step must be >= 0");
    ResetArgs a{};
    a.state = h->cfg.state;
    a.mode = h->cfg.mode;
    a.target = h->cfg.target;
    a.mask_in = mask_in;
    a.goal = h->cfg.goal;
    const bool need_scan = indices_out || count_out;
    a.mask_out = mask_out ? mask_out : (need_scan ? h->mask_buf : nullptr);
    a.block_counts = need_scan ? h->block_counts : nullptr;
    a.n = h->cfg.n;
    a.ld = h->cfg.ld;
    a.t = step;
    a.key0 = h->key0;
    a.key1 = h->key1;
    a.thr = h->thr;
    a.index_base = (uint32_t)h->cfg.index_base;
    for (int k = 0; k < 3; ++k) {
        a.lo[k] = h->cfg.reset_lo[k];
        a.hi[k] = h->cfg.reset_hi[k];
    }
    const unsigned nb = (unsigned)h->L.nblocks;
    ag_status st = launch(h, reset_mask_kernel(), dim3(nb), dim3(kResetBlock), 0, &a);
    if (st != AG_OK || !need_scan) return st;
    ScanArgs sa{h->block_counts, (int)nb, count_out};
    st = launch(h, reset_scan_kernel(), dim3(1), dim3(1024), 0, &sa);
    if (st != AG_OK || !indices_out) return st;
    ScatterArgs ca{a.mask_out, h->block_counts, indices_out, h->cfg.n};
    return launch(h, reset_scatter_kernel(), dim3(nb), dim3(kResetBlock), 0, &ca);
}

ag_status ag_randomize_obstacles(ag_handle h, int32_t n_obs, const float* slots, const float* env_lo,
                                 const float* env_hi, const float* box_lo, const float* box_hi,
                                 const uint8_t* env_mask, int64_t step, float* out, int64_t out_ld) {
    AG_CHECK_HANDLE(h);
    if (n_obs < 1 || !slots || !out) return set_err(h, AG_E_INVALID, "n_obs >= 1, slots and out are required");
    if (step < 0 || step > 4294967295LL) return set_err(h, AG_E_INVALID, "step must be in [0, 2^32)");
    const long long total = h->cfg.n * (long long)n_obs;
    if (out_ld < total) return set_err(h, AG_E_INVALID, "out_ld must be >= n * n_obs");
    if ((env_lo == nullptr) != (env_hi == nullptr)) return set_err(h, AG_E_INVALID, "env_lo and env_hi go together");
    if (!env_lo && (!box_lo || !box_hi)) return set_err(h, AG_E_INVALID, "box_lo and box_hi needed without env boxes");
    ObstArgs a{};
    a.slots = slots;
    a.env_lo = env_lo;
    a.env_hi = env_hi;
    a.mask = env_mask;
    a.out = out;
    a.n_env = h->cfg.n;
    a.ld = h->cfg.ld;
    a.out_ld = out_ld;
    a.t = step;
    a.n_obs = n_obs;
    a.key0 = h->key0;
    a.key1 = h->key1;
    a.index_base = (uint32_t)h->cfg.index_base;
    for (int d = 0; d < 3; ++d) {
        a.box_lo[d] = box_lo ? box_lo[d] : 0.0f;
        a.box_hi[d] = box_hi ? box_hi[d] : 0.0f;
    }
    return launch(h, obstacles_kernel(), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, &a);
}

ag_status ag_render_depth(ag_handle h, const ag_camera* cam, int32_t n_obs, const float* shapes, const float* obst,
                          int64_t obst_ld, int64_t first, int64_t count, float* depth) {
    AG_CHECK_HANDLE(h);
    if (!cam || !depth) return set_err(h, AG_E_INVALID, "camera and depth are required");
    if (cam->width < 1 || cam->height < 1 || !(cam->hfov > 0.0f && cam->hfov < 3.14159f) ||
        !(cam->max_depth > 0.0f))
        return set_err(h, AG_E_INVALID, "camera needs width, height >= 1, 0 < hfov < pi, max_depth > 0");
    if (n_obs < 0 || n_obs > 256 || (n_obs > 0 && (!shapes || !obst)))
        return set_err(h, AG_E_INVALID, "0 <= n_obs <= 256 with shapes and obst");
    if (first < 0 || count < 0 || first + count > h->cfg.n) return set_err(h, AG_E_INVALID, "vehicle range out of bounds");
    if (n_obs > 0 && obst_ld < h->cfg.n * (long long)n_obs) return set_err(h, AG_E_INVALID, "obst_ld must be >= n * n_obs");
    if (count == 0) return AG_OK;
    CameraArgs a{};
    a.state = h->cfg.state;
    a.shapes = shapes;
    a.obst = obst;
    a.depth = depth;
    a.ld = h->cfg.ld;
    a.obst_ld = obst_ld;
    a.n_obs = n_obs;
    a.W = cam->width;
    a.H = cam->height;
    a.has_floor = std::isnan(cam->floor_z) ? 0 : 1;
    a.floor_z = cam->floor_z;
    a.inv_f = (float)(std::tan(0.5 * (double)cam->hfov) / (0.5 * (double)cam->width));
    a.max_depth = cam->max_depth;
    for (int k = 0; k < 3; ++k) a.mount_p[k] = cam->mount_pos[k];
    for (int k = 0; k < 4; ++k) a.mount_q[k] = cam->mount_quat[k];
    const unsigned tiles = (unsigned)(((cam->width + 63) / 64) * ((cam->height + 3) / 4));
    const long long chunk = 65535;
    for (long long f0 = 0; f0 < count; f0 += chunk) {
        a.first = first + f0;
        a.depth = depth + f0 * (long long)cam->width * cam->height;
        const unsigned cnt = (unsigned)std::min(chunk, count - f0);
        ag_status st = launch(h, depth_kernel(), dim3(tiles, cnt), dim3(256), 0, &a);
        if (st != AG_OK) return st;
    }
    return AG_OK;
}

ag_status ag_apply_actions(ag_handle h, const float* actions, int64_t act_ld, int32_t mode, const float* scale,
                           const float* offset) {
    AG_CHECK_HANDLE(h);
    if (!actions || !scale || !offset) return set_err(h, AG_E_INVALID, "actions, scale and offset are required");
    if (act_ld < h->cfg.n) return set_err(h, AG_E_INVALID, "act_ld must be >= n");
    if (mode < 0 || mode > 3) return set_err(h, AG_E_INVALID, "action mode must be 0..3");
    ActArgs a{};
    a.actions = actions;
    a.target = h->cfg.target;
    a.mode = h->cfg.mode;
    a.n = h->cfg.n;
    a.ld = h->cfg.ld;
    a.act_ld = act_ld;
    a.new_mode = mode;
    for (int r = 0; r < 4; ++r) {
        a.scale[r] = scale[r];
        a.offset[r] = offset[r];
    }
    h->order_valid = false;
    return launch(h, actions_kernel(), dim3((unsigned)((h->cfg.n + 255) / 256)), dim3(256), 0, &a);
}

ag_status ag_observe(ag_handle h, const ag_task* task, int32_t advance, float* obs, int64_t obs_ld, float* reward,
                     uint8_t* done, int32_t* episode) {
    AG_CHECK_HANDLE(h);
    if (!task || !obs) return set_err(h, AG_E_INVALID, "task and obs are required");
    if (obs_ld < h->cfg.n) return set_err(h, AG_E_INVALID, "obs_ld must be >= n");
    if (advance && (!reward || !done || !episode))
        return set_err(h, AG_E_INVALID, "reward, done and episode are required when advancing");
    TaskArgs a{};
    a.state = h->cfg.state;
    a.goal = h->cfg.goal ? h->cfg.goal : h->cfg.target;
    a.goal_ld = h->cfg.ld;
    a.obs = obs;
    a.reward = reward;
    a.done = done;
    a.episode = episode;
    a.n = h->cfg.n;
    a.ld = h->cfg.ld;
    a.obs_ld = obs_ld;
    a.advance = advance ? 1 : 0;
    a.max_steps = task->max_steps;
    a.w_v = task->w_v;
    a.w_omega = task->w_omega;
    a.bonus = task->bonus;
    a.r_goal = task->r_goal;
    a.r_far = task->r_far;
    return launch(h, observe_kernel(), dim3((unsigned)((h->cfg.n + 255) / 256)), dim3(256), 0, &a);
}

ag_status ag_get_stats(ag_handle h, ag_stats* out, int32_t clear) {
    AG_CHECK_HANDLE(h);
    if (!out) return AG_E_INVALID;
    StatAcc acc{};
    AG_HIP(h, hipMemcpyAsync(&acc, h->acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    AG_HIP(h, hipStreamSynchronize(h->stream));
    out->steps = acc.steps;
    out->n_saturated = acc.n_saturated;
    out->n_resets = acc.n_resets;
    out->n_invalid_mode = acc.n_invalid_mode;
    out->n_nonfinite = acc.n_nonfinite;
    out->n_finite = acc.n_finite;
    out->n_position = acc.n_position;
    out->pos_err_sum = acc.pos_err_sum;
    out->omega_sum = acc.omega_sum;
    if (clear) {
        StatAcc z{};
        z.n_nonfinite = acc.n_nonfinite;
        z.n_finite = acc.n_finite;
        z.n_position = acc.n_position;
        z.pos_err_sum = acc.pos_err_sum;
        z.omega_sum = acc.omega_sum;
        AG_HIP(h, hipMemcpyAsync(h->acc, &z, sizeof(z), hipMemcpyHostToDevice, h->stream));
        AG_HIP(h, hipStreamSynchronize(h->stream));
    }
    return AG_OK;
}

ag_status ag_get_step(ag_handle h, int64_t* step) {
    if (!h || !step) return AG_E_INVALID;
    *step = h->t;
    return AG_OK;
}

ag_status ag_set_step(ag_handle h, int64_t step) {
    AG_CHECK_HANDLE(h);
    if (step < 0) return set_err(h, AG_E_INVALID, "step must be >= 0");
    h->t = step;
    h->dev_step_dirty = true;
    return AG_OK;
}

ag_status ag_rollout_workspace_size(ag_handle h, int32_t n_steps, int32_t ckpt_every, size_t* bytes) {
    AG_CHECK_HANDLE(h);
    if (!bytes || n_steps < 1 || ckpt_every < 1) return AG_E_INVALID;
    const long long n = h->cfg.n;
    const long long n_ckpt = (n_steps + ckpt_every - 1) / ckpt_every;
    size_t off = 0;
    off = align_up(off + (size_t)n_ckpt * AG_STATE_DIM * n * sizeof(float));
    off = align_up(off + 2 * (size_t)ckpt_every * AG_STATE_DIM * n * sizeof(float));   // two tape buffers
    off = align_up(off + (size_t)((n + 63) / 64) * sizeof(double));                    // loss partials
    *bytes = off;
    return AG_OK;
}

}  // extern "C"

namespace {

ag_status rollout_args(ag_handle h, const float* x0, const float* gains, int32_t n_steps, int32_t ckpt_every,
                       float w_omega, void* ws, size_t ws_bytes, RolloutArgs& a, LaunchShape& s) {
    if (n_steps < 1 || ckpt_every < 1) return set_err(h, AG_E_INVALID, "n_steps and ckpt_every must be >= 1");
    if (!h->cfg.vparams) return set_err(h, AG_E_UNSUPPORTED, "rollouts differentiate per-vehicle gains: vparams required");
    if (h->cfg.traj) return set_err(h, AG_E_UNSUPPORTED, "rollouts of the tracking mode are not differentiated");
    if (!std::isfinite(w_omega)) return set_err(h, AG_E_INVALID, "w_omega must be finite");
    size_t need = 0;
    ag_status st = ag_rollout_workspace_size(h, n_steps, ckpt_every, &need);
    if (st != AG_OK) return st;
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return set_err(h, AG_E_NOMEM, "rollout workspace missing, misaligned or too small");
    const long long n = h->cfg.n;
    const long long n_ckpt = (n_steps + ckpt_every - 1) / ckpt_every;
    char* base = static_cast<char*>(ws);
    const size_t ckpt_bytes = align_up((size_t)n_ckpt * AG_STATE_DIM * n * sizeof(float));
    const size_t tape_bytes = align_up(2 * (size_t)ckpt_every * AG_STATE_DIM * n * sizeof(float));
    a = RolloutArgs{};
    a.x0 = x0 ? x0 : h->cfg.state;
    a.gains = gains;
    a.mode = h->cfg.mode;
    a.target = h->cfg.target;
    a.vparams = h->cfg.vparams;
    a.gtab = h->gtab;
    a.goff = h->goff;
    a.ckpt = reinterpret_cast<float*>(base);
    a.tape = reinterpret_cast<float*>(base + ckpt_bytes);
    a.loss_part = reinterpret_cast<double*>(base + ckpt_bytes + tape_bytes);
    a.n = n;
    a.ld = h->cfg.ld;
    a.n_groups = h->cfg.n_groups;
    a.T = n_steps;
    a.m = ckpt_every;
    a.n_ckpt = (int)n_ckpt;
    a.dt = h->cfg.dt;
    a.g = h->cfg.g;
    a.w_omega = w_omega;
    const int span = tile_span(h, kRolloutBlock);
    a.span = span;
    s.span = span;
    s.shmem = lds_bytes(span);
    s.block = dim3(kRolloutBlock);
    s.grid = dim3((unsigned)((n + kRolloutBlock - 1) / kRolloutBlock));
    return AG_OK;
}

}  // namespace

extern "C" {

ag_status ag_rollout_forward(ag_handle h, const float* x0, const float* gains, int32_t n_steps, int32_t ckpt_every,
                             float w_omega, void* ws, size_t ws_bytes, float* loss_out, float* batch_loss,
                             float* final_state) {
    AG_CHECK_HANDLE(h);
    RolloutArgs a;
    LaunchShape s;
    ag_status st = rollout_args(h, x0, gains, n_steps, ckpt_every, w_omega, ws, ws_bytes, a, s);
    if (st != AG_OK) return st;
    a.loss_out = loss_out;
    a.final_state = final_state;
    if (!batch_loss) a.loss_part = nullptr;
    st = launch(h, rollout_fwd_kernel(h->nr_class), s.grid, s.block, s.shmem, &a);
    if (st != AG_OK || !batch_loss) return st;
    LossFoldArgs f{a.loss_part, (int32_t)s.grid.x, 1.0 / (double)h->cfg.n, batch_loss};
    return launch(h, loss_fold_kernel(), dim3(1), dim3(256), 0, &f);
}

ag_status ag_rollout_adjoint(ag_handle h, const float* x0, const float* gains, int32_t n_steps, int32_t ckpt_every,
                             float w_omega, float seed_grad, const float* seed_dev, void* ws, size_t ws_bytes,
                             float* dgains, float* dx0) {
    AG_CHECK_HANDLE(h);
    if (!dgains || !dx0) return set_err(h, AG_E_INVALID, "dgains and dx0 are required");
    RolloutArgs a;
    LaunchShape s;
    ag_status st = rollout_args(h, x0, gains, n_steps, ckpt_every, w_omega, ws, ws_bytes, a, s);
    if (st != AG_OK) return st;
    a.dgains = dgains;
    a.dx0 = dx0;
    a.seed_grad = seed_grad;
    a.inv_n = 1.0f / (float)h->cfg.n;
    a.seed_dev = seed_dev;
    // two wavefronts per 64 vehicles: reverse sweep and recomputation
    return launch(h, rollout_adj_kernel(h->nr_class), s.grid, dim3(2 * kRolloutBlock), s.shmem, &a);
}

ag_status ag_rollout_grad_noalloc(ag_handle h, const float* x0, const float* gains, int32_t n_steps,
                                  int32_t ckpt_every, float w_omega, float seed_grad, float* loss_out,
                                  float* batch_loss, float* dgains, float* dx0) {
    AG_CHECK_HANDLE(h);
    if (!h->noalloc_scratch)
        return hip_fail(h, h->noalloc_err, "ag_rollout_grad_noalloc: device address of the static scratch");
    size_t need = 0;
    ag_status st = ag_rollout_workspace_size(h, n_steps, ckpt_every, &need);
    if (st != AG_OK) return set_err(h, st, "n_steps and ckpt_every must be >= 1");
    if (need > kNoAllocScratchBytes) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "ag_rollout_grad_noalloc: the rollout needs %zu bytes of scratch, the static scratch holds %zu",
                      need, kNoAllocScratchBytes);
        return set_err(h, AG_E_NOMEM, msg);
    }
    st = ag_rollout_forward(h, x0, gains, n_steps, ckpt_every, w_omega, h->noalloc_scratch, kNoAllocScratchBytes,
                            loss_out, batch_loss, nullptr);
    if (st != AG_OK) return st;
    return ag_rollout_adjoint(h, x0, gains, n_steps, ckpt_every, w_omega, seed_grad, nullptr, h->noalloc_scratch,
                              kNoAllocScratchBytes, dgains, dx0);
}

ag_status ag_sync(ag_handle h) {
    if (!h) return AG_E_INVALID;
    if (h->sticky != AG_OK) return h->sticky;
    AG_HIP(h, hipStreamSynchronize(h->stream));
    return AG_OK;
}

const char* ag_last_error(ag_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
