// ag_rollout.hip -- differentiable rollout of the tracking loss (gfx950).
//
// Forward: each lane runs its vehicle for T steps from x0 with the step
// function of the simulator, accumulates its loss
//   l_i = sum_{t=1..T} |x_t - goal|^2 + w_omega |Omega_t|^2
// and writes the state every m steps to a checkpoint array.
// Adjoint: the segments between checkpoints are handled last to first.  A
// segment's states are recomputed from its checkpoint into a tape (structure-
// of-arrays in the caller's workspace), then the tape is walked backwards
// running the hand-written reverse of each step (step_core<..., GRAD = true>),
// which adds the loss gradient of the post-step state and pulls the adjoint
// back to the pre-step state while accumulating the gain adjoints.  A block
// holds 64 vehicles and two wavefronts: while wavefront 0 sweeps segment s
// backwards from tape buffer s & 1, wavefront 1 recomputes segment s - 1 into
// the other buffer, and a block barrier separates the segments.  With one
// vehicle per lane the reverse sweep alone is latency-bound (the 65,536-
// vehicle workload fills one wavefront per SIMD), so the recomputation runs
// in the issue slots it leaves idle.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ag.h"
#include "ag_internal.h"
#include "ag_step.h"

namespace ag {

__device__ __forceinline__ int rollout_find_group(const int32_t* __restrict__ goff, int n_groups, long long i) {
    int lo = 0, hi = n_groups;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((long long)goff[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Stage the groups overlapping vehicles [base, end) (every thread of the
// block calls it); returns the group entry of vehicle i.
__device__ __forceinline__ const float* rollout_stage(const RolloutArgs& a, float* lds, int* loff, int* sh,
                                                      long long base, long long end, long long i) {
    if (threadIdx.x == 0) {
        const int glo = a.n_groups == 1 ? 0 : rollout_find_group(a.goff, a.n_groups, base);
        const int ghi = a.n_groups == 1 ? 0 : rollout_find_group(a.goff, a.n_groups, end - 1);
        sh[0] = glo;
        sh[1] = ghi - glo + 1;
    }
    __syncthreads();
    const int glo = sh[0], cnt = sh[1];
    for (int e = threadIdx.x; e < cnt * GSTRIDE; e += blockDim.x) lds[e] = a.gtab[(long long)glo * GSTRIDE + e];
    for (int e = threadIdx.x; e <= cnt; e += blockDim.x) loff[e] = a.goff[glo + e];
    __syncthreads();
    int j = 0;
    while (j + 1 < cnt && i >= (long long)loff[j + 1]) ++j;
    return lds + j * GSTRIDE;
}

// The vehicle's group entry held in registers for the whole rollout: at the
// rollouts' sizes a SIMD runs one or two wavefronts, too few to hide the LDS
// latency of the allocation table on every step.
struct EntryRegs {
    float e[GSTRIDE];
};

__device__ __forceinline__ void copy_entry(EntryRegs& g, const float* gt) {
#pragma unroll
    for (int k = 0; k < GSTRIDE; ++k) g.e[k] = gt[k];
}

// The mode shared by every active lane of the wavefront if it is 0, 1 or 2
// (the step then runs that mode's specialised copy), else -1.
__device__ __forceinline__ int wave_mode(int mode) {
    const int mf = __builtin_amdgcn_readfirstlane(mode);
    return (__all(mode == mf) && mf >= 0 && mf <= 2) ? mf : -1;
}

// Call fn with std::integral_constant<int, wm> for wm in -1..2 (wm uniform
// across the wavefront).
template <typename F>
__device__ __forceinline__ void by_mode(int wm, F&& fn) {
    switch (wm) {
    case 0: fn(std::integral_constant<int, 0>{}); break;
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    default: fn(std::integral_constant<int, -1>{}); break;
    }
}

// The rollout's own gains (gains rows, when given) in place of the vparams rows.
__device__ __forceinline__ void override_gains(Params& P, const float* __restrict__ gains, long long ld,
                                               long long i) {
    if (!gains) return;
    P.kx_xy = gains[i];
    P.kx_z = gains[ld + i];
    P.kv_xy = gains[2 * ld + i];
    P.kv_z = gains[3 * ld + i];
    P.kR0 = gains[4 * ld + i];
    P.kR1 = gains[5 * ld + i];
    P.kR2 = gains[6 * ld + i];
    P.kW0 = gains[7 * ld + i];
    P.kW1 = gains[8 * ld + i];
    P.kW2 = gains[9 * ld + i];
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Forward rollout; one wavefront (64 vehicles) per block.
template <int NR>
__global__ __launch_bounds__(64) void k_rollout_fwd(RolloutArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    int* loff = reinterpret_cast<int*>(lds + a.span * GSTRIDE);
    __shared__ int sh[2];
    const long long base = (long long)blockIdx.x * blockDim.x;
    const long long i = base + threadIdx.x;
    const float* gl = rollout_stage(a, lds, loff, sh, base, base + blockDim.x < a.n ? base + blockDim.x : a.n, i);
    double loss = 0.0;
    if (i < a.n) {
        EntryRegs ge;
        copy_entry(ge, gl);
        const float* gt = ge.e;
        const long long ld = a.ld, n = a.n;
        float s[13];
#pragma unroll
        for (int r = 0; r < 13; ++r) s[r] = a.x0[r * ld + i];
        Params P;
        load_params<true>(P, gt, a.vparams, ld, i);
        override_gains(P, a.gains, ld, i);
        Cmd C;
        derive_cmd(C, (int)a.mode[i], a.target[i], a.target[ld + i], a.target[2 * ld + i], a.target[3 * ld + i]);
        const float gx = C.t0, gy = C.t1, gz = C.t2;
        by_mode(wave_mode(C.mode), [&](auto ms) {
            constexpr int MS = decltype(ms)::value;
            for (int t = 0; t < a.T; ++t) {
                if (t % a.m == 0) {
                    float* ck = a.ckpt + (long long)(t / a.m) * 13 * n;
#pragma unroll
                    for (int r = 0; r < 13; ++r) ck[r * n + i] = s[r];
                }
                step<NR, false, false, false, MS>(s, C, P, gt, a.dt, a.g, nullptr, nullptr);
                const float ex = s[0] - gx, ey = s[1] - gy, ez = s[2] - gz;
                const float lt =
                    ex * ex + ey * ey + ez * ez + a.w_omega * (s[10] * s[10] + s[11] * s[11] + s[12] * s[12]);
                loss += (double)lt;
            }
        });
        if (a.loss_out) a.loss_out[i] = (float)loss;
        if (a.final_state) {
#pragma unroll
            for (int r = 0; r < 13; ++r) a.final_state[r * ld + i] = s[r];
        }
    }
    if (a.loss_part) {
        // the block's 64 vehicle sums in a fixed butterfly order (lanes past n add 0)
        const double b = wave_sum_f64(loss);
        if (threadIdx.x == 0) a.loss_part[blockIdx.x] = b;
    }
}

// Batch loss: one block; thread t adds partials t, t + 256, ... in order, then
// the 256 sums are added in a fixed butterfly and wavefront order.
__global__ __launch_bounds__(256) void k_loss_fold(LossFoldArgs a) {
    __shared__ double w[4];
    double v = 0.0;
    for (int p = threadIdx.x; p < a.nparts; p += 256) v += a.part[p];
    v = wave_sum_f64(v);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) a.out[0] = (float)(((w[0] + w[1]) + (w[2] + w[3])) * a.inv_n);
}

// Recompute segment seg from its checkpoint: tape entry t - t0 = state before step t.
template <int NR, int MS>
__device__ __forceinline__ void recompute_segment(const RolloutArgs& a, const Params& P, const Cmd& C,
                                                  const float* gt, int seg, float* tape, long long i) {
    const long long n = a.n;
    const int t0 = seg * a.m;
    const int t1 = t0 + a.m < a.T ? t0 + a.m : a.T;
    const float* ck = a.ckpt + (long long)seg * 13 * n;
    float s[13];
#pragma unroll
    for (int r = 0; r < 13; ++r) s[r] = ck[r * n + i];
    for (int t = t0; t < t1; ++t) {
        float* tp = tape + (long long)(t - t0) * 13 * n;
#pragma unroll
        for (int r = 0; r < 13; ++r) tp[r * n + i] = s[r];
        if (t + 1 < t1) step<NR, false, false, false, MS>(s, C, P, gt, a.dt, a.g, nullptr, nullptr);
    }
}

// Reverse sweep of segment seg over its tape; the next (earlier) tape entry is
// loaded while the current step's reverse runs, hiding the load latency.
template <int NR, int MS>
__device__ __forceinline__ void reverse_segment(const RolloutArgs& a, const Params& P, const Cmd& C,
                                                const float* gt, int seg, const float* tape, long long i, Adj& A) {
    const long long n = a.n;
    const int t0 = seg * a.m;
    const int t1 = t0 + a.m < a.T ? t0 + a.m : a.T;
    float s[13], nxt[13];
    {
        const float* tp = tape + (long long)(t1 - 1 - t0) * 13 * n;
#pragma unroll
        for (int r = 0; r < 13; ++r) nxt[r] = tp[r * n + i];
    }
    for (int t = t1 - 1; t >= t0; --t) {
#pragma unroll
        for (int r = 0; r < 13; ++r) s[r] = nxt[r];
        if (t > t0) {
            const float* tp = tape + (long long)(t - 1 - t0) * 13 * n;
#pragma unroll
            for (int r = 0; r < 13; ++r) nxt[r] = tp[r * n + i];
        }
        step_core<NR, false, false, true, false, MS>(s, C, P, gt, a.dt, a.g, nullptr, nullptr, &A);
    }
}

// Block = 64 vehicles x 2 wavefronts (see the file comment).  Every thread
// passes the same barriers: no early exit, lanes past n only skip the work.
template <int NR>
__global__ __launch_bounds__(128) void k_rollout_adj(RolloutArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    int* loff = reinterpret_cast<int*>(lds + a.span * GSTRIDE);
    __shared__ int sh[2];
    const bool reverse_wave = threadIdx.x < 64;       // uniform per wavefront
    const long long base = (long long)blockIdx.x * 64;
    const long long i = base + (threadIdx.x & 63);
    const float* gl = rollout_stage(a, lds, loff, sh, base, base + 64 < a.n ? base + 64 : a.n, i);
    EntryRegs ge;
    copy_entry(ge, gl);
    const float* gt = ge.e;
    const bool act = i < a.n;
    const long long ld = a.ld;
    const long long buf = (long long)a.m * 13 * a.n;   // floats per tape buffer
    Params P = {};
    Cmd C = {};
    if (act) {
        load_params<true>(P, gt, a.vparams, ld, i);
        override_gains(P, a.gains, ld, i);
        derive_cmd(C, (int)a.mode[i], a.target[i], a.target[ld + i], a.target[2 * ld + i], a.target[3 * ld + i]);
    }
    const int last = a.n_ckpt - 1;
    // every step of this wavefront runs its mode's specialised copy when its
    // vehicles share a mode
    const int wm = wave_mode(C.mode);
    if (!reverse_wave && act)
        by_mode(wm, [&](auto ms) {
            recompute_segment<NR, decltype(ms)::value>(a, P, C, gt, last, a.tape + (last & 1) * buf, i);
        });
    __syncthreads();
    Adj A;
#pragma unroll
    for (int r = 0; r < 13; ++r) A.lam[r] = 0.0f;
#pragma unroll
    for (int r = 0; r < 10; ++r) A.gb[r] = 0.0f;
    A.gx = C.t0; A.gy = C.t1; A.gz = C.t2;
    A.w_omega = a.w_omega;
    for (int seg = last; seg >= 0; --seg) {
        if (reverse_wave) {
            if (act)
                by_mode(wm, [&](auto ms) {
                    reverse_segment<NR, decltype(ms)::value>(a, P, C, gt, seg, a.tape + (seg & 1) * buf, i, A);
                });
        } else if (seg > 0 && act) {
            by_mode(wm, [&](auto ms) {
                recompute_segment<NR, decltype(ms)::value>(a, P, C, gt, seg - 1, a.tape + ((seg - 1) & 1) * buf, i);
            });
        }
        __syncthreads();
    }
    if (reverse_wave && act) {
        // (seed_grad times the device factor, then 1/n: an upstream gradient
        // given either way yields the same bits)
        const float sc = (a.seed_dev ? a.seed_grad * a.seed_dev[0] : a.seed_grad) * a.inv_n;
#pragma unroll
        for (int r = 0; r < 10; ++r) a.dgains[r * ld + i] = A.gb[r] * sc;
#pragma unroll
        for (int r = 0; r < 13; ++r) a.dx0[r * ld + i] = A.lam[r] * sc;
    }
}

const void* rollout_fwd_kernel(int nr_class) {
    switch (nr_class) {
        case 4: return reinterpret_cast<const void*>(&k_rollout_fwd<4>);
        case 6: return reinterpret_cast<const void*>(&k_rollout_fwd<6>);
        case 8: return reinterpret_cast<const void*>(&k_rollout_fwd<8>);
        default: return reinterpret_cast<const void*>(&k_rollout_fwd<0>);
    }
}

const void* loss_fold_kernel() { return reinterpret_cast<const void*>(&k_loss_fold); }

const void* rollout_adj_kernel(int nr_class) {
    switch (nr_class) {
        case 4: return reinterpret_cast<const void*>(&k_rollout_adj<4>);
        case 6: return reinterpret_cast<const void*>(&k_rollout_adj<6>);
        case 8: return reinterpret_cast<const void*>(&k_rollout_adj<8>);
        default: return reinterpret_cast<const void*>(&k_rollout_adj<0>);
    }
}

}  // namespace ag
