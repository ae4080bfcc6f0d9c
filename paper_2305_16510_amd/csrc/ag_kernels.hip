// ag_kernels.hip -- HIP kernels of the batched multirotor step for gfx950.
//
// Layout.  State, targets, parameters and outputs are structure-of-arrays
// rows of length ld, so lane i of a wavefront touches element i of each row:
// every load and store is a fully coalesced 256-byte wavefront access.  Each
// block stages the table entries of the vehicle groups its tile overlaps in
// LDS (rotor allocation matrix and pseudo-inverse, inverses of mass and
// inertia, default gains); lanes find their group by scanning the staged
// group offsets.  A per-step launch of a single group loads its one entry
// ahead of the state, so the staging waits for the entry alone.
//
// k_step<NR, VP, RST, VPL, ONE, OBS, TRK> is both the per-step kernel (ONE: one step
// per launch, one tile per block) and the fused kernel (k steps per launch
// with the state held in registers, VPL vehicles per lane, grid-stride loop
// over tiles).  A grid that is a multiple of 8 keeps each tile on the same
// XCD (and so the same L2) from launch to launch.  Both forms run the same
// device function per step, so their results are bitwise identical.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ag.h"
#include "ag_internal.h"
#include "ag_step.h"

namespace ag {

__device__ __forceinline__ int find_group(const int32_t* __restrict__ goff, int n_groups, long long i) {
    int lo = 0, hi = n_groups;              // goff[lo] <= i < goff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((long long)goff[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Stage the group entries overlapping vehicles [base, end) into LDS.
__device__ __forceinline__ void stage_groups(float* lds, int* loff, int* sh, const float* __restrict__ gtab,
                                             const int32_t* __restrict__ goff, int n_groups,
                                             long long base, long long end) {
    if (threadIdx.x == 0) {
        const int glo = n_groups == 1 ? 0 : find_group(goff, n_groups, base);
        const int ghi = n_groups == 1 ? 0 : find_group(goff, n_groups, end - 1);
        sh[0] = glo;
        sh[1] = ghi - glo + 1;
    }
    __syncthreads();
    const int glo = sh[0], cnt = sh[1];
    for (int e = threadIdx.x; e < cnt * GSTRIDE; e += blockDim.x) lds[e] = gtab[(long long)glo * GSTRIDE + e];
    for (int e = threadIdx.x; e <= cnt; e += blockDim.x) loff[e] = goff[glo + e];
    __syncthreads();
}

__device__ __forceinline__ const float* lane_group(const float* lds, const int* loff, int cnt, long long i) {
    int j = 0;
    while (j + 1 < cnt && i >= (long long)loff[j + 1]) ++j;
    return lds + j * GSTRIDE;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block reduction of the per-lane statistics into one slot.
__device__ void block_stats(StatSlot* slots, long long c_sat, long long c_res, long long c_nonf,
                            long long c_fin, long long c_pos, double s_err, double s_w) {
    __shared__ long long red_i[16][5];
    __shared__ double red_d[16][2];
    c_sat = wave_sum(c_sat); c_res = wave_sum(c_res); c_nonf = wave_sum(c_nonf);
    c_fin = wave_sum(c_fin); c_pos = wave_sum(c_pos);
    s_err = wave_sum(s_err); s_w = wave_sum(s_w);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red_i[wid][0] = c_sat; red_i[wid][1] = c_res; red_i[wid][2] = c_nonf;
        red_i[wid][3] = c_fin; red_i[wid][4] = c_pos;
        red_d[wid][0] = s_err; red_d[wid][1] = s_w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        long long a[5] = {0, 0, 0, 0, 0};
        double d[2] = {0.0, 0.0};
        for (int w = 0; w < nw; ++w) {
            for (int k = 0; k < 5; ++k) a[k] += red_i[w][k];
            d[0] += red_d[w][0];
            d[1] += red_d[w][1];
        }
        StatSlot* s = slots + blockIdx.x;
        s->n_saturated += a[0];
        s->n_resets += a[1];
        s->n_nonfinite = a[2];
        s->n_finite = a[3];
        s->n_position = a[4];
        s->pos_err_sum = d[0];
        s->omega_sum = d[1];
    }
}

// Fused one-vehicle-per-lane kernels without trajectories carry mode-
// specialised copies of the step loop: those without resets when no observer
// is bound, and those fed by the reset events (whose loop holds only the
// event test and a copy of the redrawn state).  The other forms would exceed
// 128 registers with them.
constexpr bool spec_loops(bool one, int vpl, bool obs, bool trk, int rst) {
    return !one && vpl == 1 && !trk && ((rst == 0 && !obs) || rst == 2);
}

// s_waitcnt immediates (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVm0 = 0x0F70;                // every vector memory access done
constexpr int kWaitLgkm0 = 0xC07F;              // every LDS access done

// The tiles of one block.  UNI (per-step kernels of a single-group launch):
// the one group entry is loaded ahead of the state and written to LDS
// without the group search and its extra barrier.
template <int NR, bool VP, int RST, int VPL, bool ONE, bool OBS, bool TRK, bool UNI>
__device__ __forceinline__ void step_tiles(const StepArgs& a, float* lds, int* loff, int* sh) {
    // RST: 0 no resets; 1 resets (per-step form: found and redrawn here; fused
    // form: from the event kernels, events past the buffer redrawn here); 2
    // fused form with every event of the launch in the buffer (no redraw code)
    constexpr bool RESET = RST != 0;
    constexpr bool EV = RESET && !ONE;
    constexpr bool FB = !(EV && RST == 2);
    constexpr bool SPEC = spec_loops(ONE, VPL, OBS, TRK, RST);
    // every event of the launch in the buffer, one vehicle per lane: each
    // wavefront copies its events into LDS at tile start
    constexpr bool STAGE = EV && RST == 2 && VPL == 1;
    const int B = blockDim.x;
    const long long TILE = (long long)B * VPL;
    const long long tbase = a.d_step ? (*a.d_step + a.t_off) : a.t0;
    const int K = ONE ? 1 : a.k;
    const long long ld = a.ld;
    // OBS: some observer (wrench or rotor outputs, flags, statistics) is bound;
    // without one the saturation and reset counting compiles away.
    const bool want_out = OBS && (a.wrench_out != nullptr || a.rotor_out != nullptr);

    long long c_sat = 0, c_res = 0, c_nonf = 0, c_fin = 0, c_pos = 0;
    double s_err = 0.0, s_w = 0.0;

    auto tile_body = [&](const long long base) {
        const long long end = base + TILE < a.n ? base + TILE : a.n;
        float s[VPL][13];
        float tg[VPL][4];
        int md[VPL];
        Cmd C[VPL];
        Params P[VPL];
        const float* gt[VPL];
        long long idx[VPL];
        bool act[VPL];
        int sat_last[VPL];
        bool did_reset[VPL];
        // Single group: the entry's loads go first, so the LDS write below
        // waits for them alone (loads complete in order), not for the state.
        // (Indices are clamped into range instead of branching, so that all
        // these loads sit in one basic block and each wait is exact.)
        // Lanes past the entry's end read and later write its last float, so
        // duplicate LDS writes carry identical values.
        const int e0 = (int)threadIdx.x < GSTRIDE ? (int)threadIdx.x : GSTRIDE - 1;
        const int e1 = (int)threadIdx.x + B < GSTRIDE ? (int)threadIdx.x + B : GSTRIDE - 1;
        float te0 = 0.0f, te1 = 0.0f;
        if constexpr (UNI) {
            te0 = a.gtab[e0];
            te1 = a.gtab[e1];
        }
        // the tile's state and command loads are issued before the group-table
        // staging and its barriers, so that their latencies overlap; lanes past
        // n load vehicle n - 1 and discard it
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const long long p = base + (long long)v * B + threadIdx.x;
            act[v] = p < a.n;
            sat_last[v] = 0;
            did_reset[v] = false;
            const long long pl = act[v] ? p : a.n - 1;
            // with a mode order, lane position p steps vehicle perm[p] (same
            // group as vehicle p, so the staged table entries still apply)
            const long long il = (SPEC && a.perm) ? (long long)a.perm[pl] : pl;
            // (the other kernels store through the unclamped position, so the
            // compiler does not keep the load addresses live for the stores)
            idx[v] = SPEC ? il : p;
#pragma unroll
            for (int r = 0; r < 13; ++r) s[v][r] = a.state[r * ld + il];
            md[v] = (int)a.mode[il];
#pragma unroll
            for (int r = 0; r < 4; ++r) tg[v][r] = a.target[r * ld + il];
        }
        // fused launches with resets: this launch's reset events of each lane
        // (bit mask over the k steps, index of its first event)
        unsigned long long evb[VPL];
        int evn[VPL];          // the lane's next event (event indices are int32)
        if constexpr (EV) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const long long il = act[v] ? idx[v] : a.n - 1;
                evb[v] = act[v] ? a.ev.bits[il] : 0ull;
                evn[v] = a.ev.off[il];
            }
        }
        // The wavefront's events are consecutive in the event list (vehicle
        // order): its first kEvStage are copied into LDS by direct
        // global-to-LDS loads, so that a reset reads the redrawn state there
        // instead of waiting on memory (about half of all wavefront-steps hold
        // a reset at 1 % per step); later events are read from the buffer.
        // The range ends at lane 63's events: in a ragged last tile that lane
        // holds vehicle n - 1's offset, so the last vehicle's events are read
        // from the buffer.
        int e_lo = 0, n_st = 0;
        float* evs = lds;
        if (STAGE && a.ev_stage) {
            e_lo = __builtin_amdgcn_readfirstlane(evn[0]);
            const int e_end = __builtin_amdgcn_readlane(evn[0] + __builtin_popcountll(evb[0]), 63);
            n_st = e_end - e_lo < kEvStage ? e_end - e_lo : kEvStage;
            const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
            evs = lds + ev_stage_offset(a.span) + (size_t)w * 16 * kEvStage;
            if (n_st > 0) {
                const long long e = (long long)e_lo + (threadIdx.x & 63);
                const long long ec = e < a.ev.cap ? e : a.ev.cap - 1;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    __builtin_amdgcn_global_load_lds(a.ev.data + r * a.ev.cap + ec, evs + r * kEvStage, 4, 0, 0);
            }
        }
        int cnt = 1;
        if constexpr (UNI) {
            lds[e0] = te0;
            lds[e1] = te1;
            __syncthreads();
        } else {
            stage_groups(lds, loff, sh, a.gtab, a.goff, a.n_groups, base, end);
            cnt = sh[1];
        }
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            if (act[v]) {
                const long long i = idx[v];
                gt[v] = UNI ? lds : lane_group(lds, loff, cnt, i);
                load_params<VP>(P[v], gt[v], a.vparams, ld, i);
                derive_cmd(C[v], md[v], tg[v][0], tg[v][1], tg[v][2], tg[v][3]);
                if constexpr (TRK) derive_traj(C[v], a.traj, ld, i);
            }
        }

        if (STAGE && a.ev_stage) __builtin_amdgcn_s_waitcnt(kWaitVm0);   // the events are in LDS
        Wrench W[VPL];
        float u[VPL][RotorClass<NR>::NR];
        uint4 mw[VPL];
        long long mblk = -1;
        // one step of every lane; OUT: the step that writes the wrench and rotor
        // outputs (the launch's last), peeled off the loop so that the loop
        // does not carry its registers
        auto run_step = [&](const int st, auto out_tag, auto ms_tag) {
            constexpr bool OUT = decltype(out_tag)::value;
            constexpr int MS = decltype(ms_tag)::value;
            if constexpr (RESET && ONE) {
                // reset words of four consecutive steps come from one Philox call
                const long long tb = (tbase + st) >> 2;
                if (tb != mblk) {
                    mblk = tb;
#pragma unroll
                    for (int v = 0; v < VPL; ++v)
                        mw[v] = mask_block(a.index_base + (uint32_t)idx[v], (uint64_t)tb, a.key0, a.key1);
                }
            }
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                if (!act[v]) continue;
                if constexpr (RESET) {
                    const uint32_t gi = a.index_base + (uint32_t)idx[v];
                    bool hit;
                    if constexpr (EV) hit = (evb[v] >> st) & 1ull;
                    else hit = mask_hit(mw[v], tbase + st, a.thr);
                    if (hit) {
                        float gx, gy, gz;
                        if constexpr (EV) {
                            const int e = evn[v]++;
                            if (STAGE && e - e_lo < n_st) {
                                const float* ls = evs + (e - e_lo);
#pragma unroll
                                for (int r = 0; r < 13; ++r) s[v][r] = ls[r * kEvStage];
                                gx = ls[13 * kEvStage];
                                gy = ls[14 * kEvStage];
                                gz = ls[15 * kEvStage];
                            } else if (e < a.ev.cap) {
                                const float* ed = a.ev.data + e;
#pragma unroll
                                for (int r = 0; r < 13; ++r) s[v][r] = ed[r * a.ev.cap];
                                gx = ed[13 * a.ev.cap];
                                gy = ed[14 * a.ev.cap];
                                gz = ed[15 * a.ev.cap];
                            } else if constexpr (FB) {   // past the event buffer: redraw here
                                redraw(s[v], gx, gy, gz, gi, tbase + st, a.key0, a.key1, a.lo, a.hi);
                            }
                        } else {
                            redraw(s[v], gx, gy, gz, gi, tbase + st, a.key0, a.key1, a.lo, a.hi);
                        }
                        if (C[v].mode == 0) set_position_goal(C[v], gx, gy, gz);
                        if (a.goal) {
                            a.goal[idx[v]] = gx;
                            a.goal[ld + idx[v]] = gy;
                            a.goal[2 * ld + idx[v]] = gz;
                        }
                        did_reset[v] = true;
                        if constexpr (OBS) ++c_res;
                    }
                }
                int ns;
                if constexpr (OUT) ns = step<NR, true, true, TRK>(s[v], C[v], P[v], gt[v], a.dt, a.g, &W[v], u[v]);
                else ns = step<NR, false, false, TRK, MS>(s[v], C[v], P[v], gt[v], a.dt, a.g, nullptr, nullptr);
                if constexpr (OBS) {
                    c_sat += ns;
                    sat_last[v] = ns;
                }
            }
        };
        const int k_loop = want_out ? K - 1 : K;
        using General = std::integral_constant<int, -1>;
        auto run_loop = [&](auto ms_tag) {
            for (int st = 0; st < k_loop; ++st) run_step(st, std::false_type{}, ms_tag);
        };
        if constexpr (SPEC) {
            const int m_first = __builtin_amdgcn_readfirstlane(md[0]);
            const int wm = __all(md[0] == m_first) ? m_first : -1;
            if constexpr (RESET) {
                // the event-fed loop has one copy, position mode: resets redraw
                // goals of position-mode vehicles
                if (wm == 0) {
                    for (int st = 0; st < k_loop; ++st) run_step(st, std::false_type{}, std::integral_constant<int, 0>{});
                } else {
                    for (int st = 0; st < k_loop; ++st) run_step(st, std::false_type{}, General{});
                }
            } else {
                switch (wm) {
                case 0: run_loop(std::integral_constant<int, 0>{}); break;
                case 1: run_loop(std::integral_constant<int, 1>{}); break;
                case 2: run_loop(std::integral_constant<int, 2>{}); break;
                default: run_loop(General{}); break;
                }
            }
        } else {
            // (the plain loop, not run_loop: the per-step kernels compile to
            // fewer registers this way)
            for (int st = 0; st < k_loop; ++st) run_step(st, std::false_type{}, General{});
        }
        if (want_out) run_step(K - 1, std::true_type{}, General{});

#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            if (!act[v]) continue;
            long long i = idx[v];
            // the store addresses are formed here, not kept from the loads
            // across the step loop (they would hold 26 registers)
            if constexpr (SPEC) asm volatile("" : "+v"(i));
#pragma unroll
            for (int r = 0; r < 13; ++r) a.state[r * ld + i] = s[v][r];
            if constexpr (RESET) {
                if (did_reset[v] && C[v].mode == 0) {
                    a.target[i] = C[v].t0;
                    a.target[ld + i] = C[v].t1;
                    a.target[2 * ld + i] = C[v].t2;
                    a.target[3 * ld + i] = C[v].t3;
                }
            }
            if (want_out) {
                if (a.wrench_out) {
                    a.wrench_out[i] = W[v].f;
                    a.wrench_out[ld + i] = W[v].M0;
                    a.wrench_out[2 * ld + i] = W[v].M1;
                    a.wrench_out[3 * ld + i] = W[v].M2;
                    a.wrench_out[4 * ld + i] = W[v].fa;
                    a.wrench_out[5 * ld + i] = W[v].Ma0;
                    a.wrench_out[6 * ld + i] = W[v].Ma1;
                    a.wrench_out[7 * ld + i] = W[v].Ma2;
                }
                if (a.rotor_out) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) a.rotor_out[r * ld + i] = r < RotorClass<NR>::NR ? u[v][r] : 0.0f;
                }
            }
            bool finite = true;
#pragma unroll
            for (int r = 0; r < 13; ++r) finite = finite && isfinite(s[v][r]);
            if (OBS && a.flags_out) {
                uint8_t fl = (finite ? 0 : AG_FLAG_NONFINITE) | (sat_last[v] ? AG_FLAG_SATURATED : 0) |
                             (did_reset[v] ? AG_FLAG_RESET : 0);
                if (a.flags_accumulate) fl |= (a.flags_out[i] & AG_FLAG_RESET);
                a.flags_out[i] = fl;
            }
            if (OBS && a.slots) {
                if (finite) {
                    ++c_fin;
                    s_w += (double)sqrtf(s[v][10] * s[v][10] + s[v][11] * s[v][11] + s[v][12] * s[v][12]);
                    if (C[v].mode == 0) {
                        ++c_pos;
                        const float ex = s[v][0] - C[v].t0, ey = s[v][1] - C[v].t1, ez = s[v][2] - C[v].t2;
                        s_err += (double)sqrtf(ex * ex + ey * ey + ez * ez);
                    }
                } else {
                    ++c_nonf;
                }
            }
        }
        __syncthreads();   // LDS is restaged for the next tile
    };
    if constexpr (ONE) {
        // a per-step launch has one block per tile (its grid is the tile count),
        // and no loop: nothing written by the block precedes its table reads
        const long long base = (long long)blockIdx.x * TILE;
        if (base < a.n) tile_body(base);
    } else {
        const long long ntiles = (a.n + TILE - 1) / TILE;
        if (SPEC && NR != 0 && a.perm && (long long)gridDim.x == ntiles) {
            // In mode order, the three mode runs of a segment read the same
            // cache lines (each wavefront gathers its 64 vehicles from about
            // 192 positions).  Blocks are dealt to the 8 XCDs in turn (block i
            // to XCD i mod 8); giving each XCD a contiguous eighth of the
            // tiles lets those runs meet in one L2.  (Not for launches mixing
            // rotor counts: their groups would load the XCDs unevenly.)
            const long long i = blockIdx.x, x = i & 7, j = i >> 3;
            const long long per = ntiles >> 3, rem = ntiles & 7;
            tile_body((x * per + (x < rem ? x : rem) + j) * TILE);
        } else {
            for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) tile_body(tile * TILE);
        }
    }
    if constexpr (OBS) {
        if (a.slots) block_stats(a.slots, c_sat, c_res, c_nonf, c_fin, c_pos, s_err, s_w);
    }
}

template <int NR, bool VP, int RST, int VPL, bool ONE, bool OBS, bool TRK>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(VPL == 1 && !TRK && ((RST == 2 && !OBS) || spec_loops(ONE, VPL, OBS, TRK, RST)) ? (RST == 2 && OBS ? 3 : 4) : 1)))
void k_step(StepArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    int* loff = reinterpret_cast<int*>(lds + a.span * GSTRIDE);
    __shared__ int sh[2];
    if constexpr (RST != 0 && !ONE) {
        // both event variants are launched; the one that does not match the
        // launch's event count leaves at once (a uniform test)
        const bool fits = *a.ev.total <= a.ev.cap;
        if (fits != (RST == 2)) return;
    }
    if constexpr (ONE) {
        if (a.n_groups == 1) {     // uniform across the grid
            step_tiles<NR, VP, RST, VPL, ONE, OBS, TRK, true>(a, lds, loff, sh);
            return;
        }
    }
    step_tiles<NR, VP, RST, VPL, ONE, OBS, TRK, false>(a, lds, loff, sh);
}

// ---- fused steps from work queues, the next tile copied ahead --------------
// Persistent form of the fused kernel for single-group fleets without
// observers, resets, trajectories or per-vehicle parameters (one vehicle per
// lane, blocks of one wavefront).  The grid holds as many wavefronts as the
// chip runs at once, a multiple of the queue count.  The tiles (64 lane
// positions each) are split into kQueueSub * 8 contiguous ranges, one per
// queue, and block b serves queue (b mod 8, (b / 8) mod kQueueSub): blocks
// are dealt to the XCDs round robin, so each XCD serves one contiguous eighth
// of the tiles and the mode runs of a segment meet in one L2.  Wavefronts
// sharing a SIMD run at very different speeds (the SIMD issues from its
// oldest wavefront first), so after its first tile a wavefront takes tiles on
// demand: it asks its queue for the next one a few steps before the current
// one ends, late enough to hold on to little work the others could take.
// The next tile's rows (state and command, 17 floats per lane) are then
// copied into LDS by direct global-to-LDS loads, and its mode byte into a
// register, while the last steps of the current tile run; the waits for the
// ticket and the vehicle indices stall only this wavefront (the SIMD runs
// the others).  Each queue's two counters have a 256-byte line of their own
// (the atomics on one line are served one at a time); the last wavefront of
// a queue to finish clears them for the next launch.
constexpr int kQueueRows = 17;                  // floats per lane copied ahead
constexpr int kLead = 3;                        // steps left in a tile when the next is asked for

template <int NR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_step_q(StepArgs a) {
    extern __shared__ float4 lds4[];
    float* const lds = reinterpret_cast<float*>(lds4);   // the group entry
    float* const buf = lds + GSTRIDE;                     // [kQueueRows][64]
    const int lane = (int)threadIdx.x;
    const long long n = a.n, ld = a.ld;
    const int K = a.k;
    const long long ntiles = (n + 63) >> 6;
    constexpr int NQ = 8 * kQueueSub;
    const int qi = (int)(blockIdx.x & 7) * kQueueSub + (int)((blockIdx.x >> 3) % kQueueSub);
    const long long per = ntiles / NQ, rem = ntiles % NQ;
    const long long r0 = qi * per + (qi < rem ? qi : rem);
    const long long r1 = r0 + per + (qi < rem ? 1 : 0);
    unsigned* const q = a.queue + qi * kQueueLine;       // [0] tickets handed out, [1] wavefronts done
    const unsigned waves = gridDim.x / NQ;               // wavefronts serving this queue

    // a ticket of this queue (lane 0; the offset is an opaque zero: with a
    // visibly uniform address the compiler would combine the wavefront's
    // atomics and read the result back at once, waiting for it there)
    auto ticket = [&]() -> unsigned {
        unsigned k = 0;
        if (lane == 0) {
            int zero;
            asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
            k = atomicAdd(q + zero, 1u);
        }
        return k;
    };
    // lane position of tile t -> vehicle (mode order, or identity); positions
    // past n take vehicle n - 1 and are not stored
    auto vehicle = [&](long long t) -> int {
        const long long p = t * 64 + lane;
        const int pl = (int)(p < n ? p : n - 1);
        return a.perm ? a.perm[pl] : pl;
    };
    // copy vehicle i's rows into this lane's column of the buffer
    auto fetch = [&](int i) {
#pragma unroll
        for (int r = 0; r < 13; ++r) __builtin_amdgcn_global_load_lds(a.state + r * ld + i, buf + r * 64, 4, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) __builtin_amdgcn_global_load_lds(a.target + r * ld + i, buf + (13 + r) * 64, 4, 0, 0);
    };

    // the first tile is fixed: the wavefronts of a queue take its first tiles
    // in block order, and its tickets count the tiles after those.  Its
    // vehicles are asked for first, then the group entry (single group)
    long long t_cur = r0 + (long long)(blockIdx.x / NQ);
    int i_cur = t_cur < r1 ? vehicle(t_cur) : 0;
    for (int e = lane; e < GSTRIDE; e += 64) lds[e] = a.gtab[e];
    __syncthreads();
    const float* gt = lds;
    Params P;
    load_params<false>(P, gt, nullptr, ld, 0);
    // a SIMD issues from its oldest wavefront first, which would leave a
    // young one on its first tile until the end: a wavefront's priority
    // drops with each tile it completes, down to the lowest after three
    __builtin_amdgcn_s_setprio(3);
    int n_done = 0;
    if (t_cur < r1) {
        fetch(i_cur);
        int md = a.mode[i_cur];
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        // the next tile is asked for kLead steps before the current one ends
        // (at once for shorter launches): late enough that a wavefront holds
        // on to little work the others could take, early enough that its
        // rows arrive before they are needed
        const int s_ask = K > kLead ? K - kLead : 0;
        for (;;) {
            // the current tile's rows, from LDS
            float s[13], tg[4];
#pragma unroll
            for (int r = 0; r < 13; ++r) s[r] = buf[r * 64 + lane];
#pragma unroll
            for (int r = 0; r < 4; ++r) tg[r] = buf[(13 + r) * 64 + lane];
            const bool act = t_cur * 64 + lane < n;
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
            long long t_nxt = r1;
            int i_nxt = 0, md_nxt = 0;
            Cmd C;
            derive_cmd(C, md, tg[0], tg[1], tg[2], tg[3]);
            auto run = [&](auto ms) {
                constexpr int MS = decltype(ms)::value;
                for (int st = 0; st < s_ask; ++st) step<NR, false, false, false, MS>(s, C, P, gt, a.dt, a.g, nullptr, nullptr);
                // each ticket goes to one wavefront, and a wavefront stops
                // only at its first ticket past the queue's end, so every
                // tile of the queue is taken
                const unsigned k = ticket();
                __builtin_amdgcn_s_waitcnt(kWaitVm0);
                t_nxt = r0 + waves + (long long)(unsigned)__builtin_amdgcn_readfirstlane((int)k);
                if (t_nxt < r1) {
                    i_nxt = vehicle(t_nxt);
                    fetch(i_nxt);
                    md_nxt = a.mode[i_nxt];
                }
                for (int st = s_ask; st < K; ++st) step<NR, false, false, false, MS>(s, C, P, gt, a.dt, a.g, nullptr, nullptr);
            };
            const int m_first = __builtin_amdgcn_readfirstlane(md);
            const int wm = __all(md == m_first) ? m_first : -1;
            switch (wm) {
            case 0: run(std::integral_constant<int, 0>{}); break;
            case 1: run(std::integral_constant<int, 1>{}); break;
            case 2: run(std::integral_constant<int, 2>{}); break;
            default: run(std::integral_constant<int, -1>{}); break;
            }
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            if (act) {
#pragma unroll
                for (int r = 0; r < 13; ++r) a.state[r * ld + i_cur] = s[r];
            }
            if (t_nxt >= r1) break;
            ++n_done;
            if (n_done == 1) __builtin_amdgcn_s_setprio(2);
            else if (n_done == 2) __builtin_amdgcn_s_setprio(1);
            else if (n_done == 3) __builtin_amdgcn_s_setprio(0);
            t_cur = t_nxt;
            i_cur = i_nxt;
            md = md_nxt;
        }
    }
    // every ticket of this wavefront has been served (the waits above); the
    // last wavefront of the queue clears its counters for the next launch
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    if (lane == 0) {
        const unsigned d = atomicAdd(q + 1, 1u);
        if (d == waves - 1) {
            atomicExch(q, 0u);
            atomicExch(q + 1, 0u);
        }
    }
}

// ---- statistics fold: slots -> cumulative accumulator (one block) ---------
__global__ __launch_bounds__(256) void k_fold(FoldArgs a) {
    __shared__ long long ri[256][5];
    __shared__ double rd[256][2];
    long long c[5] = {0, 0, 0, 0, 0};
    double d[2] = {0.0, 0.0};
    for (int s = threadIdx.x; s < a.nslots; s += 256) {
        StatSlot* p = a.slots + s;
        c[0] += p->n_saturated; c[1] += p->n_resets; c[2] += p->n_nonfinite;
        c[3] += p->n_finite; c[4] += p->n_position;
        d[0] += p->pos_err_sum; d[1] += p->omega_sum;
        p->n_saturated = 0;
        p->n_resets = 0;
    }
    for (int k = 0; k < 5; ++k) ri[threadIdx.x][k] = c[k];
    rd[threadIdx.x][0] = d[0];
    rd[threadIdx.x][1] = d[1];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 5; ++k) ri[threadIdx.x][k] += ri[threadIdx.x + w][k];
            rd[threadIdx.x][0] += rd[threadIdx.x + w][0];
            rd[threadIdx.x][1] += rd[threadIdx.x + w][1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.acc->steps += a.steps;
        a.acc->n_saturated += ri[0][0];
        a.acc->n_resets += ri[0][1];
        if (a.has_final) {
            a.acc->n_nonfinite = ri[0][2];
            a.acc->n_finite = ri[0][3];
            a.acc->n_position = ri[0][4];
            a.acc->pos_err_sum = rd[0][0];
            a.acc->omega_sum = rd[0][1];
        }
    }
}

__global__ void k_clear_slots(ClearArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.nslots) {
        StatSlot z = {0, 0, 0, 0, 0, 0.0, 0.0, 0.0};
        a.slots[s] = z;
    }
}

__global__ void k_advance(CounterArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *a.d_step += a.value;
}

__global__ void k_set_step(CounterArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *a.d_step = a.value;
}

__global__ __launch_bounds__(256) void k_set_targets(SetTargetsArgs a) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.count) return;
    const long long i = a.first + j;
    if (a.mode_src) a.mode_dst[i] = a.mode_src[j];
    if (a.target_src) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a.target_dst[r * a.ld + i] = a.target_src[r * a.src_ld + j];
    }
    const int m = (int)a.mode_dst[i];
    if (m < 0 || m > 3) atomicAdd(reinterpret_cast<unsigned long long*>(&a.acc->n_invalid_mode), 1ull);
}

// ---- explicit reset: mask, redraw, per-block counts ------------------------
__global__ __launch_bounds__(kResetBlock) void k_reset_mask(ResetArgs a) {
    const long long i = (long long)blockIdx.x * kResetBlock + threadIdx.x;
    bool m = false;
    if (i < a.n) {
        const uint32_t gi = a.index_base + (uint32_t)i;
        m = a.mask_in ? (a.mask_in[i] != 0) : reset_mask(gi, a.t, a.key0, a.key1, a.thr);
        if (m) {
            float s[13], gx, gy, gz;
            redraw(s, gx, gy, gz, gi, a.t, a.key0, a.key1, a.lo, a.hi);
#pragma unroll
            for (int r = 0; r < 13; ++r) a.state[r * a.ld + i] = s[r];
            if (a.goal) {
                a.goal[i] = gx;
                a.goal[a.ld + i] = gy;
                a.goal[2 * a.ld + i] = gz;
            }
            if (a.mode[i] == 0) {
                a.target[i] = gx;
                a.target[a.ld + i] = gy;
                a.target[2 * a.ld + i] = gz;
                a.target[3 * a.ld + i] = 0.0f;
            }
        }
        if (a.mask_out) a.mask_out[i] = m ? 1 : 0;
    }
    const int c = __syncthreads_count(m);
    if (threadIdx.x == 0 && a.block_counts) a.block_counts[blockIdx.x] = c;
}

// Exclusive scan of the block counts in place (one block, fixed order).
__global__ __launch_bounds__(1024) void k_reset_scan(ScanArgs a) {
    __shared__ int buf[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < a.nblocks; base += 1024) {
        const int j = base + threadIdx.x;
        const int v = j < a.nblocks ? a.block_counts[j] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int t = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (j < a.nblocks) a.block_counts[j] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0 && a.count_out) *a.count_out = carry;
}

__global__ __launch_bounds__(kResetBlock) void k_reset_scatter(ScatterArgs a) {
    __shared__ int wave_cnt[kResetBlock / 64];
    const long long i = (long long)blockIdx.x * kResetBlock + threadIdx.x;
    const bool m = i < a.n && a.mask[i] != 0;
    const unsigned long long bal = __ballot(m);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int rank_in_wave = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wid] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; ++w) before += wave_cnt[w];
    if (m) a.indices[a.offsets[blockIdx.x] + before + rank_in_wave] = (int32_t)i;
}

// ---- reset events of a fused launch -----------------------------------------
// The counter-based reset decisions of a launch's k steps do not depend on the
// state, so they are found, counted, listed and redrawn before the launch by
// dense kernels (one lane per vehicle, then one lane per event) instead of in
// a divergent branch of the step loop.

__device__ __forceinline__ long long launch_t0(const StepArgs& a) {
    return a.d_step ? (*a.d_step + a.t_off) : a.t0;
}

__global__ __launch_bounds__(kResetBlock) void k_ev_mask(StepArgs a) {
    __shared__ int wsum[kResetBlock / 64];
    const long long i = (long long)blockIdx.x * kResetBlock + threadIdx.x;
    unsigned long long bits = 0;
    if (i < a.n) {
        const long long tb0 = launch_t0(a);
        const uint32_t gi = a.index_base + (uint32_t)i;
        long long mblk = -1;
        uint4 mw = make_uint4(0u, 0u, 0u, 0u);
        for (int j = 0; j < a.k; ++j) {
            const long long t = tb0 + j;
            if ((t >> 2) != mblk) {
                mblk = t >> 2;
                mw = mask_block(gi, (uint64_t)mblk, a.key0, a.key1);
            }
            if (mask_hit(mw, t, a.thr)) bits |= 1ull << j;
        }
        a.ev.bits[i] = bits;
    }
    const int c = wave_sum((int)__popcll(bits));
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kResetBlock / 64; ++w) t += wsum[w];
        a.ev.block_counts[blockIdx.x] = t;
    }
}

// ---- mode order of fused launches -------------------------------------------
// One block per segment of kOrderSeg vehicles.  Each piece of the segment that
// lies in one group is partitioned stably by mode bucket (0, 1, 2, other):
// every thread counts its 16 consecutive vehicles per bucket, a block-wide
// exclusive scan of the four counts (16-bit fields of one 64-bit word, each at
// most kOrderSeg) gives its offsets, and it writes its vehicles there in index
// order.
__global__ __launch_bounds__(kOrderBlock) void k_mode_order(OrderArgs a) {
    constexpr int PER = kOrderSeg / kOrderBlock;
    constexpr int NW = kOrderBlock / 64;
    __shared__ long long cut[kOrderPieces + 1];
    __shared__ int ncut;
    __shared__ unsigned long long wsum[NW];
    const long long base = (long long)blockIdx.x * kOrderSeg;
    const long long end = base + kOrderSeg < a.n ? base + kOrderSeg : a.n;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t == 0) {
        // piece boundaries: the group ends inside the segment
        int g = a.n_groups == 1 ? 0 : find_group(a.goff, a.n_groups, base);
        int c = 0;
        cut[c++] = base;
        for (;;) {
            const long long nxt = a.goff[g + 1];
            if (nxt >= end) {
                cut[c++] = end;
                break;
            }
            if (c == kOrderPieces) {
                c = -1;
                break;
            }
            cut[c++] = nxt;
            ++g;
        }
        ncut = c;
    }
    __syncthreads();
    const int nc = ncut;
    if (nc < 0) {
        for (int j = 0; j < PER; ++j) {
            const long long q = base + (long long)t * PER + j;
            if (q < end) a.perm[q] = (int32_t)q;
        }
        return;
    }
    for (int c = 0; c + 1 < nc; ++c) {
        const long long p0 = cut[c], p1 = cut[c + 1];
        const long long q0 = p0 + (long long)t * PER;
        int bk[PER];
        unsigned long long cnt = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const long long q = q0 + j;
            bk[j] = -1;
            if (q < p1) {
                const int m = a.mode[q];
                bk[j] = (m >= 0 && m <= 2) ? m : 3;
                cnt += 1ull << (16 * bk[j]);
            }
        }
        unsigned long long inc = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        unsigned long long pre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (w < wid) pre += wsum[w];
            tot += wsum[w];
        }
        const unsigned long long excl = pre + inc - cnt;
        long long at[4];
        long long start = p0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            at[b] = start + (long long)((excl >> (16 * b)) & 0xffffull);
            start += (long long)((tot >> (16 * b)) & 0xffffull);
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int b = bk[j];
            if (b >= 0) {
                long long pos = at[0];
                if (b == 1) pos = at[1];
                if (b == 2) pos = at[2];
                if (b == 3) pos = at[3];
                a.perm[pos] = (int32_t)(q0 + j);
                if (b == 0) ++at[0];
                if (b == 1) ++at[1];
                if (b == 2) ++at[2];
                if (b == 3) ++at[3];
            }
        }
        __syncthreads();   // wsum is reused by the next piece
    }
}

// Exclusive scan of the per-block event counts in place and their total (one
// block, 64-bit: totals may exceed 2^31).  Each thread sums a contiguous run
// of counts, shuffles within each wavefront and the wavefront totals combine
// the runs (one barrier), and each thread writes its run's offsets.
__global__ __launch_bounds__(1024) void k_ev_scan(StepArgs a) {
    __shared__ long long wtot[1024 / 64];
    const int nblocks = (int)((a.n + kResetBlock - 1) / kResetBlock);
    const int per = (nblocks + 1023) / 1024;
    const int b0 = (int)threadIdx.x * per;
    const int b1 = b0 + per < nblocks ? b0 + per : nblocks;
    // a thread's run (up to RUN counts, 8.4 M vehicles) is loaded into
    // registers at once, so its loads are in flight together; longer runs
    // take the plain loop
    constexpr int RUN = 32;
    long long v[RUN];
    long long run = 0;
    if (per <= RUN) {
#pragma unroll
        for (int j = 0; j < RUN; ++j) v[j] = b0 + j < b1 ? a.ev.block_counts[b0 + j] : 0;
#pragma unroll
        for (int j = 0; j < RUN; ++j) run += v[j];
    } else {
        for (int j = b0; j < b1; ++j) run += a.ev.block_counts[j];
    }
    // inclusive sums of the runs: by shuffles within each wavefront, then
    // the totals of the wavefronts before it (integer sums: exact in any order)
    const int lane = (int)threadIdx.x & 63, wid = (int)threadIdx.x >> 6;
    long long inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    for (int w = 0; w < wid; ++w) inc += wtot[w];
    long long off = inc - run;
    if (per <= RUN) {
#pragma unroll
        for (int j = 0; j < RUN; ++j) {
            if (b0 + j < b1) a.ev.block_counts[b0 + j] = off;
            off += v[j];
        }
    } else {
        for (int j = b0; j < b1; ++j) {
            const long long c = a.ev.block_counts[j];
            a.ev.block_counts[j] = off;
            off += c;
        }
    }
    if (threadIdx.x == 1023) *a.ev.total = inc;
}

// Per-vehicle first-event index (clamped to cap: events past cap are redrawn
// in the step loop) and the event list in vehicle-major, step-minor order.
__global__ __launch_bounds__(kResetBlock) void k_ev_scatter(StepArgs a) {
    __shared__ int wtot[kResetBlock / 64];
    const long long i = (long long)blockIdx.x * kResetBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long bits = i < a.n ? a.ev.bits[i] : 0ull;
    const int c = __popcll(bits);
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; ++w) before += wtot[w];
    if (i >= a.n) return;
    const long long off = a.ev.block_counts[blockIdx.x] + before + (incl - c);
    a.ev.off[i] = (int32_t)(off < a.ev.cap ? off : a.ev.cap);
    unsigned long long b = bits;
    for (long long e = off; b != 0 && e < a.ev.cap; ++e) {
        const int j = __builtin_ctzll(b);
        b &= b - 1;
        a.ev.list[e] = (i << 6) | j;
    }
}

// One lane per listed event: the redrawn state and goal.
__global__ __launch_bounds__(256) void k_ev_redraw(StepArgs a) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = *a.ev.total;
    if (e >= total || e >= a.ev.cap) return;
    const long long code = a.ev.list[e];
    const long long i = code >> 6;
    const int j = (int)(code & 63);
    float s[13], gx, gy, gz;
    redraw(s, gx, gy, gz, a.index_base + (uint32_t)i, launch_t0(a) + j, a.key0, a.key1, a.lo, a.hi);
    const long long cap = a.ev.cap;
#pragma unroll
    for (int r = 0; r < 13; ++r) a.ev.data[r * cap + e] = s[r];
    a.ev.data[13 * cap + e] = gx;
    a.ev.data[14 * cap + e] = gy;
    a.ev.data[15 * cap + e] = gz;
}

// ---- obstacle poses at environment reset -----------------------------------
// One lane per (environment, obstacle slot).  Position: fraction of the env
// box per axis drawn in [frac_lo, frac_hi]; attitude: Z-Y-X Euler angles in
// [eul_lo, eul_hi]; locked dimensions take the slot's constant.  Uniforms from
// Philox(counter = (env, lo32(t), slot, "OB" | j)), j = 0, 1.
constexpr uint32_t TAG_OBST = 0x4F420000u;

__global__ __launch_bounds__(256) void k_obstacles(ObstArgs a) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.n_env * a.n_obs) return;
    const long long e = idx / a.n_obs;
    const int k = (int)(idx - e * a.n_obs);
    if (a.mask && a.mask[e] == 0) return;
    const float* row = a.slots + (long long)k * 20;
    const uint32_t ge = a.index_base + (uint32_t)e;
    const uint4 w0 = philox(make_uint4(ge, (uint32_t)a.t, (uint32_t)k, TAG_OBST | 0u), a.key0, a.key1);
    const uint4 w1 = philox(make_uint4(ge, (uint32_t)a.t, (uint32_t)k, TAG_OBST | 1u), a.key0, a.key1);
    const float u[6] = {u24(w0.x), u24(w0.y), u24(w0.z), u24(w0.w), u24(w1.x), u24(w1.y)};
    const int bits = (int)row[12];
    float pos[3], ang[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float lo = a.env_lo ? a.env_lo[d * a.ld + e] : a.box_lo[d];
        const float hi = a.env_hi ? a.env_hi[d * a.ld + e] : a.box_hi[d];
        float fr = row[d] + (row[3 + d] - row[d]) * u[d];
        fr = (bits >> d & 1) ? row[13 + d] : fr;
        pos[d] = lo + (hi - lo) * fr;
        const float an = row[6 + d] + (row[9 + d] - row[6 + d]) * u[3 + d];
        ang[d] = (bits >> (3 + d) & 1) ? row[16 + d] : an;
    }
    float sr, cr, sp, cp, sy, cy;
    sincosf(0.5f * ang[0], &sr, &cr);
    sincosf(0.5f * ang[1], &sp, &cp);
    sincosf(0.5f * ang[2], &sy, &cy);
    // qz(yaw) (x) qy(pitch) (x) qx(roll)
    const float q[4] = {cy * cp * cr + sy * sp * sr, cy * cp * sr - sy * sp * cr,
                        cy * sp * cr + sy * cp * sr, sy * cp * cr - cy * sp * sr};
#pragma unroll
    for (int d = 0; d < 3; ++d) a.out[d * a.out_ld + idx] = pos[d];
#pragma unroll
    for (int d = 0; d < 4; ++d) a.out[(3 + d) * a.out_ld + idx] = q[d];
}

const void* obstacles_kernel() { return reinterpret_cast<const void*>(&k_obstacles); }

// ---- goal-reaching task: actions in, observation / reward / done out -------
__global__ __launch_bounds__(256) void k_actions(ActArgs a) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float u = __builtin_amdgcn_fmed3f(a.actions[r * a.act_ld + i], -1.0f, 1.0f);
        a.target[r * a.ld + i] = a.offset[r] + a.scale[r] * u;
    }
    a.mode[i] = (int8_t)a.new_mode;
}

__global__ __launch_bounds__(256) void k_observe(TaskArgs a) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    float s[13];
    bool finite = true;
#pragma unroll
    for (int r = 0; r < 13; ++r) {
        s[r] = a.state[r * a.ld + i];
        finite = finite && isfinite(s[r]);
    }
    const float ex = a.goal[i] - s[0], ey = a.goal[a.goal_ld + i] - s[1], ez = a.goal[2 * a.goal_ld + i] - s[2];
    const float o[13] = {ex, ey, ez, s[3], s[4], s[5], s[6], s[7], s[8], s[9], s[10], s[11], s[12]};
#pragma unroll
    for (int r = 0; r < 13; ++r) a.obs[r * a.obs_ld + i] = finite ? o[r] : 0.0f;
    if (!a.advance) return;
    const float dist = sqrtf(ex * ex + ey * ey + ez * ez);
    const float sp = sqrtf(s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    const float wn = sqrtf(s[10] * s[10] + s[11] * s[11] + s[12] * s[12]);
    const float rew = -dist - a.w_v * sp - a.w_omega * wn + (dist < a.r_goal ? a.bonus : 0.0f);
    const int ep = a.episode[i] + 1;
    const bool done = ep >= a.max_steps || dist > a.r_far || !finite;
    a.reward[i] = finite ? rew : 0.0f;
    a.done[i] = done ? 1 : 0;
    a.episode[i] = done ? 0 : ep;
}

const void* actions_kernel() { return reinterpret_cast<const void*>(&k_actions); }
const void* observe_kernel() { return reinterpret_cast<const void*>(&k_observe); }

// ---- kernel lookup ---------------------------------------------------------
// Kernels with trajectories (mode 4) exist for one vehicle per lane and for
// the quad and mixed rotor classes only.
template <int NR, bool VP, int RST, bool OBS, bool TRK>
static const void* pick_shape(int vpl, bool one) {
    if constexpr (RST != 2) {
        if (one) return reinterpret_cast<const void*>(&k_step<NR, VP, RST, 1, true, OBS, TRK>);
    }
    if constexpr (!TRK) {
        if (vpl == 2) return reinterpret_cast<const void*>(&k_step<NR, VP, RST, 2, false, OBS, TRK>);
    }
    return reinterpret_cast<const void*>(&k_step<NR, VP, RST, 1, false, OBS, TRK>);
}

template <int NR, bool VP, int RST, bool TRK>
static const void* pick_obs(int vpl, bool one, bool obs) {
    return obs ? pick_shape<NR, VP, RST, true, TRK>(vpl, one) : pick_shape<NR, VP, RST, false, TRK>(vpl, one);
}

template <int NR, bool VP, bool TRK>
static const void* pick_rst(int rst, int vpl, bool one, bool obs) {
    if (rst == 2) return pick_obs<NR, VP, 2, TRK>(vpl, one, obs);
    if (rst == 1) return pick_obs<NR, VP, 1, TRK>(vpl, one, obs);
    return pick_obs<NR, VP, 0, TRK>(vpl, one, obs);
}

template <int NR, bool TRK>
static const void* pick_nr(bool vp, int rst, int vpl, bool one, bool obs) {
    return vp ? pick_rst<NR, true, TRK>(rst, vpl, one, obs) : pick_rst<NR, false, TRK>(rst, vpl, one, obs);
}

const void* step_kernel(int nr_class, bool vp, int rst, int vpl, bool one_step, bool obs, bool trk) {
    if (rst == 2 && one_step) return nullptr;
    if (trk) return nr_class == 4 ? pick_nr<4, true>(vp, rst, vpl, one_step, obs)
                                  : pick_nr<0, true>(vp, rst, vpl, one_step, obs);
    switch (nr_class) {
        case 4: return pick_nr<4, false>(vp, rst, vpl, one_step, obs);
        case 6: return pick_nr<6, false>(vp, rst, vpl, one_step, obs);
        case 8: return pick_nr<8, false>(vp, rst, vpl, one_step, obs);
        default: return pick_nr<0, false>(vp, rst, vpl, one_step, obs);
    }
}

const void* step_queue_kernel(int nr_class) {
    switch (nr_class) {
        case 4: return reinterpret_cast<const void*>(&k_step_q<4>);
        case 6: return reinterpret_cast<const void*>(&k_step_q<6>);
        case 8: return reinterpret_cast<const void*>(&k_step_q<8>);
        default: return nullptr;   // one group: its rotor count is 4, 6 or 8
    }
}

size_t step_queue_lds_bytes() { return (size_t)(GSTRIDE + kQueueRows * 64) * sizeof(float); }

const void* fold_kernel() { return reinterpret_cast<const void*>(&k_fold); }
const void* advance_kernel() { return reinterpret_cast<const void*>(&k_advance); }
const void* set_step_kernel() { return reinterpret_cast<const void*>(&k_set_step); }
const void* set_targets_kernel() { return reinterpret_cast<const void*>(&k_set_targets); }
const void* reset_mask_kernel() { return reinterpret_cast<const void*>(&k_reset_mask); }
const void* reset_scan_kernel() { return reinterpret_cast<const void*>(&k_reset_scan); }
const void* reset_scatter_kernel() { return reinterpret_cast<const void*>(&k_reset_scatter); }
const void* clear_slots_kernel() { return reinterpret_cast<const void*>(&k_clear_slots); }
const void* ev_mask_kernel() { return reinterpret_cast<const void*>(&k_ev_mask); }
const void* ev_scan_kernel() { return reinterpret_cast<const void*>(&k_ev_scan); }
const void* ev_scatter_kernel() { return reinterpret_cast<const void*>(&k_ev_scatter); }
const void* ev_redraw_kernel() { return reinterpret_cast<const void*>(&k_ev_redraw); }
const void* mode_order_kernel() { return reinterpret_cast<const void*>(&k_mode_order); }

}  // namespace ag
