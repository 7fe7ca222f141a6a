// batch_kernels.h -- device side of the batched filter: one kernel launch that filters many uneven spherical patches
// (each with its own grid, fields, parities and cutoffs).
//
// The host flattens every patch's work into one list of work items: first-pass
// items (theta tiles for the forward filter, ring-pair groups for the
// adjoint), then second-pass items.  Workgroups take items in list order from
// an atomic ticket counter, so an item is only ever held by a running
// workgroup.  Two launch forms share the item code: a persistent grid whose
// workgroups loop over tickets, and a one-shot grid with one workgroup per
// item.  A second-pass item of a shell must not start before every
// first-pass item that writes that shell has finished: first-pass items bump
// one counter per shell they wrote (after a device-scope release), and
// second-pass items wait until the counters of the shells they touch reach
// the host-computed totals.  Every awaited item holds a smaller ticket than the
// waiter and never waits itself, so the wait always ends; a bounded spin
// additionally turns a logic error into a flagged error instead of a hang.
//
// The per-line work is done by the same workers as the per-plan kernels
// (line_filter.h).  Patches whose shells fit in LDS (n_phi = 2 n_theta <=
// 128) run their theta-filtered shells as fused items (both passes, one HBM
// round trip, as a plan does) and the rings of their other shells in the
// first pass: such a patch has no second-pass work.
#pragma once
#include "batch_internal.h"
#include "line_filter.h"

namespace sphfilt {

// LDS of the largest worker: the staged shells of the fused worker
// (ShellShape<128>::lds), which also covers the line scratch of every
// theta/phi group, hybrid spectra included; for the instance that also
// takes the lengths that are not powers of two (MIXED) it is the larger of
// that and their line scratch (which fits in it with the current splits).
template <int N, bool HYB>
constexpr int batch_line_lds()
{
    return lines_per_256<N>() * line_stride<Split<N>::N1, Split<N>::N2, HYB>();
}
template <bool HYB, bool MIXED>
constexpr int batch_lds()
{
    constexpr int a = ShellShape<128>::lds;
    constexpr int b = batch_line_lds<96, HYB>() > batch_line_lds<192, HYB>() ? batch_line_lds<96, HYB>()
                                                                          : batch_line_lds<192, HYB>();
    return MIXED && b > a ? b : a;
}
template <int N, bool MIXED>
constexpr bool batch_lds_fits()
{
    return batch_lds<true, MIXED>() >= batch_line_lds<N, true>() &&
           batch_lds<false, MIXED>() >= batch_line_lds<N, false>();
}
static_assert(batch_lds_fits<32, false>() && batch_lds_fits<64, false>() &&
                  batch_lds_fits<128, false>() && batch_lds_fits<256, false>() &&
                  batch_lds_fits<48, true>() && batch_lds_fits<80, true>() &&
                  batch_lds_fits<96, true>() && batch_lds_fits<160, true>() &&
                  batch_lds_fits<192, true>(),
              "batch LDS holds every worker's line scratch");
// Waves per SIMD the instances ask for (each then gets at most 256
// registers).  One-shot: two.  Persistent: two for the plain forms, one for
// the hybrid forms (about 270 registers: at two waves they would spill).
template <bool HYB, bool MIXED>
constexpr int oneshot_waves() { return 2; }
template <bool HYB, bool MIXED>
constexpr int persistent_waves() { return HYB ? 1 : 2; }

// Hybrid lines in a batch decide from their data; decisions are not recorded.
__device__ __forceinline__ HybridArgs batch_hybrid(const BatchPatchDev &pd)
{
    return HybridArgs{pd.det_eps, pd.det_threshold, nullptr, 0, pd.hybrid};
}

// A theta item runs `count` consecutive meridian tiles of its shells, a phi
// item its ring pairs in rounds of one workgroup's worth (the schedule's
// tiles and ring groups per item; the loops are workgroup-uniform, and each
// worker starts with a barrier before it touches LDS).
// The lane index goes through an opaque move at every round, so that the
// per-lane index math of a round is recomputed rather than kept live across
// rounds (which would raise the kernel's register count).
__device__ __forceinline__ int opaque_lane(int lane)
{
    unsigned v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "v"((unsigned)lane));
    return (int)v;
}

template <int N, bool HYB>
__device__ __forceinline__ void theta_item(const BatchWork &w, const BatchPatchDev &pd,
                                           const double *src, double *dst,
                                           const ThetaItem *th, const double *eneg, double *lds,
                                           double *etab, int *flags, int lane)
{
    for (int k = 0; k < w.count; ++k)
        theta_block<N, lines_per_256<N>(), HYB>(src, dst, th + w.first, w.n_valid, pd.cp_log2,
                                               w.tile + k, pd.n_theta, pd.n_phi, pd.tw_theta, eneg,
                                               lds, etab, flags, batch_hybrid(pd), opaque_lane(lane));
}

template <int N, bool HYB>
__device__ __forceinline__ void phi_item(const BatchWork &w, const BatchPatchDev &pd,
                                         const double *src, double *dst, const PhiItem *ph,
                                         const double *eneg, double *lds, double *etab, int *flags,
                                         int lane)
{
    constexpr int L = lines_per_256<N>();
    for (int g = 0; g < w.n_valid; g += L)
        phi_block<N, L, HYB>(src, dst, ph + w.first + g, min(L, w.n_valid - g), pd.n_theta,
                             pd.tw_phi, eneg, lds, etab, flags, batch_hybrid(pd), opaque_lane(lane));
}

template <int N, bool HYB>
__device__ __forceinline__ void fused_item(const BatchWork &w, const BatchPatchDev &pd,
                                           const double *src, double *dst, const ThetaItem *th,
                                           const double *fc, const double *eneg, double *lds,
                                           double *etab, int *flags, int lane)
{
    const HybridArgs h = batch_hybrid(pd);
    if (w.tile)
        shell_block<N, true, HYB>(src, dst, th + w.first, fc + w.aux, w.n_valid, pd.tw_phi, eneg,
                                  lds, etab, flags, h, h, lane);
    else
        shell_block<N, false, HYB>(src, dst, th + w.first, fc + w.aux, w.n_valid, pd.tw_phi, eneg,
                                   lds, etab, flags, h, h, lane);
}

// One work item k (workgroup-uniform): wait for its shells (second pass),
// filter, signal its shells (first pass).
// gave_up: a workgroup-shared word for the outcome of the wait.
template <bool HYB, bool MIXED>
__device__ __forceinline__ void run_item(const BatchArgs &a, int k, int lane, double *lds,
                                         double *etab, int *flags, int *gave_up)
{
    const BatchWork w = a.work[k];
    const BatchPatchDev pd = a.patches[w.patch];

    if (a.use_deps && w.second) {
        // wait until every first-pass item writing these shells is done:
        // relaxed polling, then one device-scope acquire.  If the bounded
        // spin gives up, the error word is set and the item is skipped (its
        // output is left as the first pass wrote it).
        if (lane == 0) {
            int late = 0;
            for (int i = 0; i < w.n_shells && !late; ++i) {
                const int s = a.shells[w.shell_off + i];
                const int target = a.need[s] + a.need_bias;
                int spins = 0;
                while (__hip_atomic_load(a.counters + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       target) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++spins > a.spin_limit) {
                        atomicOr(a.error, 1);
                        late = 1;
                        break;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            *gave_up = late;
        }
        __syncthreads();
        if (*gave_up) return;       // workgroup-uniform
    }

    const double *src = w.second ? a.outs[w.patch] : a.ins[w.patch];
    double *dst = a.outs[w.patch];
    if (w.pass == 0) {
        switch (pd.n_line) {
        case 32: theta_item<32, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
        case 64: theta_item<64, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
        case 128: theta_item<128, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
        default:
            if constexpr (MIXED) {
                switch (pd.n_line) {
                case 48: theta_item<48, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
                case 80: theta_item<80, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
                case 96: theta_item<96, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
                case 160: theta_item<160, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
                case 192: theta_item<192, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
                default: theta_item<256, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane); break;
                }
            } else {
                theta_item<256, HYB>(w, pd, src, dst, a.th, a.eneg, lds, etab, flags, lane);
            }
            break;
        }
    } else if (w.pass == 2) {
        switch (pd.n_phi) {
        case 32: fused_item<32, HYB>(w, pd, src, dst, a.th, a.fc, a.eneg, lds, etab, flags, lane); break;
        case 64: fused_item<64, HYB>(w, pd, src, dst, a.th, a.fc, a.eneg, lds, etab, flags, lane); break;
        default: fused_item<128, HYB>(w, pd, src, dst, a.th, a.fc, a.eneg, lds, etab, flags, lane); break;
        }
    } else {
        switch (pd.n_phi) {
        case 32: phi_item<32, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
        case 64: phi_item<64, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
        case 128: phi_item<128, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
        default:
            if constexpr (MIXED) {
                switch (pd.n_phi) {
                case 48: phi_item<48, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
                case 80: phi_item<80, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
                case 96: phi_item<96, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
                case 160: phi_item<160, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
                case 192: phi_item<192, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
                default: phi_item<256, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane); break;
                }
            } else {
                phi_item<256, HYB>(w, pd, src, dst, a.ph, a.eneg, lds, etab, flags, lane);
            }
            break;
        }
    }

    if (a.use_deps && !w.second && w.n_shells > 0 && !a.defer) {
        // Every wave waits until its own stores have reached the L2; one lane
        // then makes the L2 contents visible device-wide with a single
        // device-scope release (it acts on the whole cache) and bumps the
        // counters.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (lane == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (int i = 0; i < w.n_shells; ++i)
                __hip_atomic_fetch_add(a.counters + a.shells[w.shell_off + i], 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Deferred signals of the persistent one-kernel schedule: a workgroup keeps
// the first-pass items it finished in `pending` (LDS) and signals them all
// with one device-scope release when the list is full, before it waits on a
// second-pass item, and when it runs out of tickets.  A workgroup never waits
// while holding unsignalled items, so every wait still ends.
constexpr int kPendingItems = 32;

__device__ __forceinline__ void flush_pending(const BatchArgs &a, int *pending, int *n_pending,
                                              int lane)
{
    const int n = *n_pending;
    if (n == 0) return;                         // workgroup-uniform (read after a barrier)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (lane < 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        for (int i = 0; i < n; ++i) {
            const BatchWork &w = a.work[pending[i]];
            for (int j = lane; j < w.n_shells; j += 64)
                __hip_atomic_fetch_add(a.counters + a.shells[w.shell_off + j], 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (lane == 0) *n_pending = 0;
    __syncthreads();
}

// Take the next `count` tickets (workgroup-uniform); returns the first.
__device__ __forceinline__ int next_ticket(int *ticket, int *cur, int count = 1)
{
    if (threadIdx.x == 0) *cur = atomicAdd(ticket, count);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(*cur);
    __syncthreads();
    return k;
}

// Tickets a persistent workgroup takes at once: every workgroup of the grid
// takes from one counter, so each atomic queues behind the others' (the
// counter serialises them); runs of up to kTicketRun items cut their number,
// shrinking to single items for the last 2 x grid items so that the
// workgroups still finish together.  `seen`: the last ticket value this
// workgroup saw.
constexpr int kTicketRun = 8;

__device__ __forceinline__ int ticket_run(int seen, int n_work)
{
    const int left = n_work - seen, per = left / (2 * (int)gridDim.x);
    return per < 1 ? 1 : per > kTicketRun ? kTicketRun : per;
}

// One-shot form: the grid has one workgroup per item.  With waits between
// items a workgroup takes a ticket (so that every awaited item is held by a
// running workgroup); without, it runs item blockIdx.x and saves the atomic.
// MIXED: the instance that also takes lines of 48, 80, 96, 160 and 192 points,
// launched only for batches that have such a patch, so that the power-of-two
// instance keeps its code and register allocation.
template <bool HYB, bool MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(oneshot_waves<HYB, MIXED>()))) void batch_kernel_oneshot(BatchArgs a)
{
    __shared__ double lds[batch_lds<HYB, MIXED>()];
    __shared__ double etab[129];
    __shared__ int flags[64];
    __shared__ int cur, gave_up;
    const int k = a.use_deps ? next_ticket(a.ticket, &cur) : (int)blockIdx.x;
    if (k < a.n_work) run_item<HYB, MIXED>(a, k, threadIdx.x, lds, etab, flags, &gave_up);
}

// Persistent form: a fixed grid; each workgroup takes tickets until the list
// is exhausted.  The lane index is re-read through an opaque move every item
// so that per-lane index math is recomputed rather than kept live across
// items (it would otherwise not fit in 256 registers).
template <bool HYB, bool MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(persistent_waves<HYB, MIXED>()))) void batch_kernel_persistent(
    BatchArgs a)
{
    __shared__ double lds[batch_lds<HYB, MIXED>()];
    __shared__ double etab[129];
    __shared__ int flags[64];
    __shared__ int cur, gave_up;
    __shared__ int pending[kPendingItems], n_pending;
    if (threadIdx.x == 0) n_pending = 0;
    int seen = 0;
    for (;;) {
        const int run = ticket_run(seen, a.n_work);
        const int first = next_ticket(a.ticket, &cur, run);
        if (first >= a.n_work) break;
        seen = first + run;
        const int last = min(seen, a.n_work);
        // Items of a run go in ticket order: a run holds only tickets above
        // those of runs taken before it, and waits point to lower tickets,
        // so every chain of waits still ends.
        for (int k = first; k < last; ++k) {
            unsigned lane;
            asm volatile("v_mov_b32 %0, %1" : "=v"(lane) : "v"((unsigned)threadIdx.x));
            if (a.defer) {
                // signal what this workgroup finished before it may wait
                const BatchWork &w = a.work[k];
                if (w.second || n_pending == kPendingItems) flush_pending(a, pending, &n_pending, (int)lane);
            }
            run_item<HYB, MIXED>(a, k, (int)lane, lds, etab, flags, &gave_up);
            if (a.defer && !a.work[k].second && a.work[k].n_shells > 0) {
                __syncthreads();
                if (lane == 0) pending[n_pending++] = k;
                __syncthreads();
            }
        }
    }
    if (a.defer) flush_pending(a, pending, &n_pending, (int)threadIdx.x);
}

// Launch instance <HYB, MIXED>: grid > 0 persistent workgroups, else one
// workgroup per item.
template <bool HYB, bool MIXED>
hipError_t launch_batch_instance(int grid, const BatchArgs &a, hipStream_t s)
{
    if (grid > 0)
        batch_kernel_persistent<HYB, MIXED><<<(unsigned)grid, 256, 0, s>>>(a);
    else
        batch_kernel_oneshot<HYB, MIXED><<<(unsigned)a.n_work, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <bool HYB, bool MIXED>
int batch_instance_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel_persistent<HYB, MIXED>, 256, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace sphfilt
