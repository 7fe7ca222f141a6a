// batch_internal.h -- types shared by the batch host code and the batch
// kernels (batch.hip, batch_kernels.h and its four instance files).
#pragma once
#include "sphfilt_internal.h"

#include <cstdint>

namespace sphfilt {

// One work item of the persistent batch kernel.
//   pass      0: theta group (n_valid shells x one meridian tile);
//             1: phi group (n_valid ring pairs);
//             2: fused shells (n_valid whole shells, both passes; tile = 1
//                for the adjoint order, aux = index of the first shell's
//                ring cutoffs in the batch's fused cutoff array).
//   second    0: first pass (reads `in`, writes `out`, signals its shells);
//             1: second pass (works in place on `out`, waits for its shells).
//   first     index of the first item in the batch's concatenated theta or
//             phi item array.
//   shell_off, n_shells
//             the distinct global shell ids this item writes (first pass) or
//             touches (second pass), in the batch's shell list.
//   count     theta: meridian tiles [tile, tile + count) of the same shells;
//             phi: n_valid ring pairs in ceil(n_valid / L) workgroup rounds of
//             L = 256 / lanes-per-line pairs (count is then unused: 1).
struct BatchWork {
    int32_t patch;
    int16_t pass;
    int16_t second;
    int32_t first;
    int16_t n_valid;
    int16_t tile;
    int32_t shell_off;
    int32_t n_shells;
    int32_t aux;
    int32_t count;
};

// Per-patch constants of the batch kernel.
struct BatchPatchDev {
    const Twiddle *tw_theta;
    const Twiddle *tw_phi;
    int32_t n_theta, n_phi;
    int32_t n_line;       // 2 * n_theta
    int32_t cp_log2;      // theta sub-tile width (meridian pairs), log2
    double det_eps, det_threshold;   // hybrid kind: Jameson's detector
    int32_t hybrid;       // some field of the patch is hybrid
    int32_t pad;
};

// Arguments of the batch kernel (see batch_kernels.h).
struct BatchArgs {
    const BatchWork *work;
    int n_work;
    const BatchPatchDev *patches;
    const double *const *ins;
    double *const *outs;
    const ThetaItem *th;
    const PhiItem *ph;
    const double *fc;
    const int *shells;
    int *counters;
    const int *need;
    int *ticket;
    int *error;
    const double *eneg;
    int use_deps;
    int spin_limit;
    int need_bias;        // added to every wait target (0; 1 only to force a give-up in tests)
    int defer;            // persistent one-kernel form: first-pass items signal in batches
};

// The four kernel instances (HYB, MIXED), each in its own translation unit:
// grid > 0 persistent workgroups, else one workgroup per item.
hipError_t launch_batch_plain(int grid, const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_hybrid(int grid, const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_mixed(int grid, const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_mixed_hybrid(int grid, const BatchArgs &a, hipStream_t s);
int blocks_per_cu_plain();
int blocks_per_cu_hybrid();
int blocks_per_cu_mixed();
int blocks_per_cu_mixed_hybrid();

hipError_t launch_batch_reset(int *counters, int n_counters, int *tickets, int n_tickets,
                              int *error, hipStream_t s);
// grid > 0: persistent form with `grid` workgroups; grid <= 0: one workgroup
// per item.
// Kernel instance of a batch: kBatchHybrid when some patch has a hybrid field
// (the detector and mixed-pair mask), kBatchMixedRadix when some patch has lines
// that are not powers of two (48, 80, 96, 160 or 192 points).
constexpr int kBatchHybrid = 1, kBatchMixedRadix = 2;
hipError_t launch_batch(int grid, const BatchWork *work, int n_work, const BatchPatchDev *patches,
                        const double *const *ins, double *const *outs, const ThetaItem *th,
                        const PhiItem *ph, const double *fc, const int *shells, int *counters,
                        const int *need,
                        int *ticket, int *error, const double *eneg, int use_deps, int spin_limit,
                        int need_bias, int variant, hipStream_t s);
// (the persistent form, grid > 0, with use_deps defers its signals; see
// flush_pending in batch_kernels.h)
// Resident 256-lane workgroups of the persistent batch kernel instance
// `variant` per compute unit.
int batch_blocks_per_cu(int variant);

// ---- the allocation-free entry point's device scratch (batch.hip) --------
// One statically allocated array per device holds the batch kernel's
// counters, tickets, error word and the per-call pointer tables:
//   ints [0, 3) tickets, int 3 the error word, then (from byte 256) the
//   input and output pointer tables (kNoAllocMaxPatches pointers each), then
//   kNoAllocMaxShells shell counters.
constexpr int kNoAllocMaxPatches = 1024;
constexpr int kNoAllocMaxShells = 1 << 18;
constexpr size_t kNoAllocPtrOffset = 256;
constexpr size_t kNoAllocCounterOffset = kNoAllocPtrOffset + 2 * sizeof(void *) * kNoAllocMaxPatches;
constexpr size_t kNoAllocScratchBytes = kNoAllocCounterOffset + sizeof(int) * (size_t)kNoAllocMaxShells;
// Device address of the scratch array on the current device (looked up with
// hipGetSymbolAddress on the first call per device, then cached); returns
// hipSuccess or the lookup's error.
hipError_t noalloc_scratch(int device, unsigned char **out);
// Write n pointer pairs into the scratch tables, from index `first`, with
// kernels on stream s (the pointers travel as kernel arguments).
hipError_t noalloc_set_pointers(unsigned char *scratch, const double *const *ins,
                                double *const *outs, int n, hipStream_t s);

}  // namespace sphfilt
