// batch.hip -- host-side launchers of the batched filter's kernels: the
// counter-reset kernel and the dispatch to the kernel instance of a batch
// (the instances live in batch_plain.hip, batch_hybrid.hip, batch_mixed.hip
// and batch_mixed_hybrid.hip; their code in batch_kernels.h).
#include "batch_internal.h"

namespace sphfilt {

// Zero the shell counters, the ticket counters and the error word (a kernel,
// not a memset, so that it can sit in a captured graph).
__global__ __launch_bounds__(256) void batch_reset_kernel(int *counters, int n_counters,
                                                          int *tickets, int n_tickets, int *error)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_counters; i += gridDim.x * blockDim.x)
        counters[i] = 0;
    if (blockIdx.x == 0) {
        if ((int)threadIdx.x < n_tickets) tickets[threadIdx.x] = 0;
        if (threadIdx.x == 0) *error = 0;
    }
}

hipError_t launch_batch_reset(int *counters, int n_counters, int *tickets, int n_tickets,
                              int *error, hipStream_t s)
{
    int grid = (n_counters + 255) / 256;
    if (grid < 1) grid = 1;
    if (grid > 256) grid = 256;
    batch_reset_kernel<<<grid, 256, 0, s>>>(counters, n_counters, tickets, n_tickets, error);
    return hipGetLastError();
}

hipError_t launch_batch(int grid, const BatchWork *work, int n_work, const BatchPatchDev *patches,
                        const double *const *ins, double *const *outs, const ThetaItem *th,
                        const PhiItem *ph, const double *fc, const int *shells, int *counters,
                        const int *need, int *ticket, int *error, const double *eneg, int use_deps,
                        int spin_limit, int need_bias, int variant, hipStream_t s)
{
    if (n_work <= 0) return hipSuccess;
    const BatchArgs a{work, n_work, patches, ins, outs, th, ph, fc, shells, counters,
                      need, ticket, error, eneg, use_deps, spin_limit, need_bias};
    switch (variant & 3) {
    case 0: return launch_batch_plain(grid, a, s);
    case kBatchHybrid: return launch_batch_hybrid(grid, a, s);
    case kBatchMixedRadix: return launch_batch_mixed(grid, a, s);
    default: return launch_batch_mixed_hybrid(grid, a, s);
    }
}

int batch_blocks_per_cu(int variant)
{
    switch (variant & 3) {
    case 0: return blocks_per_cu_plain();
    case kBatchHybrid: return blocks_per_cu_hybrid();
    case kBatchMixedRadix: return blocks_per_cu_mixed();
    default: return blocks_per_cu_mixed_hybrid();
    }
}

}  // namespace sphfilt
