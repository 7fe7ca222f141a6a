// batch_hybrid.hip -- the batch kernel instance HYB = true, MIXED = false (its own
// translation unit, so that the instances compile in parallel).
#include "batch_kernels.h"

namespace sphfilt {

hipError_t launch_batch_hybrid(int grid, const BatchArgs &a, hipStream_t s)
{
    return launch_batch_instance<true, false>(grid, a, s);
}

int blocks_per_cu_hybrid() { return batch_instance_blocks_per_cu<true, false>(); }

}  // namespace sphfilt
