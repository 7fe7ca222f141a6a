// batch_mixed.hip -- the batch kernel instance HYB = false, MIXED = true (its own
// translation unit, so that the instances compile in parallel).
#include "batch_kernels.h"

namespace sphfilt {

hipError_t launch_batch_mixed(int grid, const BatchArgs &a, hipStream_t s)
{
    return launch_batch_instance<false, true>(grid, a, s);
}

int blocks_per_cu_mixed() { return batch_instance_blocks_per_cu<false, true>(); }

}  // namespace sphfilt
