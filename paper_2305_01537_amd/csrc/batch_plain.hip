// batch_plain.hip -- the batch kernel instance HYB = false, MIXED = false (its own
// translation unit, so that the instances compile in parallel).
#include "batch_kernels.h"

namespace sphfilt {

hipError_t launch_batch_plain(int grid, const BatchArgs &a, hipStream_t s)
{
    return launch_batch_instance<false, false>(grid, a, s);
}

int blocks_per_cu_plain() { return batch_instance_blocks_per_cu<false, false>(); }

}  // namespace sphfilt
