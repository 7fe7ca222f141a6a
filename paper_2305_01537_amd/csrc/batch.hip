// batch.hip -- host-side launchers of the batched filter's kernels: the
// counter-reset kernel and the dispatch to the kernel instance of a batch
// (the instances live in batch_plain.hip, batch_hybrid.hip, batch_mixed.hip
// and batch_mixed_hybrid.hip; their code in batch_kernels.h).
#include "batch_internal.h"

#include <mutex>

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
                      need, ticket, error, eneg, use_deps, spin_limit, need_bias,
                      use_deps && grid > 0 ? 1 : 0};
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

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (sphfilt_batch_apply_noalloc):
// a file-scope device array, one copy per device for the life of the process.
// Host code never uses the array's name as an address: its device address is
// looked up once per device with hipGetSymbolAddress and cached.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
unsigned char *scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, unsigned char **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_addr[device]) {
        // the caller has made `device` current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[device] = static_cast<unsigned char *>(p);
    }
    *out = scratch_addr[device];
    return hipSuccess;
}

namespace {
constexpr int kPtrChunk = 64;
struct PtrChunk {
    const double *ins[kPtrChunk];
    double *outs[kPtrChunk];
    int first, n;
};
}  // namespace

__global__ __launch_bounds__(64) void noalloc_pointers_kernel(PtrChunk c, const double **ins,
                                                             double **outs)
{
    const int t = threadIdx.x;
    if (t < c.n) {
        ins[c.first + t] = c.ins[t];
        outs[c.first + t] = c.outs[t];
    }
}

hipError_t noalloc_set_pointers(unsigned char *base, const double *const *ins, double *const *outs,
                                int n, hipStream_t s)
{
    const double **d_ins = reinterpret_cast<const double **>(base + kNoAllocPtrOffset);
    double **d_outs = reinterpret_cast<double **>(base + kNoAllocPtrOffset) + kNoAllocMaxPatches;
    for (int first = 0; first < n; first += kPtrChunk) {
        PtrChunk c{};
        c.first = first;
        c.n = n - first < kPtrChunk ? n - first : kPtrChunk;
        for (int i = 0; i < c.n; ++i) {
            c.ins[i] = ins[first + i];
            c.outs[i] = outs[first + i];
        }
        noalloc_pointers_kernel<<<1, 64, 0, s>>>(c, d_ins, d_outs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sphfilt
