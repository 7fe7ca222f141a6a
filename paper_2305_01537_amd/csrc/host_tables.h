// host_tables.h -- host-side tables shared by plans and batches.
#pragma once
#include "../../include/sphfilt.h"
#include "sphfilt_internal.h"

#include <vector>

namespace sphfilt {

// Item lists of one (n_r x n_theta x n_phi, n_fields) grid.  Items whose mask
// is 1 on every mode come after the others (active prefix, then identity).
// Fused schedule (shell_fusable grids only): theta items [0, n_fused) are the
// shells whose every theta line and ring is filtered, fused_c their ring-pair
// cutoffs (n_theta/2 per shell, j ascending); phi_rest holds the phi items of
// the shells the theta pass leaves alone (active prefix of phi_rest_active
// items, then identity), on every grid; phi_in the active phi items of the
// theta-filtered shells that are not fused.
struct HostTables {
    std::vector<ThetaItem> theta;
    std::vector<PhiItem> phi;
    int theta_active = 0;
    int phi_active = 0;
    int n_fused = 0;
    std::vector<double> fused_c;
    std::vector<PhiItem> phi_rest;
    int phi_rest_active = 0;
    std::vector<PhiItem> phi_in;
    // leading hybrid items of the active prefix of theta, of phi, of the fused
    // shells and of phi_in (hybrid fields come first; a hybrid line is never
    // identity, and the theta-idle shells of phi_rest are never hybrid)
    int theta_hyb = 0, phi_hyb = 0, fused_hyb = 0, phi_in_hyb = 0;
};

bool fault(const char *what);
bool supported_line(int n);
// exp(-2 pi i j / N) for j in [0, N)
std::vector<Twiddle> twiddles(int N);
// e^{-k} for k in [0, kExpTable)
std::vector<double> exp_table();
int validate(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
             const sphfilt_cutoff *cut);
void build_items(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
                 const sphfilt_cutoff *cut, HostTables *h);
// Detector parameters (defaults for zeros) and whether any field is hybrid.
HybridArgs hybrid_args(const sphfilt_cutoff *cut, int n_fields);
void fill_stats(int n_r, int n_theta, int n_phi, int n_fields, const HostTables &h,
                sphfilt_stats *s);

template <typename T>
int upload(T **dst, const std::vector<T> &src)
{
    const size_t bytes = sizeof(T) * (src.empty() ? 1 : src.size());
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e == hipErrorOutOfMemory) { *dst = nullptr; return SPHFILT_ENOMEM; }
    if (e != hipSuccess) { *dst = nullptr; return SPHFILT_EDEVICE; }
    if (!src.empty() && hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
        return SPHFILT_EDEVICE;
    return SPHFILT_OK;
}

// Make a device current for the duration of one call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace sphfilt
