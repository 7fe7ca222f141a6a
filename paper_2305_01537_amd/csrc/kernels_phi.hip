// kernels_phi.hip -- per-plan phi-pass kernels
// of the double FFT filter (arXiv:2305.01537, Sec. II.A) for gfx950, FP64: one
// launch per pass over a plan's item list.  The work of a workgroup is done by
// the workers in line_filter.h, which the batched kernel shares.
#include "line_filter.h"

namespace sphfilt {

// phi-pass: workgroup b handles ring pairs [b * LINES, b * LINES + LINES).
template <int N, int LINES, bool HYB>
__global__ __launch_bounds__(LINES * Split<N>::N2) __attribute__((amdgpu_waves_per_eu(pass_waves<N, LINES, HYB>()))) void phi_kernel(
    const double *in, double *out, const PhiItem *__restrict__ items, int n_items, int n_theta,
    const Twiddle *__restrict__ tw, const double *__restrict__ eneg, HybridArgs h)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    __shared__ double lds[LINES * line_stride<N1, N2, HYB>()];
    __shared__ double etab[N / 2 + 1];
    __shared__ int flags[LINES];
    const int first = blockIdx.x * LINES;
    phi_block<N, LINES, HYB>(in, out, items + first, min(LINES, n_items - first), n_theta, tw, eneg,
                        lds, etab, flags, h, threadIdx.x);
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
template <int N, int LINES>
static hipError_t phi_go(const double *in, double *out, const PhiItem *items, int n_items,
                         int n_theta, const Twiddle *tw, const double *eneg, const HybridArgs &h,
                         hipStream_t s)
{
    if constexpr (LINES * Split<N>::N2 > 256 || LINES * Split<N>::N2 < 16) {
        return hipErrorInvalidValue;
    } else {
        const dim3 grid((unsigned)((n_items + LINES - 1) / LINES)), block(LINES * Split<N>::N2);
        if (h.present)
            phi_kernel<N, LINES, true><<<grid, block, 0, s>>>(in, out, items, n_items, n_theta, tw,
                                                              eneg, h);
        else
            phi_kernel<N, LINES, false><<<grid, block, 0, s>>>(in, out, items, n_items, n_theta, tw,
                                                               eneg, h);
        return hipGetLastError();
    }
}

template <int N>
static hipError_t phi_lines(int lines, const double *in, double *out, const PhiItem *items,
                            int n_items, int n_theta, const Twiddle *tw, const double *eneg,
                            const HybridArgs &h, hipStream_t s)
{
    switch (lines) {
    case 4: return phi_go<N, 4>(in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 8: return phi_go<N, 8>(in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 16: return phi_go<N, 16>(in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 32: return phi_go<N, 32>(in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 64: return phi_go<N, 64>(in, out, items, n_items, n_theta, tw, eneg, h, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_phi(int n_line, int lines, const double *in, double *out, const PhiItem *items,
                      int n_items, int n_theta, const Twiddle *tw, const double *eneg,
                      const HybridArgs &h, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (!phi_shape_ok(n_line, lines)) return hipErrorInvalidValue;
    switch (n_line) {
    case 32: return phi_lines<32>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 48: return phi_lines<48>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 64: return phi_lines<64>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 80: return phi_lines<80>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 96: return phi_lines<96>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 128: return phi_lines<128>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 160: return phi_lines<160>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 192: return phi_lines<192>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    case 256: return phi_lines<256>(lines, in, out, items, n_items, n_theta, tw, eneg, h, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sphfilt
