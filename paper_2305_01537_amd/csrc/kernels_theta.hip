// kernels_theta.hip -- per-plan theta-pass kernels
// of the double FFT filter (arXiv:2305.01537, Sec. II.A) for gfx950, FP64: one
// launch per pass over a plan's item list.  The work of a workgroup is done by
// the workers in line_filter.h, which the batched kernel shares.
#include "line_filter.h"

namespace sphfilt {

// theta-pass: workgroup b handles shell group g = b / tiles (S = C / cp shells
// of the item list) and meridian tile b % tiles.
template <int N, int C, bool HYB>
__global__ __launch_bounds__(C * Split<N>::N2) __attribute__((amdgpu_waves_per_eu(pass_waves<N, C, HYB>()))) void theta_kernel(
    const double *in, double *out, const ThetaItem *__restrict__ items, int n_items, int cp_log2,
    int tiles, int n_theta, int n_phi, const Twiddle *__restrict__ tw,
    const double *__restrict__ eneg, HybridArgs h)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    __shared__ double lds[C * line_stride<N1, N2, HYB>()];
    __shared__ double etab[N / 2 + 1];
    __shared__ int flags[C];
    const int group = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int per_group = C >> cp_log2;
    const int first = group * per_group;
    const int n_valid = min(per_group, n_items - first);
    theta_block<N, C, HYB>(in, out, items + first, n_valid, cp_log2, tile, n_theta, n_phi, tw, eneg,
                      lds, etab, flags, h, threadIdx.x);
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
// Lanes per workgroup of the plan's plain theta kernel.  128 where that
// measured faster on dense grids (theta pass: N = 48, 64 and 96 5-7 %, 160 and
// 192 4 %, 32 1.5 %: half the waves wait at each barrier and the launch drains
// in finer steps), 256 at 80, 128 and 256 (128 lanes: 1.5 %, 10 % and 45 %
// slower).  Where pairs are adjacent (every N but 256) a line's result does
// not depend on the tile width, so both shapes give the same bits.  The
// hybrid-capable instance keeps 256 lanes.
template <int N>
constexpr int theta_plan_lanes()
{
    return N == 80 || N == 128 || N == 256 ? 256 : 128;
}

// One launch of theta_kernel<N, C, HYB> over the items; the tile width is
// `cols`, or the workgroup's C lines where that is smaller.
template <int N, int C, bool HYB>
static hipError_t theta_launch(int cols, const double *in, double *out, const ThetaItem *items,
                               int n_items, int n_theta, int n_phi, const Twiddle *tw,
                               const double *eneg, const HybridArgs &h, hipStream_t s)
{
    const int cw = cols < C ? cols : C;
    const int cp_log2 = ilog2_int(cw);
    const int per_group = C / cw;
    const int tiles = (n_phi / 2) / (2 * cw);
    const int groups = (n_items + per_group - 1) / per_group;
    theta_kernel<N, C, HYB><<<dim3((unsigned)(groups * tiles)), dim3(C * Split<N>::N2), 0, s>>>(
        in, out, items, n_items, cp_log2, tiles, n_theta, n_phi, tw, eneg, h);
    return hipGetLastError();
}

template <int N>
static hipError_t theta_go(int cols, const double *in, double *out, const ThetaItem *items,
                           int n_items, int n_theta, int n_phi, const Twiddle *tw,
                           const double *eneg, const HybridArgs &h, hipStream_t s)
{
    // the hybrid-capable variant only when the plan has hybrid fields: its
    // detector and two-kind mask cost registers the plain filter does not need
    if (h.present)
        return theta_launch<N, lines_per_256<N>(), true>(cols, in, out, items, n_items, n_theta,
                                                         n_phi, tw, eneg, h, s);
    return theta_launch<N, theta_plan_lanes<N>() / Split<N>::N2, false>(
        cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
}

hipError_t launch_theta(int n_line, int cols, const double *in, double *out,
                        const ThetaItem *items, int n_items, int n_theta, int n_phi,
                        const Twiddle *tw, const double *eneg, const HybridArgs &h,
                        hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (!theta_shape_ok(n_line, cols, n_phi) || n_line != 2 * n_theta) return hipErrorInvalidValue;
    switch (n_line) {
    case 32: return theta_go<32>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 48: return theta_go<48>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 64: return theta_go<64>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 80: return theta_go<80>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 96: return theta_go<96>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 128: return theta_go<128>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 160: return theta_go<160>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 192: return theta_go<192>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    case 256: return theta_go<256>(cols, in, out, items, n_items, n_theta, n_phi, tw, eneg, h, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sphfilt
