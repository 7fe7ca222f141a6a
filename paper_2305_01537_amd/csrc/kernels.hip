// kernels.hip -- the fused shell kernel of the per-plan path and the launch
// shapes of the pass kernels (the theta and phi kernels are in
// kernels_theta.hip and kernels_phi.hip), double FFT filter (arXiv:2305.01537,
// Sec. II.A) for gfx950, FP64.
// The work of a workgroup is done by the workers in line_filter.h, which the
// batched persistent kernel (batch.hip) shares: the same arithmetic per line
// (bit for bit where the compiler contracts multiply-adds the same way in
// both kernels, to rounding otherwise).
#include "line_filter.h"

namespace sphfilt {

// Fused shells and, in the same grid, ring pairs of the other shells: blocks
// [0, shell_groups) run shell_block on `shells`, the rest run phi_block
// (W/N2 ring pairs each) on `rings`; W lanes per workgroup.  The two sets touch different shells,
// so one launch lets the ring-pair workgroups stream while the shell
// workgroups load, filter and store their shells.  MFMA: the shells' theta
// pass as the circulant product (theta_gemm.h).
template <int N, bool ADJ, bool HYB, bool MFMA, int W>
__global__ __launch_bounds__(W) void shell_phi_kernel(
    const double *in, double *out, const ThetaItem *__restrict__ shells,
    const double *__restrict__ ring_c, int n_shells, int shell_groups,
    const PhiItem *__restrict__ rings, int n_rings, const Twiddle *__restrict__ tw,
    const double *__restrict__ eneg, HybridArgs ht, HybridArgs hp)
{
    using S = ShellShape<N, W>;
    constexpr int LINES = W / Split<N>::N2;
    static_assert(S::lds >= LINES * line_stride<Split<N>::N1, Split<N>::N2, HYB>(), "ring-pair scratch");
    __shared__ double lds[S::lds];
    __shared__ double etab[N / 2 + 1];
    __shared__ int flags[LINES];
    __shared__ double gaux[MFMA ? shell_gemm_aux<N>() : 1];
    if ((int)blockIdx.x < shell_groups) {
        const int first = blockIdx.x * S::shells;
        shell_block<N, ADJ, HYB, MFMA, W>(in, out, shells + first, ring_c + (size_t)first * S::lines,
                                       min(S::shells, n_shells - first), tw, eneg, lds, etab,
                                       flags, ht, hp, threadIdx.x, gaux);
    } else {
        const int first = ((int)blockIdx.x - shell_groups) * LINES;
        phi_block<N, LINES, HYB>(in, out, rings + first, min(LINES, n_rings - first), N / 2, tw,
                                 eneg, lds, etab, flags, hp, threadIdx.x);
    }
}

// The theta pass alone as the circulant product, on grids with n_phi =
// 2 n_theta = N in {32, 64}: each workgroup stages S = ShellShape<N>::shells
// whole shells in LDS (contiguous loads), forms their circulants, multiplies
// on the matrix cores and stores the results straight from the accumulators
// (each store instruction covers 16 consecutive doubles of 4 rows).  Items
// are active (non-identity) shells of plain kinds.
template <int N>
__global__ __launch_bounds__(256) void theta_gemm_kernel(const double *in, double *out,
                                                         const ThetaItem *__restrict__ items,
                                                         int n_items, const Twiddle *__restrict__ tw,
                                                         const double *__restrict__ eneg)
{
    using S = ShellShape<N>;
    constexpr int K = N / 2, SH = S::shells;
    constexpr size_t shell_pts = (size_t)N * N / 2;
    __shared__ double lds[S::lds];
    __shared__ double etab[N / 2 + 1];
    __shared__ double gaux[shell_gemm_aux<N>()];
    const int lane = threadIdx.x;
    const int first = blockIdx.x * SH;
    const int n_valid = min(SH, n_items - first);
    const ThetaItem *it = items + first;
    stage_exp_table<N>(etab, eneg, lane);
    const int us = lane / S::lanes;
    const bool valid_s = us < n_valid;
    const size_t base_s = valid_s ? (size_t)it[us].shell * shell_pts : 0;
    cplx v[Split<N>::N1];
    shell_stage<N, true>(in, out, lds + us * S::stride, v, base_s, valid_s, lane % S::lanes);
    __syncthreads();
    double *fq = gaux, *cosd = gaux + SH * (N / 2 + 1), *cvec = cosd + N;
    shell_circulants<N, SH>(it, n_valid, tw, etab, fq, cosd, cvec, lane);
    auto sign = [&](int sh) { return (it[sh].flags & kFlagOddParity) ? -1.0 : 1.0; };
    dv4 acc[gemm_tiles_per_wave<N, SH>()];
    shell_gemm<N, SH>(cvec, n_valid, lane, acc, [&](int sh, int m, int k, bool first_half) {
        const double *sb = lds + sh * S::stride;
        return first_half ? sb[m * S::row + k] : sign(sh) * sb[(N - 1 - m) * S::row + K + k];
    });
    shell_gemm_results<N, SH>(acc, n_valid, lane, [&](int sh, int n, int k, double y) {
        double *dst = out + (size_t)it[sh].shell * shell_pts;
        if (n < N / 2)
            st_stream<SPHFILT_NT_STORE_THETA != 0>(dst + (size_t)n * N + k, y);
        else
            st_stream<SPHFILT_NT_STORE_THETA != 0>(dst + (size_t)(N - 1 - n) * N + K + k, sign(sh) * y);
    });
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
int lanes_per_line(int n_line)
{
    switch (n_line) {
    case 32: return Split<32>::N2;
    case 48: return Split<48>::N2;
    case 64: return Split<64>::N2;
    case 80: return Split<80>::N2;
    case 96: return Split<96>::N2;
    case 128: return Split<128>::N2;
    case 160: return Split<160>::N2;
    case 192: return Split<192>::N2;
    case 256: return Split<256>::N2;
    default: return 0;
    }
}

int ilog2_int(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

int theta_lines_per_group(int n_line)
{
    return lanes_per_line(n_line) ? 256 / lanes_per_line(n_line) : 0;
}

int default_theta_cols(int n_line, int n_phi)
{
    // the widest power-of-two tile within the workgroup's lines and n_phi/4
    // whose pairs of sub-tiles divide the n_phi/2 meridian pairs
    const int c = theta_lines_per_group(n_line);
    int cols = 4;
    while (cols * 2 <= c && cols * 2 <= n_phi / 4) cols *= 2;
    while (cols > 4 && (n_phi / 2) % (2 * cols) != 0) cols /= 2;
    return cols;
}

int default_phi_lines(int n_line)
{
    return lanes_per_line(n_line) ? 256 / lanes_per_line(n_line) : 0;
}

bool theta_shape_ok(int n_line, int cols, int n_phi)
{
    const int c = theta_lines_per_group(n_line);
    return c > 0 && (cols == 4 || cols == 8 || cols == 16 || cols == 32 || cols == 64) && cols <= c &&
           (n_phi / 2) % (2 * cols) == 0;
}

bool phi_shape_ok(int n_line, int lines)
{
    const int l = lanes_per_line(n_line);
    return l > 0 && (lines == 4 || lines == 8 || lines == 16 || lines == 32 || lines == 64) &&
           l * lines <= 256 && l * lines >= 16;
}

// ---------------------------------------------------------------------------
// fused shell launcher
// ---------------------------------------------------------------------------
bool shell_fusable(int n_theta, int n_phi)
{
    return n_phi == 2 * n_theta && (n_phi == 32 || n_phi == 64 || n_phi == 128);
}

int shells_per_group(int n_phi)
{
    switch (n_phi) {
    case 32: return ShellShape<32>::shells;
    case 64: return ShellShape<64>::shells;
    case 128: return ShellShape<128>::shells;
    default: return 0;
    }
}


// Lanes per workgroup of the fused launch: 128 for plain kinds at N = 32 and
// 64 (dense fused filter 2-7 % faster: fewer waves per barrier, and the
// halved staging LDS lets twice as many workgroups share a CU), 256 for
// N = 128 (one shell takes 256 lanes), for hybrid fields (their instance
// needs more registers at 128 lanes) and for the circulant variant.
template <int N, bool ADJ, bool HYB, bool MFMA>
static hipError_t shell_phi_launch(const double *in, double *out, const ThetaItem *shells,
                                   const double *ring_c, int n_shells, const PhiItem *rings,
                                   int n_rings, const Twiddle *tw, const double *eneg,
                                   const HybridArgs &ht, const HybridArgs &hp, hipStream_t s)
{
    constexpr int W = N <= 64 && !MFMA && !HYB ? 128 : 256;
    constexpr int LINES = W / Split<N>::N2;
    const int groups = (n_shells + ShellShape<N, W>::shells - 1) / ShellShape<N, W>::shells;
    const dim3 grid((unsigned)(groups + (n_rings + LINES - 1) / LINES)), block(W);
    shell_phi_kernel<N, ADJ, HYB, MFMA, W><<<grid, block, 0, s>>>(in, out, shells, ring_c, n_shells,
                                                                  groups, rings, n_rings, tw, eneg,
                                                                  ht, hp);
    return hipGetLastError();
}

template <int N, bool MFMA>
static hipError_t shell_phi_go(bool adjoint, const double *in, double *out,
                               const ThetaItem *shells, const double *ring_c, int n_shells,
                               const PhiItem *rings, int n_rings, const Twiddle *tw,
                               const double *eneg, const HybridArgs &ht, const HybridArgs &hp,
                               hipStream_t s)
{
    const bool hyb = ht.present != 0;
#define SPHFILT_SHELL_PHI(A, H)                                                                    \
    return shell_phi_launch<N, A, H, MFMA && !H>(in, out, shells, ring_c, n_shells, rings, n_rings, \
                                                 tw, eneg, ht, hp, s)
    if (adjoint) {
        if (hyb) SPHFILT_SHELL_PHI(true, true); else SPHFILT_SHELL_PHI(true, false);
    } else {
        if (hyb) SPHFILT_SHELL_PHI(false, true); else SPHFILT_SHELL_PHI(false, false);
    }
#undef SPHFILT_SHELL_PHI
}

bool theta_gemm_ok(int n_theta, int n_phi)
{
    return n_phi == 2 * n_theta && (n_phi == 32 || n_phi == 64);
}

hipError_t launch_shell_phi(bool adjoint, int n_theta, int n_phi, const double *in, double *out,
                            const ThetaItem *shells, const double *ring_c, int n_shells,
                            const PhiItem *rings, int n_rings, const Twiddle *tw,
                            const double *eneg, const HybridArgs &ht, const HybridArgs &hp,
                            hipStream_t s, bool mfma)
{
    if (n_shells < 0 || n_rings < 0 || !shell_fusable(n_theta, n_phi)) return hipErrorInvalidValue;
    if (mfma && (!theta_gemm_ok(n_theta, n_phi) || ht.present)) return hipErrorInvalidValue;
    if (n_shells + n_rings == 0) return hipSuccess;
    switch (n_phi) {
    case 32:
        return mfma ? shell_phi_go<32, true>(adjoint, in, out, shells, ring_c, n_shells, rings, n_rings, tw, eneg, ht, hp, s)
                    : shell_phi_go<32, false>(adjoint, in, out, shells, ring_c, n_shells, rings, n_rings, tw, eneg, ht, hp, s);
    case 64:
        return mfma ? shell_phi_go<64, true>(adjoint, in, out, shells, ring_c, n_shells, rings, n_rings, tw, eneg, ht, hp, s)
                    : shell_phi_go<64, false>(adjoint, in, out, shells, ring_c, n_shells, rings, n_rings, tw, eneg, ht, hp, s);
    case 128: return shell_phi_go<128, false>(adjoint, in, out, shells, ring_c, n_shells, rings, n_rings, tw, eneg, ht, hp, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_theta_gemm(int n_theta, int n_phi, const double *in, double *out,
                             const ThetaItem *items, int n_items, const Twiddle *tw,
                             const double *eneg, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (!theta_gemm_ok(n_theta, n_phi)) return hipErrorInvalidValue;
    if (n_phi == 32) {
        const unsigned g = (unsigned)((n_items + ShellShape<32>::shells - 1) / ShellShape<32>::shells);
        theta_gemm_kernel<32><<<g, 256, 0, s>>>(in, out, items, n_items, tw, eneg);
    } else {
        const unsigned g = (unsigned)((n_items + ShellShape<64>::shells - 1) / ShellShape<64>::shells);
        theta_gemm_kernel<64><<<g, 256, 0, s>>>(in, out, items, n_items, tw, eneg);
    }
    return hipGetLastError();
}

}  // namespace sphfilt
