// kernels.hip -- theta-pass and phi-pass kernels of the double FFT filter
// (arXiv:2305.01537, Sec. II.B) for gfx950, FP64.
//
// Both passes filter independent real lines of length N: FFT, multiply mode q
// by f(|q|, cutoff), inverse FFT.  Two real lines that share one cutoff are
// packed as the real and imaginary part of one complex line; because the mask
// is real and even in q, the real and imaginary parts of the result are the
// two filtered lines.
//   theta-pass: the line is the extended great circle of meridian pair
//     (k, k + n_phi/2): rows 0..n_theta-1 of meridian k, then, times the
//     parity sign, rows n_theta-1..0 of meridian k + n_phi/2 (the paper's
//     extension across the poles).  The two real lines packed together are
//     meridian pairs k and k + C of one shell (same l_max).  Lanes walk the
//     meridians fastest, so every load and store touches whole 128-byte
//     row segments.
//   phi-pass: the line is a ring; rings j and n_theta-1-j of one shell are
//     packed together (same sin(theta), same m_max).  Lanes walk phi fastest.
// Each line is read from HBM once and written once; the transform, mask and
// inverse happen in registers and LDS in between.
#include "fft_core.h"
#include "sphfilt_internal.h"

#include <cmath>

namespace sphfilt {

// ln(0.9), the Gaussian filter's constant (eq. gaussian_filter).
constexpr double kLog09 = -0.10536051565782630123;

// Field data is streamed exactly once per pass: non-temporal loads and stores
// keep it from displacing the small tables in the caches.
#ifndef SPHFILT_NT
#define SPHFILT_NT 1
#endif
// Minimum waves per SIMD requested from the register allocator (0: compiler's
// choice).  Bounds the VGPR count of the large-N kernels.
#ifndef SPHFILT_WAVES
#define SPHFILT_WAVES 0
#endif
#if SPHFILT_WAVES > 0
#define SPHFILT_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SPHFILT_WAVES)))
#else
#define SPHFILT_OCCUPANCY
#endif

__device__ __forceinline__ double ld_stream(const double *p)
{
#if SPHFILT_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

__device__ __forceinline__ void st_stream(double *p, double v)
{
#if SPHFILT_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Mask of one line, with the inverse transform's 1/N folded in.  v holds
// X[q] at q = t + N2 r + N1 k2 in v[r N2 + k2].
//   exponential (eq. exp_filter): f = 1 for |q| <= c, else exp(-(|q| - c)).
//     With m = floor(c), |q| <= c is |q| <= m, and above the cutoff
//     exp(c - |q|) = exp(c - m - 1) * e^{-(|q| - m - 1)}: one exp per lane and
//     a table of e^{-k}, instead of one exp per mode.
//   sharp: the same with the factor above the cutoff set to 0.
//   Gaussian (eq. gaussian_filter): f = exp(log(0.9) (|q| / (c + 1))^2).
template <int N1, int N2>
__device__ __forceinline__ void apply_mask(cplx (&v)[N1], int t, int kind, double c,
                                           const double *etab)
{
    constexpr int N = N1 * N2;
    constexpr int R = N1 / N2;
    constexpr double inv_n = 1.0 / N;
    if (kind == 1) {
        const double inv = 1.0 / (c + 1.0);
        static_for<0, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            static_for<0, N2>([&](auto kk) {
                constexpr int k2 = decltype(kk)::value;
                const int q = t + N2 * r + N1 * k2;
                const double u = (double)(q <= N / 2 ? q : N - q) * inv;
                const double f = exp(kLog09 * u * u) * inv_n;
                v[r * N2 + k2].re *= f;
                v[r * N2 + k2].im *= f;
            });
        });
    } else {
        const int m = c >= (double)N ? N : (int)floor(c);
        const double g = (kind == 0 ? exp((c - (double)m) - 1.0) : 0.0) * inv_n;
        static_for<0, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            static_for<0, N2>([&](auto kk) {
                constexpr int k2 = decltype(kk)::value;
                const int q = t + N2 * r + N1 * k2;
                const int qhat = q <= N / 2 ? q : N - q;
                const double f = qhat <= m ? inv_n : g * etab[qhat > m ? qhat - m - 1 : 0];
                v[r * N2 + k2].re *= f;
                v[r * N2 + k2].im *= f;
            });
        });
    }
}

// LDS doubles per line: an N1 x (N2 + 1) padded tile plus one double, so that
// consecutive lines start on different banks.
template <int N1, int N2>
constexpr int line_lds() { return N1 * (N2 + 1) + 1; }

// Forward transpose: lane t holds Y[k1][t] in v[k1]; afterwards it holds
// Y[t + N2 r][n2] in v[r * N2 + n2].  Real and imaginary parts go through LDS
// in two rounds to halve the LDS footprint.
template <int N1, int N2>
__device__ __forceinline__ void transpose_fwd(cplx (&v)[N1], int t, double *L)
{
    constexpr int S = N2 + 1;
    static_for<0, 2>([&](auto part) {
        constexpr bool im = decltype(part)::value == 1;
        static_for<0, N1>([&](auto kk) {
            constexpr int k1 = decltype(kk)::value;
            L[k1 * S + t] = im ? v[k1].im : v[k1].re;
        });
        __syncthreads();
        static_for<0, N1 / N2>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            static_for<0, N2>([&](auto nn) {
                constexpr int n2 = decltype(nn)::value;
                const double x = L[(t + N2 * r) * S + n2];
                if constexpr (im) v[r * N2 + n2].im = x; else v[r * N2 + n2].re = x;
            });
        });
        __syncthreads();
    });
}

// Inverse of transpose_fwd.
template <int N1, int N2>
__device__ __forceinline__ void transpose_bwd(cplx (&v)[N1], int t, double *L)
{
    constexpr int S = N2 + 1;
    static_for<0, 2>([&](auto part) {
        constexpr bool im = decltype(part)::value == 1;
        static_for<0, N1 / N2>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            static_for<0, N2>([&](auto nn) {
                constexpr int n2 = decltype(nn)::value;
                L[(t + N2 * r) * S + n2] = im ? v[r * N2 + n2].im : v[r * N2 + n2].re;
            });
        });
        __syncthreads();
        static_for<0, N1>([&](auto kk) {
            constexpr int k1 = decltype(kk)::value;
            const double x = L[k1 * S + t];
            if constexpr (im) v[k1].im = x; else v[k1].re = x;
        });
        __syncthreads();
    });
}

// v[OFF + k] *= w^k (or conj(w)^k with CONJ) for k in [1, K), where
// w^j = tw[j * s].  Powers are formed as w^(4a + b) = w^(4a) * w^b from the
// table entries w^1..w^3 and w^4, w^8, ...: a handful of loads and at most
// one rounding per twiddle.  Needs (K - 1) * s < N.
template <int K, bool CONJ, int OFF, int NV>
__device__ __forceinline__ void twiddle_powers(cplx (&v)[NV], const Twiddle *__restrict__ tw, int s)
{
    cplx lo[4], hi[(K + 3) / 4];
    lo[0] = cplx{1.0, 0.0};
    hi[0] = cplx{1.0, 0.0};
    static_for<1, (K < 4 ? K : 4)>([&](auto bb) {
        constexpr int b = decltype(bb)::value;
        const Twiddle w = tw[b * s];
        lo[b] = cplx{w.re, w.im};
    });
    static_for<1, (K + 3) / 4>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        const Twiddle w = tw[4 * a * s];
        hi[a] = cplx{w.re, w.im};
    });
    static_for<1, K>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        constexpr int a = k / 4, b = k % 4;
        cplx w;
        if constexpr (a == 0) w = lo[b];
        else if constexpr (b == 0) w = hi[a];
        else w = cmul(hi[a], lo[b]);
        v[OFF + k] = CONJ ? cmulc(v[OFF + k], w) : cmul(v[OFF + k], w);
    });
}

// Filter one complex line of length N = N1 * N2 held by N2 lanes (lane t
// holds x[N2 n1 + t] in v[n1]); on return v holds the filtered values at the
// same positions.  Every lane of the workgroup calls this together.
// etab: e^{-k}, k <= N/2, in LDS, written before the first barrier here.
template <int N1, int N2>
__device__ __forceinline__ void filter_line(cplx (&v)[N1], int t, int kind, double c, double *L,
                                            const Twiddle *__restrict__ tw, const double *etab)
{
    constexpr int R = N1 / N2;
    static_assert(N1 % N2 == 0, "lane count must divide the register count");

    // forward: N1-point DFTs over n1, twiddle W_N^{t k1}
    dft_reg<N1, false>(v);
    twiddle_powers<N1, false, 0>(v, tw, t);
    transpose_fwd<N1, N2>(v, t, L);
    // N2-point DFTs over n2: v[r N2 + k2] = X[k1 + N1 k2], k1 = t + N2 r
    static_for<0, R>([&](auto rr) { dft_reg<N2, false, decltype(rr)::value * N2>(v); });

    apply_mask<N1, N2>(v, t, kind, c, etab);

    // inverse: N2-point inverse DFTs, conjugate twiddles W_N^{-n2 k1},
    // transpose back, N1-point inverse DFTs
    static_for<0, R>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        dft_reg<N2, true, r * N2>(v);
        twiddle_powers<N2, true, r * N2>(v, tw, t + N2 * r);
    });
    transpose_bwd<N1, N2>(v, t, L);
    dft_reg<N1, true>(v);
}

// Copy e^{-k}, k in [0, N/2], into the workgroup's LDS table.
template <int N>
__device__ __forceinline__ void stage_exp_table(double *etab, const double *__restrict__ eneg)
{
    for (int i = threadIdx.x; i <= N / 2; i += blockDim.x) etab[i] = eneg[i];
}

template <int N> struct Split;
template <> struct Split<32>  { static constexpr int N1 = 8,  N2 = 4; };
template <> struct Split<64>  { static constexpr int N1 = 8,  N2 = 8; };
template <> struct Split<128> { static constexpr int N1 = 16, N2 = 8; };
template <> struct Split<256> { static constexpr int N1 = 16, N2 = 16; };

// ---------------------------------------------------------------------------
// theta-pass: one workgroup = one tile of 2*C meridian pairs of one shell.
// Lane (p, t), p fastest: complex line p packs meridian pair kr = k0 + p
// (real part) and ki = k0 + C + p (imaginary part).
// ---------------------------------------------------------------------------
template <int N, int C>
__global__ __launch_bounds__(C * Split<N>::N2) SPHFILT_OCCUPANCY void theta_kernel(
    const double *in, double *out, const ThetaItem *__restrict__ items, int tiles_per_shell,
    int n_theta, int n_phi, const Twiddle *__restrict__ tw, const double *__restrict__ eneg)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    __shared__ double lds[C * line_lds<N1, N2>()];
    __shared__ double etab[N / 2 + 1];
    const int p = threadIdx.x % C, t = threadIdx.x / C;
    const int tile = blockIdx.x % tiles_per_shell;
    const ThetaItem it = items[blockIdx.x / tiles_per_shell];
    const bool filtered = !(it.flags & kFlagIdentity);
    if (filtered) stage_exp_table<N>(etab, eneg);
    const size_t base = (size_t)it.shell * (size_t)(n_theta * n_phi);
    const int half = n_phi / 2;
    const int kr = tile * 2 * C + p, ki = kr + C;
    const double s = (it.flags & kFlagOddParity) ? -1.0 : 1.0;
    // Row n1 of the lane block starts at a workgroup-uniform row; the lane adds
    // a small non-negative row offset and its column.  Rows N2 n1 + t of the
    // first half; rows n_theta - N2 (n1 - N1/2 + 1) + (N2 - 1 - t) of the
    // mirrored half, i.e. row 2 n_theta - 1 - (N2 n1 + t).
    const int off_n = t * n_phi;
    const int off_s = (N2 - 1 - t) * n_phi + half;

    cplx v[N1];
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        if constexpr (n1 < N1 / 2) {
            const double *row = in + base + (size_t)(N2 * n1) * n_phi;
            v[n1] = cplx{ld_stream(row + off_n + kr), ld_stream(row + off_n + ki)};
        } else {
            const double *row = in + base + (size_t)(N - N2 * (n1 + 1)) * n_phi;
            v[n1] = cplx{s * ld_stream(row + off_s + kr), s * ld_stream(row + off_s + ki)};
        }
    });
    if (filtered)
        filter_line<N1, N2>(v, t, it.flags & kKindMask, it.c, lds + p * line_lds<N1, N2>(), tw, etab);
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        if constexpr (n1 < N1 / 2) {
            double *row = out + base + (size_t)(N2 * n1) * n_phi;
            st_stream(row + off_n + kr, v[n1].re);
            st_stream(row + off_n + ki, v[n1].im);
        } else {
            double *row = out + base + (size_t)(N - N2 * (n1 + 1)) * n_phi;
            st_stream(row + off_s + kr, s * v[n1].re);
            st_stream(row + off_s + ki, s * v[n1].im);
        }
    });
}

// ---------------------------------------------------------------------------
// phi-pass: one workgroup = LINES ring pairs; lane (p, t), t fastest.
// ---------------------------------------------------------------------------
template <int N, int LINES>
__global__ __launch_bounds__(LINES * Split<N>::N2) SPHFILT_OCCUPANCY void phi_kernel(
    const double *in, double *out, const PhiItem *__restrict__ items, int n_items, int n_theta,
    const Twiddle *__restrict__ tw, const double *__restrict__ eneg)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    __shared__ double lds[LINES * line_lds<N1, N2>()];
    __shared__ double etab[N / 2 + 1];
    const int t = threadIdx.x % N2, p = threadIdx.x / N2;
    const int idx = blockIdx.x * LINES + p;
    const bool valid = idx < n_items;
    PhiItem it{0, kFlagIdentity, 0.0};
    if (valid) it = items[idx];
    const bool active = valid && !(it.flags & kFlagIdentity);
    const int any_active = __syncthreads_or(active);
    if (any_active) stage_exp_table<N>(etab, eneg);

    const int j = it.ring % n_theta;
    const size_t a = (size_t)it.ring * N;
    const size_t b = a + (size_t)(n_theta - 1 - 2 * j) * N;
    cplx v[N1];
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        v[n1] = valid ? cplx{ld_stream(in + a + N2 * n1 + t), ld_stream(in + b + N2 * n1 + t)}
                      : cplx{0.0, 0.0};
    });
    // Identity lines that share a workgroup with filtered ones run through the
    // transform too (the barriers are workgroup-wide) but their result is
    // dropped: they are copied exactly from `in` instead.  Such workgroups
    // only occur out of place, where `in` is not written.
    if (any_active)
        filter_line<N1, N2>(v, t, it.flags & kKindMask, active ? it.c : INFINITY,
                            lds + p * line_lds<N1, N2>(), tw, etab);
    if (valid && (active || !any_active)) {
        static_for<0, N1>([&](auto nn) {
            constexpr int n1 = decltype(nn)::value;
            st_stream(out + a + N2 * n1 + t, v[n1].re);
            st_stream(out + b + N2 * n1 + t, v[n1].im);
        });
    } else if (valid && in != out) {
        static_for<0, N1>([&](auto nn) {
            constexpr int n1 = decltype(nn)::value;
            st_stream(out + a + N2 * n1 + t, ld_stream(in + a + N2 * n1 + t));
            st_stream(out + b + N2 * n1 + t, ld_stream(in + b + N2 * n1 + t));
        });
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int default_theta_cols(int n_phi) { return n_phi >= 64 ? 16 : 8; }

int default_phi_lines(int n_line)
{
    switch (n_line) {
    case 32: return 64;
    case 64: return 32;
    case 128: return 32;
    default: return 16;
    }
}

static int lanes_per_line(int n_line)
{
    switch (n_line) {
    case 32: return Split<32>::N2;
    case 64: return Split<64>::N2;
    case 128: return Split<128>::N2;
    case 256: return Split<256>::N2;
    default: return 0;
    }
}

bool theta_shape_ok(int n_line, int cols, int n_phi)
{
    return lanes_per_line(n_line) > 0 && (cols == 8 || cols == 16) && (n_phi / 2) % (2 * cols) == 0;
}

bool phi_shape_ok(int n_line, int lines)
{
    const int l = lanes_per_line(n_line);
    return l > 0 && (lines == 4 || lines == 8 || lines == 16 || lines == 32 || lines == 64) &&
           l * lines <= 256 && l * lines >= 16;
}

template <int N, int C>
static hipError_t theta_go(const double *in, double *out, const ThetaItem *items, int n_items,
                           int n_theta, int n_phi, const Twiddle *tw, const double *eneg,
                           hipStream_t s)
{
    const int tiles = (n_phi / 2) / (2 * C);
    const dim3 grid((unsigned)(n_items * tiles)), block(C * Split<N>::N2);
    theta_kernel<N, C><<<grid, block, 0, s>>>(in, out, items, tiles, n_theta, n_phi, tw, eneg);
    return hipGetLastError();
}

hipError_t launch_theta(int n_line, int cols, const double *in, double *out,
                        const ThetaItem *items, int n_items, int n_theta, int n_phi,
                        const Twiddle *tw, const double *eneg, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (!theta_shape_ok(n_line, cols, n_phi) || n_line != 2 * n_theta) return hipErrorInvalidValue;
#define SPHFILT_THETA_CASE(NN)                                                                  \
    case NN:                                                                                    \
        return cols == 16 ? theta_go<NN, 16>(in, out, items, n_items, n_theta, n_phi, tw, eneg, s)  \
                          : theta_go<NN, 8>(in, out, items, n_items, n_theta, n_phi, tw, eneg, s);
    switch (n_line) {
        SPHFILT_THETA_CASE(32)
        SPHFILT_THETA_CASE(64)
        SPHFILT_THETA_CASE(128)
        SPHFILT_THETA_CASE(256)
    default: return hipErrorInvalidValue;
    }
#undef SPHFILT_THETA_CASE
}

template <int N, int LINES>
static hipError_t phi_go(const double *in, double *out, const PhiItem *items, int n_items,
                         int n_theta, const Twiddle *tw, const double *eneg, hipStream_t s)
{
    if constexpr (LINES * Split<N>::N2 > 256 || LINES * Split<N>::N2 < 16) {
        return hipErrorInvalidValue;
    } else {
        const dim3 grid((unsigned)((n_items + LINES - 1) / LINES)), block(LINES * Split<N>::N2);
        phi_kernel<N, LINES><<<grid, block, 0, s>>>(in, out, items, n_items, n_theta, tw, eneg);
        return hipGetLastError();
    }
}

template <int N>
static hipError_t phi_lines(int lines, const double *in, double *out, const PhiItem *items,
                            int n_items, int n_theta, const Twiddle *tw, const double *eneg,
                            hipStream_t s)
{
    switch (lines) {
    case 4: return phi_go<N, 4>(in, out, items, n_items, n_theta, tw, eneg, s);
    case 8: return phi_go<N, 8>(in, out, items, n_items, n_theta, tw, eneg, s);
    case 16: return phi_go<N, 16>(in, out, items, n_items, n_theta, tw, eneg, s);
    case 32: return phi_go<N, 32>(in, out, items, n_items, n_theta, tw, eneg, s);
    case 64: return phi_go<N, 64>(in, out, items, n_items, n_theta, tw, eneg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_phi(int n_line, int lines, const double *in, double *out, const PhiItem *items,
                      int n_items, int n_theta, const Twiddle *tw, const double *eneg,
                      hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (!phi_shape_ok(n_line, lines)) return hipErrorInvalidValue;
    switch (n_line) {
    case 32: return phi_lines<32>(lines, in, out, items, n_items, n_theta, tw, eneg, s);
    case 64: return phi_lines<64>(lines, in, out, items, n_items, n_theta, tw, eneg, s);
    case 128: return phi_lines<128>(lines, in, out, items, n_items, n_theta, tw, eneg, s);
    case 256: return phi_lines<256>(lines, in, out, items, n_items, n_theta, tw, eneg, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sphfilt
