// line_filter.h -- the per-line filter engine and the workgroup workers of
// the theta- and phi-passes, shared by the per-plan kernels and the batched
// persistent kernel (device side).
//
// Both passes filter independent real lines of length N: FFT, multiply mode q
// by f(|q|, cutoff), inverse FFT (arXiv:2305.01537, Sec. II.A).  Two real lines
// that share one cutoff are packed as the real and imaginary part of one
// complex line; because the mask is real and even in q, the real and
// imaginary parts of the result are the two filtered lines.
#pragma once
#include "fft_core.h"
#include "sphfilt_internal.h"
#include "theta_gemm.h"

#include <cmath>

namespace sphfilt {

// ln(0.9), the Gaussian filter's constant (eq. gaussian_filter).
constexpr double kLog09 = -0.10536051565782630123;

// Field data is streamed once per pass: loads are non-temporal.  Stores of
// the theta-pass (whose output the phi-pass reads next) and of the phi-pass
// can each be non-temporal or cache-allocating.
#ifndef SPHFILT_NT
#define SPHFILT_NT 1
#endif
#ifndef SPHFILT_NT_STORE_THETA
#define SPHFILT_NT_STORE_THETA 1
#endif
#ifndef SPHFILT_NT_STORE_PHI
#define SPHFILT_NT_STORE_PHI 1
#endif

__device__ __forceinline__ double ld_stream(const double *p)
{
#if SPHFILT_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Loads whose instruction reads only a piece of each 128-byte line it
// touches go through the cache instead: rings of N <= 128 points (4 or 8
// lanes per ring: 32- or 64-byte pieces) and theta rows at N = 32 (sub-tiles
// of 8 meridians).  Streamed, the other pieces of a line were fetched again
// (1.32x the algorithmic bytes for rings of 32, 1.09x for rings of 64, 1.04x
// for rings of 128; cached, the phi pass at 128 ran 1.3 % faster and the
// fused grmhd call 3 %).
template <bool CACHED>
__device__ __forceinline__ double ld_piece(const double *p)
{
    if constexpr (CACHED)
        return *p;
    else
        return ld_stream(p);
}
template <int N>
constexpr bool ring_loads_cached() { return N <= 128; }
// Ring stores of 32-byte pieces (4 lanes per ring: N = 32, 48) go through the
// cache too, so that the pieces of a line are written back together (phi pass
// at N = 32: 1.125x the algorithmic writes streamed, 1.8 % faster cached; at
// 64 and 128 streamed stores measured as fast or faster).
template <int N>
constexpr bool ring_stores_streamed() { return SPHFILT_NT_STORE_PHI != 0 && N != 32 && N != 48; }
template <int N>
constexpr bool theta_loads_cached() { return N <= 32; }

template <bool NT = true>
__device__ __forceinline__ void st_stream(double *p, double v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Two adjacent doubles at a 16-byte aligned address, moved by one 16-byte
// access: the theta pass packs adjacent meridian pairs into one complex line.
typedef double dpair __attribute__((ext_vector_type(2)));

template <bool CACHED>
__device__ __forceinline__ cplx ld_pair(const double *p)
{
    const dpair *q = reinterpret_cast<const dpair *>(p);
    dpair v;
#if SPHFILT_NT
    if constexpr (!CACHED)
        v = __builtin_nontemporal_load(q);
    else
#endif
        v = *q;
    return cplx{v.x, v.y};
}

template <bool NT = true>
__device__ __forceinline__ void st_pair(double *p, double re, double im)
{
    dpair *q = reinterpret_cast<dpair *>(p);
    const dpair v = {re, im};
    if constexpr (NT)
        __builtin_nontemporal_store(v, q);
    else
        *q = v;
}

// Which two meridian pairs a theta line packs.  Adjacent pairs k, k + 1 (one
// 16-byte access per row) for every N but 256, where pairs k and k + cp (two
// 8-byte accesses; a 16-line sub-tile's instruction still covers whole
// 128-byte lines) measured faster: dense theta pass 5.8 against 5.4 TB/s.
// Adjacent pairs gained 2-32 % on the other lengths, most where the tile is
// narrow (sub-tiles of 4 or 8 lines).
template <int N>
constexpr bool theta_pairs_adjacent() { return N != 256; }

template <bool ADJ, bool CACHED>
__device__ __forceinline__ cplx ld_two(const double *row, int kr, int ki)
{
    if constexpr (ADJ)
        return ld_pair<CACHED>(row + kr);
    else
        return cplx{ld_piece<CACHED>(row + kr), ld_piece<CACHED>(row + ki)};
}

template <bool ADJ, bool NT>
__device__ __forceinline__ void st_two(double *row, int kr, int ki, double re, double im)
{
    if constexpr (ADJ) {
        st_pair<NT>(row + kr, re, im);
    } else {
        st_stream<NT>(row + kr, re);
        st_stream<NT>(row + ki, im);
    }
}

// Gaussian factors of one second-stage row, with the 1/N folded in.  The
// row holds the modes q = q0 + N1 k2, k2 < N2 (q0 = t + N2 r < N1), whose
// folded indices |q| run along two arithmetic sequences of step N1:
//   k2 <  N2/2:  |q| = q0 + N1 k2,
//   k2 >= N2/2:  |q| = N - q = (N1 - q0) + N1 j,  j = N2 - 1 - k2.
// Along |q| = b + N1 j, with kappa = log(0.9) / (c + 1)^2, consecutive
// factors exp(kappa |q|^2) have the ratio g_j = exp(kappa N1 (2b + N1 (2j + 1))),
// and g_{j+1} = g_j exp(2 kappa N1^2): two exps per sequence and one per line
// instead of one per mode.  The j-th factor carries about j^2 / 2 roundings
// more than a direct exp (below 1e-14 relative for j < 8).  gauss_factors
// writes the factor of mode k2 to f[k2].
template <int N1>
struct GaussChain {
    double kappa, step;     // log(0.9) / (c + 1)^2, exp(2 kappa N1^2)
    __device__ __forceinline__ explicit GaussChain(double c)
    {
        const double inv = 1.0 / (c + 1.0);
        kappa = kLog09 * inv * inv;
        step = exp(2.0 * kappa * (double)(N1 * N1));
    }
};

template <int N1, int N2>
__device__ __forceinline__ void gauss_factors(int q0, const GaussChain<N1> &g, double (&f)[N2])
{
    constexpr double inv_n = 1.0 / (N1 * N2);
    constexpr double D = N1;
    static_assert(N2 % 2 == 0, "two sequences of N2 / 2 modes");
    static_for<0, 2>([&](auto hh) {
        constexpr int h = decltype(hh)::value;
        const double b = h == 0 ? (double)q0 : (double)(N1 - q0);
        double fj = exp(g.kappa * b * b) * inv_n;
        double ratio = exp(g.kappa * D * (2.0 * b + D));
        static_for<0, N2 / 2>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            f[h == 0 ? j : N2 - 1 - j] = fj;
            if constexpr (j + 1 < N2 / 2) {
                fj *= ratio;
                ratio *= g.step;
            }
        });
    });
}

// Mask of one line, with the inverse transform's 1/N folded in.  v holds
// X[q] at q = t + N2 r + N1 k2 in v[r N2 + k2].
//   exponential (eq. exp_filter): f = 1 for |q| <= c, else exp(-(|q| - c)).
//     With m = floor(c), |q| <= c is |q| <= m, and above the cutoff
//     exp(c - |q|) = exp(c - m - 1) * e^{-(|q| - m - 1)}: one exp per lane and
//     a table of e^{-k}, instead of one exp per mode.
//   sharp: the same with the factor above the cutoff set to 0.
//   Gaussian (eq. gaussian_filter): f = exp(log(0.9) (|q| / (c + 1))^2),
//     formed along the row by gauss_factors.
template <int N1, int N2, int NV>
__device__ __forceinline__ void apply_mask(cplx (&v)[NV], int t, int kind, double c,
                                           const double *etab)
{
    constexpr int N = N1 * N2;
    constexpr int R = NV / N2;
    constexpr bool PAD = NV != N1;        // padded second stage: rows k1 >= N1 are empty
    constexpr double inv_n = 1.0 / N;
    if (kind == 1) {
        const GaussChain<N1> g(c);
        static_for<0, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            if constexpr (PAD) {
                if (t + N2 * r >= N1) return;
            }
            double f[N2];
            gauss_factors<N1, N2>(t + N2 * r, g, f);
            static_for<0, N2>([&](auto kk) {
                constexpr int k2 = decltype(kk)::value;
                v[r * N2 + k2].re *= f[k2];
                v[r * N2 + k2].im *= f[k2];
            });
        });
    } else {
        const int m = c >= (double)N ? N : (int)floor(c);
        const double g = (kind == 0 ? exp((c - (double)m) - 1.0) : 0.0) * inv_n;
        static_for<0, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            if constexpr (PAD) {
                if (t + N2 * r >= N1) return;
            }
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

// Ordering of LDS accesses among the lanes of one wave: lanes of a wave see
// each other's earlier LDS writes (a wave's LDS instructions complete in
// order); the fences keep the compiler from moving accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronise the lanes of a line: a workgroup barrier, or, where the line's
// lanes all lie in one wave (WAVE: the phi layout), the wave-level ordering.
template <bool WAVE>
__device__ __forceinline__ void line_sync()
{
    if constexpr (WAVE)
        wave_lds_sync();
    else
        __syncthreads();
}

// Mask of a complex line whose two real lines take different kinds (the
// hybrid filter can pick the Gaussian for one and the exponential for the
// other).  With z = a + i b and Z its transform, A and B (the transforms of a
// and b) are (Z[q] + conj Z[-q]) / 2 and (Z[q] - conj Z[-q]) / 2i, so
//   f_a A + i f_b B = (f_a + f_b)/2 Z[q] + (f_a - f_b)/2 conj Z[N - q].
// Bin N - q lives on another lane: every lane publishes its bins through the
// line's LDS region P (2N doubles: real parts, then imaginary parts, natural
// order), so one synchronisation serves both parts.  Lines with ka == kb get
// plain f Z.  All lanes of the workgroup (WAVE: of the wave) call this
// together.  (In the theta layout one wave holds lanes of every line of the
// workgroup, so restricting the exchange to the lines that mix two kinds
// would save nothing there.)
template <int N1, int N2, bool WAVE, int NV>
__device__ __forceinline__ void apply_mask_pair(cplx (&v)[NV], int t, int ka, int kb, double c,
                                                const double *etab, double *P)
{
    constexpr int N = N1 * N2;
    constexpr int R = NV / N2;
    constexpr bool PAD = NV != N1;
    constexpr double inv_n = 1.0 / N;
    const int m = c >= (double)N ? N : (int)floor(c);
    const double g_exp = exp((c - (double)m) - 1.0) * inv_n;
    const GaussChain<N1> gc(c);
    // Each real line's kind as 0/1 weights, so that the per-mode factors are
    // blends rather than branches (a select chain on the kind was lowered to
    // a switch per mode: hundreds of divergent branches per workgroup).
    // Weights of 1 and 0 keep the blends exact.
    const double ga = ka == 1 ? 1.0 : 0.0, ea = ka == 0 ? 1.0 : 0.0, sa = ka == 2 ? 1.0 : 0.0;
    const double gb = kb == 1 ? 1.0 : 0.0, eb = kb == 0 ? 1.0 : 0.0, sb = kb == 2 ? 1.0 : 0.0;
    static_for<0, R>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        if constexpr (PAD) {
            if (t + N2 * r >= N1) return;
        }
        static_for<0, N2>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            const int q = t + N2 * r + N1 * k2;
            P[q] = v[r * N2 + k2].re;
            P[N + q] = v[r * N2 + k2].im;
        });
    });
    line_sync<WAVE>();
    static_for<0, R>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        if constexpr (PAD) {
            if (t + N2 * r >= N1) return;
        }
        double fgs[N2];
        gauss_factors<N1, N2>(t + N2 * r, gc, fgs);
        static_for<0, N2>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            const double fg = fgs[k2];
            const int q = t + N2 * r + N1 * k2;
            const int qhat = q <= N / 2 ? q : N - q;
            const double e = etab[max(qhat - m - 1, 0)];
            const bool below = qhat <= m;
            const double tail = below ? inv_n : g_exp * e;     // exponential
            const double keep = below ? inv_n : 0.0;           // sharp
            const double fa = ga * fg + ea * tail + sa * keep;
            const double fb = gb * fg + eb * tail + sb * keep;
            const double alpha = 0.5 * (fa + fb), beta = 0.5 * (fa - fb);
            const int qp = (N - q) % N;
            v[r * N2 + k2].re = alpha * v[r * N2 + k2].re + beta * P[qp];
            v[r * N2 + k2].im = alpha * v[r * N2 + k2].im - beta * P[N + qp];
        });
    });
    line_sync<WAVE>();
}

// LDS doubles per line: an N1 x (N2 + 1) padded tile plus one double, so that
// consecutive lines start on different banks.
template <int N1, int N2>
constexpr int line_lds() { return N1 * (N2 + 1) + 1; }

// LDS doubles per line of a kernel: the hybrid-capable variants also publish
// a whole spectrum (2N doubles) for the two-kind mask.
template <int N1, int N2, bool HYB>
constexpr int line_stride()
{
    return HYB && 2 * N1 * N2 + 1 > line_lds<N1, N2>() ? 2 * N1 * N2 + 1 : line_lds<N1, N2>();
}

// Forward transpose: lane t holds Y[k1][t] in v[k1]; afterwards it holds
// Y[t + N2 r][n2] in v[r * N2 + n2].  Real and imaginary parts go through LDS
// in two rounds to halve the LDS footprint.  With a padded second stage
// (NV > N1: N2 does not divide N1) the rows t + N2 r >= N1 do not exist and
// are set to zero.  Only the line's own lanes touch its region L, so with
// WAVE (the line's lanes in one wave) the wave-level ordering replaces the
// workgroup barriers.
template <int N1, int N2, bool WAVE, int NV>
__device__ __forceinline__ void transpose_fwd(cplx (&v)[NV], int t, double *L)
{
    constexpr int S = N2 + 1;
    constexpr bool PAD = NV != N1;
    static_for<0, 2>([&](auto part) {
        constexpr bool im = decltype(part)::value == 1;
        static_for<0, N1>([&](auto kk) {
            constexpr int k1 = decltype(kk)::value;
            L[k1 * S + t] = im ? v[k1].im : v[k1].re;
        });
        line_sync<WAVE>();
        static_for<0, NV / N2>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            const bool row = !PAD || t + N2 * r < N1;
            static_for<0, N2>([&](auto nn) {
                constexpr int n2 = decltype(nn)::value;
                const double x = row ? L[(t + N2 * r) * S + n2] : 0.0;
                if constexpr (im) v[r * N2 + n2].im = x; else v[r * N2 + n2].re = x;
            });
        });
        line_sync<WAVE>();
    });
}

// Inverse of transpose_fwd (padded rows are dropped).
template <int N1, int N2, bool WAVE, int NV>
__device__ __forceinline__ void transpose_bwd(cplx (&v)[NV], int t, double *L)
{
    constexpr int S = N2 + 1;
    constexpr bool PAD = NV != N1;
    static_for<0, 2>([&](auto part) {
        constexpr bool im = decltype(part)::value == 1;
        static_for<0, NV / N2>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            if constexpr (PAD) {
                if (t + N2 * r >= N1) return;
            }
            static_for<0, N2>([&](auto nn) {
                constexpr int n2 = decltype(nn)::value;
                L[(t + N2 * r) * S + n2] = im ? v[r * N2 + n2].im : v[r * N2 + n2].re;
            });
        });
        line_sync<WAVE>();
        static_for<0, N1>([&](auto kk) {
            constexpr int k1 = decltype(kk)::value;
            const double x = L[k1 * S + t];
            if constexpr (im) v[k1].im = x; else v[k1].re = x;
        });
        line_sync<WAVE>();
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
// etab: e^{-k}, k <= N/2, in LDS, written before the first barrier here
// (with WAVE: before a barrier of the caller's).  WAVE: the line's lanes lie
// in one wave, so the transposes and the two-kind mask synchronise the wave
// only, with no workgroup barrier, and `mixed` is wave-uniform.
template <int N1, int N2, bool HYB, bool WAVE = false, int NV>
__device__ __forceinline__ void filter_line(cplx (&v)[NV], int t, int kind, int kind_b, bool mixed,
                                            double c, double *L, const Twiddle *__restrict__ tw,
                                            const double *etab)
{
    // R second-stage rows per lane; when N2 does not divide N1 the last row
    // is padded (NV = R N2 > N1) and its entries k1 >= N1 are skipped
    constexpr int R = NV / N2;
    constexpr bool PAD = NV != N1;
    static_assert(NV % N2 == 0 && NV >= N1 && NV - N1 < N2, "second stage: ceil(N1 / N2) rows");

    // forward: N1-point DFTs over n1, twiddle W_N^{t k1}
    dft_reg<N1, false>(v);
    twiddle_powers<N1, false, 0>(v, tw, t);
    transpose_fwd<N1, N2, WAVE>(v, t, L);
    // N2-point DFTs over n2: v[r N2 + k2] = X[k1 + N1 k2], k1 = t + N2 r
    static_for<0, R>([&](auto rr) { dft_reg<N2, false, decltype(rr)::value * N2>(v); });

    // kind: the real part's filter; kind_b: the imaginary part's.  mixed
    // (workgroup-uniform, or wave-uniform with WAVE) is set when some line of
    // the workgroup (wave) has two; only the hybrid-capable variant (HYB)
    // carries that code.
    if constexpr (HYB) {
        if (mixed)
            apply_mask_pair<N1, N2, WAVE>(v, t, kind, kind_b, c, etab, L);
        else
            apply_mask<N1, N2>(v, t, kind, c, etab);
    } else {
        apply_mask<N1, N2>(v, t, kind, c, etab);
    }

    // inverse: N2-point inverse DFTs, conjugate twiddles W_N^{-n2 k1},
    // transpose back, N1-point inverse DFTs.  In the hybrid-capable variant
    // the table address takes an opaque zero offset here, so that the
    // inverse twiddles are not loaded before the two-kind mask and held
    // across it (that pushed the register count past the two-wave limit and
    // spilled 16-40 registers at N = 256).
    const Twiddle *tw_inv = tw;
    if constexpr (HYB) {
        int zero = 0;
        asm volatile("" : "+v"(zero));
        tw_inv = tw + zero;
    }
    static_for<0, R>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        dft_reg<N2, true, r * N2>(v);
        // a padded row's twiddles stay inside the table (its result is dropped)
        const int k1 = t + N2 * r;
        twiddle_powers<N2, true, r * N2>(v, tw_inv, PAD && k1 >= N1 ? 0 : k1);
    });
    transpose_bwd<N1, N2, WAVE>(v, t, L);
    dft_reg<N1, true>(v);
}

// Copy e^{-k}, k in [0, N/2], into the workgroup's LDS table.
template <int N>
__device__ __forceinline__ void stage_exp_table(double *etab, const double *__restrict__ eneg,
                                                int lane)
{
    for (int i = lane; i <= N / 2; i += (int)blockDim.x) etab[i] = eneg[i];
}

// N = N1 * N2: N2 lanes per line, N1 values per lane.  After the transpose
// each lane holds ceil(N1 / N2) rows of N2 second-stage values: NV values per
// lane in all (NV = N1 when N2 divides N1, else the last row is padded: 96 =
// 12 x 8 and 80 = 10 x 8 hold 16, 192 = 12 x 16 and 160 = 10 x 16 hold 16 with
// one row per lane, 4 or 6 of the 16 lanes' rows padded).  The lengths 48,
// 96 and 192 take a radix-3 stage in the N1-point transform, 80 and 160 a
// radix-5 stage.  Splits with more lanes per line were chosen over ones with
// fewer padded values (24 x 4, 24 x 8, 20 x 4, 20 x 8): wider row pieces per
// load and fewer registers.
template <int A, int B>
struct SplitOf {
    static constexpr int N1 = A, N2 = B;
    static constexpr int NV = (A + B - 1) / B * B;
};
template <int N> struct Split;
template <> struct Split<32>  : SplitOf<8, 4> {};
template <> struct Split<48>  : SplitOf<12, 4> {};
template <> struct Split<64>  : SplitOf<8, 8> {};
template <> struct Split<80>  : SplitOf<10, 8> {};
template <> struct Split<96>  : SplitOf<12, 8> {};
template <> struct Split<128> : SplitOf<16, 8> {};
template <> struct Split<160> : SplitOf<10, 16> {};
template <> struct Split<192> : SplitOf<12, 16> {};
template <> struct Split<256> : SplitOf<16, 16> {};


// One cell of Jameson's detector: sigma = num / den >= threshold (threshold
// > 0), decided as the rounded quotient decides it, mostly without the
// division.  r = num - threshold den is formed with one rounding (fma), so its
// sign is that of the exact difference: r > 0 means num / den > threshold, so
// the rounded quotient is >= threshold (fires); r below -2^-50 threshold den
// (plus a floor for tiny values) puts the exact quotient more than an ulp
// below the threshold, so the rounded one stays below (does not fire).  The
// rest (r near zero, den zero, non-finite values) is `unsure`: the caller
// decides those cells by the division itself.
struct JamesonCell {
    bool fires, unsure;
};

__device__ __forceinline__ double jameson_num(double a, double b, double c)
{
    return fabs(a - 2.0 * b + c);
}

__device__ __forceinline__ double jameson_den(double a, double b, double c, double eps)
{
    return fabs(a) + 2.0 * fabs(b) + fabs(c) + eps;
}

__device__ __forceinline__ JamesonCell jameson_cell(double a, double b, double c, double eps,
                                                    double threshold)
{
    const double num = jameson_num(a, b, c), den = jameson_den(a, b, c, eps);
    const double r = fma(-threshold, den, num);
    const double margin = fma(threshold * 0x1p-50, den, 0x1p-1000);
    return JamesonCell{r > 0.0, !(r > 0.0) && !(r < -margin)};
}

// Jameson's detector sigma_i = |u_{i-1} - 2u_i + u_{i+1}| /
// (|u_{i-1}| + 2|u_i| + |u_{i+1}| + eps) on the two real lines packed in v
// (periodic along the line).  Returns bit 0 if any cell of the real-part
// line has sigma >= threshold, bit 1 for the imaginary-part line.  Lanes
// publish both real lines through the line's LDS region L (2N doubles: the
// hybrid-capable kernels' line stride) to read their neighbours, and combine
// their findings in *flag (this line's LDS word) behind workgroup barriers;
// with WAVE (the line's N2 lanes are consecutive lanes of one wave, aligned to
// N2) a wave-level ordering and a ballot do instead.  All lanes of the
// workgroup call this together; `check` says whether this lane's line needs
// the detector at all.
template <int N1, int N2, bool WAVE, int NV>
__device__ __forceinline__ int detect_shocks(const cplx (&v)[NV], int t, double *L, int *flag,
                                             bool check, double eps, double threshold)
{
    constexpr int N = N1 * N2;
    if constexpr (!WAVE) {
        if (t == 0) *flag = 0;
    }
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        L[N2 * n1 + t] = v[n1].re;
        L[N + N2 * n1 + t] = v[n1].im;
    });
    line_sync<WAVE>();
    int bits = 0;
    if (check) {
        // straight-line sign tests over every cell of the lane; the cells they
        // leave unsure (never, with random data) go through the division in a
        // second, rarely entered loop
        int unsure = 0;
        static_for<0, 2>([&](auto part) {
            constexpr int im = decltype(part)::value;
            const double *Lp = L + im * N;
            static_for<0, N1>([&](auto nn) {
                constexpr int n1 = decltype(nn)::value;
                const int n = N2 * n1 + t;
                const double b = im ? v[n1].im : v[n1].re;
                const JamesonCell cell = jameson_cell(Lp[(n + N - 1) % N], b, Lp[(n + 1) % N], eps,
                                                      threshold);
                bits |= cell.fires ? 1 << im : 0;
                unsure |= cell.unsure ? 1 << im : 0;
            });
        });
        if (unsure) {
            static_for<0, 2>([&](auto part) {
                constexpr int im = decltype(part)::value;
                const double *Lp = L + im * N;
                static_for<0, N1>([&](auto nn) {
                    constexpr int n1 = decltype(nn)::value;
                    const int n = N2 * n1 + t;
                    const double a = Lp[(n + N - 1) % N], c = Lp[(n + 1) % N];
                    const double b = im ? v[n1].im : v[n1].re;
                    if ((unsure >> im) & 1)
                        bits |= jameson_num(a, b, c) / jameson_den(a, b, c, eps) >= threshold ? 1 << im : 0;
                });
            });
        }
    }
    if constexpr (WAVE) {
        static_assert(64 % N2 == 0, "a line's lanes lie in one wave");
        const unsigned long long re = __ballot((bits & 1) != 0), im = __ballot((bits & 2) != 0);
        const int first = (int)__lane_id() & ~(N2 - 1);
        const unsigned long long mine = (N2 == 64 ? ~0ull : ((1ull << N2) - 1)) << first;
        // the region L is rewritten next (the transposes): keep this wave's
        // neighbour reads ahead of that
        wave_lds_sync();
        return ((re & mine) ? 1 : 0) | ((im & mine) ? 2 : 0);
    } else {
        if (bits) atomicOr(flag, bits);
        __syncthreads();
        return *flag;
    }
}

// The two kinds of a packed line: a hybrid line takes the Gaussian where its
// detector fired (or its recorded decision says so), else the exponential.
// dec_a / dec_b: byte offsets of the two real lines in h.dec.  *mixed says
// whether some line takes two kinds: over the wave with WAVE (see
// detect_shocks), else over the workgroup, read from the n_lines flag words
// flags[0, n_lines) (this line's is flags[line]), which hold each line's
// detector bits (0 for lines that are not hybrid) after one barrier.
template <int N1, int N2, bool WAVE, int NV>
__device__ __forceinline__ void hybrid_kinds(const cplx (&v)[NV], int t, double *L, int *flags,
                                             int line, int n_lines, bool active, int kind,
                                             size_t dec_a, size_t dec_b, const HybridArgs &h,
                                             int *ka, int *kb, bool *mixed)
{
    *ka = kind;
    *kb = kind;
    *mixed = false;
    if (!h.present) return;
    const bool hybrid = active && kind == 3;
    int bits = 0;
    if (h.replay) {
        if (hybrid) bits = (h.dec[dec_a] ? 1 : 0) | (h.dec[dec_b] ? 2 : 0);
        if constexpr (!WAVE) {
            if (t == 0) flags[line] = bits;
            __syncthreads();
        }
    } else {
        bits = detect_shocks<N1, N2, WAVE>(v, t, L, flags + line, hybrid, h.eps, h.threshold);
        if (hybrid && h.dec && t == 0) {
            h.dec[dec_a] = (unsigned char)(bits & 1);
            h.dec[dec_b] = (unsigned char)((bits >> 1) & 1);
        }
    }
    if (hybrid) {
        *ka = (bits & 1) ? 1 : 0;
        *kb = (bits & 2) ? 1 : 0;
    }
    if constexpr (WAVE) {
        *mixed = __ballot(*ka != *kb) != 0;
    } else {
        // a line takes two kinds exactly when one of its two bits is set
        bool any = false;
        for (int i = 0; i < n_lines; ++i) {
            const int f = flags[i];
            any |= f == 1 || f == 2;
        }
        *mixed = any;
    }
}

// Lanes per line and lines per 256-lane workgroup for each supported N.
template <int N>
constexpr int lines_per_256() { return 256 / Split<N>::N2; }

// ---------------------------------------------------------------------------
// theta-pass worker.  C complex lines per workgroup (C * N2 lanes, lane
// (p, t) with p = lane % C fastest), grouped in sub-tiles of cp = 2^cp_log2
// lines.  Sub-tile u = p / cp works on shell items[u] (u < n_valid) and
// meridian pairs [k0, k0 + 2 cp), k0 = tile * 2 cp.  Its line p' packs the
// adjacent pairs k0 + 2 p' (real part) and k0 + 2 p' + 1 (imaginary part),
// whose two values of a row a lane moves with one 16-byte access; at N = 256
// it packs k0 + p' and k0 + cp + p' instead (theta_pairs_adjacent).  The
// extended line of pair k is rows 0..n_theta-1 of meridian k, then, times the
// parity sign, rows n_theta-1..0 of meridian k + n_phi/2 (the paper's
// extension across the poles).  Lanes walk the meridians fastest, so each
// load and store instruction covers whole row segments.  Where pairs are
// adjacent the pairing, and so the result, does not depend on cp.  All lanes
// of the workgroup must call this together.
// ---------------------------------------------------------------------------
template <int N, int C, bool HYB>
__device__ __forceinline__ void theta_block(const double *in, double *out,
                                            const ThetaItem *__restrict__ items, int n_valid,
                                            int cp_log2, int tile, int n_theta, int n_phi,
                                            const Twiddle *__restrict__ tw,
                                            const double *__restrict__ eneg, double *lds,
                                            double *etab, int *flags, const HybridArgs &h, int lane)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    static_assert(C * N2 == 256 || C * N2 == 128, "theta workgroups have 256 or 128 lanes");
    const int p = lane % C, t = lane / C;
    const int u = p >> cp_log2, pp = p & ((1 << cp_log2) - 1);
    const bool valid = u < n_valid;
    ThetaItem it{0, kFlagIdentity, 0.0};
    if (valid) it = items[u];
    const bool active = valid && !(it.flags & kFlagIdentity);
    const int any_active = __syncthreads_or(active);
    if (any_active) stage_exp_table<N>(etab, eneg, lane);

    const size_t base = (size_t)it.shell * (size_t)(n_theta * n_phi);
    const int half = n_phi / 2;
    constexpr bool ADJ = theta_pairs_adjacent<N>();
    const int k0 = tile << (cp_log2 + 1);
    const int kr = ADJ ? k0 + 2 * pp : k0 + pp, ki = ADJ ? kr + 1 : kr + (1 << cp_log2);
    const double s = (it.flags & kFlagOddParity) ? -1.0 : 1.0;
    // Row block n1 starts at a workgroup-uniform row; the lane adds a small
    // non-negative row offset and its column.  First half: row N2 n1 + t.
    // Mirrored half: row (N - N2 (n1 + 1)) + (N2 - 1 - t) = 2 n_theta - 1 - (N2 n1 + t).
    const int off_n = t * n_phi;
    const int off_s = (N2 - 1 - t) * n_phi + half;

    cplx v[Split<N>::NV];
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        if (!valid) {
            v[n1] = cplx{0.0, 0.0};
        } else if constexpr (n1 < N1 / 2) {
            constexpr bool cached = theta_loads_cached<N>();
            const double *row = in + base + (size_t)(N2 * n1) * n_phi;
            v[n1] = ld_two<ADJ, cached>(row + off_n, kr, ki);
        } else {
            constexpr bool cached = theta_loads_cached<N>();
            const double *row = in + base + (size_t)(N - N2 * (n1 + 1)) * n_phi;
            const cplx w = ld_two<ADJ, cached>(row + off_s, kr, ki);
            v[n1] = cplx{s * w.re, s * w.im};
        }
    });
    // Identity lines sharing a workgroup with filtered ones run through the
    // transform (the barriers are workgroup-wide) but their result is dropped;
    // they are copied exactly from `in`.  That only happens out of place.
    if (any_active) {
        double *L = lds + p * line_stride<N1, N2, HYB>();
        const size_t dline = (size_t)it.shell * (size_t)half;
        int ka = it.flags & kKindMask, kb = ka;
        bool mixed = false;
        if constexpr (HYB)
            hybrid_kinds<N1, N2, false>(v, t, L, flags, p, C, active, ka, dline + kr, dline + ki, h,
                                        &ka, &kb, &mixed);
        filter_line<N1, N2, HYB>(v, t, ka, kb, mixed, active ? it.c : INFINITY, L, tw, etab);
    }
    if (valid && (active || !any_active)) {
        static_for<0, N1>([&](auto nn) {
            constexpr int n1 = decltype(nn)::value;
            if constexpr (n1 < N1 / 2) {
                double *row = out + base + (size_t)(N2 * n1) * n_phi;
                st_two<ADJ, SPHFILT_NT_STORE_THETA != 0>(row + off_n, kr, ki, v[n1].re, v[n1].im);
            } else {
                double *row = out + base + (size_t)(N - N2 * (n1 + 1)) * n_phi;
                st_two<ADJ, SPHFILT_NT_STORE_THETA != 0>(row + off_s, kr, ki, s * v[n1].re, s * v[n1].im);
            }
        });
    } else if (valid && in != out) {
        static_for<0, N1>([&](auto nn) {
            constexpr int n1 = decltype(nn)::value;
            const size_t r = n1 < N1 / 2 ? (size_t)(N2 * n1) * n_phi + off_n
                                         : (size_t)(N - N2 * (n1 + 1)) * n_phi + off_s;
            const cplx w = ld_two<ADJ, false>(in + base + r, kr, ki);
            st_two<ADJ, SPHFILT_NT_STORE_THETA != 0>(out + base + r, kr, ki, w.re, w.im);
        });
    }
}

// ---------------------------------------------------------------------------
// phi-pass worker.  LINES ring pairs per workgroup (LINES * N2 lanes, lane
// (p, t) with t fastest): line p packs ring items[p].ring (real part) and its
// mirror ring n_theta-1-j of the same shell (imaginary part), which shares
// m_max.  Lines p >= n_valid are idle.  A line's N2 lanes are consecutive
// lanes of one wave, so the line filter synchronises per wave; the worker
// itself takes three workgroup barriers (the any-active vote, the staged
// e^{-k} table, the end).  All lanes call this together.
// ---------------------------------------------------------------------------
template <int N, int LINES, bool HYB>
__device__ __forceinline__ void phi_block(const double *in, double *out,
                                          const PhiItem *__restrict__ items, int n_valid,
                                          int n_theta, const Twiddle *__restrict__ tw,
                                          const double *__restrict__ eneg, double *lds,
                                          double *etab, int *flags, const HybridArgs &h, int lane)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    const int t = lane % N2, p = lane / N2;
    const bool valid = p < n_valid;
    PhiItem it{0, kFlagIdentity, 0.0};
    if (valid) it = items[p];
    const bool active = valid && !(it.flags & kFlagIdentity);
    const int any_active = __syncthreads_or(active);
    if (any_active) stage_exp_table<N>(etab, eneg, lane);

    const int j = it.ring % n_theta;
    const size_t a = (size_t)it.ring * N;
    const size_t b = a + (size_t)(n_theta - 1 - 2 * j) * N;
    cplx v[Split<N>::NV];
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        constexpr bool cached = ring_loads_cached<N>();
        v[n1] = valid ? cplx{ld_piece<cached>(in + a + N2 * n1 + t), ld_piece<cached>(in + b + N2 * n1 + t)}
                      : cplx{0.0, 0.0};
    });
    if (any_active) {
        // the line filter synchronises each line's wave only: the e^{-k}
        // table staged above needs this one workgroup barrier
        __syncthreads();
        double *L = lds + p * line_stride<N1, N2, HYB>();
        const size_t ring_b = (size_t)it.ring + (size_t)(n_theta - 1 - 2 * j);
        int ka = it.flags & kKindMask, kb = ka;
        bool mixed = false;
        if constexpr (HYB)
            hybrid_kinds<N1, N2, true>(v, t, L, flags, p, LINES, active, ka, (size_t)it.ring, ring_b,
                                       h, &ka, &kb, &mixed);
        filter_line<N1, N2, HYB, true>(v, t, ka, kb, mixed, active ? it.c : INFINITY, L, tw, etab);
    }
    if (valid && (active || !any_active)) {
        static_for<0, N1>([&](auto nn) {
            constexpr int n1 = decltype(nn)::value;
            st_stream<ring_stores_streamed<N>()>(out + a + N2 * n1 + t, v[n1].re);
            st_stream<ring_stores_streamed<N>()>(out + b + N2 * n1 + t, v[n1].im);
        });
    } else if (valid && in != out) {
        static_for<0, N1>([&](auto nn) {
            constexpr int n1 = decltype(nn)::value;
            st_stream<ring_stores_streamed<N>()>(out + a + N2 * n1 + t, ld_stream(in + a + N2 * n1 + t));
            st_stream<ring_stores_streamed<N>()>(out + b + N2 * n1 + t, ld_stream(in + b + N2 * n1 + t));
        });
    }
    // a caller that runs another worker next (the batch kernels) must not
    // overwrite the LDS before every wave is done with its lines
    __syncthreads();
}

}  // namespace sphfilt

namespace sphfilt {

// ---------------------------------------------------------------------------
// Fused shell worker: both passes of a shell with one HBM round trip.
// For n_phi = 2 n_theta = N a theta line and a phi ring have the same length
// N, and a shell has as many complex theta lines (meridian pairs k and
// k + N/4) as complex phi lines (ring pairs j and n_theta-1-j): N/4.  A
// workgroup of W lanes (256 or 128) takes `shells` whole shells: it loads their theta lines
// from HBM, filters them, writes the result into a padded LDS copy of the
// shells, reads it back in the phi layout, filters the rings and stores them
// to HBM (the adjoint order runs the phi pass first).  Lines are filtered as
// by theta_block and phi_block; a theta line
// here packs meridian pairs k and k + N/4 (theta_block packs adjacent pairs at
// these N), so the result is that of the two passes up to rounding.  The line
// filter's LDS scratch reuses the staging memory.
// ---------------------------------------------------------------------------
template <int N, int W = 256> struct ShellShape {
    static constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    static constexpr int lines = N / 4;                  // complex lines per shell and pass
    static constexpr int lanes = lines * N2;             // lanes per shell
    static constexpr int shells = W / lanes;             // shells per workgroup
    static constexpr int row = N + (N2 == 4 ? 4 : 8);    // padded row stride, doubles
    static constexpr int stride = (N / 2) * row + 16;    // doubles per staged shell
    static constexpr int lds = shells * stride;
    static_assert(lanes % N == 0, "a shell's lanes cover whole rows");
    static_assert(shells >= 1 && lds >= (W / N2) * line_stride<N1, N2, true>(), "scratch fits in the staging area");
};

// Staging: lane l of a shell's lanes moves elements e = k * lanes + l,
// k < 2 N1, of the shell (row e / N, column e % N).
template <int N, bool LOAD, int W = 256>
__device__ __forceinline__ void shell_stage(const double *in, double *out, double *sb, cplx (&v)[Split<N>::N1],
                                            size_t base, bool valid, int l)
{
    using S = ShellShape<N, W>;
    constexpr int R = S::lanes / N;                      // rows per k step
    const int r0 = l / N, col = l % N;
    static_for<0, 2 * S::N1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        double &x = (k & 1) ? v[k / 2].im : v[k / 2].re;
        double *s = sb + (k * R + r0) * S::row + col;
        if constexpr (LOAD) {
            x = valid ? ld_stream(in + base + (size_t)k * S::lanes + l) : 0.0;
            *s = x;
        } else {
            x = *s;
            if (valid) st_stream<true>(out + base + (size_t)k * S::lanes + l, x);
        }
    });
}

// theta layout: lane (p, t), p = lane % C fastest; line p packs meridian
// pairs kr = p % lines and ki = kr + lines of staged shell p / lines.
template <int N, bool WRITE, int W = 256>
__device__ __forceinline__ void shell_theta_io(cplx (&v)[Split<N>::N1], double *sb, int t, int kr, double s)
{
    using S = ShellShape<N, W>;
    constexpr int N1 = S::N1, N2 = S::N2, half = N / 2;
    const int ki = kr + S::lines;
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        if constexpr (n1 < N1 / 2) {
            double *r = sb + (N2 * n1 + t) * S::row;
            if constexpr (WRITE) { r[kr] = v[n1].re; r[ki] = v[n1].im; }
            else v[n1] = cplx{r[kr], r[ki]};
        } else {
            double *r = sb + (N - 1 - N2 * n1 - t) * S::row + half;
            if constexpr (WRITE) { r[kr] = s * v[n1].re; r[ki] = s * v[n1].im; }
            else v[n1] = cplx{s * r[kr], s * r[ki]};
        }
    });
}

// The theta layout straight from / to HBM (the shell at `base`, rows of N
// doubles): the same positions as shell_theta_io, with no staging copy.  A
// load or store instruction covers the lines' consecutive meridians of one
// or two rows.  Invalid shells load zeros and store nothing.
template <int N, bool LOAD, int W = 256>
__device__ __forceinline__ void shell_theta_hbm(const double *in, double *out, size_t base,
                                                cplx (&v)[Split<N>::N1], int t, int kr, double s,
                                                bool valid)
{
    using S = ShellShape<N, W>;
    constexpr int N1 = S::N1, N2 = S::N2, half = N / 2;
    constexpr bool cached = theta_loads_cached<N>();
    const int ki = kr + S::lines;
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        constexpr bool first = n1 < N1 / 2;
        const size_t row = first ? base + (size_t)(N2 * n1 + t) * N
                                 : base + (size_t)(N - 1 - N2 * n1 - t) * N + half;
        if constexpr (LOAD) {
            if (!valid) {
                v[n1] = cplx{0.0, 0.0};
            } else if constexpr (first) {
                v[n1] = cplx{ld_piece<cached>(in + row + kr), ld_piece<cached>(in + row + ki)};
            } else {
                v[n1] = cplx{s * ld_piece<cached>(in + row + kr), s * ld_piece<cached>(in + row + ki)};
            }
        } else if (valid) {
            if constexpr (first) {
                st_stream<true>(out + row + kr, v[n1].re);
                st_stream<true>(out + row + ki, v[n1].im);
            } else {
                st_stream<true>(out + row + kr, s * v[n1].re);
                st_stream<true>(out + row + ki, s * v[n1].im);
            }
        }
    });
}

// phi layout: lane (p, t), t = lane % N2 fastest; line p packs rings j and
// n_theta-1-j, j = p % lines, of staged shell p / lines.
template <int N, bool WRITE, int W = 256>
__device__ __forceinline__ void shell_phi_io(cplx (&v)[Split<N>::N1], double *sb, int t, int j)
{
    using S = ShellShape<N, W>;
    constexpr int N1 = S::N1, N2 = S::N2;
    double *ra = sb + j * S::row + t;
    double *rb = sb + (N / 2 - 1 - j) * S::row + t;
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        if constexpr (WRITE) { ra[N2 * n1] = v[n1].re; rb[N2 * n1] = v[n1].im; }
        else v[n1] = cplx{ra[N2 * n1], rb[N2 * n1]};
    });
}

// The phi layout straight from / to HBM (the shell at `base`): line j packs
// ring j and its mirror n_theta-1-j, whose rows are contiguous; a lane moves
// x[N2 n1 + t] of both.  Invalid shells load zeros and store nothing.
template <int N, bool LOAD>
__device__ __forceinline__ void shell_phi_hbm(const double *in, double *out, size_t base,
                                               cplx (&v)[Split<N>::N1], int t, int j, bool valid)
{
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    constexpr bool cached = ring_loads_cached<N>();
    const size_t a = base + (size_t)j * N + t, b = base + (size_t)(N / 2 - 1 - j) * N + t;
    static_for<0, N1>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        if constexpr (LOAD) {
            v[n1] = valid ? cplx{ld_piece<cached>(in + a + N2 * n1), ld_piece<cached>(in + b + N2 * n1)}
                          : cplx{0.0, 0.0};
        } else if (valid) {
            st_stream<true>(out + a + N2 * n1, v[n1].re);
            st_stream<true>(out + b + N2 * n1, v[n1].im);
        }
    });
}

// items: the workgroup's shells (n_valid of them); ring_c: their phi cutoffs,
// lines per shell.  ht / hp: hybrid arguments of the theta and phi passes.
// MFMA (plain kinds, N = 32 or 64 only): the theta pass is the circulant
// product of theta_gemm.h on the staged shells instead of the line FFTs;
// gaux then holds its tables (shell_gemm_aux<N>() doubles).
template <int N>
constexpr int shell_gemm_aux()
{
    return ShellShape<N>::shells * (N / 2 + 1) + N + ShellShape<N>::shells * N;
}

template <int N, bool ADJ, bool HYB, bool MFMA = false, int W = 256>
__device__ __forceinline__ void shell_block(const double *in, double *out,
                                            const ThetaItem *__restrict__ items,
                                            const double *__restrict__ ring_c, int n_valid,
                                            const Twiddle *__restrict__ tw,
                                            const double *__restrict__ eneg, double *lds,
                                            double *etab, int *flags, const HybridArgs &ht,
                                            const HybridArgs &hp, int lane, double *gaux = nullptr)
{
    static_assert(!MFMA || (!HYB && (N == 32 || N == 64)), "circulant theta: plain kinds, N = 32, 64");
    static_assert(!MFMA || W == 256, "circulant variant: 256-lane workgroups");
    using S = ShellShape<N, W>;
    constexpr int N1 = S::N1, N2 = S::N2, C = W / N2;
    constexpr size_t shell_pts = (size_t)N * N / 2;
    stage_exp_table<N>(etab, eneg, lane);

    // The theta side of the shell moves straight between HBM and registers in
    // the theta layout (row segments, as the theta kernel does).  At N = 128
    // the phi side does too, in the phi layout (ring pieces of 64 bytes, as
    // the phi kernel does), so LDS only carries the exchange between the two
    // layouts (fused forward 448 -> 431 us on the dense n_phi = 128 grid,
    // grmhd 34 -> 32 us); at N = 32 and 64 (ring pieces of 32 and 64 bytes)
    // the phi side is staged through LDS with contiguous accesses, which
    // measured as fast or faster.  The circulant (MFMA) variant stages whole
    // shells on both sides.
    constexpr bool theta_direct = !MFMA, phi_direct = !MFMA && N >= 128;
    // the first pass's input and the last pass's output are staged with
    // contiguous accesses unless that side moves directly
    constexpr bool stage_in = ADJ ? !phi_direct : !theta_direct;
    constexpr bool stage_out = ADJ ? !theta_direct : !phi_direct;
    const int us = lane / S::lanes;
    const bool valid_s = us < n_valid;
    const size_t base_s = valid_s ? (size_t)items[us].shell * shell_pts : 0;
    cplx v[N1];

    // theta layout
    const int pt = lane % C, tt = lane / C, ut = pt / S::lines, kr = pt % S::lines;
    const bool valid_t = ut < n_valid;
    const ThetaItem it = valid_t ? items[ut] : ThetaItem{0, 0, 0.0};
    const double sgn = (it.flags & kFlagOddParity) ? -1.0 : 1.0;
    const size_t base_t = valid_t ? (size_t)it.shell * shell_pts : 0;
    double *sb_t = lds + ut * S::stride;

    if constexpr (stage_in) {
        shell_stage<N, true, W>(in, out, lds + us * S::stride, v, base_s, valid_s, lane % S::lanes);
        __syncthreads();
    }
    // phi layout
    const int tp = lane % N2, pp = lane / N2, up = pp / S::lines, j = pp % S::lines;
    const bool valid_p = up < n_valid;
    const int shell_p = valid_p ? items[up].shell : 0;
    const size_t base_p = (size_t)shell_p * shell_pts;
    const int kind_p = valid_p ? (items[up].flags & kKindMask) : 0;
    const double c_p = valid_p ? ring_c[up * S::lines + j] : INFINITY;
    double *sb_p = lds + up * S::stride;

    auto theta_filter = [&]() {
        double *L = lds + pt * line_stride<N1, N2, HYB>();
        int ka = it.flags & kKindMask, kb = ka;
        bool mixed = false;
        if constexpr (HYB) {
            const size_t dline = (size_t)it.shell * (size_t)(N / 2);
            hybrid_kinds<N1, N2, false>(v, tt, L, flags, pt, C, valid_t, ka, dline + kr,
                                 dline + kr + S::lines, ht, &ka, &kb, &mixed);
        }
        filter_line<N1, N2, HYB>(v, tt, ka, kb, mixed, valid_t ? it.c : INFINITY, L, tw, etab);
    };
    auto phi_filter = [&]() {
        double *L = lds + pp * line_stride<N1, N2, HYB>();
        int ka = kind_p, kb = ka;
        bool mixed = false;
        if constexpr (HYB) {
            const size_t ring = (size_t)shell_p * (size_t)(N / 2) + j;
            hybrid_kinds<N1, N2, true>(v, tp, L, flags, pp, C, valid_p, ka, ring,
                                 ring + (size_t)(N / 2 - 1 - 2 * j), hp, &ka, &kb, &mixed);
        }
        filter_line<N1, N2, HYB, true>(v, tp, ka, kb, mixed, c_p, L, tw, etab);
        // the phi line filter synchronises each line's wave only; its LDS
        // scratch overlaps the staging area and other lines' scratch
        __syncthreads();
    };

    // the theta pass on the staged shells, ending with their contents updated
    // (no trailing barrier)
    auto theta_pass = [&]() {
        if constexpr (MFMA) {
            constexpr int K = N / 2, SH = S::shells;
            double *fq = gaux, *cosd = gaux + SH * (N / 2 + 1), *cvec = cosd + N;
            shell_circulants<N, SH>(items, n_valid, tw, etab, fq, cosd, cvec, lane);
            dv4 acc[gemm_tiles_per_wave<N, SH>()];
            auto sign = [&](int sh) { return (items[sh].flags & kFlagOddParity) ? -1.0 : 1.0; };
            shell_gemm<N, SH>(cvec, n_valid, lane, acc, [&](int sh, int m, int k, bool first) {
                const double *sb = lds + sh * S::stride;
                return first ? sb[m * S::row + k] : sign(sh) * sb[(N - 1 - m) * S::row + K + k];
            });
            __syncthreads();
            shell_gemm_results<N, SH>(acc, n_valid, lane, [&](int sh, int n, int k, double y) {
                double *sb = lds + sh * S::stride;
                if (n < N / 2)
                    sb[n * S::row + k] = y;
                else
                    sb[(N - 1 - n) * S::row + K + k] = sign(sh) * y;
            });
        } else if constexpr (!ADJ) {
            // forward: the lines come from HBM, the result goes to the staging area
            shell_theta_hbm<N, true, W>(in, out, base_t, v, tt, kr, sgn, valid_t);
            theta_filter();
            shell_theta_io<N, true, W>(v, sb_t, tt, kr, sgn);
        } else {
            // adjoint: the lines come from the staging area, the result goes to HBM
            shell_theta_io<N, false, W>(v, sb_t, tt, kr, sgn);
            __syncthreads();
            theta_filter();
            shell_theta_hbm<N, false, W>(in, out, base_t, v, tt, kr, sgn, valid_t);
        }
    };

    if constexpr (!ADJ) {
        theta_pass();
        __syncthreads();
        shell_phi_io<N, false, W>(v, sb_p, tp, j);
        __syncthreads();
        phi_filter();
        if constexpr (phi_direct)
            shell_phi_hbm<N, false>(in, out, base_p, v, tp, j, valid_p);
        else
            shell_phi_io<N, true, W>(v, sb_p, tp, j);
    } else {
        if constexpr (phi_direct) {
            shell_phi_hbm<N, true>(in, out, base_p, v, tp, j, valid_p);
            __syncthreads();                    // the e^{-k} table staged above
        } else {
            shell_phi_io<N, false, W>(v, sb_p, tp, j);
            __syncthreads();
        }
        phi_filter();
        shell_phi_io<N, true, W>(v, sb_p, tp, j);
        __syncthreads();
        theta_pass();
    }
    if constexpr (stage_out) {
        __syncthreads();
        shell_stage<N, false, W>(in, out, lds + us * S::stride, v, base_s, valid_s, lane % S::lanes);
    }
}

}  // namespace sphfilt

namespace sphfilt {

// The hybrid-capable theta and phi kernels fit two waves per SIMD (at most
// 256 registers) without spilling; two waves beat one by a wide margin (the
// share with 8 hybrid fields ran 0.81 against 1.25 ms per forward filter
// when the two-wave form still spilled a little).

// Waves per SIMD a pass kernel asks the compiler for (it caps the registers
// per lane at 512 / waves).  The hybrid-capable instances: two, where two
// workgroups' line scratch (a whole spectrum per line) fits in LDS, else one.
// The plain instances: no target (they fit two or more waves by themselves).
template <int N, int LINES, bool HYB>
constexpr int pass_waves()
{
    constexpr int bytes = 8 * LINES * line_stride<Split<N>::N1, Split<N>::N2, HYB>();
    return HYB && 2 * bytes <= 160 * 1024 - 4096 ? 2 : 1;
}

}  // namespace sphfilt
