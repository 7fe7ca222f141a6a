// theta_gemm.h -- the theta filter of whole shells as a dense circulant
// product on the matrix cores (FP64 MFMA), for grids with n_phi = 2 n_theta
// = N in {32, 64} (device side).
//
// On one extended theta line of length N the theta filter (FFT, mask,
// inverse FFT; arXiv:2305.01537, Sec. II.A, theta filter) is the circular
// convolution
//   y[n] = sum_m c[(n - m) mod N] g[m],
//   c[d] = (1/N) sum_{q=0}^{N-1} f(|q|; l_max) cos(2 pi q d / N),
// c being the inverse transform of the mask (real and even in q, so c is
// real and c[d] = c[N - d]).  Every extended line of a shell (meridian pairs
// k and k + N/2, k < K = N/2) has the same l_max, so the shell's theta pass is
// one matrix product Y = C G, C the N x N circulant, G the N x K matrix whose
// column k is the extended line of pair k:
//   G[n][k] = X[n][k]                  for n <  N/2,
//   G[n][k] = s X[N - 1 - n][k + K]    for n >= N/2   (s: parity sign),
// and Y is written back through the same map.  This costs 2N flops per point
// against ~5 log2 N for the FFT, but runs as V_MFMA_F64_16X16X4_F64 tiles
// with no transposes or twiddles; a variant, chosen per plan or batch.
//
// Operand layout of __builtin_amdgcn_mfma_f64_16x16x4f64 (D += A B, one
// wave), as measured on gfx950 with one-hot operands: lane l holds
// A[l % 16][l / 16] (A is 16 x 4), B[l / 16][l % 16] (B is 4 x 16) and, in
// register r, D[l / 16 + 4 r][l % 16] (D is 16 x 16).
#pragma once
#include "fft_core.h"
#include "sphfilt_internal.h"

#include <cmath>

namespace sphfilt {

typedef double dv4 __attribute__((ext_vector_type(4)));

template <int N>
struct GemmShape {
    static_assert(N == 32 || N == 64, "the circulant product is built for lines of 32 and 64");
    static constexpr int K = N / 2;        // columns of G: meridian pairs
    static constexpr int RB = N / 16;      // 16-row blocks of Y
    static constexpr int CT = K / 16;      // 16-column tiles of Y
    static constexpr int KS = N / 4;       // 4-deep steps of one tile's product
    static constexpr int TILES = RB * CT;  // tiles per shell
};

// Mask factor f(|q|; c) of one mode, without the 1/N (kinds as in
// apply_mask: 0 exponential, 1 Gaussian, 2 sharp; etab holds e^{-k}).
template <int N>
__device__ __forceinline__ double mask_factor(int kind, int qhat, double c, const double *etab)
{
    if (kind == 1) {
        const double u = (double)qhat / (c + 1.0);
        return exp(-0.10536051565782630123 * u * u);
    }
    const int m = c >= (double)N ? N : (int)floor(c);
    if (qhat <= m) return 1.0;
    return kind == 0 ? exp((c - (double)m) - 1.0) * etab[qhat - m - 1] : 0.0;
}

// Circulants of the workgroup's S shells (items[0, n_valid)) into
// cvec[S][N]: first the N/2 + 1 distinct mask factors of each shell into
// fq[S][N/2 + 1], then c[d] from them with the cosine table cosd[j] =
// cos(2 pi j / N) = tw[j].re.  All lanes call this together; it ends with a
// barrier.  The caller staged etab (e^{-k}, k <= N/2) before a barrier.
template <int N, int S>
__device__ __forceinline__ void shell_circulants(const ThetaItem *__restrict__ items, int n_valid,
                                                 const Twiddle *__restrict__ tw,
                                                 const double *etab, double *fq, double *cosd,
                                                 double *cvec, int lane)
{
    constexpr int H = N / 2 + 1;
    for (int i = lane; i < S * H; i += (int)blockDim.x) {
        const int s = i / H, q = i % H;
        fq[i] = s < n_valid ? mask_factor<N>(items[s].flags & kKindMask, q, items[s].c, etab) : 0.0;
    }
    for (int j = lane; j < N; j += (int)blockDim.x) cosd[j] = tw[j].re;
    __syncthreads();
    for (int i = lane; i < S * N; i += (int)blockDim.x) {
        const int s = i / N, d = i % N;
        const double *f = fq + s * H;
        double acc = 0.0;
        for (int q = 1; q < N / 2; ++q) acc += f[q] * cosd[(q * d) % N];
        const double nyq = (d & 1) ? -f[N / 2] : f[N / 2];
        cvec[i] = (f[0] + nyq + 2.0 * acc) * (1.0 / N);
    }
    __syncthreads();
}

// The products of one wave.  The workgroup's S shells have S RB (shell, row
// block) groups of CT tiles each; wave w takes groups [w GW, (w + 1) GW),
// GW = S RB / 4, loads the group's operand A (KS values of the circulant per
// lane) once and runs its CT tiles.  Operand B (G) comes from
// `load_g(shell, m, k, first_half)` (first_half: m < N/2).  The result of the
// wave's tile u = g CT + ct, lane l, register r is
// Y[shell][16 rb + l / 16 + 4 r][16 ct + l % 16], left in acc[u].  Shells
// s >= n_valid are skipped.  Wave-uniform control flow; no barrier inside.
template <int N, int S>
constexpr int gemm_tiles_per_wave() { return S * GemmShape<N>::TILES / 4; }

template <int N, int S, typename LoadG>
__device__ __forceinline__ void shell_gemm(const double *cvec, int n_valid, int lane,
                                           dv4 (&acc)[gemm_tiles_per_wave<N, S>()], LoadG &&load_g)
{
    using G = GemmShape<N>;
    constexpr int GW = S * G::RB / 4;
    static_assert(S * G::RB % 4 == 0, "four waves share the row blocks evenly");
    const int w = lane / 64, l = lane % 64;
    const int i = l % 16, kk = l / 16;
    static_for<0, GW>([&](auto gg) {
        constexpr int g = decltype(gg)::value;
        const int grp = w * GW + g;
        const int sh = grp / G::RB, rb = grp % G::RB;
        static_for<0, G::CT>([&](auto cc) { acc[g * G::CT + decltype(cc)::value] = dv4{0.0, 0.0, 0.0, 0.0}; });
        if (sh < n_valid) {
            const double *c = cvec + sh * N;
            double a[G::KS];
            static_for<0, G::KS>([&](auto tt) {
                constexpr int t = decltype(tt)::value;
                // A[i][kk] = C[16 rb + i][4 t + kk] = c[(16 rb + i - 4 t - kk) mod N]
                a[t] = c[(16 * rb + i - 4 * t - kk + 2 * N) % N];
            });
            static_for<0, G::CT>([&](auto cc) {
                constexpr int ct = decltype(cc)::value;
                static_for<0, G::KS>([&](auto tt) {
                    constexpr int t = decltype(tt)::value;
                    const double b = load_g(sh, 4 * t + kk, 16 * ct + i, t < G::KS / 2);
                    acc[g * G::CT + ct] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b, acc[g * G::CT + ct], 0, 0, 0);
                });
            });
        }
    });
}

// Hand every result of shell_gemm to `store_y(shell, n, k, value)`, for the
// valid shells.
template <int N, int S, typename StoreY>
__device__ __forceinline__ void shell_gemm_results(const dv4 (&acc)[gemm_tiles_per_wave<N, S>()],
                                                   int n_valid, int lane, StoreY &&store_y)
{
    using G = GemmShape<N>;
    constexpr int GW = S * G::RB / 4;
    const int w = lane / 64, l = lane % 64;
    static_for<0, GW>([&](auto gg) {
        constexpr int g = decltype(gg)::value;
        const int grp = w * GW + g;
        const int sh = grp / G::RB, rb = grp % G::RB;
        if (sh < n_valid) {
            static_for<0, G::CT>([&](auto cc) {
                constexpr int ct = decltype(cc)::value;
                static_for<0, 4>([&](auto rr) {
                    constexpr int r = decltype(rr)::value;
                    store_y(sh, 16 * rb + l / 16 + 4 * r, 16 * ct + l % 16, acc[g * G::CT + ct][r]);
                });
            });
        }
    });
}

}  // namespace sphfilt
