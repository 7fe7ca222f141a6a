// fft_core.h -- FP64 complex FFT building blocks for gfx950 (device side).
//
// A line of length N = N1 * N2 is spread over N2 lanes; lane t holds the N1
// elements x[N2*n1 + t].  One filtered line is the four-step transform
//
//   X[k1 + N1 k2] = sum_n2 W_N2^{n2 k2} W_N^{n2 k1} sum_n1 x[N2 n1 + n2] W_N1^{n1 k1}
//
// done as: an N1-point DFT in registers, a twiddle by W_N^{t k1}, one LDS
// transpose, ceil(N1/N2) rows of N2-point DFTs per lane in registers (the
// last row partly padding when N2 does not divide N1); then the mask; then
// the same steps in reverse (inverse DFTs, conjugate twiddles, one LDS
// transpose) so that every lane ends up with its own N1 input positions again.
// Two HBM touches per line (load, store) and two LDS transposes in between.
//
// The small in-register DFTs are radix-2 decimation in frequency with their
// twiddles as compile-time constants, with one radix-3 or radix-5 stage in
// front for sizes 3 * 2^k and 5 * 2^k; the output permutations are register
// renamings, so they cost nothing.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace sphfilt {

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
// a * w
__device__ __forceinline__ cplx cmul(cplx a, cplx w)
{
    return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}
// a * conj(w)
__device__ __forceinline__ cplx cmulc(cplx a, cplx w)
{
    return {a.re * w.re + a.im * w.im, a.im * w.re - a.re * w.im};
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// cos(a pi / 32) for a in [0, 16], to 25 digits (the compiler rounds to FP64).
constexpr double cos_pi32_q(int a)
{
    return a == 0    ? 1.0
           : a == 1  ? 0.9951847266721968862448370
           : a == 2  ? 0.9807852804032304491261822
           : a == 3  ? 0.9569403357322088649357979
           : a == 4  ? 0.9238795325112867561281832
           : a == 5  ? 0.8819212643483550297127569
           : a == 6  ? 0.8314696123025452370787884
           : a == 7  ? 0.7730104533627369608109066
           : a == 8  ? 0.7071067811865475244008444
           : a == 9  ? 0.6343932841636454982151716
           : a == 10 ? 0.5555702330196022247428308
           : a == 11 ? 0.4713967368259976485563876
           : a == 12 ? 0.3826834323650897717284600
           : a == 13 ? 0.2902846772544623676361924
           : a == 14 ? 0.1950903220161282678482849
           : a == 15 ? 0.0980171403295606019941956
                     : 0.0;
}

// cos(a pi / 32) for any integer a, by the quadrant symmetries.
constexpr double cos_pi32(int a)
{
    a = ((a % 64) + 64) % 64;
    return a <= 16 ? cos_pi32_q(a) : a <= 32 ? -cos_pi32_q(32 - a) : a <= 48 ? -cos_pi32_q(a - 32) : cos_pi32_q(64 - a);
}
constexpr double sin_pi32(int a) { return cos_pi32(16 - a); }

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int x, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1) << (bits - 1 - b);
    return r;
}

// a * W_M^I with W_M = exp(-2 pi i / M) (forward) or exp(+2 pi i / M) (INV).
// M divides 64; trivial factors (1, -1, +-i, (+-1 +-i)/sqrt2) take no multiply
// by a general constant.
template <int M, int I, bool INV>
__device__ __forceinline__ cplx twiddle_const(cplx a)
{
    static_assert(64 % M == 0, "twiddle order must divide 64");
    constexpr int ang = ((64 / M) * I) % 64;             // angle = ang * pi / 32
    constexpr int e = INV ? ang : (64 - ang) % 64;       // exp(i e pi / 32)
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 32) {
        return {-a.re, -a.im};
    } else if constexpr (e == 16) {                      // * i
        return {-a.im, a.re};
    } else if constexpr (e == 48) {                      // * -i
        return {a.im, -a.re};
    } else if constexpr (e % 16 == 8) {                  // * (+-1 +-i)/sqrt2
        constexpr double h = 0.7071067811865475244008444;
        constexpr double cr = cos_pi32(e) > 0 ? h : -h;
        constexpr double ci = sin_pi32(e) > 0 ? h : -h;
        if constexpr (cr == ci)
            return {cr * (a.re - a.im), cr * (a.re + a.im)};
        else
            return {cr * (a.re + a.im), cr * (a.im - a.re)};
    } else {
        constexpr double c = cos_pi32(e), s = sin_pi32(e);
        return {a.re * c - a.im * s, a.re * s + a.im * c};
    }
}

// cos(a pi / D) for D = 12 (a in [0, 6]: (sqrt6 +- sqrt2)/4, sqrt3/2,
// sqrt2/2, 1/2) and D = 20 (a in [0, 10]), to 25 digits; any integer a by the
// quadrant symmetries.  The twiddles of the transforms whose size divides 24
// or 40.
template <int D>
constexpr double cos_frac_q(int a)
{
    if constexpr (D == 12) {
        return a == 0   ? 1.0
               : a == 1 ? 0.9659258262890682867497432
               : a == 2 ? 0.8660254037844386467637232
               : a == 3 ? 0.7071067811865475244008444
               : a == 4 ? 0.5
               : a == 5 ? 0.2588190451025207623488988
                        : 0.0;
    } else {
        static_assert(D == 20, "tables for pi/12 and pi/20");
        return a == 0   ? 1.0
               : a == 1 ? 0.9876883405951377261900402
               : a == 2 ? 0.9510565162951535721164393
               : a == 3 ? 0.8910065241883678623597096
               : a == 4 ? 0.8090169943749474241022934
               : a == 5 ? 0.7071067811865475244008444
               : a == 6 ? 0.5877852522924731291687060
               : a == 7 ? 0.4539904997395467915604084
               : a == 8 ? 0.3090169943749474241022934
               : a == 9 ? 0.1564344650402308690101053
                        : 0.0;
    }
}
template <int D>
constexpr double cos_frac(int a)
{
    a = ((a % (2 * D)) + 2 * D) % (2 * D);
    return a <= D / 2 ? cos_frac_q<D>(a)
           : a <= D   ? -cos_frac_q<D>(D - a)
           : a <= 3 * D / 2 ? -cos_frac_q<D>(a - D)
                            : cos_frac_q<D>(2 * D - a);
}
template <int D>
constexpr double sin_frac(int a) { return cos_frac<D>(D / 2 - a); }

// a * exp(-i A pi / D) (forward) or exp(+i A pi / D) (INV).
template <int D, int A, bool INV>
__device__ __forceinline__ cplx twiddle_frac(cplx a)
{
    constexpr int a0 = ((A % (2 * D)) + 2 * D) % (2 * D);
    constexpr int e = INV ? a0 : (2 * D - a0) % (2 * D);   // exp(i e pi / D)
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == D) {
        return {-a.re, -a.im};
    } else if constexpr (2 * e == D) {
        return {-a.im, a.re};
    } else if constexpr (2 * e == 3 * D) {
        return {a.im, -a.re};
    } else {
        constexpr double c = cos_frac<D>(e), s = sin_frac<D>(e);
        return {a.re * c - a.im * s, a.re * s + a.im * c};
    }
}

// 3-point DFT of (x0, x1, x2) in place: with s = x1 + x2 and d = x1 - x2,
// X0 = x0 + s and X1, X2 = x0 - s/2 -+ i (sqrt3/2) d (forward; INV swaps the
// signs of the i (sqrt3/2) d term).
template <bool INV>
__device__ __forceinline__ void dft3(cplx &x0, cplx &x1, cplx &x2)
{
    constexpr double h = 0.8660254037844386467637232;   // sqrt(3)/2
    const cplx s = cadd(x1, x2), d = csub(x1, x2);
    const cplx m = {x0.re - 0.5 * s.re, x0.im - 0.5 * s.im};
    const cplx j = INV ? cplx{-h * d.im, h * d.re} : cplx{h * d.im, -h * d.re};   // -+i h d
    x0 = cadd(x0, s);
    x1 = cadd(m, j);
    x2 = csub(m, j);
}

// 5-point DFT in place.  With W = exp(-2 pi i / 5), c1 = cos(2pi/5),
// c2 = cos(4pi/5), s1 = sin(2pi/5), s2 = sin(4pi/5), u1 = x1 + x4,
// u2 = x2 + x3, d1 = x1 - x4, d2 = x2 - x3 (W^4 = conj W, W^3 = conj W^2):
//   X0 = x0 + u1 + u2
//   X1, X4 = x0 + c1 u1 + c2 u2 -+ i (s1 d1 + s2 d2)
//   X2, X3 = x0 + c2 u1 + c1 u2 -+ i (s2 d1 - s1 d2)
// (forward; INV swaps the signs of the i terms).
template <bool INV>
__device__ __forceinline__ void dft5(cplx &x0, cplx &x1, cplx &x2, cplx &x3, cplx &x4)
{
    constexpr double c1 = 0.3090169943749474241022934, c2 = -0.8090169943749474241022934;
    constexpr double s1 = 0.9510565162951535721164393, s2 = 0.5877852522924731291687060;
    const cplx u1 = cadd(x1, x4), u2 = cadd(x2, x3), d1 = csub(x1, x4), d2 = csub(x2, x3);
    const cplx a1 = {x0.re + c1 * u1.re + c2 * u2.re, x0.im + c1 * u1.im + c2 * u2.im};
    const cplx a2 = {x0.re + c2 * u1.re + c1 * u2.re, x0.im + c2 * u1.im + c1 * u2.im};
    const cplx b1 = {s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im};
    const cplx b2 = {s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im};
    // -i b = (b.im, -b.re); +i b = (-b.im, b.re)
    const cplx j1 = INV ? cplx{-b1.im, b1.re} : cplx{b1.im, -b1.re};
    const cplx j2 = INV ? cplx{-b2.im, b2.re} : cplx{b2.im, -b2.re};
    x0 = cadd(x0, cadd(u1, u2));
    x1 = cadd(a1, j1);
    x4 = csub(a1, j1);
    x2 = cadd(a2, j2);
    x3 = csub(a2, j2);
}

// In-register DFT of size R on v[OFF + STRIDE*i], i in [0, R): natural order
// in, natural order out.  Forward: exp(-2 pi i n k / R); INV: exp(+...),
// unnormalised.  R is a power of two up to 64, or P = 3 or 5 times a power of
// two B with R dividing 24 (P = 3) or 40 (P = 5): then, with n = b + B a and
// k = ka + P kb,
//   X[ka + P kb] = sum_b W_B^{b kb} W_R^{b ka} sum_a x[b + B a] W_P^{a ka},
// i.e. P-point DFTs over a, twiddles W_R^{b ka}, B-point DFTs over b, and a
// register renaming to natural order.
template <int R, bool INV, int OFF = 0, int STRIDE = 1, int NV>
__device__ __forceinline__ void dft_reg(cplx (&v)[NV])
{
    if constexpr (R % 3 == 0 || R % 5 == 0) {
        constexpr int P = R % 3 == 0 ? 3 : 5, D = P == 3 ? 12 : 20;
        static_assert((2 * D) % R == 0, "an odd-radix transform size must divide 24 or 40");
        constexpr int B = R / P;
        static_for<0, B>([&](auto bb) {
            constexpr int b = decltype(bb)::value;
            constexpr int p0 = OFF + STRIDE * b;
            if constexpr (P == 3) {
                dft3<INV>(v[p0], v[p0 + STRIDE * B], v[p0 + 2 * STRIDE * B]);
            } else {
                dft5<INV>(v[p0], v[p0 + STRIDE * B], v[p0 + 2 * STRIDE * B], v[p0 + 3 * STRIDE * B],
                          v[p0 + 4 * STRIDE * B]);
            }
            // W_R^{b ka} = exp(-+ i (2 D / R) b ka pi / D)
            static_for<1, P>([&](auto kk) {
                constexpr int ka = decltype(kk)::value;
                v[p0 + ka * STRIDE * B] = twiddle_frac<D, (2 * D / R) * b * ka, INV>(v[p0 + ka * STRIDE * B]);
            });
        });
        static_for<0, P>([&](auto aa) {
            dft_reg<B, INV, OFF + STRIDE * B * decltype(aa)::value, STRIDE>(v);
        });
        // X[ka + P kb] sits at position ka B + kb
        cplx tmp[R];
        static_for<0, R>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            tmp[k] = v[OFF + STRIDE * ((k % P) * B + k / P)];
        });
        static_for<0, R>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            v[OFF + STRIDE * k] = tmp[k];
        });
        return;
    }
    static_assert(R % 3 == 0 || R % 5 == 0 || ((R & (R - 1)) == 0 && R >= 1 && R <= 64),
                  "radix must be a power of two <= 64");
    if constexpr (R > 1 && R % 3 != 0 && R % 5 != 0) {
        // decimation in frequency: spans R/2, R/4, ..., 1; output bit-reversed
        static_for<0, ilog2(R)>([&](auto st) {
            constexpr int span = R >> (decltype(st)::value + 1);
            static_for<0, R / (2 * span)>([&](auto bb) {
                static_for<0, span>([&](auto ii) {
                    constexpr int i = decltype(ii)::value;
                    constexpr int p = OFF + STRIDE * (decltype(bb)::value * 2 * span + i);
                    constexpr int q = p + STRIDE * span;
                    cplx a = v[p], b = v[q];
                    v[p] = cadd(a, b);
                    v[q] = twiddle_const<2 * span, i, INV>(csub(a, b));
                });
            });
        });
        // bit-reversed -> natural: a register renaming after unrolling
        cplx tmp[R];
        static_for<0, R>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            tmp[k] = v[OFF + STRIDE * bitrev(k, ilog2(R))];
        });
        static_for<0, R>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            v[OFF + STRIDE * k] = tmp[k];
        });
    }
}

}  // namespace sphfilt
