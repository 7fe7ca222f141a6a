// fft_core.h -- FP64 complex FFT building blocks for gfx950 (device side).
//
// A line of length N = N1 * N2 is spread over N2 lanes; lane t holds the N1
// elements x[N2*n1 + t].  One filtered line is the four-step transform
//
//   X[k1 + N1 k2] = sum_n2 W_N2^{n2 k2} W_N^{n2 k1} sum_n1 x[N2 n1 + n2] W_N1^{n1 k1}
//
// done as: an N1-point DFT in registers, a twiddle by W_N^{t k1}, one LDS
// transpose, N1/N2 independent N2-point DFTs in registers; then the mask;
// then the same steps in reverse (inverse DFTs, conjugate twiddles, one LDS
// transpose) so that every lane ends up with its own N1 input positions again.
// Two HBM touches per line (load, store) and two LDS transposes in between.
//
// The small in-register DFTs are radix-2 decimation in frequency with their
// twiddles as compile-time constants; the output permutation is a register
// renaming, so it costs nothing.
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

// cos(a pi / 12) for a in [0, 6] ((sqrt6 +- sqrt2)/4, sqrt3/2, sqrt2/2, 1/2),
// to 25 digits; and for any integer a by the quadrant symmetries.
constexpr double cos_pi12_q(int a)
{
    return a == 0   ? 1.0
           : a == 1 ? 0.9659258262890682867497432
           : a == 2 ? 0.8660254037844386467637232
           : a == 3 ? 0.7071067811865475244008444
           : a == 4 ? 0.5
           : a == 5 ? 0.2588190451025207623488988
                    : 0.0;
}
constexpr double cos_pi12(int a)
{
    a = ((a % 24) + 24) % 24;
    return a <= 6 ? cos_pi12_q(a) : a <= 12 ? -cos_pi12_q(12 - a) : a <= 18 ? -cos_pi12_q(a - 12) : cos_pi12_q(24 - a);
}
constexpr double sin_pi12(int a) { return cos_pi12(6 - a); }

// a * exp(-i A pi / 12) (forward) or exp(+i A pi / 12) (INV): the twiddles of
// the transforms whose size divides 24.
template <int A, bool INV>
__device__ __forceinline__ cplx twiddle_pi12(cplx a)
{
    constexpr int a0 = ((A % 24) + 24) % 24;
    constexpr int e = INV ? a0 : (24 - a0) % 24;         // exp(i e pi / 12)
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 12) {
        return {-a.re, -a.im};
    } else if constexpr (e == 6) {
        return {-a.im, a.re};
    } else if constexpr (e == 18) {
        return {a.im, -a.re};
    } else {
        constexpr double c = cos_pi12(e), s = sin_pi12(e);
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

// In-register DFT of size R on v[OFF + STRIDE*i], i in [0, R): natural order
// in, natural order out.  Forward: exp(-2 pi i n k / R); INV: exp(+...),
// unnormalised.  R is a power of two up to 64, or 3 times a power of two
// dividing 24 (R = 3, 6, 12, 24): then, with R = 3 B, n = b + B a and
// k = ka + 3 kb,
//   X[ka + 3 kb] = sum_b W_B^{b kb} W_R^{b ka} sum_a x[b + B a] W_3^{a ka},
// i.e. 3-point DFTs over a, twiddles W_R^{b ka}, B-point DFTs over b, and a
// register renaming to natural order.
template <int R, bool INV, int OFF = 0, int STRIDE = 1, int NV>
__device__ __forceinline__ void dft_reg(cplx (&v)[NV])
{
    if constexpr (R % 3 == 0) {
        static_assert(24 % R == 0, "a radix-3 transform size must divide 24");
        constexpr int B = R / 3;
        static_for<0, B>([&](auto bb) {
            constexpr int b = decltype(bb)::value;
            constexpr int p0 = OFF + STRIDE * b, p1 = p0 + STRIDE * B, p2 = p1 + STRIDE * B;
            dft3<INV>(v[p0], v[p1], v[p2]);
            // W_R^{b ka} = exp(-+ i (24 / R) b ka pi / 12)
            v[p1] = twiddle_pi12<(24 / R) * b, INV>(v[p1]);
            v[p2] = twiddle_pi12<(24 / R) * 2 * b, INV>(v[p2]);
        });
        static_for<0, 3>([&](auto aa) {
            dft_reg<B, INV, OFF + STRIDE * B * decltype(aa)::value, STRIDE>(v);
        });
        // X[ka + 3 kb] sits at position ka B + kb
        cplx tmp[R];
        static_for<0, R>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            tmp[k] = v[OFF + STRIDE * ((k % 3) * B + k / 3)];
        });
        static_for<0, R>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            v[OFF + STRIDE * k] = tmp[k];
        });
        return;
    }
    static_assert(R % 3 == 0 || ((R & (R - 1)) == 0 && R >= 1 && R <= 64),
                  "radix must be a power of two <= 64");
    if constexpr (R > 1 && R % 3 != 0) {
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
