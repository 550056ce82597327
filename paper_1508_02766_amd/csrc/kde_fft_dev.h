// Device building blocks of the FFT convolution kernels: complex arithmetic,
// the compile-time twiddle tables, the Stockham line transform in LDS (lengths
// 2^k with radix-16/8/4/2 stages, 3 x 2^k with a radix-12 stage first), and the bodies of the row (contiguous axis) and column (strided
// axis) passes. Included by the single-instance launchers (kde_fft.hip) and
// the batched ones (kde_fft_batch.hip), so both run the same device code.
#pragma once

#include "kde_internal.h"

namespace kde {
namespace {


// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------

template <typename R>
struct cpx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
// These sources build without floating-point contraction, so every fused
// multiply-add is written out: the rounding of a product never depends on
// how the compiler fused the surrounding kernel, and the single-instance and
// batched kernels give identical bits.
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
__device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
    return {fmaR(a.re, b.re, -(a.im * b.im)), fmaR(a.re, b.im, a.im * b.re)};
}
template <typename R>
__device__ __forceinline__ cpx<R> scal(cpx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ cpx<R> conj(cpx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> mul_minus_i(cpx<R> a) { return {a.im, -a.re}; }

// ---------------------------------------------------------------------------
// compile-time twiddle table: exp(-2 pi i k / 4096), k = 0..4095
// ---------------------------------------------------------------------------

constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series on [0, pi/4]; 14 terms leave a truncation error far below
// one FP64 ulp there.
constexpr double sin_series(double x) {
    double x2 = x * x, term = x, s = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        s += term;
    }
    return s;
}
constexpr double cos_series(double x) {
    double x2 = x * x, term = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        s += term;
    }
    return s;
}

struct SinCos {
    double s, c;
};

// sin and cos of 2 pi k / N with the argument reduced exactly in integers
// (quadrant, then reflection about pi/4), N divisible by 8.
constexpr SinCos sincos_turn(long k, long N) {
    k %= N;
    if (k < 0) k += N;
    const long quarter = N / 4;
    const long quad = k / quarter, r = k % quarter;
    double s = 0.0, c = 0.0;
    if (2 * r <= quarter) {
        const double x = 2.0 * kPi * static_cast<double>(r) / static_cast<double>(N);
        s = sin_series(x);
        c = cos_series(x);
    } else {
        const double x = 2.0 * kPi * static_cast<double>(quarter - r) / static_cast<double>(N);
        s = cos_series(x);
        c = sin_series(x);
    }
    switch (quad) {
        case 0: return {s, c};
        case 1: return {c, -s};
        case 2: return {-s, -c};
        default: return {-c, s};
    }
}

template <typename R>
struct TwiddleTable {
    cpx<R> w[kMaxP];
};

template <typename R>
constexpr TwiddleTable<R> make_twiddles() {
    TwiddleTable<R> t{};
    for (int k = 0; k < kMaxP; ++k) {
        const SinCos v = sincos_turn(k, kMaxP);
        t.w[k] = cpx<R>{static_cast<R>(v.c), static_cast<R>(-v.s)};
    }
    return t;
}

__device__ constexpr TwiddleTable<float> g_tw32 = make_twiddles<float>();
__device__ constexpr TwiddleTable<double> g_tw64 = make_twiddles<double>();

template <typename R>
__device__ __forceinline__ cpx<R> twiddle(int k);
template <>
__device__ __forceinline__ cpx<float> twiddle<float>(int k) { return g_tw32.w[k]; }
template <>
__device__ __forceinline__ cpx<double> twiddle<double>(int k) { return g_tw64.w[k]; }

// exp(-2 pi i k / 3072), k = 0..3071: the twiddles of the lengths 3 x 2^k
template <typename R>
struct TwiddleTable3 {
    cpx<R> w[kMaxP3];
};

template <typename R>
constexpr TwiddleTable3<R> make_twiddles3() {
    TwiddleTable3<R> t{};
    for (int k = 0; k < kMaxP3; ++k) {
        const SinCos v = sincos_turn(k, kMaxP3);
        t.w[k] = cpx<R>{static_cast<R>(v.c), static_cast<R>(-v.s)};
    }
    return t;
}

__device__ constexpr TwiddleTable3<float> g_tw32_3 = make_twiddles3<float>();
__device__ constexpr TwiddleTable3<double> g_tw64_3 = make_twiddles3<double>();

template <typename R>
__device__ __forceinline__ cpx<R> twiddle3(int k);
template <>
__device__ __forceinline__ cpx<float> twiddle3<float>(int k) { return g_tw32_3.w[k]; }
template <>
__device__ __forceinline__ cpx<double> twiddle3<double>(int k) { return g_tw64_3.w[k]; }

// Line lengths 3 x 2^k (a radix-12 first stage, then radix 4 and 2).
__host__ __device__ constexpr bool is_tri(int P) { return P % 3 == 0; }

// multiply by the compile-time constant exp(-2 pi i m / 12)
template <int m, typename R>
__device__ __forceinline__ cpx<R> rot12(cpx<R> a) {
    constexpr int mm = ((m % 12) + 12) % 12;
    if constexpr (mm == 0) {
        return a;
    } else if constexpr (mm == 3) {
        return mul_minus_i(a);
    } else if constexpr (mm == 6) {
        return cpx<R>{-a.re, -a.im};
    } else if constexpr (mm == 9) {
        return cpx<R>{-a.im, a.re};
    } else {
        constexpr SinCos v = sincos_turn(2 * mm, 24);
        return a * cpx<R>{static_cast<R>(v.c), static_cast<R>(-v.s)};
    }
}

// multiply by the compile-time constant exp(-2 pi i m / 16)
template <int m, typename R>
__device__ __forceinline__ cpx<R> rot16(cpx<R> a) {
    constexpr int mm = ((m % 16) + 16) % 16;
    if constexpr (mm == 0) {
        return a;
    } else if constexpr (mm == 4) {
        return mul_minus_i(a);
    } else if constexpr (mm == 8) {
        return cpx<R>{-a.re, -a.im};
    } else if constexpr (mm == 12) {
        return cpx<R>{-a.im, a.re};
    } else {
        constexpr SinCos v = sincos_turn(mm, 16);
        return a * cpx<R>{static_cast<R>(v.c), static_cast<R>(-v.s)};
    }
}

// ---------------------------------------------------------------------------
// register DFTs, forward sign, natural order in and out
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ void dft4(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {
    const cpx<R> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_minus_i(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

// length-3 DFT: X_1,2 = a0 - (a1 + a2)/2 -/+ i sin(2 pi/3) (a1 - a2)
template <typename R>
__device__ __forceinline__ void dft3(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2) {
    constexpr R h = static_cast<R>(sincos_turn(8, 24).s);   // sin(2 pi / 3)
    const cpx<R> s = a1 + a2, d = a1 - a2;
    const cpx<R> m{fmaR(R(-0.5), s.re, a0.re), fmaR(R(-0.5), s.im, a0.im)};
    const cpx<R> r{d.im * h, -(d.re * h)};   // -i sin(2 pi/3) (a1 - a2)
    a0 = a0 + s;
    a1 = m + r;
    a2 = m - r;
}

template <int RAD, typename R>
__device__ __forceinline__ void dft(cpx<R> (&a)[RAD]) {
    if constexpr (RAD == 2) {
        const cpx<R> t = a[0] - a[1];
        a[0] = a[0] + a[1];
        a[1] = t;
    } else if constexpr (RAD == 4) {
        dft4(a[0], a[1], a[2], a[3]);
    } else if constexpr (RAD == 8) {
        // even and odd halves, then the radix-2 combination with exp(-2 pi i k / 8)
        dft4(a[0], a[2], a[4], a[6]);
        dft4(a[1], a[3], a[5], a[7]);
        const cpx<R> o1 = rot16<2>(a[3]), o2 = rot16<4>(a[5]), o3 = rot16<6>(a[7]);
        const cpx<R> y0 = a[0] + a[1], y4 = a[0] - a[1];
        const cpx<R> y1 = a[2] + o1, y5 = a[2] - o1;
        const cpx<R> y2 = a[4] + o2, y6 = a[4] - o2;
        const cpx<R> y3 = a[6] + o3, y7 = a[6] - o3;
        a[0] = y0; a[1] = y1; a[2] = y2; a[3] = y3;
        a[4] = y4; a[5] = y5; a[6] = y6; a[7] = y7;
    } else if constexpr (RAD == 16) {
        // 16 = 4 x 4: length-4 DFTs over n1 (input n = 4 n1 + n2), twiddle
        // exp(-2 pi i n2 k1 / 16), length-4 DFTs over n2; output k = k1 + 4 k2.
        dft4(a[0], a[4], a[8], a[12]);
        dft4(a[1], a[5], a[9], a[13]);
        dft4(a[2], a[6], a[10], a[14]);
        dft4(a[3], a[7], a[11], a[15]);
        // a[n2 + 4 k1] now holds the inner result for (n2, k1)
        a[5] = rot16<1>(a[5]);
        a[6] = rot16<2>(a[6]);
        a[7] = rot16<3>(a[7]);
        a[9] = rot16<2>(a[9]);
        a[10] = rot16<4>(a[10]);
        a[11] = rot16<6>(a[11]);
        a[13] = rot16<3>(a[13]);
        a[14] = rot16<6>(a[14]);
        a[15] = rot16<9>(a[15]);
        dft4(a[0], a[1], a[2], a[3]);
        dft4(a[4], a[5], a[6], a[7]);
        dft4(a[8], a[9], a[10], a[11]);
        dft4(a[12], a[13], a[14], a[15]);
        // a[4 k1 + k2] holds output k1 + 4 k2: transpose the 4 x 4 block
        cpx<R> y[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) y[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = y[i];
    } else if constexpr (RAD == 12) {
        // 12 = 4 x 3: length-4 DFTs over n1 (input n = 3 n1 + n2), twiddle
        // exp(-2 pi i n2 k1 / 12), length-3 DFTs over n2; output k = k1 + 4 k2.
        dft4(a[0], a[3], a[6], a[9]);
        dft4(a[1], a[4], a[7], a[10]);
        dft4(a[2], a[5], a[8], a[11]);
        // a[n2 + 3 k1] now holds the inner result for (n2, k1)
        a[4] = rot12<1>(a[4]);
        a[5] = rot12<2>(a[5]);
        a[7] = rot12<2>(a[7]);
        a[8] = rot12<4>(a[8]);
        a[10] = rot12<3>(a[10]);
        a[11] = rot12<6>(a[11]);
        dft3(a[0], a[1], a[2]);
        dft3(a[3], a[4], a[5]);
        dft3(a[6], a[7], a[8]);
        dft3(a[9], a[10], a[11]);
        // a[3 k1 + k2] holds output k1 + 4 k2
        cpx<R> y[12];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) y[k1 + 4 * k2] = a[3 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 12; ++i) a[i] = y[i];
    }
}

// First-stage DFTs of a line whose zero padding the launch knows: all inputs
// (kPruneNone); only the lower half a[0 .. RAD/2) (kPruneHalf: a zero-padded
// prefix of at most P/2 elements, Eq. 13); only a[0] and a[RAD - 1]
// (kPruneEnds: a circularly placed lag axis whose half width L is below the
// line's T threads, Eq. 12). The terms left out are additions of zero, so the
// outputs are the full DFT's (up to the sign of a zero).
enum Prune : int { kPruneNone = 0, kPruneHalf = 1, kPruneEnds = 2 };

// Pruned first stages add a second copy of a transform to a kernel. They pay
// where the passes are VALU-bound (FP32, P <= 256: the 3-D product pass at
// P = 256, 128^3, 27.9 -> 26.9 us); in FP64 the extra registers cost occupancy
// (the same pass 42.7 -> 62.7 us), and the latency-bound P = 1024 passes got
// slower by 0.4 us. Lengths 3 x 2^k run the full first stage.
template <typename R, int P>
constexpr bool kPruneFirst = sizeof(R) == 4 && P <= 256 && !is_tri(P);

template <typename R>
__device__ __forceinline__ void dft4_half(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {   // a2 = a3 = 0
    const cpx<R> x0 = a0, x1 = a1, t3 = mul_minus_i(x1);
    a0 = x0 + x1;
    a2 = x0 - x1;
    a1 = x0 + t3;
    a3 = x0 - t3;
}

template <typename R>
__device__ __forceinline__ void dft4_ends(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {   // a1 = a2 = 0
    const cpx<R> x0 = a0, x3 = a3, t3 = mul_minus_i(cpx<R>{-x3.re, -x3.im});
    a0 = x0 + x3;
    a2 = x0 - x3;
    a1 = x0 + t3;
    a3 = x0 - t3;
}

template <typename R>
__device__ __forceinline__ void dft4_last(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {   // a0 = a1 = a2 = 0
    const cpx<R> x3 = a3, t3 = mul_minus_i(cpx<R>{-x3.re, -x3.im});
    a0 = x3;
    a2 = cpx<R>{-x3.re, -x3.im};
    a1 = t3;
    a3 = cpx<R>{-t3.re, -t3.im};
}

template <int RAD, int PR, typename R>
__device__ __forceinline__ void dft_first(cpx<R> (&a)[RAD]) {
    if constexpr (PR == kPruneNone || RAD == 2 || RAD == 12) {
        dft<RAD>(a);
    } else if constexpr (RAD == 4) {
        if constexpr (PR == kPruneHalf) dft4_half(a[0], a[1], a[2], a[3]);
        else dft4_ends(a[0], a[1], a[2], a[3]);
    } else if constexpr (RAD == 8) {
        if constexpr (PR == kPruneHalf) {
            dft4_half(a[0], a[2], a[4], a[6]);
            dft4_half(a[1], a[3], a[5], a[7]);
        } else {
            a[2] = a[0];
            a[4] = a[0];
            a[6] = a[0];
            dft4_last(a[1], a[3], a[5], a[7]);
        }
        const cpx<R> o1 = rot16<2>(a[3]), o2 = rot16<4>(a[5]), o3 = rot16<6>(a[7]);
        const cpx<R> y0 = a[0] + a[1], y4 = a[0] - a[1];
        const cpx<R> y1 = a[2] + o1, y5 = a[2] - o1;
        const cpx<R> y2 = a[4] + o2, y6 = a[4] - o2;
        const cpx<R> y3 = a[6] + o3, y7 = a[6] - o3;
        a[0] = y0; a[1] = y1; a[2] = y2; a[3] = y3;
        a[4] = y4; a[5] = y5; a[6] = y6; a[7] = y7;
    } else {
        static_assert(RAD == 16, "first-stage radix 4, 8 or 16");
        if constexpr (PR == kPruneHalf) {
            dft4_half(a[0], a[4], a[8], a[12]);
            dft4_half(a[1], a[5], a[9], a[13]);
            dft4_half(a[2], a[6], a[10], a[14]);
            dft4_half(a[3], a[7], a[11], a[15]);
            a[5] = rot16<1>(a[5]);
            a[6] = rot16<2>(a[6]);
            a[9] = rot16<2>(a[9]);
            a[10] = rot16<4>(a[10]);
            a[13] = rot16<3>(a[13]);
            a[14] = rot16<6>(a[14]);
        } else {
            // rows n2 = 1, 2 of the 4 x 4 input block are zero and stay zero
            a[4] = a[0];
            a[8] = a[0];
            a[12] = a[0];
            dft4_last(a[3], a[7], a[11], a[15]);
        }
        a[7] = rot16<3>(a[7]);
        a[11] = rot16<6>(a[11]);
        a[15] = rot16<9>(a[15]);
        if constexpr (PR == kPruneHalf) {
            dft4(a[0], a[1], a[2], a[3]);
            dft4(a[4], a[5], a[6], a[7]);
            dft4(a[8], a[9], a[10], a[11]);
            dft4(a[12], a[13], a[14], a[15]);
        } else {
            dft4_ends(a[0], a[1], a[2], a[3]);
            dft4_ends(a[4], a[5], a[6], a[7]);
            dft4_ends(a[8], a[9], a[10], a[11]);
            dft4_ends(a[12], a[13], a[14], a[15]);
        }
        cpx<R> y[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) y[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = y[i];
    }
}

// ---------------------------------------------------------------------------
// in-workgroup Stockham FFT of one line of length P
// ---------------------------------------------------------------------------

// LDS index of line element p: one padding slot after every 16 elements keeps
// the stride-16 stores of the first stage off a single bank.
__device__ __forceinline__ int padi(int p) { return p + (p >> 4); }

// Points per thread E of a line transform of length P: the line's T = P / E
// threads hold element t + T m in register slot m. E = 16 up to P = 256, where
// the transform takes at most three stages. Longer lines are few (at most P/2
// per axis of a grid), so they spread over more threads: at P = 512 and 1024
// the forward row pass of the counts (the first pass after binning, alone on
// the GPU) uses 4 points per thread, the other row passes and the column
// passes 8; beyond, the fewest that keep a line within 256 threads. Lengths
// 3 x 2^k take 12 (a radix-12 stage, then radix 4 and 2). A function of P and
// the pass alone: every launch shape of a pass rounds identically.
enum RowPass : int { kRowPassCounts = 0, kRowPassSpec = 1, kRowPassInv = 2 };
__host__ __device__ constexpr int row_points(int P, int pass) {
    return is_tri(P) ? 12 : (P <= 256 ? 16 : (P <= 1024 ? (pass == kRowPassCounts ? 4 : 8) : P / 256));
}
__host__ __device__ constexpr int row_pass_of(int in_kind) {
    return in_kind == kRowCountsU64 ? kRowPassCounts : kRowPassSpec;
}
__host__ __device__ constexpr int col_points(int P) {
    return is_tri(P) ? 12 : (P <= 256 ? 16 : (P <= 1024 ? 8 : P / 256));
}

// Radix of the stage that follows the stages with product NS (3 x 2^k: 12
// first, then 4 while at least 4 remain, then 2).
template <int P, int E, int NS>
constexpr int stage_radix() {
    if constexpr (is_tri(P)) return NS == 1 ? 12 : ((P / NS) >= 4 ? 4 : 2);
    else return (P / NS) < E ? P / NS : E;
}

// j mod NS (NS a power of two, or 3 x 2^k past the first stage)
template <int NS>
__device__ __forceinline__ int mod_ns(int j) {
    if constexpr ((NS & (NS - 1)) == 0) return j & (NS - 1);
    else return j % NS;
}

// The twiddles one thread uses in the stages with product NS and after,
// loaded together at the start of the transform so their latency overlaps the
// first stage instead of stalling each later one.
template <typename R, int P, int E, int NS>
struct StageTwiddles {
    static constexpr int RAD = stage_radix<P, E, NS>();
    static constexpr int N = (E / RAD) * (RAD - 1);
    cpx<R> w[N];
    StageTwiddles<R, P, E, NS * RAD> next;
};
template <typename R, int P, int E>
struct StageTwiddles<R, P, E, P> {};

template <typename R, int P, int E, int NS>
__device__ __forceinline__ void load_twiddles(StageTwiddles<R, P, E, NS>& tw, int t) {
    if constexpr (NS < P) {
        constexpr int T = P / E, RAD = stage_radix<P, E, NS>(), NB = E / RAD;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int jm = mod_ns<NS>(t + T * u);
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                if constexpr (is_tri(P))
                    tw.w[u * (RAD - 1) + r - 1] = twiddle3<R>(r * jm * (kMaxP3 / (NS * RAD)));
                else
                    tw.w[u * (RAD - 1) + r - 1] = twiddle<R>(r * jm * (kMaxP / (NS * RAD)));
            }
        }
        load_twiddles<R, P, E, NS * RAD>(tw.next, t);
    }
}

// One radix-RAD pass with NS = product of the earlier radices. Thread t owns
// the butterflies j = t + T u, u < E/RAD; butterfly j reads elements
// j + r P/RAD and writes (j / NS) NS RAD + j % NS + r NS. Element
// t + T m always lives in register slot m. `w` holds this thread's twiddles
// exp(-2 pi i r (j mod NS) / (NS RAD)) for u, r >= 1.
template <typename R, int P, int E, int LS, int RAD, int NS, int NW, int PR = kPruneNone>
__device__ __forceinline__ void fft_stage(cpx<R> (&v)[E], cpx<R>* lds, int t, const cpx<R> (&w)[NW]) {
    constexpr int T = P / E;
    constexpr int NB = E / RAD;
    constexpr bool kFirst = (NS == 1);
    constexpr bool kLast = (NS * RAD == P);
    if constexpr (!kFirst) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = lds[padi(t + T * m) * LS];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        cpx<R> a[RAD];
#pragma unroll
        for (int r = 0; r < RAD; ++r) a[r] = v[u + r * NB];
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < RAD; ++r) a[r] = a[r] * w[u * (RAD - 1) + r - 1];
        }
        if constexpr (kFirst) dft_first<RAD, PR>(a);
        else dft<RAD>(a);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[u + r * NB] = a[r];
    }
    if constexpr (!kLast) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = t + T * u;
            const int base = (j / NS) * (NS * RAD) + mod_ns<NS>(j);
#pragma unroll
            for (int r = 0; r < RAD; ++r) lds[padi(base + r * NS) * LS] = v[u + r * NB];
        }
    }
}

template <typename R, int P, int E, int LS, int NS>
__device__ __forceinline__ void fft_stages(cpx<R> (&v)[E], cpx<R>* lds, int t, const StageTwiddles<R, P, E, NS>& tw) {
    if constexpr (NS < P) {
        constexpr int RAD = stage_radix<P, E, NS>();
        fft_stage<R, P, E, LS, RAD, NS>(v, lds, t, tw.w);
        fft_stages<R, P, E, LS, NS * RAD>(v, lds, t, tw.next);
    }
}

// Forward DFT (sign -1) of the line whose element t + T m is in v[m]; on
// return v[m] holds output t + T m. Every thread of the workgroup must call
// it (it contains barriers). LS is the LDS distance between padded elements;
// PR: the zero padding of the input the first stage may skip (dft_first).
template <typename R, int P, int E, int LS, int PR = kPruneNone>
__device__ __forceinline__ void fft_line(cpx<R> (&v)[E], cpx<R>* lds, int t) {
    static_assert((P >= 16 && P <= kMaxP && (P & (P - 1)) == 0) ||
                      (is_tri(P) && P >= 48 && P <= kMaxP3 && ((P / 3) & (P / 3 - 1)) == 0),
                  "P must be 2^k in [16, 4096] or 3 x 2^k in [48, 3072]");
    static_assert((E == 4 || E == 8 || E == 16 || (E == 12 && is_tri(P))) && E <= P,
                  "4, 8 or 16 points per thread (12 for 3 x 2^k)");
    StageTwiddles<R, P, E, E> tw;
    load_twiddles<R, P, E, E>(tw, t);
    constexpr cpx<R> none[1] = {};
    fft_stage<R, P, E, LS, E, 1, 1, PR>(v, lds, t, none);
    fft_stages<R, P, E, LS, E>(v, lds, t, tw);
}

// Unnormalised inverse DFT (sign +1) through conj(F(conj(x))).
template <typename R, int P, int E, int LS>
__device__ __forceinline__ void ifft_line(cpx<R> (&v)[E], cpx<R>* lds, int t) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].im = -v[m].im;
    fft_line<R, P, E, LS>(v, lds, t);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].im = -v[m].im;
}

template <typename R>
__device__ __forceinline__ R to_real(uint64_t x) { return static_cast<R>(x); }

template <typename R>
__device__ __forceinline__ R fexp(R x);
template <>
__device__ __forceinline__ float fexp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double fexp<double>(double x) { return exp(x); }

// ---------------------------------------------------------------------------
// rows_r2c: real rows along the contiguous axis -> half spectra (P/2 + 1 bins)
// ---------------------------------------------------------------------------

// B line pairs per workgroup: 128 threads, or half that (NARROW) for launches
// that would otherwise leave CUs idle.
template <int P, bool NARROW = false, int PASS = kRowPassCounts>
struct RowShape {
    static constexpr int E = row_points(P, PASS);
    static constexpr int T = P / E;
    static constexpr int kWide = (128 / T) >= 1 ? 128 / T : 1;
    static constexpr int B = NARROW ? (kWide >= 2 ? kWide / 2 : 1) : kWide;
    static constexpr int THREADS = T * B;
};

// q = l'Al accumulated axis by axis, each new axis k adding A_kk l_k^2 + 2 (sum_{a<k} A_ak l_a) l_k.
template <typename R, int D>
__device__ __forceinline__ R gauss_weight(const RowArgs<R>& g, R l0, R l1, R l2, R l3 = R(0)) {
    R q = g.a00 * l0 * l0;
    if constexpr (D >= 2) q = fmaR(g.a11 * l1, l1, fmaR(R(2) * g.a01 * l0, l1, q));
    if constexpr (D >= 3) q = fmaR(g.a22 * l2, l2, fmaR(R(2) * (fmaR(g.a02, l0, g.a12 * l1)), l2, q));
    if constexpr (D == 4)
        q = fmaR(g.a33 * l3, l3, fmaR(R(2) * (fmaR(g.a03, l0, fmaR(g.a13, l1, g.a23 * l2))), l3, q));
    return g.norm * fexp<R>(R(-0.5) * q);
}

// Leading lags of lag-box row r: d = 2 -> (r - L0); d = 3 -> (r / n1 - L0, r % n1 - L1);
// d = 4 -> (r / (n1 n2) - L0, (r / n2) % n1 - L1, r % n2 - L2).
template <typename R, int D>
__device__ __forceinline__ void row_lags(const RowArgs<R>& g, int64_t r, R& l0, R& l1, R& l2) {
    l2 = 0;
    if constexpr (D == 4) {
        const int64_t n1 = 2 * g.L1 + 1, n2 = 2 * g.L2 + 1;
        l0 = static_cast<R>(r / (n1 * n2) - g.L0);
        l1 = static_cast<R>((r / n2) % n1 - g.L1);
        l2 = static_cast<R>(r % n2 - g.L2);
    } else if constexpr (D == 3) {
        const int64_t n1 = 2 * g.L1 + 1;
        l0 = static_cast<R>(r / n1 - g.L0);
        l1 = static_cast<R>(r % n1 - g.L1);
    } else {
        l0 = static_cast<R>(r - g.L0);
        l1 = 0;
    }
}

// BW > 0 overrides the number of line pairs per workgroup (the caller launches
// P/E * BW threads).
template <typename R, int P, int IN_KIND, bool OUT_REAL, int D, bool NARROW = false, int BW = 0>
__device__ __forceinline__ void rows_r2c_body(const RowArgs<R>& gw, uint32_t blk) {
    using C = cpx<R>;
    using S = RowShape<P, NARROW, row_pass_of(IN_KIND)>;
    constexpr int T = S::T, B = BW > 0 ? BW : S::B, LINE = P + P / 16, E = S::E;
    __shared__ C lds[B * LINE];
    const void* __restrict__ in_ = gw.in;
    void* __restrict__ out_ = gw.out;
    const int64_t nrows = gw.nrows, in_ld = gw.in_ld, out_ld = gw.out_ld;
    const int len = gw.len;
    const int b = threadIdx.x / T, t = threadIdx.x - b * T;
    const int64_t r0 = 2 * (static_cast<int64_t>(blk) * B + b), r1 = r0 + 1;
    const bool ok0 = r0 < nrows, ok1 = r1 < nrows;
    C v[E];
    if constexpr (IN_KIND == kRowCountsU64) {
        const uint64_t* in = static_cast<const uint64_t*>(in_);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = t + T * m;
            R x = 0, y = 0;
            if (p < len) {
                if (ok0) x = to_real<R>(in[r0 * in_ld + p]);
                if (ok1) y = to_real<R>(in[r1 * in_ld + p]);
            }
            v[m] = C{x, y};
        }
    } else {
        // weights of two lag-box rows; the last-axis lag l sits at position l mod P
        R a0 = 0, b0 = 0, c0 = 0, a1 = 0, b1 = 0, c1 = 0;
        if (D > 1) {
            row_lags<R, D>(gw, r0, a0, b0, c0);
            row_lags<R, D>(gw, r1, a1, b1, c1);
        }
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = t + T * m;
            R x = 0, y = 0;
            const bool on = p <= len || p >= P - len;
            const R l = static_cast<R>(p <= len ? p : p - P);
            if (on) {
                if constexpr (D == 1) {
                    if (ok0) x = gauss_weight<R, 1>(gw, l, R(0), R(0));
                } else if constexpr (D == 2) {
                    if (ok0) x = gauss_weight<R, 2>(gw, a0, l, R(0));
                    if (ok1) y = gauss_weight<R, 2>(gw, a1, l, R(0));
                } else if constexpr (D == 3) {
                    if (ok0) x = gauss_weight<R, 3>(gw, a0, b0, l);
                    if (ok1) y = gauss_weight<R, 3>(gw, a1, b1, l);
                } else {
                    if (ok0) x = gauss_weight<R, 4>(gw, a0, b0, c0, l);
                    if (ok1) y = gauss_weight<R, 4>(gw, a1, b1, c1, l);
                }
            }
            v[m] = C{x, y};
        }
    }
    C* line = lds + b * LINE;
    // zero padding the first stage skips: counts past len (len <= P/2), or lags past L < T
    if (kPruneFirst<R, P> && (IN_KIND == kRowCountsU64 ? 2 * len <= P : len < T))
        fft_line<R, P, E, 1, IN_KIND == kRowCountsU64 ? kPruneHalf : kPruneEnds>(v, line, t);
    else
        fft_line<R, P, E, 1>(v, line, t);
    // split Z = X + iY of two real rows: X_k = (Z_k + conj Z_-k)/2, Y_k = (Z_k - conj Z_-k)/(2i)
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) line[padi(t + T * m)] = v[m];
    __syncthreads();
    const R h = R(0.5);
    for (int k = t; k <= P / 2; k += T) {
        const C zk = line[padi(k)], zn = line[padi(k == 0 ? 0 : P - k)];
        const C X{(zk.re + zn.re) * h, (zk.im - zn.im) * h};
        const C Y{(zk.im + zn.im) * h, (zn.re - zk.re) * h};
        if constexpr (OUT_REAL) {
            R* out = static_cast<R*>(out_);
            if (ok0) out[r0 * out_ld + k] = X.re;
            if (ok1) out[r1 * out_ld + k] = Y.re;
        } else {
            C* out = static_cast<C*>(out_);
            if (ok0) out[r0 * out_ld + k] = X;
            if (ok1) out[r1 * out_ld + k] = Y;
        }
    }
}

// ---------------------------------------------------------------------------
// rows_c2r: half spectra -> real rows, scaled, window [0, mout)
// ---------------------------------------------------------------------------

template <typename R, int P, bool MULT, bool NARROW = false>
__device__ __forceinline__ void rows_c2r_body(const C2RArgs<R>& a, uint32_t blk) {
    using C = cpx<R>;
    using S = RowShape<P, NARROW, kRowPassInv>;
    constexpr int T = S::T, B = S::B, LINE = P + P / 16, E = S::E;
    __shared__ C lds[B * LINE];
    const C* __restrict__ in = static_cast<const C*>(a.in);
    const R* __restrict__ mult = static_cast<const R*>(a.mult);
    R* __restrict__ out = static_cast<R*>(a.out);
    const int64_t nrows = a.nrows, in_ld = a.in_ld, out_ld = a.out_ld;
    const int mout = a.mout;
    const R scale = a.scale;
    const int b = threadIdx.x / T, t = threadIdx.x - b * T;
    const int64_t r0 = 2 * (static_cast<int64_t>(blk) * B + b), r1 = r0 + 1;
    const bool ok0 = r0 < nrows, ok1 = r1 < nrows;
    C v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int p = t + T * m;
        const bool upper = p > P / 2;
        const int src = upper ? P - p : p;
        C X{0, 0}, Y{0, 0};
        if (ok0) X = in[r0 * in_ld + src];
        if (ok1) Y = in[r1 * in_ld + src];
        if (upper) {
            X = conj(X);
            Y = conj(Y);
        }
        if constexpr (MULT) {
            const R kk = mult[src];
            X = scal(X, kk);
            Y = scal(Y, kk);
        }
        v[m] = C{X.re - Y.im, X.im + Y.re};   // Z = X + iY
    }
    ifft_line<R, P, E, 1>(v, lds + b * LINE, t);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int p = t + T * m;
        if (p < mout) {
            if (ok0) out[r0 * out_ld + p] = v[m].re * scale;
            if (ok1) out[r1 * out_ld + p] = v[m].im * scale;
        }
    }
}

// ---------------------------------------------------------------------------
// cols: transforms along a strided axis, B adjacent lines per workgroup
// ---------------------------------------------------------------------------

// B adjacent lines per workgroup: the widest that fits 72 KiB of LDS and 1024
// threads (up to 16), or 4 for launches that would otherwise leave CUs idle.
template <typename R, int P, bool NARROW>
struct ColShape {
    static constexpr int E = col_points(P);
    static constexpr int T = P / E;
    static constexpr int kLineBytes = (P + P / 16) * static_cast<int>(sizeof(cpx<R>));
    static constexpr int kCap = 73728 / kLineBytes;                 // at most 72 KiB of LDS
    static constexpr int kThr = 1024 / T;
    static constexpr int kRaw = kCap < kThr ? (kCap < 16 ? kCap : 16) : (kThr < 16 ? kThr : 16);
    static constexpr int kWide = kRaw >= 16 ? 16 : kRaw >= 8 ? 8 : kRaw >= 4 ? 4 : kRaw >= 2 ? 2 : 1;
    static constexpr int B = NARROW ? (kWide < 4 ? kWide : 4) : kWide;
    static constexpr int THREADS = T * B;
};

// BW > 0 overrides the number of lines per workgroup (a power of two; the
// caller launches P/E * BW threads).
template <typename R, int P, int MODE, bool NARROW, int BW = 0>
__device__ __forceinline__ void cols_body(const ColArgs& a, uint32_t bx, uint32_t by) {
    using C = cpx<R>;
    constexpr int T = ColShape<R, P, NARROW>::T, E = ColShape<R, P, NARROW>::E;
    constexpr int B = BW > 0 ? BW : ColShape<R, P, NARROW>::B;
    __shared__ C lds[B * (P + P / 16)];
    const int b = threadIdx.x & (B - 1), t = threadIdx.x / B;
    const int64_t w = static_cast<int64_t>(bx) * B + b;
    const int64_t o1 = a.ob ? by / a.ob : 0, o = a.ob ? by % a.ob : by;   // two-level outer index
    const bool act = w < a.W;
    const C* in = static_cast<const C*>(a.in) + o1 * a.in_os1 + o * a.in_os + w;
    C v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int p = t + T * m;
        C x{0, 0};
        if constexpr (MODE == kColFwdPrefix || MODE == kColConvLag || MODE == kColConvSpec) {
            if (act && p < a.len) x = in[p * a.in_ps];
        } else if constexpr (MODE == kColFwdCirc || MODE == kColFwdCircRe) {
            const int idx = p <= a.len ? p + a.len : (p >= P - a.len ? p - P + a.len : -1);
            if (act && idx >= 0) x = in[idx * a.in_ps];
        } else {   // kColInvPrefix
            if (act) x = in[p * a.in_ps];
        }
        v[m] = x;
    }
    if constexpr (MODE == kColConvLag) {
        // the spectrum of this line: transform of the lag column, placed circularly
        // (it is real because the lag box is centrally symmetric)
        const C* kin = static_cast<const C*>(a.kt) + o1 * a.kt_os1 + o * a.kt_os + w;
        C kv[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = t + T * m;
            const int idx = p <= a.kt_len ? p + a.kt_len : (p >= P - a.kt_len ? p - P + a.kt_len : -1);
            kv[m] = (act && idx >= 0) ? kin[idx * a.kt_ps] : C{0, 0};
        }
        if (kPruneFirst<R, P> && a.kt_len < T)
            fft_line<R, P, E, B, kPruneEnds>(kv, lds + b, t);
        else
            fft_line<R, P, E, B>(kv, lds + b, t);
        if (kPruneFirst<R, P> && 2 * a.len <= P)
            fft_line<R, P, E, B, kPruneHalf>(v, lds + b, t);
        else
            fft_line<R, P, E, B>(v, lds + b, t);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = scal(v[m], kv[m].re);
        ifft_line<R, P, E, B>(v, lds + b, t);
    } else if constexpr (MODE == kColConvSpec) {
        // the stored spectrum of this line, loaded while the data line is transformed
        const R* kin = static_cast<const R*>(a.kt) + o1 * a.kt_os1 + o * a.kt_os + w;
        R kv[E];
#pragma unroll
        for (int m = 0; m < E; ++m) kv[m] = act ? kin[(t + T * m) * a.kt_ps] : R(0);
        if (kPruneFirst<R, P> && 2 * a.len <= P)
            fft_line<R, P, E, B, kPruneHalf>(v, lds + b, t);
        else
            fft_line<R, P, E, B>(v, lds + b, t);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = scal(v[m], kv[m]);
        ifft_line<R, P, E, B>(v, lds + b, t);
    } else if constexpr (MODE == kColInvPrefix) {
        ifft_line<R, P, E, B>(v, lds + b, t);
    } else if constexpr (MODE == kColFwdPrefix) {
        if (kPruneFirst<R, P> && 2 * a.len <= P)
            fft_line<R, P, E, B, kPruneHalf>(v, lds + b, t);
        else
            fft_line<R, P, E, B>(v, lds + b, t);
    } else {   // kColFwdCirc, kColFwdCircRe: the same pruning as the lag column of kColConvLag
        if (kPruneFirst<R, P> && a.len < T)
            fft_line<R, P, E, B, kPruneEnds>(v, lds + b, t);
        else
            fft_line<R, P, E, B>(v, lds + b, t);
    }
    if (!act) return;
    if constexpr (MODE == kColFwdCircRe) {
        R* out = static_cast<R*>(a.out) + o1 * a.out_os1 + o * a.out_os + w;
#pragma unroll
        for (int m = 0; m < E; ++m) out[(t + T * m) * a.out_ps] = v[m].re;
    } else if constexpr (MODE == kColFwdPrefix || MODE == kColFwdCirc) {
        C* out = static_cast<C*>(a.out) + o1 * a.out_os1 + o * a.out_os + w;
#pragma unroll
        for (int m = 0; m < E; ++m) out[(t + T * m) * a.out_ps] = v[m];
    } else {   // kColConvLag, kColConvSpec (in place) and kColInvPrefix: keep [0, mout)
        C* out = static_cast<C*>(a.out) + o1 * a.out_os1 + o * a.out_os + w;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = t + T * m;
            if (p < a.mout) out[p * a.out_ps] = v[m];
        }
    }
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

#define KDE_FOR_EACH_P(X) \
    X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)

}  // namespace
}  // namespace kde
