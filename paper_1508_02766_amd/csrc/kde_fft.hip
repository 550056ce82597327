// gfx950 kernels of the convolution step of the binned KDE (Gramacki &
// Gramacki, arXiv 1508.02766, Section 2 third step, Eq. 7 through the
// discrete convolution theorem of Eq. 10):
//
//   * kfill      lag-box weights k_l = n^-1 K_H(delta l) over [-L, L]^d (Eq. 6, Eq. 12)
//   * rows_r2c   forward transform along the contiguous (last) axis of real rows,
//                two rows per complex FFT; input either u64 counts (zero padded)
//                or lag-box rows whose weights are computed in place and placed
//                circularly (lag l at position l mod P)
//   * cols       forward / fused forward x spectrum x inverse / inverse transforms
//                along a strided axis; a workgroup owns B adjacent lines so each
//                global access is a contiguous run of B complex values; the
//                fused pass transforms the lag column of its line in place, so
//                the spectrum of the slowest axis is never stored
//   * rows_c2r   inverse transform along the contiguous axis back to real rows,
//                with the 1/prod(P) and fixed-point scale, keeping the M window
//
// Every transform is one in-workgroup Stockham FFT of length P = 16..4096:
// 16 points per thread in registers, a radix-16 stage first, then radix-16 and
// a final radix-8/4/2 stage, exchanging through padded LDS between stages.
// Twiddles come from a table of exp(-2 pi i k / 4096) built at compile time in
// FP64 (rounded once to FP32 for the single-precision kernels).
//
// Layout used by the host (row-major, axis 1 slowest, H_d = P_d/2 + 1):
// the lag box sits circularly in the padded array (negative lags at P - |l|),
// the counts sit at the origin, so with P_k >= M_k + L_k the circular
// convolution equals Eq. (7) on the window [0, M_k) of every axis.

#include "kde_fft_dev.h"

namespace kde {
namespace {

// ---------------------------------------------------------------------------
// kfill: k_l = norm exp(-0.5 l'Al), A_ab = delta_a delta_b (H^-1)_ab (Eq. 6, Eq. 1)
// ---------------------------------------------------------------------------

template <typename R, int D>
struct KfillArgs {
    R* lags;
    int64_t count;
    int L[kMaxD];
    R A[kMaxD * kMaxD];
    R norm;
};

// Lag-box entry i in row-major order over [-L_0, L_0] x ... (last axis fastest).
template <typename R, int D>
__global__ __launch_bounds__(256) void kfill_kernel(KfillArgs<R, D> a) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    int64_t rem = i;
    R l[D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        const int64_t n = 2 * a.L[k] + 1;
        l[k] = static_cast<R>((k ? rem % n : rem) - a.L[k]);
        rem /= n;
    }
    // q = l'Al accumulated axis by axis: A_kk l_k^2 + 2 (sum_{b<k} A_bk l_b) l_k
    R q = a.A[0] * l[0] * l[0];
#pragma unroll
    for (int k = 1; k < D; ++k) {
        R cross = a.A[(k - 1) * kMaxD + k] * l[k - 1];
#pragma unroll
        for (int b = k - 2; b >= 0; --b) cross = fmaR(a.A[b * kMaxD + k], l[b], cross);
        q = fmaR(a.A[k * kMaxD + k] * l[k], l[k], fmaR(R(2) * cross, l[k], q));
    }
    a.lags[i] = a.norm * fexp<R>(R(-0.5) * q);
}

// ---------------------------------------------------------------------------
// single-instance entry points of the passes
// ---------------------------------------------------------------------------

template <typename R, int P, int IN_KIND, bool OUT_REAL, int D, bool NARROW>
__global__ __launch_bounds__((RowShape<P, NARROW, row_pass_of(IN_KIND)>::THREADS)) void rows_r2c_kernel(RowArgs<R> a) {
    rows_r2c_body<R, P, IN_KIND, OUT_REAL, D, NARROW>(a, blockIdx.x);
}

template <typename R, int P, bool MULT, bool NARROW>
__global__ __launch_bounds__((RowShape<P, NARROW, kRowPassInv>::THREADS)) void rows_c2r_kernel(C2RArgs<R> a) {
    rows_c2r_body<R, P, MULT, NARROW>(a, blockIdx.x);
}

// A one-dimensional grid over (line block, outer index), line blocks fastest,
// walked in XCD-major order (xcd_major).
template <typename R, int P, int MODE, bool NARROW>
__global__ __launch_bounds__((ColShape<R, P, NARROW>::THREADS)) void cols_kernel(ColArgs a) {
    const uint32_t nbx = static_cast<uint32_t>(ceil_div(a.W, ColShape<R, P, NARROW>::B));
    const uint32_t b = xcd_major(blockIdx.x, gridDim.x);
    cols_body<R, P, MODE, NARROW>(a, b % nbx, b / nbx);
}

// Row launches with fewer than this many workgroups use the narrow shape.
constexpr int64_t kRowNarrowBelow = 256;

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------

template <typename R, int D>
hipError_t kfill_launch(const int L[kMaxD], const double A[kMaxD * kMaxD], double norm, void* lags, hipStream_t s) {
    KfillArgs<R, D> a{};
    a.lags = static_cast<R*>(lags);
    a.count = 1;
    for (int k = 0; k < D; ++k) {
        a.L[k] = L[k];
        a.count *= 2 * L[k] + 1;
    }
    for (int k = 0; k < kMaxD * kMaxD; ++k) a.A[k] = static_cast<R>(A[k]);
    a.norm = static_cast<R>(norm);
    KDE_LAUNCH((kfill_kernel<R, D>), dim3(static_cast<unsigned>(ceil_div(a.count, 256))), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R, int P, int KIND, bool OUT_REAL, int D, bool NARROW>
hipError_t rows_r2c_go(const RowArgs<R>& a, hipStream_t s) {
    using S = RowShape<P, NARROW, row_pass_of(KIND)>;
    const dim3 g(static_cast<unsigned>(ceil_div(ceil_div(a.nrows, 2), S::B))), blk(S::THREADS);
    KDE_LAUNCH((rows_r2c_kernel<R, P, KIND, OUT_REAL, D, NARROW>), g, blk, 0, s, a);
    return hipGetLastError();
}

template <typename R, int P, int KIND, bool OUT_REAL, int D>
hipError_t rows_r2c_pick(const RowArgs<R>& a, hipStream_t s) {
    if (ceil_div(ceil_div(a.nrows, 2), RowShape<P, false, row_pass_of(KIND)>::B) < kRowNarrowBelow)
        return rows_r2c_go<R, P, KIND, OUT_REAL, D, true>(a, s);
    return rows_r2c_go<R, P, KIND, OUT_REAL, D, false>(a, s);
}

template <typename R, int P>
hipError_t rows_r2c_launch(int kind, int d, const void* args, hipStream_t s) {
    const RowArgs<R>& a = *static_cast<const RowArgs<R>*>(args);
    if (kind == kRowCountsU64) return rows_r2c_pick<R, P, kRowCountsU64, false, 1>(a, s);
    if (d == 1) return rows_r2c_pick<R, P, kRowGaussCirc, true, 1>(a, s);
    if (d == 2) return rows_r2c_pick<R, P, kRowGaussCirc, false, 2>(a, s);
    if (d == 3) return rows_r2c_pick<R, P, kRowGaussCirc, false, 3>(a, s);
    return rows_r2c_pick<R, P, kRowGaussCirc, false, 4>(a, s);
}

template <typename R, int P, bool NARROW>
hipError_t rows_c2r_launch_b(const C2RArgs<R>& a, hipStream_t s) {
    using S = RowShape<P, NARROW, kRowPassInv>;
    const dim3 g(static_cast<unsigned>(ceil_div(ceil_div(a.nrows, 2), S::B))), blk(S::THREADS);
    if (a.mult)
        KDE_LAUNCH((rows_c2r_kernel<R, P, true, NARROW>), g, blk, 0, s, a);
    else
        KDE_LAUNCH((rows_c2r_kernel<R, P, false, NARROW>), g, blk, 0, s, a);
    return hipGetLastError();
}

template <typename R, int P>
hipError_t rows_c2r_launch(const void* args, hipStream_t s) {
    const C2RArgs<R>& a = *static_cast<const C2RArgs<R>*>(args);
    if (ceil_div(ceil_div(a.nrows, 2), RowShape<P, false, kRowPassInv>::B) < kRowNarrowBelow)
        return rows_c2r_launch_b<R, P, true>(a, s);
    return rows_c2r_launch_b<R, P, false>(a, s);
}

template <typename R, int P, bool NARROW>
hipError_t cols_launch_b(int mode, const ColArgs& a, hipStream_t s) {
    constexpr int B = ColShape<R, P, NARROW>::B;
    const int64_t blocks = ceil_div(a.W, B) * a.outer;
    if (blocks <= 0 || blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 g(static_cast<unsigned>(blocks));
    const dim3 blk(ColShape<R, P, NARROW>::THREADS);
    switch (mode) {
        case kColFwdPrefix: KDE_LAUNCH((cols_kernel<R, P, kColFwdPrefix, NARROW>), g, blk, 0, s, a); break;
        case kColFwdCirc: KDE_LAUNCH((cols_kernel<R, P, kColFwdCirc, NARROW>), g, blk, 0, s, a); break;
        case kColFwdCircRe: KDE_LAUNCH((cols_kernel<R, P, kColFwdCircRe, NARROW>), g, blk, 0, s, a); break;
        case kColConvSpec: KDE_LAUNCH((cols_kernel<R, P, kColConvSpec, NARROW>), g, blk, 0, s, a); break;
        case kColInvPrefix: KDE_LAUNCH((cols_kernel<R, P, kColInvPrefix, NARROW>), g, blk, 0, s, a); break;
        case kColConvLag: KDE_LAUNCH((cols_kernel<R, P, kColConvLag, NARROW>), g, blk, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int P>
hipError_t cols_launch(int mode, int narrow, const ColArgs& a, hipStream_t s) {
    // far fewer workgroups than CUs with the wide shape: use four lines per workgroup
    if (narrow < 0) narrow = ceil_div(a.W, ColShape<R, P, false>::B) * a.outer < 128 ? 1 : 0;
    if (narrow) return cols_launch_b<R, P, true>(mode, a, s);
    return cols_launch_b<R, P, false>(mode, a, s);
}

template <typename R>
hipError_t rows_r2c_any(int P, int kind, int d, const void* args, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return rows_r2c_launch<R, PP>(kind, d, args, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t rows_c2r_any(int P, const void* args, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return rows_c2r_launch<R, PP>(args, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t cols_any(int P, int mode, int narrow, const ColArgs& a, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return cols_launch<R, PP>(mode, narrow, a, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_kfill(int prec, int d, const int L[kMaxD], const double A[kMaxD * kMaxD], double norm,
                        void* lags, hipStream_t s) {
    if (prec == 2) {
        if (d == 1) return kfill_launch<double, 1>(L, A, norm, lags, s);
        if (d == 2) return kfill_launch<double, 2>(L, A, norm, lags, s);
        if (d == 3) return kfill_launch<double, 3>(L, A, norm, lags, s);
        return kfill_launch<double, 4>(L, A, norm, lags, s);
    }
    if (d == 1) return kfill_launch<float, 1>(L, A, norm, lags, s);
    if (d == 2) return kfill_launch<float, 2>(L, A, norm, lags, s);
    if (d == 3) return kfill_launch<float, 3>(L, A, norm, lags, s);
    return kfill_launch<float, 4>(L, A, norm, lags, s);
}

hipError_t launch_rows_r2c(int prec, int P, int input_kind, int d, const void* args, hipStream_t s) {
    if (prec == 2) return rows_r2c_any<double>(P, input_kind, d, args, s);
    return rows_r2c_any<float>(P, input_kind, d, args, s);
}

hipError_t launch_rows_c2r(int prec, int P, const void* args, hipStream_t s) {
    if (prec == 2) return rows_c2r_any<double>(P, args, s);
    return rows_c2r_any<float>(P, args, s);
}

hipError_t launch_cols(int prec, int P, int mode, int narrow, const ColArgs& a, hipStream_t s) {
    if (prec == 2) return cols_any<double>(P, mode, narrow, a, s);
    return cols_any<float>(P, mode, narrow, a, s);
}

}  // namespace kde
