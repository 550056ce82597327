// Batched launches of the FFT convolution passes: one launch runs a pass for
// many independent KDE instances that share its template parameters
// (precision, P, input kind or mode). Workgroups are assigned to instances
// through the BatchMap offsets, so instances of uneven size occupy exactly
// the workgroups they need and no launch is sized by the largest instance.
// The device code is the same as in the single-instance launches.

#include "kde_fft_dev.h"

namespace kde {
namespace {

template <typename R, int P, int IN_KIND, bool OUT_REAL, int D>
__global__ __launch_bounds__((RowShape<P, false, row_pass_of(IN_KIND)>::THREADS)) void rows_r2c_batch(BatchMap m) {
    const int i = static_cast<int>(m.owner[blockIdx.x]);
    rows_r2c_body<R, P, IN_KIND, OUT_REAL, D>(static_cast<const RowArgs<R>*>(m.tab)[i], blockIdx.x - m.start[i]);
}

template <typename R, int P, bool MULT>
__global__ __launch_bounds__((RowShape<P, false, kRowPassInv>::THREADS)) void rows_c2r_batch(BatchMap m) {
    const int i = static_cast<int>(m.owner[blockIdx.x]);
    rows_c2r_body<R, P, MULT>(static_cast<const C2RArgs<R>*>(m.tab)[i], blockIdx.x - m.start[i]);
}

// An instance's workgroups cover its ceil(W / B) x outer tile grid, x fastest;
// the launch is walked in XCD-major order (xcd_major).
template <typename R, int P, int MODE, bool NARROW>
__global__ __launch_bounds__((ColShape<R, P, NARROW>::THREADS)) void cols_batch(BatchMap m) {
    const uint32_t bid = xcd_major(blockIdx.x, gridDim.x);
    const int i = static_cast<int>(m.owner[bid]);
    const ColArgs& a = static_cast<const ColArgs*>(m.tab)[i];
    const uint32_t l = bid - m.start[i];
    const uint32_t nbx = static_cast<uint32_t>(ceil_div(a.W, ColShape<R, P, NARROW>::B));
    cols_body<R, P, MODE, NARROW>(a, l % nbx, l / nbx);
}

template <typename R, int P>
hipError_t rows_r2c_batch_launch(int kind, int d, const BatchMap& m, hipStream_t s) {
    const dim3 g(m.blocks);
    const dim3 blk(kind == kRowCountsU64 ? RowShape<P, false, kRowPassCounts>::THREADS
                                         : RowShape<P, false, kRowPassSpec>::THREADS);
    if (kind == kRowCountsU64)
        KDE_LAUNCH((rows_r2c_batch<R, P, kRowCountsU64, false, 1>), g, blk, 0, s, m);
    else if (d == 1)
        KDE_LAUNCH((rows_r2c_batch<R, P, kRowGaussCirc, true, 1>), g, blk, 0, s, m);
    else if (d == 2)
        KDE_LAUNCH((rows_r2c_batch<R, P, kRowGaussCirc, false, 2>), g, blk, 0, s, m);
    else if (d == 3)
        KDE_LAUNCH((rows_r2c_batch<R, P, kRowGaussCirc, false, 3>), g, blk, 0, s, m);
    else
        KDE_LAUNCH((rows_r2c_batch<R, P, kRowGaussCirc, false, 4>), g, blk, 0, s, m);
    return hipGetLastError();
}

template <typename R, int P>
hipError_t rows_c2r_batch_launch(bool mult, const BatchMap& m, hipStream_t s) {
    const dim3 g(m.blocks), blk(RowShape<P, false, kRowPassInv>::THREADS);
    if (mult)
        KDE_LAUNCH((rows_c2r_batch<R, P, true>), g, blk, 0, s, m);
    else
        KDE_LAUNCH((rows_c2r_batch<R, P, false>), g, blk, 0, s, m);
    return hipGetLastError();
}

template <typename R, int P, bool NARROW>
hipError_t cols_batch_launch_b(int mode, const BatchMap& m, hipStream_t s) {
    const dim3 g(m.blocks), blk(ColShape<R, P, NARROW>::THREADS);
    switch (mode) {
        case kColFwdPrefix: KDE_LAUNCH((cols_batch<R, P, kColFwdPrefix, NARROW>), g, blk, 0, s, m); break;
        case kColFwdCirc: KDE_LAUNCH((cols_batch<R, P, kColFwdCirc, NARROW>), g, blk, 0, s, m); break;
        case kColInvPrefix: KDE_LAUNCH((cols_batch<R, P, kColInvPrefix, NARROW>), g, blk, 0, s, m); break;
        case kColConvLag: KDE_LAUNCH((cols_batch<R, P, kColConvLag, NARROW>), g, blk, 0, s, m); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t rows_r2c_batch_any(int P, int kind, int d, const BatchMap& m, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return rows_r2c_batch_launch<R, PP>(kind, d, m, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t rows_c2r_batch_any(int P, bool mult, const BatchMap& m, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return rows_c2r_batch_launch<R, PP>(mult, m, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t cols_batch_any(int P, int mode, bool narrow, const BatchMap& m, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP)                                                                         \
    case PP:                                                                                 \
        return narrow ? cols_batch_launch_b<R, PP, true>(mode, m, s) : cols_batch_launch_b<R, PP, false>(mode, m, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
int cols_lines_per_group(int P, bool narrow) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return narrow ? ColShape<R, PP, true>::B : ColShape<R, PP, false>::B;
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return 1;
    }
}

int rows_lines_per_group(int P, int pass) {
    switch (P) {
#define KDE_CASE(PP)                                                                         \
    case PP:                                                                                 \
        return pass == kRowPassCounts ? RowShape<PP, false, kRowPassCounts>::B                \
                                      : (pass == kRowPassSpec ? RowShape<PP, false, kRowPassSpec>::B \
                                                              : RowShape<PP, false, kRowPassInv>::B);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return 1;
    }
}

}  // namespace

int64_t rows_pass_blocks(int P, int pass, int64_t nrows) {
    return ceil_div(ceil_div(nrows, 2), rows_lines_per_group(P, pass));
}

int64_t cols_pass_blocks(int prec, int P, bool narrow, int64_t W, int64_t outer) {
    const int B = prec == 2 ? cols_lines_per_group<double>(P, narrow) : cols_lines_per_group<float>(P, narrow);
    return ceil_div(W, B) * outer;
}

hipError_t launch_rows_r2c_batch(int prec, int P, int input_kind, int d, const BatchMap& m, hipStream_t s) {
    if (m.count <= 0 || m.blocks == 0) return hipSuccess;
    if (prec == 2) return rows_r2c_batch_any<double>(P, input_kind, d, m, s);
    return rows_r2c_batch_any<float>(P, input_kind, d, m, s);
}

hipError_t launch_rows_c2r_batch(int prec, int P, bool mult, const BatchMap& m, hipStream_t s) {
    if (m.count <= 0 || m.blocks == 0) return hipSuccess;
    if (prec == 2) return rows_c2r_batch_any<double>(P, mult, m, s);
    return rows_c2r_batch_any<float>(P, mult, m, s);
}

hipError_t launch_cols_batch(int prec, int P, int mode, bool narrow, const BatchMap& m, hipStream_t s) {
    if (m.count <= 0 || m.blocks == 0) return hipSuccess;
    if (prec == 2) return cols_batch_any<double>(P, mode, narrow, m, s);
    return cols_batch_any<float>(P, mode, narrow, m, s);
}

}  // namespace kde
