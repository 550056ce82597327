// The binning histogram and the kernel-spectrum row pass in one launch.
//
// For 1-D and 2-D problems the spectrum's row pass is independent of the
// binning and too small to fill the GPU on its own, and a separate launch (or
// a second stream) costs more than its work. Here it shares the launch of the
// histogram pass: the first workgroups in XCD-major order run the row
// transforms of the lag box (Eq. 6 weights computed in place; first, so that
// they start at once and end under the histogram's longer run), the others the
// per-chunk histograms of the tiled binning, consecutive chunks on one XCD (the
// chunks' histogram columns share cache lines), with the same device code as
// the separate passes. Built like the binning sources (no floating-point
// contraction, no fast-math); the FFT code writes its fused multiply-adds
// explicitly, so it rounds as in its own launch.

#include "kde_bin_dev.h"
#include "kde_fft_dev.h"

namespace kde {
namespace {

template <int P>
constexpr int spec_pairs() {   // row pairs per workgroup
    static_assert(RowShape<P, false, kRowPassSpec>::T <= kBinThreads, "a line must fit one binning workgroup");
    return kBinThreads / RowShape<P, false, kRowPassSpec>::T;
}
template <typename R, int P>
constexpr int spec_cols() {    // column lines per workgroup
    static_assert(ColShape<R, P, false>::T <= kBinThreads, "a line must fit one binning workgroup");
    return kBinThreads / ColShape<R, P, false>::T;
}

template <int D, typename R, int P>
__global__ __launch_bounds__(kBinThreads) void hist_kspec_kernel(HistSpecArgs<R> a) {
    const uint32_t ns = static_cast<uint32_t>(ceil_div(ceil_div(a.row.nrows, 2), spec_pairs<P>()));
    const uint32_t bx = xcd_major(blockIdx.x, gridDim.x);
    if (bx < ns) {
        rows_r2c_body<R, P, kRowGaussCirc, D == 1, D, false, spec_pairs<P>()>(a.row, bx);
        return;
    }
    bin_hist_body<D>(a.bin, bx - ns);
}

// Scan and the strided pass of the 3-D spectrum: BW = 256 / (P/E) lines per
// workgroup, workgroups walk the (W / BW) x outer grid of the pass, x fastest.
template <typename R, int P>
__global__ __launch_bounds__(kBinThreads) void scan_kcol_kernel(ScanColArgs a) {
    constexpr int BW = spec_cols<R, P>();
    const uint32_t nbx = static_cast<uint32_t>(ceil_div(a.col.W, BW));
    const uint32_t nc = nbx * static_cast<uint32_t>(a.col.outer);
    if (blockIdx.x < nc) {
        cols_body<R, P, kColFwdCirc, false, BW>(a.col, blockIdx.x % nbx, blockIdx.x / nbx);
        return;
    }
    bin_scan_body<3>(a.bin, blockIdx.x - nc);
}

template <typename R, int P>
hipError_t scan_kcol_launch(const ScanColArgs& a, hipStream_t s) {
    constexpr int BW = spec_cols<R, P>();
    const dim3 g(static_cast<unsigned>(ceil_div(a.col.W, BW) * a.col.outer + a.bin.g.ntiles)), blk(kBinThreads);
    KDE_LAUNCH((scan_kcol_kernel<R, P>), g, blk, 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t scan_kcol_any(int P, const ScanColArgs& a, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return scan_kcol_launch<R, PP>(a, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int P>
hipError_t hist_kspec_launch(int d, const void* args, hipStream_t s) {
    const HistSpecArgs<R>& a = *static_cast<const HistSpecArgs<R>*>(args);
    const dim3 g(static_cast<unsigned>(a.bin.g.nchunk + ceil_div(ceil_div(a.row.nrows, 2), spec_pairs<P>())));
    const dim3 blk(kBinThreads);
    const size_t lds = bin_stage_lds(kBinHist, a.bin.g);   // the histogram's dynamic LDS
    if (d == 1)
        KDE_LAUNCH((hist_kspec_kernel<1, R, P>), g, blk, lds, s, a);
    else if (d == 2)
        KDE_LAUNCH((hist_kspec_kernel<2, R, P>), g, blk, lds, s, a);
    else
        KDE_LAUNCH((hist_kspec_kernel<3, R, P>), g, blk, lds, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t hist_kspec_any(int P, int d, const void* args, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return hist_kspec_launch<R, PP>(d, args, s);
        KDE_FOR_EACH_P(KDE_CASE)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int64_t hist_kspec_blocks(int P, int64_t nchunk, int64_t spec_rows) {
    return nchunk + ceil_div(ceil_div(spec_rows, 2), kBinThreads / (P / row_points(P, kRowPassSpec)));
}

hipError_t launch_scan_kcol(int prec, int P, const ScanColArgs& a, hipStream_t s) {
    if (prec == 2) return scan_kcol_any<double>(P, a, s);
    return scan_kcol_any<float>(P, a, s);
}

hipError_t launch_hist_kspec(int prec, int P, int d, const void* args, hipStream_t s) {
    if (d < 1 || d > 3) return hipErrorInvalidValue;
    if (prec == 2) return hist_kspec_any<double>(P, d, args, s);
    return hist_kspec_any<float>(P, d, args, s);
}

}  // namespace kde
