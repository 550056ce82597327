// The binning sort and the kernel-spectrum row pass in one launch; the
// binning plan and the 3-D spectrum's strided pass in another.
//
// The spectrum's row pass is independent of the binning and too small to fill
// the GPU on its own, and a separate launch (or a second stream) costs more
// than its work. Here it shares the launch of the binning sort: the first
// workgroups in XCD-major order run the row transforms of the lag box (Eq. 6
// weights computed in place; first, so that they start at once and end under
// the sort's longer run), the others sort chunks of samples, consecutive chunks
// on one XCD (the chunks' table columns share cache lines), with the same device
// code as the separate passes. Built like the binning sources (no
// floating-point contraction, no fast-math); the FFT code writes its fused
// multiply-adds explicitly, so it rounds as in its own launch.

#include "kde_bin_dev.h"
#include "kde_fft_dev.h"

namespace kde {
namespace {

template <int P>
constexpr int spec_pairs() {   // row pairs per workgroup
    static_assert(RowShape<P, false, kRowPassSpec>::T <= kSortThreads, "a line must fit one sort workgroup");
    return kSortThreads / RowShape<P, false, kRowPassSpec>::T;
}

template <int D, typename R, int P>
__global__ __launch_bounds__(kSortThreads) void sort_kspec_kernel(SortSpecArgs<R> a) {
    const uint32_t ns = static_cast<uint32_t>(ceil_div(ceil_div(a.row.nrows, 2), spec_pairs<P>()));
    const uint32_t bx = xcd_major(blockIdx.x, gridDim.x);
    if (bx < ns) {
        rows_r2c_body<R, P, kRowGaussCirc, D == 1, D, false, spec_pairs<P>()>(a.row, bx);
        return;
    }
    bin_sort_body<D>(a.bin, bx - ns);
}

template <typename R, int P>
constexpr int plan_cols() {    // column lines per workgroup
    static_assert(ColShape<R, P, false>::T <= kPlanThreads, "a line must fit one plan workgroup");
    return kPlanThreads / ColShape<R, P, false>::T;
}

// The plan and the strided pass of the 3-D spectrum: BW = 256 / (P/E) lines per
// workgroup, workgroups walk the (W / BW) x outer grid of the pass, x fastest.
template <typename R, int P>
__global__ __launch_bounds__(kPlanThreads) void plan_kcol_kernel(PlanColArgs a) {
    constexpr int BW = plan_cols<R, P>();
    const uint32_t nbx = static_cast<uint32_t>(ceil_div(a.col.W, BW));
    const uint32_t nc = nbx * static_cast<uint32_t>(a.col.outer);
    if (blockIdx.x < nc) {
        cols_body<R, P, kColFwdCirc, false, BW>(a.col, blockIdx.x % nbx, blockIdx.x / nbx);
        return;
    }
    bin_plan_body(a.bin, blockIdx.x - nc);
}

template <typename R, int P>
hipError_t plan_kcol_launch(const PlanColArgs& a, hipStream_t s) {
    constexpr int BW = plan_cols<R, P>();
    const dim3 g(static_cast<unsigned>(ceil_div(a.col.W, BW) * a.col.outer + a.bin.g.ntiles)), blk(kPlanThreads);
    KDE_LAUNCH((plan_kcol_kernel<R, P>), g, blk, 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t plan_kcol_any(int P, const PlanColArgs& a, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return plan_kcol_launch<R, PP>(a, s);
        KDE_CASE(16) KDE_CASE(32) KDE_CASE(64) KDE_CASE(128) KDE_CASE(256) KDE_CASE(512) KDE_CASE(1024)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int P>
hipError_t sort_kspec_launch(int d, const void* args, hipStream_t s) {
    const SortSpecArgs<R>& a = *static_cast<const SortSpecArgs<R>*>(args);
    const dim3 g(static_cast<unsigned>(a.bin.g.nchunk + ceil_div(ceil_div(a.row.nrows, 2), spec_pairs<P>())));
    const dim3 blk(kSortThreads);
    const size_t lds = bin_stage_lds(kBinSort, a.bin.g);   // the sort's dynamic LDS
    if (d == 1)
        KDE_LAUNCH((sort_kspec_kernel<1, R, P>), g, blk, lds, s, a);
    else if (d == 2)
        KDE_LAUNCH((sort_kspec_kernel<2, R, P>), g, blk, lds, s, a);
    else
        KDE_LAUNCH((sort_kspec_kernel<3, R, P>), g, blk, lds, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t sort_kspec_any(int P, int d, const void* args, hipStream_t s) {
    switch (P) {
#define KDE_CASE(PP) \
    case PP: return sort_kspec_launch<R, PP>(d, args, s);
        KDE_CASE(16) KDE_CASE(32) KDE_CASE(64) KDE_CASE(128) KDE_CASE(256) KDE_CASE(512) KDE_CASE(1024)
#undef KDE_CASE
        default: return hipErrorInvalidValue;
    }
}
static_assert(kSortSpecMaxP == 1024, "sort_kspec_any instantiates the lengths up to kSortSpecMaxP");

}  // namespace

hipError_t launch_plan_kcol(int prec, int P, const PlanColArgs& a, hipStream_t s) {
    if (prec == 2) return plan_kcol_any<double>(P, a, s);
    return plan_kcol_any<float>(P, a, s);
}

hipError_t launch_sort_kspec(int prec, int P, int d, const void* args, hipStream_t s) {
    if (d < 1 || d > 3) return hipErrorInvalidValue;
    if (prec == 2) return sort_kspec_any<double>(P, d, args, s);
    return sort_kspec_any<float>(P, d, args, s);
}

}  // namespace kde
