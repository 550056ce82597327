// Reductions of the LSCV objective (least-squares cross-validation of H).
//
// The two double sums of the objective are binned sums of the Eq. (7) form
// followed by a dot product with the counts:
//   dot(A) = sum_j c_j f_j(A),  f(A) the estimate of Eq. (7) with bandwidth A,
// so that, with phi_H(0) = (2 pi)^-d/2 |H|^-1/2,
//   LSCV(H) = dot(2H) / n - 2 (dot(H) - phi_H(0)) / (n - 1).
// Each dot is summed in FP64 in a fixed order (per-workgroup partials over
// fixed cell ranges, then one workgroup over the partials), so a result never
// depends on scheduling, and the single-problem and batched launches agree
// bit for bit. Built without floating-point contraction; the fused
// multiply-adds are explicit.

#include "kde_internal.h"

namespace kde {
namespace {

constexpr int kDotThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = red[tid] + red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Workgroup blk sums counts_j * f_j over cells [blk kDotChunk, (blk + 1) kDotChunk).
template <typename R>
__device__ __forceinline__ void dot_partial_body(const DotArgs& a, uint32_t blk) {
    __shared__ double red[kDotThreads];
    const auto* __restrict__ counts = a.counts;
    const R* __restrict__ f = static_cast<const R*>(a.f);
    const int64_t c0 = static_cast<int64_t>(blk) * kDotChunk;
    const int64_t c1 = c0 + kDotChunk < a.cells ? c0 + kDotChunk : a.cells;
    double acc = 0.0;
    for (int64_t j = c0 + threadIdx.x; j < c1; j += kDotThreads)
        acc = __builtin_fma(static_cast<double>(counts[j]), static_cast<double>(f[j]), acc);
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.partial[blk] = s * a.scale;
}

// One workgroup: out[0] = sum of the nb partials.
__device__ __forceinline__ void dot_final_body(const DotArgs& a) {
    __shared__ double red[kDotThreads];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < a.nb; i += kDotThreads) acc = acc + a.partial[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.out[0] = s;
}

template <typename R>
__global__ __launch_bounds__(kDotThreads) void dot_partial_kernel(DotArgs a) { dot_partial_body<R>(a, blockIdx.x); }

__global__ __launch_bounds__(kDotThreads) void dot_final_kernel(DotArgs a) { dot_final_body(a); }

template <typename R>
__global__ __launch_bounds__(kDotThreads) void dot_partial_batch(BatchMap m) {
    const int i = static_cast<int>(m.owner[blockIdx.x]);
    dot_partial_body<R>(static_cast<const DotArgs*>(m.tab)[i], blockIdx.x - m.start[i]);
}

__global__ __launch_bounds__(kDotThreads) void dot_final_batch(BatchMap m) {
    dot_final_body(static_cast<const DotArgs*>(m.tab)[m.owner[blockIdx.x]]);
}

// out = {LSCV, dot(2H) / n, 2 (dot(H) - phi0) / (n - 1)} from the two dots.
__global__ __launch_bounds__(64) void lscv_combine_kernel(const double* __restrict__ dots, double n, double phi0,
                                                          double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    const double t1 = dots[0] / n;
    const double t2 = 2.0 * (dots[1] - phi0) / (n - 1.0);
    out[0] = t1 - t2;
    out[1] = t1;
    out[2] = t2;
}

__global__ __launch_bounds__(64) void lscv_combine_batch_kernel(const LscvJob* __restrict__ jobs, int count) {
    const int k = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x);
    if (k >= count) return;
    const LscvJob j = jobs[k];
    const double t1 = j.dot2H[0] / j.n;
    const double t2 = 2.0 * (j.dotH[0] - j.phi0) / (j.n - 1.0);
    j.out[0] = t1 - t2;
    j.out[1] = t1;
    j.out[2] = t2;
}

}  // namespace

int64_t dot_blocks(int64_t cells) { return (cells + kDotChunk - 1) / kDotChunk; }

hipError_t launch_dot(int prec, const DotArgs& a, hipStream_t s) {
    const dim3 blk(kDotThreads), g(static_cast<unsigned>(dot_blocks(a.cells)));
    if (prec == 2)
        KDE_LAUNCH(dot_partial_kernel<double>, g, blk, 0, s, a);
    else
        KDE_LAUNCH(dot_partial_kernel<float>, g, blk, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    KDE_LAUNCH(dot_final_kernel, dim3(1), blk, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dot_batch(int prec, bool final_stage, const BatchMap& m, hipStream_t s) {
    if (m.count <= 0 || m.blocks == 0) return hipSuccess;
    const dim3 blk(kDotThreads), g(m.blocks);
    if (final_stage)
        KDE_LAUNCH(dot_final_batch, g, blk, 0, s, m);
    else if (prec == 2)
        KDE_LAUNCH(dot_partial_batch<double>, g, blk, 0, s, m);
    else
        KDE_LAUNCH(dot_partial_batch<float>, g, blk, 0, s, m);
    return hipGetLastError();
}

hipError_t launch_lscv_combine(const double* dots, double n, double phi0, double* out, hipStream_t s) {
    KDE_LAUNCH(lscv_combine_kernel, dim3(1), dim3(64), 0, s, dots, n, phi0, out);
    return hipGetLastError();
}

hipError_t launch_lscv_combine_batch(const LscvJob* jobs, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    KDE_LAUNCH(lscv_combine_batch_kernel, dim3(static_cast<unsigned>((count + 63) / 64)), dim3(64), 0, s, jobs, count);
    return hipGetLastError();
}

}  // namespace kde
