// gfx950 kernels of the binning step of the binned KDE (Gramacki & Gramacki,
// arXiv 1508.02766, Section 2 first step; the counts must sum to n, Section 3
// footnote): multilinear (2^d-corner) linear binning in integer fixed point.
//
// Per sample and axis: u = (x - lo) / delta with one IEEE FP64 subtraction and
// one correctly rounded FP64 division (this file is compiled with
// -ffp-contract=off and without fast-math so nothing is fused or
// approximated), j = min(floor u, M - 2), q = rint((u - j) 2^Q) (ties to
// even). Corner b of the cell receives prod_k (b_k ? q_k : 2^Q - q_k), an
// exact uint64, added with integer atomics, so the result does not depend on
// the order in which samples are processed.

#include "kde_internal.h"

namespace kde {
namespace {

__global__ __launch_bounds__(256) void zero_u64_kernel(uint64_t* __restrict__ p, int64_t count) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
}

template <int D>
__global__ __launch_bounds__(256) void bin_kernel(const double* __restrict__ X, int64_t n, BinConsts c,
                                                  unsigned long long* __restrict__ counts,
                                                  unsigned long long* __restrict__ n_dropped) {
    const double scale = static_cast<double>(1ull << c.Q);   // exact power of two
    const uint64_t one = 1ull << c.Q;
    unsigned long long dropped = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t j[D];
        uint64_t q[D];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double u = (X[i * D + k] - c.lo[k]) / c.delta[k];
            const bool in = (u >= 0.0) && (u <= c.top[k]);   // false for NaN
            ok = ok && in;
            double jf = floor(u);
            jf = jf < c.top[k] - 1.0 ? jf : c.top[k] - 1.0;  // a sample on the last node
            const double t = u - jf;                           // exact
            q[k] = in ? static_cast<uint64_t>(rint(t * scale)) : 0;
            j[k] = in ? static_cast<int64_t>(jf) : 0;
        }
        if (!ok) {
            ++dropped;
            continue;
        }
#pragma unroll
        for (int corner = 0; corner < (1 << D); ++corner) {
            uint64_t w = 1;
            int64_t idx = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int bit = (corner >> (D - 1 - k)) & 1;
                w *= bit ? q[k] : one - q[k];
                idx += (j[k] + bit) * c.stride[k];
            }
            if (w) atomicAdd(counts + idx, static_cast<unsigned long long>(w));
        }
    }
    if (dropped && n_dropped) atomicAdd(n_dropped, dropped);
}

}  // namespace

hipError_t launch_zero_u64(uint64_t* p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_bin(const BinConsts& c, const double* X, int64_t n, uint64_t* counts, uint64_t* n_dropped,
                      hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    auto* cc = reinterpret_cast<unsigned long long*>(counts);
    auto* nd = reinterpret_cast<unsigned long long*>(n_dropped);
    const dim3 g(static_cast<unsigned>(blocks)), blk(256);
    if (c.d == 1)
        hipLaunchKernelGGL((bin_kernel<1>), g, blk, 0, s, X, n, c, cc, nd);
    else if (c.d == 2)
        hipLaunchKernelGGL((bin_kernel<2>), g, blk, 0, s, X, n, c, cc, nd);
    else
        hipLaunchKernelGGL((bin_kernel<3>), g, blk, 0, s, X, n, c, cc, nd);
    return hipGetLastError();
}

}  // namespace kde
