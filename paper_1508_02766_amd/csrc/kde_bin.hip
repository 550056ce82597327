// gfx950 kernels of the binning step of the binned KDE (Gramacki & Gramacki,
// arXiv 1508.02766, Section 2 first step; the counts must sum to n, Section 3
// footnote): multilinear (2^d-corner) linear binning in integer fixed point.
//
// Per sample and axis: u = (x - lo) / delta with one IEEE FP64 subtraction and
// one correctly rounded FP64 division (this file is compiled with
// -ffp-contract=off and without fast-math so nothing is fused or
// approximated), j = min(floor u, M - 2), q = rint((u - j) 2^Q) (ties to
// even). Corner b of the cell receives prod_k (b_k ? q_k : 2^Q - q_k), an
// exact uint64; integer addition makes the result independent of order.
//
// Two implementations with identical results:
//
// * tiled (default): a counting sort of packed (sample, tile) records into
//   per-tile buckets, then one workgroup per segment of a bucket sums its
//   records in LDS. Four launches:
//     hist     per-chunk histogram of records per tile (LDS atomics)
//     scan     per-tile exclusive scan over chunks (one workgroup per tile);
//              zeroes the counts of tiles with more than one segment
//     scatter  block scan of the tile totals, packed records into buckets
//     accum    LDS sum of one segment (<= S records) of one tile; a tile with
//              one segment is stored with plain writes, the segments of
//              other tiles are added to the counts with 64-bit integer
//              atomics (one per nonzero cell and segment; exact in any order)
//   The scatter's workgroup 0 also writes the accumulation's work list (one
//   descriptor per segment: tile, record range, shared flag), which each
//   accumulation workgroup reads with one load.
//   A sample whose corners straddle a tile edge gets one record per tile it
//   touches, so every cell belongs to exactly one tile.
// * atomic (fallback when a record does not fit in 64 bits or the grid needs
//   more tiles than one workgroup can histogram): zero fill, then 2^d global
//   64-bit atomic adds per sample.

#include "kde_bin_dev.h"

namespace kde {
namespace {

// Single-instance and batched entry points of the four stages (see BatchMap
// for how a batched launch assigns workgroups to instances).

#define KDE_BATCH_PROLOGUE                                              \
    const auto* tab = static_cast<const BinArgs*>(m.tab);               \
    const int inst = static_cast<int>(m.owner[blockIdx.x]);             \
    const BinArgs& a = tab[inst];                                       \
    const uint32_t blk = blockIdx.x - m.start[inst];

// The batched histogram takes the chunks in XCD-major order: consecutive
// chunks write neighbouring words of the tile-major histogram, so they share
// one L2 (the batched scatter measured faster in launch order).
#define KDE_BATCH_PROLOGUE_XCD                                          \
    const auto* tab = static_cast<const BinArgs*>(m.tab);               \
    const uint32_t bid = xcd_major(blockIdx.x, gridDim.x);              \
    const int inst = static_cast<int>(m.owner[bid]);                    \
    const BinArgs& a = tab[inst];                                       \
    const uint32_t blk = bid - m.start[inst];

template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_hist_kernel(BinArgs a) { bin_hist_body<D>(a, xcd_major(blockIdx.x, gridDim.x)); }
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_hist_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE_XCD
    bin_hist_body<D>(a, blk);
}
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_scan_kernel(BinArgs a) { bin_scan_body<D>(a, blockIdx.x); }
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_scan_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE
    bin_scan_body<D>(a, blk);
}
template <int D>
__global__ __launch_bounds__(kScatterThreads) void bin_scatter_kernel(BinArgs a) { bin_scatter_body<D>(a, xcd_major(blockIdx.x, gridDim.x)); }
template <int D>
__global__ __launch_bounds__(kScatterThreads) void bin_scatter_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE
    bin_scatter_body<D>(a, blk);
}
template <int D>
__global__ __launch_bounds__(kAccumThreads) void bin_accum_kernel(BinArgs a) { bin_accum_body<D>(a, blockIdx.x); }
template <int D>
__global__ __launch_bounds__(kAccumBatchThreads) void bin_accum_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE
    bin_accum_body<D, kAccumBatchThreads>(a, blk);
}
#undef KDE_BATCH_PROLOGUE
#undef KDE_BATCH_PROLOGUE_XCD

// ---------------------------------------------------------------------------
// atomic path
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void zero_u64_kernel(uint64_t* __restrict__ p, int64_t count) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
}

template <int D>
__global__ __launch_bounds__(256) void bin_kernel(const double* __restrict__ X, int64_t n, BinConsts c,
                                                  unsigned long long* __restrict__ counts,
                                                  unsigned long long* __restrict__ n_dropped) {
    const uint64_t one = 1ull << c.Q;
    unsigned long long dropped = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        int j[D];
        uint64_t q[D];
        if (!classify<D>(X, i, c, j, q)) {
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
                idx += static_cast<int64_t>(j[k] + bit) * c.stride[k];
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
    KDE_LAUNCH(zero_u64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, count);
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
        KDE_LAUNCH((bin_kernel<1>), g, blk, 0, s, X, n, c, cc, nd);
    else if (c.d == 2)
        KDE_LAUNCH((bin_kernel<2>), g, blk, 0, s, X, n, c, cc, nd);
    else if (c.d == 3)
        KDE_LAUNCH((bin_kernel<3>), g, blk, 0, s, X, n, c, cc, nd);
    else
        KDE_LAUNCH((bin_kernel<4>), g, blk, 0, s, X, n, c, cc, nd);
    return hipGetLastError();
}

namespace {

int64_t bin_stage_extent(int stage, const TileGeom& g) {
    switch (stage) {
        case kBinHist:
        case kBinScatter: return g.nchunk;
        case kBinScan: return g.ntiles;
        default: return g.max_segments;
    }
}

template <int D>
hipError_t bin_stage_d(int stage, const BinArgs& a, hipStream_t s) {
    const dim3 blk(stage == kBinAccum ? kAccumThreads : (stage == kBinScatter ? kScatterThreads : kBinThreads));
    const dim3 grid(static_cast<unsigned>(bin_stage_extent(stage, a.g)));
    const size_t lds = bin_stage_lds(stage, a.g);
    switch (stage) {
        case kBinHist: KDE_LAUNCH((bin_hist_kernel<D>), grid, blk, lds, s, a); break;
        case kBinScan: KDE_LAUNCH((bin_scan_kernel<D>), grid, blk, 0, s, a); break;
        case kBinScatter: KDE_LAUNCH((bin_scatter_kernel<D>), grid, blk, lds, s, a); break;
        case kBinAccum: KDE_LAUNCH((bin_accum_kernel<D>), grid, blk, lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int D>
hipError_t bin_stage_batch_d(int stage, const BatchMap& m, size_t lds, hipStream_t s) {
    const dim3 blk(stage == kBinAccum ? kAccumBatchThreads : (stage == kBinScatter ? kScatterThreads : kBinThreads));
    const dim3 grid(m.blocks);
    switch (stage) {
        case kBinHist: KDE_LAUNCH((bin_hist_batch<D>), grid, blk, lds, s, m); break;
        case kBinScan: KDE_LAUNCH((bin_scan_batch<D>), grid, blk, 0, s, m); break;
        case kBinScatter: KDE_LAUNCH((bin_scatter_batch<D>), grid, blk, lds, s, m); break;
        case kBinAccum: KDE_LAUNCH((bin_accum_batch<D>), grid, blk, lds, s, m); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

size_t bin_stage_lds(int stage, const TileGeom& g) {
    switch (stage) {
        case kBinHist: return static_cast<size_t>(g.ntiles) * 4;
        case kBinScatter: return static_cast<size_t>(g.ntiles) * 8;
        case kBinAccum: return static_cast<size_t>(g.tile_cells) * 8;
        default: return 0;
    }
}

// A batched launch gives every instance its single-instance extent.
int64_t bin_stage_batch_blocks(int stage, const TileGeom& g) { return bin_stage_extent(stage, g); }

hipError_t launch_bin_stage(int stage, const BinArgs& a, hipStream_t s) {
    if (a.c.d == 1) return bin_stage_d<1>(stage, a, s);
    if (a.c.d == 2) return bin_stage_d<2>(stage, a, s);
    if (a.c.d == 3) return bin_stage_d<3>(stage, a, s);
    return bin_stage_d<4>(stage, a, s);
}

hipError_t launch_bin_stage_batch(int stage, int d, const BatchMap& m, size_t lds, hipStream_t s) {
    if (m.count <= 0 || m.blocks == 0) return hipSuccess;
    if (d == 1) return bin_stage_batch_d<1>(stage, m, lds, s);
    if (d == 2) return bin_stage_batch_d<2>(stage, m, lds, s);
    if (d == 3) return bin_stage_batch_d<3>(stage, m, lds, s);
    return bin_stage_batch_d<4>(stage, m, lds, s);
}

}  // namespace kde
