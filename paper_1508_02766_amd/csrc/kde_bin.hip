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
// * tiled (default): every (sample, tile) pair the sample's 2^d corners touch
//   becomes one packed record; three launches:
//     sort    one workgroup per chunk of 2048 samples reads them once, groups
//             the chunk's records by tile in the chunk's own region (LDS
//             counts, scan, slots) and writes one table entry per (tile,
//             chunk): the group's offset and length; it also zeroes its share
//             of the counts
//     plan    one workgroup per tile numbers the tile's records across the
//             chunks (exclusive scan of its group lengths) and cuts them into
//             segments of at most 4096, appended to a work list
//     gather  one workgroup per segment sums it in LDS; the only segment of a
//             tile is stored with plain writes, the segments of a heavier tile
//             add their sums to the zeroed counts with 64-bit integer atomics
//             (one per nonzero cell and segment; exact in any order)
//   A sample whose corners straddle a tile edge gets one record per tile it
//   touches, so every cell belongs to exactly one tile.
// * atomic (fallback when a record does not fit in 64 bits or the grid needs
//   more tiles than one workgroup can count): zero fill, then 2^d global
//   64-bit atomic adds per sample.

#include "kde_bin_dev.h"

namespace kde {
namespace {

// Single-instance and batched entry points of the three stages (see BatchMap
// for how a batched launch assigns workgroups to instances). The sort takes
// its chunks in XCD-major order: consecutive chunks write neighbouring words
// of the tile-major table, which then share one L2.

template <int D>
__global__ __launch_bounds__(kSortThreads) void bin_sort_kernel(BinArgs a) {
    bin_sort_body<D>(a, xcd_major(blockIdx.x, gridDim.x));
}
template <int D>
__global__ __launch_bounds__(kSortThreads) void bin_sort_batch(BatchMap m) {
    const auto* tab = static_cast<const BinArgs*>(m.tab);
    const uint32_t bid = xcd_major(blockIdx.x, gridDim.x);
    const int inst = static_cast<int>(m.owner[bid]);
    bin_sort_body<D>(tab[inst], bid - m.start[inst]);
}
__global__ __launch_bounds__(kPlanThreads) void bin_plan_kernel(BinArgs a) { bin_plan_body(a, blockIdx.x); }
__global__ __launch_bounds__(kPlanThreads) void bin_plan_batch(BatchMap m) {
    const auto* tab = static_cast<const BinArgs*>(m.tab);
    const int inst = static_cast<int>(m.owner[blockIdx.x]);
    bin_plan_body(tab[inst], blockIdx.x - m.start[inst]);
}
template <int D>
__global__ __launch_bounds__(kGatherThreads) void bin_gather_kernel(BinArgs a) {
    bin_gather_body<D>(a, blockIdx.x);
}
template <int D>
__global__ __launch_bounds__(kGatherThreads) void bin_gather_batch(BatchMap m) {
    const auto* tab = static_cast<const BinArgs*>(m.tab);
    const int inst = static_cast<int>(m.owner[blockIdx.x]);
    bin_gather_body<D>(tab[inst], blockIdx.x - m.start[inst]);
}

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
    return stage == kBinSort ? g.nchunk : (stage == kBinPlan ? g.ntiles : g.max_items);
}

template <int D>
hipError_t bin_stage_d(int stage, const BinArgs& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(bin_stage_extent(stage, a.g)));
    const size_t lds = bin_stage_lds(stage, a.g);
    if (stage == kBinSort)
        KDE_LAUNCH((bin_sort_kernel<D>), grid, dim3(kSortThreads), lds, s, a);
    else if (stage == kBinPlan)
        KDE_LAUNCH(bin_plan_kernel, grid, dim3(kPlanThreads), 0, s, a);
    else if (stage == kBinGather)
        KDE_LAUNCH((bin_gather_kernel<D>), grid, dim3(kGatherThreads), lds, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int D>
hipError_t bin_stage_batch_d(int stage, const BatchMap& m, size_t lds, hipStream_t s) {
    const dim3 grid(m.blocks);
    if (stage == kBinSort)
        KDE_LAUNCH((bin_sort_batch<D>), grid, dim3(kSortThreads), lds, s, m);
    else if (stage == kBinPlan)
        KDE_LAUNCH(bin_plan_batch, grid, dim3(kPlanThreads), 0, s, m);
    else if (stage == kBinGather)
        KDE_LAUNCH((bin_gather_batch<D>), grid, dim3(kGatherThreads), lds, s, m);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

size_t bin_stage_lds(int stage, const TileGeom& g) {
    if (stage == kBinSort) return static_cast<size_t>(g.ntiles) * 8;
    if (stage == kBinPlan) return 0;
    return static_cast<size_t>(g.tile_cells) * 8 + (2 * static_cast<size_t>(g.nchunk) + 1) * 4 + kSplitRecords * 4;
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
