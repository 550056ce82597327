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
//   The accumulate workgroups rebuild the segment -> tile map from the tile
//   totals in LDS, so no pass ends waiting on one workgroup's bookkeeping.
//   A sample whose corners straddle a tile edge gets one record per tile it
//   touches, so every cell belongs to exactly one tile.
// * atomic (fallback when a record does not fit in 64 bits or the grid needs
//   more tiles than one workgroup can histogram): zero fill, then 2^d global
//   64-bit atomic adds per sample.

#include "kde_internal.h"

namespace kde {
namespace {

// Classification of a sample with coordinates x: false when it lies outside
// the closed grid box (or is NaN) on some axis; otherwise the lower-corner
// node j and the fractions q.
template <int D>
__device__ __forceinline__ bool classify_x(const double (&x)[D], const BinConsts& c, int64_t (&j)[D],
                                           uint64_t (&q)[D]) {
    const double scale = static_cast<double>(1ull << c.Q);   // exact power of two
    bool ok = true;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double u = (x[k] - c.lo[k]) / c.delta[k];
        const bool in = (u >= 0.0) && (u <= c.top[k]);   // false for NaN
        ok = ok && in;
        double jf = floor(u);
        jf = jf < c.top[k] - 1.0 ? jf : c.top[k] - 1.0;  // a sample on the last node
        const double t = u - jf;                           // exact
        q[k] = in ? static_cast<uint64_t>(rint(t * scale)) : 0;
        j[k] = in ? static_cast<int64_t>(jf) : 0;
    }
    return ok;
}

template <int D>
__device__ __forceinline__ bool classify(const double* __restrict__ X, int64_t i, const BinConsts& c,
                                         int64_t (&j)[D], uint64_t (&q)[D]) {
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = X[i * D + k];
    return classify_x<D>(x, c, j, q);
}

constexpr int kPer = kBinChunk / kBinThreads;   // samples per thread in hist / scatter

// Loads this thread's kPer samples of chunk `blk` up front so that all their
// loads are in flight together; rows past n are marked invalid.
template <int D>
__device__ __forceinline__ void load_chunk(const double* __restrict__ X, int64_t n, int64_t blk, double (&x)[kPer][D],
                                           bool (&valid)[kPer]) {
    const int64_t base = blk * kBinChunk + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = base + static_cast<int64_t>(k) * kBinThreads;
        valid[k] = i < n;
        const int64_t ii = valid[k] ? i : 0;
#pragma unroll
        for (int a = 0; a < D; ++a) x[k][a] = X[ii * D + a];
    }
}

// Calls f(tile, record) for every tile the corners j..j+1 touch.
template <int D, typename F>
__device__ __forceinline__ void for_each_tile(const TileGeom& g, const int64_t (&j)[D], const uint64_t (&q)[D], F&& f) {
    int64_t tlo[D];
    int span[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        tlo[k] = j[k] >> g.logT[k];
        span[k] = static_cast<int>(((j[k] + 1) >> g.logT[k]) != tlo[k]);
    }
    uint64_t qpart = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) qpart |= q[k] << (k * g.qbits);
#pragma unroll
    for (int b = 0; b < (1 << D); ++b) {
        bool use = true;
        int64_t tile = 0;
        uint64_t rec = qpart;
        int shift = D * g.qbits;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int bk = (b >> k) & 1;
            use = use && (bk <= span[k]);
            const int64_t tk = tlo[k] + bk;
            tile = tile * g.nt[k] + tk;
            const uint64_t jl = static_cast<uint64_t>(j[k] - (tk << g.logT[k]) + 1);   // in [0, T_k]
            rec |= jl << shift;
            shift += g.jbits[k];
        }
        if (use) f(static_cast<uint32_t>(tile), rec);
    }
}

// Exclusive scan of a[0..n) in LDS by a 256-thread block; returns the total.
__device__ uint32_t block_exclusive_scan(uint32_t* a, int n, uint32_t* wave_sums) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + kBinThreads - 1) / kBinThreads;
    const int b0 = tid * per < n ? tid * per : n;
    const int b1 = b0 + per < n ? b0 + per : n;
    uint32_t s = 0;
    for (int i = b0; i < b1; ++i) s += a[i];
    uint32_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_sums[wave] = x;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kBinThreads / 64; ++w) {
        if (w < wave) before += wave_sums[w];
        total += wave_sums[w];
    }
    uint32_t run = before + x - s;
    for (int i = b0; i < b1; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------------------
// tiled path
// ---------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ void bin_hist_body(const BinArgs& a, uint32_t blk) {
    const double* __restrict__ X = a.X;
    const int64_t n = a.n;
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    uint32_t* __restrict__ hist = a.w.hist;
    uint32_t* __restrict__ drops = a.w.drops;
    extern __shared__ uint32_t h[];     // [ntiles]
    __shared__ uint32_t nd;
    const int tid = threadIdx.x;
    double x[kPer][D];
    bool valid[kPer];
    load_chunk<D>(X, n, blk, x, valid);   // in flight while the histogram is cleared
    for (int t = tid; t < g.ntiles; t += kBinThreads) h[t] = 0;
    if (tid == 0) nd = 0;
    __syncthreads();
    uint32_t dropped = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!valid[k]) continue;
        int64_t j[D];
        uint64_t q[D];
        if (!classify_x<D>(x[k], c, j, q)) {
            ++dropped;
            continue;
        }
        for_each_tile<D>(g, j, q, [&](uint32_t tile, uint64_t) { atomicAdd(&h[tile], 1u); });
    }
    if (dropped) atomicAdd(&nd, dropped);
    __syncthreads();
    // tile-major: the scan reads each tile's chunk counts contiguously
    for (int t = tid; t < g.ntiles; t += kBinThreads) hist[static_cast<int64_t>(t) * g.nchunk + blk] = h[t];
    if (tid == 0) drops[blk] = nd;
}

template <int D>
__device__ __forceinline__ void tile_frame(const BinConsts& c, const TileGeom& g, uint32_t tile, int64_t (&org)[D],
                                           int (&ext)[D]) {
    uint32_t rem = tile;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
        const uint32_t ta = rem % static_cast<uint32_t>(g.nt[a]);
        rem /= static_cast<uint32_t>(g.nt[a]);
        org[a] = static_cast<int64_t>(ta) << g.logT[a];
        const int64_t left = c.M[a] - org[a];
        ext[a] = left < g.T[a] ? static_cast<int>(left) : g.T[a];
    }
}

// Counts index of tile-local cell i (row-major over T), or -1 outside the grid.
template <int D>
__device__ __forceinline__ int64_t tile_cell_index(const BinConsts& c, const TileGeom& g, const int64_t (&org)[D],
                                                   const int (&ext)[D], int i) {
    int64_t idx = 0;
    bool inside = true;
    int rem = i;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
        const int ca = rem & (g.T[a] - 1);
        rem >>= g.logT[a];
        inside = inside && ca < ext[a];
        idx += (org[a] + ca) * c.stride[a];
    }
    return inside ? idx : -1;
}

// One workgroup per tile: exclusive scan of hist[tile][.] over the chunks
// (each thread a contiguous run of chunks, then a workgroup scan of the run
// sums), tot[tile] = the tile's record count; the counts of a tile with more
// than one segment are zeroed for the accumulation. Workgroup 0 also totals
// the dropped samples.
template <int D>
__device__ __forceinline__ void bin_scan_body(const BinArgs& a, uint32_t blk) {
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const uint32_t* __restrict__ drops = a.w.drops;
    unsigned long long* __restrict__ n_dropped = a.n_dropped;
    __shared__ uint32_t wave_sums[kBinThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = static_cast<int>(blk);
    const int64_t nch = g.nchunk;
    const int64_t per = (nch + kBinThreads - 1) / kBinThreads;
    const int64_t c0 = tid * per < nch ? tid * per : nch;
    const int64_t c1 = c0 + per < nch ? c0 + per : nch;
    uint32_t* __restrict__ row = a.w.hist + static_cast<int64_t>(tile) * nch;
    uint32_t s = 0;
    for (int64_t ch = c0; ch < c1; ++ch) s += row[ch];
    uint32_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_sums[wave] = x;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kBinThreads / 64; ++w) {
        if (w < wave) before += wave_sums[w];
        total += wave_sums[w];
    }
    uint32_t run = before + x - s;
    for (int64_t ch = c0; ch < c1; ++ch) {
        const uint32_t v = row[ch];
        row[ch] = run;
        run += v;
    }
    if (tid == 0) a.w.tot[tile] = total;
    // a tile with several segments is summed into the counts with atomics: zero it here
    if (total > static_cast<uint32_t>(g.S)) {
        int64_t org[D];
        int ext[D];
        tile_frame<D>(c, g, static_cast<uint32_t>(tile), org, ext);
        for (int i = tid; i < g.tile_cells; i += kBinThreads) {
            const int64_t idx = tile_cell_index<D>(c, g, org, ext, i);
            if (idx >= 0) a.counts[idx] = 0;
        }
    }
    if (blk == 0 && n_dropped) {
        __shared__ unsigned long long acc;
        if (tid == 0) acc = 0;
        __syncthreads();
        unsigned long long d = 0;
        for (int64_t ch = tid; ch < nch; ch += kBinThreads) d += drops[ch];
        if (d) atomicAdd(&acc, d);
        __syncthreads();
        if (tid == 0) n_dropped[0] = acc;
    }
}

template <int D>
__device__ __forceinline__ void bin_scatter_body(const BinArgs& a, uint32_t blk) {
    const double* __restrict__ X = a.X;
    const int64_t n = a.n;
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    extern __shared__ uint32_t cur[];   // [ntiles], and [ntiles] more in workgroup 0
    __shared__ uint32_t wave_sums[kBinThreads / 64];
    const int tid = threadIdx.x;
    double x[kPer][D];
    bool valid[kPer];
    load_chunk<D>(X, n, blk, x, valid);   // in flight during the prologue
    for (int t = tid; t < g.ntiles; t += kBinThreads) cur[t] = w.tot[t];
    __syncthreads();
    block_exclusive_scan(cur, g.ntiles, wave_sums);   // cur = tile starts
    if (blk == 0) {
        // the accumulation's work list: tile t owns segments [seg_first[t], seg_first[t] + max(1,
        // ceil(tot / S))), and seg_tile maps each segment back to its tile (all ones past the end)
        uint32_t* first = cur + g.ntiles;
        for (int t = tid; t < g.ntiles; t += kBinThreads) {
            w.tile_start[t] = cur[t];
            const uint32_t cnt = w.tot[t];
            first[t] = cnt == 0 ? 1u : (cnt + g.S - 1) / g.S;
        }
        __syncthreads();
        const uint32_t nsegs = block_exclusive_scan(first, g.ntiles, wave_sums);
        for (int t = tid; t < g.ntiles; t += kBinThreads) {
            w.seg_first[t] = first[t];
            const uint32_t e = t + 1 < g.ntiles ? first[t + 1] : nsegs;
            for (uint32_t q = first[t]; q < e; ++q) w.seg_tile[q] = static_cast<uint32_t>(t);
        }
        for (int64_t q = nsegs + tid; q < g.max_segments; q += kBinThreads) w.seg_tile[q] = 0xFFFFFFFFu;
    }
    for (int t = tid; t < g.ntiles; t += kBinThreads) cur[t] += w.hist[static_cast<int64_t>(t) * g.nchunk + blk];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!valid[k]) continue;
        int64_t j[D];
        uint64_t q[D];
        if (!classify_x<D>(x[k], c, j, q)) continue;
        for_each_tile<D>(g, j, q, [&](uint32_t tile, uint64_t rec) {
            const uint32_t pos = atomicAdd(&cur[tile], 1u);
            w.records[pos] = rec;
        });
    }
}

// One workgroup per segment (<= S records of one tile): sum the records'
// corner weights in LDS, then store the tile (sole segment) or add the
// segment's sums to the zeroed counts with 64-bit integer atomics (exact, in
// any order).
template <int D>
__device__ __forceinline__ void bin_accum_body(const BinArgs& a, uint32_t blk) {
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    uint64_t* __restrict__ counts = a.counts;
    extern __shared__ unsigned long long grid[];   // [tile_cells]
    const int tid = threadIdx.x;
    const uint32_t tile = w.seg_tile[blk];          // work list written by the scatter pass
    if (tile == 0xFFFFFFFFu) return;
    const uint32_t k = blk - w.seg_first[tile];
    const uint32_t tcount = w.tot[tile];
    const uint32_t r0 = w.tile_start[tile] + k * static_cast<uint32_t>(g.S);
    const uint32_t tend = w.tile_start[tile] + tcount;
    const uint32_t r1 = r0 + static_cast<uint32_t>(g.S) < tend ? r0 + static_cast<uint32_t>(g.S) : tend;
    const bool shared_tile = tcount > static_cast<uint32_t>(g.S);
    // this thread's records, loaded together
    constexpr int kRec = kSegment / kBinThreads;
    uint64_t recs[kRec];
#pragma unroll
    for (int m = 0; m < kRec; ++m) {
        const uint32_t r = r0 + tid + m * kBinThreads;
        recs[m] = r < r1 ? w.records[r] : 0;
    }
    int64_t org[D];
    int ext[D];
    tile_frame<D>(c, g, tile, org, ext);
    for (int i = tid; i < g.tile_cells; i += kBinThreads) grid[i] = 0;
    __syncthreads();
    const uint64_t one = 1ull << c.Q;
    const uint64_t qmask = (1ull << g.qbits) - 1;
#pragma unroll
    for (int m = 0; m < kRec; ++m) {
        if (r0 + tid + m * kBinThreads >= r1) break;
        const uint64_t rec = recs[m];
        uint64_t q[D];
        int jl[D];
        int shift = D * g.qbits;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            q[a] = (rec >> (a * g.qbits)) & qmask;
            jl[a] = static_cast<int>((rec >> shift) & ((1ull << g.jbits[a]) - 1)) - 1;
            shift += g.jbits[a];
        }
#pragma unroll
        for (int b = 0; b < (1 << D); ++b) {
            bool inside = true;
            int cell = 0;
            uint64_t wgt = 1;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int bit = (b >> (D - 1 - a)) & 1;
                const int ca = jl[a] + bit;
                inside = inside && ca >= 0 && ca < ext[a];
                cell = (cell << g.logT[a]) + ca;
                wgt *= bit ? q[a] : one - q[a];
            }
            if (inside && wgt) atomicAdd(&grid[cell], static_cast<unsigned long long>(wgt));
        }
    }
    __syncthreads();
    if (!shared_tile) {
        for (int i = tid; i < g.tile_cells; i += kBinThreads) {
            const int64_t idx = tile_cell_index<D>(c, g, org, ext, i);
            if (idx >= 0) counts[idx] = grid[i];
        }
    } else {
        auto* cnt = reinterpret_cast<unsigned long long*>(counts);
        for (int i = tid; i < g.tile_cells; i += kBinThreads) {
            const int64_t idx = tile_cell_index<D>(c, g, org, ext, i);
            if (idx >= 0 && grid[i]) atomicAdd(cnt + idx, grid[i]);
        }
    }
}

// Single-instance and batched entry points of the four stages (see BatchMap
// for how a batched launch assigns workgroups to instances).

#define KDE_BATCH_PROLOGUE                                              \
    const auto* tab = static_cast<const BinArgs*>(m.tab);               \
    const int inst = static_cast<int>(m.owner[blockIdx.x]);      \
    const BinArgs& a = tab[inst];                                       \
    const uint32_t blk = blockIdx.x - m.start[inst];

template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_hist_kernel(BinArgs a) { bin_hist_body<D>(a, blockIdx.x); }
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_hist_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE
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
__global__ __launch_bounds__(kBinThreads) void bin_scatter_kernel(BinArgs a) { bin_scatter_body<D>(a, blockIdx.x); }
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_scatter_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE
    bin_scatter_body<D>(a, blk);
}
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_accum_kernel(BinArgs a) { bin_accum_body<D>(a, blockIdx.x); }
template <int D>
__global__ __launch_bounds__(kBinThreads) void bin_accum_batch(BatchMap m) {
    KDE_BATCH_PROLOGUE
    bin_accum_body<D>(a, blk);
}
#undef KDE_BATCH_PROLOGUE

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
        int64_t j[D];
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
    const dim3 blk(kBinThreads), grid(static_cast<unsigned>(bin_stage_extent(stage, a.g)));
    const size_t lds = bin_stage_lds(stage, a.g);
    switch (stage) {
        case kBinHist: hipLaunchKernelGGL((bin_hist_kernel<D>), grid, blk, lds, s, a); break;
        case kBinScan: hipLaunchKernelGGL((bin_scan_kernel<D>), grid, blk, 0, s, a); break;
        case kBinScatter: hipLaunchKernelGGL((bin_scatter_kernel<D>), grid, blk, lds, s, a); break;
        case kBinAccum: hipLaunchKernelGGL((bin_accum_kernel<D>), grid, blk, lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int D>
hipError_t bin_stage_batch_d(int stage, const BatchMap& m, size_t lds, hipStream_t s) {
    const dim3 blk(kBinThreads), grid(m.blocks);
    switch (stage) {
        case kBinHist: hipLaunchKernelGGL((bin_hist_batch<D>), grid, blk, lds, s, m); break;
        case kBinScan: hipLaunchKernelGGL((bin_scan_batch<D>), grid, blk, 0, s, m); break;
        case kBinScatter: hipLaunchKernelGGL((bin_scatter_batch<D>), grid, blk, lds, s, m); break;
        case kBinAccum: hipLaunchKernelGGL((bin_accum_batch<D>), grid, blk, lds, s, m); break;
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
    return bin_stage_d<3>(stage, a, s);
}

hipError_t launch_bin_stage_batch(int stage, int d, const BatchMap& m, size_t lds, hipStream_t s) {
    if (m.count <= 0 || m.blocks == 0) return hipSuccess;
    if (d == 1) return bin_stage_batch_d<1>(stage, m, lds, s);
    if (d == 2) return bin_stage_batch_d<2>(stage, m, lds, s);
    return bin_stage_batch_d<3>(stage, m, lds, s);
}

}  // namespace kde
