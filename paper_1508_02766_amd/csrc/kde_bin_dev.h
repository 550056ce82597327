// Device code of the binning step (the two passes of the tiled binning and
// their helpers), shared by the binning launches (kde_bin.hip) and the fused
// sort + spectrum launch (kde_fused.hip). Sources including it are
// built without floating-point contraction or fast-math, so that the FP64
// coordinate arithmetic is one subtraction and one correctly rounded division.
#pragma once

#include "kde_internal.h"

namespace kde {
namespace {


// Classification of a sample with coordinates x: false when it lies outside
// the closed grid box (or is NaN) on some axis; otherwise the lower-corner
// node j and the fractions q. Nodes fit 32 bits (M_k <= 2^24); so does q
// when Q < 32, and then one 32-bit conversion replaces the 64-bit one.
template <int D>
__device__ __forceinline__ bool classify_x(const double (&x)[D], const BinConsts& c, int (&j)[D], uint64_t (&q)[D]) {
    const double scale = static_cast<double>(1ull << c.Q);   // exact power of two
    bool ok = true;
    double r[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double u = (x[k] - c.lo[k]) / c.delta[k];
        const bool in = (u >= 0.0) && (u <= c.top[k]);   // false for NaN
        ok = ok && in;
        double jf = floor(u);
        jf = jf < c.top[k] - 1.0 ? jf : c.top[k] - 1.0;  // a sample on the last node
        const double t = u - jf;                           // exact
        r[k] = in ? rint(t * scale) : 0.0;                 // in [0, 2^Q]
        j[k] = in ? static_cast<int>(jf) : 0;
    }
    if (c.Q < 32) {
#pragma unroll
        for (int k = 0; k < D; ++k) q[k] = static_cast<uint32_t>(r[k]);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) q[k] = static_cast<uint64_t>(r[k]);
    }
    return ok;
}

template <int D>
__device__ __forceinline__ bool classify(const double* __restrict__ X, int64_t i, const BinConsts& c, int (&j)[D],
                                         uint64_t (&q)[D]) {
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = X[i * D + k];
    return classify_x<D>(x, c, j, q);
}

// Samples per thread of a histogram / scatter workgroup of NT threads.
template <int NT>
constexpr int per_thread() { return kBinChunk / NT; }

// Loads this thread's samples of chunk `blk` up front so that all their loads
// are in flight together; rows past n are marked invalid.
template <int D, int NT>
__device__ __forceinline__ void load_chunk(const double* __restrict__ X, int64_t n, int64_t blk,
                                           double (&x)[per_thread<NT>()][D], bool (&valid)[per_thread<NT>()]) {
    const int64_t base = blk * kBinChunk + threadIdx.x;
#pragma unroll
    for (int k = 0; k < per_thread<NT>(); ++k) {
        const int64_t i = base + static_cast<int64_t>(k) * NT;
        valid[k] = i < n;
        const int64_t ii = valid[k] ? i : 0;
#pragma unroll
        for (int a = 0; a < D; ++a) x[k][a] = X[ii * D + a];
    }
}

// Calls f(tile, record, b) for every tile the corners j..j+1 touch (b: the
// corner of the lower node's tile offset, 0 <= b < 2^d).
template <int D, typename F>
__device__ __forceinline__ void for_each_tile(const TileGeom& g, const int (&j)[D], const uint64_t (&q)[D], F&& f) {
    int tlo[D];
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
        uint32_t tile = 0;
        uint64_t rec = qpart;
        int shift = D * g.qbits;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int bk = (b >> k) & 1;
            use = use && (bk <= span[k]);
            const int tk = tlo[k] + bk;
            tile = tile * static_cast<uint32_t>(g.nt[k]) + static_cast<uint32_t>(tk);
            const uint32_t jl = static_cast<uint32_t>(j[k] - (tk << g.logT[k]) + 1);   // in [0, T_k]
            rec |= static_cast<uint64_t>(jl) << shift;
            shift += g.jbits[k];
        }
        if (use) f(tile, rec, b);
    }
}

// Exclusive scan of a[0..n) in LDS by a block of NT threads; returns the total.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t* a, int n, uint32_t* wave_sums) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + NT - 1) / NT;
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
    for (int w = 0; w < NT / 64; ++w) {
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

// Inclusive prefix maximum of a[0..n) in LDS by a block of NT threads (each a
// contiguous run, then a wave scan and the maxima of the earlier waves).
template <int NT>
__device__ __forceinline__ void block_inclusive_max_scan(uint32_t* a, int n, uint32_t* wave_max) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + NT - 1) / NT;
    const int b0 = tid * per < n ? tid * per : n;
    const int b1 = b0 + per < n ? b0 + per : n;
    uint32_t s = 0;
    for (int i = b0; i < b1; ++i) s = a[i] > s ? a[i] : s;
    uint32_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x = y > x ? y : x;
    }
    if (lane == 63) wave_max[wave] = x;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w)
        if (w < wave) before = wave_max[w] > before ? wave_max[w] : before;
    const uint32_t up = __shfl_up(x, 1, 64);             // every lane takes part in the shuffle
    uint32_t run = lane > 0 ? up : 0;                    // maximum of the earlier lanes of this wave
    run = before > run ? before : run;
    for (int i = b0; i < b1; ++i) {
        run = a[i] > run ? a[i] : run;
        a[i] = run;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// tiled path
// ---------------------------------------------------------------------------

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

// Pass 1, one workgroup per chunk `blk` of kBinChunk samples: the samples are
// loaded once (into registers) and classified once, their records counted per
// tile (LDS atomics),
// the counts scanned into the offsets of the tile groups in the chunk's region,
// the table column of the chunk written, and the records written to their
// groups (a second LDS atomic per record gives its slot). The workgroup also
// zeroes its share of the counts, which the gather of heavy tiles adds into,
// and workgroup 0 the work-list counter of the plan.
template <int D, int NT = kSortThreads>
__device__ __forceinline__ void bin_sort_body(const BinArgs& a, uint32_t blk) {
    const double* __restrict__ X = a.X;
    const int64_t n = a.n;
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    extern __shared__ uint32_t sort_lds[];   // [ntiles] records per tile, [ntiles] cursors
    uint32_t* h = sort_lds;
    uint32_t* cur = sort_lds + g.ntiles;
    __shared__ uint32_t wave_sums[NT / 64];
    __shared__ uint32_t nd;
    const int tid = threadIdx.x;
    constexpr int kPer = per_thread<NT>();
    double x[kPer][D];
    bool valid[kPer];
    load_chunk<D, NT>(X, n, blk, x, valid);   // in flight while the counts share is cleared
    {
        const int64_t share = (g.cells + g.nchunk - 1) / g.nchunk;
        const int64_t z0 = static_cast<int64_t>(blk) * share;
        const int64_t z1 = z0 + share < g.cells ? z0 + share : g.cells;
        for (int64_t i = z0 + tid; i < z1; i += NT) a.counts[i] = 0;
    }
    for (int t = tid; t < g.ntiles; t += NT) h[t] = 0;
    if (tid == 0) nd = 0;
    if (tid == 0 && blk == 0) w.nitems[0] = 0;   // the plan appends its segments from zero
    __syncthreads();
    // each sample is classified once; its lower corner and fractions stay in registers
    // for the second round
    uint32_t dropped = 0;
    int jj[kPer][D];
    uint64_t qq[kPer][D];
    bool in[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        in[k] = valid[k] && classify_x<D>(x[k], c, jj[k], qq[k]);
        if (valid[k] && !in[k]) ++dropped;
        if (in[k]) for_each_tile<D>(g, jj[k], qq[k], [&](uint32_t tile, uint64_t, int) { atomicAdd(&h[tile], 1u); });
    }
    if (dropped) atomicAdd(&nd, dropped);
    __syncthreads();
    for (int t = tid; t < g.ntiles; t += NT) cur[t] = h[t];
    __syncthreads();
    block_exclusive_scan<NT>(cur, g.ntiles, wave_sums);   // cur = group offsets (ends with a barrier)
    // table column of this chunk, tile-major so that the gather reads a tile's row contiguously
    for (int t = tid; t < g.ntiles; t += NT) w.tab[static_cast<int64_t>(t) * g.nchunk + blk] = (cur[t] << 16) | h[t];
    if (tid == 0) w.drops[blk] = nd;
    __syncthreads();
    uint64_t* __restrict__ region = w.records + static_cast<int64_t>(blk) * g.chunk_cap;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!in[k]) continue;
        for_each_tile<D>(g, jj[k], qq[k], [&](uint32_t tile, uint64_t rec, int) {
            const uint32_t pos = atomicAdd(&cur[tile], 1u);
            region[pos] = rec;
        });
    }
}

// Adds the 2^d corner weights of one record to the tile's LDS sums.
template <int D>
__device__ __forceinline__ void accumulate_record(unsigned long long* grid, const TileGeom& g, const int (&ext)[D],
                                                  uint64_t rec, uint64_t one) {
    const uint64_t qmask = (1ull << g.qbits) - 1;
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

// Pass 2, one workgroup per tile: the exclusive scan of the tile's group
// lengths over the chunks (the index of the tile's first record in each chunk)
// goes to the tile's prefix row; the tile's R records are cut into
// m = ceil(R / kSplitRecords) segments of equal size, appended to the work
// list with one atomic add. Workgroup 0 also totals the dropped samples.
template <int NT = kPlanThreads>
__device__ __forceinline__ void bin_plan_body(const BinArgs& a, uint32_t tile) {
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    const int nch = static_cast<int>(g.nchunk);
    __shared__ uint32_t cnt[kMaxChunks];
    __shared__ uint32_t wave_sums[NT / 64];
    __shared__ uint32_t base;
    const int tid = threadIdx.x;
    if (tile == 0 && a.n_dropped) {
        __shared__ unsigned long long acc;
        if (tid == 0) acc = 0;
        __syncthreads();
        unsigned long long dsum = 0;
        for (int ch = tid; ch < nch; ch += NT) dsum += w.drops[ch];
        if (dsum) atomicAdd(&acc, dsum);
        __syncthreads();
        if (tid == 0) a.n_dropped[0] = acc;
    }
    const uint32_t* __restrict__ row = w.tab + static_cast<int64_t>(tile) * g.nchunk;
    for (int ch = tid; ch < nch; ch += NT) cnt[ch] = row[ch] & 0xFFFFu;
    __syncthreads();
    const uint32_t total = block_exclusive_scan<NT>(cnt, nch, wave_sums);   // ends with a barrier
    uint32_t* __restrict__ prow = w.pre + static_cast<int64_t>(tile) * (g.nchunk + 1);
    for (int ch = tid; ch < nch; ch += NT) prow[ch] = cnt[ch];
    if (tid == 0) prow[nch] = total;
    if (total == 0) return;                                                  // the sort zeroed the tile
    const uint32_t m = (total + kSplitRecords - 1) / kSplitRecords;
    if (tid == 0) base = atomicAdd(w.nitems, m);
    __syncthreads();
    for (uint32_t k = tid; k < m; k += NT) w.items[base + k] = make_uint4(tile, k, m, total);
}

// Pass 3, one workgroup per work-list item: segment k of the m of its tile,
// records [k R / m, (k + 1) R / m) of the tile's R (at most kSplitRecords).
// The chunk of each of them is mapped in LDS from the tile's prefix row, then
// thread i takes records i, i + NT, ... (a wave's loads run along the tile's
// groups) and adds their corner weights to the tile's LDS sums. m = 1:
// the sums are stored; m > 1: added to the counts the sort zeroed. Workgroups
// beyond the list leave at once.
template <int D, int NT = kGatherThreads>
__device__ __forceinline__ void bin_gather_body(const BinArgs& a, uint32_t blk) {
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    uint64_t* __restrict__ counts = a.counts;
    if (blk >= w.nitems[0]) return;
    const uint4 item = w.items[blk];
    const uint32_t tile = item.x, k = item.y, m = item.z, total = item.w;
    const int nch = static_cast<int>(g.nchunk);
    extern __shared__ unsigned long long gather_lds[];
    unsigned long long* grid = gather_lds;                                     // [tile_cells]
    uint32_t* pre = reinterpret_cast<uint32_t*>(gather_lds + g.tile_cells);   // [nchunk + 1]
    uint32_t* ent = pre + nch + 1;                                             // [nchunk]
    uint32_t* wmap = ent + nch;                                                // [kSplitRecords]
    __shared__ uint32_t wave_max[NT / 64];
    const int tid = threadIdx.x;
    const uint32_t* __restrict__ row = w.tab + static_cast<int64_t>(tile) * g.nchunk;
    const uint32_t* __restrict__ prow = w.pre + static_cast<int64_t>(tile) * (g.nchunk + 1);
    for (int ch = tid; ch < nch; ch += NT) {
        ent[ch] = row[ch];
        pre[ch] = prow[ch];
    }
    if (tid == 0) pre[nch] = total;
    for (int i = tid; i < g.tile_cells; i += NT) grid[i] = 0;
    int64_t org[D];
    int ext[D];
    tile_frame<D>(c, g, tile, org, ext);
    const uint32_t r0 = static_cast<uint32_t>(static_cast<uint64_t>(total) * k / m);
    const uint32_t r1 = static_cast<uint32_t>(static_cast<uint64_t>(total) * (k + 1) / m);   // r1 - r0 <= kSplitRecords
    __syncthreads();
    // the chunk of every record of the segment, in LDS: each chunk with records in [r0, r1)
    // marks the position of its first one (the largest index wins where empty chunks share
    // it), and a prefix maximum carries the marks forward; then thread i takes records
    // i, i + NT, ... (a wave's loads run along the tile's groups)
    for (int i = tid; i < kSplitRecords; i += NT) wmap[i] = 0;
    __syncthreads();
    for (int ch = tid; ch < nch; ch += NT) {
        const uint32_t p0 = pre[ch], p1 = pre[ch + 1];
        if (p1 > r0 && p0 < r1) atomicMax(&wmap[(p0 > r0 ? p0 : r0) - r0], static_cast<uint32_t>(ch));
    }
    __syncthreads();
    block_inclusive_max_scan<NT>(wmap, static_cast<int>(r1 - r0), wave_max);
    const uint64_t one = 1ull << c.Q;
    constexpr int kPer = (kSplitRecords + NT - 1) / NT;
    uint64_t rec[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t rr = r0 + static_cast<uint32_t>(tid + u * NT);
        rec[u] = 0;
        if (rr < r1) {
            const int ch = static_cast<int>(wmap[rr - r0]);
            const int64_t at = static_cast<int64_t>(ch) * g.chunk_cap + (ent[ch] >> 16) + (rr - pre[ch]);
            rec[u] = w.records[at];
        }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u)
        if (r0 + static_cast<uint32_t>(tid + u * NT) < r1) accumulate_record<D>(grid, g, ext, rec[u], one);
    __syncthreads();
    if (m == 1) {
        for (int i = tid; i < g.tile_cells; i += NT) {
            const int64_t idx = tile_cell_index<D>(c, g, org, ext, i);
            if (idx >= 0) counts[idx] = grid[i];
        }
    } else {
        auto* cnt = reinterpret_cast<unsigned long long*>(counts);
        for (int i = tid; i < g.tile_cells; i += NT) {
            const int64_t idx = tile_cell_index<D>(c, g, org, ext, i);
            if (idx >= 0 && grid[i]) atomicAdd(cnt + idx, grid[i]);
        }
    }
}

}  // namespace
}  // namespace kde
