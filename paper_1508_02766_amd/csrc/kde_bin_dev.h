// Device code of the binning step (the four passes of the tiled counting
// sort and their helpers), shared by the binning launches (kde_bin.hip) and
// the fused scan + spectrum launch (kde_fused.hip). Sources including it are
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

// Calls f(tile, record) for every tile the corners j..j+1 touch.
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
        if (use) f(tile, rec);
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
    constexpr int kPer = per_thread<kBinThreads>();
    double x[kPer][D];
    bool valid[kPer];
    load_chunk<D, kBinThreads>(X, n, blk, x, valid);   // in flight while the histogram is cleared
    for (int t = tid; t < g.ntiles; t += kBinThreads) h[t] = 0;
    if (tid == 0) nd = 0;
    __syncthreads();
    uint32_t dropped = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!valid[k]) continue;
        int j[D];
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

template <int D, int NT = kScatterThreads>
__device__ __forceinline__ void bin_scatter_body(const BinArgs& a, uint32_t blk) {
    const double* __restrict__ X = a.X;
    const int64_t n = a.n;
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    extern __shared__ uint32_t cur[];   // [ntiles] cursors, [ntiles] this chunk's offsets
    __shared__ uint32_t wave_sums[NT / 64];
    uint32_t* aux = cur + g.ntiles;
    const int tid = threadIdx.x;
    const bool lead = blk == 0;
    // The tile totals and this chunk's offsets are loaded before the samples: vector
    // memory loads return in order, so the prologue below waits for them alone while
    // the samples are still in flight (up to kPre * NT tiles in registers).
    constexpr int kPre = 4;
    uint32_t pt[kPre], ph[kPre];
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
        const int t = tid + m * NT;
        pt[m] = t < g.ntiles ? w.tot[t] : 0u;
        ph[m] = t < g.ntiles && !lead ? w.hist[static_cast<int64_t>(t) * g.nchunk + blk] : 0u;
    }
    constexpr int kPer = per_thread<NT>();
    double x[kPer][D];
    bool valid[kPer];
    load_chunk<D, NT>(X, n, blk, x, valid);
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
        const int t = tid + m * NT;
        if (t < g.ntiles) {
            cur[t] = pt[m];
            aux[t] = ph[m];
        }
    }
    for (int t = tid + kPre * NT; t < g.ntiles; t += NT) {
        cur[t] = w.tot[t];
        if (!lead) aux[t] = w.hist[static_cast<int64_t>(t) * g.nchunk + blk];
    }
    __syncthreads();
    block_exclusive_scan<NT>(cur, g.ntiles, wave_sums);   // cur = tile starts
    if (lead) {
        // the accumulation's work list: tile t owns max(1, ceil(tot / S)) consecutive segments
        // of at most S records; aux first holds the segment counts, then their offsets
        for (int t = tid; t < g.ntiles; t += NT) {
            const uint32_t cnt = w.tot[t];
            aux[t] = cnt == 0 ? 1u : (cnt + g.S - 1) / g.S;
        }
        __syncthreads();
        const uint32_t nsegs = block_exclusive_scan<NT>(aux, g.ntiles, wave_sums);
        const uint32_t S = static_cast<uint32_t>(g.S);
        for (int t = tid; t < g.ntiles; t += NT) {
            const uint32_t cnt = w.tot[t];
            const uint32_t end = cur[t] + cnt;
            const uint32_t e = t + 1 < g.ntiles ? aux[t + 1] : nsegs;
            uint32_t r = cur[t];
            for (uint32_t q = aux[t]; q < e; ++q, r += S)
                w.seg[q] = make_uint4(static_cast<uint32_t>(t), r, end - r > S ? r + S : end, cnt > S ? 1u : 0u);
            cur[t] += w.hist[static_cast<int64_t>(t) * g.nchunk + blk];
        }
        for (int64_t q = nsegs + tid; q < g.max_segments; q += NT)
            w.seg[q] = make_uint4(0xFFFFFFFFu, 0u, 0u, 0u);
    } else {
        for (int t = tid; t < g.ntiles; t += NT) cur[t] += aux[t];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!valid[k]) continue;
        int j[D];
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
template <int D, int NT = kAccumThreads>
__device__ __forceinline__ void bin_accum_body(const BinArgs& a, uint32_t blk) {
    const BinConsts& c = a.c;
    const TileGeom& g = a.g;
    const BinWork& w = a.w;
    uint64_t* __restrict__ counts = a.counts;
    extern __shared__ unsigned long long grid[];   // [tile_cells]
    const int tid = threadIdx.x;
    const uint4 sd = w.seg[blk];                    // work list written by the scatter pass
    if (sd.x == 0xFFFFFFFFu) return;
    const uint32_t tile = sd.x, r0 = sd.y, r1 = sd.z;
    const bool shared_tile = sd.w != 0;
    // this thread's records, loaded together
    constexpr int kRec = kSegment / NT;
    uint64_t recs[kRec];
#pragma unroll
    for (int m = 0; m < kRec; ++m) {
        const uint32_t r = r0 + tid + m * NT;
        recs[m] = r < r1 ? w.records[r] : 0;
    }
    int64_t org[D];
    int ext[D];
    tile_frame<D>(c, g, tile, org, ext);
    for (int i = tid; i < g.tile_cells; i += NT) grid[i] = 0;
    __syncthreads();
    const uint64_t one = 1ull << c.Q;
    const uint64_t qmask = (1ull << g.qbits) - 1;
#pragma unroll
    for (int m = 0; m < kRec; ++m) {
        if (r0 + tid + m * NT >= r1) break;
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
