// Internal interface between the host planner / C ABI (kde_api.cpp) and the
// gfx950 kernels (kde_bin.hip, kde_fft.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kde {

// Per-kernel timing. While `stop` is set on the calling thread, every launch
// hands the events to hipExtLaunchKernel, which stamps them with the kernel's
// own dispatch start (first launch only) and end: one pair times the kernels
// of one pass, without the gaps between packets that events recorded around
// the launches would add.
struct KernelTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    int launched = 0;
};
KernelTiming& kernel_timing();   // thread-local; defined with the C ABI

// Workgroup b of a launch of G workgroups, renumbered so that consecutive
// numbers run on the same XCD: the hardware deals workgroups to the 8 XCDs
// round robin, so neighbours that share 128-byte segments would otherwise
// fetch them into eight different L2 caches.
__device__ __forceinline__ uint32_t xcd_major(uint32_t b, uint32_t G) {
    const uint32_t x = b & 7u, slot = b >> 3, q = G >> 3, r = G & 7u;
    return x * q + (x < r ? x : r) + slot;
}

#define KDE_LAUNCH(kernel, grid, block, lds, stream, ...)                                          \
    do {                                                                                           \
        ::kde::KernelTiming& kt_ = ::kde::kernel_timing();                                         \
        if (kt_.stop) {                                                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, static_cast<uint32_t>(lds), stream,         \
                                  kt_.launched ? nullptr : kt_.start, kt_.stop, 0, __VA_ARGS__);   \
            ++kt_.launched;                                                                        \
        } else {                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                     \
        }                                                                                          \
    } while (0)

// Scratch array of kde_eval_noalloc (kde_static.hip): its size, and the device
// address of `dev`'s copy (looked up once per device, with that device current).
constexpr size_t kScratchBytes = size_t(256) << 20;
hipError_t scratch_address(int dev, void** out);

constexpr int kMaxD = 4;      // largest dimension
constexpr int kMaxP = 4096;   // largest padded FFT length per axis (2^k)
constexpr int kMaxP3 = 3072;  // largest padded length 3 x 2^k
constexpr int kMinP = 16;     // smallest (one radix-16 stage)

// Constants of the fixed-point binning step, prepared on the host.
struct BinConsts {
    int d;
    int Q;
    int64_t M[kMaxD];
    int64_t stride[kMaxD];  // row-major element strides of the counts array
    double lo[kMaxD];
    double delta[kMaxD];
    double top[kMaxD];      // M_k - 1 as a double
};

// Tiled binning: the grid is cut into tiles of T_1 x ... x T_d cells; every
// (sample, tile) pair the sample's 2^d corners touch becomes one packed 64-bit
// record (tile-local lower corner + 1 and the d fixed-point fractions q), the
// records are bucketed by tile with a counting sort, and each segment of a
// tile is summed in LDS, then stored (a tile's only segment) or added to the
// counts with integer atomics (tiles with several segments).
constexpr int kBinThreads = 256;
constexpr int kBinChunk = 2048;              // samples per histogram / scatter workgroup
constexpr int kMaxTiles = 8192;              // tile-indexed LDS arrays: at most 96 KiB
constexpr int kMaxTileCells = 4096;
constexpr int kSegment = 4096;                // records per accumulation segment
constexpr int kAccumThreads = 1024;           // threads of an accumulation workgroup
constexpr int kAccumBatchThreads = 256;       // the same in batched launches (many small tiles)
constexpr int kScatterThreads = 512;          // threads of a scatter workgroup (divides kBinChunk)

struct TileGeom {
    int T[kMaxD];           // tile extent (cells, power of two) per axis
    int logT[kMaxD];
    int nt[kMaxD];          // tiles per axis
    int ntiles;
    int tile_cells;         // prod T
    int jbits[kMaxD];       // record bits of (tile-local lower corner + 1) per axis
    int qbits;              // record bits of one fraction q (Q + 1)
    int S;                  // records per accumulation segment
    int64_t nchunk;         // ceil(n / kBinChunk)
    int64_t max_records;    // n 2^d
    int64_t max_segments;   // ntiles + ceil(max_records / S): accumulation workgroups
};

struct BinWork {
    uint32_t* hist;         // [ntiles][nchunk] counts, then exclusive offsets over chunks
    uint32_t* tot;          // [ntiles] records per tile
    uint32_t* drops;        // [nchunk] dropped samples per chunk
    uint64_t* records;      // [max_records]
    uint4* seg;             // [max_segments] accumulation work list: {tile, first record, end
                            // record, tile has several segments}; tile all ones: no work
};

// Everything one instance of the tiled binning reads and writes.
struct BinArgs {
    const double* X;
    int64_t n;
    BinConsts c;
    TileGeom g;
    BinWork w;
    uint64_t* counts;
    unsigned long long* n_dropped;   // may be null
};

enum BinStage : int { kBinHist = 0, kBinScan = 1, kBinScatter = 2, kBinAccum = 3 };

// One stage of the tiled binning for one instance; bin_stage_lds is the
// dynamic LDS a stage needs for the geometry g.
hipError_t launch_bin_stage(int stage, const BinArgs& a, hipStream_t s);
size_t bin_stage_lds(int stage, const TileGeom& g);

// Input kinds of the row (contiguous-axis) real-to-complex pass.
enum RowInput : int {
    kRowCountsU64 = 0,      // uint64 counts, first `len` entries of each row nonzero
    kRowGaussCirc = 1,      // kernel weights of the lag box computed in place (GaussLag),
                            // placed circularly (lag l at l mod P)
};

// k_l = norm exp(-0.5 l'Al) on the lag box [-L, L]^d; A_ab = delta_a delta_b (H^-1)_ab.
// Row r of the row pass is the lag box row with leading lags (l_1, .., l_{d-1}).
struct GaussLag {
    double A[kMaxD * kMaxD];
    double norm;
    int d;
    int L[kMaxD];
};

// Arguments of the row (contiguous-axis) r2c pass in the working precision R.
template <typename R>
struct RowArgs {
    const void* in;         // uint64 counts rows (kRowCountsU64); unused for kRowGaussCirc
    int64_t nrows, in_ld;
    int len;                // nonzero prefix of a counts row, or L of the last axis (weights)
    R a00, a01, a02, a03, a11, a12, a13, a22, a23, a33, norm;   // weights: norm exp(-0.5 l'Al)
    int L0, L1, L2;         // weights: half widths of the leading axes
    void* out;
    int64_t out_ld;
};

// Arguments of the row c2r pass (half spectra -> real rows).
template <typename R>
struct C2RArgs {
    const void* in;
    int64_t nrows, in_ld;
    const void* mult;       // optional real spectrum indexed by the bin, or null
    void* out;
    int64_t out_ld;
    int mout;
    R scale;
};

// Modes of the strided-axis pass.
enum ColMode : int {
    kColFwdPrefix = 0,      // forward FFT of rows [0, len), zero padded; store all P
    kColFwdCirc = 1,        // forward FFT of a circularly placed lag axis (L = len); store all P
    kColFwdCircRe = 2,      // as kColFwdCirc, storing the real parts only (out holds reals)
    kColConvSpec = 3,       // forward FFT of [0, len), times the stored real spectrum line
                            // (kt holds reals), inverse, keep [0, mout)
    kColInvPrefix = 4,      // inverse FFT of all P; keep [0, mout)
    kColConvLag = 5,        // forward FFT of [0, len), times the real spectrum line, inverse,
                            // keep [0, mout); the spectrum line is the FFT of the circularly
                            // placed lag column (kt, 2 kt_len + 1 entries), computed in place
};

// The outer index o of a strided pass splits as o1 = o / ob, o2 = o % ob (ob = 0:
// o2 = o, o1 = 0), the lines of o at o1 os1 + o2 os from the base: two levels,
// for the middle axes of a 4-D array whose leading and trailing axes change
// length between input and output.
struct ColArgs {
    const void* in;
    void* out;
    int64_t W;              // lines per outer index (lines are adjacent in memory)
    int64_t outer;          // number of outer indices (grid.y)
    int64_t ob;             // inner extent of the outer index (0: one level)
    int64_t in_os, in_ps;   // input: outer stride, element stride (complex elements)
    int64_t out_os, out_ps; // output: outer stride, element stride
    int64_t in_os1, out_os1, kt_os1;   // strides of o1 (two-level outer index)
    int len;                // nonzero input prefix length, or L for circular inputs
    int mout;               // kept output prefix length
    const void* kt;         // kColConvLag: lag columns transformed along the other axes;
                            // kColConvSpec: the real spectrum
    int64_t kt_os, kt_ps;   // their outer and element strides (line stride is 1)
    int kt_len;             // their half width L (2 L + 1 entries per column)
};

// Argument structs of the passes, filled on the host.
template <typename R>
RowArgs<R> make_row_args(const void* in, const GaussLag* gauss, int64_t nrows, int64_t in_ld, int len, void* out,
                         int64_t out_ld) {
    RowArgs<R> a{};
    a.in = in;
    a.nrows = nrows;
    a.in_ld = in_ld;
    a.len = len;
    a.out = out;
    a.out_ld = out_ld;
    if (gauss) {
        const double* A = gauss->A;   // row-major kMaxD x kMaxD
        a.a00 = static_cast<R>(A[0]);
        a.a01 = static_cast<R>(A[1]);
        a.a02 = static_cast<R>(A[2]);
        a.a03 = static_cast<R>(A[3]);
        a.a11 = static_cast<R>(A[kMaxD + 1]);
        a.a12 = static_cast<R>(A[kMaxD + 2]);
        a.a13 = static_cast<R>(A[kMaxD + 3]);
        a.a22 = static_cast<R>(A[2 * kMaxD + 2]);
        a.a23 = static_cast<R>(A[2 * kMaxD + 3]);
        a.a33 = static_cast<R>(A[3 * kMaxD + 3]);
        a.norm = static_cast<R>(gauss->norm);
        a.L0 = gauss->L[0];
        a.L1 = gauss->L[1];
        a.L2 = gauss->L[2];
    }
    return a;
}

template <typename R>
C2RArgs<R> make_c2r_args(const void* in, int64_t nrows, int64_t in_ld, const void* mult, void* out, int64_t out_ld,
                         int mout, double scale) {
    C2RArgs<R> a{};
    a.in = in;
    a.nrows = nrows;
    a.in_ld = in_ld;
    a.mult = mult;
    a.out = out;
    a.out_ld = out_ld;
    a.mout = mout;
    a.scale = static_cast<R>(scale);
    return a;
}

// The binning histogram and the kernel-spectrum row pass in one launch
// (d <= 2): the first workgroups transform lag-box rows, the rest histogram.
template <typename R>
struct HistSpecArgs {
    BinArgs bin;
    RowArgs<R> row;
};
hipError_t launch_hist_kspec(int prec, int P, int d, const void* args, hipStream_t s);
int64_t hist_kspec_blocks(int P, int64_t nchunk, int64_t spec_rows);

// The binning scan and the spectrum's strided pass (kColFwdCirc) in one launch
// (d = 3): the first workgroups transform lag-box columns, the rest scan.
struct ScanColArgs {
    BinArgs bin;
    ColArgs col;
};
hipError_t launch_scan_kcol(int prec, int P, const ScanColArgs& a, hipStream_t s);

// All launchers return hipSuccess or the launch error.
hipError_t launch_zero_u64(uint64_t* p, int64_t count, hipStream_t s);
hipError_t launch_bin(const BinConsts& c, const double* X, int64_t n, uint64_t* counts,
                      uint64_t* n_dropped, hipStream_t s);
// k_l = norm exp(-0.5 l'Al) on the lag box; A is kMaxD x kMaxD row-major, in FP64 from the host.
hipError_t launch_kfill(int prec, int d, const int L[kMaxD], const double A[kMaxD * kMaxD], double norm,
                        void* lags, hipStream_t s);
// Row passes: `args` points to RowArgs<R> / C2RArgs<R> of the precision prec
// (1: float, 2: double); d is the lag-box dimension of kRowGaussCirc inputs.
hipError_t launch_rows_r2c(int prec, int P, int input_kind, int d, const void* args, hipStream_t s);
hipError_t launch_rows_c2r(int prec, int P, const void* args, hipStream_t s);
// narrow: 1 four lines per workgroup, 0 the widest shape, -1 chosen from the
// launch size.
hipError_t launch_cols(int prec, int P, int mode, int narrow, const ColArgs& a, hipStream_t s);

// Batched passes: one launch runs the same pass (same kernel template) for
// `count` instances. `tab` is a device array of their argument structs
// (BinArgs, RowArgs<R>, C2RArgs<R> or ColArgs), `start` a device array of
// count + 1 workgroup offsets (start[0] = 0, start[count] = blocks) and
// `owner` a device array giving for each of the `blocks` workgroups its
// instance: workgroup b runs as workgroup b - start[owner[b]] of instance
// owner[b]. Instances with no workgroups are allowed.
struct BatchMap {
    const void* tab;
    const uint32_t* start;
    const uint32_t* owner;
    int count;
    uint32_t blocks;
};

// Workgroups one instance needs in a batched launch of each pass.
int64_t bin_stage_batch_blocks(int stage, const TileGeom& g);
int64_t rows_pass_blocks(int P, int pass, int64_t nrows);   // pass: 0 counts r2c, 1 spectrum r2c, 2 c2r
int64_t cols_pass_blocks(int prec, int P, bool narrow, int64_t W, int64_t outer);

hipError_t launch_bin_stage_batch(int stage, int d, const BatchMap& m, size_t lds, hipStream_t s);
hipError_t launch_rows_r2c_batch(int prec, int P, int input_kind, int d, const BatchMap& m, hipStream_t s);
hipError_t launch_rows_c2r_batch(int prec, int P, bool mult, const BatchMap& m, hipStream_t s);
hipError_t launch_cols_batch(int prec, int P, int mode, bool narrow, const BatchMap& m, hipStream_t s);

// Dot products of counts and densities (LSCV objective): the partial pass
// sums cells [b kDotChunk, (b + 1) kDotChunk) per workgroup b into
// partial[b] (times scale), the final pass writes the sum of the nb partials
// to out[0]. Both in FP64, in a fixed order.
constexpr int64_t kDotChunk = 8192;

struct DotArgs {
    const uint64_t* counts;
    const void* f;          // density, float or double
    int64_t cells;
    double scale;           // 2^-dQ
    double* partial;        // [nb]
    int64_t nb;
    double* out;
};

int64_t dot_blocks(int64_t cells);
hipError_t launch_dot(int prec, const DotArgs& a, hipStream_t s);
hipError_t launch_dot_batch(int prec, bool final_stage, const BatchMap& m, hipStream_t s);
// out[0..2] = {LSCV, dots[0] / n, 2 (dots[1] - phi0) / (n - 1)}.
hipError_t launch_lscv_combine(const double* dots, double n, double phi0, double* out, hipStream_t s);

// The same combination for `count` problems of a batch (one thread each).
struct LscvJob {
    const double* dot2H;    // sum_j c_j f_j with bandwidth 2H
    const double* dotH;     // the same with H
    double n;
    double phi0;            // phi_H(0) = n k_0
    double* out;            // {LSCV, first term, second term}
};
hipError_t launch_lscv_combine_batch(const LscvJob* jobs, int count, hipStream_t s);

// Learned bandwidth proposal network (kde_mlp.hip): 32 -> 128 -> 128 -> 128 -> 16.
constexpr int kMlpIn = 24, kMlpInPad = 32, kMlpHid = 128, kMlpOut = 3, kMlpOutPad = 16, kMlpRows = 64;
// FP32 parameter vector: W1 (k-major, 32 x 128), b1, W2, b2, W3, b3, W4 (128 x 16), b4
constexpr int64_t kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpInPad * kMlpHid;
constexpr int64_t kMlpW2 = kMlpB1 + kMlpHid, kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;
constexpr int64_t kMlpW3 = kMlpB2 + kMlpHid, kMlpB3 = kMlpW3 + kMlpHid * kMlpHid;
constexpr int64_t kMlpW4 = kMlpB3 + kMlpHid, kMlpB4 = kMlpW4 + kMlpHid * kMlpOutPad;
constexpr int64_t kMlpParams = kMlpB4 + kMlpOutPad;
// BF16 weight copies, same offsets in the k-major (Wk[k][n]) and n-major (Wt[n][k]) arrays
constexpr int64_t kMlpWk1 = 0, kMlpWk2 = kMlpWk1 + kMlpInPad * kMlpHid, kMlpWk3 = kMlpWk2 + kMlpHid * kMlpHid;
constexpr int64_t kMlpWk4 = kMlpWk3 + kMlpHid * kMlpHid, kMlpWeights = kMlpWk4 + kMlpHid * kMlpOutPad;
constexpr int64_t kMlpWt1 = kMlpWk1, kMlpWt2 = kMlpWk2, kMlpWt3 = kMlpWk3, kMlpWt4 = kMlpWk4;

enum MlpOp : int { kMlpOpLoad = 0, kMlpOpForward = 1, kMlpOpBackward = 2, kMlpOpReduce = 3, kMlpOpAdam = 4 };

struct MlpArgs {
    const float* P;             // master parameters (read)
    float* Pw;                  // the same, written by load / Adam
    float* m;                   // Adam moments
    float* v;
    const uint16_t* Wk;         // BF16 weights, k-major
    const uint16_t* Wt;         // BF16 weights, n-major
    uint16_t* Wkw;
    uint16_t* Wtw;
    const float* X;             // [B][24] features
    const float* T;             // [B][3] targets
    float* Y;                   // [B][3] outputs
    int64_t B;
    int64_t groups;             // ceil(B / 64)
    uint16_t* acts;             // layer inputs: [B][32], then 3 x [B][128] (BF16)
    float* partial;             // [groups][kMlpParams]
    float* loss_partial;        // [groups]
    float* grad;                // [kMlpParams]
    float* loss;                // [1] or null
    float lr, b1, b2, eps, c1, c2;   // Adam; c1 = 1 - b1^t, c2 = 1 - b2^t
};

hipError_t launch_mlp(int op, const MlpArgs& a, const float* params, hipStream_t s);

}  // namespace kde
