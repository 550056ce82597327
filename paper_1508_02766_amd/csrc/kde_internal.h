// Internal interface between the host planner / C ABI (kde_api.cpp) and the
// gfx950 kernels (kde_bin.hip, kde_fft.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kde {

constexpr int kMaxP = 4096;   // largest padded FFT length per axis
constexpr int kMinP = 16;     // smallest (one radix-16 stage)

// Constants of the fixed-point binning step, prepared on the host.
struct BinConsts {
    int d;
    int Q;
    int64_t M[3];
    int64_t stride[3];      // row-major element strides of the counts array
    double lo[3];
    double delta[3];
    double top[3];          // M_k - 1 as a double
};

// Input kinds of the row (contiguous-axis) real-to-complex pass.
enum RowInput : int {
    kRowCountsU64 = 0,      // uint64 counts, first `len` entries of each row nonzero
    kRowLagsCirc = 1,       // lag box rows of 2L+1 reals, placed circularly (lag l at l mod P)
};

// Modes of the strided-axis pass.
enum ColMode : int {
    kColFwdPrefix = 0,      // forward FFT of rows [0, len), zero padded; store all P
    kColFwdCirc = 1,        // forward FFT of a circularly placed lag axis (L = len); store all P
    kColFwdCircReal = 2,    // as kColFwdCirc, store the real part only
    kColConv = 3,           // forward FFT of [0, len), times real spectrum, inverse, keep [0, mout)
    kColInvPrefix = 4,      // inverse FFT of all P; keep [0, mout)
};

struct ColArgs {
    const void* in;
    void* out;
    const void* khat;       // real spectrum for kColConv
    int64_t W;              // lines per outer index (lines are adjacent in memory)
    int64_t outer;          // number of outer indices (grid.y)
    int64_t in_os, in_ps;   // input: outer stride, element stride (complex elements)
    int64_t out_os, out_ps; // output: outer stride, element stride
    int64_t k_ps;           // spectrum element stride (its line stride is 1)
    int len;                // nonzero input prefix length, or L for circular inputs
    int mout;               // kept output prefix length
};

// All launchers return hipSuccess or the launch error.
hipError_t launch_zero_u64(uint64_t* p, int64_t count, hipStream_t s);
hipError_t launch_bin(const BinConsts& c, const double* X, int64_t n, uint64_t* counts,
                      uint64_t* n_dropped, hipStream_t s);
// k_l = norm exp(-0.5 l'Al) on the lag box; A is d x d row-major, in FP64 from the host.
hipError_t launch_kfill(int prec, int d, const int L[3], const double A[9], double norm,
                        void* lags, hipStream_t s);
hipError_t launch_rows_r2c(int prec, int P, int input_kind, const void* in, int64_t nrows,
                           int64_t in_ld, int len, void* out, int64_t out_ld, bool out_real,
                           hipStream_t s);
hipError_t launch_rows_c2r(int prec, int P, const void* in, int64_t nrows, int64_t in_ld,
                           const void* mult, void* out, int64_t out_ld, int mout, double scale,
                           hipStream_t s);
hipError_t launch_cols(int prec, int P, int mode, const ColArgs& a, hipStream_t s);

}  // namespace kde
