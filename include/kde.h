/*
 * kde.h -- C ABI of the MI355X (gfx950) binned FFT kernel density estimator
 * with an unconstrained (full, symmetric positive definite) bandwidth matrix.
 *
 * Method: A. Gramacki and J. Gramacki, "FFT-Based Fast Computation of
 * Multivariate Kernel Density Estimators with Unconstrained Bandwidth
 * Matrices" (arXiv 1508.02766). The library computes the truncated binned
 * estimate of Eq. (7),
 *
 *     f_j = sum_{|l_k| <= L_k} c_{j-l} k_l ,   k_l = n^-1 K_H(delta_1 l_1, ..., delta_d l_d)
 *
 * on an equally spaced grid (Eq. 3, 4) from linearly binned counts c
 * (Section 2), with K the standard normal density and K_H as in Eq. (1), and
 * L_k from Eq. (15). The kernel weights cover the whole signed lag box
 * [-L, L]^d, which is the paper's correction of Wand's ordering (Section 4.2,
 * Eq. 12-13); the convolution runs through zero-padded radix-16/8/4/2 FFTs
 * (Eq. 10) written for gfx950.
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major with axis 1 slowest. X is n x d FP64, one sample
 *     per row. Densities and counts are laid out as M_1 x ... x M_d and entry
 *     j sits at g_j = lo + j * delta (0-based j).
 *   - H is a host pointer to d x d FP64 (row-major). X, counts, lags,
 *     densities, n_dropped and workspaces are device pointers owned by the
 *     caller. The library allocates no device memory and never frees
 *     caller memory.
 *   - Work is enqueued on `stream` (0 = the null stream) and returns before
 *     it finishes; no call synchronises the device. Host-side validation
 *     happens before any enqueue, so a non-zero return means nothing ran.
 *   - Return 0 (KDE_OK) or a negative kde_status; kde_strerror() names it.
 *     No C++ exception crosses the ABI. Calls are thread-safe.
 */
#ifndef KDE_MI355X_H
#define KDE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest dimension d (Section 2 states the method for general d; the library
 * builds d = 1, 2, 3 and 4). */
#define KDE_MAX_D 4

/* Arithmetic type of the FFT convolution and of densities / lag weights. */
enum kde_precision { KDE_F32 = 1, KDE_F64 = 2 };

enum kde_status {
    KDE_OK = 0,
    KDE_ERR_ARG = -1,       /* null pointer, d not in {1,2,3,4}, M_k < 2, hi_k <= lo_k,
                               non-finite box, n < 0 (n < 1 where the estimate divides by n),
                               bad override, bad precision */
    KDE_ERR_NOT_SPD = -2,   /* H not finite, not symmetric (|H - H'| > 1e-12 max|H|)
                               or not positive definite (Cholesky fails) */
    KDE_ERR_OVERFLOW = -3,  /* n * 2^(d Q) does not fit in uint64 */
    KDE_ERR_WS = -4,        /* workspace or output buffer smaller than required */
    KDE_ERR_SIZE = -5,      /* padded FFT length P_k > 4096 on some axis */
    KDE_ERR_HIP = -6        /* a HIP launch or event call failed */
};

/* Equally spaced grid, Eq. (3)-(4): g_kj = lo[k] + j delta_k, j = 0..M[k]-1,
 * delta_k = (hi[k] - lo[k]) / (M[k] - 1). Only the first d entries are read. */
typedef struct kde_grid {
    int32_t d;
    int32_t reserved;
    int64_t M[KDE_MAX_D];
    double lo[KDE_MAX_D];
    double hi[KDE_MAX_D];
} kde_grid;

/* Options; an all-zero struct (or a NULL pointer) means the defaults. */
typedef struct kde_params {
    double tau;               /* Eq. (15) constant; <= 0 selects 3.7 (Section 4.2) */
    int32_t L[KDE_MAX_D];     /* > 0: use this L_k instead of Eq. (15) (must be <= M_k - 1);
                                 0: Eq. (15) */
    int32_t Q;                /* fixed-point bits of the binning weights; 0: floor(32 / d);
                                 else 1 <= Q and d Q <= 62 */
    int32_t prec;             /* KDE_F32 (also when 0) or KDE_F64 */
    int32_t tile[KDE_MAX_D];  /* > 0: binning tile extent (cells, a power of two <= 4096) on
                                 axis k instead of the default 1024 / 32 x 32 / 8 x 16 x 32 /
                                 8 x 8 x 8 x 8;
                                 the product must stay <= 4096. Changes speed and workspace
                                 size, never the counts */
    int32_t extent;           /* lag-box half widths: 0 (default) Eq. (15), tau sqrt(lambda_max)
                                 on every axis; 1: tau sqrt(H_kk) on axis k, the half width of
                                 the ellipsoid u' H^-1 u <= tau^2 along that axis (a tighter
                                 box around the same ellipsoid; every lag left out lies outside
                                 it, as with Eq. (15)). Both capped at M_k - 1 */
    int32_t reuse_spectrum;   /* kde_conv / kde_eval only. 1: the workspace already holds the
                                 kernel spectrum written by an earlier call of the same entry
                                 point with the same H, n, grid and options; it is not
                                 recomputed. The caller guarantees the match; the result is
                                 then identical to a full call */
    int32_t store_spectrum;   /* 0 or 1; d >= 2, kde_conv / kde_eval / kde_lscv (batches
                                 return KDE_ERR_ARG; d = 1 always stores it). 0 (default): the
                                 product pass transforms each line's lag column itself (three
                                 line transforms per line of the slowest axis, Eq. 10). 1: one
                                 more spectrum pass stores the real spectrum of Eq. (10) on the
                                 whole padded grid (P_1 ... P_(d-1) x pitch(P_d) reals of the
                                 precision more workspace, pitch(P) = P/2 + 1 rounded up to a
                                 multiple of 16) and the product pass reads it (two line
                                 transforms). The same transforms either way, so the same
                                 results; 1 pays off with reuse_spectrum (serving one H on new
                                 samples), where the spectrum pass is skipped */
    int32_t lengths;          /* padded FFT lengths P_k (kde_plan.P): 0 (default) 2^j, or in 3-D
                                 and 4-D 3 x 2^j when shorter; 1: 3 x 2^j also in 2-D (pays in
                                 batches of 2-D problems, whose launches hold many lines; single
                                 2-D problems are faster with 0); 2: 2^j only; other values:
                                 KDE_ERR_ARG. Any value gives the estimate of Eq. (7) up to
                                 rounding */
    int32_t trace_capacity;   /* optional per-kernel timing: number of events in
                                 trace_events, used in pairs */
    hipEvent_t* trace_events; /* if non-NULL: the i-th pass of the call (one kernel; the two
                                 stages of a dot product count as one pass) stamps
                                 events[2i] with its dispatch start and events[2i + 1] with
                                 its end, through hipExtLaunchKernel, for the first
                                 trace_capacity / 2 passes; hipEventElapsedTime of a pair is
                                 the kernel's duration. All passes then run in order on
                                 `stream`. Events are created by the caller with timing
                                 enabled. A stream under graph capture: KDE_ERR_ARG */
    int32_t* trace_count;     /* if non-NULL: receives the number of passes stamped */
    const char** trace_names; /* if non-NULL: receives a static name for pass i
                                 (trace_capacity / 2 entries) */
} kde_params;

/* Everything the host planner derives for one problem. */
typedef struct kde_plan {
    int32_t d;
    int32_t Q;                /* fixed-point bits; counts are in units of 2^-(d Q) */
    int32_t prec;
    int32_t L[KDE_MAX_D];     /* truncation per axis: Eq. (15), the marginal extent, or the
                                 override */
    int32_t P[KDE_MAX_D];     /* padded FFT length per axis (highly composite, Section
                                 4.1): the smallest 2^j >= max(16, M_k + L_k); for d >= 3
                                 the smallest 3 x 2^j >= 48 instead when that is shorter
                                 (kde_params.lengths changes the rule) */
    int32_t reserved;
    double delta[KDE_MAX_D];  /* bin width, Eq. (4) */
    double lambda_max;        /* largest eigenvalue of H */
    double det_H;             /* |H| */
    double norm;              /* n^-1 (2 pi)^-d/2 |H|^-1/2 = k_0 */
    int64_t lag_count;        /* prod (2 L_k + 1) */
    size_t lag_bytes;         /* lag_count * sizeof(real) */
    size_t conv_ws_bytes;     /* workspace needed by kde_conv */
    size_t eval_ws_bytes;     /* workspace needed by kde_eval (counts, binning and
                                 convolution workspaces) */
    size_t density_bytes;     /* prod M_k * sizeof(real) */
    size_t bin_ws_bytes;      /* workspace needed by kde_bin (0: none) */
    size_t lscv_ws_bytes;     /* workspace needed by kde_lscv (0 when n < 2) */
} kde_plan;

/* Grid box from the data (Eq. 3-4; the paper asks for the box [g_k1, g_kM_k]
 * to contain the data's coordinates on axis k, Section 2): on host memory, no
 * device work.
 *     lo_k = min_i X_ik - nsd sqrt(H_kk),   hi_k = max_i X_ik + nsd sqrt(H_kk),
 * M_k = M on every axis, in FP64 (each bound one square root, one product and
 * one sum, rounded in that order). X: host, n x d FP64 row-major; samples with
 * a non-finite coordinate are ignored (binning drops them). H: host, d x d
 * FP64, checked as kde_plan_query checks it. nsd >= 0 and finite (the
 * workloads use 3). *out receives d, M, lo and hi.
 * Errors: KDE_ERR_ARG (null pointer, n < 1, d not in {1,2,3,4}, M < 2, bad nsd,
 * no finite sample, or a box with hi_k <= lo_k), KDE_ERR_NOT_SPD (H). */
int kde_grid_from_data(const double* X, int64_t n, int32_t d, const double* H, double nsd, int64_t M,
                       kde_grid* out);

/* Plan one problem on the host (no device work, no HIP call).
 * Validates H (Section 1: symmetric positive definite), the grid and the
 * options; computes delta (Eq. 4), lambda_max and L (Eq. 15), the padded
 * lengths P, |H|, the normalising constant k_0 (Eq. 6 with Eq. 1) and the
 * workspace sizes. n is the sample count used in the 1/n of Eq. (1); it must
 * be >= 1. With H == NULL only the binning quantities (d, Q, delta,
 * bin_ws_bytes) are filled and n >= 0 is accepted. `out` receives the plan. */
int kde_plan_query(const double* H, int64_t n, const kde_grid* grid,
                   const kde_params* params, kde_plan* out);

/* Linear binning (Section 2, first step; the counts sum to n, Section 3
 * footnote) of the n samples X (device, n x d FP64) onto the grid, in integer
 * fixed point: for each axis u = (X_ik - lo_k) / delta_k (one FP64 subtract,
 * one FP64 divide), j = min(floor u, M_k - 2), q = rint((u - j) 2^Q) with ties
 * to even; corner b of the cell receives prod_k (b_k ? q_k : 2^Q - q_k).
 * counts (device, prod M_k uint64) is overwritten, in units of 2^-(dQ); the
 * result is independent of the order of the samples. Samples with u < 0,
 * u > M_k - 1 or NaN on some axis are skipped; their number is written to
 * *n_dropped (device, may be NULL). n = 0 gives all-zero counts.
 * ws (device, 256-byte aligned, ws_bytes long) must hold plan.bin_ws_bytes
 * (kde_plan_query with H == NULL); it may be NULL when that is 0.
 * n * 2^(dQ) must fit in uint64. */
int kde_bin(const double* X, int64_t n, const kde_grid* grid, const kde_params* params,
            uint64_t* counts, uint64_t* n_dropped, void* ws, size_t ws_bytes, hipStream_t stream);

/* Kernel weights on the signed lag box (Eq. 6 and Eq. 12):
 * k_l = n^-1 (2 pi)^-d/2 |H|^-1/2 exp(-(delta l)' H^-1 (delta l) / 2) for
 * l in [-L_1, L_1] x ... x [-L_d, L_d], written to lags (device,
 * prod (2 L_k + 1) reals of the chosen precision) with entry
 * [L_1 + l_1, ..., L_d + l_d] holding k_l. lags_bytes is the buffer size. */
int kde_kernel_grid(const double* H, int64_t n, const kde_grid* grid, const kde_params* params,
                    void* lags, size_t lags_bytes, hipStream_t stream);

/* The convolution step (Section 2, third step; Eq. 7 via Eq. 10) from
 * existing fixed-point counts (device, prod M_k uint64, as written by
 * kde_bin): fills the lag box, transforms it, transforms the zero-padded
 * counts, multiplies, transforms back and writes the M_1 x ... x M_d window
 * (scaled by 2^-(dQ) / prod P_k) to density (device, reals of the chosen
 * precision). n is the total sample count of Eq. (1). ws (device) must hold
 * plan.conv_ws_bytes and be 256-byte aligned. */
int kde_conv(const uint64_t* counts, int64_t n, const double* H, const kde_grid* grid,
             const kde_params* params, void* density, void* ws, size_t ws_bytes,
             hipStream_t stream);

/* The whole estimate: kde_bin into the workspace, then kde_conv.
 * ws (device, 256-byte aligned) must hold plan.eval_ws_bytes; n_dropped may
 * be NULL. n must be >= 1. */
int kde_eval(const double* X, int64_t n, const double* H, const kde_grid* grid,
             const kde_params* params, void* density, void* ws, size_t ws_bytes,
             uint64_t* n_dropped, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): kde_eval
 * with its workspace taken from a fixed device array inside the library
 * instead of a caller buffer. The caller still passes X, density and
 * n_dropped (device, as for kde_eval). The library holds one array of
 * KDE_NOALLOC_SCRATCH_BYTES on every GPU it runs on, until the process ends;
 * the first call on a GPU looks up that GPU's copy (no allocation), and no
 * call allocates or frees device memory. Everything runs in order on `stream`.
 * Every call on a GPU uses the same array, which keeps the previous call's
 * contents: calls that overlap on one GPU race (serialise them, e.g. on one
 * stream). Returns KDE_ERR_WS when the problem's plan.eval_ws_bytes exceeds
 * KDE_NOALLOC_SCRATCH_BYTES and KDE_ERR_ARG for reuse_spectrum (the array need
 * not hold this problem's spectrum); otherwise the results are those of
 * kde_eval with the same arguments. */
#define KDE_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)
int kde_eval_noalloc(const double* X, int64_t n, const double* H, const kde_grid* grid, const kde_params* params,
                     void* density, uint64_t* n_dropped, hipStream_t stream);

/* Least-squares cross-validation objective of H from fixed-point counts
 * (bandwidth selection, the use of the binned FFT method that Section 5 points
 * to). With phi_A the N(0, A) density, the objective
 *     LSCV(H) = n^-2 sum_{i,j} phi_2H(X_i - X_j) - 2 [n (n-1)]^-1 sum_{i != j} phi_H(X_i - X_j)
 * is evaluated in binned form: each pair sum is sum_j c_j (c * kappa_A)_j with
 * kappa_A(l) = phi_A(delta l) on the lag box of Eq. (15) for A (Eq. 7 with
 * weights n * k_l), and the i = j pairs of the second sum are removed as
 * n phi_H(0). Two convolutions (2H, then H) and two FP64 dot products.
 * counts: device, prod M_k uint64 as kde_bin writes them; n >= 2 is the sample
 * count; out: device, 3 doubles = {LSCV, first term, second term}.
 * ws (device, 256-byte aligned) must hold plan.lscv_ws_bytes. */
int kde_lscv(const uint64_t* counts, int64_t n, const double* H, const kde_grid* grid,
             const kde_params* params, double* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned bandwidth proposal: a perceptron 24 -> 128 -> 128 -> 128 -> 3 (ReLU)
 * mapping summary features of a sample to Cholesky coordinates of H, trained
 * by mean squared error against LSCV-optimal bandwidths (kde_lscv), with the
 * plain LSCV search kept as fallback and reference. Products on the matrix cores
 * in BF16 with FP32 accumulation; FP32 master parameters and Adam state.
 * State (device, state_bytes, 256-byte aligned, caller-owned) holds the FP32
 * parameters, the Adam moments and the BF16 weight copies. Parameter vector
 * (FP32, n_params): W1 (32 x 128, rows >= 24 zero), b1 (128), W2 (128 x 128),
 * b2, W3, b3, W4 (128 x 16, columns >= 3 zero), b4 (16, entries >= 3 zero),
 * each W stored input-major (W[k][n] at k * n_out + n).
 * ------------------------------------------------------------------------- */

typedef struct kde_mlp_info {
    int32_t n_in, n_hidden, n_out;
    int32_t rows_per_group;   /* rows per workgroup */
    int64_t n_params;
    size_t state_bytes;
    size_t ws_bytes;          /* workspace for a batch of `batch` rows (kde_mlp_query) */
} kde_mlp_info;

int kde_mlp_query(int64_t batch, kde_mlp_info* info);

/* Load params (device, n_params FP32) into state, zero the Adam moments. */
int kde_mlp_load(void* state, const float* params, hipStream_t stream);

/* Y (device, B x 3 FP32) = network(X) for X (device, B x 24 FP32). */
int kde_mlp_forward(const void* state, const float* X, int64_t B, float* Y, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* Gradient of the loss mean_rows sum_k (Y_k - T_k)^2 w.r.t. the parameter
 * vector (device, n_params FP32) and the loss (device, 1 FP32; may be NULL);
 * Y (device, B x 3) receives the outputs. T: device, B x 3 FP32. */
int kde_mlp_grad(const void* state, const float* X, const float* T, int64_t B, float* Y, float* grad, float* loss,
                 void* ws, size_t ws_bytes, hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * on the batch (X, T); loss (device, 1 FP32, may be NULL) receives the batch
 * loss before the step. */
int kde_mlp_train_step(void* state, const float* X, const float* T, int64_t B, float lr, int32_t step, float* loss,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched evaluation: many independent estimates (each its own X, n, H and
 * grid; d may differ between items) computed together. Every pass of the
 * pipeline runs as one launch for all items that share its kernel template
 * (precision and padded length P), with each item owning exactly the
 * workgroups its own size needs, so a batch of B items takes a few dozen
 * launches instead of about 10 B. Results are bit-identical to kde_eval of
 * each item with the same params.
 * ------------------------------------------------------------------------- */

typedef struct kde_batch_item {
    const double* X;          /* device, n x d FP64 samples */
    int64_t n;                /* >= 1 */
    double H[KDE_MAX_D * KDE_MAX_D];   /* bandwidth matrix, d x d row-major in the first d*d entries */
    kde_grid grid;
    void* density;            /* device, prod M_k reals of the batch precision (output) */
    uint64_t* n_dropped;      /* device, may be NULL: samples outside the grid (as kde_bin) */
    const uint64_t* counts;   /* device, may be NULL. If set, the item starts from these
                                 fixed-point counts (as kde_bin writes them; kde_conv
                                 semantics), X and n_dropped are ignored, and n is the
                                 sample count of Eq. (1) */
    double* dot;              /* device, may be NULL. If set, receives
                                 sum_j c_j f_j (c_j the counts in real units, f the
                                 item's density) in FP64, summed in a fixed order */
} kde_batch_item;

typedef struct kde_batch kde_batch;   /* opaque; host memory only */

typedef struct kde_batch_info {
    int32_t count;            /* items */
    int32_t launches;         /* kernel launches per kde_batch_eval */
    size_t ws_bytes;          /* device workspace kde_batch_bind needs */
    int32_t tile[KDE_MAX_D];  /* binning tile in use (the autotuner may change it) */
    int32_t narrow_mask;      /* bit ceil(log2 P) (3 x 2^j lengths share the bit of the next
                                 power of two): strided-axis passes of length P use 4 lines
                                 per workgroup (else the widest shape) */
} kde_batch_info;

/* Plan `count` items with shared params (precision, tau, Q, overrides; the
 * trace fields apply to kde_batch_eval). Validates every item as kde_eval
 * would and returns the first failing status. The items' pointers are kept:
 * X, density and n_dropped must stay valid while the batch is used.
 * *out receives a host object to release with kde_batch_destroy. */
int kde_batch_create(const kde_batch_item* items, int32_t count, const kde_params* params, kde_batch** out);

int kde_batch_query(const kde_batch* b, kde_batch_info* info);

/* Attach the device workspace (256-byte aligned, info.ws_bytes long, owned by
 * the caller) and copy the launch tables into its head on `stream`. The copy
 * reads host memory owned by the batch object: keep the object alive until
 * the stream has passed this point. Must precede kde_batch_eval; binding
 * again (e.g. another workspace) is allowed. */
int kde_batch_bind(kde_batch* b, void* ws, size_t ws_bytes, hipStream_t stream);

/* Enqueue the whole batch (binning, kernel spectra, convolutions) on `stream`.
 * Only kernel launches and event records: capturable in a HIP graph, which
 * then replays the batch on whatever the items' X buffers hold. Calls on one
 * bound workspace must not overlap. */
int kde_batch_eval(const kde_batch* b, hipStream_t stream);

/* Autotuner: times kde_batch_eval (reps runs per candidate, HIP events) over
 * the binning tile shapes that fit the workspace and, for each padded length
 * on a strided axis, the wide and narrow workgroup shapes; keeps the fastest
 * and rebinds. Synchronises `stream`; overwrites the densities. None of the
 * choices changes any result bit. */
int kde_batch_tune(kde_batch* b, int32_t reps, hipStream_t stream);

void kde_batch_destroy(kde_batch* b);

/* Batched LSCV objective (bandwidth selection through the binned FFT method,
 * the use Section 5 points to): one kde_lscv per item, all computed together.
 * Each item becomes two convolutions (2H, then H) of its counts with FP64 dot
 * products, as in kde_lscv, and the batch ends with one launch that combines
 * each item's two dots on the device into item.out. The densities and dots
 * live in the batch workspace. The result is bit-identical to kde_lscv of the
 * item with the same params. Validates every item as kde_lscv would (n >= 2,
 * non-null counts and out, H and 2H within the planner's limits) and returns
 * the first failing status. The returned batch is used with kde_batch_query
 * (which counts two items per problem), kde_batch_bind, kde_batch_eval (which
 * then writes every item.out), kde_batch_tune and kde_batch_destroy. */
typedef struct kde_lscv_item {
    const uint64_t* counts;   /* device, prod M_k uint64 fixed-point counts (kde_bin) */
    int64_t n;                /* sample count, >= 2 */
    double H[KDE_MAX_D * KDE_MAX_D];   /* bandwidth matrix, d x d row-major in the first d*d entries */
    kde_grid grid;
    double* out;              /* device, 3 doubles: {LSCV, first term, second term} */
} kde_lscv_item;

int kde_lscv_batch_create(const kde_lscv_item* items, int32_t count, const kde_params* params, kde_batch** out);

/* Static description of a status code. */
const char* kde_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* KDE_MI355X_H */
