// C ABI of the binned FFT KDE (declared in include/kde.h): host planner in
// FP64 and the orchestration of the gfx950 kernels.
//
// Planner (Gramacki & Gramacki, arXiv 1508.02766):
//   delta_k = (hi_k - lo_k) / (M_k - 1)                       Eq. (4)
//   H = R R' (Cholesky), |H| = prod R_kk^2, H^-1 = R^-T R^-1  (K_H of Eq. 1)
//   lambda_max(H): closed form for d <= 2, cyclic Jacobi for d >= 3
//   L_k = min(M_k - 1, ceil(tau sqrt(lambda_max) / delta_k))  Eq. (15)
//         (or tau sqrt(H_kk) with kde_params.extent = 1)
//   P_k = smallest 2^j >= max(16, M_k + L_k), or for d >= 3 the  zero padding, Section 4.1
//         smallest 3 x 2^j >= 48 when that is shorter            (highly composite lengths;
//         (kde_params.lengths: 3 x 2^j also in 2-D, or 2^j only)  kde_params.lengths)
//   k_0 = n^-1 (2 pi)^-d/2 |H|^-1/2                            Eq. (6) with Eq. (1)
//
// The lag box is placed circularly (lag l at l mod P_k, the true negative
// lags of Eq. 12 rather than Wand's mirror of Eq. 8) and the counts at the
// origin; P_k >= M_k + L_k makes the circular convolution equal to Eq. (7) on
// the window [0, M_k), which replaces the extraction of Eq. (14).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/kde.h"
#include "kde_internal.h"

namespace kde {
KernelTiming& kernel_timing() {
    thread_local KernelTiming t;
    return t;
}
}  // namespace kde

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kTauDefault = 3.7;   // Section 4.2, after Eq. (15)
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Row pitch (complex elements) of half spectra along the last axis: P/2 + 1
// bins, padded to a multiple of 16 so that every 16-column block a strided
// pass reads starts on a 128-byte boundary.
int64_t half_pitch(int P) { return (static_cast<int64_t>(P) / 2 + 1 + 15) / 16 * 16; }

struct Layout {
    // offsets into the convolution workspace
    size_t khat = 0, kt1 = 0, kt2 = 0, kt3 = 0, z1 = 0, z2 = 0, z3 = 0, total = 0;
};

struct BinLayout {
    // offsets into the binning workspace (tiled path)
    size_t hist = 0, tot = 0, drops = 0, records = 0, seg = 0, total = 0;
};

struct Plan {
    kde_plan pub;
    int64_t M[kde::kMaxD];              // grid nodes per axis
    double A[kde::kMaxD * kde::kMaxD];  // A_ab = delta_a delta_b (H^-1)_ab at [a kMaxD + b]
    double tau;
    Layout lay;
    size_t counts_bytes;
    bool tiled;       // tiled binning (else global atomics)
    bool store;       // d >= 2: the real spectrum is stored on the whole padded grid
    kde::TileGeom tg;
    BinLayout blay;
};

// Tile geometry of the binning pass: 32 x 32 cells in 2-D, 8 x 16 x 32 in
// 3-D, 8^4 in 4-D, 1024 in 1-D, or the caller's tile (clamped to the grid),
// widened until the tile count fits the per-workgroup histogram. Returns false
// when the tiled path cannot be used: too many cells per tile, records wider
// than 64 bits, or n 2^d >= 2^32.
bool plan_tiles(int d, const int64_t* M, int Q, int64_t n, const int* tile, kde::TileGeom* tg, BinLayout* bl) {
    kde::TileGeom g{};
    static const int base[kde::kMaxD][kde::kMaxD] = {{1024}, {32, 32}, {8, 16, 32}, {8, 8, 8, 8}};
    for (int k = 0; k < d; ++k) {
        int T = tile[k] > 0 ? tile[k] : base[d - 1][k];
        while (T > 1 && T / 2 >= M[k]) T /= 2;
        g.T[k] = T;
    }
    for (;;) {
        int64_t nt = 1;
        int worst = 0;
        for (int k = 0; k < d; ++k) {
            g.nt[k] = static_cast<int>((M[k] + g.T[k] - 1) / g.T[k]);
            nt *= g.nt[k];
            if (g.nt[k] > g.nt[worst]) worst = k;
        }
        if (nt <= kde::kMaxTiles) {
            g.ntiles = static_cast<int>(nt);
            break;
        }
        g.T[worst] *= 2;
    }
    int64_t cells = 1;
    int bits = 0;
    g.qbits = Q + 1;
    for (int k = 0; k < d; ++k) {
        cells *= g.T[k];
        int lg = 0;
        while ((1 << lg) < g.T[k]) ++lg;
        g.logT[k] = lg;
        g.jbits[k] = lg + 1;
        bits += g.jbits[k] + g.qbits;
    }
    if (cells > kde::kMaxTileCells || bits > 64) return false;
    g.tile_cells = static_cast<int>(cells);
    g.max_records = n << d;
    if (n <= 0 || g.max_records >= (int64_t(1) << 32)) return false;
    g.S = kde::kSegment;
    g.nchunk = (n + kde::kBinChunk - 1) / kde::kBinChunk;
    g.max_segments = g.ntiles + (g.max_records + g.S - 1) / g.S;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    bl->hist = take(static_cast<size_t>(g.nchunk) * g.ntiles * 4);
    bl->tot = take(static_cast<size_t>(g.ntiles) * 4);
    bl->drops = take(static_cast<size_t>(g.nchunk) * 4);
    bl->records = take(static_cast<size_t>(g.max_records) * 8);
    bl->seg = take(static_cast<size_t>(g.max_segments) * 16);
    bl->total = off;
    *tg = g;
    return true;
}

// H (d x d, row-major) must be finite, symmetric (|H - H'| <= 1e-12 max|H|)
// and positive definite (Section 1): Hs = (H + H') / 2 and its Cholesky
// factor R (lower triangular, Hs = R R').
int factor_bandwidth(const double* H, int d, double (&Hs)[kde::kMaxD][kde::kMaxD],
                     double (&R)[kde::kMaxD][kde::kMaxD]) {
    double hmax = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const double v = H[i * d + j];
            if (!std::isfinite(v)) return KDE_ERR_NOT_SPD;
            hmax = std::fmax(hmax, std::fabs(v));
        }
    if (!(hmax > 0.0)) return KDE_ERR_NOT_SPD;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            if (std::fabs(H[i * d + j] - H[j * d + i]) > 1e-12 * hmax) return KDE_ERR_NOT_SPD;
            Hs[i][j] = 0.5 * (H[i * d + j] + H[j * d + i]);
        }
    for (int j = 0; j < d; ++j) {
        double s = Hs[j][j];
        for (int k = 0; k < j; ++k) s -= R[j][k] * R[j][k];
        if (!(s > 0.0)) return KDE_ERR_NOT_SPD;
        R[j][j] = std::sqrt(s);
        for (int i = j + 1; i < d; ++i) {
            double t = Hs[i][j];
            for (int k = 0; k < j; ++k) t -= R[i][k] * R[j][k];
            R[i][j] = t / R[j][j];
        }
    }
    return KDE_OK;
}

#define KDE_PLAN_CHECK(expr)           \
    do {                               \
        const int rc_ = (expr);        \
        if (rc_ != KDE_OK) return rc_; \
    } while (0)

// Validation and derived quantities. need_H: validate and factor H;
// n_min: the smallest admissible sample count (1 where Eq. 1 divides by n).
int make_plan(const double* H, int64_t n, int64_t n_min, bool need_H, const kde_grid* g,
              const kde_params* prm, Plan* out) {
    if (!g || !out) return KDE_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    kde_plan& p = out->pub;
    const int d = g->d;
    if (d < 1 || d > kde::kMaxD) return KDE_ERR_ARG;
    if (n < n_min) return KDE_ERR_ARG;
    p.d = d;
    for (int k = 0; k < d; ++k) out->M[k] = g->M[k];
    for (int k = 0; k < d; ++k) {
        if (g->M[k] < 2 || g->M[k] > (int64_t(1) << 24)) return KDE_ERR_ARG;
        if (!std::isfinite(g->lo[k]) || !std::isfinite(g->hi[k]) || !(g->hi[k] > g->lo[k])) return KDE_ERR_ARG;
        p.delta[k] = (g->hi[k] - g->lo[k]) / static_cast<double>(g->M[k] - 1);
        if (!std::isfinite(p.delta[k]) || !(p.delta[k] > 0.0)) return KDE_ERR_ARG;
    }
    // options
    double tau = kTauDefault;
    int prec = KDE_F32, Q = 32 / d;
    int Lovr[kde::kMaxD] = {}, tile[kde::kMaxD] = {};
    int extent = 0, lengths = 0;
    if (prm) {
        if (std::isnan(prm->tau) || std::isinf(prm->tau)) return KDE_ERR_ARG;
        if (prm->tau > 0.0) tau = prm->tau;
        if (prm->prec != 0) {
            if (prm->prec != KDE_F32 && prm->prec != KDE_F64) return KDE_ERR_ARG;
            prec = prm->prec;
        }
        if (prm->Q != 0) {
            if (prm->Q < 1 || d * prm->Q > 62) return KDE_ERR_ARG;
            Q = prm->Q;
        }
        for (int k = 0; k < d; ++k) {
            if (prm->L[k] < 0 || prm->L[k] > g->M[k] - 1) return KDE_ERR_ARG;
            Lovr[k] = prm->L[k];
        }
        int64_t tcells = 1;
        for (int k = 0; k < d; ++k) {
            const int T = prm->tile[k];
            if (T < 0 || T > kde::kMaxTileCells || (T & (T - 1)) != 0) return KDE_ERR_ARG;
            tile[k] = T;
            tcells *= T > 0 ? T : 1;
        }
        if (tcells > kde::kMaxTileCells) return KDE_ERR_ARG;
        if (prm->extent != 0 && prm->extent != 1) return KDE_ERR_ARG;
        if (prm->reuse_spectrum != 0 && prm->reuse_spectrum != 1) return KDE_ERR_ARG;
        if (prm->store_spectrum != 0 && prm->store_spectrum != 1) return KDE_ERR_ARG;
        if (prm->lengths < 0 || prm->lengths > 2) return KDE_ERR_ARG;
        lengths = prm->lengths;
        out->store = prm->store_spectrum == 1 && d >= 2;
        extent = prm->extent;
        if (prm->trace_events && prm->trace_capacity < 0) return KDE_ERR_ARG;
    }
    p.prec = prec;
    p.Q = Q;
    out->tau = tau;
    // n 2^(dQ) must fit in uint64 (each sample adds exactly 2^(dQ))
    if (n > 0 && (static_cast<uint64_t>(n) > (~uint64_t(0) >> (d * Q)))) return KDE_ERR_OVERFLOW;

    int64_t cells = 1;
    for (int k = 0; k < d; ++k) cells *= g->M[k];
    out->counts_bytes = static_cast<size_t>(cells) * sizeof(uint64_t);
    out->tiled = plan_tiles(d, g->M, Q, n, tile, &out->tg, &out->blay);
    p.bin_ws_bytes = out->tiled ? out->blay.total : 0;
    if (!need_H) return KDE_OK;

    // H: finite, symmetric, positive definite
    if (!H) return KDE_ERR_ARG;
    double Hs[kde::kMaxD][kde::kMaxD] = {};
    double R[kde::kMaxD][kde::kMaxD] = {};
    KDE_PLAN_CHECK(factor_bandwidth(H, d, Hs, R));
    double det = 1.0;
    for (int k = 0; k < d; ++k) det *= R[k][k] * R[k][k];
    // inverse of the lower-triangular factor, then H^-1 = R^-T R^-1
    double Ri[kde::kMaxD][kde::kMaxD] = {};
    for (int j = 0; j < d; ++j) {
        Ri[j][j] = 1.0 / R[j][j];
        for (int i = j + 1; i < d; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += R[i][k] * Ri[k][j];
            Ri[i][j] = -s / R[i][i];
        }
    }
    double Hinv[kde::kMaxD][kde::kMaxD] = {};
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += Ri[k][a] * Ri[k][b];
            Hinv[a][b] = s;
        }
    // largest eigenvalue
    double lam = 0.0;
    if (d == 1) {
        lam = Hs[0][0];
    } else if (d == 2) {
        lam = 0.5 * (Hs[0][0] + Hs[1][1]) + std::hypot(0.5 * (Hs[0][0] - Hs[1][1]), Hs[0][1]);
    } else {
        // cyclic Jacobi rotations (Golub & Van Loan, Section 8.5) until the
        // off-diagonal mass is negligible; lambda_max is the largest diagonal entry
        double a[kde::kMaxD][kde::kMaxD];
        std::memcpy(a, Hs, sizeof(a));
        for (int sweep = 0; sweep < 60; ++sweep) {
            double off = 0.0, diag = 0.0;
            for (int i = 0; i < d; ++i) {
                diag += a[i][i] * a[i][i];
                for (int j = i + 1; j < d; ++j) off += a[i][j] * a[i][j];
            }
            if (off <= 1e-36 * diag) break;
            for (int P = 0; P < d; ++P)
                for (int Qi = P + 1; Qi < d; ++Qi) {
                    const double apq = a[P][Qi];
                    if (apq == 0.0) continue;
                    const double theta = (a[Qi][Qi] - a[P][P]) / (2.0 * apq);
                    const double t =
                        (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                    const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                    a[P][P] -= t * apq;
                    a[Qi][Qi] += t * apq;
                    a[P][Qi] = a[Qi][P] = 0.0;
                    for (int r = 0; r < d; ++r) {
                        if (r == P || r == Qi) continue;
                        const double arp = a[r][P], arq = a[r][Qi];
                        a[r][P] = a[P][r] = c * arp - s * arq;
                        a[r][Qi] = a[Qi][r] = s * arp + c * arq;
                    }
                }
        }
        lam = a[0][0];
        for (int k = 1; k < d; ++k) lam = std::fmax(lam, a[k][k]);
    }
    p.lambda_max = lam;
    p.det_H = det;
    p.norm = 1.0 / (static_cast<double>(n) * std::pow(kTwoPi, 0.5 * d) * std::sqrt(det));
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) out->A[a * kde::kMaxD + b] = p.delta[a] * p.delta[b] * Hinv[a][b];

    // truncation (Eq. 15) and padded lengths
    int64_t lag_count = 1;
    for (int k = 0; k < d; ++k) {
        int L = Lovr[k];
        if (L == 0) {
            // Eq. (15), or the axis-k half width of the ellipsoid u' H^-1 u <= tau^2
            const double half = extent == 1 ? std::sqrt(Hs[k][k]) : std::sqrt(std::fabs(lam));
            const double x = std::ceil(tau * half / p.delta[k]);
            const double cap = static_cast<double>(g->M[k] - 1);
            L = static_cast<int>(x < cap ? x : cap);
        }
        p.L[k] = L;
        // the shortest highly composite length (Section 4.1) that holds the window and the
        // lags of the circular layout: 2^k, or in 3-D and 4-D 3 x 2^k when that is shorter.
        // There every pass has thousands of lines and is bound by its bytes and arithmetic;
        // in 1-D and 2-D the few long lines are latency-bound, and the 12 points per thread
        // of a 3 x 2^k line would leave most of the GPU idle (512^2: 45 -> 52 us per step).
        // kde_params.lengths takes 3 x 2^k in 2-D too (batches), or 2^k only.
        int64_t P = kde::kMinP;
        while (P < g->M[k] + L) P *= 2;
        if (P > kde::kMaxP) return KDE_ERR_SIZE;
        const bool tri = lengths == 0 ? d >= 3 : lengths == 1 && d >= 2;
        if (tri && P >= 64 && 3 * (P / 4) >= g->M[k] + L) P = 3 * (P / 4);
        p.P[k] = static_cast<int32_t>(P);
        lag_count *= 2 * L + 1;
    }
    const size_t rs = prec == KDE_F64 ? 8 : 4, cs = 2 * rs;
    p.lag_count = lag_count;
    p.lag_bytes = static_cast<size_t>(lag_count) * rs;
    p.density_bytes = static_cast<size_t>(cells) * rs;

    // workspace layout of the convolution
    Layout& L = out->lay;
    const int64_t M0 = g->M[0], M1 = d > 1 ? g->M[1] : 1;
    const int64_t P1 = d > 1 ? p.P[1] : 1;
    const int64_t Hl = d == 1 ? p.P[0] / 2 + 1 : half_pitch(p.P[d - 1]);   // row pitch of half spectra
    const int64_t n0 = 2 * p.L[0] + 1, n1 = d > 1 ? 2 * p.L[1] + 1 : 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    if (d == 1) {
        L.khat = take(static_cast<size_t>(Hl) * rs);
        L.z1 = take(static_cast<size_t>(Hl) * cs);
    } else if (d == 2) {
        L.kt1 = take(static_cast<size_t>(n0 * Hl) * cs);
        L.z1 = take(static_cast<size_t>(M0 * Hl) * cs);
    } else if (d == 3) {
        L.kt1 = take(static_cast<size_t>(n0 * n1 * Hl) * cs);
        L.kt2 = take(static_cast<size_t>(n0 * P1 * Hl) * cs);
        L.z1 = take(static_cast<size_t>(M0 * M1 * Hl) * cs);
        L.z2 = take(static_cast<size_t>(M0 * P1 * Hl) * cs);
    } else {
        // 4-D: spectrum [n0][n1][n2] -> [n0][n1][P2] -> [n0][P1][P2], counts
        // [M0][M1][M2] -> [M0][M1][P2] -> [M0][P1][P2] (rows of Hl half-spectrum bins)
        const int64_t M2 = g->M[2], P2 = p.P[2], n2 = 2 * p.L[2] + 1;
        L.kt1 = take(static_cast<size_t>(n0 * n1 * n2 * Hl) * cs);
        L.kt2 = take(static_cast<size_t>(n0 * n1 * P2 * Hl) * cs);
        L.kt3 = take(static_cast<size_t>(n0 * P1 * P2 * Hl) * cs);
        L.z1 = take(static_cast<size_t>(M0 * M1 * M2 * Hl) * cs);
        L.z2 = take(static_cast<size_t>(M0 * M1 * P2 * Hl) * cs);
        L.z3 = take(static_cast<size_t>(M0 * P1 * P2 * Hl) * cs);
    }
    if (out->store) {
        // the real spectrum [P0][P1 .. P(d-2)][Hl]
        int64_t lines = Hl;
        for (int k = 0; k < d - 1; ++k) lines *= p.P[k];
        L.khat = take(static_cast<size_t>(lines) * rs);
    }
    L.total = off;
    p.conv_ws_bytes = L.total;
    p.eval_ws_bytes = align_up(out->counts_bytes) + align_up(p.bin_ws_bytes) + L.total;
    return KDE_OK;
}

// Optional per-kernel timing (kde_params.trace_*): pass i of the call gets the
// event pair (2i, 2i + 1), stamped by its kernels' own dispatches.
struct Tracer {
    const kde_params* prm;
    hipStream_t s;
    int n = 0;
    int pairs = 0;
    bool on = false;
    Tracer(const kde_params* p, hipStream_t st) : prm(p), s(st) {
        on = prm && prm->trace_events && prm->trace_capacity >= 2;
        pairs = on ? prm->trace_capacity / 2 : 0;
    }
    // Stamped launches cannot be captured into a graph.
    int start() {
        if (!on) return KDE_OK;
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) != hipSuccess) return KDE_ERR_HIP;
        return st == hipStreamCaptureStatusNone ? KDE_OK : KDE_ERR_ARG;
    }
    // Runs f, which launches the kernels of one pass (returns a KDE_* code).
    template <typename F>
    int pass(const char* name, F&& f) {
        if (!on || n >= pairs) return f();
        kde::KernelTiming& t = kde::kernel_timing();
        t.start = prm->trace_events[2 * n];
        t.stop = prm->trace_events[2 * n + 1];
        t.launched = 0;
        const int r = f();
        const int launched = t.launched;
        t = kde::KernelTiming{};
        if (launched > 0) {
            if (prm->trace_names) prm->trace_names[n] = name;
            ++n;
        }
        return r;
    }
    void finish() {
        if (prm && prm->trace_count) *prm->trace_count = on ? n : 0;
    }
};

#define KDE_TRY(expr)                                 \
    do {                                              \
        if ((expr) != hipSuccess) return KDE_ERR_HIP; \
    } while (0)

#define KDE_CHECK(expr)              \
    do {                             \
        const int rc_ = (expr);      \
        if (rc_ != KDE_OK) return rc_; \
    } while (0)

// One kernel launch of the pipeline for one problem: which kernel (kind and
// template parameters), its argument struct, and the workgroups it takes in a
// batched launch. The single-instance path launches passes as they are
// produced; the batched path collects them and launches all passes with the
// same kernel together.
enum PassKind : int { kPassZero, kPassBinAtomic, kPassBin, kPassRowR2C, kPassRowC2R, kPassCols, kPassDotPartial,
                      kPassDotFinal, kPassHistKspec, kPassScanKcol };

struct Pass {
    PassKind kind;
    int prec = 0, P = 0, sub = 0, d = 0;   // sub: bin stage / row input kind / c2r multiplier / column mode
    int narrow = -1;                       // column passes: -1 by launch size, 0 wide, 1 four lines
    int order = 0;                         // position in the pipeline (increasing along an instance)
    const char* name = "";
    int64_t blocks = 0;                    // workgroups in a batched launch
    size_t lds = 0;                        // dynamic LDS (binning stages)
    size_t size = 0;                       // bytes of args
    alignas(16) unsigned char args[512];
    // kPassZero / kPassBinAtomic
    uint64_t* zptr = nullptr;
    int64_t zcount = 0;
    kde::BinConsts bc{};
    const double* X = nullptr;
    int64_t n = 0;
    uint64_t* counts = nullptr;
    uint64_t* n_dropped = nullptr;

    template <typename T>
    void set_args(const T& a) {
        static_assert(sizeof(T) <= sizeof(args), "argument struct too large");
        std::memcpy(args, &a, sizeof(T));
        size = sizeof(T);
    }
};

int exec_pass(const Pass& p, hipStream_t s) {
    hipError_t e = hipSuccess;
    switch (p.kind) {
        case kPassZero: e = kde::launch_zero_u64(p.zptr, p.zcount, s); break;
        case kPassBinAtomic: e = kde::launch_bin(p.bc, p.X, p.n, p.counts, p.n_dropped, s); break;
        case kPassBin:
            e = kde::launch_bin_stage(p.sub, *reinterpret_cast<const kde::BinArgs*>(p.args), s);
            break;
        case kPassRowR2C: e = kde::launch_rows_r2c(p.prec, p.P, p.sub, p.d, p.args, s); break;
        case kPassRowC2R: e = kde::launch_rows_c2r(p.prec, p.P, p.args, s); break;
        case kPassCols:
            e = kde::launch_cols(p.prec, p.P, p.sub, p.narrow, *reinterpret_cast<const kde::ColArgs*>(p.args), s);
            break;
        case kPassHistKspec: e = kde::launch_hist_kspec(p.prec, p.P, p.d, p.args, s); break;
        case kPassScanKcol:
            e = kde::launch_scan_kcol(p.prec, p.P, *reinterpret_cast<const kde::ScanColArgs*>(p.args), s);
            break;
        case kPassDotPartial:
        case kPassDotFinal:
            // the single-problem path runs both stages through launch_dot
            return KDE_ERR_ARG;
    }
    return e == hipSuccess ? KDE_OK : KDE_ERR_HIP;
}

// Consumer of the passes of one stream of work.
struct Emit {
    virtual int operator()(const Pass& p) = 0;
    virtual ~Emit() = default;
};

// Launch at once (and mark the trace).
struct Direct : Emit {
    hipStream_t s;
    Tracer& tr;
    Direct(hipStream_t st, Tracer& t) : s(st), tr(t) {}
    int operator()(const Pass& p) override {
        return tr.pass(p.name, [&] { return exec_pass(p, s); });
    }
};

// Collect for a batched launch.
struct Collect : Emit {
    std::vector<Pass>& out;
    explicit Collect(std::vector<Pass>& o) : out(o) {}
    int operator()(const Pass& p) override {
        out.push_back(p);
        return KDE_OK;
    }
};

kde::BinArgs bin_args(const Plan& pl, const kde::BinConsts& c, const double* X, int64_t n, uint64_t* counts,
                      uint64_t* n_dropped, char* ws) {
    const BinLayout& b = pl.blay;
    kde::BinArgs a{};
    a.X = X;
    a.n = n;
    a.c = c;
    a.g = pl.tg;
    a.w.hist = reinterpret_cast<uint32_t*>(ws + b.hist);
    a.w.tot = reinterpret_cast<uint32_t*>(ws + b.tot);
    a.w.drops = reinterpret_cast<uint32_t*>(ws + b.drops);
    a.w.records = reinterpret_cast<uint64_t*>(ws + b.records);
    a.w.seg = reinterpret_cast<uint4*>(ws + b.seg);
    a.counts = counts;
    a.n_dropped = reinterpret_cast<unsigned long long*>(n_dropped);
    return a;
}

kde::BinConsts bin_consts(const Plan& pl, const kde_grid* g) {
    const int d = pl.pub.d;
    kde::BinConsts c{};
    c.d = d;
    c.Q = pl.pub.Q;
    int64_t cells = 1;
    for (int k = d - 1; k >= 0; --k) {
        c.stride[k] = cells;
        cells *= g->M[k];
    }
    for (int k = 0; k < d; ++k) {
        c.M[k] = g->M[k];
        c.lo[k] = g->lo[k];
        c.delta[k] = pl.pub.delta[k];
        c.top[k] = static_cast<double>(g->M[k] - 1);
    }
    return c;
}

// Binning (Section 2, first step): the four tiled stages, or zero fill and
// global atomics where the tiled path does not apply. With `spec` (the
// kernel-spectrum row pass) the histogram stage and that pass share one
// launch; with `spec_col` (the 3-D spectrum's strided pass) the scan stage
// and that pass do.
int run_bin(const Plan& pl, const double* X, int64_t n, const kde_grid* g, uint64_t* counts, uint64_t* n_dropped,
            char* ws, Emit& emit, const Pass* spec = nullptr, const Pass* spec_col = nullptr) {
    const kde::BinConsts c = bin_consts(pl, g);
    int64_t cells = 1;
    for (int k = 0; k < pl.pub.d; ++k) cells *= g->M[k];
    if (pl.tiled && n > 0) {
        static const char* names[4] = {"bin_hist", "bin_scan", "bin_scatter", "bin_accum"};
        const kde::BinArgs a = bin_args(pl, c, X, n, counts, n_dropped, ws);
        for (int st = kde::kBinHist; st <= kde::kBinAccum; ++st) {
            if (st == kde::kBinHist && spec) {
                Pass f;
                f.kind = kPassHistKspec;
                f.prec = spec->prec;
                f.P = spec->P;
                f.d = pl.pub.d;
                f.order = st;
                f.name = "hist_kspec";
                if (spec->prec == KDE_F64) {
                    kde::HistSpecArgs<double> sa{};
                    sa.bin = a;
                    std::memcpy(&sa.row, spec->args, sizeof(sa.row));
                    f.set_args(sa);
                } else {
                    kde::HistSpecArgs<float> sa{};
                    sa.bin = a;
                    std::memcpy(&sa.row, spec->args, sizeof(sa.row));
                    f.set_args(sa);
                }
                KDE_CHECK(emit(f));
                continue;
            }
            if (st == kde::kBinScan && spec_col) {
                Pass f;
                f.kind = kPassScanKcol;
                f.prec = spec_col->prec;
                f.P = spec_col->P;
                f.d = pl.pub.d;
                f.order = st;
                f.name = "scan_kcol";
                kde::ScanColArgs sa{};
                sa.bin = a;
                std::memcpy(&sa.col, spec_col->args, sizeof(sa.col));
                f.set_args(sa);
                KDE_CHECK(emit(f));
                continue;
            }
            Pass p;
            p.kind = kPassBin;
            p.sub = st;
            p.d = pl.pub.d;
            p.order = st;
            p.name = names[st];
            p.blocks = kde::bin_stage_batch_blocks(st, pl.tg);
            p.lds = kde::bin_stage_lds(st, pl.tg);
            p.set_args(a);
            KDE_CHECK(emit(p));
        }
        return KDE_OK;
    }
    Pass z;
    z.kind = kPassZero;
    z.name = "zero_counts";
    z.zptr = counts;
    z.zcount = cells;
    KDE_CHECK(emit(z));
    if (n_dropped) {
        z.name = "zero_dropped";
        z.order = 1;
        z.zptr = n_dropped;
        z.zcount = 1;
        KDE_CHECK(emit(z));
    }
    if (n > 0) {
        Pass b;
        b.kind = kPassBinAtomic;
        b.order = 2;
        b.name = "bin";
        b.bc = c;
        b.X = X;
        b.n = n;
        b.counts = counts;
        b.n_dropped = n_dropped;
        KDE_CHECK(emit(b));
    }
    return KDE_OK;
}

// Stage views of the convolution workspace.
struct ConvBufs {
    void *khat, *kt1, *kt2, *kt3, *z1, *z2, *z3;
};

ConvBufs conv_bufs(const Plan& pl, char* ws) {
    const Layout& L = pl.lay;
    return {ws + L.khat, ws + L.kt1, ws + L.kt2, ws + L.kt3, ws + L.z1, ws + L.z2, ws + L.z3};
}

Pass row_r2c_pass(const Plan& pl, int P, int kind, const void* in, const kde::GaussLag* gl, int64_t nrows,
                  int64_t in_ld, int len, void* out, int64_t out_ld, int order, const char* name) {
    Pass p;
    p.kind = kPassRowR2C;
    p.prec = pl.pub.prec;
    p.P = P;
    p.sub = kind;
    p.d = kind == kde::kRowGaussCirc ? pl.pub.d : 1;
    p.order = order;
    p.name = name;
    p.blocks = kde::rows_pass_blocks(P, kind == kde::kRowCountsU64 ? 0 : 1, nrows);
    if (p.prec == KDE_F64)
        p.set_args(kde::make_row_args<double>(in, gl, nrows, in_ld, len, out, out_ld));
    else
        p.set_args(kde::make_row_args<float>(in, gl, nrows, in_ld, len, out, out_ld));
    return p;
}

Pass row_c2r_pass(const Plan& pl, int P, const void* in, int64_t nrows, int64_t in_ld, const void* mult, void* out,
                  int64_t out_ld, int mout, double scale, int order, const char* name) {
    Pass p;
    p.kind = kPassRowC2R;
    p.prec = pl.pub.prec;
    p.P = P;
    p.sub = mult ? 1 : 0;
    p.order = order;
    p.name = name;
    p.blocks = kde::rows_pass_blocks(P, 2, nrows);
    if (p.prec == KDE_F64)
        p.set_args(kde::make_c2r_args<double>(in, nrows, in_ld, mult, out, out_ld, mout, scale));
    else
        p.set_args(kde::make_c2r_args<float>(in, nrows, in_ld, mult, out, out_ld, mout, scale));
    return p;
}

// nmask < 0: workgroup shape chosen at launch from its size; else bit
// ceil(log2 P) of nmask selects the narrow shape for length P.
Pass cols_pass(const Plan& pl, int P, int mode, const kde::ColArgs& a, int nmask, int order, const char* name) {
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    const int narrow = nmask < 0 ? -1 : (nmask >> lg) & 1;
    Pass p;
    p.kind = kPassCols;
    p.prec = pl.pub.prec;
    p.P = P;
    p.sub = mode;
    p.narrow = narrow;
    p.order = order;
    p.name = name;
    p.blocks = kde::cols_pass_blocks(p.prec, P, narrow == 1, a.W, a.outer);
    p.set_args(a);
    return p;
}

// Kernel spectrum: lag-box weights computed in place (Eq. 6 over the signed
// box of Eq. 12), transformed along every axis but the slowest (whose
// transform the product pass computes per line unless the plan stores the
// spectrum); real because the box is centrally symmetric and placed circularly.
int run_kspec_lags(const Plan& pl, char* ws, int nmask, Emit& emit) {
    const kde_plan& p = pl.pub;
    const int d = p.d;
    const ConvBufs b = conv_bufs(pl, ws);
    kde::GaussLag gl{};
    for (int i = 0; i < kde::kMaxD * kde::kMaxD; ++i) gl.A[i] = pl.A[i];
    gl.norm = p.norm;
    gl.d = d;
    for (int k = 0; k < kde::kMaxD; ++k) gl.L[k] = k < d ? p.L[k] : 0;
    if (d == 1) {
        const int P0 = p.P[0];
        return emit(row_r2c_pass(pl, P0, kde::kRowGaussCirc, nullptr, &gl, 1, 0, p.L[0], b.khat, P0 / 2 + 1, 0,
                                 "kspec_r2c"));
    }
    if (d == 2) {
        const int P1 = p.P[1];
        const int64_t n0 = 2 * p.L[0] + 1;
        return emit(row_r2c_pass(pl, P1, kde::kRowGaussCirc, nullptr, &gl, n0, 0, p.L[1], b.kt1, half_pitch(P1), 0,
                                 "kspec_r2c"));
    }
    if (d == 4) {
        const int P1 = p.P[1], P2 = p.P[2], P3 = p.P[3];
        const int64_t H3 = P3 / 2 + 1, Hp = half_pitch(P3);
        const int64_t n0 = 2 * p.L[0] + 1, n1 = 2 * p.L[1] + 1, n2 = 2 * p.L[2] + 1;
        KDE_CHECK(emit(row_r2c_pass(pl, P3, kde::kRowGaussCirc, nullptr, &gl, n0 * n1 * n2, 0, p.L[3], b.kt1, Hp,
                                    0, "kspec_r2c")));
        // axis 2: [n0 n1][n2][Hp] -> [n0 n1][P2][Hp]
        kde::ColArgs k2{};
        k2.in = b.kt1;
        k2.out = b.kt2;
        k2.W = H3;
        k2.outer = n0 * n1;
        k2.in_os = n2 * Hp;
        k2.in_ps = Hp;
        k2.out_os = static_cast<int64_t>(P2) * Hp;
        k2.out_ps = Hp;
        k2.len = p.L[2];
        KDE_CHECK(emit(cols_pass(pl, P2, kde::kColFwdCirc, k2, nmask, 1, "kspec_col3")));
        // axis 1: [n0][n1][P2 Hp] -> [n0][P1][P2 Hp]; outer index (i0, w2)
        kde::ColArgs k1{};
        k1.in = b.kt2;
        k1.out = b.kt3;
        k1.W = H3;
        k1.outer = n0 * P2;
        k1.ob = P2;
        k1.in_os1 = n1 * P2 * Hp;
        k1.in_os = Hp;
        k1.in_ps = P2 * Hp;
        k1.out_os1 = static_cast<int64_t>(P1) * P2 * Hp;
        k1.out_os = Hp;
        k1.out_ps = P2 * Hp;
        k1.len = p.L[1];
        return emit(cols_pass(pl, P1, kde::kColFwdCirc, k1, nmask, 2, "kspec_col2"));
    }
    const int P1 = p.P[1], P2 = p.P[2];
    const int64_t H2 = P2 / 2 + 1, Hp = half_pitch(P2), n0 = 2 * p.L[0] + 1, n1 = 2 * p.L[1] + 1;
    KDE_CHECK(emit(row_r2c_pass(pl, P2, kde::kRowGaussCirc, nullptr, &gl, n0 * n1, 0, p.L[2], b.kt1, Hp, 0,
                                "kspec_r2c")));
    kde::ColArgs k1{};
    k1.in = b.kt1;
    k1.out = b.kt2;
    k1.W = H2;
    k1.outer = n0;
    k1.in_os = n1 * Hp;
    k1.in_ps = Hp;
    k1.out_os = static_cast<int64_t>(P1) * Hp;
    k1.out_ps = Hp;
    k1.len = p.L[1];
    return emit(cols_pass(pl, P1, kde::kColFwdCirc, k1, nmask, 1, "kspec_col2"));
}

// The slowest axis of the spectrum (d >= 2, stored plans): the lag columns
// transformed along the other axes, [2 L0 + 1][lines], to the real spectrum
// [P0][lines]. Its transform prunes as the product pass's own lag-column
// transform does, so both spectra are the same numbers.
int run_kspec_store(const Plan& pl, char* ws, int nmask, Emit& emit) {
    const kde_plan& p = pl.pub;
    const int d = p.d;
    const ConvBufs b = conv_bufs(pl, ws);
    const int64_t Pl = p.P[d - 1], Hp = half_pitch(static_cast<int>(Pl));
    int64_t mid = 1;   // P1 .. P(d-2)
    for (int k = 1; k < d - 1; ++k) mid *= p.P[k];
    kde::ColArgs ks{};
    ks.in = d == 2 ? b.kt1 : (d == 3 ? b.kt2 : b.kt3);
    ks.out = b.khat;
    ks.W = Pl / 2 + 1;
    ks.outer = mid;
    ks.in_os = Hp;
    ks.out_os = Hp;
    ks.in_ps = mid * Hp;
    ks.out_ps = mid * Hp;
    ks.len = p.L[0];
    return emit(cols_pass(pl, p.P[0], kde::kColFwdCircRe, ks, nmask, 3, "kspec_col1"));
}

int run_kspec(const Plan& pl, char* ws, int nmask, Emit& emit) {
    KDE_CHECK(run_kspec_lags(pl, ws, nmask, emit));
    return pl.store ? run_kspec_store(pl, ws, nmask, emit) : KDE_OK;
}

// Forward transforms of the zero-padded counts that do not need the spectrum.
int run_counts_fwd(const Plan& pl, const uint64_t* counts, const kde_grid* g, char* ws, int nmask, Emit& emit) {
    const kde_plan& p = pl.pub;
    const int d = p.d;
    const ConvBufs b = conv_bufs(pl, ws);
    const int Pl = p.P[d - 1];
    const int64_t Hl = Pl / 2 + 1, Hp = d == 1 ? Hl : half_pitch(Pl);
    const int64_t Ml = g->M[d - 1];
    int64_t rows = 1;
    for (int k = 0; k < d - 1; ++k) rows *= g->M[k];
    KDE_CHECK(emit(row_r2c_pass(pl, Pl, kde::kRowCountsU64, counts, nullptr, rows, Ml, static_cast<int>(Ml), b.z1, Hp,
                                10, "counts_r2c")));
    if (d == 3) {
        const int P1 = p.P[1];
        const int64_t M0 = g->M[0], M1 = g->M[1];
        kde::ColArgs f1{};
        f1.in = b.z1;
        f1.out = b.z2;
        f1.W = Hl;
        f1.outer = M0;
        f1.in_os = M1 * Hp;
        f1.in_ps = Hp;
        f1.out_os = static_cast<int64_t>(P1) * Hp;
        f1.out_ps = Hp;
        f1.len = static_cast<int>(M1);
        KDE_CHECK(emit(cols_pass(pl, P1, kde::kColFwdPrefix, f1, nmask, 11, "counts_col2")));
    }
    if (d == 4) {
        const int P1 = p.P[1], P2 = p.P[2];
        const int64_t M0 = g->M[0], M1 = g->M[1], M2 = g->M[2];
        // axis 2: [M0 M1][M2][Hp] -> [M0 M1][P2][Hp]
        kde::ColArgs f2{};
        f2.in = b.z1;
        f2.out = b.z2;
        f2.W = Hl;
        f2.outer = M0 * M1;
        f2.in_os = M2 * Hp;
        f2.in_ps = Hp;
        f2.out_os = static_cast<int64_t>(P2) * Hp;
        f2.out_ps = Hp;
        f2.len = static_cast<int>(M2);
        KDE_CHECK(emit(cols_pass(pl, P2, kde::kColFwdPrefix, f2, nmask, 11, "counts_col3")));
        // axis 1: [M0][M1][P2 Hp] -> [M0][P1][P2 Hp]; outer index (i0, w2)
        kde::ColArgs f1{};
        f1.in = b.z2;
        f1.out = b.z3;
        f1.W = Hl;
        f1.outer = M0 * P2;
        f1.ob = P2;
        f1.in_os1 = M1 * P2 * Hp;
        f1.in_os = Hp;
        f1.in_ps = P2 * Hp;
        f1.out_os1 = static_cast<int64_t>(P1) * P2 * Hp;
        f1.out_os = Hp;
        f1.out_ps = P2 * Hp;
        f1.len = static_cast<int>(M1);
        KDE_CHECK(emit(cols_pass(pl, P1, kde::kColFwdPrefix, f1, nmask, 12, "counts_col2")));
    }
    return KDE_OK;
}

// Product with the spectrum, inverse transforms, window [0, M_k) and the
// 2^-(dQ) / prod P_k scale.
int run_product_inv(const Plan& pl, const kde_grid* g, void* density, char* ws, int nmask, Emit& emit) {
    const kde_plan& p = pl.pub;
    const int d = p.d;
    const ConvBufs b = conv_bufs(pl, ws);
    double scale = std::ldexp(1.0, -d * p.Q);
    for (int k = 0; k < d; ++k) scale /= static_cast<double>(p.P[k]);
    // a stored spectrum has the real-spectrum layout of the data, [P0][..][Hp] (kt strides)
    const int conv_mode = pl.store ? kde::kColConvSpec : kde::kColConvLag;
    if (d == 1) {
        const int P0 = p.P[0];
        const int64_t H0 = P0 / 2 + 1, M0 = g->M[0];
        return emit(row_c2r_pass(pl, P0, b.z1, 1, H0, b.khat, density, M0, static_cast<int>(M0), scale, 20,
                                 "product_c2r"));
    }
    if (d == 2) {
        const int P0 = p.P[0], P1 = p.P[1];
        const int64_t H1 = P1 / 2 + 1, Hp = half_pitch(P1), M0 = g->M[0], M1 = g->M[1];
        kde::ColArgs ca{};
        ca.in = b.z1;
        ca.out = b.z1;
        ca.kt = pl.store ? b.khat : b.kt1;
        ca.kt_ps = Hp;
        ca.kt_len = p.L[0];
        ca.W = H1;
        ca.outer = 1;
        ca.in_ps = Hp;
        ca.out_ps = Hp;
        ca.len = static_cast<int>(M0);
        ca.mout = static_cast<int>(M0);
        KDE_CHECK(emit(cols_pass(pl, P0, conv_mode, ca, nmask, 20, "conv_col")));
        return emit(row_c2r_pass(pl, P1, b.z1, M0, Hp, nullptr, density, M1, static_cast<int>(M1), scale, 21, "c2r"));
    }
    if (d == 4) {
        const int P0 = p.P[0], P1 = p.P[1], P2 = p.P[2], P3 = p.P[3];
        const int64_t H3 = P3 / 2 + 1, Hp = half_pitch(P3);
        const int64_t M0 = g->M[0], M1 = g->M[1], M2 = g->M[2], M3 = g->M[3];
        // axis 0 over [M0][P1 P2][Hp], lines (w1 w2, w3), in place
        kde::ColArgs cv{};
        cv.in = b.z3;
        cv.out = b.z3;
        cv.kt = pl.store ? b.khat : b.kt3;
        cv.W = H3;
        cv.outer = static_cast<int64_t>(P1) * P2;
        cv.in_os = Hp;
        cv.out_os = Hp;
        cv.kt_os = Hp;
        cv.in_ps = static_cast<int64_t>(P1) * P2 * Hp;
        cv.out_ps = cv.in_ps;
        cv.kt_ps = cv.in_ps;
        cv.kt_len = p.L[0];
        cv.len = static_cast<int>(M0);
        cv.mout = static_cast<int>(M0);
        KDE_CHECK(emit(cols_pass(pl, P0, conv_mode, cv, nmask, 20, "conv_col1")));
        // axis 1: [M0][P1][P2 Hp] -> [M0][M1][P2 Hp]; outer index (i0, w2)
        kde::ColArgs i1{};
        i1.in = b.z3;
        i1.out = b.z2;
        i1.W = H3;
        i1.outer = M0 * P2;
        i1.ob = P2;
        i1.in_os1 = static_cast<int64_t>(P1) * P2 * Hp;
        i1.in_os = Hp;
        i1.in_ps = P2 * Hp;
        i1.out_os1 = M1 * P2 * Hp;
        i1.out_os = Hp;
        i1.out_ps = P2 * Hp;
        i1.mout = static_cast<int>(M1);
        KDE_CHECK(emit(cols_pass(pl, P1, kde::kColInvPrefix, i1, nmask, 21, "inv_col2")));
        // axis 2: [M0 M1][P2][Hp] -> [M0 M1][M2][Hp]
        kde::ColArgs i2{};
        i2.in = b.z2;
        i2.out = b.z1;
        i2.W = H3;
        i2.outer = M0 * M1;
        i2.in_os = static_cast<int64_t>(P2) * Hp;
        i2.in_ps = Hp;
        i2.out_os = M2 * Hp;
        i2.out_ps = Hp;
        i2.mout = static_cast<int>(M2);
        KDE_CHECK(emit(cols_pass(pl, P2, kde::kColInvPrefix, i2, nmask, 22, "inv_col3")));
        return emit(row_c2r_pass(pl, P3, b.z1, M0 * M1 * M2, Hp, nullptr, density, M3, static_cast<int>(M3), scale,
                                 23, "c2r"));
    }
    const int P0 = p.P[0], P1 = p.P[1], P2 = p.P[2];
    const int64_t H2 = P2 / 2 + 1, Hp = half_pitch(P2), M0 = g->M[0], M1 = g->M[1], M2 = g->M[2];
    kde::ColArgs cv{};
    cv.in = b.z2;
    cv.out = b.z2;
    cv.kt = pl.store ? b.khat : b.kt2;
    cv.W = H2;                                  // lines (w2, w3): outer index w2, inner w3
    cv.outer = P1;
    cv.in_os = Hp;
    cv.out_os = Hp;
    cv.kt_os = Hp;
    cv.in_ps = static_cast<int64_t>(P1) * Hp;   // axis-1 element stride
    cv.out_ps = cv.in_ps;
    cv.kt_ps = cv.in_ps;
    cv.kt_len = p.L[0];
    cv.len = static_cast<int>(M0);
    cv.mout = static_cast<int>(M0);
    KDE_CHECK(emit(cols_pass(pl, P0, conv_mode, cv, nmask, 20, "conv_col1")));
    kde::ColArgs i1{};
    i1.in = b.z2;
    i1.out = b.z1;
    i1.W = H2;
    i1.outer = M0;
    i1.in_os = static_cast<int64_t>(P1) * Hp;
    i1.in_ps = Hp;
    i1.out_os = M1 * Hp;
    i1.out_ps = Hp;
    i1.mout = static_cast<int>(M1);
    KDE_CHECK(emit(cols_pass(pl, P1, kde::kColInvPrefix, i1, nmask, 21, "inv_col2")));
    return emit(row_c2r_pass(pl, P2, b.z1, M0 * M1, Hp, nullptr, density, M2, static_cast<int>(M2), scale, 22, "c2r"));
}

// Dot product of the counts with the density (two passes: per-chunk partials,
// then their sum), for the LSCV objective.
int run_dot(const Plan& pl, const uint64_t* counts, const void* density, double* partial, double* out, Emit& emit) {
    int64_t cells = 1;
    for (int k = 0; k < pl.pub.d; ++k) cells *= pl.M[k];
    kde::DotArgs a{};
    a.counts = counts;
    a.f = density;
    a.cells = cells;
    a.scale = std::ldexp(1.0, -pl.pub.d * pl.pub.Q);
    a.partial = partial;
    a.nb = kde::dot_blocks(cells);
    a.out = out;
    Pass p;
    p.kind = kPassDotPartial;
    p.prec = pl.pub.prec;
    p.order = 30;
    p.name = "dot_partial";
    p.blocks = a.nb;
    p.set_args(a);
    KDE_CHECK(emit(p));
    p.kind = kPassDotFinal;
    p.prec = 0;
    p.order = 31;
    p.name = "dot_final";
    p.blocks = 1;
    return emit(p);
}

// A second stream per device on which the kernel spectrum is computed while
// the caller's stream bins and transforms the counts. Created once (default
// priority, non-blocking) and kept for the life of the process; the fork /
// join events order it with the caller's stream, so the work stays capturable
// in a HIP graph. The mutex keeps concurrent callers from interleaving their
// event records.
struct Aux {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool ready = false;
};
std::mutex g_aux_mu;
Aux g_aux[64];

Aux* aux_for(hipStream_t s) {
    int dev = 0;
    if (hipStreamGetDevice(s, &dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    Aux& a = g_aux[dev];
    if (a.ready) return &a;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    bool ok = hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&a.join, hipEventDisableTiming) == hipSuccess;
    if (cur != dev && hipSetDevice(cur) != hipSuccess) ok = false;
    if (!ok) return nullptr;
    a.ready = true;
    return &a;
}

// Runs the three phases of the pipeline: `spec` (the kernel spectrum) on the
// auxiliary stream, `fwd` (binning and forward transforms of the counts) on
// the caller's stream, then `inv` (product and inverse transforms) on the
// caller's stream after both. With tracing on or overlap off, everything runs
// in order on the caller's stream. The fork and join cost the host about as
// much as several kernel launches, so the overlap pays only where the GPU work
// is large and the spectrum does not already share the binning's launches:
// 3-D convolutions from counts and batches (measured with separate spectrum
// launches: 2-D 512^2 60 us serial vs 64 us overlapped; 3-D 128^3 145 vs
// 147 us; a 256-problem batch 1.10 vs 1.12 ms).
template <typename Spec, typename Fwd, typename Inv>
int run_phases(hipStream_t s, Tracer& tr, bool overlap, Spec&& spec, Fwd&& fwd, Inv&& inv) {
    if (overlap && !tr.on) {
        std::lock_guard<std::mutex> lock(g_aux_mu);
        Aux* a = aux_for(s);
        if (a) {
            KDE_TRY(hipEventRecord(a->fork, s));
            KDE_TRY(hipStreamWaitEvent(a->stream, a->fork, 0));
            KDE_CHECK(spec(a->stream));
            KDE_TRY(hipEventRecord(a->join, a->stream));
            KDE_CHECK(fwd(s));
            KDE_TRY(hipStreamWaitEvent(s, a->join, 0));
            return inv(s);
        }
    }
    KDE_CHECK(fwd(s));
    KDE_CHECK(spec(s));
    return inv(s);
}

// ---------------------------------------------------------------------------
// batched evaluation
// ---------------------------------------------------------------------------

// Passes of one kernel template, launched together.
struct Group {
    int phase = 0;                 // 0 spectrum (auxiliary stream), 1 forward, 2 inverse
    Pass key;                      // kernel and template parameters (first member)
    std::vector<int> members;      // indices into Batch::passes, in instance order
    bool batched = false;          // false: zero / atomic binning, launched one by one
    size_t tab_off = 0, start_off = 0, owner_off = 0;
    uint32_t blocks = 0;
    size_t lds = 0;
};

// Workspace of kde_lscv: one density (reused by both convolutions), the two
// dots, the partial sums, and the larger of the two convolution workspaces.
struct LscvLayout {
    size_t density = 0, dots = 0, partial = 0, conv = 0, total = 0;
};

int lscv_plans(const double* H, int64_t n, const kde_grid* g, const kde_params* prm, Plan* p1, Plan* p2,
               LscvLayout* L) {
    if (n < 2 || !H || !g) return KDE_ERR_ARG;
    KDE_CHECK(make_plan(H, n, 1, true, g, prm, p1));
    const int d = p1->pub.d;
    double H2[kde::kMaxD * kde::kMaxD] = {};
    for (int i = 0; i < d * d; ++i) H2[i] = 2.0 * H[i];
    KDE_CHECK(make_plan(H2, n, 1, true, g, prm, p2));
    int64_t cells = 1;
    for (int k = 0; k < d; ++k) cells *= g->M[k];
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L->density = take(p1->pub.density_bytes);
    L->dots = take(2 * sizeof(double));
    L->partial = take(static_cast<size_t>(kde::dot_blocks(cells)) * sizeof(double));
    L->conv = take(std::max(p1->pub.conv_ws_bytes, p2->pub.conv_ws_bytes));
    L->total = off;
    return KDE_OK;
}

bool same_kernel(const Pass& a, const Pass& b) {
    return a.kind == b.kind && a.prec == b.prec && a.P == b.P && a.sub == b.sub && a.d == b.d &&
           a.narrow == b.narrow && a.order == b.order;
}

}  // namespace

struct kde_batch {
    std::vector<kde_batch_item> items;
    kde_params prm{};
    bool has_prm = false;
    int tile[kde::kMaxD] = {};     // binning tile of the current configuration (0: default)
    int narrow_mask = 0;           // bit ceil(log2 P): narrow strided passes of length P
    std::vector<Plan> plans;
    std::vector<size_t> inst_off;  // per item: offset of its eval workspace in ws
    std::vector<char> internal;    // per item: density and dot live in the workspace (LSCV batches)
    // LSCV batches: problem k combines the dots of items 2k (2H) and 2k + 1 (H)
    std::vector<kde::LscvJob> lscv;
    size_t lscv_tab_off = 0;       // offset of the device copy of `lscv` in ws
    size_t table_cap = 0, ws_bytes = 0;
    // the current configuration, laid out for ws
    std::vector<Pass> passes;
    std::vector<Group> groups;
    std::vector<unsigned char> table;
    char* ws = nullptr;
    bool bound = false;
};

namespace {

constexpr int kAllNarrow = ((1 << 13) - 1) & ~((1 << 4) - 1);   // bits log2(P) for P = 16 .. 4096
using TileShape = std::array<int, kde::kMaxD>;
const TileShape kTuneTiles1[] = {{0}, {512}, {2048}, {4096}};
const TileShape kTuneTiles2[] = {{0}, {16, 64}, {64, 16}, {64, 64}, {16, 16}};
const TileShape kTuneTiles3[] = {{0}, {8, 16, 16}, {4, 16, 16}, {16, 16, 16}, {4, 32, 32}};
const TileShape kTuneTiles4[] = {{0}, {4, 8, 8, 16}, {4, 4, 16, 16}, {8, 8, 8, 4}};

// Workspace of one batch item, relative to its base: the counts and binning
// workspace (items that bin), the convolution workspace, the dot partials
// (items with a dot) and, for items whose outputs are internal (LSCV
// batches), the density and the dot.
struct ItemLayout {
    size_t counts = 0, bin = 0, conv = 0, partial = 0, density = 0, dot = 0, total = 0;
};

ItemLayout item_layout(const kde_batch_item& it, const Plan& pl, bool internal) {
    ItemLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    if (!it.counts) {
        L.counts = take(pl.counts_bytes);
        L.bin = take(pl.pub.bin_ws_bytes);
    }
    L.conv = take(pl.pub.conv_ws_bytes);
    int64_t cells = 1;
    for (int k = 0; k < pl.pub.d; ++k) cells *= pl.M[k];
    if (it.dot || internal) L.partial = take(static_cast<size_t>(kde::dot_blocks(cells)) * sizeof(double));
    if (internal) {
        L.density = take(pl.pub.density_bytes);
        L.dot = take(sizeof(double));
    }
    L.total = off;
    return L;
}

kde_params batch_params(const kde_batch& b, const int tile[kde::kMaxD]) {
    kde_params q = b.prm;
    for (int k = 0; k < kde::kMaxD; ++k) q.tile[k] = tile[k];
    return q;
}

int plan_item(const kde_batch& b, const kde_batch_item& it, const int tile[kde::kMaxD], Plan* pl) {
    const kde_params q = batch_params(b, tile);
    return make_plan(it.H, it.n, 1, true, &it.grid, &q, pl);
}

// Binning tile shapes the autotuner tries, the first being the one in use at
// creation: the caller's shape alone if params set one, the items differ in d
// or none of them bins; otherwise the default and the alternatives for that d.
std::vector<TileShape> tile_candidates(const kde_batch& b) {
    std::vector<TileShape> c;
    bool fixed = false;
    for (int k = 0; k < kde::kMaxD; ++k) fixed = fixed || (b.has_prm && b.prm.tile[k]);
    int d = b.items[0].grid.d;
    bool bins = false;
    for (const auto& it : b.items) {
        if (it.grid.d != d) d = 0;
        bins = bins || !it.counts;
    }
    if (fixed || d == 0 || !bins) {   // caller's shape, mixed d, or nothing to bin
        TileShape t{};
        for (int k = 0; k < kde::kMaxD; ++k) t[k] = b.has_prm ? b.prm.tile[k] : 0;
        c.push_back(t);
        return c;
    }
    auto add = [&](const TileShape* t, size_t nt) { c.insert(c.end(), t, t + nt); };
    if (d == 1) add(kTuneTiles1, std::size(kTuneTiles1));
    if (d == 2) add(kTuneTiles2, std::size(kTuneTiles2));
    if (d == 3) add(kTuneTiles3, std::size(kTuneTiles3));
    if (d == 4) add(kTuneTiles4, std::size(kTuneTiles4));
    return c;
}

// Collect every item's passes (workspace base `ws`, possibly null for sizing)
// and group them by phase, pipeline position and kernel.
int build_groups(kde_batch& b, char* ws, std::vector<Pass>& passes, std::vector<Group>& groups, size_t& table_bytes) {
    passes.clear();
    groups.clear();
    const int count = static_cast<int>(b.items.size());
    std::vector<std::vector<Pass>> ph[3];
    for (auto& v : ph) v.resize(count);
    for (int i = 0; i < count; ++i) {
        const kde_batch_item& it = b.items[i];
        const Plan& pl = b.plans[i];
        const ItemLayout lay = item_layout(it, pl, b.internal[i] != 0);
        char* base = ws + b.inst_off[i];
        uint64_t* own_counts = reinterpret_cast<uint64_t*>(base + lay.counts);
        const uint64_t* counts = it.counts ? it.counts : own_counts;
        char* bin_ws = base + lay.bin;
        char* conv_ws = base + lay.conv;
        auto* partial = reinterpret_cast<double*>(base + lay.partial);
        void* density = b.internal[i] ? static_cast<void*>(base + lay.density) : it.density;
        double* dot = b.internal[i] ? reinterpret_cast<double*>(base + lay.dot) : it.dot;
        Collect c0(ph[0][i]), c1(ph[1][i]), c2(ph[2][i]);
        KDE_CHECK(run_kspec(pl, conv_ws, b.narrow_mask, c0));
        if (!it.counts) KDE_CHECK(run_bin(pl, it.X, it.n, &it.grid, own_counts, it.n_dropped, bin_ws, c1));
        KDE_CHECK(run_counts_fwd(pl, counts, &it.grid, conv_ws, b.narrow_mask, c1));
        KDE_CHECK(run_product_inv(pl, &it.grid, density, conv_ws, b.narrow_mask, c2));
        if (dot) KDE_CHECK(run_dot(pl, counts, density, partial, dot, c2));
    }
    for (int phase = 0; phase < 3; ++phase) {
        // all (order, kernel) keys of this phase, by order then first appearance
        std::vector<Pass> keys;
        for (int i = 0; i < count; ++i)
            for (const Pass& p : ph[phase][i]) {
                bool found = false;
                for (const Pass& k : keys) found = found || same_kernel(k, p);
                if (!found) keys.push_back(p);
            }
        std::stable_sort(keys.begin(), keys.end(), [](const Pass& x, const Pass& y) { return x.order < y.order; });
        for (const Pass& k : keys) {
            Group g;
            g.phase = phase;
            g.key = k;
            g.batched = k.kind != kPassZero && k.kind != kPassBinAtomic;
            for (int i = 0; i < count; ++i)
                for (const Pass& p : ph[phase][i])
                    if (same_kernel(k, p)) {
                        g.members.push_back(static_cast<int>(passes.size()));
                        passes.push_back(p);
                    }
            groups.push_back(std::move(g));
        }
    }
    // table layout: per batched group, the argument structs then the offsets
    size_t off = 0;
    for (Group& g : groups) {
        if (!g.batched) continue;
        uint64_t total = 0;
        for (int m : g.members) {
            total += static_cast<uint64_t>(passes[m].blocks);
            g.lds = std::max(g.lds, passes[m].lds);
        }
        if (total >= (uint64_t(1) << 32)) return KDE_ERR_SIZE;
        g.blocks = static_cast<uint32_t>(total);
        g.tab_off = off;
        off = align_up(off + g.members.size() * g.key.size);
        g.start_off = off;
        off = align_up(off + (g.members.size() + 1) * sizeof(uint32_t));
        g.owner_off = off;
        off = align_up(off + static_cast<size_t>(g.blocks) * sizeof(uint32_t));
    }
    table_bytes = off;
    return KDE_OK;
}

// Fill the host copy of the launch tables for the device address `dev`.
void fill_table(const std::vector<Pass>& passes, const std::vector<Group>& groups, std::vector<unsigned char>& t,
                size_t bytes) {
    t.assign(bytes, 0);
    for (const Group& g : groups) {
        if (!g.batched) continue;
        uint32_t acc = 0;
        auto* start = reinterpret_cast<uint32_t*>(t.data() + g.start_off);
        auto* owner = reinterpret_cast<uint32_t*>(t.data() + g.owner_off);
        for (size_t j = 0; j < g.members.size(); ++j) {
            const Pass& p = passes[g.members[j]];
            std::memcpy(t.data() + g.tab_off + j * g.key.size, p.args, p.size);
            start[j] = acc;
            for (int64_t k = 0; k < p.blocks; ++k) owner[acc + k] = static_cast<uint32_t>(j);
            acc += static_cast<uint32_t>(p.blocks);
        }
        start[g.members.size()] = acc;
    }
}

int launch_group(const kde_batch& b, const Group& g, hipStream_t s) {
    if (!g.batched) {
        for (int m : g.members) KDE_CHECK(exec_pass(b.passes[m], s));
        return KDE_OK;
    }
    const char* dev = b.ws;
    kde::BatchMap m{dev + g.tab_off, reinterpret_cast<const uint32_t*>(dev + g.start_off),
                    reinterpret_cast<const uint32_t*>(dev + g.owner_off), static_cast<int>(g.members.size()),
                    g.blocks};
    const Pass& k = g.key;
    hipError_t e = hipSuccess;
    switch (k.kind) {
        case kPassBin: e = kde::launch_bin_stage_batch(k.sub, k.d, m, g.lds, s); break;
        case kPassRowR2C: e = kde::launch_rows_r2c_batch(k.prec, k.P, k.sub, k.d, m, s); break;
        case kPassRowC2R: e = kde::launch_rows_c2r_batch(k.prec, k.P, k.sub != 0, m, s); break;
        case kPassCols: e = kde::launch_cols_batch(k.prec, k.P, k.sub, k.narrow == 1, m, s); break;
        case kPassDotPartial: e = kde::launch_dot_batch(k.prec, false, m, s); break;
        case kPassDotFinal: e = kde::launch_dot_batch(k.prec, true, m, s); break;
        default: return KDE_ERR_ARG;
    }
    return e == hipSuccess ? KDE_OK : KDE_ERR_HIP;
}

int run_batch_phase(const kde_batch& b, int phase, hipStream_t s, Tracer& tr) {
    for (const Group& g : b.groups) {
        if (g.phase != phase) continue;
        KDE_CHECK(tr.pass(g.key.name, [&] { return launch_group(b, g, s); }));
    }
    return KDE_OK;
}

// Plans every item under the configuration (b.tile) and lays the items'
// workspaces out after a table region of b.table_cap bytes.
int layout_batch(kde_batch& b) {
    const int count = static_cast<int>(b.items.size());
    b.plans.assign(count, Plan{});
    for (int i = 0; i < count; ++i) KDE_CHECK(plan_item(b, b.items[i], b.tile, &b.plans[i]));
    return KDE_OK;
}

int rebind(kde_batch& b, hipStream_t s) {
    size_t tb = 0;
    KDE_CHECK(build_groups(b, b.ws, b.passes, b.groups, tb));
    if (tb > b.table_cap) return KDE_ERR_WS;
    fill_table(b.passes, b.groups, b.table, tb);
    if (!b.lscv.empty()) {
        // the combination reads the dots that items 2k and 2k + 1 write into their workspaces
        for (size_t k = 0; k < b.lscv.size(); ++k)
            for (int t = 0; t < 2; ++t) {
                const size_t i = 2 * k + t;
                const ItemLayout lay = item_layout(b.items[i], b.plans[i], true);
                const double* dot = reinterpret_cast<const double*>(b.ws + b.inst_off[i] + lay.dot);
                (t == 0 ? b.lscv[k].dot2H : b.lscv[k].dotH) = dot;
            }
        const size_t bytes = b.lscv.size() * sizeof(kde::LscvJob);
        b.table.resize(b.lscv_tab_off + bytes, 0);
        std::memcpy(b.table.data() + b.lscv_tab_off, b.lscv.data(), bytes);
        tb = b.table.size();
    }
    if (tb > 0) {
        KDE_TRY(hipMemcpyAsync(b.ws, b.table.data(), tb, hipMemcpyHostToDevice, s));
        KDE_TRY(hipStreamSynchronize(s));
    }
    b.bound = true;
    return KDE_OK;
}

// Plans the items, sizes every item's workspace for the largest binning tile
// shape the autotuner may pick, and reserves the launch tables (and the
// LSCV job table) at the head of the workspace.
int batch_create(std::vector<kde_batch_item>&& items, std::vector<char>&& internal, std::vector<kde::LscvJob>&& jobs,
                 const kde_params* params, kde_batch** out) {
    // the batched column kernels transform the lag columns in the product pass
    if (params && params->store_spectrum) return KDE_ERR_ARG;
    auto* b = new (std::nothrow) kde_batch;
    if (!b) return KDE_ERR_ARG;
    const int count = static_cast<int>(items.size());
    b->items = std::move(items);
    b->internal = std::move(internal);
    b->lscv = std::move(jobs);
    if (params) {
        b->prm = *params;
        b->has_prm = true;
    }
    for (int k = 0; k < kde::kMaxD; ++k) b->tile[k] = params ? params->tile[k] : 0;
    const std::vector<TileShape> cands = tile_candidates(*b);
    std::vector<size_t> need(count, 0);
    size_t cap = 0;
    int rc = KDE_OK;
    for (const auto& c : cands) {
        for (int k = 0; k < kde::kMaxD; ++k) b->tile[k] = c[k];
        rc = layout_batch(*b);
        if (rc != KDE_OK) break;
        for (int i = 0; i < count; ++i)
            need[i] = std::max(need[i], item_layout(b->items[i], b->plans[i], b->internal[i] != 0).total);
    }
    if (rc == KDE_OK) {
        b->inst_off.assign(count, 0);
        size_t off_items = 0;
        for (int i = 0; i < count; ++i) {
            b->inst_off[i] = off_items;
            off_items += align_up(need[i]);
        }
        // the tables of every configuration the autotuner may bind: each tile shape with the
        // strided passes wide or narrow (narrow shapes take more workgroups, so larger owner maps)
        for (const auto& c : cands) {
            for (int k = 0; k < kde::kMaxD; ++k) b->tile[k] = c[k];
            rc = layout_batch(*b);
            if (rc != KDE_OK) break;
            for (const int mask : {0, kAllNarrow}) {
                b->narrow_mask = mask;
                size_t tb = 0;
                rc = build_groups(*b, nullptr, b->passes, b->groups, tb);
                if (rc != KDE_OK) break;
                cap = std::max(cap, tb);
            }
            b->narrow_mask = 0;
            if (rc != KDE_OK) break;
        }
        b->lscv_tab_off = align_up(cap);
        b->table_cap = align_up(b->lscv_tab_off + b->lscv.size() * sizeof(kde::LscvJob));
        for (int i = 0; i < count; ++i) b->inst_off[i] += b->table_cap;
        b->ws_bytes = b->table_cap + off_items;
    }
    if (rc == KDE_OK) {
        for (int k = 0; k < kde::kMaxD; ++k) b->tile[k] = cands[0][k];
        rc = layout_batch(*b);
        size_t tb = 0;
        if (rc == KDE_OK) rc = build_groups(*b, nullptr, b->passes, b->groups, tb);
    }
    if (rc != KDE_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return KDE_OK;
}

// The whole estimate of a planned problem into the workspace ws (counts,
// binning workspace, convolution workspace); `overlap` allows the kernel
// spectrum on the second stream where it does not ride in the binning launches.
int eval_planned(const Plan& pl, const double* X, int64_t n, const kde_grid* grid, const kde_params* params,
                 void* density, char* ws, uint64_t* n_dropped, bool overlap, hipStream_t stream) {
    auto* counts = reinterpret_cast<uint64_t*>(ws);
    char* bin_ws = ws + align_up(pl.counts_bytes);
    char* conv_ws = bin_ws + align_up(pl.pub.bin_ws_bytes);
    const bool reuse = params && params->reuse_spectrum;
    // with tiled binning the spectrum rides in the binning launches: its row pass
    // in the histogram's, its strided pass (3-D) in the scan's
    std::vector<Pass> spec;
    if (pl.tiled && !reuse && pl.pub.d <= 3) {
        Collect c(spec);
        KDE_CHECK(run_kspec_lags(pl, conv_ws, -1, c));
        const size_t want = pl.pub.d == 3 ? 2 : 1;
        if (spec.size() != want || spec[0].kind != kPassRowR2C || (want == 2 && spec[1].kind != kPassCols))
            spec.clear();
    }
    Tracer tr(params, stream);
    KDE_CHECK(tr.start());
    const int r = run_phases(
        stream, tr, overlap && pl.pub.d >= 3 && spec.empty() && !reuse,
        [&](hipStream_t s) {
            Direct e(s, tr);
            return reuse || !spec.empty() ? KDE_OK : run_kspec(pl, conv_ws, -1, e);
        },
        [&](hipStream_t s) {
            Direct e(s, tr);
            KDE_CHECK(run_bin(pl, X, n, grid, counts, n_dropped, bin_ws, e, spec.empty() ? nullptr : &spec[0],
                              spec.size() == 2 ? &spec[1] : nullptr));
            // a stored spectrum's slowest axis follows the passes fused into the binning
            if (!spec.empty() && pl.store) KDE_CHECK(run_kspec_store(pl, conv_ws, -1, e));
            return run_counts_fwd(pl, counts, grid, conv_ws, -1, e);
        },
        [&](hipStream_t s) {
            Direct e(s, tr);
            return run_product_inv(pl, grid, density, conv_ws, -1, e);
        });
    tr.finish();
    return r;
}

}  // namespace

extern "C" {

int kde_grid_from_data(const double* X, int64_t n, int32_t d, const double* H, double nsd, int64_t M,
                       kde_grid* out) {
    if (!X || !H || !out || n < 1 || d < 1 || d > kde::kMaxD || M < 2 || M > (int64_t(1) << 24)) return KDE_ERR_ARG;
    if (!std::isfinite(nsd) || nsd < 0.0) return KDE_ERR_ARG;
    double Hs[kde::kMaxD][kde::kMaxD] = {}, R[kde::kMaxD][kde::kMaxD] = {};
    const int rc = factor_bandwidth(H, d, Hs, R);
    if (rc != KDE_OK) return rc;
    double mn[kde::kMaxD], mx[kde::kMaxD];
    bool any = false;
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + i * d;
        bool finite = true;
        for (int k = 0; k < d; ++k) finite = finite && std::isfinite(x[k]);
        if (!finite) continue;
        for (int k = 0; k < d; ++k) {
            mn[k] = any ? std::fmin(mn[k], x[k]) : x[k];
            mx[k] = any ? std::fmax(mx[k], x[k]) : x[k];
        }
        any = true;
    }
    if (!any) return KDE_ERR_ARG;
    kde_grid g{};
    g.d = d;
    for (int k = 0; k < d; ++k) {
        const double s = std::sqrt(H[k * d + k]);
        const double w = nsd * s;   // separate statements: no contraction into a fused multiply-add
        g.lo[k] = mn[k] - w;
        g.hi[k] = mx[k] + w;
        g.M[k] = M;
        if (!std::isfinite(g.lo[k]) || !std::isfinite(g.hi[k]) || !(g.hi[k] > g.lo[k])) return KDE_ERR_ARG;
    }
    *out = g;
    return KDE_OK;
}

int kde_plan_query(const double* H, int64_t n, const kde_grid* grid, const kde_params* params, kde_plan* out) {
    if (!out) return KDE_ERR_ARG;
    Plan pl;
    const int rc = H ? make_plan(H, n, 1, true, grid, params, &pl) : make_plan(nullptr, n, 0, false, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    *out = pl.pub;
    if (H && n >= 2) {
        Plan p1, p2;
        LscvLayout L;
        if (lscv_plans(H, n, grid, params, &p1, &p2, &L) == KDE_OK) out->lscv_ws_bytes = L.total;
    }
    return KDE_OK;
}

int kde_bin(const double* X, int64_t n, const kde_grid* grid, const kde_params* params, uint64_t* counts,
            uint64_t* n_dropped, void* ws, size_t ws_bytes, hipStream_t stream) {
    Plan pl;
    const int rc = make_plan(nullptr, n, 0, false, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    if (!counts || (n > 0 && !X)) return KDE_ERR_ARG;
    if (pl.pub.bin_ws_bytes > 0) {
        if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return KDE_ERR_ARG;
        if (ws_bytes < pl.pub.bin_ws_bytes) return KDE_ERR_WS;
    }
    Tracer tr(params, stream);
    KDE_CHECK(tr.start());
    Direct emit(stream, tr);
    const int r = run_bin(pl, X, n, grid, counts, n_dropped, static_cast<char*>(ws), emit);
    tr.finish();
    return r;
}

int kde_kernel_grid(const double* H, int64_t n, const kde_grid* grid, const kde_params* params, void* lags,
                    size_t lags_bytes, hipStream_t stream) {
    Plan pl;
    const int rc = make_plan(H, n, 1, true, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    if (!lags) return KDE_ERR_ARG;
    if (lags_bytes < pl.pub.lag_bytes) return KDE_ERR_WS;
    Tracer tr(params, stream);
    KDE_CHECK(tr.start());
    KDE_CHECK(tr.pass("kfill", [&] {
        return kde::launch_kfill(pl.pub.prec, pl.pub.d, pl.pub.L, pl.A, pl.pub.norm, lags, stream) == hipSuccess
                   ? KDE_OK
                   : KDE_ERR_HIP;
    }));
    tr.finish();
    return KDE_OK;
}

int kde_conv(const uint64_t* counts, int64_t n, const double* H, const kde_grid* grid, const kde_params* params,
             void* density, void* ws, size_t ws_bytes, hipStream_t stream) {
    Plan pl;
    const int rc = make_plan(H, n, 1, true, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    if (!counts || !density || !ws) return KDE_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return KDE_ERR_ARG;
    if (ws_bytes < pl.pub.conv_ws_bytes) return KDE_ERR_WS;
    char* conv_ws = static_cast<char*>(ws);
    const bool reuse = params && params->reuse_spectrum;
    Tracer tr(params, stream);
    KDE_CHECK(tr.start());
    const int r = run_phases(
        stream, tr, pl.pub.d >= 3 && !reuse,
        [&](hipStream_t s) {
            Direct e(s, tr);
            return reuse ? KDE_OK : run_kspec(pl, conv_ws, -1, e);
        },
        [&](hipStream_t s) {
            Direct e(s, tr);
            return run_counts_fwd(pl, counts, grid, conv_ws, -1, e);
        },
        [&](hipStream_t s) {
            Direct e(s, tr);
            return run_product_inv(pl, grid, density, conv_ws, -1, e);
        });
    tr.finish();
    return r;
}

int kde_eval(const double* X, int64_t n, const double* H, const kde_grid* grid, const kde_params* params,
             void* density, void* ws, size_t ws_bytes, uint64_t* n_dropped, hipStream_t stream) {
    Plan pl;
    const int rc = make_plan(H, n, 1, true, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    if (!X || !density || !ws) return KDE_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return KDE_ERR_ARG;
    if (ws_bytes < pl.pub.eval_ws_bytes) return KDE_ERR_WS;
    return eval_planned(pl, X, n, grid, params, density, static_cast<char*>(ws), n_dropped, true, stream);
}

int kde_eval_noalloc(const double* X, int64_t n, const double* H, const kde_grid* grid, const kde_params* params,
                     void* density, uint64_t* n_dropped, hipStream_t stream) {
    Plan pl;
    const int rc = make_plan(H, n, 1, true, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    if (!X || !density) return KDE_ERR_ARG;
    // the scratch array keeps the previous call's contents, which need not be this problem's spectrum
    if (params && params->reuse_spectrum) return KDE_ERR_ARG;
    if (pl.pub.eval_ws_bytes > kde::kScratchBytes) return KDE_ERR_WS;
    int dev = 0;
    if (hipStreamGetDevice(stream, &dev) != hipSuccess) return KDE_ERR_HIP;
    void* ws = nullptr;
    if (kde::scratch_address(dev, &ws) != hipSuccess || !ws) return KDE_ERR_HIP;
    // everything on the caller's stream (no second stream, which its first use would create)
    return eval_planned(pl, X, n, grid, params, density, static_cast<char*>(ws), n_dropped, false, stream);
}

int kde_lscv(const uint64_t* counts, int64_t n, const double* H, const kde_grid* grid, const kde_params* params,
             double* out, void* ws, size_t ws_bytes, hipStream_t stream) {
    Plan p1, p2;
    LscvLayout L;
    const int rc = lscv_plans(H, n, grid, params, &p1, &p2, &L);
    if (rc != KDE_OK) return rc;
    if (!counts || !out || !ws || reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return KDE_ERR_ARG;
    if (ws_bytes < L.total) return KDE_ERR_WS;
    char* base = static_cast<char*>(ws);
    void* density = base + L.density;
    auto* dots = reinterpret_cast<double*>(base + L.dots);
    auto* partial = reinterpret_cast<double*>(base + L.partial);
    char* conv_ws = base + L.conv;
    int64_t cells = 1;
    for (int k = 0; k < p1.pub.d; ++k) cells *= grid->M[k];
    Tracer tr(params, stream);
    KDE_CHECK(tr.start());
    // first term with 2H, then the second with H; each convolution is followed
    // by its dot product on the caller's stream
    const Plan* plans[2] = {&p2, &p1};
    for (int t = 0; t < 2; ++t) {
        const Plan& pl = *plans[t];
        KDE_CHECK(run_phases(
            stream, tr, pl.pub.d >= 3,
            [&](hipStream_t s) {
                Direct e(s, tr);
                return run_kspec(pl, conv_ws, -1, e);
            },
            [&](hipStream_t s) {
                Direct e(s, tr);
                return run_counts_fwd(pl, counts, grid, conv_ws, -1, e);
            },
            [&](hipStream_t s) {
                Direct e(s, tr);
                return run_product_inv(pl, grid, density, conv_ws, -1, e);
            }));
        kde::DotArgs a{};
        a.counts = counts;
        a.f = density;
        a.cells = cells;
        a.scale = std::ldexp(1.0, -p1.pub.d * p1.pub.Q);
        a.partial = partial;
        a.nb = kde::dot_blocks(cells);
        a.out = dots + t;
        KDE_CHECK(tr.pass("dot", [&] {
            return kde::launch_dot(pl.pub.prec, a, stream) == hipSuccess ? KDE_OK : KDE_ERR_HIP;
        }));
    }
    // phi_H(0) = (2 pi)^-d/2 |H|^-1/2 = n k_0
    const double phi0 = p1.pub.norm * static_cast<double>(n);
    KDE_CHECK(tr.pass("lscv_combine", [&] {
        return kde::launch_lscv_combine(dots, static_cast<double>(n), phi0, out, stream) == hipSuccess
                   ? KDE_OK
                   : KDE_ERR_HIP;
    }));
    tr.finish();
    return KDE_OK;
}

}  // extern "C"

namespace {

// Device layouts of the network state and workspace.
struct MlpState {
    size_t P = 0, m = 0, v = 0, Wk = 0, Wt = 0, total = 0;
};
MlpState mlp_state() {
    MlpState L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.P = take(kde::kMlpParams * sizeof(float));
    L.m = take(kde::kMlpParams * sizeof(float));
    L.v = take(kde::kMlpParams * sizeof(float));
    L.Wk = take(kde::kMlpWeights * sizeof(uint16_t));
    L.Wt = take(kde::kMlpWeights * sizeof(uint16_t));
    L.total = off;
    return L;
}
struct MlpWs {
    size_t acts = 0, Y = 0, partial = 0, lossp = 0, grad = 0, loss = 0, total = 0;
};
MlpWs mlp_ws(int64_t B) {
    MlpWs L;
    const int64_t groups = (B + kde::kMlpRows - 1) / kde::kMlpRows;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.acts = take(static_cast<size_t>(B) * (kde::kMlpInPad + 3 * kde::kMlpHid) * sizeof(uint16_t));
    L.Y = take(static_cast<size_t>(B) * kde::kMlpOut * sizeof(float));
    L.partial = take(static_cast<size_t>(groups) * kde::kMlpParams * sizeof(float));
    L.lossp = take(static_cast<size_t>(groups) * sizeof(float));
    L.grad = take(kde::kMlpParams * sizeof(float));
    L.loss = take(sizeof(float));
    L.total = off;
    return L;
}
kde::MlpArgs mlp_args(const void* state, int64_t B, char* ws) {
    const MlpState S = mlp_state();
    char* st = static_cast<char*>(const_cast<void*>(state));
    kde::MlpArgs a{};
    a.P = reinterpret_cast<const float*>(st + S.P);
    a.Pw = reinterpret_cast<float*>(st + S.P);
    a.m = reinterpret_cast<float*>(st + S.m);
    a.v = reinterpret_cast<float*>(st + S.v);
    a.Wk = reinterpret_cast<const uint16_t*>(st + S.Wk);
    a.Wt = reinterpret_cast<const uint16_t*>(st + S.Wt);
    a.Wkw = reinterpret_cast<uint16_t*>(st + S.Wk);
    a.Wtw = reinterpret_cast<uint16_t*>(st + S.Wt);
    a.B = B;
    a.groups = (B + kde::kMlpRows - 1) / kde::kMlpRows;
    if (ws) {
        const MlpWs W = mlp_ws(B);
        a.acts = reinterpret_cast<uint16_t*>(ws + W.acts);
        a.partial = reinterpret_cast<float*>(ws + W.partial);
        a.loss_partial = reinterpret_cast<float*>(ws + W.lossp);
        a.grad = reinterpret_cast<float*>(ws + W.grad);
        a.loss = reinterpret_cast<float*>(ws + W.loss);
        a.Y = reinterpret_cast<float*>(ws + W.Y);
    }
    return a;
}
bool aligned(const void* p) { return reinterpret_cast<uintptr_t>(p) % kAlign == 0; }

// forward with saved layer inputs, then the per-group and summed gradients
int mlp_grad_pass(kde::MlpArgs& a, hipStream_t s) {
    KDE_TRY(kde::launch_mlp(kde::kMlpOpForward, a, nullptr, s));
    KDE_TRY(kde::launch_mlp(kde::kMlpOpBackward, a, nullptr, s));
    KDE_TRY(kde::launch_mlp(kde::kMlpOpReduce, a, nullptr, s));
    return KDE_OK;
}

}  // namespace

extern "C" {

int kde_mlp_query(int64_t batch, kde_mlp_info* info) {
    if (!info || batch < 0) return KDE_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_in = kde::kMlpIn;
    info->n_hidden = kde::kMlpHid;
    info->n_out = kde::kMlpOut;
    info->rows_per_group = kde::kMlpRows;
    info->n_params = kde::kMlpParams;
    info->state_bytes = mlp_state().total;
    info->ws_bytes = batch > 0 ? mlp_ws(batch).total : 0;
    return KDE_OK;
}

int kde_mlp_load(void* state, const float* params, hipStream_t stream) {
    if (!state || !params || !aligned(state)) return KDE_ERR_ARG;
    kde::MlpArgs a = mlp_args(state, 0, nullptr);
    KDE_TRY(kde::launch_mlp(kde::kMlpOpLoad, a, params, stream));
    return KDE_OK;
}

int kde_mlp_forward(const void* state, const float* X, int64_t B, float* Y, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
    if (!state || !X || !Y || B < 1 || !aligned(state)) return KDE_ERR_ARG;
    (void)ws;
    (void)ws_bytes;
    kde::MlpArgs a = mlp_args(state, B, nullptr);
    a.X = X;
    a.Y = Y;
    KDE_TRY(kde::launch_mlp(kde::kMlpOpForward, a, nullptr, stream));
    return KDE_OK;
}

int kde_mlp_grad(const void* state, const float* X, const float* T, int64_t B, float* Y, float* grad, float* loss,
                 void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!state || !X || !T || !grad || B < 1 || !ws || !aligned(state) || !aligned(ws)) return KDE_ERR_ARG;
    if (ws_bytes < mlp_ws(B).total) return KDE_ERR_WS;
    kde::MlpArgs a = mlp_args(state, B, static_cast<char*>(ws));
    a.X = X;
    a.T = T;
    if (Y) a.Y = Y;
    a.grad = grad;
    a.loss = loss;
    return mlp_grad_pass(a, stream);
}

int kde_mlp_train_step(void* state, const float* X, const float* T, int64_t B, float lr, int32_t step, float* loss,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!state || !X || !T || B < 1 || step < 1 || !ws || !aligned(state) || !aligned(ws)) return KDE_ERR_ARG;
    if (!(lr > 0.f) || !std::isfinite(lr)) return KDE_ERR_ARG;
    if (ws_bytes < mlp_ws(B).total) return KDE_ERR_WS;
    kde::MlpArgs a = mlp_args(state, B, static_cast<char*>(ws));
    a.X = X;
    a.T = T;
    if (loss) a.loss = loss;
    KDE_CHECK(mlp_grad_pass(a, stream));
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.eps = 1e-8f;
    a.c1 = static_cast<float>(1.0 - std::pow(0.9, step));
    a.c2 = static_cast<float>(1.0 - std::pow(0.999, step));
    KDE_TRY(kde::launch_mlp(kde::kMlpOpAdam, a, nullptr, stream));
    return KDE_OK;
}

int kde_batch_create(const kde_batch_item* items, int32_t count, const kde_params* params, kde_batch** out) {
    if (!out) return KDE_ERR_ARG;
    *out = nullptr;
    if (!items || count < 1) return KDE_ERR_ARG;
    for (int32_t i = 0; i < count; ++i)
        if ((!items[i].X && !items[i].counts) || !items[i].density) return KDE_ERR_ARG;
    return batch_create(std::vector<kde_batch_item>(items, items + count), std::vector<char>(count, 0), {}, params,
                        out);
}

int kde_lscv_batch_create(const kde_lscv_item* items, int32_t count, const kde_params* params, kde_batch** out) {
    if (!out) return KDE_ERR_ARG;
    *out = nullptr;
    if (!items || count < 1) return KDE_ERR_ARG;
    std::vector<kde_batch_item> inner;
    std::vector<kde::LscvJob> jobs;
    inner.reserve(2 * static_cast<size_t>(count));
    jobs.reserve(count);
    for (int32_t k = 0; k < count; ++k) {
        const kde_lscv_item& it = items[k];
        if (!it.counts || !it.out) return KDE_ERR_ARG;
        Plan p1, p2;
        LscvLayout L;
        const int rc = lscv_plans(it.H, it.n, &it.grid, params, &p1, &p2, &L);
        if (rc != KDE_OK) return rc;
        // first term with 2H, second with H, as kde_lscv computes them
        kde_batch_item a{};
        a.n = it.n;
        a.grid = it.grid;
        a.counts = it.counts;
        const int d = it.grid.d;
        for (int i = 0; i < d * d; ++i) a.H[i] = 2.0 * it.H[i];
        inner.push_back(a);
        for (int i = 0; i < d * d; ++i) a.H[i] = it.H[i];
        inner.push_back(a);
        kde::LscvJob j{};
        j.n = static_cast<double>(it.n);
        j.phi0 = p1.pub.norm * static_cast<double>(it.n);   // phi_H(0) = n k_0
        j.out = it.out;
        jobs.push_back(j);
    }
    return batch_create(std::move(inner), std::vector<char>(inner.size(), 1), std::move(jobs), params, out);
}

int kde_batch_query(const kde_batch* b, kde_batch_info* info) {
    if (!b || !info) return KDE_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->count = static_cast<int32_t>(b->items.size());
    info->ws_bytes = b->ws_bytes;
    for (int k = 0; k < kde::kMaxD; ++k) info->tile[k] = b->tile[k];
    info->narrow_mask = b->narrow_mask;
    int launches = 0;
    for (const Group& g : b->groups) launches += g.batched ? 1 : static_cast<int>(g.members.size());
    info->launches = launches;
    return KDE_OK;
}

int kde_batch_bind(kde_batch* b, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!b || !ws || reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return KDE_ERR_ARG;
    if (ws_bytes < b->ws_bytes) return KDE_ERR_WS;
    b->ws = static_cast<char*>(ws);
    b->bound = false;
    return rebind(*b, stream);
}

int kde_batch_eval(const kde_batch* b, hipStream_t stream) {
    if (!b || !b->bound) return KDE_ERR_ARG;
    const kde_params* prm = b->has_prm ? &b->prm : nullptr;
    Tracer tr(prm, stream);
    KDE_CHECK(tr.start());
    int r = run_phases(
        stream, tr, true, [&](hipStream_t s) { return run_batch_phase(*b, 0, s, tr); },
        [&](hipStream_t s) { return run_batch_phase(*b, 1, s, tr); },
        [&](hipStream_t s) { return run_batch_phase(*b, 2, s, tr); });
    if (r == KDE_OK && !b->lscv.empty()) {
        const auto* jobs = reinterpret_cast<const kde::LscvJob*>(b->ws + b->lscv_tab_off);
        r = tr.pass("lscv_combine", [&] {
            return kde::launch_lscv_combine_batch(jobs, static_cast<int>(b->lscv.size()), stream) == hipSuccess
                       ? KDE_OK
                       : KDE_ERR_HIP;
        });
    }
    tr.finish();
    return r;
}

int kde_batch_tune(kde_batch* b, int32_t reps, hipStream_t stream) {
    if (!b || !b->bound || reps < 1) return KDE_ERR_ARG;
    if (b->has_prm && b->prm.trace_events) return KDE_ERR_ARG;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KDE_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return KDE_ERR_HIP;
    }
    auto time_config = [&](float* ms) -> int {
        KDE_CHECK(rebind(*b, stream));
        KDE_CHECK(kde_batch_eval(b, stream));   // warm-up
        KDE_TRY(hipEventRecord(e0, stream));
        for (int r = 0; r < reps; ++r) KDE_CHECK(kde_batch_eval(b, stream));
        KDE_TRY(hipEventRecord(e1, stream));
        KDE_TRY(hipEventSynchronize(e1));
        KDE_TRY(hipEventElapsedTime(ms, e0, e1));
        return KDE_OK;
    };
    int rc = KDE_OK;
    int best_tile[kde::kMaxD];
    std::memcpy(best_tile, b->tile, sizeof(best_tile));
    float best = 0.f;
    do {
        rc = time_config(&best);
        if (rc != KDE_OK) break;
        // binning tile shape
        const std::vector<TileShape> cands = tile_candidates(*b);
        for (size_t j = 1; j < cands.size(); ++j) {
            for (int k = 0; k < kde::kMaxD; ++k) b->tile[k] = cands[j][k];
            rc = layout_batch(*b);
            float ms = 0.f;
            if (rc == KDE_OK) rc = time_config(&ms);
            if (rc != KDE_OK) break;
            if (ms < best) {
                best = ms;
                for (int k = 0; k < kde::kMaxD; ++k) best_tile[k] = cands[j][k];
            }
        }
        if (rc != KDE_OK) break;
        for (int k = 0; k < kde::kMaxD; ++k) b->tile[k] = best_tile[k];
        rc = layout_batch(*b);
        if (rc != KDE_OK) break;
        // strided-pass shape, one padded length at a time
        int lens = 0;
        for (const auto& pl : b->plans)
            for (int k = 0; k + 1 < pl.pub.d; ++k) lens |= pl.pub.P[k];
        for (int lg = 4; lg <= 12; ++lg) {
            if (!(lens & (1 << lg))) continue;
            b->narrow_mask ^= 1 << lg;
            float ms = 0.f;
            rc = time_config(&ms);
            if (rc != KDE_OK) break;
            if (ms < best) best = ms;
            else b->narrow_mask ^= 1 << lg;
        }
        if (rc != KDE_OK) break;
        rc = rebind(*b, stream);
        if (rc == KDE_OK && hipStreamSynchronize(stream) != hipSuccess) rc = KDE_ERR_HIP;
    } while (false);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

void kde_batch_destroy(kde_batch* b) { delete b; }

const char* kde_strerror(int status) {
    switch (status) {
        case KDE_OK: return "ok";
        case KDE_ERR_ARG: return "invalid argument";
        case KDE_ERR_NOT_SPD: return "bandwidth matrix is not finite, symmetric and positive definite";
        case KDE_ERR_OVERFLOW: return "n * 2^(d Q) does not fit in uint64";
        case KDE_ERR_WS: return "workspace or output buffer too small";
        case KDE_ERR_SIZE: return "padded FFT length exceeds 4096 on some axis";
        case KDE_ERR_HIP: return "HIP launch or event call failed";
        default: return "unknown status";
    }
}

}  // extern "C"
