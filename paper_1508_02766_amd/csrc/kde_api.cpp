// C ABI of the binned FFT KDE (declared in include/kde.h): host planner in
// FP64 and the orchestration of the gfx950 kernels.
//
// Planner (Gramacki & Gramacki, arXiv 1508.02766):
//   delta_k = (hi_k - lo_k) / (M_k - 1)                       Eq. (4)
//   H = R R' (Cholesky), |H| = prod R_kk^2, H^-1 = R^-T R^-1  (K_H of Eq. 1)
//   lambda_max(H): closed form for d <= 2, cyclic Jacobi for d = 3
//   L_k = min(M_k - 1, ceil(tau sqrt(lambda_max) / delta_k))  Eq. (15)
//   P_k = smallest power of two >= max(16, M_k + L_k)          zero padding, Section 4.1
//   k_0 = n^-1 (2 pi)^-d/2 |H|^-1/2                            Eq. (6) with Eq. (1)
//
// The lag box is placed circularly (lag l at l mod P_k, the true negative
// lags of Eq. 12 rather than Wand's mirror of Eq. 8) and the counts at the
// origin; P_k >= M_k + L_k makes the circular convolution equal to Eq. (7) on
// the window [0, M_k), which replaces the extraction of Eq. (14).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/kde.h"
#include "kde_internal.h"

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
    size_t khat = 0, kt1 = 0, kt2 = 0, z1 = 0, z2 = 0, total = 0;
};

struct BinLayout {
    // offsets into the binning workspace (tiled path)
    size_t hist = 0, tot = 0, drops = 0, tile_start = 0, records = 0, partial = 0, total = 0;
};

struct Plan {
    kde_plan pub;
    double A[9];      // A_ab = delta_a delta_b (H^-1)_ab
    double tau;
    Layout lay;
    size_t counts_bytes;
    bool tiled;       // tiled binning (else global atomics)
    kde::TileGeom tg;
    BinLayout blay;
};

// Tile geometry of the binning pass: 32 x 32 cells in 2-D, 8 x 8 x 8 in 3-D,
// 1024 in 1-D (clamped to the grid), widened until the tile count fits the
// per-workgroup histogram. Returns false when the tiled path cannot be used:
// too many cells per tile, records wider than 64 bits, or n 2^d >= 2^32.
bool plan_tiles(int d, const int64_t* M, int Q, int64_t n, kde::TileGeom* tg, BinLayout* bl) {
    kde::TileGeom g{};
    static const int base[3][3] = {{1024, 0, 0}, {32, 32, 0}, {8, 16, 16}};
    for (int k = 0; k < d; ++k) {
        int T = base[d - 1][k];
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
    bl->tile_start = take(static_cast<size_t>(g.ntiles) * 4);
    bl->records = take(static_cast<size_t>(g.max_records) * 8);
    bl->partial = take(static_cast<size_t>(g.max_segments) * g.tile_cells * 8);
    bl->total = off;
    *tg = g;
    return true;
}

// Validation and derived quantities. need_H: validate and factor H;
// n_min: the smallest admissible sample count (1 where Eq. 1 divides by n).
int make_plan(const double* H, int64_t n, int64_t n_min, bool need_H, const kde_grid* g,
              const kde_params* prm, Plan* out) {
    if (!g || !out) return KDE_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    kde_plan& p = out->pub;
    const int d = g->d;
    if (d < 1 || d > 3) return KDE_ERR_ARG;
    if (n < n_min) return KDE_ERR_ARG;
    p.d = d;
    for (int k = 0; k < d; ++k) {
        if (g->M[k] < 2 || g->M[k] > (int64_t(1) << 24)) return KDE_ERR_ARG;
        if (!std::isfinite(g->lo[k]) || !std::isfinite(g->hi[k]) || !(g->hi[k] > g->lo[k])) return KDE_ERR_ARG;
        p.delta[k] = (g->hi[k] - g->lo[k]) / static_cast<double>(g->M[k] - 1);
        if (!std::isfinite(p.delta[k]) || !(p.delta[k] > 0.0)) return KDE_ERR_ARG;
    }
    // options
    double tau = kTauDefault;
    int prec = KDE_F32, Q = 32 / d;
    int Lovr[3] = {0, 0, 0};
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
    out->tiled = plan_tiles(d, g->M, Q, n, &out->tg, &out->blay);
    p.bin_ws_bytes = out->tiled ? out->blay.total : 0;
    if (!need_H) return KDE_OK;

    // H: finite, symmetric, positive definite
    if (!H) return KDE_ERR_ARG;
    double Hs[3][3] = {};
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
    double R[3][3] = {};
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
    double det = 1.0;
    for (int k = 0; k < d; ++k) det *= R[k][k] * R[k][k];
    // inverse of the lower-triangular factor, then H^-1 = R^-T R^-1
    double Ri[3][3] = {};
    for (int j = 0; j < d; ++j) {
        Ri[j][j] = 1.0 / R[j][j];
        for (int i = j + 1; i < d; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += R[i][k] * Ri[k][j];
            Ri[i][j] = -s / R[i][i];
        }
    }
    double Hinv[3][3] = {};
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
        double a[3][3];
        std::memcpy(a, Hs, sizeof(a));
        for (int sweep = 0; sweep < 60; ++sweep) {
            const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
            const double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
            if (off <= 1e-36 * diag) break;
            static const int pq[3][2] = {{0, 1}, {0, 2}, {1, 2}};
            for (const auto& e : pq) {
                const int P = e[0], Qi = e[1];
                const double apq = a[P][Qi];
                if (apq == 0.0) continue;
                const double theta = (a[Qi][Qi] - a[P][P]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                a[P][P] -= t * apq;
                a[Qi][Qi] += t * apq;
                a[P][Qi] = a[Qi][P] = 0.0;
                for (int r = 0; r < 3; ++r) {
                    if (r == P || r == Qi) continue;
                    const double arp = a[r][P], arq = a[r][Qi];
                    a[r][P] = a[P][r] = c * arp - s * arq;
                    a[r][Qi] = a[Qi][r] = s * arp + c * arq;
                }
            }
        }
        lam = std::fmax(a[0][0], std::fmax(a[1][1], a[2][2]));
    }
    p.lambda_max = lam;
    p.det_H = det;
    p.norm = 1.0 / (static_cast<double>(n) * std::pow(kTwoPi, 0.5 * d) * std::sqrt(det));
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) out->A[a * 3 + b] = p.delta[a] * p.delta[b] * Hinv[a][b];

    // truncation (Eq. 15) and padded lengths
    int64_t lag_count = 1;
    for (int k = 0; k < d; ++k) {
        int L = Lovr[k];
        if (L == 0) {
            const double x = std::ceil(tau * std::sqrt(std::fabs(lam)) / p.delta[k]);
            const double cap = static_cast<double>(g->M[k] - 1);
            L = static_cast<int>(x < cap ? x : cap);
        }
        p.L[k] = L;
        int64_t P = kde::kMinP;
        while (P < g->M[k] + L) P *= 2;
        if (P > kde::kMaxP) return KDE_ERR_SIZE;
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
    } else {
        L.kt1 = take(static_cast<size_t>(n0 * n1 * Hl) * cs);
        L.kt2 = take(static_cast<size_t>(n0 * P1 * Hl) * cs);
        L.z1 = take(static_cast<size_t>(M0 * M1 * Hl) * cs);
        L.z2 = take(static_cast<size_t>(M0 * P1 * Hl) * cs);
    }
    L.total = off;
    p.conv_ws_bytes = L.total;
    p.eval_ws_bytes = align_up(out->counts_bytes) + align_up(p.bin_ws_bytes) + L.total;
    return KDE_OK;
}

// Optional per-kernel event trace (kde_params.trace_*).
struct Tracer {
    const kde_params* prm;
    hipStream_t s;
    int n = 0;
    bool on = false;
    Tracer(const kde_params* p, hipStream_t st) : prm(p), s(st) {
        on = prm && prm->trace_events && prm->trace_capacity > 0;
    }
    hipError_t start() {
        if (!on) return hipSuccess;
        n = 1;
        return hipEventRecord(prm->trace_events[0], s);
    }
    hipError_t mark(const char* name) {
        if (!on || n >= prm->trace_capacity) return hipSuccess;
        if (prm->trace_names) prm->trace_names[n - 1] = name;
        return hipEventRecord(prm->trace_events[n++], s);
    }
    void finish() {
        if (prm && prm->trace_count) *prm->trace_count = on ? n : 0;
    }
};

#define KDE_TRY(expr)                                 \
    do {                                              \
        if ((expr) != hipSuccess) return KDE_ERR_HIP; \
    } while (0)

#define KDE_LAUNCH(expr, name)              \
    do {                                    \
        KDE_TRY(expr);                      \
        KDE_TRY(tr.mark(name));             \
    } while (0)

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
    a.w.tile_start = reinterpret_cast<uint32_t*>(ws + b.tile_start);
    a.w.records = reinterpret_cast<uint64_t*>(ws + b.records);
    a.w.partial = reinterpret_cast<uint64_t*>(ws + b.partial);
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

int run_bin(const Plan& pl, const double* X, int64_t n, const kde_grid* g, uint64_t* counts, uint64_t* n_dropped,
            char* ws, hipStream_t s, Tracer& tr) {
    const kde::BinConsts c = bin_consts(pl, g);
    int64_t cells = 1;
    for (int k = 0; k < pl.pub.d; ++k) cells *= g->M[k];
    if (pl.tiled && n > 0) {
        const kde::BinArgs a = bin_args(pl, c, X, n, counts, n_dropped, ws);
        KDE_LAUNCH(kde::launch_bin_stage(kde::kBinHist, a, s), "bin_hist");
        KDE_LAUNCH(kde::launch_bin_stage(kde::kBinScan, a, s), "bin_scan");
        KDE_LAUNCH(kde::launch_bin_stage(kde::kBinScatter, a, s), "bin_scatter");
        KDE_LAUNCH(kde::launch_bin_stage(kde::kBinAccum, a, s), "bin_accum");
        KDE_LAUNCH(kde::launch_bin_stage(kde::kBinReduce, a, s), "bin_reduce");
        return KDE_OK;
    }
    KDE_LAUNCH(kde::launch_zero_u64(counts, cells, s), "zero_counts");
    if (n_dropped) KDE_LAUNCH(kde::launch_zero_u64(n_dropped, 1, s), "zero_dropped");
    if (n > 0) KDE_LAUNCH(kde::launch_bin(c, X, n, counts, n_dropped, s), "bin");
    return KDE_OK;
}

// Stage views of the convolution workspace.
struct ConvBufs {
    void *khat, *kt1, *kt2, *z1, *z2;
};

ConvBufs conv_bufs(const Plan& pl, char* ws) {
    const Layout& L = pl.lay;
    return {ws + L.khat, ws + L.kt1, ws + L.kt2, ws + L.z1, ws + L.z2};
}

// Kernel spectrum: lag-box weights computed in place (Eq. 6 over the signed
// box of Eq. 12), transformed along every axis; real because the box is
// centrally symmetric and placed circularly.
int run_kspec(const Plan& pl, const kde_grid* g, char* ws, hipStream_t s, Tracer& tr) {
    const kde_plan& p = pl.pub;
    const int d = p.d, prec = p.prec;
    const ConvBufs b = conv_bufs(pl, ws);
    kde::GaussLag gl{};
    for (int i = 0; i < 9; ++i) gl.A[i] = pl.A[i];
    gl.norm = p.norm;
    gl.d = d;
    for (int k = 0; k < 3; ++k) gl.L[k] = k < d ? p.L[k] : 0;
    (void)g;
    if (d == 1) {
        const int P0 = p.P[0];
        KDE_LAUNCH(kde::launch_rows_r2c(prec, P0, kde::kRowGaussCirc, nullptr, &gl, 1, 0, p.L[0], b.khat, P0 / 2 + 1,
                                        true, s), "kspec_r2c");
        return KDE_OK;
    }
    if (d == 2) {
        const int P1 = p.P[1];
        const int64_t n0 = 2 * p.L[0] + 1;
        KDE_LAUNCH(kde::launch_rows_r2c(prec, P1, kde::kRowGaussCirc, nullptr, &gl, n0, 0, p.L[1], b.kt1, half_pitch(P1), false,
                                        s), "kspec_r2c");
        return KDE_OK;
    }
    const int P1 = p.P[1], P2 = p.P[2];
    const int64_t H2 = P2 / 2 + 1, Hp = half_pitch(P2), n0 = 2 * p.L[0] + 1, n1 = 2 * p.L[1] + 1;
    KDE_LAUNCH(kde::launch_rows_r2c(prec, P2, kde::kRowGaussCirc, nullptr, &gl, n0 * n1, 0, p.L[2], b.kt1, Hp, false,
                                    s), "kspec_r2c");
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
    KDE_LAUNCH(kde::launch_cols(prec, P1, kde::kColFwdCirc, k1, s), "kspec_col2");
    return KDE_OK;
}

// Forward transforms of the zero-padded counts that do not need the spectrum.
int run_counts_fwd(const Plan& pl, const uint64_t* counts, const kde_grid* g, char* ws, hipStream_t s, Tracer& tr) {
    const kde_plan& p = pl.pub;
    const int d = p.d, prec = p.prec;
    const ConvBufs b = conv_bufs(pl, ws);
    const int Pl = p.P[d - 1];
    const int64_t Hl = Pl / 2 + 1, Hp = d == 1 ? Hl : half_pitch(Pl);
    const int64_t Ml = g->M[d - 1];
    int64_t rows = 1;
    for (int k = 0; k < d - 1; ++k) rows *= g->M[k];
    KDE_LAUNCH(kde::launch_rows_r2c(prec, Pl, kde::kRowCountsU64, counts, nullptr, rows, Ml, static_cast<int>(Ml), b.z1,
                                    Hp, false, s), "counts_r2c");
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
        KDE_LAUNCH(kde::launch_cols(prec, P1, kde::kColFwdPrefix, f1, s), "counts_col2");
    }
    return KDE_OK;
}

// Product with the spectrum, inverse transforms, window [0, M_k) and the
// 2^-(dQ) / prod P_k scale.
int run_product_inv(const Plan& pl, const kde_grid* g, void* density, char* ws, hipStream_t s, Tracer& tr) {
    const kde_plan& p = pl.pub;
    const int d = p.d, prec = p.prec;
    const ConvBufs b = conv_bufs(pl, ws);
    double scale = std::ldexp(1.0, -d * p.Q);
    for (int k = 0; k < d; ++k) scale /= static_cast<double>(p.P[k]);
    if (d == 1) {
        const int P0 = p.P[0];
        const int64_t H0 = P0 / 2 + 1, M0 = g->M[0];
        KDE_LAUNCH(kde::launch_rows_c2r(prec, P0, b.z1, 1, H0, b.khat, density, M0, static_cast<int>(M0), scale, s),
                   "product_c2r");
        return KDE_OK;
    }
    if (d == 2) {
        const int P0 = p.P[0], P1 = p.P[1];
        const int64_t H1 = P1 / 2 + 1, Hp = half_pitch(P1), M0 = g->M[0], M1 = g->M[1];
        kde::ColArgs ca{};
        ca.in = b.z1;
        ca.out = b.z1;
        ca.kt = b.kt1;
        ca.kt_ps = Hp;
        ca.kt_len = p.L[0];
        ca.W = H1;
        ca.outer = 1;
        ca.in_ps = Hp;
        ca.out_ps = Hp;
        ca.len = static_cast<int>(M0);
        ca.mout = static_cast<int>(M0);
        KDE_LAUNCH(kde::launch_cols(prec, P0, kde::kColConvLag, ca, s), "conv_col");
        KDE_LAUNCH(kde::launch_rows_c2r(prec, P1, b.z1, M0, Hp, nullptr, density, M1, static_cast<int>(M1), scale, s),
                   "c2r");
        return KDE_OK;
    }
    const int P0 = p.P[0], P1 = p.P[1], P2 = p.P[2];
    const int64_t H2 = P2 / 2 + 1, Hp = half_pitch(P2), M0 = g->M[0], M1 = g->M[1], M2 = g->M[2];
    kde::ColArgs cv{};
    cv.in = b.z2;
    cv.out = b.z2;
    cv.kt = b.kt2;
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
    KDE_LAUNCH(kde::launch_cols(prec, P0, kde::kColConvLag, cv, s), "conv_col1");
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
    KDE_LAUNCH(kde::launch_cols(prec, P1, kde::kColInvPrefix, i1, s), "inv_col2");
    KDE_LAUNCH(kde::launch_rows_c2r(prec, P2, b.z1, M0 * M1, Hp, nullptr, density, M2, static_cast<int>(M2), scale, s),
               "c2r");
    return KDE_OK;
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

// The convolution of counts (already on / being computed on stream s), with
// the spectrum on the auxiliary stream unless per-kernel tracing asks for one
// serial stream. `pre` enqueues the work that produces the counts (binning)
// or nothing.
template <typename Pre>
int run_pipeline(const Plan& pl, const kde_grid* g, const uint64_t* counts, void* density, char* conv_ws, hipStream_t s,
                 Tracer& tr, Pre&& pre) {
    if (!tr.on) {
        std::lock_guard<std::mutex> lock(g_aux_mu);
        Aux* a = aux_for(s);
        if (a) {
            KDE_TRY(hipEventRecord(a->fork, s));
            KDE_TRY(hipStreamWaitEvent(a->stream, a->fork, 0));
            int r = run_kspec(pl, g, conv_ws, a->stream, tr);
            if (r != KDE_OK) return r;
            KDE_TRY(hipEventRecord(a->join, a->stream));
            r = pre();
            if (r == KDE_OK) r = run_counts_fwd(pl, counts, g, conv_ws, s, tr);
            if (r != KDE_OK) return r;
            KDE_TRY(hipStreamWaitEvent(s, a->join, 0));
            return run_product_inv(pl, g, density, conv_ws, s, tr);
        }
    }
    int r = pre();
    if (r == KDE_OK) r = run_kspec(pl, g, conv_ws, s, tr);
    if (r == KDE_OK) r = run_counts_fwd(pl, counts, g, conv_ws, s, tr);
    if (r == KDE_OK) r = run_product_inv(pl, g, density, conv_ws, s, tr);
    return r;
}

}  // namespace

extern "C" {

int kde_plan_query(const double* H, int64_t n, const kde_grid* grid, const kde_params* params, kde_plan* out) {
    if (!out) return KDE_ERR_ARG;
    Plan pl;
    const int rc = H ? make_plan(H, n, 1, true, grid, params, &pl) : make_plan(nullptr, n, 0, false, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    *out = pl.pub;
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
    KDE_TRY(tr.start());
    const int r = run_bin(pl, X, n, grid, counts, n_dropped, static_cast<char*>(ws), stream, tr);
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
    KDE_TRY(tr.start());
    KDE_LAUNCH(kde::launch_kfill(pl.pub.prec, pl.pub.d, pl.pub.L, pl.A, pl.pub.norm, lags, stream), "kfill");
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
    Tracer tr(params, stream);
    KDE_TRY(tr.start());
    const int r = run_pipeline(pl, grid, counts, density, static_cast<char*>(ws), stream, tr, [] { return KDE_OK; });
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
    auto* counts = static_cast<uint64_t*>(ws);
    char* bin_ws = static_cast<char*>(ws) + align_up(pl.counts_bytes);
    char* conv_ws = bin_ws + align_up(pl.pub.bin_ws_bytes);
    Tracer tr(params, stream);
    KDE_TRY(tr.start());
    const int r = run_pipeline(pl, grid, counts, density, conv_ws, stream, tr,
                               [&] { return run_bin(pl, X, n, grid, counts, n_dropped, bin_ws, stream, tr); });
    tr.finish();
    return r;
}

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
