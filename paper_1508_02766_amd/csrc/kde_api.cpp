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

#include "../../include/kde.h"
#include "kde_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kTauDefault = 3.7;   // Section 4.2, after Eq. (15)
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    // offsets into the convolution workspace
    size_t lags = 0, khat = 0, kt1 = 0, kt2 = 0, z1 = 0, z2 = 0, total = 0;
};

struct Plan {
    kde_plan pub;
    double A[9];      // A_ab = delta_a delta_b (H^-1)_ab
    double tau;
    Layout lay;
    size_t counts_bytes;
};

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
    const int64_t P0 = p.P[0], P1 = d > 1 ? p.P[1] : 1;
    const int64_t Hl = p.P[d - 1] / 2 + 1;   // bins kept along the last axis
    const int64_t n0 = 2 * p.L[0] + 1, n1 = d > 1 ? 2 * p.L[1] + 1 : 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.lags = take(p.lag_bytes);
    if (d == 1) {
        L.khat = take(static_cast<size_t>(Hl) * rs);
        L.z1 = take(static_cast<size_t>(Hl) * cs);
    } else if (d == 2) {
        L.khat = take(static_cast<size_t>(P0 * Hl) * rs);
        L.kt1 = take(static_cast<size_t>(n0 * Hl) * cs);
        L.z1 = take(static_cast<size_t>(M0 * Hl) * cs);
    } else {
        L.khat = take(static_cast<size_t>(P0 * P1 * Hl) * rs);
        L.kt1 = take(static_cast<size_t>(n0 * n1 * Hl) * cs);
        L.kt2 = take(static_cast<size_t>(n0 * P1 * Hl) * cs);
        L.z1 = take(static_cast<size_t>(M0 * M1 * Hl) * cs);
        L.z2 = take(static_cast<size_t>(M0 * P1 * Hl) * cs);
    }
    L.total = off;
    p.conv_ws_bytes = L.total;
    p.eval_ws_bytes = align_up(out->counts_bytes) + L.total;
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

int run_bin(const Plan& pl, const double* X, int64_t n, const kde_grid* g, uint64_t* counts, uint64_t* n_dropped,
            hipStream_t s, Tracer& tr) {
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
    KDE_LAUNCH(kde::launch_zero_u64(counts, cells, s), "zero_counts");
    if (n_dropped) KDE_LAUNCH(kde::launch_zero_u64(n_dropped, 1, s), "zero_dropped");
    if (n > 0) KDE_LAUNCH(kde::launch_bin(c, X, n, counts, n_dropped, s), "bin");
    return KDE_OK;
}

int run_conv(const Plan& pl, const uint64_t* counts, const kde_grid* g, void* density, char* ws, hipStream_t s,
             Tracer& tr) {
    const kde_plan& p = pl.pub;
    const Layout& L = pl.lay;
    const int d = p.d, prec = p.prec;
    void* lags = ws + L.lags;
    void* khat = ws + L.khat;
    void* kt1 = ws + L.kt1;
    void* kt2 = ws + L.kt2;
    void* z1 = ws + L.z1;
    void* z2 = ws + L.z2;
    double scale = std::ldexp(1.0, -d * p.Q);
    for (int k = 0; k < d; ++k) scale /= static_cast<double>(p.P[k]);

    KDE_LAUNCH(kde::launch_kfill(prec, d, p.L, pl.A, p.norm, lags, s), "kfill");
    if (d == 1) {
        const int P0 = p.P[0];
        const int64_t H0 = P0 / 2 + 1, M0 = g->M[0];
        KDE_LAUNCH(kde::launch_rows_r2c(prec, P0, kde::kRowLagsCirc, lags, 1, 2 * p.L[0] + 1, p.L[0], khat, H0,
                                        true, s), "kspec_r2c");
        KDE_LAUNCH(kde::launch_rows_r2c(prec, P0, kde::kRowCountsU64, counts, 1, M0, static_cast<int>(M0), z1, H0,
                                        false, s), "counts_r2c");
        KDE_LAUNCH(kde::launch_rows_c2r(prec, P0, z1, 1, H0, khat, density, M0, static_cast<int>(M0), scale, s),
                   "product_c2r");
        return KDE_OK;
    }
    if (d == 2) {
        const int P0 = p.P[0], P1 = p.P[1];
        const int64_t H1 = P1 / 2 + 1, M0 = g->M[0], M1 = g->M[1];
        const int64_t n0 = 2 * p.L[0] + 1, n1 = 2 * p.L[1] + 1;
        KDE_LAUNCH(kde::launch_rows_r2c(prec, P1, kde::kRowLagsCirc, lags, n0, n1, p.L[1], kt1, H1, false, s),
                   "kspec_r2c");
        kde::ColArgs ka{};
        ka.in = kt1;
        ka.out = khat;
        ka.W = H1;
        ka.outer = 1;
        ka.in_ps = H1;
        ka.out_ps = H1;
        ka.len = p.L[0];
        KDE_LAUNCH(kde::launch_cols(prec, P0, kde::kColFwdCircReal, ka, s), "kspec_col");
        KDE_LAUNCH(kde::launch_rows_r2c(prec, P1, kde::kRowCountsU64, counts, M0, M1, static_cast<int>(M1), z1, H1,
                                        false, s), "counts_r2c");
        kde::ColArgs ca{};
        ca.in = z1;
        ca.out = z1;
        ca.khat = khat;
        ca.W = H1;
        ca.outer = 1;
        ca.in_ps = H1;
        ca.out_ps = H1;
        ca.k_ps = H1;
        ca.len = static_cast<int>(M0);
        ca.mout = static_cast<int>(M0);
        KDE_LAUNCH(kde::launch_cols(prec, P0, kde::kColConv, ca, s), "conv_col");
        KDE_LAUNCH(kde::launch_rows_c2r(prec, P1, z1, M0, H1, nullptr, density, M1, static_cast<int>(M1), scale, s),
                   "c2r");
        return KDE_OK;
    }
    // d == 3
    const int P0 = p.P[0], P1 = p.P[1], P2 = p.P[2];
    const int64_t H2 = P2 / 2 + 1, M0 = g->M[0], M1 = g->M[1], M2 = g->M[2];
    const int64_t n0 = 2 * p.L[0] + 1, n1 = 2 * p.L[1] + 1, n2 = 2 * p.L[2] + 1;
    KDE_LAUNCH(kde::launch_rows_r2c(prec, P2, kde::kRowLagsCirc, lags, n0 * n1, n2, p.L[2], kt1, H2, false, s),
               "kspec_r2c");
    kde::ColArgs k1{};
    k1.in = kt1;
    k1.out = kt2;
    k1.W = H2;
    k1.outer = n0;
    k1.in_os = n1 * H2;
    k1.in_ps = H2;
    k1.out_os = static_cast<int64_t>(P1) * H2;
    k1.out_ps = H2;
    k1.len = p.L[1];
    KDE_LAUNCH(kde::launch_cols(prec, P1, kde::kColFwdCirc, k1, s), "kspec_col2");
    kde::ColArgs k0{};
    k0.in = kt2;
    k0.out = khat;
    k0.W = static_cast<int64_t>(P1) * H2;
    k0.outer = 1;
    k0.in_ps = k0.W;
    k0.out_ps = k0.W;
    k0.len = p.L[0];
    KDE_LAUNCH(kde::launch_cols(prec, P0, kde::kColFwdCircReal, k0, s), "kspec_col1");
    KDE_LAUNCH(kde::launch_rows_r2c(prec, P2, kde::kRowCountsU64, counts, M0 * M1, M2, static_cast<int>(M2), z1, H2,
                                    false, s), "counts_r2c");
    kde::ColArgs f1{};
    f1.in = z1;
    f1.out = z2;
    f1.W = H2;
    f1.outer = M0;
    f1.in_os = M1 * H2;
    f1.in_ps = H2;
    f1.out_os = static_cast<int64_t>(P1) * H2;
    f1.out_ps = H2;
    f1.len = static_cast<int>(M1);
    KDE_LAUNCH(kde::launch_cols(prec, P1, kde::kColFwdPrefix, f1, s), "counts_col2");
    kde::ColArgs cv{};
    cv.in = z2;
    cv.out = z2;
    cv.khat = khat;
    cv.W = static_cast<int64_t>(P1) * H2;
    cv.outer = 1;
    cv.in_ps = cv.W;
    cv.out_ps = cv.W;
    cv.k_ps = cv.W;
    cv.len = static_cast<int>(M0);
    cv.mout = static_cast<int>(M0);
    KDE_LAUNCH(kde::launch_cols(prec, P0, kde::kColConv, cv, s), "conv_col1");
    kde::ColArgs i1{};
    i1.in = z2;
    i1.out = z1;
    i1.W = H2;
    i1.outer = M0;
    i1.in_os = static_cast<int64_t>(P1) * H2;
    i1.in_ps = H2;
    i1.out_os = M1 * H2;
    i1.out_ps = H2;
    i1.mout = static_cast<int>(M1);
    KDE_LAUNCH(kde::launch_cols(prec, P1, kde::kColInvPrefix, i1, s), "inv_col2");
    KDE_LAUNCH(kde::launch_rows_c2r(prec, P2, z1, M0 * M1, H2, nullptr, density, M2, static_cast<int>(M2), scale, s),
               "c2r");
    return KDE_OK;
}

}  // namespace

extern "C" {

int kde_plan_query(const double* H, int64_t n, const kde_grid* grid, const kde_params* params, kde_plan* out) {
    if (!out) return KDE_ERR_ARG;
    Plan pl;
    const int rc = make_plan(H, n, 1, true, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    *out = pl.pub;
    return KDE_OK;
}

int kde_bin(const double* X, int64_t n, const kde_grid* grid, const kde_params* params, uint64_t* counts,
            uint64_t* n_dropped, hipStream_t stream) {
    Plan pl;
    const int rc = make_plan(nullptr, n, 0, false, grid, params, &pl);
    if (rc != KDE_OK) return rc;
    if (!counts || (n > 0 && !X)) return KDE_ERR_ARG;
    Tracer tr(params, stream);
    KDE_TRY(tr.start());
    const int r = run_bin(pl, X, n, grid, counts, n_dropped, stream, tr);
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
    const int r = run_conv(pl, counts, grid, density, static_cast<char*>(ws), stream, tr);
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
    char* conv_ws = static_cast<char*>(ws) + align_up(pl.counts_bytes);
    Tracer tr(params, stream);
    KDE_TRY(tr.start());
    int r = run_bin(pl, X, n, grid, counts, n_dropped, stream, tr);
    if (r == KDE_OK) r = run_conv(pl, counts, grid, density, conv_ws, stream, tr);
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
