// Lanczos evaluation of exp(-i tau H) theta (Sec. III A, Park-Light Lanczos
// exponentiation).  Krylov vectors stay in complex128 on the device; every
// iteration applies H once, subtracts the three-term recurrence, runs two
// classical Gram-Schmidt passes against all previous vectors, and reads back
// only alpha_k and ||w||^2.  The k x k tridiagonal matrix is diagonalised on
// the host; the iteration stops when beta_k |e_k^T exp(-i tau T_k) e_1| <= tol
// (a-posteriori estimate) or on a happy breakdown.
//
// Short vectors (one-workgroup recurrence step) queue several iterations
// before reading their scalars back: each step takes beta_{k-1} from the
// device, so the host synchronises once per batch instead of once per
// iteration.  Iterations queued past the stopping point only touch Krylov
// vectors that are never combined.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace tdvp {

namespace {
constexpr int kFirstBatch = 8;  // first batch when no earlier run of this length is known
constexpr int kNextBatch = 2;
}  // namespace

void tridiag_eigen(const std::vector<double>& alpha, const std::vector<double>& beta, const std::vector<int>& rows,
                   std::vector<double>& evals, std::vector<double>& z) {
    // Implicit QL iterations with Wilkinson shifts (Golub & Van Loan,
    // Sec. 8.3): each sweep chases a bulge from the bottom of the active
    // block to its top with plane rotations, which are also applied to the
    // requested rows of the eigenvector matrix.  O(k^2) work for a fixed
    // number of rows instead of the O(k^3) per sweep of dense rotations.
    const int k = (int)alpha.size();
    const int nr = (int)rows.size();
    std::vector<double> d = alpha;
    std::vector<double> e(k, 0.0);
    for (int i = 0; i + 1 < k; ++i) e[i] = beta[i];
    z.assign((size_t)nr * k, 0.0);
    for (int r = 0; r < nr; ++r) z[(size_t)r * k + rows[r]] = 1.0;
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < k; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m + 1 < k; ++m)  // first negligible coupling at or after l
                if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
            if (m == l) break;
            TDVP_REQUIRE(iter < 60, TDVP_E_NUMERIC, "Krylov: tridiagonal eigen-solver did not converge");
            // shift: the eigenvalue of the leading 2 x 2 block nearer to d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::sqrt(f * f + g * g);  // entries are of the order of ||T||
                e[i + 1] = r;
                if (r == 0.0) {  // exact zero: the block splits at i
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int q = 0; q < nr; ++q) {  // the same rotation on columns i, i + 1
                    double* zq = &z[(size_t)q * k];
                    const double zi1 = zq[i + 1];
                    zq[i + 1] = s * zq[i] + c * zi1;
                    zq[i] = c * zq[i] - s * zi1;
                }
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    evals = d;
}

namespace {

enum class KrylovMode { Exp, Ground };

// Lanczos driver.  Exp: theta <- exp(-i tau H) theta.  Ground: theta <- the
// normalised Ritz vector of the lowest Ritz value, *energy = that value.
KrylovInfo krylov_run(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau, int kmax, double tol,
                      KrylovMode mode, double* energy, bool imaginary) {
    // exp(-i tau lambda), or exp(-tau lambda) in imaginary time
    auto phase = [&](double lam) {
        return imaginary ? double2{std::exp(-tau * lam), 0.0} : double2{std::cos(-tau * lam), std::sin(-tau * lam)};
    };
    KrylovInfo info;
    TDVP_REQUIRE(kmax >= 1, TDVP_E_ARG, "krylov_max must be >= 1");
    if (n == 0) return info;
    hipStream_t s = ctx->stream;
    double2* V = static_cast<double2*>(ctx->workspace("kry_V", sizeof(double2) * (size_t)(kmax + 1) * n));
    double2* w = static_cast<double2*>(ctx->workspace("kry_w", sizeof(double2) * (size_t)n));
    double2* scal = static_cast<double2*>(ctx->workspace("kry_scal", sizeof(double2) * 4));
    double2* coef = static_cast<double2*>(ctx->workspace("kry_coef", sizeof(double2) * (size_t)(kmax + 2)));
    double2 host[2];
    const bool small = n <= kSmallLanczos && kmax < 64;
    double beta0 = 0.0;
    auto check_beta0 = [&](double nn0) {
        beta0 = std::sqrt(std::max(0.0, nn0));
        TDVP_REQUIRE(std::isfinite(beta0), TDVP_E_NUMERIC, "Krylov: non-finite input norm");
    };
    if (!small) {
        vdot_multi(ctx, theta, 0, 1, theta, n, scal + 1);
        TDVP_CHECK_HIP(hipMemcpyAsync(host, scal + 1, sizeof(double2), hipMemcpyDeviceToHost, s));
        TDVP_CHECK_HIP(hipStreamSynchronize(s));
        check_beta0(host[0].x);
        if (beta0 == 0.0) return info;
        scale_copy(V, theta, 1.0 / beta0, n, s);
    }

    std::vector<double> alphas, betas, evals, z;
    std::vector<double2> y;
    int k_used = 0;
    // Ground mode: the residual norm of the lowest Ritz pair is
    // beta_k |e_{kk-1}^T z_min| (z_min its eigenvector of T_kk).
    auto consume_ground = [&](int k, double b, int kk) -> bool {
        tridiag_eigen(alphas, betas, {kk - 1}, evals, z);
        int imin = 0;
        for (int i = 1; i < kk; ++i)
            if (evals[i] < evals[imin]) imin = i;
        double scale = 0.0;
        for (double v : alphas) scale = std::max(scale, std::fabs(v));
        for (double v : betas) scale = std::max(scale, v);
        bool stop = b * std::fabs(z[imin]) <= tol || b <= 1e-14 * scale || scale == 0.0;
        if (!stop && k + 1 == kmax) {
            info.converged = false;
            stop = true;
        }
        if (!stop) {
            betas.push_back(b);
            return false;
        }
        std::vector<int> all(kk);
        for (int j = 0; j < kk; ++j) all[j] = j;
        tridiag_eigen(alphas, betas, all, evals, z);
        imin = 0;
        for (int i = 1; i < kk; ++i)
            if (evals[i] < evals[imin]) imin = i;
        if (energy) *energy = evals[imin];
        y.assign(kk, double2{0.0, 0.0});
        for (int j = 0; j < kk; ++j) y[j].x = z[(size_t)j * kk + imin];
        k_used = kk;
        return true;
    };
    // Consumes iteration k's alpha_k and ||w||^2; returns true when the
    // iteration stops here.
    auto consume = [&](int k, double a, double nn) -> bool {
        const double b = std::sqrt(std::max(0.0, nn));
        ++info.matvecs;
        TDVP_REQUIRE(std::isfinite(a) && std::isfinite(b), TDVP_E_NUMERIC,
                     "Krylov: non-finite value in H_eff application");
        alphas.push_back(a);
        const int kk = (int)alphas.size();
        if (mode == KrylovMode::Ground) return consume_ground(k, b, kk);
        // e_{kk-1}^T exp(-i tau T) e_0 needs the first and last eigenvector rows only
        tridiag_eigen(alphas, betas, {0, kk - 1}, evals, z);
        double yr = 0.0, yi = 0.0;
        for (int i = 0; i < kk; ++i) {
            const double f = z[(size_t)kk + i] * z[i];
            const double2 e = phase(evals[i]);
            yr += f * e.x;
            yi += f * e.y;
        }
        double scale = 0.0;
        for (double v : alphas) scale = std::max(scale, std::fabs(v));
        for (double v : betas) scale = std::max(scale, v);
        const double est = b * std::hypot(yr, yi);
        bool stop = est <= tol || b <= 1e-14 * scale || scale == 0.0;
        if (!stop && k + 1 == kmax) {
            info.converged = false;
            stop = true;
        }
        if (!stop) {
            betas.push_back(b);
            return false;
        }
        // y = exp(-i tau T) e_0 in full
        std::vector<int> all(kk);
        for (int j = 0; j < kk; ++j) all[j] = j;
        tridiag_eigen(alphas, betas, all, evals, z);
        y.assign(kk, double2{0.0, 0.0});
        for (int i = 0; i < kk; ++i) {
            const double2 e = phase(evals[i]);
            const double c0 = e.x, s0 = e.y;
            const double w0 = z[i];  // row 0
            for (int j = 0; j < kk; ++j) {
                const double f = z[(size_t)j * kk + i] * w0;
                y[j].x += f * c0;
                y[j].y += f * s0;
            }
        }
        k_used = kk;
        return true;
    };
    if (small) {
        // the whole recurrence step in one workgroup (it writes v_{k+1});
        // ||theta||^2 at sc[0], scalars of iteration k at sc[1 + 2k], sc[2 + 2k]
        double* sc = static_cast<double*>(ctx->workspace("kry_small_sc", sizeof(double) * (1 + 2 * (size_t)kmax)));
        std::vector<double> hs(1 + 2 * (size_t)kmax);
        small_normalize(theta, V, n, sc, s);  // read back with the first batch
        // consecutive exponentials of one vector length need similar
        // iteration counts: the first batch is the count of the last one
        int& hint = ctx->krylov_hint[mode == KrylovMode::Exp ? n : -n];
        const int first = hint > 0 ? std::max(2, hint) : kFirstBatch;
        int queued = 0;
        bool stop = false;
        while (!stop) {
            const int end = std::min(kmax, queued + (queued == 0 ? first : kNextBatch));
            for (int k = queued; k < end; ++k) {
                op(V + (size_t)k * n, w);
                lanczos_small_step(V, n, k, w, 0.0, k > 0 ? sc + 2 * k : nullptr, sc + 1 + 2 * k, s);
            }
            const int lo = queued == 0 ? 0 : 1 + 2 * queued;
            TDVP_CHECK_HIP(hipMemcpyAsync(hs.data() + lo, sc + lo, sizeof(double) * (1 + 2 * end - lo),
                                          hipMemcpyDeviceToHost, s));
            TDVP_CHECK_HIP(hipStreamSynchronize(s));
            if (queued == 0) {
                check_beta0(hs[0]);
                if (beta0 == 0.0) return info;  // the queued steps ran on zero vectors
            }
            for (int k = queued; k < end && !stop; ++k) stop = consume(k, hs[1 + 2 * k], hs[2 + 2 * k]);
            queued = end;
        }
        hint = k_used;
    } else {
        for (int k = 0; k < kmax; ++k) {
            double2* vk = V + (size_t)k * n;
            op(vk, w);
            vdot_multi(ctx, vk, 0, 1, w, n, scal);  // alpha_k = <v_k, H v_k>
            lanczos_3term(w, vk, k > 0 ? V + (size_t)(k - 1) * n : nullptr, scal,
                          k > 0 ? betas.back() : 0.0, n, s);
            for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
                vdot_multi(ctx, V, n, k + 1, w, n, coef);
                axpy_multi(V, n, k + 1, coef, w, n, s);
            }
            vdot_multi(ctx, w, 0, 1, w, n, scal + 1);
            TDVP_CHECK_HIP(hipMemcpyAsync(host, scal, 2 * sizeof(double2), hipMemcpyDeviceToHost, s));
            TDVP_CHECK_HIP(hipStreamSynchronize(s));
            if (consume(k, host[0].x, host[1].x)) break;
            scale_copy(V + (size_t)(k + 1) * n, w, 1.0 / betas.back(), n, s);
        }
    }
    if (mode == KrylovMode::Exp) {  // the Ritz vector of Ground mode stays normalised
        for (auto& c : y) {
            c.x *= beta0;
            c.y *= beta0;
        }
    }
    // Pinned staging: the copy runs asynchronously, and every call
    // synchronises the stream before it writes the staging buffer again.
    double2* pin = static_cast<double2*>(ctx->pinned_host(sizeof(double2) * (size_t)k_used));
    std::copy(y.begin(), y.begin() + k_used, pin);
    TDVP_CHECK_HIP(hipMemcpyAsync(coef, pin, sizeof(double2) * k_used, hipMemcpyHostToDevice, s));
    combine(theta, V, n, k_used, coef, n, s);
    info.k = k_used;
    return info;
}

}  // namespace

KrylovInfo expm_krylov(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau, int kmax, double tol,
                       bool imaginary) {
    return krylov_run(ctx, op, theta, n, tau, kmax, tol, KrylovMode::Exp, nullptr, imaginary);
}

KrylovInfo ground_krylov(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, int kmax, double tol,
                         double* energy) {
    return krylov_run(ctx, op, theta, n, 0.0, kmax, tol, KrylovMode::Ground, energy, false);
}

}  // namespace tdvp
