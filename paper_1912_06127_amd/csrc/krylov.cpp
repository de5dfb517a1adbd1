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

enum class KrylovMode { Exp, Ground, Interval };

// Lanczos driver.  Exp: theta <- exp(-i tau H) theta.  Ground: theta <- the
// normalised Ritz vector of the lowest Ritz value, *energy = that value.
// Interval: kmax steps (fewer on breakdown), theta unchanged, energy[0..1] =
// [min_i (r_i - res_i), max_i (r_i + res_i)] over the Ritz values r_i with
// residual norms res_i = beta_k |e_k^T z_i| (an enclosure of the spectrum
// seen from theta; [0, 0] for a zero theta).
KrylovInfo krylov_run(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau, int kmax, double tol,
                      KrylovMode mode, double* energy, bool imaginary) {
    // exp(-i tau lambda), or exp(-tau lambda) in imaginary time
    auto phase = [&](double lam) {
        return imaginary ? double2{std::exp(-tau * lam), 0.0} : double2{std::cos(-tau * lam), std::sin(-tau * lam)};
    };
    KrylovInfo info;
    TDVP_REQUIRE(kmax >= 1, TDVP_E_ARG, "krylov_max must be >= 1");
    if (mode == KrylovMode::Interval) energy[0] = energy[1] = 0.0;
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
        beta0 = sqrt_or_nan(nn0);
        TDVP_REQUIRE(std::isfinite(beta0), TDVP_E_NUMERIC, "Krylov: non-finite input norm");
    };
    if (!small) {
        vdot_multi(ctx, theta, 0, 1, theta, n, scal + 1);
        ctx->read_back({{host, scal + 1, sizeof(double2)}});
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
        const double b = sqrt_or_nan(nn);
        ++info.matvecs;
        TDVP_REQUIRE(std::isfinite(a) && std::isfinite(b), TDVP_E_NUMERIC,
                     "Krylov: non-finite value in H_eff application");
        alphas.push_back(a);
        const int kk = (int)alphas.size();
        if (mode == KrylovMode::Ground) return consume_ground(k, b, kk);
        if (mode == KrylovMode::Interval) {
            double scale = 0.0;
            for (double v : alphas) scale = std::max(scale, std::fabs(v));
            for (double v : betas) scale = std::max(scale, v);
            if (k + 1 < kmax && b > 1e-14 * scale && scale != 0.0) {
                betas.push_back(b);
                return false;
            }
            tridiag_eigen(alphas, betas, {kk - 1}, evals, z);
            double lo = evals[0] - b * std::fabs(z[0]), hi = evals[0] + b * std::fabs(z[0]);
            for (int i = 1; i < kk; ++i) {
                lo = std::min(lo, evals[i] - b * std::fabs(z[i]));
                hi = std::max(hi, evals[i] + b * std::fabs(z[i]));
            }
            energy[0] = lo;
            energy[1] = hi;
            return true;
        }
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
        const int first = mode == KrylovMode::Interval ? kmax : (hint > 0 ? std::max(2, hint) : kFirstBatch);
        int queued = 0;
        bool stop = false;
        while (!stop) {
            const int end = std::min(kmax, queued + (queued == 0 ? first : kNextBatch));
            for (int k = queued; k < end; ++k) {
                op(V + (size_t)k * n, w);
                lanczos_small_step(V, n, k, w, 0.0, k > 0 ? sc + 2 * k : nullptr, sc + 1 + 2 * k, s);
            }
            const int lo = queued == 0 ? 0 : 1 + 2 * queued;
            ctx->read_back({{hs.data() + lo, sc + lo, sizeof(double) * (1 + 2 * end - lo)}});
            if (queued == 0) {
                check_beta0(hs[0]);
                if (beta0 == 0.0) return info;  // the queued steps ran on zero vectors
            }
            for (int k = queued; k < end && !stop; ++k) stop = consume(k, hs[1 + 2 * k], hs[2 + 2 * k]);
            queued = end;
        }
        if (mode != KrylovMode::Interval) hint = k_used;
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
            ctx->read_back({{host, scal, 2 * sizeof(double2)}});
            if (consume(k, host[0].x, host[1].x)) break;
            scale_copy(V + (size_t)(k + 1) * n, w, 1.0 / betas.back(), n, s);
        }
    }
    if (mode == KrylovMode::Interval) return info;
    if (mode == KrylovMode::Exp) {  // the Ritz vector of Ground mode stays normalised
        for (auto& c : y) {
            c.x *= beta0;
            c.y *= beta0;
        }
    }
    if (k_used <= kCombineArgs) {
        combine_args(theta, V, n, k_used, y.data(), n, s);
    } else {
        // Pinned staging: the copy runs asynchronously, and every call
        // synchronises the stream before it writes the staging buffer again.
        double2* pin = static_cast<double2*>(ctx->pinned_host(sizeof(double2) * (size_t)k_used));
        std::copy(y.begin(), y.begin() + k_used, pin);
        TDVP_CHECK_HIP(hipMemcpyAsync(coef, pin, sizeof(double2) * k_used, hipMemcpyHostToDevice, s));
        combine(theta, V, n, k_used, coef, n, s);
    }
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

namespace {
#include "taylor_theta.inc"
constexpr int kIntervalSteps = 16;
constexpr double kTaylorMaxSteps = 1e5;
}  // namespace

// Truncated Taylor series with scaling (Al-Mohy and Higham 2011), applied
// to the Hermitian H_eff through its matvec only.  The norm in the degree
// selection is the spectral norm, exact for a Hermitian operator: the
// spectrum seen from theta is enclosed by a short Lanczos run, the operator
// is shifted to the midpoint c of that enclosure (exp(-i tau H) = e^{-i tau c}
// exp(-i tau (H - c))) and ||tau (H - c)|| <= |tau| rho with rho the
// half-width, widened by 5 %.  Then (m, s) minimise m s subject to
// |tau| rho / s <= theta_m, and each of the s steps sums at most m terms,
// stopping early once two consecutive terms are below tol relative to the
// partial sum.
KrylovInfo expm_taylor(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau, double tol,
                       bool imaginary) {
    KrylovInfo info;
    if (n == 0 || tau == 0.0) return info;
    double iv[2];
    info = krylov_run(ctx, op, theta, n, 0.0, (int)std::min<int64_t>(kIntervalSteps, n), 0.0, KrylovMode::Interval,
                      iv, false);
    if (iv[0] == 0.0 && iv[1] == 0.0 && info.matvecs == 0) return info;  // theta vanishes
    const double c = 0.5 * (iv[0] + iv[1]);
    const double rho = 0.5 * (iv[1] - iv[0]) * 1.05;
    const double anorm = std::fabs(tau) * rho;
    TDVP_REQUIRE(std::isfinite(anorm), TDVP_E_NUMERIC, "Taylor exponential: non-finite spectral bound");
    TDVP_REQUIRE(anorm <= kTaylorTheta[kTaylorMaxDegree] * kTaylorMaxSteps, TDVP_E_ARG,
                 "Taylor exponential: |tau| ||H_eff|| needs more than 1e5 scaling steps");
    int m = 0, s = 1;
    if (anorm > 0.0) {
        double best = 0.0;
        for (int mm = 1; mm <= kTaylorMaxDegree; ++mm) {
            const double ss = std::max(1.0, std::ceil(anorm / kTaylorTheta[mm]));
            if (m == 0 || mm * ss < best) {
                best = mm * ss;
                m = mm;
                s = (int)ss;
            }
        }
    }
    hipStream_t st = ctx->stream;
    double2* F = static_cast<double2*>(ctx->workspace("tay_F", sizeof(double2) * (size_t)n));
    double2* b = static_cast<double2*>(ctx->workspace("tay_b", sizeof(double2) * (size_t)n));
    double2* y = static_cast<double2*>(ctx->workspace("tay_y", sizeof(double2) * (size_t)n));
    double2* nrm = static_cast<double2*>(ctx->workspace("tay_nrm", sizeof(double2) * 2));
    TDVP_CHECK_HIP(hipMemcpyAsync(F, theta, sizeof(double2) * (size_t)n, hipMemcpyDeviceToDevice, st));
    TDVP_CHECK_HIP(hipMemcpyAsync(b, theta, sizeof(double2) * (size_t)n, hipMemcpyDeviceToDevice, st));
    // A = -i tau (H - c), or -tau (H - c) in imaginary time; eta = e^{-i tau c / s} (e^{-tau c / s})
    const double2 eta = imaginary ? double2{std::exp(-tau * c / s), 0.0}
                                  : double2{std::cos(-tau * c / s), std::sin(-tau * c / s)};
    double2 h[2];
    auto norms = [&](double& nb, double& nf) {
        vdot_multi(ctx, b, 0, 1, b, n, nrm);
        vdot_multi(ctx, F, 0, 1, F, n, nrm + 1);
        TDVP_CHECK_HIP(hipMemcpyAsync(h, nrm, sizeof(h), hipMemcpyDeviceToHost, st));
        TDVP_CHECK_HIP(hipStreamSynchronize(st));
        nb = sqrt_or_nan(h[0].x);
        nf = sqrt_or_nan(h[1].x);
        TDVP_REQUIRE(std::isfinite(nb) && std::isfinite(nf), TDVP_E_NUMERIC,
                     "Taylor exponential: non-finite value in H_eff application");
    };
    int terms = 0;
    for (int i = 0; i < s; ++i) {
        double c1 = 0.0, c2 = 0.0, nf = 0.0;
        norms(c1, nf);
        for (int j = 1; j <= m; ++j) {
            op(b, y);
            ++info.matvecs;
            const double f = tau / ((double)s * j);
            const double2 alpha = imaginary ? double2{-f, 0.0} : double2{0.0, -f};
            taylor_term(b, y, F, n, alpha, c, st);
            terms = std::max(terms, j);
            norms(c2, nf);
            if (c1 + c2 <= tol * nf) break;
            c1 = c2;
        }
        taylor_rescale(F, b, n, eta, st);
    }
    TDVP_CHECK_HIP(hipMemcpyAsync(theta, F, sizeof(double2) * (size_t)n, hipMemcpyDeviceToDevice, st));
    info.k = terms;
    info.converged = true;
    return info;
}

}  // namespace tdvp
