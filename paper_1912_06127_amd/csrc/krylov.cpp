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

namespace tdvp {

namespace {
constexpr int kFirstBatch = 8;  // first batch when no earlier run of this length is known
constexpr int kNextBatch = 2;
}  // namespace

void tridiag_eigen(const std::vector<double>& alpha, const std::vector<double>& beta,
                   std::vector<double>& evals, std::vector<double>& evecs) {
    // Cyclic Jacobi rotations on the dense symmetric matrix (k <= a few dozen).
    const int k = (int)alpha.size();
    std::vector<double> A((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) A[i * k + i] = alpha[i];
    for (int i = 0; i + 1 < k; ++i) A[i * k + i + 1] = A[(i + 1) * k + i] = beta[i];
    evecs.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) evecs[i * k + i] = 1.0;
    double scale = 0.0;
    for (double v : A) scale = std::max(scale, std::fabs(v));
    for (int sweep = 0; sweep < 100 && k > 1; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) off = std::max(off, std::fabs(A[p * k + q]));
        if (off <= 1e-300 || off <= 1e-18 * scale) break;
        for (int p = 0; p < k; ++p) {
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[p * k + q];
                if (std::fabs(apq) <= 1e-300) continue;
                const double tau = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < k; ++r) {  // columns p, q
                    const double arp = A[r * k + p], arq = A[r * k + q];
                    A[r * k + p] = c * arp - s * arq;
                    A[r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {  // rows p, q
                    const double apr = A[p * k + r], aqr = A[q * k + r];
                    A[p * k + r] = c * apr - s * aqr;
                    A[q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {
                    const double vrp = evecs[r * k + p], vrq = evecs[r * k + q];
                    evecs[r * k + p] = c * vrp - s * vrq;
                    evecs[r * k + q] = s * vrp + c * vrq;
                }
            }
        }
    }
    evals.resize(k);
    for (int i = 0; i < k; ++i) evals[i] = A[i * k + i];
}

KrylovInfo expm_krylov(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau,
                       int kmax, double tol) {
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

    std::vector<double> alphas, betas, evals, evecs;
    std::vector<double2> y;
    int k_used = 0;
    // Consumes iteration k's alpha_k and ||w||^2; returns true when the
    // iteration stops here.
    auto consume = [&](int k, double a, double nn) -> bool {
        const double b = std::sqrt(std::max(0.0, nn));
        ++info.matvecs;
        TDVP_REQUIRE(std::isfinite(a) && std::isfinite(b), TDVP_E_NUMERIC,
                     "Krylov: non-finite value in H_eff application");
        alphas.push_back(a);
        tridiag_eigen(alphas, betas, evals, evecs);
        const int kk = (int)alphas.size();
        y.assign(kk, double2{0.0, 0.0});
        for (int i = 0; i < kk; ++i) {
            const double ph = -tau * evals[i];
            const double w0 = evecs[0 * kk + i];
            for (int j = 0; j < kk; ++j) {
                const double f = evecs[j * kk + i] * w0;
                y[j].x += f * std::cos(ph);
                y[j].y += f * std::sin(ph);
            }
        }
        k_used = k + 1;
        double scale = 0.0;
        for (double v : alphas) scale = std::max(scale, std::fabs(v));
        for (double v : betas) scale = std::max(scale, v);
        const double est = b * std::hypot(y[kk - 1].x, y[kk - 1].y);
        if (est <= tol || b <= 1e-14 * scale || scale == 0.0) return true;
        if (k + 1 == kmax) {
            info.converged = false;
            return true;
        }
        betas.push_back(b);
        return false;
    };
    if (small) {
        // the whole recurrence step in one workgroup (it writes v_{k+1});
        // ||theta||^2 at sc[0], scalars of iteration k at sc[1 + 2k], sc[2 + 2k]
        double* sc = static_cast<double*>(ctx->workspace("kry_small_sc", sizeof(double) * (1 + 2 * (size_t)kmax)));
        std::vector<double> hs(1 + 2 * (size_t)kmax);
        small_normalize(theta, V, n, sc, s);  // read back with the first batch
        // consecutive exponentials of one vector length need similar
        // iteration counts: the first batch is the count of the last one
        int& hint = ctx->krylov_hint[n];
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
    for (auto& c : y) {
        c.x *= beta0;
        c.y *= beta0;
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

}  // namespace tdvp
