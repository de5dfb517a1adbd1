// Sums of exponentials for power-law couplings (Sec. II C; the fit the
// Supplemental Material uses for the long-range XXX model).
//
// A power law has no compact MPO, so f(r) = r^-alpha is approximated on
// r = 1..R by Re sum_k c_k lambda_k^r, which the MPO carries with one decaying
// channel per exponential.  The paper cites Pirvu et al. for the fit without
// stating its steps; this is the matrix-pencil reading:
//   1. Hankel matrix Y[i][j] = f(i + j + 1), i = 0..R-P-1, j = 0..P, P = R/2;
//   2. its K dominant right singular vectors (one-sided Jacobi SVD, which
//      keeps small singular values accurate);
//   3. lambda_k = eigenvalues of the shift operator that maps the first P
//      entries of those vectors to the last P (least squares, then the
//      eigenvalues of a small nonsymmetric matrix by the complex
//      Hessenberg QR iteration with Wilkinson shifts);
//   4. c_k by linear least squares on all R samples (Householder QR of the
//      Vandermonde matrix).
// Optionally the result is refined: Levenberg-Marquardt on the 4K real
// parameters (real and imaginary parts of c and lambda) for the residuals
// Re(sum) - f and Im(sum) (the second keeps conjugate pairs conjugate),
// inside Lawson reweighting towards the minimax fit; the refined fit is kept
// only when its maximum error is smaller.  Host code: runs once per MPO.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace tdvp {
namespace {

using zc = std::complex<double>;

// One-sided Jacobi SVD of the real m x n matrix A (row-major): returns the
// singular values (descending) and the right singular vectors as the rows
// of Vt (n x n).
void jacobi_svd(std::vector<double> A, int m, int n, std::vector<double>& sv, std::vector<double>& Vt) {
    std::vector<double> V((size_t)n * n, 0.0);  // column-major accumulation: V[i + n*j]
    for (int i = 0; i < n; ++i) V[i + (size_t)n * i] = 1.0;
    auto col = [&](int j, int i) -> double& { return A[(size_t)i * n + j]; };
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = 0; i < m; ++i) {
                    const double x = col(p, i), y = col(q, i);
                    a += x * x;
                    b += y * y;
                    g += x * y;
                }
                if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
                off = std::max(off, std::fabs(g) / std::sqrt(a * b));
                // rotation that zeroes the (p, q) entry of the Gram matrix
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < m; ++i) {
                    const double x = col(p, i), y = col(q, i);
                    col(p, i) = cs * x - sn * y;
                    col(q, i) = sn * x + cs * y;
                }
                for (int i = 0; i < n; ++i) {
                    const double x = V[i + (size_t)n * p], y = V[i + (size_t)n * q];
                    V[i + (size_t)n * p] = cs * x - sn * y;
                    V[i + (size_t)n * q] = sn * x + cs * y;
                }
            }
        if (off <= 1e-14) break;
    }
    std::vector<double> norms(n);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += col(j, i) * col(j, i);
        norms[j] = std::sqrt(s);
    }
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return norms[x] > norms[y]; });
    sv.resize(n);
    Vt.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) {
        sv[r] = norms[order[r]];
        for (int i = 0; i < n; ++i) Vt[(size_t)r * n + i] = V[i + (size_t)n * order[r]];
    }
}

// Solve the n x n system A x = b (row-major, copied) by Gaussian elimination
// with partial pivoting; b holds nrhs right-hand sides as columns [n][nrhs].
template <class T>
void solve(std::vector<T> A, std::vector<T>& b, int n, int nrhs) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::abs(A[(size_t)i * n + k]) > std::abs(A[(size_t)piv * n + k])) piv = i;
        TDVP_REQUIRE(std::abs(A[(size_t)piv * n + k]) > 0.0, TDVP_E_NUMERIC, "exponential fit: singular system");
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
            for (int j = 0; j < nrhs; ++j) std::swap(b[(size_t)k * nrhs + j], b[(size_t)piv * nrhs + j]);
        }
        for (int i = k + 1; i < n; ++i) {
            const T f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
            if (f == T(0)) continue;
            for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
            for (int j = 0; j < nrhs; ++j) b[(size_t)i * nrhs + j] -= f * b[(size_t)k * nrhs + j];
        }
    }
    for (int k = n - 1; k >= 0; --k)
        for (int j = 0; j < nrhs; ++j) {
            T s = b[(size_t)k * nrhs + j];
            for (int i = k + 1; i < n; ++i) s -= A[(size_t)k * n + i] * b[(size_t)i * nrhs + j];
            b[(size_t)k * nrhs + j] = s / A[(size_t)k * n + k];
        }
}

// Eigenvalues of the complex n x n matrix H (row-major): Householder
// reduction to Hessenberg form, then shifted QR steps (Givens rotations,
// Wilkinson shift from the trailing 2 x 2 block) with deflation.
std::vector<zc> eigenvalues(std::vector<zc> H, int n) {
    auto h = [&](int i, int j) -> zc& { return H[(size_t)i * n + j]; };
    for (int k = 0; k + 2 < n; ++k) {  // Hessenberg reduction
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += std::norm(h(i, k));
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        std::vector<zc> v(n, 0.0);
        const zc x0 = h(k + 1, k);
        const zc ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : zc(1.0);
        for (int i = k + 1; i < n; ++i) v[i] = h(i, k);
        v[k + 1] += ph * alpha;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
        if (vn == 0.0) continue;
        // H <- (I - 2 v v^H / v^H v) H (I - 2 v v^H / v^H v)
        for (int j = 0; j < n; ++j) {
            zc s = 0.0;
            for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * h(i, j);
            s *= 2.0 / vn;
            for (int i = k + 1; i < n; ++i) h(i, j) -= v[i] * s;
        }
        for (int i = 0; i < n; ++i) {
            zc s = 0.0;
            for (int j = k + 1; j < n; ++j) s += h(i, j) * v[j];
            s *= 2.0 / vn;
            for (int j = k + 1; j < n; ++j) h(i, j) -= s * std::conj(v[j]);
        }
    }
    std::vector<zc> ev(n);
    int hi = n - 1, iter = 0;
    while (hi >= 0) {
        if (hi == 0) {
            ev[0] = h(0, 0);
            break;
        }
        int lo = hi;  // find the unreduced block [lo, hi]
        while (lo > 0) {
            const double s = std::abs(h(lo, lo)) + std::abs(h(lo - 1, lo - 1));
            if (std::abs(h(lo, lo - 1)) <= 4e-16 * (s > 0 ? s : 1.0)) {
                h(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            ev[hi] = h(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        TDVP_REQUIRE(++iter < 300, TDVP_E_NOCONV, "exponential fit: eigenvalue iteration did not converge");
        // Wilkinson shift: eigenvalue of the trailing 2 x 2 block closest to h(hi, hi)
        const zc a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
        const zc tr = a + d, disc = std::sqrt((a - d) * (a - d) + 4.0 * b * c);
        const zc m1 = 0.5 * (tr + disc), m2 = 0.5 * (tr - disc);
        zc mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        if (iter % 11 == 10) mu += std::abs(h(hi, hi - 1));  // exceptional shift
        // QR step on the active block via Givens rotations: H - mu = Q R, H <- R Q + mu
        std::vector<zc> cs(hi - lo), sn(hi - lo);
        for (int i = lo; i <= hi; ++i) h(i, i) -= mu;
        for (int k = lo; k < hi; ++k) {
            const zc x = h(k, k), y = h(k + 1, k);
            const double r = std::sqrt(std::norm(x) + std::norm(y));
            const zc cc = r > 0 ? x / r : zc(1.0), ss = r > 0 ? y / r : zc(0.0);
            cs[k - lo] = cc;
            sn[k - lo] = ss;
            for (int j = k; j < n; ++j) {  // rows k, k+1 <- G^H rows
                const zc u = h(k, j), w = h(k + 1, j);
                h(k, j) = std::conj(cc) * u + std::conj(ss) * w;
                h(k + 1, j) = -ss * u + cc * w;
            }
        }
        for (int k = lo; k < hi; ++k) {  // columns k, k+1 <- columns G
            const zc cc = cs[k - lo], ss = sn[k - lo];
            for (int i = 0; i <= std::min(k + 2, hi); ++i) {
                const zc u = h(i, k), w = h(i, k + 1);
                h(i, k) = u * cc + w * ss;
                h(i, k + 1) = -u * std::conj(ss) + w * std::conj(cc);
            }
        }
        for (int i = lo; i <= hi; ++i) h(i, i) += mu;
    }
    return ev;
}

// Least squares min ||Z x - f|| for the complex R x K matrix Z (row-major)
// by Householder QR.
std::vector<zc> lstsq(std::vector<zc> Z, std::vector<zc> f, int R, int K) {
    auto z = [&](int i, int j) -> zc& { return Z[(size_t)i * K + j]; };
    for (int k = 0; k < K; ++k) {
        double alpha = 0.0;
        for (int i = k; i < R; ++i) alpha += std::norm(z(i, k));
        alpha = std::sqrt(alpha);
        TDVP_REQUIRE(alpha > 0.0, TDVP_E_NUMERIC, "exponential fit: rank-deficient Vandermonde matrix");
        const zc x0 = z(k, k);
        const zc ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : zc(1.0);
        std::vector<zc> v(R, 0.0);
        for (int i = k; i < R; ++i) v[i] = z(i, k);
        v[k] += ph * alpha;
        double vn = 0.0;
        for (int i = k; i < R; ++i) vn += std::norm(v[i]);
        for (int j = k; j < K; ++j) {
            zc s = 0.0;
            for (int i = k; i < R; ++i) s += std::conj(v[i]) * z(i, j);
            s *= 2.0 / vn;
            for (int i = k; i < R; ++i) z(i, j) -= v[i] * s;
        }
        zc s = 0.0;
        for (int i = k; i < R; ++i) s += std::conj(v[i]) * f[i];
        s *= 2.0 / vn;
        for (int i = k; i < R; ++i) f[i] -= v[i] * s;
    }
    std::vector<zc> x(K);
    for (int k = K - 1; k >= 0; --k) {
        zc s = f[k];
        for (int j = k + 1; j < K; ++j) s -= z(k, j) * x[j];
        TDVP_REQUIRE(std::abs(z(k, k)) > 0.0, TDVP_E_NUMERIC, "exponential fit: rank-deficient Vandermonde matrix");
        x[k] = s / z(k, k);
    }
    return x;
}

double max_error(const std::vector<double>& f, const std::vector<zc>& c, const std::vector<zc>& lam) {
    double e = 0.0;
    for (size_t r = 0; r < f.size(); ++r) {
        zc s = 0.0;
        for (size_t k = 0; k < c.size(); ++k) s += c[k] * std::pow(lam[k], (double)(r + 1));
        e = std::max(e, std::fabs(s.real() - f[r]));
    }
    return e;
}

// Levenberg-Marquardt on (Re c, Im c, Re lam, Im lam) for the weighted
// residuals sqrt(w_r) (Re sum - f_r) and sqrt(w_r) Im sum, r = 1..R.
void lm_refine(const std::vector<double>& f, std::vector<zc>& c, std::vector<zc>& lam,
               const std::vector<double>& w, int iters) {
    const int R = (int)f.size(), K = (int)c.size(), P = 4 * K;
    auto residual = [&](const std::vector<zc>& cc, const std::vector<zc>& ll, std::vector<double>& res) {
        res.assign(2 * R, 0.0);
        for (int r = 0; r < R; ++r) {
            zc s = 0.0;
            for (int k = 0; k < K; ++k) s += cc[k] * std::pow(ll[k], (double)(r + 1));
            const double sw = std::sqrt(w[r]);
            res[r] = sw * (s.real() - f[r]);
            res[R + r] = sw * s.imag();
        }
    };
    std::vector<double> res, res2, J((size_t)2 * R * P);
    residual(c, lam, res);
    double cost = 0.0;
    for (double x : res) cost += x * x;
    double mu = 1e-3;
    for (int it = 0; it < iters; ++it) {
        for (int r = 0; r < R; ++r) {
            const double sw = std::sqrt(w[r]);
            for (int k = 0; k < K; ++k) {
                const zc p = std::pow(lam[k], (double)(r + 1));                       // d/dc
                const zc dp = c[k] * (double)(r + 1) * std::pow(lam[k], (double)r);   // d/dlam
                const zc cols[4] = {p, zc(0, 1) * p, dp, zc(0, 1) * dp};
                for (int q = 0; q < 4; ++q) {
                    J[(size_t)r * P + q * K + k] = sw * cols[q].real();
                    J[(size_t)(R + r) * P + q * K + k] = sw * cols[q].imag();
                }
            }
        }
        std::vector<double> A((size_t)P * P, 0.0), g(P, 0.0);
        for (int i = 0; i < 2 * R; ++i)
            for (int a = 0; a < P; ++a) {
                const double ja = J[(size_t)i * P + a];
                g[a] += ja * res[i];
                for (int b = 0; b < P; ++b) A[(size_t)a * P + b] += ja * J[(size_t)i * P + b];
            }
        std::vector<double> M = A;
        for (int a = 0; a < P; ++a) M[(size_t)a * P + a] += mu * (A[(size_t)a * P + a] + 1e-300);
        std::vector<double> step(P);
        for (int a = 0; a < P; ++a) step[a] = -g[a];
        solve(M, step, P, 1);
        std::vector<zc> c2(K), l2(K);
        bool decaying = true;
        for (int k = 0; k < K; ++k) {
            c2[k] = c[k] + zc(step[k], step[K + k]);
            l2[k] = lam[k] + zc(step[2 * K + k], step[3 * K + k]);
            decaying = decaying && std::abs(l2[k]) < 1.0;
        }
        if (!decaying) {  // keep every channel decaying
            mu *= 10.0;
            continue;
        }
        residual(c2, l2, res2);
        double cost2 = 0.0;
        for (double x : res2) cost2 += x * x;
        if (cost2 < cost) {
            const bool converged = cost - cost2 <= 1e-15 * cost;
            c = c2;
            lam = l2;
            res = res2;
            cost = cost2;
            mu = std::max(mu / 3.0, 1e-12);
            if (converged) break;
        } else {
            mu *= 10.0;
            if (mu > 1e12) break;
        }
    }
}

}  // namespace

double fit_exponentials(const std::vector<double>& f, int K, bool refine, std::vector<zc>& c, std::vector<zc>& lam) {
    const int R = (int)f.size();
    TDVP_REQUIRE(K >= 1 && R >= 2 * K, TDVP_E_ARG, "exponential fit: need K >= 1 and at least 2K samples");
    for (double v : f) TDVP_REQUIRE(std::isfinite(v), TDVP_E_NUMERIC, "exponential fit: non-finite sample");
    const int P = R / 2, rows = R - P, cols = P + 1;
    std::vector<double> Y((size_t)rows * cols);
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) Y[(size_t)i * cols + j] = f[i + j];
    std::vector<double> sv, Vt;
    jacobi_svd(Y, rows, cols, sv, Vt);
    // shift operator: top[:, 1:] = M top[:, :-1] in least squares,
    // M = top1 X^T (X X^T)^-1 with X = top[:, :-1]
    std::vector<double> G((size_t)K * K, 0.0), B((size_t)K * K, 0.0);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            double gx = 0.0, bx = 0.0;
            for (int j = 0; j < P; ++j) {
                gx += Vt[(size_t)a * cols + j] * Vt[(size_t)b * cols + j];
                bx += Vt[(size_t)a * cols + j + 1] * Vt[(size_t)b * cols + j];
            }
            G[(size_t)a * K + b] = gx;  // X X^T (symmetric)
            B[(size_t)a * K + b] = bx;  // top1 X^T
        }
    // M = B G^-1  <=>  G M^T = B^T (G symmetric)
    std::vector<double> MT((size_t)K * K);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) MT[(size_t)a * K + b] = B[(size_t)b * K + a];
    solve(G, MT, K, K);
    std::vector<zc> M((size_t)K * K);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) M[(size_t)a * K + b] = MT[(size_t)b * K + a];
    lam = eigenvalues(M, K);
    std::vector<zc> Z((size_t)R * K), fc(R);
    for (int r = 0; r < R; ++r) {
        fc[r] = f[r];
        for (int k = 0; k < K; ++k) Z[(size_t)r * K + k] = std::pow(lam[k], (double)(r + 1));
    }
    c = lstsq(Z, fc, R, K);
    double err = max_error(f, c, lam);
    if (refine) {
        std::vector<double> w(R, 1.0);
        std::vector<zc> c2 = c, l2 = lam;
        for (int pass = 0; pass < 30; ++pass) {
            lm_refine(f, c2, l2, w, 200);
            bool decaying = true;
            for (const zc& l : l2) decaying = decaying && std::abs(l) < 1.0;
            double e2 = 0.0;
            std::vector<double> res(R);
            for (int r = 0; r < R; ++r) {
                zc s = 0.0;
                for (int k = 0; k < K; ++k) s += c2[k] * std::pow(l2[k], (double)(r + 1));
                res[r] = std::fabs(s.real() - f[r]);
                e2 = std::max(e2, res[r]);
            }
            if (e2 < err && decaying) {
                c = c2;
                lam = l2;
                err = e2;
            }
            // Lawson: weights grow where the residual is large
            double tot = 0.0;
            for (int r = 0; r < R; ++r) {
                w[r] *= res[r] + 1e-3 * e2;
                tot += w[r];
            }
            for (int r = 0; r < R; ++r) w[r] *= R / tot;
        }
    }
    return err;
}

}  // namespace tdvp

using namespace tdvp;

extern "C" {

int tdvp_fit_exponentials(const double* f, int R, int K, int refine, double* c_out, double* lam_out,
                          double* max_abs_err) {
    if (!f || !c_out || !lam_out || R < 1) return TDVP_E_ARG;
    return guarded(nullptr, [&] {
        std::vector<double> fv(f, f + R);
        std::vector<zc> c, lam;
        const double err = fit_exponentials(fv, K, refine != 0, c, lam);
        for (int k = 0; k < K; ++k) {
            c_out[2 * k] = c[k].real();
            c_out[2 * k + 1] = c[k].imag();
            lam_out[2 * k] = lam[k].real();
            lam_out[2 * k + 1] = lam[k].imag();
        }
        if (max_abs_err) *max_abs_err = err;
    });
}

int tdvp_fit_power_law(double alpha, int K, int rmax, int refine, double* c_out, double* lam_out,
                       double* max_abs_err) {
    if (rmax < 1 || !std::isfinite(alpha)) return TDVP_E_ARG;
    std::vector<double> f(rmax);
    for (int r = 1; r <= rmax; ++r) f[r - 1] = std::pow((double)r, -alpha);
    return tdvp_fit_exponentials(f.data(), rmax, K, refine, c_out, lam_out, max_abs_err);
}

}  // extern "C"
