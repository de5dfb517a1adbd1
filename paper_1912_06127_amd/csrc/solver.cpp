// Dense FP64 gauge moves on the device (rocSOLVER): QR / LQ for one-site TDVP
// and the thin SVD that re-splits two-site states (Sec. III A, Fig. postupdate).
//
// rocSOLVER is column-major.  A row-major matrix M [rows][cols] is the
// column-major matrix M^T [cols][rows] in the same memory, so a row-major QR
// is a column-major LQ and vice versa, and the SVD factors swap roles:
//   M^T = U' S V'^H  =>  M = (V'^H)^T S U'^T,
// i.e. the column-major V'^H buffer read row-major is U, and the
// column-major U' buffer read row-major is V^H.  No transposition kernel is
// needed.
#include "internal.hpp"

#include <rocsolver/rocsolver.h>

namespace tdvp {

namespace {

void check_rs(rocblas_status st, const char* what) {
    if (st != rocblas_status_success)
        throw Error(TDVP_E_SOLVER, std::string(what) + " failed: " + rocblas_status_to_string(st));
}

rocblas_double_complex* rz(double2* p) { return reinterpret_cast<rocblas_double_complex*>(p); }

}  // namespace

void qr_rowmajor(tdvp_ctx ctx, const double2* M, int rows, int cols, double2* Q, double2* R) {
    if (qr_small_fits(rows, cols)) {  // rows >= cols: Q [rows][cols], R [cols][cols]
        qr_small(M, rows, cols, false, Q, R, ctx->stream);
        return;
    }
    const int k = std::min(rows, cols);
    double2* work = static_cast<double2*>(ctx->workspace("qr_work", sizeof(double2) * (size_t)rows * cols));
    double2* tau = static_cast<double2*>(ctx->workspace("qr_tau", sizeof(double2) * (size_t)k));
    TDVP_CHECK_HIP(hipMemcpyAsync(work, M, sizeof(double2) * (size_t)rows * cols, hipMemcpyDeviceToDevice, ctx->stream));
    // column-major LQ of M^T (cols x rows, lda = cols)
    check_rs(rocsolver_zgelqf(ctx->blas, cols, rows, rz(work), cols, rz(tau)), "zgelqf");
    // R[c][i] = L^T: buffer rows c < k with row stride cols, keep i >= c
    copy2d(R, cols, work, cols, k, cols, 1, ctx->stream);
    check_rs(rocsolver_zunglq(ctx->blas, k, rows, k, rz(work), cols, rz(tau)), "zunglq");
    // Q[i][c] = work[i*cols + c], c < k
    copy2d(Q, k, work, cols, rows, k, 0, ctx->stream);
}

void lq_rowmajor(tdvp_ctx ctx, const double2* M, int rows, int cols, double2* L, double2* Q) {
    if (qr_small_fits(cols, rows)) {  // rows <= cols: L [rows][rows], Q [rows][cols]
        qr_small(M, cols, rows, true, Q, L, ctx->stream);
        return;
    }
    const int k = std::min(rows, cols);
    double2* work = static_cast<double2*>(ctx->workspace("qr_work", sizeof(double2) * (size_t)rows * cols));
    double2* tau = static_cast<double2*>(ctx->workspace("qr_tau", sizeof(double2) * (size_t)k));
    TDVP_CHECK_HIP(hipMemcpyAsync(work, M, sizeof(double2) * (size_t)rows * cols, hipMemcpyDeviceToDevice, ctx->stream));
    // column-major QR of M^T (cols x rows, lda = cols)
    check_rs(rocsolver_zgeqrf(ctx->blas, cols, rows, rz(work), cols, rz(tau)), "zgeqrf");
    // L[a][c] = work[a*cols + c] for c <= a, c < k
    copy2d(L, k, work, cols, rows, k, 2, ctx->stream);
    check_rs(rocsolver_zungqr(ctx->blas, cols, k, k, rz(work), cols, rz(tau)), "zungqr");
    // Q[c][j] = work[c*cols + j]
    copy2d(Q, cols, work, cols, k, cols, 0, ctx->stream);
}

SvdResult svd_rowmajor(tdvp_ctx ctx, const double2* M, int rows, int cols) {
    SvdResult r;
    const int k = std::min(rows, cols);
    r.k = k;
    double2* work = static_cast<double2*>(ctx->workspace("svd_work", sizeof(double2) * (size_t)rows * cols));
    double2* Ubuf = static_cast<double2*>(ctx->workspace("svd_U", sizeof(double2) * (size_t)cols * k));
    double2* Vbuf = static_cast<double2*>(ctx->workspace("svd_V", sizeof(double2) * (size_t)k * rows));
    double* S = static_cast<double*>(ctx->workspace("svd_S", sizeof(double) * (size_t)k));
    double* E = static_cast<double*>(ctx->workspace("svd_E", sizeof(double) * (size_t)std::max(k, 1)));
    int* dinfo = static_cast<int*>(ctx->workspace("svd_info", sizeof(int)));
    TDVP_CHECK_HIP(hipMemcpyAsync(work, M, sizeof(double2) * (size_t)rows * cols, hipMemcpyDeviceToDevice, ctx->stream));
    // one-sided Jacobi: an order of magnitude faster than the bidiagonal
    // QR iteration of zgesvd on this device, and relatively accurate for
    // small singular values
    double* resid = static_cast<double*>(ctx->workspace("svd_resid", sizeof(double)));
    int* sweeps = static_cast<int*>(ctx->workspace("svd_sweeps", sizeof(int)));
    (void)E;
    check_rs(rocsolver_zgesvdj(ctx->blas, rocblas_svect_singular, rocblas_svect_singular, cols, rows,
                               rz(work), cols, 0.0, resid, 100, sweeps, S, rz(Ubuf), cols, rz(Vbuf), k,
                               dinfo),
             "zgesvdj");
    int hinfo = 0;
    r.S.resize(k);
    ctx->read_back({{r.S.data(), S, sizeof(double) * k}, {&hinfo, dinfo, sizeof(int)}});
    TDVP_REQUIRE(hinfo == 0, TDVP_E_SOLVER, "zgesvdj did not converge (info = " + std::to_string(hinfo) + ")");
    for (double v : r.S) TDVP_REQUIRE(std::isfinite(v), TDVP_E_NUMERIC, "SVD: non-finite singular value");
    r.U = Vbuf;   // row-major [rows][k]
    r.Vh = Ubuf;  // row-major [k][cols]
    r.S_dev = S;
    return r;
}

}  // namespace tdvp

namespace tdvp {

// Density-matrix split (Sec. III C truncation on the eigenvalues of the
// reduced density matrix).  left = true: G = Theta Theta^dag, eigenvectors
// are the left singular vectors; left = false: G = Theta^dag Theta.  The
// eigenvalues lambda = sigma^2 have absolute accuracy ~ eps ||Theta||^2, so
// this path is used only when the truncation thresholds sit far above that.
GramResult gram_eigen(tdvp_ctx ctx, const double2* M, int rows, int cols, bool left) {
    GramResult r;
    const int n = left ? rows : cols;
    r.n = n;
    double2* G = static_cast<double2*>(ctx->workspace("gram_G", sizeof(double2) * (size_t)n * n));
    double* ev = static_cast<double*>(ctx->workspace("gram_ev", sizeof(double) * (size_t)n));
    double* E = static_cast<double*>(ctx->workspace("gram_E", sizeof(double) * (size_t)n));
    int* dinfo = static_cast<int*>(ctx->workspace("gram_info", sizeof(int)));
    GemmDesc g;
    g.M = n;
    g.N = n;
    g.cdt = Dt::C128;
    g.ldc = n;
    g.C = G;
    if (left) {  // G[m][p] = sum_k M[m][k] conj(M[p][k])
        g.K = cols;
        g.A.p = M; g.A.dt = Dt::C128; g.A.ld = cols; g.A.kcontig = true;
        g.B.p = M; g.B.dt = Dt::C128; g.B.ld = cols; g.B.kcontig = true; g.B.conj = true;
    } else {     // G[m][p] = sum_k conj(M[k][m]) M[k][p]
        g.K = rows;
        g.A.p = M; g.A.dt = Dt::C128; g.A.ld = cols; g.A.kcontig = false; g.A.conj = true;
        g.B.p = M; g.B.dt = Dt::C128; g.B.ld = cols; g.B.kcontig = false;
    }
    cgemm(ctx, g, true, 4);
    if (n <= kJacobiMaxOrder) {
        // small orders: one-workgroup Jacobi instead of the ~n-launch tridiagonalisation
        r.vecs = static_cast<double2*>(ctx->workspace("gram_vecs", sizeof(double2) * (size_t)n * n));
        jacobi_eigh_small(G, n, ev, r.vecs, nullptr, ctx->stream);
        // The Jacobi eigenvalues carry ~n times the rounding of a tridiagonal
        // solve (every rotation touches the diagonal).  sigma_c is taken instead
        // as the norm of the projection u_c^dag Theta (left) or Theta v_c
        // (right): absolute error ~eps ||Theta|| in sigma, not eps ||Theta||^2
        // in sigma^2, so the discarded weight near w_max is that of an SVD.
        const int len = left ? cols : rows;
        double2* P = static_cast<double2*>(ctx->workspace("gram_P", sizeof(double2) * (size_t)n * len));
        GemmDesc p;
        p.cdt = Dt::C128;
        p.C = P;
        if (left) {  // P[c][k] = sum_i conj(u_c[i]) M[i][k]
            p.M = n; p.N = cols; p.K = rows; p.ldc = cols;
            p.A.p = r.vecs; p.A.dt = Dt::C128; p.A.ld = n; p.A.kcontig = true;
            p.B.p = M; p.B.dt = Dt::C128; p.B.ld = cols; p.B.kcontig = false;
        } else {     // P[i][c] = sum_k M[i][k] v_c[k]
            p.M = rows; p.N = n; p.K = cols; p.ldc = n;
            p.A.p = M; p.A.dt = Dt::C128; p.A.ld = cols; p.A.kcontig = true;
            p.B.p = r.vecs; p.B.dt = Dt::C128; p.B.ld = n; p.B.kcontig = true; p.B.conj = true;
        }
        cgemm(ctx, p, true, 4);
        vec_norms2(P, left ? cols : n, n, len, left, ev, ctx->stream);
        std::vector<double> s2(n);
        ctx->read_back({{s2.data(), ev, sizeof(double) * n}});
        r.s.resize(n);
        for (int c = 0; c < n; ++c) {
            TDVP_REQUIRE(std::isfinite(s2[c]), TDVP_E_NUMERIC, "density-matrix split: non-finite singular value");
            r.s[c] = std::sqrt(s2[c]);
        }
        return r;
    }
    // row-major G is the column-major conj(G): its eigenvectors W give the
    // eigenvectors conj(W) of G with the same (ascending) eigenvalues
    check_rs(rocsolver_zheevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, rz(G), n, ev, E, dinfo),
             "zheevd");
    std::vector<double> lam(n);
    int hinfo = 0;
    ctx->read_back({{lam.data(), ev, sizeof(double) * n}, {&hinfo, dinfo, sizeof(int)}});
    TDVP_REQUIRE(hinfo == 0, TDVP_E_SOLVER, "zheevd did not converge (info = " + std::to_string(hinfo) + ")");
    r.s.resize(n);
    for (int c = 0; c < n; ++c) {
        const double l = lam[n - 1 - c];
        TDVP_REQUIRE(std::isfinite(l), TDVP_E_NUMERIC, "density-matrix split: non-finite eigenvalue");
        r.s[c] = l > 0.0 ? std::sqrt(l) : 0.0;
    }
    // rows of the buffer are conj(eigenvector); reversed so row c' is the
    // c'-th largest: E[c'][i] = buf[(n-1-c') n + i] = conj(u_c'[i])
    r.vecs = static_cast<double2*>(ctx->workspace("gram_vecs", sizeof(double2) * (size_t)n * n));
    copy2d(r.vecs, n, G + (size_t)(n - 1) * n, -(int64_t)n, n, n, 0, ctx->stream);
    return r;
}

void heevd_slot(rocblas_handle h, double2* G, int ld, int n, double* ev, double* E, int* info) {
    // row-major G is the column-major conj(G): the eigenvectors it returns in
    // columns are the conjugated eigenvectors of G, i.e. rows of the row-major view
    check_rs(rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, n, rz(G), ld, ev, E, info), "zheevd");
}

}  // namespace tdvp

namespace tdvp {

namespace {

// Device bytes rocSOLVER asks for when `call` runs in size-query mode (no
// computation, only the workspace request is recorded on the handle).
template <class F>
size_t query_size(rocblas_handle h, F call) {
    size_t sz = 0;
    check_rs(rocblas_start_device_memory_size_query(h), "rocblas_start_device_memory_size_query");
    const rocblas_status st = call();
    check_rs(rocblas_stop_device_memory_size_query(h, &sz), "rocblas_stop_device_memory_size_query");
    if (st != rocblas_status_success && st != rocblas_status_size_increased && st != rocblas_status_size_unchanged)
        check_rs(st, "device memory size query");
    return sz;
}

}  // namespace

void reserve_solver_workspace(tdvp_ctx ctx, const SolverSizes& s) {
    rocblas_handle h = ctx->blas;
    size_t need = 0;
    auto ws = [&](const char* name, size_t bytes) { return ctx->workspace(name, std::max<size_t>(bytes, 16)); };
    // the query runs on the same (real, correctly sized) buffers the calls use
    if (s.eig_n > kJacobiMaxOrder) {
        const int n = s.eig_n;
        auto* G = static_cast<double2*>(ws("gram_G", sizeof(double2) * (size_t)n * n));
        auto* ev = static_cast<double*>(ws("gram_ev", sizeof(double) * (size_t)n));
        auto* E = static_cast<double*>(ws("gram_E", sizeof(double) * (size_t)n));
        auto* info = static_cast<int*>(ws("gram_info", sizeof(int)));
        ws("gram_vecs", sizeof(double2) * (size_t)n * n);
        need = std::max(need, query_size(h, [&] {
            return rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, n, rz(G), n, ev, E, info);
        }));
    }
    if (s.svd_rows > 0 && s.svd_cols > 0) {
        const int rows = s.svd_rows, cols = s.svd_cols, k = std::min(rows, cols);
        auto* work = static_cast<double2*>(ws("svd_work", sizeof(double2) * (size_t)rows * cols));
        auto* U = static_cast<double2*>(ws("svd_U", sizeof(double2) * (size_t)cols * k));
        auto* V = static_cast<double2*>(ws("svd_V", sizeof(double2) * (size_t)k * rows));
        auto* S = static_cast<double*>(ws("svd_S", sizeof(double) * (size_t)k));
        ws("svd_E", sizeof(double) * (size_t)std::max(k, 1));
        auto* info = static_cast<int*>(ws("svd_info", sizeof(int)));
        auto* resid = static_cast<double*>(ws("svd_resid", sizeof(double)));
        auto* sweeps = static_cast<int*>(ws("svd_sweeps", sizeof(int)));
        need = std::max(need, query_size(h, [&] {
            return rocsolver_zgesvdj(h, rocblas_svect_singular, rocblas_svect_singular, cols, rows, rz(work), cols,
                                     0.0, resid, 100, sweeps, S, rz(U), cols, rz(V), k, info);
        }));
    }
    auto qr_like = [&](int rows, int cols, bool lq) {
        if (rows <= 0 || cols <= 0) return;
        const int k = std::min(rows, cols);
        auto* work = static_cast<double2*>(ws("qr_work", sizeof(double2) * (size_t)rows * cols));
        auto* tau = static_cast<double2*>(ws("qr_tau", sizeof(double2) * (size_t)k));
        if (!lq) {
            need = std::max(need, query_size(h, [&] { return rocsolver_zgelqf(h, cols, rows, rz(work), cols, rz(tau)); }));
            need = std::max(need, query_size(h, [&] { return rocsolver_zunglq(h, k, rows, k, rz(work), cols, rz(tau)); }));
        } else {
            need = std::max(need, query_size(h, [&] { return rocsolver_zgeqrf(h, cols, rows, rz(work), cols, rz(tau)); }));
            need = std::max(need, query_size(h, [&] { return rocsolver_zungqr(h, cols, k, k, rz(work), cols, rz(tau)); }));
        }
    };
    qr_like(s.qr_rows, s.qr_cols, false);
    qr_like(s.lq_rows, s.lq_cols, true);
    if (need == 0) return;
    tdvp::Buffer& cur = ctx->work["rocblas_ws"];
    if (cur.bytes >= need) return;
    // the handle must let go of the old block before the workspace map frees it
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    check_rs(rocblas_set_workspace(h, nullptr, 0), "rocblas_set_workspace");
    void* p = ctx->workspace("rocblas_ws", need);
    check_rs(rocblas_set_workspace(h, p, ctx->work["rocblas_ws"].bytes), "rocblas_set_workspace");
}

}  // namespace tdvp
