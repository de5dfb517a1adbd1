// One- and two-site TDVP time steps (Sec. II D, Sec. III A) and observables
// (Sec. IV) on the device.  The MPS is kept in mixed canonical form with the
// orthogonality centre on site 1 between steps; environments L_j (sites
// 1..j-1) and R_j (sites j+1..N) are cached on the MPS and updated one site
// at a time (Sec. III A).
#include "internal.hpp"
#include <algorithm>
#include <map>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <functional>
#include <thread>

using namespace tdvp;

bool tdvp::chi_saturated(const std::vector<int>& chi, int d, int chi_max) {
    const int N = (int)chi.size() - 1;
    for (int j = 1; j < N; ++j) {
        int64_t cap = 1;  // min(chi_max, d^min(j, N - j)) without overflow
        for (int e = 0; e < std::min(j, N - j) && cap < chi_max; ++e) cap *= d;
        if (chi[j] < std::min<int64_t>(cap, chi_max)) return false;
    }
    return true;
}

int tdvp::truncation_rank(const std::vector<double>& s, const TruncRule& r, double& w) {
    const int full = (int)s.size();
    std::vector<double> tail(full + 1, 0.0);
    for (int c = full - 1; c >= 0; --c) tail[c] = tail[c + 1] + s[c] * s[c];
    int chi_w = full;
    for (int c = 1; c <= full; ++c)
        if (tail[c] <= r.w_max) {
            chi_w = c;
            break;
        }
    int chi_eps = 0;
    for (int c = 0; c < full; ++c) chi_eps += (s[c] >= r.eps * s[0]);
    int chi = std::max(1, std::min(std::min(chi_w, r.chi_max), chi_eps));
    if (r.guard)
        while (chi > 1 && chi < full && s[chi] >= (1.0 - 1e-10) * s[chi - 1]) --chi;
    w = tail[chi];
    return chi;
}

// U(1) block-sparse contractions (u1.cpp); every tensor in precision dt,
// charge labels on the host
namespace tdvp {
void heff_u1(tdvp_ctx ctx, int nsite, Dt dt, int chil, int chir, int d, int wl, int wm, int wr, const int* ql,
             const int* qr, const int* qs, const int* cl, const int* cr, const void* L, const void* W1,
             const void* W2, const void* R, const void* x, void* y);
void env_u1(tdvp_ctx ctx, int dir, Dt dt, int chil, int chir, int d, int wl, int wr, const int* ql, const int* qr,
            const int* qs, const int* cl, const int* cr, const void* env, const void* A, const void* W, void* out);
}  // namespace tdvp

namespace {

// Worker lanes for the per-sector eigensolvers of the U(1) split.  The
// solver's divide and conquer is bound by its many small launches issued
// from the host, so sectors decomposed from several host threads, each with
// its own stream and rocBLAS handle, overlap on the GPU.  A lane owns only
// its stream, handle and solver workspace (hipMalloc: the lanes never call
// the context's allocator callback); the matrices, eigenvalues and codes it
// writes are slots of buffers the owning thread allocated.
struct SolverLane {
    tdvp_ctx_s c;
    hipEvent_t done = nullptr;
    ~SolverLane() {
        if (c.stream) (void)hipStreamSynchronize(c.stream);
        c.release_all();
        if (c.blas) rocblas_destroy_handle(c.blas);
        if (c.stream) (void)hipStreamDestroy(c.stream);
        if (done) (void)hipEventDestroy(done);
    }
};

struct SolverLanes {
    std::vector<std::unique_ptr<SolverLane>> lanes;
    hipEvent_t ready = nullptr;
    ~SolverLanes() {
        lanes.clear();
        if (ready) (void)hipEventDestroy(ready);
    }
};

int solver_lane_count() {
    const char* e = getenv("TDVP_U1_LANES");
    const int n = e ? atoi(e) : 4;
    return std::max(1, std::min(n, 16));
}

SolverLanes& solver_lanes(tdvp_ctx ctx, int n) {
    if (!ctx->solver_lanes) ctx->solver_lanes = std::make_shared<SolverLanes>();
    auto& P = *static_cast<SolverLanes*>(ctx->solver_lanes.get());
    if (!P.ready) TDVP_CHECK_HIP(hipEventCreateWithFlags(&P.ready, hipEventDisableTiming));
    while ((int)P.lanes.size() < n) {
        auto L = std::make_unique<SolverLane>();
        L->c.device = ctx->device;
        L->c.alloc_fn = nullptr;
        L->c.free_fn = nullptr;
        L->c.user = nullptr;
        TDVP_CHECK_HIP(hipStreamCreateWithFlags(&L->c.stream, hipStreamNonBlocking));
        TDVP_REQUIRE(rocblas_create_handle(&L->c.blas) == rocblas_status_success, TDVP_E_HIP,
                     "rocblas_create_handle failed");
        rocblas_set_stream(L->c.blas, L->c.stream);
        TDVP_CHECK_HIP(hipEventCreateWithFlags(&L->done, hipEventDisableTiming));
        P.lanes.push_back(std::move(L));
    }
    return P;
}

// Eigen-decompositions of the slots of G (orders n[b], leading dimension ld)
// after the work queued so far on the context stream; the context stream
// waits for all of them.  ev, E: ld doubles per slot; info: one int per slot.
// `meanwhile` runs on the calling thread while the lanes work (it may queue
// independent work on the context stream).
void heevd_on_lanes(tdvp_ctx ctx, double2* G, int ld, const std::vector<int>& n, double* ev, double* E, int* info,
                    const std::function<void()>& meanwhile) {
    const int count = (int)n.size();
    const int nl = std::min(solver_lane_count(), count);
    if (nl <= 1) {
        meanwhile();
        for (int b = 0; b < count; ++b)
            heevd_slot(ctx->blas, G + (size_t)b * ld * ld, ld, n[b], ev + (size_t)b * ld, E + (size_t)b * ld, info + b);
        return;
    }
    SolverLanes& P = solver_lanes(ctx, nl);
    SolverSizes ss;
    ss.eig_n = *std::max_element(n.begin(), n.end());
    for (int l = 0; l < nl; ++l) reserve_solver_workspace(&P.lanes[l]->c, ss);
    std::vector<int> order(count);
    for (int b = 0; b < count; ++b) order[b] = b;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });  // largest first
    TDVP_CHECK_HIP(hipEventRecord(P.ready, ctx->stream));
    std::atomic<int> next{0};
    std::vector<std::exception_ptr> errs(nl);
    std::vector<std::thread> pool;
    for (int l = 0; l < nl; ++l) {
        pool.emplace_back([&, l] {
            try {
                SolverLane& L = *P.lanes[l];
                TDVP_CHECK_HIP(hipSetDevice(L.c.device));
                TDVP_CHECK_HIP(hipStreamWaitEvent(L.c.stream, P.ready, 0));
                for (int t = next++; t < count; t = next++) {
                    const int b = order[t];
                    heevd_slot(L.c.blas, G + (size_t)b * ld * ld, ld, n[b], ev + (size_t)b * ld, E + (size_t)b * ld,
                               info + b);
                }
                TDVP_CHECK_HIP(hipEventRecord(L.done, L.c.stream));
            } catch (...) {
                errs[l] = std::current_exception();
            }
        });
    }
    std::exception_ptr own;
    try {
        meanwhile();
    } catch (...) {
        own = std::current_exception();
    }
    for (auto& t : pool) t.join();
    for (int l = 0; l < nl; ++l)
        if (!errs[l]) TDVP_CHECK_HIP(hipStreamWaitEvent(ctx->stream, P.lanes[l]->done, 0));
    if (own) std::rethrow_exception(own);
    for (auto& e : errs)
        if (e) std::rethrow_exception(e);
}

struct Stepper {
    tdvp_ctx ctx;
    tdvp_mps m;
    tdvp_mpo W;
    const tdvp_opts& o;
    tdvp_stats& st;
    bool fp64;
    Dt edt;
    int form;
    // U(1) mode: the state and the MPO carry charge labels; matvecs and
    // environment updates visit only the charge-allowed blocks and the
    // two-site splits decompose every charge sector of the middle bond
    // separately (the labels of the new bond follow from the kept values)
    bool u1 = false;
    int64_t u1_min = 0;  // chi_left * chi_right from which U(1) mode uses the block kernels

    Stepper(tdvp_ctx c, tdvp_mps mp, tdvp_mpo w, const tdvp_opts& opts, tdvp_stats& stats)
        : ctx(c), m(mp), W(w), o(opts), st(stats) {
        const Dt cdt = to_dt(opts.compute);
        fp64 = cdt == Dt::C128;
        edt = cdt;
        form = opts.gemm_form == 0 ? (fp64 ? 4 : 3) : opts.gemm_form;
        TDVP_REQUIRE(form == 3 || form == 4, TDVP_E_ARG, "gemm_form must be 0, 3 or 4");
        TDVP_REQUIRE(opts.krylov_max >= 1, TDVP_E_ARG, "krylov_max must be >= 1");
        TDVP_REQUIRE(opts.chi_max >= 1, TDVP_E_ARG, "chi_max must be >= 1");
        TDVP_REQUIRE(opts.exp_method == 0 || opts.exp_method == 1, TDVP_E_ARG, "exp_method must be 0 or 1");
        TDVP_REQUIRE(opts.u1_block_min >= 0, TDVP_E_ARG, "u1_block_min must be >= 0");
        u1_min = opts.u1_block_min == 0 ? 256 * 256 : opts.u1_block_min;
        TDVP_REQUIRE(m->N == W->N && m->d == W->d, TDVP_E_SHAPE, "MPS and MPO sizes differ");
        for (int j = 0; j < m->N; ++j)
            TDVP_REQUIRE(m->chi[j] <= (int64_t)m->d * m->chi[j + 1] &&
                             m->chi[j + 1] <= (int64_t)m->d * m->chi[j],
                         TDVP_E_SHAPE, "MPS bond dimensions are not consistent");
        if (m->has_charges() && W->charge.empty()) m->clear_charges();  // a step without charges drops them
        u1 = m->has_charges() && !W->charge.empty();
        if (u1) {
            TDVP_REQUIRE((int)m->qphys.size() == m->d && (int)m->qbond.size() == m->N + 1, TDVP_E_STATE,
                         "U(1) labels do not match the state");
            for (int j = 0; j <= m->N; ++j)
                TDVP_REQUIRE((int)m->qbond[j].size() == m->chi[j] && (int)W->charge[j].size() == W->w[j],
                             TDVP_E_STATE, "U(1) labels do not match the bond dimensions");
        }
    }

    // --------------------------------------------------- U(1) contractions
    // y = H_eff x (complex128 vectors) for the local problem of HeffArgs a at
    // site j (two-site: sites j, j+1; zero-site: the bond after site j).
    void heff_u1_apply(const HeffArgs& a, int j, const double2* x, double2* y) {
        const int d = m->d;
        const int D = a.nsite == 0 ? 1 : (a.nsite == 1 ? d : d * d);
        const int64_t n = (int64_t)a.chil * D * a.chir;
        const int *ql, *qr, *cl, *cr;
        const void *W1 = nullptr, *W2 = nullptr;
        int wm = a.wl;
        if (a.nsite == 2) {
            ql = m->qbond[j].data(); qr = m->qbond[j + 2].data();
            cl = W->charge[j].data(); cr = W->charge[j + 2].data();
            W1 = W->W(j, edt); W2 = W->W(j + 1, edt); wm = W->w[j + 1];
        } else if (a.nsite == 1) {
            ql = m->qbond[j].data(); qr = m->qbond[j + 1].data();
            cl = W->charge[j].data(); cr = W->charge[j + 1].data();
            W1 = W->W(j, edt);
        } else {
            ql = qr = m->qbond[j + 1].data();
            cl = cr = W->charge[j + 1].data();
        }
        const int dd = a.nsite == 0 ? 1 : d;
        if (edt == Dt::C128) {
            heff_u1(ctx, a.nsite, edt, a.chil, a.chir, dd, a.wl, wm, a.wr, ql, qr, m->qphys.data(), cl, cr, a.L, W1, W2,
                    a.R, x, y);
            return;
        }
        void* xs = ctx->workspace("u1s_x", elem_bytes(edt) * (size_t)n);
        void* ys = ctx->workspace("u1s_y", elem_bytes(edt) * (size_t)n);
        convert(xs, edt, x, Dt::C128, n, ctx->stream);
        heff_u1(ctx, a.nsite, edt, a.chil, a.chir, dd, a.wl, wm, a.wr, ql, qr, m->qphys.data(), cl, cr, a.L, W1, W2,
                a.R, xs, ys);
        convert(y, Dt::C128, ys, edt, n, ctx->stream);
    }

    // environment update across site j (dir +1: L[j+1] from L[j], -1: R[j-1] from R[j])
    void env_u1_update(int dir, int j, const void* env_in, void* env_out) {
        const int chil = m->chi[j], chir = m->chi[j + 1];
        const void* Aj = m->A[j].ptr;
        if (edt != Dt::C128) {
            void* As = ctx->workspace("u1s_A", elem_bytes(edt) * m->tensor_elems(j));
            convert(As, edt, Aj, Dt::C128, (int64_t)m->tensor_elems(j), ctx->stream);
            Aj = As;
        }
        env_u1(ctx, dir, edt, chil, chir, m->d, W->w[j], W->w[j + 1], m->qbond[j].data(), m->qbond[j + 1].data(),
               m->qphys.data(), W->charge[j].data(), W->charge[j + 1].data(), env_in, Aj, W->W(j, edt), env_out);
    }

    // U(1) mode on a local problem of these bond dimensions: block kernels
    // from u1_min on; below it the dense kernels, which keep every entry
    // outside the blocks exactly zero (each is a sum of products with a zero
    // factor), so both give the same block structure
    bool blocks(int chil, int chir) const { return u1 && (int64_t)chil * chir >= u1_min; }

    MatVec matvec(const HeffArgs& a, int j) {
        if (blocks(a.chil, a.chir)) return [this, a, j](const double2* x, double2* y) { heff_u1_apply(a, j, x, y); };
        return [this, a](const double2* x, double2* y) { heff_apply(ctx, a, x, Dt::C128, y, Dt::C128); };
    }

    size_t esz() const { return elem_bytes(edt); }

    void env_buf(DevMem& b, size_t elems) {
        if (b.bytes < elems * esz()) b = DevMem(ctx, elems * esz());
    }

    void trivial_env(DevMem& b) {
        env_buf(b, 1);
        if (edt == Dt::C128) {
            const double2 one{1.0, 0.0};
            TDVP_CHECK_HIP(hipMemcpyAsync(b.ptr, &one, sizeof(one), hipMemcpyHostToDevice, ctx->stream));
        } else {
            const float2 one{1.0f, 0.0f};
            TDVP_CHECK_HIP(hipMemcpyAsync(b.ptr, &one, sizeof(one), hipMemcpyHostToDevice, ctx->stream));
        }
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    }

    EnvArgs env_args(int j, const Mop* mop) {
        return EnvArgs{m->chi[j], m->chi[j + 1], m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1],
                       m->A[j].ptr, m->A[j].ptr, Dt::C128, mop, fp64, form};
    }

    void update_left(int j) {  // L[j+1] from L[j], A[j], W[j]
        env_buf(m->L[j + 1], (size_t)W->w[j + 1] * m->chi[j + 1] * m->chi[j + 1]);
        if (blocks(m->chi[j], m->chi[j + 1])) {
            env_u1_update(1, j, m->L[j].ptr, m->L[j + 1].ptr);
            st.flops += env_flops(m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1]);
            return;
        }
        EnvArgs a = env_args(j, &W->mop(1, j, fp64));
        env_left(ctx, a, m->L[j].ptr, edt, m->L[j + 1].ptr, edt);
        st.flops += env_flops(m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1]);
    }

    void update_right(int j) {  // R[j-1] from R[j], A[j], W[j]
        env_buf(m->R[j - 1], (size_t)W->w[j] * m->chi[j] * m->chi[j]);
        if (blocks(m->chi[j], m->chi[j + 1])) {
            env_u1_update(-1, j, m->R[j].ptr, m->R[j - 1].ptr);
            st.flops += env_flops(m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1]);
            return;
        }
        EnvArgs a = env_args(j, &W->mop(3, j, fp64));
        env_right(ctx, a, m->R[j].ptr, edt, m->R[j - 1].ptr, edt);
        st.flops += env_flops(m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1]);
    }

    void ensure_envs() {
        if (m->env_valid && m->env_mpo == W && m->env_dt == edt) return;
        const int N = m->N;
        trivial_env(m->L[0]);
        trivial_env(m->R[N - 1]);
        for (int j = N - 1; j >= 1; --j) update_right(j);  // Sec. III A: right to left at the start
        m->env_mpo = W;
        m->env_dt = edt;
        m->env_valid = true;
    }

    // theta <- exp(-i tau H) theta for the local operator described by a.
    void evolve(const HeffArgs& a, int j, double2* theta, double tau) {
        TxRange tx("expm");
        const int D = a.nsite == 0 ? 1 : (a.nsite == 1 ? m->d : m->d * m->d);
        const int64_t n = (int64_t)a.chil * D * a.chir;
        const double f = heff_flops(a.nsite, a.chil, a.chir, m->d, a.wl, a.wr);
        MatVec op = matvec(a, j);
        KrylovInfo ki = o.exp_method == 1
                            ? expm_taylor(ctx, op, theta, n, tau, std::max(0x1p-53, o.krylov_tol), o.imaginary != 0)
                            : expm_krylov(ctx, op, theta, n, tau, o.krylov_max, o.krylov_tol, o.imaginary != 0);
        st.matvecs += ki.matvecs;
        st.flops += f * ki.matvecs;
        st.krylov_max_used = std::max(st.krylov_max_used, ki.k);
        if (!ki.converged) {
            st.flags |= 1;
            TDVP_REQUIRE(!o.strict, TDVP_E_NOCONV, "Krylov exponential did not converge within krylov_max");
        }
    }

    // theta <- lowest Ritz vector of the local operator (normalised); returns its Ritz value.
    double ground(const HeffArgs& a, int j, double2* theta) {
        const int D = a.nsite == 0 ? 1 : (a.nsite == 1 ? m->d : m->d * m->d);
        const int64_t n = (int64_t)a.chil * D * a.chir;
        const double f = heff_flops(a.nsite, a.chil, a.chir, m->d, a.wl, a.wr);
        MatVec op = matvec(a, j);
        double e = 0.0;
        KrylovInfo ki = ground_krylov(ctx, op, theta, n, o.krylov_max, o.krylov_tol, &e);
        st.matvecs += ki.matvecs;
        st.flops += f * ki.matvecs;
        st.krylov_max_used = std::max(st.krylov_max_used, ki.k);
        if (!ki.converged) {
            st.flags |= 1;
            TDVP_REQUIRE(!o.strict, TDVP_E_NOCONV, "Lanczos ground state did not converge within krylov_max");
        }
        return e;
    }

    HeffArgs h1(int j) {
        return HeffArgs{1, m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1], m->L[j].ptr, m->R[j].ptr,
                        edt, &W->mop(1, j, fp64), fp64, form};
    }
    HeffArgs h0(int j) {  // bond between sites j and j+1
        const int c = m->chi[j + 1];
        return HeffArgs{0, c, c, m->d, W->w[j + 1], W->w[j + 1], m->L[j + 1].ptr, m->R[j].ptr, edt,
                        &W->mop(0, j, fp64), fp64, form};
    }
    HeffArgs h2(int j) {
        return HeffArgs{2, m->chi[j], m->chi[j + 2], m->d, W->w[j], W->w[j + 2], m->L[j].ptr,
                        m->R[j + 1].ptr, edt, &W->mop(2, j, fp64), fp64, form};
    }

    double2* A(int j) { return m->A[j].as<double2>(); }

    // Site j <- the row-major matrix src [rows][cols] (leading dimension ld),
    // rows * cols = chil * d * chir.
    void store_site(int j, const double2* src, int chil, int chir, int rows, int cols, int64_t ld) {
        m->set_tensor_dev(j, chil, chir);
        copy2d(A(j), cols, src, ld, rows, cols, 0, ctx->stream);
    }

    // ------------------------------------------------------------- 1TDVP
    void step1(double dt) {
        TxRange tx("tdvp1_step");
        // the gauge moves of the one-site step are dense QR / LQ, which mix
        // charge sectors (a column's pivot row may carry another charge)
        TDVP_REQUIRE(!u1, TDVP_E_ARG, "one-site steps do not run in U(1) mode: clear the state's charge labels first");
        const int N = m->N, d = m->d;
        const double tau = dt / 2.0;
        ensure_envs();
        for (int j = 0; j + 1 < N; ++j) {
            evolve(h1(j), j, A(j), tau);
            const int rows = m->chi[j] * d, cols = m->chi[j + 1];
            double2* Q = static_cast<double2*>(ctx->workspace("t1_Q", sizeof(double2) * (size_t)rows * cols));
            double2* C = static_cast<double2*>(ctx->workspace("t1_C", sizeof(double2) * (size_t)cols * cols));
            qr_rowmajor(ctx, A(j), rows, cols, Q, C);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j), Q, sizeof(double2) * (size_t)rows * cols,
                                          hipMemcpyDeviceToDevice, ctx->stream));
            update_left(j);
            evolve(h0(j), j, C, -tau);
            const int n2 = d * m->chi[j + 2];
            double2* T = static_cast<double2*>(ctx->workspace("t1_T", sizeof(double2) * (size_t)cols * n2));
            zgemm_rowmajor(ctx, C, A(j + 1), T, cols, cols, n2);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j + 1), T, sizeof(double2) * (size_t)cols * n2,
                                          hipMemcpyDeviceToDevice, ctx->stream));
        }
        evolve(h1(N - 1), N - 1, A(N - 1), dt);  // merged turning point
        for (int j = N - 1; j >= 1; --j) {
            const int rows = m->chi[j], cols = d * m->chi[j + 1];
            double2* Lf = static_cast<double2*>(ctx->workspace("t1_C", sizeof(double2) * (size_t)rows * rows));
            double2* Q = static_cast<double2*>(ctx->workspace("t1_Q", sizeof(double2) * (size_t)rows * cols));
            lq_rowmajor(ctx, A(j), rows, cols, Lf, Q);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j), Q, sizeof(double2) * (size_t)rows * cols,
                                          hipMemcpyDeviceToDevice, ctx->stream));
            update_right(j);
            evolve(h0(j - 1), j - 1, Lf, -tau);
            const int m1 = m->chi[j - 1] * d;
            double2* T = static_cast<double2*>(ctx->workspace("t1_T", sizeof(double2) * (size_t)m1 * rows));
            zgemm_rowmajor(ctx, A(j - 1), Lf, T, m1, rows, rows);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j - 1), T, sizeof(double2) * (size_t)m1 * rows,
                                          hipMemcpyDeviceToDevice, ctx->stream));
            evolve(h1(j - 1), j - 1, A(j - 1), tau);
        }
    }

    // ------------------------------------------------------------- 2TDVP
    int trunc_rank(const std::vector<double>& s, double& w) {
        return truncation_rank(s, TruncRule{o.chi_max, o.w_max, o.eps_rel, o.multiplet_guard != 0}, w);
    }

    double2* form_theta(int j) {
        const int d = m->d;
        const int rows = m->chi[j] * d, mid = m->chi[j + 1], cols = d * m->chi[j + 2];
        double2* th = static_cast<double2*>(ctx->workspace("t2_theta", sizeof(double2) * (size_t)rows * cols));
        zgemm_rowmajor(ctx, A(j), A(j + 1), th, rows, mid, cols);
        return th;
    }

    // U(1) split of theta into sites j, j+1: rows (a, s1) carry q(a) + q(s1),
    // columns (s2, b) carry q(b) - q(s2), and theta connects only equal
    // charges (the charge of the new bond index).  Every charge sector is
    // decomposed on its own; the singular values of all sectors are
    // truncated together by the rule of the dense split (Eq. discweight), and
    // the kept ones, ordered by charge (then by position in the sector),
    // label the new bond.  Sectors go the way the dense split goes: with the
    // density-matrix rule every sector is decomposed through the eigenvectors
    // of its reduced density matrix (orders <= kJacobiMaxOrder by the
    // one-workgroup Jacobi, larger ones by the solver's divide and conquer,
    // spread over worker lanes), sigma taken as the norm of the projection;
    // all of it is queued and read back once.  Otherwise each sector takes an SVD.
    // Uall [rows][ktot] and Vall [ktot][cols] collect every sector's factors
    // with the singular values already on the side that keeps them (site
    // j + 1 unless centre_left).
    void split_u1(int j, double2* th, bool centre_left) {
        TxRange tx("split_u1");
        const int d = m->d, chil = m->chi[j], chir = m->chi[j + 2];
        const int rows = chil * d, cols = d * chir;
        const std::vector<int>& qa = m->qbond[j];
        const std::vector<int>& qb = m->qbond[j + 2];
        const std::vector<int>& qs = m->qphys;
        const bool gram = o.svd_mode == 2 || (o.svd_mode == 0 && o.w_max >= 1e-13);
        const bool left = !centre_left;  // the side that becomes orthonormal
        std::map<int, std::vector<int>> rsec, csec;
        for (int a = 0; a < chil; ++a)
            for (int s1 = 0; s1 < d; ++s1) rsec[qa[a] + qs[s1]].push_back(a * d + s1);
        for (int s2 = 0; s2 < d; ++s2)
            for (int b = 0; b < chir; ++b) csec[qb[b] - qs[s2]].push_back(s2 * chir + b);
        enum Path { JACOBI, SOLVER, SVD };
        struct Sec {
            int Q;
            const std::vector<int>* r;
            const std::vector<int>* c;
            int k, off;
            Path path;
            int slot;        // SOLVER: slot in the solver's buffer
            int64_t ri, ci;  // offsets of the index lists in the device table
            int64_t blk, G, vecs, P, T;  // arena offsets (complex elements), density-matrix paths
            std::vector<double> s;
        };
        std::vector<Sec> secs;
        std::vector<int> idx;  // row lists, then column lists
        int ktot = 0, nb = 0, nmax = 0;
        int64_t arena = 0;
        for (const auto& kv : rsec) {
            auto it = csec.find(kv.first);
            if (it == csec.end()) continue;
            const int nr = (int)kv.second.size(), nc = (int)it->second.size();
            Sec sc{kv.first, &kv.second, &it->second, 0, ktot, SVD, -1, 0, 0, 0, 0, 0, 0, 0, {}};
            const int n = left ? nr : nc;
            if (gram) {
                sc.path = n <= kJacobiMaxOrder ? JACOBI : SOLVER;
                sc.k = n;
                const int len = left ? nc : nr;
                sc.blk = arena; arena += (int64_t)nr * nc;
                if (sc.path == JACOBI) {
                    sc.G = arena;
                    arena += (int64_t)n * n;
                } else {
                    sc.slot = nb++;
                    nmax = std::max(nmax, n);
                }
                sc.vecs = arena; arena += (int64_t)n * n;
                sc.P = arena; arena += (int64_t)n * len;
                sc.T = arena; arena += left ? (int64_t)nr * n : 0;
            } else {
                sc.k = std::min(nr, nc);
            }
            sc.ri = (int64_t)idx.size();
            idx.insert(idx.end(), kv.second.begin(), kv.second.end());
            sc.ci = (int64_t)idx.size();
            idx.insert(idx.end(), it->second.begin(), it->second.end());
            ktot += sc.k;
            secs.push_back(sc);
        }
        TDVP_REQUIRE(ktot > 0, TDVP_E_NUMERIC, "U(1) split: no charge sector connects the two sites");
        const int64_t nidx = (int64_t)idx.size();
        int* didx = static_cast<int*>(ctx->workspace("u1s_idx", sizeof(int) * (size_t)(nidx + ktot)));
        double2* Uall = static_cast<double2*>(ctx->workspace("u1s_Uall", sizeof(double2) * (size_t)rows * ktot));
        double2* Vall = static_cast<double2*>(ctx->workspace("u1s_Vall", sizeof(double2) * (size_t)ktot * cols));
        double2* ar = static_cast<double2*>(ctx->workspace("u1s_arena", sizeof(double2) * (size_t)std::max<int64_t>(1, arena)));
        double* s2 = static_cast<double*>(ctx->workspace("u1s_s2", sizeof(double) * (size_t)ktot));
        const int64_t slot_elems = (int64_t)nmax * nmax;
        double2* Gb = nb ? static_cast<double2*>(ctx->workspace("u1s_geig", sizeof(double2) * (size_t)(nb * slot_elems)))
                         : nullptr;
        TDVP_CHECK_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int) * nidx, hipMemcpyHostToDevice, ctx->stream));
        TDVP_CHECK_HIP(hipMemsetAsync(Uall, 0, sizeof(double2) * (size_t)rows * ktot, ctx->stream));
        TDVP_CHECK_HIP(hipMemsetAsync(Vall, 0, sizeof(double2) * (size_t)ktot * cols, ctx->stream));
        auto operand = [](const double2* p, int64_t ld, bool kcontig, bool conj) {
            GemmOperand g;
            g.p = p; g.dt = Dt::C128; g.ld = ld; g.kcontig = kcontig; g.conj = conj;
            return g;
        };
        // blocks and reduced density matrices (the small ones are decomposed
        // together in one launch below, while the solver lanes work)
        std::vector<JacobiProb> jprobs;
        for (auto& sc : secs) {
            const int nr = (int)sc.r->size(), nc = (int)sc.c->size();
            if (sc.path != SVD) {
                const int n = sc.k;
                double2* blk = ar + sc.blk;
                double2* G = sc.path == JACOBI ? ar + sc.G : Gb + sc.slot * slot_elems;
                copy_idx(blk, nc, nullptr, nullptr, th, cols, didx + sc.ri, didx + sc.ci, nr, nc, ctx->stream);
                GemmDesc g;
                g.M = n; g.N = n; g.cdt = Dt::C128; g.ldc = sc.path == JACOBI ? n : nmax; g.C = G;
                if (left) {  // G = B B^dag
                    g.K = nc; g.A = operand(blk, nc, true, false); g.B = operand(blk, nc, true, true);
                } else {     // G = B^dag B
                    g.K = nr; g.A = operand(blk, nc, false, true); g.B = operand(blk, nc, false, false);
                }
                cgemm(ctx, g, true, 4);
                if (sc.path == JACOBI)  // row c of the vectors = conj(eigenvector c)
                    jprobs.push_back(JacobiProb{G, s2 + sc.off, ar + sc.vecs, n, 0});
                continue;
            }
            double2* blk = static_cast<double2*>(ctx->workspace("u1s_blk", sizeof(double2) * (size_t)nr * nc));
            copy_idx(blk, nc, nullptr, nullptr, th, cols, didx + sc.ri, didx + sc.ci, nr, nc, ctx->stream);
            SvdResult r = svd_rowmajor(ctx, blk, nr, nc);
            TDVP_REQUIRE(r.k == sc.k, TDVP_E_STATE, "U(1) split: unexpected sector rank");
            if (centre_left) scale_cols(r.U, r.k, r.S_dev, nr, r.k, ctx->stream);
            else scale_rows(r.Vh, nc, r.S_dev, r.k, nc, ctx->stream);
            // U_Q into the sector's rows of Uall, Vh_Q into its columns of Vall
            copy_idx(Uall + sc.off, ktot, didx + sc.ri, nullptr, r.U, r.k, nullptr, nullptr, nr, sc.k, ctx->stream);
            copy_idx(Vall + (int64_t)sc.off * cols, cols, nullptr, didx + sc.ci, r.Vh, nc, nullptr, nullptr, sc.k, nc,
                     ctx->stream);
            sc.s = r.S;
        }
        // the larger ones by the solver; rows in ascending order, so the c-th
        // largest of a sector of order n is row n - 1 - c of its slot
        std::vector<int> orders;
        for (const auto& sc : secs)
            if (sc.path == SOLVER) orders.push_back(sc.k);
        const int* info = nullptr;
        if (nb) {
            double* ev = static_cast<double*>(ctx->workspace("heevds_ev", sizeof(double) * (size_t)nmax * nb));
            double* E = static_cast<double*>(ctx->workspace("heevds_E", sizeof(double) * (size_t)nmax * nb));
            int* dinfo = static_cast<int*>(ctx->workspace("heevds_info", sizeof(int) * (size_t)nb));
            heevd_on_lanes(ctx, Gb, nmax, orders, ev, E, dinfo, [&] { jacobi_eigh_batched(ctx, jprobs); });
            info = dinfo;
        } else {
            jacobi_eigh_batched(ctx, jprobs);
        }
        for (auto& sc : secs)
            if (sc.path == SOLVER)
                copy2d(ar + sc.vecs, sc.k, Gb + sc.slot * slot_elems + (int64_t)(sc.k - 1) * nmax, -(int64_t)nmax, sc.k,
                       sc.k, 0, ctx->stream);
        // the other side, U^dag B (left) or B V (right): its norms are the singular values
        for (auto& sc : secs) {
            if (sc.path == SVD) continue;
            const int nr = (int)sc.r->size(), nc = (int)sc.c->size();
            const int n = sc.k, len = left ? nc : nr;
            double2 *blk = ar + sc.blk, *V = ar + sc.vecs, *P = ar + sc.P;
            GemmDesc pg;
            pg.cdt = Dt::C128; pg.C = P;
            if (left) {
                pg.M = n; pg.N = nc; pg.K = nr; pg.ldc = nc;
                pg.A = operand(V, n, true, false); pg.B = operand(blk, nc, false, false);
            } else {
                pg.M = nr; pg.N = n; pg.K = nc; pg.ldc = n;
                pg.A = operand(blk, nc, true, false); pg.B = operand(V, n, true, true);
            }
            cgemm(ctx, pg, true, 4);
            vec_norms2(P, left ? nc : n, n, len, left, s2 + sc.off, ctx->stream);
            if (left) {
                double2* T = ar + sc.T;  // T[i][c] = u_c[i]
                conj_transpose(T, n, V, n, n, nr, ctx->stream);
                copy_idx(Uall + sc.off, ktot, didx + sc.ri, nullptr, T, n, nullptr, nullptr, nr, n, ctx->stream);
                copy_idx(Vall + (int64_t)sc.off * cols, cols, nullptr, didx + sc.ci, P, nc, nullptr, nullptr, n, nc,
                         ctx->stream);
            } else {
                copy_idx(Vall + (int64_t)sc.off * cols, cols, nullptr, didx + sc.ci, V, n, nullptr, nullptr, n, nc,
                         ctx->stream);
                copy_idx(Uall + sc.off, ktot, didx + sc.ri, nullptr, P, n, nullptr, nullptr, nr, n, ctx->stream);
            }
        }
        // the density-matrix sectors' squared singular values (and the solver's codes) in one read-back
        std::vector<double> hs2(ktot, 0.0);
        std::vector<int> hinfo(nb, 0);
        if (gram) {
            if (nb)
                ctx->read_back({{hs2.data(), s2, sizeof(double) * (size_t)ktot}, {hinfo.data(), info, sizeof(int) * (size_t)nb}});
            else
                ctx->read_back({{hs2.data(), s2, sizeof(double) * (size_t)ktot}});
        }
        for (int b = 0; b < nb; ++b)
            TDVP_REQUIRE(hinfo[b] == 0, TDVP_E_SOLVER, "U(1) split: zheevd did not converge (info = " +
                                                           std::to_string(hinfo[b]) + ")");
        for (auto& sc : secs) {
            if (sc.path == SVD) continue;
            sc.s.resize(sc.k);
            for (int c = 0; c < sc.k; ++c) {
                const double v = hs2[sc.off + c];
                TDVP_REQUIRE(std::isfinite(v), TDVP_E_NUMERIC, "U(1) split: non-finite singular value");
                sc.s[c] = std::sqrt(std::max(v, 0.0));
            }
        }
        // all singular values, largest first, for the truncation rule
        std::vector<std::pair<double, std::pair<int, int>>> all;  // (s, (sector, index))
        for (int q = 0; q < (int)secs.size(); ++q)
            for (int i = 0; i < secs[q].k; ++i) all.push_back({secs[q].s[i], {q, i}});
        std::stable_sort(all.begin(), all.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
        std::vector<double> sv(all.size());
        for (size_t i = 0; i < all.size(); ++i) sv[i] = all[i].first;
        double w = 0.0;
        const int chi = trunc_rank(sv, w);
        // kept values ordered by sector charge (sectors are in ascending charge), then by position
        std::vector<std::pair<int, int>> kept(chi);
        for (int c = 0; c < chi; ++c) kept[c] = all[c].second;
        std::stable_sort(kept.begin(), kept.end(), [](const auto& x, const auto& y) {
            return x.first != y.first ? x.first < y.first : x.second < y.second;
        });
        std::vector<int> src(chi), labels(chi);
        for (int c = 0; c < chi; ++c) {
            const Sec& sc = secs[kept[c].first];
            src[c] = sc.off + kept[c].second;
            labels[c] = sc.Q;
            const double v = sc.s[kept[c].second];
            TDVP_REQUIRE(v > 0.0 && std::isfinite(v), TDVP_E_NUMERIC, "U(1) split: a kept singular value is zero or not finite");
        }
        int* dsrc = didx + nidx;
        double2* U = static_cast<double2*>(ctx->workspace("u1s_U", sizeof(double2) * (size_t)rows * chi));
        double2* Vh = static_cast<double2*>(ctx->workspace("u1s_Vh", sizeof(double2) * (size_t)chi * cols));
        TDVP_CHECK_HIP(hipMemcpyAsync(dsrc, src.data(), sizeof(int) * chi, hipMemcpyHostToDevice, ctx->stream));
        copy_idx(U, chi, nullptr, nullptr, Uall, ktot, nullptr, dsrc, rows, chi, ctx->stream);
        copy_idx(Vh, cols, nullptr, nullptr, Vall, cols, dsrc, nullptr, chi, cols, ctx->stream);
        store_site(j, U, m->chi[j], chi, rows, chi, chi);
        store_site(j + 1, Vh, chi, m->chi[j + 2], chi, cols, cols);
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));  // the host index list above goes out of scope
        st.w_step += w;
        m->chi[j + 1] = chi;
        m->qbond[j + 1] = labels;
    }

    // Split of theta into sites j, j+1 (Fig. postupdate); centre_left puts the
    // singular values into site j, otherwise into site j+1.
    void split(int j, double2* th, bool centre_left) {
        if (u1) {
            split_u1(j, th, centre_left);
            return;
        }
        TxRange tx("split");
        const int d = m->d;
        const int rows = m->chi[j] * d, cols = d * m->chi[j + 2];
        const bool gram = o.svd_mode == 2 || (o.svd_mode == 0 && o.w_max >= 1e-13);
        double w = 0.0;
        int chi;
        if (!gram) {
            SvdResult r = svd_rowmajor(ctx, th, rows, cols);
            chi = trunc_rank(r.S, w);
            if (centre_left) scale_cols(r.U, r.k, r.S_dev, rows, chi, ctx->stream);
            else scale_rows(r.Vh, cols, r.S_dev, chi, cols, ctx->stream);
            store_site(j, r.U, m->chi[j], chi, rows, chi, r.k);
            store_site(j + 1, r.Vh, chi, m->chi[j + 2], chi, cols, cols);
        } else {
            // reduced density matrix of the side that becomes orthonormal
            GramResult g = gram_eigen(ctx, th, rows, cols, !centre_left);
            chi = trunc_rank(g.s, w);
            GemmDesc gd;
            gd.cdt = Dt::C128;
            if (!centre_left) {
                // A_L(j) = U_kept, A_C(j+1) = U_kept^dag theta
                m->set_tensor_dev(j, m->chi[j], chi);
                conj_transpose(A(j), chi, g.vecs, g.n, chi, rows, ctx->stream);
                m->set_tensor_dev(j + 1, chi, m->chi[j + 2]);
                gd.M = chi; gd.N = cols; gd.K = rows;
                gd.A.p = g.vecs; gd.A.dt = Dt::C128; gd.A.ld = g.n; gd.A.kcontig = true;
                gd.B.p = th; gd.B.dt = Dt::C128; gd.B.ld = cols; gd.B.kcontig = false;
                gd.C = A(j + 1); gd.ldc = cols;
            } else {
                // B(j+1) = V_kept^dag, A_C(j) = theta V_kept
                m->set_tensor_dev(j + 1, chi, m->chi[j + 2]);
                copy2d(A(j + 1), cols, g.vecs, g.n, chi, cols, 0, ctx->stream);
                m->set_tensor_dev(j, m->chi[j], chi);
                gd.M = rows; gd.N = chi; gd.K = cols;
                gd.A.p = th; gd.A.dt = Dt::C128; gd.A.ld = cols; gd.A.kcontig = true;
                gd.B.p = g.vecs; gd.B.dt = Dt::C128; gd.B.ld = g.n; gd.B.kcontig = true; gd.B.conj = true;
                gd.C = A(j); gd.ldc = chi;
            }
            cgemm(ctx, gd, true, 4);
        }
        st.w_step += w;
        m->chi[j + 1] = chi;
    }

    void step2(double dt) {
        TxRange tx("tdvp2_step");
        const int N = m->N;
        TDVP_REQUIRE(N >= 2, TDVP_E_SHAPE, "tdvp2_step needs at least two sites");
        const double tau = dt / 2.0;
        ensure_envs();
        for (int j = 0; j + 2 < N; ++j) {
            double2* th = form_theta(j);
            evolve(h2(j), j, th, tau);
            split(j, th, false);
            update_left(j);
            evolve(h1(j + 1), j + 1, A(j + 1), -tau);
        }
        {
            const int j = N - 2;
            double2* th = form_theta(j);
            evolve(h2(j), j, th, dt);  // right-most pair once by the full step
            split(j, th, true);
            update_right(j + 1);
        }
        for (int j = N - 3; j >= 0; --j) {
            evolve(h1(j + 1), j + 1, A(j + 1), -tau);
            double2* th = form_theta(j);
            evolve(h2(j), j, th, tau);
            split(j, th, true);
            update_right(j + 1);
        }
    }

    // ------------------------------------------------------- two-site DMRG
    // One sweep of two-site DMRG (left to right, then right to left, the
    // right-most pair once at the turn), with the same environments, effective
    // Hamiltonian and truncated splits as the two-site TDVP step (Sec. III A).
    // The state is renormalised at the end.  Returns the last Ritz value.
    double dmrg2() {
        const int N = m->N;
        TDVP_REQUIRE(N >= 2, TDVP_E_SHAPE, "dmrg2_sweep needs at least two sites");
        ensure_envs();
        double e = 0.0;
        for (int j = 0; j + 2 < N; ++j) {
            double2* th = form_theta(j);
            e = ground(h2(j), j, th);
            split(j, th, false);
            update_left(j);
        }
        {
            const int j = N - 2;
            double2* th = form_theta(j);
            e = ground(h2(j), j, th);
            split(j, th, true);
            update_right(j + 1);
        }
        for (int j = N - 3; j >= 0; --j) {
            double2* th = form_theta(j);
            e = ground(h2(j), j, th);
            split(j, th, true);
            update_right(j + 1);
        }
        normalize_centre();  // the centre carries the norm (1 - discarded weight of the last split)
        return e;
    }

    // Scales the centre tensor (site 0; sites 1.. are right-orthonormal) to unit norm.
    void normalize_centre() {
        const int64_t n0 = (int64_t)m->chi[0] * m->d * m->chi[1];
        double2* nn = static_cast<double2*>(ctx->workspace("centre_nn", sizeof(double2)));
        vdot_multi(ctx, A(0), 0, 1, A(0), n0, nn);
        double2 h{0.0, 0.0};
        TDVP_CHECK_HIP(hipMemcpyAsync(&h, nn, sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        TDVP_REQUIRE(std::isfinite(h.x) && h.x > 0.0, TDVP_E_NUMERIC, "renormalisation: the state vanished");
        scale_copy(A(0), A(0), 1.0 / std::sqrt(h.x), n0, ctx->stream);
    }

    void finish(double t0) {
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        st.chi_peak = 0;
        for (int c : m->chi) st.chi_peak = std::max(st.chi_peak, c);
        m->w_total += st.w_step;
        st.w_total = m->w_total;
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
    }
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------- observables

struct Transfer {
    tdvp_ctx ctx;
    int d;
    std::vector<double> host_id;
    DevMem Wdev;
    Mop mop_id;

    explicit Transfer(tdvp_ctx c, int dd) : ctx(c), d(dd) {}

    void make_op(Mop& mop, DevMem& store, const double* op_host, int kind) {
        store = DevMem(ctx, sizeof(double2) * d * d);
        TDVP_CHECK_HIP(hipMemcpyAsync(store.ptr, op_host, sizeof(double2) * d * d, hipMemcpyHostToDevice, ctx->stream));
        mop_make(ctx, mop, kind, store.ptr, nullptr, Dt::C128, 1, 1, 1, d, true, true);
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    }

    // E'[b'][b] = sum conj(Abra) E O Aket (left), w = 1
    void left(const void* E, const void* Abra, int chil_b, int chir_b, const void* Aket, int chil,
              int chir, const Mop& mop, void* out) {
        EnvArgs a{chil, chir, chil_b, chir_b, d, 1, 1, Abra, Aket, Dt::C128, &mop, true, 4};
        env_left(ctx, a, E, Dt::C128, out, Dt::C128);
    }
    void right(const void* E, const void* A, int chil, int chir, const Mop& mop, void* out) {
        EnvArgs a{chil, chir, chil, chir, d, 1, 1, A, A, Dt::C128, &mop, true, 4};
        env_right(ctx, a, E, Dt::C128, out, Dt::C128);
    }
};

std::vector<double> identity_host(int d) {
    std::vector<double> id((size_t)d * d * 2, 0.0);
    for (int s = 0; s < d; ++s) id[(s * d + s) * 2] = 1.0;
    return id;
}

void set_one(tdvp_ctx ctx, DevMem& b) {
    b = DevMem(ctx, sizeof(double2));
    const double2 one{1.0, 0.0};
    TDVP_CHECK_HIP(hipMemcpyAsync(b.ptr, &one, sizeof(one), hipMemcpyHostToDevice, ctx->stream));
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
}

double2 read1(tdvp_ctx ctx, const void* p) {
    double2 v;
    TDVP_CHECK_HIP(hipMemcpyAsync(&v, p, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    return v;
}

// All left transfers EL[0..N] and right transfers ER[0..N-1] (ER[j] covers j+1..N-1).
void all_transfers(tdvp_ctx ctx, tdvp_mps m, Transfer& tr, std::vector<DevMem>& EL, std::vector<DevMem>& ER) {
    const int N = m->N;
    EL.resize(N + 1);
    ER.resize(N);
    set_one(ctx, EL[0]);
    for (int j = 0; j < N; ++j) {
        EL[j + 1] = DevMem(ctx, sizeof(double2) * (size_t)m->chi[j + 1] * m->chi[j + 1]);
        tr.left(EL[j].ptr, m->A[j].ptr, m->chi[j], m->chi[j + 1], m->A[j].ptr, m->chi[j], m->chi[j + 1],
                tr.mop_id, EL[j + 1].ptr);
    }
    set_one(ctx, ER[N - 1]);
    for (int j = N - 1; j >= 1; --j) {
        ER[j - 1] = DevMem(ctx, sizeof(double2) * (size_t)m->chi[j] * m->chi[j]);
        tr.right(ER[j].ptr, m->A[j].ptr, m->chi[j], m->chi[j + 1], tr.mop_id, ER[j - 1].ptr);
    }
}

}  // namespace

extern "C" {

int tdvp1_step(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double dt, const tdvp_opts* opts, tdvp_stats* stats) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && mpo && opts, TDVP_E_ARG, "tdvp1_step: null argument");
        TDVP_REQUIRE(std::isfinite(dt), TDVP_E_ARG, "tdvp1_step: dt must be finite");
        tdvp_stats local{};
        tdvp_stats& st = stats ? *stats : local;
        st = tdvp_stats{};
        const double t0 = now_s();
        Stepper s(ctx, mps, mpo, *opts, st);
        try {
            s.step1(dt);
            if (opts->imaginary) s.normalize_centre();
        } catch (...) {
            mps->env_valid = false;
            throw;
        }
        s.finish(t0);
    });
}

int tdvp2_step(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double dt, const tdvp_opts* opts, tdvp_stats* stats) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && mpo && opts, TDVP_E_ARG, "tdvp2_step: null argument");
        TDVP_REQUIRE(std::isfinite(dt), TDVP_E_ARG, "tdvp2_step: dt must be finite");
        tdvp_stats local{};
        tdvp_stats& st = stats ? *stats : local;
        st = tdvp_stats{};
        const double t0 = now_s();
        Stepper s(ctx, mps, mpo, *opts, st);
        try {
            s.step2(dt);
            if (opts->imaginary) s.normalize_centre();
        } catch (...) {
            mps->env_valid = false;
            throw;
        }
        s.finish(t0);
    });
}

int tdvp_hybrid_step(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double dt, const tdvp_opts* opts,
                     tdvp_stats* stats, int* one_site) {
    if (!ctx) return TDVP_E_ARG;
    bool saturated = false;
    const int rc = guarded(ctx, [&] {
        TDVP_REQUIRE(mps && mpo && opts, TDVP_E_ARG, "tdvp_hybrid_step: null argument");
        TDVP_REQUIRE(opts->chi_max >= 1, TDVP_E_ARG, "chi_max must be >= 1");
        saturated = chi_saturated(mps->chi, mps->d, opts->chi_max);
    });
    if (rc != TDVP_OK) return rc;
    if (one_site) *one_site = saturated ? 1 : 0;
    return saturated ? tdvp1_step(ctx, mps, mpo, dt, opts, stats) : tdvp2_step(ctx, mps, mpo, dt, opts, stats);
}

int dmrg2_sweep(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, const tdvp_opts* opts, tdvp_stats* stats,
                double* energy) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && mpo && opts, TDVP_E_ARG, "dmrg2_sweep: null argument");
        tdvp_stats local{};
        tdvp_stats& st = stats ? *stats : local;
        st = tdvp_stats{};
        const double t0 = now_s();
        Stepper s(ctx, mps, mpo, *opts, st);
        double e = 0.0;
        try {
            e = s.dmrg2();
        } catch (...) {
            mps->env_valid = false;
            throw;
        }
        s.finish(t0);
        if (energy) *energy = e;
    });
}

int norm2(tdvp_ctx ctx, tdvp_mps mps, double* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && out, TDVP_E_ARG, "norm2: null argument");
        Transfer tr(ctx, mps->d);
        DevMem idd;
        tr.make_op(tr.mop_id, idd, identity_host(mps->d).data(), 1);
        DevMem E, E2;
        set_one(ctx, E);
        for (int j = 0; j < mps->N; ++j) {
            E2 = DevMem(ctx, sizeof(double2) * (size_t)mps->chi[j + 1] * mps->chi[j + 1]);
            tr.left(E.ptr, mps->A[j].ptr, mps->chi[j], mps->chi[j + 1], mps->A[j].ptr, mps->chi[j],
                    mps->chi[j + 1], tr.mop_id, E2.ptr);
            std::swap(E, E2);
        }
        *out = read1(ctx, E.ptr).x;
    });
}

int overlap(tdvp_ctx ctx, tdvp_mps bra, tdvp_mps ket, double* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(bra && ket && out, TDVP_E_ARG, "overlap: null argument");
        TDVP_REQUIRE(bra->N == ket->N && bra->d == ket->d, TDVP_E_SHAPE, "overlap: sizes differ");
        Transfer tr(ctx, ket->d);
        DevMem idd;
        tr.make_op(tr.mop_id, idd, identity_host(ket->d).data(), 1);
        DevMem E, E2;
        set_one(ctx, E);
        for (int j = 0; j < ket->N; ++j) {
            E2 = DevMem(ctx, sizeof(double2) * (size_t)bra->chi[j + 1] * ket->chi[j + 1]);
            tr.left(E.ptr, bra->A[j].ptr, bra->chi[j], bra->chi[j + 1], ket->A[j].ptr, ket->chi[j],
                    ket->chi[j + 1], tr.mop_id, E2.ptr);
            std::swap(E, E2);
        }
        const double2 v = read1(ctx, E.ptr);
        out[0] = v.x;
        out[1] = v.y;
    });
}

int energy(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && mpo && out, TDVP_E_ARG, "energy: null argument");
        TDVP_REQUIRE(mps->N == mpo->N && mps->d == mpo->d, TDVP_E_SHAPE, "energy: sizes differ");
        DevMem E, E2;
        set_one(ctx, E);
        for (int j = 0; j < mps->N; ++j) {
            E2 = DevMem(ctx, sizeof(double2) * (size_t)mpo->w[j + 1] * mps->chi[j + 1] * mps->chi[j + 1]);
            EnvArgs a{mps->chi[j], mps->chi[j + 1], mps->chi[j], mps->chi[j + 1], mps->d, mpo->w[j],
                      mpo->w[j + 1], mps->A[j].ptr, mps->A[j].ptr, Dt::C128, &mpo->mop(1, j, true), true, 4};
            env_left(ctx, a, E.ptr, Dt::C128, E2.ptr, Dt::C128);
            std::swap(E, E2);
        }
        const double2 e = read1(ctx, E.ptr);
        double n2 = 0.0;
        int rc = norm2(ctx, mps, &n2);
        TDVP_REQUIRE(rc == TDVP_OK, rc, ctx->err);
        TDVP_REQUIRE(n2 > 0.0, TDVP_E_NUMERIC, "energy: zero norm");
        out[0] = e.x / n2;
        out[1] = e.y / n2;
    });
}

int expect(tdvp_ctx ctx, tdvp_mps mps, int n, const int* sites, const double* ops, double* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && n >= 0 && (n == 0 || (sites && ops && out)), TDVP_E_ARG, "expect: bad argument");
        const int d = mps->d;
        for (int i = 0; i < n; ++i)
            TDVP_REQUIRE(sites[i] >= 0 && sites[i] < mps->N, TDVP_E_ARG, "expect: site out of range");
        Transfer tr(ctx, d);
        DevMem idd;
        tr.make_op(tr.mop_id, idd, identity_host(d).data(), 1);
        std::vector<DevMem> EL, ER;
        all_transfers(ctx, mps, tr, EL, ER);
        const double n2 = read1(ctx, EL[mps->N].ptr).x;
        TDVP_REQUIRE(n2 > 0.0, TDVP_E_NUMERIC, "expect: zero norm");
        DevMem res(ctx, sizeof(double2));
        for (int i = 0; i < n; ++i) {
            const int j = sites[i];
            Mop mo;
            DevMem od;
            tr.make_op(mo, od, ops + (size_t)i * d * d * 2, 1);
            DevMem X(ctx, sizeof(double2) * (size_t)mps->chi[j + 1] * mps->chi[j + 1]);
            tr.left(EL[j].ptr, mps->A[j].ptr, mps->chi[j], mps->chi[j + 1], mps->A[j].ptr, mps->chi[j],
                    mps->chi[j + 1], mo, X.ptr);
            trace_xyT(ctx, X.as<double2>(), ER[j].as<double2>(), mps->chi[j + 1], res.as<double2>());
            const double2 v = read1(ctx, res.ptr);
            out[2 * i] = v.x / n2;
            out[2 * i + 1] = v.y / n2;
        }
    });
}

int mps_apply_site(tdvp_ctx ctx, tdvp_mps mps, int site, const double* op) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && op, TDVP_E_ARG, "mps_apply_site: null argument");
        TDVP_REQUIRE(site >= 0 && site < mps->N, TDVP_E_ARG, "mps_apply_site: site out of range");
        const int d = mps->d;
        double2* O = static_cast<double2*>(ctx->workspace("apply_site_op", sizeof(double2) * d * d));
        TDVP_CHECK_HIP(hipMemcpyAsync(O, op, sizeof(double2) * d * d, hipMemcpyHostToDevice, ctx->stream));
        apply_site(mps->A[site].as<double2>(), O, mps->chi[site], d, mps->chi[site + 1], ctx->stream);
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));  // op lives in caller memory
        mps->env_valid = false;
        mps->clear_charges();  // op need not conserve the charge
    });
}

int transition_expect(tdvp_ctx ctx, tdvp_mps bra, tdvp_mps ket, int n, const int* sites, const double* ops,
                      double* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(bra && ket && n >= 0 && (n == 0 || (sites && ops && out)), TDVP_E_ARG,
                     "transition_expect: bad argument");
        TDVP_REQUIRE(bra->N == ket->N && bra->d == ket->d, TDVP_E_SHAPE, "transition_expect: sizes differ");
        const int N = ket->N, d = ket->d;
        for (int i = 0; i < n; ++i)
            TDVP_REQUIRE(sites[i] >= 0 && sites[i] < N, TDVP_E_ARG, "transition_expect: site out of range");
        Transfer tr(ctx, d);
        DevMem idd;
        tr.make_op(tr.mop_id, idd, identity_host(d).data(), 1);
        // mixed transfers: EL[j] [chi_bra_j][chi_ket_j], ER[j] [chi_ket_{j+1}][chi_bra_{j+1}]
        std::vector<DevMem> EL(N + 1), ER(N);
        set_one(ctx, EL[0]);
        for (int j = 0; j < N; ++j) {
            EL[j + 1] = DevMem(ctx, sizeof(double2) * (size_t)bra->chi[j + 1] * ket->chi[j + 1]);
            tr.left(EL[j].ptr, bra->A[j].ptr, bra->chi[j], bra->chi[j + 1], ket->A[j].ptr, ket->chi[j],
                    ket->chi[j + 1], tr.mop_id, EL[j + 1].ptr);
        }
        set_one(ctx, ER[N - 1]);
        for (int j = N - 1; j >= 1; --j) {
            ER[j - 1] = DevMem(ctx, sizeof(double2) * (size_t)ket->chi[j] * bra->chi[j]);
            EnvArgs a{ket->chi[j], ket->chi[j + 1], bra->chi[j], bra->chi[j + 1], d, 1, 1,
                      bra->A[j].ptr, ket->A[j].ptr, Dt::C128, &tr.mop_id, true, 4};
            env_right(ctx, a, ER[j].ptr, Dt::C128, ER[j - 1].ptr, Dt::C128);
        }
        DevMem res(ctx, sizeof(double2));
        for (int i = 0; i < n; ++i) {
            const int j = sites[i];
            Mop mo;
            DevMem od;
            tr.make_op(mo, od, ops + (size_t)i * d * d * 2, 1);
            DevMem X(ctx, sizeof(double2) * (size_t)bra->chi[j + 1] * ket->chi[j + 1]);
            tr.left(EL[j].ptr, bra->A[j].ptr, bra->chi[j], bra->chi[j + 1], ket->A[j].ptr, ket->chi[j],
                    ket->chi[j + 1], mo, X.ptr);
            trace_xy(ctx, X.as<double2>(), ER[j].as<double2>(), bra->chi[j + 1], ket->chi[j + 1], res.as<double2>());
            const double2 v = read1(ctx, res.ptr);
            out[2 * i] = v.x;
            out[2 * i + 1] = v.y;
        }
    });
}

int expect2(tdvp_ctx ctx, tdvp_mps mps, int n, const int* ii, const int* jj, const double* Oi,
            const double* Oj, double* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(mps && n >= 0 && (n == 0 || (ii && jj && Oi && Oj && out)), TDVP_E_ARG,
                     "expect2: bad argument");
        const int d = mps->d, N = mps->N;
        Transfer tr(ctx, d);
        DevMem idd;
        tr.make_op(tr.mop_id, idd, identity_host(d).data(), 1);
        std::vector<DevMem> EL, ER;
        all_transfers(ctx, mps, tr, EL, ER);
        const double n2 = read1(ctx, EL[N].ptr).x;
        TDVP_REQUIRE(n2 > 0.0, TDVP_E_NUMERIC, "expect2: zero norm");
        DevMem res(ctx, sizeof(double2));
        for (int p = 0; p < n; ++p) {
            int a = ii[p], b = jj[p];
            TDVP_REQUIRE(a >= 0 && a < N && b >= 0 && b < N, TDVP_E_ARG, "expect2: site out of range");
            const double* oa = Oi + (size_t)p * d * d * 2;
            const double* ob = Oj + (size_t)p * d * d * 2;
            if (a > b) {
                std::swap(a, b);
                std::swap(oa, ob);
            }
            std::vector<double> prod;
            if (a == b) {  // product O_a O_b on one site
                prod.assign((size_t)d * d * 2, 0.0);
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c)
                        for (int q = 0; q < d; ++q) {
                            const double xr = oa[(r * d + q) * 2], xi = oa[(r * d + q) * 2 + 1];
                            const double yr = ob[(q * d + c) * 2], yi = ob[(q * d + c) * 2 + 1];
                            prod[(r * d + c) * 2] += xr * yr - xi * yi;
                            prod[(r * d + c) * 2 + 1] += xr * yi + xi * yr;
                        }
                oa = prod.data();
            }
            Mop ma, mb;
            DevMem da, db;
            tr.make_op(ma, da, oa, 1);
            tr.make_op(mb, db, ob, 1);
            DevMem X(ctx, sizeof(double2) * (size_t)mps->chi[a + 1] * mps->chi[a + 1]);
            tr.left(EL[a].ptr, mps->A[a].ptr, mps->chi[a], mps->chi[a + 1], mps->A[a].ptr, mps->chi[a],
                    mps->chi[a + 1], ma, X.ptr);
            for (int q = a + 1; q <= b && a != b; ++q) {
                DevMem Y(ctx, sizeof(double2) * (size_t)mps->chi[q + 1] * mps->chi[q + 1]);
                tr.left(X.ptr, mps->A[q].ptr, mps->chi[q], mps->chi[q + 1], mps->A[q].ptr, mps->chi[q],
                        mps->chi[q + 1], q == b ? mb : tr.mop_id, Y.ptr);
                TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
                X = std::move(Y);
            }
            trace_xyT(ctx, X.as<double2>(), ER[b].as<double2>(), mps->chi[b + 1], res.as<double2>());
            const double2 v = read1(ctx, res.ptr);
            out[2 * p] = v.x / n2;
            out[2 * p + 1] = v.y / n2;
        }
    });
}

}  // extern "C"
