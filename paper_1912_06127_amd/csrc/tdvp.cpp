// One- and two-site TDVP time steps (Sec. II D, Sec. III A) and observables
// (Sec. IV) on the device.  The MPS is kept in mixed canonical form with the
// orthogonality centre on site 1 between steps; environments L_j (sites
// 1..j-1) and R_j (sites j+1..N) are cached on the MPS and updated one site
// at a time (Sec. III A).
#include "internal.hpp"

#include <chrono>
#include <cmath>

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

namespace {

struct Stepper {
    tdvp_ctx ctx;
    tdvp_mps m;
    tdvp_mpo W;
    const tdvp_opts& o;
    tdvp_stats& st;
    bool fp64;
    Dt edt;
    int form;

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
        TDVP_REQUIRE(m->N == W->N && m->d == W->d, TDVP_E_SHAPE, "MPS and MPO sizes differ");
        for (int j = 0; j < m->N; ++j)
            TDVP_REQUIRE(m->chi[j] <= (int64_t)m->d * m->chi[j + 1] &&
                             m->chi[j + 1] <= (int64_t)m->d * m->chi[j],
                         TDVP_E_SHAPE, "MPS bond dimensions are not consistent");
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
        EnvArgs a = env_args(j, &W->mop(1, j, fp64));
        env_left(ctx, a, m->L[j].ptr, edt, m->L[j + 1].ptr, edt);
        st.flops += env_flops(m->chi[j], m->chi[j + 1], m->d, W->w[j], W->w[j + 1]);
    }

    void update_right(int j) {  // R[j-1] from R[j], A[j], W[j]
        env_buf(m->R[j - 1], (size_t)W->w[j] * m->chi[j] * m->chi[j]);
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
    void evolve(const HeffArgs& a, double2* theta, double tau) {
        TxRange tx("expm");
        const int D = a.nsite == 0 ? 1 : (a.nsite == 1 ? m->d : m->d * m->d);
        const int64_t n = (int64_t)a.chil * D * a.chir;
        const double f = heff_flops(a.nsite, a.chil, a.chir, m->d, a.wl, a.wr);
        MatVec op = [&](const double2* x, double2* y) { heff_apply(ctx, a, x, Dt::C128, y, Dt::C128); };
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
    double ground(const HeffArgs& a, double2* theta) {
        const int D = a.nsite == 0 ? 1 : (a.nsite == 1 ? m->d : m->d * m->d);
        const int64_t n = (int64_t)a.chil * D * a.chir;
        const double f = heff_flops(a.nsite, a.chil, a.chir, m->d, a.wl, a.wr);
        MatVec op = [&](const double2* x, double2* y) { heff_apply(ctx, a, x, Dt::C128, y, Dt::C128); };
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
        const int N = m->N, d = m->d;
        const double tau = dt / 2.0;
        ensure_envs();
        for (int j = 0; j + 1 < N; ++j) {
            evolve(h1(j), A(j), tau);
            const int rows = m->chi[j] * d, cols = m->chi[j + 1];
            double2* Q = static_cast<double2*>(ctx->workspace("t1_Q", sizeof(double2) * (size_t)rows * cols));
            double2* C = static_cast<double2*>(ctx->workspace("t1_C", sizeof(double2) * (size_t)cols * cols));
            qr_rowmajor(ctx, A(j), rows, cols, Q, C);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j), Q, sizeof(double2) * (size_t)rows * cols,
                                          hipMemcpyDeviceToDevice, ctx->stream));
            update_left(j);
            evolve(h0(j), C, -tau);
            const int n2 = d * m->chi[j + 2];
            double2* T = static_cast<double2*>(ctx->workspace("t1_T", sizeof(double2) * (size_t)cols * n2));
            zgemm_rowmajor(ctx, C, A(j + 1), T, cols, cols, n2);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j + 1), T, sizeof(double2) * (size_t)cols * n2,
                                          hipMemcpyDeviceToDevice, ctx->stream));
        }
        evolve(h1(N - 1), A(N - 1), dt);  // merged turning point
        for (int j = N - 1; j >= 1; --j) {
            const int rows = m->chi[j], cols = d * m->chi[j + 1];
            double2* Lf = static_cast<double2*>(ctx->workspace("t1_C", sizeof(double2) * (size_t)rows * rows));
            double2* Q = static_cast<double2*>(ctx->workspace("t1_Q", sizeof(double2) * (size_t)rows * cols));
            lq_rowmajor(ctx, A(j), rows, cols, Lf, Q);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j), Q, sizeof(double2) * (size_t)rows * cols,
                                          hipMemcpyDeviceToDevice, ctx->stream));
            update_right(j);
            evolve(h0(j - 1), Lf, -tau);
            const int m1 = m->chi[j - 1] * d;
            double2* T = static_cast<double2*>(ctx->workspace("t1_T", sizeof(double2) * (size_t)m1 * rows));
            zgemm_rowmajor(ctx, A(j - 1), Lf, T, m1, rows, rows);
            TDVP_CHECK_HIP(hipMemcpyAsync(A(j - 1), T, sizeof(double2) * (size_t)m1 * rows,
                                          hipMemcpyDeviceToDevice, ctx->stream));
            evolve(h1(j - 1), A(j - 1), tau);
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

    // Split of theta into sites j, j+1 (Fig. postupdate); centre_left puts the
    // singular values into site j, otherwise into site j+1.
    void split(int j, double2* th, bool centre_left) {
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
            evolve(h2(j), th, tau);
            split(j, th, false);
            update_left(j);
            evolve(h1(j + 1), A(j + 1), -tau);
        }
        {
            const int j = N - 2;
            double2* th = form_theta(j);
            evolve(h2(j), th, dt);  // right-most pair once by the full step
            split(j, th, true);
            update_right(j + 1);
        }
        for (int j = N - 3; j >= 0; --j) {
            evolve(h1(j + 1), A(j + 1), -tau);
            double2* th = form_theta(j);
            evolve(h2(j), th, tau);
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
            e = ground(h2(j), th);
            split(j, th, false);
            update_left(j);
        }
        {
            const int j = N - 2;
            double2* th = form_theta(j);
            e = ground(h2(j), th);
            split(j, th, true);
            update_right(j + 1);
        }
        for (int j = N - 3; j >= 0; --j) {
            double2* th = form_theta(j);
            e = ground(h2(j), th);
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
