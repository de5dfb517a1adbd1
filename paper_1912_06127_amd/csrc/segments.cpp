// Segment-parallel two-site TDVP on one GPU (Sec. III B, Fig. partitioning),
// with the state in the inverse canonical gauge (Sec. II A).
//
// The paper gives each segment of the chain its own process.  Here the
// segments are instances of one batch on one device.  At every phase of the
// schedule all active segments perform the same kind of local update (a
// two-site forward step or a one-site backward step), so their Lanczos
// exponentiations run together: per Krylov iteration one grouped launch per
// GEMM stage and one per MPO stage serves every instance, and the vector
// work of all instances runs in single launches over packed vectors.  Splits
// and environment refreshes remain per instance.  With static shapes every
// phase has the same packed layout from step to step, so its batched
// exponentiation is captured once in a HIP graph and replayed.
//
// Schedule (the paper's step-by-step diagrams of the parallel step are not
// part of its text; this is the reading used throughout):
//  * first half: the two central segments sweep away from the centre,
//    neighbours alternate; second half: every direction reversed;
//  * every boundary (a bond between segments, and each chain end) owns a
//    boundary pair -- (b, b+1), (0, 1) or (N-2, N-1); it is "meeting" in a
//    half when the segment(s) next to it sweep toward it;
//  * first half: departing boundary pairs forward by dt/2 before the sweeps,
//    meeting pairs forward by dt after them (merged turning point, Sec.
//    III A); second half: meeting pairs forward by dt/2 after the sweeps;
//  * a segment sweeping right over sites ls..rs (its sites, without the
//    chain-end sites) does: backward step on ls, then for j = ls..rs-1 the
//    pair (j, j+1) forward by dt/2 and a backward step on j+1 (mirror image
//    sweeping left);
//  * after a boundary-pair update both environments across that bond are
//    rebuilt; environments of a departing boundary stay as last built (out
//    of date, Sec. III D).
#include "internal.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <functional>
#include <thread>

namespace tdvp {
namespace {

struct SOp {
    bool pair;
    int j;
    double tau;
    int refresh;        // pairs: 1 left environment, 2 right, 3 both; bonds: 1 sweeping right, 2 left
    bool bond = false;  // zero-site step on the bond (j, j+1) (one-site schedule)
};
using SPhase = std::vector<SOp>;

std::vector<int> seg_dirs(int p, bool first) {
    std::vector<int> dir(p);
    if (p == 1) {
        dir[0] = first ? 1 : -1;
        return dir;
    }
    const int h = p / 2;
    for (int s = 0; s < p; ++s) {
        const int dist = s < h ? h - 1 - s : s - h;
        const int away = s < h ? -1 : 1;
        dir[s] = (dist % 2 == 0) ? away : -away;
        if (!first) dir[s] = -dir[s];
    }
    return dir;
}

std::vector<SPhase> seg_schedule(const std::vector<int>& sizes, double dt, bool first) {
    const int p = (int)sizes.size();
    int N = 0;
    std::vector<int> lo(p), hi(p);
    for (int s = 0; s < p; ++s) {
        lo[s] = N;
        N += sizes[s];
        hi[s] = N - 1;
    }
    const std::vector<int> dir = seg_dirs(p, first);
    const double half = dt / 2.0;
    SPhase before, after;
    // left chain end
    if (dir[0] == -1) after.push_back({true, 0, first ? dt : half, 3});
    else if (first) before.push_back({true, 0, half, 3});
    for (int s = 0; s + 1 < p; ++s) {
        const bool meet = dir[s] == 1 && dir[s + 1] == -1;
        if (meet) after.push_back({true, hi[s], first ? dt : half, 3});
        else if (first) before.push_back({true, hi[s], half, 3});
    }
    if (dir[p - 1] == 1) after.push_back({true, N - 2, first ? dt : half, 3});
    else if (first) before.push_back({true, N - 2, half, 3});

    std::vector<SPhase> sweeps(p);
    size_t longest = 0;
    for (int s = 0; s < p; ++s) {
        const int ls = std::max(lo[s], 1), rs = std::min(hi[s], N - 2);
        SPhase& o = sweeps[s];
        if (dir[s] == 1) {
            o.push_back({false, ls, -half, 0});
            for (int j = ls; j < rs; ++j) {
                o.push_back({true, j, half, 1});
                o.push_back({false, j + 1, -half, 0});
            }
        } else {
            o.push_back({false, rs, -half, 0});
            for (int j = rs - 1; j >= ls; --j) {
                o.push_back({true, j, half, 2});
                o.push_back({false, j, -half, 0});
            }
        }
        longest = std::max(longest, o.size());
    }
    std::vector<SPhase> out;
    if (!before.empty()) out.push_back(before);
    for (size_t i = 0; i < longest; ++i) {
        SPhase ph;
        for (int s = 0; s < p; ++s)
            if (i < sweeps[s].size()) ph.push_back(sweeps[s][i]);
        out.push_back(ph);
    }
    if (!after.empty()) out.push_back(after);
    return out;
}

// One-site schedule (the parallel one-site TDVP proposed in the Discussion;
// the boundary rule is a reading): the two-site boundary pairs and their
// timing as above, one-site sweeps inside the segments.  A segment sweeping
// right over its own sites a..z (its sites without those of boundary pairs)
// does the bond from its left boundary site backward by dt/2, site a forward
// by dt/2, then bond j backward and site j+1 forward for j = a..z-1, then the
// bond into its right boundary pair backward (mirror image sweeping left).
// Per step every boundary pair and every other site go forward by dt and
// every other bond backward by dt; at p = 1 this is the serial one-site step.
std::vector<SPhase> seg_schedule1(const std::vector<int>& sizes, double dt, bool first) {
    const int p = (int)sizes.size();
    int N = 0;
    std::vector<int> lo(p), hi(p);
    for (int s = 0; s < p; ++s) {
        lo[s] = N;
        N += sizes[s];
        hi[s] = N - 1;
    }
    const std::vector<int> dir = seg_dirs(p, first);
    const double half = dt / 2.0;
    SPhase before, after;
    for (int s = 0; s + 1 < p; ++s) {
        const bool meet = dir[s] == 1 && dir[s + 1] == -1;
        if (meet) after.push_back({true, hi[s], first ? dt : half, 3});
        else if (first) before.push_back({true, hi[s], half, 3});
    }
    std::vector<SPhase> sweeps(p);
    size_t longest = 0;
    for (int s = 0; s < p; ++s) {
        const int a = lo[s] + (s > 0 ? 1 : 0), z = hi[s] - (s + 1 < p ? 1 : 0);
        SPhase& o = sweeps[s];
        if (dir[s] == 1) {
            if (s > 0) o.push_back({false, lo[s], -half, 1, true});
            o.push_back({false, a, half, 0});
            for (int j = a; j < z; ++j) {
                o.push_back({false, j, -half, 1, true});
                o.push_back({false, j + 1, half, 0});
            }
            if (s + 1 < p) o.push_back({false, z, -half, 1, true});
        } else {
            if (s + 1 < p) o.push_back({false, z, -half, 2, true});
            o.push_back({false, z, half, 0});
            for (int j = z - 1; j >= a; --j) {
                o.push_back({false, j, -half, 2, true});
                o.push_back({false, j, half, 0});
            }
            if (s > 0) o.push_back({false, lo[s], -half, 2, true});
        }
        longest = std::max(longest, o.size());
    }
    std::vector<SPhase> out;
    if (!before.empty()) out.push_back(before);
    for (size_t i = 0; i < longest; ++i) {
        SPhase ph;
        for (int s = 0; s < p; ++s)
            if (i < sweeps[s].size()) ph.push_back(sweeps[s][i]);
        out.push_back(ph);
    }
    if (!after.empty()) out.push_back(after);
    return out;
}

// Batched exponentiation of one phase: layout, grouped H_eff plans, pointer
// tables and (optionally) its captured graph.
struct PhasePlan {
    uint64_t gen = ~uint64_t(0);
    std::vector<const void*> sig;
    SegLayout L;
    GroupedGemm A, B;
    GroupedWStage W;
    DevMem ptrs;  // device table of per-instance state pointers (gather / scatter)
    double flops_per_matvec = 0.0;
    hipGraphExec_t graph = nullptr;
    ~PhasePlan() {
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};

}  // namespace
}  // namespace tdvp

using namespace tdvp;

// A split lane: its own stream, rocBLAS handle and workspaces, so that the
// per-segment splits of one phase run concurrently (each from its own host
// thread, as the dense solvers synchronise with the host).
struct SegLane {
    tdvp_ctx_s c;
    hipEvent_t done = nullptr;
    ~SegLane() {
        if (c.stream) (void)hipStreamSynchronize(c.stream);
        c.release_all();
        if (c.blas) rocblas_destroy_handle(c.blas);
        if (c.stream) (void)hipStreamDestroy(c.stream);
        if (done) (void)hipEventDestroy(done);
    }
};

struct tdvp_seg_s {
    tdvp_ctx ctx = nullptr;
    int N = 0, d = 0;
    std::vector<int> sizes;
    std::vector<int> chi, cap;       // [N+1]; cap: initial profile (static-shape limits)
    std::vector<DevMem> Psi;         // c128 [chi_j][d][chi_{j+1}]
    std::vector<DevMem> Vd;          // double [chi_{j+1}], bond j (between sites j and j+1)
    std::vector<std::vector<double>> Vh;
    Dt edt = Dt::C64;                // environments and matvecs
    std::vector<DevMem> beta, gamma; // beta[j] [w_j][chi_j][chi_j], gamma[j] [w_{j+1}][chi_{j+1}][chi_{j+1}]
    double w_total = 0.0;
    std::map<std::string, std::unique_ptr<PhasePlan>> plans;
    DevMem flag;                     // device int: non-finite value seen during a step
    bool mixed_gauge = false;        // one-site steps left unit V on inner bonds
    hipStream_t cap_stream = nullptr; // graphs are captured here (the context stream may be the null stream)
    std::vector<std::unique_ptr<SegLane>> lanes;
    hipEvent_t ready = nullptr;

    double2* psi(int j) { return Psi[j].as<double2>(); }
    size_t psi_elems(int j) const { return (size_t)chi[j] * d * chi[j + 1]; }
    ~tdvp_seg_s() {
        plans.clear();
        lanes.clear();
        if (ready) (void)hipEventDestroy(ready);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace tdvp {
namespace {

struct SegRun {
    tdvp_ctx ctx;
    tdvp_seg sg;
    tdvp_mpo W;
    const tdvp_seg_opts& o;
    tdvp_stats& st;
    bool fp64;
    int form;

    size_t esz() const { return elem_bytes(sg->edt); }

    // State buffers always belong to the state's own context (lanes come and
    // go) and are grow-only.  The context's allocator is called from the
    // context's own thread only: before a phase runs on the split lanes every
    // buffer its ops may write is sized there (presize_split / presize_bond),
    // so a lane thread that would have to grow one reports an error instead.
    void need(DevMem& b, size_t bytes) {
        if (b.bytes >= bytes) return;
        TDVP_REQUIRE(ctx == sg->ctx, TDVP_E_STATE,
                     "segment step: a state buffer would grow on a split lane (not sized beforehand)");
        b = DevMem(sg->ctx, bytes);
    }
    void env_buf(DevMem& b, size_t elems) { need(b, elems * esz()); }

    HeffArgs h1(int j) {
        return HeffArgs{1, sg->chi[j], sg->chi[j + 1], sg->d, W->w[j], W->w[j + 1], sg->beta[j].ptr,
                        sg->gamma[j].ptr, sg->edt, &W->mop(1, j, fp64), fp64, form};
    }
    HeffArgs h2(int j) {
        return HeffArgs{2, sg->chi[j], sg->chi[j + 2], sg->d, W->w[j], W->w[j + 2], sg->beta[j].ptr,
                        sg->gamma[j + 1].ptr, sg->edt, &W->mop(2, j, fp64), fp64, form};
    }

    HeffArgs h0(int j) {  // bond between sites j and j+1
        const int c = sg->chi[j + 1];
        return HeffArgs{0, c, c, sg->d, W->w[j + 1], W->w[j + 1], sg->beta[j + 1].ptr, sg->gamma[j].ptr, sg->edt,
                        &W->mop(0, j, fp64), fp64, form};
    }

    double2* ws(const char* name, size_t elems) {
        return static_cast<double2*>(ctx->workspace(name, sizeof(double2) * std::max<size_t>(1, elems)));
    }

    // Zero-site step on bond j of the one-site schedule (Eq. proj1site).
    // refresh 1 (sweeping right): Psi_j = Q R, the bond matrix is R (V_j
    // Psi_{j+1} is right orthonormal), beta_{j+1} from Q; refresh 2 (sweeping
    // left): Psi_{j+1} = L Q', the bond matrix is L (Psi_j V_j is left
    // orthonormal), gamma_j from Q'.  C <- exp(-i tau H_0) C is absorbed into
    // the next site, Psi_{j+1} = C V_j Psi_{j+1} (or Psi_j = Psi_j V_j C), the
    // isometry stays (Psi_j = Q or Psi_{j+1} = Q') and V_j = 1: inside a
    // segment the state keeps the mixed canonical form of the serial step, and
    // only the boundary pairs restore Schmidt values.
    void bond_step(int j, double tau, int refresh) {
        ProfScope prof(ctx, "seg_bond", 0.0, 0.0);
        const int d = sg->d, chil = sg->chi[j], c = sg->chi[j + 1], chir = sg->chi[j + 2];
        const int rows = chil * d, cols = d * chir;
        TDVP_REQUIRE(rows >= c && cols >= c, TDVP_E_SHAPE, "segment bond step: bond exceeds its rank bound");
        hipStream_t s = ctx->stream;
        double2* C = ws("seg_bC", (size_t)c * c);
        double2* Q = ws("seg_bQ", (size_t)(refresh == 1 ? rows : cols) * c);
        if (refresh == 1) {
            qr_rowmajor(ctx, sg->psi(j), rows, c, Q, C);
            refresh_left(j, Q, chil, c);
        } else {
            lq_rowmajor(ctx, sg->psi(j + 1), c, cols, C, Q);
            refresh_right(j + 1, Q, c, chir);
        }
        const HeffArgs h = h0(j);
        MatVec mv = [&](const double2* a, double2* b) { heff_apply(ctx, h, a, Dt::C128, b, Dt::C128); };
        KrylovInfo ki = expm_krylov(ctx, mv, C, (int64_t)c * c, tau, o.krylov_k, 0.0);
        st.matvecs += ki.matvecs;
        st.flops += heff_flops(0, c, c, d, h.wl, h.wr) * ki.matvecs;
        st.krylov_max_used = std::max(st.krylov_max_used, ki.k);
        if (refresh == 1) {
            double2* X = ws("seg_bX", (size_t)c * cols);
            copy2d(X, cols, sg->psi(j + 1), cols, c, cols, 0, s);
            scale_rows(X, cols, sg->Vd[j].as<double>(), c, cols, s);
            zgemm_rowmajor(ctx, C, X, sg->psi(j + 1), c, c, cols);  // C V_j Psi_{j+1}
            copy2d(sg->psi(j), c, Q, c, rows, c, 0, s);
        } else {
            double2* T = ws("seg_bT", (size_t)rows * c);
            copy2d(T, c, sg->psi(j), c, rows, c, 0, s);
            scale_cols(T, c, sg->Vd[j].as<double>(), rows, c, s);
            zgemm_rowmajor(ctx, T, C, sg->psi(j), rows, c, c);  // Psi_j V_j C
            copy2d(sg->psi(j + 1), cols, Q, cols, c, cols, 0, s);
        }
        std::vector<double> one(c, 1.0);
        sg->Vh[j] = one;
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->Vd[j].ptr, one.data(), sizeof(double) * c, hipMemcpyHostToDevice, s));
        TDVP_CHECK_HIP(hipStreamSynchronize(s));  // one goes out of scope
    }

    void refresh_left(int j, const double2* A, int chil, int chir) {  // beta[j+1] from beta[j], A_j
        env_buf(sg->beta[j + 1], (size_t)W->w[j + 1] * chir * chir);
        EnvArgs a{chil, chir, chil, chir, sg->d, W->w[j], W->w[j + 1], A, A, Dt::C128, &W->mop(1, j, fp64),
                  fp64, form};
        env_left(ctx, a, sg->beta[j].ptr, sg->edt, sg->beta[j + 1].ptr, sg->edt);
        st.flops += env_flops(chil, chir, sg->d, W->w[j], W->w[j + 1]);
    }
    void refresh_right(int j, const double2* B, int chil, int chir) {  // gamma[j-1] from gamma[j], B_j
        env_buf(sg->gamma[j - 1], (size_t)W->w[j] * chil * chil);
        EnvArgs a{chil, chir, chil, chir, sg->d, W->w[j], W->w[j + 1], B, B, Dt::C128, &W->mop(3, j, fp64),
                  fp64, form};
        env_right(ctx, a, sg->gamma[j].ptr, sg->edt, sg->gamma[j - 1].ptr, sg->edt);
        st.flops += env_flops(chil, chir, sg->d, W->w[j], W->w[j + 1]);
    }

    // Theta = Psi_j V_j Psi_{j+1} written to dst [chi_j d][d chi_{j+2}].
    void form_theta(int j, double2* dst) {
        ProfScope prof(ctx, "seg_theta", 0.0, 0.0);
        const int d = sg->d, rows = sg->chi[j] * d, mid = sg->chi[j + 1], cols = d * sg->chi[j + 2];
        double2* t = static_cast<double2*>(ctx->workspace("seg_scaled", sizeof(double2) * (size_t)rows * mid));
        copy2d(t, mid, sg->psi(j), mid, rows, mid, 0, ctx->stream);
        scale_cols(t, mid, sg->Vd[j].as<double>(), rows, mid, ctx->stream);
        zgemm_rowmajor(ctx, t, sg->psi(j + 1), dst, rows, mid, cols);
    }

    // Truncated split of theta [chi_j d][d chi_{j+2}] into Psi_j = U S,
    // V_j = 1/S, Psi_{j+1} = S Vh (Fig. postupdate) and the environment
    // refresh the op asks for.
    void split(int j, const double2* th, int refresh) {
        ProfScope prof(ctx, "seg_split", 0.0, 0.0);
        const int d = sg->d, chil = sg->chi[j], chir = sg->chi[j + 2];
        const int rows = chil * d, cols = d * chir;
        int cap = o.chi_max;
        if (o.static_shapes) cap = std::min(cap, sg->cap[j + 1]);
        const TruncRule rule{cap, o.w_max, o.eps_rel, o.multiplet_guard != 0};
        double w = 0.0;
        int chi = 0;
        std::vector<double> s;
        double2* U = nullptr;   // [rows][chi] left orthonormal
        double2* SV = nullptr;  // [chi][cols] = S Vh
        bool use_svd = o.svd_mode == 1;
        if (!use_svd) {
            const bool left = rows <= cols;
            GramResult g = gram_eigen(ctx, th, rows, cols, left);
            chi = truncation_rank(g.s, rule, w);
            // the density-matrix split resolves s only to ~1e-8 s_1; fall back
            // to the SVD when smaller singular values are kept
            if (o.svd_mode == 0 && g.s[chi - 1] < 1e-6 * g.s[0]) use_svd = true;
            else {
                s.assign(g.s.begin(), g.s.begin() + chi);
                U = static_cast<double2*>(ctx->workspace("seg_U", sizeof(double2) * (size_t)rows * chi));
                SV = static_cast<double2*>(ctx->workspace("seg_SV", sizeof(double2) * (size_t)chi * cols));
                GemmDesc gd;
                gd.cdt = Dt::C128;
                if (left) {  // U = conj(vecs[:chi])^T, S Vh = vecs[:chi] theta
                    conj_transpose(U, chi, g.vecs, g.n, chi, rows, ctx->stream);
                    gd.M = chi; gd.N = cols; gd.K = rows;
                    gd.A.p = g.vecs; gd.A.dt = Dt::C128; gd.A.ld = g.n; gd.A.kcontig = true;
                    gd.B.p = th; gd.B.dt = Dt::C128; gd.B.ld = cols; gd.B.kcontig = false;
                    gd.C = SV; gd.ldc = cols;
                    cgemm(ctx, gd, true, 4);
                } else {  // Vh = vecs[:chi], U S = theta Vh^dag
                    double2* US = static_cast<double2*>(ctx->workspace("seg_US", sizeof(double2) * (size_t)rows * chi));
                    gd.M = rows; gd.N = chi; gd.K = cols;
                    gd.A.p = th; gd.A.dt = Dt::C128; gd.A.ld = cols; gd.A.kcontig = true;
                    gd.B.p = g.vecs; gd.B.dt = Dt::C128; gd.B.ld = g.n; gd.B.kcontig = true; gd.B.conj = true;
                    gd.C = US; gd.ldc = chi;
                    cgemm(ctx, gd, true, 4);
                    copy2d(SV, cols, g.vecs, g.n, chi, cols, 0, ctx->stream);
                    upload_scale(s, false);
                    scale_rows(SV, cols, scal_dev(), chi, cols, ctx->stream);
                    upload_scale(s, true);
                    copy2d(U, chi, US, chi, rows, chi, 0, ctx->stream);
                    scale_cols(U, chi, scal_dev(), rows, chi, ctx->stream);
                }
            }
        }
        if (use_svd) {
            SvdResult r = svd_rowmajor(ctx, th, rows, cols);
            chi = truncation_rank(r.S, rule, w);
            s.assign(r.S.begin(), r.S.begin() + chi);
            U = static_cast<double2*>(ctx->workspace("seg_U", sizeof(double2) * (size_t)rows * chi));
            SV = static_cast<double2*>(ctx->workspace("seg_SV", sizeof(double2) * (size_t)chi * cols));
            copy2d(U, chi, r.U, r.k, rows, chi, 0, ctx->stream);
            copy2d(SV, cols, r.Vh, cols, chi, cols, 0, ctx->stream);
            scale_rows(SV, cols, r.S_dev, chi, cols, ctx->stream);
        }
        for (double v : s)
            TDVP_REQUIRE(v > 0.0 && std::isfinite(v), TDVP_E_NUMERIC,
                         "segment split: a kept singular value is zero or not finite");
        st.w_step += w;
        // Psi_j = U S, V_j = 1/S, Psi_{j+1} = S Vh
        set_bond(j, chi);
        upload_scale(s, false);
        copy2d(sg->psi(j), chi, U, chi, rows, chi, 0, ctx->stream);
        scale_cols(sg->psi(j), chi, scal_dev(), rows, chi, ctx->stream);
        copy2d(sg->psi(j + 1), cols, SV, cols, chi, cols, 0, ctx->stream);
        std::vector<double> inv(chi);
        for (int c = 0; c < chi; ++c) inv[c] = 1.0 / s[c];
        sg->Vh[j] = inv;
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->Vd[j].ptr, inv.data(), sizeof(double) * chi, hipMemcpyHostToDevice,
                                      ctx->stream));
        if (refresh & 1) refresh_left(j, U, chil, chi);
        if (refresh & 2) {
            // B_{j+1} = V_j Psi_{j+1} = Vh
            double2* B = static_cast<double2*>(ctx->workspace("seg_B", sizeof(double2) * (size_t)chi * cols));
            copy2d(B, cols, SV, cols, chi, cols, 0, ctx->stream);
            scale_rows(B, cols, sg->Vd[j].as<double>(), chi, cols, ctx->stream);
            refresh_right(j + 1, B, chi, chir);
        }
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));  // host vectors above go out of scope
    }

    std::vector<double> scal_host;
    void upload_scale(const std::vector<double>& s, bool invert) {
        scal_host.resize(s.size());
        for (size_t c = 0; c < s.size(); ++c) scal_host[c] = invert ? 1.0 / s[c] : s[c];
        double* dv = static_cast<double*>(ctx->workspace("seg_scal", sizeof(double) * std::max<size_t>(1, s.size())));
        TDVP_CHECK_HIP(hipMemcpyAsync(dv, scal_host.data(), sizeof(double) * s.size(), hipMemcpyHostToDevice,
                                      ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    }
    const double* scal_dev() { return static_cast<const double*>(ctx->workspace("seg_scal", 8)); }

    // Bond j takes dimension chi: the two site tensors and V_j keep their
    // buffers when those are large enough (their contents are rewritten by the
    // caller).
    void set_bond(int j, int chi) {
        if (sg->chi[j + 1] == chi) return;
        sg->chi[j + 1] = chi;
        need(sg->Psi[j], sizeof(double2) * sg->psi_elems(j));
        need(sg->Psi[j + 1], sizeof(double2) * sg->psi_elems(j + 1));
        need(sg->Vd[j], sizeof(double) * chi);
    }

    // Largest bond a split of pair (j, j+1) can produce.
    int split_cap(int j) const {
        int cap = o.chi_max;
        if (o.static_shapes) cap = std::min(cap, sg->cap[j + 1]);
        return std::max(1, std::min({cap, sg->chi[j] * sg->d, sg->d * sg->chi[j + 2]}));
    }
    // On the calling thread, before a phase runs on the lanes: every state
    // buffer the op may write, at its largest size.
    void presize_split(const SOp& op) {
        const int j = op.j, c = split_cap(j), d = sg->d;
        need(sg->Psi[j], sizeof(double2) * (size_t)sg->chi[j] * d * c);
        need(sg->Psi[j + 1], sizeof(double2) * (size_t)c * d * sg->chi[j + 2]);
        need(sg->Vd[j], sizeof(double) * (size_t)c);
        if (op.refresh & 1) env_buf(sg->beta[j + 1], (size_t)W->w[j + 1] * c * c);
        if (op.refresh & 2) env_buf(sg->gamma[j], (size_t)W->w[j + 1] * c * c);
    }
    // The named workspaces a split on a lane asks for (its own, the
    // environment refresh's and the small density-matrix path's), at their
    // largest size over the phase, grown on the owning thread: a split on a
    // lane then allocates nothing.  The solver's own buffers are reserved by
    // reserve_solver_workspace.
    void presize_lane_split(tdvp_ctx_s& c, const SPhase& ph) {
        const int d = sg->d;
        const size_t esz = elem_bytes(sg->edt);
        size_t u = 1, sv = 1, k1 = 1, env = 1, gn = 0, gp = 1;
        for (const auto& op : ph) {
            const int j = op.j;
            const size_t rows = (size_t)sg->chi[j] * d, cols = (size_t)d * sg->chi[j + 2], k = (size_t)split_cap(j);
            const size_t wmax = (size_t)std::max({W->w[j], W->w[j + 1], W->w[j + 2]});
            u = std::max(u, rows * k);
            sv = std::max(sv, k * cols);
            k1 = std::max(k1, k);
            env = std::max(env, esz * wmax * std::max(rows, cols) * k);
            const size_t n = std::min(rows, cols);
            if (n <= (size_t)kJacobiMaxOrder) {
                gn = std::max(gn, n);
                gp = std::max(gp, n * std::max(rows, cols));
            }
        }
        c.workspace("seg_U", sizeof(double2) * u);
        c.workspace("seg_US", sizeof(double2) * u);
        c.workspace("seg_SV", sizeof(double2) * sv);
        c.workspace("seg_B", sizeof(double2) * sv);
        c.workspace("seg_scal", sizeof(double) * k1);
        c.workspace("env_X", env);
        c.workspace("env_Y", env);
        if (gn) {
            c.workspace("gram_G", sizeof(double2) * gn * gn);
            c.workspace("gram_vecs", sizeof(double2) * gn * gn);
            c.workspace("gram_ev", sizeof(double) * gn);
            c.workspace("gram_E", sizeof(double) * gn);
            c.workspace("gram_info", sizeof(int));
            c.workspace("gram_P", sizeof(double2) * gp);
        }
    }
    void presize_bond(const SOp& op) {
        const int j = op.j, c = sg->chi[j + 1];
        if (op.refresh == 1) env_buf(sg->beta[j + 1], (size_t)W->w[j + 1] * c * c);
        else env_buf(sg->gamma[j], (size_t)W->w[j + 1] * c * c);
    }

    // ---------------------------------------------------------- phases
    static std::string key(bool first, int idx) { return (first ? "A" : "B") + std::to_string(idx); }

    // Per-instance local problems of a phase and their packed layout.
    void build_plan(PhasePlan& P, const SPhase& ph, bool pair) {
        const int d = sg->d;
        const int D = pair ? d * d : d;
        std::vector<int64_t> n(ph.size());
        for (size_t i = 0; i < ph.size(); ++i) {
            const int j = ph[i].j;
            const int chil = sg->chi[j], chir = sg->chi[j + (pair ? 2 : 1)];
            n[i] = (int64_t)chil * D * chir;
        }
        seg_layout(ctx, n, P.L);
        const int64_t T = P.L.total;
        // matvec buffers (compute precision) and the two intermediate stages
        int64_t t1 = 0, t3 = 0;
        std::vector<int64_t> o1(ph.size()), o3(ph.size());
        for (size_t i = 0; i < ph.size(); ++i) {
            const int j = ph[i].j;
            const int wl = W->w[j], wr = W->w[j + (pair ? 2 : 1)];
            const int chil = sg->chi[j], chir = sg->chi[j + (pair ? 2 : 1)];
            o1[i] = t1;
            o3[i] = t3;
            t1 += (int64_t)wl * chil * D * chir;
            t3 += (int64_t)wr * chil * D * chir;
        }
        const size_t ce = esz();
        void* X = ctx->workspace("segb_X", ce * (size_t)std::max<int64_t>(1, T));
        void* Y = ctx->workspace("segb_Y", ce * (size_t)std::max<int64_t>(1, T));
        void* T1 = ctx->workspace("segb_T1", ce * (size_t)std::max<int64_t>(1, t1));
        void* T3 = ctx->workspace("segb_T3", ce * (size_t)std::max<int64_t>(1, t3));
        ctx->workspace("segb_theta", sizeof(double2) * (size_t)std::max<int64_t>(1, T));
        batch_expm_reserve(ctx, P.L, o.krylov_k);
        const Dt cdt = sg->edt;
        std::vector<GemmDesc> ga, gb;
        std::vector<WStageDesc> ws;
        P.flops_per_matvec = 0.0;
        for (size_t i = 0; i < ph.size(); ++i) {
            const int j = ph[i].j;
            const HeffArgs h = pair ? h2(j) : h1(j);
            const int64_t chil = h.chil, chir = h.chir;
            char* x = static_cast<char*>(X) + ce * P.L.off[i];
            char* y = static_cast<char*>(Y) + ce * P.L.off[i];
            char* p1 = static_cast<char*>(T1) + ce * o1[i];
            char* p3 = static_cast<char*>(T3) + ce * o3[i];
            GemmDesc g1;  // T1[(k a')][(s b)] = L x
            g1.M = (int)(h.wl * chil);
            g1.N = (int)(D * chir);
            g1.K = (int)chil;
            g1.A.p = h.L; g1.A.dt = cdt; g1.A.ld = chil; g1.A.kcontig = true;
            g1.B.p = x; g1.B.dt = cdt; g1.B.ld = D * chir; g1.B.kcontig = false;
            g1.C = p1; g1.cdt = cdt; g1.ldc = D * chir;
            ga.push_back(g1);
            WStageDesc w;  // T3[a'][s'][n][b] = sum M[(n s'),(k s)] T1[k][a'][s][b]
            w.in = p1; w.in_dt = cdt; w.out = p3; w.out_dt = cdt;
            w.P = (int)chil; w.Q = (int)chir; w.D = D; w.w_in = h.wl; w.w_out = h.wr;
            w.ik = chil * D * chir; w.is = chir; w.ip = D * chir;
            w.on = chir; w.os = h.wr * chir; w.op = (int64_t)D * h.wr * chir;
            w.row_ptr = h.mop->row_ptr; w.col = h.mop->col; w.val = h.mop->val; w.fp64 = fp64;
            ws.push_back(w);
            GemmDesc g2;  // y[(a' s')][b'] = T3 R
            g2.M = (int)(chil * D);
            g2.N = (int)chir;
            g2.K = (int)(h.wr * chir);
            g2.A.p = p3; g2.A.dt = cdt; g2.A.ld = h.wr * chir; g2.A.kcontig = true;
            g2.B.p = h.R; g2.B.dt = cdt; g2.B.ld = chir; g2.B.kcontig = false;
            g2.C = y; g2.cdt = cdt; g2.ldc = chir;
            gb.push_back(g2);
            P.flops_per_matvec += heff_flops(pair ? 2 : 1, (int)chil, (int)chir, d, h.wl, h.wr);
        }
        grouped_gemm_plan(ctx, ga, fp64, form, P.A);
        grouped_wstage_plan(ctx, ws, P.W);
        grouped_gemm_plan(ctx, gb, fp64, form, P.B);
        // per-instance state pointers for gather / scatter (site phases)
        std::vector<double2*> ptr(ph.size());
        for (size_t i = 0; i < ph.size(); ++i) ptr[i] = sg->psi(ph[i].j);
        P.ptrs = DevMem(ctx, sizeof(double2*) * std::max<size_t>(1, ph.size()));
        TDVP_CHECK_HIP(hipMemcpyAsync(P.ptrs.ptr, ptr.data(), sizeof(double2*) * ph.size(), hipMemcpyHostToDevice,
                                      ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        P.sig = signature(ph, pair);
        P.gen = ctx->ws_gen;
        if (P.graph) {
            (void)hipGraphExecDestroy(P.graph);
            P.graph = nullptr;
        }
    }

    std::vector<const void*> signature(const SPhase& ph, bool pair) {
        std::vector<const void*> sig;
        for (const auto& op : ph) {
            const int j = op.j, r = j + (pair ? 2 : 1);
            sig.push_back(sg->Psi[j].ptr);
            sig.push_back(sg->beta[j].ptr);
            sig.push_back(sg->gamma[r - 1].ptr);
            sig.push_back(reinterpret_cast<const void*>((intptr_t)sg->chi[j]));
            sig.push_back(reinterpret_cast<const void*>((intptr_t)sg->chi[r]));
            sig.push_back(reinterpret_cast<const void*>((intptr_t)op.j));
        }
        return sig;
    }

    // The launches of one batched exponentiation (no host synchronisation).
    void launch_batched(PhasePlan& P, bool pair, double tau) {
        const int64_t T = P.L.total;
        double2* theta = static_cast<double2*>(ctx->workspace("segb_theta", sizeof(double2) * (size_t)T));
        void* X = ctx->workspace("segb_X", esz() * (size_t)T);
        void* Y = ctx->workspace("segb_Y", esz() * (size_t)T);
        if (!pair) seg_gather(ctx, P.L, theta, static_cast<const double2* const*>(P.ptrs.ptr));
        BatchOp op = [&](const double2* x, double2* y) {
            convert(X, sg->edt, x, Dt::C128, T, ctx->stream);
            grouped_gemm_run(ctx, P.A);
            grouped_wstage_run(ctx, P.W);
            grouped_gemm_run(ctx, P.B);
            convert(y, Dt::C128, Y, sg->edt, T, ctx->stream);
        };
        BatchState bs;
        batch_expm(ctx, P.L, op, theta, tau, o.krylov_k, bs);
        seg_flag_or(ctx, bs, sg->flag.as<int>());
        if (!pair) seg_scatter(ctx, P.L, static_cast<double2* const*>(P.ptrs.ptr), theta);
    }

    // Eager launches, or the phase's graph (captured on first use).
    void exec_batched(PhasePlan& P, bool pair, double tau) {
        if (o.use_graph) {
            if (!P.graph) {
                if (!sg->cap_stream) TDVP_CHECK_HIP(hipStreamCreateWithFlags(&sg->cap_stream, hipStreamNonBlocking));
                const bool prof = ctx->prof_on;
                hipStream_t home = ctx->stream;
                ctx->prof_on = false;
                ctx->stream = sg->cap_stream;  // capture only records; nothing runs here
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    try {
                        launch_batched(P, pair, tau);
                    } catch (...) {
                        (void)hipStreamEndCapture(ctx->stream, &g);
                        if (g) (void)hipGraphDestroy(g);
                        ctx->stream = home;
                        ctx->prof_on = prof;
                        throw;
                    }
                    e = hipStreamEndCapture(ctx->stream, &g);
                }
                ctx->stream = home;
                ctx->prof_on = prof;
                TDVP_CHECK_HIP(e);
                e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                TDVP_CHECK_HIP(e);
                TDVP_REQUIRE(P.gen == ctx->ws_gen, TDVP_E_STATE, "workspace moved during graph capture");
            }
            TDVP_CHECK_HIP(hipGraphLaunch(P.graph, ctx->stream));
        } else {
            launch_batched(P, pair, tau);
        }
    }

    void run_batched(const SPhase& ph, bool pair, bool first, int idx) {
        auto& slot = sg->plans[key(first, idx)];
        if (!slot) slot = std::make_unique<PhasePlan>();
        PhasePlan& P = *slot;
        if (P.gen != ctx->ws_gen || P.sig != signature(ph, pair)) build_plan(P, ph, pair);
        if (P.gen != ctx->ws_gen) build_plan(P, ph, pair);  // a workspace moved while planning
        const double tau = ph[0].tau;
        for (const auto& op : ph) TDVP_REQUIRE(op.tau == tau, TDVP_E_STATE, "segment phase with mixed time steps");
        if (pair) {
            double2* theta = static_cast<double2*>(ctx->workspace("segb_theta", sizeof(double2) * (size_t)P.L.total));
            for (size_t i = 0; i < ph.size(); ++i) form_theta(ph[i].j, theta + P.L.off[i]);
        }
        if (P.gen != ctx->ws_gen) build_plan(P, ph, pair);
        {
            TxRange tx("seg_phase_expm");
            ProfScope ps(ctx, o.use_graph ? "seg_batched_expm_graph" : "seg_batched_expm",
                         P.flops_per_matvec * o.krylov_k, 0.0);
            exec_batched(P, pair, tau);
        }
        st.matvecs += o.krylov_k * (int)ph.size();
        st.flops += P.flops_per_matvec * o.krylov_k;
        st.krylov_max_used = std::max(st.krylov_max_used, o.krylov_k);
        if (pair) {
            const double2* theta =
                static_cast<const double2*>(ctx->workspace("segb_theta", sizeof(double2) * (size_t)P.L.total));
            TxRange tx("seg_phase_splits");
            ProfScope ps(ctx, "seg_splits", 0.0, 0.0);
            split_concurrent(ph, theta, P.L.off);
        }
    }

    static int lane_count() {
        const char* e = getenv("TDVP_SEG_LANES");
        const int n = e ? atoi(e) : 8;
        return std::max(1, std::min(n, 32));
    }

    void ensure_lanes(int n) {
        if (!sg->ready) TDVP_CHECK_HIP(hipEventCreateWithFlags(&sg->ready, hipEventDisableTiming));
        while ((int)sg->lanes.size() < n) {
            auto L = std::make_unique<SegLane>();
            // Lane workspaces come from hipMalloc, not from the context's
            // allocator callback: the lanes are library worker threads, and the
            // callback (which may re-enter an interpreter) is only called from
            // the thread that owns the context.
            L->c.device = ctx->device;
            L->c.alloc_fn = nullptr;
            L->c.free_fn = nullptr;
            L->c.user = nullptr;
            // no tile timing and no K splits on a lane: both would allocate
            // (candidate runs, split-K partials) from the worker thread
            L->c.autotune = false;
            L->c.splitk = false;
            TDVP_CHECK_HIP(hipStreamCreateWithFlags(&L->c.stream, hipStreamNonBlocking));
            TDVP_REQUIRE(rocblas_create_handle(&L->c.blas) == rocblas_status_success, TDVP_E_HIP,
                         "rocblas_create_handle failed");
            rocblas_set_stream(L->c.blas, L->c.stream);
            TDVP_CHECK_HIP(hipEventCreateWithFlags(&L->done, hipEventDisableTiming));
            sg->lanes.push_back(std::move(L));
        }
    }

    // The splits of one phase (instance i reads theta + off[i]); instances are
    // taken largest first by a pool of lanes.  Each split only touches its own
    // pair of sites, bond and environments.
    // Runs body(r, i) for the listed op indices on nl split lanes (each a
    // host thread with its own stream, rocBLAS handle and workspaces); the
    // lanes start after the work queued so far on the context stream, and the
    // context stream waits for all of them.
    void on_lanes(int nl, const std::vector<int>& order, const std::function<void(SegRun&, int)>& body) {
        ensure_lanes(nl);
        TDVP_CHECK_HIP(hipEventRecord(sg->ready, ctx->stream));
        const int n = (int)order.size();
        std::atomic<int> next{0};
        std::vector<std::exception_ptr> errs(nl);
        std::vector<tdvp_stats> lst(nl);
        std::vector<std::thread> pool;
        for (int l = 0; l < nl; ++l) {
            pool.emplace_back([&, l] {
                try {
                    TxRange tx("seg_lane");
                    SegLane& L = *sg->lanes[l];
                    TDVP_CHECK_HIP(hipSetDevice(L.c.device));
                    TDVP_CHECK_HIP(hipStreamWaitEvent(L.c.stream, sg->ready, 0));
                    lst[l] = tdvp_stats{};
                    SegRun r{&L.c, sg, W, o, lst[l], fp64, form};
                    for (int t = next++; t < n; t = next++) body(r, order[t]);
                    TDVP_CHECK_HIP(hipEventRecord(L.done, L.c.stream));
                } catch (...) {
                    errs[l] = std::current_exception();
                }
            });
        }
        for (auto& t : pool) t.join();
        for (int l = 0; l < nl; ++l) {
            if (!errs[l]) TDVP_CHECK_HIP(hipStreamWaitEvent(ctx->stream, sg->lanes[l]->done, 0));
            st.w_step += lst[l].w_step;
            st.flops += lst[l].flops;
            st.matvecs += lst[l].matvecs;
            st.krylov_max_used = std::max(st.krylov_max_used, lst[l].krylov_max_used);
        }
        for (auto& e : errs)
            if (e) std::rethrow_exception(e);
    }

    void split_concurrent(const SPhase& ph, const double2* theta, const std::vector<int64_t>& off) {
        const int n = (int)ph.size();
        const int nl = std::min(lane_count(), n);
        if (nl <= 1) {
            for (int i = 0; i < n; ++i) split(ph[i].j, theta + off[i], ph[i].refresh);
            return;
        }
        SolverSizes ss;
        for (const auto& op : ph) {  // operators are cached lazily; build them here, single-threaded
            W->mop(1, op.j, fp64);
            W->mop(3, op.j + 1, fp64);
            presize_split(op);
            const int rows = sg->chi[op.j] * sg->d, cols = sg->d * sg->chi[op.j + 2];
            if (o.svd_mode != 1) ss.eig_n = std::max(ss.eig_n, std::min(rows, cols));
            if (o.svd_mode != 2) {
                ss.svd_rows = std::max(ss.svd_rows, rows);
                ss.svd_cols = std::max(ss.svd_cols, cols);
            }
        }
        ensure_lanes(nl);
        for (int l = 0; l < nl; ++l) {
            reserve_solver_workspace(&sg->lanes[l]->c, ss);
            presize_lane_split(sg->lanes[l]->c, ph);
        }
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::sort(order.begin(), order.end(),
                  [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
        on_lanes(nl, order, [&](SegRun& r, int i) { r.split(ph[i].j, theta + off[i], ph[i].refresh); });
    }

    // The bond steps of a phase (one per segment at most, on disjoint
    // tensors and environments), concurrently on the split lanes.
    void bonds_concurrent(const SPhase& ph) {
        TxRange tx("seg_phase_bonds");
        const int n = (int)ph.size();
        const int nl = std::min(lane_count(), n);
        if (nl <= 1) {
            for (const auto& op : ph) bond_step(op.j, op.tau, op.refresh);
            return;
        }
        SolverSizes ss;
        for (const auto& op : ph) {
            W->mop(0, op.j, fp64);
            W->mop(1, op.j, fp64);
            W->mop(3, op.j + 1, fp64);
            presize_bond(op);
            const int rows = sg->chi[op.j] * sg->d, c = sg->chi[op.j + 1], cols = sg->d * sg->chi[op.j + 2];
            if (op.refresh == 1) {
                ss.qr_rows = std::max(ss.qr_rows, rows);
                ss.qr_cols = std::max(ss.qr_cols, c);
            } else {
                ss.lq_rows = std::max(ss.lq_rows, c);
                ss.lq_cols = std::max(ss.lq_cols, cols);
            }
        }
        ensure_lanes(nl);
        for (int l = 0; l < nl; ++l) reserve_solver_workspace(&sg->lanes[l]->c, ss);
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return sg->chi[ph[a].j + 1] > sg->chi[ph[b].j + 1]; });
        ProfScope ps(ctx, "seg_bonds", 0.0, 0.0);
        on_lanes(nl, order, [&](SegRun& r, int i) { r.bond_step(ph[i].j, ph[i].tau, ph[i].refresh); });
    }

    // Instance by instance (reference for the batched path).
    void run_serial(const SPhase& ph, bool pair) {
        for (const auto& op : ph) {
            const int j = op.j;
            const HeffArgs h = pair ? h2(j) : h1(j);
            const int D = pair ? sg->d * sg->d : sg->d;
            const int64_t n = (int64_t)h.chil * D * h.chir;
            double2* x;
            if (pair) {
                x = static_cast<double2*>(ctx->workspace("seg_theta1", sizeof(double2) * (size_t)n));
                form_theta(j, x);
            } else {
                x = sg->psi(j);
            }
            MatVec mv = [&](const double2* a, double2* b) { heff_apply(ctx, h, a, Dt::C128, b, Dt::C128); };
            KrylovInfo ki = expm_krylov(ctx, mv, x, n, op.tau, o.krylov_k, 0.0);
            st.matvecs += ki.matvecs;
            st.flops += heff_flops(pair ? 2 : 1, h.chil, h.chir, sg->d, h.wl, h.wr) * ki.matvecs;
            st.krylov_max_used = std::max(st.krylov_max_used, ki.k);
            if (pair) split(j, x, op.refresh);
        }
    }

    // A phase of the one-site schedule: its boundary pairs, its site
    // exponentials (batched like the two-site schedule's) and its bond steps;
    // the ops of a phase are independent, so running them kind by kind is
    // the same as any other order.
    void run_one_site_phase(const SPhase& ph, bool first, int idx) {
        SPhase pairs, sites, bonds;
        for (const auto& op : ph) (op.bond ? bonds : (op.pair ? pairs : sites)).push_back(op);
        if (!pairs.empty()) {
            if (o.batched) run_batched(pairs, true, first, 1000 + 2 * idx);
            else run_serial(pairs, true);
        }
        if (!sites.empty()) {
            if (o.batched) run_batched(sites, false, first, 1001 + 2 * idx);
            else run_serial(sites, false);
        }
        if (o.batched) bonds_concurrent(bonds);
        else
            for (const auto& op : bonds) bond_step(op.j, op.tau, op.refresh);
    }

    void step(double dt) {
        TxRange tx("seg_step");
        reset_flag(ctx, sg->flag.as<int>());
        const auto t0 = std::chrono::steady_clock::now();
        int done = 0;  // phases run so far (o.max_phases > 0 stops the step early)
        auto more = [&] { return o.max_phases <= 0 || done < o.max_phases; };
        for (int half = 0; half < 2 && more(); ++half) {
            const bool first = half == 0;
            if (o.one_site) {
                sg->mixed_gauge = true;
                const std::vector<SPhase> phases = seg_schedule1(sg->sizes, dt, first);
                for (size_t idx = 0; idx < phases.size() && more(); ++idx, ++done)
                    run_one_site_phase(phases[idx], first, (int)idx);
                continue;
            }
            const std::vector<SPhase> phases = seg_schedule(sg->sizes, dt, first);
            for (size_t idx = 0; idx < phases.size() && more(); ++idx, ++done) {
                const SPhase& ph = phases[idx];
                const bool pair = ph[0].pair;
                for (const auto& op : ph)
                    TDVP_REQUIRE(op.pair == pair, TDVP_E_STATE, "segment phase mixes pair and site updates");
                if (o.batched) run_batched(ph, pair, first, (int)idx);
                else run_serial(ph, pair);
            }
        }
        int bad = 0;
        TDVP_CHECK_HIP(hipMemcpyAsync(&bad, sg->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        TDVP_REQUIRE(!bad, TDVP_E_NUMERIC, "segment step: non-finite value in a Krylov recursion");
        sg->w_total += st.w_step;
        st.w_total = sg->w_total;
        int peak = 0;
        for (int c : sg->chi) peak = std::max(peak, c);
        st.chi_peak = peak;
    }
};

// ------------------------------------------------------------ initial state
// Any MPS -> inverse canonical gauge: right-orthonormalise by LQ, then sweep
// left to right splitting off Psi_j = U S with V_j = 1/S (the Schmidt
// coefficients of bond j); the norm stays in Psi_{N-1}.
void to_inverse_canonical(tdvp_ctx ctx, tdvp_seg sg, int svd_mode) {
    const int N = sg->N, d = sg->d;
    hipStream_t s = ctx->stream;
    for (int j = N - 1; j >= 1; --j) {
        const int rows = sg->chi[j], cols = d * sg->chi[j + 1];
        double2* Lf = static_cast<double2*>(ctx->workspace("ic_L", sizeof(double2) * (size_t)rows * rows));
        double2* Q = static_cast<double2*>(ctx->workspace("ic_Q", sizeof(double2) * (size_t)rows * cols));
        lq_rowmajor(ctx, sg->psi(j), rows, cols, Lf, Q);
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->psi(j), Q, sizeof(double2) * (size_t)rows * cols, hipMemcpyDeviceToDevice, s));
        const int m1 = sg->chi[j - 1] * d;
        double2* T = static_cast<double2*>(ctx->workspace("ic_T", sizeof(double2) * (size_t)m1 * rows));
        zgemm_rowmajor(ctx, sg->psi(j - 1), Lf, T, m1, rows, rows);
        // drop the global factor (it would overflow over a long chain)
        double2* nrm = static_cast<double2*>(ctx->workspace("ic_nrm", sizeof(double2)));
        vdot_multi(ctx, T, 0, 1, T, (int64_t)m1 * rows, nrm);
        double2 h{0.0, 0.0};
        TDVP_CHECK_HIP(hipMemcpyAsync(&h, nrm, sizeof(h), hipMemcpyDeviceToHost, s));
        TDVP_CHECK_HIP(hipStreamSynchronize(s));
        TDVP_REQUIRE(std::isfinite(h.x) && h.x > 0.0, TDVP_E_NUMERIC, "inverse canonical form: zero or non-finite tensor");
        scale_copy(sg->psi(j - 1), T, 1.0 / std::sqrt(h.x), (int64_t)m1 * rows, s);
    }
    for (int j = 0; j + 1 < N; ++j) {
        const int rows = sg->chi[j] * d, n = sg->chi[j + 1], cols2 = d * sg->chi[j + 2];
        double2* M = sg->psi(j);
        std::vector<double> sv;
        double2* Vrow = nullptr;  // [n][n] rows v_c^dagger (right singular vectors)
        bool use_svd = svd_mode == 1;
        if (!use_svd) {
            GramResult g = gram_eigen(ctx, M, rows, n, false);
            sv = g.s;
            if (svd_mode == 0 && sv[n - 1] < 1e-6 * sv[0]) use_svd = true;
            else Vrow = g.vecs;
        }
        double2* US = static_cast<double2*>(ctx->workspace("ic_US", sizeof(double2) * (size_t)rows * n));
        if (use_svd) {
            SvdResult r = svd_rowmajor(ctx, M, rows, n);
            TDVP_REQUIRE(r.k == n, TDVP_E_SHAPE, "inverse canonical form: bond dimension exceeds the rank bound");
            sv = r.S;
            copy2d(US, n, r.U, r.k, rows, n, 0, s);
            scale_cols(US, n, r.S_dev, rows, n, s);
            Vrow = static_cast<double2*>(ctx->workspace("ic_Vrow", sizeof(double2) * (size_t)n * n));
            copy2d(Vrow, n, r.Vh, n, n, n, 0, s);
        } else {
            GemmDesc gd;  // U S = M V
            gd.cdt = Dt::C128;
            gd.M = rows; gd.N = n; gd.K = n;
            gd.A.p = M; gd.A.dt = Dt::C128; gd.A.ld = n; gd.A.kcontig = true;
            gd.B.p = Vrow; gd.B.dt = Dt::C128; gd.B.ld = n; gd.B.kcontig = true; gd.B.conj = true;
            gd.C = US; gd.ldc = n;
            cgemm(ctx, gd, true, 4);
        }
        // Schmidt coefficients of the normalised state
        double ss = 0.0;
        for (double v : sv) ss += v * v;
        const double snorm = std::sqrt(ss);
        TDVP_REQUIRE(std::isfinite(snorm) && snorm > 0.0, TDVP_E_NUMERIC, "inverse canonical form: zero state");
        for (double& v : sv) v /= snorm;
        scale_copy(US, US, 1.0 / snorm, (int64_t)rows * n, s);
        for (double v : sv)
            TDVP_REQUIRE(v > 0.0 && std::isfinite(v), TDVP_E_NUMERIC,
                         "inverse canonical form: bond " + std::to_string(j) + " has a zero Schmidt coefficient");
        // next centre: S Vh Psi_{j+1}
        double2* SVT = static_cast<double2*>(ctx->workspace("ic_SVT", sizeof(double2) * (size_t)n * cols2));
        zgemm_rowmajor(ctx, Vrow, sg->psi(j + 1), SVT, n, n, cols2);
        std::vector<double> inv(n);
        for (int c = 0; c < n; ++c) inv[c] = 1.0 / sv[c];
        sg->Vh[j] = inv;
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->Vd[j].ptr, sv.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
        scale_rows(SVT, cols2, sg->Vd[j].as<double>(), n, cols2, s);
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->psi(j), US, sizeof(double2) * (size_t)rows * n, hipMemcpyDeviceToDevice, s));
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->psi(j + 1), SVT, sizeof(double2) * (size_t)n * cols2, hipMemcpyDeviceToDevice,
                                      s));
        TDVP_CHECK_HIP(hipMemcpyAsync(sg->Vd[j].ptr, inv.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
        TDVP_CHECK_HIP(hipStreamSynchronize(s));
    }
}

void build_environments(tdvp_ctx ctx, tdvp_seg sg, tdvp_mpo W) {
    const int N = sg->N, d = sg->d;
    tdvp_seg_opts o;
    tdvp_seg_opts_default(&o);
    o.compute = sg->edt == Dt::C128 ? TDVP_C128 : TDVP_C64;
    tdvp_stats st{};
    SegRun r{ctx, sg, W, o, st, sg->edt == Dt::C128, sg->edt == Dt::C128 ? 4 : 3};
    auto one = [&](DevMem& b) {
        r.env_buf(b, 1);
        if (sg->edt == Dt::C128) {
            const double2 v{1.0, 0.0};
            TDVP_CHECK_HIP(hipMemcpyAsync(b.ptr, &v, sizeof(v), hipMemcpyHostToDevice, ctx->stream));
        } else {
            const float2 v{1.0f, 0.0f};
            TDVP_CHECK_HIP(hipMemcpyAsync(b.ptr, &v, sizeof(v), hipMemcpyHostToDevice, ctx->stream));
        }
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    };
    one(sg->beta[0]);
    one(sg->gamma[N - 1]);
    for (int j = 0; j + 1 < N; ++j) {  // A_j = Psi_j V_j
        const int rows = sg->chi[j] * d, c = sg->chi[j + 1];
        double2* A = static_cast<double2*>(ctx->workspace("ic_A", sizeof(double2) * (size_t)rows * c));
        copy2d(A, c, sg->psi(j), c, rows, c, 0, ctx->stream);
        scale_cols(A, c, sg->Vd[j].as<double>(), rows, c, ctx->stream);
        r.refresh_left(j, A, sg->chi[j], c);
    }
    for (int j = N - 1; j >= 1; --j) {  // B_j = V_{j-1} Psi_j
        const int c = sg->chi[j], cols = d * sg->chi[j + 1];
        double2* B = static_cast<double2*>(ctx->workspace("ic_A", sizeof(double2) * (size_t)c * cols));
        copy2d(B, cols, sg->psi(j), cols, c, cols, 0, ctx->stream);
        scale_rows(B, cols, sg->Vd[j - 1].as<double>(), c, cols, ctx->stream);
        r.refresh_right(j, B, c, sg->chi[j + 1]);
    }
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
}

// The hybrid switch for segment runs: every bond holds its largest possible
// dimension, min(chi_max, d^min(j, N-j)) and, with static shapes, its initial
// dimension (the serial rule with the static caps added).
bool seg_saturated(const tdvp_seg_s& sg, const tdvp_seg_opts& o) {
    const int N = sg.N;
    for (int j = 1; j < N; ++j) {
        const int64_t cmax = o.static_shapes ? std::min(o.chi_max, sg.cap[j]) : o.chi_max;
        int64_t lim = 1;
        for (int e = 0; e < std::min(j, N - j) && lim < cmax; ++e) lim *= sg.d;
        if (sg.chi[j] < std::min(lim, cmax)) return false;
    }
    return true;
}

// ------------------------------------------------------------ repair
// <psi|psi> of Psi_0 V_0 Psi_1 ... Psi_{N-1} by left transfers of the
// tensors A_j = Psi_j V_j (the last tensor as it stands), FP64.
double state_norm2(tdvp_ctx ctx, tdvp_seg sg) {
    const int N = sg->N, d = sg->d;
    hipStream_t s = ctx->stream;
    std::vector<double2> id((size_t)d * d, double2{0.0, 0.0});
    for (int k = 0; k < d; ++k) id[(size_t)k * d + k] = double2{1.0, 0.0};
    DevMem idd(ctx, sizeof(double2) * d * d);
    DevMem E(ctx, sizeof(double2)), E2;
    const double2 one{1.0, 0.0};
    TDVP_CHECK_HIP(hipMemcpyAsync(idd.ptr, id.data(), sizeof(double2) * d * d, hipMemcpyHostToDevice, s));
    TDVP_CHECK_HIP(hipMemcpyAsync(E.ptr, &one, sizeof(one), hipMemcpyHostToDevice, s));
    TDVP_CHECK_HIP(hipStreamSynchronize(s));
    Mop mop;
    mop_make(ctx, mop, 1, idd.ptr, nullptr, Dt::C128, 1, 1, 1, d, true, true);
    for (int j = 0; j < N; ++j) {
        const int cl = sg->chi[j], cr = sg->chi[j + 1];
        const double2* A = sg->psi(j);
        if (j + 1 < N) {
            double2* T = static_cast<double2*>(ctx->workspace("nrm_A", sizeof(double2) * (size_t)cl * d * cr));
            copy2d(T, cr, sg->psi(j), cr, cl * d, cr, 0, s);
            scale_cols(T, cr, sg->Vd[j].as<double>(), cl * d, cr, s);
            A = T;
        }
        E2 = DevMem(ctx, sizeof(double2) * (size_t)cr * cr);
        EnvArgs a{cl, cr, cl, cr, d, 1, 1, A, A, Dt::C128, &mop, true, 4};
        env_left(ctx, a, E.ptr, Dt::C128, E2.ptr, Dt::C128);
        std::swap(E, E2);
    }
    double2 v{0.0, 0.0};
    TDVP_CHECK_HIP(hipMemcpyAsync(&v, E.ptr, sizeof(v), hipMemcpyDeviceToHost, s));
    TDVP_CHECK_HIP(hipStreamSynchronize(s));
    return v.x;
}

// Serial repair of a segment run (Sec. III D, Fig. reorth): fold the bond
// matrices into the site tensors (an ordinary MPS of the same state), bring
// it back to the inverse canonical gauge of the normalised state and rebuild
// every environment.  Bond dimensions are kept, nothing is truncated.
void reorthonormalize(tdvp_ctx ctx, tdvp_seg sg, tdvp_mpo W) {
    for (int j = 0; j + 1 < sg->N; ++j) {
        const int rows = sg->chi[j] * sg->d, c = sg->chi[j + 1];
        scale_cols(sg->psi(j), c, sg->Vd[j].as<double>(), rows, c, ctx->stream);
    }
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    to_inverse_canonical(ctx, sg, 0);
    build_environments(ctx, sg, W);
    sg->mixed_gauge = false;
}

}  // namespace
}  // namespace tdvp

extern "C" {

int tdvp_seg_opts_default(tdvp_seg_opts* o) {
    if (!o) return TDVP_E_ARG;
    o->compute = TDVP_C64;
    o->krylov_k = 8;
    o->chi_max = 1 << 30;
    o->w_max = 0.0;
    o->eps_rel = 0.0;
    o->multiplet_guard = 1;
    o->static_shapes = 1;
    o->batched = 1;
    o->use_graph = 0;
    o->svd_mode = 0;
    o->one_site = 0;
    o->max_phases = 0;
    return TDVP_OK;
}

int seg_init(tdvp_ctx ctx, tdvp_mpo mpo, int N, int d, const int* chi, const void* const* tensors, int nseg,
             const int* seg_sizes, tdvp_dtype compute, tdvp_seg* out) {
    if (!ctx || !out) return TDVP_E_ARG;
    *out = nullptr;
    return guarded(ctx, [&] {
        TxRange tx("seg_init");
        TDVP_REQUIRE(mpo && chi && tensors && seg_sizes, TDVP_E_ARG, "seg_init: null argument");
        TDVP_REQUIRE(N >= 4 && d >= 1, TDVP_E_SHAPE, "seg_init: need N >= 4 sites");
        TDVP_REQUIRE(mpo->N == N && mpo->d == d, TDVP_E_SHAPE, "seg_init: MPO size differs from the state");
        TDVP_REQUIRE(nseg == 1 || (nseg >= 2 && nseg % 2 == 0), TDVP_E_ARG,
                     "seg_init: the number of segments must be 1 or even");
        int tot = 0;
        for (int s = 0; s < nseg; ++s) {
            TDVP_REQUIRE(seg_sizes[s] >= 2, TDVP_E_SHAPE, "seg_init: every segment needs at least two sites");
            tot += seg_sizes[s];
        }
        TDVP_REQUIRE(tot == N, TDVP_E_SHAPE, "seg_init: segment sizes do not add up to N");
        TDVP_REQUIRE(chi[0] == 1 && chi[N] == 1, TDVP_E_SHAPE, "seg_init: boundary bonds must be 1");
        for (int j = 0; j < N; ++j) {
            TDVP_REQUIRE(tensors[j], TDVP_E_ARG, "seg_init: null site tensor");
            TDVP_REQUIRE(chi[j + 1] >= 1 && chi[j + 1] <= (int64_t)d * chi[j] && chi[j] <= (int64_t)d * chi[j + 1],
                         TDVP_E_SHAPE, "seg_init: bond dimensions are not isometry-feasible");
        }
        const Dt cdt = to_dt(compute);
        auto sg = std::make_unique<tdvp_seg_s>();
        sg->ctx = ctx;
        sg->N = N;
        sg->d = d;
        sg->sizes.assign(seg_sizes, seg_sizes + nseg);
        sg->chi.assign(chi, chi + N + 1);
        sg->cap = sg->chi;
        sg->edt = cdt;
        sg->Psi.resize(N);
        sg->Vd.resize(N - 1);
        sg->Vh.resize(N - 1);
        sg->beta.resize(N);
        sg->gamma.resize(N);
        sg->flag = DevMem(ctx, sizeof(int));
        for (int j = 0; j < N; ++j) {
            sg->Psi[j] = DevMem(ctx, sizeof(double2) * sg->psi_elems(j));
            TDVP_CHECK_HIP(hipMemcpyAsync(sg->Psi[j].ptr, tensors[j], sizeof(double2) * sg->psi_elems(j),
                                          hipMemcpyHostToDevice, ctx->stream));
        }
        for (int j = 0; j + 1 < N; ++j) sg->Vd[j] = DevMem(ctx, sizeof(double) * chi[j + 1]);
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        to_inverse_canonical(ctx, sg.get(), 0);
        build_environments(ctx, sg.get(), mpo);
        *out = sg.release();
    });
}

int seg_step(tdvp_ctx ctx, tdvp_seg sg, tdvp_mpo mpo, double dt, const tdvp_seg_opts* opts, tdvp_stats* stats) {
    if (!ctx || !sg) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(sg->ctx == ctx, TDVP_E_ARG, "seg_step: state belongs to another context");
        TDVP_REQUIRE(mpo && mpo->N == sg->N && mpo->d == sg->d, TDVP_E_SHAPE, "seg_step: MPO does not match");
        tdvp_seg_opts o;
        tdvp_seg_opts_default(&o);
        if (opts) o = *opts;
        TDVP_REQUIRE(to_dt(o.compute) == sg->edt, TDVP_E_DTYPE,
                     "seg_step: compute dtype must equal the one the state was created with");
        TDVP_REQUIRE(o.krylov_k >= 1 && o.krylov_k <= 16, TDVP_E_ARG, "seg_step: krylov_k must be in 1..16");
        TDVP_REQUIRE(o.chi_max >= 1, TDVP_E_ARG, "seg_step: chi_max must be >= 1");
        TDVP_REQUIRE(!o.use_graph || (o.batched && o.static_shapes), TDVP_E_ARG,
                     "seg_step: graphs need the batched path with static shapes");
        TDVP_REQUIRE(o.svd_mode >= 0 && o.svd_mode <= 2, TDVP_E_ARG, "seg_step: svd_mode must be 0, 1 or 2");
        TDVP_REQUIRE(o.one_site >= 0 && o.one_site <= 2, TDVP_E_ARG, "seg_step: one_site must be 0, 1 or 2");
        TDVP_REQUIRE(o.max_phases >= 0, TDVP_E_ARG, "seg_step: max_phases must be >= 0");
        if (o.one_site)
            for (size_t s = 1; s + 1 < sg->sizes.size(); ++s)
                TDVP_REQUIRE(sg->sizes[s] >= 3, TDVP_E_SHAPE,
                             "seg_step: the one-site schedule needs at least three sites in every inner segment");
        // 2: the hybrid scheme (two-site steps until the bond dimensions are saturated)
        const bool one = o.one_site == 1 || (o.one_site == 2 && (sg->mixed_gauge || seg_saturated(*sg, o)));
        TDVP_REQUIRE(one || !sg->mixed_gauge, TDVP_E_STATE,
                     "seg_step: after one-site steps call seg_reorthonormalize before a two-site step");
        tdvp_seg_opts oo = o;
        oo.one_site = one ? 1 : 0;
        tdvp_stats st{};
        const bool fp64 = sg->edt == Dt::C128;
        SegRun r{ctx, sg, mpo, oo, st, fp64, fp64 ? 4 : 3};
        r.step(dt);
        if (one) st.flags |= 2;
        if (stats) *stats = st;
    });
}

int seg_get_info(tdvp_seg sg, int* N, int* d, int* chi, double* w_total) {
    if (!sg) return TDVP_E_ARG;
    if (N) *N = sg->N;
    if (d) *d = sg->d;
    if (chi) std::copy(sg->chi.begin(), sg->chi.end(), chi);
    if (w_total) *w_total = sg->w_total;
    return TDVP_OK;
}

int seg_get_psi(tdvp_seg sg, int j, void* out) {
    if (!sg || !out) return TDVP_E_ARG;
    return guarded(sg->ctx, [&] {
        TDVP_REQUIRE(j >= 0 && j < sg->N, TDVP_E_ARG, "seg_get_psi: site out of range");
        TDVP_CHECK_HIP(hipMemcpyAsync(out, sg->Psi[j].ptr, sizeof(double2) * sg->psi_elems(j), hipMemcpyDeviceToHost,
                                      sg->ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(sg->ctx->stream));
    });
}

int seg_get_bond(tdvp_seg sg, int j, double* out) {
    if (!sg || !out) return TDVP_E_ARG;
    return guarded(sg->ctx, [&] {
        TDVP_REQUIRE(j >= 0 && j + 1 < sg->N, TDVP_E_ARG, "seg_get_bond: bond out of range");
        std::copy(sg->Vh[j].begin(), sg->Vh[j].end(), out);
    });
}

int seg_norm2(tdvp_ctx ctx, tdvp_seg sg, double* out) {
    if (!ctx || !sg) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TxRange tx("seg_norm2");
        TDVP_REQUIRE(out, TDVP_E_ARG, "seg_norm2: null argument");
        TDVP_REQUIRE(sg->ctx == ctx, TDVP_E_ARG, "seg_norm2: state belongs to another context");
        *out = state_norm2(ctx, sg);
    });
}

int seg_reorthonormalize(tdvp_ctx ctx, tdvp_seg sg, tdvp_mpo mpo) {
    if (!ctx || !sg) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TxRange tx("seg_reorthonormalize");
        TDVP_REQUIRE(sg->ctx == ctx, TDVP_E_ARG, "seg_reorthonormalize: state belongs to another context");
        TDVP_REQUIRE(mpo && mpo->N == sg->N && mpo->d == sg->d, TDVP_E_SHAPE,
                     "seg_reorthonormalize: MPO does not match");
        reorthonormalize(ctx, sg, mpo);
    });
}

int seg_schedule(int nseg, const int* seg_sizes, double dt, int first_half, int max_ops, int* phase, int* kind,
                 int* site, double* tau, int* n_out) {
    if (!seg_sizes || !n_out || nseg < 1 || (nseg > 1 && nseg % 2)) return TDVP_E_ARG;
    int N = 0;
    for (int s = 0; s < nseg; ++s) {
        if (seg_sizes[s] < 2) return TDVP_E_SHAPE;
        N += seg_sizes[s];
    }
    if (N < 4) return TDVP_E_SHAPE;
    const auto phases = seg_schedule(std::vector<int>(seg_sizes, seg_sizes + nseg), dt, first_half != 0);
    int n = 0;
    for (size_t p = 0; p < phases.size(); ++p)
        for (const auto& op : phases[p]) {
            if (n < max_ops && phase && kind && site && tau) {
                phase[n] = (int)p;
                kind[n] = op.pair ? 2 : 1;
                site[n] = op.j;
                tau[n] = op.tau;
            }
            ++n;
        }
    *n_out = n;
    return n <= max_ops ? TDVP_OK : TDVP_E_SHAPE;
}

int seg_schedule1(int nseg, const int* seg_sizes, double dt, int first_half, int max_ops, int* phase, int* kind,
                  int* site, double* tau, int* n_out) {
    if (!seg_sizes || !n_out || nseg < 1 || (nseg > 1 && nseg % 2)) return TDVP_E_ARG;
    int N = 0;
    for (int s = 0; s < nseg; ++s) {
        if (seg_sizes[s] < 2 || (s > 0 && s + 1 < nseg && seg_sizes[s] < 3)) return TDVP_E_SHAPE;
        N += seg_sizes[s];
    }
    if (N < 4) return TDVP_E_SHAPE;
    const auto phases = seg_schedule1(std::vector<int>(seg_sizes, seg_sizes + nseg), dt, first_half != 0);
    int n = 0;
    for (size_t p = 0; p < phases.size(); ++p)
        for (const auto& op : phases[p]) {
            if (n < max_ops && phase && kind && site && tau) {
                phase[n] = (int)p;
                kind[n] = op.bond ? (op.refresh == 1 ? 3 : 4) : (op.pair ? 2 : 1);
                site[n] = op.j;
                tau[n] = op.tau;
            }
            ++n;
        }
    *n_out = n;
    return n <= max_ops ? TDVP_OK : TDVP_E_SHAPE;
}

int seg_destroy(tdvp_seg sg) {
    if (!sg) return TDVP_E_ARG;
    (void)hipStreamSynchronize(sg->ctx->stream);
    delete sg;
    return TDVP_OK;
}

}  // extern "C"
