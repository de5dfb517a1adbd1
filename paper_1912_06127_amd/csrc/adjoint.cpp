// Adjoint of the effective-Hamiltonian application (reverse mode).
//
// y = H_eff theta is linear in theta, in L, in R and in each MPO tensor.  For
// a real loss with gradients in the convention g = dl/dRe z + i dl/dIm z
// (so dl = Re sum conj(g) dz), the gradient of a linear map y = A x with
// respect to x is A^dagger ybar, and with respect to a factor F it is the
// contraction of ybar with the conjugate of everything else:
//   theta_bar = H_eff^dagger ybar  (L^dagger, the physical adjoint of W, R^dagger)
//   L_bar[k][a'][a] = sum ybar[a' s' b'] conj((W R theta)[k][a][s'][b'])
//   R_bar[n][b][b'] = sum conj((L W theta)[a' s'][n][b]) ybar[a' s' b']
//   W_bar[k][l][s'][s] = sum conj((L theta)[k][a'][s][b]) (ybar R^dagger)[l][a'][s'][b]
// Each is a GEMM -> sparse MPO stage -> GEMM pipeline like the forward
// application, so the same kernels run it.
#include "internal.hpp"

namespace tdvp {

namespace {

GemmOperand opnd(const void* p, Dt dt, int64_t ld, bool kcontig, bool conj = false, int64_t stride = 0) {
    GemmOperand o;
    o.p = p;
    o.dt = dt;
    o.ld = ld;
    o.kcontig = kcontig;
    o.conj = conj;
    o.stride = stride;
    return o;
}

}  // namespace

struct AdjointArgs {
    int nsite, chil, chir, d, wl, wm, wr;
    const void *L, *W1, *W2, *R, *theta, *ybar;
    void *theta_bar, *L_bar, *W1_bar, *R_bar;
    Dt dt;
};

void heff_adjoint(tdvp_ctx ctx, const AdjointArgs& a) {
    const bool fp64 = a.dt == Dt::C128;
    const int form = raw_gemm_form(ctx, fp64);
    const int D = a.nsite == 0 ? 1 : (a.nsite == 1 ? a.d : a.d * a.d);
    const size_t esz = elem_bytes(a.dt);
    const int64_t chil = a.chil, chir = a.chir;
    const int wm = a.nsite == 2 ? a.wm : a.wl;

    if (a.theta_bar) {
        void* LH = ctx->workspace("adj_LH", esz * (size_t)a.wl * chil * chil);
        void* RH = ctx->workspace("adj_RH", esz * (size_t)a.wr * chir * chir);
        conj_transpose_batched(LH, a.L, a.dt, a.chil, a.wl, ctx->stream);
        conj_transpose_batched(RH, a.R, a.dt, a.chir, a.wr, ctx->stream);
        Mop m;
        mop_make(ctx, m, a.nsite == 0 ? 0 : (a.nsite == 1 ? 4 : 5), a.W1, a.W2, a.dt, a.wl, wm, a.wr, a.d, fp64, false);
        HeffArgs h{a.nsite, a.chil, a.chir, a.d, a.wl, a.wr, LH, RH, a.dt, &m, fp64, form};
        heff_apply(ctx, h, a.ybar, a.dt, a.theta_bar, a.dt);
    }

    if (a.L_bar) {
        // U[(a s)][n][b'] = sum_b theta[(a s)][b] R[n][b][b']
        void* U = ctx->workspace("adj_U", esz * (size_t)a.wr * chil * D * chir);
        GemmDesc g1;
        g1.M = (int)(chil * D);
        g1.N = (int)chir;
        g1.K = (int)chir;
        g1.batch = a.wr;
        g1.A = opnd(a.theta, a.dt, chir, true);
        g1.B = opnd(a.R, a.dt, chir, false, false, chir * chir);
        g1.C = U;
        g1.cdt = a.dt;
        g1.ldc = a.wr * chir;
        g1.strideC = chir;
        cgemm(ctx, g1, fp64, form);
        // X[k][a][s'][b'] = sum_{n,s} W[(k s'),(n s)] U[a][s][n][b']
        Mop m;
        mop_make(ctx, m, a.nsite == 0 ? 0 : (a.nsite == 1 ? 3 : 6), a.W1, a.W2, a.dt, a.wl, wm, a.wr, a.d, fp64, false);
        void* X = ctx->workspace("adj_X", esz * (size_t)a.wl * chil * D * chir);
        WStageDesc w;
        w.in = U;
        w.in_dt = a.dt;
        w.out = X;
        w.out_dt = a.dt;
        w.P = (int)chil;
        w.Q = (int)chir;
        w.D = D;
        w.w_in = a.wr;
        w.w_out = a.wl;
        w.ik = chir;
        w.is = a.wr * chir;
        w.ip = (int64_t)D * a.wr * chir;
        w.on = chil * D * chir;
        w.os = chir;
        w.op = D * chir;
        w.row_ptr = m.row_ptr;
        w.col = m.col;
        w.val = m.val;
        w.fp64 = fp64;
        wstage(ctx, w);
        // L_bar[k][a'][a] = sum_{(s' b')} ybar[a'][(s' b')] conj(X[k][a][(s' b')])
        GemmDesc g2;
        g2.M = (int)chil;
        g2.N = (int)chil;
        g2.K = (int)(D * chir);
        g2.batch = a.wl;
        g2.A = opnd(a.ybar, a.dt, D * chir, true);
        g2.B = opnd(X, a.dt, D * chir, true, true, chil * D * chir);
        g2.C = a.L_bar;
        g2.cdt = a.dt;
        g2.ldc = chil;
        g2.strideC = chil * chil;
        cgemm(ctx, g2, fp64, form);
    }

    if (a.R_bar || a.W1_bar) {
        // T1[(k a')][(s b)] = sum_a L[k][a'][a] theta[a][(s b)]
        void* T1 = ctx->workspace("adj_T1", esz * (size_t)a.wl * chil * D * chir);
        GemmDesc g1;
        g1.M = (int)(a.wl * chil);
        g1.N = (int)(D * chir);
        g1.K = (int)chil;
        g1.A = opnd(a.L, a.dt, chil, true);
        g1.B = opnd(a.theta, a.dt, D * chir, false);
        g1.C = T1;
        g1.cdt = a.dt;
        g1.ldc = D * chir;
        cgemm(ctx, g1, fp64, form);
        if (a.R_bar) {
            // T3[a'][s'][n][b] = sum_{k,s} W[(n s'),(k s)] T1[k][a'][s][b]
            Mop m;
            mop_make(ctx, m, a.nsite == 0 ? 0 : (a.nsite == 1 ? 1 : 2), a.W1, a.W2, a.dt, a.wl, wm, a.wr, a.d, fp64,
                     false);
            void* T3 = ctx->workspace("adj_T3", esz * (size_t)a.wr * chil * D * chir);
            WStageDesc w;
            w.in = T1;
            w.in_dt = a.dt;
            w.out = T3;
            w.out_dt = a.dt;
            w.P = (int)chil;
            w.Q = (int)chir;
            w.D = D;
            w.w_in = a.wl;
            w.w_out = a.wr;
            w.ik = chil * D * chir;
            w.is = chir;
            w.ip = D * chir;
            w.on = chir;
            w.os = a.wr * chir;
            w.op = (int64_t)D * a.wr * chir;
            w.row_ptr = m.row_ptr;
            w.col = m.col;
            w.val = m.val;
            w.fp64 = fp64;
            wstage(ctx, w);
            // R_bar[n][b][b'] = sum_{(a' s')} conj(T3[(a' s')][n][b]) ybar[(a' s')][b']
            GemmDesc g2;
            g2.M = (int)chir;
            g2.N = (int)chir;
            g2.K = (int)(chil * D);
            g2.batch = a.wr;
            g2.A = opnd(T3, a.dt, a.wr * chir, false, true, chir);
            g2.B = opnd(a.ybar, a.dt, chir, false);
            g2.C = a.R_bar;
            g2.cdt = a.dt;
            g2.ldc = chir;
            g2.strideC = chir * chir;
            cgemm(ctx, g2, fp64, form);
        }
        if (a.W1_bar) {
            // Z[l][a'][s'][b] = sum_{b'} ybar[(a' s')][b'] conj(R[l][b][b'])
            void* Z = ctx->workspace("adj_Z", esz * (size_t)a.wr * chil * D * chir);
            GemmDesc g3;
            g3.M = (int)(chil * D);
            g3.N = (int)chir;
            g3.K = (int)chir;
            g3.batch = a.wr;
            g3.A = opnd(a.ybar, a.dt, chir, true);
            g3.B = opnd(a.R, a.dt, chir, true, true, chir * chir);
            g3.C = Z;
            g3.cdt = a.dt;
            g3.ldc = chir;
            g3.strideC = chil * D * chir;
            cgemm(ctx, g3, fp64, form);
            wgrad(T1, Z, a.dt, a.wl, a.wr, a.d, a.chil, a.chir, a.W1_bar, ctx->stream);
        }
    }
}

// Adjoint of the environment update (Sec. III A, Fig. environments).  Left:
// L'[l][b'][b] = sum conj(A[a' s' b']) L[k][a'][a] W[k][l][s'][s] A[a s b];
// right: R'[k][a][a'] = sum A[a s b] W[k][l][s'][s] R[l][b][b'] conj(A[a' s' b']).
// Given out_bar = the gradient of R' (or L'), with Hb the blockwise conjugate
// transpose of out_bar and H = the one-site effective Hamiltonian built from
// (L, W, Hb) (left) or (Hb, W, R) (right):
//   env_bar = the opposite-direction update of out_bar with the blockwise
//             conjugate transpose of W (the map is linear in the environment),
//   A_bar   = H^dagger A + H A  (A enters once as ket, once conjugated as bra),
//   W_bar   = the MPO-tensor gradient of Re<A, H A>.
void env_adjoint(tdvp_ctx ctx, int dir, Dt dt, int chil, int chir, int d, int wl, int wr, const void* env_in,
                 const void* A, const void* W, const void* out_bar, void* env_bar, void* A_bar, void* W_bar) {
    const bool fp64 = dt == Dt::C128;
    const size_t esz = elem_bytes(dt);
    if (env_bar) {
        void* WH = ctx->workspace("envadj_WH", esz * (size_t)wl * wr * d * d);
        conj_transpose_batched(WH, W, dt, d, wl * wr, ctx->stream);
        Mop m;
        mop_make(ctx, m, dir == 1 ? 3 : 1, WH, nullptr, dt, wl, wl, wr, d, fp64, false);
        EnvArgs a{chil, chir, chil, chir, d, wl, wr, A, A, dt, &m, fp64, raw_gemm_form(ctx, fp64)};
        if (dir == 1) env_right(ctx, a, out_bar, dt, env_bar, dt);
        else env_left(ctx, a, out_bar, dt, env_bar, dt);
    }
    if (!A_bar && !W_bar) return;
    const int wo = dir == 1 ? wr : wl, co = dir == 1 ? chir : chil;
    void* Hb = ctx->workspace("envadj_Hb", esz * (size_t)wo * co * co);
    conj_transpose_batched(Hb, out_bar, dt, co, wo, ctx->stream);
    const void* Luse = dir == 1 ? env_in : Hb;
    const void* Ruse = dir == 1 ? Hb : env_in;
    AdjointArgs g{1, chil, chir, d, wl, wl, wr, Luse, W, nullptr, Ruse, A, A, A_bar, nullptr, W_bar, nullptr, dt};
    heff_adjoint(ctx, g);  // A_bar = H^dagger A, W_bar
    if (A_bar) {
        const int64_t n = (int64_t)chil * d * chir;
        void* HA = ctx->workspace("envadj_HA", esz * (size_t)n);
        Mop m;
        mop_make(ctx, m, 1, W, nullptr, dt, wl, wl, wr, d, fp64, false);
        HeffArgs h{1, chil, chir, d, wl, wr, Luse, Ruse, dt, &m, fp64, raw_gemm_form(ctx, fp64)};
        heff_apply(ctx, h, A, dt, HA, dt);
        add_inplace(A_bar, HA, dt, n, ctx->stream);
    }
}

}  // namespace tdvp

using namespace tdvp;

extern "C" {

int env_update_adjoint(tdvp_ctx ctx, int dir, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wr,
                       const void* env_in, const void* A, const void* W, const void* out_bar, void* env_bar,
                       void* A_bar, void* W_bar) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        const Dt dt = to_dt(dtype);
        TDVP_REQUIRE(dir == 1 || dir == -1, TDVP_E_ARG, "env_update_adjoint: dir must be +1 or -1");
        TDVP_REQUIRE(chil >= 1 && chir >= 1 && d >= 1 && wl >= 1 && wr >= 1, TDVP_E_SHAPE,
                     "env_update_adjoint: dimensions must be positive");
        TDVP_REQUIRE(env_in && A && W && out_bar, TDVP_E_ARG, "env_update_adjoint: null input");
        const void* ins[] = {env_in, A, W, out_bar};
        void* outs[] = {env_bar, A_bar, W_bar};
        for (void* o : outs)
            for (const void* i : ins)
                TDVP_REQUIRE(!o || o != i, TDVP_E_ARG, "env_update_adjoint: an output aliases an input");
        env_adjoint(ctx, dir, dt, chil, chir, d, wl, wr, env_in, A, W, out_bar, env_bar, A_bar, W_bar);
    });
}


int apply_heff_adjoint(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm,
                       int wr, const void* L, const void* W1, const void* W2, const void* R, const void* theta,
                       const void* ybar, void* theta_bar, void* L_bar, void* W1_bar, void* W2_bar, void* R_bar) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        const Dt dt = to_dt(dtype);
        TDVP_REQUIRE(nsite >= 0 && nsite <= 2, TDVP_E_ARG, "apply_heff_adjoint: nsite must be 0, 1 or 2");
        TDVP_REQUIRE(chil >= 1 && chir >= 1 && wl >= 1 && wr >= 1, TDVP_E_SHAPE,
                     "apply_heff_adjoint: dimensions must be positive");
        TDVP_REQUIRE(nsite == 0 || d >= 1, TDVP_E_SHAPE, "apply_heff_adjoint: d must be positive");
        TDVP_REQUIRE(nsite != 2 || wm >= 1, TDVP_E_SHAPE, "apply_heff_adjoint: wm must be positive");
        TDVP_REQUIRE(nsite != 0 || wl == wr, TDVP_E_SHAPE, "apply_heff_adjoint: zero-site needs wl == wr");
        TDVP_REQUIRE(L && R && theta && ybar, TDVP_E_ARG, "apply_heff_adjoint: null input");
        TDVP_REQUIRE(nsite < 1 || W1, TDVP_E_ARG, "apply_heff_adjoint: W1 is null");
        TDVP_REQUIRE(nsite < 2 || W2, TDVP_E_ARG, "apply_heff_adjoint: W2 is null");
        TDVP_REQUIRE(!W2_bar && (nsite == 1 || !W1_bar), TDVP_E_ARG,
                     "apply_heff_adjoint: MPO-tensor gradients are provided for nsite = 1 only");
        const void* ins[] = {L, W1, W2, R, theta, ybar};
        void* outs[] = {theta_bar, L_bar, W1_bar, R_bar};
        for (void* o : outs)
            for (const void* i : ins)
                TDVP_REQUIRE(!o || o != i, TDVP_E_ARG, "apply_heff_adjoint: an output aliases an input");
        AdjointArgs a{nsite, chil, chir, d, wl, wm, wr, L, W1, W2, R, theta, ybar, theta_bar, L_bar, W1_bar, R_bar, dt};
        heff_adjoint(ctx, a);
    });
}

}  // extern "C"
