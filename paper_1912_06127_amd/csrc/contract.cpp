// Effective-Hamiltonian application and environment updates as
// GEMM -> sparse MPO stage -> GEMM pipelines (Sec. III A, Fig. update and the
// left-environment figure; cost Eq. eqnscaling).
#include "internal.hpp"

namespace tdvp {

namespace {

GemmOperand op(const void* p, Dt dt, int64_t ld, bool kcontig, bool conj = false, int64_t stride = 0) {
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

// Complex-GEMM form of the raw-pointer entry points (tdvp_ctx_set_gemm_form).
int raw_gemm_form(tdvp_ctx ctx, bool fp64) {
    if (fp64) return 4;
    return ctx->gemm_form == 0 ? 3 : ctx->gemm_form;
}

namespace {

int pow_int(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

}  // namespace

void mop_make(tdvp_ctx ctx, Mop& m, int kind, const void* W1, const void* W2, Dt w_dt, int wl,
              int wm, int wr, int d, bool fp64, bool own) {
    int rows, cols;
    switch (kind) {
        case 0: rows = wl; cols = wl; break;
        case 1: case 4: rows = wr * d; cols = wl * d; break;
        case 2: case 5: rows = wr * d * d; cols = wl * d * d; break;
        case 3: rows = wl * d; cols = wr * d; break;
        case 6: rows = wl * d * d; cols = wr * d * d; break;
        default: throw Error(TDVP_E_ARG, "mop_make: bad kind");
    }
    const size_t nz = (size_t)rows * cols;
    const size_t vsz = fp64 ? sizeof(double2) : sizeof(float2);
    m.rows = rows;
    m.cols = cols;
    m.fp64 = fp64;
    int* rp;
    int* col;
    void* val;
    if (own) {
        m.own_rp = DevMem(ctx, sizeof(int) * (rows + 1));
        m.own_col = DevMem(ctx, sizeof(int) * nz);
        m.own_val = DevMem(ctx, vsz * nz);
        rp = m.own_rp.as<int>();
        col = m.own_col.as<int>();
        val = m.own_val.ptr;
    } else {
        rp = static_cast<int*>(ctx->workspace("mop_rp", sizeof(int) * (rows + 1)));
        col = static_cast<int*>(ctx->workspace("mop_col", sizeof(int) * nz));
        val = ctx->workspace("mop_val", vsz * nz);
    }
    double2* dense = static_cast<double2*>(ctx->workspace("mop_dense", sizeof(double2) * nz));
    mop_build(kind, W1, w_dt, W2, w_dt, wl, wm, wr, d, rows, cols, dense, rp, col, val, fp64, ctx->stream);
    m.row_ptr = rp;
    m.col = col;
    m.val = val;
}

double heff_flops(int nsite, int chil, int chir, int d, int wl, int wr) {
    const double D = nsite == 0 ? 1.0 : (double)pow_int(d, nsite);
    const double w = std::max(wl, wr);
    double f = 8.0 * wl * chil * (double)chil * D * chir + 8.0 * wr * chil * D * (double)chir * chir;
    if (nsite == 1) f += 8.0 * w * w * d * d * (double)chil * chir;
    if (nsite == 2) f += 16.0 * w * w * d * d * d * (double)chil * chir;
    return f;
}

double env_flops(int chil, int chir, int d, int wl, int wr) {
    const double w = std::max(wl, wr);
    return 8.0 * wl * chil * (double)chil * d * chir + 8.0 * wr * chir * (double)chil * d * chir +
           8.0 * w * w * d * d * (double)chil * chir;
}

void heff_apply(tdvp_ctx ctx, const HeffArgs& a, const void* x, Dt x_dt, void* y, Dt y_dt) {
    const int D = a.nsite == 0 ? 1 : pow_int(a.d, a.nsite);
    const Dt cdt = a.fp64 ? Dt::C128 : Dt::C64;
    const int64_t chil = a.chil, chir = a.chir;
    TDVP_REQUIRE(a.mop && a.mop->rows == a.wr * D && a.mop->cols == a.wl * D, TDVP_E_SHAPE,
                 "heff: MPO stage operator does not match the bond dimensions");
    const size_t xbytes = elem_bytes(x_dt) * (size_t)chil * D * chir;
    const size_t ybytes = elem_bytes(y_dt) * (size_t)chil * D * chir;
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    const bool overlap = xb < yb + ybytes && yb < xb + xbytes;
    const bool env_native = (a.env_dt == Dt::C128) == a.fp64;
    if (!overlap && env_native && heff_small_fits(a.chil, a.chir, D, a.wl, a.wr, a.fp64)) {
        HeffSmallDesc h;
        h.L = a.L; h.L_dt = a.env_dt;
        h.R = a.R; h.R_dt = a.env_dt;
        h.x = x; h.x_dt = x_dt;
        h.y = y; h.y_dt = y_dt;
        h.row_ptr = a.mop->row_ptr;
        h.col = a.mop->col;
        h.val = a.mop->val;
        h.chil = a.chil; h.chir = a.chir; h.D = D; h.wl = a.wl; h.wr = a.wr;
        h.fp64 = a.fp64;
        h.flops = heff_flops(a.nsite, a.chil, a.chir, a.d, a.wl, a.wr);
        heff_small(ctx, h);
        return;
    }
    void* T1 = ctx->workspace("heff_T1", elem_bytes(cdt) * (size_t)a.wl * chil * D * chir);
    void* T3 = ctx->workspace("heff_T3", elem_bytes(cdt) * (size_t)a.wr * chil * D * chir);

    // Stage A: T1[(k a')][(s b)] = sum_a L[k][a'][a] x[a][(s b)]
    GemmDesc g1;
    g1.M = (int)(a.wl * chil);
    g1.N = (int)(D * chir);
    g1.K = (int)chil;
    g1.A = op(a.L, a.env_dt, chil, true);
    g1.B = op(x, x_dt, D * chir, false);
    g1.C = T1;
    g1.cdt = cdt;
    g1.ldc = D * chir;
    cgemm(ctx, g1, a.fp64, a.form);

    // MPO stage: T3[a'][s'][n][b] = sum_{k,s} M[(n,s'),(k,s)] T1[k][a'][s][b]
    WStageDesc w;
    w.in = T1;
    w.in_dt = cdt;
    w.out = T3;
    w.out_dt = cdt;
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
    w.row_ptr = a.mop->row_ptr;
    w.col = a.mop->col;
    w.val = a.mop->val;
    w.fp64 = a.fp64;
    wstage(ctx, w);

    // Stage B: y[(a' s')][b'] = sum_{(n b)} T3[(a' s')][(n b)] R[(n b)][b']
    GemmDesc g2;
    g2.M = (int)(chil * D);
    g2.N = (int)chir;
    g2.K = (int)(a.wr * chir);
    g2.A = op(T3, cdt, a.wr * chir, true);
    g2.B = op(a.R, a.env_dt, chir, false);
    g2.C = y;
    g2.cdt = y_dt;
    g2.ldc = chir;
    cgemm(ctx, g2, a.fp64, a.form);
}

void env_left(tdvp_ctx ctx, const EnvArgs& a, const void* L, Dt l_dt, void* out, Dt out_dt) {
    const Dt cdt = a.fp64 ? Dt::C128 : Dt::C64;
    const int64_t d = a.d;
    const int64_t chil = a.chil, chir = a.chir, chilb = a.chil_b, chirb = a.chir_b;
    TDVP_REQUIRE(a.mop && a.mop->rows == a.wr * a.d && a.mop->cols == a.wl * a.d, TDVP_E_SHAPE,
                 "env_left: MPO stage operator does not match");
    void* X = ctx->workspace("env_X", elem_bytes(cdt) * (size_t)a.wl * chilb * d * chir);
    void* Y = ctx->workspace("env_Y", elem_bytes(cdt) * (size_t)a.wr * chilb * d * chir);

    // X[(k a')][(s b)] = sum_a L[k][a'][a] Aket[a][(s b)]
    GemmDesc g1;
    g1.M = (int)(a.wl * chilb);
    g1.N = (int)(d * chir);
    g1.K = (int)chil;
    g1.A = op(L, l_dt, chil, true);
    g1.B = op(a.Aket, a.a_dt, d * chir, false);
    g1.C = X;
    g1.cdt = cdt;
    g1.ldc = d * chir;
    cgemm(ctx, g1, a.fp64, a.form);

    // Y[l][a'][s'][b] = sum_{k,s} W[k][l][s'][s] X[k][a'][s][b]
    WStageDesc w;
    w.in = X;
    w.in_dt = cdt;
    w.out = Y;
    w.out_dt = cdt;
    w.P = (int)chilb;
    w.Q = (int)chir;
    w.D = a.d;
    w.w_in = a.wl;
    w.w_out = a.wr;
    w.ik = chilb * d * chir;
    w.is = chir;
    w.ip = d * chir;
    w.on = chilb * d * chir;
    w.os = chir;
    w.op = d * chir;
    w.row_ptr = a.mop->row_ptr;
    w.col = a.mop->col;
    w.val = a.mop->val;
    w.fp64 = a.fp64;
    wstage(ctx, w);

    // out[l][b'][b] = sum_{(a' s')} conj(Abra[(a' s')][b']) Y[l][(a' s')][b]
    GemmDesc g2;
    g2.M = (int)chirb;
    g2.N = (int)chir;
    g2.K = (int)(chilb * d);
    g2.batch = a.wr;
    g2.A = op(a.Abra, a.a_dt, chirb, false, true, 0);
    g2.B = op(Y, cdt, chir, false, false, chilb * d * chir);
    g2.C = out;
    g2.cdt = out_dt;
    g2.ldc = chir;
    g2.strideC = chirb * chir;
    cgemm(ctx, g2, a.fp64, a.form);
}

void env_right(tdvp_ctx ctx, const EnvArgs& a, const void* R, Dt r_dt, void* out, Dt out_dt) {
    const Dt cdt = a.fp64 ? Dt::C128 : Dt::C64;
    const int64_t d = a.d;
    const int64_t chil = a.chil, chir = a.chir, chilb = a.chil_b, chirb = a.chir_b;
    TDVP_REQUIRE(a.mop && a.mop->rows == a.wl * a.d && a.mop->cols == a.wr * a.d, TDVP_E_SHAPE,
                 "env_right: MPO stage operator does not match");
    void* U = ctx->workspace("env_X", elem_bytes(cdt) * (size_t)a.wr * chil * d * chirb);
    void* V = ctx->workspace("env_Y", elem_bytes(cdt) * (size_t)a.wl * chil * d * chirb);

    // U[(a s)][l][b'] = sum_b Aket[(a s)][b] R[l][b][b']    (batched over l)
    GemmDesc g1;
    g1.M = (int)(chil * d);
    g1.N = (int)chirb;
    g1.K = (int)chir;
    g1.batch = a.wr;
    g1.A = op(a.Aket, a.a_dt, chir, true, false, 0);
    g1.B = op(R, r_dt, chirb, false, false, chir * chirb);
    g1.C = U;
    g1.cdt = cdt;
    g1.ldc = a.wr * chirb;
    g1.strideC = chirb;
    cgemm(ctx, g1, a.fp64, a.form);

    // V[k][a][s'][b'] = sum_{l,s} W[k][l][s'][s] U[a][s][l][b']
    WStageDesc w;
    w.in = U;
    w.in_dt = cdt;
    w.out = V;
    w.out_dt = cdt;
    w.P = (int)chil;
    w.Q = (int)chirb;
    w.D = a.d;
    w.w_in = a.wr;
    w.w_out = a.wl;
    w.ik = chirb;
    w.is = a.wr * chirb;
    w.ip = d * a.wr * chirb;
    w.on = chil * d * chirb;
    w.os = chirb;
    w.op = d * chirb;
    w.row_ptr = a.mop->row_ptr;
    w.col = a.mop->col;
    w.val = a.mop->val;
    w.fp64 = a.fp64;
    wstage(ctx, w);

    // out[(k a)][a'] = sum_{(s' b')} V[(k a)][(s' b')] conj(Abra[a'][(s' b')])
    GemmDesc g2;
    g2.M = (int)(a.wl * chil);
    g2.N = (int)chilb;
    g2.K = (int)(d * chirb);
    g2.A = op(V, cdt, d * chirb, true);
    g2.B = op(a.Abra, a.a_dt, d * chirb, true, true);
    g2.C = out;
    g2.cdt = out_dt;
    g2.ldc = chilb;
    cgemm(ctx, g2, a.fp64, a.form);
}

}  // namespace tdvp

using namespace tdvp;

namespace tdvp {

// Argument checks, MPO-stage operator and pipeline of the raw-pointer
// H_eff call (shared by apply_heff and apply_heff_noalloc).
void heff_raw_call(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm, int wr,
                   const void* L, const void* W1, const void* W2, const void* R, const void* theta, void* out) {
    const Dt dt = to_dt(dtype);
    TDVP_REQUIRE(nsite >= 0 && nsite <= 2, TDVP_E_ARG, "apply_heff: nsite must be 0, 1 or 2");
    TDVP_REQUIRE(chil >= 1 && chir >= 1 && wl >= 1 && wr >= 1, TDVP_E_SHAPE,
                 "apply_heff: dimensions must be positive");
    TDVP_REQUIRE(nsite == 0 || d >= 1, TDVP_E_SHAPE, "apply_heff: d must be positive");
    TDVP_REQUIRE(nsite != 2 || wm >= 1, TDVP_E_SHAPE, "apply_heff: wm must be positive");
    TDVP_REQUIRE(nsite != 0 || wl == wr, TDVP_E_SHAPE, "apply_heff: zero-site needs wl == wr");
    TDVP_REQUIRE(L && R && theta && out, TDVP_E_ARG, "apply_heff: null pointer");
    TDVP_REQUIRE(nsite < 1 || W1, TDVP_E_ARG, "apply_heff: W1 is null");
    TDVP_REQUIRE(nsite < 2 || W2, TDVP_E_ARG, "apply_heff: W2 is null");
    TDVP_REQUIRE(out != theta && out != L && out != R, TDVP_E_ARG, "apply_heff: out aliases an input");
    const bool fp64 = dt == Dt::C128;
    Mop m;
    const int kind = nsite == 0 ? 0 : (nsite == 1 ? 1 : 2);
    mop_make(ctx, m, kind, W1, W2, dt, wl, nsite == 2 ? wm : wl, wr, d, fp64, false);
    HeffArgs a{nsite, chil, chir, d, wl, wr, L, R, dt, &m, fp64, raw_gemm_form(ctx, fp64)};
    heff_apply(ctx, a, theta, dt, out, dt);
}

}  // namespace tdvp

extern "C" {

int apply_heff(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm,
               int wr, const void* L, const void* W1, const void* W2, const void* R,
               const void* theta, void* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TxRange tx("apply_heff");
        heff_raw_call(ctx, nsite, dtype, chil, chir, d, wl, wm, wr, L, W1, W2, R, theta, out);
    });
}

int apply_heff_batched(tdvp_ctx ctx, tdvp_dtype dtype, int n, const tdvp_heff_desc* descs) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        const Dt dt = to_dt(dtype);
        TDVP_REQUIRE(n >= 0 && (n == 0 || descs), TDVP_E_ARG, "apply_heff_batched: null descriptor array");
        if (n == 0) return;
        const bool fp64 = dt == Dt::C128;
        const size_t esz = elem_bytes(dt);
        std::vector<Mop> mops(n);
        std::vector<int64_t> o1(n), o3(n);
        int64_t t1 = 0, t3 = 0;
        for (int i = 0; i < n; ++i) {
            const tdvp_heff_desc& q = descs[i];
            TDVP_REQUIRE(q.nsite >= 0 && q.nsite <= 2, TDVP_E_ARG, "apply_heff_batched: nsite must be 0, 1 or 2");
            TDVP_REQUIRE(q.chil >= 1 && q.chir >= 1 && q.wl >= 1 && q.wr >= 1, TDVP_E_SHAPE,
                         "apply_heff_batched: dimensions must be positive");
            TDVP_REQUIRE(q.nsite == 0 || q.d >= 1, TDVP_E_SHAPE, "apply_heff_batched: d must be positive");
            TDVP_REQUIRE(q.nsite != 2 || q.wm >= 1, TDVP_E_SHAPE, "apply_heff_batched: wm must be positive");
            TDVP_REQUIRE(q.nsite != 0 || q.wl == q.wr, TDVP_E_SHAPE, "apply_heff_batched: zero-site needs wl == wr");
            TDVP_REQUIRE(q.L && q.R && q.theta && q.out, TDVP_E_ARG, "apply_heff_batched: null pointer");
            TDVP_REQUIRE(q.nsite < 1 || q.W1, TDVP_E_ARG, "apply_heff_batched: W1 is null");
            TDVP_REQUIRE(q.nsite < 2 || q.W2, TDVP_E_ARG, "apply_heff_batched: W2 is null");
            for (int k = 0; k < n; ++k)
                TDVP_REQUIRE(q.out != descs[k].theta && q.out != descs[k].L && q.out != descs[k].R &&
                                 (k == i || q.out != descs[k].out),
                             TDVP_E_ARG, "apply_heff_batched: an output aliases an input or another output");
            const int kind = q.nsite == 0 ? 0 : (q.nsite == 1 ? 1 : 2);
            mop_make(ctx, mops[i], kind, q.W1, q.W2, dt, q.wl, q.nsite == 2 ? q.wm : q.wl, q.wr, q.d, fp64, true);
            const int64_t D = q.nsite == 0 ? 1 : pow_int(q.d, q.nsite);
            o1[i] = t1;
            o3[i] = t3;
            t1 += (int64_t)q.wl * q.chil * D * q.chir;
            t3 += (int64_t)q.wr * q.chil * D * q.chir;
        }
        char* T1 = static_cast<char*>(ctx->workspace("heffb_T1", esz * (size_t)t1));
        char* T3 = static_cast<char*>(ctx->workspace("heffb_T3", esz * (size_t)t3));
        std::vector<GemmDesc> ga(n), gb(n);
        std::vector<WStageDesc> ws(n);
        for (int i = 0; i < n; ++i) {
            const tdvp_heff_desc& q = descs[i];
            const int64_t D = q.nsite == 0 ? 1 : pow_int(q.d, q.nsite);
            const int64_t chil = q.chil, chir = q.chir;
            GemmDesc& g1 = ga[i];  // T1[(k a')][(s b)] = L x
            g1.M = (int)(q.wl * chil);
            g1.N = (int)(D * chir);
            g1.K = (int)chil;
            g1.A = op(q.L, dt, chil, true);
            g1.B = op(q.theta, dt, D * chir, false);
            g1.C = T1 + esz * o1[i];
            g1.cdt = dt;
            g1.ldc = D * chir;
            WStageDesc& w = ws[i];
            w.in = T1 + esz * o1[i]; w.in_dt = dt; w.out = T3 + esz * o3[i]; w.out_dt = dt;
            w.P = (int)chil; w.Q = (int)chir; w.D = (int)D; w.w_in = q.wl; w.w_out = q.wr;
            w.ik = chil * D * chir; w.is = chir; w.ip = D * chir;
            w.on = chir; w.os = q.wr * chir; w.op = D * q.wr * chir;
            w.row_ptr = mops[i].row_ptr; w.col = mops[i].col; w.val = mops[i].val; w.fp64 = fp64;
            GemmDesc& g2 = gb[i];  // y[(a' s')][b'] = T3 R
            g2.M = (int)(chil * D);
            g2.N = (int)chir;
            g2.K = (int)(q.wr * chir);
            g2.A = op(T3 + esz * o3[i], dt, q.wr * chir, true);
            g2.B = op(q.R, dt, chir, false);
            g2.C = q.out;
            g2.cdt = dt;
            g2.ldc = chir;
        }
        GroupedGemm A, B;
        GroupedWStage W;
        grouped_gemm_plan(ctx, ga, fp64, raw_gemm_form(ctx, fp64), A);
        grouped_wstage_plan(ctx, ws, W);
        grouped_gemm_plan(ctx, gb, fp64, raw_gemm_form(ctx, fp64), B);
        grouped_gemm_run(ctx, A);
        grouped_wstage_run(ctx, W);
        grouped_gemm_run(ctx, B);
        // the plans' tables and the operators are freed on return
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int env_update(tdvp_ctx ctx, int dir, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wr,
               const void* env_in, const void* A, const void* W, void* env_out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TxRange tx("env_update");
        const Dt dt = to_dt(dtype);
        TDVP_REQUIRE(dir == 1 || dir == -1, TDVP_E_ARG, "env_update: dir must be +1 or -1");
        TDVP_REQUIRE(chil >= 1 && chir >= 1 && d >= 1 && wl >= 1 && wr >= 1, TDVP_E_SHAPE,
                     "env_update: dimensions must be positive");
        TDVP_REQUIRE(env_in && A && W && env_out, TDVP_E_ARG, "env_update: null pointer");
        TDVP_REQUIRE(env_out != env_in && env_out != A, TDVP_E_ARG, "env_update: out aliases an input");
        const bool fp64 = dt == Dt::C128;
        Mop m;
        mop_make(ctx, m, dir == 1 ? 1 : 3, W, nullptr, dt, wl, wl, wr, d, fp64, false);
        EnvArgs a{chil, chir, chil, chir, d, wl, wr, A, A, dt, &m, fp64, raw_gemm_form(ctx, fp64)};
        if (dir == 1) env_left(ctx, a, env_in, dt, env_out, dt);
        else env_right(ctx, a, env_in, dt, env_out, dt);
    });
}

}  // extern "C"
