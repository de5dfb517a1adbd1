// U(1) block-sparse effective-Hamiltonian application and environment
// updates (quantum-number blocks).
//
// The XY and XXX chains of Sec. IV conserve the total S^z, and the paper's
// largest runs store every tensor in charge blocks (Supplemental Material,
// Implementation).  Here the tensors keep the dense layouts of the other
// entry points; bond indices are sorted by charge, so every charge sector is
// a contiguous index range, and only the blocks the charge rules allow are
// computed:
//   site / local state  T[a][s][b]      q(a) + q(s) = q(b)
//   MPO                 W[k][l][s'][s]   c(l) = c(k) + q(s') - q(s)
//   left environment    L[k][a'][a]      q(a') - q(a) = c(k)
//   right environment   R[l][b][b']      q(b') - q(b) = c(l)
// Each GEMM stage of the dense pipeline becomes one launch of block
// products (block_gemm): stage A one product per (run of equal MPO charges,
// left sector, physical index), batched over the run; stage B one output
// block per (left sector, physical index) accumulated over K chunks, one per
// run of MPO charges; the sparse MPO stage runs only on the (left sector,
// right sector) rectangles whose charge difference some MPO term can
// produce.  Entries outside the allowed blocks are zero in the outputs and
// are never read from the inputs.
#include "internal.hpp"

#include <algorithm>
#include <vector>

namespace tdvp {
namespace {

struct Sector {
    int q, off, n;
};
struct Run {
    int c, i0, n;
};

std::vector<Sector> sectors_of(const int* q, int n, const char* what) {
    std::vector<Sector> s;
    for (int i = 0; i < n;) {
        int j = i;
        while (j < n && q[j] == q[i]) ++j;
        TDVP_REQUIRE(j == n || q[j] > q[i], TDVP_E_ARG, std::string(what) + ": charge labels must be non-decreasing");
        s.push_back({q[i], i, j - i});
        i = j;
    }
    return s;
}

std::vector<Run> runs_of(const int* c, int n) {
    std::vector<Run> r;
    for (int i = 0; i < n;) {
        int j = i;
        while (j < n && c[j] == c[i]) ++j;
        r.push_back({c[i], i, j - i});
        i = j;
    }
    return r;
}

const Sector* find(const std::vector<Sector>& s, int q) {
    for (const auto& x : s)
        if (x.q == q) return &x;
    return nullptr;
}

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

const void* at(const void* p, int64_t elems, size_t esz) { return static_cast<const char*>(p) + elems * esz; }
void* at(void* p, int64_t elems, size_t esz) { return static_cast<char*>(p) + elems * esz; }

// Stage A of both pipelines: X[k][a'][s][b] = sum_a Env[k][a'][a] T[a][s][b]
// (Env [w][chil][chil], T [chil][D][chir]).
void stage_a(tdvp_ctx ctx, Dt dt, bool fp64, int form, const std::vector<Sector>& SL, const std::vector<Sector>& SR,
             const std::vector<int>& qD, const std::vector<Run>& cw, int chil, int chir, const void* env,
             const void* T, void* X) {
    const int D = (int)qD.size();
    const size_t esz = elem_bytes(dt);
    const int64_t row = (int64_t)D * chir;
    // every block of X the later stages may read is written: a block whose
    // source sector a = a' - c does not exist is written as zeros (K = 0)
    std::vector<BlockGemm> probs;
    for (const Run& r : cw)
        for (const Sector& ap : SL) {
            const Sector* a = find(SL, ap.q - r.c);
            for (int s = 0; s < D; ++s) {
                const Sector* b = find(SR, ap.q - r.c + qD[s]);
                if (!b) continue;
                BlockGemm bg;
                GemmDesc& g = bg.g;
                g.M = ap.n;
                g.N = b->n;
                g.K = a ? a->n : 0;
                g.batch = r.n;
                const int aoff = a ? a->off : 0;
                g.A = opnd(at(env, (int64_t)r.i0 * chil * chil + (int64_t)ap.off * chil + aoff, esz), dt, chil, true,
                           false, (int64_t)chil * chil);
                g.B = opnd(at(T, (int64_t)aoff * row + (int64_t)s * chir + b->off, esz), dt, row, false);
                g.C = at(X, (int64_t)r.i0 * chil * row + (int64_t)ap.off * row + (int64_t)s * chir + b->off, esz);
                g.cdt = dt;
                g.ldc = row;
                g.strideC = (int64_t)chil * row;
                probs.push_back(bg);
            }
        }
    block_gemm(ctx, probs, {}, fp64, form, "u1A");
}

// The sparse MPO stage on the (p-sector, q-sector) rectangles whose charge
// difference q - p is in `deltas`; strides as in WStageDesc.  Neighbouring
// q-sectors that both qualify are one rectangle (their indices are
// contiguous): a block of the MPO stage covers a few hundred q points, and
// single sectors of a few dozen would leave most of it idle.
void mpo_stage(tdvp_ctx ctx, const WStageDesc& base, const std::vector<Sector>& SP, const std::vector<Sector>& SQ,
               const std::vector<int>& deltas, size_t esz_in, size_t esz_out) {
    std::vector<WStageDesc> ds;
    auto wanted = [&](const Sector& p, const Sector& q) {
        return std::find(deltas.begin(), deltas.end(), q.q - p.q) != deltas.end();
    };
    for (const Sector& p : SP)
        for (size_t i = 0; i < SQ.size();) {
            if (!wanted(p, SQ[i])) {
                ++i;
                continue;
            }
            size_t e = i + 1;
            while (e < SQ.size() && wanted(p, SQ[e])) ++e;
            WStageDesc w = base;
            w.in = at(base.in, (int64_t)p.off * base.ip + SQ[i].off, esz_in);
            w.out = at(base.out, (int64_t)p.off * base.op + SQ[i].off, esz_out);
            w.P = p.n;
            w.Q = SQ[e - 1].off + SQ[e - 1].n - SQ[i].off;
            ds.push_back(w);
            i = e;
        }
    if (ds.empty()) return;
    GroupedWStage g;
    grouped_wstage_plan(ctx, ds, g, "u1_wstage_tab");
    grouped_wstage_run(ctx, g);
}

// Charge differences q(right index) - q(left index) = qD(s) + sign c(k) that
// the terms (s, k) of one side of the MPO stage produce, added to `d`.
void add_deltas(std::vector<int>& d, const std::vector<int>& qD, const int* c, int w, int sign) {
    for (int s = 0; s < (int)qD.size(); ++s)
        for (int k = 0; k < w; ++k) {
            const int v = qD[s] + sign * c[k];
            if (std::find(d.begin(), d.end(), v) == d.end()) d.push_back(v);
        }
}

}  // namespace

void heff_u1(tdvp_ctx ctx, int nsite, Dt dt, int chil, int chir, int d, int wl, int wm, int wr, const int* ql,
             const int* qr, const int* qs, const int* cl, const int* cr, const void* L, const void* W1,
             const void* W2, const void* R, const void* x, void* y) {
    const bool fp64 = dt == Dt::C128;
    const int form = raw_gemm_form(ctx, fp64);
    const size_t esz = elem_bytes(dt);
    const std::vector<Sector> SL = sectors_of(ql, chil, "apply_heff_u1 left bond");
    const std::vector<Sector> SR = sectors_of(qr, chir, "apply_heff_u1 right bond");
    std::vector<int> qD;  // charge of the local physical multi-index
    if (nsite == 0) qD = {0};
    else if (nsite == 1) qD.assign(qs, qs + d);
    else
        for (int s1 = 0; s1 < d; ++s1)
            for (int s2 = 0; s2 < d; ++s2) qD.push_back(qs[s1] + qs[s2]);
    const int D = (int)qD.size();
    const int64_t n = (int64_t)chil * D * chir;
    zero_fill(y, esz * (size_t)n, ctx->stream);
    const std::vector<Run> RL = runs_of(cl, wl), RR = runs_of(cr, wr);
    void* T1 = ctx->workspace("u1_T1", esz * (size_t)wl * n);
    void* T3 = ctx->workspace("u1_T3", esz * (size_t)wr * n);
    stage_a(ctx, dt, fp64, form, SL, SR, qD, RL, chil, chir, L, x, T1);

    // MPO stage: T3[a'][s'][n][b] = sum_{k,s} M[(n,s'),(k,s)] T1[k][a'][s][b]
    Mop m;
    mop_make(ctx, m, nsite == 0 ? 0 : (nsite == 1 ? 1 : 2), W1, W2, dt, wl, nsite == 2 ? wm : wl, wr, d, fp64, false);
    WStageDesc w;
    w.in = T1;
    w.in_dt = dt;
    w.out = T3;
    w.out_dt = dt;
    w.D = D;
    w.w_in = wl;
    w.w_out = wr;
    w.ik = n;
    w.is = chir;
    w.ip = (int64_t)D * chir;
    w.on = chir;
    w.os = (int64_t)wr * chir;
    w.op = (int64_t)D * wr * chir;
    w.row_ptr = m.row_ptr;
    w.col = m.col;
    w.val = m.val;
    w.fp64 = fp64;
    // rectangles: every charge difference of an input (k, s) or an output
    // (n, s') term, so that every block stage B reads is computed (an output
    // term without inputs comes out zero)
    std::vector<int> dlt;
    add_deltas(dlt, qD, cl, wl, -1);
    add_deltas(dlt, qD, cr, wr, -1);
    mpo_stage(ctx, w, SL, SR, dlt, esz, esz);

    // Stage B: y[a'][s'][b'] = sum_{n, b} T3[a'][s'][n][b] R[n][b][b'], one K
    // chunk per run of equal MPO charge c (b in the sector q(b') - c)
    std::vector<BlockGemm> probs;
    std::vector<BlockChunk> chunks;
    for (const Sector& a : SL)
        for (int s = 0; s < D; ++s) {
            const Sector* bp = find(SR, a.q + qD[s]);
            if (!bp) continue;
            BlockGemm bg;
            bg.chunk0 = (int)chunks.size();
            for (const Run& r : RR) {
                const Sector* b = find(SR, bp->q - r.c);
                if (!b) continue;
                BlockChunk ch;
                ch.offA = (int64_t)a.off * w.op + (int64_t)s * w.os + (int64_t)r.i0 * chir + b->off;
                ch.offB = (int64_t)r.i0 * chir * chir + (int64_t)b->off * chir + bp->off;
                ch.strideA = chir;
                ch.strideB = (int64_t)chir * chir;
                ch.K = b->n;
                ch.count = r.n;
                chunks.push_back(ch);
            }
            bg.nchunk = (int)chunks.size() - bg.chunk0;
            if (bg.nchunk == 0) continue;  // the block stays zero
            GemmDesc& g = bg.g;
            g.M = a.n;
            g.N = bp->n;
            g.K = 0;
            g.A = opnd(T3, dt, w.op, true);
            g.B = opnd(R, dt, chir, false);
            g.C = at(y, (int64_t)a.off * D * chir + (int64_t)s * chir + bp->off, esz);
            g.cdt = dt;
            g.ldc = (int64_t)D * chir;
            probs.push_back(bg);
        }
    block_gemm(ctx, probs, chunks, fp64, form, "u1B");
}

void env_u1(tdvp_ctx ctx, int dir, Dt dt, int chil, int chir, int d, int wl, int wr, const int* ql, const int* qr,
            const int* qs, const int* cl, const int* cr, const void* env, const void* A, const void* W, void* out) {
    const bool fp64 = dt == Dt::C128;
    const int form = raw_gemm_form(ctx, fp64);
    const size_t esz = elem_bytes(dt);
    const std::vector<Sector> SL = sectors_of(ql, chil, "env_update_u1 left bond");
    const std::vector<Sector> SR = sectors_of(qr, chir, "env_update_u1 right bond");
    const std::vector<int> qd(qs, qs + d);
    const int64_t n = (int64_t)chil * d * chir;
    Mop m;
    if (dir == 1) {
        zero_fill(out, esz * (size_t)wr * chir * chir, ctx->stream);
        void* X = ctx->workspace("u1_envX", esz * (size_t)wl * n);
        void* Y = ctx->workspace("u1_envY", esz * (size_t)wr * n);
        // X[k][a'][s][b] = sum_a L[k][a'][a] A[a][s][b]
        stage_a(ctx, dt, fp64, form, SL, SR, qd, runs_of(cl, wl), chil, chir, env, A, X);
        // Y[l][a'][s'][b] = sum_{k,s} W[k][l][s'][s] X[k][a'][s][b]
        mop_make(ctx, m, 1, W, nullptr, dt, wl, wl, wr, d, fp64, false);
        WStageDesc w;
        w.in = X;
        w.in_dt = dt;
        w.out = Y;
        w.out_dt = dt;
        w.D = d;
        w.w_in = wl;
        w.w_out = wr;
        w.ik = n;
        w.is = chir;
        w.ip = (int64_t)d * chir;
        w.on = n;
        w.os = chir;
        w.op = (int64_t)d * chir;
        w.row_ptr = m.row_ptr;
        w.col = m.col;
        w.val = m.val;
        w.fp64 = fp64;
        std::vector<int> dlt;
        add_deltas(dlt, qd, cl, wl, -1);
        add_deltas(dlt, qd, cr, wr, -1);
        mpo_stage(ctx, w, SL, SR, dlt, esz, esz);
        // out[l][b'][b] = sum_{a', s'} conj(A[a'][s'][b']) Y[l][a'][s'][b]: one
        // chunk per s' (a' in the sector q(b') - q(s'))
        std::vector<BlockGemm> probs;
        std::vector<BlockChunk> chunks;
        for (const Run& r : runs_of(cr, wr))
            for (const Sector& b : SR) {
                const Sector* bp = find(SR, b.q + r.c);
                if (!bp) continue;
                BlockGemm bg;
                bg.chunk0 = (int)chunks.size();
                for (int s = 0; s < d; ++s) {
                    const Sector* ap = find(SL, bp->q - qs[s]);
                    if (!ap) continue;
                    BlockChunk ch;
                    ch.offA = (int64_t)ap->off * d * chir + (int64_t)s * chir + bp->off;
                    ch.offB = (int64_t)ap->off * d * chir + (int64_t)s * chir + b.off;
                    ch.K = ap->n;
                    chunks.push_back(ch);
                }
                bg.nchunk = (int)chunks.size() - bg.chunk0;
                if (bg.nchunk == 0) continue;
                GemmDesc& g = bg.g;
                g.M = bp->n;
                g.N = b.n;
                g.batch = r.n;
                g.A = opnd(A, dt, (int64_t)d * chir, false, true, 0);
                g.B = opnd(at(Y, (int64_t)r.i0 * n, esz), dt, (int64_t)d * chir, false, false, n);
                g.C = at(out, (int64_t)r.i0 * chir * chir + (int64_t)bp->off * chir + b.off, esz);
                g.cdt = dt;
                g.ldc = chir;
                g.strideC = (int64_t)chir * chir;
                probs.push_back(bg);
            }
        block_gemm(ctx, probs, chunks, fp64, form, "u1envL");
        return;
    }
    zero_fill(out, esz * (size_t)wl * chil * chil, ctx->stream);
    void* U = ctx->workspace("u1_envX", esz * (size_t)wr * n);
    void* V = ctx->workspace("u1_envY", esz * (size_t)wl * n);
    // U[a][s][l][b'] = sum_b A[a][s][b] R[l][b][b'], batched over runs of l;
    // blocks whose source sector b = a + q(s) does not exist are zeros (K = 0)
    {
        std::vector<BlockGemm> probs;
        for (const Run& r : runs_of(cr, wr))
            for (const Sector& a : SL)
                for (int s = 0; s < d; ++s) {
                    const Sector* bp = find(SR, a.q + qs[s] + r.c);
                    if (!bp) continue;
                    const Sector* b = find(SR, a.q + qs[s]);
                    const int boff = b ? b->off : 0;
                    BlockGemm bg;
                    GemmDesc& g = bg.g;
                    g.M = a.n;
                    g.N = bp->n;
                    g.K = b ? b->n : 0;
                    g.batch = r.n;
                    g.A = opnd(at(A, (int64_t)a.off * d * chir + (int64_t)s * chir + boff, esz), dt,
                               (int64_t)d * chir, true);
                    g.B = opnd(at(env, (int64_t)r.i0 * chir * chir + (int64_t)boff * chir + bp->off, esz), dt, chir,
                               false, false, (int64_t)chir * chir);
                    g.C = at(U, (int64_t)a.off * d * wr * chir + (int64_t)s * wr * chir + (int64_t)r.i0 * chir + bp->off,
                             esz);
                    g.cdt = dt;
                    g.ldc = (int64_t)d * wr * chir;
                    g.strideC = chir;
                    probs.push_back(bg);
                }
        block_gemm(ctx, probs, {}, fp64, form, "u1envU");
    }
    // V[k][a][s'][b'] = sum_{l,s} W[k][l][s'][s] U[a][s][l][b']
    mop_make(ctx, m, 3, W, nullptr, dt, wl, wl, wr, d, fp64, false);
    WStageDesc w;
    w.in = U;
    w.in_dt = dt;
    w.out = V;
    w.out_dt = dt;
    w.D = d;
    w.w_in = wr;
    w.w_out = wl;
    w.ik = chir;
    w.is = (int64_t)wr * chir;
    w.ip = (int64_t)d * wr * chir;
    w.on = n;
    w.os = chir;
    w.op = (int64_t)d * chir;
    w.row_ptr = m.row_ptr;
    w.col = m.col;
    w.val = m.val;
    w.fp64 = fp64;
    std::vector<int> dl;  // q(b') - q(a) = q(s) + c(l) (inputs) or q(s') + c(k) (outputs)
    add_deltas(dl, qd, cr, wr, 1);
    add_deltas(dl, qd, cl, wl, 1);
    mpo_stage(ctx, w, SL, SR, dl, esz, esz);
    // out[k][a][a'] = sum_{s', b'} V[k][a][s'][b'] conj(A[a'][s'][b']): one
    // chunk per s' (b' in the sector q(a') + q(s'))
    std::vector<BlockGemm> probs;
    std::vector<BlockChunk> chunks;
    for (const Run& r : runs_of(cl, wl))
        for (const Sector& a : SL) {
            const Sector* ap = find(SL, a.q + r.c);
            if (!ap) continue;
            BlockGemm bg;
            bg.chunk0 = (int)chunks.size();
            for (int s = 0; s < d; ++s) {
                const Sector* bp = find(SR, ap->q + qs[s]);
                if (!bp) continue;
                BlockChunk ch;
                ch.offA = (int64_t)a.off * d * chir + (int64_t)s * chir + bp->off;
                ch.offB = (int64_t)ap->off * d * chir + (int64_t)s * chir + bp->off;
                ch.K = bp->n;
                chunks.push_back(ch);
            }
            bg.nchunk = (int)chunks.size() - bg.chunk0;
            if (bg.nchunk == 0) continue;
            GemmDesc& g = bg.g;
            g.M = a.n;
            g.N = ap->n;
            g.batch = r.n;
            g.A = opnd(at(V, (int64_t)r.i0 * n, esz), dt, (int64_t)d * chir, true, false, n);
            g.B = opnd(A, dt, (int64_t)d * chir, true, true, 0);
            g.C = at(out, (int64_t)r.i0 * chil * chil + (int64_t)a.off * chil + ap->off, esz);
            g.cdt = dt;
            g.ldc = chil;
            g.strideC = (int64_t)chil * chil;
            probs.push_back(bg);
        }
    block_gemm(ctx, probs, chunks, fp64, form, "u1envR");
}

}  // namespace tdvp

using namespace tdvp;

extern "C" {

int apply_heff_u1(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm, int wr,
                  const int* q_left, const int* q_right, const int* q_phys, const int* c_left, const int* c_right,
                  const void* L, const void* W1, const void* W2, const void* R, const void* theta, void* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        const Dt dt = to_dt(dtype);
        TDVP_REQUIRE(nsite >= 0 && nsite <= 2, TDVP_E_ARG, "apply_heff_u1: nsite must be 0, 1 or 2");
        TDVP_REQUIRE(chil >= 1 && chir >= 1 && wl >= 1 && wr >= 1 && (nsite == 0 || d >= 1), TDVP_E_SHAPE,
                     "apply_heff_u1: dimensions must be positive");
        TDVP_REQUIRE(nsite != 2 || wm >= 1, TDVP_E_SHAPE, "apply_heff_u1: wm must be positive");
        TDVP_REQUIRE(nsite != 0 || wl == wr, TDVP_E_SHAPE, "apply_heff_u1: zero-site needs wl == wr");
        TDVP_REQUIRE(q_left && q_right && c_left && c_right && (nsite == 0 || q_phys), TDVP_E_ARG,
                     "apply_heff_u1: null charge labels");
        TDVP_REQUIRE(L && R && theta && out && (nsite < 1 || W1) && (nsite < 2 || W2), TDVP_E_ARG,
                     "apply_heff_u1: null pointer");
        TDVP_REQUIRE(out != theta && out != L && out != R, TDVP_E_ARG, "apply_heff_u1: out aliases an input");
        heff_u1(ctx, nsite, dt, chil, chir, nsite == 0 ? 1 : d, wl, wm, wr, q_left, q_right, q_phys, c_left, c_right,
                L, W1, W2, R, theta, out);
    });
}

int env_update_u1(tdvp_ctx ctx, int dir, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wr,
                  const int* q_left, const int* q_right, const int* q_phys, const int* c_left, const int* c_right,
                  const void* env_in, const void* A, const void* W, void* env_out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        const Dt dt = to_dt(dtype);
        TDVP_REQUIRE(dir == 1 || dir == -1, TDVP_E_ARG, "env_update_u1: dir must be +1 or -1");
        TDVP_REQUIRE(chil >= 1 && chir >= 1 && d >= 1 && wl >= 1 && wr >= 1, TDVP_E_SHAPE,
                     "env_update_u1: dimensions must be positive");
        TDVP_REQUIRE(q_left && q_right && q_phys && c_left && c_right, TDVP_E_ARG, "env_update_u1: null charge labels");
        TDVP_REQUIRE(env_in && A && W && env_out, TDVP_E_ARG, "env_update_u1: null pointer");
        TDVP_REQUIRE(env_out != env_in && env_out != A, TDVP_E_ARG, "env_update_u1: out aliases an input");
        env_u1(ctx, dir, dt, chil, chir, d, wl, wr, q_left, q_right, q_phys, c_left, c_right, env_in, A, W, env_out);
    });
}

}  // extern "C"
