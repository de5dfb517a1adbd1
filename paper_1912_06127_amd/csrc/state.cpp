// MPO and MPS objects: construction, host transfer and canonical form.
#include "internal.hpp"

#include <algorithm>

#include <cmath>

namespace tdvp {

namespace {

// Row-major complex product C [m][n] = A [m][k] B [k][n] in FP64 on MFMA.
void zgemm_nn(tdvp_ctx ctx, const double2* A, const double2* B, double2* C, int m, int k, int n) {
    GemmDesc g;
    g.M = m;
    g.N = n;
    g.K = k;
    g.A.p = A; g.A.dt = Dt::C128; g.A.ld = k; g.A.kcontig = true;
    g.B.p = B; g.B.dt = Dt::C128; g.B.ld = n; g.B.kcontig = false;
    g.C = C;
    g.cdt = Dt::C128;
    g.ldc = n;
    cgemm(ctx, g, true, 4);
}

// splitmix64 (Steele, Lea, Flood 2014) -> uniform doubles -> Box-Muller normals
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    void normal2(double& a, double& b) {
        const double u = uniform(), v = uniform();
        const double r = std::sqrt(-2.0 * std::log(u));
        a = r * std::cos(2.0 * M_PI * v);
        b = r * std::sin(2.0 * M_PI * v);
    }
};

}  // namespace

void zgemm_rowmajor(tdvp_ctx ctx, const double2* A, const double2* B, double2* C, int m, int k, int n) {
    zgemm_nn(ctx, A, B, C, m, k, n);
}

}  // namespace tdvp

using namespace tdvp;

const Mop& tdvp_mpo_s::mop(int kind, int site, bool fp64) {
    auto key = std::make_tuple(kind, site, fp64);
    auto it = mops.find(key);
    if (it != mops.end()) return *it->second;
    auto m = std::make_unique<Mop>();
    const Dt dt = Dt::C128;
    switch (kind) {
        case 0:  // bond between site and site+1
            mop_make(ctx, *m, 0, nullptr, nullptr, dt, w[site + 1], w[site + 1], w[site + 1], d, fp64, true);
            break;
        case 1:
        case 3:
            mop_make(ctx, *m, kind, W(site, dt), nullptr, dt, w[site], w[site], w[site + 1], d, fp64, true);
            break;
        case 2:
            mop_make(ctx, *m, 2, W(site, dt), W(site + 1, dt), dt, w[site], w[site + 1], w[site + 2], d,
                     fp64, true);
            break;
        default:
            throw Error(TDVP_E_ARG, "bad MPO stage kind");
    }
    const Mop& ref = *m;
    mops[key] = std::move(m);
    return ref;
}

const void* tdvp_mpo_s::W(int site, Dt dt) { return dt == Dt::C128 ? dev128[site].ptr : dev64[site].ptr; }

void tdvp_mps_s::set_tensor_dev(int j, int chil, int chir) {
    const size_t need = sizeof(double2) * (size_t)chil * d * chir;
    if (A[j].bytes < need) A[j] = DevMem(ctx, need);
}

namespace {

void upload_mpo(tdvp_mpo m) {
    tdvp_ctx ctx = m->ctx;
    m->dev128.clear();
    m->dev64.clear();
    for (int j = 0; j < m->N; ++j) {
        const size_t n = (size_t)m->w[j] * m->w[j + 1] * m->d * m->d;
        m->dev128.emplace_back(ctx, n * sizeof(double2));
        m->dev64.emplace_back(ctx, n * sizeof(float2));
        TDVP_CHECK_HIP(hipMemcpyAsync(m->dev128[j].ptr, m->host[j].data(), n * sizeof(double2),
                                      hipMemcpyHostToDevice, ctx->stream));
        convert(m->dev64[j].ptr, Dt::C64, m->dev128[j].ptr, Dt::C128, (int64_t)n, ctx->stream);
    }
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
}

void validate_chi(int N, int d, const int* chi) {
    TDVP_REQUIRE(chi, TDVP_E_ARG, "chi is null");
    TDVP_REQUIRE(chi[0] == 1 && chi[N] == 1, TDVP_E_SHAPE, "chi[0] and chi[N] must be 1");
    for (int j = 1; j <= N; ++j) {
        TDVP_REQUIRE(chi[j] >= 1, TDVP_E_SHAPE, "bond dimensions must be positive");
        TDVP_REQUIRE(chi[j - 1] <= (int64_t)d * chi[j] && chi[j] <= (int64_t)d * chi[j - 1], TDVP_E_SHAPE,
                     "bond dimensions must satisfy chi[j-1] <= d chi[j] and chi[j] <= d chi[j-1]");
    }
}

void right_canonicalize(tdvp_ctx ctx, tdvp_mps m) {
    for (int j = m->N - 1; j >= 1; --j) {
        const int chil = m->chi[j], chir = m->chi[j + 1], d = m->d;
        const int k = std::min(chil, d * chir);
        double2* Lf = static_cast<double2*>(ctx->workspace("canon_L", sizeof(double2) * (size_t)chil * k));
        double2* Q = static_cast<double2*>(ctx->workspace("canon_Q", sizeof(double2) * (size_t)k * d * chir));
        lq_rowmajor(ctx, m->A[j].as<double2>(), chil, d * chir, Lf, Q);
        m->set_tensor_dev(j, k, chir);
        TDVP_CHECK_HIP(hipMemcpyAsync(m->A[j].ptr, Q, sizeof(double2) * (size_t)k * d * chir,
                                      hipMemcpyDeviceToDevice, ctx->stream));
        const int pl = m->chi[j - 1];
        double2* tmp = static_cast<double2*>(ctx->workspace("canon_T", sizeof(double2) * (size_t)pl * d * k));
        zgemm_rowmajor(ctx, m->A[j - 1].as<double2>(), Lf, tmp, pl * d, chil, k);
        m->set_tensor_dev(j - 1, pl, k);
        TDVP_CHECK_HIP(hipMemcpyAsync(m->A[j - 1].ptr, tmp, sizeof(double2) * (size_t)pl * d * k,
                                      hipMemcpyDeviceToDevice, ctx->stream));
        m->chi[j] = k;
    }
    m->env_valid = false;
    TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
}

}  // namespace

extern "C" {

int mpo_longrange(tdvp_ctx ctx, const tdvp_mpo_spec* sp, tdvp_mpo* out, double* fit_max_abs_err) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(sp && out, TDVP_E_ARG, "mpo_longrange: null argument");
        *out = nullptr;
        if (fit_max_abs_err) *fit_max_abs_err = 0.0;
        const int N = sp->N, d = sp->d, nH = sp->n_terms, K = sp->K;
        TDVP_REQUIRE(N >= 2 && d >= 1 && nH >= 0 && K >= 0, TDVP_E_SHAPE, "mpo_longrange: bad sizes");
        TDVP_REQUIRE(nH == 0 || (sp->g && sp->A_ops && sp->B_ops), TDVP_E_ARG, "mpo_longrange: null operators");
        TDVP_REQUIRE(!sp->c == !sp->lambda, TDVP_E_ARG, "mpo_longrange: give both c and lambda, or neither");
        TDVP_REQUIRE(K > 0 || nH == 0 || sp->coupling, TDVP_E_ARG, "mpo_longrange: null couplings");
        // K > 0 without c, lambda: fit f(r) = r^-alpha on r = 1..fit_rmax (Sec. II C)
        std::vector<double> fitted;
        const double* cw = sp->c;
        const double* lw = sp->lambda;
        if (K > 0 && !cw) {
            TDVP_REQUIRE(std::isfinite(sp->alpha), TDVP_E_ARG, "mpo_longrange: alpha is not finite");
            const int rmax = sp->fit_rmax > 0 ? sp->fit_rmax : N - 1;
            std::vector<double> f(rmax);
            for (int r = 1; r <= rmax; ++r) f[r - 1] = std::pow((double)r, -sp->alpha);
            std::vector<std::complex<double>> c, lam;
            const double err = fit_exponentials(f, K, sp->fit_refine != 0, c, lam);
            if (fit_max_abs_err) *fit_max_abs_err = err;
            fitted.resize(4 * K);
            for (int k = 0; k < K; ++k) {
                fitted[2 * k] = c[k].real();
                fitted[2 * k + 1] = c[k].imag();
                fitted[2 * K + 2 * k] = lam[k].real();
                fitted[2 * K + 2 * k + 1] = lam[k].imag();
            }
            cw = fitted.data();
            lw = fitted.data() + 2 * K;
        }
        const int R = N - 1;
        const int chans = K > 0 ? K : R;  // bond states per term
        const int m = nH * chans + 2;
        const size_t dd = (size_t)d * d;
        // bulk tensor Wb[k][l][s'][s], complex interleaved
        std::vector<double> Wb((size_t)m * m * dd * 2, 0.0);
        auto put = [&](int k, int l, const double* op, double cre, double cim) {
            for (size_t e = 0; e < dd; ++e) {
                const double ore = op ? op[2 * e] : 0.0, oim = op ? op[2 * e + 1] : 0.0;
                double* dst = &Wb[(((size_t)k * m + l) * dd + e) * 2];
                dst[0] += cre * ore - cim * oim;
                dst[1] += cre * oim + cim * ore;
            }
        };
        std::vector<double> id(dd * 2, 0.0);
        for (int s = 0; s < d; ++s) id[(s * d + s) * 2] = 1.0;
        put(0, 0, id.data(), 1.0, 0.0);          // nothing placed yet
        put(m - 1, m - 1, id.data(), 1.0, 0.0);  // term complete
        if (sp->onsite && sp->h != 0.0) put(0, m - 1, sp->onsite, sp->h, 0.0);
        for (int a = 0; a < nH; ++a) {
            const double* A = sp->A_ops + a * dd * 2;
            const double* B = sp->B_ops + a * dd * 2;
            const double g = sp->g[a];
            if (K > 0) {
                // channel (a, k): A opens, lambda_k per site, g c_k lambda_k B closes
                for (int k = 0; k < K; ++k) {
                    const int st = 1 + a * K + k;
                    const double lr = lw[2 * k], li = lw[2 * k + 1];
                    const double cr = cw[2 * k], ci = cw[2 * k + 1];
                    put(0, st, A, 1.0, 0.0);
                    put(st, st, id.data(), lr, li);
                    put(st, m - 1, B, g * (cr * lr - ci * li), g * (cr * li + ci * lr));
                }
            } else {
                // shift register: state (a, r) = "A_a placed r sites to the left"
                for (int r = 1; r <= R; ++r) {
                    const int st = 1 + a * R + (r - 1);
                    if (r == 1) put(0, st, A, 1.0, 0.0);
                    if (r < R) put(st, st + 1, id.data(), 1.0, 0.0);
                    put(st, m - 1, B, g * sp->coupling[r - 1], 0.0);
                }
            }
        }
        auto mp = std::make_unique<tdvp_mpo_s>();
        mp->ctx = ctx;
        mp->N = N;
        mp->d = d;
        mp->w.assign(N + 1, m);
        mp->w[0] = mp->w[N] = 1;
        for (int j = 0; j < N; ++j) {
            const int r0 = (j == 0) ? 0 : 0, r1 = (j == 0) ? 1 : m;        // rows kept
            const int c0 = (j == N - 1) ? m - 1 : 0, c1 = (j == N - 1) ? m : m;  // cols kept
            std::vector<double> t;
            for (int k = r0; k < r1; ++k)
                for (int l = c0; l < c1; ++l)
                    for (size_t e = 0; e < dd; ++e) {
                        const double* src = &Wb[(((size_t)k * m + l) * dd + e) * 2];
                        t.push_back(src[0]);
                        t.push_back(src[1]);
                    }
            mp->host.push_back(std::move(t));
        }
        upload_mpo(mp.get());
        *out = mp.release();
    });
}

int mpo_from_tensors(tdvp_ctx ctx, int N, int d, const int* w, const double* W_host, tdvp_mpo* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(out && w && W_host, TDVP_E_ARG, "mpo_from_tensors: null argument");
        *out = nullptr;
        TDVP_REQUIRE(N >= 1 && d >= 1, TDVP_E_SHAPE, "mpo_from_tensors: bad sizes");
        TDVP_REQUIRE(w[0] == 1 && w[N] == 1, TDVP_E_SHAPE, "mpo_from_tensors: w[0] and w[N] must be 1");
        auto mp = std::make_unique<tdvp_mpo_s>();
        mp->ctx = ctx;
        mp->N = N;
        mp->d = d;
        mp->w.assign(w, w + N + 1);
        size_t off = 0;
        for (int j = 0; j < N; ++j) {
            TDVP_REQUIRE(w[j + 1] >= 1, TDVP_E_SHAPE, "mpo_from_tensors: bond dimensions must be positive");
            const size_t n = (size_t)w[j] * w[j + 1] * d * d * 2;
            mp->host.emplace_back(W_host + off, W_host + off + n);
            off += n;
        }
        upload_mpo(mp.get());
        *out = mp.release();
    });
}

int mpo_get_info(tdvp_mpo mpo, int* N, int* d, int* w) {
    if (!mpo) return TDVP_E_ARG;
    if (N) *N = mpo->N;
    if (d) *d = mpo->d;
    if (w) for (int j = 0; j <= mpo->N; ++j) w[j] = mpo->w[j];
    return TDVP_OK;
}

int mpo_get_tensor(tdvp_mpo mpo, int site, double* W_host) {
    if (!mpo || !W_host || site < 0 || site >= mpo->N) return TDVP_E_ARG;
    std::memcpy(W_host, mpo->host[site].data(), mpo->host[site].size() * sizeof(double));
    return TDVP_OK;
}

int mpo_destroy(tdvp_mpo mpo) {
    if (!mpo) return TDVP_E_ARG;
    (void)hipStreamSynchronize(mpo->ctx->stream);
    delete mpo;
    return TDVP_OK;
}

int mps_init(tdvp_ctx ctx, int N, int d, const int* chi, const int* basis_state, uint64_t seed,
             tdvp_mps* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(out, TDVP_E_ARG, "mps_init: out is null");
        *out = nullptr;
        TDVP_REQUIRE(N >= 1 && d >= 1, TDVP_E_SHAPE, "mps_init: bad sizes");
        validate_chi(N, d, chi);
        auto m = std::make_unique<tdvp_mps_s>();
        m->ctx = ctx;
        m->N = N;
        m->d = d;
        m->chi.assign(chi, chi + N + 1);
        m->A.resize(N);
        m->L.resize(N);
        m->R.resize(N);
        Rng rng{seed};
        for (int j = 0; j < N; ++j) {
            const int chil = chi[j], chir = chi[j + 1];
            std::vector<double> t((size_t)chil * d * chir * 2, 0.0);
            if (basis_state) {
                const int bit = basis_state[j];
                TDVP_REQUIRE(bit >= 0 && bit < d, TDVP_E_ARG, "mps_init: basis state out of range");
                // row 0 carries the product state, other rows the remaining
                // unit vectors e_(s, b) in lexicographic order
                t[((size_t)0 * d * chir + bit * chir + 0) * 2] = 1.0;
                int r = 1;
                for (int s = 0; s < d && r < chil; ++s)
                    for (int b = 0; b < chir && r < chil; ++b) {
                        if (s == bit && b == 0) continue;
                        t[((size_t)r * d * chir + s * chir + b) * 2] = 1.0;
                        ++r;
                    }
            } else {
                for (size_t e = 0; e < t.size(); e += 2) {
                    double a, b;
                    rng.normal2(a, b);
                    t[e] = a / std::sqrt(2.0);
                    t[e + 1] = b / std::sqrt(2.0);
                }
            }
            m->set_tensor_dev(j, chil, chir);
            TDVP_CHECK_HIP(hipMemcpyAsync(m->A[j].ptr, t.data(), t.size() * sizeof(double),
                                          hipMemcpyHostToDevice, ctx->stream));
            TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        }
        if (!basis_state) {
            right_canonicalize(ctx, m.get());
            // unit norm: scale site 1
            std::vector<double> t((size_t)m->chi[0] * d * m->chi[1] * 2);
            TDVP_CHECK_HIP(hipMemcpy(t.data(), m->A[0].ptr, t.size() * sizeof(double), hipMemcpyDeviceToHost));
            double nrm = 0.0;
            for (double v : t) nrm += v * v;
            nrm = std::sqrt(nrm);
            TDVP_REQUIRE(nrm > 0.0, TDVP_E_NUMERIC, "mps_init: zero random state");
            scale_copy(m->A[0].as<double2>(), m->A[0].as<double2>(), 1.0 / nrm,
                       (int64_t)m->chi[0] * d * m->chi[1], ctx->stream);
            TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        }
        *out = m.release();
    });
}

int mps_get_info(tdvp_mps mps, int* N, int* d, int* chi) {
    if (!mps) return TDVP_E_ARG;
    if (N) *N = mps->N;
    if (d) *d = mps->d;
    if (chi) for (int j = 0; j <= mps->N; ++j) chi[j] = mps->chi[j];
    return TDVP_OK;
}

int mps_get_tensor(tdvp_mps mps, int site, double* host) {
    if (!mps) return TDVP_E_ARG;
    return guarded(mps->ctx, [&] {
        TDVP_REQUIRE(host && site >= 0 && site < mps->N, TDVP_E_ARG, "mps_get_tensor: bad argument");
        TDVP_CHECK_HIP(hipMemcpyAsync(host, mps->A[site].ptr, sizeof(double2) * mps->tensor_elems(site),
                                      hipMemcpyDeviceToHost, mps->ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(mps->ctx->stream));
    });
}

int mps_set_tensor(tdvp_mps mps, int site, const double* host, int chil, int chir) {
    if (!mps) return TDVP_E_ARG;
    return guarded(mps->ctx, [&] {
        TDVP_REQUIRE(host && site >= 0 && site < mps->N, TDVP_E_ARG, "mps_set_tensor: bad argument");
        TDVP_REQUIRE(chil >= 1 && chir >= 1, TDVP_E_SHAPE, "mps_set_tensor: bad bond dimensions");
        TDVP_REQUIRE(site != 0 || chil == 1, TDVP_E_SHAPE, "mps_set_tensor: chi_0 must be 1");
        TDVP_REQUIRE(site != mps->N - 1 || chir == 1, TDVP_E_SHAPE, "mps_set_tensor: chi_N must be 1");
        mps->set_tensor_dev(site, chil, chir);
        mps->chi[site] = chil;
        mps->chi[site + 1] = chir;
        mps->clear_charges();
        TDVP_CHECK_HIP(hipMemcpyAsync(mps->A[site].ptr, host, sizeof(double2) * (size_t)chil * mps->d * chir,
                                      hipMemcpyHostToDevice, mps->ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(mps->ctx->stream));
        mps->env_valid = false;
    });
}

int mps_set_charges(tdvp_mps mps, const int* q_phys, const int* labels) {
    if (!mps) return TDVP_E_ARG;
    return guarded(mps->ctx, [&] {
        if (!q_phys && !labels) {
            mps->clear_charges();
            return;
        }
        TDVP_REQUIRE(q_phys && labels, TDVP_E_ARG, "mps_set_charges: q_phys and labels go together");
        std::vector<std::vector<int>> q(mps->N + 1);
        const int* p = labels;
        for (int j = 0; j <= mps->N; ++j) {
            q[j].assign(p, p + mps->chi[j]);
            p += mps->chi[j];
            for (int a = 1; a < mps->chi[j]; ++a)
                TDVP_REQUIRE(q[j][a - 1] <= q[j][a], TDVP_E_ARG, "mps_set_charges: bond labels must be non-decreasing");
        }
        mps->qphys.assign(q_phys, q_phys + mps->d);
        mps->qbond = std::move(q);
    });
}

int mps_get_charges(tdvp_mps mps, int* q_phys, int* labels) {
    if (!mps) return TDVP_E_ARG;
    return guarded(mps->ctx, [&] {
        TDVP_REQUIRE(mps->has_charges(), TDVP_E_STATE, "mps_get_charges: the state carries no charge labels");
        if (q_phys) std::copy(mps->qphys.begin(), mps->qphys.end(), q_phys);
        if (labels)
            for (int j = 0; j <= mps->N; ++j) labels = std::copy(mps->qbond[j].begin(), mps->qbond[j].end(), labels);
    });
}

int mpo_set_charges(tdvp_mpo mpo, const int* charges) {
    if (!mpo) return TDVP_E_ARG;
    return guarded(mpo->ctx, [&] {
        if (!charges) {
            mpo->charge.clear();
            return;
        }
        std::vector<std::vector<int>> c(mpo->N + 1);
        const int* p = charges;
        for (int j = 0; j <= mpo->N; ++j) {
            c[j].assign(p, p + mpo->w[j]);
            p += mpo->w[j];
        }
        TDVP_REQUIRE(c[0].size() == 1 && c[mpo->N].size() == 1 && c[0][0] == 0 && c[mpo->N][0] == 0, TDVP_E_ARG,
                     "mpo_set_charges: the boundary bonds must carry charge 0");
        mpo->charge = std::move(c);
    });
}

int mps_right_canonicalize(tdvp_ctx ctx, tdvp_mps mps) {
    if (!ctx || !mps) return TDVP_E_ARG;
    return guarded(ctx, [&] { right_canonicalize(ctx, mps); });
}

int mps_destroy(tdvp_mps mps) {
    if (!mps) return TDVP_E_ARG;
    (void)hipStreamSynchronize(mps->ctx->stream);
    delete mps;
    return TDVP_OK;
}

}  // extern "C"
