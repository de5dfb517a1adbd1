// Host-side objects and algorithms of the library.
#pragma once

#include "common.hpp"

#include <complex>

#include <functional>

namespace tdvp {

// Run `body`, translating exceptions into a status code and a message on ctx.
int guarded(tdvp_ctx ctx, const std::function<void()>& body);

// ------------------------------------------------------ MPO stage operator
// CSR form of the sparse operator between the two GEMMs of a contraction.
struct Mop {
    const int* row_ptr = nullptr;
    const int* col = nullptr;
    const void* val = nullptr;
    int rows = 0, cols = 0;
    bool fp64 = false;
    DevMem own_rp, own_col, own_val;  // storage when the operator is cached
};
// kind: see mop_build.  W1/W2 device tensors of dtype w_dt.  own = true
// keeps the operator in memory owned by m; otherwise context workspaces
// (valid until the next mop_make without ownership) are used.
void mop_make(tdvp_ctx ctx, Mop& m, int kind, const void* W1, const void* W2, Dt w_dt, int wl,
              int wm, int wr, int d, bool fp64, bool own);

// ------------------------------------------------------------ contractions
// y = H_eff x for nsite = 0, 1, 2 (Sec. III A).  Env layouts L[wl][chil][chil],
// R[wr][chir][chir]; x, y of shape [chil][D][chir] with D = d^nsite (1 for
// nsite = 0).  L and R have dtype env_dt, x has x_dt, y has y_dt.
struct HeffArgs {
    int nsite, chil, chir, d, wl, wr;
    const void* L;
    const void* R;
    Dt env_dt;
    const Mop* mop;
    bool fp64;
    int form;
};
void heff_apply(tdvp_ctx ctx, const HeffArgs& a, const void* x, Dt x_dt, void* y, Dt y_dt);
// GEMM form of the raw-pointer entry points: 4 for FP64, else the context's choice (default 3).
int raw_gemm_form(tdvp_ctx ctx, bool fp64);
double heff_flops(int nsite, int chil, int chir, int d, int wl, int wr);

// Left environment update with separate bra and ket tensors (Sec. III A):
// out[l][b'][b] = sum conj(Abra[a'][s'][b']) L[k][a'][a] W[k][l][s'][s] Aket[a][s][b]
// Abra [chil_b][d][chir_b], Aket [chil][d][chir] (complex128), L [wl][chil_b][chil],
// out [wr][chir_b][chir].  mop: kind 1 for W.
struct EnvArgs {
    int chil, chir, chil_b, chir_b, d, wl, wr;
    const void* Abra;
    const void* Aket;
    Dt a_dt;
    const Mop* mop;
    bool fp64;
    int form;
};
void env_left(tdvp_ctx ctx, const EnvArgs& a, const void* L, Dt l_dt, void* out, Dt out_dt);
// Right update: out[k][a][a'] = sum Aket[a][s][b] W[k][l][s'][s] R[l][b][b'] conj(Abra[a'][s'][b'])
// R [wr][chir][chir_b], out [wl][chil][chil_b].  mop: kind 3 for W.
void env_right(tdvp_ctx ctx, const EnvArgs& a, const void* R, Dt r_dt, void* out, Dt out_dt);
double env_flops(int chil, int chir, int d, int wl, int wr);

// ------------------------------------------------------------- Lanczos
// Linear operator on complex128 device vectors.
using MatVec = std::function<void(const double2* x, double2* y)>;
struct KrylovInfo {
    int k = 0;
    int matvecs = 0;
    bool converged = true;
};
// theta <- exp(-i tau H) theta with H Hermitian (Sec. III A, Lanczos).
// imaginary = true: theta <- exp(-tau H) theta instead.
KrylovInfo expm_krylov(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau,
                       int kmax, double tol, bool imaginary = false);
// theta <- exp(-i tau H) theta (imaginary: exp(-tau H) theta) by the
// truncated Taylor series with scaling of Al-Mohy and Higham (2011): the
// degree m <= 55 and the number of steps s from the table of theta_m and a
// Lanczos enclosure of the spectrum seen from theta; each step stops early
// once two consecutive terms fall below tol relative to the partial sum.
// info.k = the largest number of terms summed in a step.
KrylovInfo expm_taylor(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, double tau, double tol,
                       bool imaginary);
// theta <- normalised Ritz vector of the lowest Ritz value of H in the
// Krylov space of theta (Lanczos with full reorthogonalisation); stops when
// the residual norm of that Ritz pair is <= tol.  *energy (nullable) = the
// Ritz value.  theta must not vanish for a meaningful result.
KrylovInfo ground_krylov(tdvp_ctx ctx, const MatVec& op, double2* theta, int64_t n, int kmax, double tol,
                         double* energy);
// Eigen-decomposition of the symmetric tridiagonal k x k matrix with
// diagonal alpha and off-diagonal beta (host): evals[k] (unordered) and
// z[r*k + c] = entry rows[r] of the c-th eigenvector, for the listed rows.
void tridiag_eigen(const std::vector<double>& alpha, const std::vector<double>& beta, const std::vector<int>& rows,
                   std::vector<double>& evals, std::vector<double>& z);

// True when every bond j = 1..N-1 of chi[0..N] holds min(chi_max, d^min(j, N-j)).
bool chi_saturated(const std::vector<int>& chi, int d, int chi_max);

// Truncation rule of a two-site split (Sec. III C, Eq. discweight; Sec. III D
// relative cut): chi_w = smallest rank whose discarded weight is <= w_max,
// chi_eps = count of s >= eps s_1, chi = max(1, min(chi_w, chi_max, chi_eps)),
// then lowered while s_{chi+1} is within 1e-10 of s_chi (multiplet guard).
// s descending; returns chi and the discarded weight in w.
struct TruncRule {
    int chi_max;
    double w_max, eps;
    bool guard;
};
int truncation_rank(const std::vector<double>& s, const TruncRule& r, double& w);

// ------------------------------------------------------------- solvers
// Row-major QR: M [rows][cols] = Q [rows][k] R [k][cols], k = min(rows, cols).
void qr_rowmajor(tdvp_ctx ctx, const double2* M, int rows, int cols, double2* Q, double2* R);
// Row-major LQ: M [rows][cols] = L [rows][k] Q [k][cols].
void lq_rowmajor(tdvp_ctx ctx, const double2* M, int rows, int cols, double2* L, double2* Q);
// Row-major thin SVD: M = U [rows][k] diag(S) Vh [k][cols]; S on host and device.
struct SvdResult {
    double2* U;   // row-major [rows][k]  (workspace)
    double2* Vh;  // row-major [k][cols]  (workspace)
    double* S_dev;
    std::vector<double> S;
    int k;
};
SvdResult svd_rowmajor(tdvp_ctx ctx, const double2* M, int rows, int cols);
// Eigen-decomposition of the Gram (reduced density) matrix of M [rows][cols]:
// left: Theta Theta^dag (n = rows), else Theta^dag Theta (n = cols).  s =
// sqrt of the eigenvalues, descending (negative rounding noise -> 0); vecs
// row-major [n][n], row c = conj of the c-th eigenvector.  Workspace-backed.
struct GramResult {
    double2* vecs;
    std::vector<double> s;
    int n;
};
GramResult gram_eigen(tdvp_ctx ctx, const double2* M, int rows, int cols, bool left);
// Eigen-decomposition of the Hermitian matrix of order n at G (row-major,
// leading dimension ld) on the given handle (its stream), nothing read back:
// on return row c is the conjugate of the eigenvector of the c-th smallest
// eigenvalue; eigenvalues to ev, n-element scratch E, solver code to info
// (0 = converged).  (rocSOLVER's strided-batched divide and conquer was not
// used for several such matrices: it returned non-finite eigenvectors for
// matrices zero-padded to a common order, whose tridiagonal form splits.)
void heevd_slot(rocblas_handle h, double2* G, int ld, int n, double* ev, double* E, int* info);
// Largest dense problems a context's solver calls will see: reserves the
// device memory rocSOLVER needs for them (rocBLAS's device-memory size query)
// and the named workspaces of the calls above, and installs that memory as
// the handle's workspace, so that the calls themselves allocate nothing.
// Sizes <= 0 are skipped.  Grow-only: a later reservation for smaller
// problems keeps the current memory.
struct SolverSizes {
    int eig_n = 0;                 // gram_eigen order above the one-workgroup Jacobi limit
    int svd_rows = 0, svd_cols = 0;
    int qr_rows = 0, qr_cols = 0;  // qr_rowmajor
    int lq_rows = 0, lq_cols = 0;  // lq_rowmajor
};
void reserve_solver_workspace(tdvp_ctx ctx, const SolverSizes& s);
// Resolves (once per device, with that device current) the device address of
// the fixed scratch array used by apply_heff_noalloc; failures are recorded
// and reported by that call.
void scratch_setup(int device);
// apply_heff body: checks, MPO-stage operator, pipeline (workspaces by name).
void heff_raw_call(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm, int wr,
                   const void* L, const void* W1, const void* W2, const void* R, const void* theta, void* out);
// Matrix-pencil fit f(r) ~ Re sum_k c_k lambda_k^r of samples f(1..R)
// (optionally refined); returns the maximum absolute error on r = 1..R.
double fit_exponentials(const std::vector<double>& f, int K, bool refine, std::vector<std::complex<double>>& c,
                        std::vector<std::complex<double>>& lam);
// Row-major complex128 product C [m][n] = A [m][k] B [k][n] (FP64 MFMA).
void zgemm_rowmajor(tdvp_ctx ctx, const double2* A, const double2* B, double2* C, int m, int k, int n);

}  // namespace tdvp

// ------------------------------------------------------------------ objects

struct tdvp_mpo_s {
    tdvp_ctx ctx = nullptr;
    int N = 0, d = 0;
    std::vector<int> w;                           // [N+1]
    std::vector<std::vector<double>> host;        // c128 interleaved per site
    std::vector<tdvp::DevMem> dev128, dev64;      // device copies
    std::map<std::tuple<int, int, bool>, std::unique_ptr<tdvp::Mop>> mops;  // (kind, site, fp64)
    std::vector<std::vector<int>> charge;         // U(1) charges of the MPO bonds [N+1][w_j] (empty: none)
    const tdvp::Mop& mop(int kind, int site, bool fp64);
    const void* W(int site, tdvp::Dt dt);
};

struct tdvp_mps_s {
    tdvp_ctx ctx = nullptr;
    int N = 0, d = 0;
    std::vector<int> chi;                 // [N+1]
    std::vector<tdvp::DevMem> A;          // c128 site tensors
    double w_total = 0.0;
    // cached environments for (mpo, dtype)
    const tdvp_mpo_s* env_mpo = nullptr;
    tdvp::Dt env_dt = tdvp::Dt::C128;
    bool env_valid = false;
    std::vector<tdvp::DevMem> L, R;       // L[j]: [w_j][chi_j][chi_j], R[j]: [w_{j+1}][chi_{j+1}][chi_{j+1}]
    // U(1) labels (empty: none): charge of each physical state and of each
    // bond index, [N+1][chi_j], non-decreasing along every bond
    std::vector<int> qphys;
    std::vector<std::vector<int>> qbond;
    bool has_charges() const { return !qbond.empty(); }
    void clear_charges() {
        qphys.clear();
        qbond.clear();
    }
    size_t tensor_elems(int j) const { return (size_t)chi[j] * d * chi[j + 1]; }
    void set_tensor_dev(int j, int chil, int chir);  // (re)allocate site j storage
};
