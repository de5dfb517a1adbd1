/*
 * tdvp.h -- C ABI of the MI355X (gfx950) TDVP library.
 *
 * Time evolution of matrix product states (MPS) under long-range matrix
 * product operator (MPO) Hamiltonians by the time-dependent variational
 * principle, after Secular et al., "Parallel time-dependent variational
 * principle algorithm for matrix product states" (arXiv:1912.06127).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Sites are 1-based in the documentation and 0-based in `site` arguments.
 *  - Complex numbers are interleaved (re, im): complex64 = 2 x float,
 *    complex128 = 2 x double, the layout of torch.complex64/complex128.
 *  - All arrays are row-major, last index fastest:
 *      MPS site tensor   A[a][s][b]        [chi_l][d][chi_r]      (Sec. II A)
 *      two-site state    Theta[a][s1][s2][b]                      (Sec. III A)
 *      bond matrix       C[a][b]           [chi_l][chi_r]
 *      MPO site tensor   W[k][l][s'][s]    [w_l][w_r][d][d], s' output (Sec. II C)
 *      left environment  L[k][a'][a]       [w][chi_bra][chi_ket]  = beta_j[a',k,a]
 *      right environment R[l][b][b']       [w][chi_ket][chi_bra]  = gamma_j[b',l,b]
 *  - Every call returns an int status (TDVP_OK = 0).  No call aborts or
 *    throws across the ABI; a failing call stores a message readable with
 *    tdvp_last_error(ctx).  Kernel faults are asynchronous and surface at
 *    the next synchronising call (tdvp_ctx_sync, any host read-back).
 *  - Raw-pointer calls (apply_heff, env_update) take device pointers owned
 *    by the caller, enqueue work on the context stream and return without
 *    synchronising; they neither free nor retain the pointers.
 *  - Handles (tdvp_ctx, tdvp_mps, tdvp_mpo) are opaque and owned by the
 *    library until the matching *_destroy call.  A context is used by one
 *    host thread at a time.
 */
#ifndef TDVP_H
#define TDVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum tdvp_status {
    TDVP_OK = 0,
    TDVP_E_ARG = 1,      /* null pointer, bad enum, negative size */
    TDVP_E_SHAPE = 2,    /* inconsistent tensor dimensions */
    TDVP_E_DTYPE = 3,    /* unsupported dtype */
    TDVP_E_NOMEM = 4,    /* device or host allocation failed */
    TDVP_E_HIP = 5,      /* HIP runtime or kernel error */
    TDVP_E_NOCONV = 6,   /* Krylov did not converge (strict mode only) */
    TDVP_E_NUMERIC = 7,  /* NaN or Inf met */
    TDVP_E_STATE = 8,    /* object in a state that does not allow the call */
    TDVP_E_SOLVER = 9    /* dense solver (QR/SVD) reported failure */
};

typedef enum { TDVP_C64 = 0, TDVP_C128 = 1 } tdvp_dtype;

typedef struct tdvp_ctx_s* tdvp_ctx;
typedef struct tdvp_mps_s* tdvp_mps;
typedef struct tdvp_mpo_s* tdvp_mpo;
typedef struct tdvp_seg_s* tdvp_seg;

/* Optional device allocator.  alloc returns a device pointer of at least
 * `bytes` bytes usable on `stream`, or NULL; free releases it.  With NULL
 * callbacks the library calls hipMalloc/hipFree itself. */
typedef void* (*tdvp_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*tdvp_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues all work on
 * `hip_stream` (a hipStream_t; NULL = the default stream). */
int tdvp_ctx_create(int device, void* hip_stream, tdvp_alloc_fn alloc_fn,
                    tdvp_free_fn free_fn, void* user, tdvp_ctx* out);
int tdvp_ctx_destroy(tdvp_ctx ctx);
/* Message of the last failing call on this context ("" if none).  The
 * string stays valid until the next call on the context. */
const char* tdvp_last_error(tdvp_ctx ctx);
/* Wait for all work on the context stream; reports asynchronous errors. */
int tdvp_ctx_sync(tdvp_ctx ctx);
/* Library version string, e.g. "tdvp-gfx950 0.1". */
const char* tdvp_version(void);

/* Kernel timing.  With profiling on, every kernel launch of the library is
 * bracketed by a HIP event pair on the context stream (a few microseconds of
 * overhead per launch).  tdvp_profile_read synchronises the stream, returns
 * per-kernel totals accumulated since the previous read and clears them:
 * names [max_entries][64] (NUL-terminated), ms = summed event time, flops /
 * bytes = summed algorithmic work (8 real flops per complex multiply-add;
 * compulsory operand bytes), count = launches; *n_out = entries written. */
int tdvp_profile_enable(tdvp_ctx ctx, int on);
/* Real-GEMM form of the complex products in apply_heff, env_update and
 * apply_heff_batched on this context: 0 = default (3M for TDVP_C64, 4M for
 * TDVP_C128), 3 = three real products (C64 only; C128 always uses 4M),
 * 4 = four real products.  TDVP_E_ARG for any other value.  Time steps take
 * the form from their options. */
int tdvp_ctx_set_gemm_form(tdvp_ctx ctx, int form);
int tdvp_profile_read(tdvp_ctx ctx, int max_entries, char* names, double* ms, double* flops,
                      double* bytes, long* count, int* n_out);

/* -------------------------------------------------------------------- MPO */

/* Long-range spin-chain Hamiltonian (Sec. II C, Sec. IV):
 *   H = sum_{i<j} f(j-i) sum_a g_a A_a(i) B_a(j) + h sum_i X(i).
 * With K > 0, f(r) = Re sum_k c_k lambda_k^r (sum of exponentials,
 * Sec. II C): bond dimension m = n_terms K + 2.  The weights and decay
 * factors are either given (c and lambda) or, with c = lambda = NULL,
 * fitted by the library to the power law f(r) = r^-alpha on
 * r = 1..fit_rmax (fit_rmax <= 0: N-1) with tdvp_fit_exponentials (the
 * couplings' strength goes into g).  With K = 0 every distance
 * r = 1..N-1 has its own chain of bond states and coupling[r-1] = f(r)
 * (exact MPO, bond dimension n_terms (N-1) + 2).
 * Operators are d x d complex128 matrices, host memory, [s'][s]. */
typedef struct {
    int N;                  /* number of sites, >= 2 */
    int d;                  /* local dimension */
    int n_terms;            /* number of long-range terms n_H */
    const double* g;        /* [n_terms] real prefactors g_a */
    const double* A_ops;    /* [n_terms][d][d] complex128 */
    const double* B_ops;    /* [n_terms][d][d] complex128 */
    int K;                  /* exponentials per term; 0 = exact MPO */
    const double* c;        /* [K] complex128 weights c_k, or NULL (fit) */
    const double* lambda;   /* [K] complex128 decay factors lambda_k, or NULL (fit) */
    const double* coupling; /* [N-1] real f(1..N-1) (K = 0) */
    const double* onsite;   /* [d][d] complex128 X, or NULL */
    double h;               /* field strength multiplying X */
    double alpha;           /* fitted power r^-alpha (K > 0, c = lambda = NULL) */
    int fit_rmax;           /* fit range r = 1..fit_rmax; <= 0: N-1 */
    int fit_refine;         /* 1: Levenberg-Marquardt refinement of the fit */
} tdvp_mpo_spec;

/* Build the MPO on the device.  fit_max_abs_err (nullable) receives the
 * maximum of |f(r) - r^-alpha| over the fit range when the library fitted
 * the exponentials, else 0.  Errors: TDVP_E_SHAPE for bad sizes,
 * TDVP_E_ARG for missing operators or only one of c / lambda, the fit's
 * errors as for tdvp_fit_exponentials. */
int mpo_longrange(tdvp_ctx ctx, const tdvp_mpo_spec* spec, tdvp_mpo* out, double* fit_max_abs_err);

/* Sum-of-exponentials fit (Sec. II C; the method of Pirvu et al. that the
 * paper cites, read as a matrix pencil): f(r) ~ Re sum_k c_k lambda_k^r for
 * the samples f[0..R-1] = f(1..R).  The Hankel matrix of the samples is cut
 * to its K dominant right singular vectors (one-sided Jacobi SVD), the
 * lambda_k are the eigenvalues of the shift operator on them and the c_k
 * follow by least squares on all samples.  refine = 1 adds
 * Levenberg-Marquardt iterations with Lawson reweighting towards the
 * minimax fit (kept only when the maximum error drops).  Host only (no
 * context, no device work).  c_out, lam_out: [K] complex128 (interleaved);
 * max_abs_err (nullable): max_r |Re sum - f(r)|.  Errors: TDVP_E_ARG for
 * K < 1, R < 2K or null pointers, TDVP_E_NUMERIC for non-finite samples or
 * a rank-deficient problem, TDVP_E_NOCONV if the eigenvalue iteration
 * fails. */
int tdvp_fit_exponentials(const double* f, int R, int K, int refine, double* c_out, double* lam_out,
                          double* max_abs_err);
/* tdvp_fit_exponentials of f(r) = r^-alpha on r = 1..rmax. */
int tdvp_fit_power_law(double alpha, int K, int rmax, int refine, double* c_out, double* lam_out,
                       double* max_abs_err);
/* MPO from explicit tensors: w[0..N] bond dimensions (w[0] = w[N] = 1),
 * W_host the concatenation of the N site tensors [w_j][w_{j+1}][d][d]
 * complex128 (host). */
int mpo_from_tensors(tdvp_ctx ctx, int N, int d, const int* w, const double* W_host,
                     tdvp_mpo* out);
int mpo_get_info(tdvp_mpo mpo, int* N, int* d, int* w /* [N+1], nullable */);
/* U(1) charges of the MPO bond indices (the quantum-number blocks the
 * paper's symmetric tensors use, Supplemental Material, Implementation):
 * charges = the concatenation of bonds 0..N, w_j integers each; index k of
 * bond j carries the charge its operator string adds, so W_j[k][l][s'][s]
 * may be non-zero only where c(l) = c(k) + q(s') - q(s).  Both boundary
 * bonds must carry 0.  NULL clears them.  With charges on both the MPO and
 * the MPS (mps_set_charges), tdvp2_step and dmrg2_sweep run in U(1) mode:
 * block-sparse matvecs and environment updates (as apply_heff_u1 /
 * env_update_u1) and, in the two-site splits, one SVD per charge sector of
 * the new bond with one truncation over all sectors.  tdvp1_step (and the
 * one-site part of tdvp_hybrid_step) refuses U(1) mode with TDVP_E_ARG: its
 * dense QR / LQ gauge moves would mix the sectors.  Errors: TDVP_E_ARG for
 * non-zero boundary charges. */
int mpo_set_charges(tdvp_mpo mpo, const int* charges);
int mpo_get_tensor(tdvp_mpo mpo, int site, double* W_host);
int mpo_destroy(tdvp_mpo mpo);

/* -------------------------------------------------------------------- MPS */

/* MPS with bond dimensions chi[0..N] (chi[0] = chi[N] = 1, chi[j-1] <=
 * d chi[j]) in right-canonical form with the orthogonality centre on
 * site 1 (Eqs. mixed-mps1/2).  basis_state[N] (entries in 0..d-1) gives a
 * product state padded to chi by unit vectors: row 0 of every site holds
 * the product state, the remaining rows are the unit vectors e_(s,b) in
 * lexicographic order.  basis_state = NULL gives a random state from
 * `seed` (complex Gaussian entries, then right-orthonormalised). */
int mps_init(tdvp_ctx ctx, int N, int d, const int* chi, const int* basis_state,
             uint64_t seed, tdvp_mps* out);
int mps_get_info(tdvp_mps mps, int* N, int* d, int* chi /* [N+1], nullable */);
/* Copy site tensor `site` (0-based) to host as complex128. */
int mps_get_tensor(tdvp_mps mps, int site, double* host);
/* Replace site tensor `site` by host complex128 data of shape
 * [chil][d][chir]; chil/chir must match the neighbours' bonds once all
 * sets are done.  Invalidates cached environments.  The caller is
 * responsible for the canonical form that tdvp*_step assumes (sites 2..N
 * right-orthonormal); mps_right_canonicalize restores it. */
int mps_set_tensor(tdvp_mps mps, int site, const double* host, int chil, int chir);
/* U(1) labels of the state: q_phys [d] the charge of each physical state,
 * labels the concatenation of bonds 0..N, chi_j integers each, non-decreasing
 * along every bond (a charge sector is a contiguous index range); bond j
 * carries the charge of the block to its left, so site j may be non-zero
 * only where q(a) + q(s) = q(b).  The caller guarantees that the tensors
 * obey these rules (the U(1) kernels read only the allowed blocks).  Both
 * NULL clears the labels; mps_set_tensor, mps_apply_site and a step with an
 * MPO without charges also clear them.  Two-site steps in U(1) mode rewrite
 * the labels of the bonds they truncate.  Errors: TDVP_E_ARG for unsorted
 * labels or only one of the two arrays. */
int mps_set_charges(tdvp_mps mps, const int* q_phys, const int* labels);
/* The current labels (layout as mps_set_charges; sizes from mps_get_info);
 * either output may be NULL.  TDVP_E_STATE if the state carries none. */
int mps_get_charges(tdvp_mps mps, int* q_phys, int* labels);
/* Right-orthonormalise sites N..2 by successive LQ decompositions; the
 * norm stays in site 1 (LQ keeps the U(1) block structure, so labels stay
 * valid). */
int mps_right_canonicalize(tdvp_ctx ctx, tdvp_mps mps);
int mps_destroy(tdvp_mps mps);
/* Apply the d x d operator op (host, complex128, op[s'][s] row-major) to
 * the physical index of one site: A[a][s'][b] <- sum_s op[s'][s] A[a][s][b]
 * (the sigma^z_k(0) of the correlation function of Sec. IV).  A unitary op
 * keeps the canonical form; for any other the norm and gauge are the
 * caller's.  d <= 16; cached environments of the MPS are invalidated. */
int mps_apply_site(tdvp_ctx ctx, tdvp_mps mps, int site, const double* op);

/* ------------------------------------------------------------- time steps */

typedef struct {
    tdvp_dtype compute;  /* TDVP_C64: H_eff and environment contractions in
                            complex FP32 on MFMA (FP32 accumulation), Lanczos,
                            QR/SVD in FP64.  TDVP_C128: everything FP64. */
    int krylov_max;      /* maximum Krylov dimension (paper: 8) */
    double krylov_tol;   /* a-posteriori error tolerance (paper: 1e-6) */
    int chi_max;         /* maximum bond dimension (2TDVP) */
    double w_max;        /* maximum discarded weight per SVD, Eq. (discweight) */
    double eps_rel;      /* relative singular-value cut eps (Sec. III D) */
    int multiplet_guard; /* 1: never cut inside a degenerate multiplet */
    int strict;          /* 1: Krylov non-convergence returns TDVP_E_NOCONV */
    int gemm_form;       /* 0 = default (3M for FP32, 4M for FP64), 3 = 3M, 4 = 4M;
                            the FP64 path always uses 4M */
    int svd_mode;        /* two-site split: 1 = SVD (one-sided Jacobi), 2 = eigen-
                            decomposition of the reduced density matrix Theta Theta^dag
                            (or Theta^dag Theta; eigenvalues = squared singular values,
                            absolute accuracy ~1e-16 ||Theta||^2), 0 = automatic:
                            density matrix when w_max >= 1e-13, else SVD */
    int imaginary;       /* 1: imaginary time (the paper's Discussion): the local
                            steps apply exp(-tau H_eff) instead of exp(-i tau H_eff)
                            (backward steps exp(+tau H_eff)) and the state is
                            renormalised after the step; dt is then the
                            imaginary-time step.  0: real time. */
    int exp_method;      /* local exponentials: 0 = Lanczos (Sec. III A), 1 = truncated
                            Taylor series with scaling (Al-Mohy and Higham 2011, the
                            alternative named with the Lanczos method in Sec. III A):
                            degree m <= 55 and s steps from the backward-error bounds
                            theta_m (unit roundoff 2^-53) and a 16-step Lanczos
                            enclosure of the spectrum, shifted to its midpoint;
                            terms stop at max(2^-53, krylov_tol) relative.
                            krylov_max does not apply; TDVP_E_ARG if |dt| ||H_eff||
                            would need more than 1e5 scaling steps.  TDVP_E_ARG for
                            other values. */
    int u1_block_min;    /* U(1) mode (charge labels on the state and the MPO):
                            local problems and environment updates with
                            chi_left * chi_right >= u1_block_min run on the
                            block-sparse kernels, smaller ones on the dense
                            kernels, which keep the blocks exactly (an entry
                            outside them is a sum of products with a zero factor);
                            the splits are sector by sector either way.  0 =
                            default (256 * 256), 1 = always blocks; TDVP_E_ARG
                            if negative. */
} tdvp_opts;

typedef struct {
    double w_step;       /* discarded weight of this step */
    double w_total;      /* cumulative discarded weight of this MPS */
    double seconds;      /* host wall time of the call */
    double flops;        /* algorithmic flops of H_eff and environment work */
    int chi_peak;        /* largest bond dimension after the step */
    int matvecs;         /* number of H_eff applications */
    int krylov_max_used; /* largest Krylov dimension used */
    int flags;           /* bit 0: a Krylov run hit krylov_max unconverged;
                            bit 1 (seg_step): the one-site schedule ran */
} tdvp_stats;

/* Fill opts with defaults: C128, krylov_max 40, tol 1e-13, chi_max
 * 1<<30, w_max 0, eps_rel 0, guard on, strict off, gemm_form 0, svd_mode 0,
 * real time, Lanczos exponentials. */
int tdvp_opts_default(tdvp_opts* opts);

/* One symmetric one-site TDVP step of size dt (Sec. II D, Eq. proj1site):
 * forward one-site and backward zero-site updates in a left-to-right and a
 * right-to-left sweep, the last site evolved once by the full dt.  Bond
 * dimensions stay fixed.  The MPS must be right-canonical with the centre
 * on site 1, and is left so. */
int tdvp1_step(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double dt,
               const tdvp_opts* opts, tdvp_stats* stats);
/* One symmetric two-site TDVP step (Sec. II D, Eq. proj2site; Sec. III A):
 * forward two-site and backward one-site updates, truncated SVD splits
 * with w_max, chi_max and eps_rel (Sec. III C, III D), the right-most pair
 * evolved once by the full dt.  Same canonical-form contract as tdvp1_step. */
int tdvp2_step(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double dt,
               const tdvp_opts* opts, tdvp_stats* stats);
/* One step of the hybrid scheme the paper's Discussion proposes: a two-site
 * step while the bond dimensions can still grow, a one-site step once
 * chi_max is saturated, i.e. once every bond j = 1..N-1 holds
 * min(opts->chi_max, d^min(j, N-j)) (the largest dimension the truncation
 * and the Hilbert space allow; one-site steps keep it so).  *one_site
 * (nullable) is set to 1 when the one-site step ran, else 0.  Same
 * canonical-form contract and errors as tdvp1_step / tdvp2_step. */
int tdvp_hybrid_step(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double dt,
                     const tdvp_opts* opts, tdvp_stats* stats, int* one_site);
/* One sweep of two-site DMRG for the ground state (the quench experiments of
 * Sec. IV start from two-site DMRG ground states; the sweep uses the same
 * environments, effective Hamiltonian and truncated splits as a 2TDVP step,
 * Sec. III A): each pair in a left-to-right and a right-to-left pass is
 * replaced by the lowest Ritz vector of its H_eff (Lanczos with full
 * reorthogonalisation, stopped when the Ritz residual is <= krylov_tol or
 * after krylov_max vectors) and split with the truncation of opts.  The
 * state is renormalised at the end; *energy (nullable) = the last Ritz
 * value, the variational energy of the state after the sweep.  Same
 * canonical-form contract as tdvp2_step; stats as for a time step (flags
 * bit 0: a Lanczos run hit krylov_max; TDVP_E_NOCONV with strict). */
int dmrg2_sweep(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, const tdvp_opts* opts,
                tdvp_stats* stats, double* energy);

/* ------------------------------------- segment-parallel two-site TDVP ---- */
/* Sec. III B (Fig. partitioning) on one device.  The state is held in the
 * inverse canonical gauge of Sec. II A: Psi_j = Lambda_{j-1} Gamma_j Lambda_j
 * (complex128 [chi_j][d][chi_{j+1}]) and V_j = 1/Lambda_j on every bond, plus
 * one stored left and right environment per site (in the compute dtype).
 * The chain is cut into p contiguous segments (p = 1 or even, each of at
 * least two sites).  A time step has two halves; in the first the two
 * central segments sweep away from the centre and neighbours alternate, in
 * the second every direction is reversed.  Each segment sweeps its own sites
 * with two-site forward steps (dt/2) and one-site backward steps (dt/2);
 * the pair straddling two segments (and each chain-end pair) is evolved
 * before the sweeps (dt/2, first half, where the segments depart), after
 * them where they meet (dt in the first half, the merged turning point of
 * Sec. III A; dt/2 in the second), by the left segment, after which both
 * environments across that bond are rebuilt.  Environments across a
 * departing boundary keep their last value (out of date, Sec. III D).  At
 * p = 1 the step equals tdvp2_step.  The paper's diagrams of the parallel
 * step are not in its text; this schedule is the library's reading.
 *
 * All segments of a phase update at once: their Lanczos exponentiations
 * (krylov_k steps each, fixed, as in the paper's runs) share one grouped
 * launch per contraction stage per Krylov iteration; splits and environment
 * refreshes run per segment.  With static_shapes every bond keeps its
 * initial dimension as its cap, so each phase has a fixed memory layout and
 * use_graph can capture its batched exponentiation in a HIP graph (captured
 * on first use, replayed afterwards, re-captured if library workspaces
 * move). */
typedef struct {
    tdvp_dtype compute;  /* matvec / environment precision; must equal the
                            dtype given to seg_init.  Lanczos and splits FP64. */
    int krylov_k;        /* Lanczos steps per exponentiation, 1..16 (paper: 8) */
    int chi_max;         /* bond dimension cap */
    double w_max;        /* discarded weight per split, Eq. (discweight) */
    double eps_rel;      /* relative singular-value cut (Sec. III D) */
    int multiplet_guard; /* 1: never cut inside a degenerate multiplet */
    int static_shapes;   /* 1: bond j never exceeds its initial dimension */
    int batched;         /* 1: one batched exponentiation per phase; 0: one
                            segment after the other (reference path) */
    int use_graph;       /* 1: replay each phase's exponentiation from a HIP
                            graph (needs batched and static_shapes) */
    int svd_mode;        /* 0: density-matrix split, SVD when a kept singular
                            value is below 1e-6 of the largest; 1: SVD; 2:
                            density matrix always */
    int one_site;        /* 1: the parallel one-site scheme proposed in the
                            Discussion, with two-site boundary pairs (a reading):
                            one-site sweeps inside the segments, zero-site bond
                            steps (QR/LQ, exponential, absorbed into the next site),
                            the boundary pairs and their timing as in the two-site
                            schedule; bond dimensions change only at boundary
                            splits.  Inner bonds then hold V_j = 1 (the mixed
                            canonical form inside segments) until
                            seg_reorthonormalize; a two-site step before that
                            returns TDVP_E_STATE.  Inner segments need at least
                            three sites (TDVP_E_SHAPE).  At one segment it is the
                            serial one-site step.  0: the two-site schedule
                            (Sec. III B).  2: the hybrid scheme of the Discussion
                            on segments: two-site steps until every bond holds
                            min(chi_max, d^min(j, N-j)) (and, with static shapes, its
                            initial dimension), one-site steps from then on
                            (stats flags bit 1 tells which ran). */
    int max_phases;      /* > 0: stop the step after this many phases of its
                            schedule (inspection and testing of single phases;
                            the state is then left mid-step and the next call
                            starts a new step); 0: the whole step */
} tdvp_seg_opts;

/* Defaults: C64, krylov_k 8, chi_max 1<<30, w_max 0, eps_rel 0, guard on,
 * static_shapes 1, batched 1, use_graph 0, svd_mode 0, one_site 0, max_phases 0. */
int tdvp_seg_opts_default(tdvp_seg_opts* opts);

/* Build the segmented state from host site tensors (complex128
 * [chi[j]][d][chi[j+1]], C order; copied, the caller keeps ownership):
 * right-orthonormalisation, then a left-to-right split sweep that yields
 * Psi_j and V_j (the Schmidt coefficients must be non-zero), then every left
 * and right environment (Sec. III B: all initial environments are built
 * sequentially).  chi must be isometry-feasible (chi_{j+1} <= d chi_j and
 * chi_j <= d chi_{j+1}) with chi_0 = chi_N = 1; compute is the dtype of the
 * environments and of the matvecs of later steps.  Errors: TDVP_E_SHAPE for
 * inconsistent sizes, TDVP_E_NUMERIC for a zero Schmidt coefficient. */
int seg_init(tdvp_ctx ctx, tdvp_mpo mpo, int N, int d, const int* chi, const void* const* tensors,
             int nseg, const int* seg_sizes, tdvp_dtype compute, tdvp_seg* out);
/* One time step of size dt.  TDVP_E_NUMERIC if a Krylov recursion produced a
 * non-finite value or a kept singular value is zero.  The per-segment splits
 * and bond steps of a phase run on up to TDVP_SEG_LANES (default 8) library
 * worker threads, each with its own stream and rocBLAS handle; their
 * workspaces come from hipMalloc (the context's allocator callback is called
 * only from the calling thread, which also sizes every state buffer and every
 * solver workspace of the phase before the workers start). */
int seg_step(tdvp_ctx ctx, tdvp_seg seg, tdvp_mpo mpo, double dt, const tdvp_seg_opts* opts,
             tdvp_stats* stats);
/* N, d, the bond dimensions chi[N+1] and the cumulative discarded weight
 * (any output may be NULL). */
int seg_get_info(tdvp_seg seg, int* N, int* d, int* chi, double* w_total);
/* Psi_j to host memory (complex128 [chi_j][d][chi_{j+1}]). */
int seg_get_psi(tdvp_seg seg, int j, void* out);
/* V_j = 1/Lambda_j of bond j (between sites j and j+1, 0-based) to host
 * memory (double [chi_{j+1}]); after one-site steps inner bonds of segments
 * hold 1 (see tdvp_seg_opts.one_site). */
int seg_get_bond(tdvp_seg seg, int j, double* out);
int seg_destroy(tdvp_seg seg);
/* <psi|psi> of the state Psi_0 V_0 Psi_1 ... Psi_{N-1} as it stands, in FP64
 * (left transfer matrices on the device).  The parallel updates break the
 * gauge conditions at the segment boundaries, so this drifts from 1 as a run
 * goes on (Sec. III D, item ii; Fig. reorth).  *out receives the value. */
int seg_norm2(tdvp_ctx ctx, tdvp_seg seg, double* out);
/* Serial repair of a segment run (Sec. III D, Fig. reorth): the bond
 * matrices are folded into the site tensors, the state is brought back to the
 * inverse canonical gauge of the normalised state (the same right
 * orthonormalisation and split sweep as seg_init) and every environment is
 * recomputed from it.  Bond dimensions are kept and nothing is truncated, so
 * the state changes only by its normalisation.  mpo must be the MPO of the
 * run.  Errors: TDVP_E_SHAPE if the MPO does not match, TDVP_E_NUMERIC if a
 * Schmidt coefficient vanished; after an error the state is unspecified and
 * must only be destroyed. */
int seg_reorthonormalize(tdvp_ctx ctx, tdvp_seg seg, tdvp_mpo mpo);
/* The operations of one half step (host only, no device work): for op n,
 * phase[n] (ops of one phase run together), kind[n] (2: pair (site, site+1)
 * forward, 1: one-site backward), site[n] (0-based) and tau[n] (forward
 * time; negative for backward steps).  n_out receives the op count;
 * TDVP_E_SHAPE if it exceeds max_ops (outputs may then be NULL). */
int seg_schedule(int nseg, const int* seg_sizes, double dt, int first_half, int max_ops, int* phase,
                 int* kind, int* site, double* tau, int* n_out);
/* The operations of one half step of the one-site schedule
 * (tdvp_seg_opts.one_site), host only, in the layout of seg_schedule: kind 2
 * boundary pair forward, 1 site forward, 3 bond (site, site+1) backward while
 * sweeping right, 4 the same while sweeping left.  TDVP_E_SHAPE also when an
 * inner segment has fewer than three sites. */
int seg_schedule1(int nseg, const int* seg_sizes, double dt, int first_half, int max_ops, int* phase,
                  int* kind, int* site, double* tau, int* n_out);

/* ------------------------------------------------------ raw-pointer kernels */

/* Effective Hamiltonian applied to a local state (Sec. III A, Fig. update;
 * cost Eq. eqnscaling):
 *   nsite = 2: out[a'][s1'][s2'][b'] = sum L[k][a'][a] W1[k][l][s1'][s1]
 *              W2[l][n][s2'][s2] R[n][b][b'] theta[a][s1][s2][b]
 *              (W1: [wl][wm][d][d], W2: [wm][wr][d][d], L: [wl][chil][chil],
 *               R: [wr][chir][chir])
 *   nsite = 1: out[a'][s'][b'] = sum L[k][a'][a] W1[k][l][s'][s] R[l][b][b'] theta[a][s][b]
 *              (W1: [wl][wr][d][d]; W2 unused, wm ignored)
 *   nsite = 0: out[a'][b'] = sum_k L[k][a'][a] C[a][b] R[k][b][b'] (bond
 *              evolution of Eq. proj1site; wl = wr; W1, W2 unused, d ignored)
 * All device pointers; every tensor has `dtype` (TDVP_C64 computes in FP32
 * on MFMA with FP32 accumulation, TDVP_C128 in FP64).  W1/W2 are device
 * copies of the MPO tensors.  `out` must not alias any input. */
int apply_heff(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d,
               int wl, int wm, int wr, const void* L, const void* W1, const void* W2,
               const void* R, const void* theta, void* out);

/* Adjoint of apply_heff for reverse-mode differentiation (gradients in the
 * convention g = dl/dRe z + i dl/dIm z for a real loss l, i.e. the
 * convention of torch's complex autograd).  Given the gradient ybar of the
 * output, computes (each output optional, NULL = skip):
 *   theta_bar = H_eff^dagger ybar                       [chil][D][chir]
 *   L_bar[k][a'][a] = sum ybar[a' s' b'] conj(W R theta)  [wl][chil][chil]
 *   R_bar[n][b][b'] = sum conj(L W theta) ybar           [wr][chir][chir]
 *   W1_bar[k][l][s'][s]  (nsite = 1 only)               [wl][wr][d][d]
 * W2_bar must be NULL (MPO gradients are provided for the one-site form used
 * by one-site TDVP).  Same shapes, layouts, dtype and stream semantics as
 * apply_heff; outputs must not alias inputs. */
int apply_heff_adjoint(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d,
                       int wl, int wm, int wr, const void* L, const void* W1, const void* W2,
                       const void* R, const void* theta, const void* ybar, void* theta_bar,
                       void* L_bar, void* W1_bar, void* W2_bar, void* R_bar);

/* Many independent effective-Hamiltonian applications at once (the
 * segments of Sec. III B as one batch): descriptor i has the meaning of the
 * arguments of apply_heff; sizes and nsite may differ between descriptors.
 * One grouped launch per contraction stage serves all of them.  All device
 * pointers of `dtype`; outputs must not alias any input or another output.
 * Synchronises the context stream before returning. */
typedef struct {
    int nsite, chil, chir, d, wl, wm, wr;
    const void *L, *W1, *W2, *R, *theta;
    void* out;
} tdvp_heff_desc;
int apply_heff_batched(tdvp_ctx ctx, tdvp_dtype dtype, int n, const tdvp_heff_desc* descs);

/* apply_heff without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layouts, ownership and result as apply_heff
 * (the caller still passes every input and the output); the MPO-stage
 * operator and the two intermediate stages live in one fixed scratch array of
 * apply_heff_noalloc_max_bytes() bytes (64 MiB) that the library holds on each
 * device it runs on until the process ends.  Problems needing more scratch
 * return TDVP_E_NOMEM before any work is queued (two-site, w = 10, d = 2:
 * chi_l * chi_r up to about 1e5 in complex64, 5e4 in complex128).  No GEMM
 * tile timing and no split-K.  Every call on one device shares that device's
 * array: calls that overlap in time on one device (from any context, stream
 * or thread) race and give wrong results; calls queued on one stream are
 * ordered and safe.  Nothing in the array needs to start at zero. */
int apply_heff_noalloc(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl,
                       int wm, int wr, const void* L, const void* W1, const void* W2, const void* R,
                       const void* theta, void* out);
size_t apply_heff_noalloc_max_bytes(void);

/* Environment update (Sec. III A, left-environment figure):
 *   dir = +1: out[l][b'][b] = sum conj(A[a'][s'][b']) env[k][a'][a] W[k][l][s'][s] A[a][s][b]
 *             (env = L_j [wl][chil][chil], out = L_{j+1} [wr][chir][chir])
 *   dir = -1: out[k][a][a'] = sum A[a][s][b] W[k][l][s'][s] env[l][b][b'] conj(A[a'][s'][b'])
 *             (env = R_j [wr][chir][chir], out = R_{j-1} [wl][chil][chil])
 * A is [chil][d][chir]; all device pointers of `dtype`. */
int env_update(tdvp_ctx ctx, int dir, tdvp_dtype dtype, int chil, int chir, int d,
               int wl, int wr, const void* env_in, const void* A, const void* W,
               void* env_out);

/* U(1) block-sparse H_eff application (quantum-number blocks; the S^z
 * conservation of the XY and XXX chains of Sec. IV, which the paper's
 * largest runs exploit through block-sparse tensors).  Same arguments,
 * layouts and result as apply_heff, plus integer charge labels (host
 * arrays): q_left [chil] and q_right [chir] of the bond indices (the charge
 * of the block to their left; each must be non-decreasing, so every charge
 * sector is a contiguous index range), q_phys [d] of the physical index, and
 * c_left [wl], c_right [wr] of the outer MPO bonds (the charge the operator
 * string to their left adds).  The inputs must obey the charge rules
 *   theta[a][s..][b]: q(a) + q(s..) = q(b);  W[k][l][s'][s]: c(l) = c(k) + q(s') - q(s);
 *   L[k][a'][a]: q(a') - q(a) = c(k);        R[l][b][b']: q(b') - q(b) = c(l);
 * entries outside the allowed blocks are never read (except that the MPO
 * must be exactly zero there), and the output is written in full (zero
 * outside its allowed blocks).  Only the allowed blocks are multiplied: the
 * two GEMM stages run as block products and the MPO stage on the sector
 * rectangles some term can reach.  Synchronises the context stream (the
 * block tables are built on the host per call).  Errors as apply_heff, plus
 * TDVP_E_ARG for unsorted labels. */
int apply_heff_u1(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm, int wr,
                  const int* q_left, const int* q_right, const int* q_phys, const int* c_left, const int* c_right,
                  const void* L, const void* W1, const void* W2, const void* R, const void* theta, void* out);
/* U(1) block-sparse env_update: same arguments and result as env_update
 * (A [chil][d][chir], W [wl][wr][d][d]), charge labels as for
 * apply_heff_u1 (q_left [chil], q_right [chir], q_phys [d], c_left [wl],
 * c_right [wr]); inputs must obey the charge rules, the output is written in
 * full.  Synchronises the context stream. */
int env_update_u1(tdvp_ctx ctx, int dir, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wr,
                  const int* q_left, const int* q_right, const int* q_phys, const int* c_left, const int* c_right,
                  const void* env_in, const void* A, const void* W, void* env_out);

/* Adjoint of env_update (reverse mode; Sec. III A, Fig. environments): for a
 * real loss and gradients in the convention g = dl/dRe z + i dl/dIm z,
 * given out_bar = the gradient of env_out, writes the gradients of the
 * inputs: env_bar (same shape as env_in), A_bar [chil][d][chir] (A enters
 * as ket and, conjugated, as bra; both contributions are summed) and W_bar
 * [wl][wr][d][d].  Any output may be NULL.  Same dimensions, layouts and
 * dtype as env_update; device pointers owned by the caller; outputs must
 * not alias inputs (TDVP_E_ARG). */
int env_update_adjoint(tdvp_ctx ctx, int dir, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wr,
                       const void* env_in, const void* A, const void* W, const void* out_bar, void* env_bar,
                       void* A_bar, void* W_bar);

/* ------------------------------------------------------------ observables */

/* <bra|O_i|ket> for n (site, O) pairs, not normalised (sites 0-based, ops
 * [n][d][d] complex128 host, out [n] complex128 host).  bra and ket need the
 * same N and d; their bond dimensions may differ.  With ket = e^{-iHt}
 * sigma_k |psi_0> and bra = |psi_0> this gives the dynamical correlation
 * function of Sec. IV (Eq. HaldaneCorrelation) up to the phase e^{i E_0 t}. */
int transition_expect(tdvp_ctx ctx, tdvp_mps bra, tdvp_mps ket, int n, const int* sites,
                      const double* ops, double* out);

/* <psi|O_i|psi>/<psi|psi> for n (site, O) pairs; sites 0-based, ops
 * [n][d][d] complex128 host, out [n] complex128 host (Sec. IV). */
int expect(tdvp_ctx ctx, tdvp_mps mps, int n, const int* sites, const double* ops,
           double* out);
/* <psi|O_i O_j|psi>/<psi|psi> for n pairs (equal-time correlator,
 * Eq. IsingCorrelation without the disconnected part). */
int expect2(tdvp_ctx ctx, tdvp_mps mps, int n, const int* i, const int* j, const double* Oi,
            const double* Oj, double* out);
/* <psi|H|psi>/<psi|psi> with H the MPO; out is complex128 (2 doubles). */
int energy(tdvp_ctx ctx, tdvp_mps mps, tdvp_mpo mpo, double* out);
/* <psi|psi> (real). */
int norm2(tdvp_ctx ctx, tdvp_mps mps, double* out);
/* <bra|ket> as complex128; infidelity (Sec. IV) follows from it. */
int overlap(tdvp_ctx ctx, tdvp_mps bra, tdvp_mps ket, double* out);

#ifdef __cplusplus
}
#endif

#endif /* TDVP_H */
