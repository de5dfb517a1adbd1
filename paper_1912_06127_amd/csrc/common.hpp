// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tdvp.h"

namespace tdvp {

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define TDVP_CHECK_HIP(expr)                                                          \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::tdvp::Error(TDVP_E_HIP, std::string(#expr) + ": " +               \
                                                hipGetErrorString(e_));               \
    } while (0)

#define TDVP_REQUIRE(cond, status, msg)                                              \
    do {                                                                              \
        if (!(cond)) throw ::tdvp::Error((status), (msg));                            \
    } while (0)

// ------------------------------------------------------------------- dtypes

enum class Dt : int { C64 = 0, C128 = 1 };
inline size_t elem_bytes(Dt d) { return d == Dt::C64 ? 8 : 16; }
inline Dt to_dt(int v) {
    TDVP_REQUIRE(v == TDVP_C64 || v == TDVP_C128, TDVP_E_DTYPE, "dtype must be TDVP_C64 or TDVP_C128");
    return v == TDVP_C64 ? Dt::C64 : Dt::C128;
}

struct cd {  // host complex double
    double re, im;
};

// ------------------------------------------------------------------ context

struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace tdvp

struct tdvp_prof_rec {
    std::string name;
    hipEvent_t start, stop;
    double flops, bytes;
};
struct tdvp_prof_total {
    double ms = 0.0, flops = 0.0, bytes = 0.0;
    long count = 0;
};

namespace tdvp {
// Square root of a squared norm: negative rounding noise gives 0, while NaN
// stays NaN (fmax/std::max would turn it into 0 and hide a non-finite value).
__host__ __device__ inline double sqrt_or_nan(double x) { return x > 0.0 ? sqrt(x) : (x <= 0.0 ? 0.0 : x); }
}  // namespace tdvp

namespace tdvp {
// Fixed device region handed out by workspace() while a call runs without
// allocating (apply_heff_noalloc): requests are carved from it in order, a
// name asked for twice gets the same block, and a request that does not fit
// is an error instead of an allocation.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    std::map<std::string, std::pair<size_t, size_t>> named;  // name -> (offset, bytes)
};
}  // namespace tdvp

struct tdvp_ctx_s {
    int device = 0;
    tdvp::Arena* arena = nullptr;               // set only inside an allocation-free call
    hipStream_t stream = nullptr;
    tdvp_alloc_fn alloc_fn = nullptr;
    tdvp_free_fn free_fn = nullptr;
    void* user = nullptr;
    rocblas_handle blas = nullptr;
    std::string err;
    std::map<std::string, tdvp::Buffer> work;  // grow-only named workspaces
    uint64_t ws_gen = 0;                        // bumped whenever a workspace moves
    bool prof_on = false;                       // HIP event pair around every launch
    bool autotune = true;                       // time GEMM tiles per shape bucket
    bool splitk = true;                         // GEMMs may split K (partial sums in a workspace)
    int gemm_form = 0;                          // raw-pointer calls: 0 default, 3 or 4
    std::map<int64_t, int> krylov_hint;         // Lanczos iterations last used per vector length
    void* pinned = nullptr;                     // page-locked host staging (pinned_host)
    size_t pinned_bytes = 0;
    void* pinned_rd = nullptr;                  // page-locked landing area of read_back
    size_t pinned_rd_bytes = 0;
    std::shared_ptr<void> solver_lanes;         // worker lanes of the U(1) split's eigensolvers (tdvp.cpp)
    std::vector<tdvp_prof_rec> prof_pending;
    std::map<std::string, tdvp_prof_total> prof_total;

    void* dev_alloc(size_t bytes);
    void dev_free(void* p, size_t bytes);
    // Named workspace of at least `bytes` bytes; contents not preserved on growth.
    void* workspace(const std::string& name, size_t bytes);
    // Page-locked host buffer of at least `bytes` bytes (grow-only; growing
    // synchronises the stream first).
    void* pinned_host(size_t bytes);
    // Small device-to-host read-backs: every span is copied into page-locked
    // memory on the context stream, the stream is awaited (polled for a
    // short while before blocking: the waits on the serial path are a few
    // microseconds of queued work) and the values are copied to dst.
    struct ReadSpan {
        void* dst;
        const void* src;
        size_t bytes;
    };
    void read_back(std::initializer_list<ReadSpan> spans);
    // Host-to-device copy of a small table on the context stream without
    // waiting for it: the bytes are staged in one of kUploadSlots page-locked
    // slots, and a slot is written again only after the copy that read it
    // has completed (its event).  Not for use under stream capture.
    static constexpr int kUploadSlots = 8;
    struct UploadSlot {
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    UploadSlot up_slot[kUploadSlots];
    char* up_base = nullptr;
    size_t up_slot_bytes = 0;
    int up_next = 0;
    void upload(void* dst, const void* src, size_t bytes);
    // Waits for the context stream like hipStreamSynchronize.
    void wait_stream();
    void release_all();
};

namespace tdvp {

// Records a HIP event pair around the launches in its scope when the
// context's profiler is on; `flops` and `bytes` are the algorithmic work.
struct ProfScope {
    tdvp_ctx ctx;
    size_t idx = (size_t)-1;
    ProfScope(tdvp_ctx c, const char* name, double flops, double bytes);
    ~ProfScope();
};

// Named range of the calling thread on the ROC-TX marker stream (shown by a
// marker trace, e.g. rocprofv3 --marker-trace); without a tool attached the
// push and pop return at once.
struct TxRange {
    explicit TxRange(const char* name) { roctxRangePushA(name); }
    ~TxRange() { roctxRangePop(); }
    TxRange(const TxRange&) = delete;
    TxRange& operator=(const TxRange&) = delete;
};

// RAII device allocation through the context allocator.
struct DevMem {
    tdvp_ctx ctx = nullptr;
    void* ptr = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(tdvp_ctx c, size_t b) : ctx(c), bytes(b) { ptr = b ? c->dev_alloc(b) : nullptr; }
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    DevMem(DevMem&& o) noexcept { *this = std::move(o); }
    DevMem& operator=(DevMem&& o) noexcept {
        reset();
        ctx = o.ctx; ptr = o.ptr; bytes = o.bytes;
        o.ptr = nullptr; o.bytes = 0;
        return *this;
    }
    ~DevMem() { reset(); }
    void reset() {
        if (ptr && ctx) ctx->dev_free(ptr, bytes);
        ptr = nullptr; bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// ------------------------------------------------------------ kernel entry

// Operand of the complex GEMM.  For the A operand the "outer" index is m,
// for B it is n.  kcontig: element (outer, k) at p[outer*ld + k], otherwise
// at p[k*ld + outer].  conj: use the complex conjugate of the stored value.
struct GemmOperand {
    const void* p = nullptr;
    Dt dt = Dt::C64;
    int64_t ld = 0;
    int64_t stride = 0;  // batch stride in elements
    bool kcontig = true;
    bool conj = false;
};

// C[z][m][n] = sum_k op(A)[z][m][k] op(B)[z][k][n], C stored row-major with ldc.
struct GemmDesc {
    int M = 0, N = 0, K = 0, batch = 1;
    GemmOperand A, B;
    void* C = nullptr;
    Dt cdt = Dt::C64;
    int64_t ldc = 0, strideC = 0;
};

// fp64: FP64 MFMA, else FP32 MFMA.  form: 3 (Gauss 3-real-product) or 4.
void cgemm(tdvp_ctx ctx, const GemmDesc& g, bool fp64, int form);

// Many independent products (batch 1 each, shapes may differ) in one launch.
// The plan uploads the problem table (device memory owned by the plan) and
// picks one tile for the group (timed once per shape signature); operands
// are referenced by pointer, so a plan can be re-run, also inside a captured
// graph, as long as those buffers stay in place.
struct GroupedGemm {
    DevMem probs;
    int nprob = 0;
    int64_t total = 0;
    int cfg = 0;
    bool fp64 = false, m3 = false, ak = true, bkc = false;
    double flops = 0.0;
};
void grouped_gemm_plan(tdvp_ctx ctx, const std::vector<GemmDesc>& g, bool fp64, int form, GroupedGemm& out);
void grouped_gemm_run(tdvp_ctx ctx, const GroupedGemm& gg);

// Block-sparse products (U(1) quantum-number blocks).  Every problem is one
// output block C (g.batch entries: entry z reads A + z A.stride, B + z
// B.stride and writes C + z strideC) summed over a list of K chunks: chunk c
// adds the product of A + offA + i strideA and B + offB + i strideB over k in
// [0, K), for i = 0..count-1 (element offsets).  nchunk = 0: one chunk over
// g.K.  All problems of one call share the operand layouts (kcontig) and
// dtypes; C blocks must not overlap.
struct BlockChunk {
    int64_t offA = 0, offB = 0, strideA = 0, strideB = 0;
    int K = 0, count = 1;
};
struct BlockGemm {
    GemmDesc g;
    int chunk0 = 0, nchunk = 0;
};
void block_gemm(tdvp_ctx ctx, const std::vector<BlockGemm>& probs, const std::vector<BlockChunk>& chunks, bool fp64,
                int form, const char* tag);
// Fills `bytes` (a multiple of 8) with zero by a kernel (no memset node under graph capture).
void zero_fill(void* p, size_t bytes, hipStream_t s);

// Sparse local-operator stage.  For every grid point (p, q):
//   out[n][s'](p, q) = sum_{k,s} M[(n,s'),(k,s)] in[k][s](p, q)
// with in offset  k*ik + s*is + p*ip + q  and out offset n*on + s'*os + p*op + q.
// M is given in CSR form by output row r = n*D + s'; col = k*D + s.
struct WStageDesc {
    const void* in = nullptr; Dt in_dt = Dt::C64;
    void* out = nullptr; Dt out_dt = Dt::C64;
    int P = 0, Q = 0, D = 1, w_in = 1, w_out = 1;
    int64_t ik = 0, is = 0, ip = 0, on = 0, os = 0, op = 0;
    const int* row_ptr = nullptr;  // device [w_out*D + 1]
    const int* col = nullptr;      // device [nnz]
    const void* val = nullptr;     // device [nnz] complex of the compute dtype
    bool fp64 = false;
};
void wstage(tdvp_ctx ctx, const WStageDesc& w);
// Fused y = H_eff x for small bonds (all three stages in one launch, one
// block per row a').  Layouts as in heff_apply: L[wl][chil][chil],
// R[wr][chir][chir], x, y [chil][D][chir]; operator rows n*D + s', columns
// k*D + s, values of the compute dtype.  x and y must not overlap.
constexpr int kHeffSmallChi = 32;
struct HeffSmallDesc {
    const void* L = nullptr; Dt L_dt = Dt::C64;
    const void* R = nullptr; Dt R_dt = Dt::C64;
    const void* x = nullptr; Dt x_dt = Dt::C64;
    void* y = nullptr; Dt y_dt = Dt::C64;
    const int* row_ptr = nullptr;
    const int* col = nullptr;
    const void* val = nullptr;
    int chil = 0, chir = 0, D = 1, wl = 1, wr = 1;
    bool fp64 = false;
    double flops = 0.0;
};
bool heff_small_fits(int chil, int chir, int D, int wl, int wr, bool fp64);
void heff_small(tdvp_ctx ctx, const HeffSmallDesc& d);
// Many MPO stages of one precision in one launch (see GroupedGemm).
struct GroupedWStage {
    DevMem probs;                  // the problem table, unless it sits in a named workspace
    const void* table = nullptr;   // the table the launch reads
    int nprob = 0, nt = 256;
    int64_t blocks = 0;
    size_t shmem = 0;
    bool fp64 = false;
    double bytes = 0.0;
};
// The table is uploaded without waiting (tdvp_ctx_s::upload); it goes into
// the workspace named table_ws when given, else into out.probs.
void grouped_wstage_plan(tdvp_ctx ctx, const std::vector<WStageDesc>& ds, GroupedWStage& out,
                         const char* table_ws = nullptr);
void grouped_wstage_run(tdvp_ctx ctx, const GroupedWStage& g);

// ------------------------------------- batched Krylov over packed instances
// Instance i of a batch owns elements [off[i], off[i+1]) of packed vectors.
struct SegLayout {
    int ninst = 0, nblk = 0;
    int64_t total = 0;
    std::vector<int64_t> off;          // host copy [ninst + 1]
    DevMem d_off, d_iblk, d_binst, d_blo;
};
void seg_layout(tdvp_ctx ctx, const std::vector<int64_t>& sizes, SegLayout& L);
// packed <- per-instance sources / per-instance destinations <- packed
// (pointer tables in device memory).
void seg_gather(tdvp_ctx ctx, const SegLayout& L, double2* packed, const double2* const* src_dev);
void seg_scatter(tdvp_ctx ctx, const SegLayout& L, double2* const* dst_dev, const double2* packed);
// y = H x for all instances at once (packed complex128 vectors).
using BatchOp = std::function<void(const double2* x, double2* y)>;
struct BatchState {
    int ninst = 0;
    int* bad = nullptr;  // device [ninst]: non-finite value seen (valid until the next call)
};
// theta_i <- exp(-i tau H_i) theta_i by K Lanczos steps per instance (two
// Gram-Schmidt passes, breakdown handled per instance), no host sync.
void batch_expm(tdvp_ctx ctx, const SegLayout& L, const BatchOp& op, double2* theta, double tau, int K,
                BatchState& st);
void batch_expm_reserve(tdvp_ctx ctx, const SegLayout& L, int K);
// flag[0] = 1 if any instance of the last batch_expm saw a non-finite value;
// reset_flag sets flag[0] = 0 (kernels, so both may sit inside a graph).
void seg_flag_or(tdvp_ctx ctx, const BatchState& st, int* flag);
void reset_flag(tdvp_ctx ctx, int* flag);

// ----------------------------------------------- FP64 vector kernels (c128)
// All pointers device; n complex elements.
// partial dot products of vectors V[0..nv) (stride vstride) with w,
// reduced into out[nv] (complex) = sum conj(V[j][i]) w[i].
void vdot_multi(tdvp_ctx ctx, const double2* V, int64_t vstride, int nv, const double2* w,
                int64_t n, double2* out);
// One Lanczos step on a short vector in a single workgroup (n <= kSmallLanczos,
// k < 64): w <- w - alpha v_k - beta_prev v_{k-1} with alpha = Re<v_k, w>, two
// Gram-Schmidt passes against V[0..k], out[0] = alpha, out[1] = ||w||^2 (device
// doubles), V[k+1] = w / ||w|| (zero if w vanishes).  V holds n-element rows.
constexpr int64_t kSmallLanczos = 8192;
// beta_{k-1} is beta_prev, or sqrt(*nn_prev) when nn_prev (device, the
// previous step's ||w||^2) is not null, so that steps can be queued
// without reading anything back.
void lanczos_small_step(double2* V, int64_t n, int k, double2* w, double beta_prev, const double* nn_prev,
                        double* out, hipStream_t s);
// nn[0] = ||x||^2 and v = x / ||x|| (zero if x vanishes) in one workgroup, n <= kSmallLanczos.
void small_normalize(const double2* x, double2* v, int64_t n, double* nn, hipStream_t s);
// Eigen-decomposition of a Hermitian n x n matrix G (row-major, n <= kJacobiMaxOrder) in
// one workgroup (cyclic Jacobi): evals descending, vecs row c = conj of the
// c-th eigenvector (row-major [n][n]), sweeps = Jacobi sweeps used (may be
// null).  All device pointers.
constexpr int kJacobiMaxOrder = 64;
void jacobi_eigh_small(const double2* G, int n, double* evals, double2* vecs, int* sweeps, hipStream_t s);
// The same for several matrices in one launch, one workgroup each (the table
// is uploaded without waiting, tdvp_ctx_s::upload).
struct JacobiProb {
    const double2* G;
    double* evals;
    double2* vecs;
    int n, pad;
};
void jacobi_eigh_batched(tdvp_ctx ctx, const std::vector<JacobiProb>& probs);
// Thin QR of an m x n matrix (m >= n, n <= kQrMaxCols, m n <= kQrMaxElems) in one
// workgroup (Householder reflectors in LDS, LAPACK's zgeqr2 / zung2r conventions).
// herm = false: M row-major [m][n] = Q [m][n] R [n][n] (R upper); herm = true: M
// row-major [n][m] = L [n][n] Q [n][m] (the LQ; L lower, rows of Q orthonormal),
// written to RL and Q.  All device pointers; every output element is written.
constexpr int kQrMaxCols = 64;
constexpr int kQrMaxElems = 4096;
bool qr_small_fits(int m, int n);
void qr_small(const double2* M, int m, int n, bool herm, double2* Q, double2* RL, hipStream_t s);
// w -= sum_j coef[j] V[j]   (coef device complex[nv])
void axpy_multi(const double2* V, int64_t vstride, int nv, const double2* coef, double2* w,
                int64_t n, hipStream_t s);
// w -= Re(alpha_dev[0]) * vk + beta * vkm1 (vkm1 may be null)
void lanczos_3term(double2* w, const double2* vk, const double2* vkm1, const double2* alpha_dev,
                   double beta, int64_t n, hipStream_t s);
// out = scale * in
void scale_copy(double2* out, const double2* in, double scale, int64_t n, hipStream_t s);
// Truncated-Taylor exponential action: b <- alpha (y - c b) and F <- F + b;
// taylor_rescale: F <- eta F and b <- F.
void taylor_term(double2* b, const double2* y, double2* F, int64_t n, double2 alpha, double c, hipStream_t s);
void taylor_rescale(double2* F, double2* b, int64_t n, double2 eta, hipStream_t s);
// out = sum_j coef[j] V[j]
void combine(double2* out, const double2* V, int64_t vstride, int nv, const double2* coef,
             int64_t n, hipStream_t s);
// The same with at most kCombineArgs host coefficients passed by value in the
// launch (no device copy of the coefficients).
constexpr int kCombineArgs = 32;
struct CombineCoef {
    double2 c[kCombineArgs];
};
void combine_args(double2* out, const double2* V, int64_t vstride, int nv, const double2* coef_host, int64_t n,
                  hipStream_t s);
// Indexed 2-D copy of complex128: dst[dr[i]][dc[k]] = src[sr[i]][sc[k]] for
// i < nr, k < nc (row-major, leading dimensions ldd / lds); a null index
// array means the identity.  Index arrays are device int arrays.
void copy_idx(double2* dst, int64_t ldd, const int* dr, const int* dc, const double2* src, int64_t lds,
              const int* sr, const int* sc, int nr, int nc, hipStream_t s);
// strided 2-D copy of complex128: dst[r*ldd + c] = src[r*lds + c] for c < cols;
// mask: 0 none, 1 zero where c < r (keep upper), 2 zero where c > r (keep lower)
void copy2d(double2* dst, int64_t ldd, const double2* src, int64_t lds, int rows, int cols,
            int mask, hipStream_t s);
// dst[c][r] = conj(src[r][c]) for r < rows, c < cols
void conj_transpose(double2* dst, int64_t ldd, const double2* src, int64_t lds, int rows, int cols,
                    hipStream_t s);
// rows of V (row-major [rows][cols]) multiplied by real sv[r]
void scale_rows(double2* V, int64_t ld, const double* sv, int rows, int cols, hipStream_t s);
// columns of U (row-major [rows][cols]) multiplied by real sv[c]
void scale_cols(double2* U, int64_t ld, const double* sv, int rows, int cols, hipStream_t s);
// out[c] = ||P row c||^2 (by_rows) or ||P column c||^2, c < count, vectors of len elements
void vec_norms2(const double2* P, int64_t ld, int count, int len, bool by_rows, double* out, hipStream_t s);
// c128 <-> c64 conversion
void convert(void* dst, Dt ddt, const void* src, Dt sdt, int64_t n, hipStream_t s);
// any NaN/Inf in n complex128 values -> flag[0] = 1 (flag must be zeroed)
void nan_check(const double2* x, int64_t n, int* flag, hipStream_t s);

}  // namespace tdvp

namespace tdvp {
// MPO-stage operator kinds (rows <- cols):
//   0 zero-site identity (w x w), 1 one-site / left environment (l,s')<-(k,s),
//   2 two-site (n,s1's2')<-(k,s1s2), 3 right environment (k,s')<-(l,s),
//   4 kind 1 with the physical adjoint conj(W[k][l][s][s']), 5 kind 2 with
//   both factors physically adjoint, 6 two-site right orientation
//   (k,s1's2')<-(n,s1s2).
void mop_build(int kind, const void* W1, Dt w1dt, const void* W2, Dt w2dt, int wl, int wm, int wr,
               int d, int rows, int cols, double2* dense, int* row_ptr, int* col, void* val,
               bool val_fp64, hipStream_t s);
// out[z] = in[z]^dagger for `batch` n x n blocks of dtype dt.
void conj_transpose_batched(void* out, const void* in, Dt dt, int n, int batch, hipStream_t s);
// y += x elementwise over n complex entries of dtype dt.
void add_inplace(void* y, const void* x, Dt dt, int64_t n, hipStream_t s);
// out[k][l][s'][s] = sum_{a',b} conj(T1[k][a'][s][b]) Z[l][a'][s'][b] (T1 [wl][chil][d][chir],
// Z [wr][chil][d][chir], out [wl][wr][d][d], all of dtype dt).
void wgrad(const void* T1, const void* Z, Dt dt, int wl, int wr, int d, int chil, int chir, void* out,
           hipStream_t s);
// out[0] = sum_{i,j} X[i][j] Y[j][i] for n x n complex128 matrices.
void trace_xyT(tdvp_ctx ctx, const double2* X, const double2* Y, int n, double2* out);
// out = tr(X Y) for X [rows][cols], Y [cols][rows] (device)
void trace_xy(tdvp_ctx ctx, const double2* X, const double2* Y, int rows, int cols, double2* out);
// A[a][s'][b] <- sum_s O[s'][s] A[a][s][b], A [chil][d][chir], O [d][d] (device), d <= 16
void apply_site(double2* A, const double2* O, int chil, int d, int chir, hipStream_t s);
}  // namespace tdvp
