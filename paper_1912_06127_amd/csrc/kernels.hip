// Memory-bound kernels of the TDVP path: the sparse MPO stage between the
// two GEMMs of H_eff and of the environment updates, the FP64 vector
// operations of Lanczos, and small reshaping helpers around the dense
// solvers.
#include "common.hpp"

namespace tdvp {
namespace {

constexpr int kVecThreads = 256;
constexpr int kDotBlocks = 512;  // fixed partial-sum count -> deterministic sums

template <typename T> struct cplx;
template <> struct cplx<float> { using t = float2; };
template <> struct cplx<double> { using t = double2; };

template <typename T>
__device__ inline void ld(const void* p, int c128, int64_t i, T& re, T& im) {
    if (c128) {
        double2 v = reinterpret_cast<const double2*>(p)[i];
        re = (T)v.x;
        im = (T)v.y;
    } else {
        float2 v = reinterpret_cast<const float2*>(p)[i];
        re = (T)v.x;
        im = (T)v.y;
    }
}

template <typename T>
__device__ inline void st(void* p, int c128, int64_t i, T re, T im) {
    if (c128) reinterpret_cast<double2*>(p)[i] = make_double2((double)re, (double)im);
    else reinterpret_cast<float2*>(p)[i] = make_float2((float)re, (float)im);
}

// ---------------------------------------------------------------- MPO stage
// One thread per grid point (p, q).  The w_in*D input values of the point
// are staged in a thread-private LDS column, then each output row is a
// short sparse dot product with the MPO entries (read with uniform
// addresses).  Loads and stores are coalesced along q.
struct WParams {
    const void* in; int in128;
    void* out; int out128;
    int P, Q, D, nin, nout;
    int64_t ik, is, ip, on, os, op;
    const int* row_ptr;
    const int* col;
    const void* val;
};

// Grid point (p, q) of one MPO stage; xin is this thread's LDS column.
template <typename T>
__device__ __forceinline__ void wstage_point(const WParams& w, int p, int q, typename cplx<T>::t* xin, int nt) {
    using C = typename cplx<T>::t;
    const int64_t pin = (int64_t)p * w.ip + q;
    for (int c = 0; c < w.nin; ++c) {
        const int k = c / w.D, s = c % w.D;
        T re, im;
        ld<T>(w.in, w.in128, pin + k * w.ik + s * w.is, re, im);
        xin[c * nt] = C{re, im};
    }
    const C* val = reinterpret_cast<const C*>(w.val);
    const int64_t pout = (int64_t)p * w.op + q;
    for (int r = 0; r < w.nout; ++r) {
        T ar = 0, ai = 0;
        const int e1 = w.row_ptr[r + 1];
        for (int e = w.row_ptr[r]; e < e1; ++e) {
            const C v = val[e];
            const C x = xin[w.col[e] * nt];
            ar += v.x * x.x - v.y * x.y;
            ai += v.x * x.y + v.y * x.x;
        }
        const int n = r / w.D, s = r % w.D;
        st<T>(w.out, w.out128, pout + n * w.on + s * w.os, ar, ai);
    }
}

template <typename T>
__global__ void wstage_kernel(WParams w) {
    using C = typename cplx<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* xin = reinterpret_cast<C*>(smem_raw);  // [nin][blockDim.x]
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= w.Q) return;  // no barrier: each thread uses only its column
    wstage_point<T>(w, blockIdx.y, q, xin + threadIdx.x, blockDim.x);
}

// Grouped MPO stage: problem g owns blocks [blk_begin, blk_begin + P*qblocks).
struct GWProblem {
    WParams w;
    int64_t blk_begin;
    int qblocks;
};

template <typename T>
__global__ void wstage_grouped_kernel(const GWProblem* __restrict__ probs, int nprob) {
    using C = typename cplx<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* xin = reinterpret_cast<C*>(smem_raw);
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].blk_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const int qb = probs[lo].qblocks;
    const int64_t local = b - probs[lo].blk_begin;
    const int p = (int)(local / qb);
    const int q = (int)(local % qb) * blockDim.x + threadIdx.x;
    const WParams w = probs[lo].w;
    if (q >= w.Q) return;
    wstage_point<T>(w, p, q, xin + threadIdx.x, blockDim.x);
}

// ------------------------------------------------------------ FP64 vectors

__global__ void vdot_partial_kernel(const double2* V, int64_t vstride, int nv, const double2* w,
                                    int64_t n, double2* partial) {
    // partial[j][block] = sum over this block's grid-stride slice of conj(V[j][i]) w[i]
    __shared__ double sre[kVecThreads], sim[kVecThreads];
    for (int j = 0; j < nv; ++j) {
        double re = 0.0, im = 0.0;
        const double2* v = V + j * vstride;
        for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * kVecThreads) {
            const double2 a = v[i], b = w[i];
            re += a.x * b.x + a.y * b.y;
            im += a.x * b.y - a.y * b.x;
        }
        sre[threadIdx.x] = re;
        sim[threadIdx.x] = im;
        __syncthreads();
        for (int h = kVecThreads / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                sre[threadIdx.x] += sre[threadIdx.x + h];
                sim[threadIdx.x] += sim[threadIdx.x + h];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = make_double2(sre[0], sim[0]);
        __syncthreads();
    }
}

__global__ void reduce_partial_kernel(const double2* partial, int nblocks, double2* out) {
    // one block per vector j
    __shared__ double sre[kVecThreads], sim[kVecThreads];
    const int j = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kVecThreads) {
        const double2 v = partial[(int64_t)j * nblocks + b];
        re += v.x;
        im += v.y;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = kVecThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = make_double2(sre[0], sim[0]);
}

__global__ void axpy_multi_kernel(const double2* V, int64_t vstride, int nv, const double2* coef,
                                  double2* w, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    double2 acc = w[i];
    for (int j = 0; j < nv; ++j) {
        const double2 c = coef[j], v = V[j * vstride + i];
        acc.x -= c.x * v.x - c.y * v.y;
        acc.y -= c.x * v.y + c.y * v.x;
    }
    w[i] = acc;
}

__global__ void lanczos_3term_kernel(double2* w, const double2* vk, const double2* vkm1,
                                     const double2* alpha, double beta, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    const double a = alpha[0].x;
    double2 x = w[i];
    const double2 v = vk[i];
    x.x -= a * v.x;
    x.y -= a * v.y;
    if (vkm1) {
        const double2 u = vkm1[i];
        x.x -= beta * u.x;
        x.y -= beta * u.y;
    }
    w[i] = x;
}

__global__ void scale_copy_kernel(double2* out, const double2* in, double scale, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    const double2 v = in[i];
    out[i] = make_double2(scale * v.x, scale * v.y);
}

__global__ void combine_kernel(double2* out, const double2* V, int64_t vstride, int nv,
                               const double2* coef, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nv; ++j) {
        const double2 c = coef[j], v = V[j * vstride + i];
        re += c.x * v.x - c.y * v.y;
        im += c.x * v.y + c.y * v.x;
    }
    out[i] = make_double2(re, im);
}

__global__ void copy2d_kernel(double2* dst, int64_t ldd, const double2* src, int64_t lds, int rows,
                              int cols, int mask) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= cols || r >= rows) return;
    double2 v = src[(int64_t)r * lds + c];
    if ((mask == 1 && c < r) || (mask == 2 && c > r)) v = make_double2(0.0, 0.0);
    dst[(int64_t)r * ldd + c] = v;
}

__global__ void conj_transpose_kernel(double2* dst, int64_t ldd, const double2* src, int64_t lds, int rows,
                                      int cols) {
    // dst[c][r] = conj(src[r][c]) for r < rows, c < cols
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= cols || r >= rows) return;
    const double2 v = src[(int64_t)r * lds + c];
    dst[(int64_t)c * ldd + r] = make_double2(v.x, -v.y);
}

// out[z][j][i] = conj(in[z][i][j]) for n x n blocks, any complex dtype
__global__ void conj_transpose_batched_kernel(void* out, const void* in, int c128, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int64_t z = blockIdx.z;
    if (j >= n) return;
    const int64_t base = z * (int64_t)n * n;
    double re, im;
    ld<double>(in, c128, base + (int64_t)i * n + j, re, im);
    st<double>(out, c128, base + (int64_t)j * n + i, re, -im);
}

// MPO-tensor gradient of the one-site effective Hamiltonian:
// out[k][l][s'][s] = sum_{a', b} conj(T1[k][a'][s][b]) Z[l][a'][s'][b],
// one block per output entry, fixed-order reduction.
template <typename T>
__global__ void wgrad_kernel(const void* T1, const void* Z, int c128, int wl, int wr, int d, int chil,
                             int chir, void* out, int out128) {
    __shared__ double sre[256], sim[256];
    const int e = blockIdx.x;  // (k, l, s', s)
    const int s = e % d, sp = (e / d) % d, l = (e / (d * d)) % wr, k = e / (d * d * wr);
    double re = 0.0, im = 0.0;
    const int64_t nn = (int64_t)chil * chir;
    for (int64_t t = threadIdx.x; t < nn; t += blockDim.x) {
        const int a = (int)(t / chir), b = (int)(t % chir);
        T xr, xi, zr, zi;
        ld<T>(T1, c128, (((int64_t)k * chil + a) * d + s) * chir + b, xr, xi);
        ld<T>(Z, c128, (((int64_t)l * chil + a) * d + sp) * chir + b, zr, zi);
        re += (double)(xr * zr + xi * zi);
        im += (double)(xr * zi - xi * zr);
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) st<double>(out, out128, e, sre[0], sim[0]);
}

__global__ void scale_rows_kernel(double2* V, int64_t ld, const double* sv, int rows, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= cols || r >= rows) return;
    const double s = sv[r];
    double2 v = V[(int64_t)r * ld + c];
    V[(int64_t)r * ld + c] = make_double2(s * v.x, s * v.y);
}

__global__ void scale_cols_kernel(double2* U, int64_t ld, const double* sv, int rows, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= cols || r >= rows) return;
    const double s = sv[c];
    double2 v = U[(int64_t)r * ld + c];
    U[(int64_t)r * ld + c] = make_double2(s * v.x, s * v.y);
}

__global__ void convert_kernel(void* dst, int d128, const void* src, int s128, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    double re, im;
    ld<double>(src, s128, i, re, im);
    st<double>(dst, d128, i, re, im);
}

__global__ void nan_check_kernel(const double2* x, int64_t n, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    const double2 v = x[i];
    if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(flag, 1);
}

// --------------------------------------------- MPO stage operator (device)
// Dense operator M[row][col] of the sparse MPO stage, built in FP64 from the
// device MPO tensors (kind as in MopKind).
__global__ void mop_dense_kernel(int kind, const void* W1, int w1_128, const void* W2, int w2_128,
                                 int wl, int wm, int wr, int d, int rows, int cols, double2* M) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int row = idx / cols, col = idx % cols;
    double re = 0.0, im = 0.0;
    if (kind == 0) {  // zero-site: identity on the MPO bond
        re = (row == col) ? 1.0 : 0.0;
    } else if (kind == 1) {  // (l, s') <- (k, s): W[k][l][s'][s]
        const int l = row / d, sp = row % d, k = col / d, s = col % d;
        ld<double>(W1, w1_128, (((int64_t)k * wr + l) * d + sp) * d + s, re, im);
    } else if (kind == 3) {  // (k, s') <- (l, s): W[k][l][s'][s]
        const int k = row / d, sp = row % d, l = col / d, s = col % d;
        ld<double>(W1, w1_128, (((int64_t)k * wr + l) * d + sp) * d + s, re, im);
    } else if (kind == 4) {  // (l, s') <- (k, s): conj(W[k][l][s][s'])  (physical adjoint)
        const int l = row / d, sp = row % d, k = col / d, s = col % d;
        ld<double>(W1, w1_128, (((int64_t)k * wr + l) * d + s) * d + sp, re, im);
        im = -im;
    } else {
        // kind 2: (n, s1' s2') <- (k, s1 s2): sum_l W1[k][l][s1'][s1] W2[l][n][s2'][s2]
        // kind 5: as kind 2 with both factors physically adjoint (conj, s <-> s')
        // kind 6: (k, s1' s2') <- (n, s1 s2): sum_l W1[k][l][s1'][s1] W2[l][n][s2'][s2]
        const int dd = d * d;
        int n, s1p, s2p, k, s1, s2;
        if (kind == 6) {
            k = row / dd; s1p = (row % dd) / d; s2p = row % d;
            n = col / dd; s1 = (col % dd) / d; s2 = col % d;
        } else {
            n = row / dd; s1p = (row % dd) / d; s2p = row % d;
            k = col / dd; s1 = (col % dd) / d; s2 = col % d;
        }
        const bool adj = kind == 5;
        for (int l = 0; l < wm; ++l) {
            double ar, ai, br, bi;
            ld<double>(W1, w1_128, (((int64_t)k * wm + l) * d + (adj ? s1 : s1p)) * d + (adj ? s1p : s1), ar, ai);
            ld<double>(W2, w2_128, (((int64_t)l * wr + n) * d + (adj ? s2 : s2p)) * d + (adj ? s2p : s2), br, bi);
            if (adj) {
                ai = -ai;
                bi = -bi;
            }
            re += ar * br - ai * bi;
            im += ar * bi + ai * br;
        }
    }
    M[idx] = make_double2(re, im);
}

// Compress the dense operator to CSR (exact zeros dropped).  One block.
__global__ void mop_csr_kernel(const double2* M, int rows, int cols, int* row_ptr, int* col,
                               void* val, int val128) {
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        int c = 0;
        for (int j = 0; j < cols; ++j) {
            const double2 v = M[(int64_t)r * cols + j];
            c += (v.x != 0.0 || v.y != 0.0);
        }
        row_ptr[r + 1] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        row_ptr[0] = 0;
        for (int r = 0; r < rows; ++r) row_ptr[r + 1] += row_ptr[r];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        int e = row_ptr[r];
        for (int j = 0; j < cols; ++j) {
            const double2 v = M[(int64_t)r * cols + j];
            if (v.x != 0.0 || v.y != 0.0) {
                col[e] = j;
                st<double>(val, val128, e, v.x, v.y);
                ++e;
            }
        }
    }
}

// out[block] = partial sums of X[i][j] * Y[j][i] (no conjugation)
__global__ void trace_xyT_partial_kernel(const double2* X, const double2* Y, int n, double2* partial) {
    __shared__ double sre[kVecThreads], sim[kVecThreads];
    double re = 0.0, im = 0.0;
    const int64_t nn = (int64_t)n * n;
    for (int64_t t = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; t < nn;
         t += (int64_t)gridDim.x * kVecThreads) {
        const int64_t i = t / n, j = t % n;
        const double2 a = X[t], b = Y[j * n + i];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = kVecThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(sre[0], sim[0]);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kVecThreads - 1) / kVecThreads); }

}  // namespace

void wstage(tdvp_ctx ctx, const WStageDesc& d) {
    hipStream_t s = ctx->stream;
    if (d.P == 0 || d.Q == 0) return;
    WParams w;
    w.in = d.in;
    w.in128 = d.in_dt == Dt::C128;
    w.out = d.out;
    w.out128 = d.out_dt == Dt::C128;
    w.P = d.P;
    w.Q = d.Q;
    w.D = d.D;
    w.nin = d.w_in * d.D;
    w.nout = d.w_out * d.D;
    w.ik = d.ik; w.is = d.is; w.ip = d.ip;
    w.on = d.on; w.os = d.os; w.op = d.op;
    w.row_ptr = d.row_ptr;
    w.col = d.col;
    w.val = d.val;
    const size_t esz = d.fp64 ? sizeof(double2) : sizeof(float2);
    int nt = 256;
    while (nt > 64 && (size_t)nt * w.nin * esz > 48 * 1024) nt /= 2;
    const size_t shmem = (size_t)nt * w.nin * esz;
    TDVP_REQUIRE(shmem <= 160 * 1024, TDVP_E_SHAPE, "wstage: MPO bond dimension too large");
    TDVP_REQUIRE(d.P <= 65535 * 1024, TDVP_E_SHAPE, "wstage: grid too large");
    dim3 grid((d.Q + nt - 1) / nt, d.P);
    const double pts = (double)d.P * d.Q;
    ProfScope prof(ctx, d.fp64 ? "wstage_f64" : "wstage_f32", 0.0,
                   pts * (w.nin * elem_bytes(d.in_dt) + w.nout * elem_bytes(d.out_dt)));
    if (d.fp64) hipLaunchKernelGGL(wstage_kernel<double>, grid, dim3(nt), shmem, s, w);
    else hipLaunchKernelGGL(wstage_kernel<float>, grid, dim3(nt), shmem, s, w);
    TDVP_CHECK_HIP(hipGetLastError());
}

void grouped_wstage_plan(tdvp_ctx ctx, const std::vector<WStageDesc>& ds, GroupedWStage& out) {
    std::vector<GWProblem> tab;
    int nin_max = 1;
    bool first = true;
    out.bytes = 0.0;
    for (const auto& d : ds) {
        if (first) {
            out.fp64 = d.fp64;
            first = false;
        }
        TDVP_REQUIRE(d.fp64 == out.fp64, TDVP_E_ARG, "grouped wstage: mixed precision");
        nin_max = std::max(nin_max, d.w_in * d.D);
    }
    const size_t esz = out.fp64 ? sizeof(double2) : sizeof(float2);
    int nt = 256;
    while (nt > 64 && (size_t)nt * nin_max * esz > 48 * 1024) nt /= 2;
    out.nt = nt;
    out.shmem = (size_t)nt * nin_max * esz;
    TDVP_REQUIRE(out.shmem <= 160 * 1024, TDVP_E_SHAPE, "wstage: MPO bond dimension too large");
    int64_t blocks = 0;
    for (const auto& d : ds) {
        if (d.P == 0 || d.Q == 0) continue;
        GWProblem g{};
        WParams& w = g.w;
        w.in = d.in;
        w.in128 = d.in_dt == Dt::C128;
        w.out = d.out;
        w.out128 = d.out_dt == Dt::C128;
        w.P = d.P;
        w.Q = d.Q;
        w.D = d.D;
        w.nin = d.w_in * d.D;
        w.nout = d.w_out * d.D;
        w.ik = d.ik; w.is = d.is; w.ip = d.ip;
        w.on = d.on; w.os = d.os; w.op = d.op;
        w.row_ptr = d.row_ptr;
        w.col = d.col;
        w.val = d.val;
        g.qblocks = (d.Q + nt - 1) / nt;
        g.blk_begin = blocks;
        blocks += (int64_t)d.P * g.qblocks;
        out.bytes += (double)d.P * d.Q * (w.nin * elem_bytes(d.in_dt) + w.nout * elem_bytes(d.out_dt));
        tab.push_back(g);
    }
    TDVP_REQUIRE(blocks <= 0x7fffffff, TDVP_E_SHAPE, "grouped wstage: grid too large");
    out.nprob = (int)tab.size();
    out.blocks = blocks;
    if (out.probs.bytes < sizeof(GWProblem) * tab.size()) out.probs = DevMem(ctx, sizeof(GWProblem) * tab.size());
    if (!tab.empty()) {
        TDVP_CHECK_HIP(hipMemcpyAsync(out.probs.ptr, tab.data(), sizeof(GWProblem) * tab.size(), hipMemcpyHostToDevice,
                                      ctx->stream));
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    }
}

void grouped_wstage_run(tdvp_ctx ctx, const GroupedWStage& g) {
    if (g.nprob == 0 || g.blocks == 0) return;
    ProfScope prof(ctx, g.fp64 ? "wstage_grouped_f64" : "wstage_grouped_f32", 0.0, g.bytes);
    const auto* pr = static_cast<const GWProblem*>(g.probs.ptr);
    if (g.fp64)
        hipLaunchKernelGGL(wstage_grouped_kernel<double>, dim3((unsigned)g.blocks), dim3(g.nt), g.shmem, ctx->stream,
                           pr, g.nprob);
    else
        hipLaunchKernelGGL(wstage_grouped_kernel<float>, dim3((unsigned)g.blocks), dim3(g.nt), g.shmem, ctx->stream,
                           pr, g.nprob);
    TDVP_CHECK_HIP(hipGetLastError());
}

void vdot_multi(tdvp_ctx ctx, const double2* V, int64_t vstride, int nv, const double2* w,
                int64_t n, double2* out) {
    if (nv <= 0) return;
    double2* partial = static_cast<double2*>(
        ctx->workspace("vdot_partial", sizeof(double2) * (size_t)kDotBlocks * nv));
    int nb = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + kVecThreads - 1) / kVecThreads));
    hipLaunchKernelGGL(vdot_partial_kernel, dim3(nb), dim3(kVecThreads), 0, ctx->stream, V, vstride,
                       nv, w, n, partial);
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(nv), dim3(kVecThreads), 0, ctx->stream, partial,
                       nb, out);
    TDVP_CHECK_HIP(hipGetLastError());
}

void axpy_multi(const double2* V, int64_t vstride, int nv, const double2* coef, double2* w,
                int64_t n, hipStream_t s) {
    if (n == 0 || nv == 0) return;
    hipLaunchKernelGGL(axpy_multi_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, V, vstride, nv,
                       coef, w, n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void lanczos_3term(double2* w, const double2* vk, const double2* vkm1, const double2* alpha_dev,
                   double beta, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(lanczos_3term_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, w, vk, vkm1,
                       alpha_dev, beta, n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void scale_copy(double2* out, const double2* in, double scale, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, out, in, scale, n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void combine(double2* out, const double2* V, int64_t vstride, int nv, const double2* coef,
             int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(combine_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, out, V, vstride, nv,
                       coef, n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void copy2d(double2* dst, int64_t ldd, const double2* src, int64_t lds, int rows, int cols,
            int mask, hipStream_t s) {
    if (rows == 0 || cols == 0) return;
    TDVP_REQUIRE(rows <= 65535, TDVP_E_SHAPE, "copy2d: too many rows");
    dim3 grid((cols + 127) / 128, rows);
    hipLaunchKernelGGL(copy2d_kernel, grid, dim3(128), 0, s, dst, ldd, src, lds, rows, cols, mask);
    TDVP_CHECK_HIP(hipGetLastError());
}

void conj_transpose(double2* dst, int64_t ldd, const double2* src, int64_t lds, int rows, int cols,
                    hipStream_t s) {
    if (rows == 0 || cols == 0) return;
    TDVP_REQUIRE(rows <= 65535, TDVP_E_SHAPE, "conj_transpose: too many rows");
    dim3 grid((cols + 127) / 128, rows);
    hipLaunchKernelGGL(conj_transpose_kernel, grid, dim3(128), 0, s, dst, ldd, src, lds, rows, cols);
    TDVP_CHECK_HIP(hipGetLastError());
}

void scale_rows(double2* V, int64_t ld, const double* sv, int rows, int cols, hipStream_t s) {
    if (rows == 0 || cols == 0) return;
    dim3 grid((cols + 127) / 128, rows);
    hipLaunchKernelGGL(scale_rows_kernel, grid, dim3(128), 0, s, V, ld, sv, rows, cols);
    TDVP_CHECK_HIP(hipGetLastError());
}

void scale_cols(double2* U, int64_t ld, const double* sv, int rows, int cols, hipStream_t s) {
    if (rows == 0 || cols == 0) return;
    dim3 grid((cols + 127) / 128, rows);
    hipLaunchKernelGGL(scale_cols_kernel, grid, dim3(128), 0, s, U, ld, sv, rows, cols);
    TDVP_CHECK_HIP(hipGetLastError());
}

void convert(void* dst, Dt ddt, const void* src, Dt sdt, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(convert_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, dst,
                       (int)(ddt == Dt::C128), src, (int)(sdt == Dt::C128), n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void nan_check(const double2* x, int64_t n, int* flag, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(nan_check_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, x, n, flag);
    TDVP_CHECK_HIP(hipGetLastError());
}

void mop_build(int kind, const void* W1, Dt w1dt, const void* W2, Dt w2dt, int wl, int wm, int wr,
               int d, int rows, int cols, double2* dense, int* row_ptr, int* col, void* val,
               bool val_fp64, hipStream_t s) {
    const int tot = rows * cols;
    if (tot == 0) return;
    hipLaunchKernelGGL(mop_dense_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, kind, W1,
                       (int)(w1dt == Dt::C128), W2, (int)(w2dt == Dt::C128), wl, wm, wr, d, rows,
                       cols, dense);
    hipLaunchKernelGGL(mop_csr_kernel, dim3(1), dim3(256), 0, s, dense, rows, cols, row_ptr, col,
                       val, (int)val_fp64);
    TDVP_CHECK_HIP(hipGetLastError());
}

void conj_transpose_batched(void* out, const void* in, Dt dt, int n, int batch, hipStream_t s) {
    if (n == 0 || batch == 0) return;
    TDVP_REQUIRE(n <= 65535 && batch <= 65535, TDVP_E_SHAPE, "conj_transpose_batched: too large");
    dim3 grid((n + 127) / 128, n, batch);
    hipLaunchKernelGGL(conj_transpose_batched_kernel, grid, dim3(128), 0, s, out, in, (int)(dt == Dt::C128), n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void wgrad(const void* T1, const void* Z, Dt dt, int wl, int wr, int d, int chil, int chir, void* out,
           hipStream_t s) {
    const int nout = wl * wr * d * d;
    if (nout == 0) return;
    if (dt == Dt::C128)
        hipLaunchKernelGGL(wgrad_kernel<double>, dim3(nout), dim3(256), 0, s, T1, Z, 1, wl, wr, d, chil, chir, out, 1);
    else
        hipLaunchKernelGGL(wgrad_kernel<float>, dim3(nout), dim3(256), 0, s, T1, Z, 0, wl, wr, d, chil, chir, out, 0);
    TDVP_CHECK_HIP(hipGetLastError());
}

void trace_xyT(tdvp_ctx ctx, const double2* X, const double2* Y, int n, double2* out) {
    double2* partial = static_cast<double2*>(ctx->workspace("trace_partial", sizeof(double2) * kDotBlocks));
    int nb = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, ((int64_t)n * n + kVecThreads - 1) / kVecThreads));
    hipLaunchKernelGGL(trace_xyT_partial_kernel, dim3(nb), dim3(kVecThreads), 0, ctx->stream, X, Y, n, partial);
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(1), dim3(kVecThreads), 0, ctx->stream, partial, nb, out);
    TDVP_CHECK_HIP(hipGetLastError());
}

}  // namespace tdvp
