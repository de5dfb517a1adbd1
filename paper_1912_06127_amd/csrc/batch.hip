// Batched Lanczos exponentiation over many local problems of different size
// (the independent segments of the segment-parallel step, Sec. III B).
//
// The Krylov vectors of all instances are packed back to back in one
// complex128 buffer; instance i owns elements [off[i], off[i+1]).  The packed
// range is cut into chunks of kChunk elements that never straddle two
// instances; every vector kernel runs one block per chunk and looks up its
// instance, so one launch serves all instances whatever their sizes.  Dot
// products write one partial per chunk and are summed per instance in chunk
// order (deterministic).  The scalar recurrences (alpha, beta, breakdown,
// exp(-i tau T_k) e_1 of the k x k tridiagonal matrix) run on the device,
// one thread per instance, so a whole exponentiation needs no host
// synchronisation and can be captured in a graph.
#include "common.hpp"

#include <cmath>

namespace tdvp {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = kThreads * 16;
constexpr int kMaxK = 16;

struct SegMap {
    const int* blk_inst;     // [nblk] instance of chunk b
    const int64_t* blk_lo;   // [nblk] first element of chunk b
    const int64_t* off;      // [ninst + 1]
};

__device__ inline int64_t chunk_hi(const SegMap& m, int b) {
    const int64_t hi = m.blk_lo[b] + kChunk;
    const int64_t e = m.off[m.blk_inst[b] + 1];
    return hi < e ? hi : e;
}

// partial[j * nblk + b] = sum_{e in chunk b} conj(V[j][e]) w[e]
__global__ void seg_dot_partial_kernel(SegMap m, const double2* V, int64_t vstride, int nv, const double2* w,
                                       int nblk, double2* partial) {
    __shared__ double sre[kThreads], sim[kThreads];
    const int b = blockIdx.x;
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b);
    for (int j = 0; j < nv; ++j) {
        const double2* v = V + (int64_t)j * vstride;
        double re = 0.0, im = 0.0;
        for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
            const double2 a = v[e], c = w[e];
            re += a.x * c.x + a.y * c.y;
            im += a.x * c.y - a.y * c.x;
        }
        sre[threadIdx.x] = re;
        sim[threadIdx.x] = im;
        __syncthreads();
        for (int h = kThreads / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                sre[threadIdx.x] += sre[threadIdx.x + h];
                sim[threadIdx.x] += sim[threadIdx.x + h];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)j * nblk + b] = make_double2(sre[0], sim[0]);
        __syncthreads();
    }
}

// out[i * ldo + j] = sum over the chunks of instance i (in order) of partial[j][.]
__global__ void seg_reduce_kernel(const double2* partial, int nblk, const int* inst_blk, double2* out, int ldo) {
    __shared__ double sre[kThreads], sim[kThreads];
    const int i = blockIdx.x, j = blockIdx.y;
    const int b0 = inst_blk[i], b1 = inst_blk[i + 1];
    double re = 0.0, im = 0.0;
    for (int b = b0 + threadIdx.x; b < b1; b += kThreads) {
        const double2 v = partial[(int64_t)j * nblk + b];
        re += v.x;
        im += v.y;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)i * ldo + j] = make_double2(sre[0], sim[0]);
}

// w[e] -= sum_j coef[inst][j] V[j][e]
__global__ void seg_axpy_kernel(SegMap m, const double2* V, int64_t vstride, int nv, const double2* coef, int ldc,
                                double2* w) {
    const int b = blockIdx.x;
    const int i = m.blk_inst[b];
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b);
    const double2* c = coef + (int64_t)i * ldc;
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        double2 acc = w[e];
        for (int j = 0; j < nv; ++j) {
            const double2 v = V[(int64_t)j * vstride + e];
            const double2 cj = c[j];
            acc.x -= cj.x * v.x - cj.y * v.y;
            acc.y -= cj.x * v.y + cj.y * v.x;
        }
        w[e] = acc;
    }
}

// w -= alpha_k v_k + beta_{k-1} v_{k-1}  (per-instance real coefficients)
__global__ void seg_3term_kernel(SegMap m, double2* w, const double2* vk, const double2* vkm1, const double* alpha,
                                 const double* beta, int k, int K) {
    const int b = blockIdx.x;
    const int i = m.blk_inst[b];
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b);
    const double a = alpha[i * K + k];
    const double bb = k > 0 ? beta[i * K + k - 1] : 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        double2 x = w[e];
        const double2 v = vk[e];
        x.x -= a * v.x;
        x.y -= a * v.y;
        if (k > 0) {
            const double2 u = vkm1[e];
            x.x -= bb * u.x;
            x.y -= bb * u.y;
        }
        w[e] = x;
    }
}

// out[e] = in[e] * s[inst]
__global__ void seg_scale_kernel(SegMap m, double2* out, const double2* in, const double* s) {
    const int b = blockIdx.x;
    const double f = s[m.blk_inst[b]];
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b);
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        const double2 v = in[e];
        out[e] = make_double2(f * v.x, f * v.y);
    }
}

// out[e] = sum_j coef[inst][j] V[j][e]
__global__ void seg_combine_kernel(SegMap m, double2* out, const double2* V, int64_t vstride, int nv,
                                   const double2* coef, int ldc) {
    const int b = blockIdx.x;
    const int i = m.blk_inst[b];
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b);
    const double2* c = coef + (int64_t)i * ldc;
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < nv; ++j) {
            const double2 v = V[(int64_t)j * vstride + e];
            const double2 cj = c[j];
            acc.x += cj.x * v.x - cj.y * v.y;
            acc.y += cj.x * v.y + cj.y * v.x;
        }
        out[e] = acc;
    }
}

// packed[e] = src[inst][e - off[inst]]   (gather), or the reverse (scatter)
__global__ void seg_gather_kernel(SegMap m, double2* packed, const double2* const* src) {
    const int b = blockIdx.x;
    const int i = m.blk_inst[b];
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b), o = m.off[i];
    const double2* s = src[i];
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) packed[e] = s[e - o];
}

__global__ void seg_scatter_kernel(SegMap m, double2* const* dst, const double2* packed) {
    const int b = blockIdx.x;
    const int i = m.blk_inst[b];
    const int64_t lo = m.blk_lo[b], hi = chunk_hi(m, b), o = m.off[i];
    double2* d = dst[i];
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) d[e - o] = packed[e];
}

// ------------------------------------------------------------ scalar steps
// Per-instance state: alpha[i*K + k], beta[i*K + k], beta0, scale, inv (1/||w||
// or 0), done (happy breakdown seen), bad (non-finite value seen).

__global__ void lz_start_kernel(int n, int K, const double2* nrm2, double* beta0, double* inv, double* alpha,
                                double* beta, double* scale, int* done, int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = sqrt_or_nan(nrm2[(int64_t)i * (K + 1)].x);
    beta0[i] = b;
    inv[i] = b > 0.0 ? 1.0 / b : 0.0;
    done[i] = b > 0.0 ? 0 : 1;
    bad[i] = isfinite(b) ? 0 : 1;
    scale[i] = 0.0;
    for (int k = 0; k < K; ++k) {
        alpha[i * K + k] = 0.0;
        beta[i * K + k] = 0.0;
    }
}

__global__ void lz_alpha_kernel(int n, int K, int k, const double2* dots, double* alpha, double* scale, int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = dots[(int64_t)i * (K + 1)].x;
    if (!isfinite(a)) bad[i] = 1;
    alpha[i * K + k] = a;
    scale[i] = fmax(scale[i], fabs(a));
}

// ||w|| -> beta_k and the scale of the next basis vector; a happy breakdown
// (||w|| tiny against the largest coefficient so far) ends the instance:
// its later basis vectors are zero and decouple from T.
__global__ void lz_beta_kernel(int n, int K, int k, const double2* nrm2, double* beta, double* scale, double* inv,
                               int* done, int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = sqrt_or_nan(nrm2[(int64_t)i * (K + 1)].x);
    if (!isfinite(b)) bad[i] = 1;
    const double sc = scale[i];
    if (done[i] || !(b > 1e-14 * sc) || sc == 0.0) {
        done[i] = 1;
        beta[i * K + k] = 0.0;
        inv[i] = 0.0;
    } else {
        beta[i * K + k] = b;
        inv[i] = 1.0 / b;
        scale[i] = fmax(sc, b);
    }
}

// coef[i][j] = beta0 (exp(-i tau T) e_1)_j with T the K x K tridiagonal matrix
// (cyclic Jacobi eigen-decomposition, one thread per instance).
__global__ void lz_expm_kernel(int n, int K, double tau, const double* alpha, const double* beta,
                               const double* beta0, double2* coef, int ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double A[kMaxK * kMaxK], E[kMaxK * kMaxK];
    for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) {
            A[r * K + c] = 0.0;
            E[r * K + c] = r == c ? 1.0 : 0.0;
        }
    for (int r = 0; r < K; ++r) A[r * K + r] = alpha[i * K + r];
    for (int r = 0; r + 1 < K; ++r) A[r * K + r + 1] = A[(r + 1) * K + r] = beta[i * K + r];
    double sc = 0.0;
    for (int r = 0; r < K * K; ++r) sc = fmax(sc, fabs(A[r]));
    for (int sweep = 0; sweep < 100 && K > 1; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < K; ++p)
            for (int q = p + 1; q < K; ++q) off = fmax(off, fabs(A[p * K + q]));
        if (off <= 1e-300 || off <= 1e-18 * sc) break;
        for (int p = 0; p < K; ++p) {
            for (int q = p + 1; q < K; ++q) {
                const double apq = A[p * K + q];
                if (fabs(apq) <= 1e-300) continue;
                const double th = (A[q * K + q] - A[p * K + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < K; ++r) {
                    const double arp = A[r * K + p], arq = A[r * K + q];
                    A[r * K + p] = c * arp - s * arq;
                    A[r * K + q] = s * arp + c * arq;
                }
                for (int r = 0; r < K; ++r) {
                    const double apr = A[p * K + r], aqr = A[q * K + r];
                    A[p * K + r] = c * apr - s * aqr;
                    A[q * K + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < K; ++r) {
                    const double vrp = E[r * K + p], vrq = E[r * K + q];
                    E[r * K + p] = c * vrp - s * vrq;
                    E[r * K + q] = s * vrp + c * vrq;
                }
            }
        }
    }
    const double b0 = beta0[i];
    for (int j = 0; j < K; ++j) {
        double re = 0.0, im = 0.0;
        for (int m = 0; m < K; ++m) {
            const double f = E[j * K + m] * E[m];  // E[0][m] = E[m]
            const double ph = -tau * A[m * K + m];
            re += f * cos(ph);
            im += f * sin(ph);
        }
        coef[(int64_t)i * ldc + j] = make_double2(b0 * re, b0 * im);
    }
}

__global__ void flag_or_kernel(int n, const int* bad, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && bad[i]) *flag = 1;  // benign race: every writer stores 1
}

__global__ void flag_reset_kernel(int* flag) { *flag = 0; }

inline unsigned sblocks(int n) { return (unsigned)((n + 63) / 64); }

}  // namespace

void seg_flag_or(tdvp_ctx ctx, const BatchState& st, int* flag) {
    if (st.ninst == 0) return;
    hipLaunchKernelGGL(flag_or_kernel, dim3(sblocks(st.ninst)), dim3(64), 0, ctx->stream, st.ninst, st.bad, flag);
    TDVP_CHECK_HIP(hipGetLastError());
}

void reset_flag(tdvp_ctx ctx, int* flag) {
    hipLaunchKernelGGL(flag_reset_kernel, dim3(1), dim3(1), 0, ctx->stream, flag);
    TDVP_CHECK_HIP(hipGetLastError());
}

void seg_layout(tdvp_ctx ctx, const std::vector<int64_t>& sizes, SegLayout& L) {
    const int n = (int)sizes.size();
    std::vector<int64_t> off(n + 1, 0), blo;
    std::vector<int> binst, iblk(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        off[i + 1] = off[i] + sizes[i];
        iblk[i] = (int)binst.size();
        for (int64_t e = off[i]; e < off[i + 1]; e += kChunk) {
            binst.push_back(i);
            blo.push_back(e);
        }
    }
    iblk[n] = (int)binst.size();
    L.ninst = n;
    L.total = off[n];
    L.nblk = (int)binst.size();
    L.off = off;
    L.d_off = DevMem(ctx, sizeof(int64_t) * (n + 1));
    L.d_iblk = DevMem(ctx, sizeof(int) * (n + 1));
    L.d_binst = DevMem(ctx, sizeof(int) * std::max(1, L.nblk));
    L.d_blo = DevMem(ctx, sizeof(int64_t) * std::max(1, L.nblk));
    hipStream_t s = ctx->stream;
    TDVP_CHECK_HIP(hipMemcpyAsync(L.d_off.ptr, off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    TDVP_CHECK_HIP(hipMemcpyAsync(L.d_iblk.ptr, iblk.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, s));
    if (L.nblk) {
        TDVP_CHECK_HIP(hipMemcpyAsync(L.d_binst.ptr, binst.data(), sizeof(int) * L.nblk, hipMemcpyHostToDevice, s));
        TDVP_CHECK_HIP(hipMemcpyAsync(L.d_blo.ptr, blo.data(), sizeof(int64_t) * L.nblk, hipMemcpyHostToDevice, s));
    }
    TDVP_CHECK_HIP(hipStreamSynchronize(s));
}

namespace {
SegMap segmap(const SegLayout& L) {
    return SegMap{L.d_binst.as<int>(), L.d_blo.as<int64_t>(), L.d_off.as<int64_t>()};
}
}  // namespace

void seg_gather(tdvp_ctx ctx, const SegLayout& L, double2* packed, const double2* const* src_dev) {
    if (!L.nblk) return;
    hipLaunchKernelGGL(seg_gather_kernel, dim3(L.nblk), dim3(kThreads), 0, ctx->stream, segmap(L), packed, src_dev);
    TDVP_CHECK_HIP(hipGetLastError());
}

void seg_scatter(tdvp_ctx ctx, const SegLayout& L, double2* const* dst_dev, const double2* packed) {
    if (!L.nblk) return;
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(L.nblk), dim3(kThreads), 0, ctx->stream, segmap(L), dst_dev, packed);
    TDVP_CHECK_HIP(hipGetLastError());
}

// The whole exponentiation: theta (packed) <- exp(-i tau H_i) theta_i for
// every instance, K matrix-vector products each (fewer on breakdown).
void batch_expm(tdvp_ctx ctx, const SegLayout& L, const BatchOp& op, double2* theta, double tau, int K,
                BatchState& st) {
    TDVP_REQUIRE(K >= 1 && K <= kMaxK, TDVP_E_ARG, "batched Krylov: k must be in 1..16");
    if (L.ninst == 0 || L.total == 0) return;
    hipStream_t s = ctx->stream;
    const int n = L.ninst;
    const int64_t T = L.total;
    const SegMap m = segmap(L);
    const unsigned nb = (unsigned)L.nblk;
    double2* V = static_cast<double2*>(ctx->workspace("bk_V", sizeof(double2) * (size_t)(K + 1) * T));
    double2* w = static_cast<double2*>(ctx->workspace("bk_w", sizeof(double2) * (size_t)T));
    double2* partial =
        static_cast<double2*>(ctx->workspace("bk_partial", sizeof(double2) * (size_t)(K + 1) * L.nblk));
    double2* dots = static_cast<double2*>(ctx->workspace("bk_dots", sizeof(double2) * (size_t)n * (K + 1)));
    double* sc = static_cast<double*>(ctx->workspace("bk_scal", sizeof(double) * (size_t)n * (2 * K + 3)));
    double* alpha = sc;
    double* beta = alpha + (size_t)n * K;
    double* beta0 = beta + (size_t)n * K;
    double* scale = beta0 + n;
    double* inv = scale + n;
    int* flags = static_cast<int*>(ctx->workspace("bk_flags", sizeof(int) * (size_t)2 * n));
    int* done = flags;
    st.bad = flags + n;
    st.ninst = n;

    auto dot = [&](const double2* Vs, int64_t vstride, int nv, const double2* x, double2* out) {
        hipLaunchKernelGGL(seg_dot_partial_kernel, dim3(nb), dim3(kThreads), 0, s, m, Vs, vstride, nv, x, L.nblk,
                           partial);
        hipLaunchKernelGGL(seg_reduce_kernel, dim3(n, nv), dim3(kThreads), 0, s, partial, L.nblk,
                           L.d_iblk.as<int>(), out, K + 1);
    };

    dot(theta, 0, 1, theta, dots);
    hipLaunchKernelGGL(lz_start_kernel, dim3(sblocks(n)), dim3(64), 0, s, n, K, dots, beta0, inv, alpha, beta, scale,
                       done, st.bad);
    hipLaunchKernelGGL(seg_scale_kernel, dim3(nb), dim3(kThreads), 0, s, m, V, theta, inv);
    for (int k = 0; k < K; ++k) {
        double2* vk = V + (size_t)k * T;
        op(vk, w);
        dot(vk, 0, 1, w, dots);  // alpha_k = <v_k, H v_k>
        hipLaunchKernelGGL(lz_alpha_kernel, dim3(sblocks(n)), dim3(64), 0, s, n, K, k, dots, alpha, scale, st.bad);
        hipLaunchKernelGGL(seg_3term_kernel, dim3(nb), dim3(kThreads), 0, s, m, w, vk,
                           k > 0 ? V + (size_t)(k - 1) * T : nullptr, alpha, beta, k, K);
        for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
            dot(V, T, k + 1, w, dots);
            hipLaunchKernelGGL(seg_axpy_kernel, dim3(nb), dim3(kThreads), 0, s, m, V, T, k + 1, dots, K + 1, w);
        }
        if (k + 1 == K) break;  // the last ||w|| is not needed
        dot(w, 0, 1, w, dots);
        hipLaunchKernelGGL(lz_beta_kernel, dim3(sblocks(n)), dim3(64), 0, s, n, K, k, dots, beta, scale, inv, done,
                           st.bad);
        hipLaunchKernelGGL(seg_scale_kernel, dim3(nb), dim3(kThreads), 0, s, m, V + (size_t)(k + 1) * T, w, inv);
    }
    double2* coef = static_cast<double2*>(ctx->workspace("bk_coef", sizeof(double2) * (size_t)n * K));
    hipLaunchKernelGGL(lz_expm_kernel, dim3(sblocks(n)), dim3(64), 0, s, n, K, tau, alpha, beta, beta0, coef, K);
    hipLaunchKernelGGL(seg_combine_kernel, dim3(nb), dim3(kThreads), 0, s, m, theta, V, T, K, coef, K);
    TDVP_CHECK_HIP(hipGetLastError());
}

// Workspace sizes batch_expm will request (so that a graph capture that
// follows does not allocate).
void batch_expm_reserve(tdvp_ctx ctx, const SegLayout& L, int K) {
    const int n = std::max(1, L.ninst);
    const int64_t T = std::max<int64_t>(1, L.total);
    ctx->workspace("bk_V", sizeof(double2) * (size_t)(K + 1) * T);
    ctx->workspace("bk_w", sizeof(double2) * (size_t)T);
    ctx->workspace("bk_partial", sizeof(double2) * (size_t)(K + 1) * std::max(1, L.nblk));
    ctx->workspace("bk_dots", sizeof(double2) * (size_t)n * (K + 1));
    ctx->workspace("bk_scal", sizeof(double) * (size_t)n * (2 * K + 3));
    ctx->workspace("bk_flags", sizeof(int) * (size_t)2 * n);
    ctx->workspace("bk_coef", sizeof(double2) * (size_t)n * K);
}

}  // namespace tdvp
