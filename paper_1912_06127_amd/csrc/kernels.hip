// Memory-bound kernels of the TDVP path: the sparse MPO stage between the
// two GEMMs of H_eff and of the environment updates, the FP64 vector
// operations of Lanczos, and small reshaping helpers around the dense
// solvers.
#include "common.hpp"

#include <algorithm>

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
// short sparse dot product with the MPO entries.  The sparse operator (a few
// hundred entries for the MPOs used here) is first copied into LDS by the
// whole block, so the inner loop reads broadcast LDS values instead of a
// chain of dependent global loads; larger operators are read from global
// memory.  Loads and stores are coalesced along q.
struct WParams {
    const void* in; int in128;
    void* out; int out128;
    int P, Q, D, nin, nout;
    int64_t ik, is, ip, on, os, op;
    const int* row_ptr;
    const int* col;
    const void* val;
};

constexpr int kWNnzCap = 512;  // operator entries staged in LDS
constexpr int kWRowCap = 512;  // operator rows staged in LDS

// bytes of the staged operator, rounded up so that the input columns behind
// it stay 16-byte aligned
template <typename T>
constexpr size_t wstage_op_bytes() {
    return ((size_t)kWNnzCap * (sizeof(typename cplx<T>::t) + sizeof(int)) + (size_t)(kWRowCap + 1) * sizeof(int) + 15) /
           16 * 16;
}

// A block handles wpts<T>() consecutive q of one p with kWSub groups of
// threads: every group loads every kWSub-th input row of those points
// (coalesced along q) into the shared [nin][points] tile, then computes every
// kWSub-th output row.
// Sharing each point over four waves keeps the LDS per thread small enough
// for several blocks per CU, so many loads are in flight.
constexpr int kWSub = 4;
// points per block: 128 in complex64 (each row of a block is 1 KiB of
// contiguous memory), 64 in complex128 (the same bytes; keeps the LDS tile
// within bounds for the widest MPO bonds)
template <typename T>
constexpr int wpts() {
    return sizeof(T) == 4 ? 128 : 64;
}
constexpr int kWRowsInFlight = 16;  // input rows per wave loaded back to back (nin <= 64)
template <typename T>
constexpr int wthreads() {
    return kWSub * wpts<T>();
}

template <typename T>
__device__ __forceinline__ void wstage_tile(const WParams& w, int p, int q0, typename cplx<T>::t* xin, const int* rp,
                                            const int* cl, const typename cplx<T>::t* vl) {
    using C = typename cplx<T>::t;
    constexpr int kWPts = wpts<T>();
    const int lane = threadIdx.x % kWPts, sub = threadIdx.x / kWPts;
    const int q = q0 + lane;
    const bool live = q < w.Q;
    const int64_t pin = (int64_t)p * w.ip + q;
    if (w.nin <= kWSub * kWRowsInFlight) {
        // every input row of this wave loaded before any is stored: all the
        // wave's loads are in flight together
        C buf[kWRowsInFlight];
#pragma unroll
        for (int i = 0; i < kWRowsInFlight; ++i) {
            const int c = sub + kWSub * i;
            T re = 0, im = 0;
            if (live && c < w.nin) ld<T>(w.in, w.in128, pin + (c / w.D) * w.ik + (c % w.D) * w.is, re, im);
            buf[i] = C{re, im};
        }
#pragma unroll
        for (int i = 0; i < kWRowsInFlight; ++i) {
            const int c = sub + kWSub * i;
            if (c < w.nin) xin[c * kWPts + lane] = buf[i];
        }
    } else {
#pragma unroll 4
        for (int c = sub; c < w.nin; c += kWSub) {
            const int k = c / w.D, s = c % w.D;
            T re = 0, im = 0;
            if (live) ld<T>(w.in, w.in128, pin + k * w.ik + s * w.is, re, im);
            xin[c * kWPts + lane] = C{re, im};
        }
    }
    __syncthreads();
    if (!live) return;  // no barrier below
    const int64_t pout = (int64_t)p * w.op + q;
    for (int r = sub; r < w.nout; r += kWSub) {
        T ar = 0, ai = 0;
        const int e1 = rp[r + 1];
        for (int e = rp[r]; e < e1; ++e) {
            const C v = vl[e];
            const C x = xin[cl[e] * kWPts + lane];
            ar += v.x * x.x - v.y * x.y;
            ai += v.x * x.y + v.y * x.x;
        }
        const int n = r / w.D, s = r % w.D;
        st<T>(w.out, w.out128, pout + n * w.on + s * w.os, ar, ai);
    }
}

// Copies the operator into LDS when it fits (block-uniform decision) and
// returns the pointers the tile should read.  Contains a barrier: every
// thread of the block must call it.
template <typename T>
__device__ __forceinline__ void wstage_stage_op(const WParams& w, unsigned char* smem, const int*& rp, const int*& cl,
                                                const typename cplx<T>::t*& vl) {
    using C = typename cplx<T>::t;
    const int nnz = w.row_ptr[w.nout];
    C* sv = reinterpret_cast<C*>(smem);
    int* sc = reinterpret_cast<int*>(sv + kWNnzCap);
    int* sr = sc + kWNnzCap;
    const bool fits = nnz <= kWNnzCap && w.nout <= kWRowCap;
    if (fits) {
        const C* gv = reinterpret_cast<const C*>(w.val);
        for (int i = threadIdx.x; i < nnz; i += blockDim.x) {
            sv[i] = gv[i];
            sc[i] = w.col[i];
        }
        for (int i = threadIdx.x; i <= w.nout; i += blockDim.x) sr[i] = w.row_ptr[i];
    }
    __syncthreads();
    rp = fits ? sr : w.row_ptr;
    cl = fits ? sc : w.col;
    vl = fits ? sv : reinterpret_cast<const C*>(w.val);
}

template <typename T>
__global__ void __launch_bounds__(wthreads<T>()) wstage_kernel(WParams w) {
    using C = typename cplx<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int* rp;
    const int* cl;
    const C* vl;
    wstage_stage_op<T>(w, smem_raw, rp, cl, vl);
    C* xin = reinterpret_cast<C*>(smem_raw + wstage_op_bytes<T>());  // [nin][kWPts]
    wstage_tile<T>(w, blockIdx.y, blockIdx.x * wpts<T>(), xin, rp, cl, vl);
}

// Grouped MPO stage: problem g owns blocks [blk_begin, blk_begin + P*qblocks).
struct GWProblem {
    WParams w;
    int64_t blk_begin;
    int qblocks;
};

template <typename T>
__global__ void __launch_bounds__(wthreads<T>()) wstage_grouped_kernel(const GWProblem* __restrict__ probs,
                                                                        int nprob) {
    using C = typename cplx<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
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
    const int q0 = (int)(local % qb) * wpts<T>();
    const WParams w = probs[lo].w;
    const int* rp;
    const int* cl;
    const C* vl;
    wstage_stage_op<T>(w, smem_raw, rp, cl, vl);  // the whole block shares problem lo
    C* xin = reinterpret_cast<C*>(smem_raw + wstage_op_bytes<T>());
    wstage_tile<T>(w, p, q0, xin, rp, cl, vl);
}

// ------------------------------------------- fused H_eff for small bonds
// For small chi_l, chi_r the three stages of y = H_eff x (Sec. III A) have
// only a few hundred points each and are bound by launch latency.  Here one
// block per output row a' and output index s' runs all of them with the
// intermediates in LDS:
//   T1[k][s][b] = sum_a L[k][a'][a] x[a][s][b]          (k < wl, s < D, b < chi_r)
//   T3[n][b]    = sum_e M[n D + s'][c_e] T1[c_e][b]     (sparse MPO stage, row s' only)
//   y[a'][s'][b'] = sum_n sum_b T3[n][b] R[n][b][b']
// The L row of a' and the MPO operator are staged in LDS, x passes through
// LDS in chunks of `rows` rows (all of x when it fits) with coalesced loads.
// Stage B gives each of G thread groups every G-th n and reads R straight
// from L2 (coalesced along b'); the partial sums meet in LDS.  Stage A is
// repeated by the D blocks of one a', which is cheap next to the latency
// it hides.
struct HsParams {
    const void* L; int L128;
    const void* R; int R128;
    const void* x; int x128;
    void* y; int y128;
    const int* row_ptr;
    const int* col;
    const void* val;
    int chil, chir, D, wl, wr, rows;
};

constexpr int kHsThreads = 256;
constexpr int kHsKC = 8;    // stage-A accumulators (values of k) per thread
constexpr int kHsRows = 8;  // x rows per chunk when the whole of x does not fit

__host__ __device__ inline int heff_small_groups(int chir, int wr) {  // stage-B groups over n
    return min(wr, kHsThreads / chir);
}

template <typename T>
size_t heff_small_smem(int chil, int chir, int D, int wl, int wr, int rows) {
    const size_t nc = (size_t)D * chir;
    const size_t red = std::max((size_t)kHsThreads, (size_t)heff_small_groups(chir, wr) * chir);
    return wstage_op_bytes<T>() +
           sizeof(typename cplx<T>::t) * (wl * nc + (size_t)wr * chir + red + (size_t)wl * chil + (size_t)rows * nc);
}

// Element i of a complex array stored as S (float2 or double2), as C.
template <typename C, typename S>
__device__ __forceinline__ C ld_as(const void* p, int64_t i) {
    const S v = reinterpret_cast<const S*>(p)[i];
    C c;
    c.x = v.x;
    c.y = v.y;
    return c;
}

// L and R are in the compute precision (the launcher checks it); x is stored
// as XS.  All loads have a compile-time width and no branch around them, so
// the staging loops issue kHsLoads loads before their first wait and the
// stage-B loop over b can keep several R loads in flight.
constexpr int kHsLoads = 4;

template <typename T, typename XS>
__global__ void __launch_bounds__(kHsThreads) heff_small_kernel(HsParams h) {
    using C = typename cplx<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WParams w;
    w.row_ptr = h.row_ptr;
    w.col = h.col;
    w.val = h.val;
    w.nout = h.wr * h.D;
    const int* rp;
    const int* cl;
    const C* vl;
    const int tid = threadIdx.x, ap = blockIdx.x, sp = blockIdx.y;
    const int NC = h.D * h.chir;
    const int G = heff_small_groups(h.chir, h.wr);
    const int NR = max(kHsThreads, G * h.chir);
    C* T1 = reinterpret_cast<C*>(smem_raw + wstage_op_bytes<T>());  // [wl][D][chir]
    C* T3 = T1 + (size_t)h.wl * NC;                                  // [wr][chir], row s' = sp
    C* red = T3 + (size_t)h.wr * h.chir;                             // [NR]
    C* Ls = red + NR;                                                // [wl][chil]
    C* xb = Ls + (size_t)h.wl * h.chil;                              // [rows][NC]
    for (int i0 = 0; i0 < h.wl * h.chil; i0 += kHsThreads * kHsLoads) {
        C buf[kHsLoads];
#pragma unroll
        for (int u = 0; u < kHsLoads; ++u) {
            const int i = i0 + u * kHsThreads + tid;
            const int ii = i < h.wl * h.chil ? i : 0;
            const int k = ii / h.chil, a = ii % h.chil;
            buf[u] = ld_as<C, C>(h.L, ((int64_t)k * h.chil + ap) * h.chil + a);
        }
#pragma unroll
        for (int u = 0; u < kHsLoads; ++u) {
            const int i = i0 + u * kHsThreads + tid;
            if (i < h.wl * h.chil) Ls[i] = buf[u];
        }
    }
    for (int i = tid; i < h.wl * NC; i += kHsThreads) T1[i] = C{T(0), T(0)};

    // stage A over chunks of x rows; item = (column (s, b), kHsKC values of k)
    const int kchunks = (h.wl + kHsKC - 1) / kHsKC;
    for (int a0 = 0; a0 < h.chil; a0 += h.rows) {
        const int na = min(h.rows, h.chil - a0);
        if (a0 > 0) __syncthreads();  // the previous chunk is consumed
        for (int i0 = 0; i0 < na * NC; i0 += kHsThreads * kHsLoads) {
            C buf[kHsLoads];
#pragma unroll
            for (int u = 0; u < kHsLoads; ++u) {
                const int i = i0 + u * kHsThreads + tid;
                buf[u] = ld_as<C, XS>(h.x, (int64_t)a0 * NC + (i < na * NC ? i : 0));
            }
#pragma unroll
            for (int u = 0; u < kHsLoads; ++u) {
                const int i = i0 + u * kHsThreads + tid;
                if (i < na * NC) xb[i] = buf[u];
            }
        }
        if (a0 == 0) wstage_stage_op<T>(w, smem_raw, rp, cl, vl);  // its barrier also publishes Ls, T1, xb
        else __syncthreads();
        for (int item = tid; item < NC * kchunks; item += kHsThreads) {
            const int c = item % NC, k0 = (item / NC) * kHsKC;
            T ar[kHsKC], ai[kHsKC];
#pragma unroll
            for (int j = 0; j < kHsKC; ++j) ar[j] = ai[j] = T(0);
            for (int a = 0; a < na; ++a) {
                const C xv = xb[a * NC + c];
#pragma unroll
                for (int j = 0; j < kHsKC; ++j) {
                    if (k0 + j < h.wl) {
                        const C l = Ls[(k0 + j) * h.chil + a0 + a];
                        ar[j] += l.x * xv.x - l.y * xv.y;
                        ai[j] += l.x * xv.y + l.y * xv.x;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kHsKC; ++j) {
                if (k0 + j < h.wl) {
                    C& t = T1[(size_t)(k0 + j) * NC + c];
                    t.x += ar[j];
                    t.y += ai[j];
                }
            }
        }
    }
    __syncthreads();

    // MPO stage for output index s': item = (n, b)
    for (int item = tid; item < h.wr * h.chir; item += kHsThreads) {
        const int n = item / h.chir, b = item % h.chir;
        const int r = n * h.D + sp;
        T ar = 0, ai = 0;
        const int e1 = rp[r + 1];
        for (int e = rp[r]; e < e1; ++e) {
            const C v = vl[e];
            const C t = T1[(size_t)cl[e] * h.chir + b];
            ar += v.x * t.x - v.y * t.y;
            ai += v.x * t.y + v.y * t.x;
        }
        T3[item] = C{ar, ai};
    }
    __syncthreads();

    // stage B: item = (b', group g over n = g, g + G, ...)
    for (int item = tid; item < G * h.chir; item += kHsThreads) {
        const int bp = item % h.chir, g = item / h.chir;
        T ar = 0, ai = 0;
        for (int n = g; n < h.wr; n += G) {
            const C* t3 = T3 + (size_t)n * h.chir;
            const C* Rn = reinterpret_cast<const C*>(h.R) + (int64_t)n * h.chir * h.chir + bp;
#pragma unroll 8
            for (int b = 0; b < h.chir; ++b) {
                const C r = Rn[(int64_t)b * h.chir];
                const C t = t3[b];
                ar += t.x * r.x - t.y * r.y;
                ai += t.x * r.y + t.y * r.x;
            }
        }
        red[item] = C{ar, ai};
    }
    __syncthreads();
    for (int bp = tid; bp < h.chir; bp += kHsThreads) {
        T ar = 0, ai = 0;
        for (int g = 0; g < G; ++g) {
            const C v = red[g * h.chir + bp];
            ar += v.x;
            ai += v.y;
        }
        st<T>(h.y, h.y128, ((int64_t)ap * h.D + sp) * h.chir + bp, ar, ai);
    }
}

// ------------------------------------------------------- small Lanczos step
// One Lanczos step for a short vector (n <= kSmallLanczos) in one workgroup:
// alpha = Re<v_k, w>, w -= alpha v_k + beta v_{k-1}, classical Gram-Schmidt
// against v_0..v_k (a second pass when the first removed more than half of
// ||w||^2), then ||w||^2 and v_{k+1} = w/||w||.
// Replaces about a dozen launches of the general path when every launch
// costs more than the arithmetic (small bond dimensions).
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kSmallMaxK = 64;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup, the same value in every thread; part holds
// kSmallWaves doubles and may be reused right after the call.
__device__ inline double block_sum_small(double v, double* part) {
    v = wave_sum(v);
    __syncthreads();  // earlier readers of part are done
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kSmallWaves; ++i) t += part[i];
    return t;
}

__global__ void __launch_bounds__(kSmallThreads) lanczos_small_kernel(double2* V, int64_t n, int k, double2* w,
                                                                      double beta_prev, const double* nn_prev,
                                                                      double* out) {
    // beta_{k-1} from the previous step's ||w||^2 when it is still on the device
    if (nn_prev) beta_prev = sqrt_or_nan(*nn_prev);
    __shared__ double sre[kSmallMaxK + 1][kSmallWaves], sim[kSmallMaxK + 1][kSmallWaves];
    __shared__ double coef_re[kSmallMaxK + 1], coef_im[kSmallMaxK + 1];
    __shared__ double part[kSmallWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double2* vk = V + (int64_t)k * n;
    // alpha_k = Re <v_k, w>
    double a = 0.0;
    for (int64_t e = tid; e < n; e += kSmallThreads) a += vk[e].x * w[e].x + vk[e].y * w[e].y;
    const double alpha = block_sum_small(a, part);
    // three-term recurrence, with ||w||^2 of the result
    double nb = 0.0;
    for (int64_t e = tid; e < n; e += kSmallThreads) {
        double2 x = w[e];
        x.x -= alpha * vk[e].x;
        x.y -= alpha * vk[e].y;
        if (k > 0) {
            const double2 u = V[(int64_t)(k - 1) * n + e];
            x.x -= beta_prev * u.x;
            x.y -= beta_prev * u.y;
        }
        w[e] = x;
        nb += x.x * x.x + x.y * x.y;
    }
    nb = block_sum_small(nb, part);
    // Classical Gram-Schmidt against v_0..v_k; a second pass only when the
    // first removed more than half of ||w||^2 (the DGKS criterion with
    // eta = 1/sqrt(2): otherwise one pass already leaves w orthogonal to
    // working precision).
    double nn = nb;
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j <= k; ++j) {  // c_j = <v_j, w>
            const double2* v = V + (int64_t)j * n;
            double re = 0.0, im = 0.0;
            for (int64_t e = tid; e < n; e += kSmallThreads) {
                re += v[e].x * w[e].x + v[e].y * w[e].y;
                im += v[e].x * w[e].y - v[e].y * w[e].x;
            }
            re = wave_sum(re);
            im = wave_sum(im);
            if (lane == 0) {
                sre[j][wave] = re;
                sim[j][wave] = im;
            }
        }
        __syncthreads();
        if (tid <= k) {
            double re = 0.0, im = 0.0;
            for (int i = 0; i < kSmallWaves; ++i) {
                re += sre[tid][i];
                im += sim[tid][i];
            }
            coef_re[tid] = re;
            coef_im[tid] = im;
        }
        __syncthreads();
        double na = 0.0;
        for (int64_t e = tid; e < n; e += kSmallThreads) {  // w -= sum_j c_j v_j
            double2 x = w[e];
            for (int j = 0; j <= k; ++j) {
                const double2 v = V[(int64_t)j * n + e];
                x.x -= coef_re[j] * v.x - coef_im[j] * v.y;
                x.y -= coef_re[j] * v.y + coef_im[j] * v.x;
            }
            w[e] = x;
            na += x.x * x.x + x.y * x.y;
        }
        const double before = nn;
        nn = block_sum_small(na, part);  // also orders the w updates before the next pass
        if (nn >= 0.5 * before) break;   // uniform: every thread holds the same sums
    }
    if (tid == 0) {
        out[0] = alpha;
        out[1] = nn;
    }
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    double2* vn = V + (int64_t)(k + 1) * n;
    for (int64_t e = tid; e < n; e += kSmallThreads) vn[e] = make_double2(w[e].x * inv, w[e].y * inv);
}

__global__ void __launch_bounds__(kSmallThreads) small_normalize_kernel(const double2* x, double2* v, int64_t n,
                                                                        double* nn_out) {
    __shared__ double part[kSmallWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double nn = 0.0;
    for (int64_t e = tid; e < n; e += kSmallThreads) nn += x[e].x * x[e].x + x[e].y * x[e].y;
    nn = wave_sum(nn);
    if (lane == 0) part[wave] = nn;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kSmallWaves; ++i) t += part[i];  // every thread forms the same sum
    if (tid == 0) nn_out[0] = t;
    const double inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
    for (int64_t e = tid; e < n; e += kSmallThreads) v[e] = make_double2(x[e].x * inv, x[e].y * inv);
}


// --------------------------------------------- small Hermitian eigensolver
// Cyclic Jacobi for a Hermitian matrix of order n <= kJacobiMax in one
// workgroup, matrix and eigenvectors resident in LDS.  Rounds follow the
// round-robin (tournament) ordering: n/2 disjoint index pairs per round,
// whose rotations commute, so all of them are applied together -- first to
// the columns of A and V, then to the rows of A.  For a_pq = |a_pq| e^{i phi}
// the rotation is U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] (a phase that
// makes a_pq real, then the real Jacobi angle); A <- U^H A U, V <- V U.
// |a_pq| is taken with hypot: sqrt(x^2 + y^2) loses its precision once the
// squares are subnormal, and a phase e^{i phi} off the unit circle scales
// an eigenvector instead of rotating it.  Entries at or below 1e-18 ||A||_F
// (a rounding-level perturbation of A) are not rotated, so repeated sweeps
// over a null space never push entries into the subnormal range.  Sweeps
// stop when the off-diagonal mass is below 1e-30 of the diagonal mass, or
// after 40 sweeps.  Outputs: eigenvalues in descending order and
// the eigenvectors as conjugated rows (row c = conj of the c-th eigenvector).
// ------------------------------------------------ small QR in one workgroup
// Thin Householder QR of an m x n complex matrix B (m >= n) held in LDS, in
// the reflector convention of LAPACK's zgeqr2 / zung2r: reflector k is
// H_k = I - tau_k v v^H with v_k = 1, built so that H_k^H maps column k below
// the diagonal onto beta_k e_k with real beta_k; B = Q R with Q = H_0 ... H_{n-1}
// (first n columns) and R upper triangular.  One wave per column for the
// reflector applications (lanes over rows, shuffle reductions).
// herm = 0: B = M (row-major [m][n]); outputs Q [m][n] and R [n][n] (upper),
// both row-major with leading dimension n.
// herm = 1: B = M^H with M row-major [n][m] (the LQ of M = R^H Q^H); outputs
// L = R^H [n][n] (lower, ld n) to RL and Q^H [n][m] (ld m) to Qout.
constexpr int kQrThreads = 256;
constexpr int kQrWaves = kQrThreads / 64;

__device__ inline double2 qr_cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 qr_cjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 qr_wave_sum(double2 v) {
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

__global__ void __launch_bounds__(kQrThreads) qr_small_kernel(const double2* __restrict__ M, int m, int n, int herm,
                                                              double2* __restrict__ Qout, double2* __restrict__ RL) {
    __shared__ double2 A[kQrMaxElems];
    __shared__ double2 Q[kQrMaxElems];
    __shared__ double2 tau[kQrMaxCols];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < m * n; e += kQrThreads) {
        const int i = e / n, j = e % n;
        if (herm) {
            const double2 x = M[(int64_t)j * m + i];
            A[e] = make_double2(x.x, -x.y);
        } else {
            A[e] = M[(int64_t)i * n + j];
        }
        Q[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (wave == 0) {
            double xn = 0.0;  // squared norm of column k below the diagonal
            for (int i = k + 1 + lane; i < m; i += 64) xn += A[i * n + k].x * A[i * n + k].x + A[i * n + k].y * A[i * n + k].y;
            for (int o = 32; o > 0; o >>= 1) xn += __shfl_xor(xn, o, 64);
            const double2 alpha = A[k * n + k];
            double2 t = make_double2(0.0, 0.0), sc = make_double2(0.0, 0.0);
            double beta = alpha.x;
            const bool reflect = !(xn == 0.0 && alpha.y == 0.0);
            if (reflect) {
                beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn), alpha.x);
                t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                // sc = 1 / (alpha - beta)
                const double dr = alpha.x - beta, di = alpha.y, dd = dr * dr + di * di;
                sc = make_double2(dr / dd, -di / dd);
            }
            for (int i = k + 1 + lane; i < m; i += 64) A[i * n + k] = reflect ? qr_cmul(A[i * n + k], sc) : A[i * n + k];
            if (lane == 0) {
                tau[k] = t;
                if (reflect) A[k * n + k] = make_double2(beta, 0.0);
            }
        }
        __syncthreads();
        // columns j > k: A(k:m, j) -= conj(tau) v (v^H A(k:m, j))
        const double2 tk = tau[k];
        for (int j = k + 1 + wave; j < n; j += kQrWaves) {
            double2 w = make_double2(0.0, 0.0);
            for (int i = k + lane; i < m; i += 64) {
                const double2 v = i == k ? make_double2(1.0, 0.0) : A[i * n + k];
                const double2 p = qr_cjmul(v, A[i * n + j]);
                w.x += p.x;
                w.y += p.y;
            }
            w = qr_wave_sum(w);
            const double2 f = qr_cjmul(tk, w);  // conj(tau) w
            for (int i = k + lane; i < m; i += 64) {
                const double2 v = i == k ? make_double2(1.0, 0.0) : A[i * n + k];
                const double2 d = qr_cmul(v, f);
                A[i * n + j].x -= d.x;
                A[i * n + j].y -= d.y;
            }
        }
        __syncthreads();
    }
    // Q = H_0 ... H_{n-1} I: reflectors applied from the last, columns j >= k
    for (int k = n - 1; k >= 0; --k) {
        const double2 tk = tau[k];
        for (int j = k + wave; j < n; j += kQrWaves) {
            double2 w = make_double2(0.0, 0.0);
            for (int i = k + lane; i < m; i += 64) {
                const double2 v = i == k ? make_double2(1.0, 0.0) : A[i * n + k];
                const double2 p = qr_cjmul(v, Q[i * n + j]);
                w.x += p.x;
                w.y += p.y;
            }
            w = qr_wave_sum(w);
            const double2 f = qr_cmul(tk, w);  // tau w
            for (int i = k + lane; i < m; i += 64) {
                const double2 v = i == k ? make_double2(1.0, 0.0) : A[i * n + k];
                const double2 d = qr_cmul(v, f);
                Q[i * n + j].x -= d.x;
                Q[i * n + j].y -= d.y;
            }
        }
        __syncthreads();
    }
    if (!herm) {
        for (int e = tid; e < m * n; e += kQrThreads) Qout[e] = Q[e];
        for (int e = tid; e < n * n; e += kQrThreads) {
            const int r = e / n, c = e % n;
            RL[e] = c >= r ? A[r * n + c] : make_double2(0.0, 0.0);
        }
    } else {
        for (int e = tid; e < m * n; e += kQrThreads) {  // Q^H [n][m]
            const int c = e / m, j = e % m;
            const double2 q = Q[j * n + c];
            Qout[e] = make_double2(q.x, -q.y);
        }
        for (int e = tid; e < n * n; e += kQrThreads) {  // L = R^H, lower
            const int a = e / n, c = e % n;
            const double2 r = A[c * n + a];
            RL[e] = c <= a ? make_double2(r.x, -r.y) : make_double2(0.0, 0.0);
        }
    }
}

constexpr int kJacobiMax = kJacobiMaxOrder;
constexpr int kJacobiThreads = 256;

__device__ __forceinline__ void jacobi_eigh_body(const double2* G, int n, double* evals, double2* vecs,
                                                 int* sweeps_out) {
    __shared__ double2 A[kJacobiMax * kJacobiMax];
    __shared__ double2 V[kJacobiMax * kJacobiMax];
    __shared__ double rc[kJacobiMax / 2], rs[kJacobiMax / 2], rpr[kJacobiMax / 2], rpi[kJacobiMax / 2];
    __shared__ int rp[kJacobiMax / 2], rq[kJacobiMax / 2];
    __shared__ double red[kJacobiThreads], red2[kJacobiThreads];
    __shared__ int done;
    const int tid = threadIdx.x;
    const int m = n + (n & 1);  // even order for the tournament (a padded index is a no-op)
    for (int i = tid; i < m * m; i += kJacobiThreads) {
        const int r = i / m, c = i % m;
        // Hermitian part of G: a rounding-level anti-Hermitian remainder could
        // never be rotated away and would hold the sweeps at their cap
        double2 a = make_double2(0.0, 0.0);
        if (r < n && c < n) {
            const double2 x = G[r * n + c], y = G[c * n + r];
            a = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
        }
        A[i] = a;
        V[i] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    if (tid == 0) done = 0;
    __syncthreads();
    const int half = m / 2;
    int sweep = 0;
    for (; sweep < 40; ++sweep) {
        // convergence test: off-diagonal vs diagonal mass
        double off = 0.0, dia = 0.0;
        for (int i = tid; i < m * m; i += kJacobiThreads) {
            const int r = i / m, c = i % m;
            const double a2 = A[i].x * A[i].x + A[i].y * A[i].y;
            if (r == c) dia += a2;
            else off += a2;
        }
        red[tid] = off;
        red2[tid] = dia;
        __syncthreads();
        for (int h = kJacobiThreads / 2; h > 0; h >>= 1) {
            if (tid < h) {
                red[tid] += red[tid + h];
                red2[tid] += red2[tid + h];
            }
            __syncthreads();
        }
        if (tid == 0) done = (red[0] <= 1e-30 * red2[0] || red[0] == 0.0) ? 1 : 0;
        __syncthreads();
        if (done) break;
        const double skip = 1e-18 * sqrt(red[0] + red2[0]);  // red[] is rewritten only in the next sweep
        for (int round = 0; round < m - 1; ++round) {
            // tournament pairs: position 0 fixed, the others rotate
            if (tid < half) {
                const int a = tid == 0 ? 0 : 1 + (tid - 1 + round) % (m - 1);
                const int b = 1 + (m - 2 - tid + round) % (m - 1);
                const int p = a < b ? a : b, q = a < b ? b : a;
                rp[tid] = p;
                rq[tid] = q;
                const double2 apq = A[p * m + q];
                const double mag = hypot(apq.x, apq.y);
                double c = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
                if (mag > skip && mag > 1e-290) {
                    const double tau = (A[q * m + q].x - A[p * m + p].x) / (2.0 * mag);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sn = t * c;
                    er = apq.x / mag;  // e^{i phi}
                    ei = apq.y / mag;
                }
                rc[tid] = c;
                rs[tid] = sn;
                rpr[tid] = er;
                rpi[tid] = ei;
            }
            __syncthreads();
            // Column rotation of pair k (V and A): col_p' = c col_p - s e^{-i phi} col_q,
            // col_q' = s col_p + c e^{-i phi} col_q; row rotation (A): row_p' = c row_p -
            // s e^{i phi} row_q, row_q' = s row_p + c e^{i phi} row_q.  The pairs
            // partition the indices, so A is updated block by block: the 2 x 2 block
            // of pairs (P, Q) takes the column rotation of Q and then the row rotation
            // of P, the same operations in the same order as a full column pass
            // followed by a full row pass, with A read and written once.
            for (int i = tid; i < half * half + half * m; i += kJacobiThreads) {
                if (i < half * half) {
                    const int P = i / half, Q = i % half;
                    const int p1 = rp[P], p2 = rq[P], q1 = rp[Q], q2 = rq[Q];
                    const double cq = rc[Q], sq = rs[Q], erq = rpr[Q], eiq = -rpi[Q];  // e^{-i phi_Q}
                    const double cp = rc[P], sp = rs[P], erp = rpr[P], eip = rpi[P];   // e^{i phi_P}
                    double2 x[2][2];
                    const int rows2[2] = {p1, p2};
                    for (int a = 0; a < 2; ++a) {  // column rotation of Q on rows p1, p2
                        const int r = rows2[a];
                        const double2 xp = A[r * m + q1], xq = A[r * m + q2];
                        const double2 eq = make_double2(erq * xq.x - eiq * xq.y, erq * xq.y + eiq * xq.x);
                        x[a][0] = make_double2(cq * xp.x - sq * eq.x, cq * xp.y - sq * eq.y);
                        x[a][1] = make_double2(sq * xp.x + cq * eq.x, sq * xp.y + cq * eq.y);
                    }
                    const int cols2[2] = {q1, q2};
                    for (int b = 0; b < 2; ++b) {  // then the row rotation of P
                        const double2 xp = x[0][b], xq = x[1][b];
                        const double2 eq = make_double2(erp * xq.x - eip * xq.y, erp * xq.y + eip * xq.x);
                        A[p1 * m + cols2[b]] = make_double2(cp * xp.x - sp * eq.x, cp * xp.y - sp * eq.y);
                        A[p2 * m + cols2[b]] = make_double2(sp * xp.x + cp * eq.x, sp * xp.y + cp * eq.y);
                    }
                } else {
                    const int i2 = i - half * half;
                    const int k = i2 / m, r = i2 % m;
                    const int p = rp[k], q = rq[k];
                    const double c = rc[k], sn = rs[k], er = rpr[k], ei = -rpi[k];  // e^{-i phi}
                    const double2 xp = V[r * m + p], xq = V[r * m + q];
                    const double2 eq = make_double2(er * xq.x - ei * xq.y, er * xq.y + ei * xq.x);
                    V[r * m + p] = make_double2(c * xp.x - sn * eq.x, c * xp.y - sn * eq.y);
                    V[r * m + q] = make_double2(sn * xp.x + c * eq.x, sn * xp.y + c * eq.y);
                }
            }
            __syncthreads();
        }
    }
    // descending order by rank (ties broken by index)
    for (int i = tid; i < n; i += kJacobiThreads) {
        const double li = A[i * m + i].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j * m + j].x;
            rank += (lj > li) || (lj == li && j < i);
        }
        evals[rank] = li;
        for (int r = 0; r < n; ++r) {
            const double2 v = V[r * m + i];
            vecs[(int64_t)rank * n + r] = make_double2(v.x, -v.y);
        }
    }
    if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

__global__ void __launch_bounds__(kJacobiThreads) jacobi_eigh_kernel(const double2* G, int n, double* evals,
                                                                       double2* vecs, int* sweeps_out) {
    jacobi_eigh_body(G, n, evals, vecs, sweeps_out);
}

// One workgroup per matrix of the table.
__global__ void __launch_bounds__(kJacobiThreads) jacobi_eigh_batched_kernel(const JacobiProb* __restrict__ tab) {
    const JacobiProb p = tab[blockIdx.x];
    jacobi_eigh_body(p.G, p.n, p.evals, p.vecs, nullptr);
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

// One term of the Taylor series: b <- alpha (y - c b), F <- F + b.
__global__ void taylor_term_kernel(double2* b, const double2* y, double2* F, int64_t n, double ar, double ai,
                                   double c) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    const double2 yi = y[i], bi = b[i], fi = F[i];
    const double ur = yi.x - c * bi.x, ui = yi.y - c * bi.y;
    const double2 nb = make_double2(ar * ur - ai * ui, ar * ui + ai * ur);
    b[i] = nb;
    F[i] = make_double2(fi.x + nb.x, fi.y + nb.y);
}

// End of one scaling step: F <- eta F, b <- F.
__global__ void taylor_rescale_kernel(double2* F, double2* b, int64_t n, double er, double ei) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    const double2 f = F[i];
    const double2 g = make_double2(er * f.x - ei * f.y, er * f.y + ei * f.x);
    F[i] = g;
    b[i] = g;
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

// combine_kernel with the coefficients passed by value (no upload)
__global__ void combine_args_kernel(double2* out, const double2* V, int64_t vstride, int nv, CombineCoef coef,
                                    int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nv; ++j) {
        const double2 c = coef.c[j], v = V[j * vstride + i];
        re += c.x * v.x - c.y * v.y;
        im += c.x * v.y + c.y * v.x;
    }
    out[i] = make_double2(re, im);
}

__global__ void copy_idx_kernel(double2* dst, int64_t ldd, const int* dr, const int* dc, const double2* src,
                                int64_t lds, const int* sr, const int* sc, int nr, int nc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (k >= nc || i >= nr) return;
    const int64_t di = dr ? dr[i] : i, dk = dc ? dc[k] : k;
    const int64_t si = sr ? sr[i] : i, sk = sc ? sc[k] : k;
    dst[di * ldd + dk] = src[si * lds + sk];
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

// y[i] += x[i] for n complex entries of one dtype
__global__ void add_inplace_kernel(void* y, const void* x, int c128, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double yr, yi, xr, xi;
        ld<double>(y, c128, i, yr, yi);
        ld<double>(x, c128, i, xr, xi);
        st<double>(y, c128, i, yr + xr, yi + xi);
    }
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

// out[c] = squared 2-norm of vector c of P: row c (by_rows) or column c,
// each of len elements; one block per vector.
__global__ void vec_norms2_kernel(const double2* P, int64_t ld, int len, int by_rows, double* out) {
    __shared__ double red[kVecThreads];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < len; k += kVecThreads) {
        const double2 v = by_rows ? P[(int64_t)c * ld + k] : P[(int64_t)k * ld + c];
        acc += v.x * v.x + v.y * v.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kVecThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
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

// ------------------------------------------------- local operator on a site
// A[a][s'][b] <- sum_s O[s'][s] A[a][s][b]; one thread per (a, b).
constexpr int kApplyMaxD = 16;

__global__ void apply_site_kernel(double2* A, const double2* O, int chil, int d, int chir) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)chil * chir) return;
    const int64_t a = t / chir, b = t % chir;
    double2 x[kApplyMaxD];
    for (int s = 0; s < d; ++s) x[s] = A[(a * d + s) * chir + b];
    for (int sp = 0; sp < d; ++sp) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < d; ++s) {
            const double2 o = O[sp * d + s];
            re += o.x * x[s].x - o.y * x[s].y;
            im += o.x * x[s].y + o.y * x[s].x;
        }
        A[(a * d + sp) * chir + b] = make_double2(re, im);
    }
}

// --------------------------------------------- MPO stage operator (device)
// Entry M[row][col] of the dense operator of the sparse MPO stage, in FP64,
// from the MPO tensors (kind as in MopKind).  W1/W2 are either the device
// tensors (w1_128/w2_128 give their precision) or complex128 copies in LDS.
__device__ __forceinline__ double2 mop_entry(int kind, const void* W1, int w1_128, const void* W2, int w2_128,
                                             int wm, int wr, int d, int row, int col) {
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
    return make_double2(re, im);
}

__global__ void mop_dense_kernel(int kind, const void* W1, int w1_128, const void* W2, int w2_128,
                                 int wm, int wr, int d, int rows, int cols, double2* M) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    M[idx] = mop_entry(kind, W1, w1_128, W2, w2_128, wm, wr, d, idx / cols, idx % cols);
}

// The whole operator build in one block when it is small (the common case):
// the MPO tensors are copied to LDS in complex128, every thread computes up
// to kMopPerThread entries (kept in registers) and marks the non-zeros in an
// LDS bit mask, the row counts and their prefix sum follow from the mask,
// and each thread writes its non-zeros at their rank within the row, so the
// column order inside a row is ascending as in the two-kernel path.
constexpr int kMopThreads = 1024;
constexpr int kMopPerThread = 8;
constexpr int kMopMaxEntries = kMopThreads * kMopPerThread;
constexpr int kMopMaxRows = 2048;
constexpr int kMopLdsW = 2560;  // complex128 MPO entries staged (40 KiB)

// number of set bits of the LDS bit mask in positions [a, b)
__device__ __forceinline__ int mask_count(const unsigned* mask, int a, int b) {
    int c = 0;
    while (a < b) {
        const int w = a >> 5, lo = a & 31;
        const int hi = min(32, lo + (b - a));  // bits [lo, hi) of word w
        const unsigned m = (hi == 32 ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        c += __popc(mask[w] & m);
        a += hi - lo;
    }
    return c;
}

__global__ void __launch_bounds__(kMopThreads) mop_fused_kernel(int kind, const void* W1, int w1_128, int n1,
                                                                const void* W2, int w2_128, int n2, int wm, int wr,
                                                                int d, int rows, int cols, int* row_ptr, int* col,
                                                                void* val, int val128) {
    __shared__ double2 sw[kMopLdsW];
    __shared__ unsigned mask[kMopMaxEntries / 32];
    __shared__ int cnt[kMopMaxRows + 1];
    const int tid = threadIdx.x, tot = rows * cols;
    for (int i = tid; i < n1 + n2; i += kMopThreads) {
        double re, im;
        if (i < n1) ld<double>(W1, w1_128, i, re, im);
        else ld<double>(W2, w2_128, i - n1, re, im);
        sw[i] = make_double2(re, im);
    }
    for (int i = tid; i < kMopMaxEntries / 32; i += kMopThreads) mask[i] = 0u;
    __syncthreads();
    double2 v[kMopPerThread];
#pragma unroll
    for (int t = 0; t < kMopPerThread; ++t) {
        const int idx = tid + t * kMopThreads;
        v[t] = make_double2(0.0, 0.0);
        if (idx < tot) {
            v[t] = mop_entry(kind, sw, 1, sw + n1, 1, wm, wr, d, idx / cols, idx % cols);
            if (v[t].x != 0.0 || v[t].y != 0.0) atomicOr(&mask[idx >> 5], 1u << (idx & 31));
        }
    }
    __syncthreads();
    // row counts from the mask (rows may straddle 32-bit words)
    for (int r = tid; r < rows; r += kMopThreads) cnt[r + 1] = mask_count(mask, r * cols, (r + 1) * cols);
    __syncthreads();
    if (tid == 0) {
        cnt[0] = 0;
        for (int r = 0; r < rows; ++r) cnt[r + 1] += cnt[r];
    }
    __syncthreads();
    for (int r = tid; r <= rows; r += kMopThreads) row_ptr[r] = cnt[r];
#pragma unroll
    for (int t = 0; t < kMopPerThread; ++t) {
        const int idx = tid + t * kMopThreads;
        if (idx >= tot || !((mask[idx >> 5] >> (idx & 31)) & 1u)) continue;
        const int r = idx / cols, c0 = r * cols;
        const int e = cnt[r] + mask_count(mask, c0, idx);
        col[e] = idx - c0;
        st<double>(val, val128, e, v[t].x, v[t].y);
    }
}

// Dense operator -> CSR (exact zeros dropped), one block: row counts and
// their prefix sum in LDS, then the column indices and values per row.
__global__ void mop_csr_kernel(const double2* M, int rows, int cols, int* row_ptr, int* col,
                               void* val, int val128) {
    extern __shared__ int cnt[];  // rows + 1
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        int c = 0;
        for (int j = 0; j < cols; ++j) {
            const double2 v = M[(int64_t)r * cols + j];
            c += (v.x != 0.0 || v.y != 0.0);
        }
        cnt[r + 1] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt[0] = 0;
        for (int r = 0; r < rows; ++r) cnt[r + 1] += cnt[r];
    }
    __syncthreads();
    for (int r = threadIdx.x; r <= rows; r += blockDim.x) row_ptr[r] = cnt[r];
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        int e = cnt[r];
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
// partial sums of tr(X Y) for X [rows][cols], Y [cols][rows]
__global__ void trace_xyT_partial_kernel(const double2* X, const double2* Y, int rows, int cols, double2* partial) {
    __shared__ double sre[kVecThreads], sim[kVecThreads];
    double re = 0.0, im = 0.0;
    const int64_t nn = (int64_t)rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; t < nn;
         t += (int64_t)gridDim.x * kVecThreads) {
        const int64_t i = t / cols, j = t % cols;
        const double2 a = X[t], b = Y[j * rows + i];
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
    const int bpts = d.fp64 ? wpts<double>() : wpts<float>();  // points per block
    const size_t shmem = (size_t)bpts * w.nin * esz + (d.fp64 ? wstage_op_bytes<double>() : wstage_op_bytes<float>());
    TDVP_REQUIRE(shmem <= 160 * 1024, TDVP_E_SHAPE, "wstage: MPO bond dimension too large");
    TDVP_REQUIRE(d.P <= 65535, TDVP_E_SHAPE, "wstage: grid too large");
    const int nt = d.fp64 ? wthreads<double>() : wthreads<float>();
    dim3 grid((d.Q + bpts - 1) / bpts, d.P);
    const double pts = (double)d.P * d.Q;
    ProfScope prof(ctx, d.fp64 ? "wstage_f64" : "wstage_f32", 0.0,
                   pts * (w.nin * elem_bytes(d.in_dt) + w.nout * elem_bytes(d.out_dt)));
    if (d.fp64) hipLaunchKernelGGL(wstage_kernel<double>, grid, dim3(nt), shmem, s, w);
    else hipLaunchKernelGGL(wstage_kernel<float>, grid, dim3(nt), shmem, s, w);
    TDVP_CHECK_HIP(hipGetLastError());
}

void grouped_wstage_plan(tdvp_ctx ctx, const std::vector<WStageDesc>& ds, GroupedWStage& out, const char* table_ws) {
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
    const int nt = out.fp64 ? wpts<double>() : wpts<float>();  // points per block
    out.nt = out.fp64 ? wthreads<double>() : wthreads<float>();
    out.shmem = (size_t)nt * nin_max * esz + (out.fp64 ? wstage_op_bytes<double>() : wstage_op_bytes<float>());
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
    const size_t tb = sizeof(GWProblem) * std::max<size_t>(1, tab.size());
    void* dst;
    if (table_ws) {
        dst = ctx->workspace(table_ws, tb);
    } else {
        if (out.probs.bytes < tb) out.probs = DevMem(ctx, tb);
        dst = out.probs.ptr;
    }
    out.table = dst;
    if (!tab.empty()) ctx->upload(dst, tab.data(), sizeof(GWProblem) * tab.size());
}

void grouped_wstage_run(tdvp_ctx ctx, const GroupedWStage& g) {
    if (g.nprob == 0 || g.blocks == 0) return;
    ProfScope prof(ctx, g.fp64 ? "wstage_grouped_f64" : "wstage_grouped_f32", 0.0, g.bytes);
    const auto* pr = static_cast<const GWProblem*>(g.table);
    if (g.fp64)
        hipLaunchKernelGGL(wstage_grouped_kernel<double>, dim3((unsigned)g.blocks), dim3(g.nt), g.shmem, ctx->stream,
                           pr, g.nprob);
    else
        hipLaunchKernelGGL(wstage_grouped_kernel<float>, dim3((unsigned)g.blocks), dim3(g.nt), g.shmem, ctx->stream,
                           pr, g.nprob);
    TDVP_CHECK_HIP(hipGetLastError());
}

namespace {
constexpr size_t kHsSmemCap = 150 * 1024;

// x rows per stage-A chunk: all of x when the LDS holds it, else kHsRows
int heff_small_rows(int chil, int chir, int D, int wl, int wr, bool fp64) {
    auto bytes = [&](int rows) {
        return fp64 ? heff_small_smem<double>(chil, chir, D, wl, wr, rows)
                    : heff_small_smem<float>(chil, chir, D, wl, wr, rows);
    };
    if (bytes(chil) <= kHsSmemCap) return chil;
    return bytes(std::min(kHsRows, chil)) <= kHsSmemCap ? std::min(kHsRows, chil) : 0;
}
}  // namespace

bool heff_small_fits(int chil, int chir, int D, int wl, int wr, bool fp64) {
    if (chil < 1 || chir < 1 || chil > kHeffSmallChi || chir > kHeffSmallChi || wl < 1 || wr < 1) return false;
    if (D < 1 || D > 65535) return false;
    return heff_small_rows(chil, chir, D, wl, wr, fp64) > 0;
}

void heff_small(tdvp_ctx ctx, const HeffSmallDesc& d) {
    TDVP_REQUIRE(heff_small_fits(d.chil, d.chir, d.D, d.wl, d.wr, d.fp64), TDVP_E_SHAPE,
                 "heff_small: shape outside the fused kernel's limits");
    TDVP_REQUIRE((d.L_dt == Dt::C128) == d.fp64 && (d.R_dt == Dt::C128) == d.fp64, TDVP_E_ARG,
                 "heff_small: environments must be in the compute precision");
    HsParams h;
    h.L = d.L; h.L128 = d.L_dt == Dt::C128;
    h.R = d.R; h.R128 = d.R_dt == Dt::C128;
    h.x = d.x; h.x128 = d.x_dt == Dt::C128;
    h.y = d.y; h.y128 = d.y_dt == Dt::C128;
    h.row_ptr = d.row_ptr;
    h.col = d.col;
    h.val = d.val;
    h.chil = d.chil; h.chir = d.chir; h.D = d.D; h.wl = d.wl; h.wr = d.wr;
    h.rows = heff_small_rows(d.chil, d.chir, d.D, d.wl, d.wr, d.fp64);
    const size_t shmem = d.fp64 ? heff_small_smem<double>(d.chil, d.chir, d.D, d.wl, d.wr, h.rows)
                                : heff_small_smem<float>(d.chil, d.chir, d.D, d.wl, d.wr, h.rows);
    const double nc = (double)d.D * d.chir;
    ProfScope prof(ctx, d.fp64 ? "heff_small_f64" : "heff_small_f32", d.flops,
                   elem_bytes(d.x_dt) * d.chil * nc + elem_bytes(d.y_dt) * d.chil * nc +
                       elem_bytes(d.L_dt) * (double)d.wl * d.chil * d.chil + elem_bytes(d.R_dt) * (double)d.wr * d.chir * d.chir);
    const dim3 grid(d.chil, d.D);
    const bool x128 = d.x_dt == Dt::C128;
    if (d.fp64) {
        if (x128) hipLaunchKernelGGL((heff_small_kernel<double, double2>), grid, dim3(kHsThreads), shmem, ctx->stream, h);
        else hipLaunchKernelGGL((heff_small_kernel<double, float2>), grid, dim3(kHsThreads), shmem, ctx->stream, h);
    } else {
        if (x128) hipLaunchKernelGGL((heff_small_kernel<float, double2>), grid, dim3(kHsThreads), shmem, ctx->stream, h);
        else hipLaunchKernelGGL((heff_small_kernel<float, float2>), grid, dim3(kHsThreads), shmem, ctx->stream, h);
    }
    TDVP_CHECK_HIP(hipGetLastError());
}

void lanczos_small_step(double2* V, int64_t n, int k, double2* w, double beta_prev, const double* nn_prev,
                        double* out, hipStream_t s) {
    TDVP_REQUIRE(n <= kSmallLanczos && k < kSmallMaxK, TDVP_E_ARG, "lanczos_small_step: vector or basis too large");
    hipLaunchKernelGGL(lanczos_small_kernel, dim3(1), dim3(kSmallThreads), 0, s, V, n, k, w, beta_prev, nn_prev, out);
    TDVP_CHECK_HIP(hipGetLastError());
}

void small_normalize(const double2* x, double2* v, int64_t n, double* nn, hipStream_t s) {
    TDVP_REQUIRE(n <= kSmallLanczos, TDVP_E_ARG, "small_normalize: vector too long");
    hipLaunchKernelGGL(small_normalize_kernel, dim3(1), dim3(kSmallThreads), 0, s, x, v, n, nn);
    TDVP_CHECK_HIP(hipGetLastError());
}

bool qr_small_fits(int m, int n) { return n >= 1 && m >= n && n <= kQrMaxCols && (int64_t)m * n <= kQrMaxElems; }

void qr_small(const double2* M, int m, int n, bool herm, double2* Q, double2* RL, hipStream_t s) {
    TDVP_REQUIRE(qr_small_fits(m, n), TDVP_E_SHAPE, "qr_small: matrix does not fit one workgroup");
    hipLaunchKernelGGL(qr_small_kernel, dim3(1), dim3(kQrThreads), 0, s, M, m, n, herm ? 1 : 0, Q, RL);
    TDVP_CHECK_HIP(hipGetLastError());
}

void jacobi_eigh_batched(tdvp_ctx ctx, const std::vector<JacobiProb>& probs) {
    if (probs.empty()) return;
    for (const auto& p : probs)
        TDVP_REQUIRE(p.n >= 1 && p.n <= kJacobiMax && p.G && p.evals && p.vecs, TDVP_E_ARG,
                     "jacobi_eigh_batched: order out of range or null pointer");
    auto* tab = static_cast<JacobiProb*>(ctx->workspace("jacobi_tab", sizeof(JacobiProb) * probs.size()));
    ctx->upload(tab, probs.data(), sizeof(JacobiProb) * probs.size());
    hipLaunchKernelGGL(jacobi_eigh_batched_kernel, dim3((unsigned)probs.size()), dim3(kJacobiThreads), 0, ctx->stream,
                       tab);
    TDVP_CHECK_HIP(hipGetLastError());
}

void jacobi_eigh_small(const double2* G, int n, double* evals, double2* vecs, int* sweeps, hipStream_t s) {
    TDVP_REQUIRE(n >= 1 && n <= kJacobiMax, TDVP_E_ARG, "jacobi_eigh_small: order out of range");
    hipLaunchKernelGGL(jacobi_eigh_kernel, dim3(1), dim3(kJacobiThreads), 0, s, G, n, evals, vecs, sweeps);
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

void taylor_term(double2* b, const double2* y, double2* F, int64_t n, double2 alpha, double c, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(taylor_term_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, b, y, F, n, alpha.x, alpha.y, c);
    TDVP_CHECK_HIP(hipGetLastError());
}

void taylor_rescale(double2* F, double2* b, int64_t n, double2 eta, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(taylor_rescale_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, F, b, n, eta.x, eta.y);
    TDVP_CHECK_HIP(hipGetLastError());
}

void combine(double2* out, const double2* V, int64_t vstride, int nv, const double2* coef,
             int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(combine_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, out, V, vstride, nv,
                       coef, n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void combine_args(double2* out, const double2* V, int64_t vstride, int nv, const double2* coef_host, int64_t n,
                  hipStream_t s) {
    TDVP_REQUIRE(nv <= kCombineArgs, TDVP_E_ARG, "combine_args: too many vectors");
    if (n == 0) return;
    CombineCoef c{};
    for (int j = 0; j < nv; ++j) c.c[j] = coef_host[j];
    hipLaunchKernelGGL(combine_args_kernel, dim3(nblk(n)), dim3(kVecThreads), 0, s, out, V, vstride, nv, c, n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void copy_idx(double2* dst, int64_t ldd, const int* dr, const int* dc, const double2* src, int64_t lds,
              const int* sr, const int* sc, int nr, int nc, hipStream_t s) {
    if (nr == 0 || nc == 0) return;
    TDVP_REQUIRE(nr <= 65535, TDVP_E_SHAPE, "copy_idx: too many rows");
    dim3 grid((nc + 127) / 128, nr);
    hipLaunchKernelGGL(copy_idx_kernel, grid, dim3(128), 0, s, dst, ldd, dr, dc, src, lds, sr, sc, nr, nc);
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

void vec_norms2(const double2* P, int64_t ld, int count, int len, bool by_rows, double* out, hipStream_t s) {
    if (count == 0) return;
    TDVP_REQUIRE(count > 0 && len >= 0, TDVP_E_ARG, "vec_norms2: negative size");
    hipLaunchKernelGGL(vec_norms2_kernel, dim3(count), dim3(kVecThreads), 0, s, P, ld, len, (int)by_rows, out);
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
    // element counts of the tensors the entries read (kinds 0, 1, 3, 4 read W1 only)
    const int n1 = kind == 0 ? 0 : (kind == 2 || kind == 5 || kind == 6) ? wl * wm * d * d : wl * wr * d * d;
    const int n2 = (kind == 2 || kind == 5 || kind == 6) ? wm * wr * d * d : 0;
    if (tot <= kMopMaxEntries && rows <= kMopMaxRows && n1 + n2 <= kMopLdsW) {
        hipLaunchKernelGGL(mop_fused_kernel, dim3(1), dim3(kMopThreads), 0, s, kind, W1, (int)(w1dt == Dt::C128), n1,
                           W2, (int)(w2dt == Dt::C128), n2, wm, wr, d, rows, cols, row_ptr, col, val,
                           (int)val_fp64);
        TDVP_CHECK_HIP(hipGetLastError());
        return;
    }
    TDVP_REQUIRE((size_t)(rows + 1) * sizeof(int) <= 64 * 1024, TDVP_E_SHAPE, "MPO stage operator: too many rows");
    hipLaunchKernelGGL(mop_dense_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, kind, W1,
                       (int)(w1dt == Dt::C128), W2, (int)(w2dt == Dt::C128), wm, wr, d, rows,
                       cols, dense);
    hipLaunchKernelGGL(mop_csr_kernel, dim3(1), dim3(256), sizeof(int) * (rows + 1), s, dense, rows, cols, row_ptr,
                       col, val, (int)val_fp64);
    TDVP_CHECK_HIP(hipGetLastError());
}

void conj_transpose_batched(void* out, const void* in, Dt dt, int n, int batch, hipStream_t s) {
    if (n == 0 || batch == 0) return;
    TDVP_REQUIRE(n <= 65535 && batch <= 65535, TDVP_E_SHAPE, "conj_transpose_batched: too large");
    dim3 grid((n + 127) / 128, n, batch);
    hipLaunchKernelGGL(conj_transpose_batched_kernel, grid, dim3(128), 0, s, out, in, (int)(dt == Dt::C128), n);
    TDVP_CHECK_HIP(hipGetLastError());
}

void add_inplace(void* y, const void* x, Dt dt, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(add_inplace_kernel, dim3(blocks), dim3(256), 0, s, y, x, (int)(dt == Dt::C128), n);
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

void apply_site(double2* A, const double2* O, int chil, int d, int chir, hipStream_t s) {
    TDVP_REQUIRE(d >= 1 && d <= kApplyMaxD, TDVP_E_ARG, "apply_site: local dimension out of range");
    const int64_t n = (int64_t)chil * chir;
    if (n == 0) return;
    hipLaunchKernelGGL(apply_site_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, O, chil, d, chir);
    TDVP_CHECK_HIP(hipGetLastError());
}

void trace_xyT(tdvp_ctx ctx, const double2* X, const double2* Y, int n, double2* out) {
    trace_xy(ctx, X, Y, n, n, out);
}

void trace_xy(tdvp_ctx ctx, const double2* X, const double2* Y, int rows, int cols, double2* out) {
    double2* partial = static_cast<double2*>(ctx->workspace("trace_partial", sizeof(double2) * kDotBlocks));
    const int64_t nn = (int64_t)rows * cols;
    int nb = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (nn + kVecThreads - 1) / kVecThreads));
    hipLaunchKernelGGL(trace_xyT_partial_kernel, dim3(nb), dim3(kVecThreads), 0, ctx->stream, X, Y, rows, cols,
                       partial);
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(1), dim3(kVecThreads), 0, ctx->stream, partial, nb, out);
    TDVP_CHECK_HIP(hipGetLastError());
}

}  // namespace tdvp
