// Complex GEMM on CDNA4 matrix cores.
//
// Every large contraction of the TDVP path (the L.Theta and T3.R stages of
// the effective Hamiltonian, Sec. III A and Eq. eqnscaling; the environment
// updates; forming two-site states) is a complex matrix product.  The
// kernel computes C = op(A) op(B) from real MFMA instructions:
//
//   4M form: Cr = Ar Br - Ai Bi,  Ci = Ar Bi + Ai Br           (4 products)
//   3M form: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
//            Cr = P1 - P2,  Ci = P3 - P1 - P2                  (3 products)
//
// FP32 uses v_mfma_f32_32x32x2f32, FP64 uses v_mfma_f64_16x16x4f64; both
// accumulate in the instruction's own precision.  Tiles are staged through
// LDS as separate real / imaginary / (sum or negated-imaginary) planes,
// stored [outer][k] so that every lane reads its k-slice with one 16-byte
// LDS load.  The k index inside a tile is permuted (lane group g handles
// k = g*S + s for instruction step s): the sum over k is order-free, so A
// and B only have to agree on the permutation.  Two LDS buffers with a
// register prefetch of the next tile give one barrier per k-tile.
//
// Inputs may be complex64 or complex128 in either precision (converted while
// staging), optionally conjugated, with k or the outer index contiguous in
// memory; output may be complex64 or complex128.  Ragged edges are handled
// by zero-filled staging and guarded stores.
#include "common.hpp"

#include <cstdio>

namespace tdvp {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;

template <> struct Mfma<float> {
    static constexpr int MT = 32;  // output tile edge
    static constexpr int KT = 2;   // k consumed per instruction
    static constexpr int NACC = 16;
    using acc_t = f32x16;
    __device__ static inline acc_t mma(float a, float b, const acc_t& c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    // A[i][k] comes from lane i + 32k, B[k][j] from lane j + 32k;
    // D[i][j] sits in lane j + 32*((i/4)%2), register (i%4) + 4*(i/8).
    __device__ static inline int row(int lane, int v) { return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); }
    __device__ static inline int col(int lane) { return lane & 31; }
};

template <> struct Mfma<double> {
    static constexpr int MT = 16;
    static constexpr int KT = 4;
    static constexpr int NACC = 4;
    using acc_t = f64x4;
    __device__ static inline acc_t mma(double a, double b, const acc_t& c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // A[i][k] from lane i + 16k, B[k][j] from lane j + 16k;
    // D[i][j] in lane j + 16*(i%4), register i/4 (checked on gfx950).
    __device__ static inline int row(int lane, int v) { return v * 4 + (lane >> 4); }
    __device__ static inline int col(int lane) { return lane & 15; }
};

struct KOperand {
    const void* p;
    int64_t ld, stride;
    int c128, kcontig, conj;
};

struct KParams {
    int M, N, K;
    int tiles_m, tiles_n;
    KOperand A, B;
    void* C;
    int c128C;
    int64_t ldc, strideC;
};

template <typename T>
__device__ inline void load_elem(const KOperand& o, int64_t idx, bool valid, T& re, T& im) {
    re = T(0);
    im = T(0);
    if (valid) {
        if (o.c128) {
            double2 v = reinterpret_cast<const double2*>(o.p)[idx];
            re = static_cast<T>(v.x);
            im = static_cast<T>(v.y);
        } else {
            float2 v = reinterpret_cast<const float2*>(o.p)[idx];
            re = static_cast<T>(v.x);
            im = static_cast<T>(v.y);
        }
        if (o.conj) im = -im;
    }
}

template <typename T, int WTM, int WTN, int BK, bool M3>
__global__ void __launch_bounds__(256, 1) cgemm_kernel(KParams p) {
    using F = Mfma<T>;
    using acc_t = typename F::acc_t;
    constexpr int MT = F::MT;
    constexpr int BM = 2 * WTM * MT;
    constexpr int BN = 2 * WTN * MT;
    constexpr int S = BK / F::KT;               // instruction steps per k-tile
    constexpr int LD = BK + (sizeof(T) == 4 ? 4 : 2);
    constexpr int AE = BM * BK / 256;           // staged A elements per thread
    constexpr int BE = BN * BK / 256;
    constexpr int NA = M3 ? 3 : 2;              // accumulators per output tile
    static_assert(AE * 256 == BM * BK && BE * 256 == BN * BK, "tile/thread mismatch");

    __shared__ __align__(16) T sA[2][3][BM * LD];
    __shared__ __align__(16) T sB[2][3][BN * LD];

    // Block -> tile.  Consecutive tiles walk down M for a fixed N panel, and
    // the hardware's round-robin dispatch over the 8 XCDs is undone so that
    // one XCD gets a contiguous run of tiles (shared panels stay in its L2).
    const int ntiles = p.tiles_m * p.tiles_n;
    int t = blockIdx.x;
    if ((ntiles & 7) == 0) t = (t & 7) * (ntiles >> 3) + (t >> 3);
    const int m0 = (t % p.tiles_m) * BM;
    const int n0 = (t / p.tiles_m) * BN;
    const int z = blockIdx.z;
    const int64_t zA = (int64_t)z * p.A.stride;
    const int64_t zB = (int64_t)z * p.B.stride;
    const int64_t zC = (int64_t)z * p.strideC;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1;
    const int wn = wave & 1;
    const int g = lane / MT;  // k group of this lane
    const int r = lane % MT;  // row (A) / column (B) of this lane

    T ar[AE], ai[AE], br[BE], bi[BE];

    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < AE; ++i) {
            const int e = tid + 256 * i;
            int o, k;
            if (p.A.kcontig) { o = e / BK; k = e % BK; } else { k = e / BM; o = e % BM; }
            const int gm = m0 + o, gk = k0 + k;
            const int64_t idx = p.A.kcontig ? (int64_t)gm * p.A.ld + gk : (int64_t)gk * p.A.ld + gm;
            load_elem<T>(p.A, zA + idx, gm < p.M && gk < p.K, ar[i], ai[i]);
        }
#pragma unroll
        for (int i = 0; i < BE; ++i) {
            const int e = tid + 256 * i;
            int o, k;
            if (p.B.kcontig) { o = e / BK; k = e % BK; } else { k = e / BN; o = e % BN; }
            const int gn = n0 + o, gk = k0 + k;
            const int64_t idx = p.B.kcontig ? (int64_t)gn * p.B.ld + gk : (int64_t)gk * p.B.ld + gn;
            load_elem<T>(p.B, zB + idx, gn < p.N && gk < p.K, br[i], bi[i]);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < AE; ++i) {
            const int e = tid + 256 * i;
            int o, k;
            if (p.A.kcontig) { o = e / BK; k = e % BK; } else { k = e / BM; o = e % BM; }
            sA[buf][0][o * LD + k] = ar[i];
            sA[buf][1][o * LD + k] = ai[i];
            sA[buf][2][o * LD + k] = M3 ? ar[i] + ai[i] : -ai[i];
        }
#pragma unroll
        for (int i = 0; i < BE; ++i) {
            const int e = tid + 256 * i;
            int o, k;
            if (p.B.kcontig) { o = e / BK; k = e % BK; } else { k = e / BN; o = e % BN; }
            sB[buf][0][o * LD + k] = br[i];
            sB[buf][1][o * LD + k] = bi[i];
            if (M3) sB[buf][2][o * LD + k] = br[i] + bi[i];
        }
    };

    acc_t acc[NA][WTM][WTN];
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
        for (int mi = 0; mi < WTM; ++mi)
#pragma unroll
            for (int ni = 0; ni < WTN; ++ni)
#pragma unroll
                for (int v = 0; v < F::NACC; ++v) acc[q][mi][ni][v] = T(0);

    const int nk = (p.K + BK - 1) / BK;
    if (nk > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);

        T fa[3][WTM][S], fb[3][WTN][S];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
#pragma unroll
            for (int mi = 0; mi < WTM; ++mi) {
                const int base = (wm * WTM * MT + mi * MT + r) * LD + g * S;
#pragma unroll
                for (int s = 0; s < S; ++s) fa[q][mi][s] = sA[cur][q][base + s];
            }
            if (q < 2 || M3) {
#pragma unroll
                for (int ni = 0; ni < WTN; ++ni) {
                    const int base = (wn * WTN * MT + ni * MT + r) * LD + g * S;
#pragma unroll
                    for (int s = 0; s < S; ++s) fb[q][ni][s] = sB[cur][q][base + s];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int mi = 0; mi < WTM; ++mi) {
#pragma unroll
                for (int ni = 0; ni < WTN; ++ni) {
                    if constexpr (M3) {
                        acc[0][mi][ni] = F::mma(fa[0][mi][s], fb[0][ni][s], acc[0][mi][ni]);
                        acc[1][mi][ni] = F::mma(fa[1][mi][s], fb[1][ni][s], acc[1][mi][ni]);
                        acc[2][mi][ni] = F::mma(fa[2][mi][s], fb[2][ni][s], acc[2][mi][ni]);
                    } else {
                        acc[0][mi][ni] = F::mma(fa[0][mi][s], fb[0][ni][s], acc[0][mi][ni]);
                        acc[0][mi][ni] = F::mma(fa[2][mi][s], fb[1][ni][s], acc[0][mi][ni]);
                        acc[1][mi][ni] = F::mma(fa[0][mi][s], fb[1][ni][s], acc[1][mi][ni]);
                        acc[1][mi][ni] = F::mma(fa[1][mi][s], fb[0][ni][s], acc[1][mi][ni]);
                    }
                }
            }
        }
        if (kt + 1 < nk) lstore(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int mi = 0; mi < WTM; ++mi) {
#pragma unroll
        for (int ni = 0; ni < WTN; ++ni) {
#pragma unroll
            for (int v = 0; v < F::NACC; ++v) {
                const int gm = m0 + wm * WTM * MT + mi * MT + F::row(lane, v);
                const int gn = n0 + wn * WTN * MT + ni * MT + F::col(lane);
                if (gm < p.M && gn < p.N) {
                    T cr, ci;
                    if constexpr (M3) {
                        const T p1 = acc[0][mi][ni][v], p2 = acc[1][mi][ni][v];
                        cr = p1 - p2;
                        ci = acc[2][mi][ni][v] - p1 - p2;
                    } else {
                        cr = acc[0][mi][ni][v];
                        ci = acc[1][mi][ni][v];
                    }
                    const int64_t idx = zC + (int64_t)gm * p.ldc + gn;
                    if (p.c128C)
                        reinterpret_cast<double2*>(p.C)[idx] = make_double2((double)cr, (double)ci);
                    else
                        reinterpret_cast<float2*>(p.C)[idx] = make_float2((float)cr, (float)ci);
                }
            }
        }
    }
}

KOperand to_k(const GemmOperand& o) {
    KOperand k;
    k.p = o.p;
    k.ld = o.ld;
    k.stride = o.stride;
    k.c128 = o.dt == Dt::C128;
    k.kcontig = o.kcontig;
    k.conj = o.conj;
    return k;
}

template <typename T, int WTM, int WTN, int BK, bool M3>
void launch(tdvp_ctx ctx, KParams kp, int batch) {
    constexpr int MT = Mfma<T>::MT;
    constexpr int BM = 2 * WTM * MT, BN = 2 * WTN * MT;
    kp.tiles_m = (kp.M + BM - 1) / BM;
    kp.tiles_n = (kp.N + BN - 1) / BN;
    dim3 grid(kp.tiles_m * kp.tiles_n, 1, batch);
    char name[64];
    snprintf(name, sizeof(name), "cgemm_%s_%s_%dx%d", sizeof(T) == 4 ? "f32" : "f64", M3 ? "3m" : "4m", BM, BN);
    const double flops = 8.0 * kp.M * (double)kp.N * kp.K * batch;
    const double bytes = (double)batch * ((double)kp.M * kp.K * (kp.A.c128 ? 16 : 8) * (kp.A.stride ? 1 : 1.0 / batch) +
                                          (double)kp.K * kp.N * (kp.B.c128 ? 16 : 8) * (kp.B.stride ? 1 : 1.0 / batch) +
                                          (double)kp.M * kp.N * (kp.c128C ? 16 : 8));
    ProfScope prof(ctx, name, flops, bytes);
    hipLaunchKernelGGL((cgemm_kernel<T, WTM, WTN, BK, M3>), grid, dim3(256), 0, ctx->stream, kp);
    TDVP_CHECK_HIP(hipGetLastError());
}

}  // namespace

void cgemm(tdvp_ctx ctx, const GemmDesc& g, bool fp64, int form) {
    TDVP_REQUIRE(g.M >= 0 && g.N >= 0 && g.K >= 0 && g.batch >= 1, TDVP_E_SHAPE, "cgemm: bad sizes");
    TDVP_REQUIRE(g.batch <= 65535, TDVP_E_SHAPE, "cgemm: batch too large");
    if (g.M == 0 || g.N == 0) return;
    TDVP_REQUIRE(g.A.p && g.B.p && g.C, TDVP_E_ARG, "cgemm: null operand");
    KParams kp{};
    kp.M = g.M;
    kp.N = g.N;
    kp.K = g.K;
    kp.A = to_k(g.A);
    kp.B = to_k(g.B);
    kp.C = g.C;
    kp.c128C = g.cdt == Dt::C128;
    kp.ldc = g.ldc;
    kp.strideC = g.strideC;
    const bool m3 = form == 3;
    if (fp64) {
        const int64_t big_tiles = ((g.M + 127) / 128) * (int64_t)((g.N + 63) / 64) * g.batch;
        if (big_tiles >= 512) {
            if (m3) launch<double, 4, 2, 8, true>(ctx, kp, g.batch);
            else launch<double, 4, 2, 8, false>(ctx, kp, g.batch);
        } else {
            if (m3) launch<double, 2, 1, 8, true>(ctx, kp, g.batch);
            else launch<double, 2, 1, 8, false>(ctx, kp, g.batch);
        }
    } else {
        const int64_t big_tiles = ((g.M + 127) / 128) * (int64_t)((g.N + 127) / 128) * g.batch;
        if (big_tiles >= 512) {
            if (m3) launch<float, 2, 2, 16, true>(ctx, kp, g.batch);
            else launch<float, 2, 2, 16, false>(ctx, kp, g.batch);
        } else {
            if (m3) launch<float, 1, 1, 16, true>(ctx, kp, g.batch);
            else launch<float, 1, 1, 16, false>(ctx, kp, g.batch);
        }
    }
}

}  // namespace tdvp
