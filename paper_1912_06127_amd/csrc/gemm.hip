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
// and B only have to agree on the permutation.  Two LDS buffers give one
// barrier per k-tile; the global loads run two k-tiles ahead of the MFMAs
// (two register sets) in the single-problem kernel and one ahead in the
// grouped kernel, whose many small products measured faster that way.  Output tiles go to the XCDs in contiguous ranges,
// and inside a range runs of kGroupM m-tiles sweep the n-tiles, so the tiles
// an XCD holds at one time share rows of A and columns of B in its L2.
//
// Inputs may be complex64 or complex128 in either precision (converted while
// staging), optionally conjugated, with k or the outer index contiguous in
// memory; output may be complex64 or complex128.  Ragged edges are handled
// by zero-filled staging and guarded stores.
#include "common.hpp"

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <tuple>
#include <type_traits>

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
    int ksplit, kchunk;  // split-K: blockIdx.z = batch * ksplit + split
    KOperand A, B;
    void* C;
    int c128C;
    int64_t ldc, strideC;
};

// Element idx of an operand as stored (re, im), without the validity and
// conjugation fix-up (applied where the value goes to LDS).  Branch-free: an
// invalid element reads element `base` (the operand's first element, which
// exists whenever the product is non-empty), so the loads of a staging pass
// issue back to back and are only waited for where the values are stored
// (a load under a branch, or a select right after it, makes the compiler
// wait for it at once).  NATIVE: the operand is stored in the compute
// precision (the common case, chosen once per tile outside the k loop);
// otherwise its precision is read from the descriptor at run time.
template <typename T, bool NATIVE>
__device__ inline void load_raw(const KOperand& o, int64_t base, int64_t idx, bool valid, T& re, T& im) {
    const int64_t at = valid ? idx : base;
    if constexpr (NATIVE) {
        using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
        const V2 v = reinterpret_cast<const V2*>(o.p)[at];
        re = v.x;
        im = v.y;
    } else if (o.c128) {
        const double2 v = reinterpret_cast<const double2*>(o.p)[at];
        re = static_cast<T>(v.x);
        im = static_cast<T>(v.y);
    } else {
        const float2 v = reinterpret_cast<const float2*>(o.p)[at];
        re = static_cast<T>(v.x);
        im = static_cast<T>(v.y);
    }
}

// Operands stored in the compute precision (complex64 for T = float,
// complex128 for T = double).
template <typename T>
__device__ inline bool native_operands(const KParams& p) {
    return sizeof(T) == 4 ? (!p.A.c128 && !p.B.c128) : (p.A.c128 && p.B.c128);
}

// Second-generation tile: two LDS planes (re, im) per operand, the third 3M
// operand (re + im) or the negated imaginary part (4M) formed in registers;
// the LDS layout follows the operand's memory order so that staging stores
// are conflict-free: k-contiguous operands are stored [outer][k] (each lane
// reads its k-slice with vector loads), outer-contiguous operands [k][outer]
// (consecutive lanes read consecutive outer indices).
template <typename T, int BM, int BN, int BK, bool AK, bool BKC>
struct TileSmem {
    static constexpr int PADK = sizeof(T) == 4 ? 4 : 2;
    static constexpr int SA = AK ? BM * (BK + PADK) : BK * (BM + PADK);
    static constexpr int SB = BKC ? BN * (BK + PADK) : BK * (BN + PADK);
    T a[2][2][SA];
    T b[2][2][SB];
};

// Accumulators of one output tile: NA planes (3M: P1, P2, P3; 4M: re, im)
// of TM x TN MFMA tiles per wave.
template <typename T, int BM, int BN, int WM, int WN, bool M3>
struct TileAcc {
    using F = Mfma<T>;
    static constexpr int TM = BM / (WM * F::MT);
    static constexpr int TN = BN / (WN * F::MT);
    static constexpr int NA = M3 ? 3 : 2;
    typename F::acc_t v[NA][TM][TN];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int q = 0; q < NA; ++q)
#pragma unroll
            for (int mi = 0; mi < TM; ++mi)
#pragma unroll
                for (int ni = 0; ni < TN; ++ni)
#pragma unroll
                    for (int e = 0; e < F::NACC; ++e) v[q][mi][ni][e] = T(0);
    }
};

// Accumulates the products of output tile (m0, n0) over k in [kbeg, kend)
// (operands offset by zA, zB elements) into acc.
// PF: k-tiles the global loads run ahead of the MFMAs (1 or 2).
template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3, bool AK, bool BKC, int PF, bool NATIVE>
__device__ __forceinline__ void gemm_tile_acc(const KParams& p, TileSmem<T, BM, BN, BK, AK, BKC>& sm, int m0, int n0,
                                              int64_t zA, int64_t zB, int kbeg, int kend,
                                              TileAcc<T, BM, BN, WM, WN, M3>& accs) {
    using F = Mfma<T>;
    using acc_t = typename F::acc_t;
    constexpr int NT = 64 * WM * WN;
    constexpr int MT = F::MT;
    constexpr int TM = BM / (WM * MT);  // MFMA tiles per wave along M
    constexpr int TN = BN / (WN * MT);
    static_assert(TM * WM * MT == BM && TN * WN * MT == BN, "tile shape");
    constexpr int S = BK / F::KT;
    constexpr int PADK = sizeof(T) == 4 ? 4 : 2;
    constexpr int LDAk = BK + PADK;       // [outer][k] row stride
    constexpr int LDAo = BM + PADK;       // [k][outer] row stride
    constexpr int LDBo = BN + PADK;
    constexpr int SA = AK ? BM * LDAk : BK * LDAo;
    constexpr int SB = BKC ? BN * LDAk : BK * LDBo;
    constexpr int AE = BM * BK / NT;
    constexpr int BE = BN * BK / NT;
    static_assert(AE * NT == BM * BK && BE * NT == BN * BK, "tile/thread mismatch");
    static_assert(AE % 2 == 0 && BE % 2 == 0, "pairwise staging");
    constexpr int NA = M3 ? 3 : 2;
    static_assert(SA == TileSmem<T, BM, BN, BK, AK, BKC>::SA && SB == TileSmem<T, BM, BN, BK, AK, BKC>::SB, "smem");
    auto& sA = sm.a;
    auto& sB = sm.b;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int g = lane / MT;
    const int r = lane % MT;

    // PF register sets: with two, the tile two steps ahead is fetched while
    // the next one is written to LDS
    static_assert(PF == 1 || PF == 2, "prefetch distance");
    T ar[PF][AE], ai[PF][AE], br[PF][BE], bi[PF][BE];
    static_assert(AE <= 32 && BE <= 32, "validity masks");
    unsigned am[PF], bm[PF];  // bit i: element i of the staged set is inside the operand
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;

    auto gload = [&](int k0, auto setc) {
        constexpr int SET = decltype(setc)::value;
        am[SET] = 0u;
        bm[SET] = 0u;
#pragma unroll
        for (int i = 0; i < AE / 2; ++i) {  // pairs along the contiguous index
            const int e = 2 * (tid + NT * i);
            const int o = AK ? e / BK : e % BM;
            const int k = AK ? e % BK : e / BM;
            const int gm = m0 + o, gk = k0 + k;
            const int64_t idx = AK ? (int64_t)gm * p.A.ld + gk : (int64_t)gk * p.A.ld + gm;
            const bool v0 = gm < p.M && gk < kend;
            const bool v1 = AK ? (gm < p.M && gk + 1 < kend) : (gm + 1 < p.M && gk < kend);
            load_raw<T, NATIVE>(p.A, zA, zA + idx, v0, ar[SET][2 * i], ai[SET][2 * i]);
            load_raw<T, NATIVE>(p.A, zA, zA + idx + 1, v1, ar[SET][2 * i + 1], ai[SET][2 * i + 1]);
            am[SET] |= (v0 ? 1u : 0u) << (2 * i) | (v1 ? 1u : 0u) << (2 * i + 1);
        }
#pragma unroll
        for (int i = 0; i < BE / 2; ++i) {
            const int e = 2 * (tid + NT * i);
            const int o = BKC ? e / BK : e % BN;
            const int k = BKC ? e % BK : e / BN;
            const int gn = n0 + o, gk = k0 + k;
            const int64_t idx = BKC ? (int64_t)gn * p.B.ld + gk : (int64_t)gk * p.B.ld + gn;
            const bool v0 = gn < p.N && gk < kend;
            const bool v1 = BKC ? (gn < p.N && gk + 1 < kend) : (gn + 1 < p.N && gk < kend);
            load_raw<T, NATIVE>(p.B, zB, zB + idx, v0, br[SET][2 * i], bi[SET][2 * i]);
            load_raw<T, NATIVE>(p.B, zB, zB + idx + 1, v1, br[SET][2 * i + 1], bi[SET][2 * i + 1]);
            bm[SET] |= (v0 ? 1u : 0u) << (2 * i) | (v1 ? 1u : 0u) << (2 * i + 1);
        }
    };
    auto lstore = [&](int buf, auto setc) {
        constexpr int SET = decltype(setc)::value;
#pragma unroll
        for (int i = 0; i < AE; ++i) {
            const int e = 2 * (tid + NT * (i / 2)) + (i & 1);
            const int off = AK ? (e / BK) * LDAk + e % BK : (e / BM) * LDAo + e % BM;
            const bool v = (am[SET] >> i) & 1u;
            sA[buf][0][off] = v ? ar[SET][i] : T(0);
            sA[buf][1][off] = v ? (p.A.conj ? -ai[SET][i] : ai[SET][i]) : T(0);
        }
#pragma unroll
        for (int i = 0; i < BE; ++i) {
            const int e = 2 * (tid + NT * (i / 2)) + (i & 1);
            const int off = BKC ? (e / BK) * LDAk + e % BK : (e / BN) * LDBo + e % BN;
            const bool v = (bm[SET] >> i) & 1u;
            sB[buf][0][off] = v ? br[SET][i] : T(0);
            sB[buf][1][off] = v ? (p.B.conj ? -bi[SET][i] : bi[SET][i]) : T(0);
        }
    };

    auto& acc = accs.v;
    (void)sizeof(acc_t);

    const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    if (nk > 0) {
        gload(kbeg, I0{});
        lstore(0, I0{});
    }
    if (PF == 2 && nk > 1) gload(kbeg + BK, std::integral_constant<int, PF - 1>{});
    __syncthreads();

    // tile kt sits in LDS buffer kt & 1; with PF = 2 it was loaded into
    // register set kt & 1, with PF = 1 the single set holds the next tile
    auto body = [&](int kt, auto setc) {
        constexpr int SET = PF == 2 ? decltype(setc)::value : 0;
        using Other = std::integral_constant<int, PF == 2 ? 1 - SET : 0>;
        const int cur = kt & 1;
        if (PF == 2 && kt + 2 < nk) gload(kbeg + (kt + 2) * BK, std::integral_constant<int, SET>{});
        if (PF == 1 && kt + 1 < nk) gload(kbeg + (kt + 1) * BK, std::integral_constant<int, 0>{});
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int kk = g * S + s;  // permuted k inside the tile
            T xa[2][TM], xb[2][TN];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
#pragma unroll
                for (int mi = 0; mi < TM; ++mi) {
                    const int o = wm * TM * MT + mi * MT + r;
                    xa[q][mi] = sA[cur][q][AK ? o * LDAk + kk : kk * LDAo + o];
                }
#pragma unroll
                for (int ni = 0; ni < TN; ++ni) {
                    const int o = wn * TN * MT + ni * MT + r;
                    xb[q][ni] = sB[cur][q][BKC ? o * LDAk + kk : kk * LDBo + o];
                }
            }
            T xa3[TM], xb3[TN];
#pragma unroll
            for (int mi = 0; mi < TM; ++mi) xa3[mi] = M3 ? xa[0][mi] + xa[1][mi] : -xa[1][mi];
#pragma unroll
            for (int ni = 0; ni < TN; ++ni) xb3[ni] = xb[0][ni] + xb[1][ni];
#pragma unroll
            for (int mi = 0; mi < TM; ++mi) {
#pragma unroll
                for (int ni = 0; ni < TN; ++ni) {
                    if constexpr (M3) {
                        acc[0][mi][ni] = F::mma(xa[0][mi], xb[0][ni], acc[0][mi][ni]);
                        acc[1][mi][ni] = F::mma(xa[1][mi], xb[1][ni], acc[1][mi][ni]);
                        acc[2][mi][ni] = F::mma(xa3[mi], xb3[ni], acc[2][mi][ni]);
                    } else {
                        acc[0][mi][ni] = F::mma(xa[0][mi], xb[0][ni], acc[0][mi][ni]);
                        acc[0][mi][ni] = F::mma(xa3[mi], xb[1][ni], acc[0][mi][ni]);
                        acc[1][mi][ni] = F::mma(xa[0][mi], xb[1][ni], acc[1][mi][ni]);
                        acc[1][mi][ni] = F::mma(xa[1][mi], xb[0][ni], acc[1][mi][ni]);
                    }
                }
            }
        }
        if (kt + 1 < nk) lstore(cur ^ 1, Other{});
        __syncthreads();
    };
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {
        body(kt, I0{});
        body(kt + 1, I1{});
    }
    if (kt < nk) body(kt, I0{});
}

// Writes the accumulated tile (m0, n0) to C (offset zC), combining the 3M
// products or taking the 4M real / imaginary planes.
template <typename T, int BM, int BN, int WM, int WN, bool M3>
__device__ __forceinline__ void gemm_tile_store(const KParams& p, int m0, int n0, int64_t zC,
                                                const TileAcc<T, BM, BN, WM, WN, M3>& accs) {
    using F = Mfma<T>;
    constexpr int MT = F::MT;
    constexpr int TM = BM / (WM * MT);
    constexpr int TN = BN / (WN * MT);
    const auto& acc = accs.v;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN;
    const int wn = wave % WN;
#pragma unroll
    for (int mi = 0; mi < TM; ++mi) {
#pragma unroll
        for (int ni = 0; ni < TN; ++ni) {
#pragma unroll
            for (int v = 0; v < F::NACC; ++v) {
                const int gm = m0 + wm * TM * MT + mi * MT + F::row(lane, v);
                const int gn = n0 + wn * TN * MT + ni * MT + F::col(lane);
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

// One output tile (m0, n0) of batch entry z over k in [kbeg, kend).
template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3, bool AK, bool BKC, int PF>
__device__ __forceinline__ void gemm_block(const KParams& p, TileSmem<T, BM, BN, BK, AK, BKC>& sm, int m0, int n0,
                                           int64_t zA, int64_t zB, int64_t zC, int kbeg, int kend) {
    TileAcc<T, BM, BN, WM, WN, M3> acc;
    acc.zero();
    if (native_operands<T>(p))
        gemm_tile_acc<T, BM, BN, BK, WM, WN, M3, AK, BKC, PF, true>(p, sm, m0, n0, zA, zB, kbeg, kend, acc);
    else
        gemm_tile_acc<T, BM, BN, BK, WM, WN, M3, AK, BKC, PF, false>(p, sm, m0, n0, zA, zB, kbeg, kend, acc);
    gemm_tile_store<T, BM, BN, WM, WN, M3>(p, m0, n0, zC, acc);
}

// Tile t (0 <= t < tiles_m * tiles_n) -> (tm, tn): runs of kGroupM m-tiles
// sweep all n-tiles (the last run may be shorter); a bijection.
constexpr int kGroupM = 4;
__device__ __forceinline__ void grouped_tile(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
    const int per_group = kGroupM * tiles_n;
    const int first_m = (t / per_group) * kGroupM;
    const int gsz = min(tiles_m - first_m, kGroupM);
    const int u = t % per_group;
    tm = first_m + u % gsz;
    tn = u / gsz;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3, bool AK, bool BKC>
__global__ void __launch_bounds__(64 * WM * WN) cgemm2_kernel(KParams p) {
    __shared__ __align__(16) TileSmem<T, BM, BN, BK, AK, BKC> sm;
    const int ntiles = p.tiles_m * p.tiles_n;
    int t = blockIdx.x;
    if ((ntiles & 7) == 0) t = (t & 7) * (ntiles >> 3) + (t >> 3);  // contiguous tile range per XCD
    int tm, tn;
    grouped_tile(t, p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM;
    const int n0 = tn * BN;
    const int z = blockIdx.z / p.ksplit;
    const int kbeg = (blockIdx.z % p.ksplit) * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);
    gemm_block<T, BM, BN, BK, WM, WN, M3, AK, BKC, 2>(p, sm, m0, n0, (int64_t)z * p.A.stride, (int64_t)z * p.B.stride,
                                                   (int64_t)blockIdx.z * p.strideC, kbeg, kend);
}

// Grouped form: many independent products of different shapes in one launch.
// Block b (after the XCD remap over all tiles) finds its problem by binary
// search over the problems' first tile indices.
struct GProblem {
    KParams p;
    int64_t tile_begin;
};

template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3, bool AK, bool BKC>
__global__ void __launch_bounds__(64 * WM * WN) cgemm2_grouped_kernel(const GProblem* __restrict__ probs, int nprob,
                                                                      int64_t total) {
    __shared__ __align__(16) TileSmem<T, BM, BN, BK, AK, BKC> sm;
    int64_t t = blockIdx.x;
    if ((total & 7) == 0) t = (t & 7) * (total >> 3) + (t >> 3);
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const KParams p = probs[lo].p;
    const int tl = (int)(t - probs[lo].tile_begin);
    int tm, tn;
    grouped_tile(tl, p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM;
    const int n0 = tn * BN;
    gemm_block<T, BM, BN, BK, WM, WN, M3, AK, BKC, 1>(p, sm, m0, n0, 0, 0, 0, 0, p.K);  // measured faster here
}

// Block-sparse form: one problem per output block, batched over z and
// accumulated over its list of K chunks before the single store.
struct BProblem {
    KParams p;
    int64_t tile_begin;
    int batch, chunk0, nchunk, pad;
};
struct BChunkDev {
    int64_t offA, offB, strideA, strideB;
    int K, count;
};

template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3, bool AK, bool BKC>
__global__ void __launch_bounds__(64 * WM * WN) cgemm2_blocks_kernel(const BProblem* __restrict__ probs, int nprob,
                                                                     const BChunkDev* __restrict__ chunks,
                                                                     int64_t total) {
    __shared__ __align__(16) TileSmem<T, BM, BN, BK, AK, BKC> sm;
    int64_t t = blockIdx.x;
    if ((total & 7) == 0) t = (t & 7) * (total >> 3) + (t >> 3);
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const BProblem& bp = probs[lo];
    const KParams p = bp.p;
    const int per = p.tiles_m * p.tiles_n;
    const int tl = (int)(t - bp.tile_begin);
    const int z = tl / per;
    int tm, tn;
    grouped_tile(tl % per, p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM;
    const int n0 = tn * BN;
    const int64_t zA = (int64_t)z * p.A.stride, zB = (int64_t)z * p.B.stride;
    TileAcc<T, BM, BN, WM, WN, M3> acc;
    acc.zero();
    auto run = [&](auto native) {
        constexpr bool NAT = decltype(native)::value;
        if (bp.nchunk == 0) {
            gemm_tile_acc<T, BM, BN, BK, WM, WN, M3, AK, BKC, 1, NAT>(p, sm, m0, n0, zA, zB, 0, p.K, acc);
        } else {
            for (int c = bp.chunk0; c < bp.chunk0 + bp.nchunk; ++c) {
                const BChunkDev ch = chunks[c];
                for (int i = 0; i < ch.count; ++i)
                    gemm_tile_acc<T, BM, BN, BK, WM, WN, M3, AK, BKC, 1, NAT>(
                        p, sm, m0, n0, zA + ch.offA + i * ch.strideA, zB + ch.offB + i * ch.strideB, 0, ch.K, acc);
            }
        }
    };
    if (native_operands<T>(p)) run(std::true_type{});
    else run(std::false_type{});
    gemm_tile_store<T, BM, BN, WM, WN, M3>(p, m0, n0, (int64_t)z * p.strideC, acc);
}

__global__ void zero_fill_kernel(uint2* p, int64_t n8) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n8; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_uint2(0u, 0u);
}

// Sum of split-K partials in a fixed order (deterministic), converted to
// the output type: C[b][m][n] = sum_s part[b][s][m][n].
template <typename T>
__global__ void splitk_reduce_kernel(const void* part, int ks, int M, int N, int batch, void* C, int c128C,
                                     int64_t ldc, int64_t strideC) {
    using C2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t mn = (int64_t)M * N;
    if (idx >= mn * batch) return;
    const int64_t b = idx / mn, r = idx % mn;
    const int m = (int)(r / N), n = (int)(r % N);
    const C2* P = reinterpret_cast<const C2*>(part) + (b * ks) * mn + r;
    T re = 0, im = 0;
    for (int s = 0; s < ks; ++s) {
        const C2 v = P[s * mn];
        re += v.x;
        im += v.y;
    }
    const int64_t o = b * strideC + (int64_t)m * ldc + n;
    if (c128C) reinterpret_cast<double2*>(C)[o] = make_double2((double)re, (double)im);
    else reinterpret_cast<float2*>(C)[o] = make_float2((float)re, (float)im);
}

// Chunk-split block products: problem q's g-th part wrote its [M][N] sum to
// part + poff + g * M * N (accumulation type); C = the parts summed in order.
struct BRed {
    void* C;
    int64_t ldc, poff;
    int M, N, parts, c128C;
};

template <typename T>
__global__ void block_reduce_kernel(const BRed* __restrict__ tab, const void* __restrict__ part) {
    using C2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    const BRed r = tab[blockIdx.x];
    const int64_t mn = (int64_t)r.M * r.N;
    const C2* P = reinterpret_cast<const C2*>(part) + r.poff;
    for (int64_t i = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; i < mn; i += (int64_t)gridDim.y * blockDim.x) {
        T re = 0, im = 0;
        for (int g = 0; g < r.parts; ++g) {
            const C2 v = P[g * mn + i];
            re += v.x;
            im += v.y;
        }
        const int64_t o = (i / r.N) * r.ldc + i % r.N;
        if (r.c128C) reinterpret_cast<double2*>(r.C)[o] = make_double2((double)re, (double)im);
        else reinterpret_cast<float2*>(r.C)[o] = make_float2((float)re, (float)im);
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

template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3>
void launch2(tdvp_ctx ctx, KParams kp, int batch) {
    kp.tiles_m = (kp.M + BM - 1) / BM;
    kp.tiles_n = (kp.N + BN - 1) / BN;
    dim3 grid(kp.tiles_m * kp.tiles_n, 1, batch * kp.ksplit);
    char name[64];
    snprintf(name, sizeof(name), "cgemm2_%s_%s_%dx%dx%d_w%dx%d%s", sizeof(T) == 4 ? "f32" : "f64", M3 ? "3m" : "4m",
             BM, BN, BK, WM, WN, kp.ksplit > 1 ? "_splitk" : "");
    const double flops = 8.0 * kp.M * (double)kp.N * kp.K * batch;
    ProfScope prof(ctx, name, flops, 0.0);
    const dim3 blk(64 * WM * WN);
    if (kp.A.kcontig && !kp.B.kcontig)
        hipLaunchKernelGGL((cgemm2_kernel<T, BM, BN, BK, WM, WN, M3, true, false>), grid, blk, 0, ctx->stream, kp);
    else if (kp.A.kcontig && kp.B.kcontig)
        hipLaunchKernelGGL((cgemm2_kernel<T, BM, BN, BK, WM, WN, M3, true, true>), grid, blk, 0, ctx->stream, kp);
    else if (!kp.A.kcontig && !kp.B.kcontig)
        hipLaunchKernelGGL((cgemm2_kernel<T, BM, BN, BK, WM, WN, M3, false, false>), grid, blk, 0, ctx->stream, kp);
    else
        hipLaunchKernelGGL((cgemm2_kernel<T, BM, BN, BK, WM, WN, M3, false, true>), grid, blk, 0, ctx->stream, kp);
    TDVP_CHECK_HIP(hipGetLastError());
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3>
void launch_grouped(tdvp_ctx ctx, const GProblem* probs, int nprob, int64_t total, bool ak, bool bkc, double flops) {
    char name[64];
    snprintf(name, sizeof(name), "cgemm2g_%s_%s_%dx%dx%d_w%dx%d", sizeof(T) == 4 ? "f32" : "f64", M3 ? "3m" : "4m", BM,
             BN, BK, WM, WN);
    ProfScope prof(ctx, name, flops, 0.0);
    const dim3 grid((unsigned)total), blk(64 * WM * WN);
    if (ak && !bkc)
        hipLaunchKernelGGL((cgemm2_grouped_kernel<T, BM, BN, BK, WM, WN, M3, true, false>), grid, blk, 0, ctx->stream,
                           probs, nprob, total);
    else if (ak && bkc)
        hipLaunchKernelGGL((cgemm2_grouped_kernel<T, BM, BN, BK, WM, WN, M3, true, true>), grid, blk, 0, ctx->stream,
                           probs, nprob, total);
    else if (!ak && !bkc)
        hipLaunchKernelGGL((cgemm2_grouped_kernel<T, BM, BN, BK, WM, WN, M3, false, false>), grid, blk, 0, ctx->stream,
                           probs, nprob, total);
    else
        hipLaunchKernelGGL((cgemm2_grouped_kernel<T, BM, BN, BK, WM, WN, M3, false, true>), grid, blk, 0, ctx->stream,
                           probs, nprob, total);
    TDVP_CHECK_HIP(hipGetLastError());
}

// Tile configurations.  f32: v_mfma_f32_32x32x2f32 (32x32 per instruction),
// f64: v_mfma_f64_16x16x4f64.  Names: BMxBNxBK, waves WMxWN.
struct TileCfg {
    int id;
    bool fp64;
    int BM, BN, BK, WM, WN;
};

constexpr TileCfg kTiles[] = {
    {2, false, 128, 128, 16, 2, 4},  {9, false, 64, 64, 32, 2, 2},   {10, false, 64, 128, 16, 2, 4},
    {12, false, 64, 64, 16, 2, 2},   {13, false, 128, 128, 16, 4, 4}, {14, false, 64, 128, 32, 2, 4},
    {15, false, 128, 64, 16, 4, 2},  {16, false, 32, 64, 16, 1, 2},
    {2, true, 128, 128, 8, 2, 4},    {9, true, 64, 64, 16, 2, 2},    {12, true, 64, 64, 8, 2, 2},
    {15, true, 128, 64, 16, 4, 2},   {16, true, 32, 64, 8, 1, 2},
};

template <typename T, int BM, int BN, int BK, int WM, int WN>
void launch_form(tdvp_ctx ctx, const KParams& kp, int batch, bool m3) {
    if constexpr (sizeof(T) == 8) {
        launch2<T, BM, BN, BK, WM, WN, false>(ctx, kp, batch);
    } else {
        if (m3) launch2<T, BM, BN, BK, WM, WN, true>(ctx, kp, batch);
        else launch2<T, BM, BN, BK, WM, WN, false>(ctx, kp, batch);
    }
}

bool launch_tile(tdvp_ctx ctx, const KParams& kp, int batch, bool fp64, bool m3, int cfg) {
    if (!fp64) {
        switch (cfg) {
            case 2: launch_form<float, 128, 128, 16, 2, 4>(ctx, kp, batch, m3); return true;
            case 9: launch_form<float, 64, 64, 32, 2, 2>(ctx, kp, batch, m3); return true;
            case 10: launch_form<float, 64, 128, 16, 2, 4>(ctx, kp, batch, m3); return true;
            case 12: launch_form<float, 64, 64, 16, 2, 2>(ctx, kp, batch, m3); return true;
            case 13: launch_form<float, 128, 128, 16, 4, 4>(ctx, kp, batch, m3); return true;
            case 14: launch_form<float, 64, 128, 32, 2, 4>(ctx, kp, batch, m3); return true;
            case 15: launch_form<float, 128, 64, 16, 4, 2>(ctx, kp, batch, m3); return true;
            case 16: launch_form<float, 32, 64, 16, 1, 2>(ctx, kp, batch, m3); return true;
            default: return false;
        }
    }
    // FP64 tiles are used in the 4M form (the 3M accumulators of the large
    // tiles do not fit the register file without spilling).
    switch (cfg) {
        case 2: launch_form<double, 128, 128, 8, 2, 4>(ctx, kp, batch, false); return true;
        case 9: launch_form<double, 64, 64, 16, 2, 2>(ctx, kp, batch, false); return true;
        case 12: launch_form<double, 64, 64, 8, 2, 2>(ctx, kp, batch, false); return true;
        case 15: launch_form<double, 128, 64, 16, 4, 2>(ctx, kp, batch, false); return true;
        case 16: launch_form<double, 32, 64, 8, 1, 2>(ctx, kp, batch, false); return true;
        default: return false;
    }
}

template <typename T, int BM, int BN, int BK, int WM, int WN>
void grouped_form(tdvp_ctx ctx, const GProblem* probs, int nprob, int64_t total, bool m3, bool ak, bool bkc,
                  double flops) {
    if constexpr (sizeof(T) == 8) {
        launch_grouped<T, BM, BN, BK, WM, WN, false>(ctx, probs, nprob, total, ak, bkc, flops);
    } else {
        if (m3) launch_grouped<T, BM, BN, BK, WM, WN, true>(ctx, probs, nprob, total, ak, bkc, flops);
        else launch_grouped<T, BM, BN, BK, WM, WN, false>(ctx, probs, nprob, total, ak, bkc, flops);
    }
}

bool launch_grouped_tile(tdvp_ctx ctx, const GProblem* probs, int nprob, int64_t total, bool fp64, bool m3, bool ak,
                         bool bkc, int cfg, double flops) {
    if (!fp64) {
        switch (cfg) {
            case 2: grouped_form<float, 128, 128, 16, 2, 4>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 9: grouped_form<float, 64, 64, 32, 2, 2>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 10: grouped_form<float, 64, 128, 16, 2, 4>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 12: grouped_form<float, 64, 64, 16, 2, 2>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 13: grouped_form<float, 128, 128, 16, 4, 4>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 14: grouped_form<float, 64, 128, 32, 2, 4>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 15: grouped_form<float, 128, 64, 16, 4, 2>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            case 16: grouped_form<float, 32, 64, 16, 1, 2>(ctx, probs, nprob, total, m3, ak, bkc, flops); return true;
            default: return false;
        }
    }
    switch (cfg) {
        case 2: grouped_form<double, 128, 128, 8, 2, 4>(ctx, probs, nprob, total, false, ak, bkc, flops); return true;
        case 9: grouped_form<double, 64, 64, 16, 2, 2>(ctx, probs, nprob, total, false, ak, bkc, flops); return true;
        case 12: grouped_form<double, 64, 64, 8, 2, 2>(ctx, probs, nprob, total, false, ak, bkc, flops); return true;
        case 15: grouped_form<double, 128, 64, 16, 4, 2>(ctx, probs, nprob, total, false, ak, bkc, flops); return true;
        case 16: grouped_form<double, 32, 64, 8, 1, 2>(ctx, probs, nprob, total, false, ak, bkc, flops); return true;
        default: return false;
    }
}

const TileCfg* find_tile(int cfg, bool fp64) {
    for (const auto& c : kTiles)
        if (c.id == cfg && c.fp64 == fp64) return &c;
    return nullptr;
}

// Launch tile `cfg` with the K range split `ks` ways: partial products go to
// a workspace in the compute precision and are summed by a second kernel.
bool launch_cfg(tdvp_ctx ctx, KParams kp, int batch, bool fp64, bool m3, int cfg, int ks) {
    const TileCfg* t = find_tile(cfg, fp64);
    if (!t) return false;
    if (ks <= 1) {
        kp.ksplit = 1;
        kp.kchunk = kp.K;
        return launch_tile(ctx, kp, batch, fp64, m3, cfg);
    }
    const int chunk = ((kp.K + ks - 1) / ks + t->BK - 1) / t->BK * t->BK;
    ks = (kp.K + chunk - 1) / chunk;
    const int64_t mn = (int64_t)kp.M * kp.N;
    const size_t esz = fp64 ? sizeof(double2) : sizeof(float2);
    void* part = ctx->workspace("gemm_splitk", esz * (size_t)mn * ks * batch);
    KParams q = kp;
    q.ksplit = ks;
    q.kchunk = chunk;
    q.C = part;
    q.c128C = fp64;
    q.ldc = kp.N;
    q.strideC = mn;
    launch_tile(ctx, q, batch, fp64, m3, cfg);
    const int64_t tot = mn * batch;
    const unsigned blocks = (unsigned)((tot + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3(blocks), dim3(256), 0, ctx->stream, part, ks, kp.M,
                           kp.N, batch, kp.C, kp.c128C, kp.ldc, kp.strideC);
    else
        hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(blocks), dim3(256), 0, ctx->stream, part, ks, kp.M,
                           kp.N, batch, kp.C, kp.c128C, kp.ldc, kp.strideC);
    TDVP_CHECK_HIP(hipGetLastError());
    return true;
}

int64_t tiles_for(const TileCfg& c, const GemmDesc& g) {
    return (int64_t)((g.M + c.BM - 1) / c.BM) * ((g.N + c.BN - 1) / c.BN) * g.batch;
}

struct Choice {
    int cfg, ks;
};

// K split that gives at least two blocks per CU while every split keeps at
// least eight k-tiles.
int default_split(const TileCfg& c, const GemmDesc& g) {
    int ks = 1;
    const int64_t tiles = tiles_for(c, g);
    while (tiles * ks < 512 && g.K / (2 * ks) >= 8 * c.BK && ks < 16) ks *= 2;
    return ks;
}

// Shape heuristic used when no tuned choice exists: the largest tile that
// still gives every CU at least one block, else a small tile with split-K.
Choice heuristic_cfg(const GemmDesc& g, bool fp64) {
    const int big = fp64 ? 2 : 10;
    const TileCfg* b = find_tile(big, fp64);
    if (tiles_for(*b, g) >= 256) return {big, 1};
    const TileCfg* s = find_tile(12, fp64);
    return {12, default_split(*s, g)};
}

// ------------------------------------------------------------- autotuner
// Per shape bucket (precision, form, operand layouts, log2 of M, N, K and
// batch) the first call times every tile configuration on the call's own
// operands (C is overwritten each time, the operation is idempotent) and
// keeps the fastest.  Choices persist across processes in the text file
// named by TDVP_TUNE_CACHE, keyed by the device architecture.
struct TuneKey {
    int fp64, form, akc, bkc, lm, ln, lk, lb;
    bool operator<(const TuneKey& o) const {
        return std::tie(fp64, form, akc, bkc, lm, ln, lk, lb) < std::tie(o.fp64, o.form, o.akc, o.bkc, o.lm, o.ln, o.lk, o.lb);
    }
};

int ilog2ceil(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

struct Tuner {
    std::mutex mu;
    std::map<TuneKey, Choice> best;
    std::string arch;
    bool loaded = false;

    std::string path() const {
        const char* p = getenv("TDVP_TUNE_CACHE");
        return p ? std::string(p) : std::string();
    }
    void load(const std::string& a) {
        if (loaded) return;
        loaded = true;
        arch = a;
        const std::string p = path();
        if (p.empty()) return;
        FILE* f = fopen(p.c_str(), "r");
        if (!f) return;
        char ar[64];
        TuneKey k;
        Choice c;
        while (fscanf(f, "%63s %d %d %d %d %d %d %d %d %d %d", ar, &k.fp64, &k.form, &k.akc, &k.bkc, &k.lm, &k.ln,
                      &k.lk, &k.lb, &c.cfg, &c.ks) == 11)
            if (arch == ar) best[k] = c;
        fclose(f);
    }
    void save() {
        const std::string p = path();
        if (p.empty()) return;
        FILE* f = fopen(p.c_str(), "w");
        if (!f) return;
        for (auto& kv : best)
            fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d\n", arch.c_str(), kv.first.fp64, kv.first.form, kv.first.akc,
                    kv.first.bkc, kv.first.lm, kv.first.ln, kv.first.lk, kv.first.lb, kv.second.cfg, kv.second.ks);
        fclose(f);
    }
};

Tuner& tuner() {
    static Tuner t;
    return t;
}

int forced_cfg() {
    const char* e = getenv("TDVP_GEMM_CFG");
    return e ? atoi(e) : -1;
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

Choice choose_cfg(tdvp_ctx ctx, const GemmDesc& g, const KParams& kp, bool fp64, bool m3) {
    const int forced = forced_cfg();
    if (forced > 0 && find_tile(forced, fp64)) {
        const char* e = getenv("TDVP_GEMM_KSPLIT");
        return {forced, e ? std::max(1, atoi(e)) : 1};
    }
    const int64_t work = (int64_t)g.M * g.N * (int64_t)g.K * g.batch;
    if (!ctx->autotune || work < (int64_t)1 << 24 || stream_capturing(ctx->stream)) return heuristic_cfg(g, fp64);
    Tuner& T = tuner();
    std::lock_guard<std::mutex> lock(T.mu);
    if (!T.loaded) {
        hipDeviceProp_t prop;
        T.load(hipGetDeviceProperties(&prop, ctx->device) == hipSuccess ? std::string(prop.gcnArchName) : "unknown");
    }
    const TuneKey key{fp64, m3 ? 3 : 4, kp.A.kcontig, kp.B.kcontig, ilog2ceil(g.M), ilog2ceil(g.N),
                      ilog2ceil(g.K), ilog2ceil(g.batch)};
    auto it = T.best.find(key);
    if (it != T.best.end()) return it->second;
    hipEvent_t e0, e1;
    TDVP_CHECK_HIP(hipEventCreate(&e0));
    TDVP_CHECK_HIP(hipEventCreate(&e1));
    Choice best = heuristic_cfg(g, fp64);
    float best_ms = 1e30f;
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    // each candidate: best of three single launches after a warm-up; a K
    // split must beat the unsplit tile by 3 % (it costs an extra pass and
    // workspace, and smaller margins are timing noise)
    for (const auto& c : kTiles) {
        if (c.fp64 != fp64) continue;
        for (int ks = 1; ks <= 16; ks *= 2) {
            if (ks > 1 && (g.K / ks < 4 * c.BK || tiles_for(c, g) * ks > 4096)) break;
            launch_cfg(ctx, kp, g.batch, fp64, m3, c.id, ks);  // warm-up / code load
            float ms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                TDVP_CHECK_HIP(hipEventRecord(e0, ctx->stream));
                launch_cfg(ctx, kp, g.batch, fp64, m3, c.id, ks);
                TDVP_CHECK_HIP(hipEventRecord(e1, ctx->stream));
                TDVP_CHECK_HIP(hipEventSynchronize(e1));
                float t = 0.f;
                TDVP_CHECK_HIP(hipEventElapsedTime(&t, e0, e1));
                ms = std::min(ms, t);
            }
            const float eff = ks > 1 ? ms * 1.03f : ms;
            if (eff < best_ms) {
                best_ms = eff;
                best = {c.id, ks};
            }
        }
    }
    ctx->prof_on = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    T.best[key] = best;
    T.save();
    return best;
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
    const bool m3 = fp64 ? false : form == 3;
    if (ctx->arena) {  // allocation-free call: no tile timing, no split-K partials
        launch_cfg(ctx, kp, g.batch, fp64, m3, heuristic_cfg(g, fp64).cfg, 1);
        return;
    }
    Choice ch = choose_cfg(ctx, g, kp, fp64, m3);
    if (!ctx->splitk) ch.ks = 1;
    if (!launch_cfg(ctx, kp, g.batch, fp64, m3, ch.cfg, ch.ks)) {
        const Choice h = heuristic_cfg(g, fp64);
        launch_cfg(ctx, kp, g.batch, fp64, m3, h.cfg, ctx->splitk ? h.ks : 1);
    }
}

namespace {

// Problem table for tile `cfg` (tile counts depend on the tile edge).
int64_t build_table(const std::vector<GemmDesc>& g, const TileCfg& c, std::vector<GProblem>& out) {
    out.clear();
    int64_t total = 0;
    for (const auto& d : g) {
        if (d.M == 0 || d.N == 0) continue;
        GProblem q{};
        q.p.M = d.M;
        q.p.N = d.N;
        q.p.K = d.K;
        q.p.tiles_m = (d.M + c.BM - 1) / c.BM;
        q.p.tiles_n = (d.N + c.BN - 1) / c.BN;
        q.p.ksplit = 1;
        q.p.kchunk = d.K;
        q.p.A = to_k(d.A);
        q.p.B = to_k(d.B);
        q.p.C = d.C;
        q.p.c128C = d.cdt == Dt::C128;
        q.p.ldc = d.ldc;
        q.p.strideC = 0;
        q.tile_begin = total;
        total += (int64_t)q.p.tiles_m * q.p.tiles_n;
        out.push_back(q);
    }
    return total;
}

struct GroupTuner {
    std::mutex mu;
    std::map<std::vector<int>, int> best;  // (fp64, form, shapes...) -> tile
};
GroupTuner& group_tuner() {
    static GroupTuner t;
    return t;
}

}  // namespace

void grouped_gemm_plan(tdvp_ctx ctx, const std::vector<GemmDesc>& g, bool fp64, int form, GroupedGemm& out) {
    out.fp64 = fp64;
    out.m3 = fp64 ? false : form == 3;
    out.flops = 0.0;
    bool first = true;
    std::vector<int> sig{fp64 ? 1 : 0, out.m3 ? 3 : 4};
    for (const auto& d : g) {
        TDVP_REQUIRE(d.batch == 1, TDVP_E_ARG, "grouped gemm: batch must be 1");
        TDVP_REQUIRE(d.M >= 0 && d.N >= 0 && d.K >= 0, TDVP_E_SHAPE, "grouped gemm: bad sizes");
        if (d.M == 0 || d.N == 0) continue;
        TDVP_REQUIRE(d.A.p && d.B.p && d.C, TDVP_E_ARG, "grouped gemm: null operand");
        if (first) {
            out.ak = d.A.kcontig;
            out.bkc = d.B.kcontig;
            first = false;
        }
        TDVP_REQUIRE(d.A.kcontig == out.ak && d.B.kcontig == out.bkc, TDVP_E_ARG,
                     "grouped gemm: all problems must share operand layouts");
        out.flops += 8.0 * d.M * (double)d.N * d.K;
        sig.push_back(d.M);
        sig.push_back(d.N);
        sig.push_back(d.K);
    }
    std::vector<GProblem> tab;
    auto upload = [&](int cfg) {
        const TileCfg* c = find_tile(cfg, fp64);
        out.total = build_table(g, *c, tab);
        out.nprob = (int)tab.size();
        out.cfg = cfg;
        if (out.probs.bytes < sizeof(GProblem) * tab.size()) out.probs = DevMem(ctx, sizeof(GProblem) * tab.size());
        if (!tab.empty())
            TDVP_CHECK_HIP(hipMemcpyAsync(out.probs.ptr, tab.data(), sizeof(GProblem) * tab.size(),
                                          hipMemcpyHostToDevice, ctx->stream));
        // the table must be on the device before the host vector goes away
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    };
    const int forced = forced_cfg();
    if (forced > 0 && find_tile(forced, fp64)) {
        upload(forced);
        return;
    }
    // heuristic: the large tile when it still gives every CU two blocks
    int cfg = fp64 ? 2 : 10;
    {
        std::vector<GProblem> t2;
        if (build_table(g, *find_tile(cfg, fp64), t2) < 512) cfg = 12;
    }
    GroupTuner& T = group_tuner();
    {
        std::lock_guard<std::mutex> lock(T.mu);
        auto it = T.best.find(sig);
        if (it != T.best.end()) cfg = it->second;
        else if (ctx->autotune && out.flops >= 1e11 && !stream_capturing(ctx->stream)) {
            hipEvent_t e0, e1;
            TDVP_CHECK_HIP(hipEventCreate(&e0));
            TDVP_CHECK_HIP(hipEventCreate(&e1));
            float best_ms = 1e30f;
            const bool prof = ctx->prof_on;
            ctx->prof_on = false;
            // candidates: the tiles that win on large ragged groups (128x128 with
            // 16 waves since the grouped tile order)
            const int cand32[] = {10, 2, 12, 15, 13}, cand64[] = {2, 12, 15};
            const int* cand = fp64 ? cand64 : cand32;
            const int ncand = fp64 ? 3 : 5;
            for (int ci = 0; ci < ncand; ++ci) {
                const TileCfg& c = *find_tile(cand[ci], fp64);
                upload(c.id);
                auto* pr = static_cast<const GProblem*>(out.probs.ptr);
                launch_grouped_tile(ctx, pr, out.nprob, out.total, fp64, out.m3, out.ak, out.bkc, c.id, out.flops);
                TDVP_CHECK_HIP(hipEventRecord(e0, ctx->stream));
                launch_grouped_tile(ctx, pr, out.nprob, out.total, fp64, out.m3, out.ak, out.bkc, c.id, out.flops);
                TDVP_CHECK_HIP(hipEventRecord(e1, ctx->stream));
                TDVP_CHECK_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                TDVP_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) {
                    best_ms = ms;
                    cfg = c.id;
                }
            }
            ctx->prof_on = prof;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            T.best[sig] = cfg;
        }
    }
    upload(cfg);
}

namespace {

template <typename T, int BM, int BN, int BK, int WM, int WN, bool M3>
void launch_blocks(tdvp_ctx ctx, const BProblem* probs, int nprob, const BChunkDev* chunks, int64_t total, bool ak,
                   bool bkc, double flops, const char* tag) {
    char name[80];
    snprintf(name, sizeof(name), "cgemm2_blocks_%s_%s_%s_%dx%dx%d", tag, sizeof(T) == 4 ? "f32" : "f64",
             M3 ? "3m" : "4m", BM, BN, BK);
    ProfScope prof(ctx, name, flops, 0.0);
    const dim3 grid((unsigned)total), blk(64 * WM * WN);
    if (ak && !bkc)
        hipLaunchKernelGGL((cgemm2_blocks_kernel<T, BM, BN, BK, WM, WN, M3, true, false>), grid, blk, 0, ctx->stream,
                           probs, nprob, chunks, total);
    else if (ak && bkc)
        hipLaunchKernelGGL((cgemm2_blocks_kernel<T, BM, BN, BK, WM, WN, M3, true, true>), grid, blk, 0, ctx->stream,
                           probs, nprob, chunks, total);
    else if (!ak && !bkc)
        hipLaunchKernelGGL((cgemm2_blocks_kernel<T, BM, BN, BK, WM, WN, M3, false, false>), grid, blk, 0, ctx->stream,
                           probs, nprob, chunks, total);
    else
        hipLaunchKernelGGL((cgemm2_blocks_kernel<T, BM, BN, BK, WM, WN, M3, false, true>), grid, blk, 0, ctx->stream,
                           probs, nprob, chunks, total);
    TDVP_CHECK_HIP(hipGetLastError());
}

}  // namespace

void zero_fill(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    TDVP_REQUIRE(bytes % 8 == 0 && ((uintptr_t)p & 7) == 0, TDVP_E_ARG, "zero_fill: 8-byte granules only");
    const int64_t n8 = (int64_t)(bytes / 8);
    const unsigned blocks = (unsigned)std::min<int64_t>((n8 + 255) / 256, 8192);
    hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint2*>(p), n8);
    TDVP_CHECK_HIP(hipGetLastError());
}

void block_gemm(tdvp_ctx ctx, const std::vector<BlockGemm>& probs, const std::vector<BlockChunk>& chunks, bool fp64,
                int form, const char* tag) {
    if (probs.empty()) return;
    const bool m3 = fp64 ? false : form == 3;
    std::vector<BProblem> hp;
    hp.reserve(probs.size());
    int64_t total = 0;
    double flops = 0.0;
    int maxmn = 0;
    const bool ak = probs[0].g.A.kcontig, bkc = probs[0].g.B.kcontig;
    for (const auto& q : probs) {
        const GemmDesc& d = q.g;
        TDVP_REQUIRE(d.A.kcontig == ak && d.B.kcontig == bkc, TDVP_E_ARG, "block gemm: mixed operand layouts");
        TDVP_REQUIRE(d.M >= 0 && d.N >= 0 && d.K >= 0 && d.batch >= 1, TDVP_E_SHAPE, "block gemm: bad sizes");
        if (d.M == 0 || d.N == 0) continue;
        TDVP_REQUIRE(q.chunk0 >= 0 && q.nchunk >= 0 && q.chunk0 + q.nchunk <= (int)chunks.size(), TDVP_E_ARG,
                     "block gemm: chunk range out of bounds");
        maxmn = std::max(maxmn, std::max(d.M, d.N));
        BProblem b{};
        b.p.M = d.M;
        b.p.N = d.N;
        b.p.K = d.K;
        b.p.A = to_k(d.A);
        b.p.B = to_k(d.B);
        b.p.C = d.C;
        b.p.c128C = d.cdt == Dt::C128;
        b.p.ldc = d.ldc;
        b.p.strideC = d.strideC;
        b.p.ksplit = 1;
        b.p.kchunk = d.K;
        b.batch = d.batch;
        b.chunk0 = q.chunk0;
        b.nchunk = q.nchunk;
        double kk = q.nchunk == 0 ? (double)d.K : 0.0;
        for (int c = q.chunk0; c < q.chunk0 + q.nchunk; ++c) kk += (double)chunks[c].K * chunks[c].count;
        flops += 8.0 * d.M * (double)d.N * kk * d.batch;
        hp.push_back(b);
    }
    if (hp.empty()) return;
    const bool small = maxmn <= 32;
    const int BM = small ? 32 : 64, BN = 64;
    for (auto& b : hp) {
        b.p.tiles_m = (b.p.M + BM - 1) / BM;
        b.p.tiles_n = (b.p.N + BN - 1) / BN;
        b.tile_begin = total;
        total += (int64_t)b.p.tiles_m * b.p.tiles_n * b.batch;
    }
    TDVP_REQUIRE(total <= 0x7fffffff, TDVP_E_SHAPE, "block gemm: too many tiles");
    std::vector<BChunkDev> hc(chunks.size());
    for (size_t c = 0; c < chunks.size(); ++c)
        hc[c] = BChunkDev{chunks[c].offA, chunks[c].offB, chunks[c].strideA, chunks[c].strideB, chunks[c].K,
                          chunks[c].count};
    // Too few tiles to fill the CUs (each walking a long chunk list): the
    // chunk list of every unbatched problem is cut into up to `parts`
    // consecutive pieces of about equal K (a chunk of count c is c unit
    // products), each piece a problem of its own that writes an [M][N]
    // partial sum; a reduction adds the pieces in order (deterministic).
    std::vector<BRed> red;
    int64_t part_elems = 0;
    char* part = nullptr;
    const int parts = total >= 512 ? 1 : (int)std::min<int64_t>(8, (512 + total - 1) / std::max<int64_t>(1, total));
    if (parts > 1) {
        std::vector<BProblem> out;
        std::vector<BChunkDev> oc;
        std::vector<int64_t> part_off;  // per problem of `out`: offset of its partial, or -1
        int64_t t2 = 0;
        for (const auto& b : hp) {
            int units = 0;
            for (int c = b.chunk0; c < b.chunk0 + b.nchunk; ++c) units += hc[c].count;
            const int np = std::min(parts, units);
            if (b.batch != 1 || b.nchunk == 0 || np < 2) {
                BProblem x = b;
                const int c0 = (int)oc.size();
                for (int c = b.chunk0; c < b.chunk0 + b.nchunk; ++c) oc.push_back(hc[c]);
                x.chunk0 = c0;
                x.tile_begin = t2;
                t2 += (int64_t)x.p.tiles_m * x.p.tiles_n * x.batch;
                out.push_back(x);
                part_off.push_back(-1);
                continue;
            }
            const int64_t mn = (int64_t)b.p.M * b.p.N;
            red.push_back(BRed{b.p.C, b.p.ldc, part_elems, b.p.M, b.p.N, np, b.p.c128C ? 1 : 0});
            // unit u of the problem = (chunk c, product i); piece g takes units [g*units/np, (g+1)*units/np)
            int c = b.chunk0, i = 0;
            for (int g = 0; g < np; ++g) {
                const int take = (int)((int64_t)(g + 1) * units / np - (int64_t)g * units / np);
                BProblem x = b;
                x.chunk0 = (int)oc.size();
                for (int left = take; left > 0;) {
                    const BChunkDev& src = hc[c];
                    const int n = std::min(left, src.count - i);
                    BChunkDev piece = src;
                    piece.offA = src.offA + (int64_t)i * src.strideA;
                    piece.offB = src.offB + (int64_t)i * src.strideB;
                    piece.count = n;
                    oc.push_back(piece);
                    left -= n;
                    i += n;
                    if (i == src.count) {
                        ++c;
                        i = 0;
                    }
                }
                x.nchunk = (int)oc.size() - x.chunk0;
                x.p.c128C = fp64;
                x.p.ldc = b.p.N;
                x.p.strideC = mn;
                x.tile_begin = t2;
                t2 += (int64_t)x.p.tiles_m * x.p.tiles_n;
                out.push_back(x);
                part_off.push_back(part_elems + g * mn);
            }
            part_elems += np * mn;
        }
        if (!red.empty()) {
            const size_t pesz = fp64 ? sizeof(double2) : sizeof(float2);
            part = static_cast<char*>(ctx->workspace(std::string("blk_") + tag + "_part", pesz * part_elems));
            for (size_t q = 0; q < out.size(); ++q)
                if (part_off[q] >= 0) out[q].p.C = part + part_off[q] * (int64_t)pesz;
            hp.swap(out);
            hc.swap(oc);
            total = t2;
            TDVP_REQUIRE(total <= 0x7fffffff, TDVP_E_SHAPE, "block gemm: too many tiles");
        }
    }
    const std::string key = std::string("blk_") + tag;
    auto* dp = static_cast<BProblem*>(ctx->workspace(key + "_p", sizeof(BProblem) * hp.size()));
    auto* dc = static_cast<BChunkDev*>(ctx->workspace(key + "_c", sizeof(BChunkDev) * std::max<size_t>(1, hc.size())));
    ctx->upload(dp, hp.data(), sizeof(BProblem) * hp.size());
    if (!hc.empty()) ctx->upload(dc, hc.data(), sizeof(BChunkDev) * hc.size());
    const int n = (int)hp.size();
    if (fp64) {
        if (small) launch_blocks<double, 32, 64, 8, 1, 2, false>(ctx, dp, n, dc, total, ak, bkc, flops, tag);
        else launch_blocks<double, 64, 64, 8, 2, 2, false>(ctx, dp, n, dc, total, ak, bkc, flops, tag);
    } else if (m3) {
        if (small) launch_blocks<float, 32, 64, 16, 1, 2, true>(ctx, dp, n, dc, total, ak, bkc, flops, tag);
        else launch_blocks<float, 64, 64, 16, 2, 2, true>(ctx, dp, n, dc, total, ak, bkc, flops, tag);
    } else {
        if (small) launch_blocks<float, 32, 64, 16, 1, 2, false>(ctx, dp, n, dc, total, ak, bkc, flops, tag);
        else launch_blocks<float, 64, 64, 16, 2, 2, false>(ctx, dp, n, dc, total, ak, bkc, flops, tag);
    }
    if (!red.empty()) {
        const std::string key2 = std::string("blk_") + tag + "_red";
        auto* dr = static_cast<BRed*>(ctx->workspace(key2, sizeof(BRed) * red.size()));
        ctx->upload(dr, red.data(), sizeof(BRed) * red.size());
        ProfScope prof(ctx, fp64 ? "block_reduce_f64" : "block_reduce_f32", 0.0, 0.0);
        // problems x slices of each problem's elements: about 2048 blocks in all
        int64_t maxmn = 1;
        for (const auto& r : red) maxmn = std::max<int64_t>(maxmn, (int64_t)r.M * r.N);
        const unsigned ys = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>((maxmn + 255) / 256, (2048 + (int64_t)red.size() - 1) / (int64_t)red.size()));
        const dim3 grid((unsigned)red.size(), ys);
        if (fp64)
            hipLaunchKernelGGL(block_reduce_kernel<double>, grid, dim3(256), 0, ctx->stream, dr, part);
        else
            hipLaunchKernelGGL(block_reduce_kernel<float>, grid, dim3(256), 0, ctx->stream, dr, part);
        TDVP_CHECK_HIP(hipGetLastError());
    }
}

void grouped_gemm_run(tdvp_ctx ctx, const GroupedGemm& gg) {
    if (gg.nprob == 0 || gg.total == 0) return;
    TDVP_REQUIRE(gg.total <= 0x7fffffff, TDVP_E_SHAPE, "grouped gemm: too many tiles");
    launch_grouped_tile(ctx, static_cast<const GProblem*>(gg.probs.ptr), gg.nprob, gg.total, gg.fp64, gg.m3, gg.ak,
                        gg.bkc, gg.cfg, gg.flops);
}

}  // namespace tdvp
