// Allocation-free H_eff application (apply_heff_noalloc), for callers that
// cannot allocate device memory: code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation.  The MPO-stage operator and the two
// intermediate stages of the H_eff pipeline live in one fixed scratch array
// that the library keeps on every device it runs on until the process ends.
#include "internal.hpp"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // this device's address of `scratch`
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

int ipow(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Scratch bytes the pipeline asks for, in the order it asks (the MPO-stage
// operator's CSR arrays and dense staging, then the two intermediate stages
// unless the fused small-bond kernel runs).  Mirrors heff_raw_call/mop_make.
size_t heff_scratch_bytes(int nsite, bool fp64, int chil, int chir, int d, int wl, int wr) {
    const int D = nsite == 0 ? 1 : ipow(d, nsite);
    const size_t rows = (size_t)wr * D, cols = (size_t)wl * D, nz = rows * cols;
    const size_t esz = fp64 ? 16 : 8;
    size_t b = up256(sizeof(int) * (rows + 1)) + up256(sizeof(int) * nz) + up256(esz * nz) + up256(16 * nz);
    if (!tdvp::heff_small_fits(chil, chir, D, wl, wr, fp64))
        b += up256(esz * (size_t)wl * chil * D * chir) + up256(esz * (size_t)wr * chil * D * chir);
    return b;
}

}  // namespace

namespace tdvp {

void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) {
        g_scratch_err[device] = hipErrorInvalidDevice;
        return;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    if (e == hipSuccess && p) {
        g_scratch_ptr[device] = p;
        g_scratch_done[device] = true;
    }
}

}  // namespace tdvp

using namespace tdvp;

extern "C" {

size_t apply_heff_noalloc_max_bytes(void) { return kScratchBytes; }

int apply_heff_noalloc(tdvp_ctx ctx, int nsite, tdvp_dtype dtype, int chil, int chir, int d, int wl, int wm,
                       int wr, const void* L, const void* W1, const void* W2, const void* R, const void* theta,
                       void* out) {
    if (!ctx) return TDVP_E_ARG;
    return guarded(ctx, [&] {
        TDVP_REQUIRE(ctx->device >= 0 && ctx->device < kMaxDevices, TDVP_E_ARG, "apply_heff_noalloc: bad device");
        void* base = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            base = g_scratch_ptr[ctx->device];
            TDVP_REQUIRE(base, TDVP_E_HIP,
                         std::string("apply_heff_noalloc: scratch address unavailable on this device: ") +
                             hipGetErrorString(g_scratch_err[ctx->device]));
        }
        TDVP_REQUIRE(dtype == TDVP_C64 || dtype == TDVP_C128, TDVP_E_DTYPE, "apply_heff_noalloc: bad dtype");
        TDVP_REQUIRE(nsite >= 0 && nsite <= 2 && chil >= 1 && chir >= 1 && wl >= 1 && wr >= 1 &&
                         (nsite == 0 || d >= 1),
                     TDVP_E_SHAPE, "apply_heff_noalloc: bad dimensions");
        const size_t need = heff_scratch_bytes(nsite, dtype == TDVP_C128, chil, chir, d, wl, wr);
        TDVP_REQUIRE(need <= kScratchBytes, TDVP_E_NOMEM,
                     "apply_heff_noalloc: this problem needs " + std::to_string(need) +
                         " bytes of scratch, the maximum is " + std::to_string(kScratchBytes));
        Arena arena;
        arena.base = static_cast<char*>(base);
        arena.cap = kScratchBytes;
        struct Reset {
            tdvp_ctx c;
            ~Reset() { c->arena = nullptr; }
        } reset{ctx};
        ctx->arena = &arena;
        heff_raw_call(ctx, nsite, dtype, chil, chir, d, wl, wm, wr, L, W1, W2, R, theta, out);
    });
}

}  // extern "C"
