// Context: device, stream, allocator, rocBLAS handle and named workspaces.
#include "internal.hpp"

#include <algorithm>

#include <rocsolver/rocsolver.h>

void* tdvp_ctx_s::dev_alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    void* p = nullptr;
    if (alloc_fn) {
        p = alloc_fn(bytes, (void*)stream, user);
        if (!p) throw tdvp::Error(TDVP_E_NOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess || !p)
            throw tdvp::Error(TDVP_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    return p;
}

void tdvp_ctx_s::dev_free(void* p, size_t bytes) {
    if (!p) return;
    if (free_fn) free_fn(p, bytes, (void*)stream, user);
    else (void)hipFree(p);
}

void* tdvp_ctx_s::workspace(const std::string& name, size_t bytes) {
    if (arena) {
        auto it = arena->named.find(name);
        if (it != arena->named.end()) {
            TDVP_REQUIRE(it->second.second >= bytes, TDVP_E_NOMEM,
                         "allocation-free call: scratch block '" + name + "' asked for twice with a larger size");
            return arena->base + it->second.first;
        }
        const size_t off = (arena->used + 255) / 256 * 256;
        TDVP_REQUIRE(off + bytes <= arena->cap, TDVP_E_NOMEM,
                     "allocation-free call: scratch exhausted (" + std::to_string(off + bytes) + " of " +
                         std::to_string(arena->cap) + " bytes)");
        arena->named[name] = {off, bytes};
        arena->used = off + bytes;
        return arena->base + off;
    }
    tdvp::Buffer& b = work[name];
    if (b.bytes < bytes) {
        if (b.ptr) {
            // the old buffer may still be read by queued kernels
            TDVP_CHECK_HIP(hipStreamSynchronize(stream));
            dev_free(b.ptr, b.bytes);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t cap = bytes + bytes / 4 + 256;
        b.ptr = dev_alloc(cap);
        b.bytes = cap;
        ++ws_gen;  // anything that recorded workspace addresses must re-record them
    }
    return b.ptr;
}

void* tdvp_ctx_s::pinned_host(size_t bytes) {
    if (pinned_bytes < bytes) {
        if (pinned) {
            TDVP_CHECK_HIP(hipStreamSynchronize(stream));  // a queued copy may still read it
            (void)hipHostFree(pinned);
            pinned = nullptr;
            pinned_bytes = 0;
        }
        const size_t cap = std::max<size_t>(bytes, 4096);
        TDVP_CHECK_HIP(hipHostMalloc(&pinned, cap, hipHostMallocDefault));
        pinned_bytes = cap;
    }
    return pinned;
}

void tdvp_ctx_s::upload(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return;
    if (bytes > up_slot_bytes) {
        // regrow: every copy out of the old slots must have completed first
        for (auto& sl : up_slot)
            if (sl.pending) {
                TDVP_CHECK_HIP(hipEventSynchronize(sl.ev));
                sl.pending = false;
            }
        if (up_base) (void)hipHostFree(up_base);
        up_base = nullptr;
        up_slot_bytes = 0;
        const size_t cap = std::max<size_t>((bytes + 255) / 256 * 256, 64 * 1024);
        void* p = nullptr;
        TDVP_CHECK_HIP(hipHostMalloc(&p, cap * kUploadSlots, hipHostMallocDefault));
        up_base = static_cast<char*>(p);
        up_slot_bytes = cap;
    }
    UploadSlot& sl = up_slot[up_next];
    char* slot = up_base + (size_t)up_next * up_slot_bytes;
    up_next = (up_next + 1) % kUploadSlots;
    if (!sl.ev) TDVP_CHECK_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    if (sl.pending) TDVP_CHECK_HIP(hipEventSynchronize(sl.ev));
    sl.pending = false;
    std::memcpy(slot, src, bytes);
    TDVP_CHECK_HIP(hipMemcpyAsync(dst, slot, bytes, hipMemcpyHostToDevice, stream));
    TDVP_CHECK_HIP(hipEventRecord(sl.ev, stream));
    sl.pending = true;
}

void tdvp_ctx_s::wait_stream() {
    for (int i = 0; i < 4096; ++i) {
        const hipError_t e = hipStreamQuery(stream);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) TDVP_CHECK_HIP(e);
    }
    TDVP_CHECK_HIP(hipStreamSynchronize(stream));
}

void tdvp_ctx_s::read_back(std::initializer_list<ReadSpan> spans) {
    size_t total = 0;
    for (const auto& r : spans) total += (r.bytes + 15) / 16 * 16;
    if (pinned_rd_bytes < total) {
        if (pinned_rd) (void)hipHostFree(pinned_rd);  // no copy into it is pending between calls
        pinned_rd = nullptr;
        pinned_rd_bytes = 0;
        const size_t cap = std::max<size_t>(total, 16384);
        TDVP_CHECK_HIP(hipHostMalloc(&pinned_rd, cap, hipHostMallocDefault));
        pinned_rd_bytes = cap;
    }
    char* p = static_cast<char*>(pinned_rd);
    size_t off = 0;
    for (const auto& r : spans) {
        if (r.bytes) TDVP_CHECK_HIP(hipMemcpyAsync(p + off, r.src, r.bytes, hipMemcpyDeviceToHost, stream));
        off += (r.bytes + 15) / 16 * 16;
    }
    wait_stream();
    off = 0;
    for (const auto& r : spans) {
        if (r.bytes) std::memcpy(r.dst, p + off, r.bytes);
        off += (r.bytes + 15) / 16 * 16;
    }
}

void tdvp_ctx_s::release_all() {
    solver_lanes.reset();  // joins nothing: the lanes only run inside a split
    for (auto& sl : up_slot) {
        if (sl.ev) {
            if (sl.pending) (void)hipEventSynchronize(sl.ev);
            (void)hipEventDestroy(sl.ev);
        }
        sl.ev = nullptr;
        sl.pending = false;
    }
    if (up_base) (void)hipHostFree(up_base);
    up_base = nullptr;
    up_slot_bytes = 0;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
    if (pinned_rd) (void)hipHostFree(pinned_rd);
    pinned_rd = nullptr;
    pinned_rd_bytes = 0;
    for (auto& kv : work) dev_free(kv.second.ptr, kv.second.bytes);
    work.clear();
}

namespace tdvp {

int guarded(tdvp_ctx ctx, const std::function<void()>& body) {
    try {
        body();
        if (ctx) ctx->err.clear();
        return TDVP_OK;
    } catch (const Error& e) {
        if (ctx) ctx->err = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->err = "host allocation failed";
        return TDVP_E_NOMEM;
    } catch (const std::exception& e) {
        if (ctx) ctx->err = e.what();
        return TDVP_E_STATE;
    } catch (...) {
        if (ctx) ctx->err = "unknown error";
        return TDVP_E_STATE;
    }
}

}  // namespace tdvp

extern "C" {

const char* tdvp_version(void) { return "tdvp-gfx950 0.1"; }

int tdvp_ctx_create(int device, void* hip_stream, tdvp_alloc_fn alloc_fn, tdvp_free_fn free_fn,
                    void* user, tdvp_ctx* out) {
    if (!out) return TDVP_E_ARG;
    *out = nullptr;
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return TDVP_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return TDVP_E_HIP;
    if (device < 0 || device >= ndev) return TDVP_E_ARG;
    auto* c = new (std::nothrow) tdvp_ctx_s();
    if (!c) return TDVP_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->alloc_fn = alloc_fn;
    c->free_fn = free_fn;
    c->user = user;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return TDVP_E_HIP;
    }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        delete c;
        return TDVP_E_HIP;
    }
    rocblas_set_stream(c->blas, c->stream);
    tdvp::scratch_setup(device);  // this device's scratch address for apply_heff_noalloc
    *out = c;
    return TDVP_OK;
}

int tdvp_ctx_destroy(tdvp_ctx ctx) {
    if (!ctx) return TDVP_E_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    ctx->release_all();
    if (ctx->blas) rocblas_destroy_handle(ctx->blas);
    delete ctx;
    return TDVP_OK;
}

const char* tdvp_last_error(tdvp_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int tdvp_ctx_sync(tdvp_ctx ctx) {
    if (!ctx) return TDVP_E_ARG;
    return tdvp::guarded(ctx, [&] { TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream)); });
}

int tdvp_opts_default(tdvp_opts* o) {
    if (!o) return TDVP_E_ARG;
    o->compute = TDVP_C128;
    o->krylov_max = 40;
    o->krylov_tol = 1e-13;
    o->chi_max = 1 << 30;
    o->w_max = 0.0;
    o->eps_rel = 0.0;
    o->multiplet_guard = 1;
    o->strict = 0;
    o->imaginary = 0;
    o->exp_method = 0;
    o->gemm_form = 0;
    o->svd_mode = 0;
    o->u1_block_min = 0;
    return TDVP_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- profiler

namespace tdvp {

ProfScope::ProfScope(tdvp_ctx c, const char* name, double flops, double bytes) : ctx(c) {
    if (!ctx || !ctx->prof_on) return;
    tdvp_prof_rec r;
    r.name = name;
    r.flops = flops;
    r.bytes = bytes;
    TDVP_CHECK_HIP(hipEventCreate(&r.start));
    TDVP_CHECK_HIP(hipEventCreate(&r.stop));
    TDVP_CHECK_HIP(hipEventRecord(r.start, ctx->stream));
    idx = ctx->prof_pending.size();
    ctx->prof_pending.push_back(r);
}

ProfScope::~ProfScope() {
    if (idx != (size_t)-1) (void)hipEventRecord(ctx->prof_pending[idx].stop, ctx->stream);
}

}  // namespace tdvp

extern "C" {

int tdvp_profile_enable(tdvp_ctx ctx, int on) {
    if (!ctx) return TDVP_E_ARG;
    ctx->prof_on = on != 0;
    return TDVP_OK;
}

int tdvp_ctx_set_gemm_form(tdvp_ctx ctx, int form) {
    if (!ctx || (form != 0 && form != 3 && form != 4)) return TDVP_E_ARG;
    ctx->gemm_form = form;
    return TDVP_OK;
}

int tdvp_profile_read(tdvp_ctx ctx, int max_entries, char* names, double* ms, double* flops,
                      double* bytes, long* count, int* n_out) {
    if (!ctx || !n_out || (max_entries > 0 && (!names || !ms || !flops || !bytes || !count))) return TDVP_E_ARG;
    return tdvp::guarded(ctx, [&] {
        TDVP_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        for (auto& r : ctx->prof_pending) {
            float t = 0.0f;
            TDVP_CHECK_HIP(hipEventElapsedTime(&t, r.start, r.stop));
            auto& tot = ctx->prof_total[r.name];
            tot.ms += t;
            tot.flops += r.flops;
            tot.bytes += r.bytes;
            tot.count += 1;
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        ctx->prof_pending.clear();
        int i = 0;
        for (auto& kv : ctx->prof_total) {
            if (i >= max_entries) break;
            std::memset(names + 64 * i, 0, 64);
            std::strncpy(names + 64 * i, kv.first.c_str(), 63);
            ms[i] = kv.second.ms;
            flops[i] = kv.second.flops;
            bytes[i] = kv.second.bytes;
            count[i] = kv.second.count;
            ++i;
        }
        *n_out = i;
        ctx->prof_total.clear();
    });
}

}  // extern "C"
