// cs_api.hip -- the C ABI of libcompton.so: argument validation, context and
// workspace management, error reporting.  Kernels live in cs_step.hip and
// cs_mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "cs_internal.h"

namespace cs {
int64_t step_scan_tmp_len(int64_t n_cells, int64_t n_chunks);
}

namespace {

thread_local std::string g_create_error;

cs_status fail(cs_ctx* ctx, cs_status code, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    return code;
}

cs_status hip_fail(cs_ctx* ctx, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(ctx, CS_ERR_HIP, m);
}

// Ensure the context workspace holds `step_bytes` of per-step area and
// `status_words` look-back status words.  Growth waits for `stream` first so
// that no queued kernel still uses the old buffer, then re-initialises the
// control block (epoch 1) and zeroes the status words (synchronous; never
// inside a captured graph, since a captured step never grows).
cs_status ensure_workspace(cs_ctx* ctx, size_t step_bytes, int64_t status_words, hipStream_t stream) {
    cs::Workspace& w = ctx->ws;
    if (w.base && w.status_cap >= status_words && w.bytes >= cs::ws_fixed_bytes(w.status_cap) + step_bytes)
        return CS_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "workspace growth: stream synchronize");
    if (w.base) {
        e = hipFree(w.base);
        w.base = nullptr;
        w.bytes = 0;
        w.status_cap = 0;
        if (e != hipSuccess) return hip_fail(ctx, e, "workspace growth: hipFree");
    }
    const int64_t cap = status_words + status_words / 4 + 64;
    const size_t fixed = cs::ws_fixed_bytes(cap);
    const size_t want = fixed + step_bytes + step_bytes / 4 + 4096;
    e = hipMalloc(&w.base, want);
    if (e != hipSuccess) {
        w.base = nullptr;
        return hip_fail(ctx, e, "workspace growth: hipMalloc");
    }
    e = hipMemset(w.base, 0, fixed);
    cs::StepControl init = {};
    init.epoch = 1;
    if (e == hipSuccess) e = hipMemcpy(w.base, &init, sizeof(init), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "workspace growth: initialisation");
    w.bytes = want;
    w.status_cap = cap;
    return CS_OK;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool species_ok(const cs_species& s) {
    if (s.n < 0) return false;
    if (s.n == 0) return true;
    return s.x && s.y && s.z && s.w;
}

}  // namespace

extern "C" {

cs_status cs_create(cs_ctx** out, int device) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "cs_create: out is NULL";
        return CS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        g_create_error = std::string("cs_create: no HIP device: ") + hipGetErrorString(e);
        return CS_ERR_HIP;
    }
    if (device < 0 || device >= n) {
        g_create_error = "cs_create: device index out of range";
        return CS_ERR_INVALID_ARG;
    }
    cs_ctx* c = new (std::nothrow) cs_ctx();
    if (!c) {
        g_create_error = "cs_create: out of host memory";
        return CS_ERR_INVALID_ARG;
    }
    c->device = device;
    *out = c;
    return CS_OK;
}

cs_status cs_destroy(cs_ctx* ctx) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    {
        DeviceGuard g(ctx->device);
        if (ctx->ws.base) {
            (void)hipDeviceSynchronize();
            (void)hipFree(ctx->ws.base);
        }
        for (auto& ev : ctx->events)
            if (ev) (void)hipEventDestroy(ev);
    }
    delete ctx;
    return CS_OK;
}

const char* cs_last_error(const cs_ctx* ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->last_error.c_str();
}

cs_status cs_sync(cs_ctx* ctx, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_sync");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_sync");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_compton_step(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                          const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                          double density_norm, uint64_t seed, uint64_t step, cs_sampler sampler,
                          const cs_mlp* mlp, cs_stats* stats, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (dtype != CS_F32 && dtype != CS_F64) return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: bad dtype");
    if (!species_ok(electrons) || !species_ok(photons))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: species arrays NULL or count negative");
    if (n_cells < 0) return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: n_cells < 0");
    if (!off_e || !off_g) return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: offsets NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: dt must be > 0");
    if (!(density_norm >= 0.0) || !std::isfinite(density_norm))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: density_norm must be >= 0");
    if (n_cells == 0 && (electrons.n != 0 || photons.n != 0))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: particles given but n_cells == 0");
    if (electrons.n >= (int64_t)1 << 31 || photons.n >= (int64_t)1 << 31)
        return fail(ctx, CS_ERR_UNSUPPORTED, "cs_compton_step: a species count >= 2^31");
    if (n_cells >= (int64_t)1 << 31) return fail(ctx, CS_ERR_UNSUPPORTED, "cs_compton_step: n_cells >= 2^31");
    if (sampler == CS_SAMPLER_PLAIN) {
        if (mlp) return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: PLAIN sampler takes mlp == NULL");
    } else if (sampler == CS_SAMPLER_MLP_F32 || sampler == CS_SAMPLER_MLP_BF16 || sampler == CS_SAMPLER_MLP_FP8) {
        if (!mlp) return fail(ctx, CS_ERR_NOT_READY, "cs_compton_step: MLP sampler without a network");
        return fail(ctx, CS_ERR_NOT_READY, "cs_compton_step: MLP sampler not prepared");
    } else {
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_compton_step: bad sampler");
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, CS_ERR_HIP, "cs_compton_step: cannot select device");
    hipStream_t st = (hipStream_t)stream;
    cs::StepShape sh;
    sh.n_cells = n_cells;
    sh.ne = electrons.n;
    sh.ng = photons.n;
    const int64_t nmin = electrons.n < photons.n ? electrons.n : photons.n;
    sh.n_chunks = (nmin + cs::kChunk - 1) / cs::kChunk;
    sh.n_collide_blocks = sh.n_chunks < 1024 ? (sh.n_chunks > 0 ? sh.n_chunks : 1) : 1024;
    sh.scan_tmp_len = cs::step_scan_tmp_len(n_cells, sh.n_chunks);
    int64_t G = ctx->chunks_per_block;
    if (G <= 0) {
        // automatic: about 512 workgroups (2 per compute unit at the fused
        // kernel's occupancy), at most 16 chunks each
        G = sh.n_chunks / 512;
        if (G > 16) G = 16;
    }
    if (G < 1) G = 1;
    sh.chunks_per_block = G;
    sh.n_step_blocks = sh.n_chunks > 0 ? (sh.n_chunks + G - 1) / G : 1;
    sh.n_prep_blocks = cs::fused_prep_blocks(n_cells);
    int64_t nd = (nmin + 63) / 64;
    sh.n_dense_blocks = nd < 1 ? 1 : (nd > 2048 ? 2048 : nd);
    const int64_t strategy = ctx->strategy;
    size_t bytes;
    int64_t status_words = sh.n_prep_blocks;
    if (strategy == CS_STRATEGY_FUSED) {
        bytes = cs::fused_workspace_bytes(sh);
    } else if (strategy == CS_STRATEGY_COMPACT) {
        sh.n_collide_blocks = sh.n_dense_blocks;
        bytes = cs::compact_workspace_bytes(sh);
        status_words += sh.n_chunks;
    } else {
        bytes = cs::step_workspace_bytes(sh);
    }
    cs_status s = ensure_workspace(ctx, bytes, status_words, st);
    if (s != CS_OK) return s;
    cs::StepParams p;
    p.dtype = dtype;
    p.e = electrons;
    p.g = photons;
    p.off_e = off_e;
    p.off_g = off_g;
    p.dt = dt;
    p.density_norm = density_norm;
    p.seed = seed;
    p.step = step;
    p.sampler = sampler;
    p.mlp = mlp;
    p.stats = stats;
    p.events = ctx->timing ? ctx->events : nullptr;
    p.use_device_step = 0;
    hipError_t e;
    if (strategy == CS_STRATEGY_FUSED) {
        cs::FusedBuffers fb;
        cs::carve_fused_buffers(ctx->ws, sh, &fb);
        e = cs::launch_fused(sh, fb, p, st);
    } else if (strategy == CS_STRATEGY_COMPACT) {
        cs::CompactBuffers cb;
        cs::carve_compact_buffers(ctx->ws, sh, &cb);
        e = cs::launch_compact(sh, cb, p, st);
    } else {
        cs::StepBuffers b;
        cs::carve_step_buffers(cs::ws_step_area(ctx->ws), sh, &b);
        e = cs::launch_step(sh, b, p, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_compton_step: launch");
    if (ctx->timing) ctx->timed_step_pending = true;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_set_option(cs_ctx* ctx, cs_option opt, int64_t value) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    switch (opt) {
        case CS_OPT_STRATEGY:
            if (value != CS_STRATEGY_FUSED && value != CS_STRATEGY_MULTI_KERNEL && value != CS_STRATEGY_COMPACT)
                return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: unknown strategy");
            ctx->strategy = value;
            break;
        case CS_OPT_CHUNKS_PER_BLOCK:
            if (value < 0 || value > 4096) return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: chunks per block");
            ctx->chunks_per_block = value;
            break;
        default:
            return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: unknown option");
    }
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_get_option(const cs_ctx* ctx, cs_option opt, int64_t* value) {
    if (!ctx || !value) return CS_ERR_INVALID_ARG;
    switch (opt) {
        case CS_OPT_STRATEGY:
            *value = ctx->strategy;
            return CS_OK;
        case CS_OPT_CHUNKS_PER_BLOCK:
            *value = ctx->chunks_per_block;
            return CS_OK;
        default:
            return CS_ERR_INVALID_ARG;
    }
}

cs_status cs_check_layout(cs_ctx* ctx, const int64_t* off, int64_t n_cells, int64_t n_particles, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!off || n_cells < 0 || n_particles < 0) return fail(ctx, CS_ERR_INVALID_ARG, "cs_check_layout: bad argument");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    cs_status s = ensure_workspace(ctx, 256, 0, st);
    if (s != CS_OK) return s;
    int32_t* flag = (int32_t*)cs::ws_step_area(ctx->ws);
    hipError_t e = cs::launch_check_layout(off, n_cells, n_particles, flag, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_check_layout: launch");
    int32_t h = 0;
    e = hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_check_layout: readback");
    if (h) return fail(ctx, CS_ERR_LAYOUT, "cs_check_layout: offsets are not a valid cell layout");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_sample_plain(cs_ctx* ctx, cs_dtype dtype, const void* x, const void* u, int64_t n, void* mu_out,
                          void* ratio_out, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (dtype != CS_F32 && dtype != CS_F64) return fail(ctx, CS_ERR_INVALID_ARG, "cs_sample_plain: bad dtype");
    if (n < 0) return fail(ctx, CS_ERR_INVALID_ARG, "cs_sample_plain: n < 0");
    if (n > 0 && (!x || !u || !mu_out || !ratio_out))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_sample_plain: NULL array");
    DeviceGuard g(ctx->device);
    hipError_t e = cs::launch_sample_plain(dtype, x, u, n, mu_out, ratio_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_sample_plain: launch");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_set_stage_timing(cs_ctx* ctx, int enable) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (enable) {
        for (auto& ev : ctx->events) {
            if (ev) continue;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(ctx, e, "cs_set_stage_timing: hipEventCreate");
        }
    }
    ctx->timing = enable != 0;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_stage_times(cs_ctx* ctx, float* ms_out, int32_t n, int32_t* n_written) {
    if (!ctx || !ms_out || n < 0) return CS_ERR_INVALID_ARG;
    if (!ctx->timed_step_pending) return fail(ctx, CS_ERR_NOT_READY, "cs_stage_times: no timed step");
    DeviceGuard g(ctx->device);
    hipError_t e = hipEventSynchronize(ctx->events[CS_STAGE_COUNT]);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_stage_times: hipEventSynchronize");
    int32_t m = n < CS_STAGE_COUNT ? n : CS_STAGE_COUNT;
    for (int32_t i = 0; i < m; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]);
        if (e != hipSuccess) return hip_fail(ctx, e, "cs_stage_times: hipEventElapsedTime");
        ms_out[i] = ms;
    }
    if (n_written) *n_written = m;
    ctx->last_error.clear();
    return CS_OK;
}

}  // extern "C"
