// cs_api.hip -- the C ABI of libcompton.so: argument validation, context and
// workspace management, error reporting.  Kernels live in cs_step.hip and
// cs_mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <utility>
#include <new>
#include <string>
#include <vector>

#include "cs_internal.h"

namespace cs {
int64_t step_scan_tmp_len(int64_t n_cells, int64_t n_chunks);
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, int64_t t, hipStream_t st);
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
cs_status ensure_workspace(cs_ctx* ctx, cs::Workspace& w, size_t step_bytes, int64_t status_words,
                           hipStream_t stream) {
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

// Scratch of cs_compton_step_noalloc: a file-scope device array holding one
// step workspace (control block, look-back status words, per-step area).
// Each device that runs the library holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (in host code it
// is a stand-in, not a device address): cs_create looks up the device address
// of its copy on each device once, with that device current, and everything
// after that uses the looked-up address.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
constexpr int64_t kStaticStatusWords = 4096;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxStaticDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxStaticDevices] = {};  // device address of `scratch`, per device

// Look up and initialise the scratch of the current device (once per device;
// called by cs_create with `device` current).  The control block starts at
// epoch 1 and the status words at zero; afterwards every step leaves them
// valid for the next one (their values carry the epoch of the step that wrote
// them), so no call has to clear anything.
cs_status setup_static_scratch(int device, std::string* err) {
    if (device < 0 || device >= kMaxStaticDevices) {
        *err = "cs_create: device index beyond the static scratch table";
        return CS_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return CS_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        *err = std::string("cs_create: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return CS_ERR_HIP;
    }
    const size_t fixed = cs::ws_fixed_bytes(kStaticStatusWords);
    e = hipMemset(ptr, 0, fixed);
    cs::StepControl init = {};
    init.epoch = 1;
    if (e == hipSuccess) e = hipMemcpy(ptr, &init, sizeof(init), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        *err = std::string("cs_create: static scratch initialisation: ") + hipGetErrorString(e);
        return CS_ERR_HIP;
    }
    g_scratch_dev[device] = ptr;
    return CS_OK;
}

void* static_scratch(int device) {
    if (device < 0 || device >= kMaxStaticDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
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
    {
        DeviceGuard g(device);
        if (!g.ok) {
            g_create_error = "cs_create: cannot select device";
            return CS_ERR_HIP;
        }
        const cs_status ss = setup_static_scratch(device, &g_create_error);
        if (ss != CS_OK) return ss;
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
        if (ctx->ws.base || ctx->bin_ws || ctx->pnet_ws || ctx->ntc.cell_ws) (void)hipDeviceSynchronize();
        if (ctx->ws.base) (void)hipFree(ctx->ws.base);
        cs::ntc_free(ctx->ntc);
        if (ctx->bin_ws) (void)hipFree(ctx->bin_ws);
        if (ctx->pnet_ws) (void)hipFree(ctx->pnet_ws);
        for (auto& ev : ctx->events)
            if (ev) (void)hipEventDestroy(ev);
        ctx->events.clear();
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

extern "C++" {
namespace {

std::string who_msg(const char* who, const char* what) { return std::string(who) + ": " + what; }

cs_status validate_step(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons, const int64_t* off_e,
                        const int64_t* off_g, int64_t n_cells, double dt, double density_norm, cs_sampler sampler,
                        const cs_mlp* mlp, int64_t strategy, const char* who) {
    if (dtype != CS_F32 && dtype != CS_F64) return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "bad dtype"));
    if (!species_ok(electrons) || !species_ok(photons))
        return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "species arrays NULL or count negative"));
    if (n_cells < 0) return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "n_cells < 0"));
    if (!off_e || !off_g) return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "offsets NULL"));
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "dt must be > 0"));
    if (!(density_norm >= 0.0) || !std::isfinite(density_norm))
        return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "density_norm must be >= 0"));
    if (n_cells == 0 && (electrons.n != 0 || photons.n != 0))
        return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "particles given but n_cells == 0"));
    if (electrons.n >= (int64_t)1 << 31 || photons.n >= (int64_t)1 << 31)
        return fail(ctx, CS_ERR_UNSUPPORTED, who_msg(who, "a species count >= 2^31"));
    if (n_cells >= (int64_t)1 << 31) return fail(ctx, CS_ERR_UNSUPPORTED, who_msg(who, "n_cells >= 2^31"));
    if (sampler == CS_SAMPLER_PLAIN) {
        if (mlp) return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "PLAIN sampler takes mlp == NULL"));
    } else if (sampler == CS_SAMPLER_MLP_F32 || sampler == CS_SAMPLER_MLP_BF16 || sampler == CS_SAMPLER_MLP_FP8) {
        if (!mlp) return fail(ctx, CS_ERR_NOT_READY, who_msg(who, "network sampler without a network"));
        if (mlp->device != ctx->device)
            return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "network lives on another device"));
        if ((sampler == CS_SAMPLER_MLP_BF16 && !mlp->bf16_ready) || (sampler == CS_SAMPLER_MLP_FP8 && !mlp->fp8_ready))
            return fail(ctx, CS_ERR_NOT_READY, who_msg(who, "network not prepared for this precision"));
        if (strategy == CS_STRATEGY_MULTI_KERNEL || strategy == CS_STRATEGY_PER_CELL)
            return fail(ctx, CS_ERR_UNSUPPORTED, who_msg(who, "the baseline strategies run the plain sampler only"));
    } else {
        return fail(ctx, CS_ERR_INVALID_ARG, who_msg(who, "bad sampler"));
    }
    return CS_OK;
}

struct Plan {
    int64_t strategy = CS_STRATEGY_FUSED;
    cs::StepShape sh = {};
    size_t bytes = 0;
    int64_t status_words = 0;
};

Plan plan_step(int64_t strategy, int64_t chunks_per_block, int64_t pairs_per_lane, int64_t n_cells, int64_t ne,
               int64_t ng, cs_sampler sampler, cs_dtype dtype) {
    Plan pl;
    pl.strategy = strategy;
    cs::StepShape& sh = pl.sh;
    sh.n_cells = n_cells;
    sh.ne = ne;
    sh.ng = ng;
    const int64_t nmin = ne < ng ? ne : ng;
    sh.n_chunks = (nmin + cs::kChunk - 1) / cs::kChunk;
    sh.n_collide_blocks = sh.n_chunks < 1024 ? (sh.n_chunks > 0 ? sh.n_chunks : 1) : 1024;
    sh.scan_tmp_len = cs::step_scan_tmp_len(n_cells, sh.n_chunks);
    int64_t G = chunks_per_block;
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
    sh.pairs_per_lane = pairs_per_lane == 1 || pairs_per_lane == 2 || pairs_per_lane == 4 ? pairs_per_lane : 1;
    // dense collide grid: one lane per accepted pair at most, capped (768
    // four-wave workgroups with the plain sampler, three per compute unit at
    // its occupancy; 512 with a network sampler, whose workgroups each load
    // the network's LDS copy)
    const int64_t dense_threads = cs::compact_collide_threads(sampler);
    const int64_t dense_cap = sampler == CS_SAMPLER_PLAIN ? 768 : 512;
    int64_t nd = (nmin + dense_threads - 1) / dense_threads;
    sh.n_dense_blocks = nd < 1 ? 1 : (nd > dense_cap ? dense_cap : nd);
    pl.status_words = sh.n_prep_blocks;
    if (strategy == CS_STRATEGY_FUSED) {
        pl.bytes = cs::fused_workspace_bytes(sh);
    } else if (strategy == CS_STRATEGY_PER_CELL) {
        sh.n_step_blocks = n_cells > 0 ? n_cells : 1;
        pl.bytes = cs::fused_workspace_bytes(sh);
    } else if (strategy == CS_STRATEGY_COMPACT) {
        // pair workgroups take G consecutive chunks, a multiple of the pairs
        // per lane and at most kCompactMaxChunks (chunk_cell held one entry
        // per lane); automatic: the fewest with which every pair workgroup
        // is resident at once (one round, the waves paced)
        const int64_t ppl = sh.pairs_per_lane;
        int64_t Gc = chunks_per_block > 0 ? chunks_per_block : cs::compact_fit_chunks(dtype, ppl, sh.n_chunks);
        Gc = (Gc + ppl - 1) / ppl * ppl;
        if (Gc < ppl) Gc = ppl;
        if (Gc > cs::kCompactMaxChunks) Gc = cs::kCompactMaxChunks;
        sh.chunks_per_block = Gc;
        sh.n_collide_blocks = sh.n_dense_blocks;
        pl.bytes = cs::compact_workspace_bytes(sh);
        pl.status_words += cs::kPairStatusStride * cs::compact_pair_blocks(sh);
    } else {
        pl.bytes = cs::step_workspace_bytes(sh);
    }
    return pl;
}

hipError_t launch_plan(const Plan& pl, const cs::Workspace& ws, const cs::StepParams& p, hipStream_t st) {
    if (pl.strategy == CS_STRATEGY_FUSED || pl.strategy == CS_STRATEGY_PER_CELL) {
        cs::FusedBuffers fb;
        cs::carve_fused_buffers(ws, pl.sh, &fb);
        return pl.strategy == CS_STRATEGY_FUSED ? cs::launch_fused(pl.sh, fb, p, st) : cs::launch_cell(pl.sh, fb, p, st);
    }
    if (pl.strategy == CS_STRATEGY_COMPACT) {
        cs::CompactBuffers cb;
        cs::carve_compact_buffers(ws, pl.sh, &cb);
        return cs::launch_compact(pl.sh, cb, p, st);
    }
    cs::StepBuffers b;
    cs::carve_step_buffers(cs::ws_step_area(ws), pl.sh, &b);
    return cs::launch_step(pl.sh, b, p, st);
}

cs::StepParams make_params(cs_dtype dtype, cs_species electrons, cs_species photons, const int64_t* off_e,
                           const int64_t* off_g, double dt, double density_norm, uint64_t seed, uint64_t step,
                           cs_sampler sampler, const cs_mlp* mlp, cs_stats* stats, int64_t wide_index) {
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
    p.net = mlp ? mlp->dev() : cs::MlpDev{nullptr, nullptr, nullptr, nullptr, {}};
    p.stats = stats;
    p.events = nullptr;
    p.use_device_step = 0;
    p.wide_index = wide_index ? 1 : 0;
    return p;
}

}  // namespace
}  // extern "C++"

cs_status cs_compton_step(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                          const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                          double density_norm, uint64_t seed, uint64_t step, cs_sampler sampler,
                          const cs_mlp* mlp, cs_stats* stats, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    cs_status s = validate_step(ctx, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm, sampler, mlp,
                                ctx->strategy, "cs_compton_step");
    if (s != CS_OK) return s;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, CS_ERR_HIP, "cs_compton_step: cannot select device");
    hipStream_t st = (hipStream_t)stream;
    const Plan pl = plan_step(ctx->strategy, ctx->chunks_per_block, ctx->pairs_per_lane, n_cells, electrons.n,
                              photons.n, sampler, dtype);
    s = ensure_workspace(ctx, ctx->ws, pl.bytes, pl.status_words, st);
    if (s != CS_OK) return s;
    cs::StepParams p = make_params(dtype, electrons, photons, off_e, off_g, dt, density_norm, seed, step, sampler, mlp,
                                   stats, ctx->wide_index);
    if (ctx->timing) {
        const int64_t slot = ctx->timed_steps % cs::kTimingRing;
        p.events = ctx->events.data() + slot * (CS_STAGE_COUNT + 1);
    }
    const hipError_t e = launch_plan(pl, ctx->ws, p, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_compton_step: launch");
    if (ctx->timing) ctx->timed_steps += 1;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_compton_step_noalloc(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                                  const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                                  double density_norm, uint64_t seed, uint64_t step, cs_sampler sampler,
                                  const cs_mlp* mlp, cs_stats* stats, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    cs_status s = validate_step(ctx, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm, sampler, mlp,
                                CS_STRATEGY_FUSED, "cs_compton_step_noalloc");
    if (s != CS_OK) return s;
    void* base = static_scratch(ctx->device);
    if (!base) return fail(ctx, CS_ERR_NOT_READY, "cs_compton_step_noalloc: no static scratch on this device");
    const Plan pl = plan_step(CS_STRATEGY_FUSED, 0, 0, n_cells, electrons.n, photons.n, sampler, dtype);
    const size_t fixed = cs::ws_fixed_bytes(kStaticStatusWords);
    if (pl.status_words > kStaticStatusWords || pl.bytes > kStaticScratchBytes - fixed) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "cs_compton_step_noalloc: the step needs %zu bytes of scratch, more than the %zu the static "
                      "buffer holds (about 24 bytes per cell and 4 per 256 pairs)",
                      pl.bytes + fixed, kStaticScratchBytes);
        return fail(ctx, CS_ERR_UNSUPPORTED, msg);
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, CS_ERR_HIP, "cs_compton_step_noalloc: cannot select device");
    cs::Workspace w;
    w.base = base;
    w.bytes = kStaticScratchBytes;
    w.status_cap = kStaticStatusWords;
    const cs::StepParams p = make_params(dtype, electrons, photons, off_e, off_g, dt, density_norm, seed, step, sampler,
                                         mlp, stats, 0);
    const hipError_t e = launch_plan(pl, w, p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_compton_step_noalloc: launch");
    ctx->last_error.clear();
    return CS_OK;
}

// ------------------------------------------------------------ graphs

struct cs_graph {
    cs_ctx* ctx = nullptr;
    int device = 0;
    cs::Workspace ws;  // the graph's own workspace (control block, step counter)
    bool is_ntc = false;
    cs::NtcState ntc;  // an NTC graph's own scratch (step word in its head)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C++" {
namespace {

__global__ void k_set_step(cs::StepControl* ctrl, uint64_t step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->step = step;
}

// Bitwise comparison of two buffers (32-bit words): number of differing words.
__global__ void k_count_diff(const uint32_t* a, const uint32_t* b, int64_t n, unsigned long long* count) {
    unsigned long long d = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d += a[i] != b[i] ? 1ull : 0ull;
    if (d) atomicAdd(count, d);
}

void free_graph(cs_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws.base) (void)hipFree(g->ws.base);
    cs::ntc_free(g->ntc);
    delete g;
}

}  // namespace
}  // extern "C++"

cs_status cs_graph_create(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                          const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                          double density_norm, uint64_t seed, cs_sampler sampler, const cs_mlp* mlp,
                          cs_stats* stats, void* stream, cs_graph** out) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!out) return fail(ctx, CS_ERR_INVALID_ARG, "cs_graph_create: out is NULL");
    *out = nullptr;
    if (!stream) return fail(ctx, CS_ERR_INVALID_ARG, "cs_graph_create: the legacy (NULL) stream cannot be captured");
    if (ctx->strategy != CS_STRATEGY_FUSED && ctx->strategy != CS_STRATEGY_COMPACT)
        return fail(ctx, CS_ERR_UNSUPPORTED, "cs_graph_create: graphs capture the fused or compact strategy");
    cs_status s = validate_step(ctx, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm, sampler, mlp,
                                ctx->strategy, "cs_graph_create");
    if (s != CS_OK) return s;
    DeviceGuard dg(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    cs_graph* g = new (std::nothrow) cs_graph();
    if (!g) return fail(ctx, CS_ERR_INVALID_ARG, "cs_graph_create: out of host memory");
    g->ctx = ctx;
    g->device = ctx->device;
    const Plan pl = plan_step(ctx->strategy, ctx->chunks_per_block, ctx->pairs_per_lane, n_cells, electrons.n,
                              photons.n, sampler, dtype);
    s = ensure_workspace(ctx, g->ws, pl.bytes, pl.status_words, st);
    if (s != CS_OK) {
        free_graph(g);
        return s;
    }
    cs::StepParams p = make_params(dtype, electrons, photons, off_e, off_g, dt, density_norm, seed, 0, sampler, mlp,
                                   stats, ctx->wide_index);
    p.use_device_step = 1;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, e, "cs_graph_create: hipStreamBeginCapture");
    }
    const hipError_t le = launch_plan(pl, g->ws, p, st);
    e = hipStreamEndCapture(st, &g->graph);
    if (le != hipSuccess || e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, le != hipSuccess ? le : e, "cs_graph_create: capture");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, e, "cs_graph_create: hipGraphInstantiate");
    }
    *out = g;
    ctx->last_error.clear();
    return CS_OK;
}

static cs_status validate_ntc(cs_ctx* ctx, cs_dtype dtype, const cs_species& electrons, const cs_species& photons,
                              const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                              double density_norm, const char* what);

cs_status cs_ntc_graph_create(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                              const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                              double density_norm, uint64_t seed, int64_t max_candidates, cs_stats* stats,
                              void* stream, cs_graph** out) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!out) return fail(ctx, CS_ERR_INVALID_ARG, "cs_ntc_graph_create: out is NULL");
    *out = nullptr;
    if (!stream)
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_ntc_graph_create: the legacy (NULL) stream cannot be captured");
    cs_status s = validate_ntc(ctx, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm,
                               "cs_ntc_graph_create");
    if (s != CS_OK) return s;
    if (max_candidates < 1 || max_candidates > ((int64_t)1 << 31) - 2)
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_ntc_graph_create: max_candidates must be in [1, 2^31 - 2]");
    if (n_cells == 0 && (electrons.n != 0 || photons.n != 0))
        return fail(ctx, CS_ERR_LAYOUT, "cs_ntc_graph_create: particles but no cells");
    DeviceGuard dg(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    cs_graph* g = new (std::nothrow) cs_graph();
    if (!g) return fail(ctx, CS_ERR_INVALID_ARG, "cs_ntc_graph_create: out of host memory");
    g->ctx = ctx;
    g->device = ctx->device;
    g->is_ntc = true;
    hipError_t e = cs::ntc_prepare_graph(g->ntc, n_cells, max_candidates, electrons.n, photons.n, st);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, e, "cs_ntc_graph_create: scratch");
    }
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, e, "cs_ntc_graph_create: hipStreamBeginCapture");
    }
    const hipError_t le =
        cs::ntc_capture(g->ntc, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm, seed, stats, st);
    e = hipStreamEndCapture(st, &g->graph);
    if (le != hipSuccess || e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, le != hipSuccess ? le : e, "cs_ntc_graph_create: capture");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_graph(g);
        return hip_fail(ctx, e, "cs_ntc_graph_create: hipGraphInstantiate");
    }
    *out = g;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_graph_set_step(cs_graph* g, uint64_t step, void* stream) {
    if (!g) return CS_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    hipError_t e = hipSuccess;
    if (g->is_ntc) {
        e = cs::ntc_set_step(g->ntc, step, (hipStream_t)stream);
    } else {
        k_set_step<<<1, 64, 0, (hipStream_t)stream>>>(cs::ws_control(g->ws), step);
        e = hipGetLastError();
    }
    return e == hipSuccess ? CS_OK : hip_fail(g->ctx, e, "cs_graph_set_step");
}

cs_status cs_graph_launch(cs_graph* g, void* stream) {
    if (!g) return CS_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    return e == hipSuccess ? CS_OK : hip_fail(g->ctx, e, "cs_graph_launch");
}

cs_status cs_graph_destroy(cs_graph* g) {
    if (!g) return CS_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    (void)hipDeviceSynchronize();
    free_graph(g);
    return CS_OK;
}

// ---------------------------------------------------------- autotune

cs_status cs_autotune(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons, const int64_t* off_e,
                      const int64_t* off_g, int64_t n_cells, double dt, double density_norm, uint64_t seed,
                      uint64_t step, cs_sampler sampler, const cs_mlp* mlp, int32_t reps, cs_tune_result* out,
                      void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (reps < 1 || reps > 100) return fail(ctx, CS_ERR_INVALID_ARG, "cs_autotune: reps must be in [1, 100]");
    cs_status s = validate_step(ctx, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm, sampler, mlp,
                                CS_STRATEGY_FUSED, "cs_autotune");
    if (s != CS_OK) return s;
    DeviceGuard dg(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t sb = dtype == CS_F64 ? 8 : 4;
    const size_t be = sb * (size_t)electrons.n, bg = sb * (size_t)photons.n;
    const size_t bytes_state = 4 * (be + bg);
    // private state, a reference result, a stats block and a diff counter
    char* buf = nullptr;
    const size_t al = 256;
    const size_t state_al = (bytes_state + al - 1) / al * al;
    hipError_t e = hipMalloc(&buf, 2 * state_al + 2 * al);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_autotune: hipMalloc");
    char* state = buf;
    char* ref = buf + state_al;
    cs_stats* st_dev = (cs_stats*)(buf + 2 * state_al);
    unsigned long long* diff = (unsigned long long*)(buf + 2 * state_al + al);
    const void* src[8] = {electrons.x, electrons.y, electrons.z, electrons.w, photons.x, photons.y, photons.z, photons.w};
    const size_t len[8] = {be, be, be, be, bg, bg, bg, bg};
    cs_species pe = {}, pg = {};
    {
        size_t o = 0;
        void** dst[8] = {&pe.x, &pe.y, &pe.z, &pe.w, &pg.x, &pg.y, &pg.z, &pg.w};
        for (int i = 0; i < 8; ++i) {
            *dst[i] = state + o;
            o += len[i];
        }
        pe.n = electrons.n;
        pg.n = photons.n;
    }
    auto restore = [&]() -> hipError_t {
        size_t o = 0;
        for (int i = 0; i < 8; ++i) {
            if (len[i]) {
                const hipError_t r = hipMemcpyAsync(state + o, src[i], len[i], hipMemcpyDeviceToDevice, st);
                if (r != hipSuccess) return r;
            }
            o += len[i];
        }
        return hipSuccess;
    };
    int32_t cand_s[CS_TUNE_MAX], cand_g[CS_TUNE_MAX], cand_p[CS_TUNE_MAX];
    int n_cand = 0;
    for (int gpb : {4, 8, 16, 32}) {
        cand_s[n_cand] = CS_STRATEGY_FUSED;
        cand_p[n_cand] = 0;
        cand_g[n_cand++] = gpb;
    }
    // compact: (pairs per lane, chunks per pair workgroup), plus for one and
    // two pairs per lane the fewest chunks with which the pair grid is
    // resident at once
    const int64_t n_chunks_tune = ((electrons.n < photons.n ? electrons.n : photons.n) + 255) / 256;
    for (const auto& pg : {std::pair<int, int>{1, 4}, {1, 8}, {1, 16}, {2, 8}, {2, 16}}) {
        cand_s[n_cand] = CS_STRATEGY_COMPACT;
        cand_p[n_cand] = pg.first;
        cand_g[n_cand++] = pg.second;
    }
    for (int ppl : {1, 2}) {
        const int g = (int)cs::compact_fit_chunks(dtype, ppl, n_chunks_tune);
        bool dup = false;
        for (int c = 0; c < n_cand; ++c) dup = dup || (cand_s[c] == CS_STRATEGY_COMPACT && cand_p[c] == ppl && cand_g[c] == g);
        if (dup) continue;
        cand_s[n_cand] = CS_STRATEGY_COMPACT;
        cand_p[n_cand] = ppl;
        cand_g[n_cand++] = g;
    }
    float ms_best = 0.f;
    int best = -1;
    float ms_all[CS_TUNE_MAX] = {};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    const int64_t saved_s = ctx->strategy, saved_g = ctx->chunks_per_block, saved_p = ctx->pairs_per_lane;
    cs_status rs = CS_OK;
    for (int c = 0; c < n_cand && e == hipSuccess && rs == CS_OK; ++c) {
        const Plan pl = plan_step(cand_s[c], cand_g[c], cand_p[c], n_cells, electrons.n, photons.n, sampler, dtype);
        rs = ensure_workspace(ctx, ctx->ws, pl.bytes, pl.status_words, st);
        if (rs != CS_OK) break;
        const cs::StepParams p = make_params(dtype, pe, pg, off_e, off_g, dt, density_norm, seed, step, sampler, mlp,
                                             st_dev, ctx->wide_index);
        // correctness: one step from the caller's state, compared bitwise
        e = restore();
        if (e == hipSuccess) e = launch_plan(pl, ctx->ws, p, st);
        if (e != hipSuccess) break;
        if (c == 0) {
            e = hipMemcpyAsync(ref, state, bytes_state, hipMemcpyDeviceToDevice, st);
        } else {
            e = hipMemsetAsync(diff, 0, sizeof(unsigned long long), st);
            if (e == hipSuccess && bytes_state >= 4) {
                k_count_diff<<<1024, 256, 0, st>>>((const uint32_t*)state, (const uint32_t*)ref,
                                                   (int64_t)(bytes_state / 4), diff);
                e = hipGetLastError();
            }
            unsigned long long nd = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&nd, diff, sizeof(nd), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e == hipSuccess && nd != 0) {
                rs = fail(ctx, CS_ERR_HIP, "cs_autotune: strategies disagree (library defect)");
                break;
            }
        }
        if (e != hipSuccess) break;
        // timing: each rep from the caller's state
        float t[100];
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = restore();
            if (e == hipSuccess) e = hipEventRecord(ev0, st);
            if (e == hipSuccess) e = launch_plan(pl, ctx->ws, p, st);
            if (e == hipSuccess) e = hipEventRecord(ev1, st);
            if (e == hipSuccess) e = hipEventSynchronize(ev1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t[r], ev0, ev1);
        }
        if (e != hipSuccess) break;
        std::sort(t, t + reps);
        ms_all[c] = t[reps / 2];
        if (best < 0 || ms_all[c] < ms_best) {
            best = c;
            ms_best = ms_all[c];
        }
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (rs != CS_OK || e != hipSuccess) {
        ctx->strategy = saved_s;
        ctx->chunks_per_block = saved_g;
        ctx->pairs_per_lane = saved_p;
        return rs != CS_OK ? rs : hip_fail(ctx, e, "cs_autotune");
    }
    ctx->strategy = cand_s[best];
    ctx->chunks_per_block = cand_g[best];
    ctx->pairs_per_lane = cand_p[best];
    if (out) {
        *out = cs_tune_result{};
        out->n = n_cand;
        out->best = best;
        for (int c = 0; c < n_cand; ++c) {
            out->strategy[c] = cand_s[c];
            out->chunks_per_block[c] = cand_g[c];
            out->pairs_per_lane[c] = cand_p[c];
            out->ms[c] = ms_all[c];
        }
    }
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_set_option(cs_ctx* ctx, cs_option opt, int64_t value) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    switch (opt) {
        case CS_OPT_STRATEGY:
            if (value != CS_STRATEGY_FUSED && value != CS_STRATEGY_MULTI_KERNEL && value != CS_STRATEGY_COMPACT &&
                value != CS_STRATEGY_PER_CELL)
                return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: unknown strategy");
            ctx->strategy = value;
            break;
        case CS_OPT_CHUNKS_PER_BLOCK:
            if (value < 0 || value > 4096) return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: chunks per block");
            ctx->chunks_per_block = value;
            break;
        case CS_OPT_PAIRS_PER_LANE:
            if (value != 0 && value != 1 && value != 2 && value != 4)
                return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: pairs per lane must be 0, 1, 2 or 4");
            ctx->pairs_per_lane = value;
            break;
        case CS_OPT_WIDE_INDEX:
            if (value != 0 && value != 1) return fail(ctx, CS_ERR_INVALID_ARG, "cs_set_option: wide index must be 0 or 1");
            ctx->wide_index = value;
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
        case CS_OPT_PAIRS_PER_LANE:
            *value = ctx->pairs_per_lane;
            return CS_OK;
        case CS_OPT_WIDE_INDEX:
            *value = ctx->wide_index;
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
    cs_status s = ensure_workspace(ctx, ctx->ws, 256, 0, st);
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

cs_status cs_pair_x(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons, int64_t n, double* x_out,
                    void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if ((dtype != CS_F32 && dtype != CS_F64) || n < 0 || n > electrons.n || n > photons.n ||
        (n > 0 && (!electrons.x || !electrons.y || !electrons.z || !photons.x || !photons.y || !photons.z || !x_out)))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_pair_x: bad arguments");
    DeviceGuard g(ctx->device);
    hipError_t e = cs::launch_pair_x(dtype, electrons, photons, n, x_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_pair_x: launch");
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

cs_status cs_bin_particles(cs_ctx* ctx, cs_dtype dtype, const int32_t* cell, cs_species in, cs_species out,
                           int64_t* off, int64_t n_cells, int64_t* n_invalid, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (dtype != CS_F32 && dtype != CS_F64) return fail(ctx, CS_ERR_INVALID_ARG, "cs_bin_particles: bad dtype");
    const int64_t n = in.n;
    if (n < 0 || n >= ((int64_t)1 << 31) || out.n != n)
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_bin_particles: need 0 <= in.n = out.n < 2^31");
    if (n_cells < 0 || n_cells >= ((int64_t)1 << 31) - 1)
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_bin_particles: need 0 <= n_cells < 2^31 - 1");
    if (!off) return fail(ctx, CS_ERR_INVALID_ARG, "cs_bin_particles: NULL offsets");
    if (n > 0 && (!cell || !in.x || !in.y || !in.z || !in.w || !out.x || !out.y || !out.z || !out.w))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_bin_particles: NULL array");
    if (n > 0) {
        const void* ins[4] = {in.x, in.y, in.z, in.w};
        const void* outs[4] = {out.x, out.y, out.z, out.w};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (ins[a] == outs[b]) return fail(ctx, CS_ERR_INVALID_ARG, "cs_bin_particles: in and out overlap");
    }
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t want = cs::bin_workspace_bytes(n);
    if (ctx->bin_bytes < want) {
        // no queued binning may still use the old scratch
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(ctx, e, "cs_bin_particles: stream synchronize");
        if (ctx->bin_ws) {
            e = hipFree(ctx->bin_ws);
            ctx->bin_ws = nullptr;
            ctx->bin_bytes = 0;
            if (e != hipSuccess) return hip_fail(ctx, e, "cs_bin_particles: hipFree");
        }
        const size_t grow = want + want / 4;
        e = hipMalloc(&ctx->bin_ws, grow);
        if (e != hipSuccess) {
            ctx->bin_ws = nullptr;
            return hip_fail(ctx, e, "cs_bin_particles: hipMalloc");
        }
        ctx->bin_bytes = grow;
    }
    void* const outp[4] = {out.x, out.y, out.z, out.w};
    const void* const inp[4] = {in.x, in.y, in.z, in.w};
    hipError_t e = cs::launch_bin(dtype, cell, n, n_cells, inp, outp, off, n_invalid, ctx->bin_ws, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_bin_particles: launch");
    ctx->last_error.clear();
    return CS_OK;
}

static cs_status validate_ntc(cs_ctx* ctx, cs_dtype dtype, const cs_species& electrons, const cs_species& photons,
                              const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                              double density_norm, const char* what) {
    const std::string w(what);
    if (dtype != CS_F32 && dtype != CS_F64) return fail(ctx, CS_ERR_INVALID_ARG, w + ": bad dtype");
    if (electrons.n < 0 || photons.n < 0 || n_cells < 0 || n_cells >= ((int64_t)1 << 31) - 1)
        return fail(ctx, CS_ERR_INVALID_ARG, w + ": negative size or n_cells >= 2^31 - 1");
    if (electrons.n >= ((int64_t)1 << 31) || photons.n >= ((int64_t)1 << 31))
        return fail(ctx, CS_ERR_UNSUPPORTED, w + ": a species count >= 2^31");
    if ((electrons.n > 0 && (!electrons.x || !electrons.y || !electrons.z || !electrons.w)) ||
        (photons.n > 0 && (!photons.x || !photons.y || !photons.z || !photons.w)) || !off_e || !off_g)
        return fail(ctx, CS_ERR_INVALID_ARG, w + ": NULL array");
    if (!(dt > 0.0) || !std::isfinite(dt) || !(density_norm >= 0.0) || !std::isfinite(density_norm))
        return fail(ctx, CS_ERR_INVALID_ARG, w + ": need finite dt > 0 and density_norm >= 0");
    return CS_OK;
}

cs_status cs_ntc_step(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons, const int64_t* off_e,
                      const int64_t* off_g, int64_t n_cells, double dt, double density_norm, uint64_t seed,
                      uint64_t step, cs_stats* stats, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    const cs_status vs =
        validate_ntc(ctx, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm, "cs_ntc_step");
    if (vs != CS_OK) return vs;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    cs::NtcOutcome out = cs::NtcOutcome::kOk;
    const hipError_t e = cs::ntc_step(ctx->ntc, dtype, electrons, photons, off_e, off_g, n_cells, dt, density_norm,
                                      seed, step, stats, st, &out);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_ntc_step");
    if (out == cs::NtcOutcome::kLayout) return fail(ctx, CS_ERR_LAYOUT, "cs_ntc_step: offsets are not a valid layout");
    if (out == cs::NtcOutcome::kTooMany)
        return fail(ctx, CS_ERR_UNSUPPORTED, "cs_ntc_step: 2^31 - 1 or more candidates in one step");
    ctx->last_error.clear();
    return CS_OK;
}

// Grow a context scratch buffer to `want` bytes (synchronises `stream` first
// so that no queued kernel still uses the old one).
static cs_status grow_scratch(cs_ctx* ctx, void** buf, size_t* bytes, size_t want, hipStream_t st,
                              const char* what) {
    if (*bytes >= want) return CS_OK;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    if (*buf) {
        e = hipFree(*buf);
        *buf = nullptr;
        *bytes = 0;
        if (e != hipSuccess) return hip_fail(ctx, e, what);
    }
    const size_t grow = want + want / 4;
    e = hipMalloc(buf, grow);
    if (e != hipSuccess) {
        *buf = nullptr;
        return hip_fail(ctx, e, what);
    }
    *bytes = grow;
    return CS_OK;
}

cs_status cs_pnet_target(cs_ctx* ctx, const float* in, int64_t n, float* y, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && (!in || !y))) return fail(ctx, CS_ERR_INVALID_ARG, "cs_pnet_target: bad arguments");
    DeviceGuard g(ctx->device);
    hipError_t e = cs::launch_pnet_target(in, n, y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_pnet_target: launch");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_pnet_forward(cs_ctx* ctx, const float* params, const float* in, int64_t n, float* y, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (n < 0 || !params || (n > 0 && (!in || !y)))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_pnet_forward: bad arguments");
    DeviceGuard g(ctx->device);
    hipError_t e = cs::launch_pnet_forward(params, in, n, y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_pnet_forward: launch");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_pnet_grad(cs_ctx* ctx, const float* params, const float* in, const float* target, int64_t n,
                       cs_loss loss, float* grad_out, float* loss_out, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (n < 0 || !params || !grad_out || (n > 0 && (!in || !target)) || (loss != CS_LOSS_MSE && loss != CS_LOSS_MAE))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_pnet_grad: bad arguments");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    cs_status rs = grow_scratch(ctx, &ctx->pnet_ws, &ctx->pnet_bytes, cs::pnet_workspace_bytes(n), st,
                                "cs_pnet_grad: scratch");
    if (rs != CS_OK) return rs;
    hipError_t e =
        cs::launch_pnet_grad(params, in, target, n, loss == CS_LOSS_MAE ? 1 : 0, grad_out, loss_out, ctx->pnet_ws, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_pnet_grad: launch");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_pnet_adam(cs_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t t, float lr,
                       void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!params || !grad || !m || !v || t < 1 || !(lr > 0.0f))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_pnet_adam: bad arguments");
    DeviceGuard g(ctx->device);
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipError_t e = cs::launch_pnet_adam(params, grad, m, v, lr, bc1, bc2, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_pnet_adam: launch");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_set_stage_timing(cs_ctx* ctx, int enable) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (enable && ctx->events.empty()) {
        ctx->events.assign((size_t)cs::kTimingRing * (CS_STAGE_COUNT + 1), nullptr);
        for (auto& ev : ctx->events) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(ctx, e, "cs_set_stage_timing: hipEventCreate");
        }
    }
    ctx->timing = enable != 0;
    ctx->timed_steps = 0;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_stage_times(cs_ctx* ctx, float* ms_out, int32_t n, int32_t* n_written) {
    if (!ctx || !ms_out || n < 0) return CS_ERR_INVALID_ARG;
    if (ctx->timed_steps == 0) return fail(ctx, CS_ERR_NOT_READY, "cs_stage_times: no timed step");
    DeviceGuard g(ctx->device);
    const int64_t n_rec = ctx->timed_steps < cs::kTimingRing ? ctx->timed_steps : cs::kTimingRing;
    const int64_t last = (ctx->timed_steps - 1) % cs::kTimingRing;
    constexpr int kEv = CS_STAGE_COUNT + 1;
    hipError_t e = hipEventSynchronize(ctx->events[last * kEv + CS_STAGE_COUNT]);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_stage_times: hipEventSynchronize");
    const int32_t m = n < CS_STAGE_COUNT ? n : CS_STAGE_COUNT;
    double acc[CS_STAGE_COUNT] = {};
    for (int64_t slot = 0; slot < n_rec; ++slot) {
        for (int32_t i = 0; i < m; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ctx->events[slot * kEv + i], ctx->events[slot * kEv + i + 1]);
            if (e != hipSuccess) return hip_fail(ctx, e, "cs_stage_times: hipEventElapsedTime");
            acc[i] += ms;
        }
    }
    for (int32_t i = 0; i < m; ++i) ms_out[i] = (float)(acc[i] / (double)n_rec);
    if (n_written) *n_written = m;
    ctx->timed_steps = 0;
    ctx->last_error.clear();
    return CS_OK;
}

// ---------------------------------------------------------------- network

extern "C++" {
namespace {

const int32_t kWidths[6] = {2, 64, 64, 64, 64, 2};
// file versions: 001 (default x range), 002 (x range stored after the Adam step)
const char kMagic1[8] = {'C', 'S', 'M', 'L', 'P', '0', '0', '1'};
const char kMagic2[8] = {'C', 'S', 'M', 'L', 'P', '0', '0', '2'};

bool domain_ok(double x_min, double x_max) {
    return std::isfinite(x_min) && std::isfinite(x_max) && x_min > 0.0 && x_max > x_min;
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h) {
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

void mlp_free(cs_mlp* m) {
    if (!m) return;
    (void)hipFree(m->params);
    (void)hipFree(m->adam_m);
    (void)hipFree(m->adam_v);
    (void)hipFree(m->frag_bf16);
    (void)hipFree(m->frag_fp8);
    (void)hipFree(m->fp8_scales);
    (void)hipFree(m->work);
    delete m;
}

cs_status mlp_alloc(cs_ctx* ctx, cs_mlp** out) {
    cs_mlp* m = new (std::nothrow) cs_mlp();
    if (!m) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_create: out of host memory");
    m->device = ctx->device;
    const size_t pb = sizeof(float) * cs::kMlpParams;
    hipError_t e = hipMalloc(&m->params, pb);
    if (e == hipSuccess) e = hipMalloc(&m->adam_m, pb);
    if (e == hipSuccess) e = hipMalloc(&m->adam_v, pb);
    if (e == hipSuccess) e = hipMalloc(&m->frag_bf16, (size_t)cs::kFragCount * 16);
    if (e == hipSuccess) e = hipMalloc(&m->frag_fp8, (size_t)cs::kFragCount * 8);
    if (e == hipSuccess) e = hipMalloc(&m->fp8_scales, 16 * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->params, 0, pb);
    if (e == hipSuccess) e = hipMemset(m->adam_m, 0, pb);
    if (e == hipSuccess) e = hipMemset(m->adam_v, 0, pb);
    if (e == hipSuccess) e = hipMemset(m->fp8_scales, 0, 16 * sizeof(float));
    if (e != hipSuccess) {
        mlp_free(m);
        return hip_fail(ctx, e, "cs_mlp_create: device allocation");
    }
    *out = m;
    return CS_OK;
}

bool widths_ok(const int32_t* w, int32_t n) {
    if (!w || n != 6) return false;
    for (int i = 0; i < 6; ++i)
        if (w[i] != kWidths[i]) return false;
    return true;
}

cs_status mlp_work(cs_ctx* ctx, cs_mlp* m, size_t bytes, hipStream_t st) {
    if (m->work_bytes >= bytes) return CS_OK;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess && m->work) e = hipFree(m->work);
    m->work = nullptr;
    m->work_bytes = 0;
    if (e == hipSuccess) e = hipMalloc(&m->work, bytes);
    if (e != hipSuccess) return hip_fail(ctx, e, "network workspace");
    m->work_bytes = bytes;
    return CS_OK;
}

cs_status check_precision(cs_ctx* ctx, const cs_mlp* m, cs_sampler p, const char* who) {
    if (p == CS_SAMPLER_MLP_F32) return CS_OK;
    if (p == CS_SAMPLER_MLP_BF16) {
        if (!m->bf16_ready) return fail(ctx, CS_ERR_NOT_READY, std::string(who) + ": BF16 weights not prepared");
        return CS_OK;
    }
    if (p == CS_SAMPLER_MLP_FP8) {
        if (!m->fp8_ready) return fail(ctx, CS_ERR_NOT_READY, std::string(who) + ": FP8 weights not prepared");
        return CS_OK;
    }
    return fail(ctx, CS_ERR_INVALID_ARG, std::string(who) + ": bad precision");
}

}  // namespace
}  // extern "C++"

cs_status cs_mlp_create(cs_ctx* ctx, const int32_t* widths, int32_t n_widths, const float* init_params_host,
                        cs_mlp** out) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!out) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_create: out is NULL");
    *out = nullptr;
    if (!widths || n_widths < 2) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_create: widths");
    if (!widths_ok(widths, n_widths))
        return fail(ctx, CS_ERR_UNSUPPORTED, "cs_mlp_create: kernels take widths {2, 64, 64, 64, 64, 2} only");
    DeviceGuard g(ctx->device);
    cs_mlp* m = nullptr;
    cs_status s = mlp_alloc(ctx, &m);
    if (s != CS_OK) return s;
    if (init_params_host) {
        hipError_t e = hipMemcpy(m->params, init_params_host, sizeof(float) * cs::kMlpParams, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            mlp_free(m);
            return hip_fail(ctx, e, "cs_mlp_create: parameter upload");
        }
    }
    *out = m;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_mlp_destroy(cs_mlp* mlp) {
    if (!mlp) return CS_ERR_INVALID_ARG;
    DeviceGuard g(mlp->device);
    (void)hipDeviceSynchronize();
    mlp_free(mlp);
    return CS_OK;
}

int64_t cs_mlp_num_params(const cs_mlp* mlp) { return mlp ? (int64_t)cs::kMlpParams : -1; }

cs_status cs_mlp_set_params(cs_mlp* mlp, const float* host, int64_t n) {
    if (!mlp || !host || n != cs::kMlpParams) return CS_ERR_INVALID_ARG;
    DeviceGuard g(mlp->device);
    if (hipDeviceSynchronize() != hipSuccess) return CS_ERR_HIP;
    if (hipMemcpy(mlp->params, host, sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess) return CS_ERR_HIP;
    mlp->bf16_ready = mlp->fp8_ready = false;
    return CS_OK;
}

cs_status cs_mlp_get_params(const cs_mlp* mlp, float* host, int64_t n) {
    if (!mlp || !host || n != cs::kMlpParams) return CS_ERR_INVALID_ARG;
    DeviceGuard g(mlp->device);
    if (hipDeviceSynchronize() != hipSuccess) return CS_ERR_HIP;
    if (hipMemcpy(host, mlp->params, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess) return CS_ERR_HIP;
    return CS_OK;
}

cs_status cs_mlp_set_domain(cs_mlp* mlp, double x_min, double x_max) {
    if (!mlp || !domain_ok(x_min, x_max)) return CS_ERR_INVALID_ARG;
    DeviceGuard g(mlp->device);
    if (hipDeviceSynchronize() != hipSuccess) return CS_ERR_HIP;  // queued work keeps the old range
    mlp->x_min = x_min;
    mlp->x_max = x_max;
    mlp->fp8_ready = false;  // the FP8 input scales were calibrated on the old features
    return CS_OK;
}

cs_status cs_mlp_get_domain(const cs_mlp* mlp, double* x_min, double* x_max) {
    if (!mlp || !x_min || !x_max) return CS_ERR_INVALID_ARG;
    *x_min = mlp->x_min;
    *x_max = mlp->x_max;
    return CS_OK;
}

cs_status cs_mlp_save(const cs_mlp* mlp, const char* path) {
    if (!mlp || !path) return CS_ERR_INVALID_ARG;
    DeviceGuard g(mlp->device);
    const size_t n = cs::kMlpParams;
    std::string buf;
    std::vector<float> p(n), m(n), v(n);
    if (hipDeviceSynchronize() != hipSuccess) return CS_ERR_HIP;
    if (hipMemcpy(p.data(), mlp->params, 4 * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(m.data(), mlp->adam_m, 4 * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(v.data(), mlp->adam_v, 4 * n, hipMemcpyDeviceToHost) != hipSuccess)
        return CS_ERR_HIP;
    const int32_t nw = 6;
    const int64_t np = (int64_t)n, t = mlp->adam_t;
    buf.append(kMagic2, 8);
    buf.append((const char*)&nw, 4);
    buf.append((const char*)kWidths, 24);
    buf.append((const char*)&np, 8);
    buf.append((const char*)&t, 8);
    buf.append((const char*)&mlp->x_min, 8);
    buf.append((const char*)&mlp->x_max, 8);
    buf.append((const char*)p.data(), 4 * n);
    buf.append((const char*)m.data(), 4 * n);
    buf.append((const char*)v.data(), 4 * n);
    const uint64_t h = fnv1a(buf.data(), buf.size(), 1469598103934665603ull);
    buf.append((const char*)&h, 8);
    FILE* f = fopen(path, "wb");
    if (!f) return CS_ERR_IO;
    const size_t wr = fwrite(buf.data(), 1, buf.size(), f);
    const int cl = fclose(f);
    return (wr == buf.size() && cl == 0) ? CS_OK : CS_ERR_IO;
}

cs_status cs_mlp_load(cs_ctx* ctx, const char* path, cs_mlp** out) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!path || !out) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_load: NULL argument");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(ctx, CS_ERR_IO, std::string("cs_mlp_load: cannot open ") + path);
    std::string buf;
    char tmp[65536];
    size_t r;
    while ((r = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.append(tmp, r);
    fclose(f);
    const size_t n = cs::kMlpParams;
    if (buf.size() < 8) return fail(ctx, CS_ERR_IO, "cs_mlp_load: wrong file size");
    const bool v2 = memcmp(buf.data(), kMagic2, 8) == 0;
    if (!v2 && memcmp(buf.data(), kMagic1, 8) != 0) return fail(ctx, CS_ERR_IO, "cs_mlp_load: bad magic");
    const size_t head = 8 + 4 + 24 + 8 + 8 + (v2 ? 16 : 0);
    const size_t need = head + 3 * 4 * n + 8;
    if (buf.size() != need) return fail(ctx, CS_ERR_IO, "cs_mlp_load: wrong file size");
    uint64_t h;
    memcpy(&h, buf.data() + need - 8, 8);
    if (fnv1a(buf.data(), need - 8, 1469598103934665603ull) != h) return fail(ctx, CS_ERR_IO, "cs_mlp_load: checksum");
    int32_t nw;
    int32_t w[6];
    int64_t np, t;
    memcpy(&nw, buf.data() + 8, 4);
    memcpy(w, buf.data() + 12, 24);
    memcpy(&np, buf.data() + 36, 8);
    memcpy(&t, buf.data() + 44, 8);
    if (!widths_ok(w, nw) || np != (int64_t)n) return fail(ctx, CS_ERR_IO, "cs_mlp_load: unsupported widths");
    double x_min = CS_MLP_X_MIN, x_max = CS_MLP_X_MAX;
    if (v2) {
        memcpy(&x_min, buf.data() + 52, 8);
        memcpy(&x_max, buf.data() + 60, 8);
        if (!domain_ok(x_min, x_max)) return fail(ctx, CS_ERR_IO, "cs_mlp_load: bad x range");
    }
    DeviceGuard g(ctx->device);
    cs_mlp* m = nullptr;
    cs_status s = mlp_alloc(ctx, &m);
    if (s != CS_OK) return s;
    m->x_min = x_min;
    m->x_max = x_max;
    const char* base = buf.data() + head;
    hipError_t e = hipMemcpy(m->params, base, 4 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->adam_m, base + 4 * n, 4 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->adam_v, base + 8 * n, 4 * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        mlp_free(m);
        return hip_fail(ctx, e, "cs_mlp_load: upload");
    }
    m->adam_t = t;
    *out = m;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_mlp_quantize(cs_ctx* ctx, cs_mlp* mlp, cs_sampler precision, const float* calib_x,
                          const float* calib_u, int64_t n, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!mlp) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_quantize: NULL network");
    if (precision == CS_SAMPLER_MLP_F32) return CS_OK;
    if (precision != CS_SAMPLER_MLP_BF16 && precision != CS_SAMPLER_MLP_FP8)
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_quantize: bad precision");
    if (precision == CS_SAMPLER_MLP_FP8 && (!calib_x || !calib_u || n <= 0))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_quantize: FP8 needs calibration samples");
    DeviceGuard g(mlp->device);
    hipError_t e = cs::launch_mlp_quantize(mlp->params, mlp->dev().dom, mlp->frag_bf16, mlp->frag_fp8, mlp->fp8_scales,
                                           precision,
                                           calib_x, calib_u, n, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_mlp_quantize: launch");
    if (precision == CS_SAMPLER_MLP_BF16)
        mlp->bf16_ready = true;
    else
        mlp->fp8_ready = true;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_mlp_forward(cs_ctx* ctx, const cs_mlp* mlp, cs_sampler precision, const float* x, const float* u,
                         int64_t n, float* y_out, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!mlp || n < 0 || (n > 0 && (!x || !u || !y_out)))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_forward: bad argument");
    cs_status s = check_precision(ctx, mlp, precision, "cs_mlp_forward");
    if (s != CS_OK) return s;
    DeviceGuard g(mlp->device);
    hipError_t e = cs::launch_mlp_forward(mlp->dev(), precision, x, u, n, y_out, nullptr, nullptr, nullptr,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_mlp_forward: launch");
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_mlp_sample(cs_ctx* ctx, const cs_mlp* mlp, cs_sampler precision, const float* x, const float* u,
                        int64_t n, float* mu_out, float* ratio_out, uint8_t* fallback_mask, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!mlp || n < 0 || (n > 0 && (!x || !u || !mu_out || !ratio_out)))
        return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_sample: bad argument");
    cs_status s = check_precision(ctx, mlp, precision, "cs_mlp_sample");
    if (s != CS_OK) return s;
    DeviceGuard g(mlp->device);
    hipError_t e = cs::launch_mlp_forward(mlp->dev(), precision, x, u, n, nullptr, mu_out, ratio_out, fallback_mask,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_mlp_sample: launch");
    ctx->last_error.clear();
    return CS_OK;
}

static cs_status mlp_grad_impl(cs_ctx* ctx, cs_mlp* mlp, const float* x, const float* u, const float* mu_t,
                               const float* r_t, int64_t n, cs_loss loss, float* grad_out, float* loss_out,
                               bool adam, float lr, void* stream, const char* who) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!mlp || n <= 0 || !x || !u || !mu_t || !r_t)
        return fail(ctx, CS_ERR_INVALID_ARG, std::string(who) + ": bad argument");
    if (loss != CS_LOSS_MSE && loss != CS_LOSS_MAE) return fail(ctx, CS_ERR_INVALID_ARG, std::string(who) + ": loss");
    if (adam && !(lr > 0.0f)) return fail(ctx, CS_ERR_INVALID_ARG, std::string(who) + ": lr must be > 0");
    DeviceGuard g(mlp->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t blocks = cs::mlp_grad_blocks(n);
    const size_t bytes = (size_t)blocks * cs::kMlpParams * 4 + (size_t)blocks * 4 + 256;
    cs_status s = mlp_work(ctx, mlp, bytes, st);
    if (s != CS_OK) return s;
    float* partials = mlp->work;
    float* loss_partials = partials + (size_t)blocks * cs::kMlpParams;
    if (adam) mlp->adam_t += 1;
    hipError_t e = cs::launch_mlp_grad(mlp->dev(), x, u, mu_t, r_t, n, (int)loss, partials, loss_partials, grad_out,
                                       loss_out, mlp->adam_m, mlp->adam_v, adam ? mlp->params : nullptr, lr,
                                       mlp->adam_t, st);
    if (e != hipSuccess) return hip_fail(ctx, e, (std::string(who) + ": launch").c_str());
    if (adam) mlp->bf16_ready = mlp->fp8_ready = false;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_mlp_grad(cs_ctx* ctx, const cs_mlp* mlp, const float* x, const float* u, const float* mu_t,
                      const float* r_t, int64_t n, cs_loss loss, float* grad_out, float* loss_out, void* stream) {
    if (ctx && mlp && !grad_out) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_grad: grad_out is NULL");
    return mlp_grad_impl(ctx, const_cast<cs_mlp*>(mlp), x, u, mu_t, r_t, n, loss, grad_out, loss_out, false, 0.0f,
                         stream, "cs_mlp_grad");
}

cs_status cs_mlp_adam_step(cs_ctx* ctx, cs_mlp* mlp, const float* grad, float lr, void* stream) {
    if (!ctx) return CS_ERR_INVALID_ARG;
    if (!mlp || !grad || !(lr > 0.0f)) return fail(ctx, CS_ERR_INVALID_ARG, "cs_mlp_adam_step: bad argument");
    DeviceGuard g(mlp->device);
    mlp->adam_t += 1;
    hipError_t e = cs::launch_mlp_adam(mlp->params, mlp->adam_m, mlp->adam_v, grad, lr, mlp->adam_t,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cs_mlp_adam_step: launch");
    mlp->bf16_ready = mlp->fp8_ready = false;
    ctx->last_error.clear();
    return CS_OK;
}

cs_status cs_mlp_train_step(cs_ctx* ctx, cs_mlp* mlp, const float* x, const float* u, const float* mu_t,
                            const float* r_t, int64_t n, float lr, cs_loss loss, float* loss_out, void* stream) {
    return mlp_grad_impl(ctx, mlp, x, u, mu_t, r_t, n, loss, nullptr, loss_out, true, lr, stream,
                         "cs_mlp_train_step");
}

}  // extern "C"
