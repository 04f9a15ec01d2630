// cs_internal.h -- host-side structures shared by the translation units of
// libcompton.so (context, workspace, launch entry points).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/compton.h"

namespace cs {

constexpr int kChunk = 256;       // pairs per workgroup of the pair kernel
constexpr int64_t kCompactMaxChunks = 32;  // compact pair kernel: chunks per workgroup
constexpr int kPairStatusStride = 16;      // compact pair kernel: look-back status words apart (one 128-byte line each)
constexpr int64_t kTimingRing = 512;  // steps whose stage events are kept
constexpr int kScanItems = 1024;  // items per workgroup of the scan kernels

// Step-to-step control block at the start of the workspace (device memory,
// zeroed with epoch = 1 when the workspace is allocated).
struct StepControl {
    uint32_t epoch;             // epoch of the current step (starts at 1)
    uint32_t done;              // workgroups of the step's last kernel finished
    uint32_t layout_epoch;      // epoch of the last step with an invalid layout
    uint32_t scan_fault_epoch;  // epoch of the last step whose scan timed out
    uint64_t step;              // device step counter (graph replay)
    uint32_t n_accepted;        // compact strategy: accepted pairs this step
    uint32_t done_pair;         // compact strategy: pair workgroups finished
    double pair_prob;           // compact strategy: reduced pair partials
    int64_t pair_clipped, pair_invalid;
    uint64_t pad[1];
};
static_assert(sizeof(StepControl) == 64, "control block size");

// Device workspace of one context: [control | look-back status words |
// per-step area].  Grown (never shrunk) on demand; growth synchronises the
// caller's stream before releasing the old buffer and re-initialises the
// control block and the status words.
struct Workspace {
    void* base = nullptr;
    size_t bytes = 0;
    int64_t status_cap = 0;  // look-back status words available
};

constexpr size_t kControlBytes = 256;

inline StepControl* ws_control(const Workspace& w) { return (StepControl*)w.base; }
inline uint64_t* ws_status(const Workspace& w) { return (uint64_t*)((char*)w.base + kControlBytes); }
inline size_t ws_fixed_bytes(int64_t status_cap) {
    return kControlBytes + (((size_t)status_cap * sizeof(uint64_t) + 255) & ~(size_t)255);
}
inline void* ws_step_area(const Workspace& w) { return (char*)w.base + ws_fixed_bytes(w.status_cap); }

// Sub-buffers of one step, carved from the workspace.
struct StepBuffers {
    int32_t* flag;         // [1] layout error flag
    int32_t* cell_np;      // [n_cells] pairs per cell
    int32_t* pair_off;     // [n_cells + 1] exclusive scan of cell_np
    uint32_t* cell_keys;   // [4 n_cells] pairing keys
    int32_t* chunk_cell;   // [n_chunks + 1] first cell of each chunk
    int2* acc_list;        // [n_chunks * kChunk] accepted (electron, photon)
    int32_t* acc_cnt;      // [n_chunks]
    int32_t* acc_off;      // [n_chunks + 1]
    double* part_prob;     // [n_chunks]
    int32_t* part_clip;    // [n_chunks]
    int32_t* part_inv;     // [n_chunks]
    double* part_energy;   // [2 n_collide_blocks]
    int32_t* part_fallback;  // [n_collide_blocks]
    int32_t* scan_tmp;     // [scan_tmp_len]
};

struct StepShape {
    int64_t n_cells;
    int64_t ne, ng;
    int64_t n_chunks;          // ceil(min(ne, ng) / kChunk): upper bound of used chunks
    int64_t n_collide_blocks;  // multi-kernel: fixed grid of the collide kernel
    int64_t scan_tmp_len;      // multi-kernel: scan scratch
    int64_t chunks_per_block;  // fused / compact pair kernel: consecutive chunks per workgroup
    int64_t n_step_blocks;     // fused: grid of k_step (>= 1)
    int64_t n_prep_blocks;     // fused / compact: grid of k_prep_scan
    int64_t n_dense_blocks;    // compact: grid of the one-wave collide kernel
    int64_t pairs_per_lane;    // compact: chunks each pair-kernel lane takes at a time (1, 2, 4)
};

// Per-workgroup partial sums of the fused step.
struct BlockPartials {
    double *prob, *e_before, *e_after;
    int64_t *clipped, *invalid, *collided, *fallback;
};

// Sub-buffers of the fused step, carved from the per-step area.
struct FusedBuffers {
    StepControl* ctrl;
    uint64_t* status;
    int32_t* pair_off;    // [n_cells + 1]
    uint32_t* cell_keys;  // [4 n_cells]
    int32_t* chunk_cell;  // [n_chunks + 1]
    BlockPartials part;   // [n_step_blocks] each
};

// Sub-buffers of the compact strategy (scan kernel, pair kernel with
// look-back compaction, dense collide kernel).
struct CompactBuffers {
    StepControl* ctrl;
    uint64_t* status;     // prep blocks, then one word per chunk
    int32_t* pair_off;    // [n_cells + 1]
    uint32_t* cell_keys;  // [4 n_cells]
    int32_t* chunk_cell;  // [n_chunks + 1]
    int32_t* list;        // [n_chunks * kChunk] stash slots of the accepted pairs, dense (workgroup, wave, pair order)
    void* stash;          // accepted pairs with their particle values: 64 G slots per pair-kernel wave
    int32_t* seg_count;   // [pair workgroups + 1] accepted pairs per pair workgroup (segmented list)
    double* chunk_prob;   // [n_chunks]
    int64_t* chunk_clip;  // [n_chunks]
    int64_t* chunk_inv;   // [n_chunks]
    double* coll_eb;      // [n_collide_blocks]
    double* coll_ea;      // [n_collide_blocks]
    int64_t* coll_fb;     // [n_collide_blocks]
};

int64_t compact_collide_threads(cs_sampler s);
// compact: the fewest chunks per pair workgroup (a multiple of the pairs per
// lane, at most kCompactMaxChunks) with which every pair workgroup of
// n_chunks chunks is resident at once on the current device
int64_t compact_fit_chunks(cs_dtype dtype, int64_t ppl, int64_t n_chunks);
int64_t compact_pair_blocks(const StepShape& s);
size_t fused_workspace_bytes(const StepShape& s);
void carve_fused_buffers(const Workspace& w, const StepShape& s, FusedBuffers* b);
int64_t fused_prep_blocks(int64_t n_cells);

size_t step_workspace_bytes(const StepShape& s);
void carve_step_buffers(void* base, const StepShape& s, StepBuffers* b);

// The x range a network answers for, as the kernels use it: its first
// feature is f1 = f_a log2(x) + f_b (log10 x mapped linearly from
// [log10 x_min, log10 x_max] onto [-1, 1]); x outside [x_lo, x_hi] (the
// bounds rounded to FP32) goes to the plain sampler.
struct NetDomain {
    float f_a, f_b;
    float x_lo, x_hi;
};
NetDomain net_domain(double x_min, double x_max);

struct MlpDev {
    const float* params;        // FP32 master
    const void* frag_bf16;      // kFragCount x 8 bf16
    const void* frag_fp8;       // kFragCount x 8 fp8 (E4M3)
    const float* fp8_scales;    // [0..2] weight scales, [3..5] input scales, [6..8] input amax
    NetDomain dom;
};

struct StepParams {
    cs_dtype dtype;
    cs_species e, g;
    const int64_t* off_e;
    const int64_t* off_g;
    double dt, density_norm;
    uint64_t seed, step;
    cs_sampler sampler;
    MlpDev net;  // device view of the network (network samplers)
    cs_stats* stats;
    hipEvent_t* events;   // CS_STAGE_COUNT + 1 events to record between stages, or nullptr
    int use_device_step;  // 1: kernels take the step from the device counter (graph replay)
    int wide_index;       // compact pair kernel: 1 = 64-bit particle indexing even where 32-bit offsets fit
};

// Launch every kernel of one step on `stream`; returns the HIP error of the
// launches (asynchronous faults surface later).
hipError_t launch_step(const StepShape& shape, const StepBuffers& buf, const StepParams& p, hipStream_t stream);
// Partial sums reduced by the finalize kernel: "a" per pair unit (chunk or
// workgroup), "b" per collide workgroup.  a_coll / b_fb may be null (then the
// accepted count comes from the control block, fallbacks are 0).
struct FinalArgs {
    StepControl* ctrl;
    const int32_t* pair_off;
    int64_t n_cells;
    const double* a_prob;
    const int64_t *a_clip, *a_inv, *a_coll;
    int64_t n_a;
    const double *b_eb, *b_ea;
    const int64_t* b_fb;
    int64_t n_b;
    cs_stats* stats;
};
hipError_t launch_finalize(const FinalArgs& f, hipStream_t st);

size_t compact_workspace_bytes(const StepShape& s);
void carve_compact_buffers(const Workspace& w, const StepShape& s, CompactBuffers* b);
hipError_t launch_compact(const StepShape& shape, const CompactBuffers& buf, const StepParams& p, hipStream_t stream);
hipError_t launch_prep(const StepShape& sh, StepControl* ctrl, uint64_t* status, int32_t* pair_off, uint32_t* keys,
                       int32_t* chunk_cell, const StepParams& p, hipStream_t st);

hipError_t launch_fused(const StepShape& shape, const FusedBuffers& buf, const StepParams& p, hipStream_t stream);
// one workgroup per cell (baseline); shape.n_step_blocks = n_cells partials
hipError_t launch_cell(const StepShape& shape, const FusedBuffers& buf, const StepParams& p, hipStream_t stream);
hipError_t launch_pair_x(cs_dtype dtype, const cs_species& e, const cs_species& g, int64_t n, double* x_out,
                         hipStream_t st);
hipError_t launch_check_layout(const int64_t* off, int64_t n_cells, int64_t n, int32_t* flag, hipStream_t stream);
hipError_t launch_sample_plain(cs_dtype dtype, const void* x, const void* u, int64_t n, void* mu, void* ratio,
                               hipStream_t stream);
// cell binning of one species (cs_bin.hip): workspace bytes for n particles,
// and the launch (in/out: x, y, z, w arrays of the dtype)
size_t bin_workspace_bytes(int64_t n);
// no-time-counter step (cs_ntc.hip): device scratch and the pinned read-back
// kept by the context (or a graph) between calls; the touch words (two sets
// of one 64-bit word per electron and per photon) keep their tags across
// steps, with the tag epoch and the replay step index in a head before them.
struct NtcState {
    void* cell_ws = nullptr;
    size_t cell_bytes = 0;
    void* cand_ws = nullptr;
    size_t cand_bytes = 0;
    int64_t cand_cap = 0;  // candidates the per-candidate launches are sized for
    void* touch = nullptr;
    int64_t cap_e = 0, cap_g = 0;
    void* host = nullptr;
    hipEvent_t ev = nullptr;
};
enum class NtcOutcome { kOk, kLayout, kTooMany };
hipError_t ntc_step(NtcState& s, cs_dtype dtype, const cs_species& e, const cs_species& g, const int64_t* off_e,
                    const int64_t* off_g, int64_t n_cells, double dt, double dn, uint64_t seed, uint64_t step,
                    cs_stats* stats, hipStream_t st, NtcOutcome* out);
// graphs: scratch for `cap` candidates (zeroed; synchronises st), the
// capturable launch sequence (step index from the device word), and the
// queued write of that word
hipError_t ntc_prepare_graph(NtcState& s, int64_t n_cells, int64_t cap, int64_t ne, int64_t ng, hipStream_t st);
hipError_t ntc_capture(const NtcState& s, cs_dtype dtype, const cs_species& e, const cs_species& g,
                       const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt, double dn,
                       uint64_t seed, cs_stats* stats, hipStream_t st);
hipError_t ntc_set_step(const NtcState& s, uint64_t step, hipStream_t st);
void ntc_free(NtcState& s);
// probability network (cs_pnet.hip)
size_t pnet_workspace_bytes(int64_t n);
hipError_t launch_pnet_target(const float* in, int64_t n, float* y, hipStream_t st);
hipError_t launch_pnet_forward(const float* params, const float* in, int64_t n, float* y, hipStream_t st);
hipError_t launch_pnet_grad(const float* params, const float* in, const float* target, int64_t n, int mae,
                            float* grad, float* loss, void* ws, hipStream_t st);
hipError_t launch_pnet_adam(float* params, const float* grad, float* m, float* v, float lr, float bc1, float bc2,
                            hipStream_t st);
hipError_t launch_bin(cs_dtype dtype, const int32_t* cell, int64_t n, int64_t n_cells, const void* const in[4],
                      void* const out[4], int64_t* off, int64_t* n_invalid, void* ws, hipStream_t stream);

// ---------------------------------------------------------------------------
// The sampler network (fixed widths 2 -> 64 x 4 -> 2).
// ---------------------------------------------------------------------------
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 12802;
// parameter offsets: W1[64][2], b1, W2[64][64], b2, W3, b3, W4, b4, W5[2][64], b5
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 4288, kOffW3 = 4352, kOffB3 = 8448,
              kOffW4 = 8512, kOffB4 = 12608, kOffW5 = 12672, kOffB5 = 12800;
// MFMA fragments of the three hidden 64x64 layers: [layer][tile_out][kstep][lane]
constexpr int kFragCount = 3 * 4 * 2 * 64;


hipError_t launch_mlp_forward(const MlpDev& m, cs_sampler prec, const float* x, const float* u, int64_t n,
                              float* y, float* mu, float* ratio, uint8_t* mask, hipStream_t st);
hipError_t launch_mlp_grad(const MlpDev& m, const float* x, const float* u, const float* mu_t, const float* r_t,
                           int64_t n, int loss, float* partials, float* loss_partials, float* grad_out,
                           float* loss_out, float* adam_m, float* adam_v, float* params_rw, float lr, int64_t t,
                           hipStream_t st);
hipError_t launch_mlp_quantize(float* params, const NetDomain& dom, void* frag_bf16, void* frag_fp8, float* scales,
                               cs_sampler prec, const float* cx, const float* cu, int64_t n, hipStream_t st);
int64_t mlp_grad_blocks(int64_t n);

}  // namespace cs

struct cs_mlp {
    int device = 0;
    int32_t widths[6] = {2, 64, 64, 64, 64, 2};
    float* params = nullptr;  // device FP32 master
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int64_t adam_t = 0;
    void* frag_bf16 = nullptr;
    void* frag_fp8 = nullptr;
    float* fp8_scales = nullptr;
    bool bf16_ready = false, fp8_ready = false;
    float* work = nullptr;  // gradient partials, loss partials, gradient
    size_t work_bytes = 0;
    double x_min = CS_MLP_X_MIN, x_max = CS_MLP_X_MAX;  // the x range the network answers for
    cs::MlpDev dev() const { return {params, frag_bf16, frag_fp8, fp8_scales, cs::net_domain(x_min, x_max)}; }
};

struct cs_ctx {
    int device = 0;
    cs::Workspace ws;
    int64_t strategy = CS_STRATEGY_FUSED;
    int64_t chunks_per_block = 0;  // 0: automatic
    int64_t pairs_per_lane = 0;    // compact pair kernel, 0: automatic
    int64_t wide_index = 0;        // compact pair kernel, 1: always 64-bit particle indexing
    std::string last_error;
    bool timing = false;
    int64_t timed_steps = 0;          // steps timed since enabling or the last read
    std::vector<hipEvent_t> events;   // kTimingRing slots of CS_STAGE_COUNT + 1 events
    void* bin_ws = nullptr;           // cell-binning scratch, grown on demand
    size_t bin_bytes = 0;
    void* pnet_ws = nullptr;          // probability-network gradient partials, grown on demand
    size_t pnet_bytes = 0;
    cs::NtcState ntc;                 // no-time-counter step scratch
};
