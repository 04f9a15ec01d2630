// cs_internal.h -- host-side structures shared by the translation units of
// libcompton.so (context, workspace, launch entry points).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/compton.h"

namespace cs {

constexpr int kChunk = 256;       // pairs per workgroup of the pair kernel
constexpr int kScanItems = 1024;  // items per workgroup of the scan kernels

// Device workspace of one context.  Grown (never shrunk) on demand; growth
// synchronises the caller's stream before releasing the old buffer.
struct Workspace {
    void* base = nullptr;
    size_t bytes = 0;
};

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
    int64_t n_chunks;         // ceil(min(ne, ng) / kChunk): upper bound of used chunks
    int64_t n_collide_blocks; // fixed grid of the collide kernel
    int64_t scan_tmp_len;
};

size_t step_workspace_bytes(const StepShape& s);
void carve_step_buffers(void* base, const StepShape& s, StepBuffers* b);

struct StepParams {
    cs_dtype dtype;
    cs_species e, g;
    const int64_t* off_e;
    const int64_t* off_g;
    double dt, density_norm;
    uint64_t seed, step;
    cs_sampler sampler;
    const cs_mlp* mlp;
    cs_stats* stats;
    hipEvent_t* events;  // CS_STAGE_COUNT + 1 events to record between stages, or nullptr
};

// Launch every kernel of one step on `stream`; returns the HIP error of the
// launches (asynchronous faults surface later).
hipError_t launch_step(const StepShape& shape, const StepBuffers& buf, const StepParams& p, hipStream_t stream);
hipError_t launch_check_layout(const int64_t* off, int64_t n_cells, int64_t n, int32_t* flag, hipStream_t stream);
hipError_t launch_sample_plain(cs_dtype dtype, const void* x, const void* u, int64_t n, void* mu, void* ratio,
                               hipStream_t stream);

}  // namespace cs

struct cs_ctx {
    int device = 0;
    cs::Workspace ws;
    std::string last_error;
    bool timing = false;
    bool timed_step_pending = false;
    hipEvent_t events[CS_STAGE_COUNT + 1] = {};
};
