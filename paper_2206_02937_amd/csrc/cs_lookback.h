// cs_lookback.h -- single-pass prefix sums across workgroups by decoupled
// look-back (Merrill & Garland, "Single-pass Parallel Prefix Scan with
// Decoupled Look-back", 2016).  Workgroup b publishes its aggregate, walks back
// over its predecessors' published words until it meets an inclusive prefix,
// and publishes its own inclusive prefix.  Status words carry the epoch of the
// step that wrote them, so the array never needs clearing.  Workgroups are
// dispatched in index order, so every predecessor is resident or finished; a
// spin limit still bounds every wait.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cs {

constexpr uint64_t kFlagAggregate = 1, kFlagPrefix = 2;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint64_t flag, uint32_t value) {
    return ((uint64_t)(epoch & 0x3FFFFFFFu) << 34) | (flag << 32) | (uint64_t)value;
}

// Called by all 64 lanes of one wave of workgroup `idx`; on a spin-limit
// overrun records the epoch in *fault and continues with the prefix gathered
// so far.  Lane l reads the status word of predecessor idx-1-l, so each round
// trip to memory covers 64 predecessors (cross-die atomic latency dominates a
// walk that reads one word at a time).  A window is complete once every
// predecessor up to the nearest inclusive prefix in it has published; the
// older ones are not needed.  Workgroup i's word is status[i S]: with S = 16
// each word has a 128-byte line of its own, which spreads the polling of many
// workgroups over the memory channels.  Returns the exclusive prefix in every
// lane.
template <int S = 1>
__device__ __forceinline__ uint32_t lookback_exclusive_wave(uint64_t* status, int64_t idx, uint32_t E,
                                                            uint32_t aggregate, uint32_t* fault) {
    const uint32_t Et = E & 0x3FFFFFFFu;
    const int lane = __lane_id();
    if (lane == 0)
        __hip_atomic_store(&status[idx * S], pack_status(E, idx == 0 ? kFlagPrefix : kFlagAggregate, aggregate),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (idx == 0) return 0;
    uint32_t excl = 0;
    int64_t base = idx - 1;
    uint32_t spins = 0;
    while (true) {
        const int64_t k = base - lane;
        const uint64_t w = k >= 0 ? __hip_atomic_load(&status[k * S], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : pack_status(E, kFlagPrefix, 0);
        const uint64_t fl = (w >> 32) & 3u;
        const bool ready = (uint32_t)(w >> 34) == Et && fl != 0;
        const uint64_t rm = __ballot(ready);
        const uint64_t pm = __ballot(ready && fl == kFlagPrefix);
        const int first = pm ? (int)__ffsll((unsigned long long)pm) - 1 : 63;
        const uint64_t need = first == 63 ? ~0ull : ((2ull << first) - 1ull);  // lanes 0 .. first
        if ((rm & need) != need) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicMax(fault, E);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint32_t val = lane <= first ? (uint32_t)w : 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) val += __shfl_xor(val, off, 64);
        excl += val;
        if (pm) break;
        base -= 64;
    }
    if (lane == 0)
        __hip_atomic_store(&status[idx * S], pack_status(E, kFlagPrefix, excl + aggregate), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

}  // namespace cs
