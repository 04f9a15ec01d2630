// cs_bin.hip -- binning of one species into collision cells (the grouping of
// particles by cell that precedes pairing, Sec. 3.1): a stable sort of the
// particles by cell id that writes the species' arrays in cell order, and
// the CSR offsets of the cells.
//
// The sort is a least-significant-digit radix sort of the cell ids with
// 8-bit digits, the lowest digit widened to up to 9 bits when that saves a
// pass (17 bits of key: 9 + 8), that moves the
// particles' values along with their keys, so that every access to the
// values is a run of consecutive elements (never a gather from random
// positions).  Every pass is stable, so the result is the stable sort;
// nothing depends on the timing of atomics, so the output is the same on
// every run.  Ids outside [0, n_cells) get the key n_cells, which sorts them
// after every valid particle.
//
//   per pass (tiles of 16 waves x 1024 keys = 16384 keys for FP32 values,
//   8 waves x 1024 = 8192 for FP64, so that a tile and one value array fit
//   in LDS together):
//   k_bin_hist    per tile, the digit counts (LDS atomics)
//   k_bin_scan    one workgroup per digit: exclusive prefix over the tiles of
//                 that digit's counts, and the digit's total
//   k_bin_scatter per tile: digit bases from the totals and the tile
//                 prefixes; each wave takes 1024 consecutive keys in 16
//                 chunks of 64, in order, and ranks each key among the
//                 chunk's keys of the same digit by one ballot per digit
//                 bit; the tile,
//                 ordered by digit in LDS, is then written out run by run
//                 with the particles' four values
//   k_bin_offsets off[c] = first sorted position with key >= c (binary
//                 search), c = 0 .. n_cells; off[n_cells] counts the valid
//                 particles
// The passes alternate between a scratch copy of the values and the output
// arrays so that the last one writes the output.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cs_block.h"
#include "cs_internal.h"

namespace cs {

constexpr int kBinThreads = 256;                          // scans and offsets
constexpr int kBinChunks = 16;                             // 64-key chunks per wave
constexpr int kBinWaveKeys = 64 * kBinChunks;             // 1024
constexpr int kBinDigits = 512;  // at most: a 9-bit digit

// Tile shape per value type: the larger the tile, the longer each digit's
// run of consecutive output positions (8-bit digits: ~64 keys per digit and
// FP32 tile, 256 bytes per value array instead of 64 with 4096-key tiles),
// so the scattered writes fill whole lines.  A tile's keys and one value
// array are staged in LDS together with the source indices and per-wave
// counts: 132 KB for FP32, 100 KB for FP64.
template <typename T>
struct BinShape {
    static constexpr int kThreads = sizeof(T) == 4 ? 1024 : 512;
    static constexpr int kWaves = kThreads / 64;
    static constexpr int kTile = kWaves * kBinWaveKeys;
    typedef typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type Word;  // a key or a value
};
constexpr int kBinTileMin = 8192;  // the smaller tile (FP64): sizes the per-tile counts of the scratch

template <typename T>
struct BinArrays {
    const T *x, *y, *z, *w;
};
template <typename T>
struct BinOut {
    T *x, *y, *z, *w;
};

// Pass key of particle i: its cell id, or n_cells for an id outside
// [0, n_cells); read from the cell ids on the first pass.
__device__ __forceinline__ uint32_t bin_key(const uint32_t* keys, const int32_t* cell, int64_t n_cells, int64_t i) {
    if (keys) return keys[i];
    const int32_t c = cell[i];
    return c >= 0 && (int64_t)c < n_cells ? (uint32_t)c : (uint32_t)n_cells;
}

// hist[d * n_tiles + t] = keys of tile t (TILE keys, THREADS threads) whose
// digit is d
template <int THREADS, int TILE>
__global__ __launch_bounds__(THREADS) void k_bin_hist(const uint32_t* keys, const int32_t* cell, int64_t n,
                                                      int64_t n_cells, int shift, int dbits, int64_t n_tiles,
                                                      uint32_t* hist) {
    __shared__ uint32_t s_cnt[kBinDigits];
    const int tid = threadIdx.x;
    const uint32_t mask = (1u << dbits) - 1u;
    const int nd = 1 << dbits;
    for (int d = tid; d < kBinDigits; d += THREADS) s_cnt[d] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * TILE;
#pragma unroll 4
    for (int j = 0; j < TILE / THREADS; ++j) {
        const int64_t i = t0 + (int64_t)j * THREADS + tid;
        if (i < n) atomicAdd(&s_cnt[(bin_key(keys, cell, n_cells, i) >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = tid; d < nd; d += THREADS) hist[(int64_t)d * n_tiles + blockIdx.x] = s_cnt[d];
}

// Workgroup d: exclusive prefix of hist[d][0 .. n_tiles) in place, the sum to
// totals[d].  The tiles are taken in blocks of 256 x 16, each thread owning
// 16 consecutive entries of a block.
__global__ __launch_bounds__(kBinThreads) void k_bin_scan(uint32_t* hist, int64_t n_tiles, uint32_t* totals) {
    __shared__ int s_scan[kBinThreads / 64 + 1];
    constexpr int kPer = 16;
    uint32_t* h = hist + (int64_t)blockIdx.x * n_tiles;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < n_tiles; b0 += (int64_t)kBinThreads * kPer) {
        const int64_t i0 = b0 + (int64_t)threadIdx.x * kPer;
        uint32_t v[kPer];
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            v[k] = i0 + k < n_tiles ? h[i0 + k] : 0u;
            const uint32_t c = v[k];
            v[k] = run;
            run += c;
        }
        int block_total;
        const uint32_t ex = carry + (uint32_t)block_exclusive_scan((int)run, s_scan, &block_total);
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (i0 + k < n_tiles) h[i0 + k] = ex + v[k];
        carry += (uint32_t)block_total;
        __syncthreads();  // s_scan reused by the next block
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of tile t: key i goes to base(digit) + (keys of the same
// digit before it in the tile), base = (keys of smaller digits in all tiles)
// + (keys of this digit in earlier tiles); the particle's values go with it.
// The tile is first ordered by digit in LDS (keys and tile-local source
// indices) and written out in that order, so that consecutive threads write
// consecutive positions of a digit's run; each value array passes through
// LDS the same way (read in order, written in digit order), so every global
// access is coalesced.
template <typename T>
__global__ __launch_bounds__(BinShape<T>::kThreads) void k_bin_scatter(const uint32_t* keys_in, const int32_t* cell,
                                                                       int64_t n, int64_t n_cells, int shift,
                                                                       int dbits, int64_t n_tiles,
                                                                       const uint32_t* hist, const uint32_t* totals,
                                                                       BinArrays<T> src, uint32_t* keys_out,
                                                                       BinOut<T> dst) {
    constexpr int kThreads = BinShape<T>::kThreads, kTile = BinShape<T>::kTile, kWaves = BinShape<T>::kWaves;
    typedef typename BinShape<T>::Word Word;
    constexpr int kPer = kTile / kThreads;            // 16 outputs per thread
    __shared__ uint32_t s_cnt[kWaves][kBinDigits];    // per wave counts, then running local bases
    __shared__ uint32_t s_toff[kBinDigits];           // tile-local start of each digit's run
    __shared__ uint32_t s_gbase[kBinDigits];          // global start of each digit's run
    __shared__ Word s_buf[kTile];                     // the tile's keys, then each value array
    __shared__ uint16_t s_src[kTile];                 // tile-local source of each output
    __shared__ int s_scan[kWaves + 1];
    static_assert(kTile <= 65536, "tile-local indices are 16-bit");
    uint32_t* s_key = (uint32_t*)s_buf;
    T* s_val = (T*)s_buf;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int64_t t = blockIdx.x;
    const int64_t t0 = t * kTile;
    const int64_t rem = n - t0;
    const int len = rem < kTile ? (int)rem : kTile;
    const int wl0 = wave * kBinWaveKeys;  // this wave's first key in the tile
    const uint32_t mask = (1u << dbits) - 1u;
    const int nd = 1 << dbits;
    // thread t < kBinDigits / 2 looks after digits 2t and 2t + 1 in the scans
    // below; the others add nothing to them
    const bool dig = tid < kBinDigits / 2;
    const int d0 = dig ? 2 * tid : 0, d1 = d0 + 1;
    if (dig) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            s_cnt[w][d0] = 0;
            s_cnt[w][d1] = 0;
        }
    }
    // digit base over all tiles: exclusive prefix of the totals
    {
        const uint32_t t0v = dig && d0 < nd ? totals[d0] : 0u, t1v = dig && d1 < nd ? totals[d1] : 0u;
        int unused;
        const uint32_t ex = (uint32_t)block_exclusive_scan((int)(t0v + t1v), s_scan, &unused);
        if (dig && d0 < nd) s_gbase[d0] = ex + hist[(int64_t)d0 * n_tiles + t];
        if (dig && d1 < nd) s_gbase[d1] = ex + t0v + hist[(int64_t)d1 * n_tiles + t];
    }
    // the tile's four value arrays, read in order (coalesced) into registers
    // first, so that their reads are in flight while the keys are ranked;
    // non-temporal, as every value is read once per pass (the stores stay
    // ordinary: a digit's run rarely fills whole lines, and the cache
    // merges the pieces that neighbouring tiles write)
    const T* srcs[4] = {src.x, src.y, src.z, src.w};
    T val[4][kPer];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = tid + q * kThreads;
            val[a][q] = j < len ? __builtin_nontemporal_load(&srcs[a][t0 + j]) : (T)0;
        }
    uint32_t key[kBinChunks];
#pragma unroll
    for (int c = 0; c < kBinChunks; ++c) {
        const int li = wl0 + c * 64 + lane;
        key[c] = li < len ? bin_key(keys_in, cell, n_cells, t0 + li) : 0u;
        if (li < len) atomicAdd(&s_cnt[wave][(key[c] >> shift) & mask], 1u);
    }
    __syncthreads();
    // the tile-local start of each digit's run, then each wave's running
    // base inside it (waves in key order)
    {
        uint32_t tc0 = 0, tc1 = 0;
        if (dig) {
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                tc0 += s_cnt[w][d0];
                tc1 += s_cnt[w][d1];
            }
        }
        int unused2;
        uint32_t run0 = (uint32_t)block_exclusive_scan((int)(tc0 + tc1), s_scan, &unused2);
        uint32_t run1 = run0 + tc0;
        if (dig) {
            s_toff[d0] = run0;
            s_toff[d1] = run1;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c0 = s_cnt[w][d0], c1 = s_cnt[w][d1];
                s_cnt[w][d0] = run0;
                s_cnt[w][d1] = run1;
                run0 += c0;
                run1 += c1;
            }
        }
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    for (int c = 0; c < kBinChunks; ++c) {
        const int li = wl0 + c * 64 + lane;  // tile-local index
        const bool act = li < len;
        const uint32_t d = (key[c] >> shift) & mask;
        uint64_t eq = __ballot(act);
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            if (b < dbits) {
                const uint64_t m = __ballot(act && ((d >> b) & 1u));
                eq &= ((d >> b) & 1u) ? m : ~m;
            }
        }
        if (act) {
            const uint32_t lp = s_cnt[wave][d] + (uint32_t)__popcll(eq & below);
            s_key[lp] = key[c];
            s_src[lp] = (uint16_t)li;
        }
        // the lowest lane of each digit group advances that digit's base (the
        // reads above precede these writes in the wave's LDS order)
        if (act && (eq & below) == 0) s_cnt[wave][d] += (uint32_t)__popcll(eq);
    }
    __syncthreads();
    // keys, in digit order; each output's global position kept for the values
    uint32_t pos[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int j = tid + q * kThreads;
        pos[q] = 0;
        if (j < len) {
            const uint32_t k = s_key[j];
            const uint32_t d = (k >> shift) & mask;
            pos[q] = s_gbase[d] + ((uint32_t)j - s_toff[d]);
            keys_out[pos[q]] = k;
        }
    }
    T* dsts[4] = {dst.x, dst.y, dst.z, dst.w};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        __syncthreads();  // s_buf free
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = tid + q * kThreads;
            if (j < len) s_val[j] = val[a][q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = tid + q * kThreads;
            if (j < len) dsts[a][pos[q]] = s_val[s_src[j]];
        }
    }
}

// off[c] = lower bound of c in the sorted keys, c = 0 .. n_cells; the thread
// of c = n_cells also reports the particles with no valid cell.
__global__ __launch_bounds__(kBinThreads) void k_bin_offsets(const uint32_t* keys, int64_t n, int64_t n_cells,
                                                             int64_t* off, int64_t* n_invalid) {
    const int64_t c = (int64_t)blockIdx.x * kBinThreads + threadIdx.x;
    if (c > n_cells) return;
    int64_t lo = 0, hi = n;  // first position with key >= c
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    off[c] = lo;
    if (c == n_cells && n_invalid) *n_invalid = n - lo;
}

// tiles of a pass (per value type); the scratch is sized for the smaller
// tile, which gives the more tiles
int64_t bin_tiles(int64_t n, int64_t tile = kBinTileMin) { return (n + tile - 1) / tile; }

// scratch: two key arrays (uint32), one copy of the four value arrays (8 B
// elements, enough for either storage type), digit counts of every tile and
// the digit totals
size_t bin_workspace_bytes(int64_t n) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t nn = n > 0 ? n : 1;
    return 2 * al(4 * (size_t)nn) + 4 * al(8 * (size_t)nn) + al(4 * (size_t)kBinDigits * bin_tiles(nn)) +
           al(4 * (size_t)kBinDigits);
}

template <typename T>
static void launch_passes(const int32_t* cell, int64_t n, int64_t n_cells, const void* const in[4],
                          void* const out[4], uint32_t* const keys[2], void* const tmp[4], uint32_t* hist,
                          uint32_t* totals, int passes, int low_bits, hipStream_t st) {
    constexpr int kThreads = BinShape<T>::kThreads, kTile = BinShape<T>::kTile;
    static_assert(kTile >= kBinTileMin, "the scratch holds counts for kBinTileMin tiles");
    const int64_t n_tiles = bin_tiles(n, kTile);
    const BinArrays<T> in_a = {(const T*)in[0], (const T*)in[1], (const T*)in[2], (const T*)in[3]};
    const BinOut<T> out_a = {(T*)out[0], (T*)out[1], (T*)out[2], (T*)out[3]};
    const BinOut<T> tmp_a = {(T*)tmp[0], (T*)tmp[1], (T*)tmp[2], (T*)tmp[3]};
    for (int ps = 0; ps < passes; ++ps) {
        // the first pass takes the low_bits lowest bits, the others 8 each
        const int shift = ps == 0 ? 0 : low_bits + 8 * (ps - 1);
        const int dbits = ps == 0 ? low_bits : 8;
        const uint32_t* kin = ps == 0 ? nullptr : keys[(ps - 1) & 1];
        // the last pass writes the output; before it the passes alternate
        // between the scratch copy and the output
        const BinOut<T> dst = ((passes - 1 - ps) & 1) == 0 ? out_a : tmp_a;
        const BinOut<T> prev = ((passes - ps) & 1) == 0 ? out_a : tmp_a;
        const BinArrays<T> src = ps == 0 ? in_a : BinArrays<T>{prev.x, prev.y, prev.z, prev.w};
        k_bin_hist<kThreads, kTile><<<(unsigned)n_tiles, kThreads, 0, st>>>(kin, cell, n, n_cells, shift, dbits,
                                                                             n_tiles, hist);
        k_bin_scan<<<1u << dbits, kBinThreads, 0, st>>>(hist, n_tiles, totals);
        k_bin_scatter<T><<<(unsigned)n_tiles, kThreads, 0, st>>>(kin, cell, n, n_cells, shift, dbits, n_tiles, hist,
                                                                 totals, src, keys[ps & 1], dst);
    }
}

hipError_t launch_bin(cs_dtype dtype, const int32_t* cell, int64_t n, int64_t n_cells, const void* const in[4],
                      void* const out[4], int64_t* off, int64_t* n_invalid, void* ws, hipStream_t st) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t nn = n > 0 ? n : 1;
    char* p = (char*)ws;
    uint32_t* keys[2];
    keys[0] = (uint32_t*)p;
    p += al(4 * (size_t)nn);
    keys[1] = (uint32_t*)p;
    p += al(4 * (size_t)nn);
    void* tmp[4];
    for (int a = 0; a < 4; ++a) {
        tmp[a] = p;
        p += al(8 * (size_t)nn);
    }
    uint32_t* hist = (uint32_t*)p;
    p += al(4 * (size_t)kBinDigits * bin_tiles(nn));
    uint32_t* totals = (uint32_t*)p;

    // the largest key is n_cells (the mark of an invalid id); at least one
    // pass, which also writes the keys the offsets are read from.  Passes of
    // 8 bits, the lowest digit up to 9 bits wide: 17 bits take 9 + 8.
    int bits = 0;
    while (bits < 32 && ((uint64_t)n_cells >> bits) != 0) ++bits;
    const int passes = bits <= 9 ? 1 : (bits - 9 + 7) / 8 + 1;
    const int low_bits = bits <= 9 ? (bits > 0 ? bits : 1) : bits - 8 * (passes - 1);
    if (n > 0) {
        if (dtype == CS_F32)
            launch_passes<float>(cell, n, n_cells, in, out, keys, tmp, hist, totals, passes, low_bits, st);
        else
            launch_passes<double>(cell, n, n_cells, in, out, keys, tmp, hist, totals, passes, low_bits, st);
    }
    const unsigned off_blocks = (unsigned)((n_cells + 1 + kBinThreads - 1) / kBinThreads);
    k_bin_offsets<<<off_blocks, kBinThreads, 0, st>>>(keys[(passes - 1) & 1], n, n_cells, off, n_invalid);
    return hipGetLastError();
}

}  // namespace cs
