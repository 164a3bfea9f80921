// Depth sort of the duplicated entries and per-tile ranges (Sec. III-C, IV-A).
//
// LSD radix sort with 8-bit digits over the significant bits of the key
// (plain: 32 + b_t bits of the 64-bit key; fast: the 32-bit key, 4 passes),
// value = Gaussian index.  The traffic model of Eq. sort_memory counts one
// read and one write of every (key, value) entry per pass; this sort meets it
// with one kernel per pass:
//   * `radix_hist` reads all keys once and builds the digit histogram of every
//     pass; `radix_scan` turns each into global digit offsets;
//   * `radix_pass` takes a tile of 4096 entries per block (ticket-ordered
//     block index), ranks each key among equal digits inside the tile with
//     wave64 ballots (stable: tile order is input order), publishes the tile's
//     digit counts and obtains each digit's offset among earlier tiles by
//     decoupled look-back, reorders the tile in LDS by digit and writes it out,
//     so consecutive threads store consecutive positions of a digit bucket.
// Ties keep input order, and the front end emits entries in Gaussian-index
// order, so equal keys end ordered by Gaussian index.
//
// Grids are sized for the workspace capacity; the entry count is read from
// the workspace header on the device, blocks beyond it return at once, so no
// host round trip sits between the front end and the sort.
#include "rgs_internal.h"

namespace rgs {

template <typename KeyT>
__device__ inline uint32_t digit_of(KeyT k, uint32_t shift) {
    return (uint32_t)(k >> shift) & (RADIX - 1);
}

__device__ inline uint32_t entry_count(const WsHeader* h) {
    uint64_t n = h->n_entries;
    uint64_t cap = h->capacity;
    return (uint32_t)(n < cap ? n : cap);
}

// Inclusive scan over a 256-thread block (one value per thread).
__device__ inline uint32_t block256_inclusive_scan(uint32_t x, uint32_t* s_wtot) {
    uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    uint32_t incl = wave_inclusive_scan(x);
    if (lane == 63) s_wtot[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if ((uint32_t)w < wave) before += s_wtot[w];
    __syncthreads();
    return incl + before;
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_radix_hist(const KeyT* __restrict__ keys, WsDev ws,
                                                    uint32_t passes, uint32_t sort_blocks_max) {
    __shared__ uint32_t s_h[MAX_PASSES * RADIX];
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += 256) s_h[i] = 0;
    const uint32_t n = entry_count(ws.header);
    // clear the look-back state of the tiles the passes will run
    const uint32_t nb = (n + SORT_TILE - 1) / SORT_TILE;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t* st = ws.lookback + (uint64_t)p * sort_blocks_max * RADIX;
        for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < (uint64_t)nb * RADIX; i += stride)
            st[i] = 0;
    }
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        KeyT k = keys[i];
        for (uint32_t p = 0; p < passes; ++p) atomicAdd(&s_h[p * RADIX + digit_of(k, 8 * p)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += 256) {
        uint32_t v = s_h[i];
        if (v) atomicAdd(&ws.hist[i], v);
    }
}

__global__ __launch_bounds__(256) void k_radix_scan(WsDev ws, uint32_t passes) {
    __shared__ uint32_t s_wtot[4];
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t v = ws.hist[p * RADIX + threadIdx.x];
        uint32_t incl = block256_inclusive_scan(v, s_wtot);
        ws.hist[p * RADIX + threadIdx.x] = incl - v;
    }
}

template <typename KeyT>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_pass(const KeyT* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin,
                                                             KeyT* __restrict__ kout,
                                                             uint32_t* __restrict__ vout, WsDev ws,
                                                             uint32_t pass, uint32_t shift,
                                                             uint32_t sort_blocks_max) {
    constexpr int WAVES = SORT_THREADS / 64;
    static_assert(SORT_THREADS == RADIX, "one thread per digit");
    __shared__ uint32_t s_vb;
    __shared__ uint32_t s_whist[WAVES * RADIX];
    __shared__ uint32_t s_bstart[RADIX];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_wtot[4];
    __shared__ KeyT s_keys[SORT_TILE];
    __shared__ uint32_t s_vals[SORT_TILE];

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    if (tid == 0) s_vb = atomicAdd(&ws.header->sort_ticket[pass], 1u);
    for (uint32_t i = tid; i < WAVES * RADIX; i += SORT_THREADS) s_whist[i] = 0;
    __syncthreads();
    const uint32_t vb = s_vb;
    const uint32_t n = entry_count(ws.header);
    const uint32_t tile_base = vb * SORT_TILE;
    if (tile_base >= n) return;
    const uint32_t n_valid = min((uint32_t)SORT_TILE, n - tile_base);

    // wave w owns entries [tile_base + w*ITEMS*64, +ITEMS*64); round r, lane l
    // holds entry tile_base + w*ITEMS*64 + r*64 + l
    const uint32_t wbase = tile_base + wave * (SORT_ITEMS * 64);
    KeyT k[SORT_ITEMS];
    uint32_t v[SORT_ITEMS];
    uint32_t rank[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        uint32_t idx = wbase + r * 64 + lane;
        bool valid = idx < n;
        k[r] = valid ? kin[idx] : (KeyT)0;
        v[r] = valid ? vin[idx] : 0u;
    }
    const uint64_t lt = lanemask_lt();
    // lanes of a wave read counters that other lanes of the same wave wrote in
    // the previous round (LDS keeps one wave's accesses in order); volatile
    // keeps the compiler from reusing an earlier read
    volatile uint32_t* my_hist = s_whist + wave * RADIX;
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        uint32_t idx = wbase + r * 64 + lane;
        bool valid = idx < n;
        uint32_t d = digit_of(k[r], shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t below = (uint32_t)__popcll(peers & lt);
        uint32_t prev = valid ? my_hist[d] : 0u;
        rank[r] = prev + below;
        if (valid && below == 0) my_hist[d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // digit d = tid: wave offsets, tile count, look-back, global base
    {
        const uint32_t d = tid;
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            uint32_t c = s_whist[w * RADIX + d];
            s_whist[w * RADIX + d] = tot;
            tot += c;
        }
        uint32_t* st = ws.lookback + ((uint64_t)pass * sort_blocks_max + vb) * RADIX;
        st_state(&st[d], (vb == 0 ? RS_PRE : RS_AGG) | tot);
        uint32_t incl = block256_inclusive_scan(tot, s_wtot);
        s_bstart[d] = incl - tot;
        uint32_t excl = 0;
        if (vb > 0) {
            int64_t j = (int64_t)vb - 1;
            uint32_t spins = 0;
            const uint32_t* base = ws.lookback + (uint64_t)pass * sort_blocks_max * RADIX + d;
            while (j >= 0) {
                uint32_t s = ld_state(base + (uint64_t)j * RADIX);
                uint32_t f = s & ~RS_VAL;
                if (f == RS_PRE) {
                    excl += s & RS_VAL;
                    break;
                }
                if (f == RS_AGG) {
                    excl += s & RS_VAL;
                    --j;
                    continue;
                }
                if (++spins > SPIN_LIMIT) {
                    atomicOr(&ws.header->error, 2u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            st_state(&st[d], RS_PRE | (excl + tot));
        }
        s_gbase[d] = ws.hist[pass * RADIX + d] + excl - (incl - tot);
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        uint32_t idx = wbase + r * 64 + lane;
        if (idx < n) {
            uint32_t d = digit_of(k[r], shift);
            uint32_t pos = s_bstart[d] + my_hist[d] + rank[r];
            s_keys[pos] = k[r];
            s_vals[pos] = v[r];
        }
    }
    __syncthreads();
    for (uint32_t p = tid; p < n_valid; p += SORT_THREADS) {
        KeyT kk = s_keys[p];
        uint32_t dst = s_gbase[digit_of(kk, shift)] + p;
        if (dst < n) {        // always true unless a look-back gave up (flagged above)
            kout[dst] = kk;
            vout[dst] = s_vals[p];
        }
    }
}

template <typename KeyT>
static void sort_typed(hipStream_t s, const WsDev& ws, uint32_t passes, uint32_t sort_blocks_max,
                       bool* result_in_b) {
    KeyT* ka = reinterpret_cast<KeyT*>(ws.keys_a);
    KeyT* kb = reinterpret_cast<KeyT*>(ws.keys_b);
    hipLaunchKernelGGL(k_radix_hist<KeyT>, dim3(HIST_BLOCKS), dim3(256), 0, s, ka, ws, passes,
                       sort_blocks_max);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(256), 0, s, ws, passes);
    for (uint32_t p = 0; p < passes; ++p) {
        bool from_a = (p % 2) == 0;
        hipLaunchKernelGGL(k_radix_pass<KeyT>, dim3(sort_blocks_max), dim3(SORT_THREADS), 0, s,
                           from_a ? ka : kb, from_a ? ws.vals_a : ws.vals_b, from_a ? kb : ka,
                           from_a ? ws.vals_b : ws.vals_a, ws, p, 8 * p, sort_blocks_max);
    }
    *result_in_b = (passes % 2) == 1;
}

void launch_sort(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes,
                 uint32_t passes, uint32_t sort_blocks_max, bool* result_in_b) {
    (void)f;
    if (key_bytes == 8) sort_typed<uint64_t>(s, ws, passes, sort_blocks_max, result_in_b);
    else sort_typed<uint32_t>(s, ws, passes, sort_blocks_max, result_in_b);
}

// ---------------------------------------------------------------------------
// Tile ranges: the run of each tile in the sorted keys.  Entry i starts a run
// when its tile differs from entry i-1's, and ends the previous run there.

template <typename KeyT>
__global__ __launch_bounds__(256) void k_ranges(const KeyT* __restrict__ keys, WsDev ws,
                                                uint32_t shift, uint32_t n_tiles) {
    const uint32_t n = entry_count(ws.header);
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t t = (uint32_t)(keys[i] >> shift);
    uint32_t tp = i ? (uint32_t)(keys[i - 1] >> shift) : 0xffffffffu;
    if (t >= n_tiles || (i && tp >= n_tiles)) {     // only after a failed sort
        atomicOr(&ws.header->error, 4u);
        return;
    }
    if (i == 0) {
        ws.ranges[2 * t] = 0;
    } else if (tp != t) {
        ws.ranges[2 * tp + 1] = i;
        ws.ranges[2 * t] = i;
    }
    if (i == n - 1) ws.ranges[2 * t + 1] = n;
}

void launch_ranges(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes,
                   bool result_in_b) {
    uint32_t blocks = (f.capacity + 255) / 256;
    if (key_bytes == 8)
        hipLaunchKernelGGL(k_ranges<uint64_t>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const uint64_t*>(result_in_b ? ws.keys_b : ws.keys_a), ws, 32u,
                           (uint32_t)f.n_tiles);
    else
        hipLaunchKernelGGL(k_ranges<uint32_t>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(result_in_b ? ws.keys_b : ws.keys_a), ws,
                           (uint32_t)f.b_d, (uint32_t)f.n_tiles);
}

}  // namespace rgs
