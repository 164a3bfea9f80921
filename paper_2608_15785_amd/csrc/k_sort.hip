// Depth sort of the duplicated entries and per-tile ranges (Sec. III-C, IV-A).
//
// LSD radix sort with 8-bit digits over the significant bits of the key
// (plain: 32 + b_t bits of the 64-bit key; fast: the 32-bit key, 4 passes),
// value = Gaussian index.  Eq. sort_memory counts one read and one write of
// every (key, value) entry per pass.  A frame's whole grid of radix tiles is
// resident on the 256 CUs at once, so the tiles cannot pass digit offsets
// along a look-back chain without waiting on each other; each pass is instead
// a reduce-then-scan:
//   * `radix_upsweep` counts each radix tile's digits (keys only; 4096-entry
//     tiles for 32-bit keys, 2048 for 64-bit keys);
//   * `radix_offsets` scans, for each digit in its own workgroup, the tiles'
//     counts into the tile's offset inside that digit's bucket, and records
//     the bucket's size;
//   * `radix_scatter` turns the 256 bucket sizes into bucket bases (one block
//     scan), ranks each key among equal digits of its tile with wave64 ballots
//     (stable: tile order is input order), reorders the tile in LDS by digit
//     and writes it out, so consecutive threads store consecutive positions of
//     a digit bucket.
// Ties keep input order, and the front end emits entries in Gaussian-index
// order, so equal keys end ordered by Gaussian index.
//
// Grids are sized for the workspace capacity; the entry count is read from
// the workspace header on the device and tiles beyond it return at once, so
// no host round trip sits between the front end and the sort.
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

// Per-tile digit counts, digit-major: counts[d * nb_max + tile].
template <typename KeyT>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_upsweep(const KeyT* __restrict__ kin, WsDev ws,
                                                                uint32_t shift, uint32_t nb_max) {
    __shared__ uint32_t s_h[RADIX];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = entry_count(ws.header);
    constexpr int SORT_ITEMS = SortTile<KeyT>::ITEMS;
    constexpr int SORT_TILE = SortTile<KeyT>::SIZE;
    const uint32_t tile_base = blockIdx.x * SORT_TILE;
    if (tile_base >= n) return;
    KeyT k[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const uint32_t idx = tile_base + r * SORT_THREADS + threadIdx.x;
        k[r] = idx < n ? kin[idx] : (KeyT)0;
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r)
        if (tile_base + r * SORT_THREADS + threadIdx.x < n) atomicAdd(&s_h[digit_of(k[r], shift)], 1u);
    __syncthreads();
    ws.tile_counts[(uint64_t)threadIdx.x * nb_max + blockIdx.x] = s_h[threadIdx.x];
}

// Digit d (one workgroup each): exclusive scan of its per-tile counts, in
// place, and the size of the digit's bucket.  Each thread scans a contiguous
// chunk of the row in registers; one block scan joins the chunks.
constexpr int OFFSETS_CHUNK = 16;

__global__ __launch_bounds__(256) void k_radix_offsets(WsDev ws, uint32_t nb_max, uint32_t tile_size) {
    __shared__ uint32_t s_wtot[4];
    const uint32_t d = blockIdx.x;
    const uint32_t n = entry_count(ws.header);
    const uint32_t nb = (n + tile_size - 1) / tile_size;
    uint32_t* row = ws.tile_counts + (uint64_t)d * nb_max;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nb; c0 += 256 * OFFSETS_CHUNK) {
        const uint32_t b = c0 + threadIdx.x * OFFSETS_CHUNK;
        uint32_t v[OFFSETS_CHUNK];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < OFFSETS_CHUNK; ++k) {
            v[k] = b + k < nb ? row[b + k] : 0u;
            sum += v[k];
        }
        const uint32_t incl = block256_inclusive_scan(sum, s_wtot);
        uint32_t run = carry + incl - sum;
#pragma unroll
        for (int k = 0; k < OFFSETS_CHUNK; ++k) {
            if (b + k < nb) row[b + k] = run;
            run += v[k];
        }
        carry += s_wtot[0] + s_wtot[1] + s_wtot[2] + s_wtot[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) ws.hist[d] = carry;
}

template <typename KeyT>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(const KeyT* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                KeyT* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, WsDev ws,
                                                                uint32_t shift, uint32_t nb_max) {
    constexpr int WAVES = SORT_THREADS / 64;
    constexpr int SORT_ITEMS = SortTile<KeyT>::ITEMS;
    constexpr int SORT_TILE = SortTile<KeyT>::SIZE;
    static_assert(SORT_THREADS == RADIX, "one thread per digit");
    __shared__ uint32_t s_whist[WAVES * RADIX];
    __shared__ uint32_t s_bstart[RADIX];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_wtot[4];
    __shared__ KeyT s_keys[SORT_TILE];
    __shared__ uint32_t s_vals[SORT_TILE];

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    const uint32_t vb = blockIdx.x;
    const uint32_t n = entry_count(ws.header);
    const uint32_t tile_base = vb * SORT_TILE;
    if (tile_base >= n) return;
    for (uint32_t i = tid; i < WAVES * RADIX; i += SORT_THREADS) s_whist[i] = 0;
    __syncthreads();
    const uint32_t n_valid = min((uint32_t)SORT_TILE, n - tile_base);
    // this tile's offset inside digit tid's bucket and the bucket's size do not
    // depend on the keys: start both loads before the keys'
    const uint32_t tile_off = ws.tile_counts[(uint64_t)tid * nb_max + vb];
    const uint32_t bucket = ws.hist[tid];

    // wave w owns entries [tile_base + w*ITEMS*64, +ITEMS*64); round r, lane l
    // holds entry tile_base + w*ITEMS*64 + r*64 + l
    const uint32_t wbase = tile_base + wave * (SORT_ITEMS * 64);
    KeyT k[SORT_ITEMS];
    uint32_t v[SORT_ITEMS];
    uint32_t rank[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const uint32_t idx = wbase + r * 64 + lane;
        const bool valid = idx < n;
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
        const uint32_t idx = wbase + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = digit_of(k[r], shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t prev = valid ? my_hist[d] : 0u;
        rank[r] = prev + below;
        if (valid && below == 0) my_hist[d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // digit d = tid: wave offsets, tile count, tile-local start, global base
    {
        const uint32_t d = tid;
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = s_whist[w * RADIX + d];
            s_whist[w * RADIX + d] = tot;
            tot += c;
        }
        const uint32_t incl = block256_inclusive_scan(tot, s_wtot);
        s_bstart[d] = incl - tot;
        const uint32_t bincl = block256_inclusive_scan(bucket, s_wtot);
        s_gbase[d] = (bincl - bucket) + tile_off - (incl - tot);
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const uint32_t idx = wbase + r * 64 + lane;
        if (idx < n) {
            const uint32_t d = digit_of(k[r], shift);
            const uint32_t pos = s_bstart[d] + s_whist[wave * RADIX + d] + rank[r];
            s_keys[pos] = k[r];
            s_vals[pos] = v[r];
        }
    }
    __syncthreads();
    for (uint32_t p = tid; p < n_valid; p += SORT_THREADS) {
        const KeyT kk = s_keys[p];
        const uint32_t dst = s_gbase[digit_of(kk, shift)] + p;
        if (dst < n) {        // always true for consistent counts; guards the bounds regardless
            kout[dst] = kk;
            vout[dst] = s_vals[p];
        }
    }
}

template <typename KeyT>
static void sort_typed(hipStream_t s, const WsDev& ws, uint32_t passes, uint32_t nb_max,
                       bool* result_in_b) {
    KeyT* ka = reinterpret_cast<KeyT*>(ws.keys_a);
    KeyT* kb = reinterpret_cast<KeyT*>(ws.keys_b);
    for (uint32_t p = 0; p < passes; ++p) {
        const bool from_a = (p % 2) == 0;
        const KeyT* kin = from_a ? ka : kb;
        hipLaunchKernelGGL(k_radix_upsweep<KeyT>, dim3(nb_max), dim3(SORT_THREADS), 0, s, kin, ws, 8 * p,
                           nb_max);
        hipLaunchKernelGGL(k_radix_offsets, dim3(RADIX), dim3(256), 0, s, ws, nb_max,
                           (uint32_t)SortTile<KeyT>::SIZE);
        hipLaunchKernelGGL(k_radix_scatter<KeyT>, dim3(nb_max), dim3(SORT_THREADS), 0, s, kin,
                           from_a ? ws.vals_a : ws.vals_b, from_a ? kb : ka, from_a ? ws.vals_b : ws.vals_a,
                           ws, 8 * p, nb_max);
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
