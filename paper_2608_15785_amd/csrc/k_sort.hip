// Depth sort of the duplicated entries and per-tile ranges (Sec. III-C, IV-A).
//
// LSD radix sort with 8-bit digits over the significant bits of the key
// (plain: 32 + b_t bits of the 64-bit key; fast: the 32-bit key, 4 passes),
// value = Gaussian index.  Eq. sort_memory counts one read and one write of
// every (key, value) entry per pass.
//
// The kernel that writes the keys (the front end) also counts every pass's
// digits into the workspace histogram and clears the first pass's look-back
// words; each pass is then one kernel over radix tiles of 4096 keys:
//   * a tile takes its index from a ticket counter, loads its keys, ranks each
//     key among equal digits of the tile with wave64 ballots (stable: tile
//     order is input order) and publishes its 256 digit counts;
//   * it then sums the counts of the tiles before it: the earlier tiles of its
//     group of SORT_GROUP, and one published total per earlier group (the last
//     tile of a group publishes the group's total).  A frame's tiles are all
//     resident at once and publish at about the same time; this two-level sum
//     keeps every tile's wait at two round trips instead of a chain through all
//     its predecessors;
//   * it reorders the tile in LDS by digit and writes it out, so consecutive
//     threads store consecutive positions of a digit bucket.
// A tile only waits on tiles with smaller tickets, which are already running,
// so the passes cannot deadlock however many tiles are resident.  The two sets
// of look-back words alternate between passes: a pass clears its tile's words
// of the set the next pass uses.
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

constexpr uint32_t SORT_READY = 0x80000000u;   // look-back word: published
constexpr int SORT_WAVES = SORT_THREADS / 64;
constexpr uint32_t SORT_SPLIT = SORT_THREADS / RADIX;   // threads per digit in the look-back
static_assert(SORT_THREADS % RADIX == 0 && SORT_THREADS >= RADIX, "whole digit rows per block");

// Exclusive scan of one value per digit (threads 0..RADIX-1; other threads
// pass anything and get an unspecified result).  Every thread of the block
// must call it: it holds two barriers.
__device__ inline uint32_t digit_exclusive_scan(uint32_t x, uint32_t* s_wtot) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    const uint32_t incl = wave_inclusive_scan(x);
    if (lane == 63 && wave < RADIX / 64) s_wtot[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < RADIX / 64; ++w)
        if ((uint32_t)w < wave) before += s_wtot[w];
    __syncthreads();
    return incl - x + before;
}

// Sum over rows r0 + s, r0 + s + SORT_SPLIT, ... < r1 of column d of a
// look-back table, waiting for each word's ready flag (bounded: on giving up
// the header's error bit 3 is set and the word counts as zero).
__device__ inline uint32_t lookback_sum(const uint32_t* tab, uint32_t r0, uint32_t r1, uint32_t s, uint32_t d,
                                        WsHeader* hdr) {
    constexpr int BATCH = 16;
    uint32_t sum = 0;
    for (uint32_t r = r0 + s; r < r1; r += BATCH * SORT_SPLIT) {
        uint32_t v[BATCH];
#pragma unroll
        for (int m = 0; m < BATCH; ++m) {
            const uint32_t rr = r + m * SORT_SPLIT;
            v[m] = rr < r1 ? ld_state(&tab[(uint64_t)rr * RADIX + d]) : SORT_READY;
        }
#pragma unroll
        for (int m = 0; m < BATCH; ++m) {
            const uint32_t rr = r + m * SORT_SPLIT;
            uint32_t spins = 0;
            while (!(v[m] & SORT_READY)) {
                if (++spins > SPIN_LIMIT) {
                    atomicOr(&hdr->error, 8u);
                    v[m] = SORT_READY;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                v[m] = ld_state(&tab[(uint64_t)rr * RADIX + d]);
            }
            sum += v[m] & ~SORT_READY;
        }
    }
    return sum;
}

template <typename KeyT>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_pass(const KeyT* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin,
                                                             KeyT* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             WsDev ws, uint32_t pass) {
    constexpr int ITEMS = SortTile<KeyT>::ITEMS;
    constexpr int SIZE = SortTile<KeyT>::SIZE;
    // per-wave digit counts, then each wave's offset inside the tile's digit
    // run; reused for the look-back's partial sums once the tile is reordered
    __shared__ uint32_t s_whist[SORT_WAVES * RADIX];
    __shared__ uint32_t s_bstart[RADIX];   // first LDS position of digit d in the reordered tile
    __shared__ uint32_t s_gbase[RADIX];    // bucket base of d, then output position minus s_bstart[d]
    __shared__ uint32_t s_tot[RADIX];      // the tile's count of digit d
    __shared__ uint32_t s_wtot[RADIX / 64];
    __shared__ uint32_t s_vb;
    __shared__ KeyT s_keys[SIZE];
    __shared__ uint32_t s_vals[SIZE];

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    // only the first ceil(n / SIZE) blocks take a ticket (tickets on one
    // address serialise); the others have no tile
    const uint32_t n = entry_count(ws.header);
    if (blockIdx.x * SIZE >= n) return;
    if (tid == 0) s_vb = atomicAdd(&ws.header->sort_ticket[pass], 1u);
    for (uint32_t i = tid; i < SORT_WAVES * RADIX; i += SORT_THREADS) s_whist[i] = 0;
    __syncthreads();
    const uint32_t vb = s_vb;
    const uint32_t tile_base = vb * SIZE;
    if (tile_base >= n) return;      // cannot happen: tickets stop at the number of blocks that take one
    const uint32_t shift = 8 * pass;
    const uint32_t n_valid = min((uint32_t)SIZE, n - tile_base);
    uint32_t* cur_tiles = sort_state_tiles(ws, pass & 1);
    uint32_t* cur_groups = sort_state_groups(ws, pass & 1);
    // the bucket sizes do not depend on this tile: start the loads first
    uint32_t bucket = 0;
    if (tid < RADIX) {
#pragma unroll
        for (int c = 0; c < HIST_COPIES; ++c) bucket += ws.hist[((uint64_t)c * MAX_PASSES + pass) * RADIX + tid];
    }

    // wave w owns entries [tile_base + w*ITEMS*64, +ITEMS*64); round r, lane l
    // holds entry tile_base + w*ITEMS*64 + r*64 + l
    const uint32_t wbase = tile_base + wave * (ITEMS * 64);
    KeyT k[ITEMS];
    uint32_t v[ITEMS];
    uint32_t rank[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = wbase + r * 64 + lane;
        const bool valid = idx < n;
        k[r] = valid ? kin[idx] : (KeyT)0;
        v[r] = valid ? vin[idx] : 0u;
    }
    // the next pass's look-back words of this tile (its set was last read by
    // the previous pass, which has finished)
    if (tid < RADIX) {
        st_state(&sort_state_tiles(ws, (pass + 1) & 1)[(uint64_t)vb * RADIX + tid], 0u);
        if (vb % SORT_GROUP == 0)
            st_state(&sort_state_groups(ws, (pass + 1) & 1)[(uint64_t)(vb / SORT_GROUP) * RADIX + tid], 0u);
    }
    const uint64_t lt = lanemask_lt();
    // Lanes of a wave read counters that other lanes of the same wave wrote in
    // the previous round.  The LDS unit executes one wave's accesses in issue
    // order; the empty asm with a memory clobber keeps the compiler from
    // moving or reusing accesses across rounds.  (A volatile pointer would do
    // the same but loses the LDS address space: every access becomes a flat
    // access that waits on all outstanding global memory operations.)
    uint32_t* my_hist = s_whist + wave * RADIX;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        asm volatile("" ::: "memory");
        const uint32_t idx = wbase + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = digit_of(k[r], shift);
        // lanes whose digit differs from this lane's: for each bit b the
        // ballot M_b of lanes holding a 1, XOR-ed with this lane's bit spread
        // to a whole word (0 or all ones), marks the lanes that disagree on b.
        // One three-input bit operation per half-mask folds M_b ^ spread into
        // the running OR (truth table 0xBE: S2 | (S0 ^ S1)).
        uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const uint32_t spread = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
            const uint64_t m = __ballot(spread != 0);
            diff_lo = __builtin_amdgcn_bitop3_b32((uint32_t)m, spread, diff_lo, 0xBE);
            diff_hi = __builtin_amdgcn_bitop3_b32((uint32_t)(m >> 32), spread, diff_hi, 0xBE);
        }
        const uint64_t vmask = __ballot(valid);
        const uint32_t peers_lo = ~diff_lo & (uint32_t)vmask, peers_hi = ~diff_hi & (uint32_t)(vmask >> 32);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(peers_hi, __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
        const uint32_t prev = valid ? my_hist[d] : 0u;
        rank[r] = prev + below;
        if (valid && below == 0) my_hist[d] = prev + (uint32_t)(__popc(peers_lo) + __popc(peers_hi));
    }
    __syncthreads();

    // digit d = tid: wave offsets and the tile's count, published at once
    uint32_t tot = 0;
    if (tid < RADIX) {
#pragma unroll
        for (int w = 0; w < SORT_WAVES; ++w) {
            const uint32_t c = s_whist[w * RADIX + tid];
            s_whist[w * RADIX + tid] = tot;
            tot += c;
        }
        st_state(&cur_tiles[(uint64_t)vb * RADIX + tid], SORT_READY | tot);
        s_tot[tid] = tot;
    }
    const uint32_t bstart = digit_exclusive_scan(tot, s_wtot);
    const uint32_t bbase = digit_exclusive_scan(bucket, s_wtot);
    if (tid < RADIX) {
        s_bstart[tid] = bstart;
        s_gbase[tid] = bbase;
    }
    __syncthreads();

    // reorder the tile by digit in LDS
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = wbase + r * 64 + lane;
        if (idx < n) {
            const uint32_t d = digit_of(k[r], shift);
            const uint32_t pos = s_bstart[d] + s_whist[wave * RADIX + d] + rank[r];
            s_keys[pos] = k[r];
            s_vals[pos] = v[r];
        }
    }
    __syncthreads();

    // keys of digit d in earlier tiles: SORT_SPLIT threads per digit share the rows
    const uint32_t d = tid % RADIX, s = tid / RADIX;
    const uint32_t g = vb / SORT_GROUP, g0 = g * SORT_GROUP;
    uint32_t* s_part = s_whist;    // [SORT_SPLIT][RADIX]
    uint32_t part = lookback_sum(cur_tiles, g0, vb, s, d, ws.header);
    if (vb % SORT_GROUP == SORT_GROUP - 1) {
        // last tile of its group: publish the group's counts before reading
        // the earlier groups, so that later groups wait as little as possible
        s_part[s * RADIX + d] = part;
        __syncthreads();
        if (tid < RADIX) {
            uint32_t gsum = s_tot[tid];
#pragma unroll
            for (uint32_t q = 0; q < SORT_SPLIT; ++q) gsum += s_part[q * RADIX + tid];
            st_state(&cur_groups[(uint64_t)g * RADIX + tid], SORT_READY | gsum);
        }
        __syncthreads();
    }
    part += lookback_sum(cur_groups, 0, g, s, d, ws.header);
    s_part[s * RADIX + d] = part;
    __syncthreads();
    if (tid < RADIX) {
        uint32_t before = 0;
#pragma unroll
        for (uint32_t q = 0; q < SORT_SPLIT; ++q) before += s_part[q * RADIX + tid];
        s_gbase[tid] = s_gbase[tid] + before - s_bstart[tid];
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
static void sort_typed(hipStream_t s, const WsDev& ws, uint32_t passes, bool* result_in_b) {
    KeyT* ka = reinterpret_cast<KeyT*>(ws.keys_a);
    KeyT* kb = reinterpret_cast<KeyT*>(ws.keys_b);
    const dim3 grid(ws.sort_rows), block(SORT_THREADS);
    for (uint32_t p = 0; p < passes; ++p) {
        const bool from_a = (p % 2) == 0;
        hipLaunchKernelGGL(k_radix_pass<KeyT>, grid, block, 0, s, from_a ? ka : kb,
                           from_a ? ws.vals_a : ws.vals_b, from_a ? kb : ka, from_a ? ws.vals_b : ws.vals_a,
                           ws, p);
    }
    *result_in_b = (passes % 2) == 1;
}

void launch_sort(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes, uint32_t passes,
                 bool* result_in_b) {
    (void)f;
    if (key_bytes == 8) sort_typed<uint64_t>(s, ws, passes, result_in_b);
    else sort_typed<uint32_t>(s, ws, passes, result_in_b);
}

// ---------------------------------------------------------------------------
// Tile ranges: the run of each tile in the sorted keys.  Entry i starts a run
// when its tile differs from entry i-1's, and ends the previous run there.
// Each thread takes RANGES_ITEMS consecutive keys with 16-byte loads.

constexpr int RANGES_ITEMS = 8;

template <typename KeyT>
__device__ inline void load_run(const KeyT* __restrict__ keys, uint64_t i0, uint32_t n, KeyT (&k)[RANGES_ITEMS]) {
    if (i0 + RANGES_ITEMS <= n) {
        // i0 is a multiple of RANGES_ITEMS and the buffers are 256-byte aligned
        const uint4* p = reinterpret_cast<const uint4*>(keys + i0);
        constexpr int VEC = RANGES_ITEMS * sizeof(KeyT) / 16;
        uint4 v[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[q] = p[q];
        __builtin_memcpy(k, v, sizeof(k));
    } else {
#pragma unroll
        for (int r = 0; r < RANGES_ITEMS; ++r) k[r] = i0 + r < n ? keys[i0 + r] : (KeyT)0;
    }
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_ranges(const KeyT* __restrict__ keys, WsDev ws,
                                                uint32_t shift, uint32_t n_tiles) {
    const uint32_t n = entry_count(ws.header);
    const uint64_t i0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * RANGES_ITEMS;
    if (i0 >= n) return;
    KeyT k[RANGES_ITEMS];
    load_run(keys, i0, n, k);
    uint32_t tp = i0 ? (uint32_t)(keys[i0 - 1] >> shift) : 0xffffffffu;
#pragma unroll
    for (int r = 0; r < RANGES_ITEMS; ++r) {
        const uint64_t i = i0 + r;
        if (i >= n) break;
        const uint32_t t = (uint32_t)(k[r] >> shift);
        if (t >= n_tiles || (i && tp >= n_tiles)) {     // only after a failed sort
            atomicOr(&ws.header->error, 4u);
            return;
        }
        if (i == 0) {
            ws.ranges[2 * t] = 0;
        } else if (tp != t) {
            ws.ranges[2 * tp + 1] = (uint32_t)i;
            ws.ranges[2 * t] = (uint32_t)i;
        }
        if (i == n - 1) ws.ranges[2 * t + 1] = n;
        tp = t;
    }
}

void launch_ranges(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes,
                   bool result_in_b) {
    const uint64_t per_block = 256ull * RANGES_ITEMS;
    const uint32_t blocks = (uint32_t)((f.capacity + per_block - 1) / per_block);
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
