// Depth sort of the duplicated entries and per-tile ranges (Sec. III-C, IV-A).
//
// LSD radix sort with 8-bit digits over the significant bits of the key
// (plain: 32 + b_t bits of the 64-bit key; fast: the 32-bit key, 4 passes),
// value = Gaussian index.  Eq. sort_memory counts one read and one write of
// every (key, value) entry per pass.
//
// The kernel that writes the keys (the front end) also counts every pass's
// digits into the workspace histogram and clears the first pass's look-back
// words; each pass is then one kernel over radix tiles of SIZE keys (4608 for
// 32-bit keys, 5632 for 64-bit ones), block b taking keys [SIZE b, SIZE (b + 1)):
//   * the tile loads its keys, ranks each key among equal digits of the tile
//     with wave64 ballots (stable: tile order is input order) and publishes
//     its 256 digit counts;
//   * it then sums the counts of the tiles before it: the earlier tiles of its
//     group of SORT_GROUP, and one published total per earlier group (the last
//     tile of a group publishes the group's total).  A frame's tiles mostly
//     run at once and publish at about the same time; this two-level sum keeps
//     every tile's wait at two round trips instead of a chain through all its
//     predecessors;
//   * it reorders the tile in LDS by digit and writes it out, so consecutive
//     threads store consecutive positions of a digit bucket.
// Nothing guarantees that the workgroups of a grid run at once or in order
// (another stream's kernels may hold the CUs), so no tile waits without
// bound: a word still unpublished after LOOKBACK_POLLS polls is replaced by
// counting that tile's keys directly (a decoupled look-back with fallback).
// Taking tiles from an atomic ticket instead, which would make waiting safe,
// costs more than the whole look-back: tickets on one address serialise at
// about 11 ns each.  The two sets of look-back words alternate between
// passes: a pass clears its tile's words of the set the next pass uses.
// Ties keep input order, and the front end emits entries in Gaussian-index
// order, so equal keys end ordered by Gaussian index.
//
// Grids are sized for the workspace capacity; the entry count is read from
// the workspace header on the device and tiles beyond it return at once, so
// no host round trip sits between the front end and the sort.
//
// The fast path's frames of 2^8 .. 2^14 tiles take the top digit first and
// the other three per bucket in LDS (the bucket sort below), which also
// writes the tile ranges.
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

// Polls of a not yet published look-back word (each a short sleep and a
// reload, a microsecond or two) before the waiting tile counts the missing row
// itself: a bound of milliseconds, far above any real wait.  When several
// streams' frames share the GPU, a running predecessor can be slow for tens of
// microseconds; 64 polls then sent ~47K rows per pass into the fallback over a
// 600-request serving burst on four streams (2040 frames/s), 4096 polls none
// (3270 frames/s).
constexpr uint32_t LOOKBACK_POLLS = 4096;

// Shared memory of the look-back (inside the pass kernel's s_whist once the
// tile is reordered): per-thread partial sums, a block-wide flag, and two
// 256-digit count rows for the fallback.
struct LookbackLds {
    uint32_t* part;     // [SORT_SPLIT][RADIX]
    uint32_t* flag;     // one word
    uint32_t* fb;       // [RADIX] digit counts of one tile
    uint32_t* acc;      // [RADIX] digit counts of one group
};

// Block-wide: fb[d] = keys of tile t (of the pass input) whose digit is d.
template <typename KeyT>
__device__ inline void count_tile(const KeyT* __restrict__ kin, uint32_t t, uint32_t n, uint32_t shift,
                                  uint32_t* fb) {
    constexpr uint32_t SIZE = SortTile<KeyT>::SIZE;
    for (uint32_t i = threadIdx.x; i < RADIX; i += SORT_THREADS) fb[i] = 0;
    __syncthreads();
    const uint32_t base = t * SIZE, cnt = min(SIZE, n - base);
    for (uint32_t i = threadIdx.x; i < cnt; i += SORT_THREADS) atomicAdd(&fb[digit_of(kin[base + i], shift)], 1u);
    __syncthreads();
}

// Block-wide: out[d] = the counts of tile row t, from its published words
// where all 256 are ready, else counted from the tile's keys.
template <typename KeyT>
__device__ inline void tile_row(const uint32_t* tiles, const KeyT* __restrict__ kin, uint32_t t, uint32_t n,
                                uint32_t shift, const LookbackLds& L, uint32_t* out, bool force) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) *L.flag = force ? 1u : 0u;
    __syncthreads();
    uint32_t w = SORT_READY;
    if (tid < RADIX && !force) {
        w = ld_state(&tiles[(uint64_t)t * RADIX + tid]);
        if (!(w & SORT_READY)) *L.flag = 1;
    }
    __syncthreads();
    if (*L.flag) {
        count_tile(kin, t, n, shift, L.fb);
        if (tid < RADIX) out[tid] = L.fb[tid];
    } else if (tid < RADIX) {
        out[tid] = w & ~SORT_READY;
    }
    __syncthreads();
}

// Keys of digit d = tid % RADIX in rows [r0, r1) of a look-back table (tile
// rows, or group rows of SORT_GROUP tiles), this thread's share: rows
// r0 + s, r0 + s + SORT_SPLIT, ... with s = tid / RADIX.  Each word is polled
// at most LOOKBACK_POLLS times; `ok` turns false when one is still unpublished.  No
// barrier: the block votes on `ok` later and, if any thread missed a word,
// takes the range again with fallback_range.
__device__ inline uint32_t poll_range(const uint32_t* tab, uint32_t r0, uint32_t r1, bool& ok) {
    constexpr int BATCH = 16;
    const uint32_t d = threadIdx.x % RADIX, s = threadIdx.x / RADIX;
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
                if (++spins > LOOKBACK_POLLS) {
                    ok = false;
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

// The same share as poll_range, taken row by row by the whole block (every
// thread calls it with the same range): each row is read from its published
// words where all 256 are there, else counted from the keys.  No tile ever
// waits on another without bound: the workgroups of a grid are not
// guaranteed to run at once.
template <typename KeyT>
__device__ uint32_t fallback_range(const WsDev& ws, uint32_t set, bool groups, uint32_t r0, uint32_t r1,
                                   const KeyT* __restrict__ kin, uint32_t n, uint32_t shift, const LookbackLds& L,
                                   bool force) {
    const uint32_t tid = threadIdx.x, d = tid % RADIX, s = tid / RADIX;
    const uint32_t* tiles = sort_state_tiles(ws, set);
    uint32_t sum = 0;
    for (uint32_t r = r0; r < r1; ++r) {
        const bool mine = (r - r0) % SORT_SPLIT == s;
        if (!groups) {
            tile_row(tiles, kin, r, n, shift, L, L.acc, force);
        } else {
            for (uint32_t i = tid; i < RADIX; i += SORT_THREADS) L.acc[i] = 0;
            __syncthreads();
            for (uint32_t t = r * SORT_GROUP; t < (r + 1) * SORT_GROUP; ++t) {
                tile_row(tiles, kin, t, n, shift, L, L.fb, force);
                if (tid < RADIX) L.acc[tid] += L.fb[tid];
                __syncthreads();
            }
        }
        if (mine) sum += L.acc[d];
        __syncthreads();
    }
    return sum;
}

// FORCE: take every look-back from the keys (fallback_range), for tests.
template <typename KeyT, bool FORCE>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_pass(const KeyT* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin,
                                                             KeyT* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             WsDev ws, uint32_t pass, uint32_t seq) {
    constexpr int ITEMS = SortTile<KeyT>::ITEMS;
    constexpr int SIZE = SortTile<KeyT>::SIZE;
    // per-wave digit counts, then each wave's offset inside the tile's digit
    // run; reused for the look-back's partial sums once the tile is reordered
    __shared__ uint32_t s_whist[SORT_WAVES * RADIX];
    __shared__ uint32_t s_bstart[RADIX];   // first LDS position of digit d in the reordered tile
    __shared__ uint32_t s_gbase[RADIX];    // bucket base of d, then output position minus s_bstart[d]
    __shared__ uint32_t s_tot[RADIX];      // the tile's count of digit d
    __shared__ uint32_t s_wtot[RADIX / 64];
    __shared__ uint32_t s_missed[2];       // look-back votes: some thread found an unpublished word
    __shared__ KeyT s_keys[SIZE];
    __shared__ uint32_t s_vals[SIZE];

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    const uint32_t n = entry_count(ws.header);
    const uint32_t vb = blockIdx.x;      // the radix tile: keys [vb * SIZE, (vb + 1) * SIZE)
    const uint32_t tile_base = vb * SIZE;
    if (tile_base >= n) return;
    for (uint32_t i = tid; i < SORT_WAVES * RADIX; i += SORT_THREADS) s_whist[i] = 0;
    if (tid < 2) s_missed[tid] = 0;
    __syncthreads();
    const uint32_t shift = 8 * pass;
    const uint32_t n_valid = min((uint32_t)SIZE, n - tile_base);
    // look-back words: set seq & 1 (launch seq of the frame's sort), the next
    // launch's set cleared below
    const uint32_t set = seq & 1;
    uint32_t* cur_tiles = sort_state_tiles(ws, set);
    uint32_t* cur_groups = sort_state_groups(ws, set);
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
        st_state(&sort_state_tiles(ws, set ^ 1u)[(uint64_t)vb * RADIX + tid], 0u);
        if (vb % SORT_GROUP == 0)
            st_state(&sort_state_groups(ws, set ^ 1u)[(uint64_t)(vb / SORT_GROUP) * RADIX + tid], 0u);
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
    const LookbackLds L{s_whist, s_whist + SORT_SPLIT * RADIX, s_whist + (SORT_SPLIT + 1) * RADIX,
                        s_whist + (SORT_SPLIT + 2) * RADIX};
    constexpr bool force = FORCE;
    bool ok = !force;
    uint32_t part = force ? 0u : poll_range(cur_tiles, g0, vb, ok);
    if (vb % SORT_GROUP == SORT_GROUP - 1) {
        // last tile of its group: publish the group's counts before reading
        // the earlier groups, so that later groups wait as little as possible
        s_part[s * RADIX + d] = part;
        if (__ballot(!ok) != 0 && lane == 0) s_missed[0] = 1;
        __syncthreads();
        if (s_missed[0]) {
            part = fallback_range(ws, set, false, g0, vb, kin, n, shift, L, force);
            s_part[s * RADIX + d] = part;
            __syncthreads();
            ok = !force;
        }
        if (tid < RADIX) {
            uint32_t gsum = s_tot[tid];
#pragma unroll
            for (uint32_t q = 0; q < SORT_SPLIT; ++q) gsum += s_part[q * RADIX + tid];
            st_state(&cur_groups[(uint64_t)g * RADIX + tid], SORT_READY | gsum);
        }
        __syncthreads();
    }
    if (!force) part += poll_range(cur_groups, 0, g, ok);
    s_part[s * RADIX + d] = part;
    if (__ballot(!ok) != 0 && lane == 0) s_missed[1] = 1;
    __syncthreads();
    if (s_missed[1]) {
        // a predecessor's counts were not published in time: take both ranges again
        part = fallback_range(ws, set, false, g0, vb, kin, n, shift, L, force) +
               fallback_range(ws, set, true, 0, g, kin, n, shift, L, force);
        s_part[s * RADIX + d] = part;
        __syncthreads();
    }
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
static void sort_typed(hipStream_t s, const WsDev& ws, uint32_t passes, bool* result_in_b, bool force) {
    KeyT* ka = reinterpret_cast<KeyT*>(ws.keys_a);
    KeyT* kb = reinterpret_cast<KeyT*>(ws.keys_b);
    const dim3 grid(ws.sort_rows), block(SORT_THREADS);
    for (uint32_t p = 0; p < passes; ++p) {
        const bool from_a = (p % 2) == 0;
        if (force)
            hipLaunchKernelGGL((k_radix_pass<KeyT, true>), grid, block, 0, s, from_a ? ka : kb,
                               from_a ? ws.vals_a : ws.vals_b, from_a ? kb : ka, from_a ? ws.vals_b : ws.vals_a,
                               ws, p, p);
        else
            hipLaunchKernelGGL((k_radix_pass<KeyT, false>), grid, block, 0, s, from_a ? ka : kb,
                               from_a ? ws.vals_a : ws.vals_b, from_a ? kb : ka, from_a ? ws.vals_b : ws.vals_a,
                               ws, p, p);
    }
    *result_in_b = (passes % 2) == 1;
}

void launch_sort(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes, uint32_t passes,
                 bool force, bool* result_in_b) {
    (void)f;
    // force (a context's RGS_DEBUG_SORT_FALLBACK, for tests): every look-back
    // counts its rows from the keys instead of reading the published words
    if (key_bytes == 8) sort_typed<uint64_t>(s, ws, passes, result_in_b, force);
    else sort_typed<uint32_t>(s, ws, passes, result_in_b, force);
}

// ---------------------------------------------------------------------------
// Bucket sort of the fast path's 32-bit keys, for frames of 2^8 .. 2^BUCKET_MAX_BT
// tile bits (FrameDev b_t).  The same stable LSD radix sort, reorganised:
//   * one radix pass as above on the top digit (key bits 24..31) moves every
//     entry to its digit's bucket, in input order.  With b_t >= 8 the top digit
//     is tile >> (b_t - 8), so a bucket holds 2^(b_t - 8) whole tiles;
//   * one workgroup per bucket then takes the bucket's three remaining digits
//     (bits 0..23), least significant first, each a stable counting pass
//     ranked through per-wave LDS digit masks (bucket_rank).  A bucket of at
//     most BK_CAP entries stays in LDS for all three; one of at most 2 BK_CAP
//     is sorted as two runs in LDS, each written back in place, and the two
//     merged; a larger one streams through global memory in chunks of BK_CAP,
//     one stable pass at a time;
//   * the same workgroup, holding its bucket sorted, writes its tiles' ranges.
// Every pass is stable and the top digit is taken first, then bits 0..23
// least significant first; as a stable sort on the top digit followed by a
// stable sort on the rest leaves the keys ordered by (top digit, rest) with
// ties in input order, the result is the LSD sort's, bit for bit.  The frame
// then needs two sort kernels instead of four passes and the ranges kernel.

constexpr int BK_THREADS = 1024;
constexpr int BK_WAVES = BK_THREADS / 64;
constexpr int BK_ITEMS = 16;
constexpr uint32_t BK_CAP = BK_THREADS * BK_ITEMS;     // 16384 entries: 128 KB of keys and values
constexpr int BK_DIGITS = 3;                             // bits 0..23 after the top digit

// Block-wide: bucket blockIdx.x is [b0, b0 + cnt) of the top-digit pass's
// output, from the front end's counts of the top digit (as that pass placed
// it), clipped to the entries the workspace holds.
__device__ inline void bucket_span(const WsDev& ws, uint32_t n, uint32_t* s_span, uint32_t* s_wtot, uint32_t& b0,
                                   uint32_t& cnt) {
    const uint32_t tid = threadIdx.x;
    uint32_t c = 0;
    if (tid < RADIX) {
#pragma unroll
        for (int h = 0; h < HIST_COPIES; ++h) c += ws.hist[((uint64_t)h * MAX_PASSES + 3) * RADIX + tid];
    }
    const uint32_t excl = digit_exclusive_scan(c, s_wtot);
    if (tid == blockIdx.x) {
        s_span[0] = excl;
        s_span[1] = c;
    }
    __syncthreads();
    b0 = s_span[0];
    cnt = b0 < n ? min(s_span[1], n - b0) : 0u;
}

// Block-wide stable ranking of up to BK_CAP keys.  Wave w holds entries
// [w R 64, (w + 1) R 64) of the chunk, round r and lane l holding entry
// (w R + r) 64 + l, with R = ceil(cnt / BK_THREADS) <= BK_ITEMS rounds, so
// that all sixteen waves share the work.  pos[r] is the key's place when the
// chunk is ordered by the digit at `shift` (ties in entry order), s_tot[d] the
// chunk's count of digit d and s_bs[d] its first place.  s_match, 4096 words
// of 64 bits, is scratch: the caller's LDS copy of the keys, which every
// thread has read into k before the call.  Every thread calls it (barriers).
//
// The lanes of a round that share a digit are found through LDS rather than
// with ballots: each lane ORs its bit into its digit's 64-bit mask in the
// wave's row of s_match, reads the mask back (a wave's LDS accesses execute
// in issue order), and the lowest lane of the digit clears it again.  Eight
// ballots and their bit operations cost about 40 VALU instructions per
// round, this a few VALU and five LDS accesses (the OR, the mask read, the
// count's read and write, the clear): the bucket kernel went from 41.9 to
// 40.2 us at 1M / 1080p.  At random digit addresses the rounds are bound by
// the LDS's bank conflicts, about half of its busy cycles.
__device__ inline void bucket_rank(const uint32_t (&k)[BK_ITEMS], uint32_t cnt, uint32_t R, uint32_t shift,
                                   uint32_t (&pos)[BK_ITEMS], uint32_t* s_whist, uint32_t* s_tot, uint32_t* s_bs,
                                   uint32_t* s_wtot, uint64_t* s_match) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    // entries of this wave that exist: round r, lane l holds one when r < R and r * 64 + l < lim
    const int lim = __builtin_amdgcn_readfirstlane((int)cnt - (int)(wave * R * 64));
    __syncthreads();            // every key read: s_match may be overwritten
    for (uint32_t i = tid; i < BK_WAVES * RADIX; i += BK_THREADS) {
        s_whist[i] = 0;
        s_match[i] = 0ull;
    }
    __syncthreads();
    uint32_t* my_hist = s_whist + wave * RADIX;
    uint64_t* my_match = s_match + wave * RADIX;
#pragma unroll
    for (int r = 0; r < BK_ITEMS; ++r) {
        if ((uint32_t)r >= R) break;
        // a wave's rounds read what its lanes wrote in the round before;
        // pos[r] holds the rank among the wave's keys of the same digit until
        // the scan below
        asm volatile("" ::: "memory");
        const bool valid = (int)lane < lim - r * 64;
        const uint32_t d = (k[r] >> shift) & (RADIX - 1);
        if (valid) atomicOr(&my_match[d], 1ull << lane);
        const uint64_t peers = valid ? my_match[d] : 0ull;
        const uint32_t below =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        const uint32_t prev = valid ? my_hist[d] : 0u;
        pos[r] = prev + below;
        if (valid && below == 0) {
            my_hist[d] = prev + (uint32_t)__popcll(peers);
            my_match[d] = 0ull;
        }
    }
    __syncthreads();
    // digit d = tid: each wave's offset inside the chunk's digit run (all
    // sixteen counts loaded before any is rewritten)
    uint32_t tot = 0;
    if (tid < RADIX) {
        uint32_t c[BK_WAVES];
#pragma unroll
        for (int w = 0; w < BK_WAVES; ++w) c[w] = s_whist[w * RADIX + tid];
#pragma unroll
        for (int w = 0; w < BK_WAVES; ++w) {
            s_whist[w * RADIX + tid] = tot;
            tot += c[w];
        }
        s_tot[tid] = tot;
    }
    const uint32_t bs = digit_exclusive_scan(tot, s_wtot);
    if (tid < RADIX) s_bs[tid] = bs;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < BK_ITEMS; ++r) {
        if ((uint32_t)r >= R) break;
        const uint32_t d = (k[r] >> shift) & (RADIX - 1);
        pos[r] += s_bs[d] + my_hist[d];
    }
}

// Sorts m <= BK_CAP entries (keys ks, values vs) by key bits 0..23 in LDS,
// three stable passes, and writes them to kd / vd.  The source may be the
// destination (everything is in LDS before the first store).  With `runs`,
// the keys are a whole bucket starting at entry b0 of the frame, and the
// tiles' runs go to ws.ranges as they are written.  Every thread calls it
// (barriers).
__device__ inline void bucket_lds_sort(const uint32_t* ks, const uint32_t* vs, uint32_t* kd, uint32_t* vd,
                                       uint32_t m, uint32_t* s_keys, uint32_t* s_vals, uint32_t* s_whist,
                                       uint32_t* s_tot, uint32_t* s_bs, uint32_t* s_wtot, uint64_t* s_match,
                                       bool runs, const WsDev& ws, uint32_t b0, uint32_t b_d, uint32_t n_tiles) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    // Entry e is held in round r < R by (wave, lane) with e = (wave R + r) 64
    // + lane, the layout of bucket_rank; the values are read after the
    // ranking, which needs only the keys.  The bounds are wave-uniform counts
    // against the lane index, so that no per-entry index stays live across
    // the passes.
    uint32_t k[BK_ITEMS], v[BK_ITEMS], pos[BK_ITEMS];
    const uint32_t R = (m + BK_THREADS - 1) / BK_THREADS;
    const uint32_t* wkeys = s_keys + wave * R * 64 + lane;
    const uint32_t* wvals = s_vals + wave * R * 64 + lane;
    const int lim = __builtin_amdgcn_readfirstlane((int)m - (int)(wave * R * 64));
    // The first pass takes its keys and values straight from global memory in
    // that layout, every load of a thread in flight at once (a load loop
    // through LDS waits for each round trip in turn).
#pragma unroll
    for (int r = 0; r < BK_ITEMS; ++r)
        k[r] = (uint32_t)r < R && (int)lane < lim - r * 64 ? ks[(wave * R + r) * 64 + lane] : 0u;
    for (int q = 0; q < BK_DIGITS; ++q) {
        if (q > 0) {
#pragma unroll
            for (int r = 0; r < BK_ITEMS; ++r)
                k[r] = (uint32_t)r < R && (int)lane < lim - r * 64 ? wkeys[r * 64] : 0u;
        }
        bucket_rank(k, m, R, 8 * q, pos, s_whist, s_tot, s_bs, s_wtot, s_match);
        if (q == 0) {
#pragma unroll
            for (int r = 0; r < BK_ITEMS; ++r)
                v[r] = (uint32_t)r < R && (int)lane < lim - r * 64 ? vs[(wave * R + r) * 64 + lane] : 0u;
        } else {
#pragma unroll
            for (int r = 0; r < BK_ITEMS; ++r)
                v[r] = (uint32_t)r < R && (int)lane < lim - r * 64 ? wvals[r * 64] : 0u;
        }
        __syncthreads();        // every entry read before any is moved
#pragma unroll
        for (int r = 0; r < BK_ITEMS; ++r)
            if ((uint32_t)r < R && (int)lane < lim - r * 64) {
                s_keys[pos[r]] = k[r];
                s_vals[pos[r]] = v[r];
            }
        __syncthreads();
    }
    for (uint32_t e = tid; e < m; e += BK_THREADS) {
        const uint32_t key = s_keys[e];
        kd[e] = key;
        vd[e] = s_vals[e];
        if (!runs) continue;
        const uint32_t t = key >> b_d;
        if (t >= n_tiles) {          // only after a failed front end
            atomicOr(&ws.header->error, 4u);
            continue;
        }
        if (e == 0 || (s_keys[e - 1] >> b_d) != t) ws.ranges[2 * t] = b0 + e;
        if (e + 1 == m || (s_keys[e + 1] >> b_d) != t) ws.ranges[2 * t + 1] = b0 + e + 1;
    }
}

// The runs of the tiles in the sorted bucket [b0, b0 + cnt) of kout, read
// back past the CU's vector cache.
__device__ inline void bucket_ranges_global(const uint32_t* kout, uint32_t b0, uint32_t cnt, const WsDev& ws,
                                            uint32_t b_d, uint32_t n_tiles) {
    for (uint32_t e = threadIdx.x; e < cnt; e += BK_THREADS) {
        const uint32_t t = ld_state(&kout[b0 + e]) >> b_d;
        if (t >= n_tiles) {
            atomicOr(&ws.header->error, 4u);
            continue;
        }
        if (e == 0 || (ld_state(&kout[b0 + e - 1]) >> b_d) != t) ws.ranges[2 * t] = b0 + e;
        if (e + 1 == cnt || (ld_state(&kout[b0 + e + 1]) >> b_d) != t) ws.ranges[2 * t + 1] = b0 + e + 1;
    }
}

// dst[e] = src[e] for e < cnt, src read past the CU's vector cache, into LDS:
// BK_LOAD_BATCH loads of a thread in flight before its LDS stores.  Every
// thread calls it.
constexpr uint32_t BK_LOAD_BATCH = 8;
__device__ inline void bucket_stage(const uint32_t* src, uint32_t cnt, uint32_t* dst) {
    for (uint32_t e0 = threadIdx.x; e0 < cnt; e0 += BK_LOAD_BATCH * BK_THREADS) {
        uint32_t t[BK_LOAD_BATCH];
#pragma unroll
        for (uint32_t j = 0; j < BK_LOAD_BATCH; ++j) {
            const uint32_t e = e0 + j * BK_THREADS;
            t[j] = e < cnt ? ld_state(&src[e]) : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < BK_LOAD_BATCH; ++j) {
            const uint32_t e = e0 + j * BK_THREADS;
            if (e < cnt) dst[e] = t[j];
        }
    }
}

// FORCE: every bucket through the global-memory path (for tests).
template <bool FORCE>
__global__ __launch_bounds__(BK_THREADS) void k_bucket_sort(const uint32_t* kin, const uint32_t* vin,
                                                            uint32_t* kout, uint32_t* vout, WsDev ws, uint32_t b_d,
                                                            uint32_t n_tiles) {
    // keys and values of up to BK_CAP entries; for a two-run merge, the keys
    // of up to 2 BK_CAP entries across both arrays
    __shared__ __align__(16) uint32_t s_lds[2 * BK_CAP];
    uint32_t* s_keys = s_lds;
    uint32_t* s_vals = s_lds + BK_CAP;
    __shared__ uint32_t s_whist[BK_WAVES * RADIX];
    // the ranking's digit masks live in the keys' LDS while the keys are in registers
    uint64_t* s_match = reinterpret_cast<uint64_t*>(s_keys);
    static_assert(BK_WAVES * RADIX * 2 <= BK_CAP, "the masks fit the keys' LDS");
    __shared__ uint32_t s_tot[RADIX];
    __shared__ uint32_t s_bs[RADIX];
    __shared__ uint32_t s_base[RADIX];
    __shared__ uint32_t s_wtot[RADIX / 64];
    __shared__ uint32_t s_span[2];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    const uint32_t n = entry_count(ws.header);
    uint32_t b0, cnt;
    bucket_span(ws, n, s_span, s_wtot, b0, cnt);
    if (cnt == 0) return;

    if (!FORCE && cnt <= 2 * BK_CAP) {
        // ---- the bucket in LDS, or in two runs: each half sorted in LDS and
        // written back in place, then the two merged ----
        const uint32_t runs = cnt <= BK_CAP ? 1u : 2u;
        const uint32_t cA = runs == 1 ? cnt : (cnt + 1) / 2, cB = cnt - cA;
        for (uint32_t h = 0; h < runs; ++h) {
            const uint32_t o = h ? cA : 0u, m = h ? cB : cA;
            uint32_t* kd = runs == 1 ? kout : const_cast<uint32_t*>(kin);
            uint32_t* vd = runs == 1 ? vout : const_cast<uint32_t*>(vin);
            bucket_lds_sort(kin + b0 + o, vin + b0 + o, kd + b0 + o, vd + b0 + o, m, s_keys, s_vals, s_whist,
                            s_tot, s_bs, s_wtot, s_match, runs == 1, ws, b0, b_d, n_tiles);
            if (h + 1 < runs) __syncthreads();     // the first run's LDS before the second's loads
        }
        if (runs == 1) return;
        // both runs' keys into LDS, read past the CU's vector cache (it may
        // hold the first run's lines from before they were sorted)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        bucket_stage(kin + b0, cnt, s_lds);
        __syncthreads();
        // Merge path: thread t writes outputs [t S, (t + 1) S).  Its first
        // output takes i entries from A and o - i from B, i the least index
        // with A[i] > B[o - i - 1]; then the two are merged sequentially, A
        // first on equal keys (A holds the earlier entries: stable).
        const uint32_t* A = s_lds;
        const uint32_t* Bk = s_lds + cA;
        const uint32_t S = (cnt + BK_THREADS - 1) / BK_THREADS;
        const uint32_t o0 = tid * S, o1 = min(o0 + S, cnt);
        if (o0 < cnt) {
            uint32_t lo = o0 > cB ? o0 - cB : 0u, hi = min(o0, cA);
            while (lo < hi) {
                const uint32_t mid = (lo + hi) / 2;
                if (A[mid] <= Bk[o0 - mid - 1]) lo = mid + 1;
                else hi = mid;
            }
            uint32_t ia = lo, ib = o0 - lo;
            // BK_LOAD_BATCH outputs at a time: their value loads in flight together
            for (uint32_t ob = o0; ob < o1; ob += BK_LOAD_BATCH) {
                uint32_t key[BK_LOAD_BATCH], val[BK_LOAD_BATCH];
#pragma unroll
                for (uint32_t j = 0; j < BK_LOAD_BATCH; ++j) {
                    if (ob + j >= o1) break;
                    const bool take_a = ib >= cB || (ia < cA && A[ia] <= Bk[ib]);
                    const uint32_t src = take_a ? ia : cA + ib;
                    key[j] = take_a ? A[ia] : Bk[ib];
                    val[j] = ld_state(&vin[b0 + src]);
                    if (take_a) ++ia;
                    else ++ib;
                }
#pragma unroll
                for (uint32_t j = 0; j < BK_LOAD_BATCH; ++j) {
                    if (ob + j >= o1) break;
                    kout[b0 + ob + j] = key[j];
                    vout[b0 + ob + j] = val[j];
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        bucket_ranges_global(kout, b0, cnt, ws, b_d, n_tiles);
        return;
    }

    uint32_t k[BK_ITEMS], v[BK_ITEMS], pos[BK_ITEMS];
    // ---- a bucket larger than the LDS ----
    // Each of the three passes streams it through global memory in chunks of
    // BK_CAP: a histogram sweep, then the chunks in order, each ranked in LDS
    // and scattered after the chunks before it.  Pass q reads src and writes
    // dst, alternating kout and the input buffer, so that the third pass ends
    // in kout.  Reads of what this workgroup wrote in the previous pass bypass
    // the CU's vector cache.
    for (int q = 0; q < BK_DIGITS; ++q) {
        const uint32_t shift = 8 * q;
        const uint32_t* ks = q == 1 ? kout : kin;
        const uint32_t* vs = q == 1 ? vout : vin;
        uint32_t* kd = q == 1 ? const_cast<uint32_t*>(kin) : kout;
        uint32_t* vd = q == 1 ? const_cast<uint32_t*>(vin) : vout;
        if (tid < RADIX) s_tot[tid] = 0;
        __syncthreads();
        for (uint32_t i0 = tid; i0 < cnt; i0 += BK_LOAD_BATCH * BK_THREADS) {
            uint32_t t[BK_LOAD_BATCH];
#pragma unroll
            for (uint32_t j = 0; j < BK_LOAD_BATCH; ++j) {
                const uint32_t i = i0 + j * BK_THREADS;
                t[j] = i < cnt ? ld_state(&ks[b0 + i]) : 0u;
            }
#pragma unroll
            for (uint32_t j = 0; j < BK_LOAD_BATCH; ++j)
                if (i0 + j * BK_THREADS < cnt) atomicAdd(&s_tot[(t[j] >> shift) & (RADIX - 1)], 1u);
        }
        __syncthreads();
        const uint32_t base = digit_exclusive_scan(tid < RADIX ? s_tot[tid] : 0u, s_wtot);
        if (tid < RADIX) s_base[tid] = base;
        __syncthreads();
        for (uint32_t c0 = 0; c0 < cnt; c0 += BK_CAP) {
            const uint32_t ccnt = min(BK_CAP, cnt - c0);
            bucket_stage(ks + b0 + c0, ccnt, s_keys);
            bucket_stage(vs + b0 + c0, ccnt, s_vals);
            __syncthreads();
            const uint32_t R = (ccnt + BK_THREADS - 1) / BK_THREADS;
            const uint32_t* wkeys = s_keys + wave * R * 64 + lane;
            const uint32_t* wvals = s_vals + wave * R * 64 + lane;
            const int lim = __builtin_amdgcn_readfirstlane((int)ccnt - (int)(wave * R * 64));
#pragma unroll
            for (int r = 0; r < BK_ITEMS; ++r)
                k[r] = (uint32_t)r < R && (int)lane < lim - r * 64 ? wkeys[r * 64] : 0u;
            bucket_rank(k, ccnt, R, shift, pos, s_whist, s_tot, s_bs, s_wtot, s_match);
#pragma unroll
            for (int r = 0; r < BK_ITEMS; ++r)
                v[r] = (uint32_t)r < R && (int)lane < lim - r * 64 ? wvals[r * 64] : 0u;
#pragma unroll
            for (int r = 0; r < BK_ITEMS; ++r) {
                if ((uint32_t)r < R && (int)lane < lim - r * 64) {
                    const uint32_t d = (k[r] >> shift) & (RADIX - 1);
                    const uint32_t dst = b0 + s_base[d] + pos[r] - s_bs[d];
                    if (dst < n) {      // always true for consistent counts
                        kd[dst] = k[r];
                        vd[dst] = v[r];
                    }
                }
            }
            // the stores reach the L2 before any thread of the workgroup reads
            // them back (the next chunk's LDS staging, the next pass, the ranges)
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid < RADIX) s_base[tid] += s_tot[tid];
            __syncthreads();
        }
    }
    bucket_ranges_global(kout, b0, cnt, ws, b_d, n_tiles);
}

bool bucket_sort_applies(const FrameDev& f, uint32_t key_bytes) {
    return key_bytes == 4 && f.b_t >= 8 && f.b_t <= BUCKET_MAX_BT;
}

void launch_sort_bucket(hipStream_t s, const FrameDev& f, const WsDev& ws, bool force, bool* result_in_b) {
    uint32_t* ka = reinterpret_cast<uint32_t*>(ws.keys_a);
    uint32_t* kb = reinterpret_cast<uint32_t*>(ws.keys_b);
    // the top digit: keys_a -> keys_b, look-back set 0 (cleared by the front end)
    if (force)
        hipLaunchKernelGGL((k_radix_pass<uint32_t, true>), dim3(ws.sort_rows), dim3(SORT_THREADS), 0, s, ka,
                           ws.vals_a, kb, ws.vals_b, ws, 3u, 0u);
    else
        hipLaunchKernelGGL((k_radix_pass<uint32_t, false>), dim3(ws.sort_rows), dim3(SORT_THREADS), 0, s, ka,
                           ws.vals_a, kb, ws.vals_b, ws, 3u, 0u);
    // each bucket: keys_b -> keys_a, with its tiles' ranges
    if (force)
        hipLaunchKernelGGL(k_bucket_sort<true>, dim3(RADIX), dim3(BK_THREADS), 0, s, kb, ws.vals_b, ka, ws.vals_a,
                           ws, (uint32_t)f.b_d, (uint32_t)f.n_tiles);
    else
        hipLaunchKernelGGL(k_bucket_sort<false>, dim3(RADIX), dim3(BK_THREADS), 0, s, kb, ws.vals_b, ka, ws.vals_a,
                           ws, (uint32_t)f.b_d, (uint32_t)f.n_tiles);
    *result_in_b = false;
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

// ---------------------------------------------------------------------------
// The rasterizers' schedule.  A tile's time grows with its list, and list
// lengths differ several-fold between tiles; workgroups are dispatched in
// grid order, so a grid that ends on long tiles leaves most CUs idle while
// they finish.  In frames that take the schedule (FrameDev::ordered),
// workgroup b renders tile order[b], where order lists the tiles of each
// chunk of ORDER_CHUNK longest first: each tile falls in one of ORDER_CLASSES
// classes of equal width in entry count (up to the chunk's longest list) and
// the classes follow one another in decreasing length (a
// longest-processing-time-first schedule; on the tile costs of the 1M / 1080p
// frame, 32 classes come within 0.2 % of an exact sort in a list-scheduling
// model).  Inside a class tiles stay in row-major order, so that tiles that
// run at about the same time still share some records in the caches.  No
// result depends on the order.
//
// One workgroup per chunk, no atomics: thread i takes tiles i, i + 1024, ...
// (round k), each wave ranks the tiles of one round within their class with
// five ballots (as the radix passes rank digits), and a scan over the
// (class, round, wave) counts places them.  The kernel takes about 10 us at
// 1M / 1080p: about 3 us to load the ranges, 2.4 us of ballots on the four
// SIMDs of a single CU, 1 us of scan and 2 us of stores; the fast rasterizer
// went from 0.123 to 0.106 ms, the plain one from 0.646 to 0.567 ms.

constexpr uint32_t ORDER_THREADS = 1024;
constexpr uint32_t ORDER_WAVES = ORDER_THREADS / 64;
constexpr uint32_t ORDER_CHUNK = 8192;
constexpr uint32_t ORDER_PER = ORDER_CHUNK / ORDER_THREADS;
constexpr uint32_t ORDER_CLASS_BITS = 5;
constexpr uint32_t ORDER_CLASSES = 1u << ORDER_CLASS_BITS;
static_assert(ORDER_CLASSES * ORDER_WAVES * ORDER_PER == 4 * ORDER_THREADS, "four (class, k, wave) groups per thread");

__global__ __launch_bounds__(ORDER_THREADS) void k_tile_order(WsDev ws, uint32_t n_tiles) {
    constexpr uint32_t GROUPS = ORDER_CLASSES * ORDER_WAVES * ORDER_PER;
    // tiles per (class, k, wave) group, class-major; the scan turns them into places
    __shared__ uint4 s_grp4[GROUPS / 4];
    __shared__ uint32_t s_red[ORDER_WAVES];
    uint32_t* s_grp = reinterpret_cast<uint32_t*>(s_grp4);
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    const uint32_t t0 = blockIdx.x * ORDER_CHUNK;
    const uint32_t t1 = min(t0 + ORDER_CHUNK, n_tiles);
    s_grp4[tid] = make_uint4(0u, 0u, 0u, 0u);
    // tile t0 + k * ORDER_THREADS + tid: its entry count, then the chunk's longest
    const uint2* __restrict__ rg = reinterpret_cast<const uint2*>(ws.ranges);
    uint32_t len[ORDER_PER];
    uint32_t longest = 0;
#pragma unroll
    for (uint32_t k = 0; k < ORDER_PER; ++k) {
        const uint32_t t = t0 + k * ORDER_THREADS + tid;
        len[k] = 0;
        if (t < t1) {
            const uint2 r = rg[t];
            len[k] = r.y > r.x ? r.y - r.x : 0u;
        }
        longest = max(longest, len[k]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) longest = max(longest, (uint32_t)__shfl_xor((int)longest, off, 64));
    if (lane == 0) s_red[wave] = longest;
    __syncthreads();
    longest = 0;
#pragma unroll
    for (uint32_t w = 0; w < ORDER_WAVES; ++w) longest = max(longest, s_red[w]);
    const float scale = (float)ORDER_CLASSES / ((float)longest + 1.0f);
    // class (0 = longest lists) and rank among the tiles of the same (wave, k) group
    uint32_t cls[ORDER_PER], rank[ORDER_PER];
#pragma unroll
    for (uint32_t k = 0; k < ORDER_PER; ++k) {
        const bool valid = t0 + k * ORDER_THREADS + tid < t1;
        const uint32_t c = ORDER_CLASSES - 1 - min(ORDER_CLASSES - 1, (uint32_t)((float)len[k] * scale));
        uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
        for (uint32_t b = 0; b < ORDER_CLASS_BITS; ++b) {
            const uint32_t spread = (uint32_t)((int32_t)(c << (31 - b)) >> 31);
            const uint64_t m = __ballot(spread != 0);
            diff_lo = __builtin_amdgcn_bitop3_b32((uint32_t)m, spread, diff_lo, 0xBE);
            diff_hi = __builtin_amdgcn_bitop3_b32((uint32_t)(m >> 32), spread, diff_hi, 0xBE);
        }
        const uint64_t vmask = __ballot(valid);
        const uint32_t peers_lo = ~diff_lo & (uint32_t)vmask, peers_hi = ~diff_hi & (uint32_t)(vmask >> 32);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(peers_hi, __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
        cls[k] = c;
        rank[k] = below;
        if (valid && below == 0)
            s_grp[(c * ORDER_PER + k) * ORDER_WAVES + wave] = (uint32_t)(__popc(peers_lo) + __popc(peers_hi));
    }
    __syncthreads();
    // places: exclusive scan of the group counts, four consecutive groups per thread
    const uint4 g = s_grp4[tid];
    const uint32_t sum4 = g.x + g.y + g.z + g.w;
    const uint32_t incl = wave_inclusive_scan(sum4);
    if (lane == 63) s_red[wave] = incl;
    __syncthreads();
    uint32_t before = incl - sum4;
    for (uint32_t w = 0; w < wave; ++w) before += s_red[w];
    s_grp4[tid] = make_uint4(before, before + g.x, before + g.x + g.y, before + g.x + g.y + g.z);
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < ORDER_PER; ++k) {
        const uint32_t t = t0 + k * ORDER_THREADS + tid;
        if (t < t1) ws.order[t0 + s_grp[(cls[k] * ORDER_PER + k) * ORDER_WAVES + wave] + rank[k]] = t;
    }
}

void launch_tile_order(hipStream_t s, const FrameDev& f, const WsDev& ws) {
    if (!f.ordered) return;
    const uint32_t n_tiles = (uint32_t)f.n_tiles;
    hipLaunchKernelGGL(k_tile_order, dim3((n_tiles + ORDER_CHUNK - 1) / ORDER_CHUNK), dim3(ORDER_THREADS), 0, s,
                       ws, n_tiles);
}

}  // namespace rgs
