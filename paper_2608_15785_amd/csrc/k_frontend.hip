// Front-end kernels: per-Gaussian preprocess, ordered duplication with keys,
// and the fused fast front end.
//
// Plain path (the 3DGS baseline, Sec. III-A/B): `preprocess_plain` projects,
// culls and colours every Gaussian and writes its record, tile rectangle,
// depth and tile count to global memory; `duplicate_plain` reads them back,
// scans the counts and emits one (64-bit key, index) entry per covered tile.
//
// Fast path (Sec. IV-A, "Preprocessing Kernel Fusion"): `frontend_fast` does
// all of it in one pass over the compact attributes.  Each thread projects one
// Gaussian and keeps its rectangle and quantised depth on chip; the block
// computes a prefix sum of the tile counts in LDS and obtains its global
// offset with one ticket atomic and a decoupled look-back over earlier blocks
// (the visible-Gaussian count rides along in the same scan, so no counter is
// incremented by every block),
// which keeps allocation in Gaussian-index order (a plain atomic per block
// would make the order, and with it the tie order of equal keys,
// nondeterministic).  The block's entries are then written cooperatively:
// consecutive threads write consecutive entries, whatever the per-Gaussian
// tile counts, so a large Gaussian does not stall its wave and the stores are
// coalesced.  Only the records of visible Gaussians and the key/index arrays
// reach global memory.
#include "rgs_internal.h"

namespace rgs {

// ---------------------------------------------------------------------------
// Spherical harmonics, degree 3, real basis with the Condon-Shortley phase
// (index l*l + l + m), evaluated in float32 (Sec. III-A: SH colour).

struct ShBasis { float y[16]; };

__device__ inline ShBasis sh_basis(float x, float y, float z) {
    ShBasis b;
    const float C0 = 0.28209479177387814f;
    const float C1 = 0.4886025119029199f;
    const float C2a = 1.0925484305920792f, C2b = 0.31539156525252005f, C2c = 0.5462742152960396f;
    const float C3a = 0.5900435899266435f, C3b = 2.890611442640554f, C3c = 0.4570457994644658f;
    const float C3d = 0.3731763325901154f, C3e = 1.445305721320277f;
    float xx = x * x, yy = y * y, zz = z * z;
    b.y[0] = C0;
    b.y[1] = -C1 * y;
    b.y[2] = C1 * z;
    b.y[3] = -C1 * x;
    b.y[4] = C2a * x * y;
    b.y[5] = -C2a * y * z;
    b.y[6] = C2b * (2.0f * zz - xx - yy);
    b.y[7] = -C2a * x * z;
    b.y[8] = C2c * (xx - yy);
    b.y[9] = -C3a * y * (3.0f * xx - yy);
    b.y[10] = C3b * x * y * z;
    b.y[11] = -C3c * y * (4.0f * zz - xx - yy);
    b.y[12] = C3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    b.y[13] = -C3c * x * (4.0f * zz - xx - yy);
    b.y[14] = C3e * z * (xx - yy);
    b.y[15] = -C3a * x * (xx - 3.0f * yy);
    return b;
}

__device__ inline ShBasis view_basis(float mx, float my, float mz, const CamDev& cam) {
    float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
    float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);     // v_rsq_f32, 1 ulp
    return sh_basis(dx * inv, dy * inv, dz * inv);
}

// FP16 bits of a non-negative value, rounded up (never below the value).
__device__ inline uint32_t half_bits_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
    if (!(f < 65504.0f)) return 0x7c00u;                 // +inf: no culling
    _Float16 h = (_Float16)f;
    uint16_t b = __builtin_bit_cast(uint16_t, h);
    if ((float)h < f) b = (uint16_t)(b + 1u);
    return b;
}

__device__ inline uint64_t pack_rect(const Projected& p) {
    return (uint64_t)(uint32_t)p.x0 | ((uint64_t)(uint32_t)p.x1 << 16) |
           ((uint64_t)(uint32_t)p.y0 << 32) | ((uint64_t)(uint32_t)p.y1 << 48);
}

__device__ inline uint32_t rect_count(uint64_t rc) {
    uint32_t x0 = rc & 0xffff, x1 = (rc >> 16) & 0xffff, y0 = (rc >> 32) & 0xffff, y1 = rc >> 48;
    return (x1 - x0 + 1) * (y1 - y0 + 1);
}

__device__ inline void write_record(Record* rec, const Projected& p, float opa, float r, float g,
                                    float b, uint32_t extra) {
    float uh = (float)p.u, vh = (float)p.v;
    float4 a = make_float4(uh, (float)(p.u - (double)uh), vh, (float)(p.v - (double)vh));
    const double idet = 1.0 / p.det;
    float4 m = make_float4((float)(p.c11 * idet), (float)(-p.c01 * idet), (float)(p.c00 * idet), opa);
    float4 c = make_float4(r, g, b, __uint_as_float(extra));
    float4* dst = reinterpret_cast<float4*>(rec);
    dst[0] = a;
    dst[1] = m;
    dst[2] = c;
}

__device__ inline void write_debug(const DebugDev& dbg, int64_t i, const Projected& p, bool vis,
                                   float r, float g, float b) {
    if (dbg.depth) dbg.depth[i] = p.d;
    if (dbg.u) dbg.u[i] = vis ? p.u : 0.0;
    if (dbg.v) dbg.v[i] = vis ? p.v : 0.0;
    if (dbg.cov2d) {
        dbg.cov2d[3 * i + 0] = vis ? p.c00 : 0.0;
        dbg.cov2d[3 * i + 1] = vis ? p.c01 : 0.0;
        dbg.cov2d[3 * i + 2] = vis ? p.c11 : 0.0;
    }
    if (dbg.rect) {
        dbg.rect[4 * i + 0] = vis ? (int32_t)p.x0 : 0;
        dbg.rect[4 * i + 1] = vis ? (int32_t)p.x1 : 0;
        dbg.rect[4 * i + 2] = vis ? (int32_t)p.y0 : 0;
        dbg.rect[4 * i + 3] = vis ? (int32_t)p.y1 : 0;
    }
    if (dbg.visible) dbg.visible[i] = vis ? 1 : 0;
    if (dbg.color) {
        dbg.color[3 * i + 0] = vis ? r : 0.0f;
        dbg.color[3 * i + 1] = vis ? g : 0.0f;
        dbg.color[3 * i + 2] = vis ? b : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Frame reset: copy the frame's parameters into the workspace, zero the
// header, the tile ranges, the front-end scan state and the digit buckets.

__global__ void k_reset(ResetArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.dst = a.prm;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_words; i += stride) {
        uint32_t v = 0;
        if (i == offsetof(WsHeader, capacity) / 4) v = a.capacity;
        if (i == offsetof(WsHeader, path) / 4) v = a.path;
        if (i == offsetof(WsHeader, passes) / 4) v = a.passes;
        a.base[i] = v;
    }
}

ResetArgs reset_args(const WsDev& ws, uint64_t zero_bytes, const FrameDev& f, uint32_t path,
                     const FrameParams& prm) {
    ResetArgs a{};
    a.base = reinterpret_cast<uint32_t*>(ws.header);
    a.n_words = zero_bytes / 4;
    a.capacity = f.capacity;
    a.path = path;
    a.passes = (uint32_t)f.passes;
    a.dst = const_cast<FrameParams*>(ws.params);
    a.prm = prm;
    return a;
}

void launch_reset(hipStream_t s, const ResetArgs& a) {
    uint32_t blocks = (uint32_t)((a.n_words + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, s, a);
}

const void* reset_kernel() { return reinterpret_cast<const void*>(&k_reset); }

// Copy the frame's outcome from the header to host-visible memory.
__global__ void k_export_status(const WsHeader* h, const FrameParams* prm, FrameStatus* dst) {
    if (threadIdx.x == 0) {
        FrameStatus st;
        st.n_entries = h->n_entries;
        st.n_visible = h->n_visible;
        st.overflow = h->overflow;
        st.error = h->error;
        st.done = 1;
        st.out = reinterpret_cast<uint64_t>(prm->out);
        *dst = st;
    }
}

void launch_export_status(hipStream_t s, const WsDev& ws, FrameStatus* dst) {
    hipLaunchKernelGGL(k_export_status, dim3(1), dim3(64), 0, s, ws.header, ws.params, dst);
}

__global__ void k_export_stamp(const WsHeader* h, const FrameParams* prm, FrameStamp* dst, uint64_t seq) {
    if (threadIdx.x == 0) {
        dst->n_entries = h->n_entries;
        dst->overflow = h->overflow;
        dst->error = h->error;
        dst->scene_tag = prm->scene_tag;
        dst->cam_hash = prm->cam_hash;
        __threadfence_system();
        __hip_atomic_store(&dst->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

void launch_export_stamp(hipStream_t s, const WsDev& ws, FrameStamp* dst, uint64_t seq) {
    hipLaunchKernelGGL(k_export_stamp, dim3(1), dim3(64), 0, s, ws.header, ws.params, dst, seq);
}

// ---------------------------------------------------------------------------
// Chained scan across blocks (decoupled look-back).  Block vb publishes its
// aggregate (entries, visible Gaussians), then sums predecessors' aggregates
// until it meets an inclusive prefix.  One wave polls 64 x LB_PER_LANE
// predecessors per round trip, nearest first.  Blocks take vb from a ticket
// counter, so a block only ever waits on blocks that are already running.

__device__ void chained_exclusive(uint64_t* states, uint32_t vb, uint64_t agg_e, uint64_t agg_v,
                                  WsHeader* hdr, uint64_t& ex_e, uint64_t& ex_v) {
    const uint32_t lane = lane_id();
    ex_e = 0;
    ex_v = 0;
    if (vb == 0) {
        if (lane == 0) st_state(&states[0], ST_PRE | st_pack(agg_e, agg_v));
        return;
    }
    if (lane == 0) st_state(&states[vb], ST_AGG | st_pack(agg_e, agg_v));
    const uint64_t my_bit = 1ull << lane;
    int64_t top = (int64_t)vb - 1;
    uint32_t spins = 0;
    while (true) {
        uint64_t s[LB_PER_LANE];
#pragma unroll
        for (int m = 0; m < LB_PER_LANE; ++m) {
            const int64_t idx = top - (int64_t)(lane * LB_PER_LANE + m);
            s[m] = idx >= 0 ? ld_state(&states[idx]) : ST_PRE;    // before block 0: prefix 0
        }
        uint64_t le = 0, lv = 0;
        bool has_pre = false, bad = false;
#pragma unroll
        for (int m = 0; m < LB_PER_LANE; ++m) {
            if (has_pre || bad) continue;
            const uint64_t f = s[m] & ~ST_VAL;
            if (f == 0) {
                bad = true;
            } else {
                le += st_entries(s[m]);
                lv += st_visible(s[m]);
                has_pre = f == ST_PRE;
            }
        }
        const uint64_t pre = __ballot(has_pre);
        const uint64_t badm = __ballot(bad);
        // lanes up to and including the nearest one holding a prefix (all if none)
        const uint64_t upto = pre ? ((pre & (~pre + 1)) << 1) - 1 : ~0ull;
        if (badm & upto) {
            if (++spins > SPIN_LIMIT) {
                if (lane == 0) atomicOr(&hdr->error, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        ex_e += wave_sum((my_bit & upto) ? le : 0ull);
        ex_v += wave_sum((my_bit & upto) ? lv : 0ull);
        if (pre) break;
        top -= 64 * LB_PER_LANE;
    }
    if (lane == 0) st_state(&states[vb], ST_PRE | st_pack(ex_e + agg_e, ex_v + agg_v));
}

// Block-wide inclusive scan of FE_ITEMS rows of per-thread counts (Gaussian
// j = k * FE_THREADS + tid of the block sits in row k), leaving s_incl[j], then
// the block's global base by chained scan.  Returns the block's entry total;
// *s_base / *s_base_v receive the exclusive entry and visible counts.  Every
// wave scans its share of all rows at once; the FE_ITEMS x WAVES wave totals
// (one wave's worth) are then scanned by wave 0 in row-major order, so the
// block takes two barriers instead of two per row.  s_wtot holds
// FE_ITEMS * WAVES + 1 words.
__device__ inline uint32_t block_scan_and_chain(const uint32_t (&count)[FE_ITEMS], uint32_t n_vis,
                                                uint32_t vb, WsDev& ws, uint32_t* s_incl,
                                                uint32_t* s_wtot, uint32_t* s_wvis, uint64_t* s_base,
                                                uint64_t* s_base_v, uint32_t* vis_total) {
    constexpr int WAVES = FE_THREADS / 64;
    static_assert(FE_ITEMS * WAVES <= 64, "one wave scans the wave totals");
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    const uint32_t wv = wave_sum(n_vis);
    if (lane == 0) s_wvis[wave] = wv;
    uint32_t incl[FE_ITEMS];
#pragma unroll
    for (int k = 0; k < FE_ITEMS; ++k) {
        incl[k] = wave_inclusive_scan(count[k]);
        if (lane == 63) s_wtot[k * WAVES + wave] = incl[k];
    }
    __syncthreads();
    if (wave == 0) {
        const uint32_t t = lane < (uint32_t)(FE_ITEMS * WAVES) ? s_wtot[lane] : 0u;
        const uint32_t in = wave_inclusive_scan(t);
        if (lane < (uint32_t)(FE_ITEMS * WAVES)) s_wtot[lane] = in - t;
        if (lane == 63) s_wtot[FE_ITEMS * WAVES] = in;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < FE_ITEMS; ++k) s_incl[k * FE_THREADS + threadIdx.x] = s_wtot[k * WAVES + wave] + incl[k];
    const uint32_t carry = s_wtot[FE_ITEMS * WAVES];
    uint32_t vtot = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) vtot += s_wvis[w];
    *vis_total = vtot;
    if (wave == 0) {
        uint64_t ex_e, ex_v;
        chained_exclusive(ws.fe_state, vb, carry, vtot, ws.header, ex_e, ex_v);
        if (lane == 0) {
            *s_base = ex_e;
            *s_base_v = ex_v;
        }
    }
    __syncthreads();
    return carry;
}

// Position of the k-th (from 0) set bit of m, which has more than k set bits.
__device__ inline uint32_t nth_set_bit(uint64_t m, uint32_t k) {
    uint32_t pos = 0;
#pragma unroll
    for (int half = 32; half > 0; half >>= 1) {
        const uint64_t low = m & ((1ull << half) - 1);
        const uint32_t c = (uint32_t)__popcll(low);
        if (k >= c) {
            k -= c;
            m >>= half;
            pos += half;
        } else {
            m = low;
        }
    }
    return pos;
}

// Entry e of the block belongs to the Gaussian j with s_incl[j-1] <= e < s_incl[j]
// and is the (e - s_incl[j-1])-th tile of j's rectangle in row-major order, or
// of its kept tiles when s_mask holds them (rectangles of at most
// EXACT_TILE_MAX_AREA tiles).
// Each stored key also counts its digits of radix passes p_first..passes-1
// into the block's LDS histogram s_h[pass][digit] (the passes before p_first
// read only the depth bits, which all entries of a Gaussian share: those are
// counted once per Gaussian by count_depth_digits).  A wave whose stored keys
// all share a digit adds it once (the high digits of neighbouring entries are
// often equal, and LDS atomics on one address serialise).
// Entries are taken EMIT_ILP per thread at a time (e, e + FE_THREADS, ...),
// whose searches for their Gaussian advance in lockstep: the search is a
// chain of dependent LDS reads, and the independent chains share its latency.
constexpr int EMIT_ILP = 4;
static_assert((FE_TILE & (FE_TILE - 1)) == 0, "the search takes log2(FE_TILE) halving steps");

template <typename KeyT, typename KeyFn>
__device__ inline void emit_entries(uint32_t total, uint64_t base, const uint32_t* s_incl,
                                    const uint64_t* s_rect, uint32_t first_gauss, int tiles_x,
                                    uint32_t capacity, KeyT* keys, uint32_t* vals, KeyFn key_of,
                                    uint32_t* s_h, uint32_t p_first, uint32_t passes, const uint64_t* s_mask) {
    for (uint32_t e0 = threadIdx.x; e0 < total; e0 += EMIT_ILP * FE_THREADS) {
        // j = #{i : s_incl[i] <= e}, the first Gaussian whose inclusive count
        // exceeds e, by binary lifting: after the steps of 2^k and above, j
        // <= FE_TILE - 2^k, so every index read is below FE_TILE (an e at or
        // past the total ends on some j < FE_TILE and is not emitted)
        uint32_t j[EMIT_ILP];
#pragma unroll
        for (int u = 0; u < EMIT_ILP; ++u) j[u] = 0;
#pragma unroll
        for (uint32_t step = FE_TILE / 2; step >= 1; step >>= 1) {
#pragma unroll
            for (int u = 0; u < EMIT_ILP; ++u)
                if (s_incl[j[u] + step - 1] <= e0 + u * FE_THREADS) j[u] += step;
        }
#pragma unroll
        for (int u = 0; u < EMIT_ILP; ++u) {
            const uint32_t e = e0 + u * FE_THREADS;
            if (e >= total) break;
            const uint32_t local = e - (j[u] ? s_incl[j[u] - 1] : 0u);
            const uint64_t rc = s_rect[j[u]];
            const uint32_t x0 = rc & 0xffff, x1 = (rc >> 16) & 0xffff, y0 = (rc >> 32) & 0xffff;
            const uint32_t w = x1 - x0 + 1;
            uint32_t b = local;            // row-major index of the tile in the rectangle
            if (s_mask && w * ((uint32_t)(rc >> 48) - y0 + 1) <= EXACT_TILE_MAX_AREA)
                b = nth_set_bit(s_mask[j[u]], local);
            // b / w and b % w: b < 2^20 (a rectangle holds at most 2^20 tiles)
            // and w <= 1024, so the float quotient is within 0.25 of b / w and
            // one correction of its truncation makes it exact
            uint32_t q = (uint32_t)((float)b * __builtin_amdgcn_rcpf((float)w));
            int32_t rem = (int32_t)b - (int32_t)(q * w);
            if (rem < 0) {
                q -= 1;
                rem += (int32_t)w;
            } else if (rem >= (int32_t)w) {
                q += 1;
                rem -= (int32_t)w;
            }
            const uint32_t ty = y0 + q;
            const uint32_t tx = x0 + (uint32_t)rem;
            const uint32_t tile = ty * (uint32_t)tiles_x + tx;
            const uint64_t pos = base + e;
            const bool stored = pos < capacity;
            const KeyT key = key_of(tile, j[u]);
            if (stored) {
                keys[pos] = key;
                vals[pos] = first_gauss + j[u];
            }
            const uint64_t active = __ballot(true);
            const bool all_stored = __ballot(stored) == active;
            for (uint32_t p = p_first; p < passes; ++p) {
                const uint32_t dg = (uint32_t)(key >> (RADIX_BITS * p)) & (RADIX - 1);
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                if (all_stored && __ballot(dg == d0) == active) {
                    if (lane_id() == (uint32_t)__builtin_ctzll(active))
                        atomicAdd(&s_h[p * RADIX + d0], (uint32_t)__popcll(active));
                } else if (stored) {
                    atomicAdd(&s_h[p * RADIX + dg], 1u);
                }
            }
        }
    }
}

// The radix sort's inputs that the front end prepares alongside the keys:
// digit counts (the block's LDS histogram added into histogram copy
// vb % HIST_COPIES) and zeroed look-back words of the first pass for every
// radix tile that starts inside this block's entries.  Call after the emission
// and a barrier.
template <typename KeyT>
__device__ inline void prepare_sort(WsDev& ws, const uint32_t* s_h, uint32_t passes, uint32_t vb, uint64_t base,
                                    uint32_t total) {
    uint32_t* copy = ws.hist + (uint64_t)(vb % HIST_COPIES) * MAX_PASSES * RADIX;
    for (uint32_t i = threadIdx.x; i < passes * RADIX; i += FE_THREADS) {
        const uint32_t c = s_h[i];
        if (c) atomicAdd(&copy[i], c);
    }
    constexpr uint64_t SIZE = SortTile<KeyT>::SIZE;
    const uint64_t t0 = (base + SIZE - 1) / SIZE;
    uint64_t t1 = (base + total + SIZE - 1) / SIZE;
    if (t1 > ws.sort_rows) t1 = ws.sort_rows;
    uint32_t* tiles = sort_state_tiles(ws, 0);
    uint32_t* groups = sort_state_groups(ws, 0);
    for (uint64_t t = t0; t < t1; ++t) {
        for (uint32_t i = threadIdx.x; i < RADIX; i += FE_THREADS) {
            st_state(&tiles[t * RADIX + i], 0u);
            if (t % SORT_GROUP == 0) st_state(&groups[(t / SORT_GROUP) * RADIX + i], 0u);
        }
    }
}

__device__ inline void zero_hist(uint32_t* s_h) {
    for (uint32_t i = threadIdx.x; i < MAX_PASSES * RADIX; i += FE_THREADS) s_h[i] = 0;
}

// Radix passes whose digit lies wholly below bit `shift` of the key (the depth
// bits) come first; their digits are the same for all entries of a Gaussian.
__device__ inline uint32_t depth_only_passes(uint32_t shift, uint32_t passes) {
    const uint32_t p = shift / RADIX_BITS;
    return p < passes ? p : passes;
}

// The entries of a block's Gaussian j share its depth bits low[j]: add the
// digits of the depth-only passes once per Gaussian, weighted by how many of
// its entries fit in the workspace (entries at or past `capacity` are not
// stored, and the sort counts only stored keys).
__device__ inline void count_depth_digits(uint32_t* s_h, const uint32_t (&count)[FE_ITEMS], const uint32_t* low,
                                          const uint32_t* s_incl, uint64_t base, uint32_t capacity,
                                          uint32_t p_depth) {
    if (p_depth == 0) return;
#pragma unroll
    for (int k = 0; k < FE_ITEMS; ++k) {
        const uint32_t j = k * FE_THREADS + threadIdx.x;
        if (!count[k]) continue;
        const uint64_t start = base + (j ? s_incl[j - 1] : 0u);
        const uint64_t room = start < capacity ? capacity - start : 0u;
        const uint32_t stored = room < count[k] ? (uint32_t)room : count[k];
        if (!stored) continue;
        for (uint32_t p = 0; p < p_depth; ++p)
            atomicAdd(&s_h[p * RADIX + ((low[j] >> (RADIX_BITS * p)) & (RADIX - 1))], stored);
    }
}

__device__ inline void finish_block(WsDev& ws, uint32_t vb, uint32_t n_blocks, uint64_t base,
                                    uint64_t base_v, uint32_t total, uint32_t vis_total,
                                    uint32_t capacity) {
    if (vb == n_blocks - 1 && threadIdx.x == 0) {
        const uint64_t n = base + total;
        ws.header->n_entries = n;
        ws.header->n_visible = (uint32_t)(base_v + vis_total);
        ws.header->overflow = n > capacity ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// Plain preprocess: one thread per Gaussian over the FP32 planes.

// TRAIN (the plain path's training variant): the same projection, colour and
// 3-sigma tile rectangle, but the record holds ln o and the FP16 box of the
// alpha >= 1/255 ellipse, as the fast path's records do, for the dual-pixel
// rasterizer with culled lists.  Entries and keys are the plain path's.
template <bool DEBUG, bool TRAIN>
__global__ __launch_bounds__(256) void k_preprocess_plain(PlainSceneDev sc, FrameDev f, WsDev ws,
                                                          DebugDev dbg) {
    const CamDev cam = ws.params->cam;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool in = i < sc.n;
    bool vis = false;
    if (in) {
        const float* P = sc.base;
        const uint64_t np = sc.n_pad;
        float mx = P[P_MX * np + i], my = P[P_MY * np + i], mz = P[P_MZ * np + i];
        Projected pr;
        const double lno = TRAIN ? (double)P[P_LNO * np + i] : 0.0;
        vis = project_gaussian(cam, mx, my, mz, P[P_QW * np + i], P[P_QX * np + i],
                               P[P_QY * np + i], P[P_QZ * np + i], P[P_SX * np + i],
                               P[P_SY * np + i], P[P_SZ * np + i], TRAIN, lno,
                               (double)f.tiles_x, (double)f.tiles_y, pr, false);
        float r = 0.f, g = 0.f, b = 0.f;
        if (vis) {
            ShBasis y = view_basis(mx, my, mz, cam);
            float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
            for (int k = 0; k < 16; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch)
                    acc[ch] = fmaf(y.y[k], P[(P_SH0 + 3 * k + ch) * np + i], acc[ch]);
            r = fmaxf(acc[0], 0.f);
            g = fmaxf(acc[1], 0.f);
            b = fmaxf(acc[2], 0.f);
            if (TRAIN) {
                // no pixel reaches alpha >= 1/255 when ln o < -ln 255: an empty box
                const uint32_t box = LN255 + lno > 0.0 ? half_bits_up(pr.ax) | (half_bits_up(pr.ay) << 16) : 0u;
                write_record(&ws.records[i], pr, (float)lno, r, g, b, box);
            } else {
                write_record(&ws.records[i], pr, P[P_OPA * np + i], r, g, b, __float_as_uint((float)pr.d));
            }
            uint64_t rc = pack_rect(pr);
            ws.rects[i] = rc;
            ws.depths[i] = (float)pr.d;
            ws.counts[i] = rect_count(rc);
        } else {
            ws.counts[i] = 0;
        }
        if (DEBUG) write_debug(dbg, i, pr, vis, r, g, b);
    }
}

void launch_preprocess_plain(hipStream_t s, const PlainSceneDev& sc, const FrameDev& f,
                             const WsDev& ws, const DebugDev* dbg, bool train) {
    const uint32_t blocks = (uint32_t)((sc.n + 255) / 256);
    const DebugDev d = dbg ? *dbg : DebugDev{};
    if (dbg && train) hipLaunchKernelGGL((k_preprocess_plain<true, true>), dim3(blocks), dim3(256), 0, s, sc, f, ws, d);
    else if (dbg) hipLaunchKernelGGL((k_preprocess_plain<true, false>), dim3(blocks), dim3(256), 0, s, sc, f, ws, d);
    else if (train) hipLaunchKernelGGL((k_preprocess_plain<false, true>), dim3(blocks), dim3(256), 0, s, sc, f, ws, d);
    else hipLaunchKernelGGL((k_preprocess_plain<false, false>), dim3(blocks), dim3(256), 0, s, sc, f, ws, d);
}

// ---------------------------------------------------------------------------
// Duplication over the stored counts (the plain path, and the fast path with
// fusion ablated): ordered allocation, then (tile << shift | low bits) keys,
// where the low bits are the float32 depth (shift 32) or the quantised depth
// (shift b_d) kept as a word in `depths`.

template <typename KeyT>
__global__ __launch_bounds__(FE_THREADS) void k_duplicate(int64_t n, FrameDev f, WsDev ws, uint32_t n_blocks,
                                                          uint32_t per,
                                                          uint32_t shift) {
    __shared__ uint32_t s_vb;
    __shared__ uint32_t s_incl[FE_TILE];
    __shared__ uint64_t s_rect[FE_TILE];
    __shared__ uint32_t s_dbits[FE_TILE];
    __shared__ uint64_t s_mask[FE_TILE];
    __shared__ uint32_t s_wtot[FE_ITEMS * FE_THREADS / 64 + 1];
    __shared__ uint32_t s_wvis[FE_THREADS / 64];
    __shared__ uint64_t s_base, s_base_v;
    __shared__ uint32_t s_h[MAX_PASSES * RADIX];
    if (threadIdx.x == 0) s_vb = atomicAdd(&ws.header->fe_ticket, 1u);
    zero_hist(s_h);
    __syncthreads();
    const uint32_t vb = s_vb;
    const uint32_t p_depth = depth_only_passes(shift, (uint32_t)f.passes);
    uint32_t count[FE_ITEMS];
    uint32_t n_vis = 0;
#pragma unroll
    for (int k = 0; k < FE_ITEMS; ++k) {
        const uint32_t j = k * FE_THREADS + threadIdx.x;
        const int64_t i = (int64_t)vb * per + j;
        count[k] = 0;
        if (j < per && i < n) {
            count[k] = ws.counts[i];
            if (count[k]) {
                s_rect[j] = ws.rects[i];
                s_dbits[j] = __float_as_uint(ws.depths[i]);
                if (ws.masks) s_mask[j] = ws.masks[i];
                ++n_vis;
            }
        }
    }
    uint32_t vis_total;
    const uint32_t total = block_scan_and_chain(count, n_vis, vb, ws, s_incl, s_wtot, s_wvis, &s_base,
                                                &s_base_v, &vis_total);
    const uint64_t base = s_base;
    // where each Gaussian's entries start in emission order (the backward pass
    // gathers a Gaussian's per-entry partials from there)
#pragma unroll
    for (int k = 0; k < FE_ITEMS; ++k) {
        const uint32_t j = k * FE_THREADS + threadIdx.x;
        const int64_t i = (int64_t)vb * per + j;
        if (j < per && i < n && count[k]) ws.offsets[i] = (uint32_t)(base + (j ? s_incl[j - 1] : 0u));
    }
    count_depth_digits(s_h, count, s_dbits, s_incl, base, f.capacity, p_depth);
    emit_entries<KeyT>(total, base, s_incl, s_rect, vb * per, f.tiles_x, f.capacity,
                       reinterpret_cast<KeyT*>(ws.keys_a), ws.vals_a,
                       [&](uint32_t tile, uint32_t j) { return ((KeyT)tile << shift) | (KeyT)s_dbits[j]; },
                       s_h, p_depth, (uint32_t)f.passes, ws.masks ? s_mask : nullptr);
    __syncthreads();
    prepare_sort<KeyT>(ws, s_h, (uint32_t)f.passes, vb, base, total);
    finish_block(ws, vb, n_blocks, base, s_base_v, total, vis_total, f.capacity);
}

void launch_duplicate(hipStream_t s, int64_t n, const FrameDev& f, const WsDev& ws, uint32_t fe_blocks, uint32_t fe_per,
                      uint32_t key_bytes) {
    if (key_bytes == 8)
        hipLaunchKernelGGL(k_duplicate<uint64_t>, dim3(fe_blocks), dim3(FE_THREADS), 0, s, n, f, ws, fe_blocks,
                           fe_per, 32u);
    else
        hipLaunchKernelGGL(k_duplicate<uint32_t>, dim3(fe_blocks), dim3(FE_THREADS), 0, s, n, f, ws, fe_blocks,
                           fe_per, (uint32_t)f.b_d);
}

// ---------------------------------------------------------------------------
// Fused fast front end over the compact planes: project, cull, colour, scan,
// allocate in order and emit 32-bit (tile << b_d | q_d) keys.

// Project, cull and colour Gaussian i of the compact planes.  Returns its tile
// count (0 when culled) and leaves its rectangle and the low part of its key
// (the quantised depth; the float32 depth bits when the 32-bit key is
// ablated).  `opts` holds the ablation bits the generic instances honour; the
// production instance passes 0 and the compiler drops every ablation branch.
template <bool DEBUG>
__device__ inline uint32_t fast_gaussian(const FastSceneDev& sc, const CamDev& cam, const FrameDev& f,
                                         WsDev& ws, const DebugDev& dbg, int64_t i, uint64_t& rect,
                                         uint32_t& klo, uint64_t& mask, uint32_t opts) {
    const uint32_t* W = sc.base;
    const uint64_t np = sc.n_pad;
    const float mx = __uint_as_float(W[F_MX * np + i]);
    const float my = __uint_as_float(W[F_MY * np + i]);
    const float mz = __uint_as_float(W[F_MZ * np + i]);
    float qw, qx, qy, qz, sx, sy, sz, lno;
    if (opts & OPT_FP16_GEOM) {
        const float* P = sc.plain;
        qw = P[P_QW * np + i]; qx = P[P_QX * np + i]; qy = P[P_QY * np + i]; qz = P[P_QZ * np + i];
        sx = P[P_SX * np + i]; sy = P[P_SY * np + i]; sz = P[P_SZ * np + i];
        lno = P[P_LNO * np + i];
    } else {
        const uint32_t qwx = W[F_QWX * np + i], qyz = W[F_QYZ * np + i];
        const uint32_t sxy = W[F_SXY * np + i], szl = W[F_SZL * np + i];
        qw = half_lo(qwx); qx = half_hi(qwx); qy = half_lo(qyz); qz = half_hi(qyz);
        sx = half_lo(sxy); sy = half_hi(sxy); sz = half_lo(szl);
        lno = half_hi(szl);
    }
    // the quantised SH words are loaded before the projection, whose FP64
    // arithmetic then covers their latency (nearly every Gaussian of a scene
    // in view is visible, so the culled ones' loads cost little)
    uint32_t qwd[12], sw[6];
    if (!(opts & OPT_INT8_SH)) {
#pragma unroll
        for (int k = 0; k < 12; ++k) qwd[k] = W[(F_SHQ0 + k) * np + i];
#pragma unroll
        for (int k = 0; k < 6; ++k) sw[k] = W[(F_SHS0 + k) * np + i];
        // keeps the compiler from sinking the loads to their use
        asm volatile("" ::: "memory");
    }
    Projected pr;
    const bool vis = project_gaussian(cam, mx, my, mz, qw, qx, qy, qz, sx, sy, sz, true, (double)lno,
                                      (double)f.tiles_x, (double)f.tiles_y, pr, !(opts & OPT_EXTENT));
    float r = 0.f, g = 0.f, b = 0.f;
    uint32_t count = 0;
    if (vis) {
        const ShBasis y = view_basis(mx, my, mz, cam);
        float acc[3] = {0.5f, 0.5f, 0.5f};
        if (opts & OPT_INT8_SH) {
            const float* P = sc.plain;
#pragma unroll
            for (int k = 0; k < 16; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) acc[ch] = fmaf(y.y[k], P[(P_SH0 + 3 * k + ch) * np + i], acc[ch]);
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int deg = k == 0 ? 0 : (k < 4 ? 1 : (k < 9 ? 2 : 3));
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const int v = 3 * k + ch;
                    const float q = (float)(int8_t)((qwd[v >> 2] >> (8 * (v & 3))) & 0xffu);
                    const int si = 3 * deg + ch;
                    const float scale = (si & 1) ? half_hi(sw[si >> 1]) : half_lo(sw[si >> 1]);
                    acc[ch] = fmaf(y.y[k], q * scale, acc[ch]);
                }
            }
        }
        r = fmaxf(acc[0], 0.f);
        g = fmaxf(acc[1], 0.f);
        b = fmaxf(acc[2], 0.f);
        write_record(&ws.records[i], pr, lno, r, g, b, half_bits_up(pr.ax) | (half_bits_up(pr.ay) << 16));
        rect = pack_rect(pr);
        klo = (opts & OPT_KEY32) ? __float_as_uint((float)pr.d) : quantize_depth(pr.d, cam.zn, cam.zf, f.b_d);
        count = rect_count(rect);
        mask = 0;
        if ((opts & OPT_EXACT_TILES) && count <= EXACT_TILE_MAX_AREA) {
            // the exact ellipse-tile test: bit r * w + c for tile (x0 + c, y0 + r)
            const uint32_t w = (uint32_t)(pr.x1 - pr.x0) + 1, h = (uint32_t)(pr.y1 - pr.y0) + 1;
            const double tau = 2.0 * (LN255 + (double)lno);
            for (uint32_t rr = 0; rr < h; ++rr)
                for (uint32_t cc = 0; cc < w; ++cc)
                    if (ellipse_meets_tile(pr.u, pr.v, pr.c00, pr.c01, pr.c11, pr.det, tau,
                                           16.0 * (pr.x0 + (double)cc), 16.0 * (pr.y0 + (double)rr)))
                        mask |= 1ull << (rr * w + cc);
            count = (uint32_t)__popcll(mask);
        }
    }
    if (DEBUG) write_debug(dbg, i, pr, vis, r, g, b);
    return count;
}

// The fused front end: project, cull, colour, scan, allocate in order, emit.
// KeyT is uint32_t for (tile << b_d | q_d) keys and uint64_t for the plain
// path's (tile << 32 | float32 depth bits) keys (the key ablation); GENERIC
// instances honour the ablation bits in `opts`, the production one ignores it.
template <bool DEBUG, bool GENERIC, typename KeyT>
__global__ __launch_bounds__(FE_THREADS) void k_frontend_fast(FastSceneDev sc, FrameDev f, WsDev ws,
                                                              uint32_t n_blocks, uint32_t per, DebugDev dbg,
                                                              uint32_t opts_arg) {
    const CamDev cam = ws.params->cam;
    const uint32_t opts = GENERIC ? opts_arg : 0u;
    __shared__ uint32_t s_vb;
    __shared__ uint32_t s_incl[FE_TILE];
    __shared__ uint64_t s_rect[FE_TILE];
    __shared__ uint32_t s_qd[FE_TILE];
    __shared__ uint64_t s_mask[FE_TILE];
    __shared__ uint32_t s_wtot[FE_ITEMS * FE_THREADS / 64 + 1];
    __shared__ uint32_t s_wvis[FE_THREADS / 64];
    __shared__ uint64_t s_base, s_base_v;
    __shared__ uint32_t s_h[MAX_PASSES * RADIX];
    if (threadIdx.x == 0) s_vb = atomicAdd(&ws.header->fe_ticket, 1u);
    zero_hist(s_h);
    __syncthreads();
    const uint32_t vb = s_vb;
    const uint32_t shift = sizeof(KeyT) == 8 ? 32u : (uint32_t)f.b_d;
    const uint32_t p_depth = depth_only_passes(shift, (uint32_t)f.passes);
    uint32_t count[FE_ITEMS];
    uint32_t n_vis = 0;
#pragma unroll
    for (int k = 0; k < FE_ITEMS; ++k) {
        const uint32_t j = k * FE_THREADS + threadIdx.x;
        const int64_t i = (int64_t)vb * per + j;
        count[k] = 0;
        if (j < per && i < sc.n) {
            uint64_t rect = 0, mask = 0;
            uint32_t klo = 0;
            count[k] = fast_gaussian<DEBUG>(sc, cam, f, ws, dbg, i, rect, klo, mask, opts);
            if (count[k]) {
                s_rect[j] = rect;
                s_qd[j] = klo;
                s_mask[j] = mask;
                ++n_vis;
            }
        }
    }
    uint32_t vis_total;
    const uint32_t total = block_scan_and_chain(count, n_vis, vb, ws, s_incl, s_wtot, s_wvis, &s_base,
                                                &s_base_v, &vis_total);
    const uint64_t base = s_base;
    count_depth_digits(s_h, count, s_qd, s_incl, base, f.capacity, p_depth);
    emit_entries<KeyT>(total, base, s_incl, s_rect, vb * per, f.tiles_x, f.capacity,
                       reinterpret_cast<KeyT*>(ws.keys_a), ws.vals_a,
                       [&](uint32_t tile, uint32_t j) { return ((KeyT)tile << shift) | (KeyT)s_qd[j]; },
                       s_h, p_depth, (uint32_t)f.passes, (opts & OPT_EXACT_TILES) ? s_mask : nullptr);
    __syncthreads();
    prepare_sort<KeyT>(ws, s_h, (uint32_t)f.passes, vb, base, total);
    finish_block(ws, vb, n_blocks, base, s_base_v, total, vis_total, f.capacity);
}

template <bool DEBUG, bool GENERIC, typename KeyT>
static void launch_fe(hipStream_t s, const FastSceneDev& sc, const FrameDev& f, const WsDev& ws,
                      uint32_t fe_blocks, uint32_t fe_per, const DebugDev* dbg, uint32_t opts) {
    hipLaunchKernelGGL((k_frontend_fast<DEBUG, GENERIC, KeyT>), dim3(fe_blocks), dim3(FE_THREADS), 0, s, sc, f,
                       ws, fe_blocks, fe_per, dbg ? *dbg : DebugDev{}, opts);
}

void launch_frontend_fast(hipStream_t s, const FastSceneDev& sc, const FrameDev& f, const WsDev& ws,
                          uint32_t fe_blocks, uint32_t fe_per, const DebugDev* dbg, uint32_t opts) {
    // only these bits change the front end; the others (the exponential, the
    // pixel layout) leave it to the production instance
    opts &= OPT_EXTENT | OPT_KEY32 | OPT_INT8_SH | OPT_FP16_GEOM | OPT_EXACT_TILES;
    const bool key64 = (opts & OPT_KEY32) != 0;
    if (opts == 0) {
        if (dbg) launch_fe<true, false, uint32_t>(s, sc, f, ws, fe_blocks, fe_per, dbg, 0);
        else launch_fe<false, false, uint32_t>(s, sc, f, ws, fe_blocks, fe_per, dbg, 0);
    } else if (key64) {
        if (dbg) launch_fe<true, true, uint64_t>(s, sc, f, ws, fe_blocks, fe_per, dbg, opts);
        else launch_fe<false, true, uint64_t>(s, sc, f, ws, fe_blocks, fe_per, dbg, opts);
    } else {
        if (dbg) launch_fe<true, true, uint32_t>(s, sc, f, ws, fe_blocks, fe_per, dbg, opts);
        else launch_fe<false, true, uint32_t>(s, sc, f, ws, fe_blocks, fe_per, dbg, opts);
    }
}

// Fusion ablated: the fast preprocess alone, one thread per Gaussian, leaving
// counts, rectangles and the low key part for the duplication kernel.
template <bool DEBUG>
__global__ __launch_bounds__(256) void k_preprocess_fast(FastSceneDev sc, FrameDev f, WsDev ws, DebugDev dbg,
                                                         uint32_t opts) {
    const CamDev cam = ws.params->cam;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    uint64_t rect = 0, mask = 0;
    uint32_t klo = 0;
    const uint32_t count = fast_gaussian<DEBUG>(sc, cam, f, ws, dbg, i, rect, klo, mask, opts);
    ws.counts[i] = count;
    if (count) {
        ws.rects[i] = rect;
        ws.depths[i] = __uint_as_float(klo);
        if (ws.masks) ws.masks[i] = mask;
    }
}

void launch_preprocess_fast(hipStream_t s, const FastSceneDev& sc, const FrameDev& f, const WsDev& ws,
                            const DebugDev* dbg, uint32_t opts) {
    const uint32_t blocks = (uint32_t)((sc.n + 255) / 256);
    if (dbg)
        hipLaunchKernelGGL(k_preprocess_fast<true>, dim3(blocks), dim3(256), 0, s, sc, f, ws, *dbg, opts);
    else
        hipLaunchKernelGGL(k_preprocess_fast<false>, dim3(blocks), dim3(256), 0, s, sc, f, ws, DebugDev{}, opts);
}

__global__ void k_widen_keys(const uint32_t* in, uint64_t* out, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

void launch_widen_keys(hipStream_t s, const uint32_t* in, uint64_t* out, uint64_t n) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_widen_keys, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
}

}  // namespace rgs
