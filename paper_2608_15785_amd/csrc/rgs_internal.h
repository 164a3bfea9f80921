// Internal definitions shared by the host library and the HIP kernels.
//
// Everything here is compiled with -ffp-contract=off: the key-defining
// front-end arithmetic below must round exactly like plain IEEE float64
// evaluated left to right, so that tile rectangles, depths and keys are
// reproducible bit for bit by an independent float64 implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rgs.h"

namespace rgs {

constexpr int TILE = RGS_TILE;
constexpr int TILE_PIX = TILE * TILE;
// ln(255) rounded to float64: -ln 255 is the opacity-cull threshold of ln o and
// the skip threshold of the folded exponent (Sec. IV-B, Eq. fast_exp_range).
constexpr double LN255 = 5.541263545158426;
constexpr float LN255F = 5.541263545158426f;
constexpr double DILATION = 0.3;     // low-pass term added to the 2D covariance (3DGS)
constexpr double J_CLAMP = 1.3;      // Jacobian clamp factor on t_x/t_z, t_y/t_z (3DGS)
constexpr float ALPHA_MAX = 0.99f;   // Eq. opacity_clamped
constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float T_MIN = 1e-4f;       // stop blending a pixel below this transmittance

constexpr int FE_THREADS = 1024;     // threads per front-end / duplication block
// Gaussians per thread (block-strided).  Four makes blocks of 4096 Gaussians:
// a 1M scene is 245 blocks, one per CU and all resident at once, and every
// block pays one ticket atomic and one look-back hop of the ordered
// allocation, so fewer, larger blocks are faster (1M at 1080p: 0.059 ms
// against 0.065 ms with two per thread).
constexpr int FE_ITEMS = 4;
constexpr int FE_TILE = FE_THREADS * FE_ITEMS;   // most Gaussians a block takes

// How n Gaussians are split over front-end workgroups.  A scene that fits in
// one round of FE_CU_QUANTUM workgroups (MI355X has 256 CUs; one workgroup
// fills a CU) is spread evenly over up to that many, at least FE_MIN_PER_BLOCK
// Gaussians each: a 1M scene becomes 253 workgroups of 3968 instead of 245 of
// 4096, which left 11 CUs idle.  Larger scenes take FE_TILE per workgroup.
constexpr uint32_t FE_CU_QUANTUM = 256;
constexpr uint32_t FE_MIN_PER_BLOCK = 1024;
inline void fe_block_shape(int64_t n, uint32_t& blocks, uint32_t& per) {
    const uint64_t un = n > 0 ? (uint64_t)n : 1u;
    uint64_t b = (un + FE_TILE - 1) / FE_TILE;
    if (b <= FE_CU_QUANTUM) {
        const uint64_t most = (un + FE_MIN_PER_BLOCK - 1) / FE_MIN_PER_BLOCK;
        b = most < FE_CU_QUANTUM ? most : FE_CU_QUANTUM;
    }
    // a multiple of 64, so that every wave's loads of an attribute plane start
    // on a 256-byte boundary (the planes are padded to 64 Gaussians)
    const uint64_t p = ((un + b - 1) / b + 63) / 64 * 64;
    per = (uint32_t)(p < (uint64_t)FE_TILE ? p : (uint64_t)FE_TILE);
    blocks = (uint32_t)((un + per - 1) / per);
}
constexpr int LB_PER_LANE = 8;       // look-back states each lane polls per round trip
constexpr int SORT_THREADS = 512;    // 8 waves per radix tile
// Keys per thread of a radix tile: 9 for 32-bit keys (4608-key tiles, 48 KB
// of LDS: keys, values, per-wave digit counts) and 11 for 64-bit keys (5632,
// 79 KB), so three or two tiles share a CU.  A pass takes as long as its most
// loaded CU: the 2.2M fast entries of a 1M / 1080p frame make 479 tiles of
// 4608, at most two per CU, where 539 tiles of 4096 left some CUs three (sort
// 0.075 -> 0.072 ms); its 2.87M plain entries make 510 tiles of 5632, one
// round of two per CU, where 702 tiles of 4096 took two rounds (plain sort
// 0.169 -> 0.135 ms).
template <typename KeyT>
struct SortTile {
    static constexpr int ITEMS = sizeof(KeyT) == 4 ? 9 : 11;
    static constexpr int SIZE = SORT_THREADS * ITEMS;
};
inline uint32_t sort_tile_size(uint32_t key_bytes) {
    return key_bytes == 8 ? (uint32_t)SortTile<uint64_t>::SIZE : (uint32_t)SortTile<uint32_t>::SIZE;
}
// Radix tiles per look-back group: the last tile of each group publishes the
// group's digit counts, so a tile reads at most SORT_GROUP - 1 tile states plus
// one state per earlier group.  32 balances the two (1M / 1080p fast sort:
// 0.0729 ms with 16, 0.0712 with 32, 0.0742 with 64, 0.0757 with 8).
constexpr uint32_t SORT_GROUP = 32;
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int MAX_PASSES = 8;
// Copies of the digit histogram that the histogram kernel's blocks spread
// their atomics over (block b adds into copy b % HIST_COPIES): device-scope
// atomics on one address serialise at about 11 ns each.
constexpr int HIST_COPIES = 16;

// Plain-format planes (float32, one per scalar, each n_pad long).
// P_LNO holds ln o rounded to float32 (computed in double on the host); only
// the fast path's FP16-geometry ablation reads it.
enum PlainPlane { P_MX = 0, P_MY, P_MZ, P_SX, P_SY, P_SZ, P_QW, P_QX, P_QY, P_QZ, P_OPA, P_SH0,
                  P_LNO = P_SH0 + 48, P_COUNT };

// Fast-path ablation bits (the path argument's bits 8..14, shifted down).
constexpr uint32_t OPT_FASTEXP = 1u, OPT_DUALPIXEL = 2u, OPT_FUSION = 4u, OPT_EXTENT = 8u, OPT_KEY32 = 16u,
                   OPT_INT8_SH = 32u, OPT_FP16_GEOM = 64u, OPT_EXACT_TILES = 128u, OPT_HW_EXP2 = 256u,
                   OPT_QUAD = 512u;
// Fast-format planes (32-bit words, one per plane, each n_pad long).
//   F_MX..F_MZ   float32 mean
//   F_QWX, F_QYZ FP16 pairs (w, x), (y, z) of the quaternion
//   F_SXY, F_SZL FP16 pairs (sx, sy), (sz, ln o)
//   F_SHQ0..11   four INT8 SH values each; value k = 4*plane + byte, k = coeff*3 + channel
//   F_SHS0..5    FP16 pairs of the 12 SH scales, scale index = degree*3 + channel
enum FastPlane { F_MX = 0, F_MY, F_MZ, F_QWX, F_QYZ, F_SXY, F_SZL, F_SHQ0,
                 F_SHS0 = F_SHQ0 + 12, F_COUNT = F_SHS0 + 6 };

struct CamDev {
    double r[9];
    double t[3];
    double fx, fy, cx, cy;
    double tanx, tany;
    double zn, zf;
    float campos[3];     // camera centre -R^T t, for the SH view direction
    float bg[3];
};

// What changes from one frame to the next at a fixed scene, resolution and
// workspace: the camera and the output image.  The reset kernel copies it into
// the workspace and every later kernel of the frame reads it from there, so a
// captured frame is replayed for another request by changing the reset
// kernel's argument block alone.
struct FrameParams {
    CamDev cam;
    float* out;          // [3][H][W]
    // What the frame was rendered from, for the backward pass's check that the
    // workspace still holds the frame it is asked to differentiate: the
    // scene's tag (new at every upload and every parameter update) and a hash
    // of the camera and the image size.
    uint64_t scene_tag;
    uint64_t cam_hash;
};
static_assert(sizeof(FrameParams) <= 256, "frame parameters fit one 256-byte slot");

struct FrameDev {
    int32_t width, height;
    int32_t tiles_x, tiles_y, n_tiles;
    int32_t b_t, b_d;
    int32_t passes;
    uint32_t capacity;
    uint32_t n_gaussians;
    uint32_t ordered;         // 1: rasterizer workgroup b takes tile ws.order[b], else tile b
};

// Frames whose rasterizers take their tiles longest list first (ws.order):
// every frame of the plain path and its training variant, and fast-path
// frames of at most ORDER_MAX_TILES tiles.  The schedule costs a kernel of
// about 10 us; it pays where the grid's last round of workgroups is a large
// share of the rasterizer's time: at 1M / 1080p (8160 tiles, about three
// rounds of the fast rasterizer's workgroups on 256 CUs) it saved 17 us of
// 123, at 3M / 4K (32400 tiles, about thirteen rounds) 4 us of 279.  The
// plain rasterizers' tiles take several times longer, so a round always
// outweighs the kernel there.
constexpr int32_t ORDER_MAX_TILES = 16384;

// Per visible Gaussian record read by the rasterizer (48 bytes).  The
// projected mean is split into float hi + lo parts so that tile-local
// coordinates keep float64 accuracy at 4K.
struct __align__(16) Record {
    float u_hi, u_lo, v_hi, v_lo;
    float A, B, C, opa;       // conic; opacity (plain) or ln o (fast, and the plain
                              // path's training variant)
    float r, g, b;            // colour
    uint32_t extra;           // plain: float32 depth bits; fast and training variant: FP16
                              // pair (hx, hy) of the alpha-ellipse box half-extents, rounded up
};

__host__ __device__ inline float half_lo(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__host__ __device__ inline float half_hi(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// Device-side header at offset 0 of every workspace.
struct WsHeader {
    uint64_t n_entries;       // entries requested by the front end
    uint32_t n_visible;
    uint32_t overflow;
    uint32_t error;           // bit 0: front-end look-back gave up;
                              // bit 2: a sorted key named a tile outside the grid;
                              // bit 3: a backward pass found another frame than its caller's
    uint32_t capacity;
    uint32_t path;
    uint32_t passes;
    uint32_t fe_ticket;
    uint64_t list_steps;      // counting renders of the fast path: list entries the waves evaluated
    uint32_t pad[52];
};
static_assert(sizeof(WsHeader) == 256, "header is one 256-byte slot");

// Byte offsets of a frame's workspace regions (all 256-byte aligned).
struct WsLayout {
    uint64_t params;
    uint64_t header, ranges, fe_state, zero_end;
    uint64_t order;
    uint64_t records, counts, rects, depths, offsets, masks;
    uint64_t keys_a, keys_b, vals_a, vals_b;
    uint64_t hist, sort_state;
    uint64_t t_final, n_proc, n_blend;
    uint64_t total;
    uint64_t capacity;
    uint32_t key_bytes, passes, fe_blocks, sort_blocks_max;   // sort_blocks_max: radix tiles at capacity
    uint32_t fe_per;          // Gaussians per front-end / duplication workgroup (<= FE_TILE)
};

// Pointers a kernel needs into the workspace.
struct WsDev {
    const FrameParams* params;
    WsHeader* header;
    uint32_t* ranges;         // [n_tiles][2]
    uint32_t* order;          // [n_tiles] tile of each rasterizer workgroup: longest lists first
    uint64_t* fe_state;       // chained-scan state per front-end block
    Record* records;          // [n]
    uint32_t* counts;         // plain: tiles touched per Gaussian
    uint64_t* rects;          // plain: packed x0 | x1 << 16 | y0 << 32 | y1 << 48
    float* depths;            // plain: float32 depth per Gaussian
    uint32_t* offsets;        // plain: position of the Gaussian's first entry in emission order
    uint64_t* masks;          // fast path, fusion ablated, exact tiles: kept tiles of the rectangle
                              // (row-major bits)
    void* keys_a;
    void* keys_b;
    uint32_t* vals_a;
    uint32_t* vals_b;
    uint32_t* hist;           // [HIST_COPIES][MAX_PASSES][RADIX] digit counts of every radix pass
    uint32_t* sort_state;     // 2 x [sort_rows + sort_groups][RADIX] look-back words, one set per
                              // pass parity: ready flag (bit 31) | digit count
    uint32_t sort_rows;       // radix tiles at capacity
    uint32_t sort_groups;     // ceil(sort_rows / SORT_GROUP)
    float* t_final;           // [H][W]
    uint32_t* n_proc;         // [H][W] list entries visited per pixel
    uint32_t* n_blend;        // [H][W] pairs blended per pixel (written by counting renders)
};

struct DebugDev {
    double* depth;
    double* u;
    double* v;
    double* cov2d;
    int32_t* rect;
    uint8_t* visible;
    float* color;
};

// ---------------------------------------------------------------------------
// Front-end arithmetic (float64, evaluated exactly as written, no contraction).

struct Projected {
    double d, u, v, c00, c01, c11, det;
    double ax, ay;            // fast path: half-extents of the ellipse where P >= -ln 255
    double x0, x1, y0, y1;    // inclusive tile bounds (integer valued)
};

// EWA projection, culling and tile extent of one Gaussian.  Returns false when
// it is culled: depth outside (zn, zf], det(Sigma') <= 0, ln o < -ln 255 (fast
// path), or an empty tile rectangle.  The evaluation order of every
// expression is part of the definition (see the header comment).
__host__ __device__ inline bool project_gaussian(const CamDev& c, double mx, double my, double mz,
                                                 double qw, double qx, double qy, double qz,
                                                 double sx, double sy, double sz, bool fast,
                                                 double lno, double tiles_x, double tiles_y,
                                                 Projected& o, bool alpha_extent = true) {
    const double* r = c.r;
    double tx = r[0] * mx + r[1] * my + r[2] * mz + c.t[0];
    double ty = r[3] * mx + r[4] * my + r[5] * mz + c.t[1];
    double d = r[6] * mx + r[7] * my + r[8] * mz + c.t[2];
    o.d = d;
    if (!(d > c.zn && d <= c.zf)) return false;
    if (fast && alpha_extent && !(lno >= -LN255)) return false;

    double inn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    double w = qw * inn, x = qx * inn, y = qy * inn, z = qz * inn;
    double R00 = 1.0 - 2.0 * (y * y + z * z);
    double R01 = 2.0 * (x * y - w * z);
    double R02 = 2.0 * (x * z + w * y);
    double R10 = 2.0 * (x * y + w * z);
    double R11 = 1.0 - 2.0 * (x * x + z * z);
    double R12 = 2.0 * (y * z - w * x);
    double R20 = 2.0 * (x * z - w * y);
    double R21 = 2.0 * (y * z + w * x);
    double R22 = 1.0 - 2.0 * (x * x + y * y);
    // M = R diag(s), Sigma = M M^T
    double M00 = R00 * sx, M01 = R01 * sy, M02 = R02 * sz;
    double M10 = R10 * sx, M11 = R11 * sy, M12 = R12 * sz;
    double M20 = R20 * sx, M21 = R21 * sy, M22 = R22 * sz;
    double S00 = M00 * M00 + M01 * M01 + M02 * M02;
    double S01 = M00 * M10 + M01 * M11 + M02 * M12;
    double S02 = M00 * M20 + M01 * M21 + M02 * M22;
    double S11 = M10 * M10 + M11 * M11 + M12 * M12;
    double S12 = M10 * M20 + M11 * M21 + M12 * M22;
    double S22 = M20 * M20 + M21 * M21 + M22 * M22;

    double limx = J_CLAMP * c.tanx;
    double limy = J_CLAMP * c.tany;
    double rd = 1.0 / d;
    double rd2 = rd * rd;
    double xc = fmin(limx, fmax(-limx, tx * rd)) * d;
    double yc = fmin(limy, fmax(-limy, ty * rd)) * d;
    double j00 = c.fx * rd;
    double j02 = -(c.fx * xc) * rd2;
    double j11 = c.fy * rd;
    double j12 = -(c.fy * yc) * rd2;
    // T = J R_w
    double T00 = j00 * r[0] + j02 * r[6];
    double T01 = j00 * r[1] + j02 * r[7];
    double T02 = j00 * r[2] + j02 * r[8];
    double T10 = j11 * r[3] + j12 * r[6];
    double T11 = j11 * r[4] + j12 * r[7];
    double T12 = j11 * r[5] + j12 * r[8];
    // U = T Sigma, Sigma' = U T^T + 0.3 I
    double U00 = T00 * S00 + T01 * S01 + T02 * S02;
    double U01 = T00 * S01 + T01 * S11 + T02 * S12;
    double U02 = T00 * S02 + T01 * S12 + T02 * S22;
    double U10 = T10 * S00 + T11 * S01 + T12 * S02;
    double U11 = T10 * S01 + T11 * S11 + T12 * S12;
    double U12 = T10 * S02 + T11 * S12 + T12 * S22;
    double c00 = U00 * T00 + U01 * T01 + U02 * T02 + DILATION;
    double c01 = U00 * T10 + U01 * T11 + U02 * T12;
    double c11 = U10 * T10 + U11 * T11 + U12 * T12 + DILATION;
    o.c00 = c00;
    o.c01 = c01;
    o.c11 = c11;
    double det = c00 * c11 - c01 * c01;
    o.det = det;
    double u = c.fx * tx * rd + c.cx;
    double v = c.fy * ty * rd + c.cy;
    o.u = u;
    o.v = v;
    if (!(det > 0.0)) return false;

    double mid = 0.5 * (c00 + c11);
    double lam = mid + sqrt(fmax(0.0, mid * mid - det));
    double rad = ceil(3.0 * sqrt(lam));
    double hx = rad, hy = rad;
    if (fast) {
        double tau = 2.0 * (LN255 + lno);
        o.ax = sqrt(tau * c00);
        o.ay = sqrt(tau * c11);
        if (alpha_extent) {
            hx = fmin(rad, o.ax);
            hy = fmin(rad, o.ay);
        }
    }
    o.x0 = fmax(0.0, floor((u - hx) / 16.0));
    o.x1 = fmin(tiles_x - 1.0, floor((u + hx) / 16.0));
    o.y0 = fmax(0.0, floor((v - hy) / 16.0));
    o.y1 = fmin(tiles_y - 1.0, floor((v + hy) / 16.0));
    return o.x0 <= o.x1 && o.y0 <= o.y1;
}

// Exact ellipse-tile test, the tile-precise half of the Speedy-Splat culling
// that the fast path adopts (Sec. IV-A): does the ellipse q(p) <= tau of a
// projected Gaussian, q(p) = (c11 dx^2 - 2 c01 dx dy + c00 dy^2) / det with
// (dx, dy) = p - (u, v) and tau = 2 (ln 255 + ln o), meet the box of a tile's
// pixel centres [X0, X0 + 15] x [Y0, Y0 + 15]?  q is convex, so the box holds
// a point of the ellipse iff it holds the mean or the least q on one of its
// edges is <= tau.  On the line x = X the least q is dx^2 / c00, at
// dy = c01 dx / c00; when that dy is off the edge, the least q on the edge is
// at the nearer corner.  Multiplying through by c00, c11 or det (all > 0)
// leaves no division or square root.  Applied to rectangles of at most
// EXACT_TILE_MAX_AREA tiles (their kept tiles fit a 64-bit mask); larger
// rectangles keep every tile.  Evaluation order as written, as everywhere in
// the key-defining arithmetic.
constexpr uint32_t EXACT_TILE_MAX_AREA = 64;
__host__ __device__ inline bool ellipse_meets_tile(double u, double v, double c00, double c01, double c11,
                                                   double det, double tau, double X0, double Y0) {
    const double X1 = X0 + 15.0, Y1 = Y0 + 15.0;
    if (u >= X0 && u <= X1 && v >= Y0 && v <= Y1) return true;
    const double rhs = tau * det;
    for (int e = 0; e < 2; ++e) {           // vertical edges x = X0, X1
        const double dx = (e ? X1 : X0) - u;
        const double t = c01 * dx;
        const double lo = (Y0 - v) * c00;
        const double hi = (Y1 - v) * c00;
        if (t >= lo && t <= hi) {
            if (dx * dx <= tau * c00) return true;
        } else {
            const double dy = t < lo ? Y0 - v : Y1 - v;
            if (c11 * dx * dx - 2.0 * c01 * dx * dy + c00 * dy * dy <= rhs) return true;
        }
    }
    for (int e = 0; e < 2; ++e) {           // horizontal edges y = Y0, Y1
        const double dy = (e ? Y1 : Y0) - v;
        const double t = c01 * dy;
        const double lo = (X0 - u) * c11;
        const double hi = (X1 - u) * c11;
        if (t >= lo && t <= hi) {
            if (dy * dy <= tau * c11) return true;
        } else {
            const double dx = t < lo ? X0 - u : X1 - u;
            if (c11 * dx * dx - 2.0 * c01 * dx * dy + c00 * dy * dy <= rhs) return true;
        }
    }
    return false;
}

// Eq. depth_quant: q = clamp(floor((d - zn) / (zf - zn) * (2^b_d - 1)), 0, 2^b_d - 1).
__host__ __device__ inline uint32_t quantize_depth(double d, double zn, double zf, int b_d) {
    double levels = (double)((1u << b_d) - 1u);
    double q = floor((d - zn) / (zf - zn) * levels);
    q = fmin(levels, fmax(0.0, q));
    return (uint32_t)q;
}

// ---------------------------------------------------------------------------
// Wave64 helpers.

__device__ inline uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ inline uint64_t lanemask_lt() {
    uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ inline T wave_inclusive_scan(T x) {
    uint32_t l = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off, 64);
        if (l >= (uint32_t)off) x += y;
    }
    return x;
}

template <typename T>
__device__ inline T wave_sum(T x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Relaxed device-scope atomics on look-back state: the value travels in the
// same word as its flag, so no ordering with other memory is needed.
__device__ inline uint64_t ld_state(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_state(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t ld_state(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_state(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back word sets of the sort: set 0 serves even passes, set 1 odd passes.
// Each set holds sort_rows tile rows, then sort_groups group rows, of RADIX
// words.
__device__ inline uint32_t* sort_state_tiles(const WsDev& ws, uint32_t set) {
    return ws.sort_state + (uint64_t)set * ((uint64_t)ws.sort_rows + ws.sort_groups) * RADIX;
}
__device__ inline uint32_t* sort_state_groups(const WsDev& ws, uint32_t set) {
    return sort_state_tiles(ws, set) + (uint64_t)ws.sort_rows * RADIX;
}

// Bounded waits: a look-back that polls this often without progress gives up,
// flags the header and lets the kernel finish.
constexpr uint32_t SPIN_LIMIT = 1u << 22;

// 64-bit chained-scan state: flag in bits 63..62 (1 aggregate, 2 inclusive
// prefix), entry count in bits 31..0 (saturating), visible count in 61..32.
constexpr uint64_t ST_AGG = 1ull << 62;
constexpr uint64_t ST_PRE = 2ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;
__host__ __device__ inline uint64_t st_pack(uint64_t entries, uint64_t visible) {
    return (entries > 0xffffffffull ? 0xffffffffull : entries) | (visible << 32);
}
__host__ __device__ inline uint64_t st_entries(uint64_t s) { return s & 0xffffffffull; }
__host__ __device__ inline uint64_t st_visible(uint64_t s) { return (s >> 32) & ((1ull << 30) - 1); }

// ---------------------------------------------------------------------------
// Host-side launch wrappers (defined in the .hip files).

struct PlainSceneDev { const float* base; uint64_t n_pad; int64_t n; };
struct FastSceneDev { const uint32_t* base; uint64_t n_pad; int64_t n; const float* plain; };

// Arguments of the reset kernel: the span it zeroes (header, tile ranges,
// scan state, digit buckets), the header fields it sets, and the frame's
// parameters with their place in the workspace.
struct ResetArgs {
    uint32_t* base;
    uint64_t n_words;
    uint32_t capacity, path, passes, pad;
    FrameParams* dst;
    FrameParams prm;
};

// A frame's outcome as the host sees it after the frame: written by the last
// kernel of a frame into host-visible memory when the caller asks for it.
struct FrameStatus {
    uint64_t n_entries;
    uint32_t n_visible, overflow, error, done;
    uint64_t out;        // output address the frame used (checks replayed parameters)
};

// A plain render's outcome and stamp, copied by the frame's last kernel into
// host-visible memory of the rendering context: the backward pass learns
// whether its frame overflowed, and that the frame is the one it expects,
// without reading the device.  seq is written last, after a system fence.
struct FrameStamp {
    uint64_t n_entries;
    uint32_t overflow, error;
    uint64_t scene_tag, cam_hash;
    uint64_t seq;
};

ResetArgs reset_args(const WsDev& ws, uint64_t zero_bytes, const FrameDev& f, uint32_t path,
                     const FrameParams& prm);
void launch_reset(hipStream_t s, const ResetArgs& a);
const void* reset_kernel();          // host handle of the reset kernel (graph node lookup)
void launch_export_status(hipStream_t s, const WsDev& ws, FrameStatus* dst);
void launch_export_stamp(hipStream_t s, const WsDev& ws, FrameStamp* dst, uint64_t seq);
void launch_preprocess_plain(hipStream_t s, const PlainSceneDev& sc, const FrameDev& f,
                             const WsDev& ws, const DebugDev* dbg, bool train);
void launch_duplicate(hipStream_t s, int64_t n, const FrameDev& f, const WsDev& ws, uint32_t fe_blocks, uint32_t fe_per,
                      uint32_t key_bytes);
void launch_frontend_fast(hipStream_t s, const FastSceneDev& sc, const FrameDev& f, const WsDev& ws,
                          uint32_t fe_blocks, uint32_t fe_per, const DebugDev* dbg, uint32_t opts);
void launch_preprocess_fast(hipStream_t s, const FastSceneDev& sc, const FrameDev& f, const WsDev& ws,
                            const DebugDev* dbg, uint32_t opts);
void launch_sort(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes, uint32_t passes,
                 bool force_fallback, bool* result_in_b);
void launch_ranges(hipStream_t s, const FrameDev& f, const WsDev& ws, uint32_t key_bytes,
                   bool result_in_b);
// The rasterizers' schedule: ws.order from the tile ranges.
void launch_tile_order(hipStream_t s, const FrameDev& f, const WsDev& ws);
// The fast path's bucket sort (frames of 8 .. BUCKET_MAX_BT tile bits, 32-bit
// keys): sorted keys and values end in keys_a / vals_a, and the tile ranges
// are written too (no launch_ranges).
constexpr int32_t BUCKET_MAX_BT = 14;
bool bucket_sort_applies(const FrameDev& f, uint32_t key_bytes);
void launch_sort_bucket(hipStream_t s, const FrameDev& f, const WsDev& ws, bool force, bool* result_in_b);
void launch_raster_plain(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count);
void launch_raster_train(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count);
void launch_raster_fast(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count,
                        uint32_t opts);
void launch_widen_keys(hipStream_t s, const uint32_t* in, uint64_t* out, uint64_t n);
void launch_probe_valu(hipStream_t s, float* out, uint32_t blocks, uint32_t iters);

// The n_proc word of a pixel: pairs visited, with this bit set when blending
// stopped at the last of them (that pair was not blended).
constexpr uint32_t N_PROC_STOPPED = 0x80000000u;

// Gradient outputs of the backward pass, [n][...] rows; screen may be NULL.
struct GradOut {
    float* means;
    float* scales;
    float* quats;
    float* opacity;
    float* sh;
    float* screen;
};

void launch_update_plain(hipStream_t s, float* planes, uint64_t n_pad, int64_t n, const float* means,
                         const float* scales, const float* quats, const float* opacity, const float* sh);
// The frame a backward pass is asked to differentiate: its scene tag and camera
// hash.  The backward kernels compare them with the workspace's frame
// parameters; on a mismatch they set header bit 3, write no partials, and the
// per-Gaussian pass writes zero gradients.
struct FrameKey {
    uint64_t scene_tag, cam_hash;
};
void launch_raster_backward(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b,
                            const float* dimg, float4* partial, FrameKey key);
void launch_raster_backward_train(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b,
                                  const float* dimg, float4* partial, FrameKey key);
// lno_opacity: the partials' opacity slot holds dL/d(ln o) (the training
// variant's), converted to dL/do here.
void launch_grad_gaussian(hipStream_t s, const PlainSceneDev& sc, const CamDev& cam, const WsDev& ws,
                          const float4* partial, const GradOut& go, bool lno_opacity, FrameKey key);

}  // namespace rgs
