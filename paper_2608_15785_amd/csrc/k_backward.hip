// Reverse mode of the plain render (differentiation of Sec. II-A / III-D's
// image definition with its discrete decisions held fixed), and the device
// update of plain attributes that a training step needs.
//
// raster_backward: one wave per 16x16 tile, four pixels per lane, the tile's
// sorted list walked back to front in batches staged in LDS.  A pixel
// starts after its last blended pair (the forward pass left its final T, the
// number of pairs it visited and whether it stopped); T before each blended
// pair is recovered as T_after / (1 - alpha), and the colour accumulated behind
// the pair plus the background's share, S' = S + T_final bg, is carried along
// (it starts at T_final bg), so that
//   dC/dc_j = alpha_j T_j,   dC/dalpha_j = c_j T_j - S'_j / (1 - alpha_j).
// The nine image-space derivatives of a pair (u, v, A, B, C, o, r, g, b) are
// summed over a lane's four pixels, then over the wave with DPP adds, and each
// entry receives one 48-byte partial at its position in emission order: no
// atomics.  Ordered allocation emitted a Gaussian's entries contiguously,
// one per tile of its rectangle in row-major order, from the offset the
// duplication kernel recorded, so that position is known from the tile.
//
// grad_gaussian: one thread per Gaussian sums its contiguous partials and
// applies the chain rule through the EWA projection and the SH colour in
// double precision; the SH gradients leave through LDS in coalesced rows.
#include "rgs_fold.h"

namespace rgs {


// ---------------------------------------------------------------------------
// Plain attributes from [n][...] rows.  A block takes 256 Gaussians.  Their
// SH rows (48 floats each, 48 KB together) are read as one contiguous span of
// 16-byte loads into LDS, each row padded to 49 floats so that the plane-wise
// reads below hit distinct banks; each thread then writes its Gaussian's 48
// coefficients into the 48 SH planes, consecutive threads at consecutive
// addresses.  Reading the rows directly, each load instruction of a wave would
// touch 64 rows 192 bytes apart.

constexpr int UPD_THREADS = 256;
constexpr int UPD_SH = 48;
constexpr int UPD_ROW = UPD_SH + 1;

__global__ __launch_bounds__(UPD_THREADS) void k_update_plain(float* __restrict__ planes, uint64_t n_pad, int64_t n,
                                                              const float* __restrict__ means,
                                                              const float* __restrict__ scales,
                                                              const float* __restrict__ quats,
                                                              const float* __restrict__ opacity,
                                                              const float* __restrict__ sh) {
    __shared__ float s_sh[UPD_THREADS * UPD_ROW];
    const int64_t first = (int64_t)blockIdx.x * UPD_THREADS;
    const int64_t rows = n - first < UPD_THREADS ? n - first : UPD_THREADS;
    const int64_t words = rows * UPD_SH;
    const float* src = sh + first * UPD_SH;
    if (rows == UPD_THREADS && (reinterpret_cast<uintptr_t>(src) % 16) == 0) {
        const float4* src4 = reinterpret_cast<const float4*>(src);
        for (int q = threadIdx.x; q < UPD_THREADS * UPD_SH / 4; q += UPD_THREADS) {
            const float4 v = src4[q];
            const float vals[4] = {v.x, v.y, v.z, v.w};
            const int w = 4 * q;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int we = w + e;
                s_sh[(we / UPD_SH) * UPD_ROW + we % UPD_SH] = vals[e];
            }
        }
    } else {
        for (int64_t w = threadIdx.x; w < words; w += UPD_THREADS)
            s_sh[(w / UPD_SH) * UPD_ROW + w % UPD_SH] = src[w];
    }
    __syncthreads();
    const int64_t i = first + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) planes[(P_MX + k) * n_pad + i] = means[3 * i + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) planes[(P_SX + k) * n_pad + i] = scales[3 * i + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) planes[(P_QW + k) * n_pad + i] = quats[4 * i + k];
    planes[P_OPA * n_pad + i] = opacity[i];
    planes[P_LNO * n_pad + i] = (float)log((double)opacity[i]);
    const float* row = s_sh + threadIdx.x * UPD_ROW;
#pragma unroll 8
    for (int k = 0; k < UPD_SH; ++k) planes[(P_SH0 + k) * n_pad + i] = row[k];
}

void launch_update_plain(hipStream_t s, float* planes, uint64_t n_pad, int64_t n, const float* means,
                         const float* scales, const float* quats, const float* opacity, const float* sh) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update_plain, dim3((uint32_t)((n + UPD_THREADS - 1) / UPD_THREADS)), dim3(UPD_THREADS), 0,
                       s, planes, n_pad, n, means, scales, quats, opacity, sh);
}

// ---------------------------------------------------------------------------
// Row sums of N values at once: after two quad permutations and two row
// shifts (each a DPP-modified add) lane 16 r + 15 holds the sum over row r of
// the wave.  The N chains are independent, so the DPP instructions of one
// value are spaced by those of the others and need no wait states.

template <int CTRL>
__device__ inline float dpp_moved(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int N>
__device__ inline void row_sums(float (&g)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) g[c] += dpp_moved<0xb1>(g[c]);     // quad_perm [1,0,3,2]
#pragma unroll
    for (int c = 0; c < N; ++c) g[c] += dpp_moved<0x4e>(g[c]);     // quad_perm [2,3,0,1]
#pragma unroll
    for (int c = 0; c < N; ++c) g[c] += dpp_moved<0x114>(g[c]);    // row_shr:4
#pragma unroll
    for (int c = 0; c < N; ++c) g[c] += dpp_moved<0x118>(g[c]);    // row_shr:8
}

// Position, in emission order, of Gaussian g's entry for tile (tx, ty).
__device__ inline uint64_t emission_pos(const WsDev& ws, uint32_t g, uint32_t tx, uint32_t ty) {
    const uint64_t rc = ws.rects[g];
    const uint32_t x0 = rc & 0xffff, x1 = (rc >> 16) & 0xffff, y0 = (rc >> 32) & 0xffff;
    return (uint64_t)ws.offsets[g] + (uint64_t)(ty - y0) * (x1 - x0 + 1) + (tx - x0);
}

// One wave per tile; lane l owns the pixels (l % 16, l / 16 + 4 k), k = 0..3,
// and adds its four pixels' terms before the wave reduction of an entry.
constexpr int BWD_LANES = 64;
constexpr int BWD_PIX = 4;
constexpr int BWD_BATCH = 32;
constexpr int BWD_ROWS = BWD_LANES / 16;     // DPP rows of the wave

// Row bands k (tile rows 4k .. 4k+3) that can hold a pixel with alpha >= 1/255
// for a Gaussian at tile-local (u, v) with conic (A, B, C) and opacity o: the
// ellipse A dx^2 + 2 B dx dy + C dy^2 <= 2 ln(255 o) spans |dy| <= sqrt(tau A / det).
// The half-height is widened by 1e-3 of itself plus 0.05 pixel, far beyond the
// float32 rounding of the exponent, so no blended pair falls outside.
__device__ inline uint32_t band_mask(float v, float A, float B, float C, float o) {
    const float tau = 2.0f * logf(255.0f * o);
    if (!(tau > 0.0f)) return 0u;                      // alpha < 1/255 everywhere
    const float det = A * C - B * B;
    if (!(det > 0.0f)) return 0xfu;
    const float hy = sqrtf(tau * A / det) * 1.001f + 0.05f;
    if (!(hy < 1e30f)) return 0xfu;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < BWD_PIX; ++k)
        if (v - hy <= (float)(4 * k + 3) && v + hy >= (float)(4 * k)) m |= 1u << k;
    return m;
}

// Whether the workspace still holds the frame the caller asked for; if not,
// the first workgroup flags it in the header and every workgroup leaves.
__device__ inline bool frame_matches(const WsDev& ws, FrameKey key) {
    const FrameParams* prm = ws.params;
    if (prm->scene_tag == key.scene_tag && prm->cam_hash == key.cam_hash) return true;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ws.header->error, 8u);
    return false;
}

__global__ __launch_bounds__(BWD_LANES) void k_raster_backward(FrameDev f, WsDev ws,
                                                               const uint32_t* __restrict__ vals,
                                                               const float* __restrict__ dimg,
                                                               float4* __restrict__ partial, FrameKey key) {
    if (!frame_matches(ws, key)) return;
    __shared__ float4 s_a[BWD_BATCH];          // u, v (tile-local), A, B
    __shared__ float4 s_b[BWD_BATCH];          // C, o, r, g
    __shared__ float s_c[BWD_BATCH];           // b
    __shared__ uint32_t s_band[BWD_BATCH];     // row bands the entry can reach
    __shared__ float4 s_acc4[9 * BWD_ROWS * BWD_BATCH / 4];   // per-row entry sums of the batch
    float* s_acc = reinterpret_cast<float*>(s_acc4);              // [9][BWD_ROWS][BWD_BATCH]
    if (blockIdx.x >= (uint32_t)f.n_tiles) return;
    const uint32_t tile = f.ordered ? ws.order[blockIdx.x] : blockIdx.x;   // the rasterizers' schedule
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t lane = threadIdx.x;
    const uint32_t lx = lane % TILE, ly0 = lane / TILE;
    const uint32_t px = tx * TILE + lx;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    const float ox = (float)(tx * TILE), oy = (float)(ty * TILE);
    const float x = (float)lx;
    const uint64_t plane = (uint64_t)f.width * f.height;
    const float bg0 = ws.params->cam.bg[0], bg1 = ws.params->cam.bg[1], bg2 = ws.params->cam.bg[2];

    float T[BWD_PIX], d[BWD_PIX][3], S[BWD_PIX][3];   // S: colour behind the pair + T_final bg
    uint32_t last[BWD_PIX];                    // pairs [start, last) may have been blended
    uint32_t lane_last = start;
#pragma unroll
    for (int k = 0; k < BWD_PIX; ++k) {
        const uint32_t py = ty * TILE + ly0 + 4 * k;
        T[k] = 1.0f;
        last[k] = start;
#pragma unroll
        for (int c = 0; c < 3; ++c) d[k][c] = 0.0f;
        if (px < (uint32_t)f.width && py < (uint32_t)f.height) {
            const uint64_t o = (uint64_t)py * f.width + px;
            T[k] = ws.t_final[o];
            const uint32_t word = ws.n_proc[o];
            last[k] = start + (word & ~N_PROC_STOPPED) - ((word & N_PROC_STOPPED) ? 1u : 0u);
            d[k][0] = dimg[o];
            d[k][1] = dimg[plane + o];
            d[k][2] = dimg[2 * plane + o];
        }
        S[k][0] = T[k] * bg0;
        S[k][1] = T[k] * bg1;
        S[k][2] = T[k] * bg2;
        lane_last = max(lane_last, last[k]);
    }
    uint32_t wave_last = lane_last;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, off));

    for (uint32_t b_end = wave_last; b_end > start;) {
        const uint32_t b0 = b_end - start > (uint32_t)BWD_BATCH ? b_end - BWD_BATCH : start;
        const uint32_t cnt = b_end - b0;
        __syncthreads();                         // the previous batch is fully read
        uint64_t my_pos = 0;
        if (lane < cnt) {
            const uint32_t g0 = vals[b0 + lane];
            const uint32_t g = g0 < f.n_gaussians ? g0 : 0u;
            const Record rec = ws.records[g];
            s_a[lane] = make_float4((rec.u_hi - ox) + rec.u_lo, (rec.v_hi - oy) + rec.v_lo, rec.A, rec.B);
            s_b[lane] = make_float4(rec.C, rec.opa, rec.r, rec.g);
            s_c[lane] = rec.b;
            s_band[lane] = band_mask((rec.v_hi - oy) + rec.v_lo, rec.A, rec.B, rec.C, rec.opa);
            my_pos = emission_pos(ws, g, tx, ty);
        }
        for (uint32_t q = lane; q < 9 * BWD_ROWS * BWD_BATCH / 4; q += BWD_LANES)
            s_acc4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        for (int j = (int)cnt - 1; j >= 0; --j) {
            const uint32_t idx = b0 + (uint32_t)j;
            if (__ballot(idx < lane_last) == 0) continue;
            const float4 a = s_a[j];
            const float4 m = s_b[j];
            const float cb = s_c[j];
            const uint32_t band = s_band[j];
            float g[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) g[c] = 0.0f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < BWD_PIX; ++k) {
                if (((band >> k) & 1u) && idx < last[k]) {
                    const float dx = x - a.x, dy = (float)(ly0 + 4 * k) - a.y;
                    const float p = fmaf(-0.5f, fmaf(a.z * dx, dx, m.x * dy * dy), -a.w * dx * dy);
                    const float e = expf(p);
                    const float raw = m.y * e;
                    const float alpha = fminf(ALPHA_MAX, raw);
                    if (alpha >= ALPHA_MIN) {
                        any = true;
                        const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
                        const float Tb = T[k] * inv;
                        const float w = alpha * Tb;
                        g[6] = fmaf(w, d[k][0], g[6]);
                        g[7] = fmaf(w, d[k][1], g[7]);
                        g[8] = fmaf(w, d[k][2], g[8]);
                        const float dA = d[k][0] * (m.z * Tb - S[k][0] * inv) +
                                         d[k][1] * (m.w * Tb - S[k][1] * inv) +
                                         d[k][2] * (cb * Tb - S[k][2] * inv);
                        S[k][0] = fmaf(m.z, w, S[k][0]);
                        S[k][1] = fmaf(m.w, w, S[k][1]);
                        S[k][2] = fmaf(cb, w, S[k][2]);
                        T[k] = Tb;
                        const float dRaw = raw <= ALPHA_MAX ? dA : 0.0f;   // a clamped alpha is constant
                        g[5] = fmaf(dRaw, e, g[5]);
                        const float dP = dRaw * raw;
                        g[0] = fmaf(dP, fmaf(a.z, dx, a.w * dy), g[0]);    // dp/du = A dx + B dy
                        g[1] = fmaf(dP, fmaf(m.x, dy, a.w * dx), g[1]);    // dp/dv = C dy + B dx
                        g[2] = fmaf(-0.5f * dP, dx * dx, g[2]);
                        g[3] = fmaf(-dP, dx * dy, g[3]);
                        g[4] = fmaf(-0.5f * dP, dy * dy, g[4]);
                    }
                }
            }
            if (__ballot(any) != 0) {
                row_sums(g);
                if ((lane & 15) == 15) {
                    const uint32_t r = lane >> 4;
#pragma unroll
                    for (int c = 0; c < 9; ++c) s_acc[(c * BWD_ROWS + r) * BWD_BATCH + j] = g[c];
                }
            }
        }
        __syncthreads();
        if (lane < cnt) {
            float4* dst = partial + 3ull * my_pos;
            float sum[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const float* row = s_acc + c * BWD_ROWS * BWD_BATCH + lane;
                sum[c] = (row[0] + row[BWD_BATCH]) + (row[2 * BWD_BATCH] + row[3 * BWD_BATCH]);
            }
            dst[0] = make_float4(sum[0], sum[1], sum[2], sum[3]);
            dst[1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
            dst[2] = make_float4(sum[8], 0.0f, 0.0f, 0.0f);
        }
        b_end = b0;
    }
    // entries no pixel of the tile reached
    for (uint32_t idx = wave_last + lane; idx < end; idx += BWD_LANES) {
        const uint32_t g = vals[idx];
        float4* dst = partial + 3ull * emission_pos(ws, g < f.n_gaussians ? g : 0u, tx, ty);
        dst[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        dst[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        dst[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

void launch_raster_backward(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b,
                            const float* dimg, float4* partial, FrameKey key) {
    const uint32_t* vals = result_in_b ? ws.vals_b : ws.vals_a;
    hipLaunchKernelGGL(k_raster_backward, dim3((uint32_t)f.n_tiles), dim3(BWD_LANES), 0, s, f, ws, vals, dimg,
                       partial, key);
}

// ---------------------------------------------------------------------------
// The training variant's backward pass.  Its forward pass is the dual-pixel
// rasterizer with culled lists over the plain records (k_raster_fast with
// EXP_HW2 and TRAIN).  Here the tile's list is replayed back to front in the
// forward's layout: two waves, wave w owning rows 8w .. 8w+7, each lane the
// dual pixel (x, y), (x, y+1).  Each batch is staged, folded and culled per
// wave by the forward's own functions (rgs_fold.h), so every exponent, alpha
// and skip decision is the forward's, bit for bit, and T before a pair is
// recovered from the forward's final T as in the plain backward.  A pair's
// exponent P = ln o + p in natural units gives dalpha/dP = alpha, and
// dP/d(ln o) = 1: the opacity slot of the partials carries dL/d(ln o), which
// the per-Gaussian pass divides by o.  Per entry, each lane's nine terms (its
// two pixels added) are summed over each half-wave with DPP row operations and
// the two half-wave sums kept in LDS; at the end of a batch each entry adds its
// four half-wave sums and writes them to its emission position.  Measured at
// 1M / 1080p (the training step's backward call): 1.02 ms with a full-wave DPP
// reduction per entry and per-channel colour sums, 0.88 ms with the sums below;
// four row sums kept instead of two, or batches of 32, made no difference;
// reading the next entry's coefficients one step ahead and keeping the
// half-wave broadcast out of the store's lane mask took it to 0.77 ms.

constexpr int TB_THREADS = 128;
constexpr int TB_BATCH = 64;

// Adds one blended pair's terms at one pixel to g[9] and steps the pixel's
// state back over the pair.  dx, dy: pixel minus mean; col: the pair's colour;
// d: dL/dC at the pixel; DS = d . S, S the colour behind the pair plus the
// background's share, so that dL/dalpha = Tb (d . col) - DS / (1 - alpha).
// The conic terms are left as moments of dL/dP: g[0] += dP dx, g[1] += dP dy,
// g[2] += dP dx^2, g[3] += dP dx dy, g[4] += dP dy^2; the wave's sums of them
// are turned into dL/d(u, v, A, B, C) once per entry (the conic is constant
// over the entry's pixels).
__device__ inline void pair_adjoint(float P, float dx, float dy, const float4& col, const float (&d)[3], float& T,
                                    float& DS, float (&g)[9]) {
    const float raw = __builtin_amdgcn_exp2f(P);
    const float alpha = fminf(ALPHA_MAX, raw);
    const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
    const float Tb = T * inv;
    const float w = alpha * Tb;
    g[6] = fmaf(w, d[0], g[6]);
    g[7] = fmaf(w, d[1], g[7]);
    g[8] = fmaf(w, d[2], g[8]);
    const float dcol = fmaf(d[0], col.x, fmaf(d[1], col.y, d[2] * col.z));
    const float dA = fmaf(Tb, dcol, -(DS * inv));
    DS = fmaf(w, dcol, DS);
    T = Tb;
    const float dP = raw <= ALPHA_MAX ? dA * raw : 0.0f;     // a clamped alpha is constant
    g[5] += dP;                                               // dL/d(ln o)
    const float ex = dP * dx, ey = dP * dy;
    g[0] += ex;
    g[1] += ey;
    g[2] = fmaf(ex, dx, g[2]);
    g[3] = fmaf(ex, dy, g[3]);
    g[4] = fmaf(ey, dy, g[4]);
}

__global__ __launch_bounds__(TB_THREADS) void k_raster_backward_train(FrameDev f, WsDev ws,
                                                                      const uint32_t* __restrict__ vals,
                                                                      const float* __restrict__ dimg,
                                                                      float4* __restrict__ partial, FrameKey key) {
    // per-wave lists of the batch's folded entries, in depth order
    __shared__ float4 s_a[2][TB_BATCH];      // C1, C2, C3, C4 (log2 units)
    __shared__ float4 s_b[2][TB_BATCH];      // C5, C6, entry index, slot in the batch (bits)
    __shared__ float4 s_m[2][TB_BATCH];      // r, g, b, v (tile-centre)
    __shared__ float4 s_q[2][TB_BATCH];      // A, B, C, u (tile-centre)
    __shared__ uint32_t s_cnt[2];
    __shared__ uint32_t s_wlast[2];
    // [wave][term][half][slot]: an entry's sums over each 32-lane half of a wave
    __shared__ float4 s_acc4[2 * 9 * 2 * TB_BATCH / 4];
    float (*s_acc)[9][2][TB_BATCH] = reinterpret_cast<float (*)[9][2][TB_BATCH]>(s_acc4);
    if (!frame_matches(ws, key)) return;
    if (blockIdx.x >= (uint32_t)f.n_tiles) return;
    const uint32_t tile = f.ordered ? ws.order[blockIdx.x] : blockIdx.x;   // the rasterizers' schedule
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64, lane = tid % 64;
    const uint32_t lx = tid % TILE, ly = 2 * (tid / TILE);
    const uint32_t px = tx * TILE + lx, py = ty * TILE + ly;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    // tile-centre coordinates, as the forward pass
    const float ox = (float)(tx * TILE) + 7.5f, oy = (float)(ty * TILE) + 7.5f;
    const float x = (float)lx - 7.5f, y = (float)ly - 7.5f;
    const float x2 = x * x, xy = x * y, y2 = y * y, y21 = fmaf(2.0f, y, 1.0f);
    const float y1 = y + 1.0f;
    const uint64_t plane = (uint64_t)f.width * f.height;
    const float bg0 = ws.params->cam.bg[0], bg1 = ws.params->cam.bg[1], bg2 = ws.params->cam.bg[2];

    // per pixel: T after the pairs behind, dL/dC, DS = dL/dC . (colour behind +
    // T_final bg), and the end of the pairs [start, last) that may have been blended
    float T[2], d[2][3], DS[2];
    uint32_t last[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        T[k] = 1.0f;
        last[k] = start;
        d[k][0] = d[k][1] = d[k][2] = 0.0f;
        if (px < (uint32_t)f.width && py + k < (uint32_t)f.height) {
            const uint64_t o = (uint64_t)(py + k) * f.width + px;
            T[k] = ws.t_final[o];
            const uint32_t word = ws.n_proc[o];
            last[k] = start + (word & ~N_PROC_STOPPED) - ((word & N_PROC_STOPPED) ? 1u : 0u);
            d[k][0] = dimg[o];
            d[k][1] = dimg[plane + o];
            d[k][2] = dimg[2 * plane + o];
        }
        DS[k] = T[k] * fmaf(d[k][0], bg0, fmaf(d[k][1], bg1, d[k][2] * bg2));
    }
    uint32_t wlast = max(last[0], last[1]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, off));
    if (lane == 0) s_wlast[wave] = wlast;
    __syncthreads();
    const uint32_t tile_last = max(s_wlast[0], s_wlast[1]);

    for (uint32_t b_end = tile_last; b_end > start;) {
        const uint32_t b0 = b_end - start > (uint32_t)TB_BATCH ? b_end - TB_BATCH : start;
        const uint32_t cnt = b_end - b0;
        __syncthreads();                         // the previous batch is fully read
        for (uint32_t q = tid; q < 2 * 9 * 2 * TB_BATCH / 4; q += TB_THREADS) s_acc4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        // ---- stage (wave 0, one entry per lane): fold, cull, compact per wave ----
        uint64_t my_pos = 0;
        float eA = 0.0f, eB = 0.0f, eC = 0.0f;     // the staged entry's conic
        if (wave == 0) {
            bool hit0 = false, hit1 = false;
            float4 ca = make_float4(0.f, 0.f, 0.f, 0.f), cbv = ca, q4 = ca;
            float u = 0.0f, v = 0.0f, cb = 0.0f;
            const uint32_t idx = b0 + lane;
            if (lane < cnt) {
                const uint32_t g0 = vals[idx];
                const uint32_t g = g0 < f.n_gaussians ? g0 : 0u;
                const Record rec = ws.records[g];
                fold_record<true>(rec, ox, oy, u, v, ca, cbv);
                cb = rec.b;
                q4 = make_float4(rec.A, rec.B, rec.C, u);
                eA = rec.A;
                eB = rec.B;
                eC = rec.C;
                cull_half_tiles(rec, u, v, hit0, hit1);
                my_pos = emission_pos(ws, g, tx, ty);
            }
            const uint64_t m0 = __ballot(hit0), m1 = __ballot(hit1);
            const uint64_t lt = lanemask_lt();
            const float4 b4 = make_float4(cbv.x, cbv.y, __uint_as_float(idx), __uint_as_float(lane));
            const float4 m4 = make_float4(cbv.z, cbv.w, cb, v);
            if (hit0) {
                const uint32_t p = (uint32_t)__popcll(m0 & lt);
                s_a[0][p] = ca;
                s_b[0][p] = b4;
                s_m[0][p] = m4;
                s_q[0][p] = q4;
            }
            if (hit1) {
                const uint32_t p = (uint32_t)__popcll(m1 & lt);
                s_a[1][p] = ca;
                s_b[1][p] = b4;
                s_m[1][p] = m4;
                s_q[1][p] = q4;
            }
            if (lane == 0) {
                s_cnt[0] = (uint32_t)__popcll(m0);
                s_cnt[1] = (uint32_t)__popcll(m1);
            }
        }
        __syncthreads();
        // ---- this wave's list, back to front ----
        const uint32_t n = __builtin_amdgcn_readfirstlane(s_cnt[wave]);
        // each step reads the next (closer) entry's exponent coefficients ahead,
        // so that their LDS latency overlaps this step's work
        float4 b4n = make_float4(0.f, 0.f, 0.f, 0.f), an = b4n;
        if (n) {
            b4n = s_b[wave][n - 1];
            an = s_a[wave][n - 1];
        }
        for (int k = (int)n - 1; k >= 0; --k) {
            const float4 b4 = b4n, a = an;
            if (k > 0) {
                b4n = s_b[wave][k - 1];
                an = s_a[wave][k - 1];
            }
            const uint32_t idx = __float_as_uint(b4.z);
            if (idx >= wlast) continue;          // no pixel of the wave got this far
            float P0, P1;
            folded_exponents(a, b4.x, b4.y, x, y, x2, xy, y2, y21, P0, P1);
            const bool pass0 = idx < last[0] && P0 >= -LOG2_255F;
            const bool pass1 = idx < last[1] && P1 >= -LOG2_255F;
            if (__ballot(pass0 || pass1) == 0) continue;
            const float4 mg = s_m[wave][k];
            const float4 abc = s_q[wave][k];
            const float dx = x - abc.w;
            float g[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) g[c] = 0.0f;
            if (pass0) pair_adjoint(P0, dx, y - mg.w, mg, d[0], T[0], DS[0], g);
            if (pass1) pair_adjoint(P1, dx, y1 - mg.w, mg, d[1], T[1], DS[1], g);
            row_sums(g);
            // row_bcast:15, taken by every lane (the compiler would otherwise move
            // the add under the store's lane mask and broadcast through extra moves)
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                g[c] += dpp_moved<0x142>(g[c]);
                asm volatile("" : "+v"(g[c]));
            }
            if ((lane & 31) == 31) {
                const uint32_t slot = __float_as_uint(b4.w), half = lane >> 5;
#pragma unroll
                for (int c = 0; c < 9; ++c) s_acc[wave][c][half][slot] = g[c];
            }
        }
        __syncthreads();
        if (tid < cnt) {
            float4* dst = partial + 3ull * my_pos;
            float sum[9];
#pragma unroll
            for (int c = 0; c < 9; ++c)
                sum[c] = (s_acc[0][c][0][tid] + s_acc[0][c][1][tid]) + (s_acc[1][c][0][tid] + s_acc[1][c][1][tid]);
            // moments of dL/dP -> dL/d(u, v, A, B, C) with the entry's conic
            const float m1 = sum[0], m2 = sum[1];
            sum[0] = fmaf(eA, m1, eB * m2);      // dp/du = A dx + B dy
            sum[1] = fmaf(eC, m2, eB * m1);      // dp/dv = C dy + B dx
            sum[2] *= -0.5f;
            sum[3] = -sum[3];
            sum[4] *= -0.5f;
            dst[0] = make_float4(sum[0], sum[1], sum[2], sum[3]);
            dst[1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
            dst[2] = make_float4(sum[8], 0.0f, 0.0f, 0.0f);
        }
        b_end = b0;
    }
    // entries no pixel of the tile reached
    for (uint32_t idx = tile_last + tid; idx < end; idx += TB_THREADS) {
        const uint32_t g = vals[idx];
        float4* dst = partial + 3ull * emission_pos(ws, g < f.n_gaussians ? g : 0u, tx, ty);
        dst[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        dst[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        dst[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

void launch_raster_backward_train(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b,
                                  const float* dimg, float4* partial, FrameKey key) {
    const uint32_t* vals = result_in_b ? ws.vals_b : ws.vals_a;
    hipLaunchKernelGGL(k_raster_backward_train, dim3((uint32_t)f.n_tiles), dim3(TB_THREADS), 0, s, f, ws, vals,
                       dimg, partial, key);
}

// ---------------------------------------------------------------------------
// Per-Gaussian gather and chain rule.

// sum_k gY_k dY_k/d(x, y, z) for the degree-3 basis written as polynomials in
// (x, y, z) (the forward basis, in double).
__device__ inline void sh_basis_backward(double x, double y, double z, const double* gY, double& gx,
                                         double& gy, double& gz) {
    const double pi = 3.14159265358979323846;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    const double xx = x * x, yy = y * y, zz = z * z;
    gx = -c1 * gY[3] + c2a * y * gY[4] - 2.0 * c2b * x * gY[6] - c2a * z * gY[7] + 2.0 * c2c * x * gY[8] -
         c3a * 6.0 * x * y * gY[9] + c3b * y * z * gY[10] + c3c * 2.0 * x * y * gY[11] -
         c3d * 6.0 * x * z * gY[12] - c3c * (4.0 * zz - 3.0 * xx - yy) * gY[13] + c3e * 2.0 * x * z * gY[14] -
         c3a * (3.0 * xx - 3.0 * yy) * gY[15];
    gy = -c1 * gY[1] + c2a * x * gY[4] - c2a * z * gY[5] - 2.0 * c2b * y * gY[6] - 2.0 * c2c * y * gY[8] -
         c3a * (3.0 * xx - 3.0 * yy) * gY[9] + c3b * x * z * gY[10] - c3c * (4.0 * zz - xx - 3.0 * yy) * gY[11] -
         c3d * 6.0 * y * z * gY[12] + c3c * 2.0 * x * y * gY[13] - c3e * 2.0 * y * z * gY[14] +
         c3a * 6.0 * x * y * gY[15];
    gz = c1 * gY[2] - c2a * y * gY[5] + 4.0 * c2b * z * gY[6] - c2a * x * gY[7] + c3b * x * y * gY[10] -
         c3c * 8.0 * y * z * gY[11] + c3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * gY[12] - c3c * 8.0 * x * z * gY[13] +
         c3e * (xx - yy) * gY[14];
}

__device__ inline void sh_basis_double(double x, double y, double z, double* Y) {
    const double pi = 3.14159265358979323846;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.5 / sqrt(pi);
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    Y[9] = -c3a * y * (3.0 * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * zz - xx - yy);
    Y[12] = c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -c3c * x * (4.0 * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0 * yy);
}

constexpr int GRAD_THREADS = 128;

// Gradients of Gaussian i: sum of its partials, then the chain rule.  The SH
// gradients go to dsh (48 floats, LDS), the rest straight to global memory.
// refused: the workspace holds another frame than the caller's; all gradients are zero.
__device__ inline void grad_one(const PlainSceneDev& sc, const CamDev& cam, const WsDev& ws,
                                const float4* __restrict__ partial, const GradOut& go, int64_t i,
                                float* dsh, bool lno_opacity, bool refused) {
    const uint32_t count = refused ? 0u : ws.counts[i];
    double gs[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) gs[c] = 0.0;
    if (count) {
        const float4* pp = partial + 3ull * ws.offsets[i];
        float acc[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[c] = 0.0f;
        for (uint32_t q = 0; q < count; ++q, pp += 3) {
            const float4 p0 = pp[0], p1 = pp[1], p2 = pp[2];
            acc[0] += p0.x; acc[1] += p0.y; acc[2] += p0.z; acc[3] += p0.w;
            acc[4] += p1.x; acc[5] += p1.y; acc[6] += p1.z; acc[7] += p1.w;
            acc[8] += p2.x;
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) gs[c] = acc[c];
        if (lno_opacity) {      // dL/do = dL/d(ln o) / o
            const double o = sc.base[P_OPA * sc.n_pad + i];
            gs[5] = o > 0.0 ? gs[5] / o : 0.0;
        }
    }
    if (go.screen) {
#pragma unroll
        for (int c = 0; c < 9; ++c) go.screen[9 * i + c] = (float)gs[c];
    }
    float* dm = go.means + 3 * i;
    float* ds = go.scales + 3 * i;
    float* dq = go.quats + 4 * i;
    if (!count) {
#pragma unroll
        for (int k = 0; k < 3; ++k) dm[k] = 0.0f, ds[k] = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) dq[k] = 0.0f;
        go.opacity[i] = 0.0f;
        for (int k = 0; k < 48; ++k) dsh[k] = 0.0f;
        return;
    }
    const float* P = sc.base;
    const uint64_t np = sc.n_pad;
    const double mx = P[P_MX * np + i], my = P[P_MY * np + i], mz = P[P_MZ * np + i];
    const double s[3] = {P[P_SX * np + i], P[P_SY * np + i], P[P_SZ * np + i]};
    const double qw0 = P[P_QW * np + i], qx0 = P[P_QX * np + i], qy0 = P[P_QY * np + i], qz0 = P[P_QZ * np + i];
    const double* r = cam.r;
    const double g_u = gs[0], g_v = gs[1], g_A = gs[2], g_B = gs[3], g_C = gs[4];

    // forward quantities (the forward pass's expressions)
    const double tx = r[0] * mx + r[1] * my + r[2] * mz + cam.t[0];
    const double ty = r[3] * mx + r[4] * my + r[5] * mz + cam.t[1];
    const double d = r[6] * mx + r[7] * my + r[8] * mz + cam.t[2];
    const double nq = sqrt(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
    const double w = qw0 / nq, x = qx0 / nq, y = qy0 / nq, z = qz0 / nq;
    double R[3][3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
    double M[3][3], S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) M[a][k] = R[a][k] * s[k];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = M[a][0] * M[b][0] + M[a][1] * M[b][1] + M[a][2] * M[b][2];
    const double limx = J_CLAMP * cam.tanx, limy = J_CLAMP * cam.tany;
    const double rx = tx / d, ry = ty / d;
    const bool inx = rx > -limx && rx < limx, iny = ry > -limy && ry < limy;
    const double xc = fmin(limx, fmax(-limx, rx)) * d;
    const double yc = fmin(limy, fmax(-limy, ry)) * d;
    const double dd = d * d;
    const double j00 = cam.fx / d, j02 = -(cam.fx * xc) / dd;
    const double j11 = cam.fy / d, j12 = -(cam.fy * yc) / dd;
    double T0[3], T1[3];
    for (int k = 0; k < 3; ++k) {
        T0[k] = j00 * r[k] + j02 * r[6 + k];
        T1[k] = j11 * r[3 + k] + j12 * r[6 + k];
    }
    double ST0[3], ST1[3];
    for (int a = 0; a < 3; ++a) {
        ST0[a] = S[a][0] * T0[0] + S[a][1] * T0[1] + S[a][2] * T0[2];
        ST1[a] = S[a][0] * T1[0] + S[a][1] * T1[1] + S[a][2] * T1[2];
    }
    const double c00 = T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2] + DILATION;
    const double c01 = T0[0] * ST1[0] + T0[1] * ST1[1] + T0[2] * ST1[2];
    const double c11 = T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2] + DILATION;
    const double det = c00 * c11 - c01 * c01;
    const double id = 1.0 / det, id2 = id * id;

    // conic (A, B, C) = (c11, -c01, c00) / det  ->  Sigma' entries
    const double g00 = g_A * (-c11 * c11 * id2) + g_B * (c01 * c11 * id2) + g_C * (id - c00 * c11 * id2);
    const double g11 = g_A * (id - c11 * c00 * id2) + g_B * (c01 * c00 * id2) + g_C * (-c00 * c00 * id2);
    const double g01 = g_A * (2.0 * c01 * c11 * id2) + g_B * (-id - 2.0 * c01 * c01 * id2) +
                       g_C * (2.0 * c00 * c01 * id2);
    // Sigma' = T Sigma T^T
    double gT0[3], gT1[3];
    for (int a = 0; a < 3; ++a) {
        gT0[a] = 2.0 * g00 * ST0[a] + g01 * ST1[a];
        gT1[a] = 2.0 * g11 * ST1[a] + g01 * ST0[a];
    }
    // symmetrised dL/dSigma: GS + GS^T with GS = g00 T0 T0^T + g01 T0 T1^T + g11 T1 T1^T
    double GSs[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            GSs[a][b] = 2.0 * g00 * T0[a] * T0[b] + g01 * (T0[a] * T1[b] + T0[b] * T1[a]) +
                        2.0 * g11 * T1[a] * T1[b];
    // T = J R_w
    const double g_j00 = gT0[0] * r[0] + gT0[1] * r[1] + gT0[2] * r[2];
    const double g_j02 = gT0[0] * r[6] + gT0[1] * r[7] + gT0[2] * r[8];
    const double g_j11 = gT1[0] * r[3] + gT1[1] * r[4] + gT1[2] * r[5];
    const double g_j12 = gT1[0] * r[6] + gT1[1] * r[7] + gT1[2] * r[8];
    // J and (u, v) -> camera-space t
    const double g_tx = g_u * cam.fx / d + (inx ? g_j02 * (-cam.fx / dd) : 0.0);
    const double g_ty = g_v * cam.fy / d + (iny ? g_j12 * (-cam.fy / dd) : 0.0);
    const double sgx = rx > 0.0 ? 1.0 : -1.0, sgy = ry > 0.0 ? 1.0 : -1.0;
    const double g_d = g_u * (-cam.fx * tx / dd) + g_v * (-cam.fy * ty / dd) + g_j00 * (-cam.fx / dd) +
                       g_j11 * (-cam.fy / dd) +
                       g_j02 * (inx ? 2.0 * cam.fx * tx / (dd * d) : cam.fx * sgx * limx / dd) +
                       g_j12 * (iny ? 2.0 * cam.fy * ty / (dd * d) : cam.fy * sgy * limy / dd);
    double gmu[3];
    for (int k = 0; k < 3; ++k) gmu[k] = r[k] * g_tx + r[3 + k] * g_ty + r[6 + k] * g_d;
    // Sigma = M M^T, M = R diag(s)
    double gM[3][3], gR[3][3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) gM[a][k] = GSs[a][0] * M[0][k] + GSs[a][1] * M[1][k] + GSs[a][2] * M[2][k];
    for (int k = 0; k < 3; ++k) ds[k] = (float)(gM[0][k] * R[0][k] + gM[1][k] * R[1][k] + gM[2][k] * R[2][k]);
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) gR[a][k] = gM[a][k] * s[k];
    // rotation of the unit quaternion (w, x, y, z)
    const double gw = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    const double gx = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] +
                             z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2]);
    const double gy = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                             w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2]);
    const double gz = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.0 * z * gR[1][1] +
                             y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    const double qdot = w * gw + x * gx + y * gy + z * gz;
    dq[0] = (float)((gw - w * qdot) / nq);
    dq[1] = (float)((gx - x * qdot) / nq);
    dq[2] = (float)((gy - y * qdot) / nq);
    dq[3] = (float)((gz - z * qdot) / nq);
    go.opacity[i] = (float)gs[5];

    // colour: a channel clamped at 0 in the forward pass has no gradient
    const Record rec = ws.records[i];
    const double ga[3] = {rec.r > 0.0f ? gs[6] : 0.0, rec.g > 0.0f ? gs[7] : 0.0, rec.b > 0.0f ? gs[8] : 0.0};
    double cp[3];
    for (int k = 0; k < 3; ++k) cp[k] = -(r[k] * cam.t[0] + r[3 + k] * cam.t[1] + r[6 + k] * cam.t[2]);
    const double vx = mx - cp[0], vy = my - cp[1], vz = mz - cp[2];
    const double vlen = sqrt(vx * vx + vy * vy + vz * vz);
    const double ux = vx / vlen, uy = vy / vlen, uz = vz / vlen;
    double Y[16], gY[16];
    sh_basis_double(ux, uy, uz, Y);
    for (int k = 0; k < 16; ++k) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) {
            dsh[3 * k + c] = (float)(Y[k] * ga[c]);
            acc += (double)P[(P_SH0 + 3 * k + c) * np + i] * ga[c];
        }
        gY[k] = acc;
    }
    double gdx, gdy, gdz;
    sh_basis_backward(ux, uy, uz, gY, gdx, gdy, gdz);
    const double dot = ux * gdx + uy * gdy + uz * gdz;
    gmu[0] += (gdx - ux * dot) / vlen;
    gmu[1] += (gdy - uy * dot) / vlen;
    gmu[2] += (gdz - uz * dot) / vlen;
    for (int k = 0; k < 3; ++k) dm[k] = (float)gmu[k];
}

template <bool LNO>
__global__ __launch_bounds__(GRAD_THREADS) void k_grad_gaussian(PlainSceneDev sc, CamDev cam, WsDev ws,
                                                                const float4* __restrict__ partial,
                                                                GradOut go, FrameKey key) {
    __shared__ float s_sh[GRAD_THREADS * 48];
    const int64_t first = (int64_t)blockIdx.x * GRAD_THREADS;
    const int64_t i = first + threadIdx.x;
    const bool refused = ws.params->scene_tag != key.scene_tag || ws.params->cam_hash != key.cam_hash;
    if (i < sc.n) grad_one(sc, cam, ws, partial, go, i, s_sh + 48 * threadIdx.x, LNO, refused);
    __syncthreads();
    const int64_t rows = sc.n - first < GRAD_THREADS ? sc.n - first : GRAD_THREADS;
    float* dst = go.sh + 48 * first;
    for (int64_t k = threadIdx.x; k < rows * 48; k += GRAD_THREADS) dst[k] = s_sh[k];
}

void launch_grad_gaussian(hipStream_t s, const PlainSceneDev& sc, const CamDev& cam, const WsDev& ws,
                          const float4* partial, const GradOut& go, bool lno_opacity, FrameKey key) {
    if (sc.n <= 0) return;
    const dim3 grid((uint32_t)((sc.n + GRAD_THREADS - 1) / GRAD_THREADS)), block(GRAD_THREADS);
    if (lno_opacity) hipLaunchKernelGGL(k_grad_gaussian<true>, grid, block, 0, s, sc, cam, ws, partial, go, key);
    else hipLaunchKernelGGL(k_grad_gaussian<false>, grid, block, 0, s, sc, cam, ws, partial, go, key);
}

}  // namespace rgs
