// Tile rasterizers (Sec. III-D, Sec. IV-B).
//
// One workgroup blends one 16x16 tile front to back over the tile's sorted
// list, staging the Gaussian records of each batch in LDS; every thread owns
// fixed pixels and keeps its transmittance T and colour in registers.  A pair
// is skipped when its opacity is below 1/255, blending of a pixel stops at the
// first pair that would take T below 1e-4, and alpha is clamped at 0.99
// (Eq. opacity_clamped).  The workgroup leaves as soon as all its pixels have
// stopped (checked at every batch).
//
// `raster_plain` is the 3DGS baseline: 256 threads, one pixel each, the exponent
// of Eq. power from (x - u, y - v) and the accurate expf.
//
// `raster_fast` applies Sec. IV-B:
//   * coefficient folding (Eqs. expand, c0, coeff, dot): while a batch is staged
//     the conic, mean and ln o are folded into C1..C6 so that the folded
//     exponent P = p + ln o (Eq. folded_exponent) is
//     C1 x^2 + C2 xy + C3 y^2 + C4 x + C5 y + C6, five FMAs per pixel with x^2,
//     xy, y^2, x, y hoisted.  The paper's b is the doubled off-diagonal of the
//     conic, so C2 = -B and the 0.5 b terms become B.  Coordinates are taken
//     relative to the tile centre, which keeps |x|, |y| <= 7.5 and the folded
//     terms small enough for float32 at any image size;
//   * dual-pixel evaluation (Eq. dual_pixel): each thread owns (x, y) and
//     (x, y+1); the second exponent is P(x,y) + C2 x + C3 (2y + 1) + C5, and
//     both pixels reuse one LDS read of the coefficients; 128 threads per tile;
//   * the range-aware bit-level exponential (Eq. fma_exp): for P in
//     [-ln 255, 0] the bits of exp(P) are built as the integer
//     floor(P 2^23 log2 e + 2^23 (127 - sigma)), sigma = 0.045677, one FMA and
//     one float-to-int conversion.  The skip test is made on P itself.
//
// Tiles are mapped to workgroups so that each of the 8 XCDs (workgroups are
// dispatched to them round-robin) works through one contiguous band of tile
// rows, which keeps the records shared by neighbouring tiles in that XCD's L2.
#include "rgs_internal.h"

namespace rgs {

__device__ inline uint32_t xcd_tile(uint32_t block, uint32_t n_tiles) {
    const uint32_t per = (n_tiles + 7u) / 8u;
    return (block % 8u) * per + block / 8u;
}

static uint32_t xcd_grid(uint32_t n_tiles) { return 8u * ((n_tiles + 7u) / 8u); }

// 2^23 log2(e) = 12102203.16 and 2^23 (127 - 0.045677) = 1064970049.55,
// rounded to the nearest float32 (spacing 1 and 64 at these magnitudes).
constexpr float FEXP_A = 12102203.0f;
constexpr float FEXP_B = 1064970048.0f;

__device__ inline float fast_exp(float P) {
    return __int_as_float((int)fmaf(P, FEXP_A, FEXP_B));
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_raster_plain(FrameDev f, CamDev cam, WsDev ws,
                                                      const uint32_t* __restrict__ vals,
                                                      float* __restrict__ out) {
    __shared__ float4 s_a[256];   // u, v (tile-local), A, B
    __shared__ float4 s_b[256];   // C, opacity, r, g
    __shared__ float s_c[256];    // b
    const uint32_t tile = xcd_tile(blockIdx.x, (uint32_t)f.n_tiles);
    if (tile >= (uint32_t)f.n_tiles) return;
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lx = tid % TILE, ly = tid / TILE;
    const uint32_t px = tx * TILE + lx, py = ty * TILE + ly;
    const bool inside = px < (uint32_t)f.width && py < (uint32_t)f.height;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    const float ox = (float)(tx * TILE), oy = (float)(ty * TILE);
    const float x = (float)lx, y = (float)ly;

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    bool done = !inside;
    uint32_t stop_at = 0xffffffffu;
    for (uint32_t b0 = start; b0 < end; b0 += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t idx = b0 + tid;
        if (idx < end) {
            const uint32_t g = vals[idx];
            const Record rec = ws.records[g < f.n_gaussians ? g : 0u];
            s_a[tid] = make_float4((rec.u_hi - ox) + rec.u_lo, (rec.v_hi - oy) + rec.v_lo, rec.A, rec.B);
            s_b[tid] = make_float4(rec.C, rec.opa, rec.r, rec.g);
            s_c[tid] = rec.b;
        }
        __syncthreads();
        const uint32_t cnt = min(256u, end - b0);
        if (!done) {
            for (uint32_t j = 0; j < cnt; ++j) {
                const float4 a = s_a[j];
                const float4 m = s_b[j];
                const float dx = x - a.x, dy = y - a.y;
                const float p = fmaf(-0.5f, fmaf(a.z * dx, dx, m.x * dy * dy), -a.w * dx * dy);
                const float alpha = fminf(ALPHA_MAX, m.y * expf(p));
                if (alpha < ALPHA_MIN) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < T_MIN) {
                    done = true;
                    stop_at = b0 + j;
                    break;
                }
                const float w = alpha * T;
                cr = fmaf(w, m.z, cr);
                cg = fmaf(w, m.w, cg);
                cb = fmaf(w, s_c[j], cb);
                T = Tn;
            }
        }
        __syncthreads();
    }
    if (inside) {
        const uint64_t plane = (uint64_t)f.width * f.height;
        const uint64_t o = (uint64_t)py * f.width + px;
        out[o] = fmaf(T, cam.bg[0], cr);
        out[plane + o] = fmaf(T, cam.bg[1], cg);
        out[2 * plane + o] = fmaf(T, cam.bg[2], cb);
        ws.t_final[o] = T;
        ws.n_proc[o] = stop_at != 0xffffffffu ? stop_at - start + 1 : end - start;
    }
}

void launch_raster_plain(hipStream_t s, const FrameDev& f, const CamDev& cam, const WsDev& ws,
                         bool result_in_b, float* out) {
    hipLaunchKernelGGL(k_raster_plain, dim3(xcd_grid(f.n_tiles)), dim3(256), 0, s, f, cam, ws,
                       result_in_b ? ws.vals_b : ws.vals_a, out);
}

// ---------------------------------------------------------------------------

constexpr int FAST_THREADS = 128;

struct PixelState {
    float T, r, g, b;
    bool done;
    uint32_t stop_at;
};

__device__ inline void blend_fast(PixelState& s, float P, float cr, float cg, float cb, uint32_t at) {
    if (!s.done && P >= -LN255F) {
        const float alpha = fminf(ALPHA_MAX, fast_exp(P));
        const float Tn = fmaf(-alpha, s.T, s.T);
        if (Tn < T_MIN) {
            s.done = true;
            s.stop_at = at;
        } else {
            const float w = alpha * s.T;
            s.r = fmaf(w, cr, s.r);
            s.g = fmaf(w, cg, s.g);
            s.b = fmaf(w, cb, s.b);
            s.T = Tn;
        }
    }
}

__global__ __launch_bounds__(FAST_THREADS) void k_raster_fast(FrameDev f, CamDev cam, WsDev ws,
                                                              const uint32_t* __restrict__ vals,
                                                              float* __restrict__ out) {
    __shared__ float4 s_a[FAST_THREADS];   // C1, C2, C3, C4
    __shared__ float4 s_b[FAST_THREADS];   // C5, C6, r, g
    __shared__ float s_c[FAST_THREADS];    // b
    const uint32_t tile = xcd_tile(blockIdx.x, (uint32_t)f.n_tiles);
    if (tile >= (uint32_t)f.n_tiles) return;
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lx = tid % TILE, ly = 2 * (tid / TILE);
    const uint32_t px = tx * TILE + lx, py = ty * TILE + ly;
    const bool in0 = px < (uint32_t)f.width && py < (uint32_t)f.height;
    const bool in1 = px < (uint32_t)f.width && py + 1 < (uint32_t)f.height;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    // tile-centre coordinates
    const float ox = (float)(tx * TILE) + 7.5f, oy = (float)(ty * TILE) + 7.5f;
    const float x = (float)lx - 7.5f, y = (float)ly - 7.5f;
    const float x2 = x * x, xy = x * y, y2 = y * y, y21 = fmaf(2.0f, y, 1.0f);

    PixelState p0{1.0f, 0.0f, 0.0f, 0.0f, !in0, 0xffffffffu};
    PixelState p1{1.0f, 0.0f, 0.0f, 0.0f, !in1, 0xffffffffu};
    for (uint32_t b0 = start; b0 < end; b0 += FAST_THREADS) {
        if (__syncthreads_count(!(p0.done && p1.done)) == 0) break;
        const uint32_t idx = b0 + tid;
        if (idx < end) {
            const uint32_t g = vals[idx];
            const Record rec = ws.records[g < f.n_gaussians ? g : 0u];
            const float u = (rec.u_hi - ox) + rec.u_lo;
            const float v = (rec.v_hi - oy) + rec.v_lo;
            const float A = rec.A, B = rec.B, C = rec.C;
            const float C0 = fmaf(A * u, u, fmaf(2.0f * B * u, v, C * v * v));
            s_a[tid] = make_float4(-0.5f * A, -B, -0.5f * C, fmaf(A, u, B * v));
            s_b[tid] = make_float4(fmaf(C, v, B * u), fmaf(-0.5f, C0, rec.opa), rec.r, rec.g);
            s_c[tid] = rec.b;
        }
        __syncthreads();
        const uint32_t cnt = min((uint32_t)FAST_THREADS, end - b0);
        for (uint32_t j = 0; j < cnt; ++j) {
            if (p0.done && p1.done) break;
            const float4 a = s_a[j];
            const float4 m = s_b[j];
            const float P0 = fmaf(a.x, x2, fmaf(a.y, xy, fmaf(a.z, y2, fmaf(a.w, x, fmaf(m.x, y, m.y)))));
            const float P1 = P0 + fmaf(a.y, x, fmaf(a.z, y21, m.x));
            const float cb = s_c[j];
            blend_fast(p0, P0, m.z, m.w, cb, b0 + j);
            blend_fast(p1, P1, m.z, m.w, cb, b0 + j);
        }
        __syncthreads();
    }
    const uint64_t plane = (uint64_t)f.width * f.height;
    if (in0) {
        const uint64_t o = (uint64_t)py * f.width + px;
        out[o] = fmaf(p0.T, cam.bg[0], p0.r);
        out[plane + o] = fmaf(p0.T, cam.bg[1], p0.g);
        out[2 * plane + o] = fmaf(p0.T, cam.bg[2], p0.b);
        ws.t_final[o] = p0.T;
        ws.n_proc[o] = p0.stop_at != 0xffffffffu ? p0.stop_at - start + 1 : end - start;
    }
    if (in1) {
        const uint64_t o = (uint64_t)(py + 1) * f.width + px;
        out[o] = fmaf(p1.T, cam.bg[0], p1.r);
        out[plane + o] = fmaf(p1.T, cam.bg[1], p1.g);
        out[2 * plane + o] = fmaf(p1.T, cam.bg[2], p1.b);
        ws.t_final[o] = p1.T;
        ws.n_proc[o] = p1.stop_at != 0xffffffffu ? p1.stop_at - start + 1 : end - start;
    }
}

void launch_raster_fast(hipStream_t s, const FrameDev& f, const CamDev& cam, const WsDev& ws,
                        bool result_in_b, float* out) {
    hipLaunchKernelGGL(k_raster_fast, dim3(xcd_grid(f.n_tiles)), dim3(FAST_THREADS), 0, s, f, cam, ws,
                       result_in_b ? ws.vals_b : ws.vals_a, out);
}

}  // namespace rgs
