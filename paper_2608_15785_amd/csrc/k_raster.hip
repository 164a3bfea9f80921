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
//     one float-to-int conversion.  The skip test is made on P itself;
//   * per-wave culled lists: while a batch is staged, each Gaussian is tested
//     against the two 16x8 half-tiles of the two waves, first with the box of
//     its alpha >= 1/255 ellipse, then with the ellipse itself (the least value
//     of its quadratic form over the half-tile), both widened far beyond the
//     float32 error of P; each wave blends only its survivors, in depth order.
//     A culled pair would have failed the skip test, so no result changes.
//
// `raster_train` is the training variant of the plain path: the dual-pixel
// rasterizer with the culled lists over the plain path's float32 records
// (which then carry ln o and the box), with log2 e folded into C1..C6 and
// alpha = min(0.99, exp2(P)) from the hardware exp2.  It also leaves each
// pixel's final T and visited-pair count; the backward pass replays the same
// lists with the same folding, so it recomputes every alpha bit for bit.
//
// Workgroup b renders tile ws.order[b] (longest lists first, so that the grid
// does not end on a few long tiles; see the tile-order kernel) in frames that
// take the schedule, else tile b in row-major order.  Workgroups are
// dispatched to the 8 XCDs round-robin, so the tiles' uneven work spreads
// evenly over the XCDs.  Giving each XCD one contiguous band of tile rows
// (for its L2) was 4 % slower than row-major at 1M / 1080p, and bands of two
// rows dealt out round-robin 8 % slower.
#include "rgs_fold.h"

namespace rgs {

// 2^23 log2(e) = 12102203.16 and 2^23 (127 - 0.045677) = 1064970049.55,
// rounded to the nearest float32 (spacing 1 and 64 at these magnitudes).
constexpr float FEXP_A = 12102203.0f;
constexpr float FEXP_B = 1064970048.0f;

// ---------------------------------------------------------------------------

template <bool COUNT>
__global__ __launch_bounds__(256) void k_raster_plain(FrameDev f, WsDev ws,
                                                      const uint32_t* __restrict__ vals) {
    __shared__ float4 s_a[256];   // u, v (tile-local), A, B
    __shared__ float4 s_b[256];   // C, opacity, r, g
    __shared__ float s_c[256];    // b
    if (blockIdx.x >= (uint32_t)f.n_tiles) return;
    const uint32_t tile = f.ordered ? ws.order[blockIdx.x] : blockIdx.x;
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
    uint32_t n_blend = 0;
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
                const float e = expf(p);
                const float alpha = fminf(ALPHA_MAX, m.y * e);
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
                if (COUNT) ++n_blend;
            }
        }
        __syncthreads();
    }
    if (inside) {
        const uint64_t plane = (uint64_t)f.width * f.height;
        const uint64_t o = (uint64_t)py * f.width + px;
        float* __restrict__ out = ws.params->out;
        const float bg0 = ws.params->cam.bg[0], bg1 = ws.params->cam.bg[1], bg2 = ws.params->cam.bg[2];
        out[o] = fmaf(T, bg0, cr);
        out[plane + o] = fmaf(T, bg1, cg);
        out[2 * plane + o] = fmaf(T, bg2, cb);
        ws.t_final[o] = T;
        ws.n_proc[o] = stop_at != 0xffffffffu ? (stop_at - start + 1) | N_PROC_STOPPED : end - start;
        if (COUNT) ws.n_blend[o] = n_blend;
    }
}

void launch_raster_plain(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count) {
    const uint32_t* vals = result_in_b ? ws.vals_b : ws.vals_a;
    const dim3 grid((uint32_t)f.n_tiles), block(256);
    if (count) hipLaunchKernelGGL(k_raster_plain<true>, grid, block, 0, s, f, ws, vals);
    else hipLaunchKernelGGL(k_raster_plain<false>, grid, block, 0, s, f, ws, vals);
}

// ---------------------------------------------------------------------------

constexpr int FAST_THREADS = 128;    // 2 waves: wave w owns tile rows 8w .. 8w+7
constexpr int FAST_BATCH = FAST_THREADS;
constexpr int LIST_UNROLL = 4;
constexpr int LIST_CAP = FAST_BATCH + LIST_UNROLL;
// How the fast rasterizer takes alpha from the folded exponent P.
enum ExpMode : int {
    EXP_BITS = 0,   // Eq. fma_exp: the bit-level exponential (the paper's fast path)
    EXP_LIBM = 1,   // min(0.99, expf(P)): the exponential's ablation
    EXP_HW2 = 2,    // min(0.99, v_exp_f32(P log2 e)) with log2 e folded into C1..C6
};

// TRAIN: the training variant of the plain path (EXP_HW2 over the plain
// path's records, which then hold ln o and the alpha-ellipse box): every
// render also leaves each pixel's final T and visited-pair count for the
// backward pass.
template <bool COUNT, int EXPM, bool TRAIN = false>
__global__ __launch_bounds__(FAST_THREADS) void k_raster_fast(FrameDev f, WsDev ws,
                                                              const uint32_t* __restrict__ vals) {
    constexpr bool EXACT = EXPM == EXP_LIBM;
    // per-wave lists of folded Gaussians, in depth order
    __shared__ float4 s_a[2][LIST_CAP];   // C1, C2, C3, C4
    __shared__ float2 s_b[2][LIST_CAP];   // C5, C6
    __shared__ float4 s_c[2][LIST_CAP];   // r, g, b, list position (as float bits)
    __shared__ uint32_t s_cnt[2][2];      // [wave of the staging thread][list]
    if (blockIdx.x >= (uint32_t)f.n_tiles) return;
    const uint32_t tile = f.ordered ? ws.order[blockIdx.x] : blockIdx.x;
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64, lane = tid % 64;
    const uint32_t lx = tid % TILE, ly = 2 * (tid / TILE);
    const uint32_t px = tx * TILE + lx, py = ty * TILE + ly;
    const bool in0 = px < (uint32_t)f.width && py < (uint32_t)f.height;
    const bool in1 = px < (uint32_t)f.width && py + 1 < (uint32_t)f.height;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    // tile-centre coordinates
    const float ox = (float)(tx * TILE) + 7.5f, oy = (float)(ty * TILE) + 7.5f;
    const float x = (float)lx - 7.5f, y = (float)ly - 7.5f;
    const float x2 = x * x, xy = x * y, y2 = y * y, y21 = fmaf(2.0f, y, 1.0f);

    float T0 = 1.0f, r0 = 0.0f, g0 = 0.0f, b0 = 0.0f;
    float T1 = 1.0f, r1 = 0.0f, g1 = 0.0f, b1 = 0.0f;
    bool live0 = in0, live1 = in1;
    uint32_t stop0 = 0xffffffffu, stop1 = 0xffffffffu;
    uint32_t nbl0 = 0, nbl1 = 0;
    uint32_t steps = 0;         // counting renders: list entries this wave evaluated

    for (uint32_t base = start; base < end; base += FAST_BATCH) {
        if (__syncthreads_count(live0 || live1) == 0) break;
        // ---- stage: fold, cull against both half-tiles, compact per wave ----
        const uint32_t idx = base + tid;
        bool hit0 = false, hit1 = false;
        float4 ca = make_float4(0.f, 0.f, 0.f, 0.f), cbv = make_float4(0.f, 0.f, 0.f, 0.f);
        float cb = 0.f;
        if (idx < end) {
            const uint32_t g = vals[idx];
            const Record rec = ws.records[g < f.n_gaussians ? g : 0u];
            float u, v;
            fold_record<EXPM == EXP_HW2>(rec, ox, oy, u, v, ca, cbv);
            cb = rec.b;
            cull_half_tiles(rec, u, v, hit0, hit1);
        }
        const uint64_t m0 = __ballot(hit0), m1 = __ballot(hit1);
        const uint64_t lt = lanemask_lt();
        if (lane == 0) {
            s_cnt[wave][0] = (uint32_t)__popcll(m0);
            s_cnt[wave][1] = (uint32_t)__popcll(m1);
        }
        __syncthreads();
        const uint32_t off0 = wave ? s_cnt[0][0] : 0u, off1 = wave ? s_cnt[0][1] : 0u;
        const float posf = __uint_as_float(idx);
        if (hit0) {
            const uint32_t p = off0 + (uint32_t)__popcll(m0 & lt);
            s_a[0][p] = ca;
            s_b[0][p] = make_float2(cbv.x, cbv.y);
            s_c[0][p] = make_float4(cbv.z, cbv.w, cb, posf);
        }
        if (hit1) {
            const uint32_t p = off1 + (uint32_t)__popcll(m1 & lt);
            s_a[1][p] = ca;
            s_b[1][p] = make_float2(cbv.x, cbv.y);
            s_c[1][p] = make_float4(cbv.z, cbv.w, cb, posf);
        }
        const uint32_t n0 = s_cnt[0][0] + s_cnt[1][0], n1 = s_cnt[0][1] + s_cnt[1][1];
        // inert padding up to a multiple of the unroll: P = -1e30 is always skipped
        if (tid < 2 * LIST_UNROLL) {
            const uint32_t w = tid / LIST_UNROLL, k = tid % LIST_UNROLL;
            const uint32_t p = (w ? n1 : n0) + k;
            s_a[w][p] = make_float4(0.f, 0.f, 0.f, 0.f);
            s_b[w][p] = make_float2(0.f, -1.0e30f);
            s_c[w][p] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();

        // ---- blend this wave's list ----
        // (the list length is the same for the whole wave: keep it scalar)
        const uint32_t n = __builtin_amdgcn_readfirstlane(wave ? n1 : n0);
        const float4* __restrict__ la = s_a[wave];
        const float2* __restrict__ lb = s_b[wave];
        const float4* __restrict__ lc = s_c[wave];
        if (__ballot(live0 || live1) != 0) {
            bool wave_done = false;     // every pixel of the wave has stopped
            for (uint32_t k0 = 0; k0 < n && !wave_done; k0 += LIST_UNROLL) {
                if (COUNT) steps += LIST_UNROLL;
                float P0s[LIST_UNROLL], P1s[LIST_UNROLL];
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    const float4 a = la[k0 + u];
                    const float2 e = lb[k0 + u];
                    folded_exponents(a, e.x, e.y, x, y, x2, xy, y2, y21, P0s[u], P1s[u]);
                }
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    const float4 c = lc[k0 + u];
                    const float P0 = P0s[u];
                    const float P1 = P1s[u];
                    constexpr float SKIP = EXPM == EXP_HW2 ? -LOG2_255F : -LN255F;
                    const bool pass0 = live0 && P0 >= SKIP;
                    const bool pass1 = live1 && P1 >= SKIP;
                    float al0, al1;
                    if (EXACT) {          // the exponential's ablation: alpha = min(0.99, exp(P))
                        al0 = pass0 ? fminf(ALPHA_MAX, expf(P0)) : 0.0f;
                        al1 = pass1 ? fminf(ALPHA_MAX, expf(P1)) : 0.0f;
                    } else if (EXPM == EXP_HW2) {
                        al0 = pass0 ? fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(P0)) : 0.0f;
                        al1 = pass1 ? fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(P1)) : 0.0f;
                    } else {
                        // alpha = min(0.99, exp_hat(P)) without the minimum, which cannot bind here:
                        // P = ln o - q/2 with ln o <= 0 and q >= 0, and for a kept pair every term of
                        // its float32 evaluation is below ~1600 in magnitude (conic entries <= 1/0.3,
                        // coordinates within a tile), so P < 1e-3 and exp_hat(P) < 0.978
                        al0 = pass0 ? __int_as_float((int)fmaf(P0, FEXP_A, FEXP_B)) : 0.0f;
                        al1 = pass1 ? __int_as_float((int)fmaf(P1, FEXP_A, FEXP_B)) : 0.0f;
                    }
                    const float w0 = al0 * T0, w1 = al1 * T1;
                    float Tn0 = T0 - w0, Tn1 = T1 - w1;
                    float nr0 = fmaf(w0, c.x, r0), ng0 = fmaf(w0, c.y, g0), nb0 = fmaf(w0, c.z, b0);
                    float nr1 = fmaf(w1, c.x, r1), ng1 = fmaf(w1, c.y, g1), nb1 = fmaf(w1, c.z, b1);
                    const bool s0 = Tn0 < T_MIN, s1 = Tn1 < T_MIN;
                    if (COUNT) {
                        nbl0 += (al0 > 0.0f && !s0) ? 1u : 0u;
                        nbl1 += (al1 > 0.0f && !s1) ? 1u : 0u;
                    }
                    if (__ballot(s0 || s1) != 0) {
                        // a pixel reached the stop: that pair is not blended
                        const uint32_t at = __float_as_uint(c.w);
                        if (s0) {
                            live0 = false;
                            stop0 = at;
                            Tn0 = T0; nr0 = r0; ng0 = g0; nb0 = b0;
                        }
                        if (s1) {
                            live1 = false;
                            stop1 = at;
                            Tn1 = T1; nr1 = r1; ng1 = g1; nb1 = b1;
                        }
                        wave_done = __ballot(live0 || live1) == 0;
                    }
                    T0 = Tn0; r0 = nr0; g0 = ng0; b0 = nb0;
                    T1 = Tn1; r1 = nr1; g1 = ng1; b1 = nb1;
                }
            }
        }
        __syncthreads();
    }
    if (COUNT && lane == 0 && steps) atomicAdd(reinterpret_cast<unsigned long long*>(&ws.header->list_steps),
                                               (unsigned long long)steps);
    const uint64_t plane = (uint64_t)f.width * f.height;
    float* __restrict__ out = ws.params->out;
    const float bg0 = ws.params->cam.bg[0], bg1 = ws.params->cam.bg[1], bg2 = ws.params->cam.bg[2];
    if (in0) {
        const uint64_t o = (uint64_t)py * f.width + px;
        out[o] = fmaf(T0, bg0, r0);
        out[plane + o] = fmaf(T0, bg1, g0);
        out[2 * plane + o] = fmaf(T0, bg2, b0);
        if (COUNT || TRAIN) {       // the debug render's and the training variant's per-pixel outputs
            ws.t_final[o] = T0;
            ws.n_proc[o] = stop0 != 0xffffffffu ? (stop0 - start + 1) | N_PROC_STOPPED : end - start;
        }
        if (COUNT) ws.n_blend[o] = nbl0;
    }
    if (in1) {
        const uint64_t o = (uint64_t)(py + 1) * f.width + px;
        out[o] = fmaf(T1, bg0, r1);
        out[plane + o] = fmaf(T1, bg1, g1);
        out[2 * plane + o] = fmaf(T1, bg2, b1);
        if (COUNT || TRAIN) {       // the debug render's and the training variant's per-pixel outputs
            ws.t_final[o] = T1;
            ws.n_proc[o] = stop1 != 0xffffffffu ? (stop1 - start + 1) | N_PROC_STOPPED : end - start;
        }
        if (COUNT) ws.n_blend[o] = nbl1;
    }
}

// One, or four, pixels per lane: the dual-pixel ablation (one pixel per
// thread, four waves of 16x4 rows) and its extension along the column (four
// pixels per lane, Eq. dual_pixel applied three times, one wave per tile).  A
// tile's workgroup has one wave per band of 4 PIX rows: the 64 lanes of a wave
// form four row groups of 16 columns, group j owning PIX consecutive rows and
// each lane PIX pixels of one column.  Staging, culling and the per-pair
// decisions are those of the dual-pixel kernel above, written for any PIX.
template <int PIX>
struct FastShape {
    static constexpr int ROWS = 4 * PIX;            // rows of a wave's band
    static constexpr int WAVES = TILE / ROWS;       // waves per tile
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int BATCH = THREADS;           // entries staged at once, one per thread
    static constexpr int CAP = BATCH + LIST_UNROLL;
};

template <int EXPM>
__device__ inline float fast_alpha(float P) {
    if (EXPM == EXP_LIBM) return fminf(ALPHA_MAX, expf(P));
    if (EXPM == EXP_HW2) return fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(P));
    // min(0.99, exp_hat(P)) without the minimum, which cannot bind here: P = ln o - q/2 with
    // ln o <= 0 and q >= 0, and for a kept pair every term of its float32 evaluation is below
    // ~1600 in magnitude (conic entries <= 1/0.3, coordinates within a tile), so P < 1e-3 and
    // exp_hat(P) < 0.978
    return __int_as_float((int)fmaf(P, FEXP_A, FEXP_B));
}

template <bool COUNT, int EXPM, int PIX>
__global__ __launch_bounds__(FastShape<PIX>::THREADS) void k_raster_fast_px(FrameDev f, WsDev ws,
                                                                         const uint32_t* __restrict__ vals) {
    using S = FastShape<PIX>;
    constexpr int WAVES = S::WAVES;
    constexpr int CAP = S::CAP;
    constexpr float SKIP = EXPM == EXP_HW2 ? -LOG2_255F : -LN255F;
    // per-wave lists of folded Gaussians, in depth order
    __shared__ float4 s_a[WAVES][CAP];               // C1, C2, C3, C4
    __shared__ float4 s_b[WAVES][CAP];               // C5, C6, r, g
    __shared__ float2 s_c[WAVES][CAP];               // b, list position (as float bits)
    __shared__ uint32_t s_cnt[WAVES][WAVES];         // [wave of the staging thread][list]
    if (blockIdx.x >= (uint32_t)f.n_tiles) return;
    const uint32_t tile = f.ordered ? ws.order[blockIdx.x] : blockIdx.x;
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64, lane = tid % 64;
    const uint32_t lx = tid % TILE, ly = PIX * (tid / TILE);
    const uint32_t px = tx * TILE + lx, py = ty * TILE + ly;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    // tile-centre coordinates
    const float ox = (float)(tx * TILE) + 7.5f, oy = (float)(ty * TILE) + 7.5f;
    const float x = (float)lx - 7.5f, y = (float)ly - 7.5f;
    const float x2 = x * x, xy = x * y, y2 = y * y;
    // the row factor 2 (y + k) + 1 of Eq. dual_pixel's step from row y + k to y + k + 1
    float yk[PIX > 1 ? PIX - 1 : 1];
#pragma unroll
    for (int k = 0; k + 1 < PIX; ++k) yk[k] = fmaf(2.0f, y + (float)k, 1.0f);

    float T[PIX], cr[PIX], cg[PIX], cb[PIX];
    uint32_t stop[PIX], nbl[PIX];
    // Whether pixel i is still blending.  Held in four scalars rather than an
    // array, so that each stays a lane mask in scalar registers (an array of
    // bools is kept as bytes in vector registers, two more VALU per pixel).
    bool live0 = px < (uint32_t)f.width && py < (uint32_t)f.height;
    bool live1 = PIX > 1 && px < (uint32_t)f.width && py + 1 < (uint32_t)f.height;
    bool live2 = PIX > 2 && px < (uint32_t)f.width && py + 2 < (uint32_t)f.height;
    bool live3 = PIX > 3 && px < (uint32_t)f.width && py + 3 < (uint32_t)f.height;
    auto live = [&](int i) -> bool& { return i == 0 ? live0 : i == 1 ? live1 : i == 2 ? live2 : live3; };
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
        T[i] = 1.0f;
        cr[i] = cg[i] = cb[i] = 0.0f;
        stop[i] = 0xffffffffu;
        nbl[i] = 0;
    }
    uint32_t steps = 0;         // counting renders: list entries this wave evaluated
    const uint64_t lt = lanemask_lt();

    for (uint32_t base = start; base < end; base += S::BATCH) {
        const bool any = live0 || live1 || live2 || live3;
        if (__syncthreads_count(any) == 0) break;
        // ---- stage: fold, cull against every wave's band, compact per wave ----
        const uint32_t idx = base + tid;
        bool hit[WAVES];
#pragma unroll
        for (int w = 0; w < WAVES; ++w) hit[w] = false;
        float4 ca = make_float4(0.f, 0.f, 0.f, 0.f), cbv = make_float4(0.f, 0.f, 0.f, 0.f);
        float cbb = 0.f;
        if (idx < end) {
            const uint32_t g = vals[idx];
            const Record rec = ws.records[g < f.n_gaussians ? g : 0u];
            const float u = (rec.u_hi - ox) + rec.u_lo;
            const float v = (rec.v_hi - oy) + rec.v_lo;
            const float A = rec.A, B = rec.B, C = rec.C;
            const float C0 = fmaf(A * u, u, fmaf(2.0f * B * u, v, C * v * v));
            ca = make_float4(-0.5f * A, -B, -0.5f * C, fmaf(A, u, B * v));
            cbv = make_float4(fmaf(C, v, B * u), fmaf(-0.5f, C0, rec.opa), rec.r, rec.g);
            cbb = rec.b;
            if (EXPM == EXP_HW2) {       // P log2 e directly: alpha = exp2 of it
                ca = make_float4(ca.x * LOG2E_F, ca.y * LOG2E_F, ca.z * LOG2E_F, ca.w * LOG2E_F);
                cbv.x *= LOG2E_F;
                cbv.y *= LOG2E_F;
            }
            // the box |x - u| <= hx, |y - v| <= hy holds every pixel with
            // P >= -ln 255 (half-extents from the front end, rounded up, then
            // widened); a band outside it has no pair that passes the skip
            // test; then the ellipse itself: the band must hold a point with
            // q <= tau = 2 (ln 255 + ln o), up to the margin.  Comparisons are
            // phrased so that a NaN keeps the Gaussian.
            const float hx = fmaf(half_lo(rec.extra), 1.0f + BOX_MARGIN_REL, BOX_MARGIN_ABS);
            const float hy = fmaf(half_hi(rec.extra), 1.0f + BOX_MARGIN_REL, BOX_MARGIN_ABS);
            const bool x_out = u - hx > 7.5f || u + hx < -7.5f;
            const float qlim = fmaf(2.0f * (LN255F + rec.opa), 1.0f + Q_MARGIN_REL, Q_MARGIN_ABS);
            // the reciprocals only place the nearest point of an edge, where q is
            // then evaluated exactly; an error of an ulp moves q by ~C (1e-6 px)^2
            const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const float y0 = (float)(w * S::ROWS) - 7.5f, y1 = y0 + (float)(S::ROWS - 1);
                hit[w] = !(x_out || v - hy > y1 || v + hy < y0);
                if (hit[w]) hit[w] = !(conic_rect_min(u, v, A, B, C, iA, iC, y0, y1) > qlim);
            }
        }
        uint64_t mk[WAVES];
#pragma unroll
        for (int w = 0; w < WAVES; ++w) mk[w] = __ballot(hit[w]);
        if (lane == 0) {
#pragma unroll
            for (int w = 0; w < WAVES; ++w) s_cnt[wave][w] = (uint32_t)__popcll(mk[w]);
        }
        __syncthreads();
        const float posf = __uint_as_float(idx);
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            if (hit[w]) {
                uint32_t p = (uint32_t)__popcll(mk[w] & lt);
                for (uint32_t sw = 0; sw < wave; ++sw) p += s_cnt[sw][w];
                s_a[w][p] = ca;
                s_b[w][p] = cbv;
                s_c[w][p] = make_float2(cbb, posf);
            }
        }
        uint32_t nl[WAVES];
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            nl[w] = 0;
#pragma unroll
            for (int sw = 0; sw < WAVES; ++sw) nl[w] += s_cnt[sw][w];
        }
        // inert padding up to a multiple of the unroll: P = -1e30 is always skipped
        if (tid < WAVES * LIST_UNROLL) {
            const uint32_t w = tid / LIST_UNROLL, k = tid % LIST_UNROLL;
            const uint32_t p = nl[w] + k;
            s_a[w][p] = make_float4(0.f, 0.f, 0.f, 0.f);
            s_b[w][p] = make_float4(0.f, -1.0e30f, 0.f, 0.f);
            s_c[w][p] = make_float2(0.f, 0.f);
        }
        __syncthreads();

        // ---- blend this wave's list ----
        // (the list length is the same for the whole wave: keep it scalar)
        const uint32_t n = __builtin_amdgcn_readfirstlane(nl[wave]);
        const float4* la = s_a[wave];
        const float4* lb = s_b[wave];
        const float2* lc = s_c[wave];
        if (__ballot(any) != 0) {
            bool wave_done = false;     // every pixel of the wave has stopped
            for (uint32_t k0 = 0; k0 < n && !wave_done; k0 += LIST_UNROLL) {
                if (COUNT) steps += LIST_UNROLL;
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    const float4 a = la[k0 + u];
                    const float4 m = lb[k0 + u];
                    const float2 c = lc[k0 + u];
                    float P[PIX];
                    P[0] = fmaf(a.x, x2, fmaf(a.y, xy, fmaf(a.z, y2, fmaf(a.w, x, fmaf(m.x, y, m.y)))));
#pragma unroll
                    for (int i = 1; i < PIX; ++i) P[i] = P[i - 1] + fmaf(a.y, x, fmaf(a.z, yk[i - 1], m.x));
                    float Tn[PIX], nr[PIX], ng[PIX], nb[PIX];
                    bool st[PIX];
                    bool any_stop = false;
#pragma unroll
                    for (int i = 0; i < PIX; ++i) {
                        // a skipped or finished pixel takes alpha = 0
                        const float al = (live(i) && P[i] >= SKIP) ? fast_alpha<EXPM>(P[i]) : 0.0f;
                        const float w = al * T[i];
                        Tn[i] = T[i] - w;
                        nr[i] = fmaf(w, m.z, cr[i]);
                        ng[i] = fmaf(w, m.w, cg[i]);
                        nb[i] = fmaf(w, c.x, cb[i]);
                        st[i] = Tn[i] < T_MIN;
                        any_stop |= st[i];
                        if (COUNT) nbl[i] += (al > 0.0f && !st[i]) ? 1u : 0u;
                    }
                    if (__ballot(any_stop) != 0) {
                        // a pixel reached the stop: that pair is not blended
                        const uint32_t at = __float_as_uint(c.y);
#pragma unroll
                        for (int i = 0; i < PIX; ++i) {
                            if (st[i]) {
                                live(i) = false;
                                stop[i] = at;
                                Tn[i] = T[i];
                                nr[i] = cr[i];
                                ng[i] = cg[i];
                                nb[i] = cb[i];
                            }
                        }
                        wave_done = __ballot(live0 || live1 || live2 || live3) == 0;
                    }
#pragma unroll
                    for (int i = 0; i < PIX; ++i) {
                        T[i] = Tn[i];
                        cr[i] = nr[i];
                        cg[i] = ng[i];
                        cb[i] = nb[i];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (COUNT && lane == 0 && steps) atomicAdd(reinterpret_cast<unsigned long long*>(&ws.header->list_steps),
                                               (unsigned long long)steps);
    const uint64_t plane = (uint64_t)f.width * f.height;
    float* __restrict__ out = ws.params->out;
    const float bg0 = ws.params->cam.bg[0], bg1 = ws.params->cam.bg[1], bg2 = ws.params->cam.bg[2];
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
        if (px < (uint32_t)f.width && py + i < (uint32_t)f.height) {
            const uint64_t o = (uint64_t)(py + i) * f.width + px;
            out[o] = fmaf(T[i], bg0, cr[i]);
            out[plane + o] = fmaf(T[i], bg1, cg[i]);
            out[2 * plane + o] = fmaf(T[i], bg2, cb[i]);
            if (COUNT) {                // the debug render's per-pixel outputs
                ws.t_final[o] = T[i];
                ws.n_proc[o] = stop[i] != 0xffffffffu ? (stop[i] - start + 1) | N_PROC_STOPPED : end - start;
                ws.n_blend[o] = nbl[i];
            }
        }
    }
}

template <int EXPM, bool TRAIN = false>
static void launch_fast_dual(hipStream_t s, const FrameDev& f, const WsDev& ws, const uint32_t* vals, bool count) {
    if (count)
        hipLaunchKernelGGL((k_raster_fast<true, EXPM, TRAIN>), dim3((uint32_t)f.n_tiles), dim3(FAST_THREADS), 0, s,
                           f, ws, vals);
    else
        hipLaunchKernelGGL((k_raster_fast<false, EXPM, TRAIN>), dim3((uint32_t)f.n_tiles), dim3(FAST_THREADS), 0, s,
                           f, ws, vals);
}

template <int EXPM, int PIX>
static void launch_fast_px(hipStream_t s, const FrameDev& f, const WsDev& ws, const uint32_t* vals, bool count) {
    const dim3 grid((uint32_t)f.n_tiles), block(FastShape<PIX>::THREADS);
    if (count)
        hipLaunchKernelGGL((k_raster_fast_px<true, EXPM, PIX>), grid, block, 0, s, f, ws, vals);
    else
        hipLaunchKernelGGL((k_raster_fast_px<false, EXPM, PIX>), grid, block, 0, s, f, ws, vals);
}

void launch_raster_fast(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count,
                        uint32_t opts) {
    const uint32_t* vals = result_in_b ? ws.vals_b : ws.vals_a;
    const bool exact = (opts & OPT_FASTEXP) != 0, single = (opts & OPT_DUALPIXEL) != 0;
    if (opts & OPT_QUAD) launch_fast_px<EXP_BITS, 4>(s, f, ws, vals, count);        // not with the two below
    else if (opts & OPT_HW_EXP2) launch_fast_dual<EXP_HW2>(s, f, ws, vals, count);  // not with the two below
    else if (!exact && !single) launch_fast_dual<EXP_BITS>(s, f, ws, vals, count);
    else if (exact && !single) launch_fast_dual<EXP_LIBM>(s, f, ws, vals, count);
    else if (!exact && single) launch_fast_px<EXP_BITS, 1>(s, f, ws, vals, count);
    else launch_fast_px<EXP_LIBM, 1>(s, f, ws, vals, count);
}

void launch_raster_train(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count) {
    launch_fast_dual<EXP_HW2, true>(s, f, ws, result_in_b ? ws.vals_b : ws.vals_a, count);
}

}  // namespace rgs
