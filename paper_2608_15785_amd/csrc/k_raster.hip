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

// ---------------------------------------------------------------------------

template <bool COUNT>
__global__ __launch_bounds__(256) void k_raster_plain(FrameDev f, WsDev ws,
                                                      const uint32_t* __restrict__ vals) {
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

void launch_raster_plain(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b,
                         bool count) {
    const uint32_t* vals = result_in_b ? ws.vals_b : ws.vals_a;
    if (count)
        hipLaunchKernelGGL(k_raster_plain<true>, dim3(xcd_grid(f.n_tiles)), dim3(256), 0, s, f, ws, vals);
    else
        hipLaunchKernelGGL(k_raster_plain<false>, dim3(xcd_grid(f.n_tiles)), dim3(256), 0, s, f, ws, vals);
}

// ---------------------------------------------------------------------------
// Fast rasterizer.
//
// Every wave of a tile's workgroup owns a band of rows and works through the
// tile's list on its own (no workgroup barrier): it stages 64 entries at a
// time (one per lane), folds each (Eqs. expand, c0, coeff), culls it against
// its band, and compacts the survivors in depth order into its own LDS list.
// The 64 lanes of a wave form four row groups of 16 columns; group j owns PIX
// consecutive rows starting at y_j and each lane PIX pixels of one column
// (PIX = 2 is Eq. dual_pixel; 1 is its ablation, 4 extends it along the
// column).  At staging the folded exponent is reduced further to each row
// group: with E_j = C2 y_j + C4 and F_j = (C3 y_j + C5) y_j + C6,
//     P(x, y_j) = C1 x^2 + E_j x + F_j                       (Eq. dot)
//     P(x, y + 1) = P(x, y) + C2 x + G(y),  G(y) = C3 (2y + 1) + C5
//                                                            (Eq. dual_pixel)
// so a lane's first pixel costs two FMAs and each further pixel an FMA and an
// add; every lane reads its group's (E, F, G) and the shared (C1, C2, colour)
// with two LDS broadcasts.
//
// The blend of a batch runs without the per-pair stop test: a pixel passing
// the skip test takes alpha, its weight alpha T, the new T and the colour in
// place, only in the lanes that pass (exec-masked).  Transmittance never
// grows, so a pixel whose T is still >= 1e-4 at the end of the batch never met
// the stop condition inside it.  If any pixel of the wave ends the batch below
// 1e-4, the wave restores the state it saved at the start of the batch and
// blends the batch again with the stop test at every pair (careful mode): the
// same operations in the same order, so both modes give the same bits.
// Counting (debug) renders always take careful mode.

constexpr int FAST_BATCH = 64;               // entries a wave stages at once, one per lane
constexpr int LIST_UNROLL = 4;
constexpr int LIST_CAP = FAST_BATCH + LIST_UNROLL;
// Margin added to the alpha-ellipse half-extents before culling a Gaussian for
// a wave: float32 rounding of the folded exponent near the 1/255 threshold
// must never hide a pair that the exact test would keep.
constexpr float BOX_MARGIN_REL = 1.0e-3f;
constexpr float BOX_MARGIN_ABS = 0.05f;
// The same safety margin on the quadratic form q = A dx^2 + 2 B dx dy + C dy^2
// (P = ln o - q / 2): a band is kept when min q <= tau (1 + 1e-3) + 0.02.
constexpr float Q_MARGIN_REL = 1.0e-3f;
constexpr float Q_MARGIN_ABS = 0.02f;

template <int PIX>
struct FastShape {
    static constexpr int ROWS = 4 * PIX;            // rows of a wave's band
    static constexpr int WAVES = TILE / ROWS;       // waves per tile
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int NG = PIX > 1 ? PIX - 1 : 1;   // row increments G per row group
    // LDS per list entry: shared float4, per-group float4 (E, F, G_0, b), per-group extra G's
    static constexpr int EXTRA = PIX > 2 ? 1 : 0;
};

// Smallest q over the rectangle [-7.5, 7.5] x [y0, y1] (tile-centre
// coordinates) for a Gaussian at (u, v) with a positive-definite conic: 0 when
// the mean is inside, else the least of the four edge minima (on an edge q is
// a parabola in the free coordinate, minimised at a clamped closed form).
__device__ inline float conic_rect_min(float u, float v, float A, float B, float C, float iA, float iC,
                                       float y0, float y1) {
    if (u >= -7.5f && u <= 7.5f && v >= y0 && v <= y1) return 0.0f;
    float best = 3.0e38f;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = (e ? 7.5f : -7.5f) - u;                 // vertical edge x = -7.5 or 7.5
        const float dy = fminf(y1, fmaxf(y0, fmaf(-B * dx, iC, v))) - v;
        best = fminf(best, fmaf(A * dx, dx, fmaf(2.0f * B * dx, dy, C * dy * dy)));
        const float ey = (e ? y1 : y0) - v;                       // horizontal edge y = y0 or y1
        const float ex = fminf(7.5f, fmaxf(-7.5f, fmaf(-B * ey, iA, u))) - u;
        best = fminf(best, fmaf(A * ex, ex, fmaf(2.0f * B * ex, ey, C * ey * ey)));
    }
    return best;
}

// How the fast rasterizer takes alpha from the folded exponent P.
enum ExpMode : int {
    EXP_BITS = 0,   // Eq. fma_exp: the bit-level exponential (the paper's fast path)
    EXP_LIBM = 1,   // min(0.99, expf(P)): the exponential's ablation
    EXP_HW2 = 2,    // min(0.99, v_exp_f32(P log2 e)) with log2 e folded into C1..C6
};
constexpr float LOG2E_F = 1.4426950408889634f;
constexpr float LOG2_255F = 7.994353436858858f;     // ln 255 * log2 e

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
__global__ __launch_bounds__(FastShape<PIX>::THREADS) void k_raster_fast(FrameDev f, WsDev ws,
                                                                         const uint32_t* __restrict__ vals) {
    using S = FastShape<PIX>;
    constexpr float SKIP = EXPM == EXP_HW2 ? -LOG2_255F : -LN255F;
    // per-wave lists of folded Gaussians, in depth order
    __shared__ float4 s_sh[S::WAVES][LIST_CAP];            // C1, C2, r, g
    __shared__ float4 s_rg[S::WAVES][LIST_CAP][4];         // E_j, F_j, G_j0, b   (row group j)
    __shared__ float4 s_rx[S::WAVES][S::EXTRA ? LIST_CAP : 1][4];   // G_j1, G_j2 (PIX = 4)
    __shared__ uint32_t s_pos[S::WAVES][LIST_CAP];         // list position of the entry
    const uint32_t tile = xcd_tile(blockIdx.x, (uint32_t)f.n_tiles);
    if (tile >= (uint32_t)f.n_tiles) return;
    const uint32_t tx = tile % (uint32_t)f.tiles_x, ty = tile / (uint32_t)f.tiles_x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    const uint32_t grp = lane / 16;
    const uint32_t lx = lane % 16, ly = wave * S::ROWS + grp * PIX;
    const uint32_t px = tx * TILE + lx, py = ty * TILE + ly;
    const uint32_t start = ws.ranges[2 * tile], end = ws.ranges[2 * tile + 1];
    // tile-centre coordinates
    const float ox = (float)(tx * TILE) + 7.5f, oy = (float)(ty * TILE) + 7.5f;
    const float x = (float)lx - 7.5f, x2 = x * x;
    const float band_lo = (float)(wave * S::ROWS) - 7.5f, band_hi = band_lo + (float)(S::ROWS - 1);

    float T[PIX], cr[PIX], cg[PIX], cb[PIX];
    bool live[PIX];
    uint32_t stop[PIX], nbl[PIX];
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
        T[i] = 1.0f;
        cr[i] = cg[i] = cb[i] = 0.0f;
        live[i] = px < (uint32_t)f.width && py + i < (uint32_t)f.height;
        stop[i] = 0xffffffffu;
        nbl[i] = 0;
    }
    const uint64_t lt = lanemask_lt();
    // LDS addresses through the per-lane wave index: the list reads of the
    // blend then take their address from a VGPR that advances once per
    // unrolled step, not from a scalar copied into a VGPR at every read
    const uint32_t wave_v = tid / 64;
    float4* lsh = s_sh[wave_v];
    uint32_t* lpos = s_pos[wave_v];

    for (uint32_t base = start; base < end; base += FAST_BATCH) {
        bool any = false;
#pragma unroll
        for (int i = 0; i < PIX; ++i) any |= live[i];
        if (__ballot(any) == 0) break;
        // ---- stage: fold, cull against this wave's band, compact ----
        const uint32_t idx = base + lane;
        bool hit = false;
        float C1 = 0.f, C2 = 0.f, C3 = 0.f, C4 = 0.f, C5 = 0.f, C6 = 0.f, rr = 0.f, rg = 0.f, rb = 0.f;
        if (idx < end) {
            const uint32_t g = vals[idx];
            const Record rec = ws.records[g < f.n_gaussians ? g : 0u];
            const float u = (rec.u_hi - ox) + rec.u_lo;
            const float v = (rec.v_hi - oy) + rec.v_lo;
            const float A = rec.A, B = rec.B, C = rec.C;
            const float C0 = fmaf(A * u, u, fmaf(2.0f * B * u, v, C * v * v));
            C1 = -0.5f * A;
            C2 = -B;
            C3 = -0.5f * C;
            C4 = fmaf(A, u, B * v);
            C5 = fmaf(C, v, B * u);
            C6 = fmaf(-0.5f, C0, rec.opa);
            if (EXPM == EXP_HW2) {       // P log2 e directly: alpha = exp2 of it
                C1 *= LOG2E_F;
                C2 *= LOG2E_F;
                C3 *= LOG2E_F;
                C4 *= LOG2E_F;
                C5 *= LOG2E_F;
                C6 *= LOG2E_F;
            }
            rr = rec.r;
            rg = rec.g;
            rb = rec.b;
            // the box |x - u| <= hx, |y - v| <= hy holds every pixel with
            // P >= -ln 255 (half-extents from the front end, rounded up, then
            // widened); a band outside it has no pair that passes the skip
            // test; then the ellipse itself: the band must hold a point with
            // q <= tau = 2 (ln 255 + ln o), up to the margin.  Comparisons are
            // phrased so that a NaN keeps the Gaussian.
            const float hx = fmaf(half_lo(rec.extra), 1.0f + BOX_MARGIN_REL, BOX_MARGIN_ABS);
            const float hy = fmaf(half_hi(rec.extra), 1.0f + BOX_MARGIN_REL, BOX_MARGIN_ABS);
            hit = !(u - hx > 7.5f || u + hx < -7.5f || v - hy > band_hi || v + hy < band_lo);
            if (hit) {
                const float qlim = fmaf(2.0f * (LN255F + rec.opa), 1.0f + Q_MARGIN_REL, Q_MARGIN_ABS);
                // the reciprocals only place the nearest point of an edge, where q is
                // then evaluated exactly; an error of an ulp moves q by ~C (1e-6 px)^2
                const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
                hit = !(conic_rect_min(u, v, A, B, C, iA, iC, band_lo, band_hi) > qlim);
            }
        }
        const uint64_t m = __ballot(hit);
        const uint32_t n = (uint32_t)__popcll(m);
        if (hit) {
            const uint32_t p = (uint32_t)__popcll(m & lt);
            lsh[p] = make_float4(C1, C2, rr, rg);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float y = band_lo + (float)(j * PIX);
                const float E = fmaf(C2, y, C4);
                const float F = fmaf(fmaf(C3, y, C5), y, C6);
                const float G0 = fmaf(C3, fmaf(2.0f, y, 1.0f), C5);
                s_rg[wave_v][p][j] = make_float4(E, F, G0, rb);
                if (S::EXTRA) {
                    const float G1 = fmaf(C3, fmaf(2.0f, y + 1.0f, 1.0f), C5);
                    const float G2 = fmaf(C3, fmaf(2.0f, y + 2.0f, 1.0f), C5);
                    s_rx[wave_v][S::EXTRA ? p : 0][j] = make_float4(G1, G2, 0.f, 0.f);
                }
            }
            lpos[p] = idx;
        }
        // inert padding up to a multiple of the unroll: P = -1e30 is always skipped
        if (lane < LIST_UNROLL) {
            const uint32_t p = n + lane;
            lsh[p] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s_rg[wave_v][p][j] = make_float4(0.f, -1.0e30f, 0.f, 0.f);
                if (S::EXTRA) s_rx[wave_v][S::EXTRA ? p : 0][j] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            lpos[p] = 0;
        }
        // the list is read by other lanes of this wave: the wave's LDS
        // accesses complete in program order, so a compiler barrier suffices
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const float4* lrg = &s_rg[wave_v][0][grp];
        const float4* lrx = &s_rx[wave_v][0][grp];
        // the exponents of this lane's pixels for list entry k
        auto exponents = [&](uint32_t k, float (&P)[PIX], float4& sh, float4& q) {
            sh = lsh[k];
            q = lrg[4 * k];
            P[0] = fmaf(sh.x, x2, fmaf(q.x, x, q.y));
            if (PIX > 1) P[1] = P[0] + fmaf(sh.y, x, q.z);
            if (PIX > 2) {
                const float4 q2 = lrx[S::EXTRA ? 4 * k : 0];
                P[2] = P[1] + fmaf(sh.y, x, q2.x);
                P[3] = P[2] + fmaf(sh.y, x, q2.y);
            }
        };
        bool careful = COUNT;
        float Ts[PIX], rs[PIX], gs[PIX], bs[PIX];
        if (!COUNT) {
#pragma unroll
            for (int i = 0; i < PIX; ++i) {
                Ts[i] = T[i];
                rs[i] = cr[i];
                gs[i] = cg[i];
                bs[i] = cb[i];
            }
            for (uint32_t k0 = 0; k0 < n; k0 += LIST_UNROLL) {
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    float P[PIX];
                    float4 sh, q;
                    exponents(k0 + u, P, sh, q);
#pragma unroll
                    for (int i = 0; i < PIX; ++i) {
                        if (live[i] && P[i] >= SKIP) {
                            const float w = fast_alpha<EXPM>(P[i]) * T[i];
                            T[i] = T[i] - w;
                            cr[i] = fmaf(w, sh.z, cr[i]);
                            cg[i] = fmaf(w, sh.w, cg[i]);
                            cb[i] = fmaf(w, q.w, cb[i]);
                        }
                    }
                }
            }
            bool below = false;
#pragma unroll
            for (int i = 0; i < PIX; ++i) below |= T[i] < T_MIN;
            careful = __ballot(below) != 0;
            if (careful) {
                // a pixel met the stop condition in this batch: start it again
#pragma unroll
                for (int i = 0; i < PIX; ++i) {
                    T[i] = Ts[i];
                    cr[i] = rs[i];
                    cg[i] = gs[i];
                    cb[i] = bs[i];
                }
            }
        }
        if (careful) {
            for (uint32_t k0 = 0; k0 < n; k0 += LIST_UNROLL) {
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) {
                    float P[PIX];
                    float4 sh, q;
                    exponents(k0 + u, P, sh, q);
#pragma unroll
                    for (int i = 0; i < PIX; ++i) {
                        if (live[i] && P[i] >= SKIP) {
                            const float w = fast_alpha<EXPM>(P[i]) * T[i];
                            const float Tn = T[i] - w;
                            if (Tn < T_MIN) {
                                // the pixel stops here: this pair is not blended
                                live[i] = false;
                                stop[i] = lpos[k0 + u];
                            } else {
                                T[i] = Tn;
                                cr[i] = fmaf(w, sh.z, cr[i]);
                                cg[i] = fmaf(w, sh.w, cg[i]);
                                cb[i] = fmaf(w, q.w, cb[i]);
                                if (COUNT) ++nbl[i];
                            }
                        }
                    }
                }
                bool any2 = false;
#pragma unroll
                for (int i = 0; i < PIX; ++i) any2 |= live[i];
                if (__ballot(any2) == 0) break;
            }
        }
        // the next batch overwrites the list: this wave's reads come first
        __builtin_amdgcn_wave_barrier();
    }
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

template <int EXPM, int PIX>
static void launch_fast(hipStream_t s, const FrameDev& f, const WsDev& ws, const uint32_t* vals, bool count) {
    const dim3 grid(xcd_grid(f.n_tiles)), block(FastShape<PIX>::THREADS);
    if (count)
        hipLaunchKernelGGL((k_raster_fast<true, EXPM, PIX>), grid, block, 0, s, f, ws, vals);
    else
        hipLaunchKernelGGL((k_raster_fast<false, EXPM, PIX>), grid, block, 0, s, f, ws, vals);
}

void launch_raster_fast(hipStream_t s, const FrameDev& f, const WsDev& ws, bool result_in_b, bool count,
                        uint32_t opts) {
    const uint32_t* vals = result_in_b ? ws.vals_b : ws.vals_a;
    const bool exact = (opts & OPT_FASTEXP) != 0, single = (opts & OPT_DUALPIXEL) != 0;
    if (opts & OPT_QUAD) {                       // not with the two above or the hardware exp2
        launch_fast<EXP_BITS, 4>(s, f, ws, vals, count);
    } else if (opts & OPT_HW_EXP2) {             // not with the two above
        launch_fast<EXP_HW2, 2>(s, f, ws, vals, count);
    } else if (!exact && !single) {
        launch_fast<EXP_BITS, 2>(s, f, ws, vals, count);
    } else if (exact && !single) {
        launch_fast<EXP_LIBM, 2>(s, f, ws, vals, count);
    } else if (!exact && single) {
        launch_fast<EXP_BITS, 1>(s, f, ws, vals, count);
    } else {
        launch_fast<EXP_LIBM, 1>(s, f, ws, vals, count);
    }
}

}  // namespace rgs
