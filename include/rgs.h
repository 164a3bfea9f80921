/*
 * rgs.h - C ABI of an MI355X (gfx950) tile-based 3D Gaussian Splatting renderer.
 *
 * The library renders one image of a scene of N 3D Gaussians (mean, rotation,
 * scale, opacity, degree-3 spherical-harmonic colour) seen by a pinhole camera,
 * with the tile-based forward pipeline of 3D Gaussian Splatting as analysed and
 * accelerated in "RoofGS: Roofline-Guided End-to-End Acceleration of 3D
 * Gaussian Splatting" (Sec. II-A, III, IV):
 *   preprocess (EWA projection, frustum/opacity culling, SH colour)
 *   -> duplicate one (key, index) entry per covered 16x16 tile
 *   -> radix sort on the key -> per-tile ranges -> per-tile alpha blending.
 *
 * Two paths render the same image definition:
 *   RGS_PATH_PLAIN  the 3DGS baseline: FP32 attributes, 64-bit (tile | FP32
 *                   depth) key, exact exponential, one pixel per thread.
 *   RGS_PATH_FAST   the paper's optimisations: INT8 SH with per-degree,
 *                   per-channel scales and FP16 rotation/scale/opacity
 *                   (Sec. IV-A, Eq. quant); 32-bit (tile | quantised depth)
 *                   key with a resolution-adaptive bit split (Eq. depth_quant);
 *                   preprocess, duplication and key generation fused in one
 *                   kernel with opacity culling; coefficient folding,
 *                   dual-pixel evaluation and the bit-level exponential in the
 *                   rasterizer (Sec. IV-B, Eqs. coeff, dot, dual_pixel, fma_exp).
 *
 * Conventions shared by every call:
 *   - every call returns an rgs_status; outputs are written only on RGS_OK;
 *     nothing throws or aborts across the ABI; rgs_last_error() gives a
 *     message for the calling thread's last failure;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory of the context's device;
 *   - GPU work is enqueued on the context's stream (a hipStream_t passed as
 *     void*; NULL means the default stream) and is asynchronous unless a
 *     call says it synchronises;
 *   - camera space is OpenCV-like (x right, y down, z forward); pixel (i, j)
 *     is sampled at image-plane position (i, j); images are float32 planar
 *     [3][H][W].
 */
#ifndef RGS_H
#define RGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rgs_status;
#define RGS_OK            0
#define RGS_E_INVALID    -1   /* bad argument; nothing was enqueued                        */
#define RGS_E_OOM        -2   /* device or host allocation failed                          */
#define RGS_E_HIP        -3   /* a HIP runtime call failed                                 */
#define RGS_E_CAPACITY   -4   /* more duplicated entries than the workspace holds          */
#define RGS_E_NODEVICE   -5   /* no usable GPU                                             */
#define RGS_E_UNSUPPORTED -6  /* entry point or option not available in this library       */
#define RGS_E_DEVICE     -7   /* a kernel reported an internal failure (bounded wait hit)  */

#define RGS_ABI_VERSION 2

#define RGS_FMT_PLAIN 1u      /* FP32 structure-of-arrays, 240 bytes per Gaussian (the
                                 plain path reads 236 of them; ln o is kept for ablations)   */
#define RGS_FMT_FAST  2u      /* compact structure-of-arrays, 100 bytes per Gaussian       */

#define RGS_PATH_PLAIN 0
#define RGS_PATH_FAST  1

/* Ablations of the fast path: each bit, OR-ed into a `path` argument together
 * with RGS_PATH_FAST, removes one of the paper's optimisations (Sec. IV) and
 * keeps the rest, for the per-step study of what each contributes.  The image
 * definition of every combination is the oracle's fast path with the matching
 * step removed. */
#define RGS_ABLATE_FASTEXP   (1 << 8)   /* alpha = min(0.99, exp(P)) instead of Eq. fma_exp        */
#define RGS_ABLATE_DUALPIXEL (1 << 9)   /* one pixel per thread instead of Eq. dual_pixel          */
#define RGS_ABLATE_FUSION    (1 << 10)  /* separate preprocess and duplication kernels             */
#define RGS_ABLATE_EXTENT    (1 << 11)  /* 3-sigma tile extent, no opacity cull                     */
#define RGS_ABLATE_KEY32     (1 << 12)  /* 64-bit (tile | FP32 depth) key of the plain path        */
#define RGS_ABLATE_INT8_SH   (1 << 13)  /* FP32 SH from the plain format (the scene needs both)    */
#define RGS_ABLATE_FP16_GEOM (1 << 14)  /* FP32 rotation, scale and ln o from the plain format     */
#define RGS_ABLATE_MASK      (0x7f << 8)

/* Extension of the fast path, OR-ed into a `path` argument like the ablation
 * bits: the exact ellipse-tile test.  Of each rectangle of at most 64 tiles it
 * keeps only the tiles whose box of pixel centres meets the ellipse where
 * alpha >= 1/255 (the tile-precise half of the Speedy-Splat culling that
 * Sec. IV-A adopts; the default fast path keeps the whole alpha-ellipse box).
 * The image is the same; the entries are fewer.  Not valid with
 * RGS_ABLATE_EXTENT or RGS_PATH_PLAIN. */
#define RGS_EXACT_TILES      (1 << 15)
/* Extension of the fast path: alpha = min(0.99, exp2(P log2 e)) by gfx950's
 * hardware exp2 instruction, with log2 e folded into the coefficients of
 * Eq. coeff, instead of the bit-level exponential of Eq. fma_exp (Sec. IV-B).
 * The image is that of the exact exponential to within the instruction's
 * 1-ulp error.  Not valid with RGS_ABLATE_FASTEXP or RGS_ABLATE_DUALPIXEL.
 * With RGS_PATH_PLAIN (and no other bit) it selects the plain path's training
 * variant: the plain front end, keys and sort (entries identical to the plain
 * path's), then the fast path's dual-pixel rasterizer with per-wave culled
 * lists over the plain path's float32 records: the exponent folded per
 * Eqs. expand, c0, coeff, dot, dual_pixel in tile-centre coordinates, and
 * alpha = min(0.99, exp2(P log2 e)) by the hardware exp2.  rgs_render_backward
 * replays the same lists with the same folding, so it recomputes the forward
 * pass's alpha bit for bit.  The image definition stays the plain one (exact
 * exponential, no quantisation); only float32 rounding differs. */
#define RGS_HW_EXP2          (1 << 16)
/* Extension of the fast path: four pixels per lane instead of two.  Eq.
 * dual_pixel is applied along the column three times, P(x, y + 1) =
 * P(x, y) + C2 x + C3 (2y + 1) + C5, so a wave of 64 lanes covers a whole
 * 16x16 tile and culls the tile's list against the tile instead of against
 * half-tiles (Sec. IV-B).  Same image definition as RGS_PATH_FAST.  Not valid
 * with RGS_ABLATE_FASTEXP, RGS_ABLATE_DUALPIXEL or RGS_HW_EXP2. */
#define RGS_QUAD_PIXEL       (1 << 17)

#define RGS_TILE 16
#define RGS_MAX_DIM 16384     /* largest accepted image width or height                    */
#define RGS_MAX_ENTRIES ((1ull << 30) - 1) /* largest entry capacity of one frame        */

/* Stages timed when a context has timing switched on (rgs_ctx_set_timing). */
#define RGS_STAGE_FRONTEND  0 /* plain: preprocess; fast: fused front end                  */
#define RGS_STAGE_DUPLICATE 1 /* plain: ordered duplication with keys; fast: unused (0)    */
#define RGS_STAGE_SORT      2 /* digit histogram + radix passes                            */
#define RGS_STAGE_RANGES    3 /* per-tile ranges                                           */
#define RGS_STAGE_RASTER    4 /* per-tile blending                                         */
#define RGS_N_STAGES        5

typedef struct rgs_ctx rgs_ctx;
typedef struct rgs_scene rgs_scene;

/* ABI version of the loaded library (RGS_ABI_VERSION of its build). */
int32_t rgs_abi_version(void);

/* Message of the calling thread's last failed call ("" if none).  The string
 * stays valid until that thread's next call into the library. */
const char* rgs_last_error(void);

/* Static name of a status code. */
const char* rgs_status_string(rgs_status s);

/* ---------------------------------------------------------------------------
 * Frame plan (host-only arithmetic, usable without a GPU).
 * Sec. IV-A, "Resolution-Adaptive Sorting-Key Encoding": N_t = T_x T_y tiles of
 * 16x16 pixels; the 32-bit key gives the tile index b_t = max(1, ceil(log2 N_t))
 * high bits and the quantised depth the b_d = 32 - b_t low bits.  The plain
 * 64-bit key has 32 + b_t significant bits.
 */
typedef struct {
    int32_t width, height;
    int32_t tiles_x, tiles_y, n_tiles;
    int32_t b_t, b_d;
    int32_t plain_key_bits;   /* 32 + b_t                                      */
    int32_t plain_passes;     /* ceil(plain_key_bits / 8) radix passes         */
    int32_t fast_passes;      /* 4 radix passes of the 32-bit key              */
} rgs_plan;

/* W, H in [1, RGS_MAX_DIM]; otherwise RGS_E_INVALID. */
rgs_status rgs_frame_plan(int32_t width, int32_t height, rgs_plan* out);

/* ---------------------------------------------------------------------------
 * Context: one device and one stream.  Create one per host thread.
 */
/* device: HIP ordinal; hip_stream: hipStream_t or NULL.  RGS_E_NODEVICE when
 * no GPU is present (safe to call on a machine without one). */
rgs_status rgs_ctx_create(int32_t device, void* hip_stream, rgs_ctx** out);
/* Releases the context (scenes must be released first).  NULL is a no-op. */
void rgs_ctx_destroy(rgs_ctx* ctx);
/* Re-targets later work to another stream of the same device. */
rgs_status rgs_ctx_set_stream(rgs_ctx* ctx, void* hip_stream);
/* Debug flags of a context's renders (0: none).  RGS_DEBUG_SORT_FALLBACK: every
 * radix tile of the sort takes the digit counts of its predecessors from their
 * keys, the path a tile takes when a predecessor's counts are not published in
 * time, so that tests can check it gives the same order.  Errors: INVALID
 * (NULL, unknown flag). */
#define RGS_DEBUG_SORT_FALLBACK 1u
rgs_status rgs_ctx_set_debug(rgs_ctx* ctx, uint32_t flags);
/* enable != 0: record HIP events around each stage of every render on the
 * context's stream.  Switching it on clears the accumulated times. */
rgs_status rgs_ctx_set_timing(rgs_ctx* ctx, int32_t enable);
/* Synchronises the stream, then returns per-stage time summed over the
 * renders recorded since timing was switched on (stage_ms[RGS_N_STAGES], ms)
 * and the number of renders.  Clears the accumulators. */
rgs_status rgs_ctx_collect_timing(rgs_ctx* ctx, double* stage_ms, int64_t* n_frames);

/* Roofline calibration probe (Sec. III measures each stage against the
 * chip's peaks).  Enqueues one kernel of `blocks` workgroups of 256 threads;
 * every wave issues exactly 8 * iters float32 FMA instructions in its main
 * loop (plus at most a few dozen other VALU instructions) with eight
 * independent chains per lane, and each thread writes one float to out.
 * Profiled together with its duration, its VALU-instruction and busy-cycle
 * counters calibrate those of the rasterizers.  out: device, blocks * 256
 * floats, caller-owned.  Asynchronous.  Errors: INVALID (NULL, blocks outside
 * [1, 2^20], iters < 0), HIP. */
rgs_status rgs_probe_valu(rgs_ctx* ctx, int32_t blocks, int32_t iters, float* out);

/* ---------------------------------------------------------------------------
 * Scene upload (once per scene, not per frame).
 * Inputs are the activated parameters a trained 3DGS scene holds, all host
 * float32, row-major; the library copies them and keeps its own device
 * copies (structure-of-arrays, one plane per scalar attribute).
 */
typedef struct {
    int64_t n;                /* number of Gaussians, >= 1                              */
    int32_t sh_degree;        /* must be 3 (16 coefficients per channel)                */
    int32_t reserved;         /* 0                                                      */
    const float* means;       /* host [n][3]                                            */
    const float* scales;      /* host [n][3], > 0 (already exp-activated)               */
    const float* quats;       /* host [n][4] as (w, x, y, z), not all zero              */
    const float* opacity;     /* host [n], in (0, 1] (already sigmoid-activated)        */
    const float* sh;          /* host [n][16][3], coefficient l*l+l+m then RGB channel  */
} rgs_scene_desc;

/* formats: RGS_FMT_PLAIN and/or RGS_FMT_FAST.  The fast format is built on
 * the host in float64 (Sec. IV-A, Eq. quant; see rgs_quantize_host) and then
 * copied.  Synchronous.  Errors: RGS_E_INVALID for a non-finite value, a
 * non-positive scale, a zero quaternion, opacity outside (0, 1], n < 1, a
 * degree other than 3, or an SH block whose FP16 scale would overflow;
 * RGS_E_OOM. */
rgs_status rgs_scene_upload(rgs_ctx* ctx, const rgs_scene_desc* desc, uint32_t formats,
                            rgs_scene** out);
/* Frees the scene's device memory.  NULL is a no-op. */
rgs_status rgs_scene_release(rgs_ctx* ctx, rgs_scene* scene);
/* Number of Gaussians, formats held, and device bytes held by the scene. */
rgs_status rgs_scene_info(const rgs_scene* scene, int64_t* n, uint32_t* formats,
                          uint64_t* device_bytes);

/* Compact storage of Sec. IV-A computed on the host (usable without a GPU):
 *   quats_f16  [n][4]     FP16 bits, round-to-nearest-even of the FP32 input
 *   scales_f16 [n][3]     FP16 bits
 *   lnopa_f16  [n]        FP16 bits of ln(opacity) evaluated in float64
 *   sh_q       [n][16][3] INT8, clamp(rint(sh / s), -127, 127), 0 when s = 0
 *   sh_scale_f16 [n][4][3] FP16 bits of s = max |sh| / 127 over the coefficients
 *                          of each degree, per Gaussian and channel (round to
 *                          nearest even); q is taken against the stored s.
 * All output arrays are caller-owned host memory. */
typedef struct {
    uint16_t* quats_f16;
    uint16_t* scales_f16;
    uint16_t* lnopa_f16;
    int8_t* sh_q;
    uint16_t* sh_scale_f16;
} rgs_fast_host;
rgs_status rgs_quantize_host(const rgs_scene_desc* desc, rgs_fast_host* out);

/* ---------------------------------------------------------------------------
 * Camera.  A world point p maps to camera space as R p + t (R row-major).
 * fx, fy, cx, cy are pinhole intrinsics in pixels; tan_half_fov{x,y} bound the
 * EWA Jacobian (3DGS clamps t_x/t_z to 1.3 tan(fovx/2)); [z_near, z_far] is
 * the predefined depth interval: Gaussians outside (z_near, z_far] are culled
 * and the fast key quantises depth over it (Eq. depth_quant).  bg is the
 * background colour added with the final transmittance.
 */
typedef struct {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double tan_half_fovx, tan_half_fovy;
    double z_near, z_far;
    float bg[3];
    float reserved;
} rgs_camera;

/* Per-frame statistics, filled when a non-NULL pointer is passed to render. */
typedef struct {
    int64_t n_gaussians;
    int64_t n_visible;        /* Gaussians that survived culling                          */
    int64_t n_entries;        /* duplicated (key, index) entries requested                */
    int64_t capacity;         /* entries the workspace holds                              */
    int32_t path;
    int32_t passes;           /* radix passes run                                         */
    int32_t overflow;         /* n_entries > capacity                                     */
    int32_t device_error;     /* bits 0, 2: a bounded wait in a kernel gave up, or a sorted
                                 key named no tile; bit 3: a backward pass found another
                                 frame in the workspace than its caller's                  */
    int64_t list_steps;       /* fast path, counting renders (rgs_render_debug) only: list
                                 entries the rasterizer's waves evaluated, each for all of
                                 the wave's pixels (64 lanes x pixels per lane); else 0      */
} rgs_frame_stats;

/* ---------------------------------------------------------------------------
 * Workspace: caller-owned device memory that holds one frame's transients
 * (per-Gaussian records, keys and indices, sort state, tile ranges, per-pixel
 * final transmittance and pair counts).  Its size depends on N, W, H, the path
 * and the entry capacity; render derives the capacity back from ws_bytes.
 * Host-only arithmetic.  max_entries in [1, RGS_MAX_ENTRIES].
 */
rgs_status rgs_workspace_size(int64_t n_gaussians, int32_t width, int32_t height, int32_t path,
                              int64_t max_entries, uint64_t* bytes);
/* Entry capacity a workspace of ws_bytes provides (0 if too small). */
rgs_status rgs_workspace_capacity(int64_t n_gaussians, int32_t width, int32_t height,
                                  int32_t path, uint64_t ws_bytes, int64_t* capacity);
/* The same sizing by a scene: the workspace bytes a render of `scene` at
 * width x height on `path` needs to hold hint_ndup duplicated entries
 * (hint_ndup = 0: 4 per Gaussian, at least 65536, at most RGS_MAX_ENTRIES).
 * The true count is known only after the front end has run; a render that
 * needs more reports RGS_E_CAPACITY with the count in its stats.  Host-only.
 * Errors: INVALID (NULL, bad size or path, hint_ndup > RGS_MAX_ENTRIES). */
rgs_status rgs_render_workspace_bound(const rgs_scene* scene, int32_t width, int32_t height, int32_t path,
                                      uint64_t hint_ndup, uint64_t* bytes);
/* Device bytes the scene holds (rgs_scene_info's third output).  Host-only.
 * Errors: INVALID (NULL). */
rgs_status rgs_scene_device_bytes(const rgs_scene* scene, uint64_t* bytes);

/* ---------------------------------------------------------------------------
 * Render one image (Sec. II-A, III, IV).
 *   workspace  device, >= rgs_workspace_size(..., 1) bytes, 256-byte aligned,
 *              not used by another render until this one has finished
 *   out_chw    device float32 [3][H][W], caller-owned
 *   stats      NULL: fully asynchronous.  Non-NULL: synchronises the stream,
 *              fills *stats and returns RGS_E_CAPACITY when the frame needed
 *              more entries than the workspace holds (the image is then
 *              incomplete; retry with a larger workspace) or RGS_E_DEVICE.
 * Without stats an overflow is still recorded in the workspace and reported by
 * rgs_workspace_check.  Kernels never write past the workspace or the image.
 * Errors: RGS_E_INVALID (W or H outside [1, RGS_MAX_DIM], z_near <= 0,
 * z_near >= z_far, non-finite camera values, path not held by the scene,
 * workspace too small or misaligned), RGS_E_HIP.
 */
rgs_status rgs_render(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                      int32_t width, int32_t height, int32_t path,
                      void* workspace, uint64_t ws_bytes, float* out_chw,
                      rgs_frame_stats* stats);

/* Allocation-free render, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  As rgs_render, but the frame's workspace is the library's own
 * static device array of RGS_STATIC_WORKSPACE_BYTES, one per device, held
 * from the first rgs_ctx_create on that device until the process ends; the
 * call allocates nothing (no hipMalloc, no events even when the context times
 * stages).  The caller still passes the scene and the output image.  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (another thread, context or stream) race and must be serialised by
 * the caller; each frame clears what it needs at its start.  The entry
 * capacity is what fits in the array (about 2.4M entries at 1M Gaussians and
 * 1920x1080 on the fast path).
 * Errors: as rgs_render; RGS_E_INVALID also when the frame's fixed part
 * (records, tile ranges, per-pixel buffers) does not fit the array, and
 * RGS_E_CAPACITY (with stats) when its entries do not. */
#define RGS_STATIC_WORKSPACE_BYTES (128ull << 20)
rgs_status rgs_render_static(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                             int32_t width, int32_t height, int32_t path, float* out_chw,
                             rgs_frame_stats* stats);

/* Synchronises the stream and reports the last frame rendered into the
 * workspace (its header sits at offset 0): RGS_E_CAPACITY on overflow,
 * RGS_E_DEVICE on a kernel failure.  stats may be NULL; n_gaussians only fills
 * stats->n_gaussians. */
rgs_status rgs_workspace_check(rgs_ctx* ctx, const void* workspace, rgs_frame_stats* stats,
                               int64_t n_gaussians);

/* ---------------------------------------------------------------------------
 * Parity access: render as rgs_render, then copy the frame's intermediates
 * into caller-owned device buffers (any pointer may be NULL).  Synchronous.
 * They are the outputs of each step of the pipeline: the preprocessing of
 * Sec. III-A (EWA projection of Sec. II-A, culling, the tile extent of
 * Sec. IV-A, the SH colour), the duplication and keys of Sec. III-B (the key
 * encoding of Sec. IV-A, Eq. depth_quant), the sort of Sec. III-C, and the
 * per-pixel outcome of the blending of Sec. III-D (Eq. alpha_computation).
 *   per Gaussian [n]:  depth, u, v (float64); cov2d [n][3] (Sigma'_00,
 *                      Sigma'_01, Sigma'_11, float64); rect [n][4] inclusive
 *                      tile bounds x0,x1,y0,y1 (int32, zeros when culled);
 *                      visible (uint8); color [n][3] (float32)
 *   entries [entry_capacity]: keys in emission order and sorted (uint64; the
 *                      fast path's 32-bit keys zero-extended), Gaussian index
 *                      per entry (uint32)
 *   ranges [n_tiles][2] (uint32 start, end); per pixel [H][W]: T_final, n_proc
 *   (list entries visited, the stopping one included) and n_blend (pairs
 *   blended: past the skip test and not stopped)
 *   tile_order [n_tiles] (uint32): the tile each rasterizer workgroup took
 *   (a schedule, not a result: within each chunk of 8192 tiles, longest
 *   lists first)
 * RGS_E_CAPACITY if entry_capacity is smaller than the frame's entry count.
 */
typedef struct {
    double* depth;
    double* u;
    double* v;
    double* cov2d;
    int32_t* rect;
    uint8_t* visible;
    float* color;
    uint64_t* keys_unsorted;
    uint32_t* vals_unsorted;
    uint64_t* keys_sorted;
    uint32_t* vals_sorted;
    int64_t entry_capacity;
    uint32_t* ranges;
    float* T_final;
    uint32_t* n_proc;
    uint32_t* n_blend;
    uint32_t* tile_order;
} rgs_debug_out;

rgs_status rgs_render_debug(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                            int32_t width, int32_t height, int32_t path,
                            void* workspace, uint64_t ws_bytes, float* out_chw,
                            rgs_debug_out* dbg, rgs_frame_stats* stats);

/* ---------------------------------------------------------------------------
 * Request server: continuous batching of view requests over resident scenes.
 * The paper renders one view at a time; this runtime serves many, and every
 * image it returns is the one rgs_render computes for the same request, bit
 * for bit.
 *
 * A request is admitted, in arrival order, as soon as (a) one of n_streams
 * frame slots is free and (b) a workspace of its (scene, width, height, path)
 * class is idle or can be allocated within mem_budget bytes (idle workspaces
 * of other classes are released, least recently used first, to make room).
 * Frames of different slots overlap on the device.  A request waits behind an
 * earlier one that cannot be admitted yet.
 *
 * With use_graphs = 1 every workspace carries a HIP graph of its whole frame
 * (reset, front end, sort, ranges, raster, status export) captured once with
 * the workspace's capacity; a request replays it after its camera and output
 * pointer are written into the argument block of the graph's reset kernel.
 * With use_graphs = 0 the kernels are launched per request.  A frame whose
 * entries exceed its workspace grows its class to the frame's entry count
 * plus a quarter, and the request returns to the head of the queue: it is
 * admitted again like any other request, in a workspace of the grown class
 * obtained within mem_budget, while frames in other slots keep running (its
 * response then has retried = 1; a second overflow fails it with
 * RGS_E_CAPACITY).
 *
 * Requests' device pointers (scenes, outputs) must stay valid, and outputs
 * untouched by other work, until rgs_serve returns.  rgs_serve synchronises:
 * it returns when every admitted frame has finished.  One thread at a time
 * may use a server.
 */
typedef struct rgs_server rgs_server;

typedef struct {
    int32_t device;
    int32_t n_streams;            /* frame slots, 1..16                                      */
    uint64_t mem_budget;          /* bytes of workspace the server may hold at once (> 0)   */
    int32_t use_graphs;           /* 1: replay captured frame graphs; 0: per-request launches */
    int32_t reserved;
    double entries_per_gaussian;  /* first workspace size of a class, entries per Gaussian
                                     (0: 4)                                                   */
} rgs_server_config;

typedef struct {
    const rgs_scene* scene;       /* resident scene on the server's device                  */
    rgs_camera camera;
    int32_t width, height;
    int32_t path;                 /* RGS_PATH_PLAIN or RGS_PATH_FAST                         */
    int32_t reserved;
    double arrival;               /* seconds after the schedule starts, non-decreasing, >= 0 */
    float* out_chw;               /* device [3][height][width], caller-owned                 */
} rgs_request;

typedef struct {
    rgs_status status;            /* RGS_OK, or why this request failed (RGS_E_OOM: its
                                     workspace alone exceeds the budget)                      */
    int32_t slot;                 /* frame slot that ran it (-1 if none)                      */
    int32_t graph;                /* 1 if the frame was a graph replay                        */
    int32_t retried;              /* 1 if it was admitted again after running out of entries   */
    double t_admit;               /* host clock, s after start, when its (last) frame was enqueued */
    double t_done;                /* device clock, s after start, when its image was complete  */
    double latency;               /* t_done - arrival                                          */
    int64_t n_entries;            /* duplicated (key, index) entries of the frame              */
} rgs_response;

typedef struct {
    double wall;                  /* s from start until the last image was complete          */
    uint64_t ws_bytes_held;       /* workspace bytes held when rgs_serve returned             */
    uint64_t ws_bytes_peak;       /* most workspace bytes held at once during the call        */
    int32_t n_workspaces;         /* workspaces held when rgs_serve returned                  */
    int32_t n_captured;           /* graphs captured during the call                          */
    int32_t n_evicted;            /* idle workspaces released to make room                    */
    int32_t max_in_flight;        /* most frames admitted and unfinished at once              */
    double mean_in_flight;        /* sum over requests of (t_done - t_admit) / wall           */
    double reserved;
} rgs_server_stats;

/* Creates the slots' streams (default priority, non-blocking) and events.
 * Errors: INVALID (NULL, device out of range, n_streams outside 1..16,
 * mem_budget 0, negative entries_per_gaussian), NODEVICE, HIP. */
rgs_status rgs_server_create(const rgs_server_config* cfg, rgs_server** out);
/* Waits for the slots' streams, then frees workspaces, graphs, streams. */
void rgs_server_destroy(rgs_server* server);
/* Runs the schedule reqs[0..n) in real time (request i becomes eligible at
 * reqs[i].arrival seconds after the call starts) and fills resp[0..n).
 * Returns RGS_OK when the schedule ran, even if single requests failed (see
 * resp[i].status); INVALID (nothing ran) if any request is malformed: NULL
 * scene or output, a scene of another device or without the path's format,
 * a bad size, camera or path, arrivals not finite, negative or decreasing;
 * HIP if the runtime failed (every admitted frame has finished or been
 * abandoned by then).  stats may be NULL. */
rgs_status rgs_serve(rgs_server* server, const rgs_request* reqs, int64_t n, rgs_response* resp,
                     rgs_server_stats* stats);

/* ---------------------------------------------------------------------------
 * Differentiation of the plain path.  The paper renders only and names
 * training pipelines as the renderer's next use (Sec. V); these calls
 * differentiate the plain image definition (Sec. II-A, III-D; Eqs.
 * alpha_computation, power, opacity_clamped) with every discrete decision of
 * the forward pass held fixed (culling, tile membership, depth order, the
 * 1/255 skip test, the 1e-4 stop test, the 0.99 alpha clamp, the EWA
 * Jacobian clamp and the clamp of each colour channel at 0).
 */

/* Activated parameters in device memory, laid out as [n][...] rows (the
 * layout of contiguous torch tensors). */
typedef struct {
    int64_t n;
    const float* means;   /* device [n][3]                       */
    const float* scales;  /* device [n][3], > 0                  */
    const float* quats;   /* device [n][4] (w, x, y, z), nonzero */
    const float* opacity; /* device [n], in (0, 1]               */
    const float* sh;      /* device [n][16][3]                   */
} rgs_device_params;

/* Overwrites the plain-format attributes of an uploaded scene with params
 * (enqueued on the context's stream; values are not checked: NaN or
 * out-of-range values propagate into the image).  The fast format, if the
 * scene has one, is left as it was.  Errors: INVALID (NULL, n differs from the
 * scene's, scene without the plain format). */
rgs_status rgs_scene_update_plain(rgs_ctx* ctx, rgs_scene* scene, const rgs_device_params* params);

typedef struct {
    float* d_means;     /* device [n][3]                                           */
    float* d_scales;    /* device [n][3]                                           */
    float* d_quats;     /* device [n][4], w.r.t. the quaternion as given            */
    float* d_opacity;   /* device [n]                                               */
    float* d_sh;        /* device [n][16][3]                                        */
    float* d_screen;    /* device [n][9] or NULL: dL/d(u, v, A, B, C, o, r, g, b),
                           the image-space quantities of each Gaussian               */
    void* scratch;      /* device, 256-byte aligned, rgs_backward_scratch_size bytes */
    uint64_t scratch_bytes;
} rgs_grads;

/* Scratch bytes rgs_render_backward needs for a plain workspace of ws_bytes
 * (one 48-byte partial per duplicated entry the workspace can hold).
 * Host-only arithmetic. */
rgs_status rgs_backward_scratch_size(int64_t n, int32_t width, int32_t height, uint64_t ws_bytes,
                                     uint64_t* bytes);

/* Gradients of a loss L with respect to the activated parameters of the
 * scene, given dL_dimg = dL/d(image) (device [3][H][W]).  workspace must hold
 * the last plain-path rgs_render of this scene with this camera and size, and
 * nothing may have rendered into it since.  Per tile, the pixels' pairs are
 * walked back to front from the last blended one; transmittance is recovered
 * from the stored final T by division instead of being stored per pair.  Each
 * tile writes one partial per sorted entry (no atomics); one thread per
 * Gaussian then gathers its entries (one per covered tile) and applies the
 * chain rule through projection and SH in double precision.  Enqueued on the
 * context's stream.  The checks below need the frame's outcome: when the
 * workspace's last frame is the one this context rendered last into it (the
 * usual training loop), the outcome comes from a stamp the frame's last kernel
 * wrote to host-visible memory, and the call only waits for that frame to
 * finish (not for later work on the stream); otherwise it reads the workspace
 * header and frame parameters synchronously.  In the first case the kernels
 * still compare the workspace's frame with the caller's: if another context
 * has rendered into the workspace since, they write zero gradients and set bit
 * 3 of the workspace's device_error, which rgs_workspace_check reports.
 * The frame may be a render of RGS_PATH_PLAIN or of its training variant
 * RGS_PATH_PLAIN | RGS_HW_EXP2; the backward pass evaluates each pair as the
 * frame did (for the variant: two waves per tile over the forward's culled
 * lists, one dual pixel per lane).
 * Errors: INVALID (NULL, bad size, a workspace whose last frame was not a
 * plain render of this scene in its current state, with this camera and
 * size, scratch too small); CAPACITY (that frame overflowed its workspace);
 * DEVICE (that frame reported an internal failure). */
rgs_status rgs_render_backward(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                               int32_t width, int32_t height, const float* dL_dimg,
                               void* workspace, uint64_t ws_bytes, rgs_grads* grads);

#ifdef __cplusplus
}
#endif

#endif /* RGS_H */
