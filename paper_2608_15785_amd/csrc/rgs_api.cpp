// Host side of the C ABI declared in rgs.h: argument checks, the compact-storage
// quantiser, scene upload, workspace layout and the per-frame kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rgs.h"
#include "rgs_host.h"
#include "rgs_internal.h"

using namespace rgs;

// ---------------------------------------------------------------------------
// Errors

static thread_local std::string g_last_error;

rgs_status rgs::fail(rgs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

rgs_status rgs::ok() {
    g_last_error.clear();
    return RGS_OK;
}

extern "C" int32_t rgs_abi_version(void) { return RGS_ABI_VERSION; }

extern "C" const char* rgs_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* rgs_status_string(rgs_status s) {
    switch (s) {
        case RGS_OK: return "RGS_OK";
        case RGS_E_INVALID: return "RGS_E_INVALID";
        case RGS_E_OOM: return "RGS_E_OOM";
        case RGS_E_HIP: return "RGS_E_HIP";
        case RGS_E_CAPACITY: return "RGS_E_CAPACITY";
        case RGS_E_NODEVICE: return "RGS_E_NODEVICE";
        case RGS_E_UNSUPPORTED: return "RGS_E_UNSUPPORTED";
        case RGS_E_DEVICE: return "RGS_E_DEVICE";
        default: return "RGS_E_UNKNOWN";
    }
}

// ---------------------------------------------------------------------------
// Frame plan (Sec. IV-A, Resolution-Adaptive Sorting-Key Encoding)

static int ceil_log2(uint32_t n) {
    int b = 0;
    while ((1ull << b) < n) ++b;
    return b;
}

extern "C" rgs_status rgs_frame_plan(int32_t width, int32_t height, rgs_plan* out) {
    if (!out) return fail(RGS_E_INVALID, "rgs_frame_plan: out is NULL");
    if (width < 1 || height < 1 || width > RGS_MAX_DIM || height > RGS_MAX_DIM)
        return fail(RGS_E_INVALID, "rgs_frame_plan: image %dx%d outside [1, %d]", width, height,
                    RGS_MAX_DIM);
    rgs_plan p;
    p.width = width;
    p.height = height;
    p.tiles_x = (width + TILE - 1) / TILE;
    p.tiles_y = (height + TILE - 1) / TILE;
    p.n_tiles = p.tiles_x * p.tiles_y;
    p.b_t = std::max(1, ceil_log2((uint32_t)p.n_tiles));
    p.b_d = 32 - p.b_t;
    p.plain_key_bits = 32 + p.b_t;
    p.plain_passes = (p.plain_key_bits + RADIX_BITS - 1) / RADIX_BITS;
    p.fast_passes = 32 / RADIX_BITS;
    *out = p;
    return ok();
}

// ---------------------------------------------------------------------------
// Compact storage (Sec. IV-A, Compact Attribute Storage, Eq. quant)

// float64 -> binary16, round to nearest even, with subnormals and overflow to inf.
static uint16_t to_half(double x) {
    uint16_t sign = std::signbit(x) ? 0x8000 : 0;
    double ax = std::fabs(x);
    if (std::isnan(x)) return sign | 0x7e00;
    if (ax == 0.0) return sign;
    int e2;
    std::frexp(ax, &e2);              // ax = m 2^e2, m in [0.5, 1): leading bit at 2^(e2-1)
    int E = std::max(e2 - 1, -14);
    double units = std::nearbyint(std::ldexp(ax, 10 - E));   // ax in units of 2^(E-10)
    uint32_t mant = (uint32_t)units;
    if (mant >= 2048) {               // rounded up to the next binade
        mant >>= 1;
        E += 1;
    }
    if (mant < 1024) return sign | (uint16_t)mant;           // subnormal (E == -14)
    if (E > 15) return sign | 0x7c00;                        // overflow
    return sign | (uint16_t)(((E + 15) << 10) | (mant - 1024));
}

static double from_half(uint16_t h) {
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0) v = std::ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = std::ldexp((double)(m + 1024), e - 25);
    return (h & 0x8000) ? -v : v;
}

static const int kDegreeStart[5] = {0, 1, 4, 9, 16};

static rgs_status validate_desc(const rgs_scene_desc* d) {
    if (!d) return fail(RGS_E_INVALID, "scene desc is NULL");
    if (d->n < 1) return fail(RGS_E_INVALID, "scene has n = %lld < 1", (long long)d->n);
    if (d->n > (int64_t)((1 << 30) - 1)) return fail(RGS_E_INVALID, "scene too large (n >= 2^30)");
    if (d->sh_degree != 3) return fail(RGS_E_INVALID, "sh_degree %d != 3", d->sh_degree);
    if (!d->means || !d->scales || !d->quats || !d->opacity || !d->sh)
        return fail(RGS_E_INVALID, "scene desc has a NULL array");
    const int64_t n = d->n;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) {
            if (!std::isfinite(d->means[3 * i + k]))
                return fail(RGS_E_INVALID, "mean %lld is not finite", (long long)i);
            float s = d->scales[3 * i + k];
            if (!std::isfinite(s) || !(s > 0.0f))
                return fail(RGS_E_INVALID, "scale %lld is not finite and positive", (long long)i);
        }
        bool nonzero = false;
        for (int k = 0; k < 4; ++k) {
            float q = d->quats[4 * i + k];
            if (!std::isfinite(q)) return fail(RGS_E_INVALID, "quaternion %lld not finite", (long long)i);
            nonzero |= q != 0.0f;
        }
        if (!nonzero) return fail(RGS_E_INVALID, "quaternion %lld is zero", (long long)i);
        float o = d->opacity[i];
        if (!(o > 0.0f && o <= 1.0f))
            return fail(RGS_E_INVALID, "opacity %lld = %g outside (0, 1]", (long long)i, (double)o);
        for (int k = 0; k < 48; ++k)
            if (!std::isfinite(d->sh[48 * i + k]))
                return fail(RGS_E_INVALID, "SH of %lld not finite", (long long)i);
    }
    return RGS_OK;
}

static rgs_status quantize_into(const rgs_scene_desc* d, rgs_fast_host* o) {
    const int64_t n = d->n;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 4; ++k) o->quats_f16[4 * i + k] = to_half((double)d->quats[4 * i + k]);
        for (int k = 0; k < 3; ++k) {
            uint16_t h = to_half((double)d->scales[3 * i + k]);
            if ((h & 0x7c00) == 0x7c00)
                return fail(RGS_E_INVALID, "scale of %lld overflows FP16", (long long)i);
            o->scales_f16[3 * i + k] = h;
        }
        o->lnopa_f16[i] = to_half(std::log((double)d->opacity[i]));
        const float* sh = d->sh + 48 * i;
        for (int deg = 0; deg < 4; ++deg) {
            for (int c = 0; c < 3; ++c) {
                double m = 0.0;
                for (int k = kDegreeStart[deg]; k < kDegreeStart[deg + 1]; ++k)
                    m = std::max(m, std::fabs((double)sh[3 * k + c]));
                uint16_t sh16 = to_half(m / 127.0);
                if ((sh16 & 0x7c00) == 0x7c00)
                    return fail(RGS_E_INVALID, "SH scale of %lld overflows FP16", (long long)i);
                o->sh_scale_f16[12 * i + 3 * deg + c] = sh16;
                double s = from_half(sh16);
                for (int k = kDegreeStart[deg]; k < kDegreeStart[deg + 1]; ++k) {
                    double q = s > 0.0 ? std::nearbyint((double)sh[3 * k + c] / s) : 0.0;
                    q = std::min(127.0, std::max(-127.0, q));
                    o->sh_q[48 * i + 3 * k + c] = (int8_t)q;
                }
            }
        }
    }
    return RGS_OK;
}

extern "C" rgs_status rgs_quantize_host(const rgs_scene_desc* desc, rgs_fast_host* out) {
    rgs_status s = validate_desc(desc);
    if (s != RGS_OK) return s;
    if (!out || !out->quats_f16 || !out->scales_f16 || !out->lnopa_f16 || !out->sh_q ||
        !out->sh_scale_f16)
        return fail(RGS_E_INVALID, "rgs_quantize_host: NULL output array");
    s = quantize_into(desc, out);
    return s == RGS_OK ? ok() : s;
}

// ---------------------------------------------------------------------------
// Context

// Stage boundaries of one timed frame.  A boundary that a path does not have
// (the fused front end has no separate duplication) is not recorded: the
// stage before it counts zero, and the next stage starts at the last recorded
// boundary.  (Two events recorded back to back measure a few microseconds of
// idle GPU, not work.)
struct FrameEvents {
    hipEvent_t ev[RGS_N_STAGES + 1];
    bool skipped[RGS_N_STAGES + 1];
};

// The last plain frame a context rendered into a workspace.  Its outcome and
// stamp arrive in stamps[slot] (host-visible memory written by the frame's
// last kernel), so that the backward pass needs no device read when it
// differentiates a frame its own context rendered.
struct FrameRecord {
    const void* ws = nullptr;     // nullptr: slot unused
    uint64_t ws_bytes = 0;
    const rgs_scene* scene = nullptr;
    uint64_t scene_tag = 0, cam_hash = 0;
    int32_t width = 0, height = 0, path = 0;
    hipStream_t stream = nullptr;
    uint64_t seq = 0;             // the stamp's sequence number once written
    uint64_t last_use = 0;
};
constexpr int N_FRAME_RECORDS = 8;

struct rgs_ctx {
    int device;
    hipStream_t stream;
    bool timing;
    uint32_t debug;      // RGS_DEBUG_* flags
    std::vector<FrameEvents> events;
    size_t events_used;
    double stage_ms[RGS_N_STAGES];
    int64_t frames;
    FrameRecord records[N_FRAME_RECORDS];
    FrameStamp* stamps = nullptr;     // [N_FRAME_RECORDS], host-visible
    uint64_t seq = 0, uses = 0;
};

// ---------------------------------------------------------------------------
// The allocation-free render's workspace: a file-scope device array, one copy
// per device, that the library holds from the first context on a device until
// the process ends.  Host code never uses the array's name as an address (on
// the host it is only a stand-in): each device's address is looked up once,
// with that device current, when the first context on it is created.

constexpr uint64_t STATIC_WS_BYTES = 128ull << 20;      // RGS_STATIC_WORKSPACE_BYTES
static_assert(STATIC_WS_BYTES == RGS_STATIC_WORKSPACE_BYTES, "static workspace size");
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES];

// With `device` current: finds that device's copy of `scratch` (once).
static rgs_status scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return fail(RGS_E_INVALID, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return RGS_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(RGS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return RGS_OK;
}

extern "C" rgs_status rgs_ctx_create(int32_t device, void* hip_stream, rgs_ctx** out) {
    if (!out) return fail(RGS_E_INVALID, "rgs_ctx_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return fail(RGS_E_NODEVICE, "no HIP device available");
    if (device < 0 || device >= count)
        return fail(RGS_E_INVALID, "device %d outside [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    rgs_status ss = scratch_setup(device);
    if (ss != RGS_OK) return ss;
    void* stamps = nullptr;
    HIP_TRY(hipHostMalloc(&stamps, N_FRAME_RECORDS * sizeof(FrameStamp), hipHostMallocCoherent));
    std::memset(stamps, 0, N_FRAME_RECORDS * sizeof(FrameStamp));
    rgs_ctx* c = new rgs_ctx();
    c->stamps = static_cast<FrameStamp*>(stamps);
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->timing = false;
    c->debug = 0;
    c->events_used = 0;
    std::fill(c->stage_ms, c->stage_ms + RGS_N_STAGES, 0.0);
    c->frames = 0;
    *out = c;
    return ok();
}

extern "C" void rgs_ctx_destroy(rgs_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (auto& fe : ctx->events)
        for (auto& e : fe.ev) (void)hipEventDestroy(e);
    // frames still queued on any stream may write their stamps
    (void)hipDeviceSynchronize();
    (void)hipHostFree(ctx->stamps);
    delete ctx;
}

extern "C" rgs_status rgs_ctx_set_stream(rgs_ctx* ctx, void* hip_stream) {
    if (!ctx) return fail(RGS_E_INVALID, "ctx is NULL");
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return ok();
}

extern "C" rgs_status rgs_ctx_set_debug(rgs_ctx* ctx, uint32_t flags) {
    if (!ctx) return fail(RGS_E_INVALID, "ctx is NULL");
    if (flags & ~RGS_DEBUG_SORT_FALLBACK) return fail(RGS_E_INVALID, "unknown debug flags 0x%x", flags);
    ctx->debug = flags;
    return ok();
}

extern "C" rgs_status rgs_ctx_set_timing(rgs_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(RGS_E_INVALID, "ctx is NULL");
    ctx->timing = enable != 0;
    ctx->events_used = 0;
    std::fill(ctx->stage_ms, ctx->stage_ms + RGS_N_STAGES, 0.0);
    ctx->frames = 0;
    return ok();
}

static rgs_status harvest_events(rgs_ctx* ctx) {
    if (ctx->events_used == 0) return RGS_OK;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (size_t f = 0; f < ctx->events_used; ++f) {
        const FrameEvents& fe = ctx->events[f];
        int last = 0;
        for (int s = 0; s < RGS_N_STAGES; ++s) {
            if (fe.skipped[s + 1]) continue;
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, fe.ev[last], fe.ev[s + 1]));
            ctx->stage_ms[s] += ms;
            last = s + 1;
        }
        ctx->frames += 1;
    }
    ctx->events_used = 0;
    return RGS_OK;
}

extern "C" rgs_status rgs_ctx_collect_timing(rgs_ctx* ctx, double* stage_ms, int64_t* n_frames) {
    if (!ctx || !stage_ms || !n_frames) return fail(RGS_E_INVALID, "rgs_ctx_collect_timing: NULL argument");
    HIP_TRY(hipSetDevice(ctx->device));
    rgs_status s = harvest_events(ctx);
    if (s != RGS_OK) return s;
    std::copy(ctx->stage_ms, ctx->stage_ms + RGS_N_STAGES, stage_ms);
    *n_frames = ctx->frames;
    std::fill(ctx->stage_ms, ctx->stage_ms + RGS_N_STAGES, 0.0);
    ctx->frames = 0;
    return ok();
}

extern "C" rgs_status rgs_probe_valu(rgs_ctx* ctx, int32_t blocks, int32_t iters, float* out) {
    if (!ctx || !out) return fail(RGS_E_INVALID, "rgs_probe_valu: NULL argument");
    if (blocks < 1 || blocks > (1 << 20) || iters < 0)
        return fail(RGS_E_INVALID, "rgs_probe_valu: blocks %d outside [1, 2^20] or iters %d < 0", blocks, iters);
    HIP_TRY(hipSetDevice(ctx->device));
    launch_probe_valu(ctx->stream, out, (uint32_t)blocks, (uint32_t)iters);
    HIP_TRY(hipGetLastError());
    return ok();
}

// Events of the next timed frame (the pool grows on demand; full pools are
// harvested, which synchronises the stream only every 1024 frames).
static rgs_status next_events(rgs_ctx* ctx, FrameEvents** fe) {
    if (ctx->events_used == 1024) {
        rgs_status s = harvest_events(ctx);
        if (s != RGS_OK) return s;
    }
    if (ctx->events_used == ctx->events.size()) {
        FrameEvents f;
        for (auto& e : f.ev) HIP_TRY(hipEventCreate(&e));
        ctx->events.push_back(f);
    }
    *fe = &ctx->events[ctx->events_used++];
    std::fill((*fe)->skipped, (*fe)->skipped + RGS_N_STAGES + 1, false);
    return RGS_OK;
}

// ---------------------------------------------------------------------------
// Scenes

struct rgs_scene {
    int device;
    uint64_t tag;        // new at upload and at every rgs_scene_update_plain
    int64_t n;
    uint64_t n_pad;
    uint32_t formats;
    float* plain;        // P_COUNT planes of n_pad floats
    uint32_t* fast;      // F_COUNT planes of n_pad words
    uint64_t bytes;
};

// Scene tags: a process-wide counter, so that no two states of any scenes
// share a tag.
static std::atomic<uint64_t> g_scene_tags{1};
static uint64_t next_scene_tag() { return g_scene_tags.fetch_add(1, std::memory_order_relaxed); }

extern "C" rgs_status rgs_scene_upload(rgs_ctx* ctx, const rgs_scene_desc* d, uint32_t formats,
                                       rgs_scene** out) {
    if (!ctx || !out) return fail(RGS_E_INVALID, "rgs_scene_upload: NULL argument");
    *out = nullptr;
    if (formats == 0 || (formats & ~(RGS_FMT_PLAIN | RGS_FMT_FAST)))
        return fail(RGS_E_INVALID, "formats 0x%x invalid", formats);
    rgs_status s = validate_desc(d);
    if (s != RGS_OK) return s;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n = d->n;
    const uint64_t np = ((uint64_t)n + 63) & ~63ull;
    rgs_scene* sc = new rgs_scene();
    sc->device = ctx->device;
    sc->tag = next_scene_tag();
    sc->n = n;
    sc->n_pad = np;
    sc->formats = formats;
    sc->plain = nullptr;
    sc->fast = nullptr;
    sc->bytes = 0;
    auto cleanup = [&]() {
        if (sc->plain) (void)hipFree(sc->plain);
        if (sc->fast) (void)hipFree(sc->fast);
        delete sc;
    };
    if (formats & RGS_FMT_PLAIN) {
        std::vector<float> h((size_t)np * P_COUNT, 0.0f);
        for (int64_t i = 0; i < n; ++i) {
            for (int k = 0; k < 3; ++k) h[(P_MX + k) * np + i] = d->means[3 * i + k];
            for (int k = 0; k < 3; ++k) h[(P_SX + k) * np + i] = d->scales[3 * i + k];
            for (int k = 0; k < 4; ++k) h[(P_QW + k) * np + i] = d->quats[4 * i + k];
            h[P_OPA * np + i] = d->opacity[i];
            h[P_LNO * np + i] = (float)std::log((double)d->opacity[i]);
            for (int k = 0; k < 48; ++k) h[(P_SH0 + k) * np + i] = d->sh[48 * i + k];
        }
        size_t bytes = h.size() * sizeof(float);
        if (hipMalloc(&sc->plain, bytes) != hipSuccess) {
            cleanup();
            return fail(RGS_E_OOM, "plain scene: %zu bytes", bytes);
        }
        if (hipMemcpy(sc->plain, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            cleanup();
            return fail(RGS_E_HIP, "plain scene copy failed");
        }
        sc->bytes += bytes;
    }
    if (formats & RGS_FMT_FAST) {
        std::vector<uint16_t> q16((size_t)n * 4), s16((size_t)n * 3), l16((size_t)n), ss16((size_t)n * 12);
        std::vector<int8_t> shq((size_t)n * 48);
        rgs_fast_host fh{q16.data(), s16.data(), l16.data(), shq.data(), ss16.data()};
        s = quantize_into(d, &fh);
        if (s != RGS_OK) {
            cleanup();
            return s;
        }
        std::vector<uint32_t> h((size_t)np * F_COUNT, 0u);
        auto pair = [](uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); };
        for (int64_t i = 0; i < n; ++i) {
            for (int k = 0; k < 3; ++k) {
                uint32_t w;
                std::memcpy(&w, &d->means[3 * i + k], 4);
                h[(F_MX + k) * np + i] = w;
            }
            h[F_QWX * np + i] = pair(q16[4 * i + 0], q16[4 * i + 1]);
            h[F_QYZ * np + i] = pair(q16[4 * i + 2], q16[4 * i + 3]);
            h[F_SXY * np + i] = pair(s16[3 * i + 0], s16[3 * i + 1]);
            h[F_SZL * np + i] = pair(s16[3 * i + 2], l16[i]);
            for (int k = 0; k < 12; ++k) {
                uint32_t w = 0;
                for (int b = 0; b < 4; ++b) w |= (uint32_t)(uint8_t)shq[48 * i + 4 * k + b] << (8 * b);
                h[(F_SHQ0 + k) * np + i] = w;
            }
            for (int k = 0; k < 6; ++k)
                h[(F_SHS0 + k) * np + i] = pair(ss16[12 * i + 2 * k], ss16[12 * i + 2 * k + 1]);
        }
        size_t bytes = h.size() * sizeof(uint32_t);
        if (hipMalloc(&sc->fast, bytes) != hipSuccess) {
            cleanup();
            return fail(RGS_E_OOM, "fast scene: %zu bytes", bytes);
        }
        if (hipMemcpy(sc->fast, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            cleanup();
            return fail(RGS_E_HIP, "fast scene copy failed");
        }
        sc->bytes += bytes;
    }
    *out = sc;
    return ok();
}

extern "C" rgs_status rgs_scene_release(rgs_ctx* ctx, rgs_scene* sc) {
    if (!sc) return ok();
    if (ctx) (void)hipSetDevice(ctx->device);
    if (sc->plain) (void)hipFree(sc->plain);
    if (sc->fast) (void)hipFree(sc->fast);
    delete sc;
    return ok();
}

extern "C" rgs_status rgs_scene_device_bytes(const rgs_scene* sc, uint64_t* bytes) {
    if (!sc || !bytes) return fail(RGS_E_INVALID, "rgs_scene_device_bytes: NULL argument");
    *bytes = sc->bytes;
    return ok();
}

extern "C" rgs_status rgs_scene_info(const rgs_scene* sc, int64_t* n, uint32_t* formats,
                                     uint64_t* device_bytes) {
    if (!sc) return fail(RGS_E_INVALID, "scene is NULL");
    if (n) *n = sc->n;
    if (formats) *formats = sc->formats;
    if (device_bytes) *device_bytes = sc->bytes;
    return ok();
}

// ---------------------------------------------------------------------------
// Workspace layout

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// The base path (RGS_PATH_PLAIN / RGS_PATH_FAST) and the ablation bits of a
// path argument.
static int32_t path_base(int32_t path) { return path & 0xff; }
static constexpr uint32_t PATH_BITS = RGS_ABLATE_MASK | RGS_EXACT_TILES | RGS_HW_EXP2 | RGS_QUAD_PIXEL;
static uint32_t path_opts(int32_t path) { return ((uint32_t)path & PATH_BITS) >> 8; }

static void make_layout(int64_t n, const rgs_plan& p, int32_t path, uint64_t capacity, WsLayout& L) {
    const bool plain = path_base(path) == RGS_PATH_PLAIN;
    const uint32_t opts = path_opts(path);
    L.capacity = capacity;
    L.key_bytes = (plain || (opts & OPT_KEY32)) ? 8 : 4;
    L.passes = L.key_bytes == 8 ? (uint32_t)p.plain_passes : (uint32_t)p.fast_passes;
    fe_block_shape(n, L.fe_blocks, L.fe_per);
    const uint64_t st = sort_tile_size(L.key_bytes);
    L.sort_blocks_max = (uint32_t)((capacity + st - 1) / st);
    uint64_t off = 0;
    L.header = off;
    off = align256(off + sizeof(WsHeader));
    L.ranges = off;
    off = align256(off + (uint64_t)p.n_tiles * 8);
    L.fe_state = off;
    off = align256(off + (uint64_t)L.fe_blocks * 8);
    L.hist = off;
    off = align256(off + (uint64_t)HIST_COPIES * MAX_PASSES * RADIX * 4);
    L.zero_end = off;
    L.params = off;                  // written by the reset kernel, outside the zeroed span
    off = align256(off + sizeof(FrameParams));
    L.order = off;                   // written whole by the tile-order kernel
    off = align256(off + (uint64_t)p.n_tiles * 4);
    L.records = off;
    off = align256(off + (uint64_t)n * sizeof(Record));
    L.counts = L.rects = L.depths = L.offsets = L.masks = 0;
    if (!plain && (opts & OPT_FUSION) && (opts & OPT_EXACT_TILES)) {
        L.masks = off;
        off = align256(off + (uint64_t)n * 8);
    }
    if (plain || (opts & OPT_FUSION)) {
        L.counts = off;
        off = align256(off + (uint64_t)n * 4);
        L.rects = off;
        off = align256(off + (uint64_t)n * 8);
        L.depths = off;
        off = align256(off + (uint64_t)n * 4);
        L.offsets = off;
        off = align256(off + (uint64_t)n * 4);
    }
    L.keys_a = off;
    off = align256(off + capacity * L.key_bytes);
    L.keys_b = off;
    off = align256(off + capacity * L.key_bytes);
    L.vals_a = off;
    off = align256(off + capacity * 4);
    L.vals_b = off;
    off = align256(off + capacity * 4);
    L.sort_state = off;
    {
        const uint64_t groups = (L.sort_blocks_max + SORT_GROUP - 1) / SORT_GROUP;
        off = align256(off + 2 * ((uint64_t)L.sort_blocks_max + groups) * RADIX * 4);
    }
    L.t_final = off;
    off = align256(off + (uint64_t)p.width * p.height * 4);
    L.n_proc = off;
    off = align256(off + (uint64_t)p.width * p.height * 4);
    L.n_blend = off;
    off = align256(off + (uint64_t)p.width * p.height * 4);
    L.total = off;
}

rgs_status rgs::check_path(int32_t path) {
    const int32_t base = path_base(path);
    if ((base != RGS_PATH_PLAIN && base != RGS_PATH_FAST) || ((uint32_t)path & ~(0xffu | PATH_BITS)))
        return fail(RGS_E_INVALID, "path 0x%x is neither RGS_PATH_PLAIN nor RGS_PATH_FAST with ablation bits", path);
    if (base == RGS_PATH_PLAIN && (path_opts(path) & ~OPT_HW_EXP2))
        return fail(RGS_E_INVALID, "ablation and extension bits other than RGS_HW_EXP2 apply to the fast path only");
    if ((path & RGS_EXACT_TILES) && (path & RGS_ABLATE_EXTENT))
        return fail(RGS_E_INVALID, "RGS_EXACT_TILES refines the alpha-ellipse extent that RGS_ABLATE_EXTENT removes");
    if ((path & RGS_HW_EXP2) && (path & (RGS_ABLATE_FASTEXP | RGS_ABLATE_DUALPIXEL)))
        return fail(RGS_E_INVALID, "RGS_HW_EXP2 replaces the exponential of the dual-pixel rasterizer; "
                                   "not with RGS_ABLATE_FASTEXP or RGS_ABLATE_DUALPIXEL");
    if ((path & RGS_QUAD_PIXEL) && (path & (RGS_ABLATE_FASTEXP | RGS_ABLATE_DUALPIXEL | RGS_HW_EXP2)))
        return fail(RGS_E_INVALID, "RGS_QUAD_PIXEL extends the dual-pixel rasterizer with the bit-level "
                                   "exponential; not with RGS_ABLATE_FASTEXP, RGS_ABLATE_DUALPIXEL or RGS_HW_EXP2");
    return RGS_OK;
}

extern "C" rgs_status rgs_workspace_size(int64_t n, int32_t width, int32_t height, int32_t path,
                                         int64_t max_entries, uint64_t* bytes) {
    if (!bytes) return fail(RGS_E_INVALID, "bytes is NULL");
    if (n < 1) return fail(RGS_E_INVALID, "n < 1");
    if (max_entries < 1 || (uint64_t)max_entries > RGS_MAX_ENTRIES)
        return fail(RGS_E_INVALID, "max_entries %lld outside [1, 2^30 - 1]", (long long)max_entries);
    rgs_status s = check_path(path);
    if (s != RGS_OK) return s;
    rgs_plan p;
    s = rgs_frame_plan(width, height, &p);
    if (s != RGS_OK) return s;
    WsLayout L;
    make_layout(n, p, path, (uint64_t)max_entries, L);
    *bytes = L.total;
    return ok();
}

extern "C" rgs_status rgs_render_workspace_bound(const rgs_scene* sc, int32_t width, int32_t height, int32_t path,
                                                 uint64_t hint_ndup, uint64_t* bytes) {
    if (!sc || !bytes) return fail(RGS_E_INVALID, "rgs_render_workspace_bound: NULL argument");
    if (hint_ndup > RGS_MAX_ENTRIES)
        return fail(RGS_E_INVALID, "hint_ndup %llu above RGS_MAX_ENTRIES", (unsigned long long)hint_ndup);
    uint64_t entries = hint_ndup;
    if (!entries) entries = std::min<uint64_t>(RGS_MAX_ENTRIES, std::max<uint64_t>(4ull * (uint64_t)sc->n, 65536ull));
    return rgs_workspace_size(sc->n, width, height, path, (int64_t)entries, bytes);
}

// Largest capacity whose layout fits in ws_bytes (0 if none).
static uint64_t capacity_for(int64_t n, const rgs_plan& p, int32_t path, uint64_t ws_bytes) {
    uint64_t lo = 0, hi = RGS_MAX_ENTRIES;
    WsLayout L;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        make_layout(n, p, path, mid, L);
        if (L.total <= ws_bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

extern "C" rgs_status rgs_workspace_capacity(int64_t n, int32_t width, int32_t height, int32_t path,
                                             uint64_t ws_bytes, int64_t* capacity) {
    if (!capacity) return fail(RGS_E_INVALID, "capacity is NULL");
    if (n < 1) return fail(RGS_E_INVALID, "n < 1");
    rgs_status s = check_path(path);
    if (s != RGS_OK) return s;
    rgs_plan p;
    s = rgs_frame_plan(width, height, &p);
    if (s != RGS_OK) return s;
    *capacity = (int64_t)capacity_for(n, p, path, ws_bytes);
    return ok();
}

static WsDev ws_pointers(void* base, const WsLayout& L) {
    char* b = static_cast<char*>(base);
    WsDev w;
    w.params = reinterpret_cast<const FrameParams*>(b + L.params);
    w.header = reinterpret_cast<WsHeader*>(b + L.header);
    w.ranges = reinterpret_cast<uint32_t*>(b + L.ranges);
    w.order = reinterpret_cast<uint32_t*>(b + L.order);
    w.fe_state = reinterpret_cast<uint64_t*>(b + L.fe_state);
    w.records = reinterpret_cast<Record*>(b + L.records);
    w.counts = L.counts ? reinterpret_cast<uint32_t*>(b + L.counts) : nullptr;
    w.rects = L.rects ? reinterpret_cast<uint64_t*>(b + L.rects) : nullptr;
    w.depths = L.depths ? reinterpret_cast<float*>(b + L.depths) : nullptr;
    w.offsets = L.offsets ? reinterpret_cast<uint32_t*>(b + L.offsets) : nullptr;
    w.masks = L.masks ? reinterpret_cast<uint64_t*>(b + L.masks) : nullptr;
    w.keys_a = b + L.keys_a;
    w.keys_b = b + L.keys_b;
    w.vals_a = reinterpret_cast<uint32_t*>(b + L.vals_a);
    w.vals_b = reinterpret_cast<uint32_t*>(b + L.vals_b);
    w.hist = reinterpret_cast<uint32_t*>(b + L.hist);
    w.sort_state = reinterpret_cast<uint32_t*>(b + L.sort_state);
    w.sort_rows = L.sort_blocks_max;
    w.sort_groups = (L.sort_blocks_max + SORT_GROUP - 1) / SORT_GROUP;
    w.t_final = reinterpret_cast<float*>(b + L.t_final);
    w.n_proc = reinterpret_cast<uint32_t*>(b + L.n_proc);
    w.n_blend = reinterpret_cast<uint32_t*>(b + L.n_blend);
    return w;
}

// ---------------------------------------------------------------------------
// Render

rgs_status rgs::check_camera(const rgs_camera* c) {
    if (!c) return fail(RGS_E_INVALID, "camera is NULL");
    const double* all[] = {c->R, c->t};
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(all[0][k])) return fail(RGS_E_INVALID, "camera R not finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(all[1][k])) return fail(RGS_E_INVALID, "camera t not finite");
    double v[] = {c->fx, c->fy, c->cx, c->cy, c->tan_half_fovx, c->tan_half_fovy, c->z_near, c->z_far};
    for (double x : v)
        if (!std::isfinite(x)) return fail(RGS_E_INVALID, "camera intrinsics not finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->bg[k])) return fail(RGS_E_INVALID, "camera background not finite");
    if (!(c->fx > 0.0 && c->fy > 0.0)) return fail(RGS_E_INVALID, "focal lengths must be positive");
    if (!(c->tan_half_fovx > 0.0 && c->tan_half_fovy > 0.0))
        return fail(RGS_E_INVALID, "tan_half_fov must be positive");
    if (!(c->z_near > 0.0 && c->z_near < c->z_far))
        return fail(RGS_E_INVALID, "need 0 < z_near < z_far (got %g, %g)", c->z_near, c->z_far);
    return RGS_OK;
}

static CamDev cam_dev(const rgs_camera* c) {
    CamDev d;
    for (int k = 0; k < 9; ++k) d.r[k] = c->R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = c->t[k];
    d.fx = c->fx;
    d.fy = c->fy;
    d.cx = c->cx;
    d.cy = c->cy;
    d.tanx = c->tan_half_fovx;
    d.tany = c->tan_half_fovy;
    d.zn = c->z_near;
    d.zf = c->z_far;
    for (int k = 0; k < 3; ++k) {
        // camera centre -R^T t
        double pos = -(c->R[0 + k] * c->t[0] + c->R[3 + k] * c->t[1] + c->R[6 + k] * c->t[2]);
        d.campos[k] = (float)pos;
        d.bg[k] = c->bg[k];
    }
    return d;
}

static rgs_status read_header(rgs_ctx* ctx, const void* ws, WsHeader* h) {
    HIP_TRY(hipMemcpyAsync(h, ws, sizeof(WsHeader), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return RGS_OK;
}

static rgs_status header_status(const WsHeader& h, rgs_frame_stats* st, int64_t n) {
    if (st) {
        st->n_gaussians = n;
        st->n_visible = h.n_visible;
        st->n_entries = (int64_t)h.n_entries;
        st->capacity = h.capacity;
        st->path = (int32_t)h.path;
        st->passes = (int32_t)h.passes;
        st->overflow = (int32_t)h.overflow;
        st->device_error = (int32_t)h.error;
        st->list_steps = (int64_t)h.list_steps;
    }
    if (h.error)
        return fail(RGS_E_DEVICE, "the frame reported device errors 0x%x (1, 4: a bounded wait gave up or a "
                    "failed sort; 8: a backward pass found another frame than its caller's)", h.error);
    if (h.overflow)
        return fail(RGS_E_CAPACITY, "frame needs %llu entries, workspace holds %u",
                    (unsigned long long)h.n_entries, h.capacity);
    return RGS_OK;
}

// FNV-1a over the camera's bytes and the image size.
static uint64_t camera_hash(const rgs_camera* c, int32_t width, int32_t height) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    mix(c, sizeof(rgs_camera));
    mix(&width, sizeof(width));
    mix(&height, sizeof(height));
    return h;
}

// Notes the frame just enqueued on ctx's stream into ws.  A plain frame gets
// a record and a stamp export after its last kernel; any other frame only
// retires the workspace's record.
static rgs_status note_frame(rgs_ctx* ctx, const FrameLaunch& fl, const void* ws, uint64_t ws_bytes,
                             const rgs_scene* sc, const FrameParams& prm, int32_t width, int32_t height,
                             int32_t path) {
    int slot = -1;
    for (int i = 0; i < N_FRAME_RECORDS; ++i)
        if (ctx->records[i].ws == ws) slot = i;
    if (fl.path != RGS_PATH_PLAIN) {
        if (slot >= 0) ctx->records[slot] = FrameRecord{};
        return RGS_OK;
    }
    if (slot < 0) {                 // an unused slot, else the least recently used
        slot = 0;
        for (int i = 0; i < N_FRAME_RECORDS; ++i) {
            if (!ctx->records[i].ws) {
                slot = i;
                break;
            }
            if (ctx->records[i].last_use < ctx->records[slot].last_use) slot = i;
        }
    }
    FrameRecord& r = ctx->records[slot];
    // a stamp export still queued on another stream must not land after this one
    if (r.ws && r.stream != ctx->stream) HIP_TRY(hipStreamSynchronize(r.stream));
    r.ws = ws;
    r.ws_bytes = ws_bytes;
    r.scene = sc;
    r.scene_tag = prm.scene_tag;
    r.cam_hash = prm.cam_hash;
    r.width = width;
    r.height = height;
    r.path = path;
    r.stream = ctx->stream;
    r.seq = ++ctx->seq;
    r.last_use = ++ctx->uses;
    launch_export_stamp(ctx->stream, fl.w, &ctx->stamps[slot], r.seq);
    HIP_TRY(hipGetLastError());
    return RGS_OK;
}

// Waits, spinning on host-visible memory, until the stamp of record `slot`
// has arrived, i.e. its frame has finished on the GPU, and copies it.
static rgs_status wait_stamp(rgs_ctx* ctx, int slot, FrameStamp* out) {
    const FrameRecord& r = ctx->records[slot];
    FrameStamp* p = &ctx->stamps[slot];
    for (uint32_t spin = 1;; ++spin) {
        if (__atomic_load_n(&p->seq, __ATOMIC_ACQUIRE) == r.seq) break;
        if (spin % 256 == 0) {      // the stream has drained, or failed, without it
            const hipError_t e = hipStreamQuery(r.stream);
            if (e == hipSuccess) {
                if (__atomic_load_n(&p->seq, __ATOMIC_ACQUIRE) == r.seq) break;
                return fail(RGS_E_HIP, "the frame's stamp was not written");
            }
            if (e != hipErrorNotReady) return fail(RGS_E_HIP, "hipStreamQuery: %s", hipGetErrorString(e));
        }
#if defined(__x86_64__)
        __builtin_ia32_pause();
#endif
    }
    out->n_entries = p->n_entries;
    out->overflow = p->overflow;
    out->error = p->error;
    out->scene_tag = p->scene_tag;
    out->cam_hash = p->cam_hash;
    out->seq = r.seq;
    return RGS_OK;
}

FrameParams rgs::frame_params(const rgs_camera* c, float* out, const rgs_scene* sc, int32_t width,
                              int32_t height) {
    FrameParams p;
    p.cam = cam_dev(c);
    p.out = out;
    p.scene_tag = sc ? sc->tag : 0;
    p.cam_hash = camera_hash(c, width, height);
    return p;
}

int rgs::scene_device(const rgs_scene* sc) { return sc->device; }

rgs_status rgs::prepare_frame(const rgs_scene* sc, int32_t W, int32_t H, int32_t path, void* ws,
                              uint64_t ws_bytes, FrameLaunch* fl) {
    if (!sc) return fail(RGS_E_INVALID, "scene is NULL");
    rgs_status s = check_path(path);
    if (s != RGS_OK) return s;
    const int32_t base = path_base(path);
    const uint32_t opts = path_opts(path);
    if (base == RGS_PATH_PLAIN && !(sc->formats & RGS_FMT_PLAIN))
        return fail(RGS_E_INVALID, "scene was uploaded without the plain format");
    if (base == RGS_PATH_FAST && !(sc->formats & RGS_FMT_FAST))
        return fail(RGS_E_INVALID, "scene was uploaded without the fast format");
    if ((opts & (OPT_INT8_SH | OPT_FP16_GEOM)) && !(sc->formats & RGS_FMT_PLAIN))
        return fail(RGS_E_INVALID, "the storage ablations read the plain format, which the scene lacks");
    s = rgs_frame_plan(W, H, &fl->plan);
    if (s != RGS_OK) return s;
    if (!ws) return fail(RGS_E_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(RGS_E_INVALID, "workspace must be 256-byte aligned");
    const rgs_plan& p = fl->plan;
    uint64_t cap = capacity_for(sc->n, p, path, ws_bytes);
    if (cap == 0) return fail(RGS_E_INVALID, "workspace of %llu bytes is too small", (unsigned long long)ws_bytes);
    fl->device = sc->device;
    fl->n = sc->n;
    fl->path = base;
    fl->opts = opts;
    fl->path_word = (uint32_t)path;
    make_layout(sc->n, p, path, cap, fl->L);
    fl->w = ws_pointers(ws, fl->L);
    FrameDev& f = fl->f;
    f.width = W;
    f.height = H;
    f.tiles_x = p.tiles_x;
    f.tiles_y = p.tiles_y;
    f.n_tiles = p.n_tiles;
    f.b_t = p.b_t;
    f.b_d = p.b_d;
    f.passes = (int32_t)fl->L.passes;
    f.capacity = (uint32_t)cap;
    f.n_gaussians = (uint32_t)sc->n;
    f.ordered = (base == RGS_PATH_PLAIN || p.n_tiles <= ORDER_MAX_TILES) ? 1u : 0u;
    fl->plain = PlainSceneDev{sc->plain, sc->n_pad, sc->n};
    fl->fast = FastSceneDev{sc->fast, sc->n_pad, sc->n, sc->plain};
    return RGS_OK;
}

rgs_status rgs::enqueue_frame(hipStream_t st, const FrameLaunch& fl, const FrameParams& prm,
                              const DebugDev* dbg, bool count, FrameStatus* status,
                              const FrameHooks* hooks, bool* result_in_b) {
    auto mark = [&](int k) {
        if (hooks && hooks->mark) hooks->mark(hooks->user, k);
    };
    const WsDev& w = fl.w;
    mark(0);
    launch_reset(st, reset_args(w, fl.L.zero_end, fl.f, fl.path_word, prm));
    if (fl.path == RGS_PATH_PLAIN) {
        launch_preprocess_plain(st, fl.plain, fl.f, w, dbg, (fl.opts & OPT_HW_EXP2) != 0);
        mark(1);
        launch_duplicate(st, fl.n, fl.f, w, fl.L.fe_blocks, fl.L.fe_per, fl.L.key_bytes);
        mark(2);
    } else if (fl.opts & OPT_FUSION) {
        launch_preprocess_fast(st, fl.fast, fl.f, w, dbg, fl.opts);
        mark(1);
        launch_duplicate(st, fl.n, fl.f, w, fl.L.fe_blocks, fl.L.fe_per, fl.L.key_bytes);
        mark(2);
    } else {
        launch_frontend_fast(st, fl.fast, fl.f, w, fl.L.fe_blocks, fl.L.fe_per, dbg, fl.opts);
        mark(1);
        mark(-2);       // no duplication stage
    }
    if (hooks && hooks->after_front) {
        rgs_status s = hooks->after_front(hooks->user);
        if (s != RGS_OK) return s;
    }
    bool in_b = false;
    if (bucket_sort_applies(fl.f, fl.L.key_bytes)) {
        launch_sort_bucket(st, fl.f, w, fl.sort_fallback, &in_b);     // the ranges come with it
        mark(3);
    } else {
        launch_sort(st, fl.f, w, fl.L.key_bytes, fl.L.passes, fl.sort_fallback, &in_b);
        mark(3);
        launch_ranges(st, fl.f, w, fl.L.key_bytes, in_b);
    }
    launch_tile_order(st, fl.f, w);
    mark(4);
    if (fl.path == RGS_PATH_PLAIN && (fl.opts & OPT_HW_EXP2)) launch_raster_train(st, fl.f, w, in_b, count);
    else if (fl.path == RGS_PATH_PLAIN) launch_raster_plain(st, fl.f, w, in_b, count);
    else launch_raster_fast(st, fl.f, w, in_b, count, fl.opts);
    mark(5);
    if (status) launch_export_status(st, w, status);
    if (result_in_b) *result_in_b = in_b;
    HIP_TRY(hipGetLastError());
    return RGS_OK;
}

namespace {

// Instrumentation of a render call: stage events and, for debug renders, the
// copies of the unsorted entries once the front end has finished.
struct RenderHooks {
    rgs_ctx* ctx;
    FrameEvents* fe;
    rgs_debug_out* dbg;
    const FrameLaunch* fl;
    void* ws;
    uint64_t n_entries;
};

void hook_mark(void* user, int k) {
    RenderHooks* h = static_cast<RenderHooks*>(user);
    if (!h->fe) return;
    if (k < 0) h->fe->skipped[-k] = true;
    else (void)hipEventRecord(h->fe->ev[k], h->ctx->stream);
}

rgs_status hook_after_front(void* user) {
    RenderHooks* h = static_cast<RenderHooks*>(user);
    rgs_debug_out* dbg = h->dbg;
    if (!dbg) return RGS_OK;
    hipStream_t st = h->ctx->stream;
    const WsDev& w = h->fl->w;
    WsHeader hd;
    rgs_status s = read_header(h->ctx, h->ws, &hd);
    if (s != RGS_OK) return s;
    h->n_entries = std::min<uint64_t>(hd.n_entries, h->fl->L.capacity);
    if (dbg->entry_capacity < (int64_t)hd.n_entries &&
        (dbg->keys_unsorted || dbg->keys_sorted || dbg->vals_unsorted || dbg->vals_sorted))
        return fail(RGS_E_CAPACITY, "debug entry buffers hold %lld, frame has %llu",
                    (long long)dbg->entry_capacity, (unsigned long long)hd.n_entries);
    const uint64_t n = h->n_entries;
    if (dbg->keys_unsorted && n) {
        if (h->fl->L.key_bytes == 8)
            HIP_TRY(hipMemcpyAsync(dbg->keys_unsorted, w.keys_a, n * 8, hipMemcpyDeviceToDevice, st));
        else
            launch_widen_keys(st, static_cast<const uint32_t*>(w.keys_a), dbg->keys_unsorted, n);
    }
    if (dbg->vals_unsorted && n)
        HIP_TRY(hipMemcpyAsync(dbg->vals_unsorted, w.vals_a, n * 4, hipMemcpyDeviceToDevice, st));
    return RGS_OK;
}

}  // namespace

static rgs_status render_impl(rgs_ctx* ctx, const rgs_scene* sc, const rgs_camera* cam, int32_t W,
                              int32_t H, int32_t path, void* ws, uint64_t ws_bytes, float* out,
                              rgs_debug_out* dbg, rgs_frame_stats* stats, bool may_time = true) {
    if (!ctx || !sc) return fail(RGS_E_INVALID, "ctx or scene is NULL");
    FrameLaunch fl;
    rgs_status s = prepare_frame(sc, W, H, path, ws, ws_bytes, &fl);
    if (s != RGS_OK) return s;
    s = check_camera(cam);
    if (s != RGS_OK) return s;
    if (!out) return fail(RGS_E_INVALID, "output is NULL");
    fl.sort_fallback = (ctx->debug & RGS_DEBUG_SORT_FALLBACK) != 0;
    HIP_TRY(hipSetDevice(ctx->device));

    DebugDev dd{};
    if (dbg) {
        dd.depth = dbg->depth;
        dd.u = dbg->u;
        dd.v = dbg->v;
        dd.cov2d = dbg->cov2d;
        dd.rect = dbg->rect;
        dd.visible = dbg->visible;
        dd.color = dbg->color;
    }
    hipStream_t st = ctx->stream;
    RenderHooks rh{ctx, nullptr, dbg, &fl, ws, 0};
    if (ctx->timing && may_time) {
        s = next_events(ctx, &rh.fe);
        if (s != RGS_OK) return s;
    }
    FrameHooks hooks{hook_mark, hook_after_front, &rh};
    bool in_b = false;
    const FrameParams prm = frame_params(cam, out, sc, W, H);
    s = enqueue_frame(st, fl, prm, dbg ? &dd : nullptr, dbg != nullptr, nullptr, (rh.fe || dbg) ? &hooks : nullptr,
                      &in_b);
    if (s != RGS_OK) return s;
    s = note_frame(ctx, fl, ws, ws_bytes, sc, prm, W, H, path);
    if (s != RGS_OK) return s;

    if (dbg) {
        const WsDev& w = fl.w;
        const uint64_t n_entries = rh.n_entries;
        const void* ks = in_b ? w.keys_b : w.keys_a;
        const uint32_t* vs = in_b ? w.vals_b : w.vals_a;
        if (dbg->keys_sorted && n_entries) {
            if (fl.L.key_bytes == 8)
                HIP_TRY(hipMemcpyAsync(dbg->keys_sorted, ks, n_entries * 8, hipMemcpyDeviceToDevice, st));
            else
                launch_widen_keys(st, static_cast<const uint32_t*>(ks), dbg->keys_sorted, n_entries);
        }
        if (dbg->vals_sorted && n_entries)
            HIP_TRY(hipMemcpyAsync(dbg->vals_sorted, vs, n_entries * 4, hipMemcpyDeviceToDevice, st));
        if (dbg->ranges)
            HIP_TRY(hipMemcpyAsync(dbg->ranges, w.ranges, (uint64_t)fl.plan.n_tiles * 8,
                                   hipMemcpyDeviceToDevice, st));
        if (dbg->T_final)
            HIP_TRY(hipMemcpyAsync(dbg->T_final, w.t_final, (uint64_t)W * H * 4, hipMemcpyDeviceToDevice, st));
        if (dbg->n_proc)
            HIP_TRY(hipMemcpyAsync(dbg->n_proc, w.n_proc, (uint64_t)W * H * 4, hipMemcpyDeviceToDevice, st));
        if (dbg->n_blend)
            HIP_TRY(hipMemcpyAsync(dbg->n_blend, w.n_blend, (uint64_t)W * H * 4, hipMemcpyDeviceToDevice, st));
        if (dbg->tile_order && fl.f.ordered) {
            HIP_TRY(hipMemcpyAsync(dbg->tile_order, w.order, (uint64_t)fl.plan.n_tiles * 4,
                                   hipMemcpyDeviceToDevice, st));
        } else if (dbg->tile_order) {
            std::vector<uint32_t> rowmajor((size_t)fl.plan.n_tiles);
            for (size_t t = 0; t < rowmajor.size(); ++t) rowmajor[t] = (uint32_t)t;
            HIP_TRY(hipMemcpyAsync(dbg->tile_order, rowmajor.data(), rowmajor.size() * 4, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        HIP_TRY(hipGetLastError());
    }
    if (stats || dbg) {
        WsHeader h;
        s = read_header(ctx, ws, &h);
        if (s != RGS_OK) return s;
        s = header_status(h, stats, sc->n);
        if (s != RGS_OK) return s;
    }
    return ok();
}

extern "C" rgs_status rgs_render(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                                 int32_t width, int32_t height, int32_t path, void* workspace,
                                 uint64_t ws_bytes, float* out_chw, rgs_frame_stats* stats) {
    return render_impl(ctx, scene, cam, width, height, path, workspace, ws_bytes, out_chw, nullptr, stats);
}

extern "C" rgs_status rgs_render_static(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                                        int32_t width, int32_t height, int32_t path, float* out_chw,
                                        rgs_frame_stats* stats) {
    if (!ctx || !scene) return fail(RGS_E_INVALID, "ctx or scene is NULL");
    void* ws = (ctx->device >= 0 && ctx->device < MAX_DEVICES) ? g_scratch_ptr[ctx->device] : nullptr;
    if (!ws) return fail(RGS_E_INVALID, "no static workspace on device %d", ctx->device);
    int64_t cap = 0;
    const rgs_status s = rgs_workspace_capacity(scene->n, width, height, path, STATIC_WS_BYTES, &cap);
    if (s != RGS_OK) return s;
    if (cap < 1)
        return fail(RGS_E_INVALID, "a %dx%d frame of %lld Gaussians needs more than the %llu-byte static workspace",
                    width, height, (long long)scene->n, (unsigned long long)STATIC_WS_BYTES);
    // no stage events: creating them could allocate
    return render_impl(ctx, scene, cam, width, height, path, ws, STATIC_WS_BYTES, out_chw, nullptr, stats, false);
}

extern "C" rgs_status rgs_render_debug(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                                       int32_t width, int32_t height, int32_t path, void* workspace,
                                       uint64_t ws_bytes, float* out_chw, rgs_debug_out* dbg,
                                       rgs_frame_stats* stats) {
    if (!dbg) return fail(RGS_E_INVALID, "rgs_render_debug: dbg is NULL");
    return render_impl(ctx, scene, cam, width, height, path, workspace, ws_bytes, out_chw, dbg, stats);
}

extern "C" rgs_status rgs_workspace_check(rgs_ctx* ctx, const void* workspace, rgs_frame_stats* stats,
                                          int64_t n_gaussians) {
    if (!ctx || !workspace) return fail(RGS_E_INVALID, "ctx or workspace is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    WsHeader h;
    rgs_status s = read_header(ctx, workspace, &h);
    if (s != RGS_OK) return s;
    s = header_status(h, stats, n_gaussians);
    return s == RGS_OK ? ok() : s;
}

extern "C" rgs_status rgs_scene_update_plain(rgs_ctx* ctx, rgs_scene* sc, const rgs_device_params* p) {
    if (!ctx || !sc || !p) return fail(RGS_E_INVALID, "rgs_scene_update_plain: NULL argument");
    if (!(sc->formats & RGS_FMT_PLAIN)) return fail(RGS_E_INVALID, "scene has no plain format");
    if (p->n != sc->n)
        return fail(RGS_E_INVALID, "params hold %lld Gaussians, the scene %lld", (long long)p->n, (long long)sc->n);
    if (!p->means || !p->scales || !p->quats || !p->opacity || !p->sh)
        return fail(RGS_E_INVALID, "rgs_scene_update_plain: NULL parameter pointer");
    HIP_TRY(hipSetDevice(ctx->device));
    launch_update_plain(ctx->stream, sc->plain, sc->n_pad, sc->n, p->means, p->scales, p->quats, p->opacity,
                        p->sh);
    HIP_TRY(hipGetLastError());
    sc->tag = next_scene_tag();
    return ok();
}

static constexpr uint64_t PARTIAL_BYTES = 48;   // three float4 per sorted entry

extern "C" rgs_status rgs_backward_scratch_size(int64_t n, int32_t width, int32_t height, uint64_t ws_bytes,
                                                uint64_t* bytes) {
    if (!bytes) return fail(RGS_E_INVALID, "bytes is NULL");
    if (n < 1 || n > RGS_MAX_ENTRIES) return fail(RGS_E_INVALID, "n = %lld out of range", (long long)n);
    rgs_plan p;
    rgs_status s = rgs_frame_plan(width, height, &p);
    if (s != RGS_OK) return s;
    const uint64_t cap = capacity_for(n, p, RGS_PATH_PLAIN, ws_bytes);
    if (cap == 0) return fail(RGS_E_INVALID, "workspace of %llu bytes is too small", (unsigned long long)ws_bytes);
    *bytes = align256(cap * PARTIAL_BYTES);
    return ok();
}

extern "C" rgs_status rgs_render_backward(rgs_ctx* ctx, const rgs_scene* scene, const rgs_camera* cam,
                                          int32_t width, int32_t height, const float* dL_dimg,
                                          void* workspace, uint64_t ws_bytes, rgs_grads* grads) {
    if (!ctx || !scene || !grads || !dL_dimg) return fail(RGS_E_INVALID, "rgs_render_backward: NULL argument");
    if (!grads->d_means || !grads->d_scales || !grads->d_quats || !grads->d_opacity || !grads->d_sh ||
        !grads->scratch)
        return fail(RGS_E_INVALID, "rgs_render_backward: NULL gradient or scratch pointer");
    if (reinterpret_cast<uintptr_t>(grads->scratch) % 256 != 0)
        return fail(RGS_E_INVALID, "scratch must be 256-byte aligned");
    FrameLaunch fl;
    rgs_status s = prepare_frame(scene, width, height, RGS_PATH_PLAIN, workspace, ws_bytes, &fl);
    if (s != RGS_OK) return s;
    s = check_camera(cam);
    if (s != RGS_OK) return s;
    if (grads->scratch_bytes < fl.L.capacity * PARTIAL_BYTES)
        return fail(RGS_E_INVALID, "scratch of %llu bytes, need %llu", (unsigned long long)grads->scratch_bytes,
                    (unsigned long long)(fl.L.capacity * PARTIAL_BYTES));
    HIP_TRY(hipSetDevice(ctx->device));
    const uint64_t hash = camera_hash(cam, width, height);
    static const char* const STALE_SCENE = "the workspace's last frame is not a render of this scene in its current "
                                           "state (another scene, or its parameters were updated since)";
    static const char* const STALE_CAMERA = "the workspace's last frame was rendered with another camera or size";
    uint32_t path_word = 0;
    int slot = -1;
    for (int i = 0; i < N_FRAME_RECORDS; ++i)
        if (ctx->records[i].ws == workspace) slot = i;
    const FrameRecord* r = slot >= 0 ? &ctx->records[slot] : nullptr;
    if (r && r->ws_bytes == ws_bytes && r->width == width && r->height == height && r->scene == scene &&
        r->scene_tag == scene->tag && r->cam_hash == hash) {
        // the last frame this context rendered into the workspace is the one
        // asked for: its stamp tells the outcome without a device read (and the
        // kernels check that no other context rendered into it since)
        FrameStamp st;
        s = wait_stamp(ctx, slot, &st);
        if (s != RGS_OK) return s;
        WsHeader h{};
        h.n_entries = st.n_entries;
        h.overflow = st.overflow;
        h.error = st.error;
        h.capacity = fl.f.capacity;
        s = header_status(h, nullptr, scene->n);
        if (s != RGS_OK) return s;
        path_word = (uint32_t)r->path;
    } else {                        // otherwise the workspace itself is asked
        WsHeader h;
        s = read_header(ctx, workspace, &h);
        if (s != RGS_OK) return s;
        if ((h.path != (uint32_t)RGS_PATH_PLAIN && h.path != (uint32_t)(RGS_PATH_PLAIN | RGS_HW_EXP2)) ||
            h.capacity != fl.f.capacity || h.passes != fl.L.passes)
            return fail(RGS_E_INVALID, "the workspace does not hold a plain render of this size");
        FrameParams prm;
        HIP_TRY(hipMemcpyAsync(&prm, static_cast<const char*>(workspace) + fl.L.params, sizeof(prm),
                               hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        if (prm.scene_tag != scene->tag) return fail(RGS_E_INVALID, "%s", STALE_SCENE);
        if (prm.cam_hash != hash) return fail(RGS_E_INVALID, "%s", STALE_CAMERA);
        s = header_status(h, nullptr, scene->n);
        if (s != RGS_OK) return s;
        path_word = h.path;
    }
    if (path_word != (uint32_t)RGS_PATH_PLAIN && path_word != (uint32_t)(RGS_PATH_PLAIN | RGS_HW_EXP2))
        return fail(RGS_E_INVALID, "the workspace does not hold a plain render of this size");
    const bool in_b = (fl.L.passes % 2) == 1;
    float4* partial = static_cast<float4*>(grads->scratch);
    const bool train = (path_word & RGS_HW_EXP2) != 0;
    const FrameKey key{scene->tag, hash};
    if (train) launch_raster_backward_train(ctx->stream, fl.f, fl.w, in_b, dL_dimg, partial, key);
    else launch_raster_backward(ctx->stream, fl.f, fl.w, in_b, dL_dimg, partial, key);
    GradOut go{grads->d_means, grads->d_scales, grads->d_quats, grads->d_opacity, grads->d_sh, grads->d_screen};
    launch_grad_gaussian(ctx->stream, fl.plain, cam_dev(cam), fl.w, partial, go, train, key);
    HIP_TRY(hipGetLastError());
    return ok();
}
