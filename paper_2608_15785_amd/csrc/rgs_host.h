// Host-side pieces shared by the render entry points and the request server:
// error reporting, argument checks and the launch sequence of one frame.
#pragma once

#include <hip/hip_runtime.h>

#include "rgs.h"
#include "rgs_internal.h"

namespace rgs {

// Sets the calling thread's last-error text and returns s.
rgs_status fail(rgs_status s, const char* fmt, ...);
// Clears the last-error text and returns RGS_OK.
rgs_status ok();

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::rgs::fail(e_ == hipErrorOutOfMemory ? RGS_E_OOM : RGS_E_HIP, "%s: %s", \
                               #expr, hipGetErrorString(e_));                               \
    } while (0)

// Everything about a frame that is fixed by the scene, the resolution, the
// path and the workspace: layout, device pointers and kernel constants.
struct FrameLaunch {
    int device;
    int64_t n;
    int32_t path;        // RGS_PATH_PLAIN or RGS_PATH_FAST
    uint32_t opts;       // ablation bits of the fast path (OPT_*)
    uint32_t path_word;  // the path argument as given, kept in the workspace header
    rgs_plan plan;
    WsLayout L;
    WsDev w;
    FrameDev f;
    PlainSceneDev plain;
    FastSceneDev fast;
    bool sort_fallback = false;   // RGS_DEBUG_SORT_FALLBACK of the rendering context
};

// Checks the scene, resolution, path and workspace and fills fl (no GPU work).
rgs_status prepare_frame(const rgs_scene* sc, int32_t width, int32_t height, int32_t path, void* ws,
                         uint64_t ws_bytes, FrameLaunch* fl);
rgs_status check_camera(const rgs_camera* c);
// A `path` argument: RGS_PATH_PLAIN, or RGS_PATH_FAST with ablation and extension bits.
rgs_status check_path(int32_t path);
// The frame parameters of a render of scene sc with camera c at W x H into out.
FrameParams frame_params(const rgs_camera* c, float* out, const rgs_scene* sc, int32_t width, int32_t height);
int scene_device(const rgs_scene* sc);

// Optional instrumentation of enqueue_frame: mark(user, k) after stage k's
// launches (k = 0 before the first), after_front(user) between the front end
// and the sort (it may read the header; a non-OK status stops the frame).
struct FrameHooks {
    // stage boundary k reached (0..RGS_N_STAGES); -k: this path has no boundary k
    void (*mark)(void* user, int k);
    rgs_status (*after_front)(void* user);
    void* user;
};

// Enqueues reset, front end, sort, ranges and raster of one frame on st.  With
// status set, a last kernel copies the header's outcome to that host-visible
// address.  *result_in_b tells which key/value buffer holds the sorted result.
rgs_status enqueue_frame(hipStream_t st, const FrameLaunch& fl, const FrameParams& prm,
                         const DebugDev* dbg, bool count, FrameStatus* status, const FrameHooks* hooks,
                         bool* result_in_b);

}  // namespace rgs
