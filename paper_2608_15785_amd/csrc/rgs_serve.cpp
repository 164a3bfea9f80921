// Request server: continuous batching of view requests over resident scenes.
//
// Frame slots (one HIP stream each) run admitted frames concurrently; a frame
// renders in a workspace of its (scene, resolution, path) class drawn from a
// pool held within a byte budget.  With graphs enabled each workspace carries a
// captured graph of its frame; a request replays it after the reset node's
// argument block is rewritten with the request's camera and output pointer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "rgs.h"
#include "rgs_host.h"
#include "rgs_internal.h"

using namespace rgs;

namespace {

constexpr int MAX_STREAMS = 16;
constexpr uint64_t MIN_ENTRIES = 65536;
constexpr double DEFAULT_ENTRIES_PER_GAUSSIAN = 4.0;
constexpr double GROWTH = 1.25;      // headroom over a frame's entry count after an overflow

struct ClassKey {
    const rgs_scene* scene;
    int32_t width, height, path;
    bool operator==(const ClassKey& o) const {
        return scene == o.scene && width == o.width && height == o.height && path == o.path;
    }
};

struct Workspace {
    ClassKey key{};
    void* mem = nullptr;
    uint64_t bytes = 0;
    uint64_t entries = 0;
    FrameLaunch fl{};
    FrameStatus* status = nullptr;           // host-visible, written by the frame's last kernel
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t reset_node = nullptr;
    hipKernelNodeParams reset_params{};
    bool busy = false;
    uint64_t last_used = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int64_t req = -1;
    Workspace* ws = nullptr;
};

struct ClassNeed {
    ClassKey key;
    uint64_t entries;
};

}  // namespace

struct rgs_server {
    int device = 0;
    rgs_server_config cfg{};
    std::vector<Slot> slots;
    std::vector<std::unique_ptr<Workspace>> pool;
    std::vector<ClassNeed> needs;
    uint64_t held = 0, peak = 0, tick = 0;
    hipEvent_t ev0 = nullptr;
    int32_t n_captured = 0, n_evicted = 0;
};

namespace {

int64_t scene_size(const rgs_scene* sc) {
    int64_t n = 0;
    uint32_t formats = 0;
    uint64_t bytes = 0;
    rgs_scene_info(sc, &n, &formats, &bytes);
    return n;
}

uint64_t& need_of(rgs_server* s, const ClassKey& k) {
    for (auto& c : s->needs)
        if (c.key == k) return c.entries;
    const double per = s->cfg.entries_per_gaussian > 0.0 ? s->cfg.entries_per_gaussian
                                                         : DEFAULT_ENTRIES_PER_GAUSSIAN;
    const uint64_t e = std::max<uint64_t>(MIN_ENTRIES, (uint64_t)std::ceil(per * (double)scene_size(k.scene)));
    s->needs.push_back(ClassNeed{k, std::min<uint64_t>(e, RGS_MAX_ENTRIES)});
    return s->needs.back().entries;
}

uint64_t class_bytes(const ClassKey& k, uint64_t entries) {
    uint64_t b = 0;
    if (rgs_workspace_size(scene_size(k.scene), k.width, k.height, k.path, (int64_t)entries, &b) != RGS_OK)
        return 0;
    return b;
}

void release(rgs_server* s, Workspace* w) {
    if (w->exec) (void)hipGraphExecDestroy(w->exec);
    if (w->graph) (void)hipGraphDestroy(w->graph);
    if (w->mem) (void)hipFree(w->mem);
    if (w->status) (void)hipHostFree(w->status);
    s->held -= w->bytes;
    for (size_t i = 0; i < s->pool.size(); ++i)
        if (s->pool[i].get() == w) {
            s->pool.erase(s->pool.begin() + (ptrdiff_t)i);
            break;
        }
}

// Records the frame of workspace w as a graph and finds its reset node.  The
// graph is recorded with the parameters of the request that first needs it, so
// that its baked arguments name real buffers.
rgs_status capture(rgs_server* s, Workspace* w, const FrameParams& first, hipStream_t st) {
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rgs_status es = enqueue_frame(st, w->fl, first, nullptr, false, w->status, nullptr, nullptr);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &g);
    if (es != RGS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return es;
    }
    if (ce != hipSuccess || !g)
        return fail(RGS_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
    w->graph = g;
    size_t count = 0;
    HIP_TRY(hipGraphGetNodes(g, nullptr, &count));
    std::vector<hipGraphNode_t> nodes(count);
    HIP_TRY(hipGraphGetNodes(g, nodes.data(), &count));
    for (size_t i = 0; i < count && !w->reset_node; ++i) {
        hipGraphNodeType type;
        HIP_TRY(hipGraphNodeGetType(nodes[i], &type));
        if (type != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams p{};
        HIP_TRY(hipGraphKernelNodeGetParams(nodes[i], &p));
        if (p.func == reset_kernel()) {
            w->reset_node = nodes[i];
            w->reset_params = p;
        }
    }
    if (!w->reset_node) return fail(RGS_E_HIP, "captured frame has no reset node");
    HIP_TRY(hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0));
    s->n_captured += 1;
    return RGS_OK;
}

rgs_status create_workspace(rgs_server* s, const ClassKey& k, uint64_t entries, uint64_t bytes,
                            const FrameParams& first, hipStream_t st, Workspace** out) {
    auto w = std::make_unique<Workspace>();
    w->key = k;
    w->entries = entries;
    w->bytes = bytes;
    HIP_TRY(hipMalloc(&w->mem, bytes));
    s->held += bytes;
    s->peak = std::max(s->peak, s->held);
    Workspace* raw = w.get();
    s->pool.push_back(std::move(w));
    void* host = nullptr;
    hipError_t e = hipHostMalloc(&host, sizeof(FrameStatus), hipHostMallocCoherent);
    if (e != hipSuccess) {
        release(s, raw);
        return fail(RGS_E_OOM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    raw->status = static_cast<FrameStatus*>(host);
    rgs_status r = prepare_frame(k.scene, k.width, k.height, k.path, raw->mem, bytes, &raw->fl);
    if (r == RGS_OK && s->cfg.use_graphs) r = capture(s, raw, first, st);
    if (r != RGS_OK) {
        release(s, raw);
        return r;
    }
    *out = raw;
    return RGS_OK;
}

// An idle workspace for class k, allocated within the budget if need be.
// *out stays NULL when the request has to wait for memory.
rgs_status acquire(rgs_server* s, const ClassKey& k, const FrameParams& first, hipStream_t st,
                   Workspace** out) {
    *out = nullptr;
    const uint64_t entries = need_of(s, k);
    for (size_t i = 0; i < s->pool.size();) {
        Workspace* w = s->pool[i].get();
        if (!w->busy && w->key == k) {
            if (w->entries >= entries) {
                *out = w;
                return RGS_OK;
            }
            release(s, w);          // too small since the class grew
            continue;
        }
        ++i;
    }
    const uint64_t bytes = class_bytes(k, entries);
    if (bytes == 0) return fail(RGS_E_INVALID, "no workspace size for this request");
    if (bytes > s->cfg.mem_budget)
        return fail(RGS_E_OOM, "one workspace needs %llu bytes, the budget is %llu",
                    (unsigned long long)bytes, (unsigned long long)s->cfg.mem_budget);
    while (s->held + bytes > s->cfg.mem_budget) {
        Workspace* lru = nullptr;
        for (auto& p : s->pool)
            if (!p->busy && (!lru || p->last_used < lru->last_used)) lru = p.get();
        if (!lru) return RGS_OK;    // wait for a frame to finish
        release(s, lru);
        s->n_evicted += 1;
    }
    return create_workspace(s, k, entries, bytes, first, st, out);
}

rgs_status launch(rgs_server* s, Slot& slot, Workspace* w, const rgs_request& r) {
    w->status->done = 0;
    const FrameParams prm = frame_params(&r.camera, r.out_chw, r.scene, r.width, r.height);
    if (w->exec) {
        ResetArgs ra = reset_args(w->fl.w, w->fl.L.zero_end, w->fl.f, w->fl.path_word, prm);
        void* args[] = {&ra};
        hipKernelNodeParams np = w->reset_params;
        np.kernelParams = args;
        np.extra = nullptr;
        HIP_TRY(hipGraphExecKernelNodeSetParams(w->exec, w->reset_node, &np));
        HIP_TRY(hipGraphLaunch(w->exec, slot.stream));
    } else {
        rgs_status e = enqueue_frame(slot.stream, w->fl, prm, nullptr, false, w->status, nullptr, nullptr);
        if (e != RGS_OK) return e;
    }
    HIP_TRY(hipEventRecord(slot.done, slot.stream));
    w->busy = true;
    w->last_used = ++s->tick;
    slot.ws = w;
    return RGS_OK;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

rgs_status check_request(const rgs_server* s, const rgs_request& r, double prev_arrival) {
    if (!r.scene) return fail(RGS_E_INVALID, "request scene is NULL");
    if (scene_device(r.scene) != s->device)
        return fail(RGS_E_INVALID, "request scene lives on device %d, the server on %d",
                    scene_device(r.scene), s->device);
    if (!r.out_chw) return fail(RGS_E_INVALID, "request output is NULL");
    if (!(std::isfinite(r.arrival) && r.arrival >= prev_arrival))
        return fail(RGS_E_INVALID, "arrivals must be finite, >= 0 and non-decreasing");
    const int32_t base = r.path & 0xff;
    if (check_path(r.path) != RGS_OK) return fail(RGS_E_INVALID, "bad path 0x%x", r.path);
    int64_t n = 0;
    uint32_t formats = 0;
    uint64_t bytes = 0;
    rgs_scene_info(r.scene, &n, &formats, &bytes);
    if (!(formats & (base == RGS_PATH_PLAIN ? RGS_FMT_PLAIN : RGS_FMT_FAST)))
        return fail(RGS_E_INVALID, "request scene lacks the format of its path");
    rgs_plan p;
    rgs_status e = rgs_frame_plan(r.width, r.height, &p);
    if (e != RGS_OK) return e;
    return check_camera(&r.camera);
}

}  // namespace

extern "C" rgs_status rgs_server_create(const rgs_server_config* cfg, rgs_server** out) {
    if (!cfg || !out) return fail(RGS_E_INVALID, "rgs_server_create: NULL argument");
    *out = nullptr;
    if (cfg->n_streams < 1 || cfg->n_streams > MAX_STREAMS)
        return fail(RGS_E_INVALID, "n_streams must be in [1, %d]", MAX_STREAMS);
    if (cfg->mem_budget == 0) return fail(RGS_E_INVALID, "mem_budget is 0");
    if (!(cfg->entries_per_gaussian >= 0.0 && std::isfinite(cfg->entries_per_gaussian)))
        return fail(RGS_E_INVALID, "entries_per_gaussian must be finite and >= 0");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(RGS_E_NODEVICE, "no HIP device available");
    if (cfg->device < 0 || cfg->device >= count)
        return fail(RGS_E_INVALID, "device %d outside [0, %d)", cfg->device, count);
    HIP_TRY(hipSetDevice(cfg->device));
    auto s = std::make_unique<rgs_server>();
    s->device = cfg->device;
    s->cfg = *cfg;
    s->slots.resize((size_t)cfg->n_streams);
    for (auto& sl : s->slots) {
        HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreate(&sl.done));
    }
    HIP_TRY(hipEventCreate(&s->ev0));
    *out = s.release();
    return ok();
}

extern "C" void rgs_server_destroy(rgs_server* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    for (auto& sl : s->slots)
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    while (!s->pool.empty()) release(s, s->pool.back().get());
    for (auto& sl : s->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    delete s;
}

extern "C" rgs_status rgs_serve(rgs_server* s, const rgs_request* reqs, int64_t n, rgs_response* resp,
                                rgs_server_stats* stats) {
    if (!s || (n > 0 && (!reqs || !resp)) || n < 0) return fail(RGS_E_INVALID, "rgs_serve: bad arguments");
    double prev = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        rgs_status e = check_request(s, reqs[i], prev);
        if (e != RGS_OK) return fail(e, "request %lld: %s", (long long)i, rgs_last_error());
        prev = reqs[i].arrival;
    }
    HIP_TRY(hipSetDevice(s->device));
    for (int64_t i = 0; i < n; ++i) {
        resp[i] = rgs_response{};
        resp[i].status = RGS_E_INVALID;
        resp[i].slot = -1;
    }
    const int32_t captured0 = s->n_captured, evicted0 = s->n_evicted;
    s->peak = s->held;

    HIP_TRY(hipEventRecord(s->ev0, s->slots[0].stream));
    HIP_TRY(hipEventSynchronize(s->ev0));
    const auto t0 = std::chrono::steady_clock::now();

    std::deque<int64_t> queue;
    int64_t next = 0, finished = 0;
    int32_t in_flight = 0, max_in_flight = 0;
    rgs_status fatal = RGS_OK;
    while (finished < n && fatal == RGS_OK) {
        bool progress = false;
        const double now = seconds_since(t0);
        while (next < n && reqs[next].arrival <= now) queue.push_back(next++);

        for (auto& sl : s->slots) {
            if (sl.req < 0) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                fatal = fail(RGS_E_HIP, "hipEventQuery: %s", hipGetErrorString(q));
                break;
            }
            rgs_response& rp = resp[sl.req];
            const rgs_request& r = reqs[sl.req];
            Workspace* w = sl.ws;
            rp.n_entries = (int64_t)w->status->n_entries;
            rp.status = RGS_OK;
            if (!w->status->done) rp.status = fail(RGS_E_HIP, "frame status was not written");
            else if (w->status->out != reinterpret_cast<uint64_t>(r.out_chw))
                rp.status = fail(RGS_E_HIP, "frame ran with another request's parameters");
            else if (w->status->error) rp.status = fail(RGS_E_DEVICE, "bounded wait gave up (0x%x)", w->status->error);
            else if (w->status->overflow) {
                // The frame needed more entries than its workspace holds.  Its
                // class grows to the frame's count plus headroom, and the
                // request goes back to the head of the queue: it is admitted
                // again like any other, in a workspace of the grown class that
                // acquire() obtains within the budget, while the other slots'
                // frames keep running.  The count is exact even on overflow, so
                // the second render fits unless the class is at the largest
                // capacity already.
                if (rp.retried || w->entries >= RGS_MAX_ENTRIES) {
                    rp.status = fail(RGS_E_CAPACITY, "the frame needs %llu entries, more than its workspace of "
                                     "%llu", (unsigned long long)w->status->n_entries,
                                     (unsigned long long)w->entries);
                } else {
                    uint64_t& need = need_of(s, w->key);
                    const uint64_t want = std::min<uint64_t>(
                        RGS_MAX_ENTRIES, (uint64_t)std::ceil(GROWTH * (double)w->status->n_entries));
                    need = std::max(need, want);
                    rp.retried = 1;
                    queue.push_front(sl.req);
                    w->busy = false;
                    sl.req = -1;
                    sl.ws = nullptr;
                    --in_flight;
                    progress = true;
                    continue;
                }
            }
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, s->ev0, sl.done) == hipSuccess) rp.t_done = ms * 1e-3;
            else rp.t_done = seconds_since(t0);
            rp.latency = rp.t_done - r.arrival;
            w->busy = false;
            sl.req = -1;
            sl.ws = nullptr;
            --in_flight;
            ++finished;
            progress = true;
        }
        if (fatal != RGS_OK) break;

        while (!queue.empty()) {
            Slot* free_slot = nullptr;
            int32_t slot_id = 0;
            for (auto& sl : s->slots) {
                if (sl.req < 0) {
                    free_slot = &sl;
                    break;
                }
                ++slot_id;
            }
            if (!free_slot) break;
            const int64_t i = queue.front();
            const rgs_request& r = reqs[i];
            const ClassKey k{r.scene, r.width, r.height, r.path};
            Workspace* w = nullptr;
            rgs_status e = acquire(s, k, frame_params(&r.camera, r.out_chw, r.scene, r.width, r.height),
                                   free_slot->stream, &w);
            if (e != RGS_OK) {             // this request cannot run at all
                resp[i].status = e;
                resp[i].t_done = resp[i].t_admit = seconds_since(t0);
                queue.pop_front();
                ++finished;
                progress = true;
                continue;
            }
            if (!w) break;                 // wait for memory
            resp[i].t_admit = seconds_since(t0);
            resp[i].slot = slot_id;
            resp[i].graph = w->exec != nullptr;
            e = launch(s, *free_slot, w, r);
            if (e != RGS_OK) {
                fatal = e;
                break;
            }
            free_slot->req = i;
            queue.pop_front();
            ++in_flight;
            max_in_flight = std::max(max_in_flight, in_flight);
            progress = true;
        }
        if (!progress && in_flight == 0 && queue.empty() && next < n) {
            // idle until the next arrival: sleep through most of the gap
            const double gap = reqs[next].arrival - seconds_since(t0);
            if (gap > 5e-4) std::this_thread::sleep_for(std::chrono::duration<double>(gap - 3e-4));
        }
    }
    for (auto& sl : s->slots) (void)hipStreamSynchronize(sl.stream);
    if (fatal != RGS_OK) {
        for (auto& sl : s->slots) {
            if (sl.ws) sl.ws->busy = false;
            sl.req = -1;
            sl.ws = nullptr;
        }
        return fatal;
    }
    if (stats) {
        double wall = 0.0, busy = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            wall = std::max(wall, resp[i].t_done);
            if (resp[i].status == RGS_OK) busy += std::max(0.0, resp[i].t_done - resp[i].t_admit);
        }
        stats->wall = wall;
        stats->ws_bytes_held = s->held;
        stats->ws_bytes_peak = s->peak;
        stats->n_workspaces = (int32_t)s->pool.size();
        stats->n_captured = s->n_captured - captured0;
        stats->n_evicted = s->n_evicted - evicted0;
        stats->max_in_flight = max_in_flight;
        stats->mean_in_flight = wall > 0.0 ? busy / wall : 0.0;
    }
    return ok();
}
