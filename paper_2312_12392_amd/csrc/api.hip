// C ABI of the renderer: argument validation, error reporting, dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "rcp_internal.hpp"

namespace rcp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

rcp_status hip_status(hipError_t e, const char* what, const char* file, int line) {
    set_error("%s: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? RCP_ERR_OUT_OF_MEMORY : RCP_ERR_DEVICE;
}

namespace {
// The current device has memory pools (the stream-ordered allocator); asked
// once per device.
bool pools_supported() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    static std::mutex mu;
    static std::map<int, bool> cache;
    std::lock_guard<std::mutex> lk(mu);
    const auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int v = 0;
    const bool ok = hipDeviceGetAttribute(&v, hipDeviceAttributeMemoryPoolsSupported, dev) == hipSuccess && v != 0;
    cache[dev] = ok;
    return ok;
}

// Test hooks (rcp_debug_set): allocations left before every later one
// fails (-1: off), and the traversal step budget of scenes built afterwards.
std::atomic<long long> g_alloc_left{-1};
std::atomic<uint32_t> g_step_budget{0};
std::atomic<int> g_list_canary{0};

}  // namespace

bool alloc_hook_fails() {
    long long left = g_alloc_left.load();
    while (left >= 0) {
        if (left == 0) return true;
        if (g_alloc_left.compare_exchange_weak(left, left - 1)) return false;
    }
    return false;
}

uint32_t debug_step_budget() { return g_step_budget.load(); }

int debug_list_canary() { return g_list_canary.load(); }

rcp_status dev_alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return RCP_OK;
    if (alloc_hook_fails()) {
        set_error("device allocation of %zu bytes failed (test hook)", bytes);
        return RCP_ERR_OUT_OF_MEMORY;
    }
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_status(e, "hipMalloc", __FILE__, __LINE__);
    }
    return RCP_OK;
}

rcp_status stream_alloc(void** p, size_t bytes, hipStream_t stream) {
    *p = nullptr;
    if (bytes == 0) return RCP_OK;
    if (alloc_hook_fails()) {
        set_error("device allocation of %zu bytes failed (test hook)", bytes);
        return RCP_ERR_OUT_OF_MEMORY;
    }
    const hipError_t e = pools_supported() ? hipMallocAsync(p, bytes, stream) : hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_status(e, "device allocation", __FILE__, __LINE__);
    }
    return RCP_OK;
}

void stream_free(void* p, hipStream_t stream) {
    if (!p) return;
    if (pools_supported()) (void)hipFreeAsync(p, stream);
    else (void)hipFree(p);
}

rcp_status take_device_error(rcp_scene* s) {
    const uint32_t e = s->err_host ? __atomic_exchange_n(s->err_host, 0u, __ATOMIC_ACQ_REL) : 0u;
    if (e == kErrListCanary) {
        set_error("a list of continuing pixels failed its canary check (an entry below the list's count left "
                  "unwritten or invalid, or one above it overwritten)");
        return RCP_ERR_INTERNAL;
    }
    if (e == kErrLdsLayout) {
        set_error("the chain kernel's dynamic LDS does not start at address 0, where the traversal reads the "
                  "staged BVH levels: nothing was rendered");
        return RCP_ERR_INTERNAL;
    }
    if (e != 0u) {
        set_error("a ray ran out of its traversal step budget (%u steps): the BVH is malformed, and that ray's "
                  "result is a miss", s->dev.step_budget);
        return RCP_ERR_INTERNAL;
    }
    return RCP_OK;
}

}  // namespace rcp

using namespace rcp;

#define FAIL(...) do { set_error(__VA_ARGS__); return RCP_ERR_INVALID_ARGUMENT; } while (0)

namespace {

bool finite_n(const float* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace

namespace rcp {

// Argument checks shared by the entry points (declared in rcp_internal.hpp).

rcp_status check_camera(const rcp_camera* c, Camera& out) {
    if (!c) FAIL("camera is NULL");
    if (!finite_n(c->eye, 3) || !finite_n(c->right, 3) || !finite_n(c->up, 3) || !finite_n(c->forward, 3) ||
        !std::isfinite(c->tan_half_fovy))
        FAIL("camera has a non-finite value");
    if (!(c->tan_half_fovy > 0.0f)) FAIL("camera tan_half_fovy must be > 0");
    const float* b[3] = {c->right, c->up, c->forward};
    for (int i = 0; i < 3; ++i) {
        double n = std::sqrt((double)b[i][0] * b[i][0] + (double)b[i][1] * b[i][1] + (double)b[i][2] * b[i][2]);
        if (std::fabs(1.0 - n) > 1e-5) FAIL("camera basis vector %d is not unit length (|v| = %.9g)", i, n);
        for (int j = i + 1; j < 3; ++j) {
            double d = (double)b[i][0] * b[j][0] + (double)b[i][1] * b[j][1] + (double)b[i][2] * b[j][2];
            if (std::fabs(d) > 1e-5) FAIL("camera basis vectors %d and %d are not orthogonal", i, j);
        }
    }
    for (int a = 0; a < 3; ++a) {
        out.eye[a] = c->eye[a];
        out.right[a] = c->right[a];
        out.up[a] = c->up[a];
        out.forward[a] = c->forward[a];
    }
    out.th = c->tan_half_fovy;
    return RCP_OK;
}

rcp_status check_disp(const rcp_displacement* d) {
    if (!d) FAIL("displacement is NULL");
    if (!std::isfinite(d->lambda_eye) || !std::isfinite(d->lambda_dir)) FAIL("displacement lambda is not finite");
    if (d->lambda_eye < 0.0f) FAIL("lambda_eye must be >= 0");
    if (!(d->lambda_dir >= 0.0f && d->lambda_dir < 1.0f)) FAIL("lambda_dir must be in [0, 1)");
    if (d->mode != RCP_MODE_COLOR && d->mode != RCP_MODE_DEPTH && d->mode != RCP_MODE_NORMAL)
        FAIL("unknown displacement mode %d", (int)d->mode);
    if (!std::isfinite(d->z0)) FAIL("z0 is not finite");
    return RCP_OK;
}

rcp_status check_size(int W, int H) {
    if (W < 1 || H < 1) FAIL("image size %dx%d: W and H must be >= 1", W, H);
    if ((long long)W * (long long)H > (1ll << 27)) FAIL("image size %dx%d exceeds 2^27 pixels", W, H);
    return RCP_OK;
}

rcp_status check_scene(const rcp_scene* s) {
    if (!s) FAIL("scene is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return RCP_ERR_DEVICE;
    }
    if (dev != s->device) FAIL("scene lives on device %d but the current device is %d", s->device, dev);
    return RCP_OK;
}

}  // namespace rcp

extern "C" {

const char* rcp_status_string(rcp_status s) {
    // A C caller may pass any int; reading it through the enum type would be
    // undefined in C++ for values outside the enumerators' range.
    int v;
    static_assert(sizeof v == sizeof s, "rcp_status is int-sized");
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
        case RCP_OK: return "ok";
        case RCP_ERR_INVALID_ARGUMENT: return "invalid argument";
        case RCP_ERR_OUT_OF_MEMORY: return "out of memory";
        case RCP_ERR_DEVICE: return "device error";
        case RCP_ERR_NOT_READY: return "not ready";
        case RCP_ERR_QUEUE_FULL: return "queue full";
        case RCP_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* rcp_last_error(void) { return g_err; }

rcp_status rcp_build_scene(const rcp_scene_desc* desc, const rcp_build_options* opts, void* hip_stream,
                           rcp_scene** out) {
    clear_error();
    if (out) *out = nullptr;
    if (!desc || !out) FAIL("desc and out must not be NULL");
    if (desc->n_tris > kMaxTris - 8) FAIL("n_tris %u exceeds the limit %u", desc->n_tris, kMaxTris - 8);
    if (!finite_n(desc->light_dir, 3) || !finite_n(desc->background, 3) || !std::isfinite(desc->k_a) ||
        !std::isfinite(desc->k_d))
        FAIL("light, shading weights and background must be finite");
    if (desc->n_tris > 0) {
        if (!desc->verts || !desc->idx || !desc->tri_rgb) FAIL("verts, idx and tri_rgb must not be NULL");
        if (desc->n_verts == 0) FAIL("n_verts is 0 but n_tris > 0");
        for (size_t i = 0; i < 3 * (size_t)desc->n_tris; ++i)
            if (desc->idx[i] >= desc->n_verts)
                FAIL("idx[%zu] = %u is out of range (n_verts = %u)", i, desc->idx[i], desc->n_verts);
        for (size_t i = 0; i < 3 * (size_t)desc->n_verts; ++i)
            if (!std::isfinite(desc->verts[i])) FAIL("vertex coordinate %zu is not finite", i);
        for (size_t i = 0; i < 3 * (size_t)desc->n_tris; ++i)
            if (!std::isfinite(desc->tri_rgb[i])) FAIL("tri_rgb[%zu] is not finite", i);
    }
    if (opts) {
        if (opts->max_leaf < 1 || opts->max_leaf > kMaxLeaf) FAIL("max_leaf must be in [1, %d]", kMaxLeaf);
        if (!(opts->c_trav > 0.0f) || !(opts->c_isect > 0.0f) || !std::isfinite(opts->c_trav) ||
            !std::isfinite(opts->c_isect))
            FAIL("SAH costs must be finite and > 0");
        if (opts->builder != RCP_BUILDER_PLOC && opts->builder != RCP_BUILDER_LBVH)
            FAIL("unknown builder %d", (int)opts->builder);
        if (opts->collapse != RCP_COLLAPSE_SAH && opts->collapse != RCP_COLLAPSE_GREEDY)
            FAIL("unknown collapse %d", (int)opts->collapse);
    }
    rcp_status st;
    try {
        st = build_scene(desc, opts, (hipStream_t)hip_stream, out);
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return RCP_ERR_OUT_OF_MEMORY;
    }
    const char* log = std::getenv("RCP_LOG");
    if (st == RCP_OK && log && std::strcmp(log, "1") == 0) {
        const rcp_scene_stats& t = (*out)->stats;
        std::fprintf(stderr,
                     "rcp: scene built: %u triangles, %u nodes, %u leaves, depth %u, max_leaf %u, SAH %.4f, "
                     "%.3f ms, %llu device bytes; leaves by triangle count 1..8: %u %u %u %u %u %u %u %u\n",
                     t.n_tris, t.n_nodes, t.n_leaves, t.max_depth, t.max_leaf, (double)t.sah_cost,
                     (double)t.build_ms, (unsigned long long)t.device_bytes, t.leaf_hist[0], t.leaf_hist[1],
                     t.leaf_hist[2], t.leaf_hist[3], t.leaf_hist[4], t.leaf_hist[5], t.leaf_hist[6],
                     t.leaf_hist[7]);
    }
    return st;
}

void rcp_destroy_scene(rcp_scene* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    if (s->nodes) (void)hipFree(s->nodes);
    if (s->tris) (void)hipFree(s->tris);
    if (s->shade) (void)hipFree(s->shade);
    if (s->normals) (void)hipFree(s->normals);
    if (s->occ.bits) (void)hipFree(s->occ.bits);
    free_workspace(s->ws, nullptr);
    free_batch_workspace(s->bws, nullptr);
    if (s->err_host) (void)hipHostFree(s->err_host);
    (void)hipDeviceSynchronize();
    delete s;
}

rcp_status rcp_scene_info(const rcp_scene* s, rcp_scene_stats* out) {
    clear_error();
    if (!s || !out) FAIL("scene and out must not be NULL");
    *out = s->stats;
    return RCP_OK;
}

static rcp_status render_common(rcp_scene* scene, const rcp_camera* cam, int W, int H, int K,
                                const rcp_displacement* disp, float* out_images, int32_t* out_ids,
                                const float* prev, const float* prev_aux, float* out_aux,
                                unsigned long long* counts, void* stream) {
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    Camera c;
    if ((st = check_camera(cam, c))) return st;
    if ((st = check_disp(disp))) return st;
    if ((st = check_size(W, H))) return st;
    if (K < 1 || K > kMaxPasses) FAIL("K = %d must be in [1, %d]", K, kMaxPasses);
    if (!out_images) FAIL("out_images must not be NULL");
    Disp d{disp->lambda_eye, disp->lambda_dir, disp->z0, disp->mode};
    return render(scene, scene->ws, c, W, H, K, d, out_images, out_ids, prev, prev_aux, out_aux, counts,
                  (hipStream_t)stream);
}

rcp_status rcp_render(rcp_scene* scene, const rcp_camera* cam, int W, int H, int K, const rcp_displacement* disp,
                      float* out_images, int32_t* out_ids, void* hip_stream) {
    return render_common(scene, cam, W, H, K, disp, out_images, out_ids, nullptr, nullptr, nullptr, nullptr,
                         hip_stream);
}

rcp_status rcp_render_pass(rcp_scene* scene, const rcp_camera* cam, int W, int H, const rcp_displacement* disp,
                           const float* prev_rgb, const float* prev_aux, float* out_rgb, int32_t* out_ids,
                           float* out_aux, void* hip_stream) {
    return render_common(scene, cam, W, H, 1, disp, out_rgb, out_ids, prev_rgb, prev_aux, out_aux, nullptr,
                         hip_stream);
}

rcp_status rcp_render_stats(rcp_scene* scene, const rcp_camera* cam, int W, int H, int K,
                            const rcp_displacement* disp, float* out_images, int32_t* out_ids, uint64_t* counts,
                            void* hip_stream) {
    if (!counts) {
        clear_error();
        FAIL("counts must not be NULL");
    }
    return render_common(scene, cam, W, H, K, disp, out_images, out_ids, nullptr, nullptr, nullptr,
                         (unsigned long long*)counts, hip_stream);
}

rcp_status rcp_generate_rays(const rcp_camera* cam, int W, int H, const rcp_displacement* disp,
                             const float* prev_rgb, const float* prev_aux, float* out_org, float* out_dir,
                             void* hip_stream) {
    clear_error();
    Camera c;
    rcp_status st;
    if ((st = check_camera(cam, c))) return st;
    if ((st = check_disp(disp))) return st;
    if ((st = check_size(W, H))) return st;
    if (!out_org || !out_dir) FAIL("out_org and out_dir must not be NULL");
    Disp d{disp->lambda_eye, disp->lambda_dir, disp->z0, disp->mode};
    return generate_rays(c, W, H, d, prev_rgb, prev_aux, out_org, out_dir, (hipStream_t)hip_stream);
}

namespace {

rcp_status check_views(const rcp_view* views, int n_views) {
    rcp_status st = RCP_OK;
    if (!views || n_views < 1 || n_views > 1024) FAIL("n_views = %d must be in [1, 1024] with views not NULL", n_views);
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int i = 0; i < n_views; ++i) {
        const rcp_view& v = views[i];
        Camera c;
        st = check_camera(&v.camera, c);
        if (!st) st = check_disp(&v.disp);
        if (!st) st = check_size(v.W, v.H);
        if (st) {
            const std::string msg = rcp_last_error();   // set_error must not read its own buffer
            set_error("view %d: %s", i, msg.c_str());
            return st;
        }
        if (v.K < 1 || v.K > kMaxPasses) FAIL("view %d: K = %d must be in [1, %d]", i, v.K, kMaxPasses);
        if (!v.out_images) FAIL("view %d: out_images must not be NULL", i);
        const size_t n = (size_t)v.W * (size_t)v.H * (size_t)v.K;
        spans.push_back({(uintptr_t)v.out_images, (uintptr_t)v.out_images + 12 * n});
        if (v.out_ids) spans.push_back({(uintptr_t)v.out_ids, (uintptr_t)v.out_ids + 4 * n});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) FAIL("output buffers of the batch overlap");
    return st;
}

void tuning_out(const Tuning& t, rcp_tuning* out) {
    out->refill_min = t.refill_min;
    out->exit_lanes = t.exit_lanes;
    out->blocks_per_cu = t.blocks_per_cu;
    out->tile_log2w = t.tile_log2w;
    out->engine = t.engine;
    out->top_levels = t.top_levels;
    out->stack_entries = t.stack;
    out->block_size = t.block;
    out->tile_order = t.tile_order;
}

}  // namespace

rcp_status rcp_render_batch(rcp_scene* scene, const rcp_view* views, int n_views, void* hip_stream) {
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    if ((st = check_views(views, n_views))) return st;
    return render_batch(scene, views, n_views, scene->bws, (hipStream_t)hip_stream);
}

rcp_status rcp_autotune_batch(rcp_scene* scene, const rcp_view* views, int n_views, int repeats, rcp_tuning* best,
                              float* best_ms, void* hip_stream) {
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    if ((st = check_views(views, n_views))) return st;
    if (!best) FAIL("best must not be NULL");
    if (repeats < 1 || repeats > 100) FAIL("repeats must be in [1, 100]");
    Tuning t;
    float ms = 0.0f;
    st = autotune_batch(scene, views, n_views, repeats, t, ms, (hipStream_t)hip_stream);
    if (st != RCP_OK) return st;
    tuning_out(t, best);
    if (best_ms) *best_ms = ms;
    return RCP_OK;
}

rcp_status rcp_graph_create(rcp_scene* scene, const rcp_camera* cam, int W, int H, int K, const rcp_displacement* disp,
                            float* out_images, int32_t* out_ids, void* hip_stream, rcp_graph** out) {
    clear_error();
    if (out) *out = nullptr;
    if (!out) FAIL("out must not be NULL");
    rcp_status st = check_scene(scene);
    if (st) return st;
    Camera c;
    if ((st = check_camera(cam, c))) return st;
    if ((st = check_disp(disp))) return st;
    if ((st = check_size(W, H))) return st;
    if (K < 1 || K > kMaxPasses) FAIL("K = %d must be in [1, %d]", K, kMaxPasses);
    if (!out_images) FAIL("out_images must not be NULL");
    // work already queued on the caller's stream must not race the capture's allocations
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) {
        set_error("hipStreamSynchronize failed");
        return RCP_ERR_DEVICE;
    }
    rcp_graph* g = new rcp_graph();
    g->scene = scene;
    g->cam = c;
    g->disp = Disp{disp->lambda_eye, disp->lambda_dir, disp->z0, disp->mode};
    g->W = W; g->H = H; g->K = K;
    g->out = out_images;
    g->ids = out_ids;
    st = graph_capture(g);
    if (st != RCP_OK) { graph_free(g); return st; }
    *out = g;
    return RCP_OK;
}

rcp_status rcp_graph_update(rcp_graph* g, const rcp_camera* cam, const rcp_displacement* disp) {
    clear_error();
    if (!g) FAIL("graph is NULL");
    Camera c;
    rcp_status st;
    if ((st = check_camera(cam, c))) return st;
    if ((st = check_disp(disp))) return st;
    if (disp->mode != g->disp.mode) FAIL("the displacement mode of a graph is fixed");
    g->cam = c;
    g->disp = Disp{disp->lambda_eye, disp->lambda_dir, disp->z0, disp->mode};
    return graph_capture(g);
}

rcp_status rcp_check(rcp_scene* scene, void* hip_stream) {
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_status(e, "hipStreamSynchronize", __FILE__, __LINE__);
    return take_device_error(scene);
}

rcp_status rcp_debug_set(int what, int64_t value) {
    clear_error();
    switch (what) {
        case RCP_DEBUG_FAIL_ALLOC_AFTER:
            g_alloc_left.store(value < 0 ? -1 : (long long)value);
            return RCP_OK;
        case RCP_DEBUG_STEP_BUDGET:
            if (value < 0 || value > 0xFFFFFFFFll) FAIL("step budget must be in [0, 2^32)");
            g_step_budget.store((uint32_t)value);
            return RCP_OK;
        case RCP_DEBUG_LIST_CANARY:
            if (value < 0 || value > 2) FAIL("list canary setting must be 0, 1 or 2");
            g_list_canary.store((int)value);
            return RCP_OK;
    }
    FAIL("unknown debug setting %d", what);
}

rcp_status rcp_graph_launch(rcp_graph* g, void* hip_stream) {
    clear_error();
    if (!g || !g->exec) FAIL("graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_status(e, "hipGraphLaunch", __FILE__, __LINE__);
    return RCP_OK;
}

void rcp_graph_destroy(rcp_graph* g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    graph_free(g);
}

rcp_status rcp_get_tuning(const rcp_scene* s, rcp_tuning* out) {
    clear_error();
    if (!s || !out) FAIL("scene and out must not be NULL");
    // the parameters as set (-1: the library's default for each launch)
    out->refill_min = s->tuning.refill_min > 0 ? s->tuning.refill_min : -1;
    out->exit_lanes = s->tuning.exit_lanes >= 0 ? s->tuning.exit_lanes : -1;
    out->blocks_per_cu = s->tuning.blocks_per_cu;
    out->tile_log2w = s->tuning.tile_log2w;
    out->engine = s->tuning.engine;
    out->top_levels = s->tuning.top_levels;
    out->stack_entries = s->tuning.stack;
    out->block_size = s->tuning.block;
    out->tile_order = s->tuning.tile_order;
    return RCP_OK;
}

rcp_status rcp_set_tuning(rcp_scene* s, const rcp_tuning* t) {
    clear_error();
    if (!s || !t) FAIL("scene and tuning must not be NULL");
    if (t->refill_min != -1 && (t->refill_min < 1 || t->refill_min > 64)) FAIL("refill_min must be -1 or in [1, 64]");
    if (t->exit_lanes < -1 || t->exit_lanes > 64) FAIL("exit_lanes must be -1 or in [0, 64]");
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) FAIL("blocks_per_cu must be in [0, 64]");
    if (t->tile_log2w < 0 || t->tile_log2w > 6) FAIL("tile_log2w must be in [0, 6]");
    if (t->engine != RCP_ENGINE_CHAIN && t->engine != RCP_ENGINE_PASSES) FAIL("unknown engine %d", t->engine);
    if (t->top_levels < 0 || t->top_levels > kTopLevels) FAIL("top_levels must be in [0, %d]", kTopLevels);
    if (t->stack_entries != 8 && t->stack_entries != 16) FAIL("stack_entries must be 8 or 16");
    if (t->block_size != 256 && t->block_size != 512) FAIL("block_size must be 256 or 512");
    if (t->tile_order != 0 && t->tile_order != 1) FAIL("tile_order must be 0 or 1");
    s->tuning.top_levels = t->top_levels;
    s->tuning.stack = t->stack_entries;
    s->tuning.block = t->block_size;
    s->tuning.tile_order = t->tile_order;
    s->tuning.refill_min = t->refill_min;
    s->tuning.exit_lanes = t->exit_lanes;
    s->tuning.blocks_per_cu = t->blocks_per_cu;
    s->tuning.tile_log2w = t->tile_log2w;
    s->tuning.engine = t->engine;
    return RCP_OK;
}

rcp_status rcp_autotune(rcp_scene* scene, const rcp_camera* cam, int W, int H, int K, const rcp_displacement* disp,
                        float* out_images, int32_t* out_ids, int repeats, rcp_tuning* best, float* best_ms,
                        void* hip_stream) {
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    Camera c;
    if ((st = check_camera(cam, c))) return st;
    if ((st = check_disp(disp))) return st;
    if ((st = check_size(W, H))) return st;
    if (K < 1 || K > kMaxPasses) FAIL("K = %d must be in [1, %d]", K, kMaxPasses);
    if (!out_images || !best) FAIL("out_images and best must not be NULL");
    if (repeats < 1 || repeats > 100) FAIL("repeats must be in [1, 100]");
    Tuning t;
    float ms = 0.0f;
    st = autotune(scene, c, W, H, K, Disp{disp->lambda_eye, disp->lambda_dir, disp->z0, disp->mode}, out_images,
                  out_ids, repeats, t, ms, (hipStream_t)hip_stream);
    if (st != RCP_OK) return st;
    tuning_out(t, best);
    if (best_ms) *best_ms = ms;
    return RCP_OK;
}

rcp_status rcp_server_create(rcp_scene* scene, uint64_t pool_bytes, int max_inflight, int queue_capacity,
                             rcp_server** out) {
    clear_error();
    if (out) *out = nullptr;
    if (!out) FAIL("out must not be NULL");
    rcp_status st = check_scene(scene);
    if (st) return st;
    if (pool_bytes < 4096) FAIL("pool_bytes must be at least 4096");
    if (max_inflight < 1 || max_inflight > 8) FAIL("max_inflight must be in [1, 8]");
    if (queue_capacity < 1) FAIL("queue_capacity must be >= 1");
    try {
        return server_create(scene, (size_t)pool_bytes, max_inflight, queue_capacity, out);
    } catch (const std::exception&) {
        set_error("host allocation or thread creation failed");
        return RCP_ERR_OUT_OF_MEMORY;
    }
}

rcp_status rcp_submit(rcp_server* server, const rcp_request* r, uint64_t* ticket) {
    clear_error();
    if (!server || !r || !ticket) FAIL("server, request and ticket must not be NULL");
    Camera c;
    rcp_status st;
    if ((st = check_camera(&r->camera, c))) return st;
    if ((st = check_disp(&r->disp))) return st;
    if ((st = check_size(r->W, r->H))) return st;
    if (r->K < 1 || r->K > kMaxPasses) FAIL("K = %d must be in [1, %d]", r->K, kMaxPasses);
    try {
        return server_submit(server, *r, *ticket);
    } catch (const std::exception&) {
        set_error("host allocation failed");
        return RCP_ERR_OUT_OF_MEMORY;
    }
}

rcp_status rcp_poll(rcp_server* server, uint64_t ticket, int32_t* state, double* times) {
    clear_error();
    if (!server || !state) FAIL("server and state must not be NULL");
    return server_poll(server, ticket, *state, times);
}

rcp_status rcp_result(rcp_server* server, uint64_t ticket, float** images, int32_t** ids) {
    clear_error();
    if (!server) FAIL("server is NULL");
    return server_result(server, ticket, images, ids);
}

rcp_status rcp_result_copy(rcp_server* server, uint64_t ticket, float* images, int32_t* ids, void* hip_stream) {
    clear_error();
    if (!server) FAIL("server is NULL");
    return server_result_copy(server, ticket, images, ids, (hipStream_t)hip_stream);
}

rcp_status rcp_release(rcp_server* server, uint64_t ticket) {
    clear_error();
    if (!server) FAIL("server is NULL");
    return server_release(server, ticket);
}

rcp_status rcp_server_stats(rcp_server* server, uint64_t out[4]) {
    clear_error();
    if (!server || !out) FAIL("server and out must not be NULL");
    return server_stats(server, out);
}

void rcp_server_destroy(rcp_server* server) {
    if (server) server_destroy(server);
}

rcp_status rcp_gather_passes(const float* in_rgb, int W, int H, int n_passes, float max_smudge, int edge_mode,
                             int centred, float* out_images, void* hip_stream) {
    clear_error();
    rcp_status st = check_size(W, H);
    if (st) return st;
    if (!in_rgb || !out_images) FAIL("in_rgb and out_images must not be NULL");
    if (n_passes < 1 || n_passes > kMaxPasses) FAIL("n_passes = %d must be in [1, %d]", n_passes, kMaxPasses);
    if (!std::isfinite(max_smudge) || max_smudge < 0.0f || max_smudge > 1e6f) FAIL("max_smudge must be in [0, 1e6]");
    if (edge_mode != RCP_EDGE_CLAMP && edge_mode != RCP_EDGE_WRAP && edge_mode != RCP_EDGE_MIRROR)
        FAIL("unknown edge mode %d", edge_mode);
    const size_t P = (size_t)W * (size_t)H;
    const uintptr_t a0 = (uintptr_t)in_rgb, a1 = a0 + 12 * P;
    const uintptr_t b0 = (uintptr_t)out_images, b1 = b0 + 12 * P * (size_t)n_passes;
    if (a0 < b1 && b0 < a1) FAIL("out_images overlaps in_rgb");
    return gather_passes(in_rgb, W, H, n_passes, max_smudge, edge_mode, centred ? 1 : 0, out_images,
                         (hipStream_t)hip_stream);
}

rcp_status rcp_trace_rays(rcp_scene* scene, const float* org, const float* dir, int n, float* out_t,
                          int32_t* out_id, int32_t* out_front, void* hip_stream) {
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    if (n < 0) FAIL("n must be >= 0");
    if (n > 0 && (!org || !dir || !out_t || !out_id)) FAIL("org, dir, out_t and out_id must not be NULL");
    return trace_rays(scene, org, dir, n, out_t, out_id, out_front, (hipStream_t)hip_stream);
}

rcp_status rcp_export_bvh(const rcp_scene* s, uint32_t* nodes, int32_t* tri_ids) {
    clear_error();
    if (!s) FAIL("scene is NULL");
    if (nodes && s->dev.n_nodes) {
        hipError_t e = hipMemcpy(nodes, s->nodes, kNodeBytes * (size_t)s->dev.n_nodes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_status(e, "export nodes", __FILE__, __LINE__);
    }
    if (tri_ids && s->dev.n_tris) {
        // original index of each packed triangle: the w word of its first vertex
        const size_t n = s->dev.n_tris;
        float4* tmp = new float4[3 * n];
        hipError_t e = hipMemcpy(tmp, s->tris, sizeof(float4) * 3 * n, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (size_t j = 0; j < n; ++j) memcpy(&tri_ids[j], &tmp[3 * j].w, 4);
        delete[] tmp;
        if (e != hipSuccess) return hip_status(e, "export triangles", __FILE__, __LINE__);
    }
    return RCP_OK;
}

rcp_status rcp_radix_sort_u64(uint64_t* keys, uint32_t* vals, int n, void* hip_stream) {
    clear_error();
    if (n < 0) FAIL("n must be >= 0");
    if (n > 0 && (!keys || !vals)) FAIL("keys and vals must not be NULL");
    if (n <= 1) return RCP_OK;
    uint64_t* k2 = nullptr;
    uint32_t* v2 = nullptr;
    rcp_status st0 = dev_alloc((void**)&k2, sizeof(uint64_t) * (size_t)n);
    if (st0 != RCP_OK) return st0;
    st0 = dev_alloc((void**)&v2, sizeof(uint32_t) * (size_t)n);
    if (st0 != RCP_OK) {
        (void)hipFree(k2);
        return st0;
    }
    rcp_status st = radix_sort_pairs(keys, vals, k2, v2, n, 64, (hipStream_t)hip_stream);
    (void)hipFree(k2);
    (void)hipFree(v2);
    return st;
}

}  // extern "C"
