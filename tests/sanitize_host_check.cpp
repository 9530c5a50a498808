// sanitize_host_check.cpp -- test driver for the library's host code built
// with the address and undefined-behaviour sanitizers (host side only; the
// device code is never instrumented).  tests/test_sanitizers.py builds the
// library's host code and this driver with them and runs the validation
// part; with --device it also drives every entry point once on the GPU
// (scene build, the K-pass render in both engines, the single pass, the
// instrumented render, batches, graphs, the server, the allocation-free
// render, the autotuner, tracing, sorting, the screen-space passes, forced
// allocation failures, the list canary and the build log) and checks that the
// paths that must agree do.
//
// Exit status 0 when every call returns what it must.  The leak check runs
// explicitly at the end of main, and the process then ends without running
// the HIP runtime's own static destructors (with the sanitizer runtime they
// abort in its device-memory bookkeeping, outside this library).
#include <hip/hip_runtime_api.h>
#include <sanitizer/lsan_interface.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "rcp.h"

static int g_fail = 0;

static void step(const char* what) { std::fprintf(stderr, "[step] %s\n", what); }

#define EXPECT(cond)                                                                      \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond,    \
                         rcp_last_error());                                               \
            g_fail = 1;                                                                   \
        }                                                                                 \
    } while (0)
#define EXPECT_STATUS(call, want) EXPECT((call) == (want))
#define OK(call) EXPECT_STATUS(call, RCP_OK)
#define HIP(call)                                                                          \
    do {                                                                                   \
        if ((call) != hipSuccess) {                                                        \
            std::fprintf(stderr, "HIP call failed %s:%d: %s\n", __FILE__, __LINE__, #call); \
            std::exit(3);                                                                  \
        }                                                                                  \
    } while (0)

// A small terrain: an n x n height-field grid (two triangles per cell) plus
// a few boxes standing on it, every value a deterministic function of the
// indices.
struct HostScene {
    std::vector<float> verts, rgb;
    std::vector<uint32_t> idx;
    rcp_scene_desc desc() const {
        rcp_scene_desc d{};
        d.verts = verts.data();
        d.n_verts = (uint32_t)(verts.size() / 3);
        d.idx = idx.data();
        d.n_tris = (uint32_t)(idx.size() / 3);
        d.tri_rgb = rgb.data();
        const float l[3] = {0.3f, 0.8f, -0.5f};
        const float n = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
        for (int c = 0; c < 3; ++c) {
            d.light_dir[c] = l[c] / n;
            d.background[c] = 0.5f;
        }
        d.k_a = 0.05f;
        d.k_d = 0.95f;
        return d;
    }
};

static HostScene terrain(int n) {
    HostScene s;
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            const float x = -1.0f + 2.0f * i / n, z = -1.0f + 2.0f * j / n;
            const float y = 0.08f * std::sin(7.0f * x) * std::cos(5.0f * z) + 0.03f * std::sin(23.0f * x * z);
            s.verts.insert(s.verts.end(), {x, y, z});
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            const uint32_t a = j * (n + 1) + i, b = a + 1, c = a + (n + 1), d = c + 1;
            s.idx.insert(s.idx.end(), {a, c, b, b, c, d});
            for (int t = 0; t < 2; ++t)
                s.rgb.insert(s.rgb.end(), {0.2f + 0.6f * i / n, 0.3f + 0.5f * j / n, 0.4f + 0.3f * t});
        }
    for (int b = 0; b < 6; ++b) {  // axis-aligned boxes, 12 triangles each
        const float cx = -0.7f + 0.28f * b, cz = 0.5f * std::sin(1.7f * b), h = 0.1f + 0.05f * b, r = 0.06f;
        const uint32_t base = (uint32_t)(s.verts.size() / 3);
        for (int k = 0; k < 8; ++k)
            s.verts.insert(s.verts.end(), {cx + ((k & 1) ? r : -r), (k & 2) ? h : -0.1f, cz + ((k & 4) ? r : -r)});
        const uint32_t f[12][3] = {{0, 1, 3}, {0, 3, 2}, {4, 6, 7}, {4, 7, 5}, {0, 4, 5}, {0, 5, 1},
                                   {2, 3, 7}, {2, 7, 6}, {0, 2, 6}, {0, 6, 4}, {1, 5, 7}, {1, 7, 3}};
        for (auto& t : f) {
            s.idx.insert(s.idx.end(), {base + t[0], base + t[1], base + t[2]});
            s.rgb.insert(s.rgb.end(), {0.9f, 0.2f + 0.1f * b, 0.1f});
        }
    }
    return s;
}

static rcp_camera look_at(const float eye[3], const float at[3], float vfov_deg) {
    rcp_camera c{};
    float f[3], len = 0.0f;
    for (int i = 0; i < 3; ++i) {
        c.eye[i] = eye[i];
        f[i] = at[i] - eye[i];
        len += f[i] * f[i];
    }
    len = std::sqrt(len);
    for (int i = 0; i < 3; ++i) c.forward[i] = f[i] / len;
    // right = up x forward with up = +y, then up = forward x right
    float r[3] = {c.forward[2], 0.0f, -c.forward[0]};
    const float rl = std::sqrt(r[0] * r[0] + r[2] * r[2]);
    for (int i = 0; i < 3; ++i) c.right[i] = r[i] / rl;
    c.up[0] = c.forward[1] * c.right[2] - c.forward[2] * c.right[1];
    c.up[1] = c.forward[2] * c.right[0] - c.forward[0] * c.right[2];
    c.up[2] = c.forward[0] * c.right[1] - c.forward[1] * c.right[0];
    c.tan_half_fovy = std::tan(0.5f * vfov_deg * 3.14159265f / 180.0f);
    return c;
}

static rcp_displacement disp(float le, float ld, int mode = RCP_MODE_COLOR, float z0 = 0.0f) {
    rcp_displacement d{};
    d.lambda_eye = le;
    d.lambda_dir = ld;
    d.mode = mode;
    d.z0 = z0;
    return d;
}

// ---------------------------------------------------------------- no device

static void validation() {
    EXPECT(std::strcmp(rcp_status_string(RCP_OK), "ok") == 0);
    EXPECT(std::strcmp(rcp_status_string((rcp_status)99), "unknown status") == 0);
    const float eye[3] = {0.0f, 0.6f, -1.5f}, at[3] = {0.0f, 0.0f, 0.0f};
    const rcp_camera cam = look_at(eye, at, 60.0f);
    const rcp_displacement d = disp(0.0f, 0.02f);
    float* fake = reinterpret_cast<float*>(uintptr_t(1) << 20);  // never dereferenced: rejected first
    EXPECT_STATUS(rcp_render(nullptr, &cam, 64, 64, 6, &d, fake, nullptr, nullptr), RCP_ERR_INVALID_ARGUMENT);
    EXPECT(std::strstr(rcp_last_error(), "scene is NULL") != nullptr);
    rcp_camera bad = cam;
    bad.right[0] *= 2.0f;
    EXPECT_STATUS(rcp_generate_rays(&bad, 8, 8, &d, nullptr, nullptr, fake, fake, nullptr),
                  RCP_ERR_INVALID_ARGUMENT);
    bad = cam;
    bad.eye[1] = NAN;
    EXPECT_STATUS(rcp_generate_rays(&bad, 8, 8, &d, nullptr, nullptr, fake, fake, nullptr),
                  RCP_ERR_INVALID_ARGUMENT);
    const rcp_displacement bad_d[] = {disp(-0.1f, 0.0f), disp(0.0f, 1.0f), disp(INFINITY, 0.0f),
                                      disp(0.0f, 0.1f, 7)};
    for (const auto& b : bad_d)
        EXPECT_STATUS(rcp_generate_rays(&cam, 8, 8, &b, nullptr, nullptr, fake, fake, nullptr),
                      RCP_ERR_INVALID_ARGUMENT);
    const int sizes[][2] = {{0, 8}, {8, 0}, {-1, 5}, {1 << 14, (1 << 13) + 1}};
    for (const auto& s : sizes)
        EXPECT_STATUS(rcp_generate_rays(&cam, s[0], s[1], &d, nullptr, nullptr, fake, fake, nullptr),
                      RCP_ERR_INVALID_ARGUMENT);
    EXPECT_STATUS(rcp_generate_rays(&cam, 8, 8, &d, nullptr, nullptr, nullptr, fake, nullptr),
                  RCP_ERR_INVALID_ARGUMENT);
    EXPECT_STATUS(rcp_render_batch(nullptr, nullptr, 0, nullptr), RCP_ERR_INVALID_ARGUMENT);
    rcp_view v{};
    v.camera = cam;
    v.W = v.H = 8;
    v.K = 65;
    v.disp = d;
    v.out_images = fake;
    EXPECT_STATUS(rcp_render_batch(nullptr, &v, 1, nullptr), RCP_ERR_INVALID_ARGUMENT);

    HostScene hs = terrain(4);
    rcp_scene_desc desc = hs.desc();
    rcp_scene* sc = reinterpret_cast<rcp_scene*>(fake);
    hs.idx[7] = desc.n_verts;
    EXPECT_STATUS(rcp_build_scene(&desc, nullptr, nullptr, &sc), RCP_ERR_INVALID_ARGUMENT);
    EXPECT(sc == nullptr);
    hs.idx[7] = 0;
    hs.verts[5] = NAN;
    EXPECT_STATUS(rcp_build_scene(&desc, nullptr, nullptr, &sc), RCP_ERR_INVALID_ARGUMENT);
    hs.verts[5] = 0.0f;
    desc.background[0] = NAN;
    EXPECT_STATUS(rcp_build_scene(&desc, nullptr, nullptr, &sc), RCP_ERR_INVALID_ARGUMENT);
    desc = hs.desc();
    const rcp_build_options bad_o[] = {{0, 1.0f, 1.0f, 0, 0}, {9, 1.0f, 1.0f, 0, 0}, {4, -1.0f, 1.0f, 0, 0},
                                       {4, 1.0f, NAN, 0, 0},  {4, 1.0f, 1.0f, 2, 0}, {4, 1.0f, 1.0f, 0, -1}};
    for (const auto& o : bad_o) EXPECT_STATUS(rcp_build_scene(&desc, &o, nullptr, &sc), RCP_ERR_INVALID_ARGUMENT);
    EXPECT_STATUS(rcp_build_scene(nullptr, nullptr, nullptr, &sc), RCP_ERR_INVALID_ARGUMENT);

    EXPECT_STATUS(rcp_trace_rays(nullptr, fake, fake, 4, fake, nullptr, nullptr, nullptr), RCP_ERR_INVALID_ARGUMENT);
    EXPECT_STATUS(rcp_radix_sort_u64(nullptr, nullptr, -1, nullptr), RCP_ERR_INVALID_ARGUMENT);
    OK(rcp_radix_sort_u64(nullptr, nullptr, 0, nullptr));
    EXPECT(rcp_last_error()[0] == '\0');
    EXPECT_STATUS(rcp_scene_info(nullptr, nullptr), RCP_ERR_INVALID_ARGUMENT);
    EXPECT(rcp_last_error()[0] != '\0');
    EXPECT_STATUS(rcp_gather_passes(nullptr, 8, 8, 1, 2.0f, RCP_EDGE_MIRROR, 1, fake, nullptr),
                  RCP_ERR_INVALID_ARGUMENT);
    EXPECT_STATUS(rcp_gather_passes(fake, 8, 8, 65, 2.0f, RCP_EDGE_MIRROR, 1, fake + (1 << 20), nullptr),
                  RCP_ERR_INVALID_ARGUMENT);
    EXPECT_STATUS(rcp_gather_passes(fake, 8, 8, 2, 2.0f, RCP_EDGE_WRAP, 1, fake + 100, nullptr),
                  RCP_ERR_INVALID_ARGUMENT);
    rcp_server* srv = nullptr;
    EXPECT_STATUS(rcp_server_create(nullptr, 1 << 20, 2, 64, &srv), RCP_ERR_INVALID_ARGUMENT);
    rcp_request rq{};
    rq.camera = cam;
    rq.W = rq.H = 8;
    rq.K = 2;
    rq.disp = d;
    uint64_t ticket = 0;
    EXPECT(rcp_submit(nullptr, &rq, &ticket) != RCP_OK);
    int32_t state = 0;
    EXPECT(rcp_poll(nullptr, 1, &state, nullptr) != RCP_OK);
    EXPECT(rcp_release(nullptr, 1) != RCP_OK);
    rcp_server_destroy(nullptr);
    rcp_destroy_scene(nullptr);
    rcp_graph_destroy(nullptr);
    EXPECT_STATUS(rcp_debug_set(99, 0), RCP_ERR_INVALID_ARGUMENT);
}

// ---------------------------------------------------------------- device

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    explicit DevBuf(size_t count) : n(count) {
        HIP(hipMalloc(&p, count * sizeof(T) + 1));
        HIP(hipMemset(p, 0, count * sizeof(T)));
    }
    ~DevBuf() { (void)hipFree(p); }
    std::vector<T> host() const {
        std::vector<T> h(n);
        HIP(hipMemcpy(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost));
        return h;
    }
};

template <class T>
static bool same(const std::vector<T>& a, const std::vector<T>& b) {
    return a.size() == b.size() && std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) == 0;
}

static void device() {
    HostScene hs = terrain(48);
    const rcp_scene_desc desc = hs.desc();
    hipStream_t st;
    HIP(hipStreamCreate(&st));

    // forced allocation failures at every point of the build, then a good one
    step("build with allocation failures");
    for (int after = 0; after < 40; ++after) {
        OK(rcp_debug_set(RCP_DEBUG_FAIL_ALLOC_AFTER, after));
        rcp_scene* s = nullptr;
        const rcp_status r = rcp_build_scene(&desc, nullptr, st, &s);
        OK(rcp_debug_set(RCP_DEBUG_FAIL_ALLOC_AFTER, -1));
        EXPECT(r == RCP_OK || r == RCP_ERR_OUT_OF_MEMORY);
        EXPECT((r == RCP_OK) == (s != nullptr));
        rcp_destroy_scene(s);
        if (r == RCP_OK) break;
    }
    rcp_scene* sc = nullptr;
    setenv("RCP_LOG", "1", 1);   // the build's log line
    OK(rcp_build_scene(&desc, nullptr, st, &sc));
    unsetenv("RCP_LOG");
    if (!sc) return;
    rcp_scene_stats info{};
    OK(rcp_scene_info(sc, &info));
    EXPECT(info.n_tris == desc.n_tris);
    std::vector<uint32_t> nodes((size_t)info.n_nodes * 32);
    std::vector<int32_t> tri_ids(info.n_tris);
    OK(rcp_export_bvh(sc, nodes.data(), tri_ids.data()));

    const float eye[3] = {0.1f, 0.7f, -1.6f}, at[3] = {0.0f, 0.0f, 0.1f};
    const rcp_camera cam = look_at(eye, at, 60.0f);
    const int W = 200, H = 120, K = 6;
    const size_t P = (size_t)W * H;
    const rcp_displacement modes[3] = {disp(0.01f, 0.02f), disp(0.0f, 0.03f, RCP_MODE_DEPTH, 1.2f),
                                       disp(0.0f, 0.03f, RCP_MODE_NORMAL)};
    for (const auto& d : modes) {
    step("renders: both engines, three mappings, single passes, counters");
        DevBuf<float> a(P * K * 3), b(P * K * 3), c(P * K * 3);
        DevBuf<int32_t> ia(P * K), ib(P * K), ic(P * K);
        rcp_tuning t{};
        OK(rcp_get_tuning(sc, &t));
        t.engine = RCP_ENGINE_CHAIN;
        OK(rcp_set_tuning(sc, &t));
        OK(rcp_render(sc, &cam, W, H, K, &d, a.p, ia.p, st));
        t.engine = RCP_ENGINE_PASSES;
        OK(rcp_set_tuning(sc, &t));
        OK(rcp_debug_set(RCP_DEBUG_LIST_CANARY, 1));   // the lists canary-checked (rcp_check below)
        OK(rcp_render(sc, &cam, W, H, K, &d, b.p, ib.p, st));
        OK(rcp_debug_set(RCP_DEBUG_LIST_CANARY, 0));
        t.engine = RCP_ENGINE_CHAIN;
        OK(rcp_set_tuning(sc, &t));
        std::vector<uint64_t> counts((size_t)K * 6);
        OK(rcp_render_stats(sc, &cam, W, H, K, &d, c.p, ic.p, counts.data(), st));
        OK(rcp_check(sc, st));
        EXPECT(same(a.host(), b.host()) && same(ia.host(), ib.host()));
        EXPECT(same(a.host(), c.host()) && same(ia.host(), ic.host()));
        EXPECT(counts[0] == P);
        // the single pass applied to image 1 gives image 2
        DevBuf<float> p1(P * 3), aux1(P * 4), p2(P * 3);
        DevBuf<int32_t> i2(P);
        OK(rcp_render_pass(sc, &cam, W, H, &d, nullptr, nullptr, p1.p, nullptr, aux1.p, st));
        OK(rcp_render_pass(sc, &cam, W, H, &d, p1.p, aux1.p, p2.p, i2.p, nullptr, st));
        HIP(hipStreamSynchronize(st));
        const std::vector<float> all = a.host();
        const std::vector<float> second(all.begin() + P * 3, all.begin() + 2 * P * 3);
        EXPECT(same(p2.host(), second));
    }

    // batch of three views against single renders; the allocation-free call
    step("batch, allocation-free render, autotuners");
    const rcp_displacement d = modes[0];
    const int sz[3][3] = {{64, 48, 3}, {W, H, K}, {17, 9, 1}};
    std::vector<DevBuf<float>*> outs;
    std::vector<DevBuf<int32_t>*> ids;
    std::vector<rcp_view> views;
    for (auto& s : sz) {
        outs.push_back(new DevBuf<float>((size_t)s[0] * s[1] * s[2] * 3));
        ids.push_back(new DevBuf<int32_t>((size_t)s[0] * s[1] * s[2]));
        rcp_view v{};
        v.camera = cam;
        v.W = s[0];
        v.H = s[1];
        v.K = s[2];
        v.disp = d;
        v.out_images = outs.back()->p;
        v.out_ids = ids.back()->p;
        views.push_back(v);
    }
    OK(rcp_render_batch(sc, views.data(), 3, st));
    for (int i = 0; i < 3; ++i) {
        DevBuf<float> o(outs[i]->n), n(outs[i]->n);
        DevBuf<int32_t> oi(ids[i]->n), ni(ids[i]->n);
        OK(rcp_render(sc, &cam, sz[i][0], sz[i][1], sz[i][2], &d, o.p, oi.p, st));
        OK(rcp_render_noalloc(sc, &cam, sz[i][0], sz[i][1], sz[i][2], &d, n.p, ni.p, st));
        HIP(hipStreamSynchronize(st));
        EXPECT(same(outs[i]->host(), o.host()) && same(ids[i]->host(), oi.host()));
        EXPECT(same(n.host(), o.host()) && same(ni.host(), oi.host()));
    }
    rcp_tuning best{};
    float best_ms = 0.0f;
    OK(rcp_autotune_batch(sc, views.data(), 3, 1, &best, &best_ms, st));
    OK(rcp_autotune(sc, &cam, W, H, K, &d, outs[1]->p, ids[1]->p, 1, &best, &best_ms, st));
    for (auto* p : outs) delete p;
    for (auto* p : ids) delete p;

    // a graph, replayed after an update
    step("graph");
    {
        DevBuf<float> g(P * K * 3), o(P * K * 3);
        DevBuf<int32_t> gi(P * K), oi(P * K);
        rcp_graph* gr = nullptr;
        OK(rcp_graph_create(sc, &cam, W, H, K, &d, g.p, gi.p, st, &gr));
        const float eye2[3] = {-0.3f, 0.5f, -1.4f};
        const rcp_camera cam2 = look_at(eye2, at, 55.0f);
        OK(rcp_graph_update(gr, &cam2, &d));
        OK(rcp_graph_launch(gr, st));
        OK(rcp_graph_launch(gr, st));
        OK(rcp_render(sc, &cam2, W, H, K, &d, o.p, oi.p, st));
        HIP(hipStreamSynchronize(st));
        EXPECT(same(g.host(), o.host()) && same(gi.host(), oi.host()));
        rcp_graph_destroy(gr);
    }

    // the server: a few requests of different sizes, results against rcp_render
    step("server");
    {
        rcp_server* srv = nullptr;
        OK(rcp_server_create(sc, 64ull << 20, 2, 64, &srv));
        std::vector<uint64_t> tickets;
        const int rs[4][3] = {{96, 64, 4}, {33, 21, 2}, {128, 128, 8}, {64, 64, 1}};
        for (auto& r : rs) {
            rcp_request q{};
            q.camera = cam;
            q.W = r[0];
            q.H = r[1];
            q.K = r[2];
            q.disp = d;
            q.with_ids = 1;
            uint64_t t = 0;
            OK(rcp_submit(srv, &q, &t));
            tickets.push_back(t);
        }
        const auto t0 = std::chrono::steady_clock::now();
        for (size_t i = 0; i < tickets.size(); ++i) {
            int32_t state = RCP_REQ_QUEUED;
            double times[3];
            while (true) {
                OK(rcp_poll(srv, tickets[i], &state, times));
                if (state == RCP_REQ_DONE || state == RCP_REQ_FAILED) break;
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) break;
                std::this_thread::sleep_for(std::chrono::microseconds(200));
            }
            EXPECT(state == RCP_REQ_DONE);
            if (state != RCP_REQ_DONE) continue;
            const size_t n = (size_t)rs[i][0] * rs[i][1] * rs[i][2];
            DevBuf<float> got(n * 3), o(n * 3);
            DevBuf<int32_t> gi(n), oi(n);
            float* img = nullptr;
            int32_t* idp = nullptr;
            OK(rcp_result(srv, tickets[i], &img, &idp));
            OK(rcp_result_copy(srv, tickets[i], got.p, gi.p, st));
            OK(rcp_render(sc, &cam, rs[i][0], rs[i][1], rs[i][2], &d, o.p, oi.p, st));
            HIP(hipStreamSynchronize(st));
            EXPECT(same(got.host(), o.host()) && same(gi.host(), oi.host()));
            OK(rcp_release(srv, tickets[i]));
        }
        uint64_t stats[4];
        OK(rcp_server_stats(srv, stats));
        EXPECT(stats[3] == 0);
        rcp_server_destroy(srv);
    }

    // single steps: rays, tracing, the sort, the screen-space passes
    step("rays, tracing, sort, screen-space passes");
    {
        const int n = 4096;
        DevBuf<float> org(n * 3), dir(n * 3), t(n);
        DevBuf<int32_t> id(n), front(n);
        OK(rcp_generate_rays(&cam, 64, 64, &d, nullptr, nullptr, org.p, dir.p, st));
        OK(rcp_trace_rays(sc, org.p, dir.p, n, t.p, id.p, front.p, st));
        std::vector<uint64_t> keys(n);
        std::vector<uint32_t> vals(n);
        for (int i = 0; i < n; ++i) {
            keys[i] = (uint64_t)(i * 2654435761u) << 13 ^ (uint64_t)(n - i);
            vals[i] = (uint32_t)i;
        }
        DevBuf<uint64_t> dk(n);
        DevBuf<uint32_t> dv(n);
        HIP(hipMemcpy(dk.p, keys.data(), n * 8, hipMemcpyHostToDevice));
        HIP(hipMemcpy(dv.p, vals.data(), n * 4, hipMemcpyHostToDevice));
        OK(rcp_radix_sort_u64(dk.p, dv.p, n, st));
        const std::vector<uint64_t> sorted = dk.host();
        for (int i = 1; i < n; ++i) EXPECT(sorted[i - 1] <= sorted[i]);
        DevBuf<float> in(P * 3), g(P * 3 * 4);
        OK(rcp_render_pass(sc, &cam, W, H, &d, nullptr, nullptr, in.p, nullptr, nullptr, st));
        for (int e = 0; e < 3; ++e) OK(rcp_gather_passes(in.p, W, H, 4, 6.0f, e, e != 1, g.p, st));
        HIP(hipStreamSynchronize(st));
    }

    // allocation failures in the render paths fail cleanly, then recover
    step("graph creation with allocation failures");
    {
        DevBuf<float> a(P * K * 3), b(P * K * 3);
        const float eye3[3] = {0.4f, 0.9f, -1.2f};
        const rcp_camera cam3 = look_at(eye3, at, 70.0f);
        OK(rcp_render(sc, &cam3, W, H, K, &d, b.p, nullptr, st));
        for (int after = 0; after < 4; ++after) {
            OK(rcp_debug_set(RCP_DEBUG_FAIL_ALLOC_AFTER, after));
            rcp_graph* gr = nullptr;
            const rcp_status r = rcp_graph_create(sc, &cam3, W, H, K, &d, a.p, nullptr, st, &gr);
            OK(rcp_debug_set(RCP_DEBUG_FAIL_ALLOC_AFTER, -1));
            EXPECT(r == RCP_OK || r == RCP_ERR_OUT_OF_MEMORY);
            rcp_graph_destroy(gr);
        }
        OK(rcp_render(sc, &cam3, W, H, K, &d, a.p, nullptr, st));
        HIP(hipStreamSynchronize(st));
        EXPECT(same(a.host(), b.host()));
    }
    OK(rcp_check(sc, st));
    rcp_destroy_scene(sc);
    HIP(hipStreamDestroy(st));
}

int main(int argc, char** argv) {
    step("argument validation");
    validation();
    const bool dev = argc > 1 && std::strcmp(argv[1], "--device") == 0;
    if (dev) device();
    step("leak check");
    __lsan_do_leak_check();  // exits with the sanitizer's exit code on a leak
    std::printf("sanitize_host_check: %s%s\n", dev ? "validation and device paths " : "validation ",
                g_fail ? "FAILED" : "ok");
    std::fflush(stdout);
    std::fflush(stderr);
    std::_Exit(g_fail ? 1 : 0);
}
