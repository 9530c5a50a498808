// Batched renderer: many views (cameras, image sizes, pass counts) of one
// scene in a single persistent launch.
//
// The recursion I_n(u,v) = F(I_{n-1}(u,v), S) is pointwise (Section 2), so a
// pixel's K passes form a chain that needs nothing from other pixels.  A work
// item is one pixel of one view (8x8 tiles per view, views back to back); a
// lane carries its pixel through the view's passes -- trace, shade, write
// image k, and, if the colour changed, displace the camera and trace again --
// and takes a new pixel as soon as the chain ends (after K passes, or when
// the colour stops changing: the next ray would be identical, so the colour
// is written to the remaining images at once).  No pass barrier is needed, so
// views of any size and pass count share the launch and its tail.
#include "traverse.hpp"

namespace rcp {
namespace {

constexpr int kMaxViews = 1024;

struct ViewDev {
    Camera cam;
    int W, H, K, tiles_x, tile_log2w;
    float le, ld;
    float* out;            // [K][H][W][3]
    int32_t* ids;          // [K][H][W] or NULL
};

struct BatchArgs {
    DevScene sc;
    const ViewDev* views;
    const uint32_t* begin;  // [n_views + 1] first work item of each view
    int n_views;
    uint32_t* fetch;
    int refill_min;
    int32_t* spill;
    uint32_t spill_stride;
};

__global__ __launch_bounds__(kBlock) void k_chain(BatchArgs a) {
    extern __shared__ float4 smem[];
    float4* top = smem;                                                   // top_count * 4
    uint32_t* vbegin = (uint32_t*)(smem + 4 * a.sc.top_count);            // n_views + 1
    int32_t* stack_area = (int32_t*)(vbegin + ((a.n_views + 4) & ~3));    // kStack * kBlock

    for (uint32_t i = threadIdx.x; i < 4 * a.sc.top_count; i += kBlock) top[i] = a.sc.nodes[i];
    for (int i = threadIdx.x; i <= a.n_views; i += kBlock) vbegin[i] = a.begin[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
    Stack st;
    st.lds = stack_area + threadIdx.x;
    st.spill = a.spill + gtid;
    st.stride = a.spill_stride;
    const uint32_t n_items = vbegin[a.n_views];
    const float seed_aux[4] = {INFINITY, 0.0f, 0.0f, 0.0f};

    bool alive = false;
    bool drained = false;      // wave-uniform
    int v = 0, k = 0, x = 0, y = 0;
    float pr = 0.5f, pg = 0.5f, pb = 0.5f;
    Trav tv;
    tv.node = -1;

    for (;;) {
        // ---- refill idle lanes with new pixels ---------------------------------
        const unsigned long long idle = __ballot(!alive);
        const uint32_t n_idle = (uint32_t)__popcll(idle);
        if (!drained && n_idle >= (uint32_t)a.refill_min) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.fetch, n_idle);
            base = __shfl(base, 0);
            if (base + n_idle >= n_items) drained = true;
            if (!alive) {
                const uint32_t item = base + lanes_below(idle);
                if (item < n_items) {
                    // the view holding this item: last begin <= item
                    int lo = 0, hi = a.n_views;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (vbegin[mid] <= item) lo = mid; else hi = mid;
                    }
                    v = lo;
                    const ViewDev& vw = a.views[v];
                    const uint32_t local = item - vbegin[v];
                    const uint32_t tile = local >> 6, l = local & 63u;
                    const uint32_t tw = 1u << vw.tile_log2w;
                    x = (int)((tile % (uint32_t)vw.tiles_x) * tw + (l & (tw - 1u)));
                    y = (int)((tile / (uint32_t)vw.tiles_x) * (64u >> vw.tile_log2w) + (l >> vw.tile_log2w));
                    if (x < vw.W && y < vw.H) {
                        k = 0;
                        pr = 0.5f; pg = 0.5f; pb = 0.5f;
                        float o[3], d[3];
                        make_ray<RCP_MODE_COLOR>(vw.cam, vw.W, vw.H, x, y, pr, pg, pb, seed_aux, 0.0f, vw.le, vw.ld,
                                                 o, d);
                        trav_init(tv, a.sc, o, d, st);
                        alive = true;
                    }
                }
            }
        }
        if (__ballot(alive) == 0ull) {
            if (drained) break;
            continue;
        }

        // ---- one traversal step -------------------------------------------------
        uint32_t dn = 0, dt = 0;
        if (alive && tv.node != -1) trav_step<false>(tv, a.sc, top, st, dn, dt);

        // ---- a finished pass: shade, write, then the next pass or the end -------
        if (alive && tv.node == -1) {
            const ViewDev& vw = a.views[v];
            float rgb[3];
            int32_t hid = -1;
            if (tv.h.id != INT_MAX) {
                const float4 c = a.sc.shade[2 * (size_t)tv.h.slot + (tv.h.front ? 0 : 1)];
                rgb[0] = c.x; rgb[1] = c.y; rgb[2] = c.z;
                hid = tv.h.id;
            } else {
                rgb[0] = a.sc.bg[0]; rgb[1] = a.sc.bg[1]; rgb[2] = a.sc.bg[2];
            }
            const size_t P = (size_t)vw.W * (size_t)vw.H;
            const size_t pix = (size_t)y * (size_t)vw.W + (size_t)x;
            const bool changed = __float_as_uint(rgb[0]) != __float_as_uint(pr) ||
                                 __float_as_uint(rgb[1]) != __float_as_uint(pg) ||
                                 __float_as_uint(rgb[2]) != __float_as_uint(pb);
            // image k, and every later image when the colour did not change
            const int k_end = changed ? k + 1 : vw.K;
            for (int kk = k; kk < k_end; ++kk) {
                float* q = vw.out + ((size_t)kk * P + pix) * 3;
                q[0] = rgb[0]; q[1] = rgb[1]; q[2] = rgb[2];
                if (vw.ids) vw.ids[(size_t)kk * P + pix] = hid;
            }
            if (changed && k + 1 < vw.K) {
                ++k;
                pr = rgb[0]; pg = rgb[1]; pb = rgb[2];
                float o[3], d[3];
                make_ray<RCP_MODE_COLOR>(vw.cam, vw.W, vw.H, x, y, pr, pg, pb, seed_aux, 0.0f, vw.le, vw.ld, o, d);
                trav_init(tv, a.sc, o, d, st);
            } else {
                alive = false;
            }
        }
    }
}

__global__ void k_clear_fetch(uint32_t* fetch) {
    if (threadIdx.x == 0) *fetch = 0u;
}

}  // namespace

rcp_status render_batch(rcp_scene* s, const rcp_view* views, int n_views, BatchWorkspace& ws, hipStream_t stream) {
    const Launch lp = launch_params(s);
    const int tw = 1 << lp.tile_log2w, th = 64 >> lp.tile_log2w;
    // host-side view table and item offsets
    std::vector<ViewDev> hv((size_t)n_views);
    std::vector<uint32_t> hb((size_t)n_views + 1);
    uint64_t items = 0;
    for (int i = 0; i < n_views; ++i) {
        const rcp_view& vi = views[i];
        ViewDev& d = hv[(size_t)i];
        for (int c = 0; c < 3; ++c) {
            d.cam.eye[c] = vi.camera.eye[c];
            d.cam.right[c] = vi.camera.right[c];
            d.cam.up[c] = vi.camera.up[c];
            d.cam.forward[c] = vi.camera.forward[c];
        }
        d.cam.th = vi.camera.tan_half_fovy;
        d.W = vi.W; d.H = vi.H; d.K = vi.K;
        d.tiles_x = (vi.W + tw - 1) / tw;
        d.tile_log2w = lp.tile_log2w;
        d.le = vi.disp.lambda_eye;
        d.ld = vi.disp.lambda_dir;
        d.out = vi.out_images;
        d.ids = vi.out_ids;
        hb[(size_t)i] = (uint32_t)items;
        items += (uint64_t)d.tiles_x * (uint64_t)((vi.H + th - 1) / th) * 64u;
    }
    if (items >= (1ull << 32)) {
        set_error("batch holds %llu work items (limit 2^32)", (unsigned long long)items);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    hb[(size_t)n_views] = (uint32_t)items;

    // persistent grid from the occupancy of this kernel and its LDS use
    const size_t smem = sizeof(float4) * 4 * (size_t)lp.staged_nodes +
                        sizeof(uint32_t) * (size_t)((n_views + 4) & ~3) + sizeof(int32_t) * kStack * kBlock;
    int per_cu = 0, dev = 0, cus = 0;
    RCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_chain, kBlock, smem));
    RCP_HIP(hipGetDevice(&dev));
    RCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu < 1) per_cu = 1;
    if (lp.blocks_per_cu > 0 && lp.blocks_per_cu < per_cu) per_cu = lp.blocks_per_cu;
    const int blocks = per_cu * cus;
    const uint32_t threads = (uint32_t)blocks * kBlock;
    const size_t spill_depth = s->dev.max_depth > (uint32_t)kStack ? s->dev.max_depth - kStack + 1 : 1;

    if ((size_t)n_views > ws.view_cap) {
        if (ws.views) { RCP_HIP(hipFree(ws.views)); ws.views = nullptr; }
        ws.view_cap = 0;
        RCP_HIP(hipMalloc(&ws.views, (sizeof(ViewDev) + sizeof(uint32_t)) * (size_t)(n_views + 1) + 256));
        ws.view_cap = (size_t)n_views;
    }
    if (!ws.fetch) RCP_HIP(hipMalloc((void**)&ws.fetch, 256));
    if (spill_depth * threads > ws.spill_cap) {
        if (ws.spill) { RCP_HIP(hipFree(ws.spill)); ws.spill = nullptr; }
        ws.spill_cap = 0;
        RCP_HIP(hipMalloc((void**)&ws.spill, sizeof(int32_t) * spill_depth * threads));
        ws.spill_cap = spill_depth * threads;
    }
    ViewDev* d_views = (ViewDev*)ws.views;
    uint32_t* d_begin = (uint32_t*)((char*)ws.views + ((sizeof(ViewDev) * (size_t)n_views + 255) & ~(size_t)255));
    // pageable sources: the copies have read them when the calls return
    RCP_HIP(hipMemcpyAsync(d_views, hv.data(), sizeof(ViewDev) * (size_t)n_views, hipMemcpyHostToDevice, stream));
    RCP_HIP(hipMemcpyAsync(d_begin, hb.data(), sizeof(uint32_t) * (size_t)(n_views + 1), hipMemcpyHostToDevice,
                           stream));
    hipLaunchKernelGGL(k_clear_fetch, dim3(1), dim3(64), 0, stream, ws.fetch);
    RCP_CHECK_LAUNCH();
    BatchArgs a{};
    a.sc = s->dev;
    a.sc.top_count = lp.staged_nodes;
    a.views = d_views;
    a.begin = d_begin;
    a.n_views = n_views;
    a.fetch = ws.fetch;
    a.refill_min = lp.refill_min;
    a.spill = ws.spill;
    a.spill_stride = threads;
    hipLaunchKernelGGL(k_chain, dim3(blocks), dim3(kBlock), smem, stream, a);
    RCP_CHECK_LAUNCH();
    return RCP_OK;
}

void free_batch_workspace(BatchWorkspace& ws) {
    if (ws.views) (void)hipFree(ws.views);
    if (ws.fetch) (void)hipFree(ws.fetch);
    if (ws.spill) (void)hipFree(ws.spill);
    ws = BatchWorkspace{};
}

}  // namespace rcp
