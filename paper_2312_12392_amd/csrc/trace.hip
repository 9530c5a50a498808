// The K-pass render: one persistent kernel launch per pass.
//
// Per pass, every wave repeatedly takes work items for its idle lanes from
// the pass's band counters (one band per XCD, see wave_fetch).  A work item
// is a pixel still being painted: at pass 0 the pixels in 64-pixel tiles
// ordered by super-tiles (with the grey seed, or a caller-supplied previous
// image), later the compact list {pixel, previous RGB} appended by the pass
// before.  For each item the lane
//   1. builds the pixel's displaced camera ray from its previous colour
//      (Section 2 ray and displacements, Section 3 colour mapping),
//   2. traverses the BVH (a short per-lane stack in LDS that overflows into
//      a per-lane global area) and runs the watertight
//      ray/triangle test at the leaves, keeping the nearest hit and, at equal
//      distance, the lowest triangle index,
//   3. looks the shaded colour up in the per-triangle table and writes
//      image k (and its hit ID),
//   4. compares the colour with the previous one: changed pixels are
//      appended to the next pass's list with one ballot, one mbcnt and one
//      atomic per wave; unchanged pixels would get the identical ray again, so
//      their colour is written to every remaining image now.
//
// Everything that decides a result (ray generation, the triangle test, the
// shade table) is FP32 evaluated left to right without contraction, with
// correctly rounded division and square root.  The box tests only prune and
// are widened so that they never reject a box the exact test would accept.
#include "traverse.hpp"

namespace rcp {
namespace {

struct PassArgs {
    DevScene sc;
    Camera cam;
    int W, H, K, k;
    float le, ld, z0;
    uint32_t n_items0;              // pass-0 items (whole super-tiles of 64-pixel tiles)
    int refill_min;                 // idle lanes that trigger a refill (1..64)
    uint32_t exit_lanes;            // searching lanes that end a traversal step early
    int tiles_x;
    int tile_log2w;                 // pass-0 tiles of 64 pixels, 2^tile_log2w wide
    int super_log2;                 // pass-0 super-tiles of 2^super_log2 tiles a side
    const float4* state_in;         // pass > 0: {pix bits, r, g, b}
    const float4* aux_in;           // pass > 0, depth/normal modes: {view depth, normal}
    const float* prev_img;          // pass 0: previous image or NULL (grey seed)
    const float* prev_aux;          // pass 0: previous [H][W][4] hit data or NULL (seed)
    float4* state_out;              // NULL: no following pass
    float4* aux_out;
    uint32_t* counters;             // [kMaxPasses] list sizes, then per pass kFetchWords band counters
                                    // at kPassFetch
    float* out;                     // [K][H][W][3]
    int32_t* ids;                   // [K][H][W] or NULL
    float* out_aux;                 // [H][W][4] of image k or NULL (single passes)
    int32_t* spill;
    uint32_t spill_stride;          // threads in the grid
    unsigned long long* stats;      // [kMaxPasses][kStatCols] or NULL
};

// The scene's counter array: list sizes, then the band counters of each pass
// (a single chain render uses the first kFetchWords words).
constexpr size_t kPassFetch = 2 * kMaxPasses + 8;
constexpr size_t kCounterWords = kPassFetch + (size_t)kMaxPasses * kFetchWords;

constexpr int kWaves = kBlock / 64;
constexpr int kStage = 128;     // per-wave staging of appended entries (flushed 64 at a time)

template <bool STATS, int MODE>
__global__ __launch_bounds__(kBlock) void k_pass(PassArgs a) {
    constexpr bool AUX = MODE != RCP_MODE_COLOR;
    extern __shared__ float4 smem[];
    float4* stage_all = smem;                                           // kWaves * kStage (x2 with aux)
    int32_t* stack_area = (int32_t*)(stage_all + (AUX ? 2 : 1) * kWaves * kStage);   // kStack * kBlock

    const int lane = threadIdx.x & 63;
    float4* stage = stage_all + (threadIdx.x >> 6) * kStage;
    float4* stage_aux = stage_all + kWaves * kStage + (threadIdx.x >> 6) * kStage;
    const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
    Stack st;
    st.lds = stack_area + threadIdx.x;
    st.spill = a.spill + gtid;
    st.stride = a.spill_stride;

    const uint32_t P = (uint32_t)a.W * (uint32_t)a.H;
    const uint32_t n_items = a.k == 0 ? a.n_items0 : a.counters[a.k];
    uint32_t* fetch = a.counters + kPassFetch + (size_t)a.k * kFetchWords;
    float* out_k = a.out + (size_t)a.k * P * 3;
    TravCount cnt;                 // STATS
    uint32_t s_rays = 0, s_app = 0;

    bool alive = false;
    bool drained = false;          // wave-uniform: the pass's list is used up
    uint32_t part = blockIdx.x % kFetchParts;   // wave-uniform: the band fetched from
    uint32_t parts_done = 0;                    // wave-uniform: bands found used up
    uint32_t fill = 0;             // wave-uniform: entries in this wave's stage
    uint32_t pix = 0;
    float pr = 0.5f, pg = 0.5f, pb = 0.5f;
    float pa[4] = {INFINITY, 0.0f, 0.0f, 0.0f};   // previous hit data (depth, normal)
    Trav tv;
    tv.node = -1;

    for (;;) {
        // ---- refill idle lanes with new work items ----------------------
        const unsigned long long idle = __ballot(!alive);
        const uint32_t n_idle = (uint32_t)__popcll(idle);
        if (!drained && n_idle >= (uint32_t)a.refill_min) {
            uint32_t base = 0, lim = 0;
            wave_fetch(fetch, n_items, n_idle, part, parts_done, drained, base, lim);
            if (!alive) {
                const uint32_t item = base + lanes_below(idle);
                bool valid = item < lim;
                int x = 0, y = 0;
                if (a.k == 0) {
                    tile_pixel(item, (uint32_t)a.tiles_x, (uint32_t)a.tile_log2w, (uint32_t)a.super_log2, x, y);
                    valid = valid && x < a.W && y < a.H;
                    pix = (uint32_t)y * (uint32_t)a.W + (uint32_t)x;
                    pr = 0.5f; pg = 0.5f; pb = 0.5f;
                    if (valid && a.prev_img) {
                        pr = a.prev_img[3 * (size_t)pix];
                        pg = a.prev_img[3 * (size_t)pix + 1];
                        pb = a.prev_img[3 * (size_t)pix + 2];
                    }
                    if (AUX) {
                        pa[0] = INFINITY; pa[1] = 0.0f; pa[2] = 0.0f; pa[3] = 0.0f;
                        if (valid && a.prev_aux) {
                            const float4 v = *(const float4*)&a.prev_aux[4 * (size_t)pix];
                            pa[0] = v.x; pa[1] = v.y; pa[2] = v.z; pa[3] = v.w;
                        }
                    }
                } else if (valid) {
                    const float4 sv = a.state_in[item];
                    pix = __float_as_uint(sv.x);
                    pr = sv.y; pg = sv.z; pb = sv.w;
                    if (AUX) {
                        const float4 v = a.aux_in[item];
                        pa[0] = v.x; pa[1] = v.y; pa[2] = v.z; pa[3] = v.w;
                    }
                    y = (int)(pix / (uint32_t)a.W);
                    x = (int)(pix - (uint32_t)y * (uint32_t)a.W);
                }
                if (valid) {
                    float ro[3], rd[3];
                    make_ray<MODE>(a.cam, half_width(a.cam.th, a.W, a.H), a.W, a.H, x, y, pr, pg, pb, pa, a.z0, a.le, a.ld, ro, rd);
                    trav_init(tv, a.sc, ro, rd, st);
                    alive = true;
                    if (STATS) ++s_rays;
                }
            }
        }
        if (__ballot(alive) == 0ull) {
            if (drained) break;
            continue;
        }

        // ---- one traversal step -------------------------------------------
        if (alive && tv.node != -1) trav_step<STATS>(tv, a.sc, st, a.exit_lanes, cnt);

        // ---- finished rays: shade, write, compact ----------------------------
        const bool done = alive && tv.node == -1;
        float rgb[3] = {0.0f, 0.0f, 0.0f};
        float na[4] = {INFINITY, 0.0f, 0.0f, 0.0f};   // this pass's hit data
        int32_t hid = -1;
        if (done) {
            if (tv.h.id != INT_MAX) {
                const float4 c = a.sc.shade[2 * (size_t)tv.h.slot + (tv.h.front ? 0 : 1)];
                rgb[0] = c.x; rgb[1] = c.y; rgb[2] = c.z;
                hid = tv.h.id;
                if (AUX || a.out_aux) {
                    // view depth of P = o + t d along the camera's forward axis; the
                    // ray is rebuilt (bit-identical) rather than kept in registers
                    const int y = (int)(pix / (uint32_t)a.W);
                    const int x = (int)(pix - (uint32_t)y * (uint32_t)a.W);
                    float ro[3], rd[3];
                    make_ray<MODE>(a.cam, half_width(a.cam.th, a.W, a.H), a.W, a.H, x, y, pr, pg, pb, pa, a.z0, a.le, a.ld, ro, rd);
                    float P3[3];
#pragma unroll
                    for (int c3 = 0; c3 < 3; ++c3) P3[c3] = ro[c3] + tv.h.t * rd[c3];
                    na[0] = ((P3[0] - a.cam.eye[0]) * a.cam.forward[0] + (P3[1] - a.cam.eye[1]) * a.cam.forward[1]) +
                            (P3[2] - a.cam.eye[2]) * a.cam.forward[2];
                    const float4 nv = a.sc.normals[tv.h.slot];
                    na[1] = nv.x; na[2] = nv.y; na[3] = nv.z;
                }
            } else {
                rgb[0] = a.sc.bg[0]; rgb[1] = a.sc.bg[1]; rgb[2] = a.sc.bg[2];
            }
            float* o3 = out_k + 3 * (size_t)pix;
            o3[0] = rgb[0]; o3[1] = rgb[1]; o3[2] = rgb[2];
            if (a.ids) a.ids[(size_t)a.k * P + pix] = hid;
            if (a.out_aux) *(float4*)&a.out_aux[4 * (size_t)pix] = make_float4(na[0], na[1], na[2], na[3]);
        }
        if (a.state_out) {
            // the next ray is a function of the colour (and, in the depth and
            // normal modes, of the hit data): unchanged inputs, unchanged result
            bool changed = done && (__float_as_uint(rgb[0]) != __float_as_uint(pr) ||
                                    __float_as_uint(rgb[1]) != __float_as_uint(pg) ||
                                    __float_as_uint(rgb[2]) != __float_as_uint(pb));
            if (AUX)
                changed = changed || (done && (__float_as_uint(na[0]) != __float_as_uint(pa[0]) ||
                                               __float_as_uint(na[1]) != __float_as_uint(pa[1]) ||
                                               __float_as_uint(na[2]) != __float_as_uint(pa[2]) ||
                                               __float_as_uint(na[3]) != __float_as_uint(pa[3])));
            const unsigned long long m = __ballot(changed);
            if (m) {
                if (changed) {
                    stage[fill + lanes_below(m)] = make_float4(__uint_as_float(pix), rgb[0], rgb[1], rgb[2]);
                    if (AUX) stage_aux[fill + lanes_below(m)] = make_float4(na[0], na[1], na[2], na[3]);
                }
                fill += (uint32_t)__popcll(m);
                if (STATS && changed) ++s_app;
                if (fill >= 64u) {
                    // flush 64 staged entries with one atomic
                    __builtin_amdgcn_wave_barrier();
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&a.counters[a.k + 1], 64u);
                    base = __shfl(base, 0);
                    a.state_out[base + lane] = stage[lane];
                    if (AUX) a.aux_out[base + lane] = stage_aux[lane];
                    __builtin_amdgcn_wave_barrier();
                    float4 rest = make_float4(0.0f, 0.0f, 0.0f, 0.0f), rest_aux = rest;
                    if ((uint32_t)lane < fill - 64u) {
                        rest = stage[64 + lane];
                        if (AUX) rest_aux = stage_aux[64 + lane];
                    }
                    __builtin_amdgcn_wave_barrier();
                    if ((uint32_t)lane < fill - 64u) {
                        stage[lane] = rest;
                        if (AUX) stage_aux[lane] = rest_aux;
                    }
                    __builtin_amdgcn_wave_barrier();
                    fill -= 64u;
                }
            }
            if (done && !changed) {
                // same inputs -> same ray -> same result in every later pass
                for (int kk = a.k + 1; kk < a.K; ++kk) {
                    float* q = a.out + ((size_t)kk * P + pix) * 3;
                    q[0] = rgb[0]; q[1] = rgb[1]; q[2] = rgb[2];
                    if (a.ids) a.ids[(size_t)kk * P + pix] = hid;
                }
            }
        }
        alive = alive && !done;
    }
    // flush what is left in the stage
    if (a.state_out && fill > 0u) {
        __builtin_amdgcn_wave_barrier();
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&a.counters[a.k + 1], fill);
        base = __shfl(base, 0);
        if ((uint32_t)lane < fill) {
            a.state_out[base + lane] = stage[lane];
            if (AUX) a.aux_out[base + lane] = stage_aux[lane];
        }
    }
    if (STATS) {
        unsigned long long* sk = a.stats + kStatCols * a.k;
        atomicAdd(&sk[0], (unsigned long long)s_rays);
        atomicAdd(&sk[1], (unsigned long long)cnt.nodes);
        atomicAdd(&sk[2], (unsigned long long)cnt.tris);
        atomicAdd(&sk[3], (unsigned long long)s_app);
        atomicAdd(&sk[4], (unsigned long long)cnt.lds);
        atomicAdd(&sk[5], (unsigned long long)cnt.spill);
    }
}

__global__ void k_clear_counters(uint32_t* c, int n, unsigned long long* stats) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0u;
    if (stats)
        for (int i = threadIdx.x; i < kStatCols * kMaxPasses; i += blockDim.x) stats[i] = 0ull;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_gen_rays(Camera cam, int W, int H, float le, float ld, float z0,
                                                      const float* __restrict__ prev, const float* __restrict__ prev_aux,
                                                      float* __restrict__ org, float* __restrict__ dir) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= (uint32_t)W * (uint32_t)H) return;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * (uint32_t)W);
    float pr = 0.5f, pg = 0.5f, pb = 0.5f;
    if (prev) { pr = prev[3 * (size_t)p]; pg = prev[3 * (size_t)p + 1]; pb = prev[3 * (size_t)p + 2]; }
    float pa[4] = {INFINITY, 0.0f, 0.0f, 0.0f};
    if (prev_aux) for (int c = 0; c < 4; ++c) pa[c] = prev_aux[4 * (size_t)p + c];
    float o[3], d[3];
    make_ray<MODE>(cam, half_width(cam.th, W, H), W, H, x, y, pr, pg, pb, pa, z0, le, ld, o, d);
    for (int c = 0; c < 3; ++c) { org[3 * (size_t)p + c] = o[c]; dir[3 * (size_t)p + c] = d[c]; }
}

__global__ __launch_bounds__(kBlock) void k_trace_rays(DevScene sc, const float* __restrict__ org,
                                                        const float* __restrict__ dir, int n, float* __restrict__ out_t,
                                                        int32_t* __restrict__ out_id, int32_t* __restrict__ out_front,
                                                        int32_t* __restrict__ spill, uint32_t stride) {
    extern __shared__ int32_t stack_area[];                             // kStack * kBlock
    const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
    Stack st;
    st.lds = stack_area + threadIdx.x;
    st.spill = spill + gtid;
    st.stride = stride;
    for (uint32_t r = gtid; r < (uint32_t)n; r += gridDim.x * kBlock) {
        float o[3], d[3];
        for (int c = 0; c < 3; ++c) { o[c] = org[3 * (size_t)r + c]; d[c] = dir[3 * (size_t)r + c]; }
        Trav tv;
        trav_init(tv, sc, o, d, st);
        TravCount cnt;
        while (tv.node != -1) trav_step<false>(tv, sc, st, 0u, cnt);
        const bool hit = tv.h.id != INT_MAX;
        out_t[r] = hit ? tv.h.t : INFINITY;
        out_id[r] = hit ? tv.h.id : -1;
        if (out_front) out_front[r] = hit && tv.h.front ? 1 : 0;
    }
}

}  // namespace

size_t counter_words() { return kCounterWords; }

namespace {

// Replace *p by a buffer of `need` elements when it holds fewer, in stream
// order on `stream`.
template <typename T>
rcp_status grow_buffer(T** p, size_t& cap, size_t need, hipStream_t stream) {
    if (need <= cap && *p) return RCP_OK;
    stream_free((void*)*p, stream);
    *p = nullptr;
    cap = 0;
    rcp_status st = stream_alloc((void**)p, sizeof(T) * need, stream);
    if (st != RCP_OK) return st;
    cap = need;
    return RCP_OK;
}

}  // namespace

rcp_status ensure_workspace(rcp_scene* s, Workspace& w, size_t n_state, size_t n_aux, size_t spill_entries,
                            hipStream_t stream) {
    (void)s;
    if (w.fixed || w.external) {
        if (n_state > w.state_cap || n_aux > w.aux_cap || spill_entries > w.spill_cap || !w.counters) {
            set_error(w.external ? "the render needs more workspace than the preallocated scratch holds"
                                 : "the render needs more workspace than was sized when the graph was created "
                                   "(launch parameters changed since); create a new graph");
            return RCP_ERR_INVALID_ARGUMENT;
        }
        return RCP_OK;
    }
    // the two lists of a pair are replaced together: the pair's capacity is
    // zero from the moment the first is released until both are allocated,
    // so a call that fails half way leaves a pair the next call regrows
    if (n_aux > w.aux_cap) {
        w.aux_cap = 0;
        for (int i = 0; i < 2; ++i) {
            size_t cap = 0;
            RCP_TRY_STATUS(grow_buffer(&w.aux[i], cap, n_aux, stream));
        }
        w.aux_cap = n_aux;
    }
    if (n_state > w.state_cap) {
        w.state_cap = 0;
        for (int i = 0; i < 2; ++i) {
            size_t cap = 0;
            RCP_TRY_STATUS(grow_buffer(&w.state[i], cap, n_state, stream));
        }
        w.state_cap = n_state;
    }
    // fixed-size buffers, each allocated once (a failed allocation leaves
    // the others as they are, and the next call tries again)
    size_t c0 = w.counters ? kCounterWords : 0;
    RCP_TRY_STATUS(grow_buffer(&w.counters, c0, kCounterWords, stream));
    size_t c1 = w.stats ? (size_t)kStatCols * kMaxPasses : 0;
    RCP_TRY_STATUS(grow_buffer(&w.stats, c1, (size_t)kStatCols * kMaxPasses, stream));
    size_t c2 = w.view ? kViewBytes : 0;
    RCP_TRY_STATUS(grow_buffer((char**)&w.view, c2, kViewBytes, stream));
    RCP_TRY_STATUS(grow_buffer(&w.spill, w.spill_cap, spill_entries, stream));
    return RCP_OK;
}

rcp_status ensure_order(Workspace& w, size_t entries, hipStream_t stream) {
    if (w.fixed || w.external) return RCP_OK;   // renders without room for it keep the screen order
    return grow_buffer(&w.order, w.order_cap, entries, stream);
}

void free_workspace(Workspace& w, hipStream_t stream) {
    if (w.external) {
        w = Workspace{};
        return;
    }
    for (int i = 0; i < 2; ++i) {
        stream_free(w.state[i], stream);
        stream_free(w.aux[i], stream);
    }
    stream_free(w.counters, stream);
    stream_free(w.spill, stream);
    stream_free(w.stats, stream);
    stream_free(w.view, stream);
    stream_free(w.order, stream);
    w = Workspace{};
}

namespace {

struct GridInfo {
    int blocks = 0;
    size_t smem = 0;
};

template <typename KernelT>
rcp_status persistent_grid(KernelT kernel, const DevScene& sc, GridInfo& g, bool aux, int blocks_per_cu) {
    g.smem = sizeof(float4) * (aux ? 2 : 1) * kWaves * kStage + sizeof(int32_t) * kStack * kBlock;
    int per_cu = 0;
    RCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, g.smem));
    int dev = 0, cus = 0;
    RCP_HIP(hipGetDevice(&dev));
    RCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu < 1) per_cu = 1;
    if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
    g.blocks = per_cu * cus;
    return RCP_OK;
}

}  // namespace

Launch launch_params(const rcp_scene* s, bool ordered) {
    Launch l;
    l.refill_min = s->tuning.refill_min > 0 ? s->tuning.refill_min
                                            : (ordered ? kDefaultRefillOrdered : kDefaultRefill);
    l.exit_lanes = s->tuning.exit_lanes >= 0 ? s->tuning.exit_lanes
                                             : (ordered ? kDefaultExitLanesOrdered : kDefaultExitLanes);
    const int lv = s->tuning.top_levels < 0 ? 0 : (s->tuning.top_levels > kTopLevels ? kTopLevels
                                                                                    : s->tuning.top_levels);
    l.top_count = s->top_nodes[lv] < kMaxStagedNodes ? s->top_nodes[lv] : kMaxStagedNodes;
    l.blocks_per_cu = s->tuning.blocks_per_cu;
    l.tile_log2w = s->tuning.tile_log2w;
    l.stack = s->tuning.stack;
    l.block = s->tuning.block;
    return l;
}

namespace {
// Debug canary of the per-pass lists (rcp_debug_set RCP_DEBUG_LIST_CANARY):
// an all-ones entry, which no list entry can be (its pixel index is below
// W * H <= 2^27 and its colours lie in [0, 1]).
__device__ inline bool is_canary(float4 v) {
    return (__float_as_uint(v.x) & __float_as_uint(v.y) & __float_as_uint(v.z) & __float_as_uint(v.w)) ==
           0xFFFFFFFFu;
}

__global__ void k_canary_fill(float4* __restrict__ st, float4* __restrict__ aux, size_t n) {
    const float4 c = make_float4(__uint_as_float(0xFFFFFFFFu), __uint_as_float(0xFFFFFFFFu),
                                 __uint_as_float(0xFFFFFFFFu), __uint_as_float(0xFFFFFFFFu));
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        st[i] = c;
        if (aux) aux[i] = c;
    }
}

// Entries [0, count - shrink) must be written, with a pixel index below P and
// colours in [0, 1]; entries [count - shrink, cap) must still hold the canary.
__global__ void k_canary_check(const float4* __restrict__ st, const float4* __restrict__ aux, size_t cap,
                               const uint32_t* __restrict__ count, uint32_t shrink, uint32_t P,
                               uint32_t* err_flag) {
    const uint32_t c = *count;
    const size_t n = c >= shrink ? c - shrink : 0;
    bool bad = (size_t)c > cap;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (size_t)gridDim.x * blockDim.x) {
        const float4 v = st[i];
        if (i < n) {
            bad = bad || is_canary(v) || __float_as_uint(v.x) >= P || !(v.y >= 0.0f && v.y <= 1.0f) ||
                  !(v.z >= 0.0f && v.z <= 1.0f) || !(v.w >= 0.0f && v.w <= 1.0f) || (aux && is_canary(aux[i]));
        } else {
            bad = bad || !is_canary(v) || (aux && !is_canary(aux[i]));
        }
    }
    if (bad) __hip_atomic_store(err_flag, kErrListCanary, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <bool STATS, int MODE>
rcp_status pass_grid(rcp_scene* s, const Launch& lp, GridInfo& g) {
    return persistent_grid(k_pass<STATS, MODE>, s->dev, g, MODE != RCP_MODE_COLOR, lp.blocks_per_cu);
}

template <bool STATS, int MODE>
rcp_status launch_passes(rcp_scene* s, Workspace& w, PassArgs& a, int K, hipStream_t stream) {
    constexpr bool AUX = MODE != RCP_MODE_COLOR;
    const Launch lp = launch_params(s);
    GridInfo g;
    rcp_status st = pass_grid<STATS, MODE>(s, lp, g);
    if (st != RCP_OK) return st;
    const uint32_t threads = (uint32_t)g.blocks * kBlock;
    const size_t P = (size_t)a.W * (size_t)a.H;
    const size_t spill_depth = spill_per_thread(s->dev);
    st = ensure_workspace(s, w, K > 1 ? P : 1, (K > 1 && AUX) ? P : 0, spill_depth * threads, stream);
    if (st != RCP_OK) return st;
    a.spill = w.spill;
    a.spill_stride = threads;
    a.counters = w.counters;
    a.stats = STATS ? w.stats : nullptr;
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(256), 0, stream, w.counters, (int)kCounterWords,
                       STATS ? w.stats : (unsigned long long*)nullptr);
    RCP_CHECK_LAUNCH();
    const int canary = debug_list_canary();
    // the lists hold P entries (the workspace may hold more)
    const size_t cap = P;
    for (int k = 0; k < K; ++k) {
        a.k = k;
        a.state_in = k == 0 ? nullptr : w.state[(k - 1) & 1];
        a.aux_in = (k == 0 || !AUX) ? nullptr : w.aux[(k - 1) & 1];
        a.state_out = k + 1 < K ? w.state[k & 1] : nullptr;
        a.aux_out = (k + 1 < K && AUX) ? w.aux[k & 1] : nullptr;
        if (k > 0) { a.prev_img = nullptr; a.prev_aux = nullptr; }
        if (canary && a.state_out) {
            hipLaunchKernelGGL(k_canary_fill, dim3(1024), dim3(256), 0, stream, a.state_out, a.aux_out, cap);
            RCP_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL((k_pass<STATS, MODE>), dim3(g.blocks), dim3(kBlock), g.smem, stream, a);
        RCP_CHECK_LAUNCH();
        if (canary && a.state_out) {
            hipLaunchKernelGGL(k_canary_check, dim3(1024), dim3(256), 0, stream, (const float4*)a.state_out,
                               (const float4*)a.aux_out, cap, (const uint32_t*)(w.counters + k + 1),
                               canary == 2 ? 1u : 0u, (uint32_t)P, s->dev.err_flag);
            RCP_CHECK_LAUNCH();
        }
    }
    return RCP_OK;
}

template <bool STATS>
rcp_status launch_mode(rcp_scene* s, Workspace& w, PassArgs& a, int K, int mode, hipStream_t stream) {
    switch (mode) {
        case RCP_MODE_DEPTH: return launch_passes<STATS, RCP_MODE_DEPTH>(s, w, a, K, stream);
        case RCP_MODE_NORMAL: return launch_passes<STATS, RCP_MODE_NORMAL>(s, w, a, K, stream);
        default: return launch_passes<STATS, RCP_MODE_COLOR>(s, w, a, K, stream);
    }
}


template <int MODE>
rcp_status prepare_mode(rcp_scene* s, Workspace& w, int W, int H, int K, hipStream_t stream) {
    const Launch lp = launch_params(s);
    GridInfo g1, g2;
    rcp_status st = pass_grid<false, MODE>(s, lp, g1);
    if (st == RCP_OK) st = pass_grid<true, MODE>(s, lp, g2);
    if (st != RCP_OK) return st;
    const uint32_t threads = (uint32_t)(g1.blocks > g2.blocks ? g1.blocks : g2.blocks) * kBlock;
    const size_t P = (size_t)W * (size_t)H;
    const size_t spill_depth = spill_per_thread(s->dev);
    return ensure_workspace(s, w, K > 1 ? P : 1, (K > 1 && MODE != RCP_MODE_COLOR) ? P : 0, spill_depth * threads,
                            stream);
}
}  // namespace

rcp_status prepare_render(rcp_scene* s, Workspace& w, int W, int H, int K, int mode, hipStream_t stream) {
    if (s->tuning.engine == RCP_ENGINE_CHAIN) return prepare_chain(s, w, W, H, mode, stream);
    switch (mode) {
        case RCP_MODE_DEPTH: return prepare_mode<RCP_MODE_DEPTH>(s, w, W, H, K, stream);
        case RCP_MODE_NORMAL: return prepare_mode<RCP_MODE_NORMAL>(s, w, W, H, K, stream);
        default: return prepare_mode<RCP_MODE_COLOR>(s, w, W, H, K, stream);
    }
}

rcp_status render(rcp_scene* s, Workspace& w, const Camera& cam, int W, int H, int K, const Disp& disp,
                  float* out_images, int32_t* out_ids, const float* prev_rgb, const float* prev_aux, float* out_aux,
                  unsigned long long* host_counts, hipStream_t stream) {
    // whole renders from the seed take the chain engine unless the per-pass
    // engine is selected; single passes with given inputs take the pass kernel
    if (s->tuning.engine == RCP_ENGINE_CHAIN && !prev_rgb && !prev_aux && !out_aux)
        return render_chain(s, w, cam, W, H, K, disp, out_images, out_ids, host_counts, stream);
    const bool stats = host_counts != nullptr;
    const Launch lp = launch_params(s);
    const int tw = 1 << lp.tile_log2w;
    const int tiles_x = (W + tw - 1) / tw;
    const int super_log2 = super_log2_for(W, H, lp.tile_log2w);
    PassArgs a{};
    a.sc = s->dev;
    a.sc.top_count = 0;          // this kernel stages nothing in LDS
    a.cam = cam;
    a.W = W; a.H = H; a.K = K;
    a.le = disp.le; a.ld = disp.ld; a.z0 = disp.z0;
    a.n_items0 = (uint32_t)view_tile_items(W, H, lp.tile_log2w, super_log2);
    a.refill_min = lp.refill_min;
    a.exit_lanes = (uint32_t)lp.exit_lanes;
    a.tiles_x = tiles_x;
    a.tile_log2w = lp.tile_log2w;
    a.super_log2 = super_log2;
    a.out = out_images;
    a.ids = out_ids;
    a.out_aux = out_aux;
    a.prev_img = prev_rgb;
    a.prev_aux = prev_aux;
    rcp_status st = stats ? launch_mode<true>(s, w, a, K, disp.mode, stream)
                          : launch_mode<false>(s, w, a, K, disp.mode, stream);
    if (st != RCP_OK) return st;
    if (stats) {
        RCP_HIP(hipMemcpyAsync(host_counts, w.stats, sizeof(unsigned long long) * kStatCols * K,
                               hipMemcpyDeviceToHost, stream));
        RCP_HIP(hipStreamSynchronize(stream));
        return take_device_error(s);
    }
    return RCP_OK;
}

rcp_status generate_rays(const Camera& cam, int W, int H, const Disp& disp, const float* prev_rgb,
                         const float* prev_aux, float* org, float* dir, hipStream_t stream) {
    const size_t P = (size_t)W * (size_t)H;
    const dim3 grid((unsigned)((P + kBlock - 1) / kBlock));
    switch (disp.mode) {
        case RCP_MODE_DEPTH:
            hipLaunchKernelGGL(k_gen_rays<RCP_MODE_DEPTH>, grid, dim3(kBlock), 0, stream, cam, W, H, disp.le, disp.ld,
                               disp.z0, prev_rgb, prev_aux, org, dir);
            break;
        case RCP_MODE_NORMAL:
            hipLaunchKernelGGL(k_gen_rays<RCP_MODE_NORMAL>, grid, dim3(kBlock), 0, stream, cam, W, H, disp.le,
                               disp.ld, disp.z0, prev_rgb, prev_aux, org, dir);
            break;
        default:
            hipLaunchKernelGGL(k_gen_rays<RCP_MODE_COLOR>, grid, dim3(kBlock), 0, stream, cam, W, H, disp.le, disp.ld,
                               disp.z0, prev_rgb, prev_aux, org, dir);
    }
    RCP_CHECK_LAUNCH();
    return RCP_OK;
}

rcp_status trace_rays(rcp_scene* s, const float* org, const float* dir, int n, float* out_t, int32_t* out_id,
                      int32_t* out_front, hipStream_t stream) {
    if (n == 0) return RCP_OK;
    GridInfo g;
    rcp_status st = persistent_grid(k_trace_rays, s->dev, g, false, 0);
    if (st != RCP_OK) return st;
    const uint32_t threads = (uint32_t)g.blocks * kBlock;
    const size_t spill_depth = spill_per_thread(s->dev);
    st = ensure_workspace(s, s->ws, 1, 0, spill_depth * threads, stream);
    if (st != RCP_OK) return st;
    DevScene sc = s->dev;
    sc.top_count = 0;            // this kernel stages nothing in LDS
    hipLaunchKernelGGL(k_trace_rays, dim3(g.blocks), dim3(kBlock), g.smem, stream, sc, org, dir, n, out_t,
                       out_id, out_front, s->ws.spill, threads);
    RCP_CHECK_LAUNCH();
    return RCP_OK;
}

}  // namespace rcp
