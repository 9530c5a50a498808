// Chain engine: every pass of a render in a single persistent launch.
//
// The recursion I_n(u,v) = F(I_{n-1}(u,v), S) is pointwise (Section 2), so a
// pixel's K passes form a chain that needs nothing from other pixels.  A work
// item is one pixel of one view (64-pixel tiles in super-tiles per view,
// views back to back, taken through one band of items per XCD); a lane
// carries its pixel through the view's passes -- trace, shade,
// write image k, and, if the inputs of the next ray changed, displace the
// camera and trace again -- and takes a new pixel as soon as the chain ends
// (after K passes, or when the colour, and in the depth and normal modes the
// hit data, stopped changing: the next ray would be identical, so the result
// is written to the remaining images at once).  No pass barrier and no
// per-pass state in HBM are needed, and views of any size, pass count and
// mode share one launch and its tail.
//
// The work that is not traversal -- finishing a traced pass (shade, write,
// decide) and setting up rays (new pixels, next passes) -- runs in setup
// rounds, when at least refill_min lanes of the wave wait for it, so that it
// runs with most of the wave's lanes instead of a few at a time.  A setup
// round also sets the wave's issue priority from the passes still ahead of
// its youngest chain: longest work first, which shortens the launch's tail
// (the last pixels handed out start chains of up to K passes).
//
// The same kernel serves rcp_render and rcp_render_batch.  Views are read
// from a device table, by each lane, or with scalar loads when the launch
// holds one view; a single render's one-entry table is written by a setup
// kernel from its by-value argument, so a captured graph holds the view and
// rcp_graph_update can change it.  (A view passed as a kernel argument lets
// the compiler hoist its uniform float math into vector registers for the
// whole loop, costing occupancy.)
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "traverse.hpp"

namespace rcp {
namespace {

struct ViewDev {
    Camera cam;
    int W, H, K, tiles_x, tile_log2w;
    int super_log2;        // log2 of the super-tile side in tiles (0: plain tile rows)
    float hw;              // half_width(cam.th, W, H)
    float le, ld, z0;
    float* out;            // [K][H][W][3]
    int32_t* ids;          // [K][H][W] or NULL
};

static_assert(sizeof(ViewDev) + 2 * sizeof(uint32_t) + 64 <= kViewBytes, "one-entry view table");

// a single render's band counters live in the scene's counter array
static_assert(kFetchWords <= 2 * kMaxPasses + 8, "band counters of a single render");

struct ChainArgs {
    DevScene sc;
    const ViewDev* views;     // [n_views]
    const uint32_t* begin;    // [n_views + 1] first work item of each view
    int n_views;
    uint32_t n_items;         // work items of the launch
    uint32_t* fetch;          // kFetchParts work counters kFetchStride words apart, zero at launch
    int refill_min;
    uint32_t exit_lanes;
    int32_t* spill;
    uint32_t spill_stride;
    unsigned long long* stats;   // [K][kStatCols] (STATS): rays, inner nodes, triangles, rays continued,
                                 // LDS node reads, stack entries spilled
    const uint32_t* order;       // single view, or NULL: item i is pixel (i & 63) of tile order[i >> 6]
};


// Lanes waiting for a setup round that start one once the bands are used up
// (measured on the terrain frame: 1 -- a round for every waiting lane --
// 0.6% slower; 4 and 12 within 0.2%; 16 and 24 slower again).
constexpr uint32_t kDrainedRound = 8;

// ONE: the launch holds a single view.  Its entry is then read with scalar
// loads (the table is constant during the launch), not per lane through the
// vector-memory path, which the traversal keeps busy.
typedef __attribute__((address_space(4))) ViewDev ConstView;

template <bool STATS, int MODE, bool ONE, int STACK, int BLOCK>
__device__ inline void chain_body(const ChainArgs& a) {
    constexpr bool AUX = MODE != RCP_MODE_COLOR;
    // LDS: the staged top levels (128-byte nodes, as in HBM, so the same
    // plane offsets serve both), then the stack area, the stats and the view
    // starts
    extern __shared__ float4 smem[];
    float4* top = smem;
    // the traversal reads staged node i at LDS byte address 128 i: the
    // dynamic LDS must begin at address 0, as it does while the kernel
    // declares no LDS of its own (otherwise the launch does nothing and
    // raises the scene's error flag)
    if ((uint32_t)(size_t)(const LdsV4*)top != 0u) {
        if (threadIdx.x == 0) __hip_atomic_store(a.sc.err_flag, kErrLdsLayout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return;
    }
    // (the stack directly after the nodes: its column addresses then carry no
    // constant offset, which the paired LDS writes of a push could not encode)
    char* lds = (char*)(smem + 8 * (size_t)a.sc.top_count);
    int32_t* stack_area = (int32_t*)lds;                                  // STACK * BLOCK
    lds += sizeof(int32_t) * STACK * BLOCK;
    unsigned long long* lstats = (unsigned long long*)lds;                // STATS: kStatCols * kMaxPasses
    if (STATS) lds += sizeof(unsigned long long) * kStatCols * kMaxPasses;
    uint32_t* vbegin = (uint32_t*)lds;                                    // n_views + 1

    const ConstView* views = (const ConstView*)a.views;
    if (!ONE)
        for (int i = threadIdx.x; i <= a.n_views; i += BLOCK) vbegin[i] = a.begin[i];
    for (uint32_t i = threadIdx.x; i < 8u * a.sc.top_count; i += BLOCK)
        if ((i & 7u) != 7u) top[i] = a.sc.nodes[i];   // the zero padding is never read
    if (STATS)
        for (int i = threadIdx.x; i < kStatCols * kMaxPasses; i += BLOCK) lstats[i] = 0ull;
    __syncthreads();

    int v = 0;                 // the lane's view

    const uint32_t gtid = blockIdx.x * BLOCK + threadIdx.x;
    StackT<STACK, BLOCK> st;
    st.lds = stack_area + threadIdx.x;
    st.spill = a.spill + gtid;
    st.stride = a.spill_stride;
    const uint32_t n_items = a.n_items;

    bool alive = false;        // tracing a ray
    bool ended = false;        // its pass is traced, waiting for a setup round to be finished
    bool pending = false;      // holds the inputs of its next pass, waiting for a setup round
    bool drained = false;      // wave-uniform
    uint32_t part = blockIdx.x % kFetchParts;   // wave-uniform: the band fetched from
    uint32_t parts_done = 0;                    // wave-uniform: bands found used up
    int k = 0, x = 0, y = 0;
    float pr = 0.5f, pg = 0.5f, pb = 0.5f;              // previous colour (the seed I_0 at pass 0)
    float pa[4] = {INFINITY, 0.0f, 0.0f, 0.0f};         // previous hit data: view depth, unit normal
    TravCount cnt;                                      // STATS: counters of the current ray
    Trav tv;
    tv.node = -1;

    for (;;) {
        // ---- setup round, when enough lanes wait: finish the traced passes,
        // fetch new pixels for idle lanes, and set up the rays of new pixels and
        // of next passes together (work done by a few lanes alone wastes the wave)
        // Once the bands are used up, lanes waiting for their next pass no
        // longer wait for refill_min idle lanes (their chains decide when the
        // launch ends), but for kDrainedRound of them, or for the wave's last
        // ray to end: a round costs the same for 1 lane as for 64.
        const unsigned long long need = wave_ballot(!alive);
        const unsigned long long waiting = wave_ballot(ended || pending);
        const uint32_t n_need = popc_u32(need), n_wait = popc_u32(waiting);
        if (n_need >= (uint32_t)a.refill_min ||
            (drained && n_wait != 0u && (n_wait >= kDrainedRound || n_need == 64u))) {
            // lanes whose pass is traced: shade, write, and keep the inputs
            // of the next pass or end the chain
            if (ended) {
                {
                    const ConstView& vw = views[ONE ? 0 : v];
                    float rgb[3];
                    float na[4] = {INFINITY, 0.0f, 0.0f, 0.0f};
                    int32_t hid = -1;
                    if (tv.h.id != INT_MAX) {
                        const float4 c = a.sc.shade[2 * (size_t)tv.h.slot + (tv.h.front ? 0 : 1)];
                        rgb[0] = c.x; rgb[1] = c.y; rgb[2] = c.z;
                        hid = tv.h.id;
                        if (AUX) {
                            // view depth of P = o + t d along the camera's forward axis; the
                            // ray is rebuilt (bit-identical) rather than kept in registers
                            float ro[3], rd[3];
                            make_ray<MODE>(vw.cam, vw.hw, vw.W, vw.H, x, y, pr, pg, pb, pa, vw.z0, vw.le, vw.ld, ro,
                                           rd);
                            float P3[3];
#pragma unroll
                            for (int c3 = 0; c3 < 3; ++c3) P3[c3] = ro[c3] + tv.h.t * rd[c3];
                            na[0] = ((P3[0] - vw.cam.eye[0]) * vw.cam.forward[0] +
                                     (P3[1] - vw.cam.eye[1]) * vw.cam.forward[1]) +
                                    (P3[2] - vw.cam.eye[2]) * vw.cam.forward[2];
                            const float4 nv = a.sc.normals[tv.h.slot];
                            na[1] = nv.x; na[2] = nv.y; na[3] = nv.z;
                        }
                    } else {
                        rgb[0] = a.sc.bg[0]; rgb[1] = a.sc.bg[1]; rgb[2] = a.sc.bg[2];
                    }
                    const size_t P = (size_t)vw.W * (size_t)vw.H;
                    const size_t pix = (size_t)y * (size_t)vw.W + (size_t)x;
                    // the next ray is a function of the colour (and, in the depth and
                    // normal modes, of the hit data): unchanged inputs, unchanged result
                    bool changed = __float_as_uint(rgb[0]) != __float_as_uint(pr) ||
                                   __float_as_uint(rgb[1]) != __float_as_uint(pg) ||
                                   __float_as_uint(rgb[2]) != __float_as_uint(pb);
                    if (AUX)
                        changed = changed || __float_as_uint(na[0]) != __float_as_uint(pa[0]) ||
                                  __float_as_uint(na[1]) != __float_as_uint(pa[1]) ||
                                  __float_as_uint(na[2]) != __float_as_uint(pa[2]) ||
                                  __float_as_uint(na[3]) != __float_as_uint(pa[3]);
                    // image k, and every later image when nothing changed
                    const int k_end = changed ? k + 1 : vw.K;
                    for (int kk = k; kk < k_end; ++kk) {
                        float* q = vw.out + ((size_t)kk * P + pix) * 3;
                        q[0] = rgb[0]; q[1] = rgb[1]; q[2] = rgb[2];
                        if (vw.ids) vw.ids[(size_t)kk * P + pix] = hid;
                    }
                    const bool next = changed && k + 1 < vw.K;
                    if (STATS) {
                        unsigned long long* sk = lstats + kStatCols * k;
                        atomicAdd(&sk[0], 1ull);
                        atomicAdd(&sk[1], (unsigned long long)cnt.nodes);
                        atomicAdd(&sk[2], (unsigned long long)cnt.tris);
                        if (next) atomicAdd(&sk[3], 1ull);
                        atomicAdd(&sk[4], (unsigned long long)cnt.lds);
                        atomicAdd(&sk[5], (unsigned long long)cnt.spill);
                        cnt = TravCount();
                    }
                    if (next) {
                        ++k;
                        pr = rgb[0]; pg = rgb[1]; pb = rgb[2];
                        if (AUX) { pa[0] = na[0]; pa[1] = na[1]; pa[2] = na[2]; pa[3] = na[3]; }
                        pending = true;
                    }
                }
                ended = false;
            }
            const unsigned long long idle = wave_ballot(!alive && !pending);
            const uint32_t n_idle = (uint32_t)__popcll(idle);
            uint32_t base = 0, lim = 0;
            const bool fetch = !drained && n_idle > 0u;
            if (fetch) wave_fetch(a.fetch, n_items, n_idle, part, parts_done, drained, base, lim);
            bool init = pending;
            if (fetch && !alive && !pending) {
                const uint32_t item = base + lanes_below(idle);
                if (item < lim) {
                    // the view holding this item: last begin <= item
                    if (!ONE) {
                        int lo = 0, hi = a.n_views;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (vbegin[mid] <= item) lo = mid; else hi = mid;
                        }
                        v = lo;
                    }
                    const uint32_t local = ONE ? (a.order ? (a.order[item >> 6] << 6) | (item & 63u) : item)
                                               : item - vbegin[v];
                    {
                        const ConstView& vw = views[ONE ? 0 : v];
                        tile_pixel(local, (uint32_t)vw.tiles_x, (uint32_t)vw.tile_log2w, (uint32_t)vw.super_log2, x, y);
                        if (x < vw.W && y < vw.H) {
                            k = 0;
                            pr = 0.5f; pg = 0.5f; pb = 0.5f;
                            pa[0] = INFINITY; pa[1] = 0.0f; pa[2] = 0.0f; pa[3] = 0.0f;
                            init = true;
                        }
                    }
                }
            }
            {
                // Longest remaining work first: the wave's issue priority follows
                // the passes still ahead of its youngest chain (at most K - k),
                // so that the chains started last, which decide when the launch
                // ends, are not slowed down by waves about to finish.
                // (Measured on the terrain frame: 3.7% faster; applied only once
                // the bands are used up, 3.0%.)
                const int kk = views[ONE ? 0 : v].K;
                const bool live = alive || init;
                const int rem = kk - k;
                if (wave_ballot(live && 3 * rem >= 2 * kk) != 0ull) __builtin_amdgcn_s_setprio(3);
                else if (wave_ballot(live && 2 * rem >= kk) != 0ull) __builtin_amdgcn_s_setprio(2);
                else if (wave_ballot(live && 3 * rem >= kk) != 0ull) __builtin_amdgcn_s_setprio(1);
                else __builtin_amdgcn_s_setprio(0);
            }
            if (init) {
                const ConstView& vw = views[ONE ? 0 : v];
                float o[3], d[3];
                make_ray<MODE>(vw.cam, vw.hw, vw.W, vw.H, x, y, pr, pg, pb, pa, vw.z0, vw.le, vw.ld, o, d);
                trav_init(tv, a.sc, o, d, st);
                if (STATS) cnt = TravCount();
                alive = true;
                pending = false;
            }
        }
        if (wave_ballot(alive) == 0ull) {
            if (drained && wave_ballot(pending || ended) == 0ull) break;
            continue;
        }

        // ---- one traversal step -------------------------------------------------
        if (alive && tv.node != -1) trav_step<STATS>(tv, a.sc, st, a.exit_lanes, cnt);

        if (alive && tv.node == -1) {   // the pass is traced: finish it in the next round
            alive = false;
            ended = true;
        }
    }

    if (STATS) {
        __syncthreads();
        for (int i = threadIdx.x; i < kStatCols * kMaxPasses; i += BLOCK)
            if (lstats[i]) atomicAdd(&a.stats[i], lstats[i]);
    }
}

// Colour mode, the default: asking for 6 waves per SIMD (at most 80 VGPRs)
// was measured faster than the 5 the compiler picks alone; 7 and 8 spill and
// are slower.  The depth and normal modes keep the compiler's choice (6
// spills there and measured 1% slower).  STACK (LDS stack entries per lane)
// and BLOCK (workgroup size) are launch parameters the autotuner chooses
// among for the colour mode's timed kernel; the instrumented kernel and the
// depth and normal modes use kStack and kBlock.
template <bool STATS, bool ONE, int STACK, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_chain(ChainArgs a) {
    chain_body<STATS, RCP_MODE_COLOR, ONE, STACK, BLOCK>(a);
}

template <bool STATS, int MODE, bool ONE>
__global__ __launch_bounds__(kBlock) void k_chain_aux(ChainArgs a) {
    chain_body<STATS, MODE, ONE, kStack, kBlock>(a);
}

// Zero the work counters (kFetchParts per launch) and the stats.
__global__ void k_clear_chain(uint32_t* fetch, int n, unsigned long long* stats) {
    for (int i = threadIdx.x; i < (int)kFetchWords * n; i += blockDim.x) fetch[i] = 0u;
    if (stats)
        for (int i = threadIdx.x; i < kStatCols * kMaxPasses; i += blockDim.x) stats[i] = 0ull;
}

// Setup of a one-view launch (a single render, or a batch of one view): its
// one-entry view table, item range, band counters and stats.
// A single render's one-entry view table, zeroed band counters (and stats).
__device__ inline void setup_single(const ViewDev& v, ViewDev* table, uint32_t* begin, uint32_t n_items,
                                    uint32_t* fetch, unsigned long long* stats) {
    if (threadIdx.x == 0) {
        *table = v;
        begin[0] = 0u;
        begin[1] = n_items;
        for (uint32_t p = 0; p < kFetchParts; ++p) fetch[kFetchStride * p] = 0u;
    }
    if (stats)
        for (int i = threadIdx.x; i < kStatCols * kMaxPasses; i += blockDim.x) stats[i] = 0ull;
}

// ---- Cost order of a single render's tiles -----------------------------------
// A tile's score is the largest number of occupied cells of the scene's
// occupancy grid that one of four undisplaced rays crosses, through the
// centres of the tile's quadrants (a voxel walk after Amanatides and Woo, "A
// Fast Voxel Traversal Algorithm for Ray Tracing", Eurographics 1987): a
// tile's wave is as slow as its slowest lane.  Each ray's segment inside the
// grid is walked in two halves by two threads, which halves the longest walk,
// the one that sets the kernel's time.  Rays that skim many occupied cells
// tend to start long chains; within each band the tiles are handed out by
// decreasing score, so that those chains start first and the launch's tail,
// set by the chains started last, gets shorter.  The order decides only when
// a pixel is rendered, never its result.
constexpr uint32_t kScoreBins = 256;

constexpr uint32_t kScoreBlock = 256;

__global__ __launch_bounds__(kScoreBlock) void k_tile_scores(ViewDev v, OccGrid g, uint32_t n_tiles, uint32_t* score) {
    extern __shared__ uint32_t occ[];
    for (uint32_t i = threadIdx.x; i < g.words; i += kScoreBlock) occ[i] = g.bits[i];
    __syncthreads();
    // eight neighbouring threads per tile: the quadrant in the low two bits,
    // the half of the ray's walk in the third; every thread reaches the
    // shuffles at the end
    const uint32_t gt = blockIdx.x * kScoreBlock + threadIdx.x;
    const uint32_t t = gt >> 3, sub = gt & 3u, half = (gt >> 2) & 1u;
    const uint32_t tw = 1u << (uint32_t)v.tile_log2w, th = 64u >> (uint32_t)v.tile_log2w;
    int x0 = 0, y0 = 0, x = 0, y = 0;
    if (t < n_tiles) tile_pixel(t << 6, (uint32_t)v.tiles_x, (uint32_t)v.tile_log2w, (uint32_t)v.super_log2, x0, y0);
    const bool live = t < n_tiles && x0 < v.W && y0 < v.H;
    const uint32_t sx = (sub & 1u) ? (3u * tw) / 4u : tw / 4u, sy = (sub & 2u) ? (3u * th) / 4u : th / 4u;
    tile_pixel((t << 6) + sy * tw + sx, (uint32_t)v.tiles_x, (uint32_t)v.tile_log2w,
               (uint32_t)v.super_log2, x, y);
    x = x < v.W ? x : v.W - 1;
    y = y < v.H ? y : v.H - 1;
    const float fx = (float)(2 * x + 1) / (float)v.W - 1.0f;
    const float fy = 1.0f - (float)(2 * y + 1) / (float)v.H;
    float o[3], d[3], inv[3];
    float tmin = 0.0f, tmax = INFINITY;
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = v.cam.eye[a];
        d[a] = v.cam.forward[a] + fx * v.hw * v.cam.right[a] + fy * v.cam.th * v.cam.up[a];
        const float lo = g.lo[a], hi = g.lo[a] + g.cell[a] * (float)g.n[a];
        if (d[a] == 0.0f) {
            inv[a] = INFINITY;
            miss = miss || o[a] < lo || o[a] > hi;
        } else {
            inv[a] = 1.0f / d[a];
            const float t0 = (lo - o[a]) * inv[a], t1 = (hi - o[a]) * inv[a];
            tmin = fmaxf(tmin, fminf(t0, t1));
            tmax = fminf(tmax, fmaxf(t0, t1));
        }
    }
    uint32_t count = 0;
    if (live && !miss && tmin <= tmax) {
        const float tmid = 0.5f * (tmin + tmax);
        const float tbeg = half ? tmid : tmin, tend = half ? tmax : tmid;
        // per axis: the next boundary's t, its spacing, the cell index stride
        // of a step and the steps left inside the grid
        float tnext[3], tdelta[3];
        int stride[3];
        uint32_t left[3];
        int cell = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float p = o[a] + tbeg * d[a];
            int q = (int)floorf((p - g.lo[a]) / g.cell[a]);
            q = q < 0 ? 0 : (q >= g.n[a] ? g.n[a] - 1 : q);
            const int step = d[a] > 0.0f ? 1 : (d[a] < 0.0f ? -1 : 0);
            tnext[a] = step == 0 ? INFINITY
                                 : (g.lo[a] + (float)(q + (step > 0 ? 1 : 0)) * g.cell[a] - o[a]) * inv[a];
            tdelta[a] = step == 0 ? INFINITY : g.cell[a] * fabsf(inv[a]);
            const int unit = a == 0 ? 1 : (a == 1 ? g.n[0] : g.n[0] * g.n[1]);
            stride[a] = step * unit;
            left[a] = step > 0 ? (uint32_t)(g.n[a] - 1 - q) : (step < 0 ? (uint32_t)q : 0u);
            cell += q * unit;
        }
        // one step per iteration, without branches: the axis whose boundary
        // comes first (x, then y, then z among equal ones); the walk ends past
        // tend or at the grid's side.  The second half's first cell is the
        // first half's last, counted there.
        const int steps = g.n[0] + g.n[1] + g.n[2];
        for (int it = 0; it < steps; ++it) {
            count += (it > 0 || half == 0u) ? (occ[(uint32_t)cell >> 5] >> ((uint32_t)cell & 31u)) & 1u : 0u;
            const bool ax = tnext[0] <= tnext[1] && tnext[0] <= tnext[2];
            const bool ay = !ax && tnext[1] <= tnext[2];
            const bool az = !ax && !ay;
            const float tn = ax ? tnext[0] : (ay ? tnext[1] : tnext[2]);
            const uint32_t l = ax ? left[0] : (ay ? left[1] : left[2]);
            if (tn > tend || l == 0u) break;
            cell += ax ? stride[0] : (ay ? stride[1] : stride[2]);
            tnext[0] += ax ? tdelta[0] : 0.0f;
            tnext[1] += ay ? tdelta[1] : 0.0f;
            tnext[2] += az ? tdelta[2] : 0.0f;
            left[0] -= ax ? 1u : 0u;
            left[1] -= ay ? 1u : 0u;
            left[2] -= az ? 1u : 0u;
        }
    }
    count += (uint32_t)__shfl_xor((int)count, 4);   // the ray's two halves
    count = max(count, (uint32_t)__shfl_xor((int)count, 1));
    count = max(count, (uint32_t)__shfl_xor((int)count, 2));
    if (sub == 0u && half == 0u && t < n_tiles) score[t] = count;
}

// One workgroup per band: a counting sort of the band's tiles by decreasing
// score (order within a score is the order of arrival, which only moves
// work in time).  Every tile of the band lands in exactly one slot of the
// band's range, so order[] is a permutation of the tiles.  One more
// workgroup does the launch's setup (the work of k_setup_single).
__global__ __launch_bounds__(1024) void k_band_order(const uint32_t* __restrict__ score, uint32_t n_items,
                                                     uint32_t* __restrict__ order, ViewDev v, ViewDev* table,
                                                     uint32_t* begin, uint32_t* fetch, unsigned long long* stats) {
    if (blockIdx.x == kFetchParts) {
        setup_single(v, table, begin, n_items, fetch, stats);
        return;
    }
    __shared__ uint32_t hist[kScoreBins];
    const uint32_t lo = part_begin(n_items, blockIdx.x) >> 6, hi = part_begin(n_items, blockIdx.x + 1u) >> 6;
    for (uint32_t i = threadIdx.x; i < kScoreBins; i += 1024) hist[i] = 0u;
    __syncthreads();
    for (uint32_t t = lo + threadIdx.x; t < hi; t += 1024) {
        const uint32_t b = score[t] < kScoreBins ? score[t] : kScoreBins - 1u;
        atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    // each bin's first slot: the tiles of all higher scores come before it
    // (a scan over the bins from the highest down, kScoreBins threads)
    __shared__ uint32_t scan[kScoreBins];
    const uint32_t own = threadIdx.x < kScoreBins ? hist[kScoreBins - 1u - threadIdx.x] : 0u;
    if (threadIdx.x < kScoreBins) scan[threadIdx.x] = own;
    __syncthreads();
    for (uint32_t off = 1; off < kScoreBins; off <<= 1) {
        const uint32_t add = (threadIdx.x < kScoreBins && threadIdx.x >= off) ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        if (threadIdx.x < kScoreBins) scan[threadIdx.x] += add;
        __syncthreads();
    }
    if (threadIdx.x < kScoreBins) hist[kScoreBins - 1u - threadIdx.x] = scan[threadIdx.x] - own;
    __syncthreads();
    for (uint32_t t = lo + threadIdx.x; t < hi; t += 1024) {
        const uint32_t b = score[t] < kScoreBins ? score[t] : kScoreBins - 1u;
        order[lo + atomicAdd(&hist[b], 1u)] = t;
    }
}

__global__ void k_setup_single(ViewDev v, ViewDev* table, uint32_t* begin, uint32_t n_items, uint32_t* fetch,
                               unsigned long long* stats) {
    setup_single(v, table, begin, n_items, fetch, stats);
}

// A chain kernel instantiation with its workgroup size and stack depth.
struct ChainKernel {
    const void* fn;
    int block;
    int stack;
};

template <bool STATS, bool ONE>
ChainKernel colour_kernel(int stack, int block) {
    if constexpr (!STATS) {
        if (stack == 8 && block == 512) return {(const void*)k_chain<false, ONE, 8, 512>, 512, 8};
        if (stack == 8) return {(const void*)k_chain<false, ONE, 8, kBlock>, kBlock, 8};
        if (block == 512) return {(const void*)k_chain<false, ONE, kStack, 512>, 512, kStack};
    }
    return {(const void*)k_chain<STATS, ONE, kStack, kBlock>, kBlock, kStack};
}

template <bool STATS, bool ONE>
ChainKernel chain_kernel1(int mode, const Launch& lp) {
    switch (mode) {
        case RCP_MODE_DEPTH: return {(const void*)k_chain_aux<STATS, RCP_MODE_DEPTH, ONE>, kBlock, kStack};
        case RCP_MODE_NORMAL: return {(const void*)k_chain_aux<STATS, RCP_MODE_NORMAL, ONE>, kBlock, kStack};
        default: return colour_kernel<STATS, ONE>(lp.stack, lp.block);
    }
}

// The kernel of a launch over n_views views in `mode` (the single-view
// kernels when n_views == 1).
ChainKernel chain_kernel(bool stats, int n_views, int mode, const Launch& lp) {
    if (stats) return n_views == 1 ? chain_kernel1<true, true>(mode, lp) : chain_kernel1<true, false>(mode, lp);
    return n_views == 1 ? chain_kernel1<false, true>(mode, lp) : chain_kernel1<false, false>(mode, lp);
}

// LDS of a workgroup: the staged top levels, the stack area and the view
// starts (and the stats).
size_t chain_smem(const Launch& lp, const ChainKernel& k, bool stats, int n_views) {
    size_t b = kNodeBytes * (size_t)lp.top_count + sizeof(int32_t) * (size_t)k.stack * (size_t)k.block +
               sizeof(uint32_t) * (size_t)((n_views + 4) & ~3);
    if (stats) b += sizeof(unsigned long long) * kStatCols * kMaxPasses;
    return b;
}

// Resident workgroups per CU and CU count of a kernel at an LDS size, on the
// current device.  The runtime's answers are cached: they cannot change in a
// process, and asking costs more than a launch.
rcp_status occupancy(const ChainKernel& k, size_t smem, int& per_cu, int& cus) {
    static std::mutex mu;
    static std::map<std::tuple<const void*, size_t, int>, std::pair<int, int>> cache;
    int dev = 0;
    RCP_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(k.fn, smem, dev);
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            per_cu = it->second.first;
            cus = it->second.second;
            return RCP_OK;
        }
    }
    RCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k.fn, k.block, smem));
    RCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = std::make_pair(per_cu, cus);
    return RCP_OK;
}

// Kernel, grid and LDS size of a launch over n_views views in `mode`.
struct ChainGrid {
    ChainKernel k;
    int blocks = 0;
    size_t smem = 0;
    uint32_t threads() const { return (uint32_t)blocks * (uint32_t)k.block; }
};

rcp_status chain_grid(const Launch& lp, bool stats, int n_views, int mode, ChainGrid& g) {
    g.k = chain_kernel(stats, n_views, mode, lp);
    g.smem = chain_smem(lp, g.k, stats, n_views);
    int per_cu = 0, cus = 0;
    const rcp_status st = occupancy(g.k, g.smem, per_cu, cus);
    if (st != RCP_OK) return st;
    if (per_cu < 1) per_cu = 1;
    // blocks_per_cu counts workgroups of kBlock threads; a larger workgroup
    // counts as several
    if (lp.blocks_per_cu > 0) {
        const int cap = std::max(1, lp.blocks_per_cu * kBlock / g.k.block);
        if (cap < per_cu) per_cu = cap;
    }
    g.blocks = per_cu * cus;
    return RCP_OK;
}

rcp_status launch_chain(const ChainGrid& g, hipStream_t stream, ChainArgs a) {
    void* args[] = {(void*)&a};
    RCP_HIP(hipLaunchKernel(g.k.fn, dim3((unsigned)g.blocks), dim3((unsigned)g.k.block), args, g.smem, stream));
    return RCP_OK;
}

size_t spill_depth_of(const rcp_scene* s, const ChainKernel& k) {
    return spill_per_thread(s->dev, k.stack);
}

ViewDev view_of(const Camera& cam, int W, int H, int K, const Disp& d, float* out, int32_t* ids, int tile_log2w) {
    ViewDev v{};
    v.cam = cam;
    v.W = W; v.H = H; v.K = K;
    v.hw = half_width(cam.th, W, H);
    v.tile_log2w = tile_log2w;
    v.tiles_x = (W + (1 << tile_log2w) - 1) >> tile_log2w;
    v.super_log2 = super_log2_for(W, H, tile_log2w);
    v.le = d.le; v.ld = d.ld; v.z0 = d.z0;
    v.out = out;
    v.ids = ids;
    return v;
}

uint64_t view_items(const ViewDev& v) {
    return view_tile_items(v.W, v.H, v.tile_log2w, v.super_log2);
}

// Entries of a view's score and order buffer: two per tile.
size_t order_entries(int W, int H, int tile_log2w) {
    return 2 * (size_t)(view_tile_items(W, H, tile_log2w, super_log2_for(W, H, tile_log2w)) >> 6);
}

}  // namespace

rcp_status prepare_chain(rcp_scene* s, Workspace& ws, int W, int H, int mode, hipStream_t stream) {
    const Launch lp = launch_params(s, chain_ordered(s));
    ChainGrid g1, g2;
    rcp_status st = chain_grid(lp, false, 1, mode, g1);
    if (st == RCP_OK) st = chain_grid(lp, true, 1, mode, g2);
    if (st != RCP_OK) return st;
    const size_t need = std::max(spill_depth_of(s, g1.k) * g1.threads(), spill_depth_of(s, g2.k) * g2.threads());
    st = ensure_workspace(s, ws, 0, 0, need, stream);
    if (st != RCP_OK) return st;
    return ensure_order(ws, order_entries(W, H, lp.tile_log2w), stream);
}

namespace {

// Enqueue the setup kernel and the chain launch of one view on a workspace
// that already fits the grid.
rcp_status launch_one_view(rcp_scene* s, Workspace& w, const Launch& lp, const ChainGrid& g, const Camera& cam,
                           int W, int H, int K, const Disp& disp, float* out_images, int32_t* out_ids, bool stats,
                           hipStream_t stream) {
    const ViewDev view = view_of(cam, W, H, K, disp, out_images, out_ids, lp.tile_log2w);
    ChainArgs a{};
    a.sc = s->dev;
    a.sc.top_count = lp.top_count;
    a.views = (const ViewDev*)w.view;
    a.begin = (const uint32_t*)((char*)w.view + ((sizeof(ViewDev) + 63) & ~(size_t)63));
    a.n_views = 1;
    a.n_items = (uint32_t)view_items(view);
    a.fetch = w.counters;
    a.refill_min = lp.refill_min;
    a.exit_lanes = (uint32_t)lp.exit_lanes;
    a.spill = w.spill;
    a.spill_stride = g.threads();
    a.stats = stats ? w.stats : nullptr;
    a.order = nullptr;
    const uint32_t n_tiles = a.n_items >> 6;
    if (s->tuning.tile_order && s->occ.bits && w.order && w.order_cap >= 2 * (size_t)n_tiles && n_tiles > 0) {
        // tile scores in the second half of the buffer, the order in the first
        uint32_t* score = w.order + n_tiles;
        hipLaunchKernelGGL(k_tile_scores, dim3((8 * n_tiles + kScoreBlock - 1) / kScoreBlock), dim3(kScoreBlock),
                           sizeof(uint32_t) * s->occ.words, stream, view, s->occ, n_tiles, score);
        hipLaunchKernelGGL(k_band_order, dim3(kFetchParts + 1), dim3(1024), 0, stream, (const uint32_t*)score,
                           a.n_items, w.order, view, (ViewDev*)a.views, (uint32_t*)a.begin, w.counters, a.stats);
        RCP_CHECK_LAUNCH();
        a.order = w.order;
    } else {
        hipLaunchKernelGGL(k_setup_single, dim3(1), dim3(256), 0, stream, view, (ViewDev*)a.views,
                           (uint32_t*)a.begin, a.n_items, w.counters, a.stats);
        RCP_CHECK_LAUNCH();
    }
    return launch_chain(g, stream, a);
}

}  // namespace

rcp_status render_chain(rcp_scene* s, Workspace& w, const Camera& cam, int W, int H, int K, const Disp& disp,
                        float* out_images, int32_t* out_ids, unsigned long long* host_counts, hipStream_t stream) {
    const bool stats = host_counts != nullptr;
    const Launch lp = launch_params(s, chain_ordered(s));
    ChainGrid g;
    rcp_status st = chain_grid(lp, stats, 1, disp.mode, g);
    if (st != RCP_OK) return st;
    st = ensure_workspace(s, w, 0, 0, spill_depth_of(s, g.k) * g.threads(), stream);
    if (st != RCP_OK) return st;
    st = ensure_order(w, order_entries(W, H, lp.tile_log2w), stream);
    if (st != RCP_OK) return st;
    st = launch_one_view(s, w, lp, g, cam, W, H, K, disp, out_images, out_ids, stats, stream);
    if (st != RCP_OK) return st;
    if (stats) {
        RCP_HIP(hipMemcpyAsync(host_counts, w.stats, sizeof(unsigned long long) * kStatCols * K,
                               hipMemcpyDeviceToHost, stream));
        RCP_HIP(hipStreamSynchronize(stream));
        return take_device_error(s);
    }
    return RCP_OK;
}

rcp_status render_chain_fixed(rcp_scene* s, Workspace& w, const Camera& cam, int W, int H, int K,
                              const Disp& disp, float* out_images, int32_t* out_ids, hipStream_t stream) {
    // the cost order where the workspace's order area holds the view's tiles
    const bool ordered = chain_ordered(s) && w.order &&
                         w.order_cap >= order_entries(W, H, launch_params(s, true).tile_log2w);
    const Launch lp = launch_params(s, ordered);
    ChainGrid g;
    rcp_status st = chain_grid(lp, false, 1, disp.mode, g);
    if (st != RCP_OK) return st;
    int dev = 0, cus = 0;
    RCP_HIP(hipGetDevice(&dev));
    RCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // as many workgroups as the overflow area holds (the grid size changes
    // the speed only), but at least one per compute unit
    const size_t per_block = spill_depth_of(s, g.k) * (size_t)g.k.block;
    const size_t fit = w.spill_cap / per_block;
    if (fit < (size_t)cus) {
        set_error("the scene's traversal stack needs %zu bytes of overflow area per compute unit's workgroup; "
                  "the preallocated scratch holds %zu for %d compute units",
                  per_block * sizeof(int32_t), w.spill_cap * sizeof(int32_t), cus);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    if ((size_t)g.blocks > fit) g.blocks = (int)fit;
    return launch_one_view(s, w, lp, g, cam, W, H, K, disp, out_images, out_ids, false, stream);
}

namespace {

// Grow a batch buffer in stream order.
template <typename T>
rcp_status grow(T** p, size_t& cap, size_t need, size_t bytes_each, hipStream_t stream) {
    if (need <= cap && *p) return RCP_OK;
    stream_free((void*)*p, stream);
    *p = nullptr;
    cap = 0;
    rcp_status st = stream_alloc((void**)p, bytes_each * need, stream);
    if (st != RCP_OK) return st;
    cap = need;
    return RCP_OK;
}

size_t view_table_bytes(size_t n_views) {
    return ((sizeof(ViewDev) * n_views + 255) & ~(size_t)255) + sizeof(uint32_t) * (n_views + 3);
}

}  // namespace

rcp_status prepare_batch_workspace(rcp_scene* s, BatchWorkspace& ws, int n_views, bool with_staging,
                                   hipStream_t stream) {
    const Launch lp = launch_params(s);
    size_t spill_need = 0;
    for (int mode = 0; mode < 3; ++mode)
        for (int nv : {1, 2}) {
            ChainGrid g;
            rcp_status st = chain_grid(lp, false, nv, mode, g);
            if (st != RCP_OK) return st;
            spill_need = std::max(spill_need, spill_depth_of(s, g.k) * g.threads());
        }
    rcp_status st = RCP_OK;
    if ((size_t)n_views > ws.view_cap || !ws.views) {
        stream_free(ws.views, stream);
        ws.views = nullptr;
        ws.view_cap = 0;
        st = stream_alloc(&ws.views, view_table_bytes((size_t)n_views), stream);
        if (st == RCP_OK) ws.view_cap = (size_t)n_views;
    }
    size_t fetch_cap = ws.fetch ? kFetchWords * 3 : 0;
    if (st == RCP_OK) st = grow(&ws.fetch, fetch_cap, kFetchWords * 3, sizeof(uint32_t), stream);
    if (st == RCP_OK)
        st = grow(&ws.spill, ws.spill_cap, spill_need, sizeof(int32_t), stream);
    if (st == RCP_OK && with_staging && ws.order_cap < 2 * kServerOrderTiles)
        st = grow(&ws.order, ws.order_cap, 2 * kServerOrderTiles, sizeof(uint32_t), stream);
    if (st == RCP_OK && with_staging && !ws.staging) {
        if (alloc_hook_fails()) {
            set_error("pinned host allocation failed (test hook)");
            return RCP_ERR_OUT_OF_MEMORY;
        }
        RCP_HIP(hipHostMalloc(&ws.staging, view_table_bytes((size_t)n_views), hipHostMallocDefault));
    }
    return st;
}

rcp_status render_batch(rcp_scene* s, const rcp_view* views, int n_views, BatchWorkspace& ws, hipStream_t stream) {
    const Launch lp = launch_params(s);
    // views grouped by displacement mode, one launch per mode present
    std::vector<int> order((size_t)n_views);
    for (int i = 0; i < n_views; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int p, int q) { return views[p].disp.mode < views[q].disp.mode; });
    std::vector<ViewDev> hv((size_t)n_views);
    std::vector<uint32_t> hb((size_t)n_views + 3);   // begin arrays of the groups, back to back
    struct Group { int mode, first, count; size_t bofs; uint32_t items; };
    std::vector<Group> groups;
    uint64_t items = 0;
    size_t bofs = 0;
    for (int j = 0; j < n_views; ++j) {
        const rcp_view& vi = views[order[(size_t)j]];
        if (groups.empty() || groups.back().mode != vi.disp.mode) {
            if (!groups.empty()) {
                hb[bofs++] = (uint32_t)items;
                groups.back().items = (uint32_t)items;
            }
            groups.push_back(Group{vi.disp.mode, j, 0, bofs, 0});
            items = 0;
        }
        Camera c{};
        for (int a = 0; a < 3; ++a) {
            c.eye[a] = vi.camera.eye[a];
            c.right[a] = vi.camera.right[a];
            c.up[a] = vi.camera.up[a];
            c.forward[a] = vi.camera.forward[a];
        }
        c.th = vi.camera.tan_half_fovy;
        const Disp d{vi.disp.lambda_eye, vi.disp.lambda_dir, vi.disp.z0, vi.disp.mode};
        hv[(size_t)j] = view_of(c, vi.W, vi.H, vi.K, d, vi.out_images, vi.out_ids, lp.tile_log2w);
        hb[bofs++] = (uint32_t)items;
        items += view_items(hv[(size_t)j]);
        if (items >= (1ull << 32) - (1ull << 24)) {   // headroom for fetches past the end
            set_error("a batch of mode %d holds %llu work items (limit 2^32 - 2^24)", vi.disp.mode,
                      (unsigned long long)items);
            return RCP_ERR_INVALID_ARGUMENT;
        }
        groups.back().count++;
    }
    hb[bofs++] = (uint32_t)items;
    groups.back().items = (uint32_t)items;

    size_t spill_need = 0;
    std::vector<ChainGrid> grids(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        rcp_status st = chain_grid(lp, false, groups[g].count, groups[g].mode, grids[g]);
        if (st != RCP_OK) return st;
        spill_need = std::max(spill_need, spill_depth_of(s, grids[g].k) * grids[g].threads());
    }

    // buffers grow in stream order (a server's slots are sized at creation
    // and never grow here)
    if ((size_t)n_views > ws.view_cap || !ws.views) {
        if (ws.staging) {
            set_error("a batch of %d views exceeds the %zu views its workspace was sized for", n_views, ws.view_cap);
            return RCP_ERR_INTERNAL;
        }
        stream_free(ws.views, stream);
        ws.views = nullptr;
        ws.view_cap = 0;
        rcp_status st = stream_alloc(&ws.views, view_table_bytes((size_t)n_views), stream);
        if (st != RCP_OK) return st;
        ws.view_cap = (size_t)n_views;
    }
    if (ws.staging && spill_need > ws.spill_cap) {
        set_error("the batch needs more stack overflow area than its workspace was sized for (launch parameters "
                  "changed since)");
        return RCP_ERR_INTERNAL;
    }
    size_t fetch_cap = ws.fetch ? kFetchWords * 3 : 0;
    rcp_status st = grow(&ws.fetch, fetch_cap, kFetchWords * 3, sizeof(uint32_t), stream);
    if (st == RCP_OK) st = grow(&ws.spill, ws.spill_cap, spill_need, sizeof(int32_t), stream);
    if (st != RCP_OK) return st;
    ViewDev* d_views = (ViewDev*)ws.views;
    const size_t begin_ofs = (sizeof(ViewDev) * (size_t)n_views + 255) & ~(size_t)255;
    uint32_t* d_begin = (uint32_t*)((char*)ws.views + begin_ofs);
    // One view (a lone request of a server, say) is a single render: its
    // tiles go out in cost order, as rcp_render's do, with the launch
    // parameters of that order.  A server slot, whose buffers never grow,
    // keeps the screen order for a view beyond its order buffer.
    const uint32_t n_tiles1 = n_views == 1 ? groups[0].items >> 6 : 0u;
    bool ordered1 = n_views == 1 && s->tuning.tile_order && s->occ.bits && n_tiles1 > 0;
    if (ordered1 && 2 * (size_t)n_tiles1 > ws.order_cap) {
        if (ws.staging) ordered1 = false;
        else if ((st = grow(&ws.order, ws.order_cap, 2 * (size_t)n_tiles1, sizeof(uint32_t), stream)) != RCP_OK)
            return st;
    }
    const Launch lpr = ordered1 ? launch_params(s, true) : lp;
    if (ordered1) {
        uint32_t* score = ws.order + n_tiles1;
        hipLaunchKernelGGL(k_tile_scores, dim3((8 * n_tiles1 + kScoreBlock - 1) / kScoreBlock), dim3(kScoreBlock),
                           sizeof(uint32_t) * s->occ.words, stream, hv[0], s->occ, n_tiles1, score);
        hipLaunchKernelGGL(k_band_order, dim3(kFetchParts + 1), dim3(1024), 0, stream, (const uint32_t*)score,
                           groups[0].items, ws.order, hv[0], d_views, d_begin, ws.fetch,
                           (unsigned long long*)nullptr);
    } else if (n_views == 1) {
        // the setup kernel writes the view's table from the by-value
        // argument, with no host copy
        hipLaunchKernelGGL(k_setup_single, dim3(1), dim3(256), 0, stream, hv[0], d_views, d_begin,
                           groups[0].items, ws.fetch, (unsigned long long*)nullptr);
    } else if (ws.staging) {
        // a server slot: copy from its pinned table (the slot's previous
        // launch, the last reader, has finished)
        std::memcpy(ws.staging, hv.data(), sizeof(ViewDev) * (size_t)n_views);
        std::memcpy((char*)ws.staging + begin_ofs, hb.data(), sizeof(uint32_t) * bofs);
        RCP_HIP(hipMemcpyAsync(d_views, ws.staging, begin_ofs + sizeof(uint32_t) * bofs, hipMemcpyHostToDevice,
                               stream));
        hipLaunchKernelGGL(k_clear_chain, dim3(1), dim3(64), 0, stream, ws.fetch, (int)groups.size(),
                           (unsigned long long*)nullptr);
    } else {
        // pageable sources: the copies have read them when the calls return
        RCP_HIP(hipMemcpyAsync(d_views, hv.data(), sizeof(ViewDev) * (size_t)n_views, hipMemcpyHostToDevice,
                               stream));
        RCP_HIP(hipMemcpyAsync(d_begin, hb.data(), sizeof(uint32_t) * bofs, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(k_clear_chain, dim3(1), dim3(64), 0, stream, ws.fetch, (int)groups.size(),
                           (unsigned long long*)nullptr);
    }
    RCP_CHECK_LAUNCH();
    for (size_t g = 0; g < groups.size(); ++g) {
        ChainArgs a{};
        a.sc = s->dev;
        a.sc.top_count = lp.top_count;
        a.views = d_views + groups[g].first;
        a.begin = d_begin + groups[g].bofs;
        a.n_views = groups[g].count;
        a.n_items = groups[g].items;
        a.fetch = ws.fetch + kFetchWords * g;
        a.refill_min = lpr.refill_min;
        a.exit_lanes = (uint32_t)lpr.exit_lanes;
        a.spill = ws.spill;
        a.spill_stride = grids[g].threads();
        a.order = ordered1 ? ws.order : nullptr;
        rcp_status st2 = launch_chain(grids[g], stream, a);
        if (st2 != RCP_OK) return st2;
    }
    return RCP_OK;
}

void free_batch_workspace(BatchWorkspace& ws, hipStream_t stream) {
    stream_free(ws.order, stream);
    stream_free(ws.views, stream);
    stream_free(ws.fetch, stream);
    stream_free(ws.spill, stream);
    if (ws.staging) (void)hipHostFree(ws.staging);
    ws = BatchWorkspace{};
}

}  // namespace rcp
