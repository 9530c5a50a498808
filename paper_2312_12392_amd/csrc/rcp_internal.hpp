// Internal declarations of the recursive camera-painting library (gfx950).
//
// Data in HBM for a built scene (all arrays in the BVH's leaf order):
//   nodes  float4[n_nodes][8]   4-wide BVH node, 128 B: lo.x, hi.x, lo.y, hi.y,
//                               lo.z, hi.z of children 0..3, their links, zero
//   tris   float4[3][n_tris][3] three copies, copy c with each vertex rotated to
//                               (x[c+1], x[c+2], x[c]) (indices mod 3): v0 +
//                               original index bits in w, v1, v2
//   shade  float4[n_tris][2]    shaded RGB seen from the front / back side
//   normal float4[n_tris]       unit geometric normal (read by the normal mapping)
// Nodes are in level order from the root; the inner children of a node sit in
// consecutive slots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "rcp.h"

// The path's results must match a plain FP32 evaluation bit for bit: no
// contraction of a*b+c into fused multiply-adds anywhere in the library.
#pragma clang fp contract(off)

namespace rcp {

// ---- link encoding of BVH children ---------------------------------------
constexpr size_t kNodeBytes = 128;           // one 4-wide BVH node
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr int kMaxLeaf = 8;                // 3 bits of count
constexpr uint32_t kMaxTris = 1u << 28;    // 28 bits of first triangle
// Unused child slot of a 4-wide node: NaN planes, which fail every box test,
// and a link to the one-triangle leaf of triangle 0, so that even a slot
// that were entered could only repeat a test (never change the closest hit).

__host__ __device__ inline uint32_t leaf_link(uint32_t first, uint32_t count) {
    return kLeafBit | (first << 3) | (count - 1u);
}

// ---- errors ----------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();
rcp_status hip_status(hipError_t e, const char* what, const char* file, int line);

// Every device allocation of the library goes through dev_alloc or
// stream_alloc, so that the test hook RCP_DEBUG_FAIL_ALLOC_AFTER can make
// them fail.  dev_alloc is a plain hipMalloc.
rcp_status dev_alloc(void** p, size_t bytes);
// True when the allocation hook says the next device allocation fails.
bool alloc_hook_fails();
// Per-ray traversal step budget of scenes built from now on (0: the bound
// that only a malformed tree can reach).
uint32_t debug_step_budget();
// Canary checks of the per-pass engine's lists: 0 off, 1 on, 2 on with each
// list taken as one entry shorter (a test of the check itself).
int debug_list_canary();
// Values of the scene's device error flag.
constexpr uint32_t kErrStepBudget = 1u;   // a ray ran out of its step budget
constexpr uint32_t kErrListCanary = 2u;   // a compaction list failed its canary check
constexpr uint32_t kErrLdsLayout = 3u;    // the chain kernel's LDS did not start at address 0

// Scratch device memory ordered on a stream: allocated for the work enqueued
// after the call, released once the stream's earlier work is done, with no
// device-wide synchronisation (hipMallocAsync / hipFreeAsync; plain
// hipMalloc / hipFree on a device without memory pools).  Free on the same
// device and stream.
rcp_status stream_alloc(void** p, size_t bytes, hipStream_t stream);
void stream_free(void* p, hipStream_t stream);

#define RCP_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) return ::rcp::hip_status(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define RCP_TRY_STATUS(expr)                                                   \
    do {                                                                       \
        rcp_status st_ = (expr);                                               \
        if (st_ != RCP_OK) return st_;                                         \
    } while (0)

#define RCP_CHECK_LAUNCH()                                                     \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) return ::rcp::hip_status(e_, "kernel launch", __FILE__, __LINE__); \
    } while (0)

// ---- argument checks of the entry points (RCP_ERR_INVALID_ARGUMENT with a
// message; check_camera also converts) --------------------------------------
struct Camera;
rcp_status check_camera(const rcp_camera* c, Camera& out);
rcp_status check_disp(const rcp_displacement* d);
rcp_status check_size(int W, int H);
rcp_status check_scene(const rcp_scene* s);

// ---- device view of a scene -------------------------------------------------
struct DevScene {
    const float4* nodes;
    const float4* tris;
    const float4* shade;
    const float4* normals;
    uint32_t n_nodes;
    uint32_t n_tris;
    uint32_t max_depth;
    uint32_t stack_bound;   // most entries a traversal stack can hold
    uint32_t top_count;     // nodes of the first kTopLevels levels, at most kMaxStagedNodes (staged in LDS)
    float radius;      // largest |coordinate| of any vertex
    float bg[3];
    uint32_t step_budget;   // traversal steps per ray (only a malformed tree reaches it)
    uint32_t* err_flag;     // host-mapped; one of the kErr values once raised
};

struct Camera {
    float eye[3], right[3], up[3], forward[3];
    float th;
};

// Occupancy of the scene's bounding box on a coarse grid (a cell is set when
// a triangle's centroid lies in it), kept for ordering the work of a render:
// the occupied cells a pixel's undisplaced ray crosses estimate how long its
// chain will take.  kOccCells cells along the box's longest axis, about
// cubic cells, and at least kOccCells / 4 along the others (a single cell
// along an axis of zero extent).
constexpr int kOccCells = 48;
struct OccGrid {
    uint32_t* bits = nullptr;   // device, one bit per cell, x fastest, then y, then z
    int n[3] = {0, 0, 0};
    float lo[3] = {0.0f, 0.0f, 0.0f};
    float cell[3] = {1.0f, 1.0f, 1.0f};
    uint32_t words = 0;
};

// Per-render workspace.  The scene owns one, grown on demand with
// stream-ordered allocations on the stream of the call that needs more room;
// a captured graph owns its own, sized at capture and never grown, so that
// later calls on the scene cannot move the buffers a graph holds.  An
// external workspace (the preallocated scratch array of the allocation-free
// entry point) is never grown or freed: a call that needs more is rejected.
struct Workspace {
    float4* state[2] = {nullptr, nullptr};    // compact {pix, rgb} lists
    float4* aux[2] = {nullptr, nullptr};      // their {view depth, normal} (depth and normal modes)
    uint32_t* order = nullptr;                 // chain engine: tile scores, then the tile order
    size_t order_cap = 0;                      // uint32 entries
    size_t aux_cap = 0;
    size_t state_cap = 0;                      // entries per list
    uint32_t* counters = nullptr;              // kCounterWords
    int32_t* spill = nullptr;                  // traversal stack overflow
    size_t spill_cap = 0;                      // int32 entries
    unsigned long long* stats = nullptr;       // [kMaxPasses][kStatCols]
    void* view = nullptr;                      // chain engine: one-entry view table (kViewBytes)
    bool fixed = false;                        // never grown: a call that needs more is rejected
    bool external = false;                     // fixed, and the memory is not the workspace's to free
};

// Release a workspace's buffers on `stream` (stream-ordered).
void free_workspace(Workspace& w, hipStream_t stream);
// Room for `entries` uint32 of tile scores and order in a growable workspace
// (fixed and external workspaces are left as they are).
rcp_status ensure_order(Workspace& w, size_t entries, hipStream_t stream);

constexpr size_t kViewBytes = 512;

constexpr int kMaxPasses = 64;
// Counters per pass of the instrumented kernels: rays traced, inner nodes
// visited, triangles tested, rays continued to the next pass, inner nodes
// read from LDS, stack entries spilled to global memory.
constexpr int kStatCols = 6;
// Defaults of the launch parameters, measured on the 1080p K=6 terrain frame.
// Launches in screen order (batches, the per-pass engine, the allocation-free
// render): refill at 56 idle lanes, early exit at 16.  Single renders with the
// tiles in cost order: a wave refills only once all its lanes are idle (it
// then takes one whole tile) and exits at 32 lanes -- 3.0% faster there, but
// 5% slower on a batch in screen order.
constexpr int kDefaultExitLanes = 16;
constexpr int kDefaultExitLanesOrdered = 32;
constexpr int kDefaultRefillOrdered = 64;
// Levels of the 4-wide BVH the chain engine reads from LDS: LDS reads bypass
// the vector-memory address unit, the busiest unit of the traversal.
// Measured: 2 levels no gain, 3 levels 2% faster, 4 levels 1% more as long as
// the workgroup's LDS still allows 6 per CU.  Staged nodes keep their
// 128-byte layout, so at most kMaxStagedNodes of the 85 nodes of 4 levels
// (10 KB next to the 16 KB stack area).
constexpr int kTopLevels = 4;
constexpr uint32_t kMaxStagedNodes = 80;
// The node array is addressed with 32-bit byte offsets.
constexpr uint32_t kMaxNodes = 1u << 25;
constexpr int kDefaultRefill = 56;
// Most triangles per leaf when the caller gives no build options: 3 measured
// 1.6-2.6% faster than 4 on the terrain frame, a 64-view batch and the 16M
// walk-through (2 and 6 slower).
constexpr int kDefaultMaxLeaf = 3;

struct Disp {
    float le, ld, z0;
    int mode;
};

// Buffers of one in-flight batch (view table, work counter, stack overflow).
// Grown with stream-ordered allocations; a server sizes its slots' sets once,
// at creation, for the largest batch.
struct BatchWorkspace {
    void* views = nullptr;
    size_t view_cap = 0;
    uint32_t* fetch = nullptr;
    int32_t* spill = nullptr;
    size_t spill_cap = 0;
    void* staging = nullptr;      // pinned host copy of the view table (servers only), view_cap views
    uint32_t* order = nullptr;    // a one-view batch's tile order and scores (chain engine, cost order)
    size_t order_cap = 0;         // uint32 entries
};

// Tiles of the largest one-view batch a server slot hands out in cost order
// (2^18 tiles: 16.8M pixels, a 4K view with room to spare); larger views keep
// the screen order, since a slot's buffers never grow.
constexpr size_t kServerOrderTiles = size_t(1) << 18;

struct Tuning {
    int refill_min = -1;          // < 0: the library default for the launch
    int exit_lanes = -1;          // likewise
    int blocks_per_cu = 0;        // 0: occupancy limit
    int tile_log2w = 3;           // 8x8 tiles
    int engine = RCP_ENGINE_CHAIN;
    int top_levels = kTopLevels;  // levels of the 4-wide tree the chain engine reads from LDS (0..kTopLevels)
    int stack = 16;               // LDS stack entries per lane of the chain engine's colour kernel (8 or 16)
    int block = 256;              // its workgroup size (256 or 512)
    int tile_order = 1;           // single renders of the chain engine: 1 hands out each band's tiles
                                  // by decreasing estimated cost, 0 in screen order
};

}  // namespace rcp

struct rcp_scene {
    int device = 0;
    rcp::DevScene dev{};
    float4* nodes = nullptr;
    float4* tris = nullptr;
    float4* shade = nullptr;
    float4* normals = nullptr;
    rcp_scene_stats stats{};
    uint32_t top_nodes[rcp::kTopLevels + 1] = {};   // nodes in the tree's first L levels, L = 0..kTopLevels
    uint32_t* err_host = nullptr;   // pinned, device-mapped error flag (DevScene::err_flag)
    rcp::OccGrid occ;
    rcp::Workspace ws;
    rcp::BatchWorkspace bws;
    rcp::Tuning tuning;
};

// A K-pass render captured as a HIP graph.
struct rcp_graph {
    rcp_scene* scene = nullptr;
    rcp::Camera cam{};
    rcp::Disp disp{};
    int W = 0, H = 0, K = 0;
    float* out = nullptr;
    int32_t* ids = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rcp::Workspace ws;           // the graph's own buffers (sized at capture)
};

namespace rcp {

// Stable LSD radix sort of (u64 key, u32 value) pairs over bits [0, end_bit).
// tmp_keys / tmp_vals: n entries each.  Result ends in keys / vals.
// In-place exclusive prefix sum of n uint32 values on the device; scratch
// holds scan_scratch_words(n) words.
size_t scan_scratch_words(long n);
rcp_status scan_exclusive_u32(uint32_t* data, long n, uint32_t* scratch, hipStream_t stream);
rcp_status radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* tmp_keys, uint32_t* tmp_vals,
                            int n, int end_bit, hipStream_t stream);

// Idle lanes that make a wave of a persistent kernel fetch new work.

rcp_status build_scene(const rcp_scene_desc* desc, const rcp_build_options* opts, hipStream_t stream,
                       rcp_scene** out);

rcp_status render(rcp_scene* s, Workspace& ws, const Camera& cam, int W, int H, int K, const Disp& disp,
                  float* out_images, int32_t* out_ids, const float* prev_rgb, const float* prev_aux, float* out_aux,
                  unsigned long long* host_counts, hipStream_t stream);

rcp_status generate_rays(const Camera& cam, int W, int H, const Disp& disp, const float* prev_rgb,
                         const float* prev_aux, float* org, float* dir, hipStream_t stream);

rcp_status gather_passes(const float* in, int W, int H, int n, float smudge, int edge, int centred, float* out,
                         hipStream_t stream);

rcp_status render_batch(rcp_scene* s, const rcp_view* views, int n_views, BatchWorkspace& ws, hipStream_t stream);
// Size a batch workspace for up to n_views views in every mode (no
// allocation in render_batch afterwards); with_staging adds the pinned view
// table the server copies from.
rcp_status prepare_batch_workspace(rcp_scene* s, BatchWorkspace& ws, int n_views, bool with_staging,
                                   hipStream_t stream);
// The chain engine for a whole render from the seed: one launch, no pass barrier.
rcp_status prepare_chain(rcp_scene* s, Workspace& ws, int W, int H, int mode, hipStream_t stream);
rcp_status render_chain(rcp_scene* s, Workspace& ws, const Camera& cam, int W, int H, int K, const Disp& disp,
                        float* out_images, int32_t* out_ids, unsigned long long* host_counts, hipStream_t stream);
// The chain engine on a caller-sized workspace that is never grown: the
// grid is limited to the blocks whose stack overflow fits spill_cap.
rcp_status render_chain_fixed(rcp_scene* s, Workspace& ws, const Camera& cam, int W, int H, int K,
                              const Disp& disp, float* out_images, int32_t* out_ids, hipStream_t stream);
void free_batch_workspace(BatchWorkspace& ws, hipStream_t stream);
// Report (and clear) a ray that ran out of its step budget since the last
// check, as RCP_ERR_INTERNAL.  Reads the host-mapped flag: the work that may
// have set it must be complete.
rcp_status take_device_error(rcp_scene* s);

// The launch parameters a render of this scene uses (tuning or defaults).
struct Launch {
    uint32_t top_count;      // top BVH nodes staged in LDS by the chain engine
    int refill_min;
    int exit_lanes;
    int blocks_per_cu;
    int tile_log2w;
    int stack;               // chain engine, colour mode: LDS stack entries per lane
    int block;               // and workgroup size
};
// ordered: a single render with its tiles in cost order (the defaults of
// refill_min and exit_lanes depend on it).
Launch launch_params(const rcp_scene* s, bool ordered = false);
// Whether single renders of the chain engine on this scene use the cost order.
inline bool chain_ordered(const rcp_scene* s) { return s->tuning.tile_order != 0 && s->occ.bits != nullptr; }

// Make sure a render workspace fits a K-pass W x H render in `mode` (no
// allocation happens in render afterwards for that size).
rcp_status prepare_render(rcp_scene* s, Workspace& ws, int W, int H, int K, int mode, hipStream_t stream);
// Grow a workspace: per-pass state and aux lists of n_state / n_aux entries
// (0 = none), the counters, and spill_entries stack overflow words.  Old
// buffers are released and new ones allocated in stream order on `stream`;
// calls on one scene are ordered (one stream, or synchronised between
// streams), so no earlier work can still use a released buffer.
rcp_status ensure_workspace(rcp_scene* s, Workspace& ws, size_t n_state, size_t n_aux, size_t spill_entries,
                            hipStream_t stream);
// Words of a workspace's counter array.
size_t counter_words();

rcp_status graph_capture(rcp_graph* g);
void graph_free(rcp_graph* g);
rcp_status autotune(rcp_scene* s, const Camera& cam, int W, int H, int K, const Disp& d, float* out, int32_t* ids,
                    int repeats, Tuning& best, float& best_ms, hipStream_t stream);
rcp_status autotune_batch(rcp_scene* s, const rcp_view* views, int n_views, int repeats, Tuning& best,
                          float& best_ms, hipStream_t stream);

size_t request_bytes(const rcp_request& r);
rcp_status server_create(rcp_scene* scene, size_t pool_bytes, int max_inflight, int queue_capacity, rcp_server** out);
void server_destroy(rcp_server* s);
rcp_status server_submit(rcp_server* s, const rcp_request& r, uint64_t& ticket);
rcp_status server_poll(rcp_server* s, uint64_t ticket, int32_t& state, double times[3]);
rcp_status server_result(rcp_server* s, uint64_t ticket, float** images, int32_t** ids);
rcp_status server_result_copy(rcp_server* s, uint64_t ticket, float* images, int32_t* ids, hipStream_t stream);
rcp_status server_release(rcp_server* s, uint64_t ticket);
rcp_status server_stats(rcp_server* s, uint64_t out[4]);

rcp_status trace_rays(rcp_scene* s, const float* org, const float* dir, int n, float* out_t,
                      int32_t* out_id, int32_t* out_front, hipStream_t stream);

}  // namespace rcp
