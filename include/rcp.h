/*
 * rcp.h -- C ABI of the recursive camera-painting renderer for MI355X (gfx950).
 *
 * Recursive camera painting (Akleman, Mullins, Morrison, Oh, "Recursive Camera
 * Painting: A Method for Real-Time Painterly Renderings of 3D Scenes") renders
 * K images I_1..I_K of one scene.  Every pixel (u,v) owns a camera: an eye
 * P_e(u,v) and an image-plane point P_p(u,v), with ray direction
 * N = (P_p - P_e) / |P_p - P_e| (Section 2).  Before pass n both points are
 * displaced from their original positions by vectors computed from the
 * previous image at the same pixel, I_n(u,v) = F(I_{n-1}(u,v), S)
 * (Section 2).  The colour mapping of Section 3 uses
 * V = lambda (2R-1, 2G-1, 2B-1) in the camera's local frame (R to the right,
 * G up, B along the view axis), starting from the grey seed I_0 = 0.5, so
 * I_1 is the ordinary ray-traced image.
 *
 * Conventions shared by every entry point:
 *   - Images are float32, row-major [H][W][3] RGB, row 0 at the top of the
 *     image.  K-image outputs are [K][H][W][3]; image 0 is I_1.
 *   - Hit-ID planes are int32 [H][W] (or [K][H][W]): the index of the hit
 *     triangle in the scene description, -1 where the ray missed.
 *   - "device" pointers are HIP device allocations (hipMalloc, or torch CUDA
 *     tensors on ROCm); "host" pointers are ordinary CPU memory.  Output
 *     buffers are owned by the caller.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Rendering
 *     calls are asynchronous: they enqueue work on the stream and return;
 *     results are valid once the stream has been synchronised.  Argument
 *     errors are reported before anything is enqueued.
 *   - Every call returns an rcp_status; no exception crosses the ABI.
 *     rcp_last_error() gives a message for the calling thread's last error.
 *   - Calls on one scene must be ordered: made on one stream, or with the
 *     earlier stream synchronised before another is used.  The scene's render
 *     workspace is shared by those calls; when a call needs more of it, the
 *     old buffers are released and new ones allocated in stream order on that
 *     call's stream (no device-wide synchronisation).
 *   - A ray that runs out of its traversal step budget (which only a
 *     malformed BVH can cause) ends as a miss and raises the scene's error
 *     flag; rcp_check, the synchronous calls and the server report it as
 *     RCP_ERR_INTERNAL.
 */
#ifndef RCP_H
#define RCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RCP_OK = 0,
    RCP_ERR_INVALID_ARGUMENT = 1,
    RCP_ERR_OUT_OF_MEMORY = 2,
    RCP_ERR_DEVICE = 3,
    RCP_ERR_NOT_READY = 4,
    RCP_ERR_QUEUE_FULL = 5,
    RCP_ERR_INTERNAL = 6
} rcp_status;

/* Opaque scene: triangles, BVH and shading table resident in HBM. */
typedef struct rcp_scene rcp_scene;

/* Scene S of Section 2.  All pointers are HOST pointers; the data is copied
 * during rcp_build_scene and may be freed afterwards.
 *   verts      [n_verts][3] float32 positions
 *   idx        [n_tris][3]  uint32 vertex indices (each < n_verts); the
 *              geometric normal is cross(v1 - v0, v2 - v0)
 *   tri_rgb    [n_tris][3]  float32 albedo per triangle
 *   light_dir  unit vector pointing toward the directional light
 *   k_a, k_d   ambient and diffuse weights of the Lambert shade
 *   background colour of rays that hit nothing
 * n_tris == 0 is allowed (every ray misses). */
typedef struct {
    const float* verts;
    uint32_t n_verts;
    const uint32_t* idx;
    uint32_t n_tris;
    const float* tri_rgb;
    float light_dir[3];
    float k_a, k_d;
    float background[3];
} rcp_scene_desc;

/* Base pinhole camera: eye P_e, orthonormal basis (right, up, forward) and
 * tan of half the vertical field of view.  The undisplaced image-plane point
 * of pixel (x, y) is P_p = eye + forward + s right + t up with
 * s = ((2x+1)/W - 1) tan_half_fovy W/H and t = (1 - (2y+1)/H) tan_half_fovy
 * (the image plane sits one unit in front of the eye). */
typedef struct {
    float eye[3];
    float right[3];
    float up[3];
    float forward[3];
    float tan_half_fovy;
} rcp_camera;

/* Displacement mapping.  Every pass displaces the base camera of each pixel
 * by a vector w computed from the previous pass at the same pixel:
 *   RCP_MODE_COLOR  (Section 3)  w = (2R-1) right + (2G-1) up + (2B-1) forward
 *   RCP_MODE_DEPTH  (Section 4)  w = |z - z0| (colour vector), z the view depth
 *                   of the previous hit along the camera's forward axis
 *                   (w = 0 after a miss)
 *   RCP_MODE_NORMAL (Section 5)  w = C x N, C the pixel's undisplaced view
 *                   direction, N the previous hit's unit geometric normal
 *                   (w = 0 after a miss)
 * and then
 *   V_e = lambda_eye w                  (eye displacement, Section 2)
 *   V_p = (lambda_eye + lambda_dir) w   (image-plane displacement)
 * so the displaced ray starts at eye + lambda_eye w with direction
 * normalize(P_p - P_e + lambda_dir w).  The paper's mappings keep the eye
 * fixed: (lambda_eye, lambda_dir) = (0, lambda).  The grey seed of pass 1 has
 * no hit, so pass 1 is the undisplaced render in every mode.
 * Valid: finite values, lambda_eye >= 0, 0 <= lambda_dir < 1; z0 is used by
 * RCP_MODE_DEPTH only. */
typedef struct {
    float lambda_eye;
    float lambda_dir;
    int32_t mode;
    float z0;
} rcp_displacement;

#define RCP_MODE_COLOR 0
#define RCP_MODE_DEPTH 1
#define RCP_MODE_NORMAL 2

/* Build options (NULL = defaults).
 *   max_leaf        most triangles per BVH leaf (1..8, default 3)
 *   c_trav, c_isect SAH costs of a node visit and a triangle test (defaults
 *                   1, 1), used when the 4-wide traversal tree is formed
 *                   from the binary tree (the SAH collapse also charges
 *                   2 * c_trav for entering a leaf)
 *   builder         how that binary tree is built from the Morton-sorted
 *                   triangles: RCP_BUILDER_PLOC (default; agglomerative
 *                   clustering of nearest neighbours, a lower SAH cost) or
 *                   RCP_BUILDER_LBVH (binary radix tree, faster to build).
 *   collapse        how the binary tree becomes the 4-wide traversal tree:
 *                   RCP_COLLAPSE_SAH (default; the wide tree of least SAH
 *                   cost over all ways to form leaves and 4-wide nodes from
 *                   the binary tree's subtrees, by dynamic programming) or
 *                   RCP_COLLAPSE_GREEDY (leaves formed in the binary tree,
 *                   then each wide node opens its children of largest area).
 * Builder and collapse change the speed of rendering only, never an image. */
#define RCP_BUILDER_PLOC 0
#define RCP_BUILDER_LBVH 1
#define RCP_COLLAPSE_SAH 0
#define RCP_COLLAPSE_GREEDY 1
typedef struct {
    int32_t max_leaf;
    float c_trav;
    float c_isect;
    int32_t builder;
    int32_t collapse;
} rcp_build_options;

/* Scene statistics filled by rcp_scene_info. */
typedef struct {
    uint32_t n_tris;
    uint32_t n_nodes;        /* 4-wide BVH nodes (node_bytes each) */
    uint32_t n_leaves;       /* leaf links in the tree */
    uint32_t max_depth;      /* levels of the tree including the leaves */
    uint32_t max_leaf;
    float sah_cost;          /* SAH cost of the 4-wide tree (c_trav per node
                                visit, 2 * c_trav per leaf entered, c_isect
                                per triangle test), relative to the root box */
    float build_ms;          /* device time of the build kernels */
    uint64_t device_bytes;   /* HBM held by the scene */
    uint32_t node_bytes;     /* bytes per packed BVH node (rcp_export_bvh) */
    uint32_t leaf_hist[8];   /* leaf links by triangle count: leaf_hist[c - 1]
                                links to leaves of c triangles (they sum to
                                n_leaves; the count times c sums to n_tris,
                                except for a scene of one leaf, whose root
                                links it twice) */
} rcp_scene_stats;

/* ---------------------------------------------------------------------- */
/* Scene                                                                   */
/* ---------------------------------------------------------------------- */

/* Copy the scene to the device and build its BVH (Morton codes, radix sort,
 * PLOC or radix binary tree, bottom-up refit with SAH leaf collapse, 4-wide
 * collapse, packing).  The call is synchronous: it returns once the scene is
 * ready.  desc pointers are host pointers (see rcp_scene_desc); opts may be
 * NULL.  Limits: n_tris <= 2^28 - 8, and at most 2^25 BVH nodes (4 GB of
 * nodes, about 10^8 triangles).
 * Errors: RCP_ERR_INVALID_ARGUMENT (NULL desc/out, idx >= n_verts, a
 * non-finite vertex, light or background value, invalid options, a scene
 * beyond the limits), RCP_ERR_OUT_OF_MEMORY, RCP_ERR_DEVICE.  On error *out
 * is set to NULL. */
rcp_status rcp_build_scene(const rcp_scene_desc* desc, const rcp_build_options* opts,
                           void* hip_stream, rcp_scene** out);
/* With the environment variable RCP_LOG=1, every successful build prints one
 * line of its statistics (rcp_scene_stats, with the leaf histogram) to
 * stderr. */

/* Release the scene's device memory (synchronises the device first).
 * NULL is ignored. */
void rcp_destroy_scene(rcp_scene* scene);

/* Fill *out with the scene's statistics (host pointer). */
rcp_status rcp_scene_info(const rcp_scene* scene, rcp_scene_stats* out);

/* ---------------------------------------------------------------------- */
/* Rendering                                                               */
/* ---------------------------------------------------------------------- */

/* K-pass recursive camera painting (Section 2 recursion, Section 3 colour
 * mapping): I_0 = 0.5 grey; for n = 1..K, every pixel's ray is displaced
 * from the base camera using I_{n-1} at the same pixel, traced to the
 * closest hit (nearest t, then lowest triangle index), and shaded.
 *   out_images  device, [K][H][W][3] float32; receives I_1..I_K
 *   out_ids     device, [K][H][W] int32 hit triangle or -1; may be NULL
 * Pixels whose colour did not change between two passes keep it (the next
 * ray would be identical) and drop out of the following passes.
 * Requires W, H >= 1, 1 <= K <= 64, W * H <= 2^27, a unit orthogonal
 * camera basis (|1 - |v|| <= 1e-5, |dot| <= 1e-5), tan_half_fovy > 0.
 * Asynchronous on hip_stream. */
rcp_status rcp_render(rcp_scene* scene, const rcp_camera* base_camera, int W, int H, int K,
                      const rcp_displacement* disp, float* out_images, int32_t* out_ids,
                      void* hip_stream);

/* rcp_render for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, validation and results as rcp_render (always the chain
 * engine); the call allocates nothing.  Its working memory (the launch's
 * view table, work counters, tile scores and order, and traversal stack
 * overflow) is a fixed area of rcp_render_noalloc_scratch_bytes() = 64 MiB
 * inside the library's device code, one per GPU, held until the process
 * ends.  Views of up to 2^16 tiles of 64 pixels (1440p and below) are
 * rendered in the cost order of the tile_order tuning, larger ones in screen
 * order (the order changes the speed only).  The launch uses as many
 * persistent workgroups as that area's overflow part holds for the scene's
 * tree (at most the occupancy limit, reached by trees of up to 15 inner
 * levels; the count changes the speed only); RCP_ERR_INVALID_ARGUMENT if it
 * cannot hold one workgroup per compute unit (a tree over 85 levels deep).
 * All calls on one GPU share the area
 * and leave their contents in it: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.
 * Asynchronous on hip_stream. */
rcp_status rcp_render_noalloc(rcp_scene* scene, const rcp_camera* base_camera, int W, int H, int K,
                              const rcp_displacement* disp, float* out_images, int32_t* out_ids,
                              void* hip_stream);
uint64_t rcp_render_noalloc_scratch_bytes(void);

/* One pass of F: out = F(prev) for a caller-supplied previous image.
 *   prev_rgb  device [H][W][3] float32, or NULL for the grey seed
 *   prev_aux  device [H][W][4] float32 (view depth, unit normal) of the
 *             previous pass's hits, as written to out_aux; NULL = the seed
 *             (no hit).  Read by RCP_MODE_DEPTH and RCP_MODE_NORMAL only.
 *   out_rgb   device [H][W][3] float32
 *   out_ids   device [H][W] int32 or NULL
 *   out_aux   device [H][W][4] float32 or NULL: view depth of the hit along
 *             the camera's forward axis and its unit normal (+inf and 0
 *             after a miss)
 * rcp_render's image k equals rcp_render_pass applied to image k-1 (and its
 * aux).  Asynchronous on hip_stream. */
rcp_status rcp_render_pass(rcp_scene* scene, const rcp_camera* base_camera, int W, int H,
                           const rcp_displacement* disp, const float* prev_rgb, const float* prev_aux,
                           float* out_rgb, int32_t* out_ids, float* out_aux, void* hip_stream);

/* rcp_render plus traversal counters (a separate instrumented kernel; not
 * for timing).  counts: HOST [K][6] uint64 per pass: rays traced, inner
 * nodes visited, triangles tested, rays continued to the next pass, inner
 * nodes read from the LDS copy of the tree's top levels (chain engine), and
 * traversal stack entries spilled from LDS to the global overflow area.
 * Synchronous; RCP_ERR_INTERNAL if a ray ran out of its step budget. */
rcp_status rcp_render_stats(rcp_scene* scene, const rcp_camera* base_camera, int W, int H, int K,
                            const rcp_displacement* disp, float* out_images, int32_t* out_ids,
                            uint64_t* counts, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Batched rendering, captured pass chains, tuning                         */
/* ---------------------------------------------------------------------- */

/* One view of a batch: its own base camera, image size, pass count and
 * displacement (any mode), and its own output buffers (device [K][H][W][3]
 * float32; ids [K][H][W] or NULL). */
typedef struct {
    rcp_camera camera;
    int32_t W, H, K;
    rcp_displacement disp;
    float* out_images;
    int32_t* out_ids;
} rcp_view;

/* Render n_views views of the scene in one persistent launch.  Each pixel's
 * K passes form an independent chain (Section 2: pass n at (u,v) needs only
 * pass n-1 at (u,v)), so a lane carries a pixel through all of its view's
 * passes and no pass barrier is needed; every view's images equal those of
 * rcp_render for that view alone.  Views are grouped by displacement mode,
 * one launch per mode present.  1 <= n_views <= 1024, each view valid as for
 * rcp_render, outputs must not overlap, and each mode's views together hold
 * fewer than 2^32 - 2^24 pixels (64-pixel tiles, rounded up per view).
 * Asynchronous on hip_stream. */
rcp_status rcp_render_batch(rcp_scene* scene, const rcp_view* views, int n_views, void* hip_stream);

/* A K-pass rcp_render call captured once as a HIP graph and replayed with a
 * single launch.  The graph holds the arguments given at creation (camera,
 * sizes, displacement, output buffers); rcp_graph_update replaces camera and
 * displacement in place.  The graph owns the buffers its kernels use
 * (allocated at creation, freed by rcp_graph_destroy), so other calls on the
 * scene between replays are safe; an update after launch parameters changed
 * so that more room is needed fails with RCP_ERR_INVALID_ARGUMENT (create a
 * new graph).  Graph, scene and outputs are used on one stream at a time.
 * Creation synchronises hip_stream. */
typedef struct rcp_graph rcp_graph;
rcp_status rcp_graph_create(rcp_scene* scene, const rcp_camera* base_camera, int W, int H, int K,
                            const rcp_displacement* disp, float* out_images, int32_t* out_ids,
                            void* hip_stream, rcp_graph** out);
rcp_status rcp_graph_update(rcp_graph* graph, const rcp_camera* base_camera, const rcp_displacement* disp);
rcp_status rcp_graph_launch(rcp_graph* graph, void* hip_stream);
void rcp_graph_destroy(rcp_graph* graph);

/* Launch parameters of the persistent kernels, per scene.  They change only
 * the speed, never an image.
 *   refill_min     lanes (1..64) needing a ray that make a wave run a setup
 *                  round (new pixels, and pixels moving to their next pass);
 *                  -1 (default): 64 for single renders with the tiles in cost
 *                  order (tile_order below), 56 for launches in screen order
 *   exit_lanes     a wave's descent to the leaves ends once no more than this
 *                  many lanes (0..64) are still looking for one and at least
 *                  as many hold one; -1 (default): 32 in cost order, 16 in
 *                  screen order
 *   blocks_per_cu  resident workgroups of 256 threads per compute unit (0 =
 *                  occupancy limit; a workgroup of 512 counts as two)
 *   tile_log2w     pixel tile of 64: width 2^tile_log2w (0..6)
 *   engine         how rcp_render (and rcp_render_stats, graphs, the
 *                  autotuner) run the K passes:
 *                  RCP_ENGINE_CHAIN  one persistent launch; each lane carries
 *                                    a pixel through all its passes (Section
 *                                    2: pass n at (u,v) needs only pass n-1
 *                                    at (u,v)); no per-pass state in HBM
 *                  RCP_ENGINE_PASSES one launch per pass; the pixels whose
 *                                    colour changed are compacted into a list
 *                                    in HBM for the next pass
 *                  rcp_render_pass always runs one pass launch.
 *   top_levels     levels of the 4-wide BVH the chain engine copies into
 *                  each workgroup's LDS and reads from there (0..4, default
 *                  4; at most 80 nodes)
 *   stack_entries  traversal stack entries per lane kept in LDS by the chain
 *                  engine's colour-mode kernel (8 or 16, default 16); deeper
 *                  entries go to a global overflow area
 *   block_size     that kernel's workgroup size (256 or 512, default 256)
 *   tile_order     single renders of the chain engine (rcp_render,
 *                  rcp_render_stats, graphs): 1 (default) hands out each
 *                  band's tiles by decreasing estimated cost -- the most
 *                  occupied cells of a coarse occupancy grid of the scene
 *                  that one of four undisplaced rays, through the centres of
 *                  the tile's quadrants, crosses, found by two small kernels
 *                  before the launch -- so that long
 *                  chains start first; 0 in screen order.  A batch of one
 *                  view follows it too (a server slot only up to 2^18
 *                  tiles, rcp_render_noalloc up to 2^16); batches of more
 *                  views always use the screen order.
 * The instrumented kernel and the depth and normal modes always use 16
 * stack entries and workgroups of 256. */
#define RCP_ENGINE_CHAIN 0
#define RCP_ENGINE_PASSES 1
typedef struct {
    int32_t refill_min;
    int32_t exit_lanes;
    int32_t blocks_per_cu;
    int32_t tile_log2w;
    int32_t engine;
    int32_t top_levels;
    int32_t stack_entries;
    int32_t block_size;
    int32_t tile_order;
} rcp_tuning;

rcp_status rcp_get_tuning(const rcp_scene* scene, rcp_tuning* out);
rcp_status rcp_set_tuning(rcp_scene* scene, const rcp_tuning* tuning);

/* Autotuner: times rcp_render of this workload (median of `repeats` runs,
 * HIP events on hip_stream) and descends over the rcp_tuning fields, one
 * field at a time with the others fixed, twice over: refill_min, exit_lanes,
 * blocks_per_cu, tile_log2w, engine, top_levels, stack_entries, block_size.
 * Sets the fastest on the scene and returns it with its time.  The outputs
 * receive a valid render.  Synchronous. */
rcp_status rcp_autotune(rcp_scene* scene, const rcp_camera* base_camera, int W, int H, int K,
                        const rcp_displacement* disp, float* out_images, int32_t* out_ids, int repeats,
                        rcp_tuning* best, float* best_ms, void* hip_stream);

/* The autotuner on a batch: times rcp_render_batch of these views over the
 * same candidates (except the engine: batches always run the chain engine),
 * sets the fastest on the scene and returns it.  The outputs receive a valid
 * render.  Synchronous. */
rcp_status rcp_autotune_batch(rcp_scene* scene, const rcp_view* views, int n_views, int repeats, rcp_tuning* best,
                              float* best_ms, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Continuous-batching server                                              */
/* ---------------------------------------------------------------------- */

/* A render request: base camera, image size, pass count, displacement (any
 * mode); with_ids != 0 also keeps the hit-ID planes. */
typedef struct {
    rcp_camera camera;
    int32_t W, H, K;
    rcp_displacement disp;
    int32_t with_ids;
} rcp_request;

#define RCP_REQ_QUEUED 0    /* waiting for pool space or a launch */
#define RCP_REQ_RUNNING 1   /* in a launched batch */
#define RCP_REQ_DONE 2      /* images ready in the pool */
#define RCP_REQ_FAILED 3

typedef struct rcp_server rcp_server;

/* Create a server on the scene's device.  pool_bytes of HBM are allocated
 * once and hold the output images of admitted requests (12 B per pixel and
 * pass, plus 4 B with ids, each rounded up to 256 B); requests are admitted
 * first-in first-out while they fit, and up to max_inflight (1..8) batched
 * launches run at once, each on its own stream.  A launch takes the
 * admitted requests of the oldest one's size class (more than 2^24 pixels
 * times passes is big), so small requests do not wait for large ones in the
 * same launch.  A request submitted while others run joins the next launch
 * of its class as soon as pool space and a launch slot are free; every
 * request's images equal those of rcp_render alone.  At most
 * queue_capacity requests wait for admission.  The scene must outlive the
 * server. */
rcp_status rcp_server_create(rcp_scene* scene, uint64_t pool_bytes, int max_inflight, int queue_capacity,
                             rcp_server** out);
/* Queue a request; *ticket identifies it.  RCP_ERR_QUEUE_FULL when
 * queue_capacity requests already wait; RCP_ERR_INVALID_ARGUMENT for an
 * invalid request or one larger than the whole pool.  Thread-safe. */
rcp_status rcp_submit(rcp_server* server, const rcp_request* request, uint64_t* ticket);
/* State of a request (RCP_REQ_*) and, if times != NULL, its submit, start
 * and completion times in seconds since the server was created (host clock;
 * completion is observed by the scheduler within ~50 us). */
rcp_status rcp_poll(rcp_server* server, uint64_t ticket, int32_t* state, double* times);
/* Device pointers of a finished request's images [K][H][W][3] and ids
 * [K][H][W] (NULL without ids), valid until rcp_release.
 * RCP_ERR_NOT_READY before RCP_REQ_DONE. */
rcp_status rcp_result(rcp_server* server, uint64_t ticket, float** images, int32_t** ids);
/* Copy a finished request's images / ids (either may be NULL) to caller
 * device buffers, asynchronously on hip_stream. */
rcp_status rcp_result_copy(rcp_server* server, uint64_t ticket, float* images, int32_t* ids, void* hip_stream);
/* Return a finished (or failed) request's pool space; the ticket ends. */
rcp_status rcp_release(rcp_server* server, uint64_t ticket);
/* out[0] launches so far, out[1] requests waiting, out[2] pool bytes in
 * use, out[3] live tickets. */
rcp_status rcp_server_stats(rcp_server* server, uint64_t out[4]);
/* Stop the scheduler (running launches finish; requests that cannot start
 * fail) and free the server.  NULL is ignored. */
void rcp_server_destroy(rcp_server* server);

/* Synchronise hip_stream, then report a ray of an earlier call on this scene
 * that ran out of its traversal step budget (RCP_ERR_INTERNAL; the flag is
 * cleared).  That ray's result was written as a miss. */
rcp_status rcp_check(rcp_scene* scene, void* hip_stream);

/* Screen-space variant (Section 6).  With the eye fixed, re-rendering a
 * pass reduces to fetching every pixel's new colour from the position its
 * own red and green point to: right by m_r and up (towards row 0) by m_g
 * times max_smudge pixels, with m = (2R-1, 2G-1) when centred != 0 (the
 * Section 3 mapping) or m = (R, G) as Section 6.1 describes.  The fetch takes
 * the pixel containing the displaced pixel centre; positions outside the
 * image follow edge_mode (Section 6.1): RCP_EDGE_CLAMP to the border,
 * RCP_EDGE_WRAP around, or RCP_EDGE_MIRROR about the border (the border
 * pixel repeated: -1 -> 0).
 *   in_rgb      device [H][W][3] float32, the image the first pass reads
 *   out_images  device [n_passes][H][W][3] float32; pass k reads image k-1
 *               (in_rgb for k = 0); must not overlap in_rgb
 * Requires W, H >= 1, W * H <= 2^27, 1 <= n_passes <= 64,
 * 0 <= max_smudge <= 1e6.  Asynchronous on hip_stream. */
#define RCP_EDGE_CLAMP 0
#define RCP_EDGE_WRAP 1
#define RCP_EDGE_MIRROR 2
rcp_status rcp_gather_passes(const float* in_rgb, int W, int H, int n_passes, float max_smudge,
                             int edge_mode, int centred, float* out_images, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Single steps of the path, for testing and measurement                   */
/* ---------------------------------------------------------------------- */

/* Displaced rays of every pixel (Section 2 ray and displacement; the
 * mapping of disp->mode) without tracing them.
 *   prev_rgb  device [H][W][3] or NULL (grey seed: the pinhole rays)
 *   prev_aux  device [H][W][4] or NULL (see rcp_render_pass)
 *   out_org, out_dir  device [H][W][3] float32
 * Asynchronous on hip_stream. */
rcp_status rcp_generate_rays(const rcp_camera* base_camera, int W, int H,
                             const rcp_displacement* disp, const float* prev_rgb, const float* prev_aux,
                             float* out_org, float* out_dir, void* hip_stream);

/* Closest hit of n arbitrary rays (org, dir device [n][3]; dir need not be
 * normalised but must be finite and non-zero).
 *   out_t      device [n] float32 (+inf on a miss)
 *   out_id     device [n] int32 triangle index or -1
 *   out_front  device [n] int32: 1 when cross(v1-v0, v2-v0) faces the ray
 * Asynchronous on hip_stream. */
rcp_status rcp_trace_rays(rcp_scene* scene, const float* org, const float* dir, int n,
                          float* out_t, int32_t* out_id, int32_t* out_front, void* hip_stream);

/* Copy the packed 4-wide BVH to HOST memory for inspection.
 *   nodes    [n_nodes][32] 32-bit words per node (node_bytes = 128 B),
 *            node 0 = root, nodes in level order:
 *            words 0-3 / 4-7     float lo.x / hi.x of children 0..3
 *            words 8-11 / 12-15  float lo.y / hi.y
 *            words 16-19 / 20-23 float lo.z / hi.z
 *            words 24-27         child links; 28-31 zero.
 *            A link with bit 31 clear is an inner node index; with bit 31
 *            set it is a leaf: bits 3..30 = first packed triangle,
 *            bits 0..2 = triangle count - 1.  An unused child slot has NaN
 *            planes (its link is the leaf of triangle 0, never entered).
 *            Boxes are slightly wider than their contents (the traversal's
 *            conservative pruning).
 *   tri_ids  [n_tris] original triangle index of each packed slot.
 * Either pointer may be NULL.  Synchronous. */
rcp_status rcp_export_bvh(const rcp_scene* scene, uint32_t* nodes, int32_t* tri_ids);

/* Stable LSD radix sort of n (uint64 key, uint32 value) pairs in device
 * memory, the sort used by the BVH build.  keys/vals are sorted in place.
 * Synchronous. */
rcp_status rcp_radix_sort_u64(uint64_t* keys, uint32_t* vals, int n, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Errors                                                                  */
/* ---------------------------------------------------------------------- */

const char* rcp_status_string(rcp_status s);
/* Message of the calling thread's last error ("" if none). */
const char* rcp_last_error(void);

/* Test hooks, process-wide, for exercising failure paths without faults:
 *   RCP_DEBUG_FAIL_ALLOC_AFTER  value >= 0: that many more device (and
 *                               pinned host) allocations of the library
 *                               succeed, every later one fails with
 *                               RCP_ERR_OUT_OF_MEMORY; value < 0: off.
 *   RCP_DEBUG_STEP_BUDGET       traversal step budget per ray of scenes built
 *                               afterwards (0: the default, which only a
 *                               malformed tree can exhaust).
 *   RCP_DEBUG_LIST_CANARY       1: the per-pass engine (Section 2's passes
 *                               one launch each) fills each pass's list of
 *                               continuing pixels, and their hit data, with an
 *                               all-ones canary before the pass and checks it
 *                               after: every entry below the list's count
 *                               written, with a pixel index below W * H and
 *                               colours in [0, 1]; every entry above it
 *                               untouched.  A violation is reported by
 *                               rcp_check and rcp_render_stats as
 *                               RCP_ERR_INTERNAL.  2: the same, with the check
 *                               told that each list is one entry shorter (a
 *                               test of the check itself: a non-empty list
 *                               then fails).  0: off (the default). */
#define RCP_DEBUG_FAIL_ALLOC_AFTER 1
#define RCP_DEBUG_STEP_BUDGET 2
#define RCP_DEBUG_LIST_CANARY 3
rcp_status rcp_debug_set(int what, int64_t value);

#ifdef __cplusplus
}
#endif
#endif /* RCP_H */
