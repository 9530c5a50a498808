/*
 * rcp_oracle.h -- CPU oracle for recursive camera painting.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * implementation of the K-pass render, written from the paper (Section 2's
 * recursion and ray definition, Section 3's colour mapping).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code with the HIP library: no headers, no helpers, no tables.
 *
 * Precision: FP32, IEEE round-to-nearest-even, no contraction (build with
 * -ffp-contract=off), correctly rounded division and square root.  FP64 is
 * used only in the watertight test's re-evaluation of zero edge functions.
 * The configurations fix FP32, and the hit ID is an argmin decided by FP32
 * arithmetic, so the oracle takes that decision in FP32 too.
 */
#ifndef RCP_ORACLE_H
#define RCP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    const float* verts;      /* [n_verts][3] */
    uint32_t n_verts;
    const uint32_t* idx;     /* [n_tris][3] */
    uint32_t n_tris;
    const float* rgb;        /* [n_tris][3] albedo */
    float light[3];          /* unit vector toward the light */
    float k_a, k_d;
    float background[3];
} orc_scene_desc;

typedef struct {
    float eye[3], right[3], up[3], forward[3];
    float tan_half_fovy;
} orc_camera;

typedef struct orc_scene orc_scene;

/* Copy the scene; build the oracle's own binned-SAH BVH when use_bvh != 0
 * (otherwise every query is brute force).  Returns NULL on bad input. */
orc_scene* orc_scene_create(const orc_scene_desc* desc, int use_bvh);
void orc_scene_destroy(orc_scene* s);
/* BVH statistics: nodes, leaves, max depth (0s for a brute-force scene). */
void orc_scene_stats(const orc_scene* s, int32_t out[3]);

/* Displacement mappings: Section 3 colour, Section 4 depth, Section 5 normal. */
#define ORC_MODE_COLOR 0
#define ORC_MODE_DEPTH 1
#define ORC_MODE_NORMAL 2

/* Ray of pixel (x, y) given the previous colour prev[3] and the previous
 * hit's data prev_aux[4] = (view depth, unit normal) or NULL for the seed
 * (Eq. N, Eq. D; Sections 3, 4, 5). */
void orc_ray(const orc_camera* cam, int W, int H, int x, int y, const float prev[3],
             const float prev_aux[4], int mode, float z0,
             float lambda_eye, float lambda_dir, float o[3], float d[3]);

/* Watertight ray/triangle test.  Returns 1 on a hit with t > 0, writing
 * t and front (1 when the geometric normal faces the ray). */
int orc_intersect(const float o[3], const float d[3], const float v0[3],
                  const float v1[3], const float v2[3], float* t, int* front);

/* Closest hit: nearest t, then lowest triangle ID.  brute != 0 forces the
 * brute-force scan.  Returns 1 on a hit. */
int orc_closest_hit(const orc_scene* s, const float o[3], const float d[3], int brute,
                    float* t, int32_t* id, int* front);

/* orc_closest_hit for n rays o[n][3], d[n][3], threaded: t[n] (+inf on a
 * miss), id[n] (-1 on a miss), front[n].  nthreads <= 0 uses every core. */
int orc_closest_hits(const orc_scene* s, const float* o, const float* d, int n, int brute,
                     float* t, int32_t* id, int32_t* front, int nthreads);

/* Shaded colour of triangle id seen from its front (1) or back (0) side. */
void orc_shade(const orc_scene* s, int32_t id, int front, float rgb[3]);
/* Unit geometric normal cross(v1-v0, v2-v0) / |...| of triangle id. */
void orc_normal(const orc_scene* s, int32_t id, float n[3]);

/* One pass: prev [H][W][3] and prev_aux [H][W][4] (NULL = the seed) ->
 * out [H][W][3], ids [H][W], out_aux [H][W][4] (view depth of the hit along
 * the camera's forward axis, unit normal; +inf and 0 after a miss).  ids and
 * out_aux may be NULL.  nthreads <= 0 uses every online core. */
int orc_render_pass(const orc_scene* s, const orc_camera* cam, int W, int H, int mode, float z0,
                    float lambda_eye, float lambda_dir, const float* prev, const float* prev_aux,
                    float* out, int32_t* ids, float* out_aux, int nthreads);

/* K passes from the grey seed: out [K][H][W][3], ids [K][H][W] or NULL. */
int orc_render(const orc_scene* s, const orc_camera* cam, int W, int H, int K, int mode, float z0,
               float lambda_eye, float lambda_dir, float* out, int32_t* ids, int nthreads);

/* Full K-pass chains of n selected pixels (index y*W + x): out [n][K][3],
 * ids [n][K] or NULL. */
int orc_render_pixels(const orc_scene* s, const orc_camera* cam, int W, int H, int K, int mode, float z0,
                      float lambda_eye, float lambda_dir, const int32_t* pix, int n,
                      float* out, int32_t* ids, int nthreads);

/* Screen-space variant (Section 6): with the eye fixed, re-rendering reduces
 * to fetching each pixel's new colour from a position displaced by its own
 * red and green, max_smudge pixels at most, with an edge rule for positions
 * outside the image (Section 6.1: clamp, wrap, mirror).  centred != 0 uses
 * (2R-1, 2G-1) as in Section 3, otherwise (R, G) as Section 6.1 describes.
 * One pass in -> out ([H][W][3]); n passes in -> out [n][H][W][3]. */
#define ORC_EDGE_CLAMP 0
#define ORC_EDGE_WRAP 1
#define ORC_EDGE_MIRROR 2
int orc_gather_pass(const float* in, int W, int H, float max_smudge, int edge, int centred, float* out);
int orc_gather(const float* in, int W, int H, int n, float max_smudge, int edge, int centred, float* out);

/* Number of threads orc_* uses for nthreads <= 0. */
int orc_default_threads(void);

#ifdef __cplusplus
}
#endif
#endif
