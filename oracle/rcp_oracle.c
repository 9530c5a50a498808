/*
 * rcp_oracle.c -- CPU oracle for recursive camera painting.
 *
 * TEST INFRASTRUCTURE ONLY (see rcp_oracle.h).  Build:
 *   gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread
 *
 * What it computes (the paper has no numbered equations; names follow the
 * paper's notation):
 *   - Section 2, recursion: I_n(u,v) = F(I_{n-1}(u,v), S(n)).  The image at
 *     (u,v) depends on the previous image at the same (u,v) only.
 *   - Section 2, ray: each (u,v) owns an eye P_e and an image-plane point
 *     P_p; the ray direction is N = (P_p - P_e) / |P_p - P_e|.  Both points
 *     are displaced from their ORIGINAL positions: P'_e = P_e + V_e,
 *     P'_p = P_p + V_p (the printed first line repeats P'_p; it is read as
 *     the eye's line).
 *   - Section 3, colour mapping: V_p = lambda (2R-1, 2G-1, 2B-1) in the
 *     camera's local frame; R moves right, G moves up, B is along the view
 *     axis.  The seed I_0 is grey 0.5, so the first rendered image is the
 *     ordinary ray-traced one.
 *   - Intersection: the watertight ray/triangle test of Woop, Benthin and
 *     Wald, "Watertight Ray/Triangle Intersection", JCGT 2013, written from
 *     its description: shear the triangle into ray space, 2-D edge functions
 *     U, V, W with an FP64 re-evaluation when one is exactly zero, reject
 *     mixed signs and det == 0, t = T / det.
 *   - Sections 4 and 5, the depth and normal mappings: the colour vector
 *     scaled by |z - z0| (z the view depth of the previous hit), and
 *     lambda (C x N) (C the pixel's view direction, N the previous hit's
 *     world normal).
 *   - Shading (the paper leaves it open): two-sided Lambert with the flat
 *     geometric normal, one directional light, clamped to [0, 1] (Section 3
 *     speaks of low-dynamic-range channels).
 *
 * Every float expression below is evaluated left to right, each product is
 * rounded, and nothing is fused.
 */
#define _GNU_SOURCE
#include "rcp_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Scene                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    float lo[3], hi[3];
    int32_t first;   /* leaf: first entry of order[]; inner: left child */
    int32_t count;   /* leaf: > 0; inner: 0 (right child = left + 1) */
} obvh_node;

struct orc_scene {
    int32_t n_tris;
    float* tri;            /* [n][9]: v0, v1, v2 in the given vertex order */
    float* rgb;            /* [n][3] */
    float light[3];
    float k_a, k_d;
    float background[3];
    double radius;         /* largest |coordinate| of any vertex */
    obvh_node* nodes;      /* NULL => brute force */
    int32_t n_nodes, n_leaves, max_depth;
    int32_t* order;        /* triangle IDs in leaf order */
};

static int finite3(const float* v) {
    return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

/* ---- binned SAH BVH (16 bins, leaves of at most 4 triangles) ------------ */

typedef struct {
    float* blo;      /* [n][3] triangle box lo */
    float* bhi;      /* [n][3] triangle box hi */
    double* cen;     /* [n][3] box centre */
    obvh_node* nodes;
    int32_t n_nodes, cap_nodes, n_leaves, max_depth;
    int32_t* order;
} obuild;

static double box_area(const float lo[3], const float hi[3]) {
    double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

static void box_empty(float lo[3], float hi[3]) {
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
}

static void box_grow(float lo[3], float hi[3], const float* l2, const float* h2) {
    for (int c = 0; c < 3; ++c) {
        if (l2[c] < lo[c]) lo[c] = l2[c];
        if (h2[c] > hi[c]) hi[c] = h2[c];
    }
}

static int32_t new_node(obuild* b) {
    if (b->n_nodes == b->cap_nodes) {
        b->cap_nodes = b->cap_nodes ? 2 * b->cap_nodes : 1024;
        b->nodes = (obvh_node*)realloc(b->nodes, sizeof(obvh_node) * (size_t)b->cap_nodes);
    }
    return b->n_nodes++;
}

#define OBINS 16
#define OLEAF 4

static void build_node(obuild* b, int32_t ni, int32_t first, int32_t count, int depth) {
    obvh_node* nd = &b->nodes[ni];
    if (depth > b->max_depth) b->max_depth = depth;
    box_empty(nd->lo, nd->hi);
    double cl[3] = {INFINITY, INFINITY, INFINITY}, ch[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = first; i < first + count; ++i) {
        int32_t t = b->order[i];
        box_grow(nd->lo, nd->hi, &b->blo[3 * t], &b->bhi[3 * t]);
        for (int c = 0; c < 3; ++c) {
            double v = b->cen[3 * t + c];
            if (v < cl[c]) cl[c] = v;
            if (v > ch[c]) ch[c] = v;
        }
    }
    if (count <= OLEAF) {
        nd->first = first; nd->count = count; b->n_leaves++;
        return;
    }
    int axis = 0;
    double ext = ch[0] - cl[0];
    for (int c = 1; c < 3; ++c) if (ch[c] - cl[c] > ext) { ext = ch[c] - cl[c]; axis = c; }
    int32_t mid;
    if (!(ext > 0.0)) {
        mid = first + count / 2;             /* all centres coincide: split by index */
    } else {
        int32_t bn[OBINS] = {0};
        float blo[OBINS][3], bhi[OBINS][3];
        for (int k = 0; k < OBINS; ++k) box_empty(blo[k], bhi[k]);
        for (int32_t i = first; i < first + count; ++i) {
            int32_t t = b->order[i];
            int k = (int)(OBINS * ((b->cen[3 * t + axis] - cl[axis]) / ext));
            if (k >= OBINS) k = OBINS - 1;
            if (k < 0) k = 0;
            bn[k]++;
            box_grow(blo[k], bhi[k], &b->blo[3 * t], &b->bhi[3 * t]);
        }
        double best = INFINITY;
        int bestk = -1;
        for (int k = 1; k < OBINS; ++k) {
            float llo[3], lhi[3], rlo[3], rhi[3];
            int32_t nl = 0, nr = 0;
            box_empty(llo, lhi); box_empty(rlo, rhi);
            for (int j = 0; j < k; ++j) if (bn[j]) { box_grow(llo, lhi, blo[j], bhi[j]); nl += bn[j]; }
            for (int j = k; j < OBINS; ++j) if (bn[j]) { box_grow(rlo, rhi, blo[j], bhi[j]); nr += bn[j]; }
            if (nl == 0 || nr == 0) continue;
            double cost = box_area(llo, lhi) * nl + box_area(rlo, rhi) * nr;
            if (cost < best) { best = cost; bestk = k; }
        }
        if (bestk < 0) {
            mid = first + count / 2;
        } else {
            /* partition: bins < bestk to the left */
            int32_t i = first, j = first + count - 1;
            while (i <= j) {
                int32_t t = b->order[i];
                int k = (int)(OBINS * ((b->cen[3 * t + axis] - cl[axis]) / ext));
                if (k >= OBINS) k = OBINS - 1;
                if (k < 0) k = 0;
                if (k < bestk) { ++i; }
                else { int32_t tmp = b->order[j]; b->order[j] = b->order[i]; b->order[i] = tmp; --j; }
            }
            mid = i;
            if (mid == first || mid == first + count) mid = first + count / 2;
        }
    }
    int32_t l = new_node(b);
    int32_t r = new_node(b);
    (void)r;
    b->nodes[ni].first = l;
    b->nodes[ni].count = 0;
    build_node(b, l, first, mid - first, depth + 1);
    build_node(b, l + 1, mid, first + count - mid, depth + 1);
}

orc_scene* orc_scene_create(const orc_scene_desc* d, int use_bvh) {
    if (!d) return NULL;
    if (d->n_tris > 0 && (!d->verts || !d->idx || !d->rgb)) return NULL;
    orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
    s->n_tris = (int32_t)d->n_tris;
    s->tri = (float*)malloc(sizeof(float) * 9 * (size_t)(d->n_tris ? d->n_tris : 1));
    s->rgb = (float*)malloc(sizeof(float) * 3 * (size_t)(d->n_tris ? d->n_tris : 1));
    for (uint32_t i = 0; i < d->n_tris; ++i) {
        for (int k = 0; k < 3; ++k) {
            uint32_t v = d->idx[3 * i + k];
            if (v >= d->n_verts) { orc_scene_destroy(s); return NULL; }
            memcpy(&s->tri[9 * i + 3 * k], &d->verts[3 * v], 3 * sizeof(float));
            if (!finite3(&d->verts[3 * v])) { orc_scene_destroy(s); return NULL; }
        }
        memcpy(&s->rgb[3 * i], &d->rgb[3 * i], 3 * sizeof(float));
        for (int k = 0; k < 9; ++k)
            if (fabs((double)s->tri[9 * i + k]) > s->radius) s->radius = fabs((double)s->tri[9 * i + k]);
    }
    memcpy(s->light, d->light, sizeof s->light);
    s->k_a = d->k_a;
    s->k_d = d->k_d;
    memcpy(s->background, d->background, sizeof s->background);
    if (use_bvh && d->n_tris > 0) {
        obuild b;
        memset(&b, 0, sizeof b);
        size_t n = d->n_tris;
        b.blo = (float*)malloc(sizeof(float) * 3 * n);
        b.bhi = (float*)malloc(sizeof(float) * 3 * n);
        b.cen = (double*)malloc(sizeof(double) * 3 * n);
        b.order = (int32_t*)malloc(sizeof(int32_t) * n);
        for (size_t i = 0; i < n; ++i) {
            const float* t = &s->tri[9 * i];
            for (int c = 0; c < 3; ++c) {
                float lo = t[c], hi = t[c];
                for (int k = 1; k < 3; ++k) {
                    if (t[3 * k + c] < lo) lo = t[3 * k + c];
                    if (t[3 * k + c] > hi) hi = t[3 * k + c];
                }
                b.blo[3 * i + c] = lo;
                b.bhi[3 * i + c] = hi;
                b.cen[3 * i + c] = 0.5 * ((double)lo + (double)hi);
            }
            b.order[i] = (int32_t)i;
        }
        int32_t root = new_node(&b);
        build_node(&b, root, 0, (int32_t)n, 0);
        s->nodes = b.nodes;
        s->n_nodes = b.n_nodes;
        s->n_leaves = b.n_leaves;
        s->max_depth = b.max_depth;
        s->order = b.order;
        free(b.blo); free(b.bhi); free(b.cen);
        if (s->max_depth + 2 > 256) {      /* traversal stack bound: fall back to brute force */
            free(s->nodes); free(s->order);
            s->nodes = NULL; s->order = NULL;
            s->n_nodes = s->n_leaves = s->max_depth = 0;
        }
    }
    return s;
}

void orc_scene_destroy(orc_scene* s) {
    if (!s) return;
    free(s->tri); free(s->rgb); free(s->nodes); free(s->order);
    free(s);
}

void orc_scene_stats(const orc_scene* s, int32_t out[3]) {
    out[0] = s ? s->n_nodes : 0;
    out[1] = s ? s->n_leaves : 0;
    out[2] = s ? s->max_depth : 0;
}

/* ------------------------------------------------------------------------ */
/* Rays (Section 2, ray definition and displacements; Section 3 mapping)     */
/* ------------------------------------------------------------------------ */

void orc_ray(const orc_camera* cam, int W, int H, int x, int y, const float prev[3],
             const float prev_aux[4], int mode, float z0,
             float lambda_eye, float lambda_dir, float o[3], float d[3]) {
    /* Pixel centre in [-1, 1]^2, row 0 at the top; vertical field of view. */
    float fx = (float)(2 * x + 1) / (float)W - 1.0f;
    float fy = 1.0f - (float)(2 * y + 1) / (float)H;
    float aspect = (float)W / (float)H;
    float s = fx * (cam->tan_half_fovy * aspect);
    float t = fy * cam->tan_half_fovy;
    /* Undisplaced P_p - P_e: the image plane sits one unit along forward. */
    float q[3];
    for (int c = 0; c < 3; ++c) q[c] = (cam->forward[c] + s * cam->right[c]) + t * cam->up[c];
    float w[3], dp[3];
    if (mode == ORC_MODE_NORMAL) {
        /* Section 5: V = lambda (C x N), C the pixel's undisplaced view
         * direction, N the world normal of the previous hit (zero after a
         * miss and for the seed, so the first image is the pinhole one). */
        static const float no_normal[3] = {0.0f, 0.0f, 0.0f};
        const float* N = prev_aux ? prev_aux + 1 : no_normal;
        float ql = sqrtf((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
        float C[3];
        for (int c = 0; c < 3; ++c) C[c] = q[c] / ql;
        w[0] = C[1] * N[2] - C[2] * N[1];
        w[1] = C[2] * N[0] - C[0] * N[2];
        w[2] = C[0] * N[1] - C[1] * N[0];
    } else {
        /* Colour mapping: (2R-1, 2G-1, 2B-1) in the camera frame (right, up, forward). */
        float mr = 2.0f * prev[0] - 1.0f;
        float mg = 2.0f * prev[1] - 1.0f;
        float mb = 2.0f * prev[2] - 1.0f;
        for (int c = 0; c < 3; ++c) w[c] = (mr * cam->right[c] + mg * cam->up[c]) + mb * cam->forward[c];
        if (mode == ORC_MODE_DEPTH) {
            /* Section 4: the colour vector scaled by |z - z0|, z the view depth
             * of the previous hit; no displacement after a miss or for the seed. */
            float z = prev_aux ? prev_aux[0] : INFINITY;
            float kz = (z < INFINITY) ? fabsf(z - z0) : 0.0f;
            for (int c = 0; c < 3; ++c) w[c] = kz * w[c];
        }
    }
    /* P'_e = P_e + V_e and P'_p = P_p + V_p with V_e = lambda_eye w and
     * V_p = (lambda_eye + lambda_dir) w, so P'_p - P'_e = q + lambda_dir w. */
    for (int c = 0; c < 3; ++c) {
        o[c] = cam->eye[c] + lambda_eye * w[c];
        dp[c] = q[c] + lambda_dir * w[c];
    }
    float len = sqrtf((dp[0] * dp[0] + dp[1] * dp[1]) + dp[2] * dp[2]);
    for (int c = 0; c < 3; ++c) d[c] = dp[c] / len;
}

/* ------------------------------------------------------------------------ */
/* Watertight ray/triangle intersection                                      */
/* ------------------------------------------------------------------------ */

int orc_intersect(const float o[3], const float d[3], const float v0[3],
                  const float v1[3], const float v2[3], float* t_out, int* front_out) {
    /* Dominant axis of the direction (first of equal magnitudes). */
    int kz = 0;
    if (fabsf(d[1]) > fabsf(d[kz])) kz = 1;
    if (fabsf(d[2]) > fabsf(d[kz])) kz = 2;
    int kx = kz + 1; if (kx == 3) kx = 0;
    int ky = kx + 1; if (ky == 3) ky = 0;
    if (d[kz] < 0.0f) { int tmp = kx; kx = ky; ky = tmp; }   /* keep the winding */
    float Sx = d[kx] / d[kz];
    float Sy = d[ky] / d[kz];
    float Sz = 1.0f / d[kz];

    /* Vertices relative to the ray origin. */
    float A[3], B[3], C[3];
    for (int c = 0; c < 3; ++c) { A[c] = v0[c] - o[c]; B[c] = v1[c] - o[c]; C[c] = v2[c] - o[c]; }
    /* Shear so that the ray runs along +z of ray space. */
    float Ax = A[kx] - Sx * A[kz];
    float Ay = A[ky] - Sy * A[kz];
    float Bx = B[kx] - Sx * B[kz];
    float By = B[ky] - Sy * B[kz];
    float Cx = C[kx] - Sx * C[kz];
    float Cy = C[ky] - Sy * C[kz];
    /* Scaled barycentrics: 2-D edge functions. */
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = U + V + W;
    if (det == 0.0f) return 0;
    float Az = Sz * A[kz];
    float Bz = Sz * B[kz];
    float Cz = Sz * C[kz];
    float T = U * Az + V * Bz + W * Cz;
    float t = T / det;
    if (!(t > 0.0f)) return 0;
    *t_out = t;
    /* det > 0 exactly when the geometric normal cross(v1-v0, v2-v0) faces
     * against the ray (the axis swap above keeps ray space right-handed). */
    *front_out = det > 0.0f;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Closest hit                                                               */
/* ------------------------------------------------------------------------ */

static int closest_brute(const orc_scene* s, const float o[3], const float d[3],
                         float* t_out, int32_t* id_out, int* front_out) {
    int found = 0;
    float best = INFINITY;
    for (int32_t i = 0; i < s->n_tris; ++i) {
        float t; int fr;
        const float* tr = &s->tri[9 * i];
        if (orc_intersect(o, d, tr, tr + 3, tr + 6, &t, &fr) && t < best) {
            best = t; *id_out = i; *front_out = fr; found = 1;
        }
    }
    if (found) *t_out = best;
    return found;
}

/* The BVH only speeds up the brute-force definition, so its box tests must
 * never reject a box holding the closest watertight hit:
 *  - the float watertight test accepts rays passing within a few ulp of
 *    (|v| + |o|) of a triangle, so boxes are widened by 2^-18 (R + max|o|);
 *  - a box is skipped as "farther than the best hit" only by the entry of the
 *    slab of the ray's dominant axis kz: the watertight t is a weighted mean
 *    of the vertices' kz distances, never below that entry, whatever the
 *    ray's angle (the full box entry is no such bound for grazing rays). */
static int slab(const obvh_node* nd, const double o[3], const double inv[3], double pad, int kz,
                double tmax_prune) {
    double t0 = 0.0, t1 = INFINITY, tk = -INFINITY;
    for (int c = 0; c < 3; ++c) {
        double lo = (double)nd->lo[c] - pad, hi = (double)nd->hi[c] + pad;
        double a, b;
        if (isinf(inv[c])) {
            if (o[c] < lo || o[c] > hi) return 0;
            continue;
        }
        a = (lo - o[c]) * inv[c];
        b = (hi - o[c]) * inv[c];
        if (a > b) { double tmp = a; a = b; b = tmp; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
        if (c == kz) tk = a;
    }
    if (t0 > t1 * (1.0 + 1e-9)) return 0;
    if (tk > tmax_prune) return 0;
    return 1;
}

static int closest_bvh(const orc_scene* s, const float o[3], const float d[3],
                       float* t_out, int32_t* id_out, int* front_out) {
    double od[3], inv[3];
    double omax = 0.0;
    for (int c = 0; c < 3; ++c) {
        od[c] = o[c];
        inv[c] = (d[c] == 0.0f) ? INFINITY : 1.0 / (double)d[c];
        if (fabs(od[c]) > omax) omax = fabs(od[c]);
    }
    int kz = 0;                                   /* dominant axis, as in orc_intersect */
    if (fabsf(d[1]) > fabsf(d[kz])) kz = 1;
    if (fabsf(d[2]) > fabsf(d[kz])) kz = 2;
    const double pad = ldexp(s->radius + omax, -18);
    int found = 0;
    float best = INFINITY;
    int32_t best_id = -1;
    int best_front = 0;
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const obvh_node* nd = &s->nodes[stack[--sp]];
        double prune = found ? (double)best * (1.0 + 1e-5) : INFINITY;
        if (!slab(nd, od, inv, pad, kz, prune)) continue;
        if (nd->count > 0) {
            for (int32_t k = nd->first; k < nd->first + nd->count; ++k) {
                int32_t id = s->order[k];
                const float* tr = &s->tri[9 * id];
                float t; int fr;
                if (orc_intersect(o, d, tr, tr + 3, tr + 6, &t, &fr)) {
                    if (!found || t < best || (t == best && id < best_id)) {
                        best = t; best_id = id; best_front = fr; found = 1;
                    }
                }
            }
        } else {
            stack[sp++] = nd->first + 1;
            stack[sp++] = nd->first;
        }
    }
    if (found) { *t_out = best; *id_out = best_id; *front_out = best_front; }
    return found;
}

int orc_closest_hit(const orc_scene* s, const float o[3], const float d[3], int brute,
                    float* t, int32_t* id, int* front) {
    if (!s || s->n_tris == 0) return 0;
    if (brute || !s->nodes) return closest_brute(s, o, d, t, id, front);
    return closest_bvh(s, o, d, t, id, front);
}

/* ------------------------------------------------------------------------ */
/* Shading                                                                   */
/* ------------------------------------------------------------------------ */

static float clamp01(float v) {
    if (!(v > 0.0f)) v = 0.0f;      /* also maps NaN to 0 */
    if (v > 1.0f) v = 1.0f;
    return v;
}

void orc_normal(const orc_scene* s, int32_t id, float n[3]) {
    const float* tr = &s->tri[9 * id];
    float e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = tr[3 + c] - tr[c]; e2[c] = tr[6 + c] - tr[c]; }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    float len = sqrtf((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
    for (int c = 0; c < 3; ++c) n[c] = n[c] / len;
}

void orc_shade(const orc_scene* s, int32_t id, int front, float rgb[3]) {
    float n[3];
    orc_normal(s, id, n);
    if (!front) for (int c = 0; c < 3; ++c) n[c] = -n[c];
    float dot = (n[0] * s->light[0] + n[1] * s->light[1]) + n[2] * s->light[2];
    float diff = dot > 0.0f ? dot : 0.0f;
    float shade = s->k_a + s->k_d * diff;
    for (int c = 0; c < 3; ++c) rgb[c] = clamp01(s->rgb[3 * id + c] * shade);
}

/* One (u,v) step of F: camera from the previous image/data, then render.
 * aux receives the data the depth and normal mappings read in the next pass:
 * the view depth of the hit along the base camera's forward axis, and the
 * hit triangle's unit geometric normal (+inf and 0 after a miss). */
static void pixel_step(const orc_scene* s, const orc_camera* cam, int W, int H, int x, int y,
                       const float prev[3], const float* prev_aux, int mode, float z0, float le,
                       float ld, float rgb[3], int32_t* id_out, float aux[4]) {
    float o[3], d[3], t;
    int32_t id;
    int front;
    orc_ray(cam, W, H, x, y, prev, prev_aux, mode, z0, le, ld, o, d);
    if (orc_closest_hit(s, o, d, 0, &t, &id, &front)) {
        orc_shade(s, id, front, rgb);
        *id_out = id;
        float P[3];
        for (int c = 0; c < 3; ++c) P[c] = o[c] + t * d[c];
        aux[0] = ((P[0] - cam->eye[0]) * cam->forward[0] + (P[1] - cam->eye[1]) * cam->forward[1]) +
                 (P[2] - cam->eye[2]) * cam->forward[2];
        orc_normal(s, id, &aux[1]);
    } else {
        for (int c = 0; c < 3; ++c) rgb[c] = s->background[c];
        *id_out = -1;
        aux[0] = INFINITY;
        aux[1] = aux[2] = aux[3] = 0.0f;
    }
}

/* ------------------------------------------------------------------------ */
/* Passes, threaded over rows                                                */
/* ------------------------------------------------------------------------ */

int orc_default_threads(void) {
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

typedef struct {
    const orc_scene* s;
    const orc_camera* cam;
    int W, H;
    int mode;
    float z0, le, ld;
    const float* prev;
    const float* prev_aux;
    float* out;
    int32_t* ids;
    float* out_aux;
    atomic_int next_row;
} pass_job;

static void* pass_worker(void* arg) {
    pass_job* j = (pass_job*)arg;
    static const float seed[3] = {0.5f, 0.5f, 0.5f};
    for (;;) {
        int y = atomic_fetch_add(&j->next_row, 1);
        if (y >= j->H) break;
        for (int x = 0; x < j->W; ++x) {
            size_t p = (size_t)y * j->W + x;
            const float* pv = j->prev ? &j->prev[3 * p] : seed;
            const float* pa = j->prev_aux ? &j->prev_aux[4 * p] : NULL;
            int32_t id;
            float aux[4];
            pixel_step(j->s, j->cam, j->W, j->H, x, y, pv, pa, j->mode, j->z0, j->le, j->ld, &j->out[3 * p],
                       &id, aux);
            if (j->ids) j->ids[p] = id;
            if (j->out_aux) memcpy(&j->out_aux[4 * p], aux, sizeof aux);
        }
    }
    return NULL;
}

static void run_threads(void* (*fn)(void*), void* job, int nthreads) {
    if (nthreads <= 0) nthreads = orc_default_threads();
    if (nthreads == 1) { fn(job); return; }
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, fn, job);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
}

/* Closest hits of n rays, spread over threads: the same query as
 * orc_closest_hit, one ray per call. */
typedef struct {
    const orc_scene* s;
    const float* o;
    const float* d;
    int n, brute;
    float* t;
    int32_t* id;
    int32_t* front;
    atomic_int next;
} hits_job;

static void* hits_worker(void* arg) {
    hits_job* j = (hits_job*)arg;
    for (;;) {
        int i = atomic_fetch_add(&j->next, 1);
        if (i >= j->n) break;
        float t;
        int32_t id;
        int fr;
        if (orc_closest_hit(j->s, &j->o[3 * (size_t)i], &j->d[3 * (size_t)i], j->brute, &t, &id, &fr)) {
            j->t[i] = t; j->id[i] = id; j->front[i] = fr;
        } else {
            j->t[i] = INFINITY; j->id[i] = -1; j->front[i] = 0;
        }
    }
    return NULL;
}

int orc_closest_hits(const orc_scene* s, const float* o, const float* d, int n, int brute,
                     float* t, int32_t* id, int32_t* front, int nthreads) {
    if (!s || n < 0 || (n > 0 && (!o || !d || !t || !id || !front))) return -1;
    hits_job j;
    j.s = s; j.o = o; j.d = d; j.n = n; j.brute = brute; j.t = t; j.id = id; j.front = front;
    atomic_init(&j.next, 0);
    run_threads(hits_worker, &j, nthreads);
    return 0;
}

int orc_render_pass(const orc_scene* s, const orc_camera* cam, int W, int H, int mode, float z0,
                    float lambda_eye, float lambda_dir, const float* prev, const float* prev_aux,
                    float* out, int32_t* ids, float* out_aux, int nthreads) {
    if (!s || !cam || W < 1 || H < 1 || !out || mode < 0 || mode > 2) return -1;
    pass_job j;
    j.s = s; j.cam = cam; j.W = W; j.H = H; j.mode = mode; j.z0 = z0; j.le = lambda_eye; j.ld = lambda_dir;
    j.prev = prev; j.prev_aux = prev_aux; j.out = out; j.ids = ids; j.out_aux = out_aux;
    atomic_init(&j.next_row, 0);
    run_threads(pass_worker, &j, nthreads);
    return 0;
}

int orc_render(const orc_scene* s, const orc_camera* cam, int W, int H, int K, int mode, float z0,
               float lambda_eye, float lambda_dir, float* out, int32_t* ids, int nthreads) {
    if (!s || !cam || W < 1 || H < 1 || K < 1 || !out || mode < 0 || mode > 2) return -1;
    size_t P = (size_t)W * H;
    float* aux[2] = {NULL, NULL};
    if (mode != ORC_MODE_COLOR) {
        aux[0] = (float*)malloc(sizeof(float) * 4 * P);
        aux[1] = (float*)malloc(sizeof(float) * 4 * P);
    }
    /* I_0 is the grey seed; image k of the output is the paper's I_{k+1}. */
    for (int k = 0; k < K; ++k) {
        const float* prev = k == 0 ? NULL : &out[(size_t)(k - 1) * P * 3];
        const float* prev_aux = k == 0 ? NULL : aux[(k - 1) & 1];
        int rc = orc_render_pass(s, cam, W, H, mode, z0, lambda_eye, lambda_dir, prev, prev_aux,
                                 &out[(size_t)k * P * 3], ids ? &ids[(size_t)k * P] : NULL, aux[k & 1],
                                 nthreads);
        if (rc) { free(aux[0]); free(aux[1]); return rc; }
    }
    free(aux[0]);
    free(aux[1]);
    return 0;
}

typedef struct {
    const orc_scene* s;
    const orc_camera* cam;
    int W, H, K;
    int mode;
    float z0, le, ld;
    const int32_t* pix;
    int n;
    float* out;
    int32_t* ids;
    atomic_int next;
} pix_job;

static void* pix_worker(void* arg) {
    pix_job* j = (pix_job*)arg;
    for (;;) {
        int i = atomic_fetch_add(&j->next, 1);
        if (i >= j->n) break;
        int p = j->pix[i];
        int x = p % j->W, y = p / j->W;
        float prev[3] = {0.5f, 0.5f, 0.5f};
        float aux[4], prev_aux[4];
        int have_aux = 0;
        for (int k = 0; k < j->K; ++k) {
            float rgb[3];
            int32_t id;
            pixel_step(j->s, j->cam, j->W, j->H, x, y, prev, have_aux ? prev_aux : NULL, j->mode, j->z0,
                       j->le, j->ld, rgb, &id, aux);
            memcpy(&j->out[((size_t)i * j->K + k) * 3], rgb, sizeof rgb);
            if (j->ids) j->ids[(size_t)i * j->K + k] = id;
            memcpy(prev, rgb, sizeof rgb);
            memcpy(prev_aux, aux, sizeof aux);
            have_aux = 1;
        }
    }
    return NULL;
}

int orc_render_pixels(const orc_scene* s, const orc_camera* cam, int W, int H, int K, int mode, float z0,
                      float lambda_eye, float lambda_dir, const int32_t* pix, int n,
                      float* out, int32_t* ids, int nthreads) {
    if (!s || !cam || W < 1 || H < 1 || K < 1 || n < 0 || (n > 0 && (!pix || !out)) || mode < 0 || mode > 2)
        return -1;
    for (int i = 0; i < n; ++i)
        if (pix[i] < 0 || (int64_t)pix[i] >= (int64_t)W * H) return -1;
    pix_job j;
    j.s = s; j.cam = cam; j.W = W; j.H = H; j.K = K; j.mode = mode; j.z0 = z0; j.le = lambda_eye;
    j.ld = lambda_dir; j.pix = pix; j.n = n; j.out = out; j.ids = ids;
    atomic_init(&j.next, 0);
    run_threads(pix_worker, &j, nthreads);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Screen-space variant (Section 6, edges Section 6.1)                       */
/* ------------------------------------------------------------------------ */

/* Edge rule for a source index i outside [0, n). */
static int edge_index(int i, int n, int edge) {
    if (edge == ORC_EDGE_CLAMP) return i < 0 ? 0 : (i >= n ? n - 1 : i);
    if (edge == ORC_EDGE_WRAP) { int m = i % n; return m < 0 ? m + n : m; }
    /* mirror about the image border, the border pixel repeated: -1 -> 0, n -> n-1 */
    int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

int orc_gather_pass(const float* in, int W, int H, float max_smudge, int edge, int centred, float* out) {
    if (!in || !out || W < 1 || H < 1 || edge < 0 || edge > 2) return -1;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const float* c = &in[3 * ((size_t)y * W + x)];
            /* the pixel's own red and green choose where its new colour comes
             * from: right for red, up for green (Section 3's axes) */
            float mr = centred ? 2.0f * c[0] - 1.0f : c[0];
            float mg = centred ? 2.0f * c[1] - 1.0f : c[1];
            float px = ((float)x + 0.5f) + mr * max_smudge;
            float py = ((float)y + 0.5f) - mg * max_smudge;
            int sx = edge_index((int)floorf(px), W, edge);
            int sy = edge_index((int)floorf(py), H, edge);
            memcpy(&out[3 * ((size_t)y * W + x)], &in[3 * ((size_t)sy * W + sx)], 3 * sizeof(float));
        }
    }
    return 0;
}

int orc_gather(const float* in, int W, int H, int n, float max_smudge, int edge, int centred, float* out) {
    if (n < 1) return -1;
    size_t P = (size_t)W * H;
    for (int k = 0; k < n; ++k) {
        int rc = orc_gather_pass(k == 0 ? in : &out[(size_t)(k - 1) * P * 3], W, H, max_smudge, edge, centred,
                                 &out[(size_t)k * P * 3]);
        if (rc) return rc;
    }
    return 0;
}
