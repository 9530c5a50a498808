/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY: a driver that runs every
 * entry point of the oracle once, so that the oracle can be built with the
 * address and undefined-behaviour sanitizers and checked for memory errors
 * (tests/test_sanitizers.py builds and runs it).
 *
 * Usage: sanitize_check SCENE_FILE
 * The scene file holds, little-endian: uint32 n_verts, uint32 n_tris, then
 * float32 verts[n_verts][3], uint32 idx[n_tris][3], float32 rgb[n_tris][3].
 * Exit status 0 when every call succeeds and the BVH agrees with the
 * brute-force scan on the rendered images.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rcp_oracle.h"

static void* read_all(FILE* f, size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (p && bytes && fread(p, 1, bytes, f) != bytes) {
        free(p);
        return NULL;
    }
    return p;
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint32_t nv = 0, nt = 0;
    if (fread(&nv, 4, 1, f) != 1 || fread(&nt, 4, 1, f) != 1) return 2;
    float* verts = (float*)read_all(f, sizeof(float) * 3 * nv);
    uint32_t* idx = (uint32_t*)read_all(f, sizeof(uint32_t) * 3 * nt);
    float* rgb = (float*)read_all(f, sizeof(float) * 3 * nt);
    fclose(f);
    if (!verts || !idx || !rgb) return 2;

    orc_scene_desc d;
    memset(&d, 0, sizeof d);
    d.verts = verts; d.n_verts = nv; d.idx = idx; d.n_tris = nt; d.rgb = rgb;
    d.light[0] = 0.3f; d.light[1] = 0.8f; d.light[2] = -0.5f;
    float ll = sqrtf(d.light[0] * d.light[0] + d.light[1] * d.light[1] + d.light[2] * d.light[2]);
    for (int c = 0; c < 3; ++c) { d.light[c] /= ll; d.background[c] = 0.5f; }
    d.k_a = 0.0f; d.k_d = 1.0f;
    orc_scene* bvh = orc_scene_create(&d, 1);
    orc_scene* brute = orc_scene_create(&d, 0);
    if (!bvh || !brute) return 3;
    int32_t st[3];
    orc_scene_stats(bvh, st);

    /* eye (0, 0.5, -1.4) looking at (0, 0.05, 0), 60 degrees */
    orc_camera cam;
    memset(&cam, 0, sizeof cam);
    cam.eye[0] = 0.0f; cam.eye[1] = 0.5f; cam.eye[2] = -1.4f;
    float fw[3] = {0.0f, 0.05f - 0.5f, 1.4f};
    float fl = sqrtf(fw[0] * fw[0] + fw[1] * fw[1] + fw[2] * fw[2]);
    for (int c = 0; c < 3; ++c) cam.forward[c] = fw[c] / fl;
    /* right = normalize(up x forward), up' = forward x right */
    float r[3] = {1.0f * cam.forward[2] - 0.0f * cam.forward[1], 0.0f * cam.forward[0] - 0.0f * cam.forward[2],
                  0.0f * cam.forward[1] - 1.0f * cam.forward[0]};
    float rl = sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int c = 0; c < 3; ++c) cam.right[c] = r[c] / rl;
    cam.up[0] = cam.forward[1] * cam.right[2] - cam.forward[2] * cam.right[1];
    cam.up[1] = cam.forward[2] * cam.right[0] - cam.forward[0] * cam.right[2];
    cam.up[2] = cam.forward[0] * cam.right[1] - cam.forward[1] * cam.right[0];
    cam.tan_half_fovy = 0.57735026f;

    const int W = 37, H = 23, K = 4;
    const size_t P = (size_t)W * H;
    int bad = 0;
    for (int mode = 0; mode < 3; ++mode) {
        float* a = (float*)malloc(sizeof(float) * 3 * P * K);
        float* b = (float*)malloc(sizeof(float) * 3 * P * K);
        int32_t* ia = (int32_t*)malloc(sizeof(int32_t) * P * K);
        int32_t* ib = (int32_t*)malloc(sizeof(int32_t) * P * K);
        if (orc_render(bvh, &cam, W, H, K, mode, 1.2f, 0.01f, 0.05f, a, ia, 3)) return 4;
        if (orc_render(brute, &cam, W, H, K, mode, 1.2f, 0.01f, 0.05f, b, ib, 1)) return 4;
        if (memcmp(a, b, sizeof(float) * 3 * P * K) || memcmp(ia, ib, sizeof(int32_t) * P * K)) bad = 1;
        /* whole chains of a few pixels */
        int32_t pix[5] = {0, (int32_t)P - 1, W + 3, (int32_t)(P / 2), 7};
        float chains[5 * 4 * 3];
        int32_t chain_ids[5 * 4];
        if (orc_render_pixels(bvh, &cam, W, H, K, mode, 1.2f, 0.01f, 0.05f, pix, 5, chains, chain_ids, 2)) return 4;
        for (int i = 0; i < 5; ++i)
            for (int k = 0; k < K; ++k)
                if (memcmp(&chains[(i * K + k) * 3], &a[((size_t)k * P + pix[i]) * 3], 12)) bad = 1;
        /* one pass with hit data */
        float* aux = (float*)malloc(sizeof(float) * 4 * P);
        if (orc_render_pass(bvh, &cam, W, H, mode, 1.2f, 0.01f, 0.05f, NULL, NULL, b, ib, aux, 2)) return 4;
        free(aux);
        free(a); free(b); free(ia); free(ib);
    }
    /* batched closest hits against single queries */
    const int n = 64;
    float o[64 * 3], dir[64 * 3], t[64];
    int32_t id[64], front[64];
    for (int i = 0; i < n; ++i) {
        orc_ray(&cam, W, H, i % W, (i * 7) % H, (const float[3]){0.5f, 0.5f, 0.5f}, NULL, 0, 0.0f, 0.0f, 0.0f,
                &o[3 * i], &dir[3 * i]);
    }
    if (orc_closest_hits(bvh, o, dir, n, 0, t, id, front, 4)) return 4;
    for (int i = 0; i < n; ++i) {
        float t1; int32_t id1 = -1; int f1 = 0;
        int hit = orc_closest_hit(brute, &o[3 * i], &dir[3 * i], 1, &t1, &id1, &f1);
        if (hit != (id[i] >= 0) || (hit && (t1 != t[i] || id1 != id[i] || f1 != front[i]))) bad = 1;
    }
    /* shading, normals, the screen-space passes */
    float rgbv[3], nrm[3];
    if (nt > 0) {
        orc_shade(bvh, 0, 1, rgbv);
        orc_normal(bvh, (int32_t)nt - 1, nrm);
    }
    float* img = (float*)malloc(sizeof(float) * 3 * P);
    for (size_t i = 0; i < 3 * P; ++i) img[i] = (float)((i * 37) % 101) / 100.0f;
    float* g = (float*)malloc(sizeof(float) * 3 * P * 3);
    for (int edge = 0; edge < 3; ++edge)
        if (orc_gather(img, W, H, 3, 4.5f, edge, edge != 1, g)) return 4;
    free(img);
    free(g);
    orc_scene_destroy(bvh);
    orc_scene_destroy(brute);
    free(verts); free(idx); free(rgb);
    printf("sanitize_check: %u triangles, %d BVH nodes, %s\n", nt, st[0], bad ? "MISMATCH" : "ok");
    return bad ? 5 : 0;
}
