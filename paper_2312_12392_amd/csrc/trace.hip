// The K-pass render: one persistent kernel launch per pass.
//
// Per pass, every wave repeatedly takes 64 work items from a pass counter.
// A work item is a pixel still being painted: at pass 0 the pixels in 8x8
// tiles (with the grey seed, or a caller-supplied previous image), later the
// compact list {pixel, previous RGB} appended by the pass before.  For each
// item the lane
//   1. builds the pixel's displaced camera ray from its previous colour
//      (Section 2 ray and displacements, Section 3 colour mapping),
//   2. traverses the BVH (top levels from LDS, a short per-lane stack in LDS
//      that overflows into a per-lane global area) and runs the watertight
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
#include <climits>
#include <cstdlib>

#include "rcp_internal.hpp"

namespace rcp {
namespace {

constexpr int kBlock = 256;
#ifndef RCP_STACK
#define RCP_STACK 8
#endif
constexpr int kStack = RCP_STACK;                // per-lane LDS stack entries (power of two not required)
constexpr float kSlack = 1.0f + 1.0f / 65536.0f; // widening of box intervals

struct PassArgs {
    DevScene sc;
    Camera cam;
    int W, H, K, k;
    float le, ld, z0;
    uint32_t n_items0;              // pass-0 items (8x8 tiles * 64)
    int refill_min;                 // idle lanes that trigger a refill (1..64)
    int tiles_x;
    const float4* state_in;         // pass > 0: {pix bits, r, g, b}
    const float4* aux_in;           // pass > 0, depth/normal modes: {view depth, normal}
    const float* prev_img;          // pass 0: previous image or NULL (grey seed)
    const float* prev_aux;          // pass 0: previous [H][W][4] hit data or NULL (seed)
    float4* state_out;              // NULL: no following pass
    float4* aux_out;
    uint32_t* counters;             // [kMaxPasses] list sizes, [kMaxPasses..] fetch
    float* out;                     // [K][H][W][3]
    int32_t* ids;                   // [K][H][W] or NULL
    float* out_aux;                 // [H][W][4] of image k or NULL (single passes)
    int32_t* spill;
    uint32_t spill_stride;          // threads in the grid
    unsigned long long* stats;      // [kMaxPasses][4] or NULL
};

__device__ inline float sel3(float x, float y, float z, int k) {
    return k == 0 ? x : (k == 1 ? y : z);
}

__device__ inline uint32_t lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Ray of pixel (x, y): P'_e = P_e + V_e, N = normalize(P'_p - P'_e), with
// w from the pixel's previous colour and hit data `aux` (view depth, unit
// normal): the colour vector (2R-1) right + (2G-1) up + (2B-1) forward
// (Section 3), that vector times |z - z0| (Section 4, none after a miss), or
// C x N with C the undisplaced view direction (Section 5).
template <int MODE>
__device__ inline void make_ray(const Camera& c, int W, int H, int x, int y, float pr, float pg, float pb,
                                const float aux[4], float z0, float le, float ld, float o[3], float d[3]) {
    const float fx = (float)(2 * x + 1) / (float)W - 1.0f;
    const float fy = 1.0f - (float)(2 * y + 1) / (float)H;
    const float aspect = (float)W / (float)H;
    const float s = fx * (c.th * aspect);
    const float t = fy * c.th;
    float q[3], w[3], dp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = (c.forward[a] + s * c.right[a]) + t * c.up[a];
    if (MODE == RCP_MODE_NORMAL) {
        const float ql = sqrtf((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
        const float C0 = q[0] / ql, C1 = q[1] / ql, C2 = q[2] / ql;
        w[0] = C1 * aux[3] - C2 * aux[2];
        w[1] = C2 * aux[1] - C0 * aux[3];
        w[2] = C0 * aux[2] - C1 * aux[1];
    } else {
        const float mr = 2.0f * pr - 1.0f;
        const float mg = 2.0f * pg - 1.0f;
        const float mb = 2.0f * pb - 1.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a] = (mr * c.right[a] + mg * c.up[a]) + mb * c.forward[a];
        if (MODE == RCP_MODE_DEPTH) {
            const float kz = (aux[0] < INFINITY) ? fabsf(aux[0] - z0) : 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) w[a] = kz * w[a];
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = c.eye[a] + le * w[a];
        dp[a] = q[a] + ld * w[a];
    }
    const float len = sqrtf((dp[0] * dp[0] + dp[1] * dp[1]) + dp[2] * dp[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = dp[a] / len;
}

// Ray constants of the watertight test (Woop, Benthin, Wald, JCGT 2013):
// the dominant direction axis kz (first of equal magnitudes), kx and ky
// following it cyclically and swapped when d[kz] < 0, and the shear.
struct RayW {
    int kx, ky, kz;
    float Sx, Sy, Sz;
    float ox, oy, oz;     // origin components along kx, ky, kz
};

__device__ inline RayW ray_setup(const float o[3], const float d[3]) {
    RayW r;
    int kz = 0;
    if (fabsf(d[1]) > fabsf(d[0])) kz = 1;
    if (fabsf(d[2]) > fabsf(sel3(d[0], d[1], d[2], kz))) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    const float dz = sel3(d[0], d[1], d[2], kz);
    if (dz < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.Sx = sel3(d[0], d[1], d[2], kx) / dz;
    r.Sy = sel3(d[0], d[1], d[2], ky) / dz;
    r.Sz = 1.0f / dz;
    r.ox = sel3(o[0], o[1], o[2], kx);
    r.oy = sel3(o[0], o[1], o[2], ky);
    r.oz = sel3(o[0], o[1], o[2], kz);
    return r;
}

// Watertight test against triangle (v0, v1, v2).  On a hit with t > 0
// returns true with t and front (det > 0: the normal cross(v1-v0, v2-v0)
// faces against the ray).
__device__ inline bool hit_triangle(const RayW& r, const float4& v0, const float4& v1, const float4& v2,
                                    float& t_out, bool& front) {
    const float Akx = sel3(v0.x, v0.y, v0.z, r.kx) - r.ox;
    const float Aky = sel3(v0.x, v0.y, v0.z, r.ky) - r.oy;
    const float Akz = sel3(v0.x, v0.y, v0.z, r.kz) - r.oz;
    const float Bkx = sel3(v1.x, v1.y, v1.z, r.kx) - r.ox;
    const float Bky = sel3(v1.x, v1.y, v1.z, r.ky) - r.oy;
    const float Bkz = sel3(v1.x, v1.y, v1.z, r.kz) - r.oz;
    const float Ckx = sel3(v2.x, v2.y, v2.z, r.kx) - r.ox;
    const float Cky = sel3(v2.x, v2.y, v2.z, r.ky) - r.oy;
    const float Ckz = sel3(v2.x, v2.y, v2.z, r.kz) - r.oz;
    const float Ax = Akx - r.Sx * Akz;
    const float Ay = Aky - r.Sy * Akz;
    const float Bx = Bkx - r.Sx * Bkz;
    const float By = Bky - r.Sy * Bkz;
    const float Cx = Ckx - r.Sx * Ckz;
    const float Cy = Cky - r.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        // exact products in FP64, one rounding of each difference
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = U + V + W;
    if (det == 0.0f) return false;
    const float Az = r.Sz * Akz;
    const float Bz = r.Sz * Bkz;
    const float Cz = r.Sz * Ckz;
    const float T = U * Az + V * Bz + W * Cz;
    const float t = T / det;
    if (!(t > 0.0f)) return false;
    t_out = t;
    front = det > 0.0f;
    return true;
}

struct Hit {
    float t;
    int32_t id;        // original triangle index, INT_MAX when none
    uint32_t slot;     // packed triangle index
    bool front;
};

// Per-lane traversal stack: the newest kStack entries live in LDS (column
// `lane_col` of the block's stack area), older ones in the lane's global
// overflow area.
struct Stack {
    int32_t* lds;       // &stack_area[tid]; entry e at lds[(e % kStack) * kBlock]
    int32_t* spill;     // &spill[gtid]; entry e at spill[e * stride]
    uint32_t stride;
    int sp, lo;         // entries [0, lo) spilled, [lo, sp) in LDS

    __device__ inline void push(int32_t v) {
        if (sp - lo == kStack) {
            spill[(size_t)lo * stride] = lds[(lo % kStack) * kBlock];
            ++lo;
        }
        lds[(sp % kStack) * kBlock] = v;
        ++sp;
    }
    __device__ inline int32_t pop() {
        if (sp == 0) return -1;
        --sp;
        if (sp < lo) {       // the LDS part is empty: take the newest spilled entry
            lo = sp;
            return spill[(size_t)sp * stride];
        }
        return lds[(sp % kStack) * kBlock];
    }
};

// Box tests never decide a result, they only prune, so they are built to
// never reject a box that holds the closest hit of the watertight test:
//  - the watertight test accepts rays passing within about 4 ulp of
//    (|v| + |o|) of a triangle, so every box is widened by
//    2^-18 (R + max|o|) on each side (R: largest |coordinate| in the scene),
//    folded into one origin per slab side;
//  - the test against the best hit so far uses only the slab of the ray's
//    dominant axis kz: the watertight t is a weighted mean of the vertices'
//    kz distances, so it is never below that slab's entry, whatever the ray's
//    angle to the triangle (the full box entry is not such a bound for
//    grazing rays);
//  - zero direction components use a large finite reciprocal (no inf * 0).
//
// The traversal state of one ray lives in registers (plus its stack), so a
// lane can advance its ray one step at a time and take a new ray as soon as
// the current one is finished.
struct Trav {
    RayW rw;
    float ix, iy, iz;       // reciprocal direction
    float lx, ly, lz;       // (o + pad) * inv: used against lo planes
    float hx, hy, hz;       // (o - pad) * inv: used against hi planes
    int32_t node;           // >= 0 inner node, other negative: leaf link, -1: finished
    uint32_t budget;
    Hit h;
};

__device__ inline void trav_init(Trav& tv, const DevScene& sc, const float o[3], const float d[3], Stack& st) {
    tv.rw = ray_setup(o, d);
    float inv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) inv[a] = fabsf(d[a]) > 1e-30f ? 1.0f / d[a] : copysignf(1e30f, d[a]);
    tv.ix = inv[0]; tv.iy = inv[1]; tv.iz = inv[2];
    // A plane at coordinate c is reached at t = c * inv - (o -/+ pad) * inv,
    // one fused multiply-add per plane.  Its rounding (a few ulp of |o * inv|)
    // is far inside the 2^-18 (R + max|o|) widening, so the bounds stay safe.
    const float pad = (sc.radius + fmaxf(fmaxf(fabsf(o[0]), fabsf(o[1])), fabsf(o[2]))) * 3.814697265625e-6f;
    tv.lx = (o[0] + pad) * inv[0]; tv.hx = (o[0] - pad) * inv[0];
    tv.ly = (o[1] + pad) * inv[1]; tv.hy = (o[1] - pad) * inv[1];
    tv.lz = (o[2] + pad) * inv[2]; tv.hz = (o[2] - pad) * inv[2];
    tv.node = sc.n_nodes > 0 ? 0 : -1;
    // Every node and leaf is entered at most once per ray; the bound only
    // guarantees termination should the tree ever be malformed.
    tv.budget = 2u * sc.n_nodes + 16u;
    tv.h.t = INFINITY;
    tv.h.id = INT_MAX;
    tv.h.slot = 0;
    tv.h.front = false;
    st.sp = 0;
    st.lo = 0;
}

// Visit one inner node: test both child boxes, continue with the nearer hit
// child, push the farther one, or pop when neither is hit.
template <bool STATS>
__device__ inline int32_t visit_inner(Trav& tv, int32_t node, const DevScene& sc, const float4* __restrict__ top,
                                      Stack& st, uint32_t& n_nodes) {
    const int kz = tv.rw.kz;
    float4 n0, n1, n2, n3;
    if ((uint32_t)node < sc.top_count) {
        n0 = top[4 * node + 0];
        n1 = top[4 * node + 1];
        n2 = top[4 * node + 2];
        n3 = top[4 * node + 3];
    } else {
        const float4* p = sc.nodes + 4 * (size_t)node;
        n0 = p[0];
        n1 = p[1];
        n2 = p[2];
        n3 = p[3];
    }
    if (STATS) ++n_nodes;
    const float lim = tv.h.t * kSlack;
    // child 0
    const float a0 = __builtin_fmaf(n0.x, tv.ix, -tv.lx), a1 = __builtin_fmaf(n0.y, tv.ix, -tv.hx);
    const float a2 = __builtin_fmaf(n0.z, tv.iy, -tv.ly), a3 = __builtin_fmaf(n0.w, tv.iy, -tv.hy);
    const float a4 = __builtin_fmaf(n2.x, tv.iz, -tv.lz), a5 = __builtin_fmaf(n2.y, tv.iz, -tv.hz);
    const float ex0 = fminf(a0, a1), ey0 = fminf(a2, a3), ez0 = fminf(a4, a5);
    const float tmin0 = fmaxf(fmaxf(ex0, ey0), fmaxf(ez0, 0.0f));
    const float tmax0 = fminf(fminf(fmaxf(a0, a1), fmaxf(a2, a3)), fmaxf(a4, a5)) * kSlack;
    const float near0 = kz == 0 ? ex0 : (kz == 1 ? ey0 : ez0);
    // child 1
    const float b0 = __builtin_fmaf(n1.x, tv.ix, -tv.lx), b1 = __builtin_fmaf(n1.y, tv.ix, -tv.hx);
    const float b2 = __builtin_fmaf(n1.z, tv.iy, -tv.ly), b3 = __builtin_fmaf(n1.w, tv.iy, -tv.hy);
    const float b4 = __builtin_fmaf(n2.z, tv.iz, -tv.lz), b5 = __builtin_fmaf(n2.w, tv.iz, -tv.hz);
    const float ex1 = fminf(b0, b1), ey1 = fminf(b2, b3), ez1 = fminf(b4, b5);
    const float tmin1 = fmaxf(fmaxf(ex1, ey1), fmaxf(ez1, 0.0f));
    const float tmax1 = fminf(fminf(fmaxf(b0, b1), fmaxf(b2, b3)), fmaxf(b4, b5)) * kSlack;
    const float near1 = kz == 0 ? ex1 : (kz == 1 ? ey1 : ez1);
    const bool hit0 = tmin0 <= tmax0 && near0 <= lim;
    const bool hit1 = tmin1 <= tmax1 && near1 <= lim;
    const int32_t c0 = __float_as_int(n3.x);
    const int32_t c1 = __float_as_int(n3.y);
    if (hit0 && hit1) {
        const bool first0 = tmin0 <= tmin1;
        st.push(first0 ? c1 : c0);
        node = first0 ? c0 : c1;
    } else if (hit0) {
        node = c0;
    } else if (hit1) {
        node = c1;
    } else {
        node = st.pop();
    }
    return node;
}

// Test the triangles of leaf `link` against the ray, keeping the closest hit.
template <bool STATS>
__device__ inline void visit_leaf(Trav& tv, int32_t link, const DevScene& sc, uint32_t& n_tris) {
    const int32_t node = link;
    // leaf: triangles [first, first + count)
    const uint32_t first = ((uint32_t)node >> 3) & 0x0FFFFFFFu;
    const uint32_t count = ((uint32_t)node & 7u) + 1u;
    for (uint32_t j = 0; j < count; ++j) {
        const float4* tp = sc.tris + 3 * (size_t)(first + j);
        const float4 v0 = tp[0], v1 = tp[1], v2 = tp[2];
        if (STATS) ++n_tris;
        float t;
        bool front;
        if (hit_triangle(tv.rw, v0, v1, v2, t, front)) {
            const int32_t id = __float_as_int(v0.w);
            if (t < tv.h.t || (t == tv.h.t && id < tv.h.id)) {
                tv.h.t = t;
                tv.h.id = id;
                tv.h.slot = first + j;
                tv.h.front = front;
            }
        }
    }
}

// One step: descend through inner nodes to a leaf and test it; sets
// tv.node = -1 once the ray is finished.  Speculation (after Aila and Laine,
// "Understanding the Efficiency of Ray Traversal on GPUs", HPG 2009): a lane
// that reaches a leaf keeps descending while other lanes of the wave are still
// looking for theirs, and holds the next leaf it meets for the following
// step, so the wave's leaf tests run together.
template <bool STATS>
__device__ inline void trav_step(Trav& tv, const DevScene& sc, const float4* __restrict__ top, Stack& st,
                                 uint32_t& n_nodes, uint32_t& n_tris) {
    int32_t node = tv.node;
    int32_t leaf = -1;
    for (;;) {
        if (node < -1 && leaf == -1) { leaf = node; node = st.pop(); }
        if (!__any(leaf == -1 && node >= 0)) break;
        if (node >= 0) {
            if (--tv.budget == 0u) { node = -1; leaf = -1; break; }
            node = visit_inner<STATS>(tv, node, sc, top, st, n_nodes);
        }
    }
    if (leaf != -1) visit_leaf<STATS>(tv, leaf, sc, n_tris);
    tv.node = node;
}

constexpr int kWaves = kBlock / 64;
constexpr int kStage = 128;     // per-wave staging of appended entries (flushed 64 at a time)

#ifndef RCP_WAVES_PER_EU
#define RCP_WAVES_PER_EU 1
#endif

template <bool STATS, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RCP_WAVES_PER_EU))) void k_pass(PassArgs a) {
    constexpr bool AUX = MODE != RCP_MODE_COLOR;
    extern __shared__ float4 smem[];
    float4* top = smem;                                                 // top_count * 4
    float4* stage_all = smem + 4 * a.sc.top_count;                      // kWaves * kStage (x2 with aux)
    int32_t* stack_area = (int32_t*)(stage_all + (AUX ? 2 : 1) * kWaves * kStage);   // kStack * kBlock

    for (uint32_t i = threadIdx.x; i < 4 * a.sc.top_count; i += kBlock) top[i] = a.sc.nodes[i];
    __syncthreads();

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
    uint32_t* fetch = &a.counters[kMaxPasses + a.k];
    float* out_k = a.out + (size_t)a.k * P * 3;
    uint32_t s_nodes = 0, s_tris = 0, s_rays = 0, s_app = 0;

    bool alive = false;
    bool drained = false;          // wave-uniform: the pass's list is used up
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
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(fetch, n_idle);
            base = __shfl(base, 0);
            if (base + n_idle >= n_items) drained = true;
            if (!alive) {
                const uint32_t item = base + lanes_below(idle);
                bool valid = item < n_items;
                int x = 0, y = 0;
                if (a.k == 0) {
                    const uint32_t tile = item >> 6;
                    const uint32_t l = item & 63u;
                    x = (int)((tile % (uint32_t)a.tiles_x) * 8u + (l & 7u));
                    y = (int)((tile / (uint32_t)a.tiles_x) * 8u + (l >> 3));
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
                    make_ray<MODE>(a.cam, a.W, a.H, x, y, pr, pg, pb, pa, a.z0, a.le, a.ld, ro, rd);
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
        if (alive && tv.node != -1) trav_step<STATS>(tv, a.sc, top, st, s_nodes, s_tris);

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
                    make_ray<MODE>(a.cam, a.W, a.H, x, y, pr, pg, pb, pa, a.z0, a.le, a.ld, ro, rd);
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
        unsigned long long* sk = a.stats + 4 * a.k;
        atomicAdd(&sk[0], (unsigned long long)s_rays);
        atomicAdd(&sk[1], (unsigned long long)s_nodes);
        atomicAdd(&sk[2], (unsigned long long)s_tris);
        atomicAdd(&sk[3], (unsigned long long)s_app);
    }
}

__global__ void k_clear_counters(uint32_t* c, int n, unsigned long long* stats) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0u;
    if (stats)
        for (int i = threadIdx.x; i < 4 * kMaxPasses; i += blockDim.x) stats[i] = 0ull;
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
    make_ray<MODE>(cam, W, H, x, y, pr, pg, pb, pa, z0, le, ld, o, d);
    for (int c = 0; c < 3; ++c) { org[3 * (size_t)p + c] = o[c]; dir[3 * (size_t)p + c] = d[c]; }
}

__global__ __launch_bounds__(kBlock) void k_trace_rays(DevScene sc, const float* __restrict__ org,
                                                        const float* __restrict__ dir, int n, float* __restrict__ out_t,
                                                        int32_t* __restrict__ out_id, int32_t* __restrict__ out_front,
                                                        int32_t* __restrict__ spill, uint32_t stride) {
    extern __shared__ float4 smem[];
    float4* top = smem;
    int32_t* stack_area = (int32_t*)(smem + 4 * sc.top_count + kWaves * kStage);
    for (uint32_t i = threadIdx.x; i < 4 * sc.top_count; i += kBlock) top[i] = sc.nodes[i];
    __syncthreads();
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
        uint32_t dn = 0, dt = 0;
        while (tv.node != -1) trav_step<false>(tv, sc, top, st, dn, dt);
        const bool hit = tv.h.id != INT_MAX;
        out_t[r] = hit ? tv.h.t : INFINITY;
        out_id[r] = hit ? tv.h.id : -1;
        if (out_front) out_front[r] = hit && tv.h.front ? 1 : 0;
    }
}

rcp_status ensure_workspace(rcp_scene* s, size_t n_state, size_t n_aux, size_t spill_entries) {
    Workspace& w = s->ws;
    if (n_aux > w.aux_cap) {
        for (int i = 0; i < 2; ++i) {
            if (w.aux[i]) { RCP_HIP(hipFree(w.aux[i])); w.aux[i] = nullptr; }
        }
        w.aux_cap = 0;
        for (int i = 0; i < 2; ++i) RCP_HIP(hipMalloc((void**)&w.aux[i], sizeof(float4) * n_aux));
        w.aux_cap = n_aux;
    }
    if (!w.counters) {
        RCP_HIP(hipMalloc((void**)&w.counters, sizeof(uint32_t) * (2 * kMaxPasses + 8)));
        RCP_HIP(hipMalloc((void**)&w.stats, sizeof(unsigned long long) * 4 * kMaxPasses));
    }
    if (n_state > w.state_cap) {
        for (int i = 0; i < 2; ++i) {
            if (w.state[i]) { RCP_HIP(hipFree(w.state[i])); w.state[i] = nullptr; }
        }
        w.state_cap = 0;
        for (int i = 0; i < 2; ++i) RCP_HIP(hipMalloc((void**)&w.state[i], sizeof(float4) * n_state));
        w.state_cap = n_state;
    }
    if (spill_entries > w.spill_cap) {
        if (w.spill) { RCP_HIP(hipFree(w.spill)); w.spill = nullptr; }
        w.spill_cap = 0;
        RCP_HIP(hipMalloc((void**)&w.spill, sizeof(int32_t) * spill_entries));
        w.spill_cap = spill_entries;
    }
    return RCP_OK;
}

// Idle lanes that make a wave fetch new work (RCP_REFILL_MIN, default 40).
int refill_min() {
    static int v = [] {
        const char* e = getenv("RCP_REFILL_MIN");
        int x = e ? atoi(e) : 40;
        return x < 1 ? 1 : (x > 64 ? 64 : x);
    }();
    return v;
}

struct GridInfo {
    int blocks = 0;
    size_t smem = 0;
};

template <typename KernelT>
rcp_status persistent_grid(KernelT kernel, const DevScene& sc, GridInfo& g, bool aux = false) {
    g.smem = sizeof(float4) * (4 * (size_t)sc.top_count + (aux ? 2 : 1) * kWaves * kStage) +
             sizeof(int32_t) * kStack * kBlock;
    int per_cu = 0;
    RCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, g.smem));
    int dev = 0, cus = 0;
    RCP_HIP(hipGetDevice(&dev));
    RCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu < 1) per_cu = 1;
    g.blocks = per_cu * cus;
    return RCP_OK;
}

}  // namespace

namespace {
template <bool STATS, int MODE>
rcp_status launch_passes(rcp_scene* s, PassArgs& a, int K, hipStream_t stream) {
    constexpr bool AUX = MODE != RCP_MODE_COLOR;
    GridInfo g;
    rcp_status st = persistent_grid(k_pass<STATS, MODE>, s->dev, g, AUX);
    if (st != RCP_OK) return st;
    const uint32_t threads = (uint32_t)g.blocks * kBlock;
    const size_t P = (size_t)a.W * (size_t)a.H;
    const size_t spill_depth = s->dev.max_depth > (uint32_t)kStack ? s->dev.max_depth - kStack + 1 : 1;
    st = ensure_workspace(s, K > 1 ? P : 1, (K > 1 && AUX) ? P : 0, spill_depth * threads);
    if (st != RCP_OK) return st;
    Workspace& w = s->ws;
    a.spill = w.spill;
    a.spill_stride = threads;
    a.counters = w.counters;
    a.stats = STATS ? w.stats : nullptr;
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(256), 0, stream, w.counters, 2 * kMaxPasses + 8,
                       STATS ? w.stats : (unsigned long long*)nullptr);
    RCP_CHECK_LAUNCH();
    for (int k = 0; k < K; ++k) {
        a.k = k;
        a.state_in = k == 0 ? nullptr : w.state[(k - 1) & 1];
        a.aux_in = (k == 0 || !AUX) ? nullptr : w.aux[(k - 1) & 1];
        a.state_out = k + 1 < K ? w.state[k & 1] : nullptr;
        a.aux_out = (k + 1 < K && AUX) ? w.aux[k & 1] : nullptr;
        if (k > 0) { a.prev_img = nullptr; a.prev_aux = nullptr; }
        hipLaunchKernelGGL((k_pass<STATS, MODE>), dim3(g.blocks), dim3(kBlock), g.smem, stream, a);
        RCP_CHECK_LAUNCH();
    }
    return RCP_OK;
}

template <bool STATS>
rcp_status launch_mode(rcp_scene* s, PassArgs& a, int K, int mode, hipStream_t stream) {
    switch (mode) {
        case RCP_MODE_DEPTH: return launch_passes<STATS, RCP_MODE_DEPTH>(s, a, K, stream);
        case RCP_MODE_NORMAL: return launch_passes<STATS, RCP_MODE_NORMAL>(s, a, K, stream);
        default: return launch_passes<STATS, RCP_MODE_COLOR>(s, a, K, stream);
    }
}
}  // namespace

rcp_status render(rcp_scene* s, const Camera& cam, int W, int H, int K, const Disp& disp, float* out_images,
                  int32_t* out_ids, const float* prev_rgb, const float* prev_aux, float* out_aux,
                  unsigned long long* host_counts, hipStream_t stream) {
    const bool stats = host_counts != nullptr;
    const int tiles_x = (W + 7) / 8, tiles_y = (H + 7) / 8;
    PassArgs a{};
    a.sc = s->dev;
    a.cam = cam;
    a.W = W; a.H = H; a.K = K;
    a.le = disp.le; a.ld = disp.ld; a.z0 = disp.z0;
    a.n_items0 = (uint32_t)tiles_x * (uint32_t)tiles_y * 64u;
    a.refill_min = refill_min();
    a.tiles_x = tiles_x;
    a.out = out_images;
    a.ids = out_ids;
    a.out_aux = out_aux;
    a.prev_img = prev_rgb;
    a.prev_aux = prev_aux;
    rcp_status st = stats ? launch_mode<true>(s, a, K, disp.mode, stream)
                          : launch_mode<false>(s, a, K, disp.mode, stream);
    if (st != RCP_OK) return st;
    if (stats) {
        RCP_HIP(hipMemcpyAsync(host_counts, s->ws.stats, sizeof(unsigned long long) * 4 * K, hipMemcpyDeviceToHost,
                               stream));
        RCP_HIP(hipStreamSynchronize(stream));
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
    rcp_status st = persistent_grid(k_trace_rays, s->dev, g);
    if (st != RCP_OK) return st;
    const uint32_t threads = (uint32_t)g.blocks * kBlock;
    const size_t spill_depth = s->dev.max_depth > (uint32_t)kStack ? s->dev.max_depth - kStack + 1 : 1;
    st = ensure_workspace(s, 1, 0, spill_depth * threads);
    if (st != RCP_OK) return st;
    hipLaunchKernelGGL(k_trace_rays, dim3(g.blocks), dim3(kBlock), g.smem, stream, s->dev, org, dir, n, out_t,
                       out_id, out_front, s->ws.spill, threads);
    RCP_CHECK_LAUNCH();
    return RCP_OK;
}

}  // namespace rcp
