// Device functions of one ray's life, shared by the pass kernels and the
// batched chain kernel: ray generation from the previous pass (Section 2 ray
// and displacements; Sections 3, 4, 5 mappings), the watertight ray/triangle
// test, the per-lane traversal stack and the BVH traversal step.
//
// Everything that decides a result (ray generation, the triangle test, the
// shade table) is FP32 evaluated left to right without contraction, with
// correctly rounded division and square root.  The box tests only prune and
// are widened so that they never reject a box the exact test would accept.
#pragma once
#include <climits>
#include <cstdlib>

#include "rcp_internal.hpp"

namespace rcp {
namespace {

constexpr int kBlock = 256;
constexpr int kStack = 16;                       // per-lane LDS stack entries
constexpr float kSlack = 1.0f + 1.0f / 65536.0f; // relative widening of the best-hit bound

// Global overflow entries per thread.  The LDS part holds `stack` entries
// (kStack unless the chain engine is tuned otherwise), and entries move to
// the overflow area stack / 2 at a time, when a push finds fewer than three
// free LDS slots: at most stack_bound - (stack - 2) + stack / 2 entries
// are then in the overflow area (three more kept as a margin).
inline size_t spill_per_thread(const DevScene& d, int stack = kStack) {
    const uint32_t keep = (uint32_t)(stack - stack / 2);
    return d.stack_bound + 3u > keep ? d.stack_bound + 3u - keep : 1u;
}


__device__ inline float sel3(float x, float y, float z, int k) {
    return k == 0 ? x : (k == 1 ? y : z);
}

// Mask of the wave's lanes where p holds (straight to a scalar register).
__device__ inline unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Lanes set in a wave mask, counted as two 32-bit halves: a count taken on
// the 64-bit value was compared in 64 bits, which the scalar unit cannot do.
__device__ inline uint32_t popc_u32(unsigned long long m) {
    return (uint32_t)__builtin_popcount((uint32_t)m) + (uint32_t)__builtin_popcount((uint32_t)(m >> 32));
}

__device__ inline uint32_t lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- work distribution ------------------------------------------------------
// A launch's work items are split into kFetchParts contiguous ranges (bands),
// one per XCD, each with its own counter (kFetchStride words apart).
// Workgroups are dispatched to the XCDs round robin, so the waves of one XCD
// start on their own band: neighbouring pixels trace through the same parts
// of the tree, and each XCD's L2 holds the nodes of its band.  A wave whose
// band is used up takes work from the next band, so no work is left undone.
constexpr uint32_t kFetchParts = 8;
constexpr uint32_t kFetchStride = 16;     // words between counters (64 bytes)
constexpr uint32_t kFetchWords = kFetchParts * kFetchStride;

__device__ inline uint32_t part_begin(uint32_t n_items, uint32_t p) {
    return p >= kFetchParts ? n_items : (uint32_t)(((uint64_t)n_items * p / kFetchParts) & ~63ull);
}

// Items [base, lim) for the wave's n_idle idle lanes (the lanes below lim
// get one each).  part and parts_done are wave-uniform (start: the
// workgroup's XCD, 0); drained is set once every band is used up.  Called by
// the whole wave.
__device__ inline void wave_fetch(uint32_t* ctr, uint32_t n_items, uint32_t n_idle, uint32_t& part,
                                  uint32_t& parts_done, bool& drained, uint32_t& base, uint32_t& lim) {
    // own band first, then the next ones; every attempt either takes items
    // or retires a band, so the loop ends
    if ((threadIdx.x & 63) == 0) {
        for (;;) {
            const uint32_t lo = part_begin(n_items, part), hi = part_begin(n_items, part + 1u);
            const uint32_t got = lo < hi ? atomicAdd(&ctr[kFetchStride * part], n_idle) : hi - lo;
            if (got < hi - lo) { base = lo + got; lim = hi; break; }
            part = (part + 1u) % kFetchParts;
            if (++parts_done >= kFetchParts) { base = lim = n_items; break; }
        }
    }
    // lane 0 is the first active lane (the whole wave is here)
    base = __builtin_amdgcn_readfirstlane(base);
    lim = __builtin_amdgcn_readfirstlane(lim);
    part = __builtin_amdgcn_readfirstlane(part);
    parts_done = __builtin_amdgcn_readfirstlane(parts_done);
    if (base + n_idle >= lim) {   // this band is used up now
        part = (part + 1u) % kFetchParts;
        ++parts_done;
    }
    if (parts_done >= kFetchParts) drained = true;
}

// Work item -> pixel.  Items come in 64-pixel tiles 2^tile_log2w wide;
// tiles are ordered by super-tiles of 2^super_log2 x 2^super_log2 tiles, row
// by row, so that the pixels in flight on one XCD form a compact patch of the
// screen (their rays share more of the tree than a thin strip of whole tile
// rows does).  The super-tile grid covers the image, so the items of its
// tiles beyond the image edges are skipped; views smaller than a super-tile
// keep plain tile rows (super_log2 = 0).  (Measured on the terrain frame:
// 8 x 8 tiles 1.8% faster than plain tile rows, 16 x 16 3.5%; super-tiles
// clipped to the image instead of padded were 2% slower than padded ones.)
constexpr int kSuperLog2 = 4;

inline int super_log2_for(int W, int H, int tile_log2w) {
    const int tiles_x = (W + (1 << tile_log2w) - 1) >> tile_log2w;
    const int tiles_y = (H + (64 >> tile_log2w) - 1) / (64 >> tile_log2w);
    return (tiles_x >= (1 << kSuperLog2) && tiles_y >= (1 << kSuperLog2)) ? kSuperLog2 : 0;
}

// Work items of a W x H view (a whole number of super-tiles).
inline uint64_t view_tile_items(int W, int H, int tile_log2w, int super_log2) {
    const uint64_t tw = 1ull << tile_log2w, th = 64u >> tile_log2w, side = 1ull << super_log2;
    const uint64_t sx = (((uint64_t)W + tw - 1u) / tw + side - 1u) / side;
    const uint64_t sy = (((uint64_t)H + th - 1u) / th + side - 1u) / side;
    return sx * sy * side * side * 64u;
}

__device__ inline void tile_pixel(uint32_t local, uint32_t tiles_x, uint32_t tile_log2w, uint32_t super_log2, int& x,
                                  int& y) {
    const uint32_t tile = local >> 6, l = local & 63u;
    const uint32_t tw = 1u << tile_log2w;
    const uint32_t sl = super_log2, sm = (1u << sl) - 1u;
    const uint32_t st = tile >> (2u * sl), w = tile & ((1u << (2u * sl)) - 1u);
    const uint32_t sx = (tiles_x + sm) >> sl;   // super-tiles per row
    const uint32_t tx = ((st % sx) << sl) + (w & sm), ty = ((st / sx) << sl) + (w >> sl);
    x = (int)(tx * tw + (l & (tw - 1u)));
    y = (int)(ty * (64u >> tile_log2w) + (l >> tile_log2w));
}

// Horizontal half extent of the image plane, tan(fovy / 2) * W / H: one value
// per view, the same bits on the host and the device.
__host__ __device__ inline float half_width(float th, int W, int H) {
    const float aspect = (float)W / (float)H;
    return th * aspect;
}

// Ray of pixel (x, y): P'_e = P_e + V_e, N = normalize(P'_p - P'_e), with
// w from the pixel's previous colour and hit data `aux` (view depth, unit
// normal): the colour vector (2R-1) right + (2G-1) up + (2B-1) forward
// (Section 3), that vector times |z - z0| (Section 4, none after a miss), or
// C x N with C the undisplaced view direction (Section 5).
// hw is half_width(c.th, W, H).  Cam is Camera, in any address space.
template <int MODE, class Cam>
__device__ inline void make_ray(const Cam& c, float hw, int W, int H, int x, int y, float pr, float pg, float pb,
                                const float aux[4], float z0, float le, float ld, float o[3], float d[3]) {
    const float fx = (float)(2 * x + 1) / (float)W - 1.0f;
    const float fy = 1.0f - (float)(2 * y + 1) / (float)H;
    const float s = fx * hw;
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
// following it cyclically, and the shear.  The test swaps kx and ky when
// d[kz] < 0; here they stay in cyclic order and the swap is applied to the
// result instead (see hit_triangle).
struct RayW {
    uint32_t tri_base;    // kz * n_tris: the first triangle of the copy rotated to (kx, ky, kz)
    bool swap;            // d[kz] < 0
    float Sx, Sy, Sz;
    float ox, oy, oz;     // origin components along kx, ky, kz
};

// kz of a direction (first of equal magnitudes).
__device__ inline int dominant_axis(const float d[3]) {
    int kz = 0;
    if (fabsf(d[1]) > fabsf(d[0])) kz = 1;
    if (fabsf(d[2]) > fabsf(sel3(d[0], d[1], d[2], kz))) kz = 2;
    return kz;
}

__device__ inline RayW ray_setup(const float o[3], const float d[3], int kz, uint32_t n_tris) {
    RayW r;
    const int kx = kz == 2 ? 0 : kz + 1;
    const int ky = kx == 2 ? 0 : kx + 1;
    const float dz = sel3(d[0], d[1], d[2], kz);
    r.tri_base = (uint32_t)kz * n_tris;
    r.swap = dz < 0.0f;
    r.Sx = sel3(d[0], d[1], d[2], kx) / dz;
    r.Sy = sel3(d[0], d[1], d[2], ky) / dz;
    r.Sz = 1.0f / dz;
    r.ox = sel3(o[0], o[1], o[2], kx);
    r.oy = sel3(o[0], o[1], o[2], ky);
    r.oz = sel3(o[0], o[1], o[2], kz);
    return r;
}

// Watertight test against triangle (v0, v1, v2), whose coordinates come
// rotated to the ray's (kx, ky, kz) (the triangle array holds one copy per
// kz).  On a hit with t > 0 returns true with t and front (det > 0 in the
// test's own axis order: the normal cross(v1-v0, v2-v0) faces against the
// ray).
//
// The test proper swaps kx and ky when d[kz] < 0.  That swap exchanges the
// x and y terms, so it turns every edge function into the same two
// products subtracted the other way round; rounding to nearest is symmetric,
// so each of U, V, W, det and T comes out exactly negated, or zero in both
// orders.  A zero edge function is neither negative nor positive to the sign
// test, and a zero det or T (t = 0) is rejected in both orders.  t = T / det
// is then the same number, and only the sign of det, the front flag, flips.
__device__ inline bool hit_triangle(const RayW& r, const float4& v0, const float4& v1, const float4& v2,
                                    float& t_out, bool& front) {
    const float Akx = v0.x - r.ox;
    const float Aky = v0.y - r.oy;
    const float Akz = v0.z - r.oz;
    const float Bkx = v1.x - r.ox;
    const float Bky = v1.y - r.oy;
    const float Bkz = v1.z - r.oz;
    const float Ckx = v2.x - r.ox;
    const float Cky = v2.y - r.oy;
    const float Ckz = v2.z - r.oz;
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
    front = (det > 0.0f) != r.swap;
    return true;
}

typedef __attribute__((address_space(3))) int32_t LdsI32;

struct Hit {
    float t;
    int32_t id;        // original triangle index, INT_MAX when none
    uint32_t slot;     // packed triangle index
    bool front;
};

// Per-lane traversal stack: the newest entries live in LDS (column
// threadIdx.x of the workgroup's STACK x BLOCK stack area, LDS entry i at
// lds[i * BLOCK]), older ones in the lane's global overflow area (entry j at
// spill[j * stride]).  A push that would not fit moves the oldest STACK / 2
// LDS entries to the overflow area and the others down; a pop with no LDS
// entry takes the newest overflow entry directly.  The order of the entries
// is that of one plain stack, and LDS addresses are linear in the stack
// pointer: one address per push or pop, the pushed entries at constant
// offsets from it.
template <int STACK, int BLOCK>
struct StackT {
    static_assert(STACK / 2 >= 3, "moving half the LDS entries leaves room for three pushes");
    static constexpr uint32_t kMove = STACK / 2;
    int32_t* lds;       // &stack_area[tid]
    int32_t* spill;     // &spill[gtid]
    uint32_t stride;
    uint32_t sp;        // entries in LDS
    uint32_t ns;        // entries in the overflow area (all older than those in LDS)

    // Push np (1..3) entries, e0 deepest, with one check for room: three LDS
    // slots are written whatever np is (those above the new top are unused).
    // n_spill counts the entries moved to the global area.
    __device__ inline void push_up_to_3(int32_t e0, int32_t e1, int32_t e2, uint32_t np, uint32_t& n_spill) {
        LdsI32* l = (LdsI32*)lds;
        if (sp + 3u > (uint32_t)STACK) {
#pragma unroll
            for (uint32_t i = 0; i < kMove; ++i) spill[(size_t)(ns + i) * stride] = l[i * BLOCK];
#pragma unroll
            for (uint32_t i = kMove; i < (uint32_t)STACK; ++i)
                if (i < sp) l[(i - kMove) * BLOCK] = l[i * BLOCK];
            ns += kMove;
            sp -= kMove;
            n_spill += kMove;
        }
        LdsI32* top = l + sp * BLOCK;
        top[0] = e0;
        top[BLOCK] = e1;
        top[2 * BLOCK] = e2;
        sp += np;
    }
    __device__ inline int32_t pop() {
        if (sp != 0u) {
            --sp;
            return ((LdsI32*)lds)[sp * BLOCK];
        }
        if (ns == 0u) return -1;
        --ns;
        return spill[(size_t)ns * stride];
    }
};

// Box tests never decide a result, they only prune, so they are built to
// never reject a box that holds the closest hit of the watertight test:
//  - the watertight test accepts rays passing within about 4 ulp of
//    (|v| + |o|) of a triangle, so every box is widened by
//    2^-18 (R + max|o|) on each side (R: largest |coordinate| in the scene),
//    folded into one origin per slab side;
//  - the overlap test tmin <= tmax needs no slack: a slab's entry and exit
//    are computed with a few ulp of (R + max|o|) |inv| of rounding (the
//    reciprocal within 1 ulp, one rounding per product and fused
//    multiply-add), far below the widening of 2^-18 (R + max|o|) |inv| they
//    move each plane by, so a ray through the exact box at t gets every
//    computed entry below t and every exit above it;
//  - the test against the best hit so far uses only the slab of the ray's
//    dominant axis kz: the watertight t is a weighted mean of the vertices'
//    kz distances, so it is never below that slab's entry, whatever the ray's
//    angle to the triangle (the full box entry is not such a bound for
//    grazing rays); the best hit is widened by a relative 2^-16 there, which
//    covers the rounding of both sides;
//  - zero direction components use a large finite reciprocal (no inf * 0).
//
// The traversal state of one ray lives in registers (plus its stack), so a
// lane can advance its ray one step at a time and take a new ray as soon as
// the current one is finished.
using Stack = StackT<kStack, kBlock>;   // the stack of the per-pass and single-step kernels

struct Trav {
    RayW rw;
    // Box test constants per axis, in the order kx, ky, kz of the watertight
    // test, so that the dominant axis is always the third.  For each axis the
    // ray enters a slab through the plane facing it (lo when the direction
    // component is positive, hi otherwise) and leaves through the other, so
    // the lane loads the entry and exit planes directly and needs no min/max
    // per slab.
    float inv[3];           // reciprocal direction component
    float ent[3];           // (o -/+ pad) * inv for the entry plane (lo: o + pad, hi: o - pad)
    float ext[3];           // the same for the exit plane
    uint32_t off[3];        // byte offset of the entry plane in a node: 32 * axis + 16 * (inv < 0);
                            // the exit plane is at off ^ 16
    int32_t node;           // >= 0 inner node, other negative: leaf link, -1: finished
    uint32_t budget;
    float lim;              // h.t * kSlack
    Hit h;
};

template <class Stack>
__device__ inline void trav_init(Trav& tv, const DevScene& sc, const float o[3], const float d[3], Stack& st) {
    const int kz = dominant_axis(d);
    tv.rw = ray_setup(o, d, kz, sc.n_tris);
    float inv[3];
#pragma unroll
    // The reciprocals only prune: the hardware reciprocal (within 1 ulp) is
    // far inside the box widening, so no correctly rounded division here.
    for (int a = 0; a < 3; ++a)
        inv[a] = fabsf(d[a]) > 1e-30f ? __builtin_amdgcn_rcpf(d[a]) : copysignf(1e30f, d[a]);
    // A plane at coordinate c is reached at t = c * inv - (o -/+ pad) * inv,
    // one fused multiply-add per plane.  Its rounding (a few ulp of |o * inv|)
    // is far inside the 2^-18 (R + max|o|) widening, so the bounds stay safe.
    // Rounding is monotonic, so the entry plane's t is never above the exit
    // plane's: the same values a min/max over the two planes would give.
    const float pad = (sc.radius + fmaxf(fmaxf(fabsf(o[0]), fabsf(o[1])), fabsf(o[2]))) * 3.814697265625e-6f;
    const int ax[3] = {kz == 2 ? 0 : kz + 1, kz == 0 ? 2 : kz - 1, kz};   // kx, ky, kz
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float iv = sel3(inv[0], inv[1], inv[2], ax[j]);
        const float oa = sel3(o[0], o[1], o[2], ax[j]);
        const float lo_term = (oa + pad) * iv;   // against lo planes
        const float hi_term = (oa - pad) * iv;   // against hi planes
        const bool neg = iv < 0.0f;
        tv.inv[j] = iv;
        tv.ent[j] = neg ? hi_term : lo_term;
        tv.ext[j] = neg ? lo_term : hi_term;
        tv.off[j] = 32u * (uint32_t)ax[j] + (neg ? 16u : 0u);
    }
    tv.node = sc.n_nodes > 0 ? 0 : -1;
    // Every step of a ray enters a node or a leaf, each at most once per ray
    // (a wide node has at most 4 children); the bound on steps
    // (5 n_nodes + 16 unless a test lowers it) only guarantees termination
    // should the tree ever be malformed.
    tv.budget = sc.step_budget;
    tv.h.t = INFINITY;
    tv.lim = INFINITY;
    tv.h.id = INT_MAX;
    tv.h.slot = 0;
    tv.h.front = false;
    st.sp = 0;
    st.ns = 0;
}

// Traversal counters of the instrumented kernels (dead code otherwise).
struct TravCount {
    uint32_t nodes = 0;   // inner nodes visited
    uint32_t tris = 0;    // triangles tested
    uint32_t lds = 0;     // inner nodes read from the LDS copy of the top levels
    uint32_t spill = 0;   // stack entries moved to the global overflow area
};

__device__ inline float lane_of(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

__device__ inline void order2(uint32_t& ka, int32_t& va, uint32_t& kb, int32_t& vb) {
    const bool s = kb < ka;
    const uint32_t k0 = s ? kb : ka, k1 = s ? ka : kb;
    const int32_t v0 = s ? vb : va, v1 = s ? va : vb;
    ka = k0; kb = k1; va = v0; vb = v1;
}

// Visit one 4-wide node: test the four child boxes (same conservative rules
// as above), continue with the nearest hit child and push the other hit
// children farthest first, or pop when none is hit.  Node layout (8 float4,
// 128 bytes): lo.x, hi.x, lo.y, hi.y, lo.z, hi.z of children 0..3, then their
// links.  The first sc.top_count nodes, when a kernel stages them, sit in LDS
// from address 0 of the workgroup's LDS in the same layout, so one set of
// byte offsets addresses a node in either place.
typedef float V4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) V4 LdsV4;

__device__ inline float4 f4(V4 v) { return make_float4(v.x, v.y, v.z, v.w); }

// The 16 bytes at LDS byte address `byte` of the workgroup.
__device__ inline float4 lds_f4(uint32_t byte) { return f4(*(const LdsV4*)(size_t)byte); }

template <bool STATS, class Stack>
__device__ inline int32_t visit_inner4(Trav& tv, int32_t node, const DevScene& sc, Stack& st, TravCount& cnt) {
    // byte offsets of the entry and exit planes of the three axes (the
    // node array is limited to 4 GB, so offsets fit 32 bits), the same in
    // LDS and in the node array
    const uint32_t base = (uint32_t)node << 7;
    const uint32_t e0 = base + tv.off[0], e1 = base + tv.off[1], e2 = base + tv.off[2];
    const uint32_t f0 = e0 ^ 16u, f1 = e1 ^ 16u, f2 = e2 ^ 16u;
    float4 n0, x0, n1, x1, n2, x2, lk;
    if ((uint32_t)node < sc.top_count) {
        // the top levels, staged in LDS: LDS reads do not use the vector
        // memory address path (the compiler barrier keeps the two paths from
        // being merged into flat loads)
        n0 = lds_f4(e0); x0 = lds_f4(f0);
        n1 = lds_f4(e1); x1 = lds_f4(f1);
        n2 = lds_f4(e2); x2 = lds_f4(f2);
        lk = lds_f4(base + 96u);
        __asm__ volatile("" ::: "memory");
    } else {
        const char* g = (const char*)sc.nodes;
        n0 = *(const float4*)(g + e0); x0 = *(const float4*)(g + f0);
        n1 = *(const float4*)(g + e1); x1 = *(const float4*)(g + f1);
        n2 = *(const float4*)(g + e2); x2 = *(const float4*)(g + f2);
        lk = *(const float4*)(g + base + 96u);
    }
    if (STATS) {
        ++cnt.nodes;
        if ((uint32_t)node < sc.top_count) ++cnt.lds;
    }
    const float lim = tv.lim;
    uint32_t key[4];    // entry distance bits of hit children (t >= 0), all ones for the rest
    int32_t val[4];
    bool any = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float a0 = __builtin_fmaf(lane_of(n0, i), tv.inv[0], -tv.ent[0]);
        const float b0 = __builtin_fmaf(lane_of(x0, i), tv.inv[0], -tv.ext[0]);
        const float a1 = __builtin_fmaf(lane_of(n1, i), tv.inv[1], -tv.ent[1]);
        const float b1 = __builtin_fmaf(lane_of(x1, i), tv.inv[1], -tv.ext[1]);
        const float a2 = __builtin_fmaf(lane_of(n2, i), tv.inv[2], -tv.ent[2]);
        const float b2 = __builtin_fmaf(lane_of(x2, i), tv.inv[2], -tv.ext[2]);
        const float tmin = fmaxf(fmaxf(a0, a1), fmaxf(a2, 0.0f));
        const float tmax = fminf(fminf(b0, b1), b2);
        const uint32_t link = __float_as_uint(lane_of(lk, i));
        // a2 is the entry of the dominant axis's slab (see above).  An unused
        // slot has NaN planes: tmax and a2 are NaN and both tests fail (its
        // link, a one-triangle leaf, is never followed)
        const bool hit = tmin <= tmax && a2 <= lim;
        key[i] = hit ? __float_as_uint(tmin) : 0xFFFFFFFFu;   // a hit's tmin is never NaN
        val[i] = (int32_t)link;
        any = any || hit;
    }
    // a full sorting network: hits ascending, then the misses, so that the
    // hit children are val[0 .. n) for the n keys that are not all ones
    order2(key[0], val[0], key[1], val[1]);
    order2(key[2], val[2], key[3], val[3]);
    order2(key[0], val[0], key[2], val[2]);
    order2(key[1], val[1], key[3], val[3]);
    order2(key[1], val[1], key[2], val[2]);
    if (!any) return st.pop();
    if (key[1] != 0xFFFFFFFFu) {   // two hits or more: push all but the nearest
        const bool h2 = key[2] != 0xFFFFFFFFu, h3 = key[3] != 0xFFFFFFFFu;
        const int32_t e0 = h3 ? val[3] : (h2 ? val[2] : val[1]);
        const int32_t e1 = h3 ? val[2] : val[1];
        st.push_up_to_3(e0, e1, val[1], 1u + (h2 ? 1u : 0u) + (h3 ? 1u : 0u), cnt.spill);
    }
    return val[0];
}

// Test the triangles of leaf `link` against the ray, keeping the closest hit.
template <bool STATS>
__device__ inline void visit_leaf(Trav& tv, int32_t link, const DevScene& sc, TravCount& cnt) {
    const int32_t node = link;
    // leaf: triangles [first, first + count)
    const uint32_t first = ((uint32_t)node >> 3) & 0x0FFFFFFFu;
    const uint32_t count = ((uint32_t)node & 7u) + 1u;
    for (uint32_t j = 0; j < count; ++j) {
        const float4* tp = sc.tris + 3 * (size_t)(tv.rw.tri_base + first + j);
        const float4 v0 = tp[0], v1 = tp[1], v2 = tp[2];
        if (STATS) ++cnt.tris;
        float t;
        bool front;
        if (hit_triangle(tv.rw, v0, v1, v2, t, front)) {
            const int32_t id = __float_as_int(v0.w);
            if (t < tv.h.t || (t == tv.h.t && id < tv.h.id)) {
                tv.h.t = t;
                tv.lim = t * kSlack;
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
// step, so the wave's leaf tests run together.  The descent ends early, after
// at least one node per searching lane, once no more than `exit_lanes` lanes
// are still looking for a leaf and at least as many hold one: a few deep
// searches would otherwise keep the waiting lanes idle.  Those lanes resume
// where they were next step.  (Without the second condition, a sparse wave --
// late in a launch, when few of its lanes still carry a ray -- stopped after
// every node; with it, the terrain frame got 2.6% faster at the same
// threshold and 5% faster at the new default of 16.)
constexpr int kMaxDescent = 256;   // node visits of one step (the step ends, the ray goes on)

template <bool STATS, class Stack>
__device__ inline void trav_step(Trav& tv, const DevScene& sc, Stack& st, uint32_t exit_lanes, TravCount& cnt) {
    if (--tv.budget == 0u) {
        // only a malformed tree gets here: end the ray and raise the scene's
        // error flag, which the host reports as an internal error
        __hip_atomic_store(sc.err_flag, kErrStepBudget, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        tv.node = -1;
        return;
    }
    int32_t node = tv.node;
    int32_t leaf = -1;
    for (int it = 0; it < kMaxDescent; ++it) {
        if (node < -1 && leaf == -1) { leaf = node; node = st.pop(); }
        // (the ballot of each compare alone maps onto one VALU compare; a
        // ballot of their conjunction was materialised through a select)
        const unsigned long long holding = wave_ballot(leaf != -1);
        const unsigned long long searching = ~holding & wave_ballot(node >= 0);
        if (searching == 0ull) break;
        // only a few lanes still looking for a leaf: let the others test
        // theirs (every searching lane has advanced one node this step)
        const uint32_t n_search = popc_u32(searching);
        if (it > 0 && n_search <= exit_lanes && popc_u32(holding) >= n_search) break;
        if (node >= 0) node = visit_inner4<STATS>(tv, node, sc, st, cnt);
    }
    if (leaf != -1) visit_leaf<STATS>(tv, leaf, sc, cnt);
    tv.node = node;
}

}  // namespace
}  // namespace rcp
