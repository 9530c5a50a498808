// Device BVH build for the renderer's scenes.
//
// The paper does not say how its ray tracer built its acceleration structure
// (Section 6 used a GPU ray-tracing engine), so this is a standard GPU build:
//   1. per-triangle boxes and the centroid bounds (wave reductions + atomics)
//   2. 63-bit Morton codes of the box centres (21 bits per axis, one scale)
//   3. stable LSD radix sort of (code, triangle) pairs
//   4. binary radix tree over the sorted codes, one thread per inner node
//      (Karras, "Maximizing Parallelism in the Construction of BVHs, Octrees,
//      and k-d Trees", HPG 2012), duplicate codes split by index
//      (or, by default, PLOC: agglomerative clustering of Morton neighbours)
//   5. the 4-wide tree the traversal uses, 128-byte nodes, by default from
//      an SAH-optimal collapse of the binary tree: a bottom-up dynamic
//      programme over the subtrees (one launch per tree level), then
//      emission level by level.  The greedy alternative: a bottom-up refit that collapses
//      subtrees into leaves (<= max_leaf triangles) where the binary SAH says
//      so, packing of the binary tree in depth-first order, and wide nodes
//      that open their children of largest area
//   6. packing of 48-byte triangles, a per-triangle table of the two shaded
//      colours and the unit normals.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rcp_internal.hpp"

namespace rcp {
namespace {

constexpr int kB = 256;

// Entering a leaf costs the traversal a step of its own (the lane holds the
// leaf, and its triangles are tested after the descent), so the cost model
// charges a leaf kLeafEntry * c_trav on top of its triangle tests (the SAH
// collapse optimises it, and the reported SAH cost includes it).  Measured
// on the terrain frames against the greedy collapse: 0 (plain SAH) split
// two-triangle cells into one-triangle leaves and was 4% slower, 1 was 3%
// slower, 2 equal at 1M triangles and 1% faster at 16M (20% fewer nodes), 3
// 4% slower again.
constexpr float kLeafEntry = 2.0f;

__device__ inline uint32_t f2o(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __host__ inline float o2f(uint32_t u) {
    uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

__device__ inline float3 ld3(const float* p, uint32_t i) {
    return make_float3(p[3 * (size_t)i], p[3 * (size_t)i + 1], p[3 * (size_t)i + 2]);
}

__device__ inline float half_area(float3 lo, float3 hi) {
    float dx = fmaxf(hi.x - lo.x, 0.0f), dy = fmaxf(hi.y - lo.y, 0.0f), dz = fmaxf(hi.z - lo.z, 0.0f);
    return dx * dy + dy * dz + dz * dx;
}

__device__ inline float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// bounds[0..2] = ordered min of centres, bounds[3..5] = ordered max.
__global__ void k_init_bounds(uint32_t* bounds) {
    if (threadIdx.x < 3) bounds[threadIdx.x] = 0xFFFFFFFFu;
    else if (threadIdx.x < 6) bounds[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(kB) void k_tri_prep(const float* __restrict__ verts, const uint32_t* __restrict__ idx,
                                                  uint32_t n, float4* __restrict__ tlo, float4* __restrict__ thi,
                                                  uint32_t* __restrict__ bounds) {
    // grid-stride over the triangles; the centroid bounds are reduced per
    // thread, per wave and per workgroup before six atomics per workgroup
    float3 cmin = make_float3(INFINITY, INFINITY, INFINITY);
    float3 cmax = make_float3(-INFINITY, -INFINITY, -INFINITY);
    for (uint32_t i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB) {
        float3 a = ld3(verts, idx[3 * (size_t)i]);
        float3 b = ld3(verts, idx[3 * (size_t)i + 1]);
        float3 d = ld3(verts, idx[3 * (size_t)i + 2]);
        float3 lo = make_float3(fminf(fminf(a.x, b.x), d.x), fminf(fminf(a.y, b.y), d.y), fminf(fminf(a.z, b.z), d.z));
        float3 hi = make_float3(fmaxf(fmaxf(a.x, b.x), d.x), fmaxf(fmaxf(a.y, b.y), d.y), fmaxf(fmaxf(a.z, b.z), d.z));
        tlo[i] = make_float4(lo.x, lo.y, lo.z, 0.0f);
        thi[i] = make_float4(hi.x, hi.y, hi.z, 0.0f);
        const float3 c = make_float3(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z));
        cmin = make_float3(fminf(cmin.x, c.x), fminf(cmin.y, c.y), fminf(cmin.z, c.z));
        cmax = make_float3(fmaxf(cmax.x, c.x), fmaxf(cmax.y, c.y), fmaxf(cmax.z, c.z));
    }
    __shared__ float red[kB / 64][6];
    const int wave = threadIdx.x >> 6;
    const float r[6] = {wave_min(cmin.x), wave_min(cmin.y), wave_min(cmin.z),
                        wave_max(cmax.x), wave_max(cmax.y), wave_max(cmax.z)};
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) red[wave][k] = r[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        float v[6];
        for (int k = 0; k < 6; ++k) v[k] = red[0][k];
        for (int w = 1; w < kB / 64; ++w) {
            for (int k = 0; k < 3; ++k) v[k] = fminf(v[k], red[w][k]);
            for (int k = 3; k < 6; ++k) v[k] = fmaxf(v[k], red[w][k]);
        }
        if (v[0] <= v[3]) {
            atomicMin(&bounds[0], f2o(v[0])); atomicMin(&bounds[1], f2o(v[1])); atomicMin(&bounds[2], f2o(v[2]));
            atomicMax(&bounds[3], f2o(v[3])); atomicMax(&bounds[4], f2o(v[4])); atomicMax(&bounds[5], f2o(v[5]));
        }
    }
}

__device__ inline uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint32_t quant21(float v, float lo, float scale) {
    float q = (v - lo) * scale;
    q = fminf(fmaxf(q, 0.0f), 2097151.0f);
    return (uint32_t)q;
}

__global__ __launch_bounds__(kB) void k_morton(const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                                uint32_t n, const uint32_t* __restrict__ bounds,
                                                uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    // One scale for all axes (a cube around the centroid bounds): the code's
    // bit order then splits the longest extents first, instead of giving a
    // thin axis (a terrain's height) as many top-level splits as the others.
    float lo[3], ext = 0.0f;
    for (int c = 0; c < 3; ++c) {
        lo[c] = o2f(bounds[c]);
        ext = fmaxf(ext, o2f(bounds[3 + c]) - lo[c]);
    }
    const float scale = ext > 0.0f ? 2097152.0f / ext : 0.0f;
    float4 a = tlo[i], b = thi[i];
    float cx = 0.5f * (a.x + b.x), cy = 0.5f * (a.y + b.y), cz = 0.5f * (a.z + b.z);
    uint32_t qx = quant21(cx, lo[0], scale);
    uint32_t qy = quant21(cy, lo[1], scale);
    uint32_t qz = quant21(cz, lo[2], scale);
    keys[i] = (spread21(qx) << 2) | (spread21(qy) << 1) | spread21(qz);
    vals[i] = i;
}

// Length of the common prefix of sorted keys i and j, extended by the index
// bits when the keys are equal; -1 outside [0, n).
__device__ inline int prefix_len(const uint64_t* __restrict__ k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((uint32_t)i ^ (uint32_t)j);
    return __clzll(a ^ b);
}

// Children: >= 0 inner node, kLeafBit | j for sorted triangle j.
__global__ __launch_bounds__(kB) void k_radix_tree(const uint64_t* __restrict__ keys, int n,
                                                    int32_t* __restrict__ left, int32_t* __restrict__ right,
                                                    int32_t* __restrict__ parent, int32_t* __restrict__ rfirst,
                                                    int32_t* __restrict__ rlast) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (prefix_len(keys, n, i, i + 1) - prefix_len(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix_len(keys, n, i, i - d);
    int lmax = 2;
    while (prefix_len(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(keys, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + (d < 0 ? -1 : 0);
    const int lo = min(i, j), hi = max(i, j);
    int32_t lc = (lo == gamma) ? (int32_t)(kLeafBit | (uint32_t)gamma) : gamma;
    int32_t rc = (hi == gamma + 1) ? (int32_t)(kLeafBit | (uint32_t)(gamma + 1)) : gamma + 1;
    left[i] = lc;
    right[i] = rc;
    rfirst[i] = lo;
    rlast[i] = hi;
    // parents: inner nodes at [0, n-1), leaves at [n-1, 2n-1)
    parent[lc < 0 ? (n - 1 + gamma) : lc] = i;
    parent[rc < 0 ? (n - 1 + gamma + 1) : rc] = i;
    if (i == 0) parent[0] = -1;
}

// ---------------------------------------------------------------------------
// PLOC: parallel locally-ordered clustering (Meister and Bittner, "Parallel
// Locally-Ordered Clustering for Bounding Volume Hierarchy Construction",
// IEEE TVCG 2018).  Clusters start as the triangles in Morton order.  Each
// round every cluster finds its nearest neighbour among the kPlocRadius
// clusters on each side -- the one whose merged box has the smallest surface
// area --, mutual nearest neighbours merge into a new inner node, and the
// clusters are compacted in order.  Equal areas are ordered by index
// distance, then pairs with an even lower index first, then by the lower
// index: a strict order on pairs, so the globally best pair is always mutual
// and every round merges, and exact duplicates pair off (0,1), (2,3), ...
// Inner nodes are numbered downward from n - 2, so the last merge, the root,
// is node 0.  The tree is then renumbered so that every subtree holds a
// contiguous range of triangles (depth-first leaf order).
// ---------------------------------------------------------------------------
constexpr int kPlocRadius = 16;

__global__ __launch_bounds__(kB) void k_ploc_init(int n, const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                                   const uint32_t* __restrict__ sorted, int32_t* __restrict__ id,
                                                   float4* __restrict__ lo, float4* __restrict__ hi) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    id[i] = (int32_t)(kLeafBit | (uint32_t)i);
    lo[i] = tlo[sorted[i]];
    hi[i] = thi[sorted[i]];
}

__global__ __launch_bounds__(kB) void k_ploc_nn(int m, const float4* __restrict__ lo, const float4* __restrict__ hi,
                                                 int32_t* __restrict__ nn) {
    constexpr int kW = kB + 2 * kPlocRadius;
    __shared__ float s[6][kW];
    const int base = (int)(blockIdx.x * kB) - kPlocRadius;
    for (int t = threadIdx.x; t < kW; t += kB) {
        const int g = base + t;
        if (g >= 0 && g < m) {
            const float4 a = lo[g], b = hi[g];
            s[0][t] = a.x; s[1][t] = a.y; s[2][t] = a.z;
            s[3][t] = b.x; s[4][t] = b.y; s[5][t] = b.z;
        }
    }
    __syncthreads();
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= m) return;
    const int li = threadIdx.x + kPlocRadius;
    float best = INFINITY;
    int bj = -1, bdist = 0, bmin = 0;
    for (int d = -kPlocRadius; d <= kPlocRadius; ++d) {
        const int j = i + d;
        if (d == 0 || j < 0 || j >= m) continue;
        const int lj = li + d;
        const float3 a = make_float3(fminf(s[0][li], s[0][lj]), fminf(s[1][li], s[1][lj]), fminf(s[2][li], s[2][lj]));
        const float3 b = make_float3(fmaxf(s[3][li], s[3][lj]), fmaxf(s[4][li], s[4][lj]), fmaxf(s[5][li], s[5][lj]));
        const float ar = half_area(a, b);
        const int dist = d < 0 ? -d : d;
        const int mn = j < i ? j : i;
        bool take = ar < best;
        if (!take && ar == best) {
            if (dist != bdist) take = dist < bdist;
            else if ((mn & 1) != (bmin & 1)) take = (mn & 1) == 0;
            else take = mn < bmin;
        }
        if (take || bj < 0) { best = ar; bj = j; bdist = dist; bmin = mn; }
    }
    nn[i] = bj;
}

__device__ inline int node_slot(int32_t c, int n) {
    return c < 0 ? n - 1 + (int)((uint32_t)c & ~kLeafBit) : c;
}

__global__ __launch_bounds__(kB) void k_ploc_merge(int m, int n, const int32_t* __restrict__ nn,
                                                    const int32_t* __restrict__ id, const float4* __restrict__ lo,
                                                    const float4* __restrict__ hi, int32_t* __restrict__ id2,
                                                    float4* __restrict__ lo2, float4* __restrict__ hi2,
                                                    uint32_t* __restrict__ pos, uint32_t* __restrict__ keep,
                                                    int32_t* __restrict__ next_id, int32_t* __restrict__ left,
                                                    int32_t* __restrict__ right, int32_t* __restrict__ parent) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= m) return;
    const int j = nn[i];
    uint32_t k = 1u;
    if (j >= 0 && nn[j] == i) {
        if (i < j) {
            const int32_t node = atomicSub(next_id, 1);
            const int32_t a = id[i], b = id[j];
            left[node] = a;
            right[node] = b;
            parent[node_slot(a, n)] = node;
            parent[node_slot(b, n)] = node;
            const float4 la = lo[i], lb = lo[j], ha = hi[i], hb = hi[j];
            id2[i] = node;
            lo2[i] = make_float4(fminf(la.x, lb.x), fminf(la.y, lb.y), fminf(la.z, lb.z), 0.0f);
            hi2[i] = make_float4(fmaxf(ha.x, hb.x), fmaxf(ha.y, hb.y), fmaxf(ha.z, hb.z), 0.0f);
        } else {
            k = 0u;   // merged into cluster j
        }
    } else {
        id2[i] = id[i];
        lo2[i] = lo[i];
        hi2[i] = hi[i];
    }
    pos[i] = k;
    keep[i] = k;
}

__global__ __launch_bounds__(kB) void k_ploc_compact(int m, const uint32_t* __restrict__ pos,
                                                      const uint32_t* __restrict__ keep,
                                                      const int32_t* __restrict__ id2, const float4* __restrict__ lo2,
                                                      const float4* __restrict__ hi2, int32_t* __restrict__ id,
                                                      float4* __restrict__ lo, float4* __restrict__ hi,
                                                      uint32_t* __restrict__ m_out) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= m) return;
    if (keep[i]) {
        const uint32_t p = pos[i];
        id[p] = id2[i];
        lo[p] = lo2[i];
        hi[p] = hi2[i];
    }
    if (i == m - 1) *m_out = pos[i] + keep[i];
}

// The last rounds of PLOC, once at most kPlocSmall clusters remain, in one
// workgroup: the same neighbour search (the same order of candidates and of
// ties), the same merge rule and the same order-keeping compaction as the
// per-round kernels above, so the tree is the same; the clusters stay in LDS
// and a workgroup barrier stands in for each launch and host read.  Thread i
// holds cluster i.  Ends with the cluster count in *m_out (1 when done; more
// if max_rounds ran out).
constexpr int kPlocSmall = 1024;

__global__ __launch_bounds__(kPlocSmall) void k_ploc_finish(int m, int n, int max_rounds,
                                                             const int32_t* __restrict__ id_in,
                                                             const float4* __restrict__ lo_in,
                                                             const float4* __restrict__ hi_in,
                                                             int32_t* __restrict__ next_id, int32_t* __restrict__ left,
                                                             int32_t* __restrict__ right, int32_t* __restrict__ parent,
                                                             uint32_t* __restrict__ m_out) {
    __shared__ float s[6][kPlocSmall];                 // lo.x, lo.y, lo.z, hi.x, hi.y, hi.z
    __shared__ int32_t s_id[kPlocSmall];
    __shared__ int32_t s_nn[kPlocSmall];
    __shared__ uint32_t s_wave[kPlocSmall / 64];
    const int i = threadIdx.x;
    if (i < m) {
        const float4 a = lo_in[i], b = hi_in[i];
        s[0][i] = a.x; s[1][i] = a.y; s[2][i] = a.z;
        s[3][i] = b.x; s[4][i] = b.y; s[5][i] = b.z;
        s_id[i] = id_in[i];
    }
    __syncthreads();
    for (int round = 0; m > 1 && round < max_rounds; ++round) {   // m is the same in every thread
        // nearest neighbour among kPlocRadius clusters on each side (as k_ploc_nn)
        if (i < m) {
            float best = INFINITY;
            int bj = -1, bdist = 0, bmin = 0;
            for (int d = -kPlocRadius; d <= kPlocRadius; ++d) {
                const int j = i + d;
                if (d == 0 || j < 0 || j >= m) continue;
                const float3 a = make_float3(fminf(s[0][i], s[0][j]), fminf(s[1][i], s[1][j]), fminf(s[2][i], s[2][j]));
                const float3 b = make_float3(fmaxf(s[3][i], s[3][j]), fmaxf(s[4][i], s[4][j]), fmaxf(s[5][i], s[5][j]));
                const float ar = half_area(a, b);
                const int dist = d < 0 ? -d : d;
                const int mn = j < i ? j : i;
                bool take = ar < best;
                if (!take && ar == best) {
                    if (dist != bdist) take = dist < bdist;
                    else if ((mn & 1) != (bmin & 1)) take = (mn & 1) == 0;
                    else take = mn < bmin;
                }
                if (take || bj < 0) { best = ar; bj = j; bdist = dist; bmin = mn; }
            }
            s_nn[i] = bj;
        }
        __syncthreads();
        // merge mutual pairs into the lower slot (as k_ploc_merge)
        bool keep = i < m;
        int32_t nid = 0;
        float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f, b3 = 0.0f, b4 = 0.0f, b5 = 0.0f;
        if (i < m) {
            nid = s_id[i];
            b0 = s[0][i]; b1 = s[1][i]; b2 = s[2][i]; b3 = s[3][i]; b4 = s[4][i]; b5 = s[5][i];
            const int j = s_nn[i];
            if (j >= 0 && s_nn[j] == i) {
                if (i < j) {
                    const int32_t node = atomicSub(next_id, 1);
                    const int32_t ca = s_id[i], cb = s_id[j];
                    left[node] = ca;
                    right[node] = cb;
                    parent[node_slot(ca, n)] = node;
                    parent[node_slot(cb, n)] = node;
                    nid = node;
                    b0 = fminf(b0, s[0][j]); b1 = fminf(b1, s[1][j]); b2 = fminf(b2, s[2][j]);
                    b3 = fmaxf(b3, s[3][j]); b4 = fmaxf(b4, s[4][j]); b5 = fmaxf(b5, s[5][j]);
                } else {
                    keep = false;   // merged into cluster j
                }
            }
        }
        // order-keeping compaction: exclusive prefix count of the kept clusters
        const unsigned long long kb = __builtin_amdgcn_ballot_w64(keep);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(kb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u));
        if ((i & 63) == 0) s_wave[i >> 6] = (uint32_t)__popcll(kb);
        __syncthreads();   // every read of this round's clusters is done
        uint32_t pos = below, total = 0;
        for (int w = 0; w < kPlocSmall / 64; ++w) {
            const uint32_t c = s_wave[w];
            if (w < (i >> 6)) pos += c;
            total += c;
        }
        if (keep) {
            s[0][pos] = b0; s[1][pos] = b1; s[2][pos] = b2; s[3][pos] = b3; s[4][pos] = b4; s[5][pos] = b5;
            s_id[pos] = nid;
        }
        m = (int)total;
        __syncthreads();
    }
    if (i == 0) *m_out = (uint32_t)m;
}

// ---- bottom-up passes -----------------------------------------------------
// A pass computes each inner node from its two children, one launch per tree
// level, deepest first: the inner nodes are sorted by depth, and kernel
// boundaries order the levels, so no fences are needed.  (Walks up from the
// leaves, where the second thread to reach a node computes it, need
// device-scope fences around every arrival counter; on 8 XCDs with their own
// L2s those cost 5-7 ms per pass at 1M triangles, the levels 0.3 ms.)
template <class Body>
__global__ __launch_bounds__(kB) void k_level(const int32_t* __restrict__ ids, uint32_t count, Body body) {
    const uint32_t i = blockIdx.x * kB + threadIdx.x;
    if (i < count) body(ids[i]);
}

// Depth of every inner node (walk up to the root), as a sort key.
__global__ __launch_bounds__(kB) void k_node_depth(int n, const int32_t* __restrict__ parent,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                                    uint32_t* __restrict__ max_depth) {
    const int x = blockIdx.x * kB + threadIdx.x;
    uint32_t d = 0;
    if (x < n - 1) {
        for (int p = parent[x]; p >= 0 && d < (uint32_t)n; p = parent[p]) ++d;
        keys[x] = d;
        ids[x] = (uint32_t)x;
    }
    for (int o = 32; o > 0; o >>= 1) d = max(d, (uint32_t)__shfl_xor((int)d, o));
    if ((threadIdx.x & 63) == 0 && x < n - 1 + 64) atomicMax(max_depth, d);
}

// First position of each depth in the depth-sorted order.
__global__ __launch_bounds__(kB) void k_level_starts(int m, const uint64_t* __restrict__ keys,
                                                      uint32_t* __restrict__ starts) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i < m && (i == 0 || keys[i] != keys[i - 1])) starts[keys[i]] = (uint32_t)i;
}

// Leaves under every inner node.
struct LeafCountBody {
    const int32_t* left;
    const int32_t* right;
    int32_t* cnt;
    __device__ void operator()(int node) const {
        const int32_t l = left[node], r = right[node];
        cnt[node] = (l < 0 ? 1 : cnt[l]) + (r < 0 ? 1 : cnt[r]);
    }
};

__global__ __launch_bounds__(kB) void k_dfs_first(int n, const int32_t* __restrict__ left,
                                                   const int32_t* __restrict__ right, const int32_t* __restrict__ parent,
                                                   const int32_t* __restrict__ cnt, int32_t* __restrict__ first) {
    const int x = blockIdx.x * kB + threadIdx.x;
    if (x >= 2 * n - 1) return;
    int32_t code = x < n - 1 ? x : (int32_t)(kLeafBit | (uint32_t)(x - (n - 1)));
    int node = parent[x];
    int r = 0;
    while (node >= 0) {
        if (right[node] == code) {
            const int32_t l = left[node];
            r += l < 0 ? 1 : cnt[l];
        }
        code = node;
        node = parent[node];
    }
    first[x] = r;
}

// Renumber the triangles in depth-first leaf order: the sorted array, the
// leaves' parents, leaf children, and each inner node's range.
__global__ __launch_bounds__(kB) void k_dfs_renumber(int n, const int32_t* __restrict__ first,
                                                      const int32_t* __restrict__ cnt,
                                                      const uint32_t* __restrict__ sorted_in,
                                                      const int32_t* __restrict__ parent_in,
                                                      uint32_t* __restrict__ sorted_out, int32_t* __restrict__ parent_out,
                                                      int32_t* __restrict__ left, int32_t* __restrict__ right,
                                                      int32_t* __restrict__ rfirst, int32_t* __restrict__ rlast) {
    const int x = blockIdx.x * kB + threadIdx.x;
    if (x >= 2 * n - 1) return;
    if (x >= n - 1) {
        const int p = x - (n - 1), r = first[x];
        sorted_out[r] = sorted_in[p];
        parent_out[n - 1 + r] = parent_in[x];
    } else {
        parent_out[x] = parent_in[x];
        const int32_t l = left[x], rr = right[x];
        if (l < 0) left[x] = (int32_t)(kLeafBit | (uint32_t)first[n - 1 + (int)((uint32_t)l & ~kLeafBit)]);
        if (rr < 0) right[x] = (int32_t)(kLeafBit | (uint32_t)first[n - 1 + (int)((uint32_t)rr & ~kLeafBit)]);
        rfirst[x] = first[x];
        rlast[x] = first[x] + cnt[x] - 1;
    }
}

__global__ void k_set_i32(int32_t* p, int32_t v) {
    if (threadIdx.x == 0) *p = v;
}

struct NodeData {
    float4* lo;        // box lo, w unused
    float4* hi;
    float* cost;
    int32_t* n_inner;  // emitted inner nodes in the subtree (0 when collapsed)
    int32_t* collapse;
};

__device__ inline void child_info(int32_t c, const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                  const uint32_t* __restrict__ sorted, NodeData nd, float c_isect,
                                  float3& lo, float3& hi, float& cost, int& ninner) {
    if (c < 0) {
        uint32_t t = sorted[(uint32_t)c & ~kLeafBit];
        float4 a = tlo[t], b = thi[t];
        lo = make_float3(a.x, a.y, a.z);
        hi = make_float3(b.x, b.y, b.z);
        cost = c_isect * half_area(lo, hi);
        ninner = 0;
    } else {
        // computed earlier in the pass (a deeper level, or the sibling's walk)
        float4 a = nd.lo[c];
        float4 b = nd.hi[c];
        lo = make_float3(a.x, a.y, a.z);
        hi = make_float3(b.x, b.y, b.z);
        cost = nd.cost[c];
        ninner = nd.n_inner[c];
    }
}

struct RefitBody {
    const int32_t* left;
    const int32_t* right;
    const int32_t* rfirst;
    const int32_t* rlast;
    const float4* tlo;
    const float4* thi;
    const uint32_t* sorted;
    NodeData nd;
    int max_leaf;
    float c_trav, c_isect;
    __device__ void operator()(int node) const {
        float3 llo, lhi, rlo, rhi;
        float cl, cr;
        int nl, nr;
        child_info(left[node], tlo, thi, sorted, nd, c_isect, llo, lhi, cl, nl);
        child_info(right[node], tlo, thi, sorted, nd, c_isect, rlo, rhi, cr, nr);
        float3 lo = make_float3(fminf(llo.x, rlo.x), fminf(llo.y, rlo.y), fminf(llo.z, rlo.z));
        float3 hi = make_float3(fmaxf(lhi.x, rhi.x), fmaxf(lhi.y, rhi.y), fmaxf(lhi.z, rhi.z));
        const int cnt = rlast[node] - rfirst[node] + 1;
        const float a = half_area(lo, hi);
        const float leaf_cost = c_isect * (float)cnt * a;
        const float split_cost = c_trav * a + cl + cr;
        const bool col = cnt <= max_leaf && leaf_cost <= split_cost;
        nd.lo[node] = make_float4(lo.x, lo.y, lo.z, 0.0f);
        nd.hi[node] = make_float4(hi.x, hi.y, hi.z, 0.0f);
        nd.cost[node] = col ? leaf_cost : split_cost;
        nd.n_inner[node] = col ? 0 : 1 + nl + nr;
        nd.collapse[node] = col ? 1 : 0;
    }
};

// Summary read back by the host: [0] collapse(root), [1] n_inner(root),
// [2] top count, [3] max depth of inner nodes; floats follow.
struct Summary {
    int32_t root_collapsed;
    int32_t n_inner;
    float root_cost;
    float root_area;
    float bbox[6];
};

__global__ void k_summary_root(NodeData nd, Summary* sm) {
    sm->root_collapsed = nd.collapse[0];
    sm->n_inner = nd.n_inner[0];
    sm->root_cost = nd.cost[0];
    float4 a = nd.lo[0], b = nd.hi[0];
    sm->root_area = half_area(make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z));
    sm->bbox[0] = a.x; sm->bbox[1] = a.y; sm->bbox[2] = a.z;
    sm->bbox[3] = b.x; sm->bbox[4] = b.y; sm->bbox[5] = b.z;
}

// Depth-first rank (among emitted inner nodes) of each inner node, by walking
// up to the root: the binary nodes are packed in depth-first order.  Nodes
// inside a collapsed subtree get -1.
__global__ __launch_bounds__(kB) void k_layout_walk(int n, const int32_t* __restrict__ left,
                                                     const int32_t* __restrict__ parent, NodeData nd,
                                                     int32_t* __restrict__ newidx) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n - 1) return;
    newidx[i] = -1;
    if (nd.collapse[i]) return;
    int x = i, idx = 0;
    while (x != 0) {
        const int p = parent[x];
        if (nd.collapse[p]) return;
        const int32_t lp = left[p];
        idx += 1;
        if (lp != x && lp >= 0) idx += nd.n_inner[lp];
        x = p;
    }
    newidx[i] = idx;
}

__device__ inline float pad_lo(float v) { return v - (fabsf(v) * 4.8e-7f + 1e-30f); }
__device__ inline float pad_hi(float v) { return v + (fabsf(v) * 4.8e-7f + 1e-30f); }

__global__ __launch_bounds__(kB) void k_pack_nodes(int n, const int32_t* __restrict__ left,
                                                    const int32_t* __restrict__ right,
                                                    const int32_t* __restrict__ rfirst,
                                                    const int32_t* __restrict__ rlast, const float4* __restrict__ tlo,
                                                    const float4* __restrict__ thi, const uint32_t* __restrict__ sorted,
                                                    NodeData nd, const int32_t* __restrict__ newidx,
                                                    float4* __restrict__ nodes) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n - 1) return;
    const int ni = newidx[i];
    if (ni < 0) return;
    float3 lo[2], hi[2];
    uint32_t link[2];
    const int32_t ch[2] = {left[i], right[i]};
    for (int c = 0; c < 2; ++c) {
        const int32_t x = ch[c];
        if (x < 0) {
            const uint32_t j = (uint32_t)x & ~kLeafBit;
            const uint32_t t = sorted[j];
            float4 a = tlo[t], b = thi[t];
            lo[c] = make_float3(a.x, a.y, a.z);
            hi[c] = make_float3(b.x, b.y, b.z);
            link[c] = leaf_link(j, 1);
        } else {
            float4 a = nd.lo[x], b = nd.hi[x];
            lo[c] = make_float3(a.x, a.y, a.z);
            hi[c] = make_float3(b.x, b.y, b.z);
            if (nd.collapse[x]) link[c] = leaf_link((uint32_t)rfirst[x], (uint32_t)(rlast[x] - rfirst[x] + 1));
            else link[c] = (uint32_t)newidx[x];
        }
    }
    float4* o = nodes + 4 * (size_t)ni;
    o[0] = make_float4(pad_lo(lo[0].x), pad_hi(hi[0].x), pad_lo(lo[0].y), pad_hi(hi[0].y));
    o[1] = make_float4(pad_lo(lo[1].x), pad_hi(hi[1].x), pad_lo(lo[1].y), pad_hi(hi[1].y));
    o[2] = make_float4(pad_lo(lo[0].z), pad_hi(hi[0].z), pad_lo(lo[1].z), pad_hi(hi[1].z));
    o[3] = make_float4(__uint_as_float(link[0]), __uint_as_float(link[1]), 0.0f, 0.0f);
}

// Occupancy grid of the scene box: the cell of each triangle's centroid is
// set.  Most triangles find their cell already set, so the word is read
// first and only a clear bit takes an atomic.
__global__ void k_occupancy(const float* __restrict__ verts, const uint32_t* __restrict__ idx, uint32_t n,
                            OccGrid g, uint32_t* bits) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        int q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float c = (verts[3 * (size_t)idx[3 * (size_t)t] + a] + verts[3 * (size_t)idx[3 * (size_t)t + 1] + a] +
                             verts[3 * (size_t)idx[3 * (size_t)t + 2] + a]) * (1.0f / 3.0f);
            const int v = (int)floorf((c - g.lo[a]) / g.cell[a]);
            q[a] = v < 0 ? 0 : (v >= g.n[a] ? g.n[a] - 1 : v);
        }
        const uint32_t cell = (uint32_t)((q[2] * g.n[1] + q[1]) * g.n[0] + q[0]);
        const uint32_t m = 1u << (cell & 31u);
        if (!(__hip_atomic_load(&bits[cell >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & m))
            atomicOr(&bits[cell >> 5], m);
    }
}

// Whole scene in one leaf (n <= max_leaf): a root whose two children are the
// same leaf; visiting it twice cannot change the closest hit.
__global__ void k_pack_single(int n, const float4* __restrict__ tlo, const float4* __restrict__ thi,
                              float4* __restrict__ nodes) {
    float3 lo = make_float3(INFINITY, INFINITY, INFINITY), hi = make_float3(-INFINITY, -INFINITY, -INFINITY);
    for (int t = 0; t < n; ++t) {
        float4 a = tlo[t], b = thi[t];
        lo = make_float3(fminf(lo.x, a.x), fminf(lo.y, a.y), fminf(lo.z, a.z));
        hi = make_float3(fmaxf(hi.x, b.x), fmaxf(hi.y, b.y), fmaxf(hi.z, b.z));
    }
    const uint32_t link = leaf_link(0, (uint32_t)n);
    nodes[0] = make_float4(pad_lo(lo.x), pad_hi(hi.x), pad_lo(lo.y), pad_hi(hi.y));
    nodes[1] = nodes[0];
    nodes[2] = make_float4(pad_lo(lo.z), pad_hi(hi.z), pad_lo(lo.z), pad_hi(hi.z));
    nodes[3] = make_float4(__uint_as_float(link), __uint_as_float(link), 0.0f, 0.0f);
}

// ---------------------------------------------------------------------------
// 4-wide nodes from the packed binary tree.  A wide node starts from one
// binary node's two children and repeatedly replaces the inner child with the
// largest box surface area by its two children, until it has four children
// or only leaves.  Boxes are copied from the binary nodes (already widened),
// so the wide tree prunes exactly as conservatively.  Built level by level:
// the nodes of one level are slots [begin, end), each records the binary
// node it expands in src[], and its inner children get slots of the next
// level from one counter.
// ---------------------------------------------------------------------------
// Statistics of the emitted wide tree, accumulated exactly: leaf links, the
// SAH cost relative to the root box in 2^-32 fixed point, and the leaves by
// their triangle count (hist[c - 1] leaves of c triangles).
struct WideStats {
    unsigned long long leaves;
    unsigned long long sah_fx;
    unsigned long long hist[8];
};

// leaf_sizes: the node's leaves by size in 4-bit fields (field c counts the
// leaves of c + 1 triangles; a node has at most 4).  Every atomic has the
// same address in all lanes, so the compiler sums each over the wave first:
// one memory atomic per wave and counter.
__device__ inline void wide_stat(WideStats* ws, float node_area, float leaf_cost, uint32_t n_leaves,
                                 uint32_t leaf_sizes, float c_trav, float inv_root_area) {
    const float rel = (c_trav * node_area + leaf_cost) * inv_root_area;
    atomicAdd(&ws->sah_fx, (unsigned long long)((double)rel * 4294967296.0 + 0.5));
    if (n_leaves) atomicAdd(&ws->leaves, (unsigned long long)n_leaves);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t v = (leaf_sizes >> (4 * c)) & 15u;
        if (v) atomicAdd(&ws->hist[c], (unsigned long long)v);
    }
}

struct WideCand {
    float lo[3], hi[3];
    uint32_t link;
    float area;
};

__device__ inline float half_area(const WideCand& c) {
    const float dx = c.hi[0] - c.lo[0], dy = c.hi[1] - c.lo[1], dz = c.hi[2] - c.lo[2];
    return dx * dy + dy * dz + dz * dx;
}

__device__ inline void wide_children(const float4* __restrict__ n2, uint32_t node, WideCand& a, WideCand& b) {
    const float4* p = n2 + 4 * (size_t)node;
    const float4 c0 = p[0], c1 = p[1], z = p[2], l = p[3];
    a.lo[0] = c0.x; a.hi[0] = c0.y; a.lo[1] = c0.z; a.hi[1] = c0.w; a.lo[2] = z.x; a.hi[2] = z.y;
    b.lo[0] = c1.x; b.hi[0] = c1.y; b.lo[1] = c1.z; b.hi[1] = c1.w; b.lo[2] = z.z; b.hi[2] = z.w;
    a.link = __float_as_uint(l.x);
    b.link = __float_as_uint(l.y);
    a.area = half_area(a);
    b.area = half_area(b);
}

__global__ __launch_bounds__(kB) void k_collapse4(const float4* __restrict__ n2, uint32_t begin, uint32_t end,
                                                   uint32_t* __restrict__ src, uint32_t* __restrict__ counter,
                                                   float4* __restrict__ n4, WideStats* stats, float c_trav,
                                                   float c_isect, float inv_root_area) {
    const uint32_t slot = begin + blockIdx.x * kB + threadIdx.x;
    if (slot >= end) return;
    WideCand c[4];
    int m = 2;
    wide_children(n2, src[slot], c[0], c[1]);
    while (m < 4) {
        int best = -1;
        float best_area = -1.0f;
        for (int i = 0; i < m; ++i)
            if (!(c[i].link & kLeafBit) && c[i].area > best_area) { best = i; best_area = c[i].area; }
        if (best < 0) break;
        WideCand a, b;
        wide_children(n2, c[best].link, a, b);
        c[best] = a;
        c[m++] = b;
    }
    int n_inner = 0;
    for (int i = 0; i < m; ++i) n_inner += (c[i].link & kLeafBit) ? 0 : 1;
    const uint32_t base = n_inner ? atomicAdd(counter, (uint32_t)n_inner) : 0u;
    float lo[3][4], hi[3][4];
    uint32_t link[4];
    int k = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < m) {
            for (int a = 0; a < 3; ++a) { lo[a][i] = c[i].lo[a]; hi[a][i] = c[i].hi[a]; }
            if (c[i].link & kLeafBit) {
                link[i] = c[i].link;
            } else {
                link[i] = base + (uint32_t)k;
                src[base + (uint32_t)k] = c[i].link;
                ++k;
            }
        } else {   // unused slot: NaN planes fail every box test
            for (int a = 0; a < 3; ++a) { lo[a][i] = __int_as_float(0x7FC00000); hi[a][i] = lo[a][i]; }
            link[i] = leaf_link(0u, 1u);
        }
    }
    float4* o = n4 + 8 * (size_t)slot;
    for (int a = 0; a < 3; ++a) {
        o[2 * a] = make_float4(lo[a][0], lo[a][1], lo[a][2], lo[a][3]);
        o[2 * a + 1] = make_float4(hi[a][0], hi[a][1], hi[a][2], hi[a][3]);
    }
    o[6] = make_float4(__uint_as_float(link[0]), __uint_as_float(link[1]), __uint_as_float(link[2]),
                       __uint_as_float(link[3]));
    o[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    WideCand u = c[0];
    float leaf_cost = 0.0f;
    uint32_t n_leaves = 0, leaf_sizes = 0;
    for (int i = 0; i < m; ++i) {
        for (int a = 0; a < 3; ++a) { u.lo[a] = fminf(u.lo[a], c[i].lo[a]); u.hi[a] = fmaxf(u.hi[a], c[i].hi[a]); }
        if (c[i].link & kLeafBit) {
            leaf_cost += (c_isect * (float)((c[i].link & 7u) + 1u) + kLeafEntry * c_trav) * c[i].area;
            ++n_leaves;
            leaf_sizes += 1u << (4u * (c[i].link & 7u));
        }
    }
    wide_stat(stats, half_area(u), leaf_cost, n_leaves, leaf_sizes, c_trav, inv_root_area);
}

// ---------------------------------------------------------------------------
// SAH-optimal collapse into 4-wide nodes (after Ylitie, Karras and Laine,
// "Efficient Incoherent Ray Traversal on GPUs Through Compressed Wide BVHs",
// HPG 2017, here for 4 children).  C(i, j) is the least SAH cost of the
// binary subtree i when it may fill j (1..4) child slots of its wide parent:
//   C(i, 1)  = min(leaf: (c_isect * count + c_leaf) * A(i) if count <= max_leaf,
//                  wide node: c_trav * A(i) + min_k C(l, k) + C(r, 4 - k))
//   C(i, j)  = min(C(i, j - 1), min_k C(l, k) + C(r, j - k))
// with A the box surface area and c_leaf = kLeafEntry * c_trav; a single
// triangle costs (c_isect + c_leaf) * A(tri) whatever j.  One bottom-up pass computes
// the costs, the decisions and the number of wide nodes each choice makes;
// the wide nodes are then emitted level by level from the decisions.
// Decision word of inner node i: bit 0 leaf at j = 1; bits 1-2 the left
// child's slots k of the wide node rooted at i; bits 2j-1..2j the left
// child's slots for j = 2, 3, 4 (0: j - 1 slots of i itself suffice).
// ---------------------------------------------------------------------------

struct WideDP {
    float4* cost;      // C(i, 1..4)
    int4* count;       // wide nodes of each choice
    uint32_t* dec;
};

__device__ inline void dp_child(int32_t c, const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                const uint32_t* __restrict__ sorted, NodeData nd, WideDP wd, float c_isect,
                                float c_entry, float3& lo, float3& hi, float C[5], int W[5]) {
    if (c < 0) {
        const uint32_t t = sorted[(uint32_t)c & ~kLeafBit];
        const float4 a = tlo[t], b = thi[t];
        lo = make_float3(a.x, a.y, a.z);
        hi = make_float3(b.x, b.y, b.z);
        const float ct = (c_isect + c_entry) * half_area(lo, hi);
        for (int j = 1; j <= 4; ++j) { C[j] = ct; W[j] = 0; }
    } else {
        // computed earlier in the pass (a deeper level, or the sibling's walk)
        const float4 a = nd.lo[c], b = nd.hi[c];
        lo = make_float3(a.x, a.y, a.z);
        hi = make_float3(b.x, b.y, b.z);
        const float4 cc = wd.cost[c];
        const int4 ww = wd.count[c];
        C[1] = cc.x; C[2] = cc.y; C[3] = cc.z; C[4] = cc.w;
        W[1] = ww.x; W[2] = ww.y; W[3] = ww.z; W[4] = ww.w;
    }
}

struct WideDPBody {
    const int32_t* left;
    const int32_t* right;
    const int32_t* rfirst;
    const int32_t* rlast;
    const float4* tlo;
    const float4* thi;
    const uint32_t* sorted;
    NodeData nd;
    WideDP wd;
    int max_leaf;
    float c_trav, c_isect;
    __device__ void operator()(int node) const {
        const float c_entry = kLeafEntry * c_trav;
        float3 llo, lhi, rlo, rhi;
        float Cl[5], Cr[5];
        int Wl[5], Wr[5];
        dp_child(left[node], tlo, thi, sorted, nd, wd, c_isect, c_entry, llo, lhi, Cl, Wl);
        dp_child(right[node], tlo, thi, sorted, nd, wd, c_isect, c_entry, rlo, rhi, Cr, Wr);
        const float3 lo = make_float3(fminf(llo.x, rlo.x), fminf(llo.y, rlo.y), fminf(llo.z, rlo.z));
        const float3 hi = make_float3(fmaxf(lhi.x, rhi.x), fmaxf(lhi.y, rhi.y), fmaxf(lhi.z, rhi.z));
        const float a = half_area(lo, hi);
        const int cnt = rlast[node] - rfirst[node] + 1;
        // the wide node rooted here: its four slots split between the children
        int kint = 1;
        float best4 = Cl[1] + Cr[3];
        for (int k = 2; k <= 3; ++k) {
            const float c = Cl[k] + Cr[4 - k];
            if (c < best4) { best4 = c; kint = k; }
        }
        const float c_int = c_trav * a + best4;
        const float c_leaf = cnt <= max_leaf ? (c_isect * (float)cnt + c_entry) * a : INFINITY;
        const bool leaf = c_leaf <= c_int;
        float C[5];
        int W[5];
        C[1] = leaf ? c_leaf : c_int;
        W[1] = leaf ? 0 : 1 + Wl[kint] + Wr[4 - kint];
        uint32_t dec = (leaf ? 1u : 0u) | ((uint32_t)kint << 1);
        for (int j = 2; j <= 4; ++j) {
            float best = C[j - 1];
            int d = 0;
            for (int k = 1; k < j; ++k) {
                const float c = Cl[k] + Cr[j - k];
                if (c < best) { best = c; d = k; }
            }
            C[j] = best;
            W[j] = d ? Wl[d] + Wr[j - d] : W[j - 1];
            dec |= (uint32_t)d << (2 * j - 1);
        }
        nd.lo[node] = make_float4(lo.x, lo.y, lo.z, 0.0f);
        nd.hi[node] = make_float4(hi.x, hi.y, hi.z, 0.0f);
        wd.cost[node] = make_float4(C[1], C[2], C[3], C[4]);
        wd.count[node] = make_int4(W[1], W[2], W[3], W[4]);
        wd.dec[node] = dec;
    }
};

// Wide nodes of the whole tree (the root is always a wide node) and the root box.
struct WideSummary {
    int32_t n_wide;
    float bbox[6];
};

__global__ void k_wide_summary(const int32_t* __restrict__ left, const int32_t* __restrict__ right, NodeData nd,
                               WideDP wd, WideSummary* sm) {
    const int kint = (int)((wd.dec[0] >> 1) & 3u);
    const int32_t l = left[0], r = right[0];
    const int wl = l < 0 ? 0 : (&wd.count[l].x)[kint - 1];
    const int wr = r < 0 ? 0 : (&wd.count[r].x)[4 - kint - 1];
    sm->n_wide = 1 + wl + wr;
    const float4 a = nd.lo[0], b = nd.hi[0];
    sm->bbox[0] = a.x; sm->bbox[1] = a.y; sm->bbox[2] = a.z;
    sm->bbox[3] = b.x; sm->bbox[4] = b.y; sm->bbox[5] = b.z;
}

// One level of the optimal collapse: slot s expands binary node src[s].
__global__ __launch_bounds__(kB) void k_emit4(const int32_t* __restrict__ left, const int32_t* __restrict__ right,
                                               const int32_t* __restrict__ rfirst, const int32_t* __restrict__ rlast,
                                               const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                               const uint32_t* __restrict__ sorted, NodeData nd, WideDP wd,
                                               uint32_t begin, uint32_t end, uint32_t* __restrict__ src,
                                               uint32_t* __restrict__ counter, float4* __restrict__ n4,
                                               WideStats* stats, float c_trav, float c_isect, float inv_root_area,
                                               uint32_t cap, uint32_t* __restrict__ error) {
    const uint32_t slot = begin + blockIdx.x * kB + threadIdx.x;
    if (slot >= end) return;
    const int32_t x = (int32_t)src[slot];
    const int kint = (int)((wd.dec[x] >> 1) & 3u);
    // work list of (binary child, slots it may fill); the slots of its
    // entries never sum to more than 4, so it holds at most 4 entries
    int32_t wn[4];
    int wj[4];
    int sp = 0;
    wn[sp] = right[x]; wj[sp++] = 4 - kint;
    wn[sp] = left[x]; wj[sp++] = kint;
    float lo[3][4], hi[3][4];
    uint32_t link[4];
    int32_t inner[4];
    int m = 0;
    float leaf_cost = 0.0f;
    uint32_t n_leaves = 0, leaf_sizes = 0;
    for (int guard = 0; sp > 0 && guard < 256; ++guard) {
        const int32_t c = wn[--sp];
        const int j = wj[sp];
        if (c >= 0 && j > 1) {
            const int d = (int)((wd.dec[c] >> (2 * j - 1)) & 3u);
            if (sp + 2 > 4 || d >= j) { atomicOr(error, 1u); return; }
            if (d == 0) {
                wn[sp] = c; wj[sp++] = j - 1;
            } else {
                wn[sp] = right[c]; wj[sp++] = j - d;
                wn[sp] = left[c]; wj[sp++] = d;
            }
            continue;
        }
        if (m >= 4) { atomicOr(error, 1u); return; }
        float4 a, b;
        if (c < 0) {   // one triangle
            const uint32_t pos = (uint32_t)c & ~kLeafBit;
            const uint32_t t = sorted[pos];
            a = tlo[t]; b = thi[t];
            link[m] = leaf_link(pos, 1u);
            inner[m] = -1;
        } else {
            a = nd.lo[c]; b = nd.hi[c];
            if (wd.dec[c] & 1u) {
                link[m] = leaf_link((uint32_t)rfirst[c], (uint32_t)(rlast[c] - rfirst[c] + 1));
                inner[m] = -1;
            } else {
                link[m] = 0u;
                inner[m] = c;
            }
        }
        if (inner[m] < 0) {
            const uint32_t cnt = (link[m] & 7u) + 1u;
            leaf_cost += (c_isect * (float)cnt + kLeafEntry * c_trav) *
                         half_area(make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z));
            ++n_leaves;
            leaf_sizes += 1u << (4u * (cnt - 1u));
        }
        lo[0][m] = pad_lo(a.x); hi[0][m] = pad_hi(b.x);
        lo[1][m] = pad_lo(a.y); hi[1][m] = pad_hi(b.y);
        lo[2][m] = pad_lo(a.z); hi[2][m] = pad_hi(b.z);
        ++m;
    }
    if (sp > 0 || m < 2) { atomicOr(error, 1u); return; }
    int n_inner = 0;
    for (int i = 0; i < m; ++i) n_inner += inner[i] >= 0 ? 1 : 0;
    const uint32_t base = n_inner ? atomicAdd(counter, (uint32_t)n_inner) : 0u;
    if (base + (uint32_t)n_inner > cap) { atomicOr(error, 2u); return; }   // more nodes than counted
    int k = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < m) {
            if (inner[i] >= 0) {
                link[i] = base + (uint32_t)k;
                src[base + (uint32_t)k] = (uint32_t)inner[i];
                ++k;
            }
        } else {   // unused slot: NaN planes fail every box test
            for (int a = 0; a < 3; ++a) { lo[a][i] = __int_as_float(0x7FC00000); hi[a][i] = lo[a][i]; }
            link[i] = leaf_link(0u, 1u);
        }
    }
    float4* o = n4 + 8 * (size_t)slot;
    for (int a = 0; a < 3; ++a) {
        o[2 * a] = make_float4(lo[a][0], lo[a][1], lo[a][2], lo[a][3]);
        o[2 * a + 1] = make_float4(hi[a][0], hi[a][1], hi[a][2], hi[a][3]);
    }
    o[6] = make_float4(__uint_as_float(link[0]), __uint_as_float(link[1]), __uint_as_float(link[2]),
                       __uint_as_float(link[3]));
    o[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float4 xa = nd.lo[x], xb = nd.hi[x];
    wide_stat(stats, half_area(make_float3(xa.x, xa.y, xa.z), make_float3(xb.x, xb.y, xb.z)), leaf_cost, n_leaves,
              leaf_sizes, c_trav, inv_root_area);
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) {
    if (threadIdx.x == 0) *p = v;
}

__device__ inline float clamp01(float v) {
    v = (v > 0.0f) ? v : 0.0f;   // NaN -> 0
    return (v > 1.0f) ? 1.0f : v;
}

struct ShadeParams {
    float light[3];
    float k_a, k_d;
};

// Triangles in leaf order, in three copies (copy c, for rays whose dominant
// axis is c, stores each vertex as (x[c+1], x[c+2], x[c]), indices mod 3: the
// watertight test's axis order, so it needs no per-vertex selects), the
// original index in the w word of the first vertex of each copy; plus their
// two shaded colours.  Shading: two-sided
// Lambert with the flat geometric normal n = cross(v1 - v0, v2 - v0) (flipped
// for the back side), one directional light, clamped to [0, 1]; evaluated in
// FP32 left to right without contraction.
__global__ __launch_bounds__(kB) void k_pack_tris(uint32_t n, const float* __restrict__ verts,
                                                   const uint32_t* __restrict__ idx, const float* __restrict__ albedo,
                                                   const uint32_t* __restrict__ sorted, ShadeParams sp,
                                                   float4* __restrict__ tris, float4* __restrict__ shade,
                                                   float4* __restrict__ normals) {
    const uint32_t j = blockIdx.x * kB + threadIdx.x;
    if (j >= n) return;
    const uint32_t t = sorted ? sorted[j] : j;
    const float3 a = ld3(verts, idx[3 * (size_t)t]);
    const float3 b = ld3(verts, idx[3 * (size_t)t + 1]);
    const float3 c = ld3(verts, idx[3 * (size_t)t + 2]);
    const float id = __uint_as_float(t);
    tris[3 * (size_t)j + 0] = make_float4(a.y, a.z, a.x, id);   // kz = x
    tris[3 * (size_t)j + 1] = make_float4(b.y, b.z, b.x, 0.0f);
    tris[3 * (size_t)j + 2] = make_float4(c.y, c.z, c.x, 0.0f);
    tris[3 * ((size_t)n + j) + 0] = make_float4(a.z, a.x, a.y, id);   // kz = y
    tris[3 * ((size_t)n + j) + 1] = make_float4(b.z, b.x, b.y, 0.0f);
    tris[3 * ((size_t)n + j) + 2] = make_float4(c.z, c.x, c.y, 0.0f);
    tris[3 * (2 * (size_t)n + j) + 0] = make_float4(a.x, a.y, a.z, id);   // kz = z
    tris[3 * (2 * (size_t)n + j) + 1] = make_float4(b.x, b.y, b.z, 0.0f);
    tris[3 * (2 * (size_t)n + j) + 2] = make_float4(c.x, c.y, c.z, 0.0f);

    const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    float nx = e1y * e2z - e1z * e2y;
    float ny = e1z * e2x - e1x * e2z;
    float nz = e1x * e2y - e1y * e2x;
    const float len = sqrtf((nx * nx + ny * ny) + nz * nz);
    nx = nx / len;
    ny = ny / len;
    nz = nz / len;
    normals[j] = make_float4(nx, ny, nz, 0.0f);
    const float3 alb = ld3(albedo, t);
    for (int side = 0; side < 2; ++side) {
        const float sx = side ? -nx : nx, sy = side ? -ny : ny, sz = side ? -nz : nz;
        const float dot = (sx * sp.light[0] + sy * sp.light[1]) + sz * sp.light[2];
        const float diff = dot > 0.0f ? dot : 0.0f;
        const float s = sp.k_a + sp.k_d * diff;
        shade[2 * (size_t)j + side] = make_float4(clamp01(alb.x * s), clamp01(alb.y * s), clamp01(alb.z * s), 0.0f);
    }
}

template <typename T>
rcp_status dalloc(T** p, size_t count) {
    return dev_alloc((void**)p, sizeof(T) * count);
}

// Scratch buffers of a build, released on its stream when the set goes out
// of scope (stream-ordered, so no device-wide synchronisation).
struct TempSet {
    hipStream_t stream;
    std::vector<void*> ptrs;
    explicit TempSet(hipStream_t s) : stream(s) {}
    ~TempSet() {
        for (void* p : ptrs) stream_free(p, stream);
    }
    template <typename T>
    rcp_status alloc(T** p, size_t count) {
        rcp_status st = stream_alloc((void**)p, sizeof(T) * count, stream);
        if (st == RCP_OK && *p) ptrs.push_back((void*)*p);
        return st;
    }
};

#define RCP_TRY(expr) do { rcp_status st_ = (expr); if (st_ != RCP_OK) return st_; } while (0)

inline unsigned blocks(long n) { return (unsigned)((n + kB - 1) / kB); }

// Inner nodes sorted by depth, and where each depth starts (host copy), for
// the bottom-up passes.  A PLOC tree is at most as deep as its rounds (at
// most 64 + 16 log2 n <= 512), a radix tree at most 64 key bits plus log2 n
// for equal keys, so kMaxLevels is never reached by a tree built here.
constexpr uint32_t kMaxLevels = 1024;

struct LevelOrder {
    int32_t* ids = nullptr;
    std::vector<uint32_t> starts;   // depth d: ids[starts[d] .. starts[d + 1])
};

rcp_status level_order(int n, const int32_t* parent, TempSet& tmp, LevelOrder& lo, hipStream_t stream) {
    const int m = n - 1;
    uint64_t *keys, *keys2;
    uint32_t *ids, *ids2, *max_depth, *starts;
    RCP_TRY(tmp.alloc(&keys, (size_t)m));
    RCP_TRY(tmp.alloc(&keys2, (size_t)m));
    RCP_TRY(tmp.alloc(&ids, (size_t)m));
    RCP_TRY(tmp.alloc(&ids2, (size_t)m));
    RCP_TRY(tmp.alloc(&max_depth, 1));
    RCP_TRY(tmp.alloc(&starts, kMaxLevels + 1));
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, max_depth, 0u);
    hipLaunchKernelGGL(k_node_depth, dim3(blocks(m)), dim3(kB), 0, stream, n, parent, keys, ids, max_depth);
    RCP_CHECK_LAUNCH();
    uint32_t depth = 0;
    RCP_HIP(hipMemcpyAsync(&depth, max_depth, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    RCP_HIP(hipStreamSynchronize(stream));
    lo.ids = nullptr;
    lo.starts.clear();
    if (depth + 1 > kMaxLevels) {
        set_error("binary tree of depth %u (limit %u)", depth, kMaxLevels - 1);
        return RCP_ERR_INTERNAL;
    }
    int bits = 8;
    while ((1u << bits) <= depth) bits += 8;
    RCP_TRY(radix_sort_pairs(keys, ids, keys2, ids2, m, bits, stream));
    hipLaunchKernelGGL(k_level_starts, dim3(blocks(m)), dim3(kB), 0, stream, m, (const uint64_t*)keys, starts);
    RCP_CHECK_LAUNCH();
    lo.starts.resize(depth + 2);
    RCP_HIP(hipMemcpyAsync(lo.starts.data(), starts, sizeof(uint32_t) * (depth + 1), hipMemcpyDeviceToHost, stream));
    RCP_HIP(hipStreamSynchronize(stream));
    lo.starts[depth + 1] = (uint32_t)m;
    lo.ids = (int32_t*)ids;
    return RCP_OK;
}

// Run a bottom-up pass over the tree, deepest level first.
template <class Body>
rcp_status bottom_up(const LevelOrder& lo, const Body& body, hipStream_t stream) {
    for (int d = (int)lo.starts.size() - 2; d >= 0; --d) {
        const uint32_t c = lo.starts[(size_t)d + 1] - lo.starts[(size_t)d];
        if (c == 0) continue;
        hipLaunchKernelGGL(k_level<Body>, dim3(blocks(c)), dim3(kB), 0, stream,
                           (const int32_t*)lo.ids + lo.starts[(size_t)d], c, body);
    }
    RCP_CHECK_LAUNCH();
    return RCP_OK;
}

// PLOC tree over the Morton-sorted triangles, renumbered in depth-first leaf
// order (sorted is permuted in place).  Returns RCP_ERR_NOT_READY when the
// rounds do not converge within the cap; the caller then builds the radix
// tree from the untouched sorted order instead.
rcp_status ploc_build(int n, const float4* tlo, const float4* thi, uint32_t* sorted, int32_t* left, int32_t* right,
                      int32_t* parent, int32_t* rfirst, int32_t* rlast, TempSet& outer, LevelOrder& levels,
                      hipStream_t stream) {
    TempSet tmp(stream);
    int32_t *id, *id2, *nn, *next_id, *cnt, *first, *parent_tmp;
    float4 *lo, *hi, *lo2, *hi2;
    uint32_t *pos, *keep, *m_out, *scratch, *sorted2;
    const size_t un = (size_t)n;
    RCP_TRY(tmp.alloc(&id, un));
    RCP_TRY(tmp.alloc(&id2, un));
    RCP_TRY(tmp.alloc(&nn, un));
    RCP_TRY(tmp.alloc(&next_id, 1));
    RCP_TRY(tmp.alloc(&cnt, un));
    RCP_TRY(tmp.alloc(&first, 2 * un));
    RCP_TRY(tmp.alloc(&parent_tmp, 2 * un));
    RCP_TRY(tmp.alloc(&lo, un));
    RCP_TRY(tmp.alloc(&hi, un));
    RCP_TRY(tmp.alloc(&lo2, un));
    RCP_TRY(tmp.alloc(&hi2, un));
    RCP_TRY(tmp.alloc(&pos, un));
    RCP_TRY(tmp.alloc(&keep, un));
    RCP_TRY(tmp.alloc(&m_out, 1));
    RCP_TRY(tmp.alloc(&scratch, scan_scratch_words(n)));
    RCP_TRY(tmp.alloc(&sorted2, un));
    // every entry gets its parent from a merge; -1 until then, so that a walk
    // to the root ends whatever happens
    RCP_HIP(hipMemsetAsync(parent_tmp, 0xFF, sizeof(int32_t) * 2 * un, stream));
    hipLaunchKernelGGL(k_ploc_init, dim3(blocks(n)), dim3(kB), 0, stream, n, tlo, thi, (const uint32_t*)sorted, id,
                       lo, hi);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, stream, next_id, (int32_t)(n - 2));
    RCP_CHECK_LAUNCH();
    int log2n = 0;
    while ((1 << log2n) < n) ++log2n;
    const int max_rounds = 64 + 16 * log2n;
    int m = n, rounds = 0;
    while (m > 1) {
        if (m <= kPlocSmall) {   // the remaining rounds in one workgroup
            hipLaunchKernelGGL(k_ploc_finish, dim3(1), dim3(kPlocSmall), 0, stream, m, n, max_rounds - rounds,
                               (const int32_t*)id, (const float4*)lo, (const float4*)hi, next_id, left, right,
                               parent_tmp, m_out);
            RCP_CHECK_LAUNCH();
            uint32_t fin = 0;
            RCP_HIP(hipMemcpyAsync(&fin, m_out, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
            RCP_HIP(hipStreamSynchronize(stream));
            if (fin != 1u) {
                set_error("PLOC's last rounds ended with %u of %d clusters", fin, m);
                return RCP_ERR_INTERNAL;
            }
            m = 1;
            break;
        }
        if (++rounds > max_rounds) return RCP_ERR_NOT_READY;
        hipLaunchKernelGGL(k_ploc_nn, dim3(blocks(m)), dim3(kB), 0, stream, m, (const float4*)lo, (const float4*)hi,
                           nn);
        hipLaunchKernelGGL(k_ploc_merge, dim3(blocks(m)), dim3(kB), 0, stream, m, n, (const int32_t*)nn,
                           (const int32_t*)id, (const float4*)lo, (const float4*)hi, id2, lo2, hi2, pos, keep, next_id,
                           left, right, parent_tmp);
        RCP_CHECK_LAUNCH();
        RCP_TRY(scan_exclusive_u32(pos, m, scratch, stream));
        hipLaunchKernelGGL(k_ploc_compact, dim3(blocks(m)), dim3(kB), 0, stream, m, (const uint32_t*)pos,
                           (const uint32_t*)keep, (const int32_t*)id2, (const float4*)lo2, (const float4*)hi2, id, lo,
                           hi, m_out);
        RCP_CHECK_LAUNCH();
        uint32_t next = 0;
        RCP_HIP(hipMemcpyAsync(&next, m_out, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        RCP_HIP(hipStreamSynchronize(stream));
        if (next < 1u || next >= (uint32_t)m) {
            set_error("PLOC round %d went from %d to %u clusters", rounds, m, next);
            return RCP_ERR_INTERNAL;
        }
        m = (int)next;
    }
    int32_t last = 0;
    RCP_HIP(hipMemcpyAsync(&last, next_id, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    RCP_HIP(hipStreamSynchronize(stream));
    if (last != -1) {
        set_error("PLOC made %d inner nodes, expected %d", n - 2 - last, n - 1);
        return RCP_ERR_INTERNAL;
    }
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, stream, parent_tmp, -1);   // the root
    RCP_CHECK_LAUNCH();
    // the depth order of the inner nodes holds for the renumbered tree too
    // (inner nodes keep their numbers)
    RCP_TRY(level_order(n, parent_tmp, outer, levels, stream));
    RCP_TRY(bottom_up(levels, LeafCountBody{left, right, cnt}, stream));
    hipLaunchKernelGGL(k_dfs_first, dim3(blocks(2L * n - 1)), dim3(kB), 0, stream, n, (const int32_t*)left,
                       (const int32_t*)right, (const int32_t*)parent_tmp, (const int32_t*)cnt, first);
    hipLaunchKernelGGL(k_dfs_renumber, dim3(blocks(2L * n - 1)), dim3(kB), 0, stream, n, (const int32_t*)first,
                       (const int32_t*)cnt, (const uint32_t*)sorted, (const int32_t*)parent_tmp, sorted2, parent,
                       left, right, rfirst, rlast);
    RCP_CHECK_LAUNCH();
    RCP_HIP(hipMemcpyAsync(sorted, sorted2, sizeof(uint32_t) * un, hipMemcpyDeviceToDevice, stream));
    RCP_HIP(hipStreamSynchronize(stream));
    return RCP_OK;
}

}  // namespace

rcp_status build_scene(const rcp_scene_desc* desc, const rcp_build_options* opts, hipStream_t stream,
                       rcp_scene** out) {
    const uint32_t n = desc->n_tris;
    const int max_leaf = opts ? opts->max_leaf : kDefaultMaxLeaf;
    const float c_trav = opts ? opts->c_trav : 1.0f;
    const float c_isect = opts ? opts->c_isect : 1.0f;
    const int builder = opts ? opts->builder : RCP_BUILDER_PLOC;
    const int collapse = opts ? opts->collapse : RCP_COLLAPSE_SAH;

    rcp_scene* s = new rcp_scene();
    struct Guard {
        rcp_scene*& s;
        bool ok = false;
        ~Guard() {
            if (!ok && s) {
                if (s->nodes) (void)hipFree(s->nodes);
                if (s->tris) (void)hipFree(s->tris);
                if (s->shade) (void)hipFree(s->shade);
                if (s->normals) (void)hipFree(s->normals);
                if (s->occ.bits) (void)hipFree(s->occ.bits);
                if (s->err_host) (void)hipHostFree(s->err_host);
                delete s;
                s = nullptr;
            }
        }
    } guard{s};

    RCP_HIP(hipGetDevice(&s->device));
    s->dev.bg[0] = desc->background[0];
    s->dev.bg[1] = desc->background[1];
    s->dev.bg[2] = desc->background[2];
    s->stats.n_tris = n;
    s->stats.max_leaf = (uint32_t)max_leaf;

    hipEvent_t e0, e1;
    RCP_HIP(hipEventCreate(&e0));
    RCP_HIP(hipEventCreate(&e1));
    struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evg{e0, e1};

    // the box of the vertices (for the occupancy grid) and the largest
    // |coordinate| (for the traversal's box widening), in one pass
    float blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float radius = 0.0f;
    for (size_t i = 0; i < (size_t)desc->n_verts && n > 0; ++i)
        for (int a = 0; a < 3; ++a) {
            const float v = desc->verts[3 * i + a];
            blo[a] = fminf(blo[a], v);
            bhi[a] = fmaxf(bhi[a], v);
            radius = fmaxf(radius, fabsf(v));
        }

    TempSet tmp(stream);
    float* d_verts = nullptr;
    uint32_t* d_idx = nullptr;
    float* d_rgb = nullptr;
    if (n > 0) {
        RCP_TRY(tmp.alloc(&d_verts, 3 * (size_t)desc->n_verts));
        RCP_TRY(tmp.alloc(&d_idx, 3 * (size_t)n));
        RCP_TRY(tmp.alloc(&d_rgb, 3 * (size_t)n));
        RCP_HIP(hipMemcpyAsync(d_verts, desc->verts, sizeof(float) * 3 * (size_t)desc->n_verts,
                               hipMemcpyHostToDevice, stream));
        RCP_HIP(hipMemcpyAsync(d_idx, desc->idx, sizeof(uint32_t) * 3 * (size_t)n, hipMemcpyHostToDevice, stream));
        RCP_HIP(hipMemcpyAsync(d_rgb, desc->tri_rgb, sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice, stream));
    }
    RCP_HIP(hipEventRecord(e0, stream));
    if (n > 0) {
        // the occupancy grid over the box of the vertices
        const float emax = fmaxf(fmaxf(bhi[0] - blo[0], bhi[1] - blo[1]), bhi[2] - blo[2]);
        OccGrid& g = s->occ;
        for (int a = 0; a < 3; ++a) {
            const float ext = bhi[a] - blo[a];
            const int c = emax > 0.0f ? (int)ceilf((float)kOccCells * ext / emax) : 1;
            // about cubic cells, but at least a quarter of the longest axis's
            // count along a thin axis (a flat scene's height still resolves)
            g.n[a] = ext <= 0.0f ? 1 : (c < kOccCells / 4 ? kOccCells / 4 : (c > kOccCells ? kOccCells : c));
            g.lo[a] = blo[a];
            g.cell[a] = ext > 0.0f ? ext / (float)g.n[a] : 1.0f;
        }
        g.words = (uint32_t)(((size_t)g.n[0] * g.n[1] * g.n[2] + 31) / 32);
        RCP_TRY(dalloc(&g.bits, g.words));
        RCP_HIP(hipMemsetAsync(g.bits, 0, sizeof(uint32_t) * g.words, stream));
        hipLaunchKernelGGL(k_occupancy, dim3(std::min(blocks(n), 4096u)), dim3(kB), 0, stream, (const float*)d_verts,
                           (const uint32_t*)d_idx, n, g, g.bits);
        RCP_CHECK_LAUNCH();
    }

    uint32_t n_nodes = 0, n_leaves = 0, max_depth = 0, stack_bound = 0, top_count = 0;
    float sah = 0.0f;
    uint32_t* sorted = nullptr;
    float4 *tlo = nullptr, *thi = nullptr;
    if (n > 0) {
        uint32_t* bounds;
        uint64_t *keys, *keys2;
        uint32_t* vals2;
        RCP_TRY(tmp.alloc(&tlo, n));
        RCP_TRY(tmp.alloc(&thi, n));
        RCP_TRY(tmp.alloc(&bounds, 8));
        RCP_TRY(tmp.alloc(&keys, n));
        RCP_TRY(tmp.alloc(&keys2, n));
        RCP_TRY(tmp.alloc(&sorted, n));
        RCP_TRY(tmp.alloc(&vals2, n));
        hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, stream, bounds);
        hipLaunchKernelGGL(k_tri_prep, dim3(std::min(blocks(n), 2048u)), dim3(kB), 0, stream, (const float*)d_verts,
                           (const uint32_t*)d_idx, n, tlo, thi, bounds);
        hipLaunchKernelGGL(k_morton, dim3(blocks(n)), dim3(kB), 0, stream, (const float4*)tlo,
                           (const float4*)thi, n, (const uint32_t*)bounds, keys, sorted);
        RCP_CHECK_LAUNCH();
        RCP_TRY(radix_sort_pairs(keys, sorted, keys2, vals2, (int)n, 64, stream));

        Summary* sm;
        WideSummary* wsm;
        WideStats* wst;
        uint32_t* err;
        RCP_TRY(tmp.alloc(&sm, 1));
        RCP_TRY(tmp.alloc(&wsm, 1));
        RCP_TRY(tmp.alloc(&wst, 1));
        RCP_TRY(tmp.alloc(&err, 1));
        RCP_HIP(hipMemsetAsync(wst, 0, sizeof(WideStats), stream));
        RCP_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), stream));
        Summary hs{};
        WideSummary hw{};
        bool single = n <= 1;
        int32_t *left = nullptr, *right = nullptr, *parent = nullptr, *rfirst = nullptr, *rlast = nullptr;
        NodeData nd{};
        WideDP wd{};
        float bbox[6] = {0, 0, 0, 0, 0, 0};
        if (!single) {
            const long ni = (long)n - 1;
            RCP_TRY(tmp.alloc(&left, ni));
            RCP_TRY(tmp.alloc(&right, ni));
            RCP_TRY(tmp.alloc(&parent, 2 * (size_t)n - 1));
            RCP_TRY(tmp.alloc(&rfirst, ni));
            RCP_TRY(tmp.alloc(&rlast, ni));
            RCP_TRY(tmp.alloc(&nd.lo, ni));
            RCP_TRY(tmp.alloc(&nd.hi, ni));
            rcp_status tree = RCP_ERR_NOT_READY;
            LevelOrder levels;
            if (builder == RCP_BUILDER_PLOC)
                tree = ploc_build((int)n, tlo, thi, sorted, left, right, parent, rfirst, rlast, tmp, levels, stream);
            if (tree == RCP_ERR_NOT_READY) {   // the radix tree, or PLOC did not converge
                hipLaunchKernelGGL(k_radix_tree, dim3(blocks(ni)), dim3(kB), 0, stream, (const uint64_t*)keys,
                                   (int)n, left, right, parent, rfirst, rlast);
                RCP_CHECK_LAUNCH();
                tree = level_order((int)n, parent, tmp, levels, stream);
            }
            if (tree != RCP_OK) return tree;
            if (collapse == RCP_COLLAPSE_SAH) {
                RCP_TRY(tmp.alloc(&wd.cost, ni));
                RCP_TRY(tmp.alloc(&wd.count, ni));
                RCP_TRY(tmp.alloc(&wd.dec, ni));
                RCP_TRY(bottom_up(levels,
                                  WideDPBody{left, right, rfirst, rlast, tlo, thi, sorted, nd, wd, max_leaf, c_trav,
                                             c_isect},
                                  stream));
                hipLaunchKernelGGL(k_wide_summary, dim3(1), dim3(1), 0, stream, (const int32_t*)left,
                                   (const int32_t*)right, nd, wd, wsm);
                RCP_CHECK_LAUNCH();
                RCP_HIP(hipMemcpyAsync(&hw, wsm, sizeof(WideSummary), hipMemcpyDeviceToHost, stream));
                RCP_HIP(hipStreamSynchronize(stream));
                memcpy(bbox, hw.bbox, sizeof(bbox));
                if (hw.n_wide < 1 || (uint32_t)hw.n_wide > (uint32_t)ni) {
                    set_error("optimal collapse counted %d wide nodes for %ld binary nodes", hw.n_wide, ni);
                    return RCP_ERR_INTERNAL;
                }
            } else {
                RCP_TRY(tmp.alloc(&nd.cost, ni));
                RCP_TRY(tmp.alloc(&nd.n_inner, ni));
                RCP_TRY(tmp.alloc(&nd.collapse, ni));
                RCP_TRY(bottom_up(levels,
                                  RefitBody{left, right, rfirst, rlast, tlo, thi, sorted, nd, max_leaf, c_trav, c_isect},
                                  stream));
                hipLaunchKernelGGL(k_summary_root, dim3(1), dim3(1), 0, stream, nd, sm);
                RCP_CHECK_LAUNCH();
                RCP_HIP(hipMemcpyAsync(&hs, sm, sizeof(Summary), hipMemcpyDeviceToHost, stream));
                RCP_HIP(hipStreamSynchronize(stream));
                memcpy(bbox, hs.bbox, sizeof(bbox));
                single = hs.root_collapsed != 0;
            }
        }
        const float root_area = (bbox[3] - bbox[0]) * (bbox[4] - bbox[1]) + (bbox[4] - bbox[1]) * (bbox[5] - bbox[2]) +
                                (bbox[5] - bbox[2]) * (bbox[3] - bbox[0]);
        const float inv_root_area = root_area > 0.0f ? 1.0f / root_area : 0.0f;
        uint32_t levels = 0;
        if (!single && collapse == RCP_COLLAPSE_SAH) {
            // the optimal collapse, one launch per level of wide nodes
            n_nodes = (uint32_t)hw.n_wide;
            uint32_t *src, *counter;
            RCP_TRY(tmp.alloc(&src, n_nodes));
            RCP_TRY(tmp.alloc(&counter, 1));
            RCP_TRY(dalloc(&s->nodes, 8 * (size_t)n_nodes));
            hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, src, 0u);
            hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, counter, 1u);
            RCP_CHECK_LAUNCH();
            uint32_t begin = 0, end = 1;
            while (begin < end) {
                hipLaunchKernelGGL(k_emit4, dim3(blocks(end - begin)), dim3(kB), 0, stream, (const int32_t*)left,
                                   (const int32_t*)right, (const int32_t*)rfirst, (const int32_t*)rlast,
                                   (const float4*)tlo, (const float4*)thi, (const uint32_t*)sorted, nd, wd, begin,
                                   end, src, counter, s->nodes, wst, c_trav, c_isect, inv_root_area, n_nodes,
                                   err);
                RCP_CHECK_LAUNCH();
                uint32_t next = 0, bad = 0;
                RCP_HIP(hipMemcpyAsync(&next, counter, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
                RCP_HIP(hipMemcpyAsync(&bad, err, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
                RCP_HIP(hipStreamSynchronize(stream));
                if (bad || next > n_nodes || next < end) {
                    set_error("optimal collapse: level %u ended at %u of %u nodes (error %u)", levels, next, n_nodes,
                              bad);
                    return RCP_ERR_INTERNAL;
                }
                begin = end;
                end = next;
                ++levels;
                if (levels <= (uint32_t)kTopLevels) s->top_nodes[levels] = begin;   // nodes of levels < `levels`
            }
            if (end != n_nodes) {
                set_error("optimal collapse emitted %u of %u wide nodes", end, n_nodes);
                return RCP_ERR_INTERNAL;
            }
        } else {
            if (single) {
                n_nodes = 1;
                RCP_TRY(dalloc(&s->nodes, 4));
                hipLaunchKernelGGL(k_pack_single, dim3(1), dim3(1), 0, stream, (int)n, (const float4*)tlo,
                                   (const float4*)thi, s->nodes);
                RCP_CHECK_LAUNCH();
            } else {
                const long ni = (long)n - 1;
                int32_t* newidx;
                RCP_TRY(tmp.alloc(&newidx, ni));
                hipLaunchKernelGGL(k_layout_walk, dim3(blocks(ni)), dim3(kB), 0, stream, (int)n,
                                   (const int32_t*)left, (const int32_t*)parent, nd, newidx);
                RCP_CHECK_LAUNCH();
                n_nodes = (uint32_t)hs.n_inner;
                RCP_TRY(dalloc(&s->nodes, 4 * (size_t)n_nodes));
                hipLaunchKernelGGL(k_pack_nodes, dim3(blocks(ni)), dim3(kB), 0, stream, (int)n,
                                   (const int32_t*)left, (const int32_t*)right, (const int32_t*)rfirst,
                                   (const int32_t*)rlast, (const float4*)tlo, (const float4*)thi,
                                   (const uint32_t*)sorted, nd, (const int32_t*)newidx, s->nodes);
                RCP_CHECK_LAUNCH();
            }
            // greedy collapse of the packed binary tree into 4-wide nodes, one
            // launch per level; the binary nodes are freed with the other
            // temporaries
            float4* n2 = s->nodes;
            tmp.ptrs.push_back((void*)n2);
            s->nodes = nullptr;
            uint32_t *src, *counter;
            RCP_TRY(tmp.alloc(&src, n_nodes));
            RCP_TRY(tmp.alloc(&counter, 1));
            RCP_TRY(dalloc(&s->nodes, 8 * (size_t)n_nodes));
            hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, src, 0u);
            hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, stream, counter, 1u);
            RCP_CHECK_LAUNCH();
            uint32_t begin = 0, end = 1;
            while (begin < end) {
                hipLaunchKernelGGL(k_collapse4, dim3(blocks(end - begin)), dim3(kB), 0, stream, (const float4*)n2,
                                   begin, end, src, counter, s->nodes, wst, c_trav, c_isect, inv_root_area);
                RCP_CHECK_LAUNCH();
                uint32_t next = 0;
                RCP_HIP(hipMemcpyAsync(&next, counter, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
                RCP_HIP(hipStreamSynchronize(stream));
                if (next > n_nodes || next < end) {
                    set_error("wide BVH collapse produced %u nodes from %u binary nodes", next, n_nodes);
                    return RCP_ERR_INTERNAL;
                }
                begin = end;
                end = next;
                ++levels;
                if (levels <= (uint32_t)kTopLevels) s->top_nodes[levels] = begin;   // nodes of levels < `levels`
            }
            n_nodes = end;
        }
        // a tree of fewer levels is staged whole
        for (uint32_t l = levels + 1u; l <= (uint32_t)kTopLevels; ++l) s->top_nodes[l] = n_nodes;
        top_count = std::min(s->top_nodes[kTopLevels], kMaxStagedNodes);
        if (n_nodes > kMaxNodes) {
            set_error("the scene needs %u BVH nodes, more than the %u a scene can hold", n_nodes, kMaxNodes);
            return RCP_ERR_INVALID_ARGUMENT;
        }
        max_depth = levels + 1;          // leaves sit one level below the deepest wide node
        stack_bound = 3u * levels + 1u;  // at most three pushes per level
        {
            WideStats hst{};
            RCP_HIP(hipMemcpyAsync(&hst, wst, sizeof(WideStats), hipMemcpyDeviceToHost, stream));
            RCP_HIP(hipStreamSynchronize(stream));
            n_leaves = (uint32_t)hst.leaves;
            sah = (float)((double)hst.sah_fx / 4294967296.0);
            for (int c = 0; c < 8; ++c) s->stats.leaf_hist[c] = (uint32_t)hst.hist[c];
            if (single) sah = c_isect * (float)n;   // one leaf of every triangle, relative to its own box
        }
        RCP_TRY(dalloc(&s->tris, 9 * (size_t)n));   // three rotated copies
        RCP_TRY(dalloc(&s->shade, 2 * (size_t)n));
        RCP_TRY(dalloc(&s->normals, (size_t)n));
        ShadeParams sp{{desc->light_dir[0], desc->light_dir[1], desc->light_dir[2]}, desc->k_a, desc->k_d};
        hipLaunchKernelGGL(k_pack_tris, dim3(blocks(n)), dim3(kB), 0, stream, n, (const float*)d_verts,
                           (const uint32_t*)d_idx, (const float*)d_rgb, (const uint32_t*)sorted, sp, s->tris,
                           s->shade, s->normals);
        RCP_CHECK_LAUNCH();
    }
    RCP_HIP(hipEventRecord(e1, stream));
    RCP_HIP(hipStreamSynchronize(stream));
    float ms = 0.0f;
    RCP_HIP(hipEventElapsedTime(&ms, e0, e1));

    s->dev.nodes = s->nodes;
    s->dev.tris = s->tris;
    s->dev.shade = s->shade;
    s->dev.normals = s->normals;
    s->dev.radius = radius;
    s->dev.n_nodes = n_nodes;
    s->dev.n_tris = n;
    s->dev.max_depth = max_depth;
    s->dev.stack_bound = stack_bound;
    s->dev.top_count = top_count;
    // every step of a ray enters a node or a leaf, each at most once
    const uint64_t bound = 5ull * n_nodes + 16ull;
    const uint32_t hook = debug_step_budget();
    s->dev.step_budget = hook ? hook : (uint32_t)std::min<uint64_t>(bound, 0xFFFFFFFFull);
    // the error flag the kernels raise when a ray runs out of that budget:
    // pinned host memory, mapped into the device's address space
    if (alloc_hook_fails()) {
        set_error("pinned host allocation failed (test hook)");
        return RCP_ERR_OUT_OF_MEMORY;
    }
    RCP_HIP(hipHostMalloc((void**)&s->err_host, sizeof(uint32_t), hipHostMallocMapped));
    *s->err_host = 0u;
    RCP_HIP(hipHostGetDevicePointer((void**)&s->dev.err_flag, s->err_host, 0));
    s->stats.n_nodes = n_nodes;
    s->stats.n_leaves = n_leaves;
    s->stats.max_depth = max_depth;
    s->stats.sah_cost = sah;
    s->stats.build_ms = ms;
    s->stats.node_bytes = (uint32_t)kNodeBytes;
    s->stats.device_bytes = (uint64_t)kNodeBytes * n_nodes + 3ull * 48ull * n + 32ull * n + 16ull * n;
    guard.ok = true;
    *out = s;
    return RCP_OK;
}

}  // namespace rcp
