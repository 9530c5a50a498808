// Screen-space variant of recursive camera painting.
//
// With the eye fixed (Section 3's colour mapping has V_e = 0), the rendered
// image already holds most directions a displaced camera would see, so a
// pass reduces to fetching each pixel's new colour from a position displaced
// by its own red and green (Section 6).  Positions outside the image follow
// an edge rule: clamp, wrap or mirror (Section 6.1).  One launch per pass;
// each reads the previous pass's image.  HBM-bound: 8 B of the own pixel,
// 12 B of the source pixel, 12 B written per pixel and pass.
#include "rcp_internal.hpp"

namespace rcp {
namespace {

constexpr int kB = 256;

__device__ inline int edge_index(int i, int n, int edge) {
    if (edge == RCP_EDGE_CLAMP) return i < 0 ? 0 : (i >= n ? n - 1 : i);
    if (edge == RCP_EDGE_WRAP) {
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    // mirror about the border, the border pixel repeated: -1 -> 0, n -> n - 1
    const int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

__global__ __launch_bounds__(kB) void k_gather(const float* __restrict__ in, float* __restrict__ out, int W, int H,
                                                float smudge, int edge, int centred) {
    const uint32_t p = blockIdx.x * kB + threadIdx.x;
    if (p >= (uint32_t)W * (uint32_t)H) return;
    const int y = (int)(p / (uint32_t)W);
    const int x = (int)(p - (uint32_t)y * (uint32_t)W);
    const float r = in[3 * (size_t)p];
    const float g = in[3 * (size_t)p + 1];
    // red moves the sample right, green up (towards row 0)
    const float mr = centred ? 2.0f * r - 1.0f : r;
    const float mg = centred ? 2.0f * g - 1.0f : g;
    const float px = ((float)x + 0.5f) + mr * smudge;
    const float py = ((float)y + 0.5f) - mg * smudge;
    const int sx = edge_index((int)floorf(px), W, edge);
    const int sy = edge_index((int)floorf(py), H, edge);
    const float* src = in + 3 * ((size_t)sy * (size_t)W + (size_t)sx);
    float* dst = out + 3 * (size_t)p;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
}

}  // namespace

rcp_status gather_passes(const float* in, int W, int H, int n, float smudge, int edge, int centred, float* out,
                         hipStream_t stream) {
    const size_t P = (size_t)W * (size_t)H;
    const dim3 grid((unsigned)((P + kB - 1) / kB));
    for (int k = 0; k < n; ++k) {
        const float* src = k == 0 ? in : out + (size_t)(k - 1) * P * 3;
        hipLaunchKernelGGL(k_gather, grid, dim3(kB), 0, stream, src, out + (size_t)k * P * 3, W, H, smudge, edge,
                           centred);
        RCP_CHECK_LAUNCH();
    }
    return RCP_OK;
}

}  // namespace rcp
