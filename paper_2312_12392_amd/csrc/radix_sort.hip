// Stable LSD radix sort of (uint64 key, uint32 value) pairs, 8-bit digits.
//
// Each pass: (1) per-tile digit histograms, (2) one exclusive scan over the
// digit-major histogram table, (3) a stable scatter.  In the scatter each
// wave owns a contiguous slice of its tile and walks it in 64-key chunks;
// equal digits inside a chunk are grouped with 8 ballots and ranked with
// mbcnt, so keys keep their input order within each digit.
#include "rcp_internal.hpp"

namespace rcp {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;      // 2048 keys per block
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ inline uint32_t lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(kBlock) void k_digit_hist(const uint64_t* __restrict__ keys, int n,
                                                        int shift, uint32_t* __restrict__ hist,
                                                        int n_tiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long base = (long)blockIdx.x * kTile;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        long i = base + (long)j * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(long)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Block-level exclusive scan of kScanTile elements; writes the block total.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t* __restrict__ data, long n,
                                                        uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t part[kBlock];
    const long base = (long)blockIdx.x * kScanTile + (long)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? data[base + j] : 0u;
        sum += v[j];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele over the 256 partial sums.
    for (int off = 1; off < kBlock; off <<= 1) {
        uint32_t add = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    if (threadIdx.x == kBlock - 1 && block_sums) block_sums[blockIdx.x] = part[kBlock - 1];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) data[base + j] = run;
        run += v[j];
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t* __restrict__ data, long n,
                                                      const uint32_t* __restrict__ block_offsets) {
    const long base = (long)blockIdx.x * kScanTile;
    const uint32_t add = block_offsets[blockIdx.x];
    for (int j = threadIdx.x; j < kScanTile; j += kBlock) {
        long i = base + j;
        if (i < n) data[i] += add;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t* __restrict__ keys_in,
                                                     const uint32_t* __restrict__ vals_in,
                                                     uint64_t* __restrict__ keys_out,
                                                     uint32_t* __restrict__ vals_out, int n, int shift,
                                                     const uint32_t* __restrict__ offsets, int n_tiles) {
    __shared__ uint32_t wcount[kWaves][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * 256; d += kBlock) (&wcount[0][0])[d] = 0;
    __syncthreads();

    const long wbase = (long)blockIdx.x * kTile + (long)wave * (kTile / kWaves);
    uint64_t key[kItems];
    uint32_t val[kItems];
    uint32_t local[kItems];
#pragma unroll
    for (int c = 0; c < kItems; ++c) {
        const long i = wbase + (long)c * 64 + lane;
        const bool valid = i < n;
        key[c] = valid ? keys_in[i] : 0ull;
        val[c] = valid ? vals_in[i] : 0u;
        const uint32_t digit = (uint32_t)(key[c] >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = lanes_below(peers);
        const uint32_t before = wcount[wave][digit];
        local[c] = before + rank;
        // The lowest lane of each digit group bumps the wave's counter after
        // every lane of the chunk has read it.
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcount[wave][digit] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // Exclusive prefix of each digit over the waves of the block.
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            uint32_t t = wcount[w][d];
            wcount[w][d] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kItems; ++c) {
        const long i = wbase + (long)c * 64 + lane;
        if (i < n) {
            const uint32_t digit = (uint32_t)(key[c] >> shift) & 255u;
            const uint32_t pos = offsets[(long)digit * n_tiles + blockIdx.x] + wcount[wave][digit] + local[c];
            keys_out[pos] = key[c];
            vals_out[pos] = val[c];
        }
    }
}

// In-place exclusive scan of n uint32 values (n < 2^31), recursive over tiles.
rcp_status scan_exclusive(uint32_t* data, long n, uint32_t* scratch, hipStream_t stream) {
    const long tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, stream, data, n, (uint32_t*)nullptr);
        RCP_CHECK_LAUNCH();
        return RCP_OK;
    }
    uint32_t* sums = scratch;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kBlock), 0, stream, data, n, sums);
    RCP_CHECK_LAUNCH();
    rcp_status st = scan_exclusive(sums, tiles, scratch + tiles, stream);
    if (st != RCP_OK) return st;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kBlock), 0, stream, data, n,
                       (const uint32_t*)sums);
    RCP_CHECK_LAUNCH();
    return RCP_OK;
}

}  // namespace

size_t scan_scratch_words(long n) { return (size_t)(n / (kScanTile - 1) + 64); }

rcp_status scan_exclusive_u32(uint32_t* data, long n, uint32_t* scratch, hipStream_t stream) {
    if (n <= 0) return RCP_OK;
    return scan_exclusive(data, n, scratch, stream);
}

rcp_status radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* tmp_keys, uint32_t* tmp_vals,
                            int n, int end_bit, hipStream_t stream) {
    if (n <= 1) return RCP_OK;
    const int n_tiles = (n + kTile - 1) / kTile;
    const long hist_n = 256L * n_tiles;
    // histogram table + scan scratch (a geometric series bounded by hist_n / 2047 + levels)
    const long scratch_n = hist_n / (kScanTile - 1) + 64;
    uint32_t* hist = nullptr;
    {
        const rcp_status ast = stream_alloc((void**)&hist, sizeof(uint32_t) * (size_t)(hist_n + scratch_n), stream);
        if (ast != RCP_OK) return ast;
    }
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = tmp_keys;
    uint32_t* vb = tmp_vals;
    rcp_status st = RCP_OK;
    for (int shift = 0; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(k_digit_hist, dim3(n_tiles), dim3(kBlock), 0, stream, (const uint64_t*)ka, n,
                           shift, hist, n_tiles);
        if (hipGetLastError() != hipSuccess) { st = RCP_ERR_DEVICE; break; }
        st = scan_exclusive(hist, hist_n, hist + hist_n, stream);
        if (st != RCP_OK) break;
        hipLaunchKernelGGL(k_scatter, dim3(n_tiles), dim3(kBlock), 0, stream, (const uint64_t*)ka,
                           (const uint32_t*)va, kb, vb, n, shift, (const uint32_t*)hist, n_tiles);
        if (hipGetLastError() != hipSuccess) { st = RCP_ERR_DEVICE; break; }
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    if (st == RCP_OK && ka != keys) {
        if (hipMemcpyAsync(keys, ka, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(vals, va, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
            st = RCP_ERR_DEVICE;
    }
    stream_free(hist, stream);
    hipError_t se = hipStreamSynchronize(stream);
    if (st == RCP_OK && se != hipSuccess) return hip_status(se, "radix sort", __FILE__, __LINE__);
    if (st != RCP_OK) {
        if (st == RCP_ERR_DEVICE) set_error("radix sort: kernel launch failed");
        return st;
    }
    return RCP_OK;
}

}  // namespace rcp
