// Device-wide exclusive prefix sum (three launches: tile sums, scan of the
// tile sums, tile-local scans) and fill kernels.
#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = kScanTile / kScanThreads;  // 8

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ int64_t block_excl_scan(int64_t v, int64_t* smem /* >= 4 */, int64_t& excl) {
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    int64_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) smem[wave] = incl;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        int64_t t = smem[w];
        if (w < wave) before += t;
        total += t;
    }
    excl = before + incl - v;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kScanThreads) void tile_sums(const int32_t* in, int64_t n, int64_t* sums) {
    __shared__ int64_t smem[kScanThreads / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kScanThreads + threadIdx.x;
        if (i < n) acc += in[i];
    }
    int64_t excl;
    int64_t total = block_excl_scan(acc, smem, excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block: exclusive scan of the tile sums in place; writes the grand total.
__global__ __launch_bounds__(kScanThreads) void scan_sums(int64_t* sums, int64_t nt, int64_t* total) {
    __shared__ int64_t smem[kScanThreads / kWave];
    int64_t carry = 0;
    for (int64_t base = 0; base < nt; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        int64_t v = (i < nt) ? sums[i] : 0;
        int64_t excl;
        int64_t t = block_excl_scan(v, smem, excl);
        if (i < nt) sums[i] = carry + excl;
        carry += t;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void tile_scan(const int32_t* in, int32_t* out, int64_t n,
                                                          const int64_t* sums) {
    __shared__ int64_t smem[kScanThreads / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        acc += v[k];
    }
    int64_t excl;
    block_excl_scan(acc, smem, excl);
    int64_t run = sums[blockIdx.x] + excl;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = static_cast<int32_t>(run);
        run += v[k];
    }
}

template <class T>
__global__ void fill_kernel(T* p, T v, size_t n) {
    size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <class T>
kmg_status fill(T* p, T v, size_t n, hipStream_t s) {
    if (n == 0) return KMG_OK;
    unsigned blocks = static_cast<unsigned>(std::min<size_t>((n + 255) / 256, 4096));
    fill_kernel<T><<<blocks, 256, 0, s>>>(p, v, n);
    return launch_status();
}

}  // namespace

size_t scan_temp_elems(int64_t n) { return static_cast<size_t>((n + kScanTile - 1) / kScanTile) + 1; }

kmg_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int64_t* total, int64_t* temp,
                          hipStream_t s) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt > 0) {
        tile_sums<<<static_cast<unsigned>(nt), kScanThreads, 0, s>>>(in, n, temp);
        KMG_TRY(launch_status());
    }
    scan_sums<<<1, kScanThreads, 0, s>>>(temp, nt, total);
    KMG_TRY(launch_status());
    if (nt > 0) {
        tile_scan<<<static_cast<unsigned>(nt), kScanThreads, 0, s>>>(in, out, n, temp);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

kmg_status fill_u8(uint8_t* p, uint8_t v, size_t n, hipStream_t s) { return fill<uint8_t>(p, v, n, s); }
kmg_status fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) { return fill<uint32_t>(p, v, n, s); }
kmg_status fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) { return fill<uint64_t>(p, v, n, s); }

}  // namespace kmg
