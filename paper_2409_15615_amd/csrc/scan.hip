// Device-wide exclusive prefix sum (two launches: tile sums, then tile-local
// scans whose blocks each add up the tile sums before them; or one launch
// whose blocks look back at the sums their predecessors publish) and fill
// kernels.
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

__device__ __forceinline__ int64_t live_count(int64_t n, const int32_t* live) {
    if (!live) return n;
    const int64_t l = *live;
    return l < n ? (l < 0 ? 0 : l) : n;
}

__global__ __launch_bounds__(kScanThreads) void tile_sums(const int32_t* in, int64_t n, const int32_t* live,
                                                          int64_t* sums) {
    __shared__ int64_t smem[kScanThreads / kWave];
    const int64_t nl = live_count(n, live);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kScanThreads + threadIdx.x;
        if (i < nl) acc += in[i];
    }
    int64_t excl;
    int64_t total = block_excl_scan(acc, smem, excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Each block sums the tile sums before its own (at most a few thousand, read
// once per block) for its prefix; the last block writes the grand total.
__global__ __launch_bounds__(kScanThreads) void tile_scan(const int32_t* in, int32_t* out, int64_t n,
                                                          const int32_t* live, const int64_t* sums, int64_t* total,
                                                          int32_t* list) {
    __shared__ int64_t smem[kScanThreads / kWave];
    const int64_t nl = live_count(n, live);
    int64_t before = 0;
    for (int64_t k = threadIdx.x; k < static_cast<int64_t>(blockIdx.x); k += kScanThreads) before += sums[k];
    int64_t prefix, unused;
    prefix = block_excl_scan(before, smem, unused);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < nl) ? in[i] : 0;
        acc += v[k];
    }
    int64_t excl;
    const int64_t tile_total = block_excl_scan(acc, smem, excl);
    int64_t run = prefix + excl;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) {
            out[i] = static_cast<int32_t>(run);
            if (list && v[k] == 1) list[run] = static_cast<int32_t>(i);
        }
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = prefix + tile_total;
}

__global__ __launch_bounds__(kScanThreads) void scan_onepass(const int32_t* in, int32_t* out, int64_t n,
                                                             const int32_t* live, uint64_t* status, int64_t* total,
                                                             int32_t* list, int32_t* err) {
    __shared__ int64_t smem[kScanThreads / kWave];
    __shared__ int s_tile;
    __shared__ int64_t s_prefix;
    const int64_t nt = gridDim.x;
    if (threadIdx.x == 0) s_tile = look_back_ticket(status, nt);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t nl = live_count(n, live);
    const int64_t base = tile * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = (i < nl) ? in[i] : 0;
        acc += v[k];
    }
    int64_t excl;
    const int64_t tile_total = block_excl_scan(acc, smem, excl);
    if (threadIdx.x < kWave) {
        const int64_t prefix = look_back(status, tile, tile_total, err);
        if (threadIdx.x == 0) s_prefix = prefix;
    }
    __syncthreads();
    int64_t run = s_prefix + excl;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < n) {
            out[i] = static_cast<int32_t>(run);
            if (list && v[k] == 1) list[run] = static_cast<int32_t>(i);
        }
        run += v[k];
    }
    if (tile == nt - 1 && threadIdx.x == 0) *total = s_prefix + tile_total;
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
                          hipStream_t s, const int32_t* live, int32_t* list) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0) return fill_u64(reinterpret_cast<uint64_t*>(total), 0ull, 1, s);
    tile_sums<<<static_cast<unsigned>(nt), kScanThreads, 0, s>>>(in, n, live, temp);
    KMG_TRY(launch_status());
    tile_scan<<<static_cast<unsigned>(nt), kScanThreads, 0, s>>>(in, out, n, live, temp, total, list);
    return launch_status();
}

kmg_status scan_exclusive_summed(const int32_t* in, int32_t* out, int64_t n, int64_t* total, int64_t* temp,
                                 hipStream_t s) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0) return fill_u64(reinterpret_cast<uint64_t*>(total), 0ull, 1, s);
    tile_scan<<<static_cast<unsigned>(nt), kScanThreads, 0, s>>>(in, out, n, nullptr, temp, total, nullptr);
    return launch_status();
}

kmg_status scan_exclusive_onepass(const int32_t* in, int32_t* out, int64_t n, int64_t* total, uint64_t* status,
                                  int32_t* err, hipStream_t s, const int32_t* live, int32_t* list) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0) return fill_u64(reinterpret_cast<uint64_t*>(total), 0ull, 1, s);
    // past kOnePassMaxTiles the look-back chains cost more than the second launch:
    // the two-launch form, with the words as its tile sums
    if (nt > kOnePassMaxTiles)
        return scan_exclusive(in, out, n, total, reinterpret_cast<int64_t*>(status), s, live, list);
    scan_onepass<<<static_cast<unsigned>(nt), kScanThreads, 0, s>>>(in, out, n, live, status, total, list, err);
    return launch_status();
}

kmg_status fill_u8(uint8_t* p, uint8_t v, size_t n, hipStream_t s) { return fill<uint8_t>(p, v, n, s); }
kmg_status fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) { return fill<uint32_t>(p, v, n, s); }
kmg_status fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) { return fill<uint64_t>(p, v, n, s); }

}  // namespace kmg
