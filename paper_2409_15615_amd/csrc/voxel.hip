// Voxel downsampling on a device hash table.
//
// The method takes clouds voxelized with voxel size v (Section III-A).  Every
// finite point gets the FP64 key floor(x / v) per axis; the voxel keeps its
// lowest-index point (atomicMin on the table slot), and kept points are
// compacted in ascending input index by a prefix sum over the kept flags.
#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void voxel_insert(const float* __restrict__ xyz, int n, double v,
                                                       uint64_t* keys, int32_t* mins, uint32_t mask,
                                                       int32_t* __restrict__ slot, DevStatus* st) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float x = xyz[i], y = xyz[n + i], z = xyz[2 * static_cast<int64_t>(n) + i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        slot[i] = -1;
        return;
    }
    // IEEE FP64 division and floor: the same keys as any IEEE implementation.
    double kx = floor(static_cast<double>(x) / v);
    double ky = floor(static_cast<double>(y) / v);
    double kz = floor(static_cast<double>(z) / v);
    if (!key_in_range(kx) || !key_in_range(ky) || !key_in_range(kz)) {
        atomicOr(&st->err_range, 1);
        slot[i] = -1;
        return;
    }
    uint64_t key = pack_key(static_cast<int64_t>(kx), static_cast<int64_t>(ky), static_cast<int64_t>(kz));
    uint32_t h = hash_insert(keys, mask, key);
    atomicMin(mins + h, i);
    slot[i] = static_cast<int32_t>(h);
}

__global__ __launch_bounds__(kBlock) void voxel_mark(const int32_t* __restrict__ slot, const int32_t* mins, int n,
                                                     int32_t* __restrict__ flag) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int h = slot[i];
    flag[i] = (h >= 0 && mins[h] == i) ? 1 : 0;
}

// Writes kept point j = pos[i] (row stride = the kept count m).
__global__ __launch_bounds__(kBlock) void voxel_emit(const float* __restrict__ xyz, int n,
                                                     const int32_t* __restrict__ flag,
                                                     const int32_t* __restrict__ pos, const int64_t* total,
                                                     int64_t cap, int32_t* __restrict__ kept_idx,
                                                     float* __restrict__ kept_xyz) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int64_t m = *total;
    if (m > cap) return;
    const int64_t j = pos[i];
    kept_idx[j] = i;
    kept_xyz[j] = xyz[i];
    kept_xyz[m + j] = xyz[n + i];
    kept_xyz[2 * m + j] = xyz[2 * static_cast<int64_t>(n) + i];
}

struct VoxelWs {
    DevStatus* st;
    uint64_t* keys;
    int32_t* mins;
    int32_t* slot;
    int32_t* flag;
    int32_t* pos;
    int64_t* total;
    int64_t* scan_tmp;
    uint32_t cap_table;
};

VoxelWs carve(Carver& c, int64_t n) {
    VoxelWs w;
    w.cap_table = next_pow2(static_cast<uint64_t>(std::max<int64_t>(2 * n, 64)));
    w.st = c.take<DevStatus>(1);
    w.keys = c.take<uint64_t>(w.cap_table);
    w.mins = c.take<int32_t>(w.cap_table);
    w.slot = c.take<int32_t>(static_cast<size_t>(n));
    w.flag = c.take<int32_t>(static_cast<size_t>(n));
    w.pos = c.take<int32_t>(static_cast<size_t>(n));
    w.total = c.take<int64_t>(2);
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(n));
    return w;
}

}  // namespace

size_t voxelize_ws(int64_t n) {
    Carver c(nullptr, 0);
    carve(c, n);
    return c.off;
}

kmg_status voxelize(const float* xyz, int64_t n, double voxel, int32_t* kept_idx, float* kept_xyz, int64_t cap,
                    int64_t* n_kept_host, void* ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    VoxelWs w = carve(c, n);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.st), 0u, sizeof(DevStatus) / 4, s));
    KMG_TRY(fill_u64(w.keys, kEmptyKey, w.cap_table, s));
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.mins), 0x7fffffffu, w.cap_table, s));
    const int ni = static_cast<int>(n);
    {
    StageScope sc(ST_VOXELIZE, s);
    if (n > 0) {
        voxel_insert<<<grid_for(n, kBlock), kBlock, 0, s>>>(xyz, ni, voxel, w.keys, w.mins, w.cap_table - 1,
                                                           w.slot, w.st);
        KMG_TRY(launch_status());
        voxel_mark<<<grid_for(n, kBlock), kBlock, 0, s>>>(w.slot, w.mins, ni, w.flag);
        KMG_TRY(launch_status());
    }
    KMG_TRY(scan_exclusive(w.flag, w.pos, n, w.total, w.scan_tmp, s));
    if (n > 0) {
        voxel_emit<<<grid_for(n, kBlock), kBlock, 0, s>>>(xyz, ni, w.flag, w.pos, w.total, cap, kept_idx,
                                                         kept_xyz);
        KMG_TRY(launch_status());
    }
    }
    int64_t m = 0;
    DevStatus st;
    KMG_TRY_HIP(hipMemcpyAsync(&m, w.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipMemcpyAsync(&st, w.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    timer_collect();
    if (st.err_range) return KMG_ERR_RANGE;
    *n_kept_host = m;
    if (m > cap) return KMG_ERR_CAPACITY;
    return KMG_OK;
}

}  // namespace kmg
