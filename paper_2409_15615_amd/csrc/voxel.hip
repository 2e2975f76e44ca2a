// Voxel downsampling on a device hash table (all clouds of a batch at once).
//
// The method takes clouds voxelized with voxel size v (Section III-A).  Every
// finite point gets the FP64 key floor(x / v) per axis, tagged with its cloud;
// each voxel keeps its lowest-index point (atomicMin on the table slot), and
// kept points are compacted in (cloud, ascending input index) order by a
// prefix sum over the kept flags.
#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;

// Consecutive raw points often share a voxel (a spinning scan lists its
// points along each ring): only the first lane of a run of equal keys on
// consecutive lanes inserts the key and takes the minimum (its index is the
// run's smallest); the others take its slot by a shuffle.
__global__ __launch_bounds__(kBlock) void voxel_insert(const CloudDev* __restrict__ cl, int n_clouds, int64_t n_cap,
                                                       uint64_t* keys, int32_t* mins, uint32_t mask,
                                                       int32_t* __restrict__ slot, DevStatus* st) {
    const int64_t n = clamp_count(st->n_raw, n_cap);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    const int lane = lane_id();
    // every lane of a wave runs the same rounds (the run detection shuffles)
    for (int64_t t0 = static_cast<int64_t>(blockIdx.x) * kBlock + (threadIdx.x & ~(kWave - 1)); t0 < n_cap;
         t0 += stride) {
        const int64_t t = t0 + lane;
        uint64_t key = kEmptyKey;
        if (t < n) {
            const int c = cloud_of_raw(cl, n_clouds, t);
            const int64_t i = t - cl[c].raw_off;
            const int64_t nc = cl[c].n_raw;
            const float* raw = cl[c].raw;
            const float x = raw[i], y = raw[nc + i], z = raw[2 * nc + i];
            if (isfinite(x) && isfinite(y) && isfinite(z)) {
                // IEEE FP64 division and floor: the same keys as any IEEE implementation.
                const double v = cl[c].voxel;
                const double kx = floor(static_cast<double>(x) / v);
                const double ky = floor(static_cast<double>(y) / v);
                const double kz = floor(static_cast<double>(z) / v);
                if (!key_in_range(kx) || !key_in_range(ky) || !key_in_range(kz)) atomicOr(&st->err_range, 1);
                else key = pack_key(c, static_cast<int64_t>(kx), static_cast<int64_t>(ky), static_cast<int64_t>(kz));
            }
        }
        const LaneRun run = lane_run(key);
        int h = -1;
        if (run.head && key != kEmptyKey) {
            h = static_cast<int>(hash_insert(keys, mask, key));
            atomicMin(mins + h, static_cast<int32_t>(t));
        }
        h = __shfl(h, run.lead, kWave);
        if (t < n_cap) slot[t] = key == kEmptyKey ? -1 : h;
    }
}

// One block per scan tile (kScanTile points, eight per thread): the flags and
// the tile's sum for the scan that numbers the kept points.
__global__ __launch_bounds__(kBlock) void voxel_mark(const int32_t* __restrict__ slot, const int32_t* mins,
                                                     int64_t n_cap, int32_t* __restrict__ flag,
                                                     int64_t* __restrict__ tile_sum) {
    static_assert(kScanTile % kBlock == 0, "whole tiles per block");
    __shared__ int s_part[kBlock / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int acc = 0;
#pragma unroll
    for (int k = 0; k < kScanTile / kBlock; ++k) {
        const int64_t t = base + k * kBlock + threadIdx.x;
        if (t < n_cap) {
            const int h = slot[t];
            const int f = (h >= 0 && mins[h] == t) ? 1 : 0;
            flag[t] = f;
            acc += f;
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) tot += s_part[w];
        tile_sum[blockIdx.x] = tot;
    }
}

// voxel_mark and the scan in one launch: the kept flags of a tile of
// kScanTile raw points (eight per thread, in order), the tile's exclusive
// scan (each kept point's index) and the kept count, the tiles chained through
// the look-back words `status` (zeroed beforehand).
__global__ __launch_bounds__(kBlock) void voxel_number(const int32_t* __restrict__ slot, const int32_t* mins,
                                                       int64_t n_cap, int32_t* __restrict__ flag,
                                                       int32_t* __restrict__ pos, uint64_t* status, DevStatus* st) {
    constexpr int kItems = kScanTile / kBlock;
    static_assert(kItems * kBlock == kScanTile, "whole tiles per block");
    __shared__ int64_t s_wave[kBlock / kWave];
    __shared__ int s_tile;
    __shared__ int64_t s_prefix;
    const int64_t nt = gridDim.x;
    if (threadIdx.x == 0) s_tile = look_back_ticket(status, nt);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * kScanTile + static_cast<int64_t>(threadIdx.x) * kItems;
    int f[kItems];
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t t = base + k;
        f[k] = 0;
        if (t < n_cap) {
            const int h = slot[t];
            f[k] = (h >= 0 && mins[h] == t) ? 1 : 0;
            flag[t] = f[k];
        }
        acc += f[k];
    }
    const int wv = threadIdx.x / kWave;
    const int64_t incl = wave_incl_scan(acc);
    if (lane_id() == kWave - 1) s_wave[wv] = incl;
    __syncthreads();
    int64_t before = 0, tile_total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        const int64_t t = s_wave[w];
        if (w < wv) before += t;
        tile_total += t;
    }
    if (threadIdx.x < kWave) {
        const int64_t prefix = look_back(status, tile, tile_total, &st->err_sync);
        if (threadIdx.x == 0) s_prefix = prefix;
    }
    __syncthreads();
    int64_t run = s_prefix + before + incl - acc;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t t = base + k;
        if (t < n_cap) pos[t] = static_cast<int32_t>(run);
        run += f[k];
    }
    if (tile == nt - 1 && threadIdx.x == 0) st->m_kept = s_prefix + tile_total;
}

// Kept point j = pos[t]; row stride `stride` (0: the kept count).  With
// gi.keys, the kept points also go into the cell hash of the radius search
// (what cell_insert does for the kept points in kept order).
__global__ __launch_bounds__(kBlock) void voxel_emit(const CloudDev* __restrict__ cl, int n_clouds, int64_t n_cap,
                                                     const int32_t* __restrict__ flag,
                                                     const int32_t* __restrict__ pos, const DevStatus* st,
                                                     int64_t out_cap, int64_t out_stride,
                                                     int32_t* __restrict__ kept_idx, float* __restrict__ kept_xyz,
                                                     int32_t* __restrict__ kept_cloud, CloudState* cs,
                                                     GridInsert gi) {
    const int64_t n = clamp_count(st->n_raw, n_cap);
    const int64_t m = st->m_kept;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    // per-cloud kept ranges (cs given): the exclusive scan at the cloud's first raw index
    if (cs) {
        for (int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; c < n_clouds; c += stride) {
            const int64_t a = cl[c].raw_off;
            const int64_t b = a + cl[c].n_raw;
            const int64_t ka = a < n ? pos[a] : m;
            const int64_t kb = b < n ? pos[b] : m;
            cs[c].kept_off = static_cast<int32_t>(ka);
            cs[c].kept_cnt = static_cast<int32_t>(kb - ka);
        }
    }
    if (m > out_cap) return;
    const int64_t ks = out_stride ? out_stride : m;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    __shared__ int s_src[kBlock / kWave][kWave];  // packed lane -> kept lane
    // every lane of a wave runs the same rounds (the run detection of the cell insert shuffles)
    for (int64_t t0 = static_cast<int64_t>(blockIdx.x) * kBlock + (threadIdx.x & ~(kWave - 1)); t0 < n;
         t0 += stride) {
        const int64_t t = t0 + lane;
        const bool kept = t < n && flag[t];
        int64_t j = 0;
        uint64_t key = kEmptyKey;
        if (kept) {
            const int c = cloud_of_raw(cl, n_clouds, t);
            const int64_t i = t - cl[c].raw_off;
            const int64_t nc = cl[c].n_raw;
            const float* raw = cl[c].raw;
            j = pos[t];
            const float x = raw[i], y = raw[nc + i], z = raw[2 * nc + i];
            kept_idx[j] = static_cast<int32_t>(i);
            kept_xyz[j] = x;
            kept_xyz[ks + j] = y;
            kept_xyz[2 * ks + j] = z;
            if (kept_cloud) kept_cloud[j] = c;
            if (gi.keys) {
                const double inv_c = cl[c].inv_cell;
                const double kx = floor(static_cast<double>(x) * inv_c);
                const double ky = floor(static_cast<double>(y) * inv_c);
                const double kz = floor(static_cast<double>(z) * inv_c);
                // one cell of headroom, so that the 27-cell stencil stays packable
                if (!key_in_range(kx - 1) || !key_in_range(kx + 1) || !key_in_range(ky - 1) ||
                    !key_in_range(ky + 1) || !key_in_range(kz - 1) || !key_in_range(kz + 1))
                    atomicOr(&gi.st->err_range, 1);
                else
                    key = pack_key(c, static_cast<int64_t>(kx), static_cast<int64_t>(ky),
                                   static_cast<int64_t>(kz));
            }
        }
        if (gi.keys) {
            // the kept lanes' keys packed to the front of the wave in lane order, so
            // that the lanes of dropped points do not break up the runs of one cell;
            // a run inserts once
            const uint64_t live = ballot(key != kEmptyKey);
            const int n_live = __popcll(live);
            const int rank = __popcll(live & ((1ull << lane) - 1ull));
            if (key != kEmptyKey) s_src[wv][rank] = lane;
            __builtin_amdgcn_wave_barrier();
            const int src = lane < n_live ? s_src[wv][lane] : lane;
            const uint64_t packed = __shfl(key, src, kWave);
            const uint64_t ckey = lane < n_live ? packed : kEmptyKey;
            const LaneRun run = lane_run(ckey);
            int h = -1;
            if (run.head && ckey != kEmptyKey) {
                h = static_cast<int>(hash_insert(gi.keys, gi.mask, ckey));
                atomicAdd(gi.cnt + h, run.len);
            }
            h = __shfl(h, run.lead, kWave);  // the run's slot, in packed lanes
            h = __shfl(h, rank, kWave);      // back to the kept lane
            if (kept) gi.pslot[j] = key == kEmptyKey ? -1 : h;
            __builtin_amdgcn_wave_barrier();  // s_src is free for the next round
        }
    }
}

// Per-cloud kept ranges: the exclusive scan at the cloud's first raw index
// (voxel_emit writes them itself when it runs).
__global__ void cloud_ranges(const CloudDev* __restrict__ cl, int n_clouds, int64_t n_cap,
                             const int32_t* __restrict__ pos, const DevStatus* st, CloudState* cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_clouds) return;
    const int64_t n = clamp_count(st->n_raw, n_cap);
    const int64_t m = st->m_kept;
    const int64_t a = cl[c].raw_off;
    const int64_t b = a + cl[c].n_raw;
    const int64_t ka = a < n ? pos[a] : m;
    const int64_t kb = b < n ? pos[b] : m;
    cs[c].kept_off = static_cast<int32_t>(ka);
    cs[c].kept_cnt = static_cast<int32_t>(kb - ka);
}

}  // namespace

VoxelWs carve_voxel(Carver& c, int64_t n_cap) {
    VoxelWs w;
    w.cap_table = next_pow2(static_cast<uint64_t>(std::max<int64_t>(2 * n_cap, 64)));
    w.keys = c.take<uint64_t>(w.cap_table);
    w.mins = c.take<int32_t>(w.cap_table);
    w.slot = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(n_cap, 1)));
    w.flag = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(n_cap, 1)));
    w.pos = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(n_cap, 1)));
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(n_cap));
    return w;
}

kmg_status voxelize_batch(const CloudDev* cl, int n_clouds, int64_t n_cap, DevStatus* st, const VoxelWs& w,
                          int64_t out_cap, int64_t out_stride, int32_t* kept_idx, float* kept_xyz,
                          int32_t* kept_cloud, CloudState* cs, hipStream_t s, bool cleared,
                          const GridInsert* grid, uint64_t* scan_status) {
    StageScope sc(ST_VOXELIZE, s);
    if (!cleared) {
        KMG_TRY(fill_u64(w.keys, kEmptyKey, w.cap_table, s));
        KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.mins), 0x7fffffffu, w.cap_table, s));
    }
    if (n_cap > 0) {
        voxel_insert<<<grid_cap(n_cap, kBlock), kBlock, 0, s>>>(cl, n_clouds, n_cap, w.keys, w.mins,
                                                               w.cap_table - 1, w.slot, st);
        KMG_TRY(launch_status());
        const unsigned nt = static_cast<unsigned>((n_cap + kScanTile - 1) / kScanTile);
        if (nt > kOnePassMaxTiles) scan_status = nullptr;  // long look-back chains: two launches
        if (scan_status) {
            voxel_number<<<nt, kBlock, 0, s>>>(w.slot, w.mins, n_cap, w.flag, w.pos, scan_status, st);
        } else {
            voxel_mark<<<nt, kBlock, 0, s>>>(w.slot, w.mins, n_cap, w.flag, w.scan_tmp);
        }
        KMG_TRY(launch_status());
    }
    if (!scan_status || n_cap <= 0)
        KMG_TRY(scan_exclusive_summed(w.flag, w.pos, n_cap, &st->m_kept, w.scan_tmp, s));
    if (n_cap > 0) {
        voxel_emit<<<grid_cap(n_cap, kBlock), kBlock, 0, s>>>(cl, n_clouds, n_cap, w.flag, w.pos, st, out_cap,
                                                             out_stride, kept_idx, kept_xyz, kept_cloud, cs,
                                                             grid ? *grid : GridInsert{});
        KMG_TRY(launch_status());
    } else if (cs) {
        cloud_ranges<<<grid_for(n_clouds, 256), 256, 0, s>>>(cl, n_clouds, n_cap, w.pos, st, cs);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

}  // namespace kmg
