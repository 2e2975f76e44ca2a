// Device-side helpers shared by the libkmg kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kmg_internal.h"

namespace kmg {

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & (kWave - 1)); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Global wave index and wave count of a grid-stride kernel.
__device__ __forceinline__ int global_wave() {
    return static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
}
__device__ __forceinline__ int wave_count() { return static_cast<int>(gridDim.x * blockDim.x / kWave); }

// XCD-aware split of items [0, n) over the wavefronts of a launch, balanced
// by work.  The blocks of a launch are dealt to the eight XCDs in turn (block
// b runs on XCD b % 8; the grid G is a multiple of 8), so XCD x takes the
// items whose work prefix start(i) (non-decreasing, total `work`) lies in
// [x work / 8, (x + 1) work / 8), and its wavefronts deal those out in turn
// (item first + k stride).  Items in input order are spatially coherent (a
// scan lists its points ring by ring), so each XCD's L2 then holds the
// neighbourhood of its own eighth rather than of the whole cloud.
constexpr int kXcds = 8;
struct XcdItems {
    int64_t first, end, stride;
};
// Wavefront index of the launch in the XCD-aware order: the waves of XCD x
// (blocks b with b % 8 == x) take indices [x W / 8, (x + 1) W / 8) of the W
// waves, in block order.
__device__ __forceinline__ int64_t xcd_block_index() {
    const int64_t G = gridDim.x;
    const int64_t b = blockIdx.x;
    return (G % kXcds == 0) ? (b % kXcds) * (G / kXcds) + b / kXcds : b;
}
__device__ __forceinline__ int64_t xcd_wave_index() {
    return xcd_block_index() * (blockDim.x / kWave) + threadIdx.x / kWave;
}

// The plain split: item i to wavefront i mod (wavefronts of the launch).
__device__ __forceinline__ XcdItems cyclic_items(int64_t n) {
    return XcdItems{static_cast<int64_t>(global_wave()), n, static_cast<int64_t>(wave_count())};
}
template <class F>
__device__ __forceinline__ XcdItems xcd_items(int64_t n, int64_t work, F start) {
    const int64_t G = gridDim.x;
    const int64_t wpb = blockDim.x / kWave;
    const int64_t wv = threadIdx.x / kWave;
    if (G % kXcds != 0 || n <= 0) return XcdItems{blockIdx.x * wpb + wv, n, G * wpb};
    const int64_t x = blockIdx.x % kXcds;
    // first item whose start reaches t: a 64-way search by the wavefront
    auto first_at = [&](int64_t t) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {  // uniform over the wave
            const int64_t step = (hi - lo + kWave - 1) / kWave;
            const int64_t probe = lo + (lane_id() + 1) * step - 1;
            const bool b = probe < hi && start(probe) < t;
            const int cnt = __popcll(ballot(b));
            const int64_t nlo = lo + cnt * step;
            hi = min(hi, lo + (cnt + 1) * step - 1);
            lo = nlo;
        }
        return lo;
    };
    const int64_t b0 = x == 0 ? 0 : first_at((work * x) / kXcds);
    const int64_t b1 = x == kXcds - 1 ? n : first_at((work * (x + 1)) / kXcds);
    return XcdItems{b0 + (blockIdx.x / kXcds) * wpb + wv, b1, (G / kXcds) * wpb};
}

// 64-bit mixing function (the MurmurHash3 fmix64 finaliser).
__device__ __forceinline__ uint32_t hash_key(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return static_cast<uint32_t>(k);
}

__device__ __forceinline__ bool key_in_range(double k) {
    return k >= -static_cast<double>(kKeyBias) && k < static_cast<double>(kKeyBias);
}

// 10 bits of cloud id, then 18 bits per axis.
__device__ __forceinline__ uint64_t pack_key(int cloud, int64_t kx, int64_t ky, int64_t kz) {
    return (static_cast<uint64_t>(cloud) << (3 * kAxisBits)) |
           (static_cast<uint64_t>(kx + kKeyBias) << (2 * kAxisBits)) |
           (static_cast<uint64_t>(ky + kKeyBias) << kAxisBits) | static_cast<uint64_t>(kz + kKeyBias);
}

// Open-addressing lookup; returns the slot or -1.
__device__ __forceinline__ int hash_find(const uint64_t* keys, uint32_t mask, uint64_t key) {
    uint32_t h = hash_key(key) & mask;
    while (true) {
        uint64_t k = keys[h];
        if (k == key) return static_cast<int>(h);
        if (k == kEmptyKey) return -1;
        h = (h + 1) & mask;
    }
}

// Open-addressing insert (the table always has a free slot); returns the slot.
__device__ __forceinline__ uint32_t hash_insert(uint64_t* keys, uint32_t mask, uint64_t key) {
    uint32_t h = hash_key(key) & mask;
    while (true) {
        unsigned long long prev =
            atomicCAS(reinterpret_cast<unsigned long long*>(keys + h), static_cast<unsigned long long>(kEmptyKey),
                      static_cast<unsigned long long>(key));
        if (prev == kEmptyKey || prev == key) return h;
        h = (h + 1) & mask;
    }
}

// Squared distance exactly as ((dx*dx) + dy*dy) + dz*dz in FP64 with
// dx = (double)x_s - (double)x_q, every operation rounded separately.
__device__ __forceinline__ double d2_exact(float qx, float qy, float qz, float sx, float sy, float sz) {
#pragma clang fp contract(off)
    double dx = static_cast<double>(sx) - static_cast<double>(qx);
    double dy = static_cast<double>(sy) - static_cast<double>(qy);
    double dz = static_cast<double>(sz) - static_cast<double>(qz);
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    return d2;
}

__device__ __forceinline__ bool in_radius(const RadiusTest& t, float qx, float qy, float qz, float sx, float sy,
                                          float sz) {
    const float dx = sx - qx, dy = sy - qy, dz = sz - qz;
    const float d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < t.lo2) return true;
    if (d2 > t.hi2) return false;
    return d2_exact(qx, qy, qz, sx, sy, sz) < t.r2;
}

// Cloud of a raw index: the last cloud whose raw_off <= t.
__device__ __forceinline__ int cloud_of_raw(const CloudDev* cl, int n_clouds, int64_t t) {
    int lo = 0, hi = n_clouds - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cl[mid].raw_off <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t clamp_count(int64_t v, int64_t cap) { return v < cap ? v : cap; }

// List-first radius search: each list of at most this many entries sits in
// row q of a pad of pad_cap entries (the rows share the pad evenly among the
// m kept points, in whole 128-byte lines once a row holds one); longer lists
// sit at their CSR places.
__device__ __forceinline__ int pad_stride(int64_t pad_cap, int64_t m) {
    const int r = m > 0 ? static_cast<int>(min<int64_t>(kListSmall, pad_cap / m)) : 0;
    return r >= 32 ? (r & ~31) : r;
}

// First entry of point q's list (CSR range [b, e)); row = pad_stride(...).
__device__ __forceinline__ const int32_t* list_of(const NbrLists& L, int row, int64_t q, int b, int e) {
    return (L.pad && e - b <= row) ? L.pad + q * row : L.nbr + b;
}

// Runs of equal keys on consecutive lanes (a lane with key kEmptyKey is a run
// of its own).  The whole wavefront must be active.  head: this lane starts a
// run; lead: the first lane of this lane's run; len: the run's lane count
// (meaningful on the head).
struct LaneRun {
    bool head;
    int lead;
    int len;
};
__device__ __forceinline__ LaneRun lane_run(uint64_t key) {
    const int lane = lane_id();
    const uint64_t prev = __shfl_up(key, 1, kWave);
    const bool head = lane == 0 || key == kEmptyKey || key != prev;
    const uint64_t heads = ballot(head);
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    LaneRun r;
    r.head = head;
    r.lead = 63 - __clzll(static_cast<long long>(heads & upto));
    const uint64_t above = heads & ~upto;
    r.len = (above ? __ffsll(static_cast<unsigned long long>(above)) - 1 : kWave) - lane;
    return r;
}

// Decoupled look-back for one-launch prefix sums over tiles.  status[t] of
// tile t: 0 until the tile's block publishes its own sum (kAggregate) and then
// the sum of every tile up to and including it (kInclusive), in the low 62
// bits; status[nt] hands out the tiles in launch order (look_back_ticket), so
// a block only ever waits on tiles whose blocks are running already.  The
// caller zeroes status[0 .. nt] before the launch.
constexpr uint64_t kAggregate = 1ull << 62;
constexpr uint64_t kInclusive = 2ull << 62;
constexpr uint64_t kScanValue = (1ull << 62) - 1;
constexpr uint32_t kLookSpinLimit = 1u << 18;  // a bounded wait (never reached in practice)
constexpr int kLookBack = 4;                    // 64-tile slots per lane and look-back window

__device__ __forceinline__ int look_back_ticket(uint64_t* status, int64_t nt) {
    return static_cast<int>(atomicAdd(reinterpret_cast<unsigned long long*>(status + nt), 1ull));
}

// Called by one whole wavefront of the tile's block: publishes the tile's sum,
// returns (to every lane) the sum of the tiles before it and publishes the
// inclusive sum.  The predecessors are read kLookBack x 64 at a time, nearest
// first (lane l, slot u: tile hi - l - 64 u), down to the nearest inclusive
// sum; tiles before 0 count as an inclusive 0.  A wait that gives up (never
// expected) sets *err and counts the tile as 0.
__device__ __forceinline__ int64_t look_back(uint64_t* status, int64_t tile, int64_t tile_total, int32_t* err) {
    const int lane = lane_id();
    if (lane == 0)
        __hip_atomic_store(status + tile, static_cast<uint64_t>(tile_total) | (tile == 0 ? kInclusive : kAggregate),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t prefix = 0;
    for (int64_t hi = tile - 1; hi >= 0; hi -= kLookBack * kWave) {
        uint64_t w[kLookBack];
#pragma unroll
        for (int u = 0; u < kLookBack; ++u) {
            const int64_t j = hi - lane - u * kWave;
            w[u] = j >= 0 ? __hip_atomic_load(status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kInclusive;
        }
        for (uint32_t spins = 0;; ++spins) {
            bool pending = false;
#pragma unroll
            for (int u = 0; u < kLookBack; ++u) pending |= (w[u] >> 62) == 0;
            if (!pending) break;
            if (spins > kLookSpinLimit) {
                atomicOr(err, 1);
#pragma unroll
                for (int u = 0; u < kLookBack; ++u)
                    if ((w[u] >> 62) == 0) w[u] = kInclusive;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int u = 0; u < kLookBack; ++u)
                if ((w[u] >> 62) == 0)
                    w[u] = __hip_atomic_load(status + (hi - lane - u * kWave), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        }
        int found = kLookBack, last = kWave - 1;
#pragma unroll
        for (int u = kLookBack - 1; u >= 0; --u) {
            const uint64_t incl = ballot((w[u] >> 62) == 2);
            if (incl) {
                found = u;
                last = __ffsll(static_cast<unsigned long long>(incl)) - 1;
            }
        }
        int64_t add = 0;
#pragma unroll
        for (int u = 0; u < kLookBack; ++u)
            if (u < found || (u == found && lane <= last)) add += static_cast<int64_t>(w[u] & kScanValue);
        prefix += wave_sum(add);
        if (found < kLookBack) break;
    }
    if (lane == 0 && tile > 0)
        __hip_atomic_store(status + tile, static_cast<uint64_t>(prefix + tile_total) | kInclusive, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return prefix;
}

}  // namespace kmg
