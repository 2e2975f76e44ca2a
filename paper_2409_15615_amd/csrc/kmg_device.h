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

__device__ __forceinline__ uint64_t pack_key(int64_t kx, int64_t ky, int64_t kz) {
    return (static_cast<uint64_t>(kx + kKeyBias) << 42) | (static_cast<uint64_t>(ky + kKeyBias) << 21) |
           static_cast<uint64_t>(kz + kKeyBias);
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

// Strict radius test d2 < r^2: an FP32 screen decides everything farther than
// a relative band of 4e-6 from the sphere (the FP32 error is below 1e-6
// relative); inside the band the FP64 expression above decides.
struct RadiusTest {
    float lo2, hi2;  // FP32 band edges around r^2
    double r2;       // r * r in FP64
    __device__ __forceinline__ bool operator()(float qx, float qy, float qz, float sx, float sy, float sz) const {
        float dx = sx - qx, dy = sy - qy, dz = sz - qz;
        float d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < lo2) return true;
        if (d2 > hi2) return false;
        return d2_exact(qx, qy, qz, sx, sy, sz) < r2;
    }
};

inline RadiusTest make_radius_test(double r) {
    RadiusTest t;
    t.r2 = r * r;
    t.lo2 = static_cast<float>(t.r2 * (1.0 - 4e-6));
    t.hi2 = static_cast<float>(t.r2 * (1.0 + 4e-6));
    return t;
}

}  // namespace kmg
