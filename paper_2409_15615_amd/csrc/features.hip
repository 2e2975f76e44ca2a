// Algorithm 1 Step 2, Darboux-frame pair features (Eq. A2), bins (Eq. A3),
// SPFH (Eq. A4) and FPFH (Eq. A5).
//
// All clouds of a batch are processed by the same launches (grid-stride over
// the kept points; each point reads its cloud's tau_num).
//
// SPFH: one wavefront per point q; lanes take the neighbours k of q, 64 at a
// time.  Each lane computes the three features of (q, k) in FP32 and bins
// them; a feature set that lies within a guard band of a bin edge or of an
// ill-conditioned frame, or near the a/b selection tie with the two role
// assignments binning differently, is recomputed in FP64 with the operation
// order of the plain definition, so the bins equal the FP64 definition's.
// Bin counts are formed with one ballot + popcount per (feature, bin): no
// atomics, deterministic.  The FPFH pass keeps the counts (uint16, 66 bytes
// per row of 33) and 100 / P_q per point, not the FP64 SPFH values: the
// gather of a neighbour's row moves a quarter of the bytes.
//
// FPFH: one wavefront per point q in J; lanes first compute the weights
// (1 / ||a_k - a_q||) (100 / P_k) of a chunk of neighbours (FP64) and compact
// them into LDS, then each lane owns descriptor bins and accumulates weight x
// count over the chunk in ascending k, in FP64 (the term (1 / w_k) SPFH(k) of
// Eq. A5); the query's own SPFH value is 100 c / P_q, divided exactly.
#include <math.h>

#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;
// Work of a point in the XCD split, in list entries: its fixed cost (the list
// bounds, its own row and the dependent loads before the first neighbour) plus
// one per neighbour.
constexpr int64_t kItemWork = 32;
constexpr int kWaves = kBlock / kWave;
constexpr int kBatch = 8;          // SPFH rows loaded together in the FPFH sum

struct V3f {
    float x, y, z;
};

__device__ __forceinline__ V3f sub(V3f a, V3f b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ float dotf(V3f a, V3f b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3f crossf(V3f a, V3f b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3f scalef(V3f a, float s) { return {a.x * s, a.y * s, a.z * s}; }

// FP32 features and bins for a given role assignment (qa: a = q, b = k).
// Returns false when a decision is too close to call in FP32: a short frame
// axis (||d x u|| < 0.2), a near-degenerate f1 argument (|(w.n_b, u.n_b)| <
// 0.2), or a scaled feature within 2e-4 of an integer.  The FP32 error of the
// scaled features is below 2e-5 outside those cases.
__device__ __forceinline__ bool bins_f32_roles(V3f d0, float dl, V3f nq, V3f nk, bool qa, int H, int bins[3]) {
    const V3f u = qa ? nq : nk;
    const V3f nb = qa ? nk : nq;
    const V3f d = scalef(d0, (qa ? 1.0f : -1.0f) / dl);
    V3f v = crossf(d, u);
    const float vl = sqrtf(dotf(v, v));
    if (vl < 0.2f) return false;
    v = scalef(v, 1.0f / vl);
    const V3f w = crossf(u, v);
    const float y = dotf(w, nb), x = dotf(u, nb);
    if (x * x + y * y < 0.04f) return false;
    const float f[3] = {atan2f(y, x), dotf(v, nb), dotf(u, d)};
    const float lo[3] = {-3.14159265358979323846f, -1.0f, -1.0f};
    const float sc[3] = {H / 6.28318530717958647692f, 0.5f * H, 0.5f * H};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const float s = (f[l] - lo[l]) * sc[l];
        if (fabsf(s - rintf(s)) < 2e-4f) return false;
        bins[l] = min(max(static_cast<int>(floorf(s)), 0), H - 1);
    }
    return true;
}

// FP32 features and bins.  The a/b roles follow the unsigned angle; when
// |n_q.d0| and |n_k.d0| lie within 1e-5 ||d0|| of each other (coplanar
// neighbours with nearly equal normals, the common case on planes) both role
// assignments are evaluated, and if both are reliable and give the same bins,
// the bins are those of either FP64 decision.  Returns false when the FP64
// path has to decide.
__device__ __forceinline__ bool bins_f32(V3f pq, V3f nq, V3f pk, V3f nk, int H, int bins[3]) {
    const V3f d0 = sub(pk, pq);
    const float aq = fabsf(dotf(nq, d0));
    const float ak = fabsf(dotf(nk, d0));
    const float dl = sqrtf(dotf(d0, d0));
    if (fabsf(aq - ak) > 1e-5f * dl) return bins_f32_roles(d0, dl, nq, nk, aq >= ak, H, bins);
    int other[3];
    if (!bins_f32_roles(d0, dl, nq, nk, true, H, bins)) return false;
    if (!bins_f32_roles(d0, dl, nq, nk, false, H, other)) return false;
    return bins[0] == other[0] && bins[1] == other[1] && bins[2] == other[2];
}

__device__ __forceinline__ double dotd(const double a[3], const double b[3]) {
#pragma clang fp contract(off)
    double s = a[0] * b[0];
    s = s + a[1] * b[1];
    s = s + a[2] * b[2];
    return s;
}

__device__ __forceinline__ void crossd(const double a[3], const double b[3], double o[3]) {
#pragma clang fp contract(off)
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// FP64 features and bins by the plain definition: a/b by the unsigned
// angle, d = (a_b - a_a) / ||.||, u = n_a, v = d x u normalised, w = u x v,
// f = (atan2(w.n_b, u.n_b), v.n_b, u.d); f = (0, 0, u.d) when d x u = 0.
// Bin h = floor(H (f - lo) / (hi - lo)) clamped to [0, H-1].
// Out of line: the FP64 recomputation is rare, and inlined it would hold the
// registers of the whole SPFH loop.  The bins come back by value (in
// registers), so the caller's bins never live in scratch memory.
struct BinsF64 {
    int b[3];
    int edge;  // some feature within 1e-9 bins of a bin edge
};
__device__ __attribute__((noinline)) BinsF64 bins_f64(V3f pq32, V3f nq32, V3f pk32, V3f nk32, int H) {
#pragma clang fp contract(off)
    BinsF64 r;
    r.edge = 0;
    const double nq[3] = {nq32.x, nq32.y, nq32.z}, nk[3] = {nk32.x, nk32.y, nk32.z};
    const double d0[3] = {static_cast<double>(pk32.x) - pq32.x, static_cast<double>(pk32.y) - pq32.y,
                          static_cast<double>(pk32.z) - pq32.z};
    const bool qa = fabs(dotd(nq, d0)) >= fabs(dotd(nk, d0));
    // a, b and their normals by value selects (no pointers to local arrays)
    const double pa[3] = {qa ? pq32.x : pk32.x, qa ? pq32.y : pk32.y, qa ? pq32.z : pk32.z};
    const double pb[3] = {qa ? pk32.x : pq32.x, qa ? pk32.y : pq32.y, qa ? pk32.z : pq32.z};
    const double u[3] = {qa ? nq[0] : nk[0], qa ? nq[1] : nk[1], qa ? nq[2] : nk[2]};
    const double nb[3] = {qa ? nk[0] : nq[0], qa ? nk[1] : nq[1], qa ? nk[2] : nq[2]};
    double d[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
    const double dl = sqrt(dotd(d, d));
    for (int c = 0; c < 3; ++c) d[c] = d[c] / dl;
    double v[3];
    crossd(d, u, v);
    const double vl = sqrt(dotd(v, v));
    double f[3];
    if (vl == 0.0) {
        f[0] = 0.0;
        f[1] = 0.0;
        f[2] = dotd(u, d);
    } else {
        for (int c = 0; c < 3; ++c) v[c] = v[c] / vl;
        double w[3];
        crossd(u, v, w);
        f[0] = atan2(dotd(w, nb) + 0.0, dotd(u, nb));
        f[1] = dotd(v, nb);
        f[2] = dotd(u, d);
    }
    const double lo[3] = {-M_PI, -1.0, -1.0};
    const double hi[3] = {M_PI, 1.0, 1.0};
    for (int l = 0; l < 3; ++l) {
        const double s = (static_cast<double>(H) * (f[l] - lo[l])) / (hi[l] - lo[l]);
        const double fl = floor(s);
        if (fabs(s - fl) < 1e-9 || fabs(s - (fl + 1.0)) < 1e-9) r.edge = 1;
        r.b[l] = min(max(static_cast<int>(fl), 0), H - 1);
    }
    return r;
}

// SPFH value of a bin (Eq. A4): 100 * count / P_q in FP64, 0 when P_q = 0.
__device__ __forceinline__ double spfh_value(int count, int P) {
    return P > 0 ? (100.0 * static_cast<double>(count)) / static_cast<double>(P) : 0.0;
}

__device__ __forceinline__ int cloud_of(const int32_t* kept_cloud, int64_t q) {
    return kept_cloud ? kept_cloud[q] : 0;
}

// Lists of a mean of at most kHalfListMean entries per point: two points per
// wavefront, one per half of 32 lanes (each lane one neighbour of its half's
// point per round, adding its three bins to the half's LDS histogram with
// integer atomics; lane h of a half then reads bin h).  Longer lists:
// spfh_kernel, one point per wavefront.  Each kernel checks the mean and
// returns at once when the other one serves it
// (one kernel holding both bodies was measured slower: its one-wave body runs
// slower than alone, 64.7 -> 70.5 us for the pass on the LiDAR pair, more than
// the launch it saves).  The threshold is measured: the 64-pair batch (mean
// 22.5) runs 1.5x faster in pairs, the LiDAR pair (mean 29, but a long tail of
// structure points next to scattered outliers with a few neighbours) 8% slower.
constexpr int kHalfListMean = 24;  // the default of tuning().spfh_pair_mean

__device__ __forceinline__ void spfh_pairs_body(const CloudDev* __restrict__ cl, const float* __restrict__ xyz,
                                           int64_t stride, const int32_t* __restrict__ kept_cloud, int64_t m,
                                           const float* __restrict__ nrm, int64_t nrm_stride,
                                           const uint8_t* __restrict__ flags, const int32_t* __restrict__ off,
                                           NbrLists nb, int H, uint16_t* __restrict__ cnt16,
                                           float* __restrict__ spfh_out, int32_t* __restrict__ Pq,
                                           double* __restrict__ inv100, int32_t* __restrict__ jflag, int xcd,
                                           DevStatus* st, uint32_t* s_hist) {
    constexpr int kHalf = kWave / 2;
    const int lane = lane_id();
    const int hf = lane / kHalf, hl = lane % kHalf, sh = kHalf * hf;
    const int D = 3 * H;
    const int64_t s2 = 2 * stride, n2 = 2 * nrm_stride;
    uint32_t n64 = 0, nedge = 0;
    const int prow = nb.pad ? pad_stride(nb.pad_cap, m) : 0;
    const XcdItems it = xcd ? xcd_items((m + 1) / 2, off[m] + kItemWork * m,
                                        [&](int64_t i) { return off[2 * i] + kItemWork * 2 * i; })
                            : cyclic_items((m + 1) / 2);
    for (int64_t pw = it.first; pw < it.end; pw += it.stride) {
        const int64_t q = 2 * pw + hf;
        const bool live = q < m;
        const bool has_b = live && (flags[q] & 1);
        V3f pq = {0.f, 0.f, 0.f}, nq = {0.f, 0.f, 0.f};
        int b = 0, e = 0;
        if (has_b) {
            pq = {xyz[q], xyz[stride + q], xyz[s2 + q]};
            nq = {nrm[q], nrm[nrm_stride + q], nrm[n2 + q]};
            b = off[q];
            e = off[q + 1];
        }
        const int len = e - b;
        const int32_t* lp = list_of(nb, prow, q, b, e);
        const int lmax = max(len, __shfl_xor(len, kHalf, kWave));
        int n_valid = 0;
        // the half's histogram in LDS (3H counters), one atomic per lane and feature
        uint32_t* hist = s_hist + hf * 3 * kMaxBins;
        for (int t = hl; t < D; t += kHalf) hist[t] = 0u;
        __builtin_amdgcn_wave_barrier();
        for (int base = 0; base < lmax; base += kHalf) {
            bool valid = false;
            int bn[3] = {-1, -1, -1};
            if (base + hl < len) {
                const int k = lp[base + hl];
                valid = (flags[k] & 1) != 0;
                if (valid && k != q) {
                    const V3f pk = {xyz[k], xyz[stride + k], xyz[s2 + k]};
                    const V3f nk = {nrm[k], nrm[nrm_stride + k], nrm[n2 + k]};
                    if (!bins_f32(pq, nq, pk, nk, H, bn)) {
                        const BinsF64 r = bins_f64(pq, nq, pk, nk, H);
                        bn[0] = r.b[0];
                        bn[1] = r.b[1];
                        bn[2] = r.b[2];
                        ++n64;
                        nedge += r.edge ? 1u : 0u;
                    }
                }
            }
            n_valid += __popc(static_cast<uint32_t>(ballot(valid) >> sh));
            if (bn[0] >= 0) {
                atomicAdd(hist + bn[0], 1u);
                atomicAdd(hist + H + bn[1], 1u);
                atomicAdd(hist + 2 * H + bn[2], 1u);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // lane h of a half holds the counts of bin h for the three features
        int c0 = 0, c1 = 0, c2 = 0;
        if (hl < H) {
            c0 = static_cast<int>(hist[hl]);
            c1 = static_cast<int>(hist[H + hl]);
            c2 = static_cast<int>(hist[2 * H + hl]);
        }
        __builtin_amdgcn_wave_barrier();  // the histogram is free for the next pair of points
        if (!live) continue;
        uint16_t* row = cnt16 + q * spfh_row(H);
        if (!has_b) {
            for (int t = hl; t < D; t += kHalf) {
                row[t] = 0;
                if (spfh_out) spfh_out[q * D + t] = 0.0f;
            }
            if (hl == 0) {
                Pq[q] = 0;
                inv100[q] = 0.0;
                jflag[q] = 0;
            }
            continue;
        }
        const int P = n_valid - 1;
        if (hl < H) {
            const int cs[3] = {c0, c1, c2};
            for (int l = 0; l < 3; ++l) {
                row[l * H + hl] = static_cast<uint16_t>(cs[l]);
                if (spfh_out) spfh_out[q * D + l * H + hl] = static_cast<float>(spfh_value(cs[l], P));
            }
        }
        if (hl == 0) {
            Pq[q] = P;
            inv100[q] = P > 0 ? 100.0 / static_cast<double>(P) : 0.0;
            jflag[q] = (n_valid >= cl[cloud_of(kept_cloud, q)].tau_j) ? 1 : 0;
        }
    }
    // the FP64 recomputation counts, once per wave
    n64 = wave_sum(n64);
    nedge = wave_sum(nedge);
    if (lane == 0) {
        if (n64) atomicAdd(&st->feat_fp64, n64);
        if (nedge) atomicAdd(&st->feat_edge, nedge);
    }
}

// SPFH of point q (Eq. A2-A4) by one wavefront: the body of spfh_kernel.
__device__ __forceinline__ void spfh_point(const CloudDev* __restrict__ cl, const float* __restrict__ xyz,
                                           int64_t stride, const int32_t* __restrict__ kept_cloud,
                                           const float* __restrict__ nrm, int64_t nrm_stride,
                                           const uint8_t* __restrict__ flags, const int32_t* __restrict__ off,
                                           NbrLists nb, int H, uint16_t* __restrict__ cnt16,
                                           float* __restrict__ spfh_out, int32_t* __restrict__ Pq,
                                           double* __restrict__ inv100, int32_t* __restrict__ jflag, DevStatus* st,
                                           int64_t q, uint32_t* s_hist, int prow) {
    const int lane = lane_id();
    const int D = 3 * H;
    const int64_t s2 = 2 * stride, n2 = 2 * nrm_stride;
    uint16_t* row = cnt16 + q * spfh_row(H);
    if (!(flags[q] & 1)) {
        for (int t = lane; t < D; t += kWave) {
            row[t] = 0;
            if (spfh_out) spfh_out[q * D + t] = 0.0f;
        }
        if (lane == 0) {
            Pq[q] = 0;
            inv100[q] = 0.0;
            jflag[q] = 0;
        }
        return;
    }
    const V3f pq = {xyz[q], xyz[stride + q], xyz[s2 + q]};
    const V3f nq = {nrm[q], nrm[nrm_stride + q], nrm[n2 + q]};
    const int b = off[q], e = off[q + 1];
    const int32_t* lp = list_of(nb, prow, q, b, e);
    // the wavefront's histogram in LDS (3H counters), one atomic per lane and feature
    for (int t = lane; t < D; t += kWave) s_hist[t] = 0u;
    __builtin_amdgcn_wave_barrier();
    int n_valid = 0;
    uint32_t n64 = 0, nedge = 0;
    for (int base = b; base < e; base += kWave) {
        const int t = base + lane;
        bool valid = false;
        int bn[3] = {-1, -1, -1};
        if (t < e) {
            const int k = lp[t - b];
            valid = (flags[k] & 1) != 0;
            if (valid && k != q) {
                const V3f pk = {xyz[k], xyz[stride + k], xyz[s2 + k]};
                const V3f nk = {nrm[k], nrm[nrm_stride + k], nrm[n2 + k]};
                if (!bins_f32(pq, nq, pk, nk, H, bn)) {
                    const BinsF64 r = bins_f64(pq, nq, pk, nk, H);
                    bn[0] = r.b[0];
                    bn[1] = r.b[1];
                    bn[2] = r.b[2];
                    ++n64;
                    nedge += r.edge ? 1u : 0u;
                }
            }
        }
        n_valid += __popcll(ballot(valid));
        if (bn[0] >= 0) {
            atomicAdd(s_hist + bn[0], 1u);
            atomicAdd(s_hist + H + bn[1], 1u);
            atomicAdd(s_hist + 2 * H + bn[2], 1u);
        }
    }
    __builtin_amdgcn_wave_barrier();
    // lane h holds the counts of bin h for the three features
    int c0 = 0, c1 = 0, c2 = 0;
    if (lane < H) {
        c0 = static_cast<int>(s_hist[lane]);
        c1 = static_cast<int>(s_hist[H + lane]);
        c2 = static_cast<int>(s_hist[2 * H + lane]);
    }
    __builtin_amdgcn_wave_barrier();  // the histogram is free for the wavefront's next point
    n64 = wave_sum(n64);
    nedge = wave_sum(nedge);
    const int P = n_valid - 1;
    if (lane < H) {
        const int cs[3] = {c0, c1, c2};
        for (int l = 0; l < 3; ++l) {
            row[l * H + lane] = static_cast<uint16_t>(cs[l]);
            if (spfh_out) spfh_out[q * D + l * H + lane] = static_cast<float>(spfh_value(cs[l], P));
        }
    }
    if (lane == 0) {
        Pq[q] = P;
        inv100[q] = P > 0 ? 100.0 / static_cast<double>(P) : 0.0;
        jflag[q] = (n_valid >= cl[cloud_of(kept_cloud, q)].tau_j) ? 1 : 0;
        if (n64) atomicAdd(&st->feat_fp64, n64);
        if (nedge) atomicAdd(&st->feat_edge, nedge);
    }
}

__global__ __launch_bounds__(kBlock) void spfh_pairs(const CloudDev* __restrict__ cl, const float* __restrict__ xyz,
                                                     int64_t stride, const int32_t* __restrict__ kept_cloud,
                                                     int64_t m_cap, const float* __restrict__ nrm,
                                                     int64_t nrm_stride, const uint8_t* __restrict__ flags,
                                                     const int32_t* __restrict__ off,
                                                     NbrLists nb, int H,
                                                     uint16_t* __restrict__ cnt16, float* __restrict__ spfh_out,
                                                     int32_t* __restrict__ Pq, double* __restrict__ inv100,
                                                     int32_t* __restrict__ jflag, int pair_mean, int xcd,
                                                     DevStatus* st) {
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (st->err_range || st->err_capacity) return;  // the neighbour lists are incomplete
    // long lists: spfh_kernel (0 = always spfh_kernel, kMaxDegree = always this pass)
    if (pair_mean < kMaxDegree && (pair_mean == 0 || st->nnz > pair_mean * m)) return;
    __shared__ uint32_t s_hist[kWaves][2 * 3 * kMaxBins];
    spfh_pairs_body(cl, xyz, stride, kept_cloud, m, nrm, nrm_stride, flags, off, nb, H, cnt16, spfh_out, Pq, inv100,
                    jflag, xcd, st, s_hist[threadIdx.x / kWave]);
}

// SPFH (Eq. A2-A4) of every kept point when the mean list length exceeds
// pair_mean, one point per wavefront; xcd selects the XCD-aware split of the
// points over the wavefronts.
__global__ __launch_bounds__(kBlock) void spfh_kernel(const CloudDev* __restrict__ cl, const float* __restrict__ xyz,
                                                      int64_t stride, const int32_t* __restrict__ kept_cloud,
                                                      int64_t m_cap, const float* __restrict__ nrm,
                                                      int64_t nrm_stride, const uint8_t* __restrict__ flags,
                                                      const int32_t* __restrict__ off,
                                                      NbrLists nb, int H,
                                                      uint16_t* __restrict__ cnt16, float* __restrict__ spfh_out,
                                                      int32_t* __restrict__ Pq, double* __restrict__ inv100,
                                                      int32_t* __restrict__ jflag, int pair_mean, int xcd,
                                                      DevStatus* st) {
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (st->err_range || st->err_capacity) return;  // the neighbour lists are incomplete
    // short lists: spfh_pairs (0 = always this pass, kMaxDegree = always spfh_pairs)
    if (pair_mean >= kMaxDegree || (pair_mean > 0 && st->nnz <= pair_mean * m)) return;
    const XcdItems it = xcd ? xcd_items(m, off[m] + kItemWork * m, [&](int64_t i) { return off[i] + kItemWork * i; })
                            : cyclic_items(m);
    __shared__ uint32_t s_hist[kWaves][3 * kMaxBins];
    const int prow = nb.pad ? pad_stride(nb.pad_cap, m) : 0;
    for (int64_t q = it.first; q < it.end; q += it.stride)
        spfh_point(cl, xyz, stride, kept_cloud, nrm, nrm_stride, flags, off, nb, H, cnt16, spfh_out, Pq, inv100,
                   jflag, st, q, s_hist[threadIdx.x / kWave], prow);
}

// FPFH of rows of at most 64 values over the J list, two points per
// wavefront: a half of 32 lanes per point, lane l of the half summing bins l
// and l + 32.  The neighbours of a round of 32 are compacted in order into
// the half's LDS list and their SPFH rows summed in that order, term by term
// the sum fpfh_kernel forms.  The rows of the other kept points are zeroed.
template <int kBatchNarrow>
__global__ __launch_bounds__(kBlock) void fpfh_pairs(const float* __restrict__ xyz, int64_t stride, int64_t m_cap,
                                                     const uint8_t* __restrict__ flags,
                                                     const int32_t* __restrict__ jflag,
                                                     const int32_t* __restrict__ j_list,
                                                     const int32_t* __restrict__ off,
                                                     NbrLists nb, int H,
                                                     const uint16_t* __restrict__ cnt16,
                                                     const int32_t* __restrict__ Pq,
                                                     const double* __restrict__ inv100, float* __restrict__ fpfh,
                                                     int xcd, const DevStatus* st) {
#pragma clang fp contract(off)
    constexpr int kHalf = kWave / 2;
    __shared__ double s_w[kWaves][2][kHalf];
    // the SPFH rows of a round of 32 neighbours, one per lane, R entries each (dynamic)
    extern __shared__ uint4 s_dyn[];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int hf = lane / kHalf, hl = lane % kHalf, sh = kHalf * hf;
    const uint32_t below = (1u << hl) - 1u;
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (st->err_range || st->err_capacity) return;  // the neighbour lists are incomplete
    const int D = 3 * H;
    const int R = spfh_row(H);
    const int R8 = R / 8;  // 16-byte pieces of a row
    uint4* s_rows = s_dyn + (wv * 2 + hf) * kHalf * R8;
    const int64_t s2 = 2 * stride;
    const int64_t gt = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < m * D; t += gt)
        if (!jflag[t / D]) fpfh[t] = 0.0f;
    const int64_t n_j = clamp_count(st->n_j, m);
    const int prow = nb.pad ? pad_stride(nb.pad_cap, m) : 0;
    const XcdItems it = xcd ? xcd_items((n_j + 1) / 2, off[m] + kItemWork * n_j,
                                        [&](int64_t i) { return off[j_list[2 * i]] + kItemWork * 2 * i; })
                            : cyclic_items((n_j + 1) / 2);
    for (int64_t pw = it.first; pw < it.end; pw += it.stride) {
        const bool live = 2 * pw + hf < n_j;
        const int64_t q = live ? j_list[2 * pw + hf] : 0;
        float qx = 0.f, qy = 0.f, qz = 0.f;
        int b = 0, e = 0;
        if (live) {
            qx = xyz[q];
            qy = xyz[stride + q];
            qz = xyz[s2 + q];
            b = off[q];
            e = off[q + 1];
        }
        const int len = e - b;
        const int32_t* lp = list_of(nb, prow, q, b, e);
        const int lmax = max(len, __shfl_xor(len, kHalf, kWave));
        // lanes own bins hl and hl + 32; lanes past D read bin D - 1 and are never stored
        const int lb0 = min(hl, D - 1), lb1 = min(hl + kHalf, D - 1);
        double acc0 = 0.0, acc1 = 0.0;
        for (int base = 0; base < lmax; base += kHalf) {
            bool use = false;
            double w = 0.0;
            int k = 0;
            if (base + hl < len) {
                k = lp[base + hl];
                const float kx = xyz[k], ky = xyz[stride + k], kz = xyz[s2 + k];
                use = (k != q) && (flags[k] & 1);
                // the weight of SPFH(k) = c (100 / P_k) folded with 1 / w_k (P_k >= 1: q is in M[k]);
                // 100 / P_k is loaded beside the coordinates (the weight of an unused lane is dropped)
                w = (1.0 / sqrt(d2_exact(qx, qy, qz, kx, ky, kz))) * inv100[k];
            }
            const uint32_t bm = static_cast<uint32_t>(ballot(use) >> sh);
            __builtin_amdgcn_wave_barrier();
            if (use) {
                // the lane's whole row in 16-byte pieces, every row of the round in flight at once
                const int at = __popc(bm & below);
                const uint4* src = reinterpret_cast<const uint4*>(cnt16 + static_cast<int64_t>(k) * R);
                uint4* dst = s_rows + at * R8;
                for (int i = 0; i < R8; ++i) dst[i] = src[i];
                s_w[wv][hf][at] = w;
            }
            __builtin_amdgcn_wave_barrier();
            const int nuse = __popc(bm);
            const int numax = max(nuse, __shfl_xor(nuse, kHalf, kWave));
            // the rows summed in ascending neighbour order, bin by bin from LDS
            const uint16_t* rows = reinterpret_cast<const uint16_t*>(s_rows);
            for (int j = 0; j < numax; j += kBatchNarrow) {
                double v0[kBatchNarrow], v1[kBatchNarrow], wj[kBatchNarrow];
#pragma unroll
                for (int u = 0; u < kBatchNarrow; ++u) {
                    const int r = min(j + u, kHalf - 1);
                    v0[u] = static_cast<double>(rows[r * R + lb0]);
                    v1[u] = static_cast<double>(rows[r * R + lb1]);
                    wj[u] = s_w[wv][hf][r];
                }
#pragma unroll
                for (int u = 0; u < kBatchNarrow; ++u) {
                    if (j + u < nuse) {
                        acc0 = acc0 + wj[u] * v0[u];
                        acc1 = acc1 + wj[u] * v1[u];
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (!live) continue;
        float* out = fpfh + q * D;
        const int P = Pq[q];
        const uint16_t* sq = cnt16 + q * R;
        if (P == 0) {
            if (hl < D) out[hl] = 0.0f;
            if (hl + kHalf < D) out[hl + kHalf] = 0.0f;
            continue;
        }
        const double inv = 1.0 / static_cast<double>(P);
        if (hl < D) out[hl] = static_cast<float>(spfh_value(sq[hl], P) + inv * acc0);
        if (hl + kHalf < D) out[hl + kHalf] = static_cast<float>(spfh_value(sq[hl + kHalf], P) + inv * acc1);
    }
}

// FPFH of point q in J (Eq. A5) by one wavefront, with the wave's LDS lists
// s_k / s_w: the body of fpfh_kernel.
template <int kBatchNarrow>
__device__ __forceinline__ void fpfh_point(const float* __restrict__ xyz, int64_t stride,
                                           const uint8_t* __restrict__ flags, const int32_t* __restrict__ off,
                                           NbrLists nb, int H, const uint16_t* __restrict__ cnt16,
                                           const int32_t* __restrict__ Pq, const double* __restrict__ inv100,
                                           float* __restrict__ fpfh, int32_t* s_k, double* s_w, int64_t q,
                                           int prow) {
#pragma clang fp contract(off)
    const int lane = lane_id();
    const int D = 3 * H;
    const int R = spfh_row(H);
    const int64_t s2 = 2 * stride;
    float* out = fpfh + q * D;
    const float qx = xyz[q], qy = xyz[stride + q], qz = xyz[s2 + q];
    const int b = off[q], e = off[q + 1];
    const int32_t* lp = list_of(nb, prow, q, b, e);
    // lanes own bins lane and lane + 64; lanes past D read bin D - 1 and are never stored
    const int lb0 = min(lane, D - 1), lb1 = min(lane + kWave, D - 1);
    double acc0 = 0.0, acc1 = 0.0;
    for (int base = b; base < e; base += kWave) {
        // every load is unconditional (indices clamped), the mask applies afterwards
        const int t = min(base + lane, e - 1);
        const int k = lp[t - b];
        const float kx = xyz[k], ky = xyz[stride + k], kz = xyz[s2 + k];
        const bool use = (base + lane < e) && (k != q) && (flags[k] & 1);
        // the weight of SPFH(k) = c (100 / P_k) folded with 1 / w_k (P_k >= 1: q is in M[k]);
        // 100 / P_k is loaded beside the coordinates (the weight of an unused lane is dropped)
        const double w = (1.0 / sqrt(d2_exact(qx, qy, qz, kx, ky, kz))) * inv100[k];
        const uint64_t bm = ballot(use);
        __builtin_amdgcn_wave_barrier();
        if (use) {
            const int at = lanes_below(bm);
            s_k[at] = k;
            s_w[at] = w;
        }
        __builtin_amdgcn_wave_barrier();
        const int nuse = __popcll(bm);
        // SPFH rows in flight kBatchNarrow (rows of at most 64 values) or kBatch at a time,
        // accumulated in ascending neighbour order
        int j = 0;
        if (D <= kWave) {
            for (; j + kBatchNarrow <= nuse; j += kBatchNarrow) {
                double v0[kBatchNarrow];
#pragma unroll
                for (int u = 0; u < kBatchNarrow; ++u)
                    v0[u] = static_cast<double>(cnt16[static_cast<int64_t>(s_k[j + u]) * R + lb0]);
#pragma unroll
                for (int u = 0; u < kBatchNarrow; ++u) acc0 = acc0 + s_w[j + u] * v0[u];
            }
        }
        for (; j + kBatch <= nuse; j += kBatch) {
            double v0[kBatch], v1[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const uint16_t* sk = cnt16 + static_cast<int64_t>(s_k[j + u]) * R;
                v0[u] = static_cast<double>(sk[lb0]);
                v1[u] = D > kWave ? static_cast<double>(sk[lb1]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const double wj = s_w[j + u];
                acc0 = acc0 + wj * v0[u];
                acc1 = acc1 + wj * v1[u];
            }
        }
        for (; j < nuse; ++j) {
            const double wj = s_w[j];
            const uint16_t* sk = cnt16 + static_cast<int64_t>(s_k[j]) * R;
            acc0 = acc0 + wj * static_cast<double>(sk[lb0]);
            if (D > kWave) acc1 = acc1 + wj * static_cast<double>(sk[lb1]);
        }
    }
    const int P = Pq[q];
    const uint16_t* sq = cnt16 + q * R;
    if (P == 0) {
        if (lane < D) out[lane] = 0.0f;
        if (lane + kWave < D) out[lane + kWave] = 0.0f;
        return;
    }
    const double inv = 1.0 / static_cast<double>(P);
    if (lane < D) out[lane] = static_cast<float>(spfh_value(sq[lane], P) + inv * acc0);
    if (lane + kWave < D) out[lane + kWave] = static_cast<float>(spfh_value(sq[lane + kWave], P) + inv * acc1);
}

// One wavefront per point of the J list (j_list[0 .. n_j), from the J scan);
// the rows of the other kept points are zeroed by a grid-stride pass first.
template <int kBatchNarrow>
__global__ __launch_bounds__(kBlock) void fpfh_kernel(const float* __restrict__ xyz, int64_t stride, int64_t m_cap,
                                                      const uint8_t* __restrict__ flags,
                                                      const int32_t* __restrict__ jflag,
                                                      const int32_t* __restrict__ j_list,
                                                      const int32_t* __restrict__ off,
                                                      NbrLists nb, int H,
                                                      const uint16_t* __restrict__ cnt16,
                                                      const int32_t* __restrict__ Pq,
                                                      const double* __restrict__ inv100, float* __restrict__ fpfh,
                                                      int xcd, const DevStatus* st) {
    __shared__ int32_t s_k[kWaves][kWave];
    __shared__ double s_w[kWaves][kWave];
    const int wv = threadIdx.x / kWave;
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (st->err_range || st->err_capacity) return;  // the neighbour lists are incomplete
    const int D = 3 * H;
    const int64_t gt = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < m * D; t += gt)
        if (!jflag[t / D]) fpfh[t] = 0.0f;
    const int64_t n_j = clamp_count(st->n_j, m);
    const XcdItems it = xcd ? xcd_items(n_j, off[m] + kItemWork * n_j,
                                        [&](int64_t i) { return off[j_list[i]] + kItemWork * i; })
                            : cyclic_items(n_j);
    const int prow = nb.pad ? pad_stride(nb.pad_cap, m) : 0;
    for (int64_t g = it.first; g < it.end; g += it.stride)
        fpfh_point<kBatchNarrow>(xyz, stride, flags, off, nb, H, cnt16, Pq, inv100, fpfh, s_k[wv], s_w[wv],
                                 j_list[g], prow);
}

// SPFH and FPFH in one persistent launch.  Wavefronts take work items from a
// queue (one counter): first every SPFH item (kFuseChunk consecutive kept
// points), then every FPFH item (the same chunks); the FPFH of q in cloud c
// may start once every point of c has its SPFH, which a per-cloud readiness
// counter tells: an SPFH item adds its points to their clouds' counters after
// a release fence, an FPFH item waits (s_sleep polling, bounded) for its
// cloud's counter to reach the cloud's kept count and then acquires.  Items
// are handed out in order, so a waiting wavefront only ever waits for SPFH
// items that running wavefronts hold.  Non-J rows of the FPFH are zeroed by
// their FPFH items.  The same per-point bodies as spfh_kernel and fpfh_kernel:
// bit-identical outputs.
constexpr int kFuseChunk = 16;
constexpr uint32_t kFuseSpinLimit = 1u << 22;

__device__ __forceinline__ int64_t cloud_kept(const CloudState* cs, int c, int64_t m) {
    return cs ? cs[c].kept_cnt : m;
}

template <int kBatchNarrow>
__global__ __launch_bounds__(kBlock) void features_fused(
    const CloudDev* __restrict__ cl, const float* __restrict__ xyz, int64_t stride,
    const int32_t* __restrict__ kept_cloud, int64_t m_cap, const float* __restrict__ nrm, int64_t nrm_stride,
    uint8_t* __restrict__ flags, const int32_t* __restrict__ off, NbrLists nb, int H,
    uint16_t* __restrict__ cnt16, float* __restrict__ spfh_out, int32_t* __restrict__ Pq, double* __restrict__ inv100,
    int32_t* __restrict__ jflag, float* __restrict__ fpfh, const CloudState* __restrict__ cs, uint32_t* queue,
    int32_t* ready, DevStatus* st) {
    __shared__ int32_t s_k[kWaves][kWave];
    __shared__ double s_w[kWaves][kWave];
    __shared__ uint32_t s_hist[kWaves][3 * kMaxBins];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (st->err_range || st->err_capacity) return;  // the neighbour lists are incomplete
    const int D = 3 * H;
    const int prow = nb.pad ? pad_stride(nb.pad_cap, m) : 0;
    const int64_t n_chunks = (m + kFuseChunk - 1) / kFuseChunk;
    int known = -1;  // a cloud whose SPFH this wavefront has seen complete (and acquired)
    while (true) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(queue, 1u);
        item = __shfl(item, 0, kWave);
        if (item >= 2 * n_chunks) break;
        if (item < n_chunks) {
            const int64_t p0 = static_cast<int64_t>(item) * kFuseChunk;
            const int64_t p1 = min(p0 + kFuseChunk, m);
            for (int64_t q = p0; q < p1; ++q)
                spfh_point(cl, xyz, stride, kept_cloud, nrm, nrm_stride, flags, off, nb, H, cnt16, spfh_out, Pq,
                           inv100, jflag, st, q, s_hist[wv], prow);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) {
                // the chunk's points by cloud (a chunk rarely crosses a cloud boundary)
                int c = cloud_of(kept_cloud, p0), n = 0;
                for (int64_t q = p0; q < p1; ++q) {
                    const int cq = cloud_of(kept_cloud, q);
                    if (cq != c) {
                        atomicAdd(ready + c, n);
                        c = cq;
                        n = 0;
                    }
                    ++n;
                }
                atomicAdd(ready + c, n);
            }
            continue;
        }
        const int64_t p0 = static_cast<int64_t>(item - n_chunks) * kFuseChunk;
        const int64_t p1 = min(p0 + kFuseChunk, m);
        for (int64_t q = p0; q < p1; ++q) {
            const int c = cloud_of(kept_cloud, q);
            if (c != known) {
                const int64_t need = cloud_kept(cs, c, m);
                int ok = 0;
                if (lane == 0) {
                    uint32_t spins = 0;
                    while (__hip_atomic_load(ready + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > kFuseSpinLimit) break;
                    }
                    ok = spins <= kFuseSpinLimit;
                    if (!ok) atomicOr(&st->err_sync, 1);
                }
                ok = __shfl(ok, 0, kWave);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (ok) known = c;
            }
            if (jflag[q]) {
                fpfh_point<kBatchNarrow>(xyz, stride, flags, off, nb, H, cnt16, Pq, inv100, fpfh, s_k[wv], s_w[wv],
                                         q, prow);
            } else {
                for (int t = lane; t < D; t += kWave) fpfh[q * D + t] = 0.0f;
            }
        }
    }
}

// The FPFH launch with kRows SPFH rows in flight per lane (4, 8 or 16; the
// accumulation order, ascending neighbours, is the same for every choice).
template <bool kPairs, int kRows>
kmg_status fpfh_as(const float* xyz, int64_t stride, int64_t m_cap, const uint8_t* flags, const int32_t* jflag,
                   const int32_t* j_idx, const int32_t* off, NbrLists nb, int H, const uint16_t* cnt16,
                   const int32_t* Pq, const double* inv100, float* fpfh_out, const DevStatus* st, hipStream_t s) {
    if (kPairs) {
        // dynamic LDS: one SPFH row per lane of the block
        const size_t rows_lds = static_cast<size_t>(kBlock) * spfh_row(H) * sizeof(uint16_t);
        fpfh_pairs<kRows><<<grid_cap((m_cap + 1) / 2, kWaves), kBlock, rows_lds, s>>>(xyz, stride, m_cap, flags, jflag, j_idx,
                                                                              off, nb, H, cnt16, Pq, inv100, fpfh_out,
                                                                              (tuning().xcd_split >> 1) & 1, st);
    } else {
        fpfh_kernel<kRows><<<grid_cap(m_cap, kWaves), kBlock, 0, s>>>(xyz, stride, m_cap, flags, jflag, j_idx, off,
                                                                     nb, H, cnt16, Pq, inv100, fpfh_out,
                                                                     (tuning().xcd_split >> 1) & 1, st);
    }
    return launch_status();
}

template <bool kPairs>
kmg_status launch_fpfh(int rows, const float* xyz, int64_t stride, int64_t m_cap, const uint8_t* flags,
                       const int32_t* jflag, const int32_t* j_idx, const int32_t* off, NbrLists nb, int H,
                       const uint16_t* cnt16, const int32_t* Pq, const double* inv100, float* fpfh_out,
                       const DevStatus* st, hipStream_t s) {
    switch (rows) {
        case 1:
            return fpfh_as<kPairs, 1>(xyz, stride, m_cap, flags, jflag, j_idx, off, nb, H, cnt16, Pq, inv100,
                                      fpfh_out, st, s);
        case 2:
            return fpfh_as<kPairs, 2>(xyz, stride, m_cap, flags, jflag, j_idx, off, nb, H, cnt16, Pq, inv100,
                                      fpfh_out, st, s);
        case 4:
            return fpfh_as<kPairs, 4>(xyz, stride, m_cap, flags, jflag, j_idx, off, nb, H, cnt16, Pq, inv100,
                                      fpfh_out, st, s);
        case 16:
            return fpfh_as<kPairs, 16>(xyz, stride, m_cap, flags, jflag, j_idx, off, nb, H, cnt16, Pq, inv100,
                                       fpfh_out, st, s);
        default:
            return fpfh_as<kPairs, 8>(xyz, stride, m_cap, flags, jflag, j_idx, off, nb, H, cnt16, Pq, inv100,
                                      fpfh_out, st, s);
    }
}

// flags |= J << 1; j_idx[jpos[q]] = q, the kept index in the batch's global
// kept space (for one cloud, its own kept index).
// With sets (the batch form): block 0 also writes each cloud's J range (from
// the scan at its first and one-past-last kept point) and its matching set:
// the J rows of the cloud (global kept indices into fpfh), reported back as
// cloud-local kept indices.
__global__ __launch_bounds__(kBlock) void j_emit(const int32_t* __restrict__ jflag, const int32_t* __restrict__ pos,
                                                 int64_t m_cap, uint8_t* __restrict__ flags,
                                                 int32_t* __restrict__ j_idx, const DevStatus* st, CloudState* cs,
                                                 int n_clouds, const float* fpfh, MatchSet* sets) {
    const int64_t m = clamp_count(st->m_kept, m_cap);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < m; q += gs) {
        const int j = jflag[q];
        flags[q] = static_cast<uint8_t>((flags[q] & 1) | (j << 1));
        if (j) j_idx[pos[q]] = static_cast<int32_t>(q);
    }
    if (sets && blockIdx.x == 0) {
        const int64_t nj = st->n_j;
        for (int c = threadIdx.x; c < n_clouds; c += kBlock) {
            const int64_t a = cs[c].kept_off, b = a + cs[c].kept_cnt;
            const int64_t ja = a < m ? pos[a] : nj;
            const int64_t jb = b < m ? pos[b] : nj;
            cs[c].j_off = static_cast<int32_t>(ja);
            cs[c].j_cnt = static_cast<int32_t>(jb - ja);
            MatchSet ms;
            ms.desc = fpfh;
            ms.rows = j_idx + ja;
            ms.n = &cs[c].j_cnt;
            ms.row_base = cs[c].kept_off;
            ms.flags = 0;
            sets[c] = ms;
        }
    }
}

// Per-cloud J ranges from the exclusive scan at the cloud's first kept point.
__global__ void cloud_j_ranges(int n_clouds, int64_t m_cap, const int32_t* __restrict__ pos, const DevStatus* st,
                               CloudState* cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_clouds) return;
    const int64_t m = clamp_count(st->m_kept, m_cap);
    const int64_t nj = st->n_j;
    const int64_t a = cs[c].kept_off, b = a + cs[c].kept_cnt;
    const int64_t ja = a < m ? pos[a] : nj;
    const int64_t jb = b < m ? pos[b] : nj;
    cs[c].j_off = static_cast<int32_t>(ja);
    cs[c].j_cnt = static_cast<int32_t>(jb - ja);
}

}  // namespace

FeatWs carve_feat(Carver& c, int64_t m_cap, int H) {
    FeatWs w;
    const size_t mc = static_cast<size_t>(std::max<int64_t>(m_cap, 1));
    w.cnt16 = c.take<uint16_t>(mc * spfh_row(H));
    w.inv100 = c.take<double>(mc);
    w.queue = c.take<uint32_t>(1);
    w.ready = c.take<int32_t>(kMaxClouds);
    w.Pq = c.take<int32_t>(mc);
    w.jflag = c.take<int32_t>(mc);
    w.pos = c.take<int32_t>(mc);
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(m_cap));
    return w;
}

kmg_status spfh_batch(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                      int64_t m_cap, int H, DevStatus* st, const FeatWs& w, const int32_t* off, NbrLists nb,
                      const float* nrm, int64_t nrm_stride, uint8_t* flags, float* spfh_out, hipStream_t s,
                      bool cleared) {
    if (!cleared)
        KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.jflag), 0u, static_cast<size_t>(std::max<int64_t>(m_cap, 1)),
                         s));
    if (m_cap > 0) {
        StageScope sc(ST_SPFH, s);
        const int pair_mean = tuning().spfh_pair_mean;
        // the two forms split on the mean list length on the device; at the ends of
        // the range (0: one point per wavefront, kMaxDegree: two) the choice is made
        // here, and only that form is launched
        if (pair_mean < kMaxDegree) {
            spfh_kernel<<<grid_cap(m_cap, kWaves), kBlock, 0, s>>>(cl, xyz, stride, kept_cloud, m_cap, nrm,
                                                                  nrm_stride, flags, off, nb, H, w.cnt16, spfh_out,
                                                                  w.Pq, w.inv100, w.jflag, pair_mean,
                                                                  tuning().xcd_split & 1, st);
            KMG_TRY(launch_status());
        }
        if (pair_mean > 0) {
            spfh_pairs<<<grid_cap((m_cap + 1) / 2, kWaves), kBlock, 0, s>>>(cl, xyz, stride, kept_cloud, m_cap, nrm,
                                                                           nrm_stride, flags, off, nb, H, w.cnt16,
                                                                           spfh_out, w.Pq, w.inv100, w.jflag,
                                                                           pair_mean, tuning().xcd_split & 1, st);
            KMG_TRY(launch_status());
        }
    }
    return KMG_OK;
}

kmg_status fpfh_batch(int n_clouds, const float* xyz, int64_t stride, int64_t m_cap, int H, DevStatus* st,
                      const FeatWs& w, const int32_t* off, NbrLists nb, uint8_t* flags, float* fpfh_out,
                      int32_t* j_idx, CloudState* cs, hipStream_t s, MatchSet* sets, uint64_t* j_scan_status) {
    if (sets && !cs) return KMG_ERR_ARG;
    {
        // the J list first: the FPFH sums run over it
        StageScope sc(ST_J_COMPACT, s);
        if (j_scan_status)
            KMG_TRY(scan_exclusive_onepass(w.jflag, w.pos, m_cap, &st->n_j, j_scan_status, &st->err_sync, s));
        else
            KMG_TRY(scan_exclusive(w.jflag, w.pos, m_cap, &st->n_j, w.scan_tmp, s));
        if (m_cap > 0 || sets) {
            j_emit<<<std::max(grid_cap(m_cap, kBlock), 1u), kBlock, 0, s>>>(w.jflag, w.pos, m_cap, flags, j_idx, st,
                                                                          cs, n_clouds, fpfh_out, sets);
            KMG_TRY(launch_status());
        }
        if (cs && !sets) {
            cloud_j_ranges<<<grid_for(n_clouds, 256), 256, 0, s>>>(n_clouds, m_cap, w.pos, st, cs);
            KMG_TRY(launch_status());
        }
    }
    if (m_cap > 0) {
        StageScope sc(ST_FPFH, s);
        if (3 * H <= kWave) {
            KMG_TRY(launch_fpfh<true>(tuning().fpfh_rows, xyz, stride, m_cap, flags, w.jflag, j_idx, off, nb, H,
                                      w.cnt16, w.Pq, w.inv100, fpfh_out, st, s));
        } else {
            KMG_TRY(launch_fpfh<false>(tuning().fpfh_rows, xyz, stride, m_cap, flags, w.jflag, j_idx, off, nb, H,
                                       w.cnt16, w.Pq, w.inv100, fpfh_out, st, s));
        }
    }
    return KMG_OK;
}

// SPFH and FPFH in the fused persistent launch, then the J list.
template <int kRows>
void launch_fused(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud, int64_t m_cap,
                  const float* nrm, int64_t nrm_stride, uint8_t* flags, const int32_t* off, NbrLists nb, int H,
                  const FeatWs& w, float* spfh_out, float* fpfh_out, const CloudState* cs, DevStatus* st,
                  hipStream_t s) {
    features_fused<kRows><<<grid_cap(m_cap, kWaves), kBlock, 0, s>>>(cl, xyz, stride, kept_cloud, m_cap, nrm,
                                                                      nrm_stride, flags, off, nb, H, w.cnt16, spfh_out,
                                                                      w.Pq, w.inv100, w.jflag, fpfh_out, cs, w.queue,
                                                                      w.ready, st);
}

kmg_status features_fused_batch(const CloudDev* cl, int n_clouds, const float* xyz, int64_t stride,
                                const int32_t* kept_cloud, int64_t m_cap, int H, DevStatus* st, const FeatWs& w,
                                const int32_t* off, NbrLists nb, const float* nrm, int64_t nrm_stride,
                                uint8_t* flags, float* spfh_out, float* fpfh_out, int32_t* j_idx, CloudState* cs,
                                hipStream_t s, bool cleared, MatchSet* sets) {
    if (sets && !cs) return KMG_ERR_ARG;
    if (!cleared)
        KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.jflag), 0u, static_cast<size_t>(std::max<int64_t>(m_cap, 1)),
                         s));
    KMG_TRY(fill_u32(w.queue, 0u, 1, s));
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.ready), 0u, static_cast<size_t>(std::max(n_clouds, 1)), s));
    if (m_cap > 0) {
        StageScope sc(ST_SPFH, s);  // SPFH and FPFH together
        switch (tuning().fpfh_rows) {
            case 4: launch_fused<4>(cl, xyz, stride, kept_cloud, m_cap, nrm, nrm_stride, flags, off, nb, H, w,
                                    spfh_out, fpfh_out, cs, st, s); break;
            case 16: launch_fused<16>(cl, xyz, stride, kept_cloud, m_cap, nrm, nrm_stride, flags, off, nb, H, w,
                                      spfh_out, fpfh_out, cs, st, s); break;
            default: launch_fused<8>(cl, xyz, stride, kept_cloud, m_cap, nrm, nrm_stride, flags, off, nb, H, w,
                                     spfh_out, fpfh_out, cs, st, s); break;
        }
        KMG_TRY(launch_status());
    }
    StageScope sc(ST_J_COMPACT, s);
    KMG_TRY(scan_exclusive(w.jflag, w.pos, m_cap, &st->n_j, w.scan_tmp, s));
    if (m_cap > 0 || sets) {
        j_emit<<<std::max(grid_cap(m_cap, kBlock), 1u), kBlock, 0, s>>>(w.jflag, w.pos, m_cap, flags, j_idx, st, cs,
                                                                      n_clouds, fpfh_out, sets);
        KMG_TRY(launch_status());
    }
    if (cs && !sets) {
        cloud_j_ranges<<<grid_for(n_clouds, 256), 256, 0, s>>>(n_clouds, m_cap, w.pos, st, cs);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

kmg_status features_batch(const CloudDev* cl, int n_clouds, const float* xyz, int64_t stride,
                          const int32_t* kept_cloud, int64_t m_cap, int H, DevStatus* st, const FeatWs& w,
                          const int32_t* off, NbrLists nb, const float* nrm, int64_t nrm_stride,
                          uint8_t* flags, float* spfh_out, float* fpfh_out, int32_t* j_idx, CloudState* cs,
                          hipStream_t s, bool cleared, MatchSet* sets, uint64_t* j_scan_status) {
    if (tuning().fuse_features)
        return features_fused_batch(cl, n_clouds, xyz, stride, kept_cloud, m_cap, H, st, w, off, nb, nrm,
                                    nrm_stride, flags, spfh_out, fpfh_out, j_idx, cs, s, cleared, sets);
    KMG_TRY(spfh_batch(cl, xyz, stride, kept_cloud, m_cap, H, st, w, off, nb, nrm, nrm_stride, flags, spfh_out, s,
                       cleared));
    return fpfh_batch(n_clouds, xyz, stride, m_cap, H, st, w, off, nb, flags, fpfh_out, j_idx, cs, s, sets,
                      j_scan_status);
}

}  // namespace kmg
