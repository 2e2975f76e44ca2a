// Downstream of matching (Section III-D): the ratio filter that keeps the
// N_tau correspondences with the lowest descriptor distance ratio, the
// pairwise-invariant compatibility graph of Eq. (3), and its maximum k-core.
//
// Ratio filter.  The key of correspondence e is its ratio d1/d2 in FP64 from
// the float32 distances (0 when both are 0, +inf when only d2 is 0); keys are
// non-negative, so their bit patterns order like the values.  Correspondences
// are ranked by (key, position) by counting, which is exact and needs no sort;
// the first N_tau ranks are the graph's vertices, vertex v = rank v.
//
// Graph.  Vertices u != v are adjacent iff | ||b_u - b_v|| - ||a_u - a_v|| |
// <= 2 beta, with both norms evaluated in FP64 as sqrt((dx dx + dy dy) + dz dz)
// from the float32 kept coordinates (contraction off).  One wavefront per
// row tests 64 columns at a time: a count pass, a scan, then a fill pass that
// writes every row ascending.
//
// k-core.  Core numbers by level-synchronous peeling in one block: at level
// k, every vertex whose remaining degree is <= k is removed (core number k)
// and its alive neighbours lose one degree, round after round until none is
// left at that level.  Core numbers are unique, so the parallel order of
// removals cannot change them.  The maximum k-core is the set of vertices
// whose core number is the largest.
#include <math.h>

#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;
constexpr int kPeelThreads = 1024;
constexpr int kMaxKcore = KMG_MAX_KCORE_VERTICES;  // LDS: 4 + 2 + 1 bytes per vertex

__global__ __launch_bounds__(kBlock) void ratio_keys(const float* __restrict__ d1, const float* __restrict__ d2,
                                                     int64_t k, uint64_t* __restrict__ keys) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < k;
         e += static_cast<int64_t>(gridDim.x) * kBlock) {
        const double a = d1[e], b = d2[e];
        const double r = b > 0.0 ? a / b : (a > 0.0 ? INFINITY : 0.0);
        keys[e] = static_cast<uint64_t>(__double_as_longlong(r));
    }
}

// Block-stride over e; the block's threads walk the keys together through an
// LDS tile, so every key is read once per block.
__global__ __launch_bounds__(kBlock) void rank_select(const uint64_t* __restrict__ keys, int64_t k, int32_t n_tau,
                                                      int32_t* __restrict__ sel) {
    __shared__ uint64_t s_key[kBlock];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t e0 = static_cast<int64_t>(blockIdx.x) * kBlock; e0 < k; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        const bool live = e < k;
        const uint64_t me = live ? keys[e] : 0ull;
        int64_t rank = 0;
        for (int64_t f0 = 0; f0 < k; f0 += kBlock) {
            __syncthreads();
            if (f0 + threadIdx.x < k) s_key[threadIdx.x] = keys[f0 + threadIdx.x];
            __syncthreads();
            const int nf = static_cast<int>(min<int64_t>(kBlock, k - f0));
            for (int t = 0; t < nf; ++t) {
                const uint64_t o = s_key[t];
                rank += (o < me || (o == me && f0 + t < e)) ? 1 : 0;
            }
        }
        if (live && rank < n_tau) sel[rank] = static_cast<int32_t>(e);
    }
}

// Correspondence indices outside the clouds set err and read point 0 instead.
__global__ __launch_bounds__(kBlock) void gather_vertices(const float* __restrict__ src, int64_t src_stride,
                                                          const float* __restrict__ tgt, int64_t tgt_stride,
                                                          const int32_t* __restrict__ pairs,
                                                          const int32_t* __restrict__ sel, int32_t n,
                                                          float4* __restrict__ va, float4* __restrict__ vb,
                                                          int32_t* __restrict__ err) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int64_t e = sel[v];
        int i = pairs[2 * e], j = pairs[2 * e + 1];
        if (i < 0 || i >= src_stride || j < 0 || j >= tgt_stride) {
            atomicOr(err, 1);
            i = 0;
            j = 0;
        }
        va[v] = make_float4(src[i], src[src_stride + i], src[2 * src_stride + i], 0.0f);
        vb[v] = make_float4(tgt[j], tgt[tgt_stride + j], tgt[2 * tgt_stride + j], 0.0f);
    }
}

__device__ __forceinline__ double norm_between(float4 p, float4 q) {
#pragma clang fp contract(off)
    const double dx = static_cast<double>(p.x) - static_cast<double>(q.x);
    const double dy = static_cast<double>(p.y) - static_cast<double>(q.y);
    const double dz = static_cast<double>(p.z) - static_cast<double>(q.z);
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

// Eq. (3) for vertices u != v.
__device__ __forceinline__ bool compatible(float4 au, float4 bu, float4 av, float4 bv, double two_beta) {
#pragma clang fp contract(off)
    const double da = norm_between(au, av);
    const double db = norm_between(bu, bv);
    return fabs(db - da) <= two_beta;
}

template <bool kFill>
__global__ __launch_bounds__(kBlock) void graph_rows(const float4* __restrict__ va, const float4* __restrict__ vb,
                                                     int32_t n, double beta, int32_t* __restrict__ deg,
                                                     const int32_t* __restrict__ off, int32_t* __restrict__ adj) {
    const int lane = lane_id();
    const double two_beta = 2.0 * beta;
    for (int64_t u = global_wave(); u < n; u += wave_count()) {
        const float4 au = va[u], bu = vb[u];
        int found = 0;
        int32_t* out = kFill ? adj + off[u] : nullptr;
        for (int base = 0; base < n; base += kWave) {
            const int v = base + lane;
            const int vc = min(v, n - 1);  // unconditional loads; the mask applies afterwards
            const bool e = v < n && v != u && compatible(au, bu, va[vc], vb[vc], two_beta);
            const uint64_t b = ballot(e);
            if (kFill && e) out[found + lanes_below(b)] = v;
            found += __popcll(b);
        }
        if (!kFill && lane == 0) deg[u] = found;
    }
}

// One block: core numbers of the graph (off, adj) on n <= kMaxKcore vertices.
// Degrees, core numbers and the removal flags live in LDS, so the block's
// atomics and plain reads see one coherent copy.
__global__ __launch_bounds__(kPeelThreads) void kcore_peel(const int32_t* __restrict__ off,
                                                           const int32_t* __restrict__ adj, int32_t n,
                                                           int32_t* __restrict__ core_out,
                                                           int32_t* __restrict__ info) {
    __shared__ int32_t s_deg[kMaxKcore];
    __shared__ int16_t s_core[kMaxKcore];
    __shared__ uint8_t s_fresh[kMaxKcore];
    __shared__ int s_changed, s_left, s_max;
    for (int v = threadIdx.x; v < n; v += kPeelThreads) {
        s_deg[v] = off[v + 1] - off[v];
        s_core[v] = -1;
        s_fresh[v] = 0;
    }
    if (threadIdx.x == 0) {
        s_left = n;
        s_max = -1;
    }
    int level = 0;
    while (true) {
        __syncthreads();
        if (s_left == 0) break;
        if (threadIdx.x == 0) s_changed = 0;
        __syncthreads();
        // removals of this round: alive vertices whose remaining degree is <= level
        int removed = 0;
        for (int v = threadIdx.x; v < n; v += kPeelThreads) {
            if (s_core[v] < 0 && s_deg[v] <= level) {
                s_core[v] = static_cast<int16_t>(level);
                s_fresh[v] = 1;
                ++removed;
            }
        }
        if (removed) {
            atomicAdd(&s_changed, 1);
            atomicSub(&s_left, removed);
        }
        __syncthreads();
        if (!s_changed) {
            ++level;  // nothing left at this level
            continue;
        }
        for (int v = threadIdx.x; v < n; v += kPeelThreads) {
            if (!s_fresh[v]) continue;
            s_fresh[v] = 0;
            for (int t = off[v]; t < off[v + 1]; ++t) {
                const int u = adj[t];
                if (u < 0 || u >= n) {  // not a vertex: reported, never followed
                    info[2] = 1;
                    continue;
                }
                if (s_core[u] < 0) atomicSub(&s_deg[u], 1);
            }
        }
    }
    int mx = -1;
    for (int v = threadIdx.x; v < n; v += kPeelThreads) {
        core_out[v] = s_core[v];
        mx = max(mx, static_cast<int>(s_core[v]));
    }
    atomicMax(&s_max, mx);
    __syncthreads();
    if (threadIdx.x == 0) info[0] = s_max;
}

// members: vertices with the largest core number, ascending (one block).
__global__ __launch_bounds__(kPeelThreads) void kcore_members(const int32_t* __restrict__ core, int32_t n,
                                                              int32_t* __restrict__ members,
                                                              int32_t* __restrict__ info) {
    __shared__ int s_base;
    __shared__ int s_wave[kPeelThreads / kWave];
    const int mx = info[0];
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int v0 = 0; v0 < n; v0 += kPeelThreads) {
        const int v = v0 + threadIdx.x;
        const bool in = v < n && core[v] == mx;
        const uint64_t b = ballot(in);
        if (lane == 0) s_wave[wv] = __popcll(b);
        __syncthreads();
        int before = s_base;
        for (int w = 0; w < wv; ++w) before += s_wave[w];
        if (in) members[before + lanes_below(b)] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < kPeelThreads / kWave; ++w) tot += s_wave[w];
            s_base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) info[1] = s_base;
}

struct GraphWs {
    uint64_t* keys;
    float4* va;
    float4* vb;
    int32_t* deg;
    int64_t* nnz;
    int32_t* err;
    int64_t* scan_tmp;
};

GraphWs carve_graph(Carver& c, int64_t n_corr, int32_t n_tau) {
    GraphWs w;
    w.keys = c.take<uint64_t>(static_cast<size_t>(std::max<int64_t>(n_corr, 1)));
    w.va = c.take<float4>(static_cast<size_t>(std::max(n_tau, 1)));
    w.vb = c.take<float4>(static_cast<size_t>(std::max(n_tau, 1)));
    w.deg = c.take<int32_t>(static_cast<size_t>(n_tau) + 1);
    w.nnz = c.take<int64_t>(1);
    w.err = c.take<int32_t>(1);
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(static_cast<int64_t>(n_tau) + 1));
    return w;
}

struct KcoreWs {
    int32_t* info;
};

KcoreWs carve_kcore(Carver& c, int32_t) {
    KcoreWs w;
    w.info = c.take<int32_t>(3);  // max core, members, bad index flag
    return w;
}

}  // namespace

size_t graph_ws(int64_t n_corr, int32_t n_tau) {
    Carver c(nullptr, 0);
    carve_graph(c, n_corr, n_tau);
    return c.off;
}

size_t kcore_ws(int32_t n) {
    Carver c(nullptr, 0);
    carve_kcore(c, n);
    return c.off;
}

kmg_status corr_graph(const float* src, int64_t src_stride, const float* tgt, int64_t tgt_stride,
                      const int32_t* pairs, const float* d1, const float* d2, int64_t n_corr, int32_t n_tau,
                      double beta, int32_t* sel, int32_t* off, int32_t* adj, int64_t adj_cap, int32_t* n_sel_host,
                      int64_t* nnz_host, void* ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    GraphWs w = carve_graph(c, n_corr, n_tau);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    const int32_t n = static_cast<int32_t>(std::min<int64_t>(n_corr, n_tau));
    *n_sel_host = n;
    *nnz_host = 0;
    if (n == 0) {
        KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(off), 0u, 1, s));
        return KMG_OK;
    }
    ratio_keys<<<grid_cap(n_corr, kBlock), kBlock, 0, s>>>(d1, d2, n_corr, w.keys);
    KMG_TRY(launch_status());
    rank_select<<<grid_cap(n_corr, kBlock), kBlock, 0, s>>>(w.keys, n_corr, n_tau, sel);
    KMG_TRY(launch_status());
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.err), 0u, 1, s));
    gather_vertices<<<grid_cap(n, kBlock), kBlock, 0, s>>>(src, src_stride, tgt, tgt_stride, pairs, sel, n, w.va,
                                                           w.vb, w.err);
    KMG_TRY(launch_status());
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.deg), 0u, static_cast<size_t>(n) + 1, s));
    graph_rows<false><<<grid_cap(n, kBlock / kWave), kBlock, 0, s>>>(w.va, w.vb, n, beta, w.deg, nullptr, nullptr);
    KMG_TRY(launch_status());
    KMG_TRY(scan_exclusive(w.deg, off, static_cast<int64_t>(n) + 1, w.nnz, w.scan_tmp, s));
    int64_t nnz = 0;
    int32_t err = 0;
    KMG_TRY_HIP(hipMemcpyAsync(&nnz, w.nnz, sizeof(nnz), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipMemcpyAsync(&err, w.err, sizeof(err), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    if (err) return KMG_ERR_RANGE;
    *nnz_host = nnz;
    if (nnz > adj_cap) return KMG_ERR_CAPACITY;
    graph_rows<true><<<grid_cap(n, kBlock / kWave), kBlock, 0, s>>>(w.va, w.vb, n, beta, nullptr, off, adj);
    KMG_TRY(launch_status());
    return KMG_OK;
}

kmg_status max_kcore(const int32_t* off, const int32_t* adj, int32_t n, int32_t* core, int32_t* members,
                     int32_t* n_members_host, int32_t* max_core_host, void* ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    KcoreWs w = carve_kcore(c, n);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    *n_members_host = 0;
    *max_core_host = -1;
    if (n == 0) return KMG_OK;
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.info), 0u, 3, s));
    kcore_peel<<<1, kPeelThreads, 0, s>>>(off, adj, n, core, w.info);
    KMG_TRY(launch_status());
    kcore_members<<<1, kPeelThreads, 0, s>>>(core, n, members, w.info);
    KMG_TRY(launch_status());
    int32_t info[3];
    KMG_TRY_HIP(hipMemcpyAsync(info, w.info, sizeof(info), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    if (info[2]) return KMG_ERR_RANGE;
    *max_core_host = info[0];
    *n_members_host = info[1];
    return KMG_OK;
}

}  // namespace kmg
