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
// left at that level; then the level jumps to the smallest remaining degree.  Core numbers are unique, so the parallel order of
// removals cannot change them.  The maximum k-core is the set of vertices
// whose core number is the largest.
#include <climits>
#include <math.h>

#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;
constexpr int kPeelThreads = 1024;
constexpr int kMaxKcore = KMG_MAX_KCORE_VERTICES;  // LDS: 4 + 2 + 2 bytes per vertex

__global__ __launch_bounds__(kBlock) void ratio_keys(const float* __restrict__ d1, const float* __restrict__ d2,
                                                     int64_t k, uint64_t* __restrict__ keys) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < k;
         e += static_cast<int64_t>(gridDim.x) * kBlock) {
        const double a = d1[e], b = d2[e];
        const double r = b > 0.0 ? a / b : (a > 0.0 ? INFINITY : 0.0);
        keys[e] = static_cast<uint64_t>(__double_as_longlong(r));
    }
}

// rank[e] = number of correspondences f ordered before e by (key, position).
// Block (x, y) counts, for the keys of tile x, the keys of tiles y, y + gy, ...
// (staged in LDS) that come first, and adds its counts with one atomic per key;
// rank_emit then writes sel[rank] = e for the first n_tau ranks.
constexpr int kRankTiles = 64;  // y tiles of the counting grid

__global__ __launch_bounds__(kBlock) void rank_count(const uint64_t* __restrict__ keys, int64_t k,
                                                     int32_t* __restrict__ rank) {
    __shared__ uint64_t s_key[kBlock];
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool live = e < k;
    const uint64_t me = live ? keys[e] : 0ull;
    int cnt = 0;
    for (int64_t f0 = static_cast<int64_t>(blockIdx.y) * kBlock; f0 < k;
         f0 += static_cast<int64_t>(gridDim.y) * kBlock) {
        __syncthreads();
        if (f0 + threadIdx.x < k) s_key[threadIdx.x] = keys[f0 + threadIdx.x];
        __syncthreads();
        const int nf = static_cast<int>(min<int64_t>(kBlock, k - f0));
        for (int t = 0; t < nf; ++t) {
            const uint64_t o = s_key[t];
            cnt += (o < me || (o == me && f0 + t < e)) ? 1 : 0;
        }
    }
    if (live && cnt) atomicAdd(rank + e, cnt);
}

__global__ __launch_bounds__(kBlock) void rank_emit(const int32_t* __restrict__ rank, int64_t k, int32_t n_tau,
                                                    int32_t* __restrict__ sel) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; e < k;
         e += static_cast<int64_t>(gridDim.x) * kBlock)
        if (rank[e] < n_tau) sel[rank[e]] = static_cast<int32_t>(e);
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

// Core numbers as the fixed point of the h-index operator: start from h = degree
// and replace h[v] by the largest x <= h[v] such that at least x neighbours u
// have h[u] >= x.  Values only decrease and never fall below the core numbers;
// a sweep that changes nothing proves a fixed point, and a fixed point reached
// from above is the core numbers (if h[v] >= x, v has x neighbours with h >= x,
// so {h >= x} lies in the x-core).  Updates are in place (a neighbour's newer,
// smaller value only speeds convergence).  Sweep k runs only if sweep k - 1
// changed something (flag[k] set); one wavefront per vertex.
constexpr int kHSweeps = 48;  // sweeps launched; the block peel finishes graphs that need more
constexpr int kHRegs = 8;     // neighbour values held in registers per lane (deg <= 512)

__global__ __launch_bounds__(kBlock) void kcore_hinit(const int32_t* __restrict__ off, int32_t n,
                                                      int32_t* __restrict__ h, int32_t* __restrict__ flag) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) h[v] = off[v + 1] - off[v];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i <= kHSweeps; i += gridDim.x * kBlock) flag[i] = i == 0;
}

__global__ __launch_bounds__(kBlock) void kcore_hsweep(const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ adj, int32_t n, int32_t* h,
                                                       int32_t* flag, int sweep, int32_t* __restrict__ info) {
    if (flag[sweep] == 0) return;  // converged
    const int lane = lane_id();
    bool changed = false;
    for (int64_t vw = global_wave(); vw < n; vw += wave_count()) {
        const int v = static_cast<int>(vw);
        const int cap = h[v];
        if (cap == 0) continue;
        const int b = off[v], deg = off[v + 1] - b;
        int hi = min(cap, deg);
        int lo = 0;
        int val[kHRegs];
        const bool in_regs = deg <= kHRegs * kWave;
#pragma unroll
        for (int r = 0; r < kHRegs; ++r) {
            const int t = r * kWave + lane;
            val[r] = -1;
            if (in_regs && t < deg) {
                const int u = adj[b + t];
                if (u < 0 || u >= n) info[2] = 1;  // not a vertex: reported, never followed
                else val[r] = h[u];
            }
        }
        // count of neighbour values >= x (from registers, or re-read for long rows)
        auto count_ge = [&](int x) {
            int c = 0;
            if (in_regs) {
#pragma unroll
                for (int r = 0; r < kHRegs; ++r) c += __popcll(ballot(val[r] >= x));
            } else {
                for (int t0 = 0; t0 < deg; t0 += kWave) {
                    const int t = t0 + lane;
                    int w = -1;
                    if (t < deg) {
                        const int u = adj[b + t];
                        if (u < 0 || u >= n) info[2] = 1;
                        else w = h[u];
                    }
                    c += __popcll(ballot(w >= x));
                }
            }
            return c;
        };
        if (count_ge(hi) >= hi) {
            lo = hi;
        } else {
            --hi;  // invariant: count_ge(lo) >= lo, count_ge(hi + 1) < hi + 1
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (count_ge(mid) >= mid) lo = mid;
                else hi = mid - 1;
            }
        }
        if (lo < cap) {
            if (lane == 0) h[v] = lo;
            changed = true;
        }
    }
    if (changed && lane == 0) flag[sweep + 1] = 1;
}

// After the sweeps: if they converged, the core numbers are h (and their maximum
// goes to info[0]); otherwise the block peel has written both.
__global__ __launch_bounds__(kBlock) void kcore_hfinish(const int32_t* __restrict__ h, int32_t n,
                                                        const int32_t* __restrict__ flag, int32_t* __restrict__ core,
                                                        int32_t* __restrict__ info) {
    if (flag[kHSweeps] != 0) return;
    int mx = -1;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        core[v] = h[v];
        mx = max(mx, h[v]);
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) mx = max(mx, __shfl_xor(mx, d, kWave));
    if (lane_id() == 0 && mx >= 0) atomicMax(info, mx);
}

// One block: core numbers of the graph (off, adj) on n <= kMaxKcore vertices.
// Remaining degrees, core numbers and the list of the round's removals live in
// LDS (dynamic, 8 bytes per vertex), so the block's atomics and plain reads see
// one coherent copy.  A round removes every alive vertex whose remaining
// degree is <= the level (core number = level) and lists it; the block's
// wavefronts then take the listed vertices and their lanes walk each one's
// adjacency, decrementing alive neighbours.  A round that removes nothing
// raises the level to the smallest remaining degree (no round is spent on
// an empty level).
__global__ __launch_bounds__(kPeelThreads) void kcore_peel(const int32_t* __restrict__ off,
                                                           const int32_t* __restrict__ adj, int32_t n,
                                                           int32_t* __restrict__ core_out,
                                                           int32_t* __restrict__ info,
                                                           const int32_t* __restrict__ skip) {
    if (skip && *skip == 0) return;  // the h-index sweeps converged
    extern __shared__ int32_t s_mem[];
    int32_t* s_deg = s_mem;
    int16_t* s_core = reinterpret_cast<int16_t*>(s_deg + n);
    int16_t* s_list = s_core + n;
    __shared__ int s_cnt, s_left, s_min, s_max;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    constexpr int kWaves = kPeelThreads / kWave;
    for (int v = threadIdx.x; v < n; v += kPeelThreads) {
        s_deg[v] = off[v + 1] - off[v];
        s_core[v] = -1;
    }
    if (threadIdx.x == 0) {
        s_left = n;
        s_max = -1;
    }
    int level = 0;
    while (true) {
        __syncthreads();
        if (s_left == 0) break;
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_min = INT_MAX;
        }
        __syncthreads();
        int low = INT_MAX;
        for (int v0 = 0; v0 < n; v0 += kPeelThreads) {
            const int v = v0 + threadIdx.x;
            bool rm = false;
            if (v < n && s_core[v] < 0) {
                const int d = s_deg[v];
                if (d <= level) {
                    s_core[v] = static_cast<int16_t>(level);
                    rm = true;
                } else {
                    low = min(low, d);
                }
            }
            const uint64_t b = ballot(rm);
            int base = 0;
            if (lane == 0 && b) base = atomicAdd(&s_cnt, __popcll(b));
            base = __shfl(base, 0, kWave);
            if (rm) s_list[base + lanes_below(b)] = static_cast<int16_t>(v);
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) low = min(low, __shfl_xor(low, d, kWave));
        if (lane == 0 && low != INT_MAX) atomicMin(&s_min, low);
        __syncthreads();
        const int nrem = s_cnt;
        if (nrem == 0) {
            level = max(level + 1, s_min);  // every alive vertex has a larger degree
            continue;
        }
        if (threadIdx.x == 0) s_left -= nrem;
        for (int i = wv; i < nrem; i += kWaves) {
            const int f = s_list[i];
            const int e = off[f + 1];
            for (int t = off[f] + lane; t < e; t += kWave) {
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

size_t kcore_lds_bytes(int32_t n) { return static_cast<size_t>(n) * 8 + 16; }

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
    int32_t* rank;
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
    w.rank = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(n_corr, 1)));
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
    int32_t* h;
    int32_t* flag;
};

KcoreWs carve_kcore(Carver& c, int32_t n) {
    KcoreWs w;
    w.info = c.take<int32_t>(3);  // max core, members, bad index flag
    w.h = c.take<int32_t>(static_cast<size_t>(std::max(n, 1)));
    w.flag = c.take<int32_t>(kHSweeps + 1);
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
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.rank), 0u, static_cast<size_t>(n_corr), s));
    {
        const int64_t tiles = (n_corr + kBlock - 1) / kBlock;
        const dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(std::min<int64_t>(tiles, kRankTiles)));
        rank_count<<<grid, kBlock, 0, s>>>(w.keys, n_corr, w.rank);
        KMG_TRY(launch_status());
    }
    rank_emit<<<grid_cap(n_corr, kBlock), kBlock, 0, s>>>(w.rank, n_corr, n_tau, sel);
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
    const size_t lds = kcore_lds_bytes(n);
    if (lds > 65536) {
        static const hipError_t raised = hipFuncSetAttribute(reinterpret_cast<const void*>(&kcore_peel),
                                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                                             static_cast<int>(kcore_lds_bytes(kMaxKcore)));
        if (raised != hipSuccess) return KMG_ERR_RANGE;  // this device cannot hold the graph's state on chip
    }
    {
        const unsigned g = grid_cap(std::max<int64_t>(n, kHSweeps + 1), kBlock);
        kcore_hinit<<<g, kBlock, 0, s>>>(off, n, w.h, w.flag);
        KMG_TRY(launch_status());
        const unsigned gw = grid_cap(n, kBlock / kWave);
        for (int k = 0; k < kHSweeps; ++k) {
            kcore_hsweep<<<gw, kBlock, 0, s>>>(off, adj, n, w.h, w.flag, k, w.info);
            KMG_TRY(launch_status());
        }
    }
    kcore_peel<<<1, kPeelThreads, lds, s>>>(off, adj, n, core, w.info, w.flag + kHSweeps);
    KMG_TRY(launch_status());
    kcore_hfinish<<<grid_cap(n, kBlock), kBlock, 0, s>>>(w.h, n, w.flag, core, w.info);
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
