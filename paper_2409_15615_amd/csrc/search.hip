// Radius search on a voxel-cell hash and PCA normals (Algorithm 1, Step 1),
// for all clouds of a batch at once.
//
// Cells have edge c = r_FPFH * (1 + 1e-4) (per cloud), so every point within
// r_FPFH of a query lies in the 27 cells around the query's cell.  Cell keys
// carry the cloud id, so one table serves the batch and a query only ever
// sees its own cloud.  Points are counting-sorted by cell into an AoS float4
// array (x, y, z, kept index), and each query is served by half a wavefront
// (a whole one for the longest lists) whose lanes walk the flattened candidate
// list of the 27 cells.  The search runs twice: a count pass (|N(q)|), then,
// after a prefix sum has placed every list, a fill pass that collects the
// accepted indices in LDS and writes them in ascending order.  Batches may
// instead search once (the list-first form): each list goes to a row of a pad
// with its length, the offsets follow from the lengths, and the later passes
// read the lists from their rows (the longer lists, searched again, from
// their CSR places).  Normals are then estimated by four lanes per point from
// the stored list: FP64 moments of the r_normal subset, a cyclic Jacobi
// eigen-solver in FP64, the linearity test and viewpoint orientation.
#include <climits>

#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;
constexpr int kNormalLanes = 4;  // lanes per point in the normal estimation

struct Grid {
    const float4* pts;     // cell-sorted points; w = bit pattern of the kept index
    const uint64_t* keys;  // cell hash table
    const int32_t* start;  // first sorted position of each cell slot
    const int32_t* count;  // points in each cell slot
    uint32_t mask;
};

__device__ __forceinline__ int64_t cell_coord(float x, double inv_c) {
    return static_cast<int64_t>(floor(static_cast<double>(x) * inv_c));
}

__device__ __forceinline__ int cloud_of(const int32_t* kept_cloud, int64_t q) {
    return kept_cloud ? kept_cloud[q] : 0;
}

// Kept points in input order often share a cell: only the first lane of a run
// of equal keys on consecutive lanes inserts the key and adds the run's length
// to the cell's count; cell_scatter places a run the same way, in lane order.
__global__ __launch_bounds__(kBlock) void cell_insert(const CloudDev* __restrict__ cl,
                                                      const float* __restrict__ xyz, int64_t stride,
                                                      const int32_t* __restrict__ kept_cloud, int64_t m_cap,
                                                      uint64_t* keys, int32_t* cnt, uint32_t mask,
                                                      int32_t* __restrict__ pslot, DevStatus* st) {
    const int64_t m = clamp_count(st->m_kept, m_cap);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    const int lane = lane_id();
    // every lane of a wave runs the same rounds (the run detection shuffles)
    for (int64_t p0 = static_cast<int64_t>(blockIdx.x) * kBlock + (threadIdx.x & ~(kWave - 1)); p0 < m; p0 += gs) {
        const int64_t p = p0 + lane;
        uint64_t key = kEmptyKey;
        if (p < m) {
            const int c = cloud_of(kept_cloud, p);
            const double inv_c = cl[c].inv_cell;
            const double kx = floor(static_cast<double>(xyz[p]) * inv_c);
            const double ky = floor(static_cast<double>(xyz[stride + p]) * inv_c);
            const double kz = floor(static_cast<double>(xyz[2 * stride + p]) * inv_c);
            // keep one cell of headroom so that the 27-cell stencil stays packable
            if (!key_in_range(kx - 1) || !key_in_range(kx + 1) || !key_in_range(ky - 1) || !key_in_range(ky + 1) ||
                !key_in_range(kz - 1) || !key_in_range(kz + 1))
                atomicOr(&st->err_range, 1);
            else
                key = pack_key(c, static_cast<int64_t>(kx), static_cast<int64_t>(ky), static_cast<int64_t>(kz));
        }
        const LaneRun run = lane_run(key);
        int h = -1;
        if (run.head && key != kEmptyKey) {
            h = static_cast<int>(hash_insert(keys, mask, key));
            atomicAdd(cnt + h, run.len);
        }
        h = __shfl(h, run.lead, kWave);
        if (p < m) pslot[p] = key == kEmptyKey ? -1 : h;
    }
}

__global__ __launch_bounds__(kBlock) void cell_scatter(const float* __restrict__ xyz, int64_t stride, int64_t m_cap,
                                                       const int32_t* __restrict__ pslot,
                                                       const int32_t* __restrict__ start, int32_t* fill,
                                                       float4* __restrict__ pts, const DevStatus* st) {
    const int64_t m = clamp_count(st->m_kept, m_cap);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    const int lane = lane_id();
    for (int64_t p0 = static_cast<int64_t>(blockIdx.x) * kBlock + (threadIdx.x & ~(kWave - 1)); p0 < m; p0 += gs) {
        const int64_t p = p0 + lane;
        const int h = p < m ? pslot[p] : -1;
        const LaneRun run = lane_run(h < 0 ? kEmptyKey : static_cast<uint64_t>(h));
        int base = 0;
        if (run.head && h >= 0) base = start[h] + atomicAdd(fill + h, run.len);
        base = __shfl(base, run.lead, kWave);
        if (h >= 0) pts[base + (lane - run.lead)] = make_float4(xyz[p], xyz[stride + p], xyz[2 * stride + p],
                                                               __int_as_float(static_cast<int>(p)));
    }
}

// Ascending sort of n <= W E distinct indices held in LDS, written to out, by
// a group of W lanes (a wavefront or half of one; gl = lane in the group): a
// bitonic network over W E values, value i = W u + gl in register u (partners
// closer than the group trade through shuffles within the group).
template <int E, int W>
__device__ __forceinline__ void group_sort_write(const int32_t* list, int n, int32_t* out, int gl) {
    int v[E];
#pragma unroll
    for (int u = 0; u < E; ++u) v[u] = (u * W + gl < n) ? list[u * W + gl] : INT_MAX;
#pragma unroll
    for (int k = 2; k <= E * W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= W) {
                const int ju = j / W;
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    if (u & ju) continue;
                    const int i = u * W + gl;
                    const int a = v[u], b = v[u | ju];
                    const bool asc = (i & k) == 0;
                    v[u] = asc ? min(a, b) : max(a, b);
                    v[u | ju] = asc ? max(a, b) : min(a, b);
                }
            } else {
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const int i = u * W + gl;
                    const int o = __shfl_xor(v[u], j, W);
                    v[u] = (((i & j) == 0) == ((i & k) == 0)) ? min(v[u], o) : max(v[u], o);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < E; ++u)
        if (u * W + gl < n) out[u * W + gl] = v[u];
}

template <int E>
__device__ __forceinline__ void wave_sort_write(const int32_t* list, int n, int32_t* out) {
    group_sort_write<E, kWave>(list, n, out, lane_id());
}

constexpr int kCandRounds = 4;  // candidate loads in flight per lane (list fill)
constexpr int kNbrRounds = 4;   // neighbour-list entries in flight per lane (normals)

// One wavefront per query, queries visited in cell-sorted order (grid-stride).
// kFill = false: writes |N(q)| to deg[q].
// kFill = true : writes N(q) ascending at nbr[off[q]..]; lists longer than
//                kCap are skipped (dense = 0) or are the only ones served
//                (dense = 1: the lists longer than the common fill pass
//                keeps, kListSmall, or in the list-first form (pad_cap > 0)
//                longer than a pad row: then only the cell-sorted positions
//                in long_q[0 .. st->n_long) are visited).
template <bool kFill, int kCap, int kWaves>
__global__ __launch_bounds__(kWaves* kWave) void radius_search(const CloudDev* __restrict__ cl, Grid g,
                                                               const int32_t* __restrict__ kept_cloud,
                                                               int64_t m_cap, int32_t* __restrict__ deg,
                                                               const int32_t* __restrict__ off,
                                                               int32_t* __restrict__ nbr, int64_t nbr_cap,
                                                               int dense, int use_rn, DevStatus* st,
                                                               int64_t pad_cap = 0,
                                                               const int32_t* __restrict__ long_q = nullptr) {
    __shared__ int32_t s_incl[kWaves][32];
    __shared__ int32_t s_start[kWaves][32];
    __shared__ int32_t s_list[kWaves][kFill ? kCap : 1];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t m = clamp_count(st->m_kept, m_cap);
    // lists that would overrun the caller's capacity are reported once (by the main fill pass)
    if (kFill && !dense && blockIdx.x == 0 && threadIdx.x == 0 && st->nnz > nbr_cap) st->err_capacity = 1;
    // no search over a partial grid; no fill beyond the caller's list capacity
    if (st->err_range) return;
    if (kFill && st->nnz > nbr_cap) return;
    if (kFill && dense && !(st->dense & 1)) return;  // no list exceeds the common LDS size (or a pad row)
    const int served_above = pad_cap > 0 ? pad_stride(pad_cap, m) : kListSmall;
    const int64_t n_visit = long_q ? clamp_count(st->n_long, m) : m;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWaves + wv; i < n_visit;
         i += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t w = long_q ? long_q[i] : i;
        if (w < 0 || w >= m) continue;
        const float4 qp = g.pts[w];
        const int q = __float_as_int(qp.w);
        if (q < 0 || q >= m) continue;
        if (kFill) {
            const int d = off[q + 1] - off[q];
            if (dense ? (d <= served_above) : (d > kCap)) continue;
        }
        const int c = cloud_of(kept_cloud, q);
        const double inv_c = cl[c].inv_cell;
        const RadiusTest rt = use_rn ? cl[c].rn : cl[c].rf;
        // the 27 neighbour cells: lanes 0..26 look one up each
        int cc = 0, cs = 0;
        if (lane < 27) {
            const int64_t cx = cell_coord(qp.x, inv_c) + (lane % 3) - 1;
            const int64_t cy = cell_coord(qp.y, inv_c) + (lane / 3) % 3 - 1;
            const int64_t cz = cell_coord(qp.z, inv_c) + lane / 9 - 1;
            const int h = hash_find(g.keys, g.mask, pack_key(c, cx, cy, cz));
            if (h >= 0) {
                cs = g.start[h];
                cc = g.count[h];
            }
        }
        const int incl = wave_incl_scan(cc);
        const int total = __shfl(incl, 26, kWave);
        __builtin_amdgcn_wave_barrier();
        if (lane < 32) {
            s_incl[wv][lane] = (lane < 27) ? incl : INT_MAX;
            s_start[wv][lane] = cs;
        }
        __builtin_amdgcn_wave_barrier();
        // candidates in rounds of kRounds x 64: the round's loads are all in
        // flight before the first test, and the tests keep candidate order
        constexpr int kRounds = kFill ? kCandRounds : 1;
        int found = 0;
        for (int base = 0; base < total; base += kRounds * kWave) {
            float4 sp[kRounds];
#pragma unroll
            for (int u = 0; u < kRounds; ++u) {
                const int t = base + u * kWave + lane;
                sp[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < total) {
                    int lo = 0, hi = 26;  // first cell whose inclusive prefix exceeds t
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_incl[wv][mid] > t) hi = mid;
                        else lo = mid + 1;
                    }
                    const int before = lo ? s_incl[wv][lo - 1] : 0;
                    sp[u] = g.pts[s_start[wv][lo] + (t - before)];
                }
            }
#pragma unroll
            for (int u = 0; u < kRounds; ++u) {
                const bool in = base + u * kWave + lane < total &&
                                in_radius(rt, qp.x, qp.y, qp.z, sp[u].x, sp[u].y, sp[u].z);
                const uint64_t b = ballot(in);
                if (kFill && in) {
                    const int at = found + lanes_below(b);
                    if (at < kCap) s_list[wv][at] = __float_as_int(sp[u].w);
                }
                found += __popcll(b);
            }
        }
        if (!kFill) {
            if (lane == 0) {
                deg[q] = found;
                // rare events only: no contended atomic per query
                if (found > kListSmall) atomicOr(&st->dense, found > kMaxDegree ? 3 : 1);
                if (found > kMaxDegree) atomicOr(&st->err_range, 1);  // a list beyond the supported length
            }
            continue;
        }
        __builtin_amdgcn_wave_barrier();
        int32_t* out = nbr + off[q];
        const int nf = found < kCap ? found : kCap;
        if (nf <= kWave) {
            wave_sort_write<1>(s_list[wv], nf, out);
        } else if (nf <= 2 * kWave) {
            wave_sort_write<2>(s_list[wv], nf, out);
        } else if (nf <= 4 * kWave) {
            wave_sort_write<4>(s_list[wv], nf, out);
        } else {
            // ranks are unique (distinct indices): scatter each entry to its sorted slot
            for (int e = lane; e < nf; e += kWave) {
                const int v = s_list[wv][e];
                int r = 0;
                for (int k = 0; k < nf; ++k) r += (s_list[wv][k] < v) ? 1 : 0;
                out[r] = v;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// The count pass with kCountGroups queries per wavefront, one per group of
// G = 64 / kCountGroups lanes: lane l of a group looks up cells l, l + G, ...
// of the 27, the group scans the cell counts, and the group's lanes test its
// query's candidates G at a time; the memory round trips of the wavefront's
// queries overlap.  Queries kCountGroups pw .. of the cell-sorted order go to
// wave pw; writes |N(q)| to deg[q].  kCountGroups (1, 2 or 4) and the waves
// per block are launch choices (tuning).
template <int kWaves, int kCountGroups>
__global__ __launch_bounds__(kWaves* kWave) void radius_count2(const CloudDev* __restrict__ cl, Grid g,
                                                               const int32_t* __restrict__ kept_cloud,
                                                               int64_t m_cap, int32_t* __restrict__ deg, int use_rn,
                                                               DevStatus* st) {
    constexpr int G = kWave / kCountGroups;
    constexpr int kPer = (27 + G - 1) / G;  // cells per lane
    __shared__ int32_t s_incl[kWaves][kCountGroups][32];
    __shared__ int32_t s_start[kWaves][kCountGroups][32];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int gi = lane / G, gl = lane % G, sh = G * gi;
    const uint64_t gmask = (G == kWave) ? ~0ull : (((1ull << G) - 1ull) << sh);
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (st->err_range) return;  // no search over a partial grid
    for (int64_t pw = static_cast<int64_t>(blockIdx.x) * kWaves + wv; kCountGroups * pw < m;
         pw += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t w = kCountGroups * pw + gi;
        const float4 qp = w < m ? g.pts[w] : make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
        const int q = __float_as_int(qp.w);
        const bool act = q >= 0 && q < m;
        const int c = act ? cloud_of(kept_cloud, q) : 0;
        const double inv_c = cl[c].inv_cell;
        const RadiusTest rt = use_rn ? cl[c].rn : cl[c].rf;
        // cells gl, gl + G, ... : their counts and starts
        int cc[kPer], cs[kPer];
        int mine = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int cell = gl + u * G;
            cc[u] = 0;
            cs[u] = 0;
            if (act && cell < 27) {
                const int64_t cx = cell_coord(qp.x, inv_c) + (cell % 3) - 1;
                const int64_t cy = cell_coord(qp.y, inv_c) + (cell / 3) % 3 - 1;
                const int64_t cz = cell_coord(qp.z, inv_c) + cell / 9 - 1;
                const int h = hash_find(g.keys, g.mask, pack_key(c, cx, cy, cz));
                if (h >= 0) {
                    cs[u] = g.start[h];
                    cc[u] = g.count[h];
                }
            }
            mine += cc[u];
        }
        // the group's inclusive scan of cells in order gl, gl + G, ... is taken per round u
        int base_u = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            int incl = cc[u];
#pragma unroll
            for (int d = 1; d < G; d <<= 1) {
                const int t = __shfl_up(incl, d, G);
                if (gl >= d) incl += t;
            }
            const int cell = gl + u * G;
            if (cell < 32) {
                s_incl[wv][gi][cell] = (cell < 27) ? base_u + incl : INT_MAX;
                s_start[wv][gi][cell] = cs[u];
            }
            base_u += __shfl(incl, sh + G - 1, kWave);
        }
        (void)mine;
        const int total = base_u;
        int tmax = total;
#pragma unroll
        for (int d = G; d < kWave; d <<= 1) tmax = max(tmax, __shfl_xor(tmax, d, kWave));
        __builtin_amdgcn_wave_barrier();
        int found = 0;
        for (int b0 = 0; b0 < tmax; b0 += G) {
            const int t = b0 + gl;
            bool in = false;
            if (t < total) {
                int lo = 0, hi = 26;  // first cell whose inclusive prefix exceeds t
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_incl[wv][gi][mid] > t) hi = mid;
                    else lo = mid + 1;
                }
                const int before = lo ? s_incl[wv][gi][lo - 1] : 0;
                const float4 sp = g.pts[s_start[wv][gi][lo] + (t - before)];
                in = in_radius(rt, qp.x, qp.y, qp.z, sp.x, sp.y, sp.z);
            }
            found += __popcll(ballot(in) & gmask);
        }
        if (act && gl == 0) {
            deg[q] = found;
            // rare events only: no contended atomic per query
            if (found > kListSmall) atomicOr(&st->dense, found > kMaxDegree ? 3 : 1);
            if (found > kMaxDegree) atomicOr(&st->err_range, 1);  // a list beyond the supported length
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// The common fill pass (lists of at most kListSmall entries) with two queries
// per wavefront, one per half of 32 lanes: lookups and candidate tests as the
// count pass, the found indices gathered in candidate order in the half's LDS
// list, then sorted by the half and written ascending at nbr[off[q]..].
// kFirst (the list-first form, no count pass before it): every query is
// searched, |N(q)| goes to deg[q] and the list, if it fits a row of the pad
// (nbr = pad of nbr_cap entries, row stride pad_stride), to row q, else the
// query's cell-sorted position to long_q (m entries); the later passes read
// the lists from the rows.
template <int kWaves, bool kFirst>
__global__ __launch_bounds__(kWaves* kWave) void radius_fill2(const CloudDev* __restrict__ cl, Grid g,
                                                              const int32_t* __restrict__ kept_cloud, int64_t m_cap,
                                                              const int32_t* __restrict__ off,
                                                              int32_t* __restrict__ nbr, int64_t nbr_cap,
                                                              int32_t* __restrict__ deg,
                                                              int32_t* __restrict__ long_q, int use_rn,
                                                              DevStatus* st) {
    constexpr int kHalf = kWave / 2;
    __shared__ int32_t s_incl[kWaves][2][kHalf];
    __shared__ int32_t s_start[kWaves][2][kHalf];
    __shared__ int32_t s_list[kWaves][2][kListSmall];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int hf = lane / kHalf, hl = lane % kHalf;
    const int64_t m = clamp_count(st->m_kept, m_cap);
    if (!kFirst) {
        // lists that would overrun the caller's capacity are reported once
        if (blockIdx.x == 0 && threadIdx.x == 0 && st->nnz > nbr_cap) st->err_capacity = 1;
        if (st->nnz > nbr_cap) return;  // no fill beyond the caller's list capacity
    }
    if (st->err_range) return;  // no search over a partial grid
    const int row = kFirst ? pad_stride(nbr_cap, m) : 0;
    for (int64_t pw = static_cast<int64_t>(blockIdx.x) * kWaves + wv; 2 * pw < m;
         pw += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t w = 2 * pw + hf;
        const float4 qp = w < m ? g.pts[w] : make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
        const int q = __float_as_int(qp.w);
        // longer lists are the dense pass's
        const bool act = q >= 0 && q < m && (kFirst || off[q + 1] - off[q] <= kListSmall);
        const int c = act ? cloud_of(kept_cloud, q) : 0;
        const double inv_c = cl[c].inv_cell;
        const RadiusTest rt = use_rn ? cl[c].rn : cl[c].rf;
        int cc = 0, cs = 0;
        if (act && hl < 27) {
            const int64_t cx = cell_coord(qp.x, inv_c) + (hl % 3) - 1;
            const int64_t cy = cell_coord(qp.y, inv_c) + (hl / 3) % 3 - 1;
            const int64_t cz = cell_coord(qp.z, inv_c) + hl / 9 - 1;
            const int h = hash_find(g.keys, g.mask, pack_key(c, cx, cy, cz));
            if (h >= 0) {
                cs = g.start[h];
                cc = g.count[h];
            }
        }
        int incl = cc;  // inclusive scan within the half
#pragma unroll
        for (int d = 1; d < kHalf; d <<= 1) {
            const int t = __shfl_up(incl, d, kHalf);
            if (hl >= d) incl += t;
        }
        const int total = __shfl(incl, hf * kHalf + 26, kWave);
        const int tmax = max(total, __shfl_xor(total, kHalf, kWave));
        __builtin_amdgcn_wave_barrier();
        s_incl[wv][hf][hl] = (hl < 27) ? incl : INT_MAX;
        s_start[wv][hf][hl] = cs;
        __builtin_amdgcn_wave_barrier();
        // candidates in rounds of kCandRounds x 32: the round's loads are all in
        // flight before the first test, and the tests keep candidate order
        int found = 0;
        const uint32_t below = (1u << hl) - 1u;
        for (int base = 0; base < tmax; base += kCandRounds * kHalf) {
            float4 sp[kCandRounds];
#pragma unroll
            for (int u = 0; u < kCandRounds; ++u) {
                const int t = base + u * kHalf + hl;
                sp[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < total) {
                    int lo = 0, hi = 26;  // first cell whose inclusive prefix exceeds t
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_incl[wv][hf][mid] > t) hi = mid;
                        else lo = mid + 1;
                    }
                    const int before = lo ? s_incl[wv][hf][lo - 1] : 0;
                    sp[u] = g.pts[s_start[wv][hf][lo] + (t - before)];
                }
            }
#pragma unroll
            for (int u = 0; u < kCandRounds; ++u) {
                const bool in = base + u * kHalf + hl < total &&
                                in_radius(rt, qp.x, qp.y, qp.z, sp[u].x, sp[u].y, sp[u].z);
                const uint32_t b = static_cast<uint32_t>(ballot(in) >> (kHalf * hf));
                if (in) {
                    const int at = found + __popc(b & below);
                    if (at < kListSmall) s_list[wv][hf][at] = __float_as_int(sp[u].w);
                }
                found += __popc(b);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (kFirst && act && hl == 0) {
            deg[q] = found;
            // lists beyond a pad row are listed (by cell-sorted position) for the dense pass
            if (found > row) {
                atomicOr(&st->dense, found > kMaxDegree ? 3 : 1);
                if (found > kMaxDegree) atomicOr(&st->err_range, 1);  // a list beyond the supported length
                long_q[atomicAdd(&st->n_long, 1)] = static_cast<int32_t>(w);
            }
        }
        const int nf = act && (!kFirst || found <= row) ? min(found, kListSmall) : 0;
        const int nmax = max(nf, __shfl_xor(nf, kHalf, kWave));
        int32_t* out = nbr + (act ? (kFirst ? static_cast<int64_t>(q) * row : off[q]) : 0);
        const int32_t* lst = s_list[wv][hf];
        if (nmax <= kHalf) {
            group_sort_write<1, kHalf>(lst, nf, out, hl);
        } else if (nmax <= 2 * kHalf) {
            group_sort_write<2, kHalf>(lst, nf, out, hl);
        } else if (nmax <= 4 * kHalf) {
            group_sort_write<4, kHalf>(lst, nf, out, hl);
        } else if (nmax <= 8 * kHalf) {
            group_sort_write<8, kHalf>(lst, nf, out, hl);
        } else {
            // ranks are unique (distinct indices): scatter each entry to its sorted slot
            for (int e = hl; e < nf; e += kHalf) {
                const int v = lst[e];
                int r = 0;
                for (int k = 0; k < nf; ++k) r += (lst[k] < v) ? 1 : 0;
                out[r] = v;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Cyclic Jacobi rotation in the (p, q) plane of a symmetric 3x3 matrix held
// as its six distinct entries; r is the remaining index.  V accumulates the
// eigenvectors as columns.
__device__ __forceinline__ void jacobi_plane(double& app, double& aqq, double& apq, double& arp, double& arq,
                                             double V[3][3], int p, int q) {
    if (apq == 0.0) return;
    if (fabs(apq) <= 1e-18 * (fabs(app) + fabs(aqq))) {
        apq = 0.0;
        return;
    }
    const double tau = (aqq - app) / (2.0 * apq);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = t * c;
    app -= t * apq;
    aqq += t * apq;
    apq = 0.0;
    const double rp = arp, rq = arq;
    arp = c * rp - s * rq;
    arq = s * rp + c * rq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vp = V[k][p], vq = V[k][q];
        V[k][p] = c * vp - s * vq;
        V[k][q] = s * vp + c * vq;
    }
}

__global__ __launch_bounds__(kBlock) void normals_kernel(const CloudDev* __restrict__ cl,
                                                         const float* __restrict__ xyz, int64_t stride,
                                                         const int32_t* __restrict__ kept_cloud, int64_t m_cap,
                                                         const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ nbr, int64_t nbr_cap,
                                                         float* __restrict__ nrm, int64_t nrm_stride,
                                                         uint8_t* __restrict__ flags, int32_t* __restrict__ n_normal,
                                                         DevStatus* st, const int32_t* __restrict__ pad = nullptr,
                                                         int64_t pad_cap = 0) {
    const int64_t m = clamp_count(st->m_kept, m_cap);
    // list-first form: the lists stay in their pad rows; a list volume beyond
    // the caller's capacity is reported here
    if (pad && blockIdx.x == 0 && threadIdx.x == 0 && st->nnz > nbr_cap) st->err_capacity = 1;
    if (st->err_range || st->nnz > nbr_cap) return;
    const int row = pad ? pad_stride(pad_cap, m) : 0;
    const NbrLists lists{nbr, pad, pad_cap};
    // kNormalLanes lanes per point: each sums every kNormalLanes-th list entry, then
    // the group adds up its partial moments (every lane ends with the totals)
    const int sub = lane_id() % kNormalLanes;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * (kBlock / kNormalLanes);
    for (int64_t q = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kNormalLanes; q < m; q += gs) {
        const int c = cloud_of(kept_cloud, q);
        const RadiusTest rn = cl[c].rn;
        const float qx = xyz[q], qy = xyz[stride + q], qz = xyz[2 * stride + q];
        const int b = off[q], e = off[q + 1];
        const int32_t* src = list_of(lists, row, q, b, e);
        int nn = 0;
        // moments of the r_normal subset, shifted to the query (FP64)
        double sx = 0, sy = 0, sz = 0, sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
        // kNbrRounds list entries per lane and round: their loads are in flight together
        for (int k0 = b + sub; k0 < e; k0 += kNormalLanes * kNbrRounds) {
            int id[kNbrRounds];
#pragma unroll
            for (int u = 0; u < kNbrRounds; ++u) {
                const int k = k0 + u * kNormalLanes;
                id[u] = k < e ? src[k - b] : -1;
            }
            float px[kNbrRounds], py[kNbrRounds], pz[kNbrRounds];
#pragma unroll
            for (int u = 0; u < kNbrRounds; ++u) {
                const int s = id[u] < 0 ? 0 : id[u];
                px[u] = xyz[s];
                py[u] = xyz[stride + s];
                pz[u] = xyz[2 * stride + s];
            }
#pragma unroll
            for (int u = 0; u < kNbrRounds; ++u) {
                if (id[u] < 0 || !in_radius(rn, qx, qy, qz, px[u], py[u], pz[u])) continue;
                ++nn;
                const double dx = static_cast<double>(px[u]) - qx, dy = static_cast<double>(py[u]) - qy,
                             dz = static_cast<double>(pz[u]) - qz;
                sx += dx;
                sy += dy;
                sz += dz;
                sxx += dx * dx;
                sxy += dx * dy;
                sxz += dx * dz;
                syy += dy * dy;
                syz += dy * dz;
                szz += dz * dz;
            }
        }
#pragma unroll
        for (int d = 1; d < kNormalLanes; d <<= 1) {
            nn += __shfl_xor(nn, d, kNormalLanes);
            sx += __shfl_xor(sx, d, kNormalLanes);
            sy += __shfl_xor(sy, d, kNormalLanes);
            sz += __shfl_xor(sz, d, kNormalLanes);
            sxx += __shfl_xor(sxx, d, kNormalLanes);
            sxy += __shfl_xor(sxy, d, kNormalLanes);
            sxz += __shfl_xor(sxz, d, kNormalLanes);
            syy += __shfl_xor(syy, d, kNormalLanes);
            syz += __shfl_xor(syz, d, kNormalLanes);
            szz += __shfl_xor(szz, d, kNormalLanes);
        }
        if (sub != 0) continue;  // the group's first lane finishes the point
        if (n_normal) n_normal[q] = nn;
        const int tau_num = cl[c].tau_num;
        if (e - b < tau_num || nn < tau_num) {
            nrm[q] = nrm[nrm_stride + q] = nrm[2 * nrm_stride + q] = 0.0f;
            flags[q] = 0;
            continue;
        }
        const double inv = 1.0 / nn;
        const double mx = sx * inv, my = sy * inv, mz = sz * inv;
        double a00 = sxx * inv - mx * mx, a01 = sxy * inv - mx * my, a02 = sxz * inv - mx * mz;
        double a11 = syy * inv - my * my, a12 = syz * inv - my * mz, a22 = szz * inv - mz * mz;
        double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int sweep = 0; sweep < 16; ++sweep) {
            if (a01 == 0.0 && a02 == 0.0 && a12 == 0.0) break;
            jacobi_plane(a00, a11, a01, a02, a12, V, 0, 1);
            jacobi_plane(a00, a22, a02, a01, a12, V, 0, 2);
            jacobi_plane(a11, a22, a12, a01, a02, V, 1, 2);
        }
        const double d[3] = {a00, a11, a22};
        int imax = 0, imin = 0;
#pragma unroll
        for (int i = 1; i < 3; ++i) {
            if (d[i] > d[imax]) imax = i;
            if (d[i] < d[imin]) imin = i;
        }
        if (imax == imin) {  // all eigenvalues equal
            imax = 0;
            imin = 2;
        }
        const int imid = 3 - imax - imin;
        const double l1 = d[imax], l2 = d[imid];
        double n0 = V[0][imin], n1 = V[1][imin], n2 = V[2][imin];
        const double nl = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        n0 /= nl;
        n1 /= nl;
        n2 /= nl;
        const double tx = cl[c].vp[0] - qx, ty = cl[c].vp[1] - qy, tz = cl[c].vp[2] - qz;
        const double dot = n0 * tx + n1 * ty + n2 * tz;
        bool flip = dot < 0.0;
        if (dot == 0.0) flip = (n0 != 0.0) ? (n0 < 0.0) : ((n1 != 0.0) ? (n1 < 0.0) : (n2 < 0.0));
        if (flip) {
            n0 = -n0;
            n1 = -n1;
            n2 = -n2;
        }
        if (fabs(dot) < 1e-12 * sqrt(tx * tx + ty * ty + tz * tz)) atomicAdd(&st->amb_orientation, 1u);
        const double plin = (l1 - l2) / l1;
        if (fabs(plin - cl[c].tau_lin) < 1e-12) atomicAdd(&st->amb_linearity, 1u);
        nrm[q] = static_cast<float>(n0);
        nrm[nrm_stride + q] = static_cast<float>(n1);
        nrm[2 * nrm_stride + q] = static_cast<float>(n2);
        flags[q] = (plin < cl[c].tau_lin) ? 1 : 0;
    }
}

template <int kWaves, int kGroups>
kmg_status count_as(const CloudDev* cl, Grid g, const int32_t* kept_cloud, int64_t m_cap, int32_t* deg, int use_rn,
                    DevStatus* st, hipStream_t s) {
    radius_count2<kWaves, kGroups><<<grid_cap((m_cap + kGroups - 1) / kGroups, kWaves), kWaves * kWave, 0, s>>>(
        cl, g, kept_cloud, m_cap, deg, use_rn, st);
    return launch_status();
}

template <int kWaves>
kmg_status count_waves(int groups, const CloudDev* cl, Grid g, const int32_t* kept_cloud, int64_t m_cap,
                       int32_t* deg, int use_rn, DevStatus* st, hipStream_t s) {
    switch (groups) {
        case 1: return count_as<kWaves, 1>(cl, g, kept_cloud, m_cap, deg, use_rn, st, s);
        case 4: return count_as<kWaves, 4>(cl, g, kept_cloud, m_cap, deg, use_rn, st, s);
        default: return count_as<kWaves, 2>(cl, g, kept_cloud, m_cap, deg, use_rn, st, s);
    }
}

kmg_status launch_count(int waves, int groups, const CloudDev* cl, Grid g, const int32_t* kept_cloud, int64_t m_cap,
                        int32_t* deg, int use_rn, DevStatus* st, hipStream_t s) {
    switch (waves) {
        case 2: return count_waves<2>(groups, cl, g, kept_cloud, m_cap, deg, use_rn, st, s);
        case 8: return count_waves<8>(groups, cl, g, kept_cloud, m_cap, deg, use_rn, st, s);
        default: return count_waves<4>(groups, cl, g, kept_cloud, m_cap, deg, use_rn, st, s);
    }
}

struct FillOut {
    const int32_t* off;  // nullptr: the list-first pass
    int32_t* nbr;        // the lists, or the pad of the list-first pass
    int64_t nbr_cap;
    int32_t* deg;        // list-first: |N(q)|
    int32_t* long_q;     // list-first: positions of the lists beyond a pad row
};

template <int kWaves, bool kFirst>
kmg_status fill_as(const CloudDev* cl, Grid g, const int32_t* kept_cloud, int64_t m_cap, const FillOut& o,
                   int use_rn, DevStatus* st, hipStream_t s) {
    radius_fill2<kWaves, kFirst><<<grid_cap((m_cap + 1) / 2, kWaves), kWaves * kWave, 0, s>>>(
        cl, g, kept_cloud, m_cap, o.off, o.nbr, o.nbr_cap, o.deg, o.long_q, use_rn, st);
    return launch_status();
}

template <bool kFirst>
kmg_status fill_form(int waves, const CloudDev* cl, Grid g, const int32_t* kept_cloud, int64_t m_cap,
                     const FillOut& o, int use_rn, DevStatus* st, hipStream_t s) {
    switch (waves) {
        case 2: return fill_as<2, kFirst>(cl, g, kept_cloud, m_cap, o, use_rn, st, s);
        case 8: return fill_as<8, kFirst>(cl, g, kept_cloud, m_cap, o, use_rn, st, s);
        default: return fill_as<4, kFirst>(cl, g, kept_cloud, m_cap, o, use_rn, st, s);
    }
}

kmg_status launch_fill(int waves, const CloudDev* cl, Grid g, const int32_t* kept_cloud, int64_t m_cap,
                       const FillOut& o, int use_rn, DevStatus* st, hipStream_t s) {
    return o.off ? fill_form<false>(waves, cl, g, kept_cloud, m_cap, o, use_rn, st, s)
                 : fill_form<true>(waves, cl, g, kept_cloud, m_cap, o, use_rn, st, s);
}

Grid grid_of(const SearchWs& w) {
    Grid g;
    g.pts = w.pts;
    g.keys = w.keys;
    g.start = w.cstart;
    g.count = w.ccount;
    g.mask = w.cap_table - 1;
    return g;
}

}  // namespace

SearchWs carve_search(Carver& c, int64_t m_cap) {
    SearchWs w;
    w.cap_table = next_pow2(static_cast<uint64_t>(std::max<int64_t>(2 * m_cap, 64)));
    w.keys = c.take<uint64_t>(w.cap_table);
    w.ccount = c.take<int32_t>(w.cap_table);
    w.cstart = c.take<int32_t>(w.cap_table);
    w.cfill = c.take<int32_t>(w.cap_table);
    w.pslot = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(m_cap, 1)));
    w.pts = c.take<float4>(static_cast<size_t>(std::max<int64_t>(m_cap, 1)));
    w.deg = c.take<int32_t>(static_cast<size_t>(m_cap) + 1);
    w.scan_tmp = c.take<int64_t>(std::max(scan_temp_elems(m_cap + 1), scan_temp_elems(w.cap_table)));
    return w;
}

namespace {

// inserted: the kept points are in the cell hash already (voxelize_batch put
// them there as it emitted them); the counts are then scanned and scattered.
kmg_status build_grid(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud, int64_t m_cap,
                      DevStatus* st, const SearchWs& w, hipStream_t s, bool cleared, bool inserted,
                      uint64_t* scan_status = nullptr) {
    StageScope sc(ST_GRID, s);
    if (!cleared) {
        KMG_TRY(fill_u64(w.keys, kEmptyKey, w.cap_table, s));
        KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.ccount), 0u, w.cap_table, s));
        KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.cfill), 0u, w.cap_table, s));
    }
    if (m_cap > 0 && !inserted) {
        cell_insert<<<grid_cap(m_cap, kBlock), kBlock, 0, s>>>(cl, xyz, stride, kept_cloud, m_cap, w.keys,
                                                              w.ccount, w.cap_table - 1, w.pslot, st);
        KMG_TRY(launch_status());
    }
    if (scan_status)
        KMG_TRY(scan_exclusive_onepass(w.ccount, w.cstart, w.cap_table, &st->n_cells, scan_status, &st->err_sync, s));
    else
        KMG_TRY(scan_exclusive(w.ccount, w.cstart, w.cap_table, &st->n_cells, w.scan_tmp, s));
    if (m_cap > 0) {
        cell_scatter<<<grid_cap(m_cap, kBlock), kBlock, 0, s>>>(xyz, stride, m_cap, w.pslot, w.cstart, w.cfill,
                                                               w.pts, st);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

}  // namespace

kmg_status search_count_batch(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                              int64_t m_cap, DevStatus* st, const SearchWs& w, int32_t* off, hipStream_t s,
                              bool grid, int use_rn, bool cleared, bool inserted) {
    if (grid) KMG_TRY(build_grid(cl, xyz, stride, kept_cloud, m_cap, st, w, s, cleared, inserted));
    {
        StageScope sc(ST_SEARCH_COUNT, s);
        if (!cleared) KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.deg), 0u, static_cast<size_t>(m_cap) + 1, s));
        if (m_cap > 0) {
            const Tuning& t = tuning();
            KMG_TRY(launch_count(t.search_waves, t.count_queries, cl, grid_of(w), kept_cloud, m_cap, w.deg, use_rn,
                                 st, s));
        }
        KMG_TRY(scan_exclusive(w.deg, off, m_cap + 1, &st->nnz, w.scan_tmp, s));
    }
    return KMG_OK;
}

size_t search_scan_status_elems(const SearchWs& w, int64_t m_cap) {
    return scan_temp_elems(w.cap_table) + scan_temp_elems(m_cap + 1);
}

kmg_status search_lists_first(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                              int64_t m_cap, int64_t nbr_cap, DevStatus* st, const SearchWs& w, int32_t* off,
                              int32_t* nbr, int32_t* pad, int64_t pad_cap, int32_t* long_q, float* nrm,
                              int64_t nrm_stride, uint8_t* flags, hipStream_t s, bool inserted,
                              uint64_t* scan_status) {
    KMG_TRY(build_grid(cl, xyz, stride, kept_cloud, m_cap, st, w, s, true, inserted, scan_status));
    if (m_cap > 0) {
        StageScope sc(ST_SEARCH_FILL, s);
        KMG_TRY(launch_fill(tuning().search_waves, cl, grid_of(w), kept_cloud, m_cap,
                            FillOut{nullptr, pad, pad_cap, w.deg, long_q}, 0, st, s));
    }
    {
        StageScope sc(ST_SEARCH_COUNT, s);
        if (scan_status)
            KMG_TRY(scan_exclusive_onepass(w.deg, off, m_cap + 1, &st->nnz, scan_status + scan_temp_elems(w.cap_table),
                                           &st->err_sync, s));
        else
            KMG_TRY(scan_exclusive(w.deg, off, m_cap + 1, &st->nnz, w.scan_tmp, s));
    }
    if (m_cap <= 0) return KMG_OK;
    {
        StageScope sc(ST_SEARCH_FILL, s);
        radius_search<true, kMaxDegree, 1><<<grid_cap(m_cap, 1), kWave, 0, s>>>(
            cl, grid_of(w), kept_cloud, m_cap, nullptr, off, nbr, nbr_cap, 1, 0, st, pad_cap, long_q);
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_NORMALS, s);
        normals_kernel<<<grid_cap(m_cap * kNormalLanes, kBlock), kBlock, 0, s>>>(
            cl, xyz, stride, kept_cloud, m_cap, off, nbr, nbr_cap, nrm, nrm_stride, flags, nullptr, st, pad, pad_cap);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

kmg_status search_fill_batch(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                             int64_t m_cap, int64_t nbr_cap, bool dense_pass, DevStatus* st, const SearchWs& w,
                             const int32_t* off, int32_t* nbr, float* nrm, int64_t nrm_stride, uint8_t* flags,
                             int32_t* n_normal, hipStream_t s, int use_rn, bool with_normals) {
    if (m_cap <= 0) return KMG_OK;
    {
        StageScope sc(ST_SEARCH_FILL, s);
        KMG_TRY(launch_fill(tuning().search_waves, cl, grid_of(w), kept_cloud, m_cap,
                            FillOut{off, nbr, nbr_cap, nullptr, nullptr}, use_rn, st, s));
        if (dense_pass) {
            radius_search<true, kMaxDegree, 1><<<grid_cap(m_cap, 1), kWave, 0, s>>>(
                cl, grid_of(w), kept_cloud, m_cap, nullptr, off, nbr, nbr_cap, 1, use_rn, st);
            KMG_TRY(launch_status());
        }
    }
    if (with_normals) {
        StageScope sc(ST_NORMALS, s);
        normals_kernel<<<grid_cap(m_cap * kNormalLanes, kBlock), kBlock, 0, s>>>(
            cl, xyz, stride, kept_cloud, m_cap, off, nbr, nbr_cap, nrm, nrm_stride, flags, n_normal, st);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

}  // namespace kmg
