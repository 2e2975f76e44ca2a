// Mutual nearest-neighbour matching of descriptor rows (reciprocity test,
// Section III-C) on gfx950 matrix cores, with exact FP64 decisions.
//
// Candidate generation.  For a query row y and swept rows x_i, the NN ranks
// D(i) = ||x_i||^2 + ||y||^2 - 2 x_i.y by t_i = ||x_i||^2 - 2 x_i.y.  FPFH rows
// cluster tightly (nearest-neighbour distances are often 1e-5 of the squared
// norms), so this expanded form is evaluated on FP64 matrix cores: rows are
// packed k-major in 16-row chunks with the squared norm appended as an extra
// "dimension" (A = [x, ||x||^2]), queries use B = [-2 y, 1], and one
// v_mfma_f64_16x16x4_f64 chain of ceil((dim+1)/4) steps yields a 16x16 tile
// of t.  Lane l owns query column l % 16 and tile rows l / 16 + {0, 4, 8, 12}
// (result register r holds row 4 r + l / 16), and keeps a running top-4 of t
// in registers.  A wave holds 64 query
// columns (four chains), a block of four waves 256, and the swept rows are
// split into S segments; block b takes segment b % S (S is a multiple of 8
// when possible, so each of the eight XCDs streams one eighth of the rows
// through its own L2).
//
// Exact decision.  The per-segment top-4 lists are merged, the four
// candidates are re-scored with the plain FP64 sum of squared differences in
// dimension order, and the result is certified: every non-candidate has
// t >= t_4 (the 4th candidate's value) and |t - exact| <= E with
// E = 128 u (2 max ||x||^2 + 2 ||y||^2), u = 2^-53 (the dot-product rounding
// bound is (dim + 2) u times ||x||^2 + 2 x.y <= 2 ||x||^2 + ||y||^2).  If the
// exact second-best distance is below t_4 + ||y||^2 - E, the exact best and
// second-best over all rows are among the candidates; otherwise the query is
// re-scanned exactly in FP64.
#include <math.h>

#include "kmg_device.h"

namespace kmg {

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kTileRows = 16;     // rows per packed chunk (MFMA M)
constexpr int kTileCols = 16;     // query columns per MFMA tile (MFMA N)
constexpr int kTilesPerWave = 4;  // 64 query columns per wave
constexpr int kColsPerWave = kTileCols * kTilesPerWave;
constexpr int kWavesPerBlock = 4;
constexpr int kColsPerBlock = kColsPerWave * kWavesPerBlock;
constexpr int kBlock = 256;

struct Packed {
    const double* pk;  // [chunks][kp][16]
    int n;             // rows
    int chunks;
    int kp;            // packed depth (multiple of 4)
};

// ---------------------------------------------------------------- packing --

__global__ __launch_bounds__(kBlock) void row_norms(const float* __restrict__ desc, const int32_t* __restrict__ rows,
                                                    int n, int dim, double* __restrict__ nrm2,
                                                    unsigned long long* max_bits) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float* x = desc + static_cast<int64_t>(rows ? rows[i] : i) * dim;
    double acc = 0.0;
    for (int t = 0; t < dim; ++t) {
        const double v = x[t];
        acc = acc + v * v;
    }
    nrm2[i] = acc;
    atomicMax(max_bits, static_cast<unsigned long long>(__double_as_longlong(acc)));
}

__global__ __launch_bounds__(kBlock) void pack_rows(const float* __restrict__ desc, const int32_t* __restrict__ rows,
                                                    int n, int dim, int kp, int chunks,
                                                    const double* __restrict__ nrm2, double* __restrict__ pk) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t total = static_cast<int64_t>(chunks) * kp * kTileRows;
    if (t >= total) return;
    const int ii = static_cast<int>(t % kTileRows);
    const int k = static_cast<int>((t / kTileRows) % kp);
    const int c = static_cast<int>(t / (static_cast<int64_t>(kTileRows) * kp));
    const int i = c * kTileRows + ii;
    double v = 0.0;
    if (i < n) {
        if (k < dim) v = desc[static_cast<int64_t>(rows ? rows[i] : i) * dim + k];
        else if (k == dim) v = nrm2[i];
    } else if (k == dim) {
        v = INFINITY;  // padding rows never enter a top-k list
    }
    pk[t] = v;
}

// ----------------------------------------------------------- top-4 passes --

struct Top4 {
    double v0, v1, v2, v3;
    int i0, i1, i2, i3;
    __device__ void init() {
        v0 = v1 = v2 = v3 = INFINITY;
        i0 = i1 = i2 = i3 = -1;
    }
    __device__ __forceinline__ void push(double v, int i) {
        if (!(v < v3)) return;
        if (v < v2) {
            v3 = v2;
            i3 = i2;
            if (v < v1) {
                v2 = v1;
                i2 = i1;
                if (v < v0) {
                    v1 = v0;
                    i1 = i0;
                    v0 = v;
                    i0 = i;
                } else {
                    v1 = v;
                    i1 = i;
                }
            } else {
                v2 = v;
                i2 = i;
            }
        } else {
            v3 = v;
            i3 = i;
        }
    }
};

// (value, index) order used wherever lists are merged: deterministic.
__device__ __forceinline__ bool before(double va, int ia, double vb, int ib) {
    return va < vb || (va == vb && static_cast<unsigned>(ia) < static_cast<unsigned>(ib));
}

// Insertion into a sorted Top4 under the (value, index) order.
__device__ __forceinline__ void push_ordered(Top4& t, double v, int ix) {
    if (!before(v, ix, t.v3, t.i3)) return;
    if (before(v, ix, t.v2, t.i2)) {
        t.v3 = t.v2;
        t.i3 = t.i2;
        if (before(v, ix, t.v1, t.i1)) {
            t.v2 = t.v1;
            t.i2 = t.i1;
            if (before(v, ix, t.v0, t.i0)) {
                t.v1 = t.v0;
                t.i1 = t.i0;
                t.v0 = v;
                t.i0 = ix;
            } else {
                t.v1 = v;
                t.i1 = ix;
            }
        } else {
            t.v2 = v;
            t.i2 = ix;
        }
    } else {
        t.v3 = v;
        t.i3 = ix;
    }
}

// Merges the top-4 list of lane l ^ d into this lane's list.
__device__ __forceinline__ void merge_lanes(Top4& t, int d) {
    const double v0 = __shfl_xor(t.v0, d, kWave), v1 = __shfl_xor(t.v1, d, kWave);
    const double v2 = __shfl_xor(t.v2, d, kWave), v3 = __shfl_xor(t.v3, d, kWave);
    const int i0 = __shfl_xor(t.i0, d, kWave), i1 = __shfl_xor(t.i1, d, kWave);
    const int i2 = __shfl_xor(t.i2, d, kWave), i3 = __shfl_xor(t.i3, d, kWave);
    push_ordered(t, v0, i0);
    push_ordered(t, v1, i1);
    push_ordered(t, v2, i2);
    push_ordered(t, v3, i3);
}

template <int KS>
__global__ __launch_bounds__(kBlock) void topk_pass(Packed A, Packed B, int dim, int segs, int chunks_per_seg,
                                                    double* __restrict__ part_v, int32_t* __restrict__ part_i) {
    const int seg = blockIdx.x % segs;
    const int cblk = blockIdx.x / segs;
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int col0 = cblk * kColsPerBlock + wv * kColsPerWave;
    if (col0 >= B.n) return;
    const int g = lane >> 4;   // k offset within a step for the operands; row group for the result
    const int l16 = lane & 15;
    // query operand: B[k][j] = -2 y_j[k] (k < dim), 1 (k = dim), 0 beyond
    double bq[kTilesPerWave][KS];
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        const int chunk = col0 / kTileCols + t;
        const bool have = chunk < B.chunks;
        const double* src = B.pk + static_cast<int64_t>(have ? chunk : 0) * B.kp * kTileRows;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + g;
            const double v = (have && k < B.kp) ? src[k * kTileRows + l16] : 0.0;
            bq[t][s] = (k < dim) ? -2.0 * v : (k == dim ? 1.0 : 0.0);
        }
    }
    Top4 top[kTilesPerWave];
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) top[t].init();
    const int c_begin = seg * chunks_per_seg;
    const int c_end = min(c_begin + chunks_per_seg, A.chunks);
    // the A operand of chunk c + 1 is loaded while chunk c is multiplied
    double a_next[KS];
    if (c_begin < c_end) {
        const double* src = A.pk + static_cast<int64_t>(c_begin) * A.kp * kTileRows;
#pragma unroll
        for (int s = 0; s < KS; ++s) a_next[s] = (4 * s + g < A.kp) ? src[s * 4 * kTileRows + lane] : 0.0;
    }
    for (int c = c_begin; c < c_end; ++c) {
        double a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = a_next[s];
        if (c + 1 < c_end) {
            const double* src = A.pk + static_cast<int64_t>(c + 1) * A.kp * kTileRows;
#pragma unroll
            for (int s = 0; s < KS; ++s) a_next[s] = (4 * s + g < A.kp) ? src[s * 4 * kTileRows + lane] : 0.0;
        }
        doublex4 acc[kTilesPerWave];
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
            for (int t = 0; t < kTilesPerWave; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bq[t][s], acc[t], 0, 0, 0);
        }
        // result register r of lane l holds tile row 4 r + l / 16, column l % 16
        const int row0 = c * kTileRows + g;
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) {
            const double mn = fmin(fmin(acc[t][0], acc[t][1]), fmin(acc[t][2], acc[t][3]));
            if (mn < top[t].v3) {
#pragma unroll
                for (int r = 0; r < 4; ++r) top[t].push(acc[t][r], row0 + 4 * r);
            }
        }
    }
    // the four row groups of a column (lanes l, l ^ 16, l ^ 32, l ^ 48) merge their lists
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        merge_lanes(top[t], 16);
        merge_lanes(top[t], 32);
        const int col = col0 + kTileCols * t + l16;
        if (g == 0 && col < B.n) {
            const int64_t base = (static_cast<int64_t>(seg) * B.n + col) * kTopK;
            part_v[base + 0] = top[t].v0;
            part_v[base + 1] = top[t].v1;
            part_v[base + 2] = top[t].v2;
            part_v[base + 3] = top[t].v3;
            part_i[base + 0] = top[t].i0;
            part_i[base + 1] = top[t].i1;
            part_i[base + 2] = top[t].i2;
            part_i[base + 3] = top[t].i3;
        }
    }
}

// ------------------------------------------------------ exact re-scoring --

__device__ __forceinline__ double exact_d2(const float* __restrict__ x, const float* __restrict__ y, int dim) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int t = 0; t < dim; ++t) {
        const double df = static_cast<double>(x[t]) - static_cast<double>(y[t]);
        acc = acc + df * df;
    }
    return acc;
}

struct Side {
    const float* desc;
    const int32_t* rows;
    int n;
    __device__ const float* row(int i, int dim) const {
        return desc + static_cast<int64_t>(rows ? rows[i] : i) * dim;
    }
};

// One thread per query: merge the S x 4 partial candidates, re-score the best
// four exactly, certify or queue the query for an exact scan.
__global__ __launch_bounds__(kBlock) void rescore(Side X, Side Y, int dim, int segs,
                                                  const double* __restrict__ part_v, const int32_t* __restrict__ part_i,
                                                  const double* __restrict__ ny2,
                                                  const unsigned long long* __restrict__ max_x_bits,
                                                  int32_t* __restrict__ nn, double* __restrict__ best,
                                                  double* __restrict__ second, int32_t* __restrict__ fb_list,
                                                  uint32_t* fb_count) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= Y.n) return;
    Top4 t;
    t.init();
    for (int sg = 0; sg < segs; ++sg) {
        const int64_t base = (static_cast<int64_t>(sg) * Y.n + j) * kTopK;
#pragma unroll
        for (int e = 0; e < kTopK; ++e) {
            const double v = part_v[base + e];
            const int ix = part_i[base + e];
            if (ix < 0 || ix >= X.n) continue;  // only real rows are ever candidates
            push_ordered(t, v, ix);
        }
    }
    const float* y = Y.row(j, dim);
    const int cand[4] = {t.i0, t.i1, t.i2, t.i3};
    double b1 = INFINITY, b2 = INFINITY;
    int j1 = -1;
    int ncand = 0;
    for (int r = 0; r < 4; ++r) {
        const int i = cand[r];
        if (i < 0) continue;
        ++ncand;
        const double d = exact_d2(X.row(i, dim), y, dim);
        if (d < b1 || (d == b1 && i < j1)) {
            b2 = b1;
            b1 = d;
            j1 = i;
        } else if (d < b2) {
            b2 = d;
        }
    }
    bool ok;
    if (ncand >= X.n) {
        ok = true;  // every row was a candidate
    } else {
        const double mx = __longlong_as_double(static_cast<long long>(*max_x_bits));
        const double E = 128.0 * 1.1102230246251565e-16 * (2.0 * mx + 2.0 * ny2[j]) + 1e-300;
        const double bound = t.v3 + ny2[j] - E;
        ok = ncand == 4 && b2 < bound;
    }
    if (ok) {
        nn[j] = j1;
        best[j] = b1;
        second[j] = b2;
    } else {
        const uint32_t at = atomicAdd(fb_count, 1u);
        fb_list[at] = j;
    }
}

// One wavefront per queued query: exact FP64 scan over all rows of X.
__global__ __launch_bounds__(kBlock) void exact_scan(Side X, Side Y, int dim, const int32_t* __restrict__ fb_list,
                                                     const uint32_t* fb_count, int32_t* __restrict__ nn,
                                                     double* __restrict__ best, double* __restrict__ second) {
    const int w = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (w >= static_cast<int>(*fb_count)) return;
    const int lane = lane_id();
    const int j = fb_list[w];
    const float* y = Y.row(j, dim);
    double b1 = INFINITY, b2 = INFINITY;
    int j1 = INT32_MAX;
    for (int i = lane; i < X.n; i += kWave) {  // ascending per lane
        const double d = exact_d2(X.row(i, dim), y, dim);
        if (d < b1) {
            b2 = b1;
            b1 = d;
            j1 = i;
        } else if (d < b2) {
            b2 = d;
        }
    }
    // combine lanes: smallest (b1, j1); second = min of the other b1s and all b2s
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const double ob1 = __shfl_xor(b1, d, kWave);
        const double ob2 = __shfl_xor(b2, d, kWave);
        const int oj1 = __shfl_xor(j1, d, kWave);
        const bool mine = (b1 < ob1) || (b1 == ob1 && j1 < oj1);
        const double nb2 = mine ? fmin(b2, ob1) : fmin(ob2, b1);
        if (!mine) {
            b1 = ob1;
            j1 = oj1;
        }
        b2 = nb2;
    }
    if (lane == 0) {
        nn[j] = (j1 == INT32_MAX) ? -1 : j1;
        best[j] = b1;
        second[j] = b2;
    }
}

__global__ __launch_bounds__(kBlock) void mutual_flags(const int32_t* __restrict__ nn_pq,
                                                       const int32_t* __restrict__ nn_qp, int np,
                                                       int32_t* __restrict__ flag) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= np) return;
    const int j = nn_pq[i];
    flag[i] = (j >= 0 && nn_qp[j] == i) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void emit_pairs(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                                     const int32_t* __restrict__ nn_pq, const double* __restrict__ best,
                                                     const double* __restrict__ second,
                                                     const int32_t* __restrict__ rows_p,
                                                     const int32_t* __restrict__ rows_q, int np, const int64_t* total,
                                                     int64_t cap, int32_t* __restrict__ pairs, float* __restrict__ d1,
                                                     float* __restrict__ d2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= np || !flag[i]) return;
    if (*total > cap) return;
    const int at = pos[i];
    const int j = nn_pq[i];
    pairs[2 * at] = rows_p ? rows_p[i] : i;
    pairs[2 * at + 1] = rows_q ? rows_q[j] : j;
    d1[at] = static_cast<float>(sqrt(best[i]));
    d2[at] = static_cast<float>(sqrt(second[i]));
}

int choose_segments(int chunks_a, int n_queries) {
    const int cblocks = (n_queries + kColsPerBlock - 1) / kColsPerBlock;
    int s = std::max(1, 1024 / std::max(1, cblocks));
    if (s >= 8) s &= ~7;
    s = std::min(s, std::max(1, chunks_a));
    return s;
}

struct Dir {
    int segs;
    double* part_v;
    int32_t* part_i;
    int32_t* nn;
    double* best;
    double* second;
    int32_t* fb_list;
    uint32_t* fb_count;
};

struct MatchWs {
    DevStatus* st;
    double* pk_p;
    double* pk_q;
    double* n2_p;
    double* n2_q;
    unsigned long long* max_bits;  // [0] P, [1] Q
    Dir dir[2];                    // 0: queries P over rows Q; 1: queries Q over rows P
    int32_t* flag;
    int32_t* pos;
    int64_t* total;
    int64_t* scan_tmp;
    int kp, chunks_p, chunks_q;
};

MatchWs carve(Carver& c, int64_t np, int64_t nq, int dim) {
    MatchWs w;
    w.kp = (dim + 1 + 3) / 4 * 4;
    w.chunks_p = static_cast<int>((np + kTileRows - 1) / kTileRows);
    w.chunks_q = static_cast<int>((nq + kTileRows - 1) / kTileRows);
    w.st = c.take<DevStatus>(1);
    w.pk_p = c.take<double>(static_cast<size_t>(w.chunks_p) * w.kp * kTileRows);
    w.pk_q = c.take<double>(static_cast<size_t>(w.chunks_q) * w.kp * kTileRows);
    w.n2_p = c.take<double>(static_cast<size_t>(np));
    w.n2_q = c.take<double>(static_cast<size_t>(nq));
    w.max_bits = c.take<unsigned long long>(2);
    const int64_t nqry[2] = {np, nq};
    const int rows_chunks[2] = {w.chunks_q, w.chunks_p};
    for (int d = 0; d < 2; ++d) {
        Dir& D = w.dir[d];
        D.segs = choose_segments(rows_chunks[d], static_cast<int>(nqry[d]));
        D.part_v = c.take<double>(static_cast<size_t>(nqry[d]) * D.segs * kTopK);
        D.part_i = c.take<int32_t>(static_cast<size_t>(nqry[d]) * D.segs * kTopK);
        D.nn = c.take<int32_t>(static_cast<size_t>(nqry[d]));
        D.best = c.take<double>(static_cast<size_t>(nqry[d]));
        D.second = c.take<double>(static_cast<size_t>(nqry[d]));
        D.fb_list = c.take<int32_t>(static_cast<size_t>(nqry[d]));
        D.fb_count = c.take<uint32_t>(1);
    }
    w.flag = c.take<int32_t>(static_cast<size_t>(np));
    w.pos = c.take<int32_t>(static_cast<size_t>(np));
    w.total = c.take<int64_t>(2);
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(np));
    return w;
}

template <int KS>
kmg_status run_pass(const Packed& A, const Packed& B, int dim, const Dir& D, hipStream_t s) {
    const int cps = (A.chunks + D.segs - 1) / D.segs;
    const int cblocks = (B.n + kColsPerBlock - 1) / kColsPerBlock;
    topk_pass<KS><<<static_cast<unsigned>(cblocks * D.segs), kBlock, 0, s>>>(A, B, dim, D.segs, cps, D.part_v,
                                                                           D.part_i);
    return launch_status();
}

}  // namespace

size_t match_ws(int64_t np, int64_t nq, int dim) {
    Carver c(nullptr, 0);
    carve(c, np, nq, dim);
    return c.off;
}

kmg_status match(const float* dp, const int32_t* rp, int64_t np, const float* dq, const int32_t* rq, int64_t nq,
                 int dim, int prec, int32_t* pairs, float* d1, float* d2, int64_t cap, int64_t* n_pairs_host,
                 int64_t* n_fallback_host, void* ws, size_t ws_bytes, hipStream_t s) {
    if (prec != KMG_FP32) return KMG_ERR_ARG;
    Carver c(ws, ws_bytes);
    MatchWs w = carve(c, np, nq, dim);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    *n_pairs_host = 0;
    if (n_fallback_host) *n_fallback_host = 0;
    if (np == 0 || nq == 0) return KMG_OK;
    const int npi = static_cast<int>(np), nqi = static_cast<int>(nq);
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.st), 0u, sizeof(DevStatus) / 4, s));
    KMG_TRY(fill_u64(reinterpret_cast<uint64_t*>(w.max_bits), 0ull, 2, s));
    {
    StageScope sc(ST_MATCH_PACK, s);
    row_norms<<<grid_for(np, kBlock), kBlock, 0, s>>>(dp, rp, npi, dim, w.n2_p, w.max_bits);
    KMG_TRY(launch_status());
    row_norms<<<grid_for(nq, kBlock), kBlock, 0, s>>>(dq, rq, nqi, dim, w.n2_q, w.max_bits + 1);
    KMG_TRY(launch_status());
    const int64_t tp = static_cast<int64_t>(w.chunks_p) * w.kp * kTileRows;
    const int64_t tq = static_cast<int64_t>(w.chunks_q) * w.kp * kTileRows;
    pack_rows<<<grid_for(tp, kBlock), kBlock, 0, s>>>(dp, rp, npi, dim, w.kp, w.chunks_p, w.n2_p, w.pk_p);
    KMG_TRY(launch_status());
    pack_rows<<<grid_for(tq, kBlock), kBlock, 0, s>>>(dq, rq, nqi, dim, w.kp, w.chunks_q, w.n2_q, w.pk_q);
    KMG_TRY(launch_status());
    }
    const Packed P{w.pk_p, npi, w.chunks_p, w.kp};
    const Packed Q{w.pk_q, nqi, w.chunks_q, w.kp};
    const Side SP{dp, rp, npi}, SQ{dq, rq, nqi};
    // direction 0: queries P over rows Q; direction 1: queries Q over rows P
    const int ks = w.kp / 4;
    for (int d = 0; d < 2; ++d) {
        const Packed& A = d == 0 ? Q : P;
        const Packed& B = d == 0 ? P : Q;
        KMG_TRY(fill_u32(w.dir[d].fb_count, 0u, 1, s));
        StageScope sc(ST_MATCH_TOPK, s);
        if (ks <= 9) {
            KMG_TRY(run_pass<9>(A, B, dim, w.dir[d], s));
        } else if (ks <= 17) {
            KMG_TRY(run_pass<17>(A, B, dim, w.dir[d], s));
        } else {
            return KMG_ERR_ARG;
        }
    }
    for (int d = 0; d < 2; ++d) {
        const Side& X = d == 0 ? SQ : SP;
        const Side& Y = d == 0 ? SP : SQ;
        const Dir& D = w.dir[d];
        StageScope sc(ST_MATCH_RESCORE, s);
        rescore<<<grid_for(Y.n, kBlock), kBlock, 0, s>>>(X, Y, dim, D.segs, D.part_v, D.part_i,
                                                        d == 0 ? w.n2_p : w.n2_q, w.max_bits + (d == 0 ? 1 : 0),
                                                        D.nn, D.best, D.second, D.fb_list, D.fb_count);
        KMG_TRY(launch_status());
        // one wave per queued query; waves beyond the queue length exit at once
        exact_scan<<<grid_for(Y.n, kBlock / kWave), kBlock, 0, s>>>(X, Y, dim, D.fb_list, D.fb_count, D.nn,
                                                                   D.best, D.second);
        KMG_TRY(launch_status());
    }
    {
    StageScope sc(ST_MATCH_MUTUAL, s);
    mutual_flags<<<grid_for(np, kBlock), kBlock, 0, s>>>(w.dir[0].nn, w.dir[1].nn, npi, w.flag);
    KMG_TRY(launch_status());
    KMG_TRY(scan_exclusive(w.flag, w.pos, np, w.total, w.scan_tmp, s));
    emit_pairs<<<grid_for(np, kBlock), kBlock, 0, s>>>(w.flag, w.pos, w.dir[0].nn, w.dir[0].best, w.dir[0].second,
                                                      rp, rq, npi, w.total, cap, pairs, d1, d2);
    KMG_TRY(launch_status());
    }
    int64_t npairs = 0;
    uint32_t fb[2] = {0, 0};
    KMG_TRY_HIP(hipMemcpyAsync(&npairs, w.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipMemcpyAsync(&fb[0], w.dir[0].fb_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipMemcpyAsync(&fb[1], w.dir[1].fb_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    timer_collect();
    *n_pairs_host = npairs;
    if (n_fallback_host) *n_fallback_host = static_cast<int64_t>(fb[0]) + fb[1];
    if (npairs > cap) return KMG_ERR_CAPACITY;
    return KMG_OK;
}

}  // namespace kmg
