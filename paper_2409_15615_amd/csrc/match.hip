// Mutual nearest-neighbour matching of descriptor rows (reciprocity test,
// Section III-C) on gfx950 matrix cores, with exact FP64 decisions, for every
// pair of a batch at once.
//
// Sets.  Descriptor sets 2i and 2i+1 form pair i; each set is matched against
// its partner in both directions.  Set sizes live on the device; a one-block
// planner lays out query slots, packed chunks, tiles and candidate buffers.
//
// Candidate generation.  For a query row y and swept rows x_i, the NN ranks
// D(i) = ||x_i||^2 + ||y||^2 - 2 x_i.y by t_i = ||x_i||^2 - 2 x_i.y.  FPFH rows
// cluster tightly (nearest-neighbour distances are often 1e-5 of the squared
// norms), so this expanded form is evaluated on FP64 matrix cores: rows are
// packed k-major in 16-row chunks with the squared norm appended as an extra
// "dimension" (A = [x, ||x||^2]), queries use B = [-2 y, 1], and one
// v_mfma_f64_16x16x4_f64 chain of ceil((dim+1)/4) steps yields a 16x16 tile
// of t.  Lane l owns query column l % 16 and tile rows l / 16 + {0, 4, 8, 12}
// (result register r holds row 4 r + l / 16).  Each score carries its row
// index in its low mantissa bits, and every lane keeps a running top-4 of
// encoded scores with min/max networks.  A wave holds 64 query columns (four
// chains), a block of four waves 256.  A tile is (set, 256-query block,
// segment of the partner's rows); a persistent grid pulls tiles from an
// atomic queue until it is empty, so uneven pairs share one launch.
//
// Exact decision.  The per-segment lists are merged, the four candidates are
// re-scored with the plain FP64 sum of squared differences in dimension
// order, and the result is certified: every non-candidate has an encoded
// score >= t_4 (the 4th candidate's), its computed t is within 2^(bits-52)|t|
// of the encoded one, and |t - exact| <= 128 u (2 max ||x||^2 + 2 ||y||^2),
// u = 2^-53 (the dot-product rounding bound is (dim + 2) u times
// ||x||^2 + 2 x.y <= 2 ||x||^2 + ||y||^2).  If the exact second-best distance
// is below t_4 + ||y||^2 minus both bounds, the exact best and second-best
// over all rows are among the candidates; otherwise the query is re-scanned
// exactly in FP64.
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
constexpr int kPlanThreads = 1024;
constexpr int kTargetTiles = 8192;  // tiles per launch the partial buffer is sized for
constexpr int kMaxSegs = 128;
constexpr double kTileOverhead = 2.0;  // fixed cost of a tile, in partner chunks
constexpr int kSegChunks = 64;     // deepest tile (partner chunks) once a set needs more segments
constexpr int kTopkBlocks = 512;    // persistent grid of the tile kernel (2 blocks per CU)
constexpr double kPadScore = 0x1p1000;  // score of padding rows: finite, so it can carry an index
constexpr double kNoScore = 0x1p999;    // list entries at or above this are no row

// Set of a flattened index given non-decreasing starts (last s with start <= t).
template <class F>
__device__ __forceinline__ int find_set(int n_sets, int64_t t, F start) {
    int lo = 0, hi = n_sets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start(mid) <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ const float* set_row(const MatchSet& s, int i, int dim) {
    return s.desc + static_cast<int64_t>(s.rows ? s.rows[i] : i) * dim;
}

// ------------------------------------------------------------------ sets --

__global__ void write_pair_sets(MatchSet* sets, int32_t* counts, MatchSet a, MatchSet b, int32_t na, int32_t nb,
                                PairOutDev* outs, PairOutDev out) {
    counts[0] = na;
    counts[1] = nb;
    a.n = counts;
    b.n = counts + 1;
    sets[0] = a;
    sets[1] = b;
    outs[0] = out;
}

// ------------------------------------------------------------------ plan --

__device__ int64_t block_excl_scan64(int64_t v, int64_t* smem, int64_t& total) {
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int64_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) smem[wave] = incl;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int w = 0; w < kPlanThreads / kWave; ++w) {
        const int64_t t = smem[w];
        if (w < wave) before += t;
        total += t;
    }
    __syncthreads();
    return before + incl - v;
}

// Common segment count.  The persistent grid takes the tiles in rounds of
// kTopkBlocks; a tile costs its sweep of partner chunks plus a fixed overhead
// (query operands, list merges and stores) of about kTileOverhead chunks.  The
// count with the least modelled time wins: enough tiles to keep every block
// busy to the end, few enough that the overhead stays small.  From 8 on only
// multiples of 8 are tried.
__device__ int common_segs(int64_t col_blocks, int64_t chunk_work) {
    if (col_blocks <= 0 || chunk_work <= 0) return 1;
    int best = 1;
    double best_t = INFINITY;
    for (int S = 1; S <= kMaxSegs; S = S < 8 ? S + 1 : S + 8) {
        const int64_t tiles = col_blocks * S;
        const int64_t rounds = (tiles + kTopkBlocks - 1) / kTopkBlocks;
        const double t = static_cast<double>(rounds) *
                         (static_cast<double>(chunk_work) / static_cast<double>(tiles) + kTileOverhead);
        if (t < best_t) {
            best_t = t;
            best = S;
        }
    }
    return best;
}

__global__ __launch_bounds__(kPlanThreads) void plan_sets(const MatchSet* __restrict__ sets, int n_sets, int kp,
                                                         int64_t part_cap, SetPlan* plan, DevStatus* st,
                                                         int32_t* __restrict__ grp_done, int64_t n_grp) {
    __shared__ int64_t smem[kPlanThreads / kWave];
    __shared__ int s_segs;
    __shared__ int s_chunks[kPlanThreads];
    __shared__ int s_n[kPlanThreads];
    for (int64_t g = threadIdx.x; g < n_grp; g += kPlanThreads) grp_done[g] = 0;  // for the exact scans
    const int c = threadIdx.x;
    const bool live = c < n_sets;
    const bool rows_only = live && (sets[c].flags & kSetRowsOnly);
    int n = live ? *sets[c].n : 0;
    if (rows_only && (c ^ 1) < n_sets) {
        // rows that no query is matched against need neither slots nor packing
        const MatchSet& o = sets[c ^ 1];
        if ((o.flags & kSetRowsOnly) || *o.n == 0) n = 0;
    }
    const int chunks = (n + kTileRows - 1) / kTileRows;
    const int cblocks = rows_only ? 0 : (n + kColsPerBlock - 1) / kColsPerBlock;
    const int n_q = rows_only ? 0 : n;  // queries that need partial lists
    int64_t tq, tc, tb;
    const int64_t q_off = block_excl_scan64(n, smem, tq);
    const int64_t c_off = block_excl_scan64(chunks, smem, tc);
    block_excl_scan64(cblocks, smem, tb);
    s_chunks[c] = chunks;
    s_n[c] = n;
    // one buffer descriptor spans a set's packed rows: keep them below 2 GiB
    if (static_cast<int64_t>(chunks) * kp * kTileRows * 8 > INT32_MAX) st->err_capacity = 1;
    __syncthreads();
    // the partner's rows are split into segments (sets pair up as 2i, 2i + 1): at least the
    // common count, and enough that no tile sweeps more than kSegChunks chunks, so the tiles
    // of uneven batches stay comparable in size
    const int p = c ^ 1;
    const int pch = (live && p < n_sets) ? s_chunks[p] : 0;
    const int pn = (live && p < n_sets) ? s_n[p] : 0;
    int64_t tw;
    block_excl_scan64((live && pn > 0) ? static_cast<int64_t>(cblocks) * pch : 0, smem, tw);
    if (c == 0) s_segs = common_segs(tb, tw);
    __syncthreads();
    const int deep = (pch + kSegChunks - 1) / kSegChunks;
    int segs = s_segs > deep ? s_segs : deep;
    segs = segs < pch ? segs : (pch > 0 ? pch : 1);
    int64_t tpart;
    block_excl_scan64(live ? static_cast<int64_t>(n_q) * segs * kTopK : 0, smem, tpart);
    if (tpart > part_cap) {
        // too many partial lists for the buffer: one common count, halved until they fit
        // (one segment per set always fits, the buffer holds kTopK entries per query)
        if (c == 0) {
            int S = s_segs;
            while (S > 1 && tq * S * kTopK > part_cap) S >>= 1;
            s_segs = S;
        }
        __syncthreads();
        segs = s_segs < pch ? s_segs : (pch > 0 ? pch : 1);
    }
    const int tiles = (live && pn > 0) ? cblocks * segs : 0;
    int64_t tt;
    const int64_t t_off = block_excl_scan64(tiles, smem, tt);
    const int64_t p_off = block_excl_scan64(live ? static_cast<int64_t>(n_q) * segs * kTopK : 0, smem, tpart);
    if (live) {
        SetPlan pl;
        pl.n = n;
        pl.q_off = static_cast<int32_t>(q_off);
        pl.chunk_off = static_cast<int32_t>(c_off);
        pl.chunks = chunks;
        pl.tile_off = static_cast<int32_t>(t_off);
        pl.cblocks = cblocks;
        pl.segs = segs;
        pl.n_fb = 0;
        pl.part_off = p_off;
        pl.max_norm_bits = 0ull;
        pl.wave_off = 0;
        pl.n_img = 0;
        plan[c] = pl;
    }
    if (c == 0) {
        st->total_queries = static_cast<int32_t>(tq);
        st->total_chunks = tc;
        st->total_tiles = static_cast<int32_t>(tt);
        st->tile_next = 0;
        st->n_fallback = 0;
        if (tpart > part_cap) st->err_capacity = 1;
    }
}

// ------------------------------------------------------------- packing --

// plan[c].max_norm_bits = max(.., v) (v >= 0): one atomic per wave when the
// wave's live lanes share a set (the common case).
__device__ __forceinline__ void wave_max_norm(SetPlan* plan, int c, double v) {
    const uint64_t live = ballot(true);
    const int c0 = __shfl(c, __ffsll(static_cast<unsigned long long>(live)) - 1, kWave);
    const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(v));
    if (ballot(c == c0) == live) {
        unsigned long long mx = bits;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const unsigned long long o = __shfl_xor(mx, d, kWave);
            const bool o_live = (live >> (lane_id() ^ d)) & 1ull;
            if (o_live && o > mx) mx = o;
        }
        if (lane_id() == __ffsll(static_cast<unsigned long long>(live)) - 1) atomicMax(&plan[c].max_norm_bits, mx);
    } else {
        atomicMax(&plan[c].max_norm_bits, bits);
    }
}

// Squared norms per slot (and rank[slot] = 0 when rank is given).
__global__ __launch_bounds__(kBlock) void row_norms(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                    int dim, double* __restrict__ n2, const DevStatus* st,
                                                    int32_t* __restrict__ rank) {
#pragma clang fp contract(off)
    const int64_t total = st->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total; t += gs) {
        const int c = find_set(n_sets, t, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const float* x = set_row(sets[c], static_cast<int>(t - plan[c].q_off), dim);
        double acc = 0.0;
        int k = 0;
        for (; k + 8 <= dim; k += 8) {  // eight loads in flight, the sum in order
            float xs[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) xs[u] = x[k + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double v = xs[u];
                acc = acc + v * v;
            }
        }
        for (; k < dim; ++k) {
            const double v = x[k];
            acc = acc + v * v;
        }
        n2[t] = acc;
        if (rank) rank[t] = 0;
        wave_max_norm(plan, c, acc);
    }
}

__global__ __launch_bounds__(kBlock) void pack_rows(const MatchSet* __restrict__ sets,
                                                    const SetPlan* __restrict__ plan, int n_sets, int dim, int kp,
                                                    const double* __restrict__ n2, double* __restrict__ pk,
                                                    const DevStatus* st) {
    const int64_t total = st->total_chunks * kp * kTileRows;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total; t += gs) {
        const int ii = static_cast<int>(t % kTileRows);
        const int k = static_cast<int>((t / kTileRows) % kp);
        const int64_t g = t / (static_cast<int64_t>(kTileRows) * kp);
        const int c = find_set(n_sets, g, [&](int s) { return static_cast<int64_t>(plan[s].chunk_off); });
        const int i = static_cast<int>(g - plan[c].chunk_off) * kTileRows + ii;
        double v = 0.0;
        if (i < plan[c].n) {
            if (k < dim) v = set_row(sets[c], i, dim)[k];
            else if (k == dim) v = n2[plan[c].q_off + i];
        } else if (k == dim) {
            v = kPadScore;  // padding rows never enter a top-k list
        }
        pk[t] = v;
    }
}

// ------------------------------------------------------ candidate lists --
//
// A candidate is a score t with its partner row index written into the low
// `bits` mantissa bits, bits = the width of the partner's padded row count.
// Encoded scores of distinct rows never compare equal, so a top-4 list is four
// doubles kept ascending by min/max networks: no branches and no index
// registers.  An encoded score differs from t by less than 2^(bits - 52) |t|,
// which the certificate adds to its error bound.

__device__ __forceinline__ int row_bits(int chunks) {
    const unsigned rows = static_cast<unsigned>(chunks) * kTileRows;  // >= 16
    return 32 - __clz(static_cast<int>(rows - 1u));
}

__device__ __forceinline__ unsigned keep_mask(int bits) { return bits >= 32 ? 0u : ~((1u << bits) - 1u); }

__device__ __forceinline__ double encode(double t, unsigned keep, unsigned row) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(t));
    const unsigned lo = (static_cast<unsigned>(u) & keep) | row;
    return __longlong_as_double(static_cast<long long>((u & 0xffffffff00000000ull) | lo));
}

__device__ __forceinline__ int decode_row(double v, unsigned keep) {
    return static_cast<int>(static_cast<unsigned>(__double_as_longlong(v)) & ~keep);
}

__device__ __forceinline__ void cex(double& a, double& b) {
    const double lo = fmin(a, b), hi = fmax(a, b);
    a = lo;
    b = hi;
}

// Ascending sort of four values: five compare-exchanges.
__device__ __forceinline__ void sort4(double& a, double& b, double& c, double& d) {
    cex(a, b);
    cex(c, d);
    cex(a, c);
    cex(b, d);
    cex(b, c);
}

// top <- the four smallest of top and w, both ascending (bitonic merge).
__device__ __forceinline__ void merge4(double* top, double w0, double w1, double w2, double w3) {
    double m0 = fmin(top[0], w3), m1 = fmin(top[1], w2), m2 = fmin(top[2], w1), m3 = fmin(top[3], w0);
    cex(m0, m2);
    cex(m1, m3);
    cex(m0, m1);
    cex(m2, m3);
    top[0] = m0;
    top[1] = m1;
    top[2] = m2;
    top[3] = m3;
}

// Merges the list of lane l ^ d into this lane's list.
__device__ __forceinline__ void merge_lane(double* top, int d) {
    const double o0 = __shfl_xor(top[0], d, kWave), o1 = __shfl_xor(top[1], d, kWave);
    const double o2 = __shfl_xor(top[2], d, kWave), o3 = __shfl_xor(top[3], d, kWave);
    merge4(top, o0, o1, o2, o3);
}

// Folds the four scores of one result register set (rows row0 + 4 r) into top.
__device__ __forceinline__ void absorb(double* top, const doublex4& acc, unsigned row0, unsigned keep) {
    double w0 = encode(acc[0], keep, row0), w1 = encode(acc[1], keep, row0 + 4u);
    double w2 = encode(acc[2], keep, row0 + 8u), w3 = encode(acc[3], keep, row0 + 12u);
    sort4(w0, w1, w2, w3);
    merge4(top, w0, w1, w2, w3);
}

template <int KS>
__device__ __forceinline__ void chunk_mfma(doublex4* acc, const double* a, const double (*bq)[KS]) {
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bq[t][s], acc[t], 0, 0, 0);
    }
}

// A packed chunk (4 KS x 16 doubles, k-major) moves through LDS in 16-byte
// pieces: each thread of the block stages kPieces of them in registers.  The
// loads are raw buffer loads on a descriptor that spans the partner's packed
// rows: they keep their place before the products (plain global loads get
// sunk to their first use), and an offset past the range reads zeros instead
// of faulting.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr unsigned kBufferWord3 = 0x00020000u;  // raw buffer, 32-bit data format (gfx9)

template <int KS>
struct ChunkStage {
    static constexpr int kPiecesPerChunk = 4 * KS * kTileRows / 2;
    static constexpr int kPieces = (kPiecesPerChunk + kBlock - 1) / kBlock;
    double2 r[kPieces];
    // indices past the chunk are clamped: those threads load and store the last piece again
    __device__ __forceinline__ static int piece(int e) {
        return min(static_cast<int>(threadIdx.x) + e * kBlock, kPiecesPerChunk - 1);
    }
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rows, int chunk) {
#pragma unroll
        for (int e = 0; e < kPieces; ++e) {
            const int off = (chunk * kPiecesPerChunk + piece(e)) * 16;
            r[e] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rows, off, 0, 0));
        }
    }
    __device__ __forceinline__ void store(double2* buf) const {
#pragma unroll
        for (int e = 0; e < kPieces; ++e) buf[piece(e)] = r[e];
    }
};

// One block: four waves of 64 query columns each (set qc, local columns from
// col0) against the partner's chunks [c_begin, c_end).  The chunk sequence is
// shared by the four waves through a double-buffered LDS stage: the raw
// buffer loads of chunk c + 1 issue before the products of chunk c and land in
// LDS after its list update, one barrier per chunk.  Query chunks past the
// set's end are clamped to its last chunk (their columns are >= n and never
// written), so every wave runs the same loop.
template <int KS>
__device__ __forceinline__ void tile_block(const double* __restrict__ pk, int dim, const SetPlan& qc,
                                           const SetPlan& pc, int col0, int c_begin, int c_end, int seg,
                                           double* __restrict__ part, double2* lds) {
    constexpr int kp = 4 * KS;
    constexpr int kChunk = kp * kTileRows;  // doubles per packed chunk
    const int lane = lane_id();
    const int g = lane >> 4;  // k offset within a step for the operands; row group for the result
    const int l16 = lane & 15;
    // query operand: B[k][j] = -2 y_j[k] (k < dim), 1 (k = dim), 0 beyond
    double bq[kTilesPerWave][KS];
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        const int chunk = min(col0 / kTileCols + t, qc.chunks - 1);
        const double* src = pk + static_cast<int64_t>(qc.chunk_off + chunk) * kChunk;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            // arithmetic rather than a select, so that the load is never predicated
            const int k = 4 * s + g;
            const double scale = k < dim ? -2.0 : 0.0;
            const double add = k == dim ? 1.0 : 0.0;
            bq[t][s] = src[k * kTileRows + l16] * scale + add;
        }
    }
    double top[kTilesPerWave][4];
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) top[t][0] = top[t][1] = top[t][2] = top[t][3] = INFINITY;
    const unsigned keep = keep_mask(row_bits(pc.chunks));
    if (c_begin < c_end) {  // uniform over the block
        // the planner flags sets whose packed rows exceed 2 GiB, the reach used for one descriptor
        const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double*>(pk + static_cast<int64_t>(pc.chunk_off) * kChunk), 0,
            static_cast<int>(min(static_cast<int64_t>(pc.chunks) * kChunk * 8, static_cast<int64_t>(INT32_MAX))),
            static_cast<int>(kBufferWord3));
        constexpr int kBuf = kChunk / 2;  // double2 per LDS buffer
        const double* lds_d = reinterpret_cast<const double*>(lds);
        ChunkStage<KS> stage;
        stage.load(rows, c_begin);
        stage.store(lds);
        __syncthreads();
        for (int c = c_begin; c < c_end; ++c) {
            const int buf = (c - c_begin) & 1;
            double a[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) a[s] = lds_d[buf * kChunk + s * 4 * kTileRows + lane];
            stage.load(rows, min(c + 1, c_end - 1));
            // keep the loads ahead of the products and the LDS stores after the
            // list update: the load latency then hides behind a whole chunk
            __builtin_amdgcn_sched_barrier(0);
            doublex4 acc[kTilesPerWave];
            chunk_mfma<KS>(acc, a, bq);
            // result register r of lane l holds tile row 4 r + l / 16, column l % 16
            const unsigned row0 = static_cast<unsigned>(c * kTileRows + g);
#pragma unroll
            for (int t = 0; t < kTilesPerWave; ++t) absorb(top[t], acc[t], row0, keep);
            __builtin_amdgcn_sched_barrier(0);
            stage.store(lds + (buf ^ 1) * kBuf);
            __syncthreads();
        }
    }
    // the four row groups of a column (lanes l, l ^ 16, l ^ 32, l ^ 48) merge their lists
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        merge_lane(top[t], 16);
        merge_lane(top[t], 32);
        const int col = col0 + kTileCols * t + l16;
        if (g == 0 && col < qc.n) {
            double* dst = part + qc.part_off + (static_cast<int64_t>(seg) * qc.n + col) * kTopK;
            dst[0] = top[t][0];
            dst[1] = top[t][1];
            dst[2] = top[t][2];
            dst[3] = top[t][3];
        }
    }
}

// Persistent tile kernel: blocks pull (set, column block, segment) tiles from
// an atomic queue; every block leaves once the queue runs past the tile count.
// Two waves per SIMD for the 36-deep form (the second wave covers the
// barrier, LDS and load latencies of the first); the 68-deep form needs the
// whole register file of one.
template <int KS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KS <= 9 ? 2 : 1))) void topk_tiles(const SetPlan* __restrict__ plan, int n_sets,
                                                     const double* __restrict__ pk, int dim,
                                                     double* __restrict__ part, DevStatus* st) {
    __shared__ double2 lds[2 * 4 * KS * kTileRows / 2];
    __shared__ int s_tile;
    const int wv = threadIdx.x / kWave;
    const int total = st->err_capacity ? 0 : st->total_tiles;
    // the first tile of every block is fixed (XCD-aware order), the rest come from the queue
    // counted from kTopkBlocks: one round takes no atomic
    for (int tile = static_cast<int>(xcd_block_index()); tile < total;) {
        const int c = find_set(n_sets, tile, [&](int s) { return static_cast<int64_t>(plan[s].tile_off); });
        const SetPlan qc = plan[c];
        const SetPlan pc = plan[c ^ 1];
        const int local = tile - qc.tile_off;
        const int seg = local % qc.segs;
        const int cblk = local / qc.segs;
        const int cps = (pc.chunks + qc.segs - 1) / qc.segs;
        const int c_begin = seg * cps;
        const int c_end = min(c_begin + cps, pc.chunks);
        const int col0 = cblk * kColsPerBlock + wv * kColsPerWave;
        tile_block<KS>(pk, dim, qc, pc, col0, c_begin, c_end, seg, part, lds);
        if (total <= kTopkBlocks) break;  // uniform: every tile was a first tile
        __syncthreads();                  // every thread has read s_tile
        if (threadIdx.x == 0) s_tile = kTopkBlocks + static_cast<int>(atomicAdd(&st->tile_next, 1u));
        __syncthreads();
        tile = s_tile;
    }
}

// ------------------------------------------------------ exact re-scoring --

// The plain FP64 sum in dimension order; the loads of eight dimensions issue
// together (the sum keeps its order).
// Adds one to plan[c].n_fb for every active lane (c its set), with one atomic
// per distinct set among them: tens of thousands of open queries of one set
// would otherwise queue on a single address.
__device__ __forceinline__ void count_open(SetPlan* plan, int c) {
    uint64_t pending = ballot(true);
    while (pending) {  // uniform over the active lanes
        const int lead = __ffsll(static_cast<unsigned long long>(pending)) - 1;
        const int cl = __shfl(c, lead, kWave);
        const uint64_t same = ballot(c == cl);
        if (lane_id() == lead) atomicAdd(&plan[cl].n_fb, static_cast<int32_t>(__popcll(same)));
        pending &= ~same;
    }
}

// As count_open, and each active lane's slot lands at fl[q_off + its place]
// in its set's range; the list total grows by the number of active lanes.
__device__ __forceinline__ void append_open(SetPlan* plan, int c, int64_t q_off, int32_t slot, int32_t* fl,
                                            int64_t* f_total) {
    const uint64_t act = ballot(true);
    uint64_t pending = act;
    int k = 0;
    while (pending) {  // uniform over the active lanes
        const int lead = __ffsll(static_cast<unsigned long long>(pending)) - 1;
        const int cl = __shfl(c, lead, kWave);
        const uint64_t same = ballot(c == cl);
        int at = 0;
        if (lane_id() == lead) at = atomicAdd(&plan[cl].n_fb, static_cast<int32_t>(__popcll(same)));
        at = __shfl(at, lead, kWave);
        if (c == cl) k = at + lanes_below(same);
        pending &= ~same;
    }
    fl[q_off + k] = slot;
    if (lane_id() == __ffsll(static_cast<unsigned long long>(act)) - 1)
        atomicAdd(reinterpret_cast<unsigned long long*>(f_total), static_cast<unsigned long long>(__popcll(act)));
}

__device__ __forceinline__ double exact_d2(const float* __restrict__ x, const float* __restrict__ y, int dim) {
#pragma clang fp contract(off)
    double acc = 0.0;
    int t = 0;
    for (; t + 8 <= dim; t += 8) {
        float xs[8], ys[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            xs[u] = x[t + u];
            ys[u] = y[t + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double df = static_cast<double>(xs[u]) - static_cast<double>(ys[u]);
            acc = acc + df * df;
        }
    }
    for (; t < dim; ++t) {
        const double df = static_cast<double>(x[t]) - static_cast<double>(y[t]);
        acc = acc + df * df;
    }
    return acc;
}

constexpr int kQuad = 4;  // lanes per query in the re-scoring kernel

// Four lanes per query slot: lane q merges the segment lists q, q + 4, ..,
// the quad merges its lists, lane q re-scores candidate q exactly, and the
// first lane certifies the result or flags the query for an exact scan.
__global__ __launch_bounds__(kBlock) void rescore(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                  int dim, const double* __restrict__ part,
                                                  const double* __restrict__ n2, int32_t* __restrict__ nn,
                                                  double* __restrict__ best, double* __restrict__ second,
                                                  int32_t* __restrict__ failed, DevStatus* st) {
    const int64_t total = st->total_queries;
    const int q = lane_id() & (kQuad - 1);
    const int quad0 = lane_id() & ~(kQuad - 1);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * (kBlock / kQuad);
    for (int64_t slot = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kQuad; slot < total;
         slot += gs) {
        const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        if (sets[c].flags & kSetRowsOnly) {  // uniform over the quad: no queries
            if (q == 0) failed[slot] = 0;
            continue;
        }
        const int p = c ^ 1;
        const SetPlan qc = plan[c];
        const int j = static_cast<int>(slot - qc.q_off);
        const int np = p < n_sets ? plan[p].n : 0;
        if (np == 0) {
            if (q == 0) {
                nn[slot] = -1;
                best[slot] = INFINITY;
                second[slot] = INFINITY;
                failed[slot] = 0;
            }
            continue;
        }
        double top[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
        for (int sg = q; sg < qc.segs; sg += kQuad) {
            const double* src = part + qc.part_off + (static_cast<int64_t>(sg) * qc.n + j) * kTopK;
            merge4(top, src[0], src[1], src[2], src[3]);
        }
        merge_lane(top, 1);
        merge_lane(top, 2);
        const int bits = row_bits(plan[p].chunks);
        const double mine = q == 0 ? top[0] : (q == 1 ? top[1] : (q == 2 ? top[2] : top[3]));
        int row = -1;
        if (mine < kNoScore) {
            row = decode_row(mine, keep_mask(bits));
            if (row >= np) row = -1;  // only real rows are ever candidates
        }
        const double d = row >= 0 ? exact_d2(set_row(sets[p], row, dim), set_row(sets[c], j, dim), dim) : INFINITY;
        double dq[kQuad];
        int rq[kQuad];
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            dq[k] = __shfl(d, quad0 + k, kWave);
            rq[k] = __shfl(row, quad0 + k, kWave);
        }
        if (q != 0) continue;
        double b1 = INFINITY, b2 = INFINITY;
        int j1 = -1;
        int ncand = 0;
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            const int i = rq[k];
            if (i < 0) continue;
            ++ncand;
            const double dk = dq[k];
            if (dk < b1 || (dk == b1 && i < j1)) {
                b2 = b1;
                b1 = dk;
                j1 = i;
            } else if (dk < b2) {
                b2 = dk;
            }
        }
        bool ok;
        if (ncand >= np) {
            ok = true;  // every row was a candidate
        } else {
            // MFMA error 128 u (2 max ||x||^2 + 2 ||y||^2) plus the encoding error
            // 2^(bits - 52) |t| with |t| <= 2 ||x||^2 + ||y||^2
            const double mx = __longlong_as_double(static_cast<long long>(plan[p].max_norm_bits));
            const double rel = 0x1p-46 + ldexp(1.0, bits - 52);
            const double E = rel * (2.0 * mx + 2.0 * n2[slot]) + 1e-300;
            const double bound = top[3] + n2[slot] - E;
            ok = ncand == 4 && b2 < bound;
        }
        if (ok) {
            nn[slot] = j1;
            best[slot] = b1;
            second[slot] = b2;
        } else {
            count_open(plan, c);
        }
        failed[slot] = ok ? 0 : 1;
    }
}

// Combines two (best, its index, second) triples: smallest (b1, j1) first;
// the second is the smallest of the other best and both seconds.
__device__ __forceinline__ void combine_best(double& b1, int& j1, double& b2, double ob1, int oj1, double ob2) {
    const bool mine = (b1 < ob1) || (b1 == ob1 && j1 < oj1);
    const double nb2 = mine ? fmin(b2, ob1) : fmin(ob2, b1);
    if (!mine) {
        b1 = ob1;
        j1 = oj1;
    }
    b2 = nb2;
}

constexpr int kXSegMax = 32;  // row segments per group of the exact scan

// Row segments of the exact scan: as many as the partial buffer holds for F
// listed queries, at most kXSegMax.
__device__ __forceinline__ int exact_segs(int64_t F, int64_t part_cap) {
    const int64_t s = F > 0 ? part_cap / (3 * F) : 1;
    return static_cast<int>(s < 1 ? 1 : (s > kXSegMax ? kXSegMax : s));
}

// Exact FP64 scans for the listed queries, *f_total of them: fl[0 .. F) in
// any order (slot order keeps a group within few sets), or (per_set) the
// lists of the sets, plan[c].n_fb entries from fl[plan[c].q_off] on, in
// groups that never span two sets.  A work item is (group of up to 64 entries, row
// segment): lane L of every wave holds entry L in registers as FP64, padded with
// zeros to 4 KS values, the partner rows of the segment stream through LDS as
// FP64 with the same zero padding (a padded term adds an exact zero), and each
// wave scores every fourth row, ascending, two rows at a time, with the plain
// FP64 sum in dimension order.  The four waves merge their (best, index, second) and write
// them as the segment's partial result; a group that spans several sets visits
// their partners one after another.  The block that finishes a group's last
// segment (counted in grp_done, which the planner zeroed) merges the group's
// partials in segment order into nn, best and second, and resets the count.
template <int KS>
__global__ __launch_bounds__(kBlock) void exact_grouped(const MatchSet* __restrict__ sets,
                                                        const SetPlan* __restrict__ plan, int n_sets, int dim,
                                                        const int32_t* __restrict__ fl,
                                                        const int64_t* __restrict__ f_total, int per_set,
                                                        int64_t part_cap, double* __restrict__ part,
                                                        int32_t* __restrict__ grp_done,
                                                        int32_t* __restrict__ nn, double* __restrict__ best,
                                                        double* __restrict__ second) {
#pragma clang fp contract(off)
    constexpr int kD = 4 * KS;                   // padded row length
    constexpr int kXRows = KS <= 9 ? 128 : 64;   // partner rows per LDS tile
    __shared__ __attribute__((aligned(16))) double s_x[kXRows * kD];
    __shared__ const float* s_row[kXRows];
    __shared__ double s_b1[kBlock], s_b2[kBlock];
    __shared__ int s_j1[kBlock];
    __shared__ int s_next;
    __shared__ int s_pre[kPlanThreads + 1];   // per-set lists: the sets' first entries
    __shared__ int s_gpre[kPlanThreads + 1];  // and first groups
    constexpr int kWaves = kBlock / kWave;
    const int L = threadIdx.x % kWave;
    const int wv = threadIdx.x / kWave;
    const int64_t F = *f_total;
    if (F == 0) return;  // uniform: nothing listed
    for (int i = threadIdx.x; i < kXRows * (kD - dim); i += kBlock)  // the padding, zero for good
        s_x[(i / (kD - dim)) * kD + dim + i % (kD - dim)] = 0.0;
    if (per_set) {
        if (wv == 0) {  // lane L sums sets [kPer L, kPer (L + 1)), then the wave scans the sums
            constexpr int kPer = (kPlanThreads + kWave) / kWave;
            int v[kPer];
            int sum = 0, gsum = 0;
            for (int k = 0; k < kPer; ++k) {
                const int c = L * kPer + k;
                v[k] = c < n_sets ? plan[c].n_fb : 0;
                sum += v[k];
                gsum += (v[k] + kWave - 1) / kWave;
            }
            int run = wave_incl_scan(sum) - sum;
            int grun = wave_incl_scan(gsum) - gsum;
            for (int k = 0; k < kPer; ++k) {
                const int c = L * kPer + k;
                if (c <= n_sets) {
                    s_pre[c] = run;
                    s_gpre[c] = grun;
                }
                run += v[k];
                grun += (v[k] + kWave - 1) / kWave;
            }
        }
        __syncthreads();
    }
    const int S = exact_segs(F, part_cap);
    double* pb1 = part;
    double* pb2 = part + F * S;
    int32_t* pj1 = reinterpret_cast<int32_t*>(part + 2 * F * S);
    const int64_t groups = per_set ? s_gpre[n_sets] : (F + kWave - 1) / kWave;
    const int64_t items = groups * S;
    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t g = item / S;
        const int sg = static_cast<int>(item % S);
        // lane L: the group's entry L (dense index e into the partials) and its slot
        int64_t e;
        bool have;
        int64_t slot = 0;
        if (!per_set) {
            e = g * kWave + L;
            have = e < F;
            if (have) slot = fl[e];
        } else {
            int lo = 0, hi = n_sets - 1;  // the group's set: the last whose first group is <= g
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_gpre[mid] <= g) lo = mid;
                else hi = mid - 1;
            }
            const int local = static_cast<int>(g - s_gpre[lo]) * kWave + L;
            have = local < s_pre[lo + 1] - s_pre[lo];
            e = s_pre[lo] + local;
            if (have) slot = fl[plan[lo].q_off + local];
        }
        const int c_e = have ? find_set(n_sets, slot, [&](int q) { return static_cast<int64_t>(plan[q].q_off); })
                             : INT_MAX;
        double y[kD];
        {
            const float* yr = have ? set_row(sets[c_e], static_cast<int>(slot - plan[c_e].q_off), dim) : nullptr;
#pragma unroll
            for (int t = 0; t < kD; ++t) y[t] = (have && t < dim) ? static_cast<double>(yr[t]) : 0.0;
        }
        // the group's sets in increasing order, from the smallest (the list may come in any order)
        if (threadIdx.x == 0) s_next = INT_MAX;
        __syncthreads();
        if (c_e != INT_MAX) atomicMin(&s_next, c_e);
        __syncthreads();
        int c_cur = s_next;
        double b1 = INFINITY, b2 = INFINITY;
        int j1 = INT_MAX;
        while (true) {
            const int p = c_cur ^ 1;
            const int np = p < n_sets ? plan[p].n : 0;
            const int len = (np + S - 1) / S;
            const int r_begin = min(np, sg * len), r_end = min(np, r_begin + len);
            for (int r0 = r_begin; r0 < r_end; r0 += kXRows) {
                const int nr = min(kXRows, r_end - r0);
                __syncthreads();
                // the tile's rows: their addresses first, then all values by all threads,
                // eight loads in flight per thread
                if (static_cast<int>(threadIdx.x) < nr)
                    s_row[threadIdx.x] = set_row(sets[p], r0 + static_cast<int>(threadIdx.x), dim);
                __syncthreads();
                const int n_el = nr * dim;
                for (int e0 = static_cast<int>(threadIdx.x); e0 < n_el; e0 += 8 * kBlock) {
                    float v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kBlock;
                        v[u] = e < n_el ? s_row[e / dim][e % dim] : 0.0f;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kBlock;
                        if (e < n_el) s_x[(e / dim) * kD + e % dim] = static_cast<double>(v[u]);
                    }
                }
                __syncthreads();
                if (c_e == c_cur) {
                    auto take = [&](double acc, int j) {
                        if (acc < b1) {
                            b2 = b1;
                            b1 = acc;
                            j1 = j;
                        } else if (acc < b2) {
                            b2 = acc;
                        }
                    };
                    for (int r = wv; r < nr; r += 2 * kWaves) {
                        const bool two = r + kWaves < nr;  // wave-uniform
                        const double2* xa = reinterpret_cast<const double2*>(s_x + r * kD);
                        const double2* xb = reinterpret_cast<const double2*>(s_x + (two ? r + kWaves : r) * kD);
                        double a = 0.0, b = 0.0;
#pragma unroll
                        for (int t = 0; t < kD / 2; ++t) {
                            const double2 va = xa[t], vb = xb[t];
                            const double da0 = va.x - y[2 * t], db0 = vb.x - y[2 * t];
                            a = a + da0 * da0;
                            b = b + db0 * db0;
                            const double da1 = va.y - y[2 * t + 1], db1 = vb.y - y[2 * t + 1];
                            a = a + da1 * da1;
                            b = b + db1 * db1;
                        }
                        take(a, r0 + r);
                        if (two) take(b, r0 + r + kWaves);
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) s_next = INT_MAX;
            __syncthreads();
            if (c_e != INT_MAX && c_e > c_cur) atomicMin(&s_next, c_e);
            __syncthreads();
            const int nx = s_next;
            if (nx == INT_MAX) break;
            c_cur = nx;
        }
        s_b1[threadIdx.x] = b1;
        s_b2[threadIdx.x] = b2;
        s_j1[threadIdx.x] = j1;
        __syncthreads();
        if (wv == 0 && have) {
            for (int o = 1; o < kWaves; ++o)
                combine_best(b1, j1, b2, s_b1[o * kWave + L], s_j1[o * kWave + L], s_b2[o * kWave + L]);
            pb1[e * S + sg] = b1;
            pb2[e * S + sg] = b2;
            pj1[e * S + sg] = j1;
        }
        // wave 0 wrote the partials: it publishes them and counts the segment
        if (wv == 0) {
            __threadfence();
            int last = 0;
            if (L == 0) last = atomicAdd(&grp_done[g], 1) == S - 1;
            last = __shfl(last, 0, kWave);
            if (last) {
                __threadfence();  // the other segments' partials are visible from here on
                if (have) {
                    double m1 = pb1[e * S], m2 = pb2[e * S];
                    int mj = pj1[e * S];
                    for (int k = 1; k < S; ++k) combine_best(m1, mj, m2, pb1[e * S + k], pj1[e * S + k], pb2[e * S + k]);
                    nn[slot] = (mj == INT_MAX) ? -1 : mj;
                    best[slot] = m1;
                    second[slot] = m2;
                }
                if (L == 0) grp_done[g] = 0;  // ready for a later scan on this workspace
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void mutual_flags(const SetPlan* __restrict__ plan, int n_sets,
                                                       const int32_t* __restrict__ nn, int64_t q_cap,
                                                       int32_t* __restrict__ flag, const DevStatus* st) {
    const int64_t total = st->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t slot = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; slot < q_cap; slot += gs) {
        int f = 0;
        if (slot < total) {
            const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
            if (!(c & 1) && c + 1 < n_sets) {
                const int j = nn[slot];
                f = (j >= 0 && nn[plan[c + 1].q_off + j] == slot - plan[c].q_off) ? 1 : 0;
            }
        }
        flag[slot] = f;
    }
}

__global__ __launch_bounds__(kBlock) void emit_pairs(const MatchSet* __restrict__ sets,
                                                     const SetPlan* __restrict__ plan, int n_sets,
                                                     const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                                     const int32_t* __restrict__ nn, const double* __restrict__ best,
                                                     const double* __restrict__ second,
                                                     const PairOutDev* __restrict__ outs, const DevStatus* st,
                                                     int64_t* counts, int stride, const CloudState* cs,
                                                     int64_t nnz_cap) {
    const int64_t total = st->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (2 * tid + 1 < n_sets) {
        // per pair: correspondences (the pair's mutual flags counted by pos) and exact re-scans
        const int i = static_cast<int>(tid);
        const int64_t a = plan[2 * i].q_off, b = plan[2 * i + 1].q_off;
        const int64_t pa = a < total ? pos[a] : st->pairs_total;
        const int64_t pb = b < total ? pos[b] : st->pairs_total;
        int64_t* o = counts + static_cast<int64_t>(i) * stride;
        o[0] = pb - pa;
        o[5] = plan[2 * i].n_fb + plan[2 * i + 1].n_fb;
        if (cs) {  // the batch form: sizes of the pair and its status
            o[1] = cs[2 * i].kept_cnt;
            o[2] = cs[2 * i + 1].kept_cnt;
            o[3] = cs[2 * i].j_cnt;
            o[4] = cs[2 * i + 1].j_cnt;
            o[7] = st->nnz;
            int64_t status = KMG_OK;
            if (st->err_sync) status = KMG_ERR_DEVICE;  // a bounded wait gave up (never expected)
            else if (st->err_range || (st->dense & 2)) status = KMG_ERR_RANGE;
            else if (st->err_capacity || st->nnz > nnz_cap) status = KMG_ERR_WORKSPACE;
            else if (o[0] > outs[i].cap) status = KMG_ERR_CAPACITY;
            o[6] = status;
        }
    }
    for (int64_t slot = tid; slot < total; slot += gs) {
        if (!flag[slot]) continue;
        const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const PairOutDev o = outs[c >> 1];
        const int64_t at = pos[slot] - pos[plan[c].q_off];
        if (at >= o.cap) continue;
        const int j = static_cast<int>(slot - plan[c].q_off);
        const int i = nn[slot];
        const MatchSet& a = sets[c];
        const MatchSet& b = sets[c + 1];
        o.pairs[2 * at] = (a.rows ? a.rows[j] : j) - a.row_base;
        o.pairs[2 * at + 1] = (b.rows ? b.rows[i] : i) - b.row_base;
        o.d1[at] = static_cast<float>(sqrt(best[slot]));
        o.d2[at] = static_cast<float>(sqrt(second[slot]));
    }
}

// ------------------------------------------------ reduced-precision tiles --
//
// FP16 / BF16 candidate generation.  Rows of each pair are centred on the
// pair's mean mu (FP64) and scaled by a power of two s (max |x - mu| s <= 2^14),
// and every centred, scaled value v is split into hi = T(v) and lo = T(v - hi).
// 16x16x32 MFMA steps form hi.hi of each K half (accumulators h0, h1) and
// hi.lo + lo.hi over both halves (accumulator c), FP32 accumulation; the
// product lo.lo is dropped.  With x' = x - mu, y' = y - mu, D = ||x' - y'||^2 = T + ||y'||^2 where
// T = ||x'||^2 - 2 x'.y', and the tile computes, in FP64,
//   L = a_x - 2 (h0 + h1 + c) / s^2 - k_y nx,
// with a_x = ||x'||^2 (1 - 2^-46) and nx = ||x'||: a lower bound of T when
// k_y = 2 e ||y'|| + 2^-22 sqrt(dim) / s bounds the dot-product error per unit
// of nx (e from the split and accumulation error analysis below).  Rows are
// ranked by L, so a non-candidate row has T >= L_4 and
// D >= L_4 + ||y'||^2 - 2^-22 sqrt(dim) ||y'|| / s (the per-query part of the
// split floor term); the exact second distance below that certifies the
// query, as in the FP64 form.
//
// Error per unit ||x'|| ||y'|| of the dot product (eps = 2^-11 for FP16 and
// 2^-8 for BF16, each widened by 2^-12 for the rounding through FP32 on the
// way): split 3 eps^2; h0, h1: at
// most 33 FP32 roundings each of sums bounded by S = sum |v_x v_y| <=
// ||v_x|| ||v_y||, counted twice for directed rounding; c: 129 roundings of a
// sum bounded by 2 eps S.  FP16 subnormals add 2^-24 per element, the 2^-22 sqrt(dim) / s
// terms above.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLpPieces = 2 * 2 * kWave;  // 16-byte pieces per chunk: K half x {hi, lo} x lane (4 KB)
constexpr int kLpSample = 1024;           // rows averaged for a pair's centre

template <class T>
struct Lp;
template <>
struct Lp<_Float16> {
    using vec = f16x8;
    static constexpr double kEps = 0x1p-11 * (1.0 + 0x1p-12);  // rounding through FP32 adds 2^-24 relative
    __device__ static f32x4 mfma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
    __device__ static _Float16 from(double v) { return static_cast<_Float16>(static_cast<float>(v)); }
};
template <>
struct Lp<__bf16> {
    using vec = bf16x8;
    static constexpr double kEps = 0x1p-8 * (1.0 + 0x1p-12);
    __device__ static f32x4 mfma(vec a, vec b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static __bf16 from(double v) { return static_cast<__bf16>(static_cast<float>(v)); }
};

template <class T>
__host__ __device__ constexpr double lp_dot_err() {
    return 3.0 * Lp<T>::kEps * Lp<T>::kEps + 2.0 * 33.0 * 0x1p-24 + 2.0 * 129.0 * 0x1p-24 * 2.0 * Lp<T>::kEps;
}

// One block per pair: mu = the mean (FP64, four fixed partial sums per
// dimension) of up to kLpSample rows taken at even strides over both sets.
// Any fixed mu is valid, since every bound is stated in ||x - mu||; a mean of
// the bulk keeps those norms, and the errors, small.
__global__ __launch_bounds__(kBlock) void lp_center(const MatchSet* __restrict__ sets, const SetPlan* __restrict__ plan,
                                                    int n_sets, int dim, PairLp* __restrict__ pp) {
    __shared__ double s_part[kBlock];
    const int pair = blockIdx.x;
    const int a = 2 * pair, b = 2 * pair + 1;
    const int na = plan[a].n, nb = b < n_sets ? plan[b].n : 0;
    const int64_t nt = static_cast<int64_t>(na) + nb;
    const int ns = static_cast<int>(nt < kLpSample ? nt : kLpSample);
    const int d = threadIdx.x % kLpMaxDim, g = threadIdx.x / kLpMaxDim;
    constexpr int kGroups = kBlock / kLpMaxDim;
    double sum = 0.0;
    if (d < dim) {
#pragma unroll 8
        for (int k = g; k < ns; k += kGroups) {
            const int r = static_cast<int>(static_cast<int64_t>(k) * nt / ns);
            const float* x = r < na ? set_row(sets[a], r, dim) : set_row(sets[b], r - na, dim);
            sum += static_cast<double>(x[d]);
        }
    }
    s_part[threadIdx.x] = sum;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < kGroups; ++q) t += s_part[q * kLpMaxDim + d];
        pp[pair].mu[d] = (d < dim && ns > 0) ? t / static_cast<double>(ns) : 0.0;
    }
    if (threadIdx.x == 0) pp[pair].maxabs_bits = 0ull;
}

// The scale of each pair from the largest |x - mu| (after lp_rows).
__global__ void lp_scale(PairLp* __restrict__ pp, int n_pairs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pairs) return;
    const double m = __longlong_as_double(static_cast<long long>(pp[i].maxabs_bits));
    int e = 0;
    if (m > 0.0) {
        frexp(m, &e);  // m < 2^e: scale 2^(14 - e) keeps every |v| below 2^14
        e = 14 - e;
    }
    e = e > 60 ? 60 : (e < -60 ? -60 : e);
    pp[i].scale = ldexp(1.0, e);
    pp[i].inv_s2 = ldexp(1.0, -2 * e);
}

// one atomic per wave for the common case of a wave within one pair
__device__ __forceinline__ void wave_max_abs(PairLp* pp, int pair, double v) {
    const uint64_t live = ballot(true);
    const int p0 = __shfl(pair, __ffsll(static_cast<unsigned long long>(live)) - 1, kWave);
    const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(v));
    if (ballot(pair == p0) == live) {
        unsigned long long mx = bits;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const unsigned long long o = __shfl_xor(mx, d, kWave);
            const bool o_live = (live >> (lane_id() ^ d)) & 1ull;
            if (o_live && o > mx) mx = o;
        }
        if (lane_id() == __ffsll(static_cast<unsigned long long>(live)) - 1) atomicMax(&pp[pair].maxabs_bits, mx);
    } else {
        atomicMax(&pp[pair].maxabs_bits, bits);
    }
}

// Per query slot: a = ||x'||^2 (1 - 2^-46) and nx = ||x'|| (FP64); the largest
// ||x'||^2 of each set goes to plan[c].max_norm_bits.
__global__ __launch_bounds__(kBlock) void lp_rows(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                  int dim, PairLp* __restrict__ pp, double* __restrict__ lp_a,
                                                  double* __restrict__ lp_nx, const DevStatus* st) {
#pragma clang fp contract(off)
    const int64_t total = st->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total; t += gs) {
        const int c = find_set(n_sets, t, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const float* x = set_row(sets[c], static_cast<int>(t - plan[c].q_off), dim);
        const double* mu = pp[c >> 1].mu;
        double acc = 0.0, mabs = 0.0;
        for (int k = 0; k < dim; ++k) {
            const double v = static_cast<double>(x[k]) - mu[k];
            acc = acc + v * v;
            mabs = fmax(mabs, fabs(v));
        }
        lp_a[t] = acc - acc * 0x1p-46;
        lp_nx[t] = sqrt(acc);
        wave_max_norm(plan, c, acc);
        wave_max_abs(pp, c >> 1, mabs);
    }
}

// Thread per 16-byte piece: chunk g, K half s, part p (hi / lo), lane l holds
// rows (or query columns) l % 16 of the chunk and k = 32 s + 8 (l / 16) + 0..7.
template <class T>
__global__ __launch_bounds__(kBlock) void lp_pack(const MatchSet* __restrict__ sets, const SetPlan* __restrict__ plan,
                                                  int n_sets, int dim, const PairLp* __restrict__ pp,
                                                  uint4* __restrict__ pk, const DevStatus* st) {
    const int64_t total = st->total_chunks * kLpPieces;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total; t += gs) {
        const int l = static_cast<int>(t % kWave);
        const int part = static_cast<int>((t / kWave) % 2);
        const int s = static_cast<int>((t / (2 * kWave)) % 2);
        const int64_t g = t / kLpPieces;
        const int c = find_set(n_sets, g, [&](int q) { return static_cast<int64_t>(plan[q].chunk_off); });
        const int i = static_cast<int>(g - plan[c].chunk_off) * kTileRows + l % kTileRows;
        const PairLp& P = pp[c >> 1];
        typename Lp<T>::vec out;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * s + 8 * (l / kTileRows) + e;
            double v = 0.0;
            if (i < plan[c].n && k < dim) v = (static_cast<double>(set_row(sets[c], i, dim)[k]) - P.mu[k]) * P.scale;
            const T hi = Lp<T>::from(v);
            out[e] = part == 0 ? hi : Lp<T>::from(v - static_cast<double>(hi));
        }
        pk[t] = __builtin_bit_cast(uint4, out);
    }
}

__device__ __forceinline__ void absorb4(double* top, double w0, double w1, double w2, double w3) {
    sort4(w0, w1, w2, w3);
    merge4(top, w0, w1, w2, w3);
}

// One block of four waves, as the FP64 tile: 64 query columns per wave
// against the partner's chunks [c_begin, c_end), chunks staged in LDS
// (4 KB of packed halves + the 16 rows' a and nx).
template <class T>
__device__ __forceinline__ void tile_block_lp(const uint4* __restrict__ pk, const double* __restrict__ lp_a,
                                              const double* __restrict__ lp_nx, int dim, const SetPlan& qc,
                                              const SetPlan& pc, const PairLp& P, int col0, int c_begin, int c_end,
                                              int seg, double* __restrict__ part, uint4* lds_pk, double* lds_rows) {
    using V = typename Lp<T>::vec;
    const int lane = lane_id();
    const int g = lane >> 4;
    const int l16 = lane & 15;
    V bh[kTilesPerWave][2], bl[kTilesPerWave][2];
    double ky[kTilesPerWave];
    const double kdot = 2.0 * lp_dot_err<T>() + 0x1p-48;
    const double kfloor = 0x1p-22 * sqrt(static_cast<double>(dim)) / P.scale;
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        const int chunk = min(col0 / kTileCols + t, qc.chunks - 1);
        const uint4* src = pk + static_cast<int64_t>(qc.chunk_off + chunk) * kLpPieces;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bh[t][s] = __builtin_bit_cast(V, src[(2 * s + 0) * kWave + lane]);
            bl[t][s] = __builtin_bit_cast(V, src[(2 * s + 1) * kWave + lane]);
        }
        const int col = min(col0 + kTileCols * t + l16, qc.n - 1);
        ky[t] = kdot * lp_nx[qc.q_off + col] + kfloor;
    }
    double top[kTilesPerWave][4];
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) top[t][0] = top[t][1] = top[t][2] = top[t][3] = INFINITY;
    const unsigned keep = keep_mask(row_bits(pc.chunks));
    const double m2is2 = -2.0 * P.inv_s2;
    if (c_begin < c_end) {  // uniform over the block
        const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint4*>(pk + static_cast<int64_t>(pc.chunk_off) * kLpPieces), 0,
            static_cast<int>(min(static_cast<int64_t>(pc.chunks) * kLpPieces * 16, static_cast<int64_t>(INT32_MAX))),
            static_cast<int>(kBufferWord3));
        // stage: piece threadIdx.x of the chunk, and row value min(threadIdx.x, 31): a (0..15), nx (16..31)
        const int rv = min(static_cast<int>(threadIdx.x), 31);
        auto load = [&](int c, uint4& piece, double& rowv) {
            piece = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rows, (c * kLpPieces + static_cast<int>(threadIdx.x)) * 16, 0, 0));
            const int i = c * kTileRows + (rv & 15);
            const int ic = min(i, pc.n - 1);
            const double* rsrc = rv < 16 ? lp_a : lp_nx;  // one unpredicated load
            const double v = rsrc[pc.q_off + ic];
            rowv = i < pc.n ? v : (rv < 16 ? kPadScore : 0.0);
        };
        uint4 piece;
        double rowv;
        load(c_begin, piece, rowv);
        lds_pk[threadIdx.x] = piece;
        lds_rows[rv] = rowv;
        __syncthreads();
        for (int c = c_begin; c < c_end; ++c) {
            const int buf = (c - c_begin) & 1;
            const uint4* sp = lds_pk + buf * kLpPieces;
            const double* sr = lds_rows + buf * 32;
            const V ah0 = __builtin_bit_cast(V, sp[0 * kWave + lane]), al0 = __builtin_bit_cast(V, sp[1 * kWave + lane]);
            const V ah1 = __builtin_bit_cast(V, sp[2 * kWave + lane]), al1 = __builtin_bit_cast(V, sp[3 * kWave + lane]);
            double ar[4], nr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ar[r] = sr[4 * g + r];
                nr[r] = sr[16 + 4 * g + r];
            }
            load(min(c + 1, c_end - 1), piece, rowv);
            __builtin_amdgcn_sched_barrier(0);
            // result register r of lane l holds tile row 4 (l / 16) + r, column l % 16
            const unsigned row0 = static_cast<unsigned>(c * kTileRows + 4 * g);
#pragma unroll
            for (int t = 0; t < kTilesPerWave; ++t) {
                const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                const f32x4 h0 = Lp<T>::mfma(ah0, bh[t][0], z);
                const f32x4 h1 = Lp<T>::mfma(ah1, bh[t][1], z);
                f32x4 x = Lp<T>::mfma(ah0, bl[t][0], z);
                x = Lp<T>::mfma(al0, bh[t][0], x);
                x = Lp<T>::mfma(ah1, bl[t][1], x);
                x = Lp<T>::mfma(al1, bh[t][1], x);
                double w[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double dot = (static_cast<double>(h0[r]) + static_cast<double>(h1[r])) + static_cast<double>(x[r]);
                    const double lb = fma(-ky[t], nr[r], fma(dot, m2is2, ar[r]));
                    w[r] = encode(lb, keep, row0 + r);
                }
                // the wave skips the merge when no lane's four bounds undercut its fourth best
                // (the scores are unique, so such a merge leaves top as it is)
                const double wmin = fmin(fmin(w[0], w[1]), fmin(w[2], w[3]));
                if (ballot(wmin < top[t][3])) absorb4(top[t], w[0], w[1], w[2], w[3]);
            }
            __builtin_amdgcn_sched_barrier(0);
            lds_pk[(buf ^ 1) * kLpPieces + threadIdx.x] = piece;
            lds_rows[(buf ^ 1) * 32 + rv] = rowv;
            __syncthreads();
        }
    }
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        merge_lane(top[t], 16);
        merge_lane(top[t], 32);
        const int col = col0 + kTileCols * t + l16;
        if (g == 0 && col < qc.n) {
            double* dst = part + qc.part_off + (static_cast<int64_t>(seg) * qc.n + col) * kTopK;
            dst[0] = top[t][0];
            dst[1] = top[t][1];
            dst[2] = top[t][2];
            dst[3] = top[t][3];
        }
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void topk_lp(
    const SetPlan* __restrict__ plan, int n_sets, const uint4* __restrict__ pk, const double* __restrict__ lp_a,
    const double* __restrict__ lp_nx, const PairLp* __restrict__ pp, int dim, double* __restrict__ part,
    DevStatus* st) {
    __shared__ uint4 lds_pk[2 * kLpPieces];
    __shared__ double lds_rows[2 * 32];
    __shared__ int s_tile;
    const int wv = threadIdx.x / kWave;
    const int total = st->err_capacity ? 0 : st->total_tiles;
    // the first tile of every block is fixed (XCD-aware order), the rest come from the queue
    // counted from kTopkBlocks: one round takes no atomic
    for (int tile = static_cast<int>(xcd_block_index()); tile < total;) {
        const int c = find_set(n_sets, tile, [&](int s) { return static_cast<int64_t>(plan[s].tile_off); });
        const SetPlan qc = plan[c];
        const SetPlan pc = plan[c ^ 1];
        const int local = tile - qc.tile_off;
        const int seg = local % qc.segs;
        const int cblk = local / qc.segs;
        const int cps = (pc.chunks + qc.segs - 1) / qc.segs;
        const int c_begin = seg * cps;
        const int c_end = min(c_begin + cps, pc.chunks);
        const int col0 = cblk * kColsPerBlock + wv * kColsPerWave;
        tile_block_lp<T>(pk, lp_a, lp_nx, dim, qc, pc, pp[c >> 1], col0, c_begin, c_end, seg, part, lds_pk,
                         lds_rows);
        if (total <= kTopkBlocks) break;  // uniform: every tile was a first tile
        __syncthreads();                  // every thread has read s_tile
        if (threadIdx.x == 0) s_tile = kTopkBlocks + static_cast<int>(atomicAdd(&st->tile_next, 1u));
        __syncthreads();
        tile = s_tile;
    }
}

// As rescore, with the lower-bound certificate of the reduced-precision tiles.
__global__ __launch_bounds__(kBlock) void rescore_lp(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                     int dim, const double* __restrict__ part,
                                                     const double* __restrict__ lp_nx,
                                                     const PairLp* __restrict__ pp, int32_t* __restrict__ nn,
                                                     double* __restrict__ best, double* __restrict__ second,
                                                     int32_t* __restrict__ failed, DevStatus* st) {
    const int64_t total = st->total_queries;
    const int q = lane_id() & (kQuad - 1);
    const int quad0 = lane_id() & ~(kQuad - 1);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * (kBlock / kQuad);
    for (int64_t slot = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kQuad; slot < total;
         slot += gs) {
        const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        if (sets[c].flags & kSetRowsOnly) {  // uniform over the quad: no queries
            if (q == 0) failed[slot] = 0;
            continue;
        }
        const int p = c ^ 1;
        const SetPlan qc = plan[c];
        const int j = static_cast<int>(slot - qc.q_off);
        const int np = p < n_sets ? plan[p].n : 0;
        if (np == 0) {
            if (q == 0) {
                nn[slot] = -1;
                best[slot] = INFINITY;
                second[slot] = INFINITY;
                failed[slot] = 0;
            }
            continue;
        }
        double top[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
        for (int sg = q; sg < qc.segs; sg += kQuad) {
            const double* src = part + qc.part_off + (static_cast<int64_t>(sg) * qc.n + j) * kTopK;
            merge4(top, src[0], src[1], src[2], src[3]);
        }
        merge_lane(top, 1);
        merge_lane(top, 2);
        const int bits = row_bits(plan[p].chunks);
        const double mine = q == 0 ? top[0] : (q == 1 ? top[1] : (q == 2 ? top[2] : top[3]));
        int row = -1;
        if (mine < kNoScore) {
            row = decode_row(mine, keep_mask(bits));
            if (row >= np) row = -1;
        }
        const double d = row >= 0 ? exact_d2(set_row(sets[p], row, dim), set_row(sets[c], j, dim), dim) : INFINITY;
        double dq[kQuad];
        int rq[kQuad];
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            dq[k] = __shfl(d, quad0 + k, kWave);
            rq[k] = __shfl(row, quad0 + k, kWave);
        }
        if (q != 0) continue;
        double b1 = INFINITY, b2 = INFINITY;
        int j1 = -1;
        int ncand = 0;
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            const int i = rq[k];
            if (i < 0) continue;
            ++ncand;
            const double dk = dq[k];
            if (dk < b1 || (dk == b1 && i < j1)) {
                b2 = b1;
                b1 = dk;
                j1 = i;
            } else if (dk < b2) {
                b2 = dk;
            }
        }
        bool ok;
        if (ncand >= np) {
            ok = true;
        } else {
            const double mx = __longlong_as_double(static_cast<long long>(plan[p].max_norm_bits));
            const double ny = lp_nx[slot];
            const double ny2 = ny * ny;
            const double cz = 0x1p-22 * sqrt(static_cast<double>(dim)) * ny / pp[c >> 1].scale;
            const double enc_err = ldexp(1.0, bits - 52) * (4.0 * mx + 4.0 * ny2 + 4.0);
            const double slack = 0x1p-44 * (fabs(top[3]) + ny2 + b2 + 4.0 * mx) + 1e-300;
            const double bound = top[3] + ny2 - cz - enc_err - slack;
            ok = ncand == 4 && b2 < bound;
        }
        if (ok) {
            nn[slot] = j1;
            best[slot] = b1;
            second[slot] = b2;
        } else {
            count_open(plan, c);
        }
        failed[slot] = ok ? 0 : 1;
    }
}

// ---------------------------------------------------- FP64 re-run lists --

// The lists of an FP64 re-run (the queries the reduced-precision
// certificate left open, or the image rows of the one-sided form), flagged in
// `failed` and counted by pos: f_slot[f] = main slot, f_row[f] = its row;
// set 2c of the re-run holds the listed queries of main set c, set 2c + 1 the
// full partner of c, rows only; the re-run's status is cleared.
__global__ __launch_bounds__(kBlock) void rerun_lists(const MatchSet* __restrict__ sets,
                                                      const SetPlan* __restrict__ plan, int n_sets,
                                                      const int32_t* __restrict__ failed,
                                                      const int32_t* __restrict__ pos,
                                                      const int64_t* __restrict__ f_total, int64_t q_cap,
                                                      int32_t* __restrict__ f_slot, int32_t* __restrict__ f_row,
                                                      int32_t* __restrict__ f_count, MatchSet* __restrict__ rr,
                                                      DevStatus* st2, const DevStatus* st) {
    const int64_t total = st->total_queries;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t slot = tid; slot < total; slot += gs) {
        if (!failed[slot]) continue;
        const int c = find_set(n_sets, slot, [&](int q) { return static_cast<int64_t>(plan[q].q_off); });
        const int j = static_cast<int>(slot - plan[c].q_off);
        const int f = pos[slot];
        f_slot[f] = static_cast<int32_t>(slot);
        f_row[f] = sets[c].rows ? sets[c].rows[j] : j;
    }
    if (tid < n_sets) {
        const int c = static_cast<int>(tid);
        auto start = [&](int k) -> int64_t {
            return (k < n_sets && plan[k].q_off < q_cap) ? pos[plan[k].q_off] : *f_total;
        };
        const int64_t b = start(c), e = start(c + 1);
        f_count[c] = static_cast<int32_t>(e - b);
        MatchSet q = sets[c];
        q.rows = f_row + b;
        q.n = f_count + c;
        q.flags = 0;
        MatchSet r = sets[c ^ 1];
        r.flags |= kSetRowsOnly;
        rr[2 * c] = q;
        rr[2 * c + 1] = r;
    }
    if (tid < static_cast<int64_t>(sizeof(DevStatus) / 4)) reinterpret_cast<uint32_t*>(st2)[tid] = 0u;
}

// Copies the re-run's answers to the main query slots (set c's list starts at
// pos[its first slot], or, without pos, at its first slot: the image lists).
// With flag (the matching back of the one-sided form): also the mutual flags.
// Image row j of set c whose nearest neighbour back is row i of the query set
// c ^ 1 forms a mutual pair iff the query's nearest neighbour is j; the flag
// sits on the slot of the pair's even set (the query slots come in cleared,
// the image rows' claims are overwritten).
__global__ __launch_bounds__(kBlock) void rerun_scatter(const SetPlan* __restrict__ plan2, int n_sets2,
                                                        const DevStatus* st2, const int32_t* __restrict__ nn2,
                                                        const double* __restrict__ best2,
                                                        const double* __restrict__ second2,
                                                        SetPlan* __restrict__ plan, const int32_t* __restrict__ pos,
                                                        const int32_t* __restrict__ f_slot, int32_t* __restrict__ nn,
                                                        double* __restrict__ best, double* __restrict__ second,
                                                        DevStatus* st, int add_rescans,
                                                        int32_t* __restrict__ flag) {
    const int64_t total = st2->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    // with add_rescans: the re-run's exact re-scans are counted with the queries they answer
    if (add_rescans && tid < n_sets2 / 2) plan[tid].n_fb += plan2[2 * tid].n_fb;
    for (int64_t t = tid; t < total; t += gs) {
        const int c2 = find_set(n_sets2, t, [&](int q) { return static_cast<int64_t>(plan2[q].q_off); });
        if (c2 & 1) continue;  // rows-only sets have no answers
        const int i = static_cast<int>(t - plan2[c2].q_off);
        const int c = c2 >> 1;
        const int64_t slot = f_slot[(pos ? pos[plan[c].q_off] : plan[c].q_off) + i];
        const int back = nn2[t];
        nn[slot] = back;
        best[slot] = best2[t];
        second[slot] = second2[t];
        if (flag) {
            const int qs = c ^ 1;  // the query set (the image rows are in set c)
            const int64_t qslot = back >= 0 ? plan[qs].q_off + back : -1;
            const bool mutual = back >= 0 && nn[qslot] == static_cast<int>(slot - plan[c].q_off);
            if (!(c & 1)) {
                flag[slot] = mutual ? 1 : 0;
            } else {
                flag[slot] = 0;
                if (mutual) flag[qslot] = 1;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && st2->err_capacity) st->err_capacity = 1;
}

// ------------------------------------------- both directions in full --
//
// Each pair as four sets, (set 2i as queries, set 2i+1 rows only) and (set
// 2i+1 as queries, set 2i rows only), matched in one band pass: no second pass
// over the image, at the price of matching every row of the larger set back.
// A pair (j, i) is mutual when j's nearest neighbour is i and i's is j.  The
// band planner writes the four sets (plan_band with `both`).

// The flags also come summed per scan tile (tile_sums, cleared by the planner):
// a wavefront's 64 slots lie in one tile, so one atomic per wavefront that
// found a pair.
static_assert(kScanTile % kWave == 0 && kBlock % kWave == 0, "a wavefront's slots lie in one scan tile");
__global__ __launch_bounds__(kBlock) void mutual_both(const SetPlan* __restrict__ plan, int n_sets2,
                                                      const int32_t* __restrict__ nn, int64_t q_cap,
                                                      int32_t* __restrict__ flag, int64_t* __restrict__ tile_sums,
                                                      const DevStatus* st2) {
    const int64_t total = st2->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t slot = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; slot < q_cap; slot += gs) {
        int f = 0;
        if (slot < total) {
            const int c = find_set(n_sets2, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
            if ((c & 3) == 0 && c + 2 < n_sets2) {  // the first set of a pair as queries
                const int j = nn[slot];
                f = (j >= 0 && nn[plan[c + 2].q_off + j] == slot - plan[c].q_off) ? 1 : 0;
            }
        }
        flag[slot] = f;
        const int cnt = __popcll(ballot(f != 0));
        if (lane_id() == 0 && cnt) atomicAdd(reinterpret_cast<unsigned long long*>(tile_sums + slot / kScanTile),
                                             static_cast<unsigned long long>(cnt));
    }
}

__global__ __launch_bounds__(kBlock) void emit_both(const MatchSet* __restrict__ sets,
                                                    const SetPlan* __restrict__ plan, int n_sets2,
                                                    const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                                    const int32_t* __restrict__ nn, const double* __restrict__ best,
                                                    const double* __restrict__ second,
                                                    const PairOutDev* __restrict__ outs, const DevStatus* st,
                                                    const DevStatus* st2, int64_t* counts, int stride,
                                                    const CloudState* cs, int64_t nnz_cap) {
    const int64_t total = st2->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (4 * tid + 3 < n_sets2) {
        const int i = static_cast<int>(tid);
        const int64_t a = plan[4 * i].q_off, b = plan[4 * i + 1].q_off;
        const int64_t pa = a < total ? pos[a] : st2->pairs_total;
        const int64_t pb = b < total ? pos[b] : st2->pairs_total;
        int64_t* o = counts + static_cast<int64_t>(i) * stride;
        o[0] = pb - pa;
        o[5] = plan[4 * i].n_fb + plan[4 * i + 2].n_fb;
        if (cs) {
            o[1] = cs[2 * i].kept_cnt;
            o[2] = cs[2 * i + 1].kept_cnt;
            o[3] = cs[2 * i].j_cnt;
            o[4] = cs[2 * i + 1].j_cnt;
            o[7] = st->nnz;
            int64_t status = KMG_OK;
            if (st->err_sync) status = KMG_ERR_DEVICE;  // a bounded wait gave up (never expected)
            else if (st->err_range || (st->dense & 2)) status = KMG_ERR_RANGE;
            else if (st->err_capacity || st2->err_capacity || st->nnz > nnz_cap) status = KMG_ERR_WORKSPACE;
            else if (o[0] > outs[i].cap) status = KMG_ERR_CAPACITY;
            o[6] = status;
        }
    }
    for (int64_t slot = tid; slot < total; slot += gs) {
        if (!flag[slot]) continue;
        const int c = find_set(n_sets2, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const int pr = c >> 2;
        const PairOutDev o = outs[pr];
        const int64_t at = pos[slot] - pos[plan[c].q_off];
        if (at >= o.cap) continue;
        const int j = static_cast<int>(slot - plan[c].q_off);
        const int i = nn[slot];
        const MatchSet& a = sets[2 * pr];
        const MatchSet& b = sets[2 * pr + 1];
        o.pairs[2 * at] = (a.rows ? a.rows[j] : j) - a.row_base;
        o.pairs[2 * at + 1] = (b.rows ? b.rows[i] : i) - b.row_base;
        o.d1[at] = static_cast<float>(sqrt(best[slot]));
        o.d2[at] = static_cast<float>(sqrt(second[slot]));
    }
}

// ------------------------------------------------------ one-sided form --
//
// A row can only be in a mutual pair if it is the nearest neighbour of some
// row of the other set.  So each pair is matched in one direction first, with
// the smaller set as queries (the other set rows only), and then only the
// image of that nearest-neighbour map is matched back.

// Copy of the sets with the larger set of each pair (the second on a tie)
// marked rows-only.
__global__ void one_sided_sets(const MatchSet* __restrict__ sets, int n_sets, MatchSet* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_sets) return;
    MatchSet m = sets[c];
    if ((c ^ 1) < n_sets) {
        const int mine = *m.n, other = *sets[c ^ 1].n;
        const bool rows_only = (c & 1) ? mine >= other : mine > other;
        if (rows_only) m.flags |= kSetRowsOnly;
    }
    out[c] = m;
}

// The image of the first direction, listed for the matching back in one pass:
// every rows-only row that some query has as its nearest neighbour is claimed
// once (its flag goes 0 -> 1; the re-score left the rows-only flags at 0) and
// appended, in no particular order, to its set's own range of the re-run lists
// (f_slot, f_row from the set's first slot on, counted in plan[c].n_img, which
// the planner zeroed).  nn of the rows-only slots <- -1 until the matching back
// fills the listed ones.  Also writes the re-run sets (set c's listed rows as
// queries against its partner's rows) and clears the re-run status.
__global__ __launch_bounds__(kBlock) void image_lists(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                      int32_t* __restrict__ nn, int32_t* __restrict__ flag,
                                                      int32_t* __restrict__ f_slot, int32_t* __restrict__ f_row,
                                                      MatchSet* __restrict__ rr, DevStatus* st2,
                                                      const DevStatus* st) {
    const int64_t total = st->total_queries;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    const int lane = lane_id();
    // wave-uniform trip count: the appends are counted once per wave and set
    for (int64_t w0 = tid - lane; w0 < total; w0 += gs) {
        const int64_t slot = w0 + lane;
        bool claim = false;
        int p = 0, j = 0;
        int32_t base = 0;
        if (slot < total) {
            const int c = find_set(n_sets, slot, [&](int q) { return static_cast<int64_t>(plan[q].q_off); });
            if (sets[c].flags & kSetRowsOnly) {
                nn[slot] = -1;
            } else {
                flag[slot] = 0;  // the mutual flags of the matching back start cleared
                j = nn[slot];
                p = c ^ 1;
                if (j >= 0 && p < n_sets) {
                    base = plan[p].q_off;
                    claim = atomicExch(&flag[base + j], 1) == 0;  // else another query has the row
                }
            }
        }
        uint64_t pending = ballot(claim);
        int k = 0;
        while (pending) {
            const int lead = __ffsll(static_cast<unsigned long long>(pending)) - 1;
            const int pl = __shfl(p, lead, kWave);
            const uint64_t same = ballot(claim && p == pl);
            int at = 0;
            if (lane == lead) at = atomicAdd(&plan[pl].n_img, __popcll(same));
            at = __shfl(at, lead, kWave);
            if (claim && p == pl) k = at + lanes_below(same);
            pending &= ~same;
        }
        if (claim) {
            f_slot[base + k] = base + j;
            f_row[base + k] = sets[p].rows ? sets[p].rows[j] : j;
        }
    }
    if (tid < n_sets) {
        const int c = static_cast<int>(tid);
        MatchSet q = sets[c];
        q.rows = f_row + plan[c].q_off;
        q.n = &plan[c].n_img;
        q.flags = 0;
        MatchSet r = sets[c ^ 1];
        r.flags |= kSetRowsOnly;
        rr[2 * c] = q;
        rr[2 * c + 1] = r;
    }
    if (tid < static_cast<int64_t>(sizeof(DevStatus) / 4)) reinterpret_cast<uint32_t*>(st2)[tid] = 0u;
}

// ------------------------------------------------------------ norm bands --
//
// Exact pruning of the FP64 form by the triangle inequality
// ||x - y|| >= | ||x|| - ||y|| |.  For every query the exact distances to the
// 64 partner rows nearest to it in norm give R^2 (the second smallest of
// them): the true second nearest neighbour is no farther, so a partner row
// whose norm differs from the query's by more than R (widened for rounding)
// can be neither of the two nearest, ties included.  Partner rows are packed
// in order of (squared norm, index), so the chunks' norm ranges ascend and a
// band of norms is a contiguous chunk range; queries are packed in order of
// (class of R, norm, index), so that the 64 queries of one wavefront need one
// narrow band.  Each wave's band is cut into tiles of at most T chunks; the
// tile lists are merged, re-scored and certified as in the full form (the rows
// outside the band are farther than R, and two rows inside are within it).

constexpr int kBandWave = kColsPerWave;  // queries per band wave (one wavefront)
constexpr int kSortTile = 1024;          // elements per LDS-sorted tile of the ordering
constexpr int kSortThreads = 256;
constexpr int kRankGroupDiv = 8;       // a set of m tiles ranks against max(1, m / 8) B tiles per item
constexpr int kBandTiles = 8192;         // band tiles the partial buffer holds beyond one per wave
constexpr int kSeedRows = kWave;         // partner rows around the query's norm for R
// Persistent grid of the band tile kernel: two blocks per CU, two waves per
// SIMD (measured: four waves per SIMD, with tiles of half the length, take
// twice as long).
constexpr int kBandBlocks = 512;
constexpr int kBandSlots = kBandBlocks * kWavesPerBlock;  // wavefronts of the band tile kernel

// Block-wide exclusive scan of K int32 values per thread in one pass (two
// barriers): v[k] <- the sum over lower threads, tot[k] <- the block total.
template <int K>
__device__ __forceinline__ void block_scan_k(int* v, int* tot, int* smem /* K x waves */) {
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    constexpr int kWaves = kPlanThreads / kWave;
    int incl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) incl[k] = wave_incl_scan(v[k]);
    if (lane == kWave - 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) smem[k * kWaves + wave] = incl[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int before = 0, total = 0;
        for (int w = 0; w < kWaves; ++w) {
            const int t = smem[k * kWaves + w];
            before += w < wave ? t : 0;
            total += t;
        }
        v[k] = before + incl[k] - v[k];
        tot[k] = total;
    }
    __syncthreads();
}

// The plan of one set per thread (thread c: set c, n rows, its partner n_other
// rows): slots, chunks, query waves, sort tiles and cross-rank items by block
// scans, and the status counts of the pass.
__device__ __forceinline__ void plan_sets_band(int c, bool live, bool paired, int n, int n_other, bool rows_only,
                                               bool other_rows, int kp, SetPlan* plan, DevStatus* st,
                                               int64_t* fb_total, int* s_scan) {
    // rows that no query is matched against need neither slots nor packing
    if (rows_only && (!paired || other_rows || n_other == 0)) n = 0;
    const int chunks = (n + kTileRows - 1) / kTileRows;
    const int waves = (live && !rows_only) ? (n + kBandWave - 1) / kBandWave : 0;
    const int sort_tiles = (n + kSortTile - 1) / kSortTile;
    // the counts of a plan stay below 2^31 (slots are int32)
    int v[5] = {n, chunks, waves, sort_tiles, sort_tiles * sort_tiles};
    int tot[5];
    block_scan_k<5>(v, tot, s_scan);
    const int q_off = v[0], c_off = v[1], w_off = v[2], s_off = v[3], i_off = v[4];
    const int tq = tot[0], tc = tot[1], tw = tot[2], ts = tot[3], ti = tot[4];
    // one buffer descriptor spans a set's packed rows: keep them below 2 GiB
    if (static_cast<int64_t>(chunks) * kp * kTileRows * 8 > INT32_MAX) st->err_capacity = 1;
    if (live) {
        SetPlan pl;
        pl.n = n;
        pl.q_off = static_cast<int32_t>(q_off);
        pl.chunk_off = static_cast<int32_t>(c_off);
        pl.chunks = chunks;
        pl.tile_off = static_cast<int32_t>(s_off);
        pl.cblocks = waves;
        pl.segs = 0;
        pl.n_fb = 0;
        pl.part_off = 0;
        pl.max_norm_bits = 0ull;
        pl.wave_off = static_cast<int32_t>(w_off);
        pl.rank_off = static_cast<int32_t>(i_off);
        pl.n_img = 0;
        plan[c] = pl;
    }
    if (c == 0) {
        st->total_queries = static_cast<int32_t>(tq);
        st->total_chunks = tc;
        st->total_waves = static_cast<int32_t>(tw);
        st->rank_items = static_cast<int32_t>(ti);
        st->sort_items = static_cast<int32_t>(ts);
        st->total_tiles = 0;
        st->tile_next = 0;
        st->n_fallback = 0;
        st->band_step = 0;
        *fb_total = 0;  // the re-score counts the uncertified queries from zero
    }
}

// With `oside`, the sets are first made one-sided (the larger set of each
// pair, the second on a tie, becomes rows-only) and written there; the
// kernels after the planner then read oside.  With `both` as well, the
// n_sets / 2 input sets are expanded there into the sets of both directions
// in full, and the status block of that pass is cleared first.
__global__ __launch_bounds__(kPlanThreads) void plan_band(const MatchSet* __restrict__ sets, int n_sets, int kp,
                                                         SetPlan* plan, DevStatus* st, MatchSet* __restrict__ oside,
                                                         int both, int64_t* __restrict__ fb_total,
                                                         int32_t* __restrict__ grp_done, int64_t n_grp,
                                                         int64_t* __restrict__ scan_tmp, int64_t n_tmp) {
    __shared__ int s_scan[5 * (kPlanThreads / kWave)];
    for (int64_t g = threadIdx.x; g < n_grp; g += kPlanThreads) grp_done[g] = 0;  // for the exact scans
    if (both)  // the tile sums of the mutual flags, accumulated by mutual_both
        for (int64_t g = threadIdx.x; g < n_tmp; g += kPlanThreads) scan_tmp[g] = 0;
    const int c = threadIdx.x;
    const bool live = c < n_sets;
    const bool paired = live && (c ^ 1) < n_sets;
    if (both) {
        // both directions in full: the n_sets / 2 input sets become set 2t (t as queries) and
        // set 2t + 1 (t's partner as rows only), planned on a status block of their own
        for (int k = c; k < static_cast<int>(sizeof(DevStatus) / 4); k += kPlanThreads)
            reinterpret_cast<uint32_t*>(st)[k] = 0u;
        __syncthreads();
        const int t = c >> 1;
        MatchSet m;
        int n = 0, n_other = 0;
        if (live) {
            m = sets[(c & 1) ? (t ^ 1) : t];
            m.flags = (c & 1) ? (m.flags | kSetRowsOnly) : (m.flags & ~kSetRowsOnly);
            oside[c] = m;
            n = *m.n;
            n_other = *sets[(c & 1) ? t : (t ^ 1)].n;
        }
        plan_sets_band(c, live, live, n, n_other, live && (c & 1), live && !(c & 1), kp, plan, st, fb_total, s_scan);
        return;
    }
    int n = live ? *sets[c].n : 0;
    const int n_other = paired ? *sets[c ^ 1].n : 0;
    bool rows_only = live && (sets[c].flags & kSetRowsOnly);
    bool other_rows = paired && (sets[c ^ 1].flags & kSetRowsOnly);
    if (oside) {
        if (paired) {
            rows_only = (c & 1) ? n >= n_other : n > n_other;
            other_rows = !rows_only;
        }
        if (live) {
            MatchSet m = sets[c];
            m.flags = rows_only ? (m.flags | kSetRowsOnly) : (m.flags & ~kSetRowsOnly);
            oside[c] = m;
        }
    }
    plan_sets_band(c, live, paired, n, n_other, rows_only, other_rows, kp, plan, st, fb_total, s_scan);
}

// 32-bit sort key of a slot.  Partners: the top 32 bits of the squared norm's
// FP64 pattern (an order-preserving truncation: a key k stands for squared
// norms in [dec(k), dec(k + 1)), dec(k) = the double with bits k << 32).
// Queries: (class of R^2, top 23 bits of the squared norm), the class being
// the binary exponent of R^2 halved (R in octaves).
__device__ __forceinline__ uint32_t norm_key(double n2) {
    return static_cast<uint32_t>(static_cast<unsigned long long>(__double_as_longlong(n2)) >> 32);
}

__device__ __forceinline__ uint32_t band_key(bool partner, double n2, double r2) {
    const unsigned long long nb = static_cast<unsigned long long>(__double_as_longlong(n2));
    if (partner) return static_cast<uint32_t>(nb >> 32);
    const int e = static_cast<int>((static_cast<unsigned long long>(__double_as_longlong(r2)) >> 52) & 0x7ffull);
    const int cls = min(max(e - 1023 + 256, 0), 511) >> 1;
    return (static_cast<uint32_t>(cls) << 24) | static_cast<uint32_t>(nb >> 40);
}

// Ordering of the sets of one role (rows-only partners, or query sets) by
// (key, local index), a unique 64-bit value: rank[slot] = the element's packed
// position.  tile_sort sorts every tile of kSortTile consecutive elements of a
// set (bitonic, one element per thread) and stores the tile's sorted values and each element's
// place in its tile as its first rank term; cross_rank takes a tile A of one
// set and a group of its other tiles B and adds to every element of A the
// count of B's values below its own (binary searches in each B's sorted
// values, staged in LDS).

__device__ __forceinline__ unsigned long long rank_value(bool partner, double n2, double r2, int idx) {
    return (static_cast<unsigned long long>(band_key(partner, n2, r2)) << 32) | static_cast<uint32_t>(idx);
}

// One element per thread: compare-exchange partners closer than a wavefront
// trade through shuffles, farther ones through LDS (ten of the 55 stages).
__global__ __launch_bounds__(kSortTile) void tile_sort(const MatchSet* __restrict__ sets,
                                                       const SetPlan* __restrict__ plan, int n_sets, int partner,
                                                       const double* __restrict__ n2, const double* __restrict__ r2,
                                                       unsigned long long* __restrict__ sorted,
                                                       int32_t* __restrict__ rank, const DevStatus* st) {
    __shared__ unsigned long long s_v[kSortTile];
    const bool pr = partner != 0;
    const int r = threadIdx.x;
    const int64_t total = st->sort_items;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_set(n_sets, item, [&](int s) { return static_cast<int64_t>(plan[s].tile_off); });
        if (((sets[c].flags & kSetRowsOnly) != 0) != pr) continue;  // uniform over the block
        const SetPlan pc = plan[c];
        const int e0 = static_cast<int>(item - pc.tile_off) * kSortTile;
        const int cnt = min(kSortTile, pc.n - e0);
        const int64_t sl = pc.q_off + e0 + r;
        unsigned long long v = r < cnt ? rank_value(pr, n2[sl], pr ? 0.0 : r2[sl], e0 + r) : ~0ull;  // ~0 sorts last
        for (int k = 2; k <= kSortTile; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                unsigned long long o;
                if (j >= kWave) {  // uniform over the block
                    __syncthreads();  // the last exchange's values are read
                    s_v[r] = v;
                    __syncthreads();
                    o = s_v[r ^ j];
                } else {
                    o = __shfl_xor(v, j, kWave);
                }
                const bool keep_min = ((r & j) == 0) == ((r & k) == 0);
                v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
            }
        }
        if (r < cnt) {
            sorted[pc.q_off + e0 + r] = v;
            rank[pc.q_off + static_cast<int>(v & 0xffffffffull)] = r;
        }
        __syncthreads();  // s_v is free for the next item
    }
}

__global__ __launch_bounds__(kSortThreads) void cross_rank(const MatchSet* __restrict__ sets,
                                                           const SetPlan* __restrict__ plan, int n_sets, int partner,
                                                           const unsigned long long* __restrict__ sorted,
                                                           int32_t* __restrict__ rank, const DevStatus* st) {
    __shared__ unsigned long long s_b[kSortTile];
    const bool pr = partner != 0;
    const int64_t total = st->rank_items;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_set(n_sets, item, [&](int s) { return static_cast<int64_t>(plan[s].rank_off); });
        if (((sets[c].flags & kSetRowsOnly) != 0) != pr) continue;  // uniform over the block
        const SetPlan pc = plan[c];
        const int m = (pc.n + kSortTile - 1) / kSortTile;
        const int local = static_cast<int>(item - pc.rank_off);
        const int ta = local / m, tb = local % m;
        // a set of many tiles takes G of them as B per item, one atomic per element and item
        // (the items of the other B tiles of the group return at once)
        const int G = max(1, m / kRankGroupDiv);
        if (tb % G != 0) continue;  // uniform over the block
        const int a0 = ta * kSortTile, na = min(kSortTile, pc.n - a0);
        constexpr int kPer = kSortTile / kSortThreads;
        unsigned long long v[kPer];
        int cnt[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int r = static_cast<int>(threadIdx.x) + kSortThreads * i;
            v[i] = r < na ? sorted[pc.q_off + a0 + r] : 0ull;
            cnt[i] = 0;
        }
        for (int b = tb; b < min(tb + G, m); ++b) {
            if (b == ta) continue;  // the tile's own order is the first rank term
            const int b0 = b * kSortTile, nb = min(kSortTile, pc.n - b0);
            __syncthreads();
            for (int r = threadIdx.x; r < nb; r += kSortThreads) s_b[r] = sorted[pc.q_off + b0 + r];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                int lo = 0, hi = nb;  // first of B's values not below v
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_b[mid] < v[i]) lo = mid + 1;
                    else hi = mid;
                }
                cnt[i] += lo;
            }
        }
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int r = static_cast<int>(threadIdx.x) + kSortThreads * i;
            if (r < na && cnt[i]) atomicAdd(&rank[pc.q_off + static_cast<int>(v[i] & 0xffffffffull)], cnt[i]);
        }
    }
}

// Both directions in full: the query set of a cloud is ordered by (class of R,
// norm) as a stable partition by class of the norm order that the rows-only
// set of the same cloud already has (the partners' ordering), in place of
// tile_sort and cross_rank.  Any order of the queries gives the same results;
// this one keeps each class in norm order.  A query set whose cloud has no
// ordered rows set (its partner cloud has no queries) keeps the slot order.
__device__ __forceinline__ int band_class(double r2) {
    const int e = static_cast<int>((static_cast<unsigned long long>(__double_as_longlong(r2)) >> 52) & 0x7ffull);
    return min(max(e - 1023 + 256, 0), 511) >> 1;
}
constexpr int kClasses = 256;

// The rows-only set of query set c's own cloud (sets 2t: cloud t as queries,
// 2t + 1: cloud t^1 as rows), or -1 when it holds no ordered copy.
__device__ __forceinline__ int same_cloud_rows(const SetPlan* plan, int n_sets, int c) {
    const int cr = 2 * ((c >> 1) ^ 1) + 1;
    return (cr < n_sets && plan[cr].n == plan[c].n) ? cr : -1;
}

// Class histogram of every sort tile of the query sets, in the norm order.
__global__ __launch_bounds__(kSortTile) void class_hist(const MatchSet* __restrict__ sets,
                                                        const SetPlan* __restrict__ plan, int n_sets,
                                                        const double* __restrict__ r2,
                                                        const int32_t* __restrict__ perm, int32_t* __restrict__ hist,
                                                        const DevStatus* st) {
    __shared__ int s_h[kClasses];
    const int r = threadIdx.x;
    const int64_t total = st->sort_items;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_set(n_sets, item, [&](int s) { return static_cast<int64_t>(plan[s].tile_off); });
        if (sets[c].flags & kSetRowsOnly) continue;  // uniform over the block
        const int cr = same_cloud_rows(plan, n_sets, c);
        if (cr < 0) continue;
        const SetPlan pc = plan[c];
        const int e0 = static_cast<int>(item - pc.tile_off) * kSortTile;
        const int cnt = min(kSortTile, pc.n - e0);
        if (r < kClasses) s_h[r] = 0;
        __syncthreads();
        if (r < cnt) {
            const int j = perm[plan[cr].q_off + e0 + r];
            if (j >= 0 && j < pc.n) atomicAdd(&s_h[band_class(r2[pc.q_off + j])], 1);  // (a valid order: always)
        }
        __syncthreads();
        if (r < kClasses) hist[item * kClasses + r] = s_h[r];
        __syncthreads();  // s_h is free for the next item
    }
}

// perm[position] = the query's slot, with position = class offset + the
// class's count in earlier tiles + its count earlier in this tile (waves in
// order, lanes in order within a wave).  The reads of the rows set's part of
// perm and the writes of the query set's part never overlap; gather_pack then
// packs the queries in that order.
__global__ __launch_bounds__(kSortTile) void class_rank(const MatchSet* __restrict__ sets,
                                                        const SetPlan* __restrict__ plan, int n_sets,
                                                        const double* __restrict__ r2, int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ hist, const DevStatus* st) {
    constexpr int kWaves = kSortTile / kWave;
    __shared__ int s_tot[kClasses], s_off[kClasses];
    __shared__ int s_wcnt[kWaves][kClasses];
    const int r = threadIdx.x;
    const int lane = lane_id();
    const int wv = r / kWave;
    const int64_t total = st->sort_items;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_set(n_sets, item, [&](int s) { return static_cast<int64_t>(plan[s].tile_off); });
        if (sets[c].flags & kSetRowsOnly) continue;  // uniform over the block
        const int cr = same_cloud_rows(plan, n_sets, c);
        const SetPlan pc = plan[c];
        const int e0 = static_cast<int>(item - pc.tile_off) * kSortTile;
        const int cnt = min(kSortTile, pc.n - e0);
        if (cr < 0) {
            if (r < cnt) perm[pc.q_off + e0 + r] = e0 + r;
            continue;
        }
        const int jp = r < cnt ? perm[plan[cr].q_off + e0 + r] : -1;
        const bool ok = jp >= 0 && jp < pc.n;  // (a valid order: always)
        const int j = ok ? jp : 0;
        const int cls = ok ? band_class(r2[pc.q_off + j]) : -1;
        // the set's class totals and the counts of its tiles before this one
        const int nt = (pc.n + kSortTile - 1) / kSortTile;
        const int me = static_cast<int>(item - pc.tile_off);
        if (r < kClasses) {
            int tot = 0, pre = 0;
            for (int t = 0; t < nt; ++t) {
                const int h = hist[(static_cast<int64_t>(pc.tile_off) + t) * kClasses + r];
                tot += h;
                pre += t < me ? h : 0;
            }
            s_tot[r] = tot;
            s_off[r] = pre;
        }
        for (int k = r; k < kWaves * kClasses; k += kSortTile) (&s_wcnt[0][0])[k] = 0;
        __syncthreads();
        if (r < kWave) {  // wave 0: exclusive scan of the class totals, four classes per lane
            int v[kClasses / kWave], sum = 0;
#pragma unroll
            for (int u = 0; u < kClasses / kWave; ++u) {
                v[u] = s_tot[r * (kClasses / kWave) + u];
                sum += v[u];
            }
            int run = wave_incl_scan(sum) - sum;
#pragma unroll
            for (int u = 0; u < kClasses / kWave; ++u) {
                s_off[r * (kClasses / kWave) + u] += run;
                run += v[u];
            }
        }
        // the element's place among the earlier elements of its class in its wave
        int in_wave = 0;
        unsigned long long pending = ballot(cls >= 0);
        while (pending) {  // uniform over the wave: one round per class present
            const int lead = __ffsll(static_cast<long long>(pending)) - 1;
            const int lc = __shfl(cls, lead, kWave);
            const unsigned long long m = ballot(cls == lc);
            if (cls == lc) in_wave = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == lead) s_wcnt[wv][lc] = __popcll(m);
            pending &= ~m;
        }
        __syncthreads();
        if (cls >= 0) {
            int before = 0;
            for (int w = 0; w < wv; ++w) before += s_wcnt[w][cls];
            perm[pc.q_off + s_off[cls] + before + in_wave] = j;
        }
        __syncthreads();  // the LDS tables are free for the next item
    }
}

// The query sets' packed chunks once perm holds their order (both directions
// in full), so that the 16 lanes of a quarter write whole 128-byte lines
// (scatter_pack writes each slot's values where its rank puts them, one value
// per line); padding rows as scatter_pack writes them.  pack_band_waves runs
// it for the chunks of each query wave before the wave's bands.
// One query chunk g (global chunk index, of query set c) packed by one
// wavefront: lane 4 r + q writes quarter q of the kp values of row r.
__device__ __forceinline__ void pack_chunk(const MatchSet* __restrict__ sets, const SetPlan& pc, int c, int dim,
                                           int kp, const double* __restrict__ n2, const int32_t* __restrict__ perm,
                                           double* __restrict__ pk, DevStatus* st, int64_t g) {
    const int ks = kp / 4;
    const int lane = lane_id();
    const int r = lane >> 2, q = lane & 3;
    const int pos = static_cast<int>(g - pc.chunk_off) * kTileRows + r;
    double* dst = pk + g * kp * kTileRows + r;
    const int k0 = q * ks;
    if (pos < pc.n) {
        const int j = perm[pc.q_off + pos];
        if (j < 0 || j >= pc.n) {  // never: the order is a permutation
            st->err_capacity = 1;
            return;
        }
        const float* x = set_row(sets[c], j, dim);
        double v[17];
#pragma unroll
        for (int u = 0; u < 17; ++u) {
            const int k = k0 + u;
            v[u] = (u < ks && k < dim) ? static_cast<double>(x[k]) : 0.0;
        }
        const double nn = n2[pc.q_off + j];
#pragma unroll
        for (int u = 0; u < 17; ++u) {
            const int k = k0 + u;
            if (u < ks) dst[k * kTileRows] = k == dim ? nn : v[u];
        }
    } else {
#pragma unroll
        for (int u = 0; u < 17; ++u) {
            const int k = k0 + u;
            if (u < ks) dst[k * kTileRows] = k == dim ? kPadScore : 0.0;
        }
    }
}

// Packs the rows of the sets of one role at their ranks (layout of pack_rows:
// k-major chunks of 16 rows, the squared norm at k = dim, padding rows scored
// kPadScore) and records perm[q_off + position] = local row (and, for
// partners, the sort key of the position).
__global__ __launch_bounds__(kBlock) void scatter_pack(const MatchSet* __restrict__ sets,
                                                       const SetPlan* __restrict__ plan, int n_sets, int dim, int kp,
                                                       int partner, const double* __restrict__ n2,
                                                       const int32_t* __restrict__ rank, double* __restrict__ pk,
                                                       int32_t* __restrict__ perm, uint32_t* __restrict__ skey,
                                                       int32_t* __restrict__ flag, DevStatus* st) {
    const bool pr = partner != 0;
    // four threads per slot (each finds the slot's set, row and position, then
    // writes a quarter of its kp = 4 KS values with all of their loads in flight);
    // padding rows after them, one thread per (set, padding row)
    const int ks = kp / 4;
    const int64_t total = static_cast<int64_t>(st->total_queries) * 4;
    const int64_t pads = static_cast<int64_t>(n_sets) * kTileRows;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total + pads; t += gs) {
        if (t < total) {
            const int64_t slot = t / 4;
            const int k0 = static_cast<int>(t % 4) * ks;
            const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
            if (((sets[c].flags & kSetRowsOnly) != 0) != pr) continue;
            const SetPlan pc = plan[c];
            const int j = static_cast<int>(slot - pc.q_off);
            const int pos = rank[slot];
            if (pos < 0 || pos >= pc.n) {  // ranks are a permutation of 0 .. n - 1
                st->err_capacity = 1;
                continue;
            }
            const float* x = set_row(sets[c], j, dim);
            double* dst = pk + static_cast<int64_t>(pc.chunk_off + pos / kTileRows) * kp * kTileRows + pos % kTileRows;
            double v[17];
#pragma unroll
            for (int u = 0; u < 17; ++u) {
                const int k = k0 + u;
                v[u] = (u < ks && k < dim) ? static_cast<double>(x[k]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 17; ++u) {
                const int k = k0 + u;
                if (u < ks) dst[k * kTileRows] = k == dim ? n2[slot] : v[u];
            }
            if (k0 == 0) {
                perm[pc.q_off + pos] = j;
                if (pr) {
                    skey[pc.q_off + pos] = norm_key(n2[slot]);
                    flag[slot] = 0;  // rows-only slots: never uncertified (the matching back claims them)
                }
            }
        } else {
            const int64_t u = t - total;
            const int c = static_cast<int>(u / kTileRows);
            const int i = static_cast<int>(u % kTileRows);
            if (((sets[c].flags & kSetRowsOnly) != 0) != pr) continue;
            const SetPlan pc = plan[c];
            const int pos = pc.n + i;
            if (pos >= pc.chunks * kTileRows) continue;
            double* dst = pk + static_cast<int64_t>(pc.chunk_off + pos / kTileRows) * kp * kTileRows + pos % kTileRows;
            for (int k = 0; k < kp; ++k) dst[k * kTileRows] = k == dim ? kPadScore : 0.0;
        }
    }
}

// First position in [0, n) at which below(position) is false, where below
// holds on a prefix: a 64-way search by one wavefront (three rounds for 2^18).
template <class F>
__device__ __forceinline__ int wave_search(int n, F below) {
    int lo = 0, hi = n;
    while (lo < hi) {  // uniform over the wave
        const int stride = (hi - lo + kWave - 1) / kWave;
        const int probe = lo + (lane_id() + 1) * stride - 1;
        const bool b = probe < hi && below(probe);
        const int cnt = __popcll(ballot(b));
        const int nlo = lo + cnt * stride;
        hi = min(hi, lo + (cnt + 1) * stride - 1);
        lo = nlo;
    }
    return lo;
}

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v = fmin(v, __shfl_xor(v, d, kWave));
    return v;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
    return v;
}

// As wave_search, by each group of 16 lanes for its own prefix predicate (the
// four groups of a wavefront search at once; a group with n = 0 idles).
template <class F>
__device__ __forceinline__ int group_search16(int n, F below) {
    const int gl = lane_id() & 15;
    const int sh = lane_id() & ~15;
    int lo = 0, hi = n;
    while (ballot(lo < hi)) {  // uniform over the wave
        const bool open = lo < hi;
        const int stride = open ? (hi - lo + 15) / 16 : 1;
        const int probe = lo + (gl + 1) * stride - 1;
        const bool b = open && probe < hi && below(probe);
        const int cnt = __popcll((ballot(b) >> sh) & 0xffffull);
        if (open) {
            const int nlo = lo + cnt * stride;
            hi = min(hi, lo + (cnt + 1) * stride - 1);
            lo = nlo;
        }
    }
    return lo;
}

// R^2 of each query slot = the second smallest exact distance (the plain FP64
// sum in dimension order, as exact_d2) to the kSeedRows partner rows around
// the query's norm key in the partner's packed order; infinite when the
// partner has fewer than two rows.  A group of 16 lanes takes one query (four
// per wavefront, whose chains of dependent loads overlap), each lane four rows
// of the window.  The query's own values are loaded before the search, which
// they do not depend on.
template <int KS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void band_seeds(
    const MatchSet* __restrict__ sets, const SetPlan* __restrict__ plan, int n_sets, int dim,
    const double* __restrict__ pk, const double* __restrict__ n2, const uint32_t* __restrict__ skey,
    double* __restrict__ r2, const DevStatus* st) {
#pragma clang fp contract(off)
    constexpr int kp = 4 * KS;
    constexpr int kG = 16;                   // lanes per query
    constexpr int kRows = kSeedRows / kG;    // rows per lane
    constexpr int kYv = (kp + kG - 1) / kG;  // query values per lane
    const int lane = lane_id();
    const int gl = lane & (kG - 1);
    // the queries only: index g = 64 (query wave) + position, rows-only sets have no waves
    const int64_t total = static_cast<int64_t>(st->total_waves) * kBandWave;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (kBlock / kG);
    for (int64_t base = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave * (kWave / kG);
         base < total; base += stride) {  // uniform over the wave
        const int64_t g = base + lane / kG;
        bool live = g < total;
        int c = 0, jq = 0, np = 0;
        int64_t slot = 0;
        if (live) {
            const int64_t wq = g / kBandWave;
            c = find_set(n_sets, wq, [&](int s) { return static_cast<int64_t>(plan[s].wave_off); });
            jq = static_cast<int>(wq - plan[c].wave_off) * kBandWave + static_cast<int>(g % kBandWave);
            live = jq < plan[c].n;  // the last wave's padding
        }
        if (live) {
            slot = plan[c].q_off + jq;
            np = (c ^ 1) < n_sets ? plan[c ^ 1].n : 0;
            if (np < 2) {
                if (gl == 0) r2[slot] = INFINITY;
                live = false;
            }
        }
        float yv[kYv];  // lane gl holds the query's values gl, gl + 16, ...
        {
            const float* y = live ? set_row(sets[c], jq, dim) : nullptr;
#pragma unroll
            for (int j = 0; j < kYv; ++j) yv[j] = (live && j * kG + gl < dim) ? y[j * kG + gl] : 0.0f;
        }
        int64_t chunk_off = 0;
        uint32_t kq = 0;
        const uint32_t* pkey = skey;
        if (live) {
            const SetPlan pc = plan[c ^ 1];
            chunk_off = pc.chunk_off;
            kq = norm_key(n2[slot]);
            pkey = skey + pc.q_off;
        }
        const int at = group_search16(live ? np : 0, [&](int pos) { return pkey[pos] < kq; });
        const int nw = min(np, kSeedRows);
        const int w0 = min(max(at - nw / 2, 0), np - nw);
        const double* xr[kRows];
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            const int pos = live ? w0 + min(j * kG + gl, nw - 1) : 0;
            xr[j] = pk + (chunk_off + pos / kTileRows) * kp * kTileRows + pos % kTileRows;
        }
        double acc[kRows];
#pragma unroll
        for (int j = 0; j < kRows; ++j) acc[j] = 0.0;
#pragma unroll
        for (int kb = 0; kb < kp; kb += 2) {
            if (kb < dim) {  // uniform; the row holds kp values, those past dim are loaded, not used
                double xs[kRows][2];
#pragma unroll
                for (int j = 0; j < kRows; ++j)
#pragma unroll
                    for (int u = 0; u < 2; ++u) xs[j][u] = xr[j][(kb + u) * kTileRows];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int k = kb + u;
                    if (k < dim) {
                        const double yk = static_cast<double>(__shfl(yv[k / kG], k % kG, kG));
#pragma unroll
                        for (int j = 0; j < kRows; ++j) {
                            const double df = xs[j][u] - yk;
                            acc[j] = acc[j] + df * df;
                        }
                    }
                }
            }
        }
        double d[kRows];
        double m1 = INFINITY;
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            d[j] = (live && j * kG + gl < nw) ? acc[j] : INFINITY;
            m1 = fmin(m1, d[j]);
        }
#pragma unroll
        for (int o = 1; o < kG; o <<= 1) m1 = fmin(m1, __shfl_xor(m1, o, kG));
        int n_eq = 0;
        double m2 = INFINITY;
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            n_eq += d[j] == m1 ? 1 : 0;
            m2 = d[j] == m1 ? m2 : fmin(m2, d[j]);
        }
#pragma unroll
        for (int o = 1; o < kG; o <<= 1) {
            n_eq += __shfl_xor(n_eq, o, kG);
            m2 = fmin(m2, __shfl_xor(m2, o, kG));
        }
        if (live && gl == 0) r2[slot] = n_eq >= 2 ? m1 : m2;
    }
}

// One wavefront per query wave: the band of norms each 16-query tile of the
// wave needs, [nu - R - m, nu + R + m] over the tile's queries with
// m = 2^-38 (nu + R) for the rounding of the norms and distances, and the
// partner chunks that can hold a squared norm in [lo^2 (1 - 2^-50),
// hi^2 (1 + 2^-50)], found on the chunks' first and last sort keys (a key k
// holds squared norms in [dec(k), dec(k + 1))); the wave's range is the union
// of its tiles' ranges.
__device__ __forceinline__ void wave_band(const SetPlan* __restrict__ plan, int n_sets,
                                          const double* __restrict__ n2, const double* __restrict__ r2,
                                          const int32_t* __restrict__ perm, const uint32_t* __restrict__ skey,
                                          int32_t* __restrict__ wave_c0, int32_t* __restrict__ wave_len,
                                          int2* __restrict__ wave_sub, int64_t w) {
    const int lane = lane_id();
    const int c = find_set(n_sets, w, [&](int s) { return static_cast<int64_t>(plan[s].wave_off); });
    const SetPlan qc = plan[c];
    const int p = c ^ 1;
    const int np = p < n_sets ? plan[p].n : 0;
    const int pos = static_cast<int>(w - qc.wave_off) * kBandWave + lane;
    double lo = INFINITY, hi = -INFINITY;
    const int jq = pos < qc.n ? perm[qc.q_off + pos] : -1;
    if (jq >= 0 && jq < qc.n) {
        const int64_t sl = qc.q_off + jq;
        const double nu = sqrt(n2[sl]);
        const double R = sqrt(r2[sl]);
        const double m = 0x1p-38 * (nu + R);
        lo = nu - R - m;
        hi = nu + R + m;
    }
    // the band of each 16-query tile of the wave (lanes 16 t .. 16 t + 15); the wave's
    // band is their union
#pragma unroll
    for (int d = 1; d < kTileCols; d <<= 1) {
        lo = fmin(lo, __shfl_xor(lo, d, kWave));
        hi = fmax(hi, __shfl_xor(hi, d, kWave));
    }
    const bool live = np > 0 && lo <= hi;
    int k0 = 0, k1 = 0;
    if (ballot(live)) {  // uniform over the wave
        const SetPlan pc = plan[p];
        const uint32_t* pkey = skey + pc.q_off;
        const int pch = pc.chunks;
        // chunks whose last key is below that of lo^2 hold only squared norms below it
        const uint32_t klo = norm_key(lo > 0.0 ? lo * lo * (1.0 - 0x1p-50) : 0.0);
        const int s0 = group_search16(live && lo > 0.0 ? pch : 0, [&](int k) {
            return pkey[min(k * kTileRows + kTileRows - 1, np - 1)] < klo;
        });
        // chunks whose first key is above that of hi^2 hold only squared norms above it
        const uint32_t khi = norm_key(hi == INFINITY ? 0.0 : hi * hi * (1.0 + 0x1p-50));
        const int s1 = group_search16(live && hi != INFINITY ? pch : 0,
                                      [&](int k) { return pkey[k * kTileRows] <= khi; });
        if (live) {
            k0 = s0;
            k1 = hi == INFINITY ? pch : max(s1, s0);
        }
    }
    if ((lane & (kTileCols - 1)) == 0) wave_sub[w * kTilesPerWave + lane / kTileCols] = make_int2(k0, k1);
    // the union: the smallest start and the largest end of the non-empty tile ranges
    int u0 = k1 > k0 ? k0 : INT_MAX, u1 = k1 > k0 ? k1 : 0;
#pragma unroll
    for (int d = kTileCols; d < kWave; d <<= 1) {
        u0 = min(u0, __shfl_xor(u0, d, kWave));
        u1 = max(u1, __shfl_xor(u1, d, kWave));
    }
    if (lane == 0) {
        wave_c0[w] = u1 > 0 ? u0 : 0;
        wave_len[w] = u1 > 0 ? u1 - u0 : 0;
    }
}

__global__ __launch_bounds__(kBlock) void band_waves(const MatchSet* __restrict__ sets,
                                                     const SetPlan* __restrict__ plan, int n_sets,
                                                     const double* __restrict__ n2, const double* __restrict__ r2,
                                                     const int32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ skey,
                                                     int32_t* __restrict__ wave_c0, int32_t* __restrict__ wave_len,
                                                     int2* __restrict__ wave_sub, const DevStatus* st) {
    const int64_t total = st->total_waves;
    const int64_t gw = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    for (int64_t w = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave; w < total; w += gw)
        wave_band(plan, n_sets, n2, r2, perm, skey, wave_c0, wave_len, wave_sub, w);
}

// Both directions in full: one wavefront per query chunk packs it, and the
// wavefront of the first chunk of each query wave also finds the wave's bands
// (band_waves' work), in one launch.
__global__ __launch_bounds__(kBlock) void pack_band_waves(const MatchSet* __restrict__ sets,
                                                          const SetPlan* __restrict__ plan, int n_sets, int dim,
                                                          int kp, const double* __restrict__ n2,
                                                          const double* __restrict__ r2,
                                                          const int32_t* __restrict__ perm,
                                                          const uint32_t* __restrict__ skey, double* __restrict__ pk,
                                                          int32_t* __restrict__ wave_c0,
                                                          int32_t* __restrict__ wave_len, int2* __restrict__ wave_sub,
                                                          DevStatus* st) {
    const int64_t total = st->total_chunks;
    const int64_t gw = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    for (int64_t g = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave; g < total; g += gw) {
        const int c = find_set(n_sets, g, [&](int s) { return static_cast<int64_t>(plan[s].chunk_off); });
        if (sets[c].flags & kSetRowsOnly) continue;  // uniform over the wave
        const SetPlan qc = plan[c];
        const int local = static_cast<int>(g - qc.chunk_off);
        pack_chunk(sets, qc, c, dim, kp, n2, perm, pk, st, g);
        if (local % (kBandWave / kTileRows) == 0)
            wave_band(plan, n_sets, n2, r2, perm, skey, wave_c0, wave_len, wave_sub,
                      qc.wave_off + local / (kBandWave / kTileRows));
    }
}

// Candidate tile lengths of the band plan: every length 1 .. 64, then four per
// octave (80, 96, 112, 128, 160, ...) up to 4096.  The plan takes the one with
// the least modelled time: with at most one tile per wavefront slot the
// longest tile, min(T, longest band) plus the fixed cost; with more, the mean
// load per slot (chunks plus the fixed cost of every tile) plus half a tile
// for the tail.
constexpr int kTileCands = 88;
__host__ __device__ constexpr int tile_len_cand(int i) {
    return i < 64 ? i + 1 : (64 << ((i - 64) / 4)) + (16 << ((i - 64) / 4)) * ((i - 64) % 4 + 1);
}
static_assert(tile_len_cand(kTileCands - 1) == 4096, "candidate lengths end at 4096");

}  // namespace

bool band_tile_candidate(int T) {
    for (int i = 0; i < kTileCands; ++i)
        if (tile_len_cand(i) == T) return true;
    return false;
}

namespace {

// Threads per candidate length when the plan counts tiles: 88 x 11 threads,
// thread (i, k) sums ceil(L_w / T_i) over the waves w = k mod 11.  Beyond
// kExactTileWaves waves (many rounds of tiles, where the count matters less
// than its cost) the count is estimated as total / T + waves / 2 and bounded by
// total / T + waves.
constexpr int kCandThreads = 11;
constexpr int kExactTileWaves = 4096;
static_assert(kTileCands * kCandThreads <= kPlanThreads, "one thread per (candidate, stripe)");

// Cuts the bands into tiles of at most T chunks (T the candidate length with
// the least modelled time over the band kernel's wavefront slots), then writes
// each wave's first tile and every tile's {wave, set, first chunk, end}.
__global__ __launch_bounds__(kPlanThreads) void band_plan(const SetPlan* __restrict__ plan, int n_sets,
                                                          const int32_t* __restrict__ wave_c0,
                                                          const int32_t* __restrict__ wave_len,
                                                          const int2* __restrict__ wave_sub,
                                                          int32_t* __restrict__ wave_tile, int4* __restrict__ tinfo,
                                                          int64_t tile_cap, int forced_T, DevStatus* st) {
    __shared__ int64_t smem[kPlanThreads / kWave];
    __shared__ int s_cnt[kTileCands][kCandThreads];  // tiles of each candidate length, per stripe of waves
    __shared__ int s_lmax[kPlanThreads / kWave];
    __shared__ int s_T;
    const int W = st->total_waves;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    int64_t len_sum = 0;
    int lmax = 0;
    for (int w = threadIdx.x; w < W; w += kPlanThreads) {
        len_sum += wave_len[w];
        lmax = max(lmax, wave_len[w]);
    }
    int64_t tot_len;
    block_excl_scan64(len_sum, smem, tot_len);
    // a length fixed by the tuning is taken whenever its tiles fit: counted first, the
    // model below is then not needed
    bool forced_fits = false;
    if (forced_T > 0) {
        int64_t cnt = 0;
        for (int w = threadIdx.x; w < W; w += kPlanThreads) cnt += (wave_len[w] + forced_T - 1) / forced_T;
        int64_t tiles;
        block_excl_scan64(cnt, smem, tiles);
        forced_fits = tiles <= tile_cap;
    }
    // exact tile counts sum_w ceil(L_w / T) of every candidate length; the quotient
    // from a float reciprocal, corrected to the exact one (L + T - 1 < 2^24)
    const bool exact = W <= kExactTileWaves;
    if (!forced_fits && exact && threadIdx.x < kTileCands * kCandThreads) {
        const int i = threadIdx.x / kCandThreads, k = threadIdx.x % kCandThreads;
        const int T = tile_len_cand(i);
        const float inv = 1.0f / static_cast<float>(T);
        int cnt = 0;
        for (int w = k; w < W; w += kCandThreads) {
            const int x = wave_len[w] + T - 1;
            int q = static_cast<int>(static_cast<float>(x) * inv);
            if ((q + 1) * T <= x) ++q;
            if (q * T > x) --q;
            cnt += q;
        }
        s_cnt[i][k] = cnt;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) lmax = max(lmax, __shfl_xor(lmax, d, kWave));
    if (lane == 0) s_lmax[wv] = lmax;
    __syncthreads();
    // wave 0: the modelled time of each candidate (lanes L and L + 64), the least wins,
    // the shorter length on a tie
    if (forced_fits) {
        if (threadIdx.x == 0) s_T = forced_T;
    } else if (wv == 0) {
        int lm = 0;
        for (int k = 0; k < kPlanThreads / kWave; ++k) lm = max(lm, s_lmax[k]);
        double t_best = INFINITY;
        int i_best = kTileCands;
        for (int i = lane; i < kTileCands; i += kWave) {
            const int Ti = tile_len_cand(i);
            int64_t tiles = 0, bound;
            if (exact) {
                for (int k = 0; k < kCandThreads; ++k) tiles += s_cnt[i][k];
                bound = tiles;
            } else {
                tiles = (tot_len + Ti - 1) / Ti + W / 2;
                bound = (tot_len + Ti - 1) / Ti + W;
            }
            const double len = static_cast<double>(min(Ti, max(lm, 1)));
            double t = INFINITY;
            if (bound <= tile_cap) {
                t = tiles <= kBandSlots
                        ? len + kTileOverhead
                        : (static_cast<double>(tot_len) + static_cast<double>(tiles) * kTileOverhead) / kBandSlots +
                              0.5 * (len + kTileOverhead);
                if (Ti == forced_T) t = -1.0;  // a length fixed by the tuning wins whenever its tiles fit
            }
            if (t < t_best) {
                t_best = t;
                i_best = i;
            }
        }
        const double m = wave_min_d(t_best);
        const int cand = t_best == m ? i_best : kTileCands;
        int first = cand;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) first = min(first, __shfl_xor(first, d, kWave));
        if (lane == 0) s_T = (m < INFINITY) ? tile_len_cand(first) : (1 << 30);  // one tile per wave always fits
    }
    __syncthreads();
    const int T = s_T;
    __shared__ int s_off[kPlanThreads], s_c0[kPlanThreads], s_len[kPlanThreads], s_set[kPlanThreads];
    int64_t carry = 0;
    int64_t pairs = 0;  // query-row products of the tiles (real queries and rows)
    for (int base = 0; base < W; base += kPlanThreads) {
        const int w = base + static_cast<int>(threadIdx.x);
        const int L = w < W ? wave_len[w] : 0;
        const int nt = (L + T - 1) / T;
        int64_t round_total;
        const int64_t rel = block_excl_scan64(nt, smem, round_total);
        int c = 0, c0 = 0;
        if (w < W) {
            wave_tile[w] = static_cast<int32_t>(carry + rel);
            c = find_set(n_sets, w, [&](int s) { return static_cast<int64_t>(plan[s].wave_off); });
            c0 = wave_c0[w];
            if (L > 0) {
                // each 16-query tile over its own chunk range
                const int nq = min(kBandWave, plan[c].n - (w - plan[c].wave_off) * kBandWave);
                const int np = plan[c ^ 1].n;
                for (int t = 0; t < kTilesPerWave; ++t) {
                    const int2 r = wave_sub[static_cast<int64_t>(w) * kTilesPerWave + t];
                    const int nq_t = min(kTileCols, max(0, nq - t * kTileCols));
                    if (r.y > r.x) pairs += static_cast<int64_t>(nq_t) * (min(r.y * kTileRows, np) - r.x * kTileRows);
                }
            }
        }
        s_off[threadIdx.x] = static_cast<int>(rel);
        s_c0[threadIdx.x] = c0;
        s_len[threadIdx.x] = L;
        s_set[threadIdx.x] = c;
        __syncthreads();
        // the round's tiles, a contiguous run per thread: the owning wave of the run's first
        // tile is the last whose first tile is <= it, and the run walks on from there
        const int in_round = min(kPlanThreads, W - base);
        const int64_t per = (round_total + kPlanThreads - 1) / kPlanThreads;
        const int64_t t_begin = min(round_total, static_cast<int64_t>(threadIdx.x) * per);
        const int64_t t_end = min(round_total, t_begin + per);
        if (t_begin < t_end) {
            int lo = 0, hi = in_round - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= t_begin) lo = mid;
                else hi = mid - 1;
            }
            for (int64_t t = t_begin; t < t_end; ++t) {
                if (carry + t >= tile_cap) break;
                while (lo + 1 < in_round && s_off[lo + 1] <= t) ++lo;  // waves without tiles are passed over
                const int k = static_cast<int>(t - s_off[lo]);
                const int a = s_c0[lo] + k * T;
                tinfo[carry + t] = make_int4(base + lo, s_set[lo], a, min(a + T, s_c0[lo] + s_len[lo]));
            }
        }
        __syncthreads();
        carry += round_total;
    }
    int64_t pairs_total;
    block_excl_scan64(pairs, smem, pairs_total);
    if (threadIdx.x == 0) {
        st->band_pairs = pairs_total;
        wave_tile[W] = static_cast<int32_t>(carry);
        st->total_tiles = static_cast<int32_t>(carry);
        st->tile_next = 0;
        st->band_step = T;
        if (carry > tile_cap) st->err_capacity = 1;
    }
}

// As absorb, skipped when no lane's four scores undercut its fourth best (the
// encoded scores are unique, so such a merge leaves top as it is).
__device__ __forceinline__ void absorb_some(double* top, const doublex4& acc, unsigned row0, unsigned keep) {
    double w0 = encode(acc[0], keep, row0), w1 = encode(acc[1], keep, row0 + 4u);
    double w2 = encode(acc[2], keep, row0 + 8u), w3 = encode(acc[3], keep, row0 + 12u);
    if (ballot(fmin(fmin(w0, w1), fmin(w2, w3)) < top[3])) {
        sort4(w0, w1, w2, w3);
        merge4(top, w0, w1, w2, w3);
    }
}

// Band tiles: each wavefront pulls tiles (64 queries of one wave against a
// range of partner chunks) from an atomic queue.  The partner chunk operands
// come straight from memory with raw buffer loads, ahead of the products; the
// waves share no data, so there is no barrier.  Each 16-query tile of the wave
// needs only the chunks of its own band: the four tiles take the chunks every
// one of them needs together (four products per chunk operand), and each tile
// takes the rest of its own band alone.  Every tile meets each of its chunks
// once, and a tile's product does not depend on the others', so the lists are
// those of the four tiles over their own bands.
// kBack only names the launch: 0 for the first direction of the one-sided
// form, 1 for the matching back, the FP64 re-runs and both directions in full
// (so that profiles tell them apart).
template <int KS, int kBack>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KS <= 9 ? 2 : 1))) void band_tiles(
    const SetPlan* __restrict__ plan, const double* __restrict__ pk, int dim, const int4* __restrict__ tinfo,
    const int2* __restrict__ wave_sub, double* __restrict__ part, DevStatus* st) {
    constexpr int kp = 4 * KS;
    constexpr int kChunk = kp * kTileRows;
    const int lane = lane_id();
    const int g = lane >> 4;
    const int l16 = lane & 15;
    const int total = st->err_capacity ? 0 : st->total_tiles;
    // The first tile of every wavefront is fixed, in the XCD-aware order (the waves of one XCD
    // take one contiguous range of the tile list: adjacent bands, whose partner chunks then stay
    // in that XCD's L2); only the tiles beyond one per wavefront come from the queue, counted
    // from kBandSlots.  A plan of at most one round takes no atomic at all (a queue that every
    // wavefront hits at once serialises on its one counter).
    // uniform from here on: the tile's descriptor, plans and buffer resources live in scalar
    // registers (a per-lane value would wrap every buffer load in a waterfall loop)
    int tile = __builtin_amdgcn_readfirstlane(static_cast<int>(xcd_wave_index()));
    for (; tile < total;) {
        const int4 ti = tinfo[tile];
        const SetPlan qc = plan[ti.y];
        const SetPlan pc = plan[ti.y ^ 1];
        const int col0 = (ti.x - qc.wave_off) * kBandWave;
        // the tiles' own chunk ranges within this tile's [c_begin, c_end), and the part
        // all of the tiles with a band share (tiles without queries have empty ranges)
        const int c_begin = ti.z, c_end = ti.w;
        int2 own[kTilesPerWave];
        int core0 = c_begin, core1 = c_end;
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) {
            const int2 r = wave_sub[static_cast<int64_t>(ti.x) * kTilesPerWave + t];
            own[t] = make_int2(max(r.x, c_begin), min(r.y, c_end));
            if (r.y > r.x) {
                core0 = max(core0, r.x);
                core1 = min(core1, r.y);
            }
        }
        double bq[kTilesPerWave][KS];
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) {
            const int chunk = min(col0 / kTileCols + t, qc.chunks - 1);
            const double* src = pk + static_cast<int64_t>(qc.chunk_off + chunk) * kChunk;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int k = 4 * s + g;
                const double scale = k < dim ? -2.0 : 0.0;
                const double add = k == dim ? 1.0 : 0.0;
                bq[t][s] = src[k * kTileRows + l16] * scale + add;
            }
        }
        double top[kTilesPerWave][4];
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) top[t][0] = top[t][1] = top[t][2] = top[t][3] = INFINITY;
        const unsigned keep = keep_mask(row_bits(pc.chunks));
        const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double*>(pk + static_cast<int64_t>(pc.chunk_off) * kChunk), 0,
            static_cast<int>(min(static_cast<int64_t>(pc.chunks) * kChunk * 8, static_cast<int64_t>(INT32_MAX))),
            static_cast<int>(kBufferWord3));
        const auto load_chunk = [&](double* dst, int c) {
#pragma unroll
            for (int s = 0; s < KS; ++s)
                dst[s] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                        rows, ((c * kChunk) + s * 4 * kTileRows + lane) * 8, 0, 0));
        };
        const bool has_core = core0 < core1;  // uniform over the wave
        if (has_core) {
            // two chunks in flight ahead of the products (a miss in L2 outlasts one chunk's products)
            double a[KS], an[KS];
            load_chunk(a, core0);
            load_chunk(an, min(core0 + 1, core1 - 1));
            for (int c = core0; c < core1; ++c) {
                double ann[KS];
                load_chunk(ann, min(c + 2, core1 - 1));
                __builtin_amdgcn_sched_barrier(0);
                doublex4 acc[kTilesPerWave];
                chunk_mfma<KS>(acc, a, bq);
                const unsigned row0 = static_cast<unsigned>(c * kTileRows + g);
#pragma unroll
                for (int t = 0; t < kTilesPerWave; ++t) absorb_some(top[t], acc[t], row0, keep);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    a[s] = an[s];
                    an[s] = ann[s];
                }
            }
        }
        // each tile alone over its range outside the shared part, one chunk in flight ahead
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) {
            const int e1 = own[t].y;
            const auto after = [&](int c) { return (has_core && c >= core0 && c < core1) ? core1 : c; };
            int c = after(own[t].x);
            if (c < e1) {  // uniform over the wave
                double a[KS];
                load_chunk(a, c);
                while (c < e1) {
                    const int cn = after(c + 1);
                    double an[KS];
                    load_chunk(an, min(cn, e1 - 1));
                    __builtin_amdgcn_sched_barrier(0);
                    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bq[t][s], acc, 0, 0, 0);
                    absorb_some(top[t], acc, static_cast<unsigned>(c * kTileRows + g), keep);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s = 0; s < KS; ++s) a[s] = an[s];
                    c = cn;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kTilesPerWave; ++t) {
            merge_lane(top[t], 16);
            merge_lane(top[t], 32);
            const int col = kTileCols * t + l16;
            if (g == 0 && col0 + col < qc.n) {
                double* dst = part + (static_cast<int64_t>(tile) * kBandWave + col) * kTopK;
                dst[0] = top[t][0];
                dst[1] = top[t][1];
                dst[2] = top[t][2];
                dst[3] = top[t][3];
            }
        }
        if (total <= kBandSlots) break;  // uniform: every tile was a first tile
        int next = 0;
        if (lane == 0) next = kBandSlots + static_cast<int>(atomicAdd(&st->tile_next, 1u));
        tile = __builtin_amdgcn_readfirstlane(next);
    }
}

// As rescore, for the band tiles: the query's lists are those of its wave's
// tiles, and candidates are packed partner positions mapped back through perm.
__global__ __launch_bounds__(kBlock) void rescore_band(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                       int dim, const double* __restrict__ part,
                                                       const double* __restrict__ n2, const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ wave_tile, int32_t* __restrict__ nn,
                                                       double* __restrict__ best, double* __restrict__ second,
                                                       int32_t* __restrict__ failed, int32_t* __restrict__ fb_list,
                                                       int64_t* __restrict__ fb_total, DevStatus* st) {
    // the queries only: index g = 64 (query wave) + packed position (scatter_pack clears the
    // flags of the rows-only slots)
    const int64_t total = static_cast<int64_t>(st->total_waves) * kBandWave;
    const bool no_tiles = st->err_capacity != 0;  // the results are void; the flags stay well defined
    const int q = lane_id() & (kQuad - 1);
    const int quad0 = lane_id() & ~(kQuad - 1);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * (kBlock / kQuad);
    for (int64_t g = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kQuad; g < total; g += gs) {
        const int64_t wq = g / kBandWave;
        const int c = find_set(n_sets, wq, [&](int s) { return static_cast<int64_t>(plan[s].wave_off); });
        const SetPlan qc = plan[c];
        // g runs over the packed (sorted) positions: the quads of a wave read adjacent columns
        // of the same tile lists, and the query's slot comes from perm beside those loads
        const int pos = static_cast<int>(wq - qc.wave_off) * kBandWave + static_cast<int>(g % kBandWave);
        if (pos >= qc.n) continue;  // the last wave's padding (uniform over the quad)
        if (no_tiles) {
            if (q == 0) failed[qc.q_off + pos] = 0;  // every slot of the set once
            continue;
        }
        const int j = perm[qc.q_off + pos];
        if (j < 0 || j >= qc.n) continue;  // never: the ranks are a permutation
        const int64_t slot = qc.q_off + j;
        const int p = c ^ 1;
        const int np = p < n_sets ? plan[p].n : 0;
        if (np == 0) {
            if (q == 0) {
                nn[slot] = -1;
                best[slot] = INFINITY;
                second[slot] = INFINITY;
                failed[slot] = 0;
            }
            continue;
        }
        const int w = static_cast<int>(wq);
        const int col = pos % kBandWave;
        const int t0 = wave_tile[w], t1 = wave_tile[w + 1];
        double top[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
        // the lane's lists four at a time: their loads in flight together
        for (int t = t0 + q; t < t1; t += 4 * kQuad) {
            double v[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tu = t + u * kQuad;
                const double* src = part + (static_cast<int64_t>(tu < t1 ? tu : t) * kBandWave + col) * kTopK;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[u][r] = src[r];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (t + u * kQuad < t1) merge4(top, v[u][0], v[u][1], v[u][2], v[u][3]);
        }
        merge_lane(top, 1);
        merge_lane(top, 2);
        const SetPlan pc = plan[p];
        const int bits = row_bits(pc.chunks);
        const double mine = q == 0 ? top[0] : (q == 1 ? top[1] : (q == 2 ? top[2] : top[3]));
        int row = -1;
        if (mine < kNoScore) {
            const int at = decode_row(mine, keep_mask(bits));
            if (at < np) row = perm[pc.q_off + at];  // only real rows are ever candidates
            if (row >= np) row = -1;
        }
        const double d = row >= 0 ? exact_d2(set_row(sets[p], row, dim), set_row(sets[c], j, dim), dim) : INFINITY;
        double dq[kQuad];
        int rq[kQuad];
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            dq[k] = __shfl(d, quad0 + k, kWave);
            rq[k] = __shfl(row, quad0 + k, kWave);
        }
        if (q != 0) continue;
        double b1 = INFINITY, b2 = INFINITY;
        int j1 = -1;
        int ncand = 0;
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            const int i = rq[k];
            if (i < 0) continue;
            ++ncand;
            const double dk = dq[k];
            if (dk < b1 || (dk == b1 && i < j1)) {
                b2 = b1;
                b1 = dk;
                j1 = i;
            } else if (dk < b2) {
                b2 = dk;
            }
        }
        bool ok;
        if (ncand >= np) {
            ok = true;  // every row was a candidate
        } else {
            // rows outside the band are farther than R >= the second distance; inside it,
            // the bound of the full form: MFMA error 128 u (2 max ||x||^2 + 2 ||y||^2)
            // plus the encoding error 2^(bits - 52) |t|
            const double mx = __longlong_as_double(static_cast<long long>(pc.max_norm_bits));
            const double rel = 0x1p-46 + ldexp(1.0, bits - 52);
            const double E = rel * (2.0 * mx + 2.0 * n2[slot]) + 1e-300;
            const double bound = top[3] + n2[slot] - E;
            ok = ncand == 4 && b2 < bound;
        }
        if (ok) {
            nn[slot] = j1;
            best[slot] = b1;
            second[slot] = b2;
        } else {
            // listed for the exact scan in the set's own range (in any order: each query's scan stands alone)
            append_open(plan, c, qc.q_off, static_cast<int32_t>(slot), fb_list, fb_total);
        }
        failed[slot] = ok ? 0 : 1;
    }
}


}  // namespace

MatchWs carve_match(Carver& c, int n_sets, int64_t q_cap, int dim, bool rerun) {
    MatchWs w;
    w.kp = (dim + 1 <= 36) ? 36 : 68;  // 4 KS for the two kernel instantiations (dim <= 64)
    w.q_cap = std::max<int64_t>(q_cap, 1);
    w.chunk_cap = q_cap / kTileRows + n_sets + 1;
    // the modelled segment counts keep queries x segments within about kTargetTiles x kColsPerBlock
    w.part_cap = kTopK * (w.q_cap + static_cast<int64_t>(kTargetTiles) * kColsPerBlock);
    // the band tiles hold kBandWave lists each
    w.part_cap = std::max<int64_t>(w.part_cap, kTopK * kBandWave * (kBandTiles + w.q_cap / kBandWave + n_sets + 1));
    w.plan = c.take<SetPlan>(static_cast<size_t>(std::max(n_sets, 1)));
    w.pk = c.take<double>(static_cast<size_t>(w.chunk_cap) * w.kp * kTileRows);
    w.n2 = c.take<double>(static_cast<size_t>(w.q_cap));
    w.lp_nx = c.take<double>(static_cast<size_t>(w.q_cap));
    w.lp_pairs = c.take<PairLp>(static_cast<size_t>(n_sets / 2 + 1));
    w.part = c.take<double>(static_cast<size_t>(w.part_cap));
    w.nn = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.best = c.take<double>(static_cast<size_t>(w.q_cap));
    w.second = c.take<double>(static_cast<size_t>(w.q_cap));
    w.fb_list = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.fb_total = c.take<int64_t>(1);
    w.n_grp = w.q_cap / kWave + n_sets + 1;  // per-set groups: at most one partial group per set
    w.grp_done = c.take<int32_t>(static_cast<size_t>(w.n_grp));
    w.flag = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.pos = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(w.q_cap));
    w.wave_cap = w.q_cap / kBandWave + n_sets + 1;
    w.tile_cap = kBandTiles + w.wave_cap;
    w.rank = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.perm = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.r2 = c.take<double>(static_cast<size_t>(w.q_cap));
    w.skey = c.take<uint32_t>(static_cast<size_t>(w.q_cap));
    w.wave_c0 = c.take<int32_t>(static_cast<size_t>(w.wave_cap));
    w.wave_len = c.take<int32_t>(static_cast<size_t>(w.wave_cap));
    w.wave_sub = c.take<int2>(static_cast<size_t>(w.wave_cap) * kTilesPerWave);
    // class histograms of the query sort tiles (at most q_cap / kSortTile + n_sets of them)
    w.chist = c.take<int32_t>(static_cast<size_t>(w.q_cap / kSortTile + n_sets + 1) * kClasses);
    w.wave_tile = c.take<int32_t>(static_cast<size_t>(w.wave_cap + 1));
    w.tinfo = c.take<int4>(static_cast<size_t>(w.tile_cap));
    w.rr = RerunWs{};
    w.one_sided = nullptr;
    if (rerun && 2 * n_sets <= kPlanThreads) {
        w.one_sided = c.take<MatchSet>(static_cast<size_t>(n_sets));
        w.rr.st = c.take<DevStatus>(1);
        w.rr.sets = c.take<MatchSet>(static_cast<size_t>(2 * n_sets));
        w.rr.f_slot = c.take<int32_t>(static_cast<size_t>(w.q_cap));
        w.rr.f_row = c.take<int32_t>(static_cast<size_t>(w.q_cap));
        w.rr.f_count = c.take<int32_t>(static_cast<size_t>(std::max(n_sets, 1)));
        w.rr.f_total = c.take<int64_t>(1);
        Carver probe(nullptr, 0);
        carve_match(probe, 2 * n_sets, 2 * w.q_cap, dim, false);
        w.rr.region_bytes = probe.off;
        w.rr.region = c.take<char>(probe.off);
    }
    return w;
}

kmg_status match_lp(const MatchSet* sets, int n_sets, int dim, int prec, DevStatus* st, const MatchWs& w,
                    hipStream_t s);
kmg_status match_fp64(const MatchSet* sets, int n_sets, int dim, DevStatus* st, const MatchWs& w, hipStream_t s);
// With oside, the sets are made one-sided by the planner and written there;
// with both as well, the n_sets / 2 input sets are expanded there into the
// n_sets sets of both directions in full (and st is cleared first).
kmg_status match_band(const MatchSet* sets, int n_sets, int dim, DevStatus* st, const MatchWs& w, hipStream_t s,
                      MatchSet* oside = nullptr, bool both = false);
kmg_status exact_fallback(const MatchSet* sets, int n_sets, int dim, DevStatus* st, const MatchWs& w,
                          hipStream_t s);
kmg_status exact_listed(const MatchSet* sets, int n_sets, int dim, const MatchWs& w, hipStream_t s,
                        bool per_set = false);

kmg_status match_back(const MatchSet* sets1, int n_sets, int dim, DevStatus* st, const MatchWs& w, hipStream_t s);

// Both directions in full in one band pass (the four-set form above).
kmg_status match_both(const MatchSet* sets, int n_sets, int dim, DevStatus* st, const MatchWs& w,
                      const PairOutDev* outs, int64_t* counts, int counts_stride, hipStream_t s,
                      const CloudState* cs, int64_t nnz_cap) {
    Carver c2(w.rr.region, w.rr.region_bytes);
    const MatchWs w2 = carve_match(c2, 2 * n_sets, 2 * w.q_cap, dim, false);
    if (!c2.fits()) return KMG_ERR_WORKSPACE;
    // the planner writes the four sets of each pair to rr.sets and clears rr.st
    KMG_TRY(match_band(sets, 2 * n_sets, dim, w.rr.st, w2, s, w.rr.sets, true));
    StageScope sc(ST_MATCH_MUTUAL, s);
    mutual_both<<<grid_cap(w2.q_cap, kBlock), kBlock, 0, s>>>(w2.plan, 2 * n_sets, w2.nn, w2.q_cap, w2.flag,
                                                              w2.scan_tmp, w.rr.st);
    KMG_TRY(launch_status());
    KMG_TRY(scan_exclusive_summed(w2.flag, w2.pos, w2.q_cap, &w.rr.st->pairs_total, w2.scan_tmp, s));
    emit_both<<<std::max(grid_cap(w2.q_cap, kBlock), grid_for(n_sets, kBlock)), kBlock, 0, s>>>(
        sets, w2.plan, 2 * n_sets, w2.flag, w2.pos, w2.nn, w2.best, w2.second, outs, st, w.rr.st, counts,
        counts_stride, cs, nnz_cap);
    return launch_status();
}

kmg_status match_batch(const MatchSet* sets, int n_sets, int dim, int prec, DevStatus* st, const MatchWs& w,
                       const PairOutDev* outs, int64_t* counts, int counts_stride, hipStream_t s,
                       const CloudState* cs, int64_t nnz_cap) {
    if (n_sets < 2 || n_sets > kMaxClouds) return KMG_ERR_ARG;
    if (tuning().match_form == 1 && w.one_sided && prec != KMG_FP16 && prec != KMG_BF16)
        return match_both(sets, n_sets, dim, st, w, outs, counts, counts_stride, s, cs, nnz_cap);
    // one-sided form when the workspace holds the second plan, else both directions in full
    const MatchSet* first = w.one_sided ? w.one_sided : sets;
    if (prec == KMG_FP16 || prec == KMG_BF16) {
        if (w.one_sided) {
            one_sided_sets<<<grid_for(n_sets, 64), 64, 0, s>>>(sets, n_sets, w.one_sided);
            KMG_TRY(launch_status());
        }
        KMG_TRY(match_lp(first, n_sets, dim, prec, st, w, s));
    } else if (w.one_sided) {
        KMG_TRY(match_band(sets, n_sets, dim, st, w, s, w.one_sided));  // the planner writes the one-sided sets
    } else {
        KMG_TRY(match_fp64(first, n_sets, dim, st, w, s));
    }
    if (w.one_sided) KMG_TRY(match_back(first, n_sets, dim, st, w, s));
    {
        StageScope sc(ST_MATCH_MUTUAL, s);
        if (w.one_sided) {
            // the matching back wrote the flags of the live slots
            KMG_TRY(scan_exclusive(w.flag, w.pos, w.q_cap, &st->pairs_total, w.scan_tmp, s, &st->total_queries));
        } else {
            mutual_flags<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(w.plan, n_sets, w.nn, w.q_cap, w.flag, st);
            KMG_TRY(launch_status());
            KMG_TRY(scan_exclusive(w.flag, w.pos, w.q_cap, &st->pairs_total, w.scan_tmp, s));
        }
        emit_pairs<<<std::max(grid_cap(w.q_cap, kBlock), grid_for(n_sets, kBlock)), kBlock, 0, s>>>(
            sets, w.plan, n_sets, w.flag, w.pos, w.nn, w.best, w.second, outs, st, counts, counts_stride, cs,
            nnz_cap);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

// Candidates in FP16 / BF16 with FP32 accumulation (lower-bound ranking),
// exact FP64 re-score and certificate; the queries left uncertified re-run
// through the FP64 form against their full partner sets (or, when the batch
// has too many sets for a second plan, are re-scanned exactly).
kmg_status match_lp(const MatchSet* sets, int n_sets, int dim, int prec, DevStatus* st, const MatchWs& w,
                    hipStream_t s) {
    if (dim > kLpMaxDim) return KMG_ERR_ARG;
    uint4* pk = reinterpret_cast<uint4*>(w.pk);  // a chunk of halves (4 KB) fits a 36-deep FP64 chunk
    const int n_pairs = n_sets / 2;
    {
        StageScope sc(ST_MATCH_PACK, s);
        plan_sets<<<1, kPlanThreads, 0, s>>>(sets, n_sets, w.kp, w.part_cap, w.plan, st, w.grp_done, w.n_grp);
        KMG_TRY(launch_status());
        lp_center<<<n_pairs, kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.lp_pairs);
        KMG_TRY(launch_status());
        lp_rows<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.lp_pairs, w.n2, w.lp_nx,
                                                            st);
        KMG_TRY(launch_status());
        lp_scale<<<grid_for(n_pairs, 64), 64, 0, s>>>(w.lp_pairs, n_pairs);
        KMG_TRY(launch_status());
        if (prec == KMG_FP16) {
            lp_pack<_Float16><<<grid_cap(w.chunk_cap * kLpPieces, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim,
                                                                                        w.lp_pairs, pk, st);
        } else {
            lp_pack<__bf16><<<grid_cap(w.chunk_cap * kLpPieces, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim,
                                                                                      w.lp_pairs, pk, st);
        }
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_MATCH_TOPK, s);
        if (prec == KMG_FP16) {
            topk_lp<_Float16><<<kTopkBlocks, kBlock, 0, s>>>(w.plan, n_sets, pk, w.n2, w.lp_nx, w.lp_pairs, dim,
                                                             w.part, st);
        } else {
            topk_lp<__bf16><<<kTopkBlocks, kBlock, 0, s>>>(w.plan, n_sets, pk, w.n2, w.lp_nx, w.lp_pairs, dim,
                                                           w.part, st);
        }
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_MATCH_RESCORE, s);
        rescore_lp<<<grid_cap(w.q_cap * kQuad, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.part, w.lp_nx,
                                                                        w.lp_pairs, w.nn, w.best, w.second, w.flag,
                                                                        st);
        KMG_TRY(launch_status());
        if (!w.rr.region) return exact_fallback(sets, n_sets, dim, st, w, s);
        KMG_TRY(scan_exclusive(w.flag, w.pos, w.q_cap, w.rr.f_total, w.scan_tmp, s, &st->total_queries));
        rerun_lists<<<std::max(grid_cap(w.q_cap, kBlock), grid_for(n_sets + 64, kBlock)), kBlock, 0, s>>>(sets, w.plan, n_sets, w.flag, w.pos, w.rr.f_total,
                                                                w.q_cap, w.rr.f_slot, w.rr.f_row, w.rr.f_count,
                                                                w.rr.sets, w.rr.st, st);
        KMG_TRY(launch_status());
    }
    Carver c2(w.rr.region, w.rr.region_bytes);
    const MatchWs w2 = carve_match(c2, 2 * n_sets, 2 * w.q_cap, dim, false);
    if (!c2.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(match_band(w.rr.sets, 2 * n_sets, dim, w.rr.st, w2, s));
    {
        StageScope sc(ST_MATCH_RESCORE, s);
        rerun_scatter<<<grid_cap(w2.q_cap, kBlock), kBlock, 0, s>>>(w2.plan, 2 * n_sets, w.rr.st, w2.nn, w2.best,
                                                                   w2.second, w.plan, w.pos, w.rr.f_slot, w.nn,
                                                                   w.best, w.second, st, 0, nullptr);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
}

// Candidates on FP64 matrix cores, exact re-score and certificate, exact
// scans for the rest.
kmg_status match_fp64(const MatchSet* sets, int n_sets, int dim, DevStatus* st, const MatchWs& w, hipStream_t s) {
    const int ks = w.kp / 4;  // 9 or 17: the packed depth equals the kernel's 4 KS
    {
        StageScope sc(ST_MATCH_PACK, s);
        plan_sets<<<1, kPlanThreads, 0, s>>>(sets, n_sets, w.kp, w.part_cap, w.plan, st, w.grp_done, w.n_grp);
        KMG_TRY(launch_status());
        row_norms<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.n2, st, nullptr);
        KMG_TRY(launch_status());
        pack_rows<<<grid_cap(w.chunk_cap * w.kp * kTileRows, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim,
                                                                                     w.kp, w.n2, w.pk, st);
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_MATCH_TOPK, s);
        if (ks <= 9) {
            topk_tiles<9><<<kTopkBlocks, kBlock, 0, s>>>(w.plan, n_sets, w.pk, dim, w.part, st);
        } else if (ks <= 17) {
            topk_tiles<17><<<kTopkBlocks, kBlock, 0, s>>>(w.plan, n_sets, w.pk, dim, w.part, st);
        } else {
            return KMG_ERR_ARG;
        }
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_MATCH_RESCORE, s);
        rescore<<<grid_cap(w.q_cap * kQuad, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.part, w.n2, w.nn,
                                                                    w.best, w.second, w.flag, st);
        KMG_TRY(launch_status());
        KMG_TRY(exact_fallback(sets, n_sets, dim, st, w, s));
    }
    return KMG_OK;
}

// The matching back of the one-sided form: the rows-only rows that are some
// query's nearest neighbour are matched in FP64 against their full partner
// sets (the re-run machinery with the image as its list), and the answers
// land in their main slots.
kmg_status match_back(const MatchSet* sets1, int n_sets, int dim, DevStatus* st, const MatchWs& w, hipStream_t s) {
    StageScope sc(ST_MATCH_IMAGE, s);
    image_lists<<<std::max(grid_cap(w.q_cap, kBlock), grid_for(n_sets + 64, kBlock)), kBlock, 0, s>>>(
        sets1, w.plan, n_sets, w.nn, w.flag, w.rr.f_slot, w.rr.f_row, w.rr.sets, w.rr.st, st);
    KMG_TRY(launch_status());
    Carver c2(w.rr.region, w.rr.region_bytes);
    const MatchWs w2 = carve_match(c2, 2 * n_sets, 2 * w.q_cap, dim, false);
    if (!c2.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(match_band(w.rr.sets, 2 * n_sets, dim, w.rr.st, w2, s));
    rerun_scatter<<<std::max(grid_cap(w2.q_cap, kBlock), grid_for(n_sets, kBlock)), kBlock, 0, s>>>(
        w2.plan, 2 * n_sets, w.rr.st, w2.nn, w2.best, w2.second, w.plan, nullptr, w.rr.f_slot, w.nn, w.best,
        w.second, st, 1, w.flag);
    return launch_status();
}

// The FP64 form with norm bands, for sets paired as (queries, rows-only
// partner) in either order: partner rows ranked and packed by norm, seed
// bounds, queries ranked by (class, norm) and packed, bands, band tiles, exact
// re-score and certificate, exact scans for the rest.
kmg_status match_band(const MatchSet* sets_in, int n_sets, int dim, DevStatus* st, const MatchWs& w, hipStream_t s,
                      MatchSet* oside, bool both) {
    const int ks = w.kp / 4;  // 9 or 17: the packed depth equals the kernel's 4 KS
    if (ks != 9 && ks != 17) return KMG_ERR_ARG;
    const MatchSet* sets = oside ? oside : sets_in;
    const bool first = oside && !both;  // the launch name: the one-sided first direction, or the rest
    {
        StageScope sc(ST_MATCH_PACK, s);
        plan_band<<<1, kPlanThreads, 0, s>>>(sets_in, n_sets, w.kp, w.plan, st, oside, both ? 1 : 0, w.fb_total,
                                             w.grp_done, w.n_grp, w.scan_tmp,
                                             static_cast<int64_t>(scan_temp_elems(w.q_cap)));
        KMG_TRY(launch_status());
        row_norms<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.n2, st, nullptr);
        KMG_TRY(launch_status());
        // the sorted tile values live in best, which the re-score writes only afterwards
        unsigned long long* sorted = reinterpret_cast<unsigned long long*>(w.best);
        for (int role = 1; role >= 0; --role) {  // partners first: the seeds need their order
            if (role == 0) {
                const unsigned gs = grid_cap(w.q_cap * 16, kBlock);
                if (ks == 9)
                    band_seeds<9><<<gs, kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.pk, w.n2, w.skey, w.r2, st);
                else
                    band_seeds<17><<<gs, kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.pk, w.n2, w.skey, w.r2, st);
                KMG_TRY(launch_status());
            }
            const unsigned gt = grid_cap((w.q_cap / kSortTile + n_sets + 1) * kBlock, kBlock);
            if (both && role == 0) {  // the queries: a partition by class of their cloud's norm order
                class_hist<<<gt, kSortTile, 0, s>>>(sets, w.plan, n_sets, w.r2, w.perm, w.chist, st);
                KMG_TRY(launch_status());
                class_rank<<<gt, kSortTile, 0, s>>>(sets, w.plan, n_sets, w.r2, w.perm, w.chist, st);
                KMG_TRY(launch_status());
            } else {
                tile_sort<<<gt, kSortTile, 0, s>>>(sets, w.plan, n_sets, role, w.n2, w.r2, sorted, w.rank, st);
                KMG_TRY(launch_status());
                cross_rank<<<kPersistBlocks, kSortThreads, 0, s>>>(sets, w.plan, n_sets, role, sorted, w.rank, st);
                KMG_TRY(launch_status());
            }
            if (both && role == 0) {  // perm holds the queries' order: each wave packs its chunks, then its bands
                pack_band_waves<<<grid_cap(w.chunk_cap * kWave, kBlock), kBlock, 0, s>>>(
                    sets, w.plan, n_sets, dim, w.kp, w.n2, w.r2, w.perm, w.skey, w.pk, w.wave_c0, w.wave_len,
                    w.wave_sub, st);
            } else {
                scatter_pack<<<grid_cap(w.q_cap * 4, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.kp, role,
                                                                                 w.n2, w.rank, w.pk, w.perm, w.skey,
                                                                                 w.flag, st);
            }
            KMG_TRY(launch_status());
        }
        if (!both) {  // (both directions in full: pack_band_waves found the bands)
            band_waves<<<grid_cap(w.wave_cap * kWave, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, w.n2, w.r2,
                                                                               w.perm, w.skey, w.wave_c0, w.wave_len,
                                                                               w.wave_sub, st);
            KMG_TRY(launch_status());
        }
        band_plan<<<1, kPlanThreads, 0, s>>>(w.plan, n_sets, w.wave_c0, w.wave_len, w.wave_sub, w.wave_tile, w.tinfo,
                                             w.tile_cap, tuning().band_tile, st);
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_MATCH_TOPK, s);
        if (ks == 9) {
            if (first) band_tiles<9, 0><<<kBandBlocks, kBlock, 0, s>>>(w.plan, w.pk, dim, w.tinfo, w.wave_sub, w.part, st);
            else band_tiles<9, 1><<<kBandBlocks, kBlock, 0, s>>>(w.plan, w.pk, dim, w.tinfo, w.wave_sub, w.part, st);
        } else {
            if (first) band_tiles<17, 0><<<kBandBlocks, kBlock, 0, s>>>(w.plan, w.pk, dim, w.tinfo, w.wave_sub, w.part, st);
            else band_tiles<17, 1><<<kBandBlocks, kBlock, 0, s>>>(w.plan, w.pk, dim, w.tinfo, w.wave_sub, w.part, st);
        }
        KMG_TRY(launch_status());
        timer_note_work(&st->band_pairs);
    }
    {
        StageScope sc(ST_MATCH_RESCORE, s);
        rescore_band<<<grid_cap(w.q_cap * kQuad, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.part, w.n2,
                                                                          w.perm, w.wave_tile, w.nn, w.best, w.second,
                                                                          w.flag, w.fb_list, w.fb_total, st);
        KMG_TRY(launch_status());
        KMG_TRY(exact_listed(sets, n_sets, dim, w, s, true));
    }
    return KMG_OK;
}

// Exact scans of the queries flagged in w.flag, grouped in slot order.
kmg_status exact_fallback(const MatchSet* sets, int n_sets, int dim, DevStatus* st, const MatchWs& w,
                          hipStream_t s) {
    KMG_TRY(scan_exclusive(w.flag, w.pos, w.q_cap, w.fb_total, w.scan_tmp, s, &st->total_queries, w.fb_list));
    return exact_listed(sets, n_sets, dim, w, s);
}

// Exact scans of the queries already listed in w.fb_list: *w.fb_total of them,
// in slot order, or (per_set) plan[c].n_fb of set c from slot plan[c].q_off on.
kmg_status exact_listed(const MatchSet* sets, int n_sets, int dim, const MatchWs& w, hipStream_t s, bool per_set) {
    if (dim < 1 || dim > 4 * 17) return KMG_ERR_ARG;
    if (dim <= 4 * 9)
        exact_grouped<9><<<kPersistBlocks, kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.fb_list, w.fb_total,
                                                          per_set ? 1 : 0, w.part_cap, w.part, w.grp_done, w.nn,
                                                          w.best, w.second);
    else
        exact_grouped<17><<<kPersistBlocks, kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.fb_list, w.fb_total,
                                                           per_set ? 1 : 0, w.part_cap, w.part, w.grp_done, w.nn,
                                                           w.best, w.second);
    return launch_status();
}

// ---------------------------------------------------- single pair entry --

size_t match_ws(int64_t np, int64_t nq, int dim) {
    Carver c(nullptr, 0);
    c.take<DevStatus>(1);
    c.take<MatchSet>(2);
    c.take<int32_t>(2);
    c.take<PairOutDev>(1);
    c.take<int64_t>(8);
    carve_match(c, 2, np + nq, dim);
    return c.off;
}

kmg_status match(const float* dp, const int32_t* rp, int64_t np, const float* dq, const int32_t* rq, int64_t nq,
                 int dim, int prec, int32_t* pairs, float* d1, float* d2, int64_t cap, int64_t* n_pairs_host,
                 int64_t* n_fallback_host, void* ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    DevStatus* st = c.take<DevStatus>(1);
    MatchSet* sets = c.take<MatchSet>(2);
    int32_t* cnt = c.take<int32_t>(2);
    PairOutDev* outs = c.take<PairOutDev>(1);
    int64_t* counts = c.take<int64_t>(8);
    MatchWs w = carve_match(c, 2, np + nq, dim);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    *n_pairs_host = 0;
    if (n_fallback_host) *n_fallback_host = 0;
    if (np == 0 || nq == 0) return KMG_OK;
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(st), 0u, sizeof(DevStatus) / 4, s));
    KMG_TRY(fill_u64(reinterpret_cast<uint64_t*>(counts), 0ull, 8, s));
    MatchSet a{dp, rp, nullptr, 0, 0}, b{dq, rq, nullptr, 0, 0};  // query sets, flags 0
    PairOutDev o{pairs, d1, d2, cap};
    write_pair_sets<<<1, 1, 0, s>>>(sets, cnt, a, b, static_cast<int32_t>(np), static_cast<int32_t>(nq), outs, o);
    KMG_TRY(launch_status());
    KMG_TRY(match_batch(sets, 2, dim, prec, st, w, outs, counts, 8, s));
    int64_t hc[8];
    DevStatus hs;
    KMG_TRY_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    timer_collect();
    if (hs.err_capacity) return KMG_ERR_WORKSPACE;
    *n_pairs_host = hc[0];
    if (n_fallback_host) *n_fallback_host = hc[5];
    if (hc[0] > cap) return KMG_ERR_CAPACITY;
    return KMG_OK;
}

}  // namespace kmg
