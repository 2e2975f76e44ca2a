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
constexpr int kTargetTiles = 4096;  // tiles wanted per launch (8 per persistent block)
constexpr int kMaxSegs = 32;
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

__global__ __launch_bounds__(kPlanThreads) void plan_sets(const MatchSet* __restrict__ sets, int n_sets, int kp,
                                                         int64_t part_cap, SetPlan* plan, DevStatus* st) {
    __shared__ int64_t smem[kPlanThreads / kWave];
    __shared__ int s_segs;
    __shared__ int s_chunks[kPlanThreads];
    __shared__ int s_n[kPlanThreads];
    const int c = threadIdx.x;
    const bool live = c < n_sets;
    const int n = live ? *sets[c].n : 0;
    const int chunks = (n + kTileRows - 1) / kTileRows;
    const int cblocks = (n + kColsPerBlock - 1) / kColsPerBlock;
    int64_t tq, tc, tb;
    const int64_t q_off = block_excl_scan64(n, smem, tq);
    const int64_t c_off = block_excl_scan64(chunks, smem, tc);
    block_excl_scan64(cblocks, smem, tb);
    s_chunks[c] = chunks;
    s_n[c] = n;
    // one buffer descriptor spans a set's packed rows: keep them below 2 GiB
    if (static_cast<int64_t>(chunks) * kp * kTileRows * 8 > INT32_MAX) st->err_capacity = 1;
    if (c == 0) {
        int S = static_cast<int>(tb > 0 ? kTargetTiles / tb : 1);
        S = S < 1 ? 1 : (S > kMaxSegs ? kMaxSegs : S);
        if (S >= 8) S &= ~7;  // a multiple of 8: the tiles of a column block spread over the eight XCDs
        s_segs = S;
    }
    __syncthreads();
    // the partner's rows are split into segments (sets pair up as 2i, 2i + 1): at least the
    // common count, and enough that no tile sweeps more than kSegChunks chunks, so the tiles
    // of uneven batches stay comparable in size
    const int p = c ^ 1;
    const int pch = (live && p < n_sets) ? s_chunks[p] : 0;
    const int pn = (live && p < n_sets) ? s_n[p] : 0;
    const int deep = (pch + kSegChunks - 1) / kSegChunks;
    int segs = s_segs > deep ? s_segs : deep;
    segs = segs < pch ? segs : (pch > 0 ? pch : 1);
    int64_t tpart;
    block_excl_scan64(live ? static_cast<int64_t>(n) * segs * kTopK : 0, smem, tpart);
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
    const int64_t p_off = block_excl_scan64(live ? static_cast<int64_t>(n) * segs * kTopK : 0, smem, tpart);
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

__global__ __launch_bounds__(kBlock) void row_norms(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                    int dim, double* __restrict__ n2, const DevStatus* st) {
#pragma clang fp contract(off)
    const int64_t total = st->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < total; t += gs) {
        const int c = find_set(n_sets, t, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const float* x = set_row(sets[c], static_cast<int>(t - plan[c].q_off), dim);
        double acc = 0.0;
        for (int k = 0; k < dim; ++k) {
            const double v = x[k];
            acc = acc + v * v;
        }
        n2[t] = acc;
        // one atomic per wave when the wave's rows share a set (the common case)
        const uint64_t live = ballot(true);
        const int c0 = __shfl(c, __ffsll(static_cast<unsigned long long>(live)) - 1, kWave);
        const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(acc));
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
    while (true) {
        if (threadIdx.x == 0) s_tile = static_cast<int>(atomicAdd(&st->tile_next, 1u));
        __syncthreads();
        const int tile = s_tile;
        __syncthreads();
        if (tile >= total) break;
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

constexpr int kQuad = 4;  // lanes per query in the re-scoring kernel

// Four lanes per query slot: lane q merges the segment lists q, q + 4, ..,
// the quad merges its lists, lane q re-scores candidate q exactly, and the
// first lane certifies the result or queues the query for an exact scan.
__global__ __launch_bounds__(kBlock) void rescore(const MatchSet* __restrict__ sets, SetPlan* plan, int n_sets,
                                                  int dim, const double* __restrict__ part,
                                                  const double* __restrict__ n2, int32_t* __restrict__ nn,
                                                  double* __restrict__ best, double* __restrict__ second,
                                                  int32_t* __restrict__ fb_list, DevStatus* st) {
    const int64_t total = st->total_queries;
    const int q = lane_id() & (kQuad - 1);
    const int quad0 = lane_id() & ~(kQuad - 1);
    const int64_t gs = static_cast<int64_t>(gridDim.x) * (kBlock / kQuad);
    for (int64_t slot = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kQuad; slot < total;
         slot += gs) {
        const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const int p = c ^ 1;
        const SetPlan qc = plan[c];
        const int j = static_cast<int>(slot - qc.q_off);
        const int np = p < n_sets ? plan[p].n : 0;
        if (np == 0) {
            if (q == 0) {
                nn[slot] = -1;
                best[slot] = INFINITY;
                second[slot] = INFINITY;
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
            const uint32_t at = atomicAdd(&st->n_fallback, 1u);
            fb_list[at] = static_cast<int32_t>(slot);
            atomicAdd(&plan[c].n_fb, 1);
        }
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

// One block per queued query: exact FP64 scan over all partner rows.
__global__ __launch_bounds__(kBlock) void exact_scan(const MatchSet* __restrict__ sets,
                                                     const SetPlan* __restrict__ plan, int n_sets, int dim,
                                                     const int32_t* __restrict__ fb_list, const DevStatus* st,
                                                     int32_t* __restrict__ nn, double* __restrict__ best,
                                                     double* __restrict__ second) {
    __shared__ double s_b1[kBlock / kWave], s_b2[kBlock / kWave];
    __shared__ int s_j1[kBlock / kWave];
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int nfb = static_cast<int>(st->n_fallback);
    for (int w = blockIdx.x; w < nfb; w += gridDim.x) {
        const int64_t slot = fb_list[w];
        const int c = find_set(n_sets, slot, [&](int s) { return static_cast<int64_t>(plan[s].q_off); });
        const int p = c ^ 1;
        const int j = static_cast<int>(slot - plan[c].q_off);
        const int np = plan[p].n;
        const float* y = set_row(sets[c], j, dim);
        double b1 = INFINITY, b2 = INFINITY;
        int j1 = INT32_MAX;
        for (int i = threadIdx.x; i < np; i += kBlock) {  // ascending per thread
            const double d = exact_d2(set_row(sets[p], i, dim), y, dim);
            if (d < b1) {
                b2 = b1;
                b1 = d;
                j1 = i;
            } else if (d < b2) {
                b2 = d;
            }
        }
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const double ob1 = __shfl_xor(b1, d, kWave);
            const double ob2 = __shfl_xor(b2, d, kWave);
            const int oj1 = __shfl_xor(j1, d, kWave);
            combine_best(b1, j1, b2, ob1, oj1, ob2);
        }
        if (lane == 0) {
            s_b1[wv] = b1;
            s_b2[wv] = b2;
            s_j1[wv] = j1;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int o = 1; o < kBlock / kWave; ++o) combine_best(b1, j1, b2, s_b1[o], s_j1[o], s_b2[o]);
            nn[slot] = (j1 == INT32_MAX) ? -1 : j1;
            best[slot] = b1;
            second[slot] = b2;
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
                                                     const PairOutDev* __restrict__ outs, const DevStatus* st) {
    const int64_t total = st->total_queries;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t slot = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; slot < total; slot += gs) {
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

__global__ void pair_counts(const SetPlan* __restrict__ plan, int n_sets, const int32_t* __restrict__ pos,
                            const DevStatus* st, int64_t* counts, int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * i + 1 >= n_sets) return;
    const int64_t total = st->total_queries;
    const int64_t a = plan[2 * i].q_off, b = plan[2 * i + 1].q_off;
    const int64_t pa = a < total ? pos[a] : st->pairs_total;
    const int64_t pb = b < total ? pos[b] : st->pairs_total;
    counts[static_cast<int64_t>(i) * stride + 0] = pb - pa;
    counts[static_cast<int64_t>(i) * stride + 5] = plan[2 * i].n_fb + plan[2 * i + 1].n_fb;
}

}  // namespace

MatchWs carve_match(Carver& c, int n_sets, int64_t q_cap, int dim) {
    MatchWs w;
    w.kp = (dim + 1 <= 36) ? 36 : 68;  // 4 KS for the two kernel instantiations (dim <= 64)
    w.q_cap = std::max<int64_t>(q_cap, 1);
    w.chunk_cap = q_cap / kTileRows + n_sets + 1;
    // segments are chosen so that queries x segments stays near kTargetTiles x kColsPerBlock
    w.part_cap = kTopK * (w.q_cap + 2 * static_cast<int64_t>(kTargetTiles) * kColsPerBlock);
    w.plan = c.take<SetPlan>(static_cast<size_t>(std::max(n_sets, 1)));
    w.pk = c.take<double>(static_cast<size_t>(w.chunk_cap) * w.kp * kTileRows);
    w.n2 = c.take<double>(static_cast<size_t>(w.q_cap));
    w.part = c.take<double>(static_cast<size_t>(w.part_cap));
    w.nn = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.best = c.take<double>(static_cast<size_t>(w.q_cap));
    w.second = c.take<double>(static_cast<size_t>(w.q_cap));
    w.fb_list = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.flag = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.pos = c.take<int32_t>(static_cast<size_t>(w.q_cap));
    w.scan_tmp = c.take<int64_t>(scan_temp_elems(w.q_cap));
    return w;
}

kmg_status match_batch(const MatchSet* sets, int n_sets, int dim, int prec, DevStatus* st, const MatchWs& w,
                       const PairOutDev* outs, int64_t* counts, int counts_stride, hipStream_t s) {
    (void)prec;
    if (n_sets < 2 || n_sets > kMaxClouds) return KMG_ERR_ARG;
    const int ks = w.kp / 4;  // 9 or 17: the packed depth equals the kernel's 4 KS
    {
        StageScope sc(ST_MATCH_PACK, s);
        plan_sets<<<1, kPlanThreads, 0, s>>>(sets, n_sets, w.kp, w.part_cap, w.plan, st);
        KMG_TRY(launch_status());
        row_norms<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.n2, st);
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
                                                                    w.best, w.second, w.fb_list, st);
        KMG_TRY(launch_status());
        exact_scan<<<grid_cap(w.q_cap, 1), kBlock, 0, s>>>(sets, w.plan, n_sets, dim, w.fb_list, st, w.nn, w.best,
                                                          w.second);
        KMG_TRY(launch_status());
    }
    {
        StageScope sc(ST_MATCH_MUTUAL, s);
        mutual_flags<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(w.plan, n_sets, w.nn, w.q_cap, w.flag, st);
        KMG_TRY(launch_status());
        KMG_TRY(scan_exclusive(w.flag, w.pos, w.q_cap, &st->pairs_total, w.scan_tmp, s));
        emit_pairs<<<grid_cap(w.q_cap, kBlock), kBlock, 0, s>>>(sets, w.plan, n_sets, w.flag, w.pos, w.nn, w.best,
                                                               w.second, outs, st);
        KMG_TRY(launch_status());
        pair_counts<<<grid_for(n_sets / 2, 64), 64, 0, s>>>(w.plan, n_sets, w.pos, st, counts, counts_stride);
        KMG_TRY(launch_status());
    }
    return KMG_OK;
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
    MatchSet a{dp, rp, nullptr, 0, 0}, b{dq, rq, nullptr, 0, 0};
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
