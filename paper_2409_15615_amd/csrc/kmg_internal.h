// Internal declarations shared by the libkmg translation units.
//
// Every kernel works on a batch of clouds laid out in flattened index
// spaces: raw points of all clouds back to back, kept points back to back
// (cloud order, then ascending input index), one CSR over all kept points,
// one list of J rows.  Each point knows its cloud id; hash keys carry the
// cloud id, so one voxel table and one cell table serve the whole batch.
// Item counts are read from device memory and kernels loop over them with a
// fixed grid, so a whole batch runs without host synchronisation (and can be
// captured in a hipGraph).  The single-cloud entry points are batches of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kmg.h"

namespace kmg {

constexpr int kWave = 64;
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kAxisBits = 18;                                // packed keys: 18 bits per axis
constexpr int64_t kKeyBias = int64_t(1) << (kAxisBits - 1);  // axis keys in [-2^17, 2^17)
constexpr int kMaxClouds = 1022;                             // 10 bits of cloud id (1023 is reserved)
constexpr int kListSmall = 1024;                             // LDS neighbour list of the common fill pass
constexpr int kMaxDegree = 8192;                             // largest |N(q)| accepted
constexpr int kMaxBins = 32;                                 // largest H (3H <= 96 descriptor values)
constexpr int kMaxMatchDim = 64;                             // longest descriptor the matcher takes
constexpr int kTopK = 4;                                     // candidates kept per query before re-scoring
constexpr int kPersistBlocks = 2048;                         // grid of the grid-stride kernels

// Strict radius test d2 < r^2: an FP32 screen decides everything farther than
// a relative band of 4e-6 from the sphere (the FP32 error is below 1e-6
// relative); inside the band the exact FP64 expression decides.
struct RadiusTest {
    float lo2, hi2;  // FP32 band edges around r^2
    double r2;       // r * r in FP64
};

inline RadiusTest make_radius_test(double r) {
    RadiusTest t;
    t.r2 = r * r;
    t.lo2 = static_cast<float>(t.r2 * (1.0 - 4e-6));
    t.hi2 = static_cast<float>(t.r2 * (1.0 + 4e-6));
    return t;
}

// Per-cloud constants (uploaded once per batch).
struct CloudDev {
    const float* raw;  // raw SoA 3 x n_raw (row stride n_raw); unused by the single-cloud stages
    int32_t n_raw;
    int32_t raw_off;   // first raw index of the cloud in the batch
    int32_t tau_num;
    int32_t H;
    double voxel;
    double inv_cell;   // 1 / (r_FPFH * (1 + 1e-4)): cell edge of the search grid
    double tau_lin;
    double vp[3];
    RadiusTest rf, rn;
    int32_t tau_j;     // |M[q]| needed for J (tau_num; 1 in the classic mode, where J = B)
    int32_t mode;      // KMG_MODE_*
};

// Per-cloud values produced on the device.
struct CloudState {
    int32_t kept_off, kept_cnt;  // range in the kept space
    int32_t j_off, j_cnt;        // range in the J list
};

// A descriptor set for matching: rows desc[rows[i]] (or desc[i]), i < *n.
struct MatchSet {
    const float* desc;
    const int32_t* rows;  // nullable
    const int32_t* n;     // device count
    int32_t row_base;     // subtracted from rows[i] in the output
    int32_t flags;        // kSetRowsOnly: rows for the partner only, no queries
};
constexpr int32_t kSetRowsOnly = 1;

// Per-set plan written by the device planner.
struct SetPlan {
    int32_t n;          // rows
    int32_t q_off;      // first query slot in the flattened query space
    int32_t chunk_off;  // first packed 16-row chunk
    int32_t chunks;
    int32_t tile_off;   // first tile of this set as the query side (norm bands: first sorted tile)
    int32_t cblocks;    // 256-query column blocks
    int32_t segs;       // segments of the partner's rows
    int32_t n_fb;       // queries of this set re-scanned exactly
    int64_t part_off;   // first partial entry
    unsigned long long max_norm_bits;  // max squared norm (FP64 bits, non-negative)
    int32_t wave_off;   // norm-band matching: first query wave of the set
    int32_t rank_off;   // norm-band matching: first tile pair of the set's cross ranking
    int32_t n_img;      // one-sided form: rows of this set listed for the matching back
};

// Matching output of one pair (device buffers).
struct PairOutDev {
    int32_t* pairs;
    float* d1;
    float* d2;
    int64_t cap;
};

// Device status block carved at the start of every workspace.
struct DevStatus {
    int32_t err_range;        // a key left the packable range, or a list exceeds kMaxDegree
    int32_t dense;            // bit 0: some |N(q)| > kListSmall; bit 1: some |N(q)| > kMaxDegree
    int32_t err_capacity;     // a capacity bound was exceeded (CSR or partials)
    int32_t n_long;           // list-first search: lists longer than a pad row
    int64_t n_raw;            // raw points in the batch
    int64_t m_kept;           // kept points
    int64_t nnz;              // neighbour entries
    int64_t n_j;              // J rows
    int64_t n_cells;
    uint32_t amb_linearity;   // |p_lin - tau_lin| < 1e-12 (FP64)
    uint32_t amb_orientation; // |n . (vp - a_q)| tiny (FP64)
    uint32_t feat_fp64;       // pair features recomputed in FP64
    uint32_t feat_edge;       // FP64 features within 1e-9 of a bin edge
    uint32_t n_fallback;      // queries re-scanned exactly
    int32_t total_tiles;      // matching tiles
    uint32_t tile_next;       // persistent tile queue
    int32_t total_queries;
    int64_t total_chunks;
    int64_t pairs_total;      // correspondences over the batch
    int32_t total_waves;      // norm-band matching: query waves
    int32_t band_step;        // norm-band matching: chunks per tile
    int32_t rank_items;       // norm-band matching: tile pairs of the cross ranking
    int32_t sort_items;       // norm-band matching: sorted tiles
    int64_t band_pairs;       // norm-band matching: query-row products evaluated by the tiles
    int32_t err_sync;         // a bounded wait inside a persistent kernel gave up (never expected)
    int32_t pad1;
};

// Linear workspace allocator; with base == nullptr it only measures.
struct Carver {
    char* base;
    size_t cap;
    size_t off = 0;
    Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    bool fits() const { return off <= cap; }
};

#define KMG_TRY_HIP(expr)                                   \
    do {                                                    \
        hipError_t kmg_e_ = (expr);                         \
        if (kmg_e_ != hipSuccess) return KMG_ERR_DEVICE;    \
    } while (0)

#define KMG_TRY(expr)                                       \
    do {                                                    \
        kmg_status kmg_s_ = (expr);                         \
        if (kmg_s_ != KMG_OK) return kmg_s_;                \
    } while (0)

inline kmg_status launch_status() {
    return hipGetLastError() == hipSuccess ? KMG_OK : KMG_ERR_DEVICE;
}

inline uint32_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return static_cast<uint32_t>(p);
}

inline unsigned grid_for(int64_t n, int block) { return static_cast<unsigned>((n + block - 1) / block); }
inline unsigned grid_cap(int64_t n, int block) {
    const int64_t g = (n + block - 1) / block;
    return static_cast<unsigned>(g < 1 ? 1 : (g > kPersistBlocks ? kPersistBlocks : g));
}

CloudDev make_cloud(const kmg_params& p, const float* raw, int64_t n_raw, int64_t raw_off);

// ---- timing.hip -----------------------------------------------------------
enum Stage {
    ST_VOXELIZE = 0,
    ST_GRID,
    ST_SEARCH_COUNT,
    ST_SEARCH_FILL,
    ST_NORMALS,
    ST_SPFH,
    ST_FPFH,
    ST_J_COMPACT,
    ST_MATCH_PACK,
    ST_MATCH_TOPK,
    ST_MATCH_RESCORE,
    ST_MATCH_MUTUAL,
    ST_MATCH_IMAGE,
    kStageCount
};
void timer_begin(int stage, hipStream_t s);
void timer_end(int stage, hipStream_t s);
void timer_collect();  // call after the stream has been synchronised
int timer_enable(int on);
int timer_read(double* ms, int64_t* launches, int n);
// The open stage's work units live in *dev (a device counter read back by timer_work).
void timer_note_work(const int64_t* dev);
int timer_work(int64_t* work, int n);
const char* stage_name(int stage);

// Brackets the launches of one stage in the current scope.
struct StageScope {
    int stage;
    hipStream_t s;
    StageScope(int st, hipStream_t str) : stage(st), s(str) { timer_begin(stage, s); }
    ~StageScope() { timer_end(stage, s); }
};

// ---- scan.hip -------------------------------------------------------------
constexpr int kScanTile = 2048;  // items per scan block (256 threads x 8)
size_t scan_temp_elems(int64_t n);
// Exclusive prefix sum of n int32 values; the int64 total goes to *total
// (device).  `temp` holds scan_temp_elems(n) int64 values.  With `live`
// (device), values at positions >= *live count as 0 and are not read.  With
// `list`, every position i with in[i] == 1 is also written to list[out[i]]
// (a stream compaction of 0/1 flags, in position order).  Two launches.
kmg_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int64_t* total, int64_t* temp,
                          hipStream_t s, const int32_t* live = nullptr, int32_t* list = nullptr);
// The second launch alone, for producers that wrote the tile sums themselves:
// temp[b] = the sum of in[b kScanTile .. (b + 1) kScanTile) for every tile b.
kmg_status scan_exclusive_summed(const int32_t* in, int32_t* out, int64_t n, int64_t* total, int64_t* temp,
                                 hipStream_t s);
// One launch: each block publishes its tile's sum in status[tile] and adds up
// those of the tiles before it (decoupled look-back).  status holds
// scan_temp_elems(n) words, all zero at the launch (the scan leaves them
// nonzero); a wait that gives up (never expected) sets *err.  Beyond
// kOnePassMaxTiles tiles the two-launch form runs instead (the words as its
// temp).
constexpr int64_t kOnePassMaxTiles = 512;
kmg_status scan_exclusive_onepass(const int32_t* in, int32_t* out, int64_t n, int64_t* total, uint64_t* status,
                                  int32_t* err, hipStream_t s, const int32_t* live = nullptr,
                                  int32_t* list = nullptr);
kmg_status fill_u8(uint8_t* p, uint8_t v, size_t n, hipStream_t s);
// Up to kMaxFillJobs fills (4- or 8-byte elements) done by one grid-stride pass.
struct FillJob {
    void* p;
    uint64_t v;
    int64_t n;
    int32_t bytes;
};
constexpr int kMaxFillJobs = 10;
struct FillJobs {
    FillJob job[kMaxFillJobs];
    int32_t n_jobs;
};
__device__ __forceinline__ void run_fill_jobs(const FillJobs& f) {
    const int64_t gs = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int k = 0; k < f.n_jobs; ++k) {
        const FillJob j = f.job[k];
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < j.n; i += gs) {
            if (j.bytes == 8) static_cast<uint64_t*>(j.p)[i] = j.v;
            else static_cast<uint32_t*>(j.p)[i] = static_cast<uint32_t>(j.v);
        }
    }
}
kmg_status fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
kmg_status fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);

// ---- voxel.hip ------------------------------------------------------------
struct VoxelWs {
    uint64_t* keys;
    int32_t* mins;
    int32_t* slot;
    int32_t* flag;
    int32_t* pos;
    int64_t* scan_tmp;
    uint32_t cap_table;
};
VoxelWs carve_voxel(Carver& c, int64_t n_cap);
// Voxelizes every cloud of the table (raw total on the device in st->n_raw,
// at most n_cap).  Kept points go to kept_xyz (SoA, row stride out_stride,
// or the kept count when out_stride == 0), their cloud-local raw index to
// kept_idx and their cloud to kept_cloud (nullable); per-cloud ranges to cs
// (nullable).  Nothing is written when the kept count exceeds out_cap.
// cleared: the caller has already emptied the voxel table (keys, mins).
// The cell hash of the radius search, filled by voxelize_batch as it emits the
// kept points (the tables cleared beforehand); keys == nullptr: not filled.
struct GridInsert {
    uint64_t* keys = nullptr;
    int32_t* cnt = nullptr;
    uint32_t mask = 0;
    int32_t* pslot = nullptr;
    DevStatus* st = nullptr;
};
// scan_status (optional): scan_temp_elems(n_cap) zeroed look-back words, for
// numbering the kept points in one launch.
kmg_status voxelize_batch(const CloudDev* cl, int n_clouds, int64_t n_cap, DevStatus* st, const VoxelWs& w,
                          int64_t out_cap, int64_t out_stride, int32_t* kept_idx, float* kept_xyz,
                          int32_t* kept_cloud, CloudState* cs, hipStream_t s, bool cleared = false,
                          const GridInsert* grid = nullptr, uint64_t* scan_status = nullptr);

// ---- search.hip -----------------------------------------------------------
// The neighbour lists as the feature passes read them: the CSR lists, or
// (pad != nullptr) the pad rows of the list-first search (pad_cap entries)
// with the lists longer than a row at their CSR places.
struct NbrLists {
    const int32_t* nbr = nullptr;
    const int32_t* pad = nullptr;
    int64_t pad_cap = 0;
};

struct SearchWs {
    uint64_t* keys;
    int32_t* ccount;
    int32_t* cstart;
    int32_t* cfill;
    int32_t* pslot;
    float4* pts;
    int32_t* deg;
    int64_t* scan_tmp;
    uint32_t cap_table;
};
SearchWs carve_search(Carver& c, int64_t m_cap);
// Grid build and the count pass over the kept points (count st->m_kept <=
// m_cap, SoA stride `stride`, cloud ids kept_cloud (nullable = cloud 0)).
// off receives m_cap + 1 offsets; the total goes to st->nnz.
// use_rn: search at r_normal instead of r_FPFH; build_grid false reuses the
// cell grid of an earlier call on the same workspace.  cleared: the caller
// has already emptied the cell table (keys, ccount, cfill) and zeroed deg.
kmg_status search_count_batch(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                              int64_t m_cap, DevStatus* st, const SearchWs& w, int32_t* off, hipStream_t s,
                              bool build_grid = true, int use_rn = 0, bool cleared = false, bool inserted = false);
// Fill pass (lists ascending) and normals.  Writes nothing into nbr when
// st->nnz > nbr_cap (device-side check; st->err_capacity is set).
kmg_status search_fill_batch(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                             int64_t m_cap, int64_t nbr_cap, bool dense_pass, DevStatus* st, const SearchWs& w,
                             const int32_t* off, int32_t* nbr, float* nrm, int64_t nrm_stride, uint8_t* flags,
                             int32_t* n_normal, hipStream_t s, int use_rn = 0, bool with_normals = true);
// The list-first form of the grid build, search and normals (r_FPFH lists,
// tables cleared beforehand): one search pass writes |N(q)| and each list
// that fits a row of the pad (pad_cap entries shared evenly by the kept
// points), the offsets follow from the degrees, the dense pass serves the
// longer lists (listed in long_q, m_cap entries) into their CSR places in
// nbr, and the normals pass reads the lists where they are (NbrLists).
// inserted: the cell hash is filled already (voxelize_batch).  scan_status
// (optional): zeroed look-back words for the two scans (cell counts, then
// degrees), search_scan_status_elems(w, m_cap) of them.
kmg_status search_lists_first(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                              int64_t m_cap, int64_t nbr_cap, DevStatus* st, const SearchWs& w, int32_t* off,
                              int32_t* nbr, int32_t* pad, int64_t pad_cap, int32_t* long_q, float* nrm,
                              int64_t nrm_stride, uint8_t* flags, hipStream_t s, bool inserted = false,
                              uint64_t* scan_status = nullptr);
size_t search_scan_status_elems(const SearchWs& w, int64_t m_cap);

// ---- features.hip ---------------------------------------------------------
// Row stride of the SPFH counts, in entries: 3H rounded up to a multiple of 8,
// so that every row starts on a 16-byte boundary and is read with 16-byte loads.
__host__ __device__ constexpr int spfh_row(int H) { return (3 * H + 7) & ~7; }

struct FeatWs {
    uint16_t* cnt16;  // SPFH bin counts (Eq. A4 numerators), m rows of spfh_row(H) (3H used)
    double* inv100;   // 100 / P_q (0 when P_q = 0)
    uint32_t* queue;  // work queue of the fused SPFH / FPFH launch
    int32_t* ready;   // per cloud: points whose SPFH is written (fused launch)
    int32_t* Pq;
    int32_t* jflag;
    int32_t* pos;
    int64_t* scan_tmp;
};
FeatWs carve_feat(Carver& c, int64_t m_cap, int H);
// Step 2, SPFH, FPFH and the J list over the kept points (count st->m_kept).
// j_idx receives the kept indices of the J points (in the batch's global kept
// space); cs, when given, receives the per-cloud J ranges, and sets (with cs)
// each cloud's matching set.  cleared: jflag is zero already.
kmg_status features_batch(const CloudDev* cl, int n_clouds, const float* xyz, int64_t stride,
                          const int32_t* kept_cloud, int64_t m_cap, int H, DevStatus* st, const FeatWs& w,
                          const int32_t* off, NbrLists nb, const float* nrm, int64_t nrm_stride,
                          uint8_t* flags, float* spfh_out, float* fpfh_out, int32_t* j_idx, CloudState* cs,
                          hipStream_t s, bool cleared = false, MatchSet* sets = nullptr,
                          uint64_t* j_scan_status = nullptr);
// The two halves of features_batch: SPFH (and J) over (off, nb); then the
// FPFH sum over (off, nb) and the J list.
kmg_status spfh_batch(const CloudDev* cl, const float* xyz, int64_t stride, const int32_t* kept_cloud,
                      int64_t m_cap, int H, DevStatus* st, const FeatWs& w, const int32_t* off, NbrLists nb,
                      const float* nrm, int64_t nrm_stride, uint8_t* flags, float* spfh_out, hipStream_t s,
                      bool cleared = false);
kmg_status fpfh_batch(int n_clouds, const float* xyz, int64_t stride, int64_t m_cap, int H, DevStatus* st,
                      const FeatWs& w, const int32_t* off, NbrLists nb, uint8_t* flags, float* fpfh_out,
                      int32_t* j_idx, CloudState* cs, hipStream_t s, MatchSet* sets = nullptr,
                      uint64_t* j_scan_status = nullptr);

// ---- match.hip ------------------------------------------------------------
constexpr int kLpMaxDim = 64;  // descriptor length of the FP16 / BF16 tiles (two K = 32 steps)
// Per pair of the reduced-precision form: the centre of both sets' rows and a
// power-of-two scale (max |x - mu| * scale <= 2^14).
struct PairLp {
    double mu[kLpMaxDim];
    double scale;
    double inv_s2;
    unsigned long long maxabs_bits;  // max |x - mu| over both sets (FP64 bits)
};
// Re-run of the queries the reduced-precision certificate left open: their
// own sets (query rows listed through f_row) against the full partner sets
// (rows only), through the FP64 form with its own status block and its own
// workspace region (carved on the host when used).
struct RerunWs {
    DevStatus* st;
    MatchSet* sets;      // 2 per main set
    int32_t* f_slot;     // main query slot of each listed query
    int32_t* f_row;      // its descriptor row
    int32_t* f_count;    // listed queries per main set
    int64_t* f_total;
    char* region;        // nullptr when not carved
    size_t region_bytes;
};
struct MatchWs {
    SetPlan* plan;
    double* pk;           // packed rows
    double* n2;           // exact squared norms per query slot
    double* part;         // per-segment top-4 lists of encoded scores
    double* lp_nx;        // reduced-precision form: ||x - mu|| per query slot
    PairLp* lp_pairs;     // reduced-precision form: per pair centre and scale
    RerunWs rr;           // FP64 re-runs: uncertified queries, the one-sided form's matching back
    MatchSet* one_sided;  // the sets of the one-sided form's first direction (null: both in full)
    int32_t* rank;        // norm-band matching: packed position of every query slot in its set
    int32_t* perm;        // norm-band matching: local row of every packed position
    double* r2;           // norm-band matching: seed bound R^2 per query slot
    uint32_t* skey;       // norm-band matching: sort key of every packed partner position
    int32_t* wave_c0;     // norm-band matching: first partner chunk of every query wave's band
    int32_t* wave_len;    // norm-band matching: chunks in the band
    int2* wave_sub;       // norm-band matching: chunk range of each 16-query tile of every wave
    int32_t* chist;       // norm-band matching, both directions: class histogram of every query sort tile
    int32_t* wave_tile;   // norm-band matching: first tile of every wave (wave_cap + 1 entries)
    int4* tinfo;          // norm-band matching: per tile {wave, set, first chunk, end chunk}
    int64_t wave_cap;
    int64_t tile_cap;
    int32_t* nn;
    double* best;
    double* second;
    int32_t* fb_list;     // queries left to the exact scan (slot order, or any order from the band re-score)
    int64_t* fb_total;
    int32_t* grp_done;    // exact scan: finished segments per 64-entry group (the planners zero them)
    int64_t n_grp;
    int32_t* flag;
    int32_t* pos;
    int64_t* scan_tmp;
    int64_t q_cap;        // total query slots
    int64_t chunk_cap;    // packed chunks
    int64_t part_cap;     // partial entries
    int kp;
};
MatchWs carve_match(Carver& c, int n_sets, int64_t q_cap, int dim, bool rerun = true);
// Matches sets 2i and 2i+1 for every pair i (both directions, mutual check).
// counts[i * counts_stride + 0] receives the number of correspondences of
// pair i and [.. + 5] the number of exact re-scans of its queries.
// With cs (the batch form), counts also receive per pair the kept points and
// |J| of both clouds (from cs), the neighbour entries and the pair's status
// (nnz_cap: the neighbour-list capacity the status is judged against).
kmg_status match_batch(const MatchSet* sets, int n_sets, int dim, int prec, DevStatus* st, const MatchWs& w,
                       const PairOutDev* outs, int64_t* counts, int counts_stride, hipStream_t s,
                       const CloudState* cs = nullptr, int64_t nnz_cap = 0);

// ---- graph.hip: ratio filter, Eq. (3) graph, max k-core ----------------------
size_t graph_ws(int64_t n_corr, int32_t n_tau);
size_t kcore_ws(int32_t n);
kmg_status corr_graph(const float* src, int64_t src_stride, const float* tgt, int64_t tgt_stride,
                      const int32_t* pairs, const float* d1, const float* d2, int64_t n_corr, int32_t n_tau,
                      double beta, int32_t* sel, int32_t* off, int32_t* adj, int64_t adj_cap, int32_t* n_sel_host,
                      int64_t* nnz_host, void* ws, size_t ws_bytes, hipStream_t s);
kmg_status max_kcore(const int32_t* off, const int32_t* adj, int32_t n, int32_t* core, int32_t* members,
                     int32_t* n_members_host, int32_t* max_core_host, void* ws, size_t ws_bytes, hipStream_t s);

// ---- stages.hip: single-cloud entry points --------------------------------
size_t voxelize_ws(int64_t n);
kmg_status voxelize(const float* xyz, int64_t n, double voxel, int32_t* kept_idx, float* kept_xyz, int64_t cap,
                    int64_t* n_kept_host, void* ws, size_t ws_bytes, hipStream_t s);
size_t normals_ws(int64_t m, int mode = 0, int64_t nbr_cap = 0);
kmg_status normals(const float* xyz, int64_t m, const kmg_params& p, float* nrm, uint8_t* flags, int32_t* off,
                   int32_t* nbr, int64_t nbr_cap, int64_t* nnz_host, int32_t* n_normal, void* ws, size_t ws_bytes,
                   hipStream_t s);
size_t fpfh_ws(int64_t m, int H, int mode = 0, int64_t nnz = 0);
kmg_status fpfh(const float* xyz, const float* nrm, uint8_t* flags, const int32_t* off, const int32_t* nbr,
                int64_t m, const kmg_params& p, float* spfh_out, float* fpfh_out, int32_t* j_idx, int64_t* n_j_host,
                int64_t* stats_host, void* ws, size_t ws_bytes, hipStream_t s);
size_t match_ws(int64_t np, int64_t nq, int dim);
kmg_status match(const float* dp, const int32_t* rp, int64_t np, const float* dq, const int32_t* rq, int64_t nq,
                 int dim, int prec, int32_t* pairs, float* d1, float* d2, int64_t cap, int64_t* n_pairs_host,
                 int64_t* n_fallback_host, void* ws, size_t ws_bytes, hipStream_t s);

// ---- tuning.hip -----------------------------------------------------------
// Launch shapes that change how work is scheduled, never what is computed or in
// which order floating-point terms are summed (every choice gives bit-identical
// outputs); set process-wide by kmg_set_tuning, read at launch time.
struct Tuning {
    int search_waves = 4;     // waves per block of the radius count and fill passes (2, 4, 8)
    int count_queries = 2;    // queries per wavefront in the count pass (1, 2, 4)
    int spfh_pair_mean = 24;  // mean list length up to which SPFH takes two points per wavefront
    int fpfh_rows = 2;        // SPFH rows per unrolled step of the FPFH sum (1, 2, 4, 8, 16)
    int band_tile = 0;        // partner chunks per band tile; 0 = the tile-length model's choice
    int fuse_features = 0;    // 1: SPFH and FPFH in one persistent launch (per-cloud readiness counters)
    int xcd_split = 2;        // bit 0 SPFH, bit 1 FPFH: XCD-aware split of the points over the wavefronts
    int match_form = 0;       // 0: one-sided matching then the image back; 1: both directions in one pass
    int search_form = 1;      // batches: 0 count pass then fill pass; 1 list-first (one search pass, a pad)
};
const Tuning& tuning();
bool set_tuning(const Tuning& t);
bool band_tile_candidate(int T);  // T is one of the band planner's candidate lengths

// ---- batch.hip ------------------------------------------------------------
size_t batch_ws(int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H);
kmg_status batch_upload(const kmg_cloud* clouds, const kmg_match_out* outs, int n_pairs, int64_t raw_cap,
                        int64_t nnz_cap, int H, void* ws, size_t ws_bytes, hipStream_t s);
kmg_status batch_run(int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H, int prec, int64_t* counts, void* ws,
                     size_t ws_bytes, hipStream_t s);
kmg_status batch_export_cloud(int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H, int cloud, float* fpfh_out,
                              int64_t cap_rows, int32_t* j_out, int64_t cap_j, void* ws, size_t ws_bytes,
                              hipStream_t s);

}  // namespace kmg
