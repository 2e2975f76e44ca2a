// Internal declarations shared by the libkmg translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kmg.h"

namespace kmg {

constexpr int kWave = 64;
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int64_t kKeyBias = int64_t(1) << 20;  // packed keys hold [-2^20, 2^20) per axis
constexpr int kMaxDegree = 8192;                 // largest |N(q)| the sorted-list kernels accept
constexpr int kMaxBins = 32;                     // largest H (3H <= 96 descriptor values)
constexpr int kTopK = 4;                         // candidates kept per row before exact re-scoring

// Device status block carved at the start of every workspace.
struct DevStatus {
    int32_t err_range;   // a key left the packable range
    int32_t dense;       // some |N(q)| exceeds the common LDS list (bit 0) or the largest one (bit 1)
    int32_t total_a;     // scan totals
    int32_t total_b;
    uint32_t amb_linearity;   // |p_lin - tau_lin| < 1e-12 (FP64)
    uint32_t amb_orientation; // |n . (vp - a_q)| tiny (FP64)
    uint32_t feat_fp64;       // pair features recomputed in FP64
    uint32_t feat_edge;       // FP64 features within 1e-9 of a bin edge
    uint32_t n_fallback;      // matching columns re-scanned exactly
    uint32_t pad[7];
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
    kStageCount
};
void timer_begin(int stage, hipStream_t s);
void timer_end(int stage, hipStream_t s);
void timer_collect();  // call after the stream has been synchronised
int timer_enable(int on);
int timer_read(double* ms, int64_t* launches, int n);
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
// (device).  `temp` holds scan_temp_elems(n) int64 values.
kmg_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int64_t* total, int64_t* temp,
                          hipStream_t s);
kmg_status fill_u8(uint8_t* p, uint8_t v, size_t n, hipStream_t s);
kmg_status fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
kmg_status fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);

// ---- voxel.hip ------------------------------------------------------------
size_t voxelize_ws(int64_t n);
kmg_status voxelize(const float* xyz, int64_t n, double voxel, int32_t* kept_idx, float* kept_xyz, int64_t cap,
                    int64_t* n_kept_host, void* ws, size_t ws_bytes, hipStream_t s);

// ---- search.hip -----------------------------------------------------------
size_t normals_ws(int64_t m);
kmg_status normals(const float* xyz, int64_t m, const kmg_params& p, float* nrm, uint8_t* flags, int32_t* off,
                   int32_t* nbr, int64_t nbr_cap, int64_t* nnz_host, int32_t* n_normal, void* ws, size_t ws_bytes,
                   hipStream_t s);

// ---- features.hip ---------------------------------------------------------
size_t fpfh_ws(int64_t m, int H);
kmg_status fpfh(const float* xyz, const float* nrm, uint8_t* flags, const int32_t* off, const int32_t* nbr,
                int64_t m, const kmg_params& p, float* spfh_out, float* fpfh_out, int32_t* j_idx, int64_t* n_j_host,
                int64_t* stats_host, void* ws, size_t ws_bytes, hipStream_t s);

// ---- match.hip ------------------------------------------------------------
size_t match_ws(int64_t np, int64_t nq, int dim);
kmg_status match(const float* dp, const int32_t* rp, int64_t np, const float* dq, const int32_t* rq, int64_t nq,
                 int dim, int prec, int32_t* pairs, float* d1, float* d2, int64_t cap, int64_t* n_pairs_host,
                 int64_t* n_fallback_host, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace kmg
