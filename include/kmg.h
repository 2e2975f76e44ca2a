/*
 * kmg.h -- C ABI of libkmg: the data-parallel hot path of KISS-Matcher
 * (arXiv 2409.15615) on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem: two voxelized
 * clouds (Section III-A) are turned into Faster-PFH descriptors (Section
 * III-C, Appendix A: Algorithm 1 and Eq. A1-A5) and matched by the mutual
 * nearest-neighbour (reciprocity) test of Section III-C.  Pruning (Eq. 3,
 * k-core) and the pose solver are not part of this library.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller, unless a
 *    parameter is documented as a host pointer.  The library never allocates
 *    device memory: scratch space comes from the caller's workspace `ws` of
 *    `ws_bytes` bytes, sized by kmg_workspace_bytes().  `ws` must be
 *    256-byte aligned.  (kmg_normals_static takes no workspace: its scratch
 *    is a fixed array inside the library.)
 *  - Point clouds are float32 structure-of-arrays: x[0..n), y[0..n),
 *    z[0..n) stored back to back (3*n floats, row stride n).
 *  - Descriptors are row-major float32, 3*H values per point (H = n_bins).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; calls that return a count through a host
 *    pointer synchronise that stream before returning.
 *  - Indices are int32 and refer to the kept (voxelized) cloud, except
 *    kept_idx, which maps kept points back to raw input indices.
 *  - Errors are returned as kmg_status; no call aborts or throws.  On
 *    KMG_ERR_CAPACITY the required size is written to the count pointer and
 *    the other outputs are unspecified.
 *  - Determinism: identical inputs give bit-identical integer outputs and
 *    bit-identical floating-point outputs on every call.
 */
#ifndef KMG_H
#define KMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KMG_OK = 0,
    KMG_ERR_ARG = -1,      /* invalid argument (null pointer, bad size or parameter) */
    KMG_ERR_CAPACITY = -2, /* an output buffer is too small; required size reported */
    KMG_ERR_DEVICE = -3,   /* a HIP runtime call or kernel launch failed */
    KMG_ERR_RANGE = -4,    /* input outside the supported range (see each call) */
    KMG_ERR_WORKSPACE = -5 /* ws_bytes smaller than kmg_workspace_bytes() */
} kmg_status;

typedef enum { KMG_FP32 = 0, KMG_BF16 = 1, KMG_FP16 = 2 } kmg_precision;

/* Faster-PFH parameters.  Section IV-B states them in units of the voxel
 * size v: r_normal = 3.5 v, r_FPFH = 5 v, tau_num = 3, tau_lin = 0.99.
 * Requirements: voxel > 0; 0 < r_normal <= r_fpfh (Section III-C relies on
 * r_normal <= r_FPFH to subsample the normal neighbourhood from the single
 * r_FPFH search); tau_num >= 1; 0 < tau_lin <= 1; 1 <= n_bins <= 32.
 * viewpoint: the normals are oriented so that n . (viewpoint - a_q) >= 0. */
typedef struct {
    double voxel;
    double r_normal;
    double r_fpfh;
    double tau_lin;
    int32_t tau_num;
    int32_t n_bins;
    double viewpoint[3];
    int32_t mode;      /* KMG_MODE_FASTER_PFH (default) or KMG_MODE_CLASSIC_FPFH */
    int32_t reserved;  /* must be 0 */
} kmg_params;

/*
 * Descriptor pipelines (kmg_params.mode).
 *   KMG_MODE_FASTER_PFH: Faster-PFH (Section III-C, Algorithm 1): one radius
 *     search at r_FPFH serves both the normals (its r_normal subset) and the
 *     features; the tau_num and tau_lin filters decide B and J.
 *   KMG_MODE_CLASSIC_FPFH: the FPFH of Rusu et al. as Section III-C describes
 *     it (Fig. 3a): normals from their own radius search at r_normal (any
 *     point with >= 3 neighbours there, q included, gets a normal; no
 *     linearity filter), angular features and SPFH over a second search at
 *     r_FPFH, and the FPFH sum over a third search at r_FPFH; every point with
 *     a normal gets a descriptor.  tau_num and tau_lin are ignored.  The
 *     per-stage entry points only; the batch form runs Faster-PFH.
 */
#define KMG_MODE_FASTER_PFH 0
#define KMG_MODE_CLASSIC_FPFH 1

/* Operation codes for kmg_workspace_bytes(). */
enum {
    KMG_OP_VOXELIZE = 0, /* n0 = raw points */
    KMG_OP_NORMALS = 1,  /* n0 = kept points m; classic mode: n1 = neighbour capacity of the r_normal search */
    KMG_OP_FPFH = 2,     /* n0 = kept points m; classic mode: n1 = neighbour entries of the r_FPFH lists */
    KMG_OP_MATCH = 3,    /* n0 = rows of P (np), n1 = rows of Q (nq) */
    KMG_OP_GRAPH = 4,    /* n0 = correspondences, n1 = N_tau */
    KMG_OP_KCORE = 5     /* n0 = graph vertices */
};

/* Largest graph kmg_max_kcore accepts (its state lives in on-chip memory,
 * 8 bytes per vertex: 128 KiB of the CU's 160 KiB LDS at the limit). */
#define KMG_MAX_KCORE_VERTICES 16384

/* Workspace size in bytes needed by `op` for the given sizes (a host call;
 * touches no device).  For KMG_OP_MATCH the descriptor length is
 * 3 * p->n_bins (33 when p is NULL); a workspace sized for a longer
 * descriptor also serves a shorter one.  Returns 0 for an unknown op or
 * invalid sizes. */
size_t kmg_workspace_bytes(int32_t op, int64_t n0, int64_t n1, const kmg_params* p);

/* Human-readable name of a status code (static storage). */
const char* kmg_status_string(int32_t status);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t kmg_version(void);

/*
 * Diagnostics: per-stage device time.  kmg_timing_enable(1) resets the
 * totals and makes every later call bracket its kernel launches with HIP
 * events on its stream; the elapsed times are added to process-wide
 * per-stage totals when the call completes (each call then also waits for
 * its stream).  Not thread-safe: for single-threaded profiling runs.
 * kmg_timing_enable(0) stops timing.  Returns 0, or -1 if events could not
 * be created.  kmg_timing_read copies up to n stage totals (milliseconds and
 * number of bracketed launches; match_topk is the candidate tile launch of
 * the first matching direction, match_image the whole matching back) and
 * returns the number of stages; kmg_stage_name(i) names stage i (static
 * storage).  kmg_timing_work copies up to n per-stage work counts of the
 * stage's last timed launch (for match_topk and match_image with the norm
 * bands: query-row products the tiles evaluated, each 16-query tile over its
 * own chunk range; 0 where a stage counts
 * none, -1 if the count could not be read) and returns the number of stages;
 * it reads device memory of the last call's workspace, which must still be
 * allocated.
 */
int32_t kmg_timing_enable(int32_t on);
int32_t kmg_timing_read(double* ms, int64_t* launches, int32_t n);
int32_t kmg_timing_work(int64_t* work, int32_t n);
const char* kmg_stage_name(int32_t stage);

/*
 * Launch tuning.  Work-distribution choices of the hot-path kernels, picked
 * per workload by the autotuner in paper_2409_15615_amd/tune.py (every value
 * gives bit-identical outputs: they change how work is scheduled, never what
 * is computed or the order of any floating-point sum).  Process-wide; read
 * when a call enqueues its kernels, so a captured hipGraph keeps the shapes
 * in force at capture time.  Not synchronised with concurrent calls.
 *   search_waves    waves per block of the radius count and fill passes
 *                   (Eq. A1): 2, 4 (default) or 8.
 *   count_queries   queries per wavefront in the count pass (the per-stage
 *                   calls, and batches under search_form 0): 1, 2 (default)
 *                   or 4.
 *   spfh_pair_mean  mean neighbour-list length up to which the SPFH pass
 *                   (Eq. A2-A4) takes two points per wavefront (default 24;
 *                   0 = never, 8192 = always).
 *   fpfh_rows       SPFH rows per unrolled step of the FPFH sum (Eq. A5):
 *                   rows read from LDS per step where two J points share a
 *                   wavefront (3H <= 64), rows in flight per lane otherwise;
 *                   1, 2 (default), 4, 8 or 16.
 *   band_tile       partner chunks per distance tile of matching (a length
 *                   of the planner's candidate set: 1..64, then four per
 *                   octave up to 4096), used whenever its tiles fit; 0
 *                   (default) = the planner's modelled choice.
 *   fuse_features   1: SPFH and FPFH (Eq. A2-A5) in one persistent launch
 *                   that takes work items from a queue, the FPFH of a cloud
 *                   starting once every SPFH of that cloud is written
 *                   (per-cloud readiness counters); 0 (default): two launches.
 *   xcd_split       bit 0 (SPFH, Eq. A2-A4) and bit 1 (FPFH, Eq. A5): deal
 *                   the points to wavefronts XCD-aware (each of the eight
 *                   XCDs takes one contiguous eighth of the points, balanced
 *                   by neighbour-list volume, so that its L2 holds that
 *                   eighth's neighbourhood) rather than in turn; 0..3,
 *                   default 2 (measured: the FPFH gather reads its
 *                   neighbours' rows and gains, the SPFH pass loses).
 *   match_form      FP64 matching (Section III-C reciprocity test) of a batch
 *                   that fits the one-sided form: 0 (default) matches the
 *                   smaller set of each pair against the larger, then only
 *                   the rows that are some query's nearest neighbour back;
 *                   1 matches both directions in full in one band pass (more
 *                   distance tiles, fewer launches).  The same
 *                   correspondences, d1 and d2 either way.
 *   search_form     radius search (Eq. A1) of a batch (kmg_batch_run):
 *                   0 a count pass, the offsets, then the fill pass;
 *                   1 (default) one search pass that writes |N(q)| and each list
 *                   into a row of a pad in the workspace (64 entries per raw
 *                   point, shared evenly by the kept points) and the
 *                   offsets, the longer lists searched again into their
 *                   CSR places; the normal and feature passes read each
 *                   list where it is.  The same lists either way.
 * kmg_set_tuning(NULL) restores the defaults; unsupported values give
 * KMG_ERR_ARG and leave the tuning unchanged.
 */
typedef struct {
    int32_t search_waves;
    int32_t count_queries;
    int32_t spfh_pair_mean;
    int32_t fpfh_rows;
    int32_t band_tile;
    int32_t fuse_features;
    int32_t xcd_split;
    int32_t match_form;
    int32_t search_form;
} kmg_tuning;
kmg_status kmg_set_tuning(const kmg_tuning* t);
kmg_status kmg_get_tuning(kmg_tuning* t);

/*
 * kmg_voxelize -- voxel downsampling of a raw cloud (Section III-A: the
 * method takes clouds voxelized with voxel size v).
 *
 * Every finite point i gets the key (floor(x_i / v), floor(y_i / v),
 * floor(z_i / v)), evaluated in FP64.  For each occupied voxel the point of
 * lowest input index is kept; kept points are written in ascending input
 * index.  Non-finite points are dropped.
 *   xyz       [in]  SoA 3 x n float32.
 *   n         [in]  number of raw points (0 <= n < 2^31).
 *   voxel     [in]  voxel size v > 0.
 *   kept_idx  [out] int32[cap]: raw index of each kept point.
 *   kept_xyz  [out] float32[3 * cap]: kept points as a packed SoA 3 x m block
 *                   (row stride m = *n_kept, not cap).
 *   cap       [in]  capacity in points of kept_idx and kept_xyz.
 *   n_kept    [out, HOST] number of kept points m.
 * Errors: KMG_ERR_RANGE if a key does not fit in [-2^17, 2^17) per axis.
 */
kmg_status kmg_voxelize(const float* xyz, int64_t n, double voxel, int32_t* kept_idx, float* kept_xyz,
                        int64_t cap, int64_t* n_kept, void* ws, size_t ws_bytes, void* stream);

/*
 * kmg_normals -- Algorithm 1, Step 1: one radius search per point at
 * r_FPFH (Eq. A1: N(q) = { s : ||a_s - a_q|| < r_FPFH }, the query
 * included), the r_normal subset P_normal(q) taken from it, the
 * cardinality tests |N(q)| >= tau_num and |P_normal(q)| >= tau_num, the
 * PCA normal (unit eigenvector of the smallest covariance eigenvalue of
 * P_normal) and the linearity p_lin = (l1 - l2) / l1 with the test
 * p_lin < tau_lin.
 *   xyz       [in]  SoA 3 x m float32, a voxelized cloud.
 *   normals   [out] SoA 3 x m float32; zero where no normal was estimated.
 *   flags     [out] uint8[m]; bit 0 = B[q] (a reliable normal after Step 1).
 *   nbr_off   [out] int32[m + 1]: CSR offsets of N(q).
 *   nbr_idx   [out] int32[nbr_cap]: N(q) for every q, each list ascending.
 *   nbr_cap   [in]  capacity of nbr_idx.
 *   nnz       [out, HOST] total number of neighbour entries.
 *   n_normal  [out, optional] int32[m]: |P_normal(q)|, or NULL.
 * Distances are decided exactly as the FP64 expression
 * ((dx*dx) + dy*dy) + dz*dz < r*r with dx = (double)x_s - (double)x_q.
 * Errors: KMG_ERR_CAPACITY (nnz > nbr_cap); KMG_ERR_RANGE if some |N(q)|
 * exceeds 8192 or nnz exceeds 2^31 - 1, or a cell key overflows.
 */
kmg_status kmg_normals(const float* xyz, int64_t m, const kmg_params* p, float* normals, uint8_t* flags,
                       int32_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap, int64_t* nnz, int32_t* n_normal,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * kmg_normals_static -- kmg_normals for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid it).  The same computation, arguments and errors as
 * kmg_normals, without the workspace: the scratch is one array of 20 MiB per
 * GPU inside the library, held until the process ends.
 *   m          at most KMG_STATIC_MAX_POINTS (KMG_ERR_RANGE beyond).
 *   p->mode    KMG_MODE_FASTER_PFH only (KMG_ERR_ARG otherwise).
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * device (two streams, two threads) race and must be serialised by the
 * caller.  The call itself allocates nothing; like kmg_normals it
 * synchronises `stream` to return *nnz.
 */
#define KMG_STATIC_MAX_POINTS 262144
kmg_status kmg_normals_static(const float* xyz, int64_t m, const kmg_params* p, float* normals, uint8_t* flags,
                              int32_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap, int64_t* nnz, int32_t* n_normal,
                              void* stream);

/*
 * kmg_fpfh -- Algorithm 1, Step 2 and Eq. A2-A5.
 * M[q] = { k in N(q) : B[k] }; J = { q : B[q] and |M[q]| >= tau_num }.
 * For every q with B[q], SPFH(q) (Eq. A4) histograms the Darboux-frame
 * features (Eq. A2) of the pairs (q, k), k in M[q] \ {q}, into H bins per
 * feature (Eq. A3, bounds [-pi, pi], [-1, 1], [-1, 1]), normalised to 100
 * by P_q = |M[q]| - 1.  For q in J, FPFH(q) = SPFH(q) + (1 / P_q) *
 * sum_{k in M[q] \ {q}} SPFH(k) / ||a_k - a_q|| (Eq. A5).
 *   xyz, normals, nbr_off, nbr_idx [in] as produced by kmg_normals.
 *   flags     [in/out] bit 0 = B (read); bit 1 = q in J (written).
 *   spfh      [out, optional] float32[m * 3H] or NULL; zero rows where not B.
 *   fpfh      [out] float32[m * 3H]; zero rows outside J.
 *   j_idx     [out] int32[m]: the points of J in ascending order.
 *   n_j       [out, HOST] |J|.
 *   stats     [out, optional HOST] int64[2] or NULL: number of pair
 *             features decided in FP64 near a bin edge or a selection tie,
 *             and the number within 1e-9 of a bin edge in FP64.
 */
kmg_status kmg_fpfh(const float* xyz, const float* normals, uint8_t* flags, const int32_t* nbr_off,
                    const int32_t* nbr_idx, int64_t m, const kmg_params* p, float* spfh, float* fpfh,
                    int32_t* j_idx, int64_t* n_j, int64_t* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * kmg_match -- mutual nearest-neighbour matching (the reciprocity test of
 * Section III-C) between descriptor rows of P and Q.
 * Distance D(i, j) = sum_t ((double)x_it - (double)y_jt)^2 in dimension
 * order (squared L2).  NN_Q(i) = argmin_j D(i, j), ties to the smaller j;
 * NN_P(j) likewise.  (i, j) is a correspondence iff NN_Q(i) = j and
 * NN_P(j) = i.  Candidates are found on matrix cores (precision `prec`)
 * and every reported decision is re-scored exactly in FP64; rows whose
 * candidate set cannot be certified are re-scanned exactly.
 *   desc_p    [in]  float32 row-major, rows addressed through rows_p.
 *   rows_p    [in]  int32[np]: row of desc_p for each P entry, or NULL for
 *                   rows 0..np-1.  The same for desc_q / rows_q / nq.
 *   dim       [in]  descriptor length (1 <= dim <= 64).
 *   prec      [in]  KMG_FP32 (KMG_BF16 / KMG_FP16: candidate generation in
 *                   16-bit with FP32 accumulation; same exact result).
 *   pairs     [out] int32[cap * 2]: (rows_p[i], rows_q[j]) sorted by i.
 *   d1, d2    [out] float32[cap]: sqrt of the smallest and second-smallest
 *                   D over row i (d2 = +inf if nq < 2).
 *   n_pairs   [out, HOST] number of correspondences.
 *   n_fallback[out, optional HOST] rows (both directions) re-scanned exactly.
 * Descriptors must be finite and non-negative (FPFH rows are).
 */
kmg_status kmg_match(const float* desc_p, const int32_t* rows_p, int64_t np, const float* desc_q,
                     const int32_t* rows_q, int64_t nq, int32_t dim, int32_t prec, int32_t* pairs, float* d1,
                     float* d2, int64_t cap, int64_t* n_pairs, int64_t* n_fallback, void* ws, size_t ws_bytes,
                     void* stream);

/*
 * Batched registration: the whole hot path (voxelize, radius search and
 * normals, SPFH/FPFH, mutual matching) for many pairs of raw clouds, uneven
 * sizes allowed, each stage one kernel launch over the whole batch.
 *
 * Cloud 2i is the source and cloud 2i+1 the target of pair i.  Every cloud
 * carries its own parameters (n_bins must be equal across the batch) and
 * viewpoint.  Correspondences of pair i are written to outs[i] as
 * (source kept index, target kept index) sorted by the source index, with
 * d1, d2 as in kmg_match; kept indices refer to each cloud voxelized alone
 * (ascending input index), so every result equals the result of running the
 * pair alone through the single-cloud calls.
 *
 * counts [out, DEVICE] int64[8 * n_pairs]: per pair, 0 correspondences,
 * 1 kept source points, 2 kept target points, 3 |J| source, 4 |J| target,
 * 5 queries re-scanned exactly (a work statistic: it depends on the matching
 * form of the launch tuning, the other entries do not), 6 status (a kmg_status; KMG_ERR_WORKSPACE
 * when the batch's neighbour entries exceed nnz_cap, KMG_ERR_CAPACITY when
 * outs[i].cap is too small, KMG_ERR_DEVICE if a bounded wait between the
 * blocks of a kernel gave up, which is never expected), 7 neighbour entries
 * of the whole batch.
 *
 * Capacities: raw_cap >= total raw points of the batch; nnz_cap = neighbour
 * entries reserved for the batch; at most 511 pairs.  The batch matches the
 * descriptors, so 3 * n_bins <= 64 (n_bins <= 21; KMG_ERR_ARG beyond, and a
 * zero workspace size).
 *
 * kmg_batch_upload copies the cloud and output tables into the workspace
 * (host call; returns after the copy).  kmg_batch_run enqueues the batch on
 * `stream` without any host synchronisation, memset or host copy, so a
 * caller may capture it in a hipGraph and replay it after uploading a new
 * batch with the same n_pairs, raw_cap, nnz_cap and n_bins.
 * kmg_register_batch = upload + run.  Results are valid once the stream has
 * completed.
 */
typedef struct {
    const float* xyz;  /* device SoA 3 x n raw points (row stride n) */
    int64_t n;
    kmg_params params;
} kmg_cloud;

typedef struct {
    int32_t* pairs; /* device int32[cap * 2] */
    float* d1;      /* device float32[cap] */
    float* d2;      /* device float32[cap] */
    int64_t cap;
} kmg_match_out;

size_t kmg_batch_workspace_bytes(int32_t n_pairs, int64_t raw_cap, int64_t nnz_cap, int32_t n_bins);

/*
 * kmg_batch_descriptors -- after a kmg_batch_run (on `stream`, in stream
 * order), copies cloud `cloud`'s Faster-PFH descriptors (Eq. A5) out of the
 * batch workspace, so that a caller may keep them resident and match them
 * again (kmg_match with rows = j_idx gives the batch's correspondences):
 *   fpfh   [out] float32[cap_rows * 3 * n_bins]: the cloud's kept-point rows
 *                (row i = kept point i of that cloud; zero outside J).
 *   j_idx  [out] int32[cap_j]: the cloud's J points as its own kept indices,
 *                ascending.
 * The counts table of the run gives the sizes (kept points, |J|); at most
 * cap_rows rows and cap_j indices are written.  The batch arguments must be
 * those of the run.  Enqueued on `stream`; no host synchronisation.
 */
kmg_status kmg_batch_descriptors(int32_t n_pairs, int64_t raw_cap, int64_t nnz_cap, int32_t n_bins, int32_t cloud,
                                 float* fpfh, int64_t cap_rows, int32_t* j_idx, int64_t cap_j, void* ws,
                                 size_t ws_bytes, void* stream);
kmg_status kmg_batch_upload(const kmg_cloud* clouds, const kmg_match_out* outs, int32_t n_pairs, int64_t raw_cap,
                            int64_t nnz_cap, void* ws, size_t ws_bytes, void* stream);
kmg_status kmg_batch_run(int32_t n_pairs, int64_t raw_cap, int64_t nnz_cap, int32_t n_bins, int32_t prec,
                         int64_t* counts, void* ws, size_t ws_bytes, void* stream);
kmg_status kmg_register_batch(const kmg_cloud* clouds, const kmg_match_out* outs, int32_t n_pairs,
                              int64_t raw_cap, int64_t nnz_cap, int32_t prec, int64_t* counts, void* ws,
                              size_t ws_bytes, void* stream);

/*
 * Downstream of matching, Section III-D: the ratio filter, the pairwise-
 * invariant compatibility graph of Eq. (3), and its maximum k-core.
 *
 * kmg_corr_graph: src_xyz / tgt_xyz are the kept clouds (device float32 SoA,
 * 3 x m_src and 3 x m_tgt); pairs (device int32[n_corr * 2]), d1 and d2
 * (device float32[n_corr]) are a correspondence set as kmg_match writes it.
 * The n_sel = min(n_corr, n_tau) correspondences with the lowest ratio d1/d2
 * (computed in FP64; 0 when d1 = d2 = 0, +inf when only d2 = 0; ties by
 * position) become the graph's vertices in that order: sel[v] (device
 * int32[n_tau]) is the correspondence of vertex v.  Vertices u != v are
 * adjacent iff | ||b_u - b_v|| - ||a_u - a_v|| | <= 2 beta (Eq. 3) with both
 * norms in FP64 from the float32 coordinates, a = source point, b = target
 * point of the correspondence.  The graph is written as CSR: off (device
 * int32[n_tau + 1], off[n_sel] = nnz) and adj (device int32[adj_cap]), every
 * row ascending, no self loops.  The caller owns every buffer.  *n_sel and
 * *nnz are host pointers (the call synchronises the stream); when
 * nnz > adj_cap, *nnz is the needed capacity, adj is untouched and the call
 * returns KMG_ERR_CAPACITY.  Correspondence indices outside [0, m) give
 * KMG_ERR_RANGE.  Requires 1 <= n_tau <= KMG_MAX_KCORE_VERTICES and
 * beta > 0.
 *
 * kmg_max_kcore: core numbers of the graph (off, adj) on n vertices
 * (n <= KMG_MAX_KCORE_VERTICES; adj entries in [0, n), rows need not be
 * sorted): core (device int32[n]); members (device int32[n]) receives the
 * vertices of the maximum k-core, ascending, *n_members (host) their count and
 * *max_core (host) the largest core number (-1 for n = 0).  An adj entry
 * outside [0, n) gives KMG_ERR_RANGE, and so does a graph above 8,192
 * vertices on a device that cannot give one workgroup more than 64 KiB of
 * LDS.  Synchronises the stream.
 */
kmg_status kmg_corr_graph(const float* src_xyz, int64_t m_src, const float* tgt_xyz, int64_t m_tgt,
                          const int32_t* pairs, const float* d1, const float* d2, int64_t n_corr, int32_t n_tau,
                          double beta, int32_t* sel, int32_t* off, int32_t* adj, int64_t adj_cap, int32_t* n_sel,
                          int64_t* nnz, void* ws, size_t ws_bytes, void* stream);
kmg_status kmg_max_kcore(const int32_t* off, const int32_t* adj, int32_t n, int32_t* core, int32_t* members,
                         int32_t* n_members, int32_t* max_core, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KMG_H */
