// Batched registration: many uneven pairs through every stage in one launch
// per kernel.  kmg_batch_upload copies the per-cloud table into the
// workspace; kmg_batch_run only launches kernels (no host synchronisation,
// no memset or host-memory copy nodes), so it can be captured in a hipGraph
// and replayed after each new upload of equal or smaller sizes.
#include "kmg_device.h"

namespace kmg {

namespace {

// counts[i * 8 + k]: 0 correspondences, 1-2 kept points, 3-4 |J|, 5 exact
// re-scans, 6 status, 7 neighbour entries of the batch.
constexpr int kCountsStride = 8;
// Pad entries per raw point for the list-first search (rows of about 240
// entries when a quarter of the points are kept).
constexpr int64_t kPadPerRaw = 64;

struct BatchWs {
    DevStatus* st;
    CloudDev* cl;
    CloudState* cs;
    PairOutDev* outs;
    MatchSet* sets;
    VoxelWs vox;
    int32_t* kept_idx;
    float* kept_xyz;
    int32_t* kept_cloud;
    SearchWs srch;
    int32_t* off;
    int32_t* nbr;
    int32_t* pad;     // list-first search: the lists, a row per kept point
    int64_t pad_cap;
    int32_t* long_q;  // list-first search: the queries whose lists exceed a row
    uint64_t* scan_status;  // look-back words: the voxel numbering, the search's two scans, the J scan
    size_t n_vox_status;
    size_t n_search_status;
    size_t n_scan_status;
    float* nrm;
    uint8_t* flags;
    FeatWs feat;
    float* fpfh;
    int32_t* jlist;
    MatchWs match;
};

BatchWs carve_batch(Carver& c, int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H) {
    const int C = 2 * n_pairs;
    const size_t rc = static_cast<size_t>(std::max<int64_t>(raw_cap, 1));
    BatchWs w;
    w.st = c.take<DevStatus>(1);
    w.cl = c.take<CloudDev>(C);
    w.cs = c.take<CloudState>(C);
    w.outs = c.take<PairOutDev>(n_pairs);
    w.sets = c.take<MatchSet>(C);
    w.vox = carve_voxel(c, raw_cap);
    w.kept_idx = c.take<int32_t>(rc);
    w.kept_xyz = c.take<float>(3 * rc);
    w.kept_cloud = c.take<int32_t>(rc);
    w.srch = carve_search(c, raw_cap);
    w.off = c.take<int32_t>(rc + 1);
    w.nbr = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(nnz_cap, 1)));
    w.pad_cap = static_cast<int64_t>(rc) * kPadPerRaw;
    w.pad = c.take<int32_t>(static_cast<size_t>(w.pad_cap));
    w.long_q = c.take<int32_t>(rc);
    w.n_vox_status = scan_temp_elems(raw_cap);
    w.n_search_status = search_scan_status_elems(w.srch, raw_cap);
    w.n_scan_status = w.n_vox_status + w.n_search_status + scan_temp_elems(raw_cap);
    w.scan_status = c.take<uint64_t>(w.n_scan_status);
    w.nrm = c.take<float>(3 * rc);
    w.flags = c.take<uint8_t>(rc);
    w.feat = carve_feat(c, raw_cap, H);
    w.fpfh = c.take<float>(rc * 3 * H);
    w.jlist = c.take<int32_t>(rc);
    w.match = carve_match(c, C, raw_cap, 3 * H);
    return w;
}

// Clears the status (block 0) and does every fill the step needs before its
// first stage: the count table, the voxel and cell tables, the degrees, the J
// flags and the look-back words of the one-launch scans (the stages are told
// that they come in cleared).
__global__ __launch_bounds__(256) void batch_init(DevStatus* st, const CloudDev* cl, int n_clouds, FillJobs fills) {
    if (blockIdx.x == 0) {
        uint32_t* w = reinterpret_cast<uint32_t*>(st);
        for (int k = threadIdx.x; k < static_cast<int>(sizeof(DevStatus) / 4); k += blockDim.x) w[k] = 0u;
        __syncthreads();
        if (threadIdx.x == 0) st->n_raw = static_cast<int64_t>(cl[n_clouds - 1].raw_off) + cl[n_clouds - 1].n_raw;
    }
    run_fill_jobs(fills);
}

// Copies cloud `cloud`'s descriptor rows (kept-space rows, zero outside J) and
// its J list as kept indices of that cloud, at most the given capacities.
__global__ __launch_bounds__(256) void batch_export(const CloudState* __restrict__ cs, int cloud,
                                                    const float* __restrict__ fpfh, const int32_t* __restrict__ jlist,
                                                    int D, float* __restrict__ fpfh_out, int64_t cap_rows,
                                                    int32_t* __restrict__ j_out, int64_t cap_j) {
    const CloudState c = cs[cloud];
    const int64_t rows = c.kept_cnt < cap_rows ? c.kept_cnt : cap_rows;
    const int64_t nj = c.j_cnt < cap_j ? c.j_cnt : cap_j;
    const int64_t gs = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const float* src = fpfh + static_cast<int64_t>(c.kept_off) * D;
    for (int64_t t = t0; t < rows * D; t += gs) fpfh_out[t] = src[t];
    for (int64_t i = t0; i < nj; i += gs) j_out[i] = jlist[c.j_off + i] - c.kept_off;
}

}  // namespace

kmg_status batch_export_cloud(int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H, int cloud, float* fpfh_out,
                              int64_t cap_rows, int32_t* j_out, int64_t cap_j, void* ws, size_t ws_bytes,
                              hipStream_t s) {
    Carver c(ws, ws_bytes);
    BatchWs w = carve_batch(c, n_pairs, raw_cap, nnz_cap, H);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    const int64_t most = std::max<int64_t>(cap_rows * 3 * H, cap_j);
    batch_export<<<static_cast<unsigned>(std::min<int64_t>(std::max<int64_t>((most + 255) / 256, 1), 1024)), 256, 0,
                   s>>>(w.cs, cloud, w.fpfh, w.jlist, 3 * H, fpfh_out, cap_rows, j_out, cap_j);
    return launch_status();
}

size_t batch_ws(int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H) {
    Carver c(nullptr, 0);
    carve_batch(c, n_pairs, raw_cap, nnz_cap, H);
    return c.off;
}

kmg_status batch_upload(const kmg_cloud* clouds, const kmg_match_out* outs, int n_pairs, int64_t raw_cap,
                        int64_t nnz_cap, int H, void* ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    BatchWs w = carve_batch(c, n_pairs, raw_cap, nnz_cap, H);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    const int C = 2 * n_pairs;
    CloudDev* table = new CloudDev[C];
    PairOutDev* otab = new PairOutDev[n_pairs];
    int64_t off = 0;
    for (int k = 0; k < C; ++k) {
        table[k] = make_cloud(clouds[k].params, clouds[k].xyz, clouds[k].n, off);
        off += clouds[k].n;
    }
    for (int i = 0; i < n_pairs; ++i) otab[i] = PairOutDev{outs[i].pairs, outs[i].d1, outs[i].d2, outs[i].cap};
    hipError_t e1 = hipMemcpyAsync(w.cl, table, sizeof(CloudDev) * C, hipMemcpyHostToDevice, s);
    hipError_t e2 = hipMemcpyAsync(w.outs, otab, sizeof(PairOutDev) * n_pairs, hipMemcpyHostToDevice, s);
    // the tables live on the host stack of this call: wait for the copies
    hipError_t e3 = hipStreamSynchronize(s);
    delete[] table;
    delete[] otab;
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return KMG_ERR_DEVICE;
    return KMG_OK;
}

kmg_status batch_run(int n_pairs, int64_t raw_cap, int64_t nnz_cap, int H, int prec, int64_t* counts, void* ws,
                     size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    BatchWs w = carve_batch(c, n_pairs, raw_cap, nnz_cap, H);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    const int C = 2 * n_pairs;
    const int D = 3 * H;
    const int64_t rc = std::max<int64_t>(raw_cap, 1);
    FillJobs fills{};
    fills.job[0] = FillJob{counts, 0ull, static_cast<int64_t>(n_pairs) * kCountsStride, 8};
    fills.job[1] = FillJob{w.vox.keys, kEmptyKey, w.vox.cap_table, 8};
    fills.job[2] = FillJob{w.vox.mins, 0x7fffffffull, w.vox.cap_table, 4};
    fills.job[3] = FillJob{w.srch.keys, kEmptyKey, w.srch.cap_table, 8};
    fills.job[4] = FillJob{w.srch.ccount, 0ull, w.srch.cap_table, 4};
    fills.job[5] = FillJob{w.srch.cfill, 0ull, w.srch.cap_table, 4};
    fills.job[6] = FillJob{w.srch.deg, 0ull, raw_cap + 1, 4};
    fills.job[7] = FillJob{w.feat.jflag, 0ull, rc, 4};
    fills.job[8] = FillJob{w.scan_status, 0ull, static_cast<int64_t>(w.n_scan_status), 8};
    fills.n_jobs = 9;
    const int64_t most = std::max<int64_t>({static_cast<int64_t>(w.vox.cap_table), w.srch.cap_table, rc + 1});
    batch_init<<<static_cast<unsigned>(std::min<int64_t>((most + 255) / 256, 4096)), 256, 0, s>>>(w.st, w.cl, C,
                                                                                                  fills);
    KMG_TRY(launch_status());
    // the kept points go into the cleared cell hash of the search as they are emitted
    const GridInsert gi{w.srch.keys, w.srch.ccount, w.srch.cap_table - 1, w.srch.pslot, w.st};
    KMG_TRY(voxelize_batch(w.cl, C, raw_cap, w.st, w.vox, raw_cap, raw_cap, w.kept_idx, w.kept_xyz, w.kept_cloud,
                           w.cs, s, true, &gi, w.scan_status));
    const bool list_first = tuning().search_form == 1;
    if (list_first) {
        KMG_TRY(search_lists_first(w.cl, w.kept_xyz, raw_cap, w.kept_cloud, raw_cap, nnz_cap, w.st, w.srch, w.off,
                                   w.nbr, w.pad, w.pad_cap, w.long_q, w.nrm, raw_cap, w.flags, s, true,
                                   w.scan_status + w.n_vox_status));
    } else {
        KMG_TRY(search_count_batch(w.cl, w.kept_xyz, raw_cap, w.kept_cloud, raw_cap, w.st, w.srch, w.off, s, true,
                                   0, true, true));
        KMG_TRY(search_fill_batch(w.cl, w.kept_xyz, raw_cap, w.kept_cloud, raw_cap, nnz_cap, true, w.st, w.srch,
                                  w.off, w.nbr, w.nrm, raw_cap, w.flags, nullptr, s));
    }
    // the list-first search leaves the lists in the pad rows (the longer ones in nbr);
    // the J list emission also writes the clouds' J ranges and matching sets
    const NbrLists nb = list_first ? NbrLists{w.nbr, w.pad, w.pad_cap} : NbrLists{w.nbr};
    KMG_TRY(features_batch(w.cl, C, w.kept_xyz, raw_cap, w.kept_cloud, raw_cap, H, w.st, w.feat, w.off, nb,
                           w.nrm, raw_cap, w.flags, nullptr, w.fpfh, w.jlist, w.cs, s, true, w.sets,
                           w.scan_status + w.n_vox_status + w.n_search_status));
    // the pair counts and statuses come with the correspondences
    KMG_TRY(match_batch(w.sets, C, D, prec, w.st, w.match, w.outs, counts, kCountsStride, s, w.cs, nnz_cap));
    timer_collect();  // waits for the stream only while timing is enabled
    return KMG_OK;
}

}  // namespace kmg
