// Single-cloud entry points: batches of one cloud run through the batch
// kernels, with the counts brought back to the host at the end of each call.
#include "kmg_device.h"

namespace kmg {

namespace {

// off (optional): the caller's neighbour lists, whose volume off[m_kept] goes
// to st->nnz.
__global__ void init_single(DevStatus* st, CloudDev* cl, CloudDev v, int64_t n_raw, int64_t m_kept,
                            const int32_t* off) {
    const int i = threadIdx.x;
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    for (int k = i; k < static_cast<int>(sizeof(DevStatus) / 4); k += blockDim.x) w[k] = 0u;
    __syncthreads();
    if (i == 0) {
        st->n_raw = n_raw;
        st->m_kept = m_kept;
        if (off) st->nnz = off[m_kept];
        cl[0] = v;
    }
}

kmg_status init(DevStatus* st, CloudDev* cl, const CloudDev& v, int64_t n_raw, int64_t m_kept, hipStream_t s,
                const int32_t* off = nullptr) {
    init_single<<<1, 64, 0, s>>>(st, cl, v, n_raw, m_kept, off);
    return launch_status();
}

kmg_status read_status(DevStatus* st, DevStatus* host, hipStream_t s) {
    KMG_TRY_HIP(hipMemcpyAsync(host, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    timer_collect();
    return KMG_OK;
}

}  // namespace

CloudDev make_cloud(const kmg_params& p, const float* raw, int64_t n_raw, int64_t raw_off) {
    CloudDev c{};
    c.raw = raw;
    c.n_raw = static_cast<int32_t>(n_raw);
    c.raw_off = static_cast<int32_t>(raw_off);
    c.tau_num = p.tau_num;
    c.H = p.n_bins;
    c.voxel = p.voxel;
    c.inv_cell = 1.0 / (p.r_fpfh * (1.0 + 1e-4));
    c.tau_lin = p.tau_lin;
    for (int k = 0; k < 3; ++k) c.vp[k] = p.viewpoint[k];
    c.rf = make_radius_test(p.r_fpfh);
    c.rn = make_radius_test(p.r_normal);
    c.mode = p.mode;
    c.tau_j = p.tau_num;
    if (p.mode == KMG_MODE_CLASSIC_FPFH) {
        // classic FPFH: a normal for any point with >= 3 r_normal neighbours, no
        // linearity filter, a descriptor for every point with a normal
        c.tau_num = 3;
        c.tau_lin = 1.0;
        c.tau_j = 1;
    }
    return c;
}

size_t voxelize_ws(int64_t n) {
    Carver c(nullptr, 0);
    c.take<DevStatus>(1);
    c.take<CloudDev>(1);
    carve_voxel(c, n);
    return c.off;
}

kmg_status voxelize(const float* xyz, int64_t n, double voxel, int32_t* kept_idx, float* kept_xyz, int64_t cap,
                    int64_t* n_kept_host, void* ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    DevStatus* st = c.take<DevStatus>(1);
    CloudDev* cl = c.take<CloudDev>(1);
    VoxelWs w = carve_voxel(c, n);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    kmg_params p{};
    p.voxel = voxel;
    p.r_normal = p.r_fpfh = voxel;
    p.tau_lin = 1.0;
    p.tau_num = 1;
    p.n_bins = 1;
    KMG_TRY(init(st, cl, make_cloud(p, xyz, n, 0), n, 0, s));
    KMG_TRY(voxelize_batch(cl, 1, n, st, w, cap, 0, kept_idx, kept_xyz, nullptr, nullptr, s));
    DevStatus h;
    KMG_TRY(read_status(st, &h, s));
    if (h.err_range) return KMG_ERR_RANGE;
    *n_kept_host = h.m_kept;
    if (h.m_kept > cap) return KMG_ERR_CAPACITY;
    return KMG_OK;
}

size_t normals_ws(int64_t m, int mode, int64_t nbr_cap) {
    Carver c(nullptr, 0);
    c.take<DevStatus>(1);
    c.take<CloudDev>(1);
    carve_search(c, m);
    if (mode == KMG_MODE_CLASSIC_FPFH) {  // the separate r_normal lists
        c.take<int32_t>(static_cast<size_t>(m) + 1);
        c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(nbr_cap, 1)));
    }
    return c.off;
}

kmg_status normals(const float* xyz, int64_t m, const kmg_params& p, float* nrm, uint8_t* flags, int32_t* off,
                   int32_t* nbr, int64_t nbr_cap, int64_t* nnz_host, int32_t* n_normal, void* ws, size_t ws_bytes,
                   hipStream_t s) {
    Carver c(ws, ws_bytes);
    DevStatus* st = c.take<DevStatus>(1);
    CloudDev* cl = c.take<CloudDev>(1);
    SearchWs w = carve_search(c, m);
    const bool classic = p.mode == KMG_MODE_CLASSIC_FPFH;
    int32_t* off_n = nullptr;
    int32_t* nbr_n = nullptr;
    int64_t nbr_n_cap = 0;
    if (classic) {
        off_n = c.take<int32_t>(static_cast<size_t>(m) + 1);
        nbr_n_cap = std::max<int64_t>(nbr_cap, 1);
        nbr_n = c.take<int32_t>(static_cast<size_t>(nbr_n_cap));
    }
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(init(st, cl, make_cloud(p, nullptr, 0, 0), 0, m, s));
    DevStatus h;
    if (classic) {
        // search 1 (r_normal) and the normals from its lists
        KMG_TRY(search_count_batch(cl, xyz, m, nullptr, m, st, w, off_n, s, true, 1));
        KMG_TRY(read_status(st, &h, s));
        if (h.err_range || (h.dense & 2) || h.nnz > INT32_MAX) return KMG_ERR_RANGE;
        if (h.nnz > nbr_n_cap) {
            *nnz_host = h.nnz;
            return KMG_ERR_CAPACITY;
        }
        KMG_TRY(search_fill_batch(cl, xyz, m, nullptr, m, nbr_n_cap, (h.dense & 1) != 0, st, w, off_n, nbr_n, nrm, m,
                                  flags, n_normal, s, 1, true));
    }
    // Faster-PFH: the one search at r_FPFH; classic: search 2, lists only
    KMG_TRY(search_count_batch(cl, xyz, m, nullptr, m, st, w, off, s, !classic, 0));
    KMG_TRY(read_status(st, &h, s));
    if (h.err_range || (h.dense & 2) || h.nnz > INT32_MAX) return KMG_ERR_RANGE;
    *nnz_host = h.nnz;
    if (h.nnz > nbr_cap) return KMG_ERR_CAPACITY;
    KMG_TRY(search_fill_batch(cl, xyz, m, nullptr, m, nbr_cap, (h.dense & 1) != 0, st, w, off, nbr, nrm, m, flags,
                              n_normal, s, 0, !classic));
    timer_collect();
    return KMG_OK;
}

size_t fpfh_ws(int64_t m, int H, int mode, int64_t nnz) {
    Carver c(nullptr, 0);
    c.take<DevStatus>(1);
    c.take<CloudDev>(1);
    carve_feat(c, m, H);
    if (mode == KMG_MODE_CLASSIC_FPFH) {  // search 3: its own grid and lists
        carve_search(c, m);
        c.take<int32_t>(static_cast<size_t>(m) + 1);
        c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
    }
    return c.off;
}

kmg_status fpfh(const float* xyz, const float* nrm, uint8_t* flags, const int32_t* off, const int32_t* nbr,
                int64_t m, const kmg_params& p, float* spfh_out, float* fpfh_out, int32_t* j_idx, int64_t* n_j_host,
                int64_t* stats_host, void* ws, size_t ws_bytes, hipStream_t s) {
    const int H = p.n_bins;
    Carver c(ws, ws_bytes);
    DevStatus* st = c.take<DevStatus>(1);
    CloudDev* cl = c.take<CloudDev>(1);
    FeatWs w = carve_feat(c, m, H);
    const bool classic = p.mode == KMG_MODE_CLASSIC_FPFH;
    SearchWs sw{};
    int32_t* off3 = nullptr;
    int32_t* nbr3 = nullptr;
    int64_t nnz3_cap = 0;
    if (classic) {
        sw = carve_search(c, m);
        off3 = c.take<int32_t>(static_cast<size_t>(m) + 1);
        // the rest of the workspace holds search 3's lists (less the carver's alignment)
        nnz3_cap = static_cast<int64_t>((ws_bytes > c.off + 512 ? ws_bytes - c.off - 512 : 0) / sizeof(int32_t));
        nbr3 = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(nnz3_cap, 1)));
    }
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(init(st, cl, make_cloud(p, nullptr, 0, 0), 0, m, s, off));
    if (!classic) {
        KMG_TRY(features_batch(cl, 1, xyz, m, nullptr, m, H, st, w, off, NbrLists{nbr}, nrm, m, flags, spfh_out,
                               fpfh_out, j_idx, nullptr, s));
    } else {
        // SPFH over the lists of search 2; search 3 (r_FPFH again) for the FPFH sum
        KMG_TRY(spfh_batch(cl, xyz, m, nullptr, m, H, st, w, off, NbrLists{nbr}, nrm, m, flags, spfh_out, s));
        KMG_TRY(search_count_batch(cl, xyz, m, nullptr, m, st, sw, off3, s, true, 0));
        DevStatus h3;
        KMG_TRY(read_status(st, &h3, s));
        if (h3.err_range || (h3.dense & 2)) return KMG_ERR_RANGE;
        if (h3.nnz > nnz3_cap) return KMG_ERR_WORKSPACE;
        KMG_TRY(search_fill_batch(cl, xyz, m, nullptr, m, nnz3_cap, (h3.dense & 1) != 0, st, sw, off3, nbr3, nullptr,
                                  m, flags, nullptr, s, 0, false));
        KMG_TRY(fpfh_batch(1, xyz, m, m, H, st, w, off3, NbrLists{nbr3}, flags, fpfh_out, j_idx, nullptr, s));
    }
    DevStatus h;
    KMG_TRY(read_status(st, &h, s));
    *n_j_host = h.n_j;
    if (stats_host) {
        stats_host[0] = h.feat_fp64;
        stats_host[1] = h.feat_edge;
    }
    return KMG_OK;
}

}  // namespace kmg
