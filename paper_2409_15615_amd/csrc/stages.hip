// Single-cloud entry points: batches of one cloud run through the batch
// kernels, with the counts brought back to the host at the end of each call.
#include "kmg_device.h"

namespace kmg {

namespace {

__global__ void init_single(DevStatus* st, CloudDev* cl, CloudDev v, int64_t n_raw, int64_t m_kept) {
    const int i = threadIdx.x;
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    for (int k = i; k < static_cast<int>(sizeof(DevStatus) / 4); k += blockDim.x) w[k] = 0u;
    __syncthreads();
    if (i == 0) {
        st->n_raw = n_raw;
        st->m_kept = m_kept;
        cl[0] = v;
    }
}

kmg_status init(DevStatus* st, CloudDev* cl, const CloudDev& v, int64_t n_raw, int64_t m_kept, hipStream_t s) {
    init_single<<<1, 64, 0, s>>>(st, cl, v, n_raw, m_kept);
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

size_t normals_ws(int64_t m) {
    Carver c(nullptr, 0);
    c.take<DevStatus>(1);
    c.take<CloudDev>(1);
    carve_search(c, m);
    return c.off;
}

kmg_status normals(const float* xyz, int64_t m, const kmg_params& p, float* nrm, uint8_t* flags, int32_t* off,
                   int32_t* nbr, int64_t nbr_cap, int64_t* nnz_host, int32_t* n_normal, void* ws, size_t ws_bytes,
                   hipStream_t s) {
    Carver c(ws, ws_bytes);
    DevStatus* st = c.take<DevStatus>(1);
    CloudDev* cl = c.take<CloudDev>(1);
    SearchWs w = carve_search(c, m);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(init(st, cl, make_cloud(p, nullptr, 0, 0), 0, m, s));
    KMG_TRY(search_count_batch(cl, xyz, m, nullptr, m, st, w, off, s));
    DevStatus h;
    KMG_TRY(read_status(st, &h, s));
    if (h.err_range || (h.dense & 2) || h.nnz > INT32_MAX) return KMG_ERR_RANGE;
    *nnz_host = h.nnz;
    if (h.nnz > nbr_cap) return KMG_ERR_CAPACITY;
    KMG_TRY(search_fill_batch(cl, xyz, m, nullptr, m, nbr_cap, (h.dense & 1) != 0, st, w, off, nbr, nrm, m, flags,
                              n_normal, s));
    timer_collect();
    return KMG_OK;
}

size_t fpfh_ws(int64_t m, int H) {
    Carver c(nullptr, 0);
    c.take<DevStatus>(1);
    c.take<CloudDev>(1);
    carve_feat(c, m, H);
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
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    KMG_TRY(init(st, cl, make_cloud(p, nullptr, 0, 0), 0, m, s));
    KMG_TRY(features_batch(cl, 1, xyz, m, nullptr, m, H, st, w, off, nbr, nrm, m, flags, spfh_out, fpfh_out, j_idx,
                           nullptr, s));
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
