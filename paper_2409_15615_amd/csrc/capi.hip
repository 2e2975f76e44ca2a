// extern "C" entry points of libkmg: argument validation, workspace checks and
// dispatch to the kernels.  No call aborts; every failure is a kmg_status.
#include <math.h>

#include "kmg_internal.h"

namespace {

bool params_ok(const kmg_params* p) {
    if (!p) return false;
    if (!(p->voxel > 0.0) || !isfinite(p->voxel)) return false;
    if (!(p->r_normal > 0.0) || !(p->r_fpfh > 0.0) || !isfinite(p->r_fpfh)) return false;
    if (p->r_normal > p->r_fpfh) return false;  // the normal subset is taken from the r_FPFH search
    if (p->tau_num < 1) return false;
    if (!(p->tau_lin > 0.0) || p->tau_lin > 1.0) return false;
    if (p->n_bins < 1 || p->n_bins > kmg::kMaxBins) return false;
    for (int c = 0; c < 3; ++c)
        if (!isfinite(p->viewpoint[c])) return false;
    if (p->mode != KMG_MODE_FASTER_PFH && p->mode != KMG_MODE_CLASSIC_FPFH) return false;
    if (p->reserved != 0) return false;
    return true;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

#define KMG_EXPORT __attribute__((visibility("default")))

extern "C" {

KMG_EXPORT int32_t kmg_version(void) { return 10000; }

KMG_EXPORT const char* kmg_status_string(int32_t status) {
    switch (status) {
        case KMG_OK: return "ok";
        case KMG_ERR_ARG: return "invalid argument";
        case KMG_ERR_CAPACITY: return "output capacity too small";
        case KMG_ERR_DEVICE: return "HIP device error";
        case KMG_ERR_RANGE: return "input outside the supported range";
        case KMG_ERR_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

KMG_EXPORT size_t kmg_workspace_bytes(int32_t op, int64_t n0, int64_t n1, const kmg_params* p) {
    if (n0 < 0 || n1 < 0 || n0 > INT32_MAX || n1 > INT32_MAX) return 0;
    switch (op) {
        case KMG_OP_VOXELIZE: return kmg::voxelize_ws(n0);
        case KMG_OP_NORMALS: return kmg::normals_ws(n0, p ? p->mode : 0, n1);
        case KMG_OP_FPFH: return kmg::fpfh_ws(n0, p ? p->n_bins : 11, p ? p->mode : 0, n1);
        case KMG_OP_MATCH: return kmg::match_ws(n0, n1, p ? 3 * p->n_bins : 33);
        case KMG_OP_GRAPH:
            if (n1 < 1 || n1 > KMG_MAX_KCORE_VERTICES) return 0;
            return kmg::graph_ws(n0, static_cast<int32_t>(n1));
        case KMG_OP_KCORE:
            if (n0 > KMG_MAX_KCORE_VERTICES) return 0;
            return kmg::kcore_ws(static_cast<int32_t>(n0));
        default: return 0;
    }
}

KMG_EXPORT int32_t kmg_timing_enable(int32_t on) { return kmg::timer_enable(on); }

KMG_EXPORT int32_t kmg_timing_read(double* ms, int64_t* launches, int32_t n) {
    return kmg::timer_read(ms, launches, n);
}

KMG_EXPORT int32_t kmg_timing_work(int64_t* work, int32_t n) { return kmg::timer_work(work, n); }

KMG_EXPORT const char* kmg_stage_name(int32_t stage) { return kmg::stage_name(stage); }

KMG_EXPORT kmg_status kmg_voxelize(const float* xyz, int64_t n, double voxel, int32_t* kept_idx, float* kept_xyz,
                        int64_t cap, int64_t* n_kept, void* ws, size_t ws_bytes, void* stream) {
    if (!n_kept || n < 0 || n > INT32_MAX - 1 || cap < 0) return KMG_ERR_ARG;
    if (!(voxel > 0.0) || !isfinite(voxel)) return KMG_ERR_ARG;
    if (n > 0 && (!xyz || !kept_idx || !kept_xyz)) return KMG_ERR_ARG;
    if (!ws) return KMG_ERR_ARG;
    if (ws_bytes < kmg::voxelize_ws(n)) return KMG_ERR_WORKSPACE;
    return kmg::voxelize(xyz, n, voxel, kept_idx, kept_xyz, cap, n_kept, ws, ws_bytes, as_stream(stream));
}

KMG_EXPORT kmg_status kmg_normals(const float* xyz, int64_t m, const kmg_params* p, float* normals, uint8_t* flags,
                       int32_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap, int64_t* nnz, int32_t* n_normal,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!params_ok(p) || !nnz || m < 0 || m > INT32_MAX - 1 || nbr_cap < 0) return KMG_ERR_ARG;
    if (!nbr_off || !ws) return KMG_ERR_ARG;
    if (m > 0 && (!xyz || !normals || !flags)) return KMG_ERR_ARG;
    if (nbr_cap > 0 && !nbr_idx) return KMG_ERR_ARG;
    const int64_t nbr_n = p->mode == KMG_MODE_CLASSIC_FPFH ? nbr_cap : 0;
    if (ws_bytes < kmg::normals_ws(m, p->mode, nbr_n)) return KMG_ERR_WORKSPACE;
    return kmg::normals(xyz, m, *p, normals, flags, nbr_off, nbr_idx, nbr_cap, nnz, n_normal, ws, ws_bytes,
                        as_stream(stream));
}

KMG_EXPORT kmg_status kmg_fpfh(const float* xyz, const float* normals, uint8_t* flags, const int32_t* nbr_off,
                    const int32_t* nbr_idx, int64_t m, const kmg_params* p, float* spfh, float* fpfh,
                    int32_t* j_idx, int64_t* n_j, int64_t* stats, void* ws, size_t ws_bytes, void* stream) {
    if (!params_ok(p) || !n_j || m < 0 || m > INT32_MAX - 1 || !ws) return KMG_ERR_ARG;
    if (m > 0 && (!xyz || !normals || !flags || !nbr_off || !nbr_idx || !fpfh || !j_idx)) return KMG_ERR_ARG;
    if (ws_bytes < kmg::fpfh_ws(m, p->n_bins, p->mode, 0)) return KMG_ERR_WORKSPACE;
    return kmg::fpfh(xyz, normals, flags, nbr_off, nbr_idx, m, *p, spfh, fpfh, j_idx, n_j, stats, ws, ws_bytes,
                     as_stream(stream));
}

KMG_EXPORT size_t kmg_batch_workspace_bytes(int32_t n_pairs, int64_t raw_cap, int64_t nnz_cap, int32_t n_bins) {
    if (n_pairs < 1 || 2 * n_pairs > kmg::kMaxClouds || raw_cap < 0 || raw_cap > INT32_MAX / 2 || nnz_cap < 0 ||
        nnz_cap > INT32_MAX || n_bins < 1 || 3 * n_bins > kmg::kMaxMatchDim)
        return 0;
    return kmg::batch_ws(n_pairs, raw_cap, nnz_cap, n_bins);
}

KMG_EXPORT kmg_status kmg_batch_upload(const kmg_cloud* clouds, const kmg_match_out* outs, int32_t n_pairs,
                                       int64_t raw_cap, int64_t nnz_cap, void* ws, size_t ws_bytes, void* stream) {
    if (!clouds || !outs || !ws || n_pairs < 1 || 2 * n_pairs > kmg::kMaxClouds) return KMG_ERR_ARG;
    if (raw_cap < 0 || raw_cap > INT32_MAX / 2 || nnz_cap < 0 || nnz_cap > INT32_MAX) return KMG_ERR_ARG;
    const int H = clouds[0].params.n_bins;
    if (3 * H > kmg::kMaxMatchDim) return KMG_ERR_ARG;  // the batch form matches the descriptors
    int64_t total = 0;
    for (int k = 0; k < 2 * n_pairs; ++k) {
        if (!params_ok(&clouds[k].params) || clouds[k].params.n_bins != H) return KMG_ERR_ARG;
        if (clouds[k].params.mode != KMG_MODE_FASTER_PFH) return KMG_ERR_ARG;  // the batch form is Faster-PFH
        if (clouds[k].n < 0 || (clouds[k].n > 0 && !clouds[k].xyz)) return KMG_ERR_ARG;
        total += clouds[k].n;
    }
    for (int i = 0; i < n_pairs; ++i)
        if (outs[i].cap < 0 || (outs[i].cap > 0 && (!outs[i].pairs || !outs[i].d1 || !outs[i].d2)))
            return KMG_ERR_ARG;
    if (total > raw_cap) return KMG_ERR_ARG;
    if (ws_bytes < kmg::batch_ws(n_pairs, raw_cap, nnz_cap, H)) return KMG_ERR_WORKSPACE;
    return kmg::batch_upload(clouds, outs, n_pairs, raw_cap, nnz_cap, H, ws, ws_bytes, as_stream(stream));
}

KMG_EXPORT kmg_status kmg_batch_run(int32_t n_pairs, int64_t raw_cap, int64_t nnz_cap, int32_t n_bins,
                                    int32_t prec, int64_t* counts, void* ws, size_t ws_bytes, void* stream) {
    if (!counts || !ws || n_pairs < 1 || 2 * n_pairs > kmg::kMaxClouds) return KMG_ERR_ARG;
    if (raw_cap < 0 || raw_cap > INT32_MAX / 2 || nnz_cap < 0 || nnz_cap > INT32_MAX) return KMG_ERR_ARG;
    if (n_bins < 1 || 3 * n_bins > kmg::kMaxMatchDim) return KMG_ERR_ARG;
    if (prec != KMG_FP32 && prec != KMG_BF16 && prec != KMG_FP16) return KMG_ERR_ARG;
    if (ws_bytes < kmg::batch_ws(n_pairs, raw_cap, nnz_cap, n_bins)) return KMG_ERR_WORKSPACE;
    return kmg::batch_run(n_pairs, raw_cap, nnz_cap, n_bins, prec, counts, ws, ws_bytes, as_stream(stream));
}

KMG_EXPORT kmg_status kmg_register_batch(const kmg_cloud* clouds, const kmg_match_out* outs, int32_t n_pairs,
                                         int64_t raw_cap, int64_t nnz_cap, int32_t prec, int64_t* counts, void* ws,
                                         size_t ws_bytes, void* stream) {
    kmg_status st = kmg_batch_upload(clouds, outs, n_pairs, raw_cap, nnz_cap, ws, ws_bytes, stream);
    if (st != KMG_OK) return st;
    return kmg_batch_run(n_pairs, raw_cap, nnz_cap, clouds[0].params.n_bins, prec, counts, ws, ws_bytes, stream);
}

KMG_EXPORT kmg_status kmg_batch_descriptors(int32_t n_pairs, int64_t raw_cap, int64_t nnz_cap, int32_t n_bins,
                                            int32_t cloud, float* fpfh, int64_t cap_rows, int32_t* j_idx,
                                            int64_t cap_j, void* ws, size_t ws_bytes, void* stream) {
    if (!ws || n_pairs < 1 || 2 * n_pairs > kmg::kMaxClouds) return KMG_ERR_ARG;
    if (raw_cap < 0 || raw_cap > INT32_MAX / 2 || nnz_cap < 0 || nnz_cap > INT32_MAX) return KMG_ERR_ARG;
    if (n_bins < 1 || 3 * n_bins > kmg::kMaxMatchDim || cloud < 0 || cloud >= 2 * n_pairs) return KMG_ERR_ARG;
    if (cap_rows < 0 || cap_j < 0 || (cap_rows > 0 && !fpfh) || (cap_j > 0 && !j_idx)) return KMG_ERR_ARG;
    if (ws_bytes < kmg::batch_ws(n_pairs, raw_cap, nnz_cap, n_bins)) return KMG_ERR_WORKSPACE;
    return kmg::batch_export_cloud(n_pairs, raw_cap, nnz_cap, n_bins, cloud, fpfh, cap_rows, j_idx, cap_j, ws,
                                   ws_bytes, as_stream(stream));
}

KMG_EXPORT kmg_status kmg_match(const float* desc_p, const int32_t* rows_p, int64_t np, const float* desc_q,
                     const int32_t* rows_q, int64_t nq, int32_t dim, int32_t prec, int32_t* pairs, float* d1,
                     float* d2, int64_t cap, int64_t* n_pairs, int64_t* n_fallback, void* ws, size_t ws_bytes,
                     void* stream) {
    if (!n_pairs || np < 0 || nq < 0 || np > INT32_MAX / 2 || nq > INT32_MAX / 2 || cap < 0) return KMG_ERR_ARG;
    if (dim < 1 || dim > kmg::kMaxMatchDim || !ws) return KMG_ERR_ARG;
    if (prec != KMG_FP32 && prec != KMG_BF16 && prec != KMG_FP16) return KMG_ERR_ARG;
    if ((np > 0 && !desc_p) || (nq > 0 && !desc_q)) return KMG_ERR_ARG;
    if (cap > 0 && (!pairs || !d1 || !d2)) return KMG_ERR_ARG;
    if (ws_bytes < kmg::match_ws(np, nq, dim)) return KMG_ERR_WORKSPACE;
    return kmg::match(desc_p, rows_p, np, desc_q, rows_q, nq, dim, prec, pairs, d1, d2, cap, n_pairs, n_fallback,
                      ws, ws_bytes, as_stream(stream));
}

}  // extern "C"

KMG_EXPORT kmg_status kmg_corr_graph(const float* src_xyz, int64_t m_src, const float* tgt_xyz, int64_t m_tgt,
                                     const int32_t* pairs, const float* d1, const float* d2, int64_t n_corr,
                                     int32_t n_tau, double beta, int32_t* sel, int32_t* off, int32_t* adj,
                                     int64_t adj_cap, int32_t* n_sel, int64_t* nnz, void* ws, size_t ws_bytes,
                                     void* stream) {
    if (!n_sel || !nnz || !off || !ws) return KMG_ERR_ARG;
    if (n_corr < 0 || n_corr > INT32_MAX || m_src < 0 || m_tgt < 0 || adj_cap < 0) return KMG_ERR_ARG;
    if (n_tau < 1 || n_tau > KMG_MAX_KCORE_VERTICES || !(beta > 0.0) || !isfinite(beta)) return KMG_ERR_ARG;
    if (n_corr > 0 && (!src_xyz || !tgt_xyz || !pairs || !d1 || !d2 || !sel || m_src == 0 || m_tgt == 0))
        return KMG_ERR_ARG;
    if (adj_cap > 0 && !adj) return KMG_ERR_ARG;
    if (ws_bytes < kmg::graph_ws(n_corr, n_tau)) return KMG_ERR_WORKSPACE;
    return kmg::corr_graph(src_xyz, m_src, tgt_xyz, m_tgt, pairs, d1, d2, n_corr, n_tau, beta, sel, off, adj,
                           adj_cap, n_sel, nnz, ws, ws_bytes, as_stream(stream));
}

KMG_EXPORT kmg_status kmg_max_kcore(const int32_t* off, const int32_t* adj, int32_t n, int32_t* core,
                                    int32_t* members, int32_t* n_members, int32_t* max_core, void* ws,
                                    size_t ws_bytes, void* stream) {
    if (!n_members || !max_core || !ws || n < 0 || n > KMG_MAX_KCORE_VERTICES) return KMG_ERR_ARG;
    if (n > 0 && (!off || !core || !members)) return KMG_ERR_ARG;
    if (ws_bytes < kmg::kcore_ws(n)) return KMG_ERR_WORKSPACE;
    return kmg::max_kcore(off, adj, n, core, members, n_members, max_core, ws, ws_bytes, as_stream(stream));
}
