// Radius search on a voxel-cell hash and PCA normals (Algorithm 1, Step 1).
//
// Cells have edge c = r_FPFH * (1 + 1e-4), so every point within r_FPFH of
// a query lies in the 27 cells around the query's cell.  Points are
// counting-sorted by cell into an AoS float4 array (x, y, z, kept index), and
// each query is served by one wavefront whose lanes walk the flattened
// candidate list of the 27 cells.  The search runs twice: a count pass
// (|N(q)|, max degree), then, after a prefix sum has placed every list, a
// fill pass that collects the accepted indices in LDS and writes them in
// ascending order (rank sort).  Normals are then estimated one thread per
// point from the stored list: FP64 moments of the r_normal subset, a cyclic
// Jacobi eigen-solver in FP64, the linearity test and viewpoint orientation.
#include <climits>

#include "kmg_device.h"

namespace kmg {

namespace {

constexpr int kBlock = 256;
constexpr int kSearchWaves = 4;     // waves (queries) per block in the count and fill passes
constexpr int kListSmall = 1024;    // LDS list per wave in the common fill pass
constexpr int kListBig = 8192;      // LDS list of the single-wave pass for dense queries
constexpr double kCellMargin = 1.0 + 1e-4;

struct Grid {
    const float4* pts;     // cell-sorted points; w = bit pattern of the kept index
    const uint64_t* keys;  // cell hash table
    const int32_t* start;  // first sorted position of each cell slot
    const int32_t* count;  // points in each cell slot
    uint32_t mask;
    double inv_c;
};

__device__ __forceinline__ int64_t cell_coord(float x, double inv_c) {
    return static_cast<int64_t>(floor(static_cast<double>(x) * inv_c));
}

__global__ __launch_bounds__(kBlock) void cell_insert(const float* __restrict__ xyz, int m, double inv_c,
                                                      uint64_t* keys, int32_t* cnt, uint32_t mask,
                                                      int32_t* __restrict__ pslot, DevStatus* st) {
    int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    double kx = floor(static_cast<double>(xyz[p]) * inv_c);
    double ky = floor(static_cast<double>(xyz[m + p]) * inv_c);
    double kz = floor(static_cast<double>(xyz[2 * static_cast<int64_t>(m) + p]) * inv_c);
    // keep one cell of headroom so that the 27-cell stencil stays packable
    if (!key_in_range(kx - 1) || !key_in_range(kx + 1) || !key_in_range(ky - 1) || !key_in_range(ky + 1) ||
        !key_in_range(kz - 1) || !key_in_range(kz + 1)) {
        atomicOr(&st->err_range, 1);
        pslot[p] = -1;
        return;
    }
    uint64_t key = pack_key(static_cast<int64_t>(kx), static_cast<int64_t>(ky), static_cast<int64_t>(kz));
    uint32_t h = hash_insert(keys, mask, key);
    atomicAdd(cnt + h, 1);
    pslot[p] = static_cast<int32_t>(h);
}

__global__ __launch_bounds__(kBlock) void cell_scatter(const float* __restrict__ xyz, int m,
                                                       const int32_t* __restrict__ pslot,
                                                       const int32_t* __restrict__ start, int32_t* fill,
                                                       float4* __restrict__ pts) {
    int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    int h = pslot[p];
    if (h < 0) return;
    int pos = start[h] + atomicAdd(fill + h, 1);
    pts[pos] = make_float4(xyz[p], xyz[m + p], xyz[2 * static_cast<int64_t>(m) + p], __int_as_float(p));
}

// One wavefront per query (queries visited in cell-sorted order).
// kFill = false: writes |N(q)| and the max degree.
// kFill = true : writes N(q) ascending at nbr[off[q]..]; lists longer than
//                kCap are skipped (dense = false) or are the only ones served
//                (dense = true).
template <bool kFill, int kCap, int kWaves>
__global__ __launch_bounds__(kWaves* kWave) void radius_search(Grid g, int m, RadiusTest rt,
                                                               int32_t* __restrict__ cnt,
                                                               const int32_t* __restrict__ off,
                                                               int32_t* __restrict__ nbr, int dense,
                                                               DevStatus* st) {
    __shared__ int32_t s_incl[kWaves][32];
    __shared__ int32_t s_start[kWaves][32];
    __shared__ int32_t s_list[kWaves][kFill ? kCap : 1];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    const int w = blockIdx.x * kWaves + wv;
    if (w >= m || st->err_range) return;  // uniform across the wave; no search over a partial grid
    const float4 qp = g.pts[w];
    const int q = __float_as_int(qp.w);
    if (q < 0 || q >= m) return;
    if (kFill) {
        int deg = off[q + 1] - off[q];
        if (dense ? (deg <= kListSmall) : (deg > kCap)) return;
    }
    // the 27 neighbour cells: lanes 0..26 look one up each
    int cc = 0, cs = 0;
    if (lane < 27) {
        int64_t cx = cell_coord(qp.x, g.inv_c) + (lane % 3) - 1;
        int64_t cy = cell_coord(qp.y, g.inv_c) + (lane / 3) % 3 - 1;
        int64_t cz = cell_coord(qp.z, g.inv_c) + lane / 9 - 1;
        int h = hash_find(g.keys, g.mask, pack_key(cx, cy, cz));
        if (h >= 0) {
            cs = g.start[h];
            cc = g.count[h];
        }
    }
    const int incl = wave_incl_scan(cc);
    const int total = __shfl(incl, 26, kWave);
    if (lane < 32) {
        s_incl[wv][lane] = (lane < 27) ? incl : INT_MAX;
        s_start[wv][lane] = cs;
    }
    __builtin_amdgcn_wave_barrier();
    int found = 0;
    for (int base = 0; base < total; base += kWave) {
        const int t = base + lane;
        bool in = false;
        int s = 0;
        if (t < total) {
            int lo = 0, hi = 26;  // first cell whose inclusive prefix exceeds t
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (s_incl[wv][mid] > t) hi = mid;
                else lo = mid + 1;
            }
            const int before = lo ? s_incl[wv][lo - 1] : 0;
            const float4 sp = g.pts[s_start[wv][lo] + (t - before)];
            in = rt(qp.x, qp.y, qp.z, sp.x, sp.y, sp.z);
            s = __float_as_int(sp.w);
        }
        const uint64_t b = ballot(in);
        if (kFill && in) {
            int at = found + lanes_below(b);
            if (at < kCap) s_list[wv][at] = s;
        }
        found += __popcll(b);
    }
    if (!kFill) {
        if (lane == 0) {
            cnt[q] = found;
            // rare events only: no contended atomic per query
            if (found > kListSmall) atomicOr(&st->dense, found > kListBig ? 3 : 1);
        }
        return;
    }
    __builtin_amdgcn_wave_barrier();
    // ranks are unique (distinct indices): scatter each entry to its sorted slot
    int32_t* out = nbr + off[q];
    for (int e = lane; e < found; e += kWave) {
        const int v = s_list[wv][e];
        int r = 0;
        for (int k = 0; k < found; ++k) r += (s_list[wv][k] < v) ? 1 : 0;
        out[r] = v;
    }
}

// Cyclic Jacobi rotation in the (p, q) plane of a symmetric 3x3 matrix held
// as its six distinct entries; r is the remaining index.  V accumulates the
// eigenvectors as columns.
__device__ __forceinline__ void jacobi_plane(double& app, double& aqq, double& apq, double& arp, double& arq,
                                             double V[3][3], int p, int q) {
    if (apq == 0.0) return;
    if (fabs(apq) <= 1e-18 * (fabs(app) + fabs(aqq))) {
        apq = 0.0;
        return;
    }
    const double tau = (aqq - app) / (2.0 * apq);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = t * c;
    app -= t * apq;
    aqq += t * apq;
    apq = 0.0;
    const double rp = arp, rq = arq;
    arp = c * rp - s * rq;
    arq = s * rp + c * rq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vp = V[k][p], vq = V[k][q];
        V[k][p] = c * vp - s * vq;
        V[k][q] = s * vp + c * vq;
    }
}

__global__ __launch_bounds__(kBlock) void normals_kernel(const float* __restrict__ xyz, int m,
                                                         const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ nbr, RadiusTest rn,
                                                         int tau_num, double tau_lin, double vpx, double vpy,
                                                         double vpz, float* __restrict__ nrm,
                                                         uint8_t* __restrict__ flags, int32_t* __restrict__ n_normal,
                                                         DevStatus* st) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= m) return;
    const int64_t m2 = 2 * static_cast<int64_t>(m);
    const float qx = xyz[q], qy = xyz[m + q], qz = xyz[m2 + q];
    const int b = off[q], e = off[q + 1];
    int nn = 0;
    // moments of the r_normal subset, shifted to the query (FP64)
    double sx = 0, sy = 0, sz = 0, sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
    for (int k = b; k < e; ++k) {
        const int s = nbr[k];
        const float x = xyz[s], y = xyz[m + s], z = xyz[m2 + s];
        if (!rn(qx, qy, qz, x, y, z)) continue;
        ++nn;
        const double dx = static_cast<double>(x) - qx, dy = static_cast<double>(y) - qy,
                     dz = static_cast<double>(z) - qz;
        sx += dx;
        sy += dy;
        sz += dz;
        sxx += dx * dx;
        sxy += dx * dy;
        sxz += dx * dz;
        syy += dy * dy;
        syz += dy * dz;
        szz += dz * dz;
    }
    if (n_normal) n_normal[q] = nn;
    if (e - b < tau_num || nn < tau_num) {
        nrm[q] = nrm[m + q] = nrm[m2 + q] = 0.0f;
        flags[q] = 0;
        return;
    }
    const double inv = 1.0 / nn;
    const double mx = sx * inv, my = sy * inv, mz = sz * inv;
    double a00 = sxx * inv - mx * mx, a01 = sxy * inv - mx * my, a02 = sxz * inv - mx * mz;
    double a11 = syy * inv - my * my, a12 = syz * inv - my * mz, a22 = szz * inv - mz * mz;
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 16; ++sweep) {
        if (a01 == 0.0 && a02 == 0.0 && a12 == 0.0) break;
        jacobi_plane(a00, a11, a01, a02, a12, V, 0, 1);
        jacobi_plane(a00, a22, a02, a01, a12, V, 0, 2);
        jacobi_plane(a11, a22, a12, a01, a02, V, 1, 2);
    }
    const double d[3] = {a00, a11, a22};
    int imax = 0, imin = 0;
#pragma unroll
    for (int i = 1; i < 3; ++i) {
        if (d[i] > d[imax]) imax = i;
        if (d[i] < d[imin]) imin = i;
    }
    if (imax == imin) {  // all eigenvalues equal
        imax = 0;
        imin = 2;
    }
    const int imid = 3 - imax - imin;
    const double l1 = d[imax], l2 = d[imid];
    double n0 = V[0][imin], n1 = V[1][imin], n2 = V[2][imin];
    const double nl = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    n0 /= nl;
    n1 /= nl;
    n2 /= nl;
    const double tx = vpx - qx, ty = vpy - qy, tz = vpz - qz;
    const double dot = n0 * tx + n1 * ty + n2 * tz;
    bool flip = dot < 0.0;
    if (dot == 0.0) flip = (n0 != 0.0) ? (n0 < 0.0) : ((n1 != 0.0) ? (n1 < 0.0) : (n2 < 0.0));
    if (flip) {
        n0 = -n0;
        n1 = -n1;
        n2 = -n2;
    }
    if (fabs(dot) < 1e-12 * sqrt(tx * tx + ty * ty + tz * tz)) atomicAdd(&st->amb_orientation, 1u);
    const double plin = (l1 - l2) / l1;
    if (fabs(plin - tau_lin) < 1e-12) atomicAdd(&st->amb_linearity, 1u);
    nrm[q] = static_cast<float>(n0);
    nrm[m + q] = static_cast<float>(n1);
    nrm[m2 + q] = static_cast<float>(n2);
    flags[q] = (plin < tau_lin) ? 1 : 0;
}

struct SearchWs {
    DevStatus* st;
    uint64_t* keys;
    int32_t* ccount;
    int32_t* cstart;
    int32_t* cfill;
    int32_t* pslot;
    float4* pts;
    int32_t* deg;
    int64_t* total;
    int64_t* scan_tmp;
    uint32_t cap_table;
};

SearchWs carve(Carver& c, int64_t m) {
    SearchWs w;
    w.cap_table = next_pow2(static_cast<uint64_t>(std::max<int64_t>(2 * m, 64)));
    w.st = c.take<DevStatus>(1);
    w.keys = c.take<uint64_t>(w.cap_table);
    w.ccount = c.take<int32_t>(w.cap_table);
    w.cstart = c.take<int32_t>(w.cap_table);
    w.cfill = c.take<int32_t>(w.cap_table);
    w.pslot = c.take<int32_t>(static_cast<size_t>(m));
    w.pts = c.take<float4>(static_cast<size_t>(m));
    w.deg = c.take<int32_t>(static_cast<size_t>(m) + 1);
    w.total = c.take<int64_t>(2);
    w.scan_tmp = c.take<int64_t>(std::max(scan_temp_elems(m + 1), scan_temp_elems(w.cap_table)));
    return w;
}

}  // namespace

size_t normals_ws(int64_t m) {
    Carver c(nullptr, 0);
    carve(c, m);
    return c.off;
}

kmg_status normals(const float* xyz, int64_t m, const kmg_params& p, float* nrm, uint8_t* flags, int32_t* off,
                   int32_t* nbr, int64_t nbr_cap, int64_t* nnz_host, int32_t* n_normal, void* ws, size_t ws_bytes,
                   hipStream_t s) {
    Carver c(ws, ws_bytes);
    SearchWs w = carve(c, m);
    if (!c.fits()) return KMG_ERR_WORKSPACE;
    const int mi = static_cast<int>(m);
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.st), 0u, sizeof(DevStatus) / 4, s));
    KMG_TRY(fill_u64(w.keys, kEmptyKey, w.cap_table, s));
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.ccount), 0u, w.cap_table, s));
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.cfill), 0u, w.cap_table, s));
    Grid g;
    g.inv_c = 1.0 / (p.r_fpfh * kCellMargin);
    g.mask = w.cap_table - 1;
    g.pts = w.pts;
    g.keys = w.keys;
    g.start = w.cstart;
    g.count = w.ccount;
    {
    StageScope sc(ST_GRID, s);
    if (m > 0) {
        cell_insert<<<grid_for(m, kBlock), kBlock, 0, s>>>(xyz, mi, g.inv_c, w.keys, w.ccount, g.mask, w.pslot,
                                                          w.st);
        KMG_TRY(launch_status());
    }
    KMG_TRY(scan_exclusive(w.ccount, w.cstart, w.cap_table, w.total + 1, w.scan_tmp, s));
    if (m > 0) {
        cell_scatter<<<grid_for(m, kBlock), kBlock, 0, s>>>(xyz, mi, w.pslot, w.cstart, w.cfill, w.pts);
        KMG_TRY(launch_status());
    }
    }
    const RadiusTest rf = make_radius_test(p.r_fpfh);
    // count pass
    if (m > 0) {
        StageScope sc(ST_SEARCH_COUNT, s);
        radius_search<false, 1, kSearchWaves><<<grid_for(m, kSearchWaves), kSearchWaves * kWave, 0, s>>>(
            g, mi, rf, w.deg, nullptr, nullptr, 0, w.st);
        KMG_TRY(launch_status());
    }
    KMG_TRY(fill_u32(reinterpret_cast<uint32_t*>(w.deg + m), 0u, 1, s));
    KMG_TRY(scan_exclusive(w.deg, off, m + 1, w.total, w.scan_tmp, s));
    int64_t nnz = 0;
    DevStatus st;
    KMG_TRY_HIP(hipMemcpyAsync(&nnz, w.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipMemcpyAsync(&st, w.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    KMG_TRY_HIP(hipStreamSynchronize(s));
    timer_collect();
    if (st.err_range) return KMG_ERR_RANGE;
    if (nnz > INT32_MAX || (st.dense & 2)) return KMG_ERR_RANGE;
    *nnz_host = nnz;
    if (nnz > nbr_cap) return KMG_ERR_CAPACITY;
    if (m > 0) {
        {
        StageScope sc(ST_SEARCH_FILL, s);
        radius_search<true, kListSmall, kSearchWaves><<<grid_for(m, kSearchWaves), kSearchWaves * kWave, 0, s>>>(
            g, mi, rf, nullptr, off, nbr, 0, w.st);
        KMG_TRY(launch_status());
        if (st.dense & 1) {
            radius_search<true, kListBig, 1><<<static_cast<unsigned>(m), kWave, 0, s>>>(g, mi, rf, nullptr, off, nbr,
                                                                                      1, w.st);
            KMG_TRY(launch_status());
        }
        }
        const RadiusTest rn = make_radius_test(p.r_normal);
        StageScope sc(ST_NORMALS, s);
        normals_kernel<<<grid_for(m, kBlock), kBlock, 0, s>>>(xyz, mi, off, nbr, rn, p.tau_num, p.tau_lin,
                                                             p.viewpoint[0], p.viewpoint[1], p.viewpoint[2], nrm,
                                                             flags, n_normal, w.st);
        KMG_TRY(launch_status());
    }  // the stage scope closes here, before the collection below
    timer_collect();
    return KMG_OK;
}

}  // namespace kmg
