/*
 * kmg_oracle.c -- plain, slow, FP64 CPU oracle for the Faster-PFH + mutual
 * nearest-neighbour matching hot path of KISS-Matcher (arXiv 2409.15615).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * called from the tests, from the smoke check and from the benchmark's CPU
 * baseline leg.  The product library never links, loads or calls it, and it
 * shares no code, header, table or constant with the GPU path.
 *
 * Every step follows the paper's definitions written out directly, in FP64,
 * with no blocking or reordering: brute-force O(m^2) radius search (and, for
 * clouds too large for it, the same test over the candidates of a uniform
 * grid, checked against the brute force by the tests), a cyclic
 * Jacobi eigen-solver, direct evaluation of the angular features, histogram
 * bins, SPFH and FPFH, and brute-force O(|P||Q|) descriptor distances.
 * Build with -O2 -ffp-contract=off (no FMA contraction, no fast-math).
 *
 * Conventions where the paper is silent (the same ones the GPU path uses):
 *  - voxel representative = lowest input index in each voxel; kept points
 *    are emitted in ascending input index; keys are floor(x / v) in FP64;
 *  - squared distance d2(q,s) = ((dx*dx) + dy*dy) + dz*dz with
 *    dx = (double)x_s - (double)x_q, compared strictly against r*r;
 *  - covariance is mean-centred over the r_normal subset, scaled by 1/n;
 *  - normals are oriented so that n . (vp - a_q) >= 0;
 *  - the pair point "a" is the one whose normal makes the smaller unsigned
 *    angle with the connecting line (ties -> the query);
 *  - histogram bounds are [-pi, pi], [-1, 1], [-1, 1]; bins are clamped;
 *  - the SPFH normaliser is the number of valid neighbours other than q.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* threads                                                                   */
/* ------------------------------------------------------------------------ */

int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Voxel downsampling (Section III-A: inputs are voxelized clouds of size v) */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t k[3];
    int64_t idx;
} orc_keyed;

static int orc_keyed_cmp(const void* a, const void* b) {
    const orc_keyed* x = (const orc_keyed*)a;
    const orc_keyed* y = (const orc_keyed*)b;
    for (int c = 0; c < 3; ++c) {
        if (x->k[c] < y->k[c]) return -1;
        if (x->k[c] > y->k[c]) return 1;
    }
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

static int orc_i32_cmp(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x < y) ? -1 : (x > y);
}

/* Voxel key of one coordinate: floor((double)x / v). */
static int64_t orc_voxel_key(float x, double v) { return (int64_t)floor((double)x / v); }

/* Keeps, for every occupied voxel, the finite input point of lowest index.
 * xyz is SoA (x[n], y[n], z[n]).  Writes kept indices in ascending order and
 * their keys (SoA, 3 x m); returns m. */
int64_t orc_voxelize(const float* xyz, int64_t n, double v, int32_t* kept, int64_t* keys) {
    const float* X = xyz;
    const float* Y = xyz + n;
    const float* Z = xyz + 2 * n;
    orc_keyed* a = (orc_keyed*)malloc(sizeof(orc_keyed) * (size_t)(n > 0 ? n : 1));
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(X[i]) || !isfinite(Y[i]) || !isfinite(Z[i])) continue;
        a[cnt].k[0] = orc_voxel_key(X[i], v);
        a[cnt].k[1] = orc_voxel_key(Y[i], v);
        a[cnt].k[2] = orc_voxel_key(Z[i], v);
        a[cnt].idx = i;
        ++cnt;
    }
    qsort(a, (size_t)cnt, sizeof(orc_keyed), orc_keyed_cmp);
    int64_t m = 0;
    /* sorted by (key, index): the first entry of each key run has the lowest index */
    for (int64_t i = 0; i < cnt; ++i) {
        int same_key = (i > 0) && a[i].k[0] == a[i - 1].k[0] && a[i].k[1] == a[i - 1].k[1] &&
                       a[i].k[2] == a[i - 1].k[2];
        if (!same_key) kept[m++] = (int32_t)a[i].idx;
    }
    qsort(kept, (size_t)m, sizeof(int32_t), orc_i32_cmp);
    if (keys) {
        for (int64_t j = 0; j < m; ++j) {
            int32_t i = kept[j];
            keys[j] = orc_voxel_key(X[i], v);
            keys[m + j] = orc_voxel_key(Y[i], v);
            keys[2 * m + j] = orc_voxel_key(Z[i], v);
        }
    }
    free(a);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Radius search (Eq. A1): N(q) = { s : ||a_s - a_q|| < r }, q included      */
/* ------------------------------------------------------------------------ */

static double orc_d2(const float* xyz, int64_t m, int64_t q, int64_t s) {
    double dx = (double)xyz[s] - (double)xyz[q];
    double dy = (double)xyz[m + s] - (double)xyz[m + q];
    double dz = (double)xyz[2 * m + s] - (double)xyz[2 * m + q];
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    return d2;
}

/* Pass 1: counts |N(q)| by brute force over all points. */
int64_t orc_radius_count(const float* xyz, int64_t m, double r, int32_t* cnt) {
    const double r2 = r * r;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t q = 0; q < m; ++q) {
        int32_t c = 0;
        for (int64_t s = 0; s < m; ++s)
            if (orc_d2(xyz, m, q, s) < r2) ++c;
        cnt[q] = c;
        total += c;
    }
    return total;
}

/* Pass 2: writes N(q) in ascending index order at off[q]..off[q+1]. */
void orc_radius_fill(const float* xyz, int64_t m, double r, const int64_t* off, int32_t* idx) {
    const double r2 = r * r;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < m; ++q) {
        int64_t w = off[q];
        for (int64_t s = 0; s < m; ++s)
            if (orc_d2(xyz, m, q, s) < r2) idx[w++] = (int32_t)s;
    }
}

/* The same two passes over candidates taken from a uniform grid of cell size
 * c = r (1 + 1e-7): a point within r of q lies in one of the 27 cells around
 * q's cell (|dx| < r < c, so floor(x_s / c) and floor(x_q / c) differ by at
 * most 1 even after the rounding of the divisions), and every candidate is
 * decided by the same strict FP64 test as the brute force.  For clouds whose
 * O(m^2) brute force is too slow; tests check it against the brute force. */
typedef struct {
    int64_t key[3];
    int32_t idx;
} orc_cell;

static int orc_cell_cmp(const void* a, const void* b) {
    const orc_cell* x = (const orc_cell*)a;
    const orc_cell* y = (const orc_cell*)b;
    for (int c = 0; c < 3; ++c) {
        if (x->key[c] < y->key[c]) return -1;
        if (x->key[c] > y->key[c]) return 1;
    }
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

/* First entry of cells[0..n) whose key is >= k (lexicographic). */
static int64_t orc_cell_lower(const orc_cell* cells, int64_t n, const int64_t k[3]) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int less = 0;
        for (int c = 0; c < 3; ++c) {
            if (cells[mid].key[c] < k[c]) { less = 1; break; }
            if (cells[mid].key[c] > k[c]) break;
        }
        if (less) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static orc_cell* orc_grid_build(const float* xyz, int64_t m, double c) {
    orc_cell* cells = (orc_cell*)malloc(sizeof(orc_cell) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) {
        for (int a = 0; a < 3; ++a) cells[i].key[a] = (int64_t)floor((double)xyz[a * m + i] / c);
        cells[i].idx = (int32_t)i;
    }
    qsort(cells, (size_t)m, sizeof(orc_cell), orc_cell_cmp);
    return cells;
}

/* Visits the candidates of q (the 27 cells around its cell) and keeps those with
 * d2 < r^2: counts them, or, when out != NULL, writes them and sorts them. */
static int32_t orc_grid_query(const float* xyz, int64_t m, const orc_cell* cells, double c, double r2, int64_t q,
                              int32_t* out) {
    int64_t kq[3];
    for (int a = 0; a < 3; ++a) kq[a] = (int64_t)floor((double)xyz[a * m + q] / c);
    int32_t cnt = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int64_t k[3] = {kq[0] + dx, kq[1] + dy, kq[2] + dz};
                for (int64_t e = orc_cell_lower(cells, m, k); e < m; ++e) {
                    if (cells[e].key[0] != k[0] || cells[e].key[1] != k[1] || cells[e].key[2] != k[2]) break;
                    if (orc_d2(xyz, m, q, cells[e].idx) < r2) {
                        if (out) out[cnt] = cells[e].idx;
                        ++cnt;
                    }
                }
            }
    if (out) qsort(out, (size_t)cnt, sizeof(int32_t), orc_i32_cmp);
    return cnt;
}

int64_t orc_radius_count_grid(const float* xyz, int64_t m, double r, int32_t* cnt) {
    const double c = r * (1.0 + 1e-7);
    orc_cell* cells = orc_grid_build(xyz, m, c);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
    for (int64_t q = 0; q < m; ++q) {
        cnt[q] = orc_grid_query(xyz, m, cells, c, r * r, q, NULL);
        total += cnt[q];
    }
    free(cells);
    return total;
}

void orc_radius_fill_grid(const float* xyz, int64_t m, double r, const int64_t* off, int32_t* idx) {
    const double c = r * (1.0 + 1e-7);
    orc_cell* cells = orc_grid_build(xyz, m, c);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < m; ++q) orc_grid_query(xyz, m, cells, c, r * r, q, idx + off[q]);
    free(cells);
}

/* ------------------------------------------------------------------------ */
/* Normal estimation by PCA (Section III-C; Algorithm 1, Step 1)            */
/* ------------------------------------------------------------------------ */

/* Cyclic Jacobi on a symmetric 3x3 matrix A (row-major, destroyed).  On exit
 * A's diagonal holds the eigenvalues and V's columns the eigenvectors. */
void orc_jacobi3(double A[9], double V[9]) {
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        if (off == 0.0) break;
        int rotated = 0;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                double app = A[3 * p + p], aqq = A[3 * q + q];
                /* skip rotations that cannot change the diagonal in FP64 */
                if (fabs(apq) <= 1e-300 ||
                    (fabs(app) + 100.0 * fabs(apq) == fabs(app) && fabs(aqq) + 100.0 * fabs(apq) == fabs(aqq))) {
                    A[3 * p + q] = 0.0;
                    A[3 * q + p] = 0.0;
                    continue;
                }
                double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                /* A <- J^T A J with J the (p,q) rotation */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = c * akp - s * akq;
                    A[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = c * apk - s * aqk;
                    A[3 * q + k] = s * apk + c * aqk;
                }
                A[3 * p + q] = 0.0;
                A[3 * q + p] = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - s * vkq;
                    V[3 * k + q] = s * vkp + c * vkq;
                }
                rotated = 1;
            }
        }
        if (!rotated) break;
    }
}

/* Eigen-decomposition sorted descending: lam[0] >= lam[1] >= lam[2]; vec is
 * column-major per eigenvalue (vec[3*i + c] = component c of eigenvector i). */
void orc_eig3_sorted(const double C[9], double lam[3], double vec[9]) {
    double A[9], V[9];
    memcpy(A, C, sizeof(A));
    orc_jacobi3(A, V);
    int ord[3] = {0, 1, 2};
    double d[3] = {A[0], A[4], A[8]};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (d[ord[j]] > d[ord[i]]) {
                int t = ord[i];
                ord[i] = ord[j];
                ord[j] = t;
            }
    for (int i = 0; i < 3; ++i) {
        lam[i] = d[ord[i]];
        for (int c = 0; c < 3; ++c) vec[3 * i + c] = V[3 * c + ord[i]];
    }
}

/* For every point q: |N(q)| and |P_normal(q)| (strict d2 < r_normal^2 within
 * N(q)); if both reach tau_num, PCA over P_normal gives lambda1>=lambda2>=lambda3,
 * the linearity p_lin = (l1 - l2) / l1 and the unit eigenvector of l3 oriented
 * toward the viewpoint; B[q] = (p_lin < tau_lin).  normals is SoA 3 x m and is
 * zero where no normal was estimated.  gap[q] = (l2 - l3) / l1 (NaN if none). */
void orc_normals(const float* xyz, int64_t m, const int64_t* off, const int32_t* idx, double r_normal,
                 int32_t tau_num, double tau_lin, const double vp[3], double* normals, double* plin,
                 double* gap, int32_t* n_normal, uint8_t* B) {
    const double rn2 = r_normal * r_normal;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < m; ++q) {
        int64_t nN = off[q + 1] - off[q];
        normals[q] = normals[m + q] = normals[2 * m + q] = 0.0;
        plin[q] = NAN;
        gap[q] = NAN;
        n_normal[q] = 0;
        B[q] = 0;
        int32_t nn = 0;
        for (int64_t e = off[q]; e < off[q + 1]; ++e)
            if (orc_d2(xyz, m, q, idx[e]) < rn2) ++nn;
        n_normal[q] = nn;
        if (nN < tau_num) continue;
        if (nn < tau_num) continue;
        double mu[3] = {0.0, 0.0, 0.0};
        for (int64_t e = off[q]; e < off[q + 1]; ++e) {
            int32_t s = idx[e];
            if (!(orc_d2(xyz, m, q, s) < rn2)) continue;
            mu[0] += (double)xyz[s];
            mu[1] += (double)xyz[m + s];
            mu[2] += (double)xyz[2 * m + s];
        }
        for (int c = 0; c < 3; ++c) mu[c] = mu[c] / (double)nn;
        double C[9] = {0};
        for (int64_t e = off[q]; e < off[q + 1]; ++e) {
            int32_t s = idx[e];
            if (!(orc_d2(xyz, m, q, s) < rn2)) continue;
            double p[3] = {(double)xyz[s] - mu[0], (double)xyz[m + s] - mu[1], (double)xyz[2 * m + s] - mu[2]};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) C[3 * i + j] += p[i] * p[j];
        }
        for (int i = 0; i < 9; ++i) C[i] = C[i] / (double)nn;
        double lam[3], vec[9];
        orc_eig3_sorted(C, lam, vec);
        double n[3] = {vec[6], vec[7], vec[8]};
        double nrm = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int c = 0; c < 3; ++c) n[c] = n[c] / nrm;
        double to_vp[3] = {vp[0] - (double)xyz[q], vp[1] - (double)xyz[m + q], vp[2] - (double)xyz[2 * m + q]};
        double dot = n[0] * to_vp[0] + n[1] * to_vp[1] + n[2] * to_vp[2];
        int flip = 0;
        if (dot < 0.0) {
            flip = 1;
        } else if (dot == 0.0) {
            for (int c = 0; c < 3; ++c)
                if (n[c] != 0.0) {
                    flip = n[c] < 0.0;
                    break;
                }
        }
        if (flip)
            for (int c = 0; c < 3; ++c) n[c] = -n[c];
        double pl = (lam[0] - lam[1]) / lam[0];
        plin[q] = pl;
        gap[q] = (lam[1] - lam[2]) / lam[0];
        normals[q] = n[0];
        normals[m + q] = n[1];
        normals[2 * m + q] = n[2];
        B[q] = (pl < tau_lin) ? 1 : 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Angular features (Eq. A2), bins (Eq. A3), SPFH (Eq. A4), FPFH (Eq. A5)    */
/* ------------------------------------------------------------------------ */

static double orc_dot(const double a[3], const double b[3]) {
    double s = a[0] * b[0];
    s = s + a[1] * b[1];
    s = s + a[2] * b[2];
    return s;
}

static void orc_cross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Features f1, f2, f3 of the pair (q, k).  pq, pk are points, nq, nk normals. */
void orc_pair_features(const double pq[3], const double nq[3], const double pk[3], const double nk[3],
                       double f[3]) {
    double d0[3] = {pk[0] - pq[0], pk[1] - pq[1], pk[2] - pq[2]};
    double aq = fabs(orc_dot(nq, d0));
    double ak = fabs(orc_dot(nk, d0));
    const double *pa, *pb, *na, *nb;
    if (aq >= ak) {
        pa = pq; na = nq; pb = pk; nb = nk;
    } else {
        pa = pk; na = nk; pb = pq; nb = nq;
    }
    double d[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
    double dl = sqrt(orc_dot(d, d));
    for (int c = 0; c < 3; ++c) d[c] = d[c] / dl;
    const double* u = na;
    double v[3];
    orc_cross(d, u, v);
    double vl = sqrt(orc_dot(v, v));
    if (vl == 0.0) {
        f[0] = 0.0;
        f[1] = 0.0;
        f[2] = orc_dot(u, d);
        return;
    }
    for (int c = 0; c < 3; ++c) v[c] = v[c] / vl;
    double w[3];
    orc_cross(u, v, w);
    f[0] = atan2(orc_dot(w, nb) + 0.0, orc_dot(u, nb));
    f[1] = orc_dot(v, nb);
    f[2] = orc_dot(u, d);
}

/* Bin of a feature value inside [lo, hi] with H bins, clamped to [0, H-1].
 * *edge is set when the scaled coordinate lies within 1e-9 of an integer. */
int orc_bin(double f, double lo, double hi, int H, int* edge) {
    double s = (double)H * (f - lo) / (hi - lo);
    double fl = floor(s);
    if (edge) *edge = (fabs(s - fl) < 1e-9) || (fabs(s - (fl + 1.0)) < 1e-9);
    int b = (int)fl;
    if (b < 0) b = 0;
    if (b > H - 1) b = H - 1;
    return b;
}

/* Step 2 of Algorithm 1 plus SPFH (Eq. A4) for every point with B[q]:
 * M[q] = { k in N(q) : B[k] }, P_q = |M[q]| - 1, J[q] = B[q] && |M[q]| >= tau_num.
 * counts[q*3H + l*H + h] = number of k in M[q]\{q} whose feature l falls in bin h;
 * spfh = 100 * counts / P_q (0 when P_q = 0).  normals SoA 3 x m, FP64.
 * Returns the number of feature values that landed within 1e-9 of a bin edge. */
int64_t orc_spfh(const float* xyz, const double* normals, int64_t m, const int64_t* off, const int32_t* idx,
                 const uint8_t* B, int32_t tau_num, int32_t H, int32_t* counts, double* spfh, int32_t* Pq,
                 uint8_t* J) {
    const int D = 3 * H;
    const double lo[3] = {-ORC_PI, -1.0, -1.0};
    const double hi[3] = {ORC_PI, 1.0, 1.0};
    int64_t edges = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : edges)
    for (int64_t q = 0; q < m; ++q) {
        int32_t* cq = counts + q * D;
        double* sq = spfh + q * D;
        for (int i = 0; i < D; ++i) {
            cq[i] = 0;
            sq[i] = 0.0;
        }
        Pq[q] = 0;
        J[q] = 0;
        if (!B[q]) continue;
        int32_t nm = 0;
        for (int64_t e = off[q]; e < off[q + 1]; ++e)
            if (B[idx[e]]) ++nm;
        Pq[q] = nm - 1;
        J[q] = (nm >= tau_num) ? 1 : 0;
        double pq[3] = {(double)xyz[q], (double)xyz[m + q], (double)xyz[2 * m + q]};
        double nq[3] = {normals[q], normals[m + q], normals[2 * m + q]};
        for (int64_t e = off[q]; e < off[q + 1]; ++e) {
            int32_t k = idx[e];
            if (k == q || !B[k]) continue;
            double pk[3] = {(double)xyz[k], (double)xyz[m + k], (double)xyz[2 * m + k]};
            double nk[3] = {normals[k], normals[m + k], normals[2 * m + k]};
            double f[3];
            orc_pair_features(pq, nq, pk, nk, f);
            for (int l = 0; l < 3; ++l) {
                int edge = 0;
                int b = orc_bin(f[l], lo[l], hi[l], H, &edge);
                cq[l * H + b] += 1;
                edges += edge;
            }
        }
        if (Pq[q] > 0)
            for (int i = 0; i < D; ++i) sq[i] = (100.0 * (double)cq[i]) / (double)Pq[q];
    }
    return edges;
}

/* FPFH (Eq. A5) for q in J:
 * FPFH(q) = SPFH(q) + (1 / P_q) * sum_{k in M[q], k != q} (1 / w_k) * SPFH(k),
 * w_k = sqrt(d2(q, k)), summed in ascending k.  Rows outside J are zero. */
void orc_fpfh(const float* xyz, int64_t m, const int64_t* off, const int32_t* idx, const uint8_t* B,
              const uint8_t* J, const double* spfh, const int32_t* Pq, int32_t H, double* fpfh) {
    const int D = 3 * H;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < m; ++q) {
        double* out = fpfh + q * D;
        for (int i = 0; i < D; ++i) out[i] = 0.0;
        if (!J[q]) continue;
        double acc[3 * 64];
        for (int i = 0; i < D; ++i) acc[i] = 0.0;
        for (int64_t e = off[q]; e < off[q + 1]; ++e) {
            int32_t k = idx[e];
            if (k == q || !B[k]) continue;
            double w = 1.0 / sqrt(orc_d2(xyz, m, q, k));
            const double* sk = spfh + (int64_t)k * D;
            for (int i = 0; i < D; ++i) acc[i] = acc[i] + w * sk[i];
        }
        const double* sq = spfh + q * D;
        if (Pq[q] == 0) {
            for (int i = 0; i < D; ++i) out[i] = sq[i];
            continue;
        }
        double inv = 1.0 / (double)Pq[q];
        for (int i = 0; i < D; ++i) out[i] = sq[i] + inv * acc[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Mutual nearest-neighbour matching (Section III-C, reciprocity test)       */
/* ------------------------------------------------------------------------ */

/* D(i, j) = sum_t ((double)x_it - (double)y_jt)^2 in dimension order. */
static double orc_desc_d2(const float* x, const float* y, int dim) {
    double acc = 0.0;
    for (int t = 0; t < dim; ++t) {
        double df = (double)x[t] - (double)y[t];
        acc = acc + df * df;
    }
    return acc;
}

/* For each row i in rows[0..nr) of X (nx x dim, row-major), the nearest row of
 * Y (ny x dim) under D, ties to the smaller index; best = D at nn, second = the
 * second-smallest D over j != nn (+inf if ny < 2).  nn = -1 when ny == 0. */
void orc_nn_rows(const float* X, const float* Y, int64_t ny, int dim, const int64_t* rows, int64_t nr,
                 int32_t* nn, double* best, double* second) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; ++r) {
        const float* x = X + rows[r] * dim;
        double b1 = INFINITY, b2 = INFINITY;
        int32_t j1 = -1;
        for (int64_t j = 0; j < ny; ++j) {
            double d = orc_desc_d2(x, Y + j * dim, dim);
            if (d < b1) {
                b2 = b1;
                b1 = d;
                j1 = (int32_t)j;
            } else if (d < b2) {
                b2 = d;
            }
        }
        nn[r] = j1;
        best[r] = b1;
        second[r] = b2;
    }
}
