"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests re-types an oracle formula: each compares the oracle with
a brute force, a library routine, a hand-derived closed form (tests/golden),
or an invariant that a dropped term, a wrong sign or index, or a transposed
operand would break.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Voxelization (Section III-A: voxelized inputs; lowest-index representative)
# ---------------------------------------------------------------------------

def test_voxelize_matches_dict_brute_force(orc):
    rng = np.random.default_rng(7)
    for trial in range(4):
        n = 3000
        pts = rng.uniform(-3, 3, (n, 3)).astype(np.float32)
        if trial == 1:
            pts[::7] = pts[3::7][: pts[::7].shape[0]]  # duplicates
        if trial == 2:
            pts[5] = np.nan
            pts[9, 1] = np.inf
        v = [0.25, 0.5, 0.1, 1.0][trial]
        first = {}
        for i, p in enumerate(pts):
            if not np.all(np.isfinite(p)):
                continue
            key = tuple(math.floor(float(c) / v) for c in p)
            first.setdefault(key, i)
        expect = np.array(sorted(first.values()), np.int32)
        kept, keys = orc.voxelize(pts.T, v)
        np.testing.assert_array_equal(kept, expect)
        for j in range(0, kept.size, 97):
            assert tuple(keys[:, j]) == tuple(math.floor(float(c) / v) for c in pts[kept[j]])


def test_voxelize_half_offset_lattice_keeps_every_point(orc):
    v = 0.125
    g = (np.arange(-6, 6) + 0.5) * v
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()]).astype(np.float32)
    perm = np.random.default_rng(3).permutation(pts.shape[1])
    pts = np.ascontiguousarray(pts[:, perm])
    kept, _ = orc.voxelize(pts, v)
    np.testing.assert_array_equal(kept, np.arange(pts.shape[1]))
    # two copies of the lattice: only the first copy (lower indices) survives
    both = np.ascontiguousarray(np.concatenate([pts, pts + np.float32(0.01)], axis=1))
    kept2, _ = orc.voxelize(both, v)
    np.testing.assert_array_equal(kept2, np.arange(pts.shape[1]))


def test_voxelize_empty(orc):
    kept, keys = orc.voxelize(np.zeros((3, 0), np.float32), 0.1)
    assert kept.size == 0 and keys.shape == (3, 0)


# ---------------------------------------------------------------------------
# Radius search (Eq. A1: strict <, the query included)
# ---------------------------------------------------------------------------

def test_radius_search_matches_kdtree(orc):
    rng = np.random.default_rng(11)
    pts = rng.uniform(0, 2, (1500, 3)).astype(np.float32)
    r = 0.23
    off, idx = orc.radius_search(pts.T, r)
    tree = cKDTree(pts.astype(np.float64))
    d_all = tree.query_ball_point(pts.astype(np.float64), r + 1e-6)
    for q in range(pts.shape[0]):
        mine = set(idx[off[q]:off[q + 1]].tolist())
        lib = set(d_all[q])
        # points within 1e-9 relative of the sphere are decided by the strict FP64 test only
        diff = mine.symmetric_difference(lib)
        for s in diff:
            dist = np.linalg.norm(pts[s].astype(np.float64) - pts[q].astype(np.float64))
            assert abs(dist - r) < 1e-6, (q, s, dist)
        assert q in mine
        lst = idx[off[q]:off[q + 1]]
        assert np.all(np.diff(lst) > 0), "lists are ascending"


def test_radius_search_strict_boundary_and_symmetry(orc):
    r = 0.25  # exactly representable: a point at exactly r along an axis is excluded
    pts = np.array([[0, 0, 0], [0.25, 0, 0], [0, -0.25, 0], [0.2499999, 0, 0], [0, 0, 0.125], [1, 1, 1]],
                   np.float32)
    off, idx = orc.radius_search(pts.T, r)
    n0 = set(idx[off[0]:off[1]].tolist())
    assert n0 == {0, 3, 4}
    rng = np.random.default_rng(5)
    p = rng.uniform(0, 1, (600, 3)).astype(np.float32)
    off, idx = orc.radius_search(p.T, 0.15)
    sets = [set(idx[off[q]:off[q + 1]].tolist()) for q in range(600)]
    for q in range(600):
        assert q in sets[q]
        for s in sets[q]:
            assert q in sets[s]


# ---------------------------------------------------------------------------
# PCA normals (Algorithm 1, Step 1)
# ---------------------------------------------------------------------------

def test_jacobi_matches_numpy_eigh(orc):
    rng = np.random.default_rng(2)
    for trial in range(200):
        A = rng.standard_normal((3, 3))
        C = A @ A.T
        if trial % 5 == 0:
            C[2, :] = C[:, 2] = 0.0  # planar: one zero eigenvalue
        if trial % 7 == 0:
            Q = np.linalg.qr(rng.standard_normal((3, 3)))[0]
            C = Q @ np.diag([2.0, 1.0, 1.0]) @ Q.T  # repeated eigenvalue
        lam, vec = orc.eig3(C)
        ref_lam, ref_vec = np.linalg.eigh(C)
        np.testing.assert_allclose(lam, ref_lam[::-1], rtol=1e-12, atol=1e-12 * abs(ref_lam).max())
        for i in range(3):
            np.testing.assert_allclose(C @ vec[i], lam[i] * vec[i], atol=1e-11 * abs(ref_lam).max())
        np.testing.assert_allclose(vec @ vec.T, np.eye(3), atol=1e-12)


def test_plane_normals_are_exact_and_face_the_viewpoint(orc):
    rng = np.random.default_rng(4)
    pts = np.zeros((3, 800), np.float32)
    pts[0] = rng.uniform(0, 1, 800)
    pts[1] = rng.uniform(0, 1, 800)
    for vp, sign in (([0.5, 0.5, 2.0], 1.0), ([0.5, 0.5, -2.0], -1.0)):
        off, idx = orc.radius_search(pts, 0.12)
        nr = orc.normals(pts, off, idx, 0.08, 3, 0.99, np.array(vp))
        ok = nr["B"].astype(bool)
        assert ok.sum() > 700
        np.testing.assert_array_equal(nr["normals"][2, ok], sign)
        np.testing.assert_array_equal(nr["normals"][:2, ok], 0.0)


def test_strip_linearity_and_filter(orc):
    """A uniform strip of width w and length L has p_lin -> 1 - (w/L)^2, the linearity
    filter keeps p_lin < tau_lin (Section III-C), and collinear points are dropped."""
    rng = np.random.default_rng(8)
    for wl, keep in ((0.05, False), (0.2, True)):
        n = 20000
        pts = np.zeros((3, n), np.float32)
        pts[0] = rng.uniform(-1, 1, n)
        pts[1] = rng.uniform(-wl, wl, n)
        off = np.array([0, n], np.int64)
        idx = np.arange(n, dtype=np.int32)
        # single query at the origin whose neighbour list is the whole strip
        q = np.concatenate([np.zeros((3, 1), np.float32), pts], axis=1)
        off = np.array([0, n + 1] + [n + 1] * n, np.int64)
        idx = np.arange(n + 1, dtype=np.int32)
        nr = orc.normals(q, off, idx, 10.0, 3, 0.99, np.array([0, 0, 1.0]))
        assert abs(nr["plin"][0] - (1 - wl * wl)) < 2e-3
        assert bool(nr["B"][0]) == keep
    line = np.zeros((3, 50), np.float32)
    line[0] = np.linspace(0, 1, 50)
    off, idx = orc.radius_search(line, 0.2)
    nr = orc.normals(line, off, idx, 0.2, 3, 0.99, np.array([0, 0, 1.0]))
    assert nr["B"].sum() == 0


def test_cardinality_filters(orc):
    """Fewer than tau_num points in N(q) or in the r_normal subset -> no normal (Algorithm 1)."""
    pts = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [5, 5, 5], [5.5, 5, 5], [5, 5.5, 5]], np.float32).T.copy()
    off, idx = orc.radius_search(pts, 1.0)
    nr = orc.normals(pts, off, idx, 0.2, 3, 0.99, np.array([0, 0, 1.0]))
    assert nr["n_normal"].tolist() == [3, 3, 3, 1, 1, 1]
    assert nr["B"].tolist() == [1, 1, 1, 0, 0, 0]
    nr4 = orc.normals(pts, off, idx, 0.2, 4, 0.99, np.array([0, 0, 1.0]))
    assert nr4["B"].sum() == 0


def test_four_point_golden(orc):
    g = _gold("four_points.json")
    pts = np.array(g["points"], np.float32).T.copy()
    off, idx = orc.radius_search(pts, g["r_fpfh"])
    nr = orc.normals(pts, off, idx, g["r_normal"], g["tau_num"], g["tau_lin"], np.array(g["viewpoint"]))
    np.testing.assert_allclose(nr["plin"], g["plin"], rtol=1e-14)
    np.testing.assert_allclose(nr["normals"].T, np.tile(g["normal"], (4, 1)), atol=1e-15)
    sp = orc.spfh(pts, nr["normals"], off, idx, nr["B"], g["tau_num"], g["H"])
    fp = orc.fpfh(pts, off, idx, nr["B"], sp["J"], sp["spfh"], sp["Pq"], g["H"])
    sup = g["spfh_support"]
    for q in range(4):
        expect = np.zeros(33)
        expect[sup] = 100.0
        np.testing.assert_allclose(sp["spfh"][q], expect, atol=1e-12)
        e2 = np.zeros(33)
        e2[sup] = g["fpfh_support_value"][q]
        np.testing.assert_allclose(fp[q], e2, rtol=1e-13, atol=1e-12)


# ---------------------------------------------------------------------------
# Angular features and bins (Eq. A2, Eq. A3)
# ---------------------------------------------------------------------------

def test_pair_feature_golden(orc):
    g = _gold("pair_features.json")
    lo = np.array([-math.pi, -1.0, -1.0])
    for c in g["cases"]:
        f = orc.pair_features(c["pq"], c["nq"], c["pk"], c["nk"])
        np.testing.assert_allclose(f, c["f"], atol=1e-15)
        bins = [int(min(10, max(0, math.floor(11 * (f[l] - lo[l]) / (2 * -lo[l]))))) for l in range(3)]
        assert bins == c["bins"]
        f2 = orc.pair_features(c["pk"], c["nk"], c["pq"], c["nq"])
        if c.get("query_dependent"):
            # an exact tie of the two angles makes the query the point a
            np.testing.assert_allclose(f2, c["f_swapped"], atol=1e-15)
        else:
            # otherwise the features do not depend on which point is the query
            np.testing.assert_allclose(f2, f, atol=1e-15)


def test_degenerate_frame_spfh(orc):
    """Normals along the connecting line (Eq. A2 with d x u = 0): f = (0, 0, u.d) with
    u.d = +1 toward a neighbour ahead of q along its normal and -1 behind it.  f3 = 1 is
    the top of the range, whose scaled value H (f - lo) / (hi - lo) is exactly H: it lands
    in the last bin (Eq. A3, clamped)."""
    pts = np.zeros((3, 3), np.float32)
    pts[0] = [0.0, 1.0, 2.0]
    nrm = np.zeros((3, 3))
    nrm[0] = 1.0
    off, idx = orc.radius_search(pts, 5.0)
    sp = orc.spfh(pts, nrm, off, idx, np.ones(3, np.uint8), 3, 11)
    for q, (behind, ahead) in enumerate([(0, 2), (1, 1), (2, 0)]):
        cnt = np.zeros(33, np.int32)
        cnt[5] = cnt[16] = 2
        cnt[22] += behind
        cnt[32] += ahead
        np.testing.assert_array_equal(sp["counts"][q], cnt)


@pytest.mark.parametrize("inward", [True, False])
def test_sphere_closed_form(orc, inward):
    """Points on a sphere of radius R with radial normals: chord c, phi = 2 asin(c / 2R);
    inward normals give f = (-phi, 0, c/2R), outward normals f = (phi, 0, -c/2R)."""
    rng = np.random.default_rng(12)
    R = 0.7
    ctr = np.array([0.3, -0.2, 1.1])
    for _ in range(300):
        a = rng.standard_normal(3)
        a /= np.linalg.norm(a)
        b = a + 0.6 * rng.standard_normal(3)
        b /= np.linalg.norm(b)
        pq, pk = ctr + R * a, ctr + R * b
        nq, nk = (-a, -b) if inward else (a, b)
        c = np.linalg.norm(pk - pq)
        phi = 2 * math.asin(c / (2 * R))
        f = orc.pair_features(pq, nq, pk, nk)
        expect = (-phi, 0.0, c / (2 * R)) if inward else (phi, 0.0, -c / (2 * R))
        np.testing.assert_allclose(f, expect, atol=1e-12)


def test_collinear_closed_form(orc):
    """Points on a line e with unit normals n = sin(t) e + cos(t) m (m a unit vector normal
    to e): n . d0 = +-sin(t), so a is the point of larger |sin t|, and Eq. A2 reduces to
    f = (s (t_b - t_a), 0, s sin t_a) with s the sign of the step from a to b along e."""
    rng = np.random.default_rng(17)
    for _ in range(400):
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        m = np.cross(e, rng.standard_normal(3))
        m /= np.linalg.norm(m)
        o = rng.uniform(-2, 2, 3)
        xq, xk = rng.uniform(-1, 1, 2)
        tq, tk = rng.uniform(-1.5, 1.5, 2)
        pq, pk = o + xq * e, o + xk * e
        nq = math.sin(tq) * e + math.cos(tq) * m
        nk = math.sin(tk) * e + math.cos(tk) * m
        if abs(math.sin(tq)) >= abs(math.sin(tk)):
            (xa, ta), (xb, tb) = (xq, tq), (xk, tk)
        else:
            (xa, ta), (xb, tb) = (xk, tk), (xq, tq)
        s = 1.0 if xb > xa else -1.0
        f = orc.pair_features(pq, nq, pk, nk)
        np.testing.assert_allclose(f, (s * (tb - ta), 0.0, s * math.sin(ta)), atol=1e-12)


def test_collinear_fpfh_golden(orc):
    """Four collinear points with given normals whose SPFH rows all differ: the hand-derived
    SPFH counts (Eq. A2-A4) and FPFH rows (Eq. A5) of tests/golden/collinear_fpfh.json.
    Every neighbour contributes its own SPFH row, weighted by 1 / distance."""
    g = _gold("collinear_fpfh.json")
    n = len(g["x"])
    pts = np.zeros((3, n), np.float32)
    pts[0] = g["x"]
    t = np.radians(g["normal_angle_deg"])
    nrm = np.stack([np.sin(t), np.zeros(n), np.cos(t)])
    off, idx = orc.radius_search(pts, g["r"])
    assert np.array_equal(np.diff(off), [n] * n)
    B = np.ones(n, np.uint8)
    H = g["H"]
    sp = orc.spfh(pts, nrm, off, idx, B, g["tau_num"], H)
    assert sp["J"].tolist() == [1] * n and sp["Pq"].tolist() == [n - 1] * n
    c = 100.0 / (n - 1)
    for q in range(n):
        cnt = np.zeros(3 * H, np.int32)
        for b, v in g["spfh_counts"][q].items():
            cnt[int(b)] = v
        np.testing.assert_array_equal(sp["counts"][q], cnt)
        np.testing.assert_allclose(sp["spfh"][q], c * cnt, rtol=1e-15, atol=0)
    fp = orc.fpfh(pts, off, idx, B, sp["J"], sp["spfh"], sp["Pq"], H)
    for q in range(n):
        expect = np.zeros(3 * H)
        for b, (num, den) in g["fpfh_over_c"][q].items():
            expect[int(b)] = c * num / den
        np.testing.assert_allclose(fp[q], expect, rtol=1e-13, atol=1e-12)


def test_orientation_exact_zero(orc):
    """Normal sign (viewpoint rule with the exact-zero convention): on planes through the
    viewpoint n . (vp - a_q) is often exactly 0; there the first nonzero component of n is
    positive, elsewhere n . (vp - a_q) > 0.  Axis planes give n = +e exactly."""
    rng = np.random.default_rng(3)
    n = 300
    ties = 0
    for (i, j), s in [((0, 1), 1), ((0, 1), -1), ((0, 2), 1), ((0, 2), -1), ((1, 2), 1), ((1, 2), -1)]:
        k = 3 - i - j
        t = rng.uniform(-1, 1, n).astype(np.float32)
        f = rng.uniform(-1, 1, n).astype(np.float32)
        xyz = np.zeros((3, n), np.float32)
        xyz[i], xyz[j], xyz[k] = t, s * t, f
        vp = np.zeros(3)
        vp[i], vp[j], vp[k] = 0.7, s * 0.7, 3.0
        off, idx = orc.radius_search(xyz, 0.3)
        nr = orc.normals(xyz, off, idx, 0.3, 3, 0.99, vp)
        ok = nr["B"] == 1
        assert ok.sum() == n
        nn = nr["normals"]
        to_vp = vp[:, None] - xyz.astype(np.float64)
        dot = (nn[0] * to_vp[0] + nn[1] * to_vp[1]) + nn[2] * to_vp[2]
        assert np.all(dot >= 0.0)
        zero = dot == 0.0
        ties += int(zero.sum())
        for q in np.nonzero(zero)[0]:
            first = nn[np.nonzero(nn[:, q])[0][0], q]
            assert first > 0.0, ((i, j, s), q, nn[:, q])
    assert ties >= 700
    for axis in range(3):
        xyz = np.ascontiguousarray(rng.uniform(-1, 1, (3, n)).astype(np.float32))
        xyz[axis] = 0.0
        vp = np.array([0.4, -0.9, 0.6])
        vp[axis] = 0.0
        off, idx = orc.radius_search(xyz, 0.3)
        nr = orc.normals(xyz, off, idx, 0.3, 3, 0.99, vp)
        ok = nr["B"] == 1
        assert ok.sum() > 0.9 * n
        expect = np.zeros(3)
        expect[axis] = 1.0
        np.testing.assert_array_equal(nr["normals"][:, ok].T, np.tile(expect, (int(ok.sum()), 1)))


def test_bin_map(orc):
    lib = orc.load()
    import ctypes

    e = ctypes.c_int(0)
    assert lib.orc_bin(math.pi, -math.pi, math.pi, 11, ctypes.byref(e)) == 10  # f = max -> last bin
    assert lib.orc_bin(-math.pi, -math.pi, math.pi, 11, ctypes.byref(e)) == 0
    assert lib.orc_bin(-1.0 + 2.0 / 11 * 3, -1.0, 1.0, 11, ctypes.byref(e)) in (2, 3) and e.value == 1
    assert lib.orc_bin(0.0, -1.0, 1.0, 11, ctypes.byref(e)) == 5 and e.value == 0
    for h in range(11):
        f = -1.0 + (h + 0.5) * 2.0 / 11
        assert lib.orc_bin(f, -1.0, 1.0, 11, None) == h


# ---------------------------------------------------------------------------
# SPFH / FPFH invariants (Eq. A4, A5) and Algorithm 1 Step 2
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c0_src(orc):
    d = synth.c0_pair(0)
    p = d["params"]
    kept, _ = orc.voxelize(d["src"], p.voxel)
    xyz = np.ascontiguousarray(d["src"][:, kept])
    return xyz, p, d["vp_src"], orc.faster_pfh(xyz, p, d["vp_src"], boundary_fp32=False)


def test_spfh_subhistograms_sum_to_100(c0_src):
    xyz, p, vp, fp = c0_src
    H = p.n_bins
    has = fp["Pq"] > 0
    assert has.sum() > 1000
    for l in range(3):
        s = fp["spfh"][has, l * H:(l + 1) * H].sum(1)
        np.testing.assert_allclose(s, 100.0, rtol=1e-12)
        np.testing.assert_array_equal(fp["counts"][has, l * H:(l + 1) * H].sum(1), fp["Pq"][has])


def test_fpfh_subhistogram_sums(c0_src):
    """Each FPFH sub-histogram sums to 100 (1 + (1/P_q) sum_k 1/w_k) over valid k != q."""
    xyz, p, vp, fp = c0_src
    H = p.n_bins
    P = xyz.T.astype(np.float64)
    J = np.nonzero(fp["J"])[0]
    for q in J[:: max(1, J.size // 400)]:
        nb = fp["idx"][fp["off"][q]:fp["off"][q + 1]]
        nb = nb[(nb != q) & (fp["B"][nb] == 1)]
        s = 100.0 * (1.0 + np.sum(1.0 / np.linalg.norm(P[nb] - P[q], axis=1)) / fp["Pq"][q])
        for l in range(3):
            np.testing.assert_allclose(fp["fpfh"][q, l * H:(l + 1) * H].sum(), s, rtol=1e-12)


def test_step2_single_pass(c0_src):
    """J = B and |M[q]| >= tau_num with M[q] = N(q) restricted to B (Algorithm 1, Step 2)."""
    xyz, p, vp, fp = c0_src
    for q in range(xyz.shape[1]):
        nb = fp["idx"][fp["off"][q]:fp["off"][q + 1]]
        nm = int(fp["B"][nb].sum())
        assert fp["J"][q] == (fp["B"][q] == 1 and nm >= p.tau_num)
        if fp["B"][q]:
            assert fp["Pq"][q] == nm - 1


def test_rigid_invariance(orc, c0_src):
    """Descriptors of a rigidly moved cloud (viewpoint moved with it) are unchanged,
    except where a bin decision sits on an edge within the rounding of the move."""
    xyz, p, vp, fp = c0_src
    rng = np.random.default_rng(21)
    R = synth.random_rotation(rng)
    t = rng.uniform(-1, 1, 3)
    xyz2 = (R @ xyz.astype(np.float64) + t[:, None]).astype(np.float32)
    fp2 = orc.faster_pfh(np.ascontiguousarray(xyz2), p, R @ vp + t, boundary_fp32=False)
    same_nbrs = np.array([np.array_equal(fp["idx"][fp["off"][q]:fp["off"][q + 1]],
                                         fp2["idx"][fp2["off"][q]:fp2["off"][q + 1]]) for q in range(xyz.shape[1])])
    assert same_nbrs.mean() > 0.99
    np.testing.assert_array_equal(fp["B"][same_nbrs], fp2["B"][same_nbrs])
    both = (fp["J"] == 1) & (fp2["J"] == 1) & same_nbrs
    err = np.abs(fp["fpfh"][both] - fp2["fpfh"][both]).max(axis=1)
    scale = fp["fpfh"][both, :11].sum(1) / 100.0
    close = err <= 1e-3 * scale
    assert close.mean() > 0.97, close.mean()


# ---------------------------------------------------------------------------
# Mutual matching (reciprocity test) and pose recovery
# ---------------------------------------------------------------------------

def test_nn_matches_brute_force(orc):
    rng = np.random.default_rng(31)
    X = rng.integers(0, 5, (300, 33)).astype(np.float32)  # small integers: many exact ties
    Y = rng.integers(0, 5, (250, 33)).astype(np.float32)
    D = ((X.astype(np.float64)[:, None, :] - Y.astype(np.float64)[None, :, :]) ** 2).sum(-1)
    nn, best, second = orc.nn_rows(X, Y)
    np.testing.assert_array_equal(nn, np.argmin(D, axis=1))  # argmin: first (smallest) index on ties
    np.testing.assert_array_equal(best, D.min(1))
    np.testing.assert_array_equal(second, np.sort(D, axis=1)[:, 1])
    mm = orc.mutual_match(X, Y)
    nyx = np.argmin(D, axis=0)
    ref = [(i, j) for i, j in enumerate(np.argmin(D, axis=1)) if nyx[j] == i]
    assert [tuple(p) for p in mm["pairs"]] == ref


def test_self_match_pin(orc):
    """Matching a set against itself gives (i, i) for the smallest index of each class of
    identical rows."""
    rng = np.random.default_rng(6)
    X = rng.uniform(0, 50, (400, 33)).astype(np.float32)
    X[100:110] = X[5]
    X[300] = X[299]
    mm = orc.mutual_match(X, X)
    expect = [i for i in range(400) if not (100 <= i < 110) and i != 300]
    assert mm["pairs"][:, 0].tolist() == expect
    assert mm["pairs"][:, 1].tolist() == expect


def test_empty_match(orc):
    X = np.zeros((0, 33), np.float32)
    Y = np.ones((5, 33), np.float32)
    assert orc.mutual_match(X, Y)["pairs"].shape == (0, 2)
    assert orc.mutual_match(Y, X)["pairs"].shape == (0, 2)


def test_exact_transform_recovery(orc):
    """Noiseless pre-voxelized pair (target = exact rigid image of the source, permuted):
    Faster-PFH, mutual matching, Eq. (3) graph, max k-core and GNC recover (R, t)."""
    from oracle import pose

    d = synth.lattice_pair(0)
    p = d["params"]
    a = orc.faster_pfh(d["src"], p, d["vp_src"])
    b = orc.faster_pfh(d["tgt"], p, d["vp_tgt"])
    X = a["fpfh"][a["j_idx"]].astype(np.float32)
    Y = b["fpfh"][b["j_idx"]].astype(np.float32)
    mm = orc.mutual_match(X, Y)
    pairs = np.stack([a["j_idx"][mm["pairs"][:, 0]], b["j_idx"][mm["pairs"][:, 1]]], 1)
    correct = d["perm"][pairs[:, 1]] == pairs[:, 0]
    assert correct.sum() >= 30
    R, t, n_inl = pose.register(d["src"], d["tgt"], pairs, mm["d1"], mm["d2"], p.voxel)
    ang = math.acos(max(-1.0, min(1.0, (np.trace(R.T @ d["R"]) - 1) / 2)))
    assert ang < 1e-5, ang
    assert np.linalg.norm(t - d["t"]) < 1e-5
    assert n_inl >= 30


def test_unrelated_pair_has_few_inliers(orc):
    """An unrelated pair yields a small final inlier set (Section III-E validity check)."""
    from oracle import pose

    d0 = synth.lattice_pair(0)
    d1 = synth.lattice_pair(1, spacing=0.06)
    p = d0["params"]
    a = orc.faster_pfh(d0["src"], p, d0["vp_src"])
    rng = np.random.default_rng(1)
    junk = np.ascontiguousarray(rng.uniform(-1, 3, d1["src"].shape).astype(np.float32))
    b = orc.faster_pfh(junk, p, np.array([1.0, 1.0, 5.0]))
    X = a["fpfh"][a["j_idx"]].astype(np.float32)
    Y = b["fpfh"][b["j_idx"]].astype(np.float32)
    if Y.shape[0] == 0:
        return
    mm = orc.mutual_match(X, Y)
    pairs = np.stack([a["j_idx"][mm["pairs"][:, 0]], b["j_idx"][mm["pairs"][:, 1]]], 1)
    if len(pairs) < 3:
        return
    _, _, n_inl = pose.register(d0["src"], junk, pairs, mm["d1"], mm["d2"], p.voxel)
    assert n_inl < 30


def test_grid_radius_search_equals_brute_force(orc):
    """The grid form of the radius search (cell size r) returns exactly the brute-force
    sets of Eq. A1, including points at exactly r, on cell faces and far from the origin."""
    rng = np.random.default_rng(23)
    r = 0.25
    clouds = [rng.uniform(0, 2, (3, 3000)).astype(np.float32),
              (rng.uniform(-1, 1, (3, 2000)) + 400.0).astype(np.float32),
              (np.round(rng.uniform(-1, 1, (3, 2500)) * 8) / 8).astype(np.float32)]  # lattice at r / 2
    axis = np.zeros((3, 9), np.float32)
    axis[0] = np.arange(9) * 0.25  # neighbours at exactly r: excluded (strict)
    clouds.append(axis)
    for xyz in clouds:
        xyz = np.ascontiguousarray(xyz)
        ob, ib = orc.radius_search(xyz, r)
        og, ig = orc.radius_search(xyz, r, grid=True)
        np.testing.assert_array_equal(og, ob)
        np.testing.assert_array_equal(ig, ib)
    assert np.array_equal(np.diff(og), [1] * 9)
