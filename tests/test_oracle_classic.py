"""Pins of the oracle's classical FPFH mode (Section III-C, Fig. 3a): normals
from the r_normal neighbourhood with no linearity filter, a descriptor for
every point with a normal."""

import numpy as np

import synth


def kept_cloud(orc, d):
    kept, _ = orc.voxelize(d["src"], d["params"].voxel)
    return np.ascontiguousarray(d["src"][:, kept])


def test_classic_J_is_every_point_with_a_normal(orc):
    d = synth.c0_pair(0)
    xyz = kept_cloud(orc, d)
    out = orc.faster_pfh(xyz, d["params"], d["vp_src"], classical=True)
    np.testing.assert_array_equal(out["J"], out["B"])
    # B: at least 3 points within r_normal (q included) and a non-degenerate normal
    assert np.all(out["n_normal"][out["B"] == 1] >= 3)
    assert np.all(out["plin"][out["B"] == 1] < 1.0)


def test_classic_equals_faster_pfh_without_filters(orc):
    """With tau_num = 3 and tau_lin = 1 the two modes share normals, B and
    SPFH; FPFH agrees on every point the Faster-PFH J keeps."""
    d = synth.c0_pair(1)
    xyz = kept_cloud(orc, d)
    p = d["params"]
    unfiltered = synth.Params(voxel=p.voxel, r_normal=p.r_normal, r_fpfh=p.r_fpfh, tau_num=3, tau_lin=1.0,
                              n_bins=p.n_bins)
    a = orc.faster_pfh(xyz, unfiltered, d["vp_src"])
    b = orc.faster_pfh(xyz, p, d["vp_src"], classical=True)
    np.testing.assert_array_equal(a["B"], b["B"])
    np.testing.assert_array_equal(a["spfh"], b["spfh"])
    assert np.all(b["J"][a["J"] == 1] == 1)
    np.testing.assert_array_equal(a["fpfh"][a["J"] == 1], b["fpfh"][a["J"] == 1])
    assert b["J"].sum() >= a["J"].sum()


def test_classic_keeps_what_faster_pfh_filters(orc):
    """A collinear-ish strip (high linearity) and sparse points: Faster-PFH
    drops them, the classical mode describes every point with 3+ normal
    neighbours."""
    rng = np.random.default_rng(4)
    strip = np.zeros((3, 400), np.float32)
    strip[0] = rng.uniform(0, 4, 400)
    strip[1] = rng.uniform(0, 0.004, 400)  # width 0.004 over a 0.2 m window: p_lin ~ 0.9996
    p = synth.Params(voxel=0.01, r_normal=0.1, r_fpfh=0.25)
    a = orc.faster_pfh(strip, p, np.array([0, 0, 5.0]))
    b = orc.faster_pfh(strip, p, np.array([0, 0, 5.0]), classical=True)
    assert a["J"].sum() == 0 < b["J"].sum()


def test_classic_plane_closed_form(orc):
    """Coplanar points: every SPFH is 100 at bins 5, 16 and 27 in either mode."""
    rng = np.random.default_rng(5)
    pts = np.zeros((3, 600), np.float32)
    pts[:2] = rng.uniform(0, 2, (2, 600))
    p = synth.Params(voxel=0.01, r_normal=0.15, r_fpfh=0.3)
    out = orc.faster_pfh(pts, p, np.array([0, 0, 1.0]), classical=True)
    has = out["B"] == 1
    expect = np.zeros(33)
    expect[[5, 16, 27]] = 100.0
    rows = out["spfh"][has & (out["Pq"] > 0)]
    np.testing.assert_allclose(rows, np.broadcast_to(expect, rows.shape), atol=1e-9)
