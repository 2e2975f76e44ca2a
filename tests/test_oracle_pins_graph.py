"""Pins of the oracle's ratio filter, Eq. (3) compatibility graph and k-core
(Section III-D) against brute force, closed cases and the definitions."""

import itertools
import math

import numpy as np
import pytest

from oracle import pose


def brute_ratio_order(d1, d2):
    def key(e):
        a, b = float(d1[e]), float(d2[e])
        r = a / b if b > 0 else (math.inf if a > 0 else 0.0)
        return (r, e)

    return sorted(range(len(d1)), key=key)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ratio_filter_matches_sorting(seed):
    rng = np.random.default_rng(seed)
    k = 400
    d2 = rng.uniform(0.5, 2.0, k).astype(np.float32)
    d1 = (d2 * rng.uniform(0.2, 1.0, k)).astype(np.float32)
    # ties: repeated rows, and the two zero conventions
    d1[10:20] = d1[5]
    d2[10:20] = d2[5]
    d1[30], d2[30] = 0.0, 0.0
    d1[31], d2[31] = 0.5, 0.0
    order = brute_ratio_order(d1, d2)
    for n_tau in (1, 7, 100, 400, 1000):
        got = pose.ratio_filter(d1, d2, n_tau)
        assert list(got) == order[:n_tau]


def test_ratio_filter_zero_conventions():
    d1 = np.array([0.0, 0.3, 0.0, 0.1], np.float32)
    d2 = np.array([0.0, 0.0, 0.5, 0.2], np.float32)
    # ratios 0, inf, 0, 0.5: ties keep position order
    assert list(pose.ratio_filter(d1, d2, 4)) == [0, 2, 3, 1]


def test_graph_of_a_rigid_copy_is_complete():
    rng = np.random.default_rng(3)
    a = rng.uniform(-10, 10, (60, 3))
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    b = a @ R.T + np.array([1.0, -2.0, 3.0])
    adj = pose.compat_graph(a, b, 1e-9)
    assert adj.sum() == 60 * 59
    assert not adj.diagonal().any()


def test_graph_boundary_is_inclusive():
    a = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 0, 0]])
    b = np.array([[0.0, 0, 0], [1.5, 0, 0], [0.0, 0, 0]])
    beta = 0.25  # |1.5 - 1.0| = 0.5 = 2 beta exactly: an edge
    adj = pose.compat_graph(a, b, beta)
    assert adj[0, 1] and adj[1, 0]
    b[1, 0] = np.nextafter(1.5, 2.0)
    adj = pose.compat_graph(a, b, beta)
    assert not adj[0, 1] and not adj[1, 0]
    assert adj[0, 2]  # both distances 0


def test_graph_symmetric_and_relabel_invariant():
    rng = np.random.default_rng(4)
    a = rng.uniform(0, 5, (50, 3))
    b = a + rng.normal(0, 0.3, (50, 3))
    adj = pose.compat_graph(a, b, 0.2)
    assert (adj == adj.T).all()
    perm = rng.permutation(50)
    adj_p = pose.compat_graph(a[perm], b[perm], 0.2)
    assert (adj_p == adj[np.ix_(perm, perm)]).all()


def brute_core_numbers(adj):
    """Core number by the definition: the largest k such that v lies in a
    subgraph whose every vertex has degree >= k inside it (the k-core, found
    by removing vertices of degree < k until none is left)."""
    n = adj.shape[0]
    core = np.zeros(n, np.int64)
    for k in range(1, n):
        alive = np.ones(n, bool)
        while True:
            deg = (adj & alive[None, :]).sum(1)
            drop = alive & (deg < k)
            if not drop.any():
                break
            alive &= ~drop
        if not alive.any():
            break
        core[alive] = k
    return core


def graph_from_edges(n, edges):
    adj = np.zeros((n, n), bool)
    for u, v in edges:
        adj[u, v] = adj[v, u] = True
    return adj


@pytest.mark.parametrize("name,n,edges,expect", [
    ("K5", 5, list(itertools.combinations(range(5), 2)), [4] * 5),
    ("star", 6, [(0, i) for i in range(1, 6)], [1] * 6),
    ("cycle", 7, [(i, (i + 1) % 7) for i in range(7)], [2] * 7),
    ("path", 5, [(i, i + 1) for i in range(4)], [1] * 5),
    ("K4+K3+isolated", 8, list(itertools.combinations(range(4), 2)) + list(itertools.combinations(range(4, 7), 2)),
     [3, 3, 3, 3, 2, 2, 2, 0]),
])
def test_core_numbers_closed_cases(name, n, edges, expect):
    adj = graph_from_edges(n, edges)
    assert list(pose.core_numbers(adj)) == expect
    mx = max(expect)
    assert list(pose.max_kcore(adj)) == [v for v in range(n) if expect[v] == mx]


@pytest.mark.parametrize("seed", range(6))
def test_core_numbers_match_definition(seed):
    rng = np.random.default_rng(10 + seed)
    n = 40
    p = [0.05, 0.1, 0.2, 0.4, 0.6, 0.9][seed]
    upper = np.triu(rng.random((n, n)) < p, 1)
    adj = upper | upper.T
    np.testing.assert_array_equal(pose.core_numbers(adj), brute_core_numbers(adj))
