"""Pins for the float64 Maximus reference (CPU only).

Checks the reference index against what Section III fixes: the bound of
Eq. (appx_bound) in hand-worked cases, the bound never falls below
u.i/||u|| for users of the cluster, the lists are monotone, and the walk
returns exactly the brute-force top-K (the paper's exactness argument), also
in the degenerate cases C = n_u (theta_b = 0) and theta_b = pi (norm order).
"""
import json
import os

import numpy as np
import pytest

import mipsgen
from oracle import maximus as M
from oracle import topk as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_bound_golden_values():
    with open(os.path.join(GOLDEN, "maximus_bound_example.json")) as fh:
        g = json.load(fh)
    b = M.cbound(np.array(g["centroid"], float), np.array(g["items"], float), g["theta_b"])
    np.testing.assert_allclose(b, g["expected_bound"], rtol=1e-15, atol=1e-15)


def test_stable_angle_special_values():
    a = np.array([[1.0, 0.0], [1.0, 0.0], [1.0, 0.0], [1.0, 1e-9], [3.0, 4.0]])
    b = np.array([[0.0, 5.0], [-2.0, 0.0], [7.0, 0.0], [1.0, 0.0], [-4.0, 3.0]])
    ang = M.stable_angle(a, b)
    np.testing.assert_allclose(ang, [np.pi / 2, np.pi, 0.0, 1e-9, np.pi / 2], rtol=1e-12, atol=1e-300)
    # arccos of a rounded cosine would give ~1.5e-8 for the 1e-9 case
    assert abs(ang[3] - 1e-9) < 1e-20


def _lemma_and_property(U, I, ix):
    U64 = U.astype(np.float64)
    un = np.linalg.norm(U64, axis=1)
    f = U.shape[1]
    worst = 0.0
    for u in range(U.shape[0]):
        j = ix["assign"][u]
        keys = T.user_keys(U[u], I)
        lhs = un[u] * ix["bounds"][j]
        slack = M.stop_slack(f) * un[u] * np.linalg.norm(I.astype(np.float64), axis=1).max()
        worst = max(worst, float((keys - lhs).max()) / (slack + 1e-300))
        assert np.all(lhs * (1 + M.stop_slack(f)) + slack >= keys)
    for j in range(ix["bounds"].shape[0]):
        b = ix["bounds"][j][ix["lists"][j]]
        assert np.all(np.diff(b) <= 0)
    return worst


@pytest.mark.parametrize("C", [1, 3, 8])
def test_lemma_property_theorem_tiny(oracle_lib, C):
    U, I = mipsgen.generate("clustered", 2, n_users=200, n_items=500, f=12)
    ix = M.build_index(U, I, C, iters=3, seed=1)
    # user-centroid angles never exceed theta_b
    ang = M.stable_angle(U, ix["centroids"][ix["assign"]])
    assert np.all(ang <= ix["theta_b"][ix["assign"]])
    _lemma_and_property(U, I, ix)
    for K in (1, 10, 37):
        idx, key, w = M.query(ix, U, I, K)
        ri, rk = T.topk(U, I, K)
        np.testing.assert_array_equal(idx, ri)
        np.testing.assert_array_equal(key, rk)


def test_theorem_clustered_workload_shape(oracle_lib):
    U, I = mipsgen.generate("clustered", 0, n_users=1500, n_items=4000)
    for C in (8, 64):
        ix = M.build_index(U, I, C, iters=3, seed=0)
        idx, key, w = M.query(ix, U, I, 10)
        ri, rk = T.topk(U, I, 10)
        np.testing.assert_array_equal(idx, ri)
        # pruning really happens on this data
        assert w.mean() < 0.25 * I.shape[0]


def test_singleton_clusters_theta_zero(oracle_lib):
    U, I = mipsgen.generate("mf", 3, n_users=40, n_items=600, f=10)
    ix = M.build_index(U, I, C=40, iters=2, seed=0)
    assert np.all(ix["theta_b"] < 1e-7)
    # with theta_b = 0 the bound is u.i/||u||: the walk stops right after the K-th item
    idx, key, w = M.query(ix, U, I, 5)
    ri, _ = T.topk(U, I, 5)
    np.testing.assert_array_equal(idx, ri)
    assert w.max() <= 5 + 3


def test_theta_pi_is_norm_order(oracle_lib):
    U, I = mipsgen.generate("mf", 4, n_users=50, n_items=400, f=8)
    ix = M.build_index(U, I, C=4, iters=2, seed=0, force_theta_pi=True)
    inorm = np.linalg.norm(I.astype(np.float64), axis=1)
    for j in range(4):
        np.testing.assert_allclose(ix["bounds"][j], inorm, rtol=1e-15)
        np.testing.assert_array_equal(ix["lists"][j], np.lexsort((np.arange(400), -inorm)))
    idx, _, _ = M.query(ix, U, I, 7)
    np.testing.assert_array_equal(idx, T.topk(U, I, 7)[0])


def test_zero_users_and_duplicate_items(oracle_lib):
    U, I = mipsgen.generate("clustered", 5, n_users=120, n_items=300, f=6)
    U[7] = 0.0
    U[50] = 0.0
    I[10] = I[20]
    I[100] = I[20]
    ix = M.build_index(U, I, C=5, iters=3, seed=3)
    idx, key, _ = M.query(ix, U, I, 12)
    ri, rk = T.topk(U, I, 12)
    np.testing.assert_array_equal(idx, ri)
    np.testing.assert_array_equal(idx[7], np.arange(12))


def test_kmeans_objective_non_increasing():
    U, _ = mipsgen.generate("clustered", 6, n_users=800, n_items=10, f=8)
    prev = np.inf
    for it in range(0, 5):
        c, a = M.kmeans(U, 16, it, seed=2)
        obj = ((U.astype(np.float64) - c[a]) ** 2).sum()
        assert obj <= prev * (1 + 1e-12)
        prev = obj
