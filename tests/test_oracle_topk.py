"""Pins for the top-K oracle (CPU only).

The oracle's result definition is the brute force of Section II-C evaluated
in float64 with a fixed left-to-right sum and ties to the lower item index.
It is pinned here by things other than itself: exact rational arithmetic on
tiny inputs, an independent numpy evaluation, and closed forms.
"""
from fractions import Fraction
import json
import os

import numpy as np
import pytest

import mipsgen
from oracle import topk as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _exact_rank(U, I, K):
    """Top-K by exact rational scores, ties by lower index."""
    Uf = [[Fraction(float(x)) for x in row] for row in U]
    If = [[Fraction(float(x)) for x in row] for row in I]
    out = []
    exact = []
    for u in Uf:
        s = [sum(a * b for a, b in zip(u, it)) for it in If]
        order = sorted(range(len(If)), key=lambda i: (-s[i], i))
        out.append(order[:K])
        exact.append([s[i] for i in order[:K]])
    return np.array(out, dtype=np.int32), exact


def _tiny_inputs(seed, n_u, n_i, f, ties=True, zeros=True):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n_u, f)).astype(np.float32)
    I = rng.standard_normal((n_i, f)).astype(np.float32)
    if ties and n_i >= 6:
        I[5] = I[2]           # exact duplicate items -> exact ties
        I[n_i - 1] = I[0]
    if zeros:
        U[0] = 0.0            # zero user: all keys 0 -> indices 0..K-1
        if n_i > 3:
            I[3] = 0.0        # zero item
    return U, I


@pytest.mark.parametrize("seed,n_u,n_i,f,K", [
    (0, 12, 40, 8, 5), (1, 9, 33, 1, 7), (2, 16, 64, 16, 10), (3, 5, 20, 3, 20), (4, 7, 50, 31, 1)])
def test_exact_rational_brute_force(oracle_lib, seed, n_u, n_i, f, K):
    U, I = _tiny_inputs(seed, n_u, n_i, f)
    ref_idx, ref_exact = _exact_rank(U, I, K)
    for mode in (0, 1):
        idx, key = T.topk(U, I, K, mode=mode)
        np.testing.assert_array_equal(idx, ref_idx)
        # the FP64 key of a left-to-right sum is within f * 2^-53 * sum|u_j i_j| of the exact value
        for u in range(n_u):
            for k in range(K):
                i = idx[u, k]
                bound = f * 2.0 ** -53 * float(np.abs(U[u].astype(np.float64) * I[i].astype(np.float64)).sum())
                assert abs(Fraction(key[u, k]) - ref_exact[u][k]) <= Fraction(bound)


def test_key_is_left_to_right_sum(oracle_lib):
    # 1 + 2^-53 + 2^-53 summed left to right is 1 (each half-ulp tie rounds to even);
    # summed right to left it is 1 + 2^-52.  Products here are exact.
    u = np.array([1.0, 2.0 ** -27, 2.0 ** -27], dtype=np.float32)
    i = np.array([1.0, 2.0 ** -26, 2.0 ** -26], dtype=np.float32)
    assert T.key(u, i) == 1.0
    assert T.key(u[::-1].copy(), i[::-1].copy()) == 1.0 + 2.0 ** -52


def _numpy_topk(U, I, K):
    """Independent route: FP64 accumulation over j in order, then lexsort."""
    U64 = U.astype(np.float64)
    I64 = I.astype(np.float64)
    acc = np.zeros((U.shape[0], I.shape[0]))
    for j in range(U.shape[1]):
        acc = acc + U64[:, j:j + 1] * I64[None, :, j]
    n_i = I.shape[0]
    idx = np.empty((U.shape[0], K), dtype=np.int32)
    key = np.empty((U.shape[0], K))
    cols = np.arange(n_i)
    for u in range(U.shape[0]):
        order = np.lexsort((cols, -acc[u]))[:K]
        idx[u] = order
        key[u] = acc[u, order]
    return idx, key


@pytest.mark.parametrize("K", [1, 10])
def test_matches_independent_numpy_tiny_workload(oracle_lib, K):
    U, I = mipsgen.generate("tiny", 0)
    ref_idx, ref_key = _numpy_topk(U, I, K)
    for mode in (0, 1):
        idx, key = T.topk(U, I, K, mode=mode)
        np.testing.assert_array_equal(idx, ref_idx)
        np.testing.assert_array_equal(key, ref_key)


def test_full_sort_equals_insertion_list_mf(oracle_lib):
    U, I = mipsgen.generate("mf", 0, n_users=300, n_items=2000)
    for K in (1, 5, 50):
        a, ka = T.topk(U, I, K, mode=0)
        b, kb = T.topk(U, I, K, mode=1)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(ka, kb)


def test_closed_form_f1(oracle_lib):
    rng = np.random.default_rng(5)
    I = rng.integers(-4, 5, size=(30, 1)).astype(np.float32)   # many exact ties
    U = np.array([[2.0], [-0.5], [0.0]], dtype=np.float32)
    K = 12
    idx, _ = T.topk(U, I, K)
    cols = np.arange(30)
    np.testing.assert_array_equal(idx[0], np.lexsort((cols, -I[:, 0]))[:K])
    np.testing.assert_array_equal(idx[1], np.lexsort((cols, I[:, 0]))[:K])
    np.testing.assert_array_equal(idx[2], np.arange(K))


def test_closed_form_identity_items(oracle_lib):
    f = 24
    I = np.eye(f, dtype=np.float32)
    rng = np.random.default_rng(6)
    U = rng.standard_normal((20, f)).astype(np.float32)
    U[3, 5] = U[3, 9] = 10.0   # tie between coordinates 5 and 9
    idx, key = T.topk(U, I, f)
    cols = np.arange(f)
    for u in range(20):
        np.testing.assert_array_equal(idx[u], np.lexsort((cols, -U[u])))
        np.testing.assert_array_equal(key[u], U[u][idx[u]].astype(np.float64))


def test_full_ranking_K_equals_n_items(oracle_lib):
    U, I = mipsgen.generate("tiny", 1, n_users=10, n_items=64)
    idx, key = T.topk(U, I, 64)
    for u in range(10):
        assert sorted(idx[u].tolist()) == list(range(64))
        assert np.all(np.diff(key[u]) <= 0)


def test_argument_errors(oracle_lib):
    U, I = mipsgen.generate("tiny", 0, n_users=4, n_items=8)
    with pytest.raises(ValueError):
        T.topk(U, I, 0)
    with pytest.raises(ValueError):
        T.topk(U, I, 9)


def test_golden_hand_example(oracle_lib):
    with open(os.path.join(GOLDEN, "topk_hand_example.json")) as fh:
        g = json.load(fh)
    U = np.array(g["U"], dtype=np.float32)
    I = np.array(g["I"], dtype=np.float32)
    idx, key = T.topk(U, I, g["K"])
    np.testing.assert_array_equal(idx, np.array(g["expected_idx"]))
    np.testing.assert_array_equal(key, np.array(g["expected_key"], dtype=np.float64))


def test_pair_keys_independent_numpy_and_hand_example(oracle_lib):
    """pair_keys against the independent left-to-right numpy sum (random
    pairs) and the hand-worked integer ratings."""
    U, I = mipsgen.generate("mf", 3, n_users=200, n_items=700, f=50)
    rng = np.random.default_rng(7)
    idx = rng.integers(0, I.shape[0], size=(U.shape[0], 12)).astype(np.int32)
    U64 = U.astype(np.float64)
    I64 = I.astype(np.float64)[idx]            # [n_u, 12, f]
    acc = np.zeros(idx.shape)
    for j in range(U.shape[1]):
        acc = acc + U64[:, None, j] * I64[:, :, j]
    np.testing.assert_array_equal(T.pair_keys(U, I, idx), acc)
    with open(os.path.join(GOLDEN, "topk_hand_example.json")) as fh:
        g = json.load(fh)
    Ug = np.array(g["U"], dtype=np.float32)
    Ig = np.array(g["I"], dtype=np.float32)
    all_idx = np.tile(np.arange(Ig.shape[0], dtype=np.int32), (Ug.shape[0], 1))
    np.testing.assert_array_equal(T.pair_keys(Ug, Ig, all_idx),
                                  np.array(g["ratings_by_hand"], dtype=np.float64))
    with pytest.raises(ValueError):
        T.pair_keys(Ug, Ig, all_idx + 1)
