"""Float64 reference of the Maximus pruning index.  TEST INFRASTRUCTURE ONLY.

Follows Section III of the paper: cluster users with k-means (Section III-A),
for each cluster take the largest user-to-centroid angle theta_b and order all
items by the bound of Eq. (appx_bound) (Section III-B, Algorithm 1,
ConstructIndex), then answer a user's top-K by walking its cluster's list and
stopping once the bound can no longer reach the K-th best rating
(Section III-C, Algorithm 1, QueryIndex).  The paper's correctness argument
(monotone lists, the bound never below u.i/||u||, the walk is exact) is what
the tests check against this module.

Readings where the paper is silent or loose (all listed with reasons in the
design notes):
* k-means: Forgy initialisation (C distinct users drawn from the seed),
  Euclidean distance, ties to the lower centroid index, an empty cluster keeps
  its centroid, ``iters`` Lloyd updates, then one final assignment; theta_b
  uses that final (assignment, centroid) pair.
* Angles: Kahan's stable form theta(a, b) = 2 atan2(||a^ - b^||, ||a^ + b^||)
  with x^ = x / ||x||.
* Bound: ||i|| cos(max(theta_ic - theta_b, 0)); this equals both branches of
  Eq. (appx_bound) because cos(0) = 1.  Negative values are kept.  A zero
  centroid gets theta_b = pi; a zero item has bound 0.
* The walk's stop test compares ||u|| * bound with the K-th best rating (the
  bound is a bound on u.i / ||u||), strictly, with a small outward slack for
  float64 evaluation error.
* Ratings are the oracle's FP64 keys (left-to-right sums); the heap order is
  (key desc, item index asc).
"""
from __future__ import annotations

import numpy as np

from . import topk as _topk


def _norms(X):
    X = np.asarray(X, dtype=np.float64)
    return np.sqrt(np.einsum("ij,ij->i", X, X))


def stable_angle(A, B):
    """Angle between rows of A and rows of B (broadcast), Kahan's formula.

    Rows of zero length give angle 0 (the caller decides what a zero vector
    means for the bound)."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    na = _norms(A)[:, None]
    nb = _norms(B)[:, None]
    Ah = np.divide(A, na, out=np.zeros_like(A), where=na > 0)
    Bh = np.divide(B, nb, out=np.zeros_like(B), where=nb > 0)
    d = _norms(Ah - Bh)
    s = _norms(Ah + Bh)
    ang = 2.0 * np.arctan2(d, s)
    zero = (na[:, 0] == 0) | (nb[:, 0] == 0) if A.shape[0] == B.shape[0] else None
    if zero is not None:
        ang = np.where(zero, 0.0, ang)
    return ang


def kmeans(U, C: int, iters: int, seed: int):
    """Lloyd's k-means (Section III-A).  Returns (centroids [C, f] float64,
    assignment [n_u] int64) where the assignment is the final one after the
    last centroid update."""
    U = np.asarray(U, dtype=np.float64)
    n_u = U.shape[0]
    if not 1 <= C <= n_u:
        raise ValueError("need 1 <= C <= n_users")
    rng = np.random.default_rng(np.random.SeedSequence([7, int(seed)]))
    cent = U[np.sort(rng.choice(n_u, size=C, replace=False))].copy()

    def assign(cent):
        # ||u - c||^2 computed directly; argmin takes the first (lowest) index on ties.
        d = ((U[:, None, :] - cent[None, :, :]) ** 2).sum(axis=2) if n_u * C <= 4_000_000 else None
        if d is None:
            out = np.empty(n_u, dtype=np.int64)
            step = max(1, 4_000_000 // C)
            for s in range(0, n_u, step):
                dd = ((U[s:s + step, None, :] - cent[None, :, :]) ** 2).sum(axis=2)
                out[s:s + step] = np.argmin(dd, axis=1)
            return out
        return np.argmin(d, axis=1)

    for _ in range(iters):
        a = assign(cent)
        for j in range(C):
            m = a == j
            if m.any():
                cent[j] = U[m].mean(axis=0)
    return cent, assign(cent)


def theta_b(U, cent, assign):
    """theta_bj = max over users of cluster j of the user-centroid angle
    (Algorithm 1, ConstructIndex).  Zero users are left out; a zero centroid
    gets pi; an empty cluster gets 0."""
    U = np.asarray(U, dtype=np.float64)
    C = cent.shape[0]
    tb = np.zeros(C)
    cn = _norms(cent)
    un = _norms(U)
    ang = stable_angle(U, cent[assign])
    for j in range(C):
        if cn[j] == 0:
            tb[j] = np.pi
            continue
        m = (assign == j) & (un > 0)
        if m.any():
            tb[j] = ang[m].max()
    return tb


def cbound(cent_j, I, tb_j):
    """Bound of Eq. (appx_bound) for one centroid against every item:
    ||i|| cos(max(theta_ic - theta_b, 0))."""
    I = np.asarray(I, dtype=np.float64)
    inorm = _norms(I)
    th = stable_angle(I, np.broadcast_to(np.asarray(cent_j, dtype=np.float64), I.shape))
    return inorm * np.cos(np.maximum(th - tb_j, 0.0))


def build_index(U, I, C: int, iters: int = 3, seed: int = 0, force_theta_pi: bool = False):
    """ConstructIndex: clusters, theta_b, bounds [C, n_i] and per-cluster lists
    sorted by (bound desc, item index asc)."""
    cent, a = kmeans(U, C, iters, seed)
    tb = theta_b(U, cent, a)
    if force_theta_pi:
        tb = np.full_like(tb, np.pi)
    n_i = np.asarray(I).shape[0]
    bounds = np.empty((C, n_i))
    lists = np.empty((C, n_i), dtype=np.int64)
    idx = np.arange(n_i)
    for j in range(C):
        b = cbound(cent[j], I, tb[j])
        bounds[j] = b
        lists[j] = np.lexsort((idx, -b))
    return {"centroids": cent, "assign": a, "theta_b": tb, "bounds": bounds, "lists": lists}


def stop_slack(f: int) -> float:
    """Relative outward slack for the walk's stop test in float64."""
    return (f + 64) * 2.0 ** -50


def query(index, U, I, K: int):
    """QueryIndex for every user: returns (idx [n_u, K] int32, key [n_u, K]
    float64, visited [n_u] int64).  The heap is seeded with the first K items
    of the user's list; the walk stops at the first item whose scaled bound is
    strictly below the K-th best key."""
    U32 = np.ascontiguousarray(U, dtype=np.float32)
    I32 = np.ascontiguousarray(I, dtype=np.float32)
    n_u, f = U32.shape
    n_i = I32.shape[0]
    if not 1 <= K <= n_i:
        raise ValueError("need 1 <= K <= n_items")
    unorm = _norms(U32)
    imax = _norms(I32).max()
    slack = stop_slack(f)
    out_idx = np.empty((n_u, K), dtype=np.int32)
    out_key = np.empty((n_u, K))
    visited = np.empty(n_u, dtype=np.int64)
    for u in range(n_u):
        j = index["assign"][u]
        L = index["lists"][j]
        bnd = index["bounds"][j]
        keys = _topk.user_keys(U32[u], I32)
        # heap as a sorted list of (key, idx), best first
        H = sorted(((keys[i], int(i)) for i in L[:K]), key=lambda t: (-t[0], t[1]))
        w = K
        for p in range(K, n_i):
            i = int(L[p])
            tau = H[-1][0]
            if unorm[u] * bnd[i] * (1.0 + slack) + slack * unorm[u] * imax < tau:
                break
            w = p + 1
            cand = (keys[i], i)
            worst = H[-1]
            if cand[0] > worst[0] or (cand[0] == worst[0] and cand[1] < worst[1]):
                H[-1] = cand
                H.sort(key=lambda t: (-t[0], t[1]))
        visited[u] = w
        out_idx[u] = [t[1] for t in H]
        out_key[u] = [t[0] for t in H]
    return out_idx, out_key, visited
