"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the CPU oracle element by element."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import topk as oracle_topk

DEV = "cuda:0"


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]


def gpu_topk(U, I, K, prec, stats=False):
    import paper_1706_01449_amd as mips
    Ut, It = to_dev(U, I)
    out = mips.bmm_topk(Ut, It, K, prec, stats=stats)
    torch.cuda.synchronize()
    idx = out[0].cpu().numpy()
    score = out[1].cpu().numpy()
    return (idx, score, out[2]) if stats else (idx, score)


def assert_parity(idx, score, U, I, K, users=None):
    """Indices bit-equal to the oracle, scores bit-equal (the float64 keys)."""
    Us = U if users is None else U[users]
    ri, rk = oracle_topk.topk(Us, I, K)
    gi = idx if users is None else idx[users]
    gs = score if users is None else score[users]
    bad = np.nonzero((gi != ri).any(axis=1))[0]
    assert bad.size == 0, (f"{bad.size} users differ; first user {bad[0]}: gpu {gi[bad[0]][:12]} "
                           f"oracle {ri[bad[0]][:12]}")
    np.testing.assert_array_equal(gs, rk)


def assert_properties_all_users(idx, score, U, I, K):
    """Checks that hold at any size, on every user: each returned score is
    the oracle's key of its (user, item) pair, bit for bit; items are
    distinct and in range; rows are ordered by (key desc, index asc)."""
    n_u = U.shape[0]
    assert idx.shape == (n_u, K) and score.shape == (n_u, K)
    assert idx.min() >= 0 and idx.max() < I.shape[0]
    np.testing.assert_array_equal(score, oracle_topk.pair_keys(U, I, idx))
    if K > 1:
        s = np.sort(idx, axis=1)
        assert np.all(s[:, 1:] != s[:, :-1]), "duplicate items in a row"
        d = score[:, :-1] - score[:, 1:]
        ok = (d > 0) | ((d == 0) & (idx[:, :-1] < idx[:, 1:]))
        assert np.all(ok), "a row is not ordered by (key desc, index asc)"
