"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the CPU oracle element by element."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import torch

from oracle import topk as oracle_topk

MANIFESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "manifests")

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


def _sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def load_manifest(workload: str, seed: int, K: int) -> dict:
    path = os.path.join(MANIFESTS, f"{workload}_seed{seed}_K{K}.json")
    with open(path) as fh:
        return json.load(fh)


def assert_manifest(idx, score, U, I, workload: str, seed: int, K: int, what: str = ""):
    """Every user's answer equals the oracle's, bit for bit: the SHA-256 of
    the GPU's idx (int32) and score (float64) bytes must equal the hashes the
    oracle's full run wrote (tests/golden/make_manifests.py).  The inputs'
    own hashes are checked first, so a changed generator is reported as such.
    On a mismatch the differing blocks of users are named and a few users of
    the first such block are compared element by element with the oracle."""
    m = load_manifest(workload, seed, K)
    assert _sha(U) == m["U_sha256"] and _sha(I) == m["I_sha256"], \
        f"{workload} seed {seed}: input bytes differ from the ones the manifest was written for"
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    score = np.ascontiguousarray(score, dtype=np.float64)
    assert idx.shape == (m["n_users"], K) and score.shape == (m["n_users"], K)
    if _sha(idx) == m["idx_sha256"] and _sha(score) == m["key_sha256"]:
        return
    B = m["block_users"]
    bad = [b for b in range(len(m["idx_block_sha256"]))
           if _sha(idx[b * B:(b + 1) * B]) != m["idx_block_sha256"][b]
           or _sha(score[b * B:(b + 1) * B]) != m["key_block_sha256"][b]]
    msg = f"{what}: {len(bad)} of {len(m['idx_block_sha256'])} blocks of {B} users differ from the oracle"
    if bad:
        users = np.arange(bad[0] * B, min((bad[0] + 1) * B, m["n_users"]))[:256]
        ri, rk = oracle_topk.topk(U[users], I, K)
        diff = np.nonzero((idx[users] != ri).any(axis=1) | (score[users] != rk).any(axis=1))[0]
        if diff.size:
            u = users[diff[0]]
            msg += (f"; user {u}: gpu {idx[u][:12]} {score[u][:4]} "
                    f"oracle {ri[diff[0]][:12]} {rk[diff[0]][:4]}")
    raise AssertionError(msg)
