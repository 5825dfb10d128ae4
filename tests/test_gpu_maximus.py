"""GPU parity of the Maximus index (Section III): the built index satisfies
the invariants the paper's correctness argument rests on, checked with the
float64 oracle functions, and the blocked walk returns exactly the oracle's
top-K (and the brute force's) for every user."""
import numpy as np
import pytest
import torch

import mipsgen
from gpu_util import assert_properties_all_users, assert_parity, log, to_dev
from oracle import maximus as M
from oracle import topk as oracle_topk

pytestmark = pytest.mark.gpu


def _build(U, I, C, iters=3, seed=0, block_items=0):
    import paper_1706_01449_amd as mips
    Ut, It = to_dev(U, I)
    ix = mips.maximus_build(Ut, It, C, iters, seed, block_items)
    return ix


def _query(ix, K, prec, stats=False):
    out = ix.query(K, prec, stats=stats)
    torch.cuda.synchronize()
    res = [out[0].cpu().numpy(), out[1].cpu().numpy()]
    return res + [out[2]] if stats else res


@pytest.mark.parametrize("C", [1, 8, 64])
def test_index_invariants(C):
    """Lists are permutations sorted by non-increasing bound; theta_b equals
    the float64 max user-centroid angle for the GPU's own clustering; the
    stored bound never undercuts the float64 bound; every user sits in a
    nearest cluster."""
    log(f"index invariants C={C}")
    U, I = mipsgen.generate("clustered", 1, n_users=6000, n_items=2500, f=24)
    ix = _build(U, I, C)
    ex = ix.export()
    cent, tb, asg, lists, bnd = ex["centroids"], ex["theta_b"], ex["assign"], ex["lists"], ex["bounds"]
    n_i = I.shape[0]
    for c in range(C):
        assert np.array_equal(np.sort(lists[c]), np.arange(n_i))
        assert np.all(np.diff(bnd[c].astype(np.float64)) <= 0)            # Property
        # ties in the stored bound are ordered by item index
        same = np.diff(bnd[c]) == 0
        assert np.all(np.diff(lists[c])[same] > 0)
    # theta_b from the GPU's (assignment, centroids) pair, float64 oracle formula
    ref_tb = M.theta_b(U, cent, asg.astype(np.int64))
    np.testing.assert_allclose(tb, ref_tb, rtol=0, atol=1e-12)
    # stored (rounded-up) bound >= float64 bound of Eq. (appx_bound)
    for c in range(C):
        ref = M.cbound(cent[c], I, tb[c])
        stored = np.empty(n_i)
        stored[lists[c]] = bnd[c]
        assert np.all(stored >= ref - 1e-12 * np.abs(ref))
    # Lemma: ||u|| * bound >= key for every pair of sampled users
    un = np.linalg.norm(U.astype(np.float64), axis=1)
    for u in mipsgen.sample_users(U.shape[0], 60, seed=C):
        keys = oracle_topk.user_keys(U[u], I)
        stored = np.empty(n_i)
        stored[lists[asg[u]]] = bnd[asg[u]]
        assert np.all(un[u] * stored * (1 + 2 ** -30) + 1e-12 >= keys)
    # nearest centroid (float32 distances on the GPU: allow a tiny slack)
    d = ((U[:, None, :].astype(np.float64) - cent[None, :, :]) ** 2).sum(-1)
    mine = d[np.arange(U.shape[0]), asg]
    assert np.all(mine <= d.min(axis=1) * (1 + 1e-4) + 1e-6)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("C,K", [(1, 10), (8, 10), (64, 1), (64, 50), (256, 5)])
def test_query_small_all_users(prec, C, K):
    log(f"maximus small prec={prec} C={C} K={K}")
    U, I = mipsgen.generate("clustered", 2, n_users=5000, n_items=3000, f=50)
    ix = _build(U, I, C)
    idx, score, st = _query(ix, K, prec, stats=True)
    assert_parity(idx, score, U, I, K)
    if C >= 8 and prec != "fp8":
        # the walk stops early; the coarse E4M3 screen's looser lower bounds
        # keep tau lower and make it walk further (same answer)
        assert st["mean_items_visited"] < 0.5 * I.shape[0]


@pytest.mark.parametrize("mode", ["wave-cascade", "wave", "group"])
@pytest.mark.parametrize("prec,K", [("fp32", 32), ("bf16", 50), ("fp8", 10), ("fp8", 40)])
def test_query_certification_kernels(mode, prec, K, monkeypatch):
    """The walk's candidates certified by either certification kernel, with
    and without the bfloat16 cascade of E4M3 candidates."""
    log(f"maximus certify {mode} prec={prec} K={K}")
    U, I = mipsgen.generate("clustered", 5, n_users=3000, n_items=2500, f=50)
    ix = _build(U, I, 16)
    monkeypatch.setenv("MIPS_DEBUG_CERTIFY", mode.split("-")[0])
    monkeypatch.setenv("MIPS_CERTIFY_CASCADE", "1" if mode.endswith("cascade") else "0")
    idx, score = _query(ix, K, prec)
    monkeypatch.delenv("MIPS_DEBUG_CERTIFY")
    monkeypatch.delenv("MIPS_CERTIFY_CASCADE")
    assert_parity(idx, score, U, I, K)


@pytest.mark.parametrize("cap", [12, 40])
def test_e4m3_walk_forced_overflow(cap, monkeypatch):
    """A test-only cap of a few candidate slots per lane overflows the E4M3
    walk's lists for many users, which then take the exact float64 path; the
    answer must not change."""
    log(f"maximus e4m3 forced overflow cap={cap}")
    U, I = mipsgen.generate("clustered", 6, n_users=3000, n_items=2500, f=50)
    ix = _build(U, I, 16)
    monkeypatch.setenv("MIPS_DEBUG_CAND_CAP", str(cap))
    idx, score, st = _query(ix, 10, "fp8", stats=True)
    monkeypatch.delenv("MIPS_DEBUG_CAND_CAP")
    log(f"  overflow users {st['overflow_users']} of {U.shape[0]}")
    assert_parity(idx, score, U, I, 10)


def test_singleton_clusters_and_degenerate_rows():
    U, I = mipsgen.generate("mf", 3, n_users=300, n_items=900, f=20)
    U[5] = 0.0
    I[7] = I[8]
    I[10] = 0.0
    ix = _build(U, I, C=300, iters=2)
    idx, score, st = _query(ix, 7, "bf16", stats=True)
    assert_parity(idx, score, U, I, 7)
    ix = _build(U, I, C=1, iters=0)
    idx, score = _query(ix, 7, "fp32")
    assert_parity(idx, score, U, I, 7)


@pytest.mark.parametrize("block_items", [0, 32, 4096])
def test_shared_leading_block(block_items):
    """The paper's B: the first B list items are scored for every user of a
    cluster before any may stop; the answer never changes."""
    U, I = mipsgen.generate("clustered", 4, n_users=4000, n_items=6000, f=50)
    ix = _build(U, I, 8, block_items=block_items)
    idx, score, st = _query(ix, 10, "bf16", stats=True)
    assert_parity(idx, score, U, I, 10)
    if block_items == 4096:
        assert st["mean_items_visited"] >= 4096


@pytest.mark.parametrize("C", [8, 64, 256])
def test_clustered_full_size_matches_oracle_and_bmm(C):
    """480,000 x 17,770, f = 50, users from a 64-component mixture and
    power-law item norms; K = 10.  Maximus (bf16 screen) equals the
    brute force on every user and the oracle on 1,000 sampled users."""
    import paper_1706_01449_amd as mips
    log(f"clustered full size C={C}")
    U, I = _clustered_full()
    Ut, It = to_dev(U, I)
    ix = mips.maximus_build(Ut, It, C, 3, 0, 0)
    out = ix.query(10, "bf16", stats=True)
    bmm = mips.bmm_topk(Ut, It, 10, "bf16")
    torch.cuda.synchronize()
    idx, score, st = out[0].cpu().numpy(), out[1].cpu().numpy(), out[2]
    log(f"  stats {st}")
    np.testing.assert_array_equal(idx, bmm[0].cpu().numpy())
    np.testing.assert_array_equal(score, bmm[1].cpu().numpy())
    users = mipsgen.sample_users(U.shape[0], 1000, seed=C)
    assert_parity(idx, score, U, I, 10, users=users)
    assert_properties_all_users(idx, score, U, I, 10)
    assert st["mean_items_visited"] < 0.1 * I.shape[0]
    assert st["overflow_users"] <= U.shape[0] // 1000


_CL = {}


def _clustered_full():
    if "x" not in _CL:
        _CL["x"] = mipsgen.generate("clustered", 0)
    return _CL["x"]
