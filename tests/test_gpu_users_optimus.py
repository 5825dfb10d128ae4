"""GPU parity of queries for arbitrary user vectors against a Maximus index
(new users, subsets: Section III-E) and of the Optimus selector (Section IV),
through the C ABI.  Bar: indices and float64 keys bit-equal to the oracle."""
import numpy as np
import pytest
import torch

import mipsgen
from gpu_util import assert_manifest, assert_parity, log, to_dev

pytestmark = pytest.mark.gpu


def _build(U, I, C, iters=3, seed=0):
    import paper_1706_01449_amd as mips
    Ut, It = to_dev(U, I)
    return mips.maximus_build(Ut, It, C, iters, seed, 0)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_query_users_with_index_users_equals_query(prec):
    """Every indexed user is covered by its own cluster, so querying the
    index's users as vectors gives the walk's answer, bit for bit."""
    log(f"query_users = query prec={prec}")
    U, I = mipsgen.generate("clustered", 4, n_users=4000, n_items=2500, f=32)
    ix = _build(U, I, 16)
    a_idx, a_sc = ix.query(10, prec)
    (Uq,) = to_dev(U)
    b_idx, b_sc, st = ix.query_users(Uq, 10, prec, stats=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(b_idx.cpu().numpy(), a_idx.cpu().numpy())
    np.testing.assert_array_equal(b_sc.cpu().numpy(), a_sc.cpu().numpy())
    assert_parity(b_idx.cpu().numpy(), b_sc.cpu().numpy(), U, I, 10)
    # the coarse E4M3 screen sends some users to the exact path (same answer)
    assert st["overflow_users"] <= (U.shape[0] // 10 if prec == "fp8" else 0)
    assert st["mean_items_visited"] < 0.5 * I.shape[0]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("K", [1, 10, 50])
def test_query_users_new_users(prec, K):
    """New users: fresh draws from the same mixture (mostly covered), isotropic
    directions far from every cluster (mostly not covered: exact path), a zero
    row, rescaled rows, and a subset of the indexed users, in one batch."""
    log(f"query_users new users prec={prec} K={K}")
    U, I = mipsgen.generate("clustered", 5, n_users=6000, n_items=3000, f=24)
    ix = _build(U, I, 32)
    # same seed, more users: the same mixture components, fresh draws
    more, _ = mipsgen.generate("clustered", 5, n_users=6700, n_items=3000, f=24)
    fresh = more[6000:]
    far, _ = mipsgen.generate("tiny", 7, n_users=300, n_items=1, f=24)
    Uq = np.concatenate([fresh, far * 5.0, np.zeros((1, 24), np.float32), fresh[:50] * 1e3,
                         U[::37]]).astype(np.float32)
    (Uqt,) = to_dev(Uq)
    idx, sc, st = ix.query_users(Uqt, K, prec, stats=True)
    torch.cuda.synchronize()
    idx, sc = idx.cpu().numpy(), sc.cpu().numpy()
    assert_parity(idx, sc, Uq, I, K)
    log(f"  stats {st}")
    # the zero row takes the exact path, as do far rows outside every
    # cluster's cone; most fresh draws of the same mixture are covered
    assert 1 <= st["overflow_users"] <= Uq.shape[0] - 500


def test_query_users_zero_and_single_row():
    U, I = mipsgen.generate("clustered", 8, n_users=500, n_items=700, f=16)
    ix = _build(U, I, 4)
    for Uq in (np.zeros((1, 16), np.float32), U[3:4].copy()):
        (Uqt,) = to_dev(Uq)
        idx, sc = ix.query_users(Uqt, 5, "bf16")
        torch.cuda.synchronize()
        assert_parity(idx.cpu().numpy(), sc.cpu().numpy(), Uq, I, 5)


@pytest.mark.parametrize("workload", ["mf", "clustered"])
@pytest.mark.parametrize("sample", [0, 700])
def test_optimus_small_exact(workload, sample):
    """Whatever it picks, the answer is the oracle's; the sampled users'
    answers are reused and the others computed by the chosen method."""
    import paper_1706_01449_amd as mips
    log(f"optimus small {workload} sample={sample}")
    U, I = mipsgen.generate(workload, 9, n_users=3000, n_items=2000, f=32)
    Ut, It = to_dev(U, I)
    idx, sc, rep = mips.optimus_topk(Ut, It, 10, "bf16", n_clusters=16, sample_users=sample)
    torch.cuda.synchronize()
    log(f"  report {rep}")
    assert_parity(idx.cpu().numpy(), sc.cpu().numpy(), U, I, 10)
    assert rep["sample_users"] == (sample if sample else 3000)
    assert rep["choice"] in ("bmm", "maximus")
    assert rep["est_bmm_ms"] > 0 and rep["est_maximus_ms"] >= rep["build_ms"]


@pytest.mark.parametrize("workload", ["mf", "clustered"])
def test_optimus_full_size(workload):
    """480,000 x 17,770, f = 50, K = 10 with the default sample: every user's
    answer equals the oracle's, whichever method the selector picks."""
    import paper_1706_01449_amd as mips
    log(f"optimus full size {workload}")
    U, I = mipsgen.generate(workload, 0)
    Ut, It = to_dev(U, I)
    idx, sc, rep = mips.optimus_topk(Ut, It, 10, "bf16", n_clusters=64)
    torch.cuda.synchronize()
    log(f"  report {rep}")
    assert_manifest(idx.cpu().numpy(), sc.cpu().numpy(), U, I, workload, 0, 10,
                    what=f"optimus {workload}")
