"""GPU parity of the top-K backward (dU gather, dI atomic scatter-add) with
the float64 oracle, directly through the C ABI and through the autograd
Function."""
import numpy as np
import pytest
import torch

import mipsgen
from gpu_util import DEV, assert_manifest, log, to_dev
from oracle import backward as B
from oracle import topk as oracle_topk

pytestmark = pytest.mark.gpu


def _softmax_rows(S):
    S = np.asarray(S, dtype=np.float64)
    e = np.exp(S - S.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def _close(gpu, ref, rtol=1e-5):
    ref = np.asarray(ref)
    atol = 1e-6 * float(np.abs(ref).max())
    np.testing.assert_allclose(gpu, ref, rtol=rtol, atol=atol)


def test_full_size_grad_workload_direct():
    """65,536 x 100,000 users/items, f = 64, K = 32: forward on the GPU, then
    the backward kernel against the float64 scatter/gather definition."""
    import paper_1706_01449_amd as mips
    log("grad workload full size")
    U, I = mipsgen.generate("grad", 0)
    Ut, It = to_dev(U, I)
    idx, score = mips.bmm_topk(Ut, It, 32, "bf16")
    S = score.cpu().numpy().astype(np.float32)
    G = _softmax_rows(S).astype(np.float32)
    dU, dI = mips.topk_backward(Ut, It, idx, torch.from_numpy(G).to(DEV))
    torch.cuda.synchronize()
    idx_h = idx.cpu().numpy()
    assert_manifest(idx_h, score.cpu().numpy(), U, I, "grad", 0, 32, what="grad forward")
    rU, rI = B.scatter_gather_grads(U, I, idx_h, G)
    _close(dU.cpu().numpy(), rU)
    _close(dI.cpu().numpy(), rI)


@pytest.mark.parametrize("recompute", [False, True])
def test_autograd_matches_float64_autograd(recompute):
    import paper_1706_01449_amd as mips
    U, I = mipsgen.generate("grad", 1, n_users=3000, n_items=6000, f=64)
    Ut, It = to_dev(U, I)
    Ut.requires_grad_(True)
    It.requires_grad_(True)
    s, idx = mips.topk_scores(Ut, It, 32, "bf16", recompute_idx=recompute)
    loss = torch.logsumexp(s, dim=1).sum()
    loss.backward()
    torch.cuda.synchronize()
    idx_h = idx.cpu().numpy()
    ri, _ = oracle_topk.topk(U, I, 32)
    np.testing.assert_array_equal(idx_h, ri)
    rU, rI = B.autograd_grads(U, I, idx_h)
    _close(Ut.grad.cpu().numpy(), rU)
    _close(It.grad.cpu().numpy(), rI)


def test_recompute_gives_same_gradients():
    import paper_1706_01449_amd as mips
    U, I = mipsgen.generate("grad", 2, n_users=1000, n_items=3000, f=64)
    grads = []
    for rec in (False, True):
        Ut, It = to_dev(U, I)
        Ut.requires_grad_(True)
        It.requires_grad_(True)
        s, _ = mips.topk_scores(Ut, It, 16, "fp32", recompute_idx=rec)
        (s * torch.arange(16, device=DEV, dtype=torch.float32)).sum().backward()
        torch.cuda.synchronize()
        grads.append((Ut.grad.cpu().numpy(), It.grad.cpu().numpy()))
    np.testing.assert_array_equal(grads[0][0], grads[1][0])   # dU is deterministic
    _close(grads[0][1], grads[1][1], rtol=1e-6)


def test_slice_matches_finite_difference_pinned_oracle():
    """The 64 x 512, f = 16 slice whose float64 gradient is pinned to finite
    differences in the CPU suite: the GPU gradient of the same (float32)
    inputs matches the oracle's."""
    import paper_1706_01449_amd as mips
    U64, I64 = mipsgen.grad_slice(0)
    U, I = U64.astype(np.float32), I64.astype(np.float32)
    Ut, It = to_dev(U, I)
    Ut.requires_grad_(True)
    It.requires_grad_(True)
    s, idx = mips.topk_scores(Ut, It, 32, "fp32")
    torch.logsumexp(s, dim=1).sum().backward()
    torch.cuda.synchronize()
    rU, rI = B.autograd_grads(U, I, idx.cpu().numpy())
    _close(Ut.grad.cpu().numpy(), rU)
    _close(It.grad.cpu().numpy(), rI)


def test_out_of_range_indices_are_skipped():
    import paper_1706_01449_amd as mips
    U, I = mipsgen.generate("grad", 3, n_users=64, n_items=100, f=20)
    Ut, It = to_dev(U, I)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 100, size=(64, 4)).astype(np.int32)
    idx[0, 1] = -5
    idx[3, 2] = 100
    G = rng.standard_normal((64, 4)).astype(np.float32)
    dU, dI = mips.topk_backward(Ut, It, torch.from_numpy(idx).to(DEV), torch.from_numpy(G).to(DEV))
    torch.cuda.synchronize()
    keep = (idx >= 0) & (idx < 100)
    G2 = np.where(keep, G, 0.0)
    idx2 = np.where(keep, idx, 0)
    rU, rI = B.scatter_gather_grads(U, I, idx2, G2)
    _close(dU.cpu().numpy(), rU)
    _close(dI.cpu().numpy(), rI)


def test_grouping_with_colliding_items_and_popular_items():
    """The dI grouping counts pairs per item in per-workgroup hash tables: items
    whose hashes collide (probe sequences past the table's limit take the
    global path) and a few items shared by almost every user (long runs that
    span workgroups) must still give the plain gather/scatter result."""
    import paper_1706_01449_amd as mips
    n_i, f, n_u, K = 1 << 20, 4, 600, 24
    # items whose 13-bit multiplicative hash is equal: they probe the same slots
    h = ((np.arange(n_i, dtype=np.uint64) * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)) >> np.uint64(19)
    same = np.nonzero(h == h[12345])[0][:100].astype(np.int32)
    assert same.size == 100
    rng = np.random.default_rng(5)
    U = rng.standard_normal((n_u, f)).astype(np.float32)
    I = rng.standard_normal((n_i, f)).astype(np.float32)
    idx = np.empty((n_u, K), dtype=np.int32)
    for u in range(n_u):
        idx[u, :16] = rng.choice(same, 16, replace=False)   # colliding items
        idx[u, 16:20] = [7, 8, 9, 10]                        # items of every user
        idx[u, 20:] = rng.integers(0, n_i, 4)
    G = rng.standard_normal((n_u, K)).astype(np.float32)
    Ut, It = to_dev(U, I)
    dU, dI = mips.topk_backward(Ut, It, torch.from_numpy(idx).to(DEV), torch.from_numpy(G).to(DEV))
    torch.cuda.synchronize()
    rU, rI = B.scatter_gather_grads(U, I, idx, G)
    _close(dU.cpu().numpy(), rU)
    _close(dI.cpu().numpy(), rI)
