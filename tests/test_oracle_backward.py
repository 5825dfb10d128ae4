"""Pins for the backward oracle (CPU only): finite differences of the true
loss (top-K recomputed) and two independent routes to the gradient."""
import numpy as np

import mipsgen
from oracle import backward as B


def _topk_idx64(U, I, K):
    S = U @ I.T
    cols = np.arange(I.shape[0])
    return np.stack([np.lexsort((cols, -S[u]))[:K] for u in range(U.shape[0])])


def _per_user_loss(U, I, K):
    """logsumexp of each user's top-K scores (top-K recomputed)."""
    idx = _topk_idx64(U, I, K)
    S = np.einsum("uf,ukf->uk", U, I[idx])
    m = S.max(axis=1)
    return m + np.log(np.exp(S - m[:, None]).sum(axis=1)), idx


def test_autograd_equals_closed_form():
    U, I = mipsgen.grad_slice(0)
    idx = _topk_idx64(U, I, 32)
    S = np.einsum("uf,ukf->uk", U, I[idx])
    G = B.logsumexp_grad_scores(S)
    dU1, dI1 = B.scatter_gather_grads(U, I, idx, G)
    dU2, dI2 = B.autograd_grads(U, I, idx)
    np.testing.assert_allclose(dU1, dU2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(dI1, dI2, rtol=1e-12, atol=1e-14)


def test_finite_differences_slice():
    K = 32
    U, I = mipsgen.grad_slice(0)
    L0, idx0 = _per_user_loss(U, I, K)
    assert abs(L0.sum() - B.logsumexp_loss(U, I, idx0)) < 1e-9
    dU, dI = B.autograd_grads(U, I, idx0)
    checked = skipped = 0
    for X, dX, is_u in ((U, dU, True), (I, dI, False)):
        for r in range(X.shape[0]):
            for c in range(X.shape[1]):
                x = X[r, c]
                # per-user differences: users the coordinate does not touch cancel exactly
                h = 2.0 ** -17 * max(1.0, abs(x))
                X[r, c] = x + h
                Lp, ip = _per_user_loss(U, I, K)
                X[r, c] = x - h
                Lm, im = _per_user_loss(U, I, K)
                X[r, c] = x
                if not (np.array_equal(np.sort(ip, 1), np.sort(idx0, 1)) and
                        np.array_equal(np.sort(im, 1), np.sort(idx0, 1))):
                    skipped += 1
                    continue
                fd = float(np.sum(Lp - Lm)) / (2 * h)
                assert abs(fd - dX[r, c]) <= 1e-6 * abs(dX[r, c]) + 1e-9, (is_u, r, c, fd, dX[r, c])
                checked += 1
    assert checked > 0.9 * (U.size + I.size)
