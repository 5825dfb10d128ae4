"""Gradients of a loss on the top-K scores.  TEST INFRASTRUCTURE ONLY.

The top-K indices are piecewise constant in U and I, so the gradient of any
loss on the top-K scores S[u, k] = u . I[idx[u, k]] is taken with idx held
fixed:

    dL/dU[u]  = sum_k G[u, k] * I[idx[u, k]]
    dL/dI[i]  = sum over (u, k) with idx[u, k] = i of G[u, k] * U[u]

with G = dL/dS.  For L = sum_u logsumexp_k S[u, k], G[u, :] = softmax(S[u, :]).
Everything here is float64.
"""
from __future__ import annotations

import numpy as np
import torch


def scatter_gather_grads(U, I, idx, G):
    """Plain definition of the two gradients for a given G (float64)."""
    U = np.asarray(U, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    G = np.asarray(G, dtype=np.float64)
    n_u, K = idx.shape
    dU = np.zeros_like(U)
    for k in range(K):
        dU += G[:, k:k + 1] * I[idx[:, k]]
    dI = np.zeros_like(I)
    for k in range(K):
        np.add.at(dI, idx[:, k], G[:, k:k + 1] * U)
    return dU, dI


def logsumexp_grad_scores(S):
    """G = softmax of each user's top-K scores (closed form of dL/dS)."""
    S = np.asarray(S, dtype=np.float64)
    m = S.max(axis=1, keepdims=True)
    e = np.exp(S - m)
    return e / e.sum(axis=1, keepdims=True)


def logsumexp_loss(U, I, idx):
    """L = sum_u logsumexp_k (U[u] . I[idx[u, k]]) in float64."""
    U = np.asarray(U, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    S = np.einsum("uf,ukf->uk", U, I[idx])
    m = S.max(axis=1)
    return float(np.sum(m + np.log(np.exp(S - m[:, None]).sum(axis=1))))


def autograd_grads(U, I, idx):
    """dL/dU, dL/dI of the logsumexp loss by torch autograd (float64, CPU)."""
    Ut = torch.tensor(np.asarray(U, dtype=np.float64), requires_grad=True)
    It = torch.tensor(np.asarray(I, dtype=np.float64), requires_grad=True)
    ix = torch.as_tensor(np.asarray(idx, dtype=np.int64))
    S = (Ut[:, None, :] * It[ix]).sum(-1)
    L = torch.logsumexp(S, dim=1).sum()
    dU, dI = torch.autograd.grad(L, (Ut, It))
    return dU.numpy(), dI.numpy()
