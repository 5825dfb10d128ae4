"""The allocation-free backward (mips_topk_backward_noalloc) against the
allocating one (mips_topk_backward) and the float64 scatter/gather
definition, on two calls in a row, the second smaller (the static scratch
keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

import mipsgen
from gpu_util import DEV, log, to_dev
from oracle import backward as B

pytestmark = pytest.mark.gpu


def _close(gpu, ref, rtol=1e-5):
    ref = np.asarray(ref)
    atol = 1e-6 * float(np.abs(ref).max())
    np.testing.assert_allclose(gpu, ref, rtol=rtol, atol=atol)


def _case(n_u, n_i, f, K, seed):
    import paper_1706_01449_amd as mips
    log(f"noalloc backward: n_u={n_u} n_i={n_i} f={f} K={K} seed={seed}")
    U, I = mipsgen.generate("grad", seed, n_users=n_u, n_items=n_i, f=f)
    Ut, It = to_dev(U, I)
    idx, score = mips.bmm_topk(Ut, It, K, "bf16")
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n_u, K)).astype(np.float32)
    Gt = torch.from_numpy(G).to(DEV)
    dU0, dI0 = mips.topk_backward(Ut, It, idx, Gt)
    dU1, dI1 = mips.topk_backward(Ut, It, idx, Gt, noalloc=True)
    torch.cuda.synchronize()
    # dU is summed in k order on both paths: identical bits
    np.testing.assert_array_equal(dU1.cpu().numpy(), dU0.cpu().numpy())
    # dI: float32 atomics in run order, so the last bits may differ
    _close(dI1.cpu().numpy(), dI0.cpu().numpy(), rtol=1e-6)
    rU, rI = B.scatter_gather_grads(U, I, idx.cpu().numpy(), G)
    _close(dU1.cpu().numpy(), rU)
    _close(dI1.cpu().numpy(), rI)


def test_noalloc_backward_two_calls_second_smaller():
    _case(4000, 20000, 64, 32, 11)
    _case(700, 3000, 16, 8, 12)


def test_noalloc_backward_rejects_calls_beyond_its_scratch():
    import paper_1706_01449_amd as mips
    L = mips.lib()
    n_i, f = 6_000_000, 1          # 12 n_i bytes > 64 MiB
    U = torch.zeros((1, f), dtype=torch.float32, device=DEV)
    I = torch.zeros((n_i, f), dtype=torch.float32, device=DEV)
    idx = torch.zeros((1, 1), dtype=torch.int32, device=DEV)
    G = torch.ones((1, 1), dtype=torch.float32, device=DEV)
    dU = torch.empty_like(U)
    dI = torch.empty_like(I)
    rc = L.mips_topk_backward_noalloc(U.data_ptr(), I.data_ptr(), 1, n_i, f, 1, idx.data_ptr(),
                                      G.data_ptr(), dU.data_ptr(), dI.data_ptr(), None)
    assert rc == -6
    assert b"static scratch" in L.mips_last_error_message()
