"""Host-side checks of libmips that need no GPU: the library loads, exports
every function include/mips.h declares, and rejects bad arguments before it
touches the device."""
import ctypes

import pytest

import paper_1706_01449_amd as mips


@pytest.fixture(scope="module")
def L():
    return mips.lib()


def test_exports_every_declared_symbol(L):
    names = mips.header_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    assert L.mips_status_string(0) == b"MIPS_OK"
    assert L.mips_status_string(-1) == b"MIPS_ERR_ARG"
    assert L.mips_status_string(-4) == b"MIPS_ERR_WORKSPACE"
    assert L.mips_status_string(-6) == b"MIPS_ERR_UNSUPPORTED"


@pytest.mark.parametrize("n_u,n_i,f,K,prec,code", [
    (0, 10, 4, 1, 1, -1),          # no users
    (5, 0, 4, 1, 1, -1),           # no items
    (5, 10, 0, 1, 1, -1),          # f < 1
    (5, 10, 300, 1, 1, -1),        # f > 256
    (5, 10, 4, 0, 1, -1),          # K < 1
    (5, 10, 4, 11, 1, -1),         # K > n_i
    (5, 10, 4, 1, 7, -1),          # bad precision
    (5, 1 << 31, 4, 1, 1, -1),     # n_i >= 2^31
    (5, 10000, 4, 5000, 1, -6),    # K above the supported maximum
])
def test_argument_errors_before_launch(L, n_u, n_i, f, K, prec, code):
    assert L.mips_bmm_topk_workspace_size(n_u, n_i, f, K, prec) == 0
    rc = L.mips_bmm_topk(ctypes.c_void_p(16), n_u, ctypes.c_void_p(16), n_i, f, K, prec,
                         ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(256), 1 << 40,
                         None, None)
    assert rc == code
    assert L.mips_last_error_message()


def test_null_pointers_and_workspace(L):
    need = L.mips_bmm_topk_workspace_size(100, 50, 8, 5, 1)
    assert need > 0
    p = ctypes.c_void_p(256)
    assert L.mips_bmm_topk(None, 100, p, 50, 8, 5, 1, p, p, p, need, None, None) == -1
    assert L.mips_bmm_topk(p, 100, p, 50, 8, 5, 1, p, p, None, need, None, None) == -4
    assert L.mips_bmm_topk(p, 100, p, 50, 8, 5, 1, p, p, p, need - 1, None, None) == -4
    assert L.mips_bmm_topk(p, 100, p, 50, 8, 5, 1, p, p, ctypes.c_void_p(257), need, None,
                           None) == -1


def test_workspace_grows_with_precision_candidates(L):
    a = L.mips_bmm_topk_workspace_size(480000, 17770, 50, 10, 1)
    b = L.mips_bmm_topk_workspace_size(480000, 17770, 50, 10, 2)
    assert 0 < a < b


def test_backward_argument_errors(L):
    p = ctypes.c_void_p(256)
    assert L.mips_topk_backward(None, p, 4, 4, 4, 2, p, p, p, p, None) == -1
    assert L.mips_topk_backward(p, p, 0, 4, 4, 2, p, p, p, p, None) == -1
    assert L.mips_topk_backward(p, p, 4, 4, 0, 2, p, p, p, p, None) == -1
    assert L.mips_topk_backward(p, p, 4, 4, 4, 0, p, p, p, p, None) == -1
