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


P = ctypes.c_void_p(256)


@pytest.mark.parametrize("args,code", [
    # (U, n_u, I, n_i, f, C, iters, seed, block_items, out)
    ((None, 100, P, 50, 8, 4, 3, 0, 0, True), -1),       # U is NULL
    ((P, 100, None, 50, 8, 4, 3, 0, 0, True), -1),       # I is NULL
    ((P, 100, P, 50, 8, 4, 3, 0, 0, False), -1),         # out_index is NULL
    ((P, 0, P, 50, 8, 1, 3, 0, 0, True), -1),            # no users
    ((P, 100, P, 0, 8, 4, 3, 0, 0, True), -1),           # no items
    ((P, 100, P, 50, 0, 4, 3, 0, 0, True), -1),          # f < 1
    ((P, 100, P, 50, 257, 4, 3, 0, 0, True), -1),        # f > 256
    ((P, 100, P, 50, 8, 0, 3, 0, 0, True), -1),          # no clusters
    ((P, 100, P, 50, 8, 101, 3, 0, 0, True), -1),        # more clusters than users
    ((P, 10000, P, 50, 8, 4097, 3, 0, 0, True), -1),     # more than 4096 clusters
    ((P, 100, P, 50, 8, 4, -1, 0, 0, True), -1),         # negative Lloyd iterations
    ((P, 100, P, 50, 8, 4, 101, 0, 0, True), -1),        # too many Lloyd iterations
    ((P, 100, P, 50, 8, 4, 3, 0, -32, True), -1),        # negative block
])
def test_maximus_build_argument_errors(L, args, code):
    U, n_u, I, n_i, f, C, iters, seed, blk, want_out = args
    h = ctypes.c_void_p(12345)
    out = ctypes.byref(h) if want_out else None
    rc = L.mips_maximus_build(U, n_u, I, n_i, f, C, iters, seed, blk, None, out)
    assert rc == code
    assert L.mips_last_error_message()
    if want_out:
        assert not h.value            # cleared: no index was built


def test_maximus_query_argument_errors(L):
    # without an index every query and size function refuses before any launch
    assert L.mips_maximus_query(None, 10, 1, P, P, P, 1 << 30, None, None) == -1
    assert L.mips_maximus_query_workspace_size(None, 10, 1) == 0
    assert L.mips_maximus_query_users(None, P, 10, 5, 1, P, P, P, 1 << 30, None, None) == -1
    assert L.mips_maximus_query_users_workspace_size(None, 10, 5, 1) == 0
    L.mips_maximus_free(None)      # NULL is ignored


@pytest.mark.parametrize("args,code", [
    # (U, n_u, I, n_i, f, K, prec, C, iters, sample, out)
    ((None, 100, P, 50, 8, 5, 1, 4, 3, 0, True), -1),     # U is NULL
    ((P, 100, P, 50, 8, 5, 1, 4, 3, 0, False), -1),       # outputs NULL
    ((P, 0, P, 50, 8, 5, 1, 1, 3, 0, True), -1),          # no users
    ((P, 100, P, 50, 8, 0, 1, 4, 3, 0, True), -1),        # K < 1
    ((P, 100, P, 50, 8, 51, 1, 4, 3, 0, True), -1),       # K > n_i
    ((P, 100, P, 50, 8, 5, 9, 4, 3, 0, True), -1),        # bad precision
    ((P, 100, P, 50, 8, 5, 1, 0, 3, 0, True), -1),        # no clusters
    ((P, 100, P, 50, 8, 5, 1, 101, 3, 0, True), -1),      # more clusters than users
    ((P, 100, P, 50, 8, 5, 1, 4, -2, 0, True), -1),       # negative Lloyd iterations
    ((P, 100, P, 50, 8, 5, 1, 4, 3, -7, True), -1),       # negative sample
    ((P, 100, P, 9000, 8, 5000, 1, 4, 3, 0, True), -6),   # K above the supported maximum
])
def test_optimus_argument_errors(L, args, code):
    U, n_u, I, n_i, f, K, prec, C, iters, sample, want_out = args
    o = P if want_out else None
    rc = L.mips_optimus_topk(U, n_u, I, n_i, f, K, prec, C, iters, 0, sample, o, o, None, None)
    assert rc == code
    assert L.mips_last_error_message()


def test_cascade_precision_code(L):
    # the E4M3 screen with the bfloat16 cascade shares the E4M3 workspace
    a = L.mips_bmm_topk_workspace_size(1000, 500, 32, 10, 2)
    b = L.mips_bmm_topk_workspace_size(1000, 500, 32, 10, 3)
    assert a == b > 0
    assert L.mips_bmm_topk_workspace_size(1000, 500, 32, 10, 4) == 0


def test_debug_knob_arguments(L):
    assert L.mips_debug_set(7, 1) == -1          # unknown knob
    assert L.mips_debug_set(0, -1) == -1         # negative value
    assert L.mips_debug_set(1, 3) == -1          # no such certification kernel
    assert L.mips_debug_set(0, 0) == 0
    assert L.mips_debug_set(1, 0) == 0
