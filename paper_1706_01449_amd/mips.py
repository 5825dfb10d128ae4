"""ctypes binding of libmips.  Argument marshalling only: the arrays are
passed to the C ABI as device pointers together with the current HIP stream
of their device."""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_lib", "libmips.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "mips.h")
_lib = None

PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2, "fp8_e4m3": 2, "fp8_bf16": 3}
DEBUG_KNOBS = {"cand_cap": 0, "certify_kernel": 1}
PROFILE_PHASES = ["item_prep", "screen", "certify", "fallback", "build", "walk", "backward"]


class MipsError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(message)
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("candidates_total", ctypes.c_int64),
        ("candidates_max_per_user", ctypes.c_int64),
        ("rescored_pairs", ctypes.c_int64),
        ("overflow_users", ctypes.c_int64),
        ("items_scored", ctypes.c_int64),
        ("mean_items_visited", ctypes.c_double),
        ("max_screen_abs_err", ctypes.c_double),
        ("max_screen_rel_err", ctypes.c_double),
        ("nonfinite_input", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class OptimusReport(ctypes.Structure):
    _fields_ = [
        ("choice", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("sample_users", ctypes.c_int64),
        ("build_ms", ctypes.c_double),
        ("bmm_sample_ms", ctypes.c_double),
        ("maximus_sample_ms", ctypes.c_double),
        ("est_bmm_ms", ctypes.c_double),
        ("est_maximus_ms", ctypes.c_double),
        ("finish_ms", ctypes.c_double),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}
        d["choice"] = "maximus" if self.choice == 1 else "bmm"
        return d


def lib_path() -> str:
    return _LIB_PATH


def header_symbols() -> list[str]:
    """Function names declared in include/mips.h."""
    with open(_HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(mips_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def lib():
    """Load libmips.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise MipsError(-6, f"libmips.so not found at {_LIB_PATH}; build it with "
                            "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(_LIB_PATH)
    c_i32, c_i64, c_u64, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    vp = ctypes.c_void_p
    L.mips_bmm_topk_workspace_size.restype = c_sz
    L.mips_bmm_topk_workspace_size.argtypes = [c_i64, c_i64, c_i32, c_i32, c_i32]
    L.mips_bmm_topk.restype = ctypes.c_int
    L.mips_bmm_topk.argtypes = [vp, c_i64, vp, c_i64, c_i32, c_i32, c_i32, vp, vp, vp, c_sz, vp,
                                ctypes.POINTER(Stats)]
    L.mips_norm_pruned_topk.restype = ctypes.c_int
    L.mips_norm_pruned_topk.argtypes = L.mips_bmm_topk.argtypes
    L.mips_maximus_build.restype = ctypes.c_int
    L.mips_maximus_build.argtypes = [vp, c_i64, vp, c_i64, c_i32, c_i32, c_i32, c_u64, c_i32, vp,
                                     ctypes.POINTER(vp)]
    L.mips_maximus_query_workspace_size.restype = c_sz
    L.mips_maximus_query_workspace_size.argtypes = [vp, c_i32, c_i32]
    L.mips_maximus_query.restype = ctypes.c_int
    L.mips_maximus_query.argtypes = [vp, c_i32, c_i32, vp, vp, vp, c_sz, vp, ctypes.POINTER(Stats)]
    L.mips_maximus_query_users_workspace_size.restype = c_sz
    L.mips_maximus_query_users_workspace_size.argtypes = [vp, c_i64, c_i32, c_i32]
    L.mips_maximus_query_users.restype = ctypes.c_int
    L.mips_maximus_query_users.argtypes = [vp, vp, c_i64, c_i32, c_i32, vp, vp, vp, c_sz, vp,
                                           ctypes.POINTER(Stats)]
    L.mips_optimus_topk.restype = ctypes.c_int
    L.mips_optimus_topk.argtypes = [vp, c_i64, vp, c_i64, c_i32, c_i32, c_i32, c_i32, c_i32, c_u64,
                                    c_i64, vp, vp, vp, ctypes.POINTER(OptimusReport)]
    L.mips_maximus_free.restype = None
    L.mips_maximus_free.argtypes = [vp]
    L.mips_maximus_export.restype = ctypes.c_int
    L.mips_maximus_export.argtypes = [vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                                      ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), vp, vp, vp, vp,
                                      vp, vp]
    L.mips_topk_backward.restype = ctypes.c_int
    L.mips_topk_backward.argtypes = [vp, vp, c_i64, c_i64, c_i32, c_i32, vp, vp, vp, vp, vp]
    L.mips_topk_backward_noalloc.restype = ctypes.c_int
    L.mips_topk_backward_noalloc.argtypes = L.mips_topk_backward.argtypes
    L.mips_status_string.restype = ctypes.c_char_p
    L.mips_status_string.argtypes = [ctypes.c_int]
    L.mips_last_error_message.restype = ctypes.c_char_p
    L.mips_last_error_message.argtypes = []
    L.mips_debug_set.restype = ctypes.c_int
    L.mips_debug_set.argtypes = [c_i32, c_i32]
    L.mips_profile_enable.restype = ctypes.c_int
    L.mips_profile_enable.argtypes = [ctypes.c_int]
    L.mips_profile_read.restype = ctypes.c_int
    L.mips_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_i64)]
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        L = lib()
        raise MipsError(rc, f"{L.mips_status_string(rc).decode()}: "
                            f"{L.mips_last_error_message().decode()}")


def _prec(p) -> int:
    if isinstance(p, int):
        return p
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"unknown precision {p!r}; use one of {sorted(PRECISIONS)}") from None


def _mat(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or x.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device (got {x.device})")
    if x.dtype != torch.float32:
        raise ValueError(f"{name} must be float32 (got {x.dtype})")
    return x.contiguous()


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def bmm_topk(U: torch.Tensor, I: torch.Tensor, K: int, precision="bf16", stats: bool = False,
             workspace: torch.Tensor | None = None):
    """Exact top-K items of every user by brute force (blocked matrix multiply
    fused with a streaming top-K).  Returns (idx int32 [n_u, K], score float64
    [n_u, K]) and, with ``stats=True``, a dict of counters (synchronises)."""
    return _bmm_call("mips_bmm_topk", U, I, K, precision, stats, workspace)


def norm_pruned_topk(U: torch.Tensor, I: torch.Tensor, K: int, precision="bf16",
                     stats: bool = False, workspace: torch.Tensor | None = None):
    """Brute force with per-user early termination on the item norms (the
    Maximus stop test with theta_b = pi).  Same result as bmm_topk."""
    return _bmm_call("mips_norm_pruned_topk", U, I, K, precision, stats, workspace)


def _bmm_call(fn: str, U, I, K, precision, stats, workspace):
    U = _mat(U, "U")
    I = _mat(I, "I")
    if U.shape[1] != I.shape[1]:
        raise ValueError("U and I must have the same number of columns")
    if U.device != I.device:
        raise ValueError("U and I must be on the same device")
    L = lib()
    n_u, f = U.shape
    n_i = I.shape[0]
    p = _prec(precision)
    need = L.mips_bmm_topk_workspace_size(n_u, n_i, f, int(K), p)
    if need == 0:
        # let the library produce the argument error message
        _check(L.mips_bmm_topk(U.data_ptr(), n_u, I.data_ptr(), n_i, f, int(K), p, None, None,
                               None, 0, None, None) or -1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=U.device)
    idx = torch.empty((n_u, K), dtype=torch.int32, device=U.device)
    score = torch.empty((n_u, K), dtype=torch.float64, device=U.device)
    st = Stats() if stats else None
    rc = getattr(L, fn)(U.data_ptr(), n_u, I.data_ptr(), n_i, f, int(K), p, idx.data_ptr(),
                        score.data_ptr(), workspace.data_ptr(), workspace.numel(),
                        _stream(U.device), ctypes.byref(st) if st is not None else None)
    _check(rc)
    if stats:
        return idx, score, st.as_dict()
    return idx, score


class MaximusIndex:
    """Maximus index (k-means clusters, per-cluster bound-ordered item lists)
    owned by libmips; freed when this object is garbage collected."""

    def __init__(self, handle, device, n_u, n_i, f):
        self._h = handle
        self.device = device
        self.n_u, self.n_i, self.f = n_u, n_i, f

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            try:
                lib().mips_maximus_free(h)
            except Exception:
                pass

    def query(self, K: int, precision="bf16", stats: bool = False,
              workspace: torch.Tensor | None = None):
        L = lib()
        p = _prec(precision)
        need = L.mips_maximus_query_workspace_size(self._h, int(K), p)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        idx = torch.empty((self.n_u, K), dtype=torch.int32, device=self.device)
        score = torch.empty((self.n_u, K), dtype=torch.float64, device=self.device)
        st = Stats() if stats else None
        rc = L.mips_maximus_query(self._h, int(K), p, idx.data_ptr(), score.data_ptr(),
                                  workspace.data_ptr(), workspace.numel(), _stream(self.device),
                                  ctypes.byref(st) if st is not None else None)
        _check(rc)
        if stats:
            return idx, score, st.as_dict()
        return idx, score

    def query_users(self, Uq: torch.Tensor, K: int, precision="bf16", stats: bool = False,
                    workspace: torch.Tensor | None = None):
        """Top-K of arbitrary user vectors (new users or any subset) against
        the index's items."""
        L = lib()
        p = _prec(precision)
        Uq = _mat(Uq, "Uq")
        if Uq.shape[1] != self.f:
            raise MipsError(-1, f"Uq has {Uq.shape[1]} factors, the index {self.f}")
        n_q = Uq.shape[0]
        need = L.mips_maximus_query_users_workspace_size(self._h, n_q, int(K), p)
        if need == 0:
            raise MipsError(-1, "invalid query sizes")
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        idx = torch.empty((n_q, K), dtype=torch.int32, device=self.device)
        score = torch.empty((n_q, K), dtype=torch.float64, device=self.device)
        st = Stats() if stats else None
        rc = L.mips_maximus_query_users(self._h, Uq.data_ptr(), n_q, int(K), p, idx.data_ptr(),
                                        score.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                        _stream(self.device),
                                        ctypes.byref(st) if st is not None else None)
        _check(rc)
        if stats:
            return idx, score, st.as_dict()
        return idx, score

    def export(self):
        """Host copies of the index: centroids, theta_b, assignment, lists, bounds."""
        import numpy as np
        L = lib()
        C = ctypes.c_int32()
        f = ctypes.c_int32()
        nu = ctypes.c_int64()
        ni = ctypes.c_int64()
        _check(L.mips_maximus_export(self._h, ctypes.byref(C), ctypes.byref(f), ctypes.byref(nu),
                                     ctypes.byref(ni), None, None, None, None, None,
                                     _stream(self.device)))
        C, f, nu, ni = C.value, f.value, nu.value, ni.value
        cent = np.empty((C, f), dtype=np.float64)
        tb = np.empty(C, dtype=np.float64)
        assign = np.empty(nu, dtype=np.int32)
        lists = np.empty((C, ni), dtype=np.int32)
        bounds = np.empty((C, ni), dtype=np.float32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(L.mips_maximus_export(self._h, None, None, None, None, ptr(cent), ptr(tb),
                                     ptr(assign), ptr(lists), ptr(bounds), _stream(self.device)))
        return {"centroids": cent, "theta_b": tb, "assign": assign, "lists": lists,
                "bounds": bounds}


def maximus_build(U: torch.Tensor, I: torch.Tensor, n_clusters: int = 8, kmeans_iters: int = 3,
                  seed: int = 0, block_items: int = 0) -> MaximusIndex:
    """Build the Maximus index (paper Section III)."""
    U = _mat(U, "U")
    I = _mat(I, "I")
    if U.shape[1] != I.shape[1]:
        raise ValueError("U and I must have the same number of columns")
    L = lib()
    h = ctypes.c_void_p()
    rc = L.mips_maximus_build(U.data_ptr(), U.shape[0], I.data_ptr(), I.shape[0], U.shape[1],
                              int(n_clusters), int(kmeans_iters), int(seed), int(block_items),
                              _stream(U.device), ctypes.byref(h))
    _check(rc)
    return MaximusIndex(h.value, U.device, U.shape[0], I.shape[0], U.shape[1])


def optimus_topk(U: torch.Tensor, I: torch.Tensor, K: int, precision="bf16", n_clusters: int = 64,
                 kmeans_iters: int = 3, seed: int = 0, sample_users: int = 0):
    """Exact top-K of every user with the method Optimus picks online (paper
    Section IV).  Returns (idx, score, report dict)."""
    U = _mat(U, "U")
    I = _mat(I, "I")
    if U.shape[1] != I.shape[1]:
        raise ValueError("U and I must have the same number of columns")
    n_u, f = U.shape
    idx = torch.empty((n_u, K), dtype=torch.int32, device=U.device)
    score = torch.empty((n_u, K), dtype=torch.float64, device=U.device)
    rep = OptimusReport()
    _check(lib().mips_optimus_topk(U.data_ptr(), n_u, I.data_ptr(), I.shape[0], f, int(K),
                                   _prec(precision), int(n_clusters), int(kmeans_iters), int(seed),
                                   int(sample_users), idx.data_ptr(), score.data_ptr(),
                                   _stream(U.device), ctypes.byref(rep)))
    return idx, score, rep.as_dict()


def topk_backward(U: torch.Tensor, I: torch.Tensor, idx: torch.Tensor, grad_scores: torch.Tensor,
                  noalloc: bool = False):
    """dU, dI of a loss on the top-K scores given dL/dS at the top-K positions.
    noalloc=True calls mips_topk_backward_noalloc (the library's static
    scratch, no device allocation inside the call)."""
    U = _mat(U, "U")
    I = _mat(I, "I")
    n_u, f = U.shape
    n_i = I.shape[0]
    K = idx.shape[1]
    idx = idx.to(torch.int32).contiguous()
    g = grad_scores.to(torch.float32).contiguous()
    if idx.shape != (n_u, K) or g.shape != (n_u, K):
        raise ValueError("idx and grad_scores must be n_u x K")
    dU = torch.empty_like(U)
    dI = torch.empty_like(I)
    fn = lib().mips_topk_backward_noalloc if noalloc else lib().mips_topk_backward
    _check(fn(U.data_ptr(), I.data_ptr(), n_u, n_i, f, K, idx.data_ptr(), g.data_ptr(),
              dU.data_ptr(), dI.data_ptr(), _stream(U.device)))
    return dU, dI


def debug_set(knob: str, value: int):
    """Set a test knob of the library (see mips_debug_set); 0 restores the
    normal behaviour."""
    _check(lib().mips_debug_set(DEBUG_KNOBS[knob], int(value)))


class debug_knob:
    """Context manager: a test knob set for the duration of a block."""

    def __init__(self, knob: str, value: int):
        self.knob, self.value = knob, value

    def __enter__(self):
        debug_set(self.knob, self.value)
        return self

    def __exit__(self, *exc):
        debug_set(self.knob, 0)
        return False


def profile_enable(on: bool = True):
    _check(lib().mips_profile_enable(1 if on else 0))


def profile_read():
    """Per-phase kernel milliseconds and launch counts since the last read
    (waits for the recorded events)."""
    n = len(PROFILE_PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().mips_profile_read(ms, cnt))
    return {PROFILE_PHASES[i]: (ms[i], cnt[i]) for i in range(n)}
