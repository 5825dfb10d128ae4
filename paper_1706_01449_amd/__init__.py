"""Exact batch maximum inner product search on AMD Instinct MI355X.

Python binding of ``libmips`` (HIP kernels for gfx950 behind the C ABI of
``include/mips.h``).  PyTorch supplies device memory and streams; every step
of the computation runs in the library's kernels.  There is no CPU path: if
the compiled library is missing the calls raise.
"""
from .mips import (  # noqa: F401
    MipsError, PRECISIONS, bmm_topk, norm_pruned_topk, maximus_build, MaximusIndex, optimus_topk, topk_backward,
    lib, lib_path, profile_enable, profile_read, PROFILE_PHASES, header_symbols, debug_set, debug_knob,
)
from .autograd import TopKScores, topk_scores  # noqa: F401
