"""GPU parity of the brute-force path (score tiles + streaming top-K +
certification + float64 rescore) against the CPU oracle, through the C ABI.

Bar: indices bit-equal, scores (float64 keys) bit-equal, for every precision
of the screen."""
import numpy as np
import pytest

import mipsgen
from gpu_util import assert_manifest, assert_parity, gpu_topk, log

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16", "fp8"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("K", [1, 10])
def test_tiny_workload_all_users(prec, K):
    log(f"tiny workload prec={prec} K={K}")
    U, I = mipsgen.generate("tiny", 0)
    idx, score, st = gpu_topk(U, I, K, prec, stats=True)
    assert_parity(idx, score, U, I, K)
    assert st["nonfinite_input"] == 0
    assert st["items_scored"] == U.shape[0] * I.shape[0]


# (n_u, n_i, f, K): ragged tails in every dimension, f not a multiple of the
# matrix-core K-step, K across the compiled list sizes.
SHAPES = [
    (1, 1, 1, 1), (3, 2, 5, 2), (33, 70, 17, 5), (100, 31, 3, 31), (70, 1000, 50, 64),
    (65, 300, 128, 16), (40, 513, 100, 10), (257, 129, 64, 50), (129, 64, 16, 64),
    (31, 95, 33, 8), (64, 1025, 7, 32),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_ragged_shapes(prec, shape):
    n_u, n_i, f, K = shape
    log(f"ragged {shape} prec={prec}")
    U, I = mipsgen.generate("mf", 7, n_users=n_u, n_items=n_i, f=f)
    idx, score = gpu_topk(U, I, K, prec)
    assert_parity(idx, score, U, I, K)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
@pytest.mark.parametrize("shape", [(50, 300, 16, 65), (20, 300, 12, 300), (30, 400, 200, 10),
                                   (10, 5000, 8, 1000)], ids=lambda s: "x".join(map(str, s)))
def test_generic_exact_path(prec, shape):
    # K > 64 or f > 128 runs on the exact float64 kernel for every user
    n_u, n_i, f, K = shape
    log(f"generic {shape} prec={prec}")
    U, I = mipsgen.generate("tiny", 3, n_users=n_u, n_items=n_i, f=f)
    idx, score, st = gpu_topk(U, I, K, prec, stats=True)
    assert_parity(idx, score, U, I, K)
    assert st["overflow_users"] == n_u


@pytest.mark.parametrize("prec", PRECS)
def test_ties_zero_rows_duplicates(prec):
    log(f"ties prec={prec}")
    U, I = mipsgen.generate("mf", 11, n_users=150, n_items=900, f=24)
    U[0] = 0.0                   # zero user: all keys 0 -> items 0..K-1
    U[77] = 0.0
    I[5] = I[100]                # exact duplicates tie; lower index first
    I[6] = I[100]
    I[899] = I[100]
    I[300] = 0.0                 # zero item
    U[10] = -U[11]
    idx, score = gpu_topk(U, I, 20, prec)
    assert_parity(idx, score, U, I, 20)
    np.testing.assert_array_equal(idx[0], np.arange(20))


@pytest.mark.parametrize("prec", PRECS)
def test_integer_massive_ties(prec):
    # f = 1 with small integers: thousands of exact ties per user
    log(f"massive ties prec={prec}")
    rng = np.random.default_rng(3)
    U = rng.integers(-3, 4, size=(90, 1)).astype(np.float32)
    I = rng.integers(-5, 6, size=(2000, 1)).astype(np.float32)
    idx, score, st = gpu_topk(U, I, 16, prec, stats=True)
    assert_parity(idx, score, U, I, 16)


@pytest.mark.parametrize("prec", PRECS)
def test_identity_items_closed_form(prec):
    f = 40
    I = np.eye(f, dtype=np.float32)
    rng = np.random.default_rng(9)
    U = rng.standard_normal((70, f)).astype(np.float32)
    idx, score = gpu_topk(U, I, f, prec)
    cols = np.arange(f)
    for u in range(70):
        np.testing.assert_array_equal(idx[u], np.lexsort((cols, -U[u])))


@pytest.mark.parametrize("prec", PRECS)
def test_wide_dynamic_range(prec):
    log(f"dynamic range prec={prec}")
    U, I = mipsgen.generate("mf", 5, n_users=200, n_items=1500, f=32)
    I[:500] *= 1e-6
    I[500:510] *= 1e3
    U[:50] *= 1e-8
    U[50:60] *= 1e8
    idx, score = gpu_topk(U, I, 10, prec)
    assert_parity(idx, score, U, I, 10)


def test_nonfinite_input_reported():
    import paper_1706_01449_amd as mips
    U, I = mipsgen.generate("tiny", 0, n_users=64, n_items=128)
    I[3, 2] = np.nan
    with pytest.raises(mips.MipsError) as ei:
        gpu_topk(U, I, 5, "bf16", stats=True)
    assert ei.value.code == -2


def test_deterministic_repeat():
    U, I = mipsgen.generate("mf", 2, n_users=3000, n_items=4000, f=50)
    a = gpu_topk(U, I, 10, "bf16")
    b = gpu_topk(U, I, 10, "bf16")
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("K", [1, 5, 10, 50])
def test_mf_full_size_all_users(prec, K):
    """480,000 x 17,770, f = 50 (the Netflix shape) in the benchmark's
    configuration: every user's indices and float64 keys equal the oracle's
    (hashes of the oracle's full run)."""
    log(f"mf full size prec={prec} K={K}")
    U, I = _mf_full()
    idx, score, st = gpu_topk(U, I, K, prec, stats=True)
    log(f"  stats {st}")
    assert_manifest(idx, score, U, I, "mf", 0, K, what=f"mf {prec} K={K}")
    # Users whose screen candidates overflow finish on the exact float64
    # fallback (same answer, slower).
    assert st["overflow_users"] <= _overflow_limit(U.shape[0], prec, K)


def _overflow_limit(n_u, prec, K):
    # the coarse E4M3 screen at large K keeps hundreds of candidates per
    # user, so more users take the exact path there
    return n_u // 100 if (prec == "fp8" and K >= 32) else n_u // 1000


@pytest.mark.parametrize("prec", PRECS)
def test_precision_workload_full_size(prec):
    """1,000,000 x 136,000, f = 100, K = 10 (the precision form): every
    user's indices and float64 keys equal the oracle's."""
    log(f"precision workload full size prec={prec}")
    U, I = _precision_full()
    idx, score, st = gpu_topk(U, I, 10, prec, stats=True)
    log(f"  stats {st}")
    assert_manifest(idx, score, U, I, "precision", 0, 10, what=f"precision {prec}")
    assert st["overflow_users"] <= U.shape[0] // 1000


_PR = {}


def _precision_full():
    if "x" not in _PR:
        _MF.clear()
        _PR["x"] = mipsgen.generate("precision", 0)
    return _PR["x"]


_MF = {}


def _mf_full():
    if "x" not in _MF:
        _MF["x"] = mipsgen.generate("mf", 0)
    return _MF["x"]


@pytest.mark.parametrize("prec", PRECS)
def test_forced_candidate_overflow_stays_exact(prec):
    """A test knob of 2 candidate slots per lane forces most users onto the
    exact float64 fallback; the answer must not change."""
    import paper_1706_01449_amd as mips
    U, I = mipsgen.generate("mf", 4, n_users=700, n_items=3000, f=50)
    with mips.debug_knob("cand_cap", 2):
        idx, score, st = gpu_topk(U, I, 10, prec, stats=True)
    assert st["overflow_users"] > 600
    assert_parity(idx, score, U, I, 10)


@pytest.mark.parametrize("mode", ["wave-cascade", "wave", "group"])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(300, 2000, 50, 10), (200, 1500, 64, 32), (150, 1000, 33, 50),
                                   (97, 700, 100, 64), (64, 40, 7, 40)],
                         ids=lambda s: "x".join(map(str, s)))
def test_certification_kernels(mode, prec, shape):
    """Both certification kernels (one wave per user with LDS-staged rows and
    a rising threshold, with or without the bfloat16 cascade of E4M3
    candidates, or a group of lanes per user) give the oracle's answer: f
    odd, even and a multiple of 4 (row loads of 1, 2 and 4 floats), K past
    the fused sizes, duplicate rows that tie."""
    n_u, n_i, f, K = shape
    log(f"certify {mode} {shape} prec={prec}")
    U, I = mipsgen.generate("mf", 9, n_users=n_u, n_items=n_i, f=f)
    I[3] = I[n_i // 2]
    I[n_i - 1] = I[n_i // 2]
    import paper_1706_01449_amd as mips
    if mode == "wave-cascade" and prec != "fp8":
        pytest.skip("the bfloat16 cascade re-screens E4M3 candidates only")
    cascade = mode == "wave-cascade"
    with mips.debug_knob("certify_kernel", 1 if mode.startswith("wave") else 2):
        idx, score, st = gpu_topk(U, I, K, "fp8_bf16" if cascade else prec, stats=True)
    assert_parity(idx, score, U, I, K)
    assert st["rescored_pairs"] <= st["candidates_total"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(300, 1000, 16, 10), (257, 3001, 50, 1), (129, 2000, 100, 50)],
                         ids=lambda s: "x".join(map(str, s)))
def test_norm_pruned_small(prec, shape):
    """Norm-pruned brute force (stop test with theta_b = pi) returns the
    oracle's answer; ragged shapes, ties from duplicate rows, a zero row."""
    import paper_1706_01449_amd as mips
    import torch
    from gpu_util import to_dev
    n_u, n_i, f, K = shape
    U, I = mipsgen.generate("mf", 12, n_users=n_u, n_items=n_i, f=f)
    I[7] = I[3]
    U[2] = 0.0
    Ut, It = to_dev(U, I)
    idx, sc, st = mips.norm_pruned_topk(Ut, It, K, prec, stats=True)
    torch.cuda.synchronize()
    assert_parity(idx.cpu().numpy(), sc.cpu().numpy(), U, I, K)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("f", [50, 100])
@pytest.mark.parametrize("n_i", [417, 449, 800, 801, 1025])
def test_sweep_tile_count_parity(prec, f, n_i):
    """The sweep takes tiles in pairs and an odd last tile alone: both
    parities of the tile count left after the warm-up (14, 15, 25, 26, 33
    tiles), for the brute force (four user blocks per wave in bfloat16 at
    f = 50, two at f = 100, one in float32 at f = 100) and the norm-pruned
    sweep, return the oracle's answer; 300 users leave a partial block."""
    import paper_1706_01449_amd as mips
    import torch
    from gpu_util import to_dev
    log(f"tile-count parity n_i={n_i} f={f} prec={prec}")
    U, I = mipsgen.generate("mf", 21, n_users=300, n_items=n_i, f=f)
    idx, score = gpu_topk(U, I, 10, prec)
    assert_parity(idx, score, U, I, 10)
    Ut, It = to_dev(U, I)
    pidx, psc = mips.norm_pruned_topk(Ut, It, 10, prec)
    torch.cuda.synchronize()
    assert_parity(pidx.cpu().numpy(), psc.cpu().numpy(), U, I, 10)


@pytest.mark.parametrize("prec", PRECS)
def test_norm_pruned_mf_full_size(prec):
    """480,000 x 17,770, f = 50, K = 10: every user's answer equals the
    oracle's, with fewer items scored than the brute force."""
    import paper_1706_01449_amd as mips
    import torch
    from gpu_util import to_dev
    log(f"norm-pruned mf full size prec={prec}")
    U, I = _mf_full()
    Ut, It = to_dev(U, I)
    idx, sc, st = mips.norm_pruned_topk(Ut, It, 10, prec, stats=True)
    torch.cuda.synchronize()
    log(f"  stats {st}")
    assert_manifest(idx.cpu().numpy(), sc.cpu().numpy(), U, I, "mf", 0, 10,
                    what=f"norm-pruned {prec}")
    assert st["mean_items_visited"] < I.shape[0]
