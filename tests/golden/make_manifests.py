"""Write SHA-256 manifests of the oracle's answer on every user of the
full-size workloads.

The answer is the one defined in Section II-B (problem statement) and
computed by the brute force of Section II-C: for each user the K items with
the largest float64 key, ties to the lower item index.  This script calls
only the CPU oracle (``oracle.topk``) and the seeded input generator
(``mipsgen``); nothing from the HIP library.

For each (workload, seed, K) it stores
  * the SHA-256 of the float32 input bytes of U and I (so a test can tell a
    changed generator from a changed answer),
  * the SHA-256 of the oracle's idx (int32, n_u x K, C order, little endian)
    and key (float64) bytes over all users,
  * the same two hashes per block of ``BLOCK`` consecutive users, so that a
    failing test can name the blocks that differ and diff a few of their
    users element by element against the oracle.

Usage: ``python tests/golden/make_manifests.py [workload[:K] ...]``; with no
arguments every case below is written to ``tests/golden/manifests/``.  The
full set takes about half an hour on 8 cores, most of it the
1,000,000 x 136,000, f = 100 case.
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import mipsgen  # noqa: E402
from oracle import topk as oracle_topk  # noqa: E402

OUT = os.path.join(HERE, "manifests")
BLOCK = 16384
SEED = 0

# (workload, K): the full-size configurations the GPU tests run.
CASES = [
    ("mf", 1), ("mf", 5), ("mf", 10), ("mf", 50),
    ("clustered", 10),
    ("grad", 32),
    ("precision", 10),
]


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def block_hashes(a: np.ndarray, block: int = BLOCK) -> list[str]:
    return [sha(a[s:s + block]) for s in range(0, a.shape[0], block)]


def manifest_path(workload: str, seed: int, K: int) -> str:
    return os.path.join(OUT, f"{workload}_seed{seed}_K{K}.json")


def write_case(workload: str, K: int, seed: int = SEED) -> str:
    U, I = mipsgen.generate(workload, seed)
    t0 = time.time()
    idx, key = oracle_topk.topk(U, I, K, mode=1)
    dt = time.time() - t0
    assert idx.dtype == np.int32 and key.dtype == np.float64
    m = {
        "what": ("oracle top-K (float64 left-to-right keys, order (key desc, index asc); "
                 "Section II-B problem statement, Section II-C brute force) on every user"),
        "workload": workload, "seed": seed, "K": K,
        "n_users": int(U.shape[0]), "n_items": int(I.shape[0]), "f": int(U.shape[1]),
        "U_sha256": sha(U), "I_sha256": sha(I),
        "idx_dtype": "int32", "key_dtype": "float64",
        "idx_sha256": sha(idx), "key_sha256": sha(key),
        "block_users": BLOCK,
        "idx_block_sha256": block_hashes(idx),
        "key_block_sha256": block_hashes(key),
        "written_by": "tests/golden/make_manifests.py (calls oracle.topk and mipsgen only)",
        "oracle_seconds": round(dt, 1),
        "oracle_threads": oracle_topk.num_threads(0),
        "numpy": np.__version__,
        "machine": platform.machine(),
    }
    os.makedirs(OUT, exist_ok=True)
    path = manifest_path(workload, seed, K)
    with open(path + ".tmp", "w") as fh:
        json.dump(m, fh, indent=1)
        fh.write("\n")
    os.replace(path + ".tmp", path)
    return path


def main(argv: list[str]) -> int:
    cases = CASES
    if argv:
        cases = []
        for a in argv:
            w, _, k = a.partition(":")
            cases += [(w, int(k))] if k else [c for c in CASES if c[0] == w]
    for w, K in cases:
        t0 = time.time()
        p = write_case(w, K)
        print(f"{w} K={K}: {os.path.relpath(p, ROOT)} ({time.time() - t0:.1f} s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
