"""Seeded synthetic inputs for exact batch MIPS (user and item factor matrices).

This module only draws random numbers; it holds none of the method's
arithmetic (no inner products, norms used for ranking, bounds or sorting).
Both the CPU oracle tests and the GPU path read their inputs from here, so
both sides see byte-identical FP32 matrices for a given (workload, seed).

The paper evaluates on matrix-factorisation models trained on Netflix, Yahoo
Music and GloVe data (Section V-A, Table I).  Those datasets and trained
models are not available, so every workload below is a synthetic stand-in
with the shape of one of them:

* ``tiny``       users 2,000 x 16, items 1,000 x 16, entries i.i.d. N(0, 1).
* ``mf``         MF-shaped factors: each row is r * g / ||g||, g ~ N(0, I_f),
                 r ~ LogNormal(0, 0.5).  The Netflix shape is 480,000 users x
                 17,770 items at f = 50.
* ``clustered``  users from a 64-component Gaussian mixture (means N(0, I_f),
                 per-coordinate spread 0.3, components uniform); item
                 directions uniform on the sphere with a rank power-law norm
                 ||i|| = rho^-1.1 / median(rho^-1.1), rho a random permutation
                 of 1..n_i.  Used for the pruning index (Section III).
* ``precision``  MF-shaped rows at 1,000,000 x 100 users, 136,000 x 100 items
                 (the Yahoo R2 item count, rounded).
* ``grad``       MF-shaped rows at 65,536 x 64 users, 100,000 x 64 items.

Draw order is fixed: all user draws, then all item draws.  Values are drawn
in float64 and rounded to float32 (round-to-nearest-even) at the end.
"""
from __future__ import annotations

import numpy as np

WORKLOAD_IDS = {"tiny": 1, "mf": 2, "clustered": 3, "precision": 4, "grad": 5}

# Full sizes of each workload: (n_users, n_items, f).
FULL_SIZES = {
    "tiny": (2_000, 1_000, 16),
    "mf": (480_000, 17_770, 50),
    "clustered": (480_000, 17_770, 50),
    "precision": (1_000_000, 136_000, 100),
    "grad": (65_536, 100_000, 64),
}


def rng_for(workload: str, seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([WORKLOAD_IDS[workload], int(seed)]))


def _normal_rows(rng, n, f):
    return rng.standard_normal((n, f))


def _mf_rows(rng, n, f):
    g = rng.standard_normal((n, f))
    r = rng.lognormal(mean=0.0, sigma=0.5, size=n)
    nrm = np.sqrt(np.einsum("ij,ij->i", g, g))
    nrm[nrm == 0.0] = 1.0
    return g * (r / nrm)[:, None]


def _mixture_users(rng, n, f, n_comp=64, spread=0.3):
    means = rng.standard_normal((n_comp, f))
    comp = rng.integers(0, n_comp, size=n)
    return means[comp] + spread * rng.standard_normal((n, f))


def _powerlaw_items(rng, n, f, exponent=1.1):
    g = rng.standard_normal((n, f))
    nrm = np.sqrt(np.einsum("ij,ij->i", g, g))
    nrm[nrm == 0.0] = 1.0
    rank = rng.permutation(n) + 1.0
    length = rank ** (-exponent)
    length = length / np.median(length)
    return g * (length / nrm)[:, None]


def generate(workload: str, seed: int = 0, n_users: int | None = None,
             n_items: int | None = None, f: int | None = None):
    """Return (U, I) as C-contiguous float32 arrays for a workload.

    Sizes default to the workload's full size; smaller sizes draw from the
    same distribution (used for quick parity cases).
    """
    nu0, ni0, f0 = FULL_SIZES[workload]
    nu = nu0 if n_users is None else int(n_users)
    ni = ni0 if n_items is None else int(n_items)
    ff = f0 if f is None else int(f)
    rng = rng_for(workload, seed)
    if workload == "tiny":
        U = _normal_rows(rng, nu, ff)
        I = _normal_rows(rng, ni, ff)
    elif workload in ("mf", "precision", "grad"):
        U = _mf_rows(rng, nu, ff)
        I = _mf_rows(rng, ni, ff)
    elif workload == "clustered":
        U = _mixture_users(rng, nu, ff)
        I = _powerlaw_items(rng, ni, ff)
    else:
        raise ValueError(workload)
    return (np.ascontiguousarray(U.astype(np.float32)),
            np.ascontiguousarray(I.astype(np.float32)))


def grad_slice(seed: int = 0):
    """Small float64 slice for finite-difference gradient checks:
    users 64 x 16, items 512 x 16, MF-shaped rows."""
    rng = np.random.default_rng(np.random.SeedSequence([WORKLOAD_IDS["grad"], 1000 + int(seed)]))
    U = _mf_rows(rng, 64, 16)
    I = _mf_rows(rng, 512, 16)
    return np.ascontiguousarray(U), np.ascontiguousarray(I)


def sample_users(n_users: int, n_sample: int, seed: int = 0) -> np.ndarray:
    """Sorted random subset of user indices for sampled parity checks."""
    rng = np.random.default_rng(np.random.SeedSequence([99, int(seed), int(n_users)]))
    k = min(n_sample, n_users)
    return np.sort(rng.choice(n_users, size=k, replace=False)).astype(np.int64)
