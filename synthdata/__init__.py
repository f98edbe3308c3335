"""Seeded synthetic inputs shaped like the paper's simulation workloads.

This module only draws data. It holds none of the estimator's arithmetic and is
shared by the tests, the benchmark and the CPU oracle's callers; the oracle and
the HIP library never import each other.

Data model (paper Section 5, "Simulations"): inliers are N(0, Sigma) with unit
diagonal; a fraction eps of the rows, chosen uniformly without replacement, is
replaced by outliers.  Outlier types:

* ``shift``   -- N(mu_C, Sigma)
* ``cluster`` -- N(mu_C, 0.05^2 I)
* ``point``   -- every outlier sits at mu_C
* ``scatter`` -- N(0, s^2 I) (wide scattered noise)
* ``offset``  -- N(c e_1, 0.01 I)

where mu_C = gamma * v and v is the eigenvector of Sigma with the smallest
eigenvalue, rescaled so that v^T Sigma^{-1} v = p (Section 5, shift
contamination).

Covariance families: AR(rho) with Sigma_jk = rho^|j-k| (the A09 family of
Section 5 is rho = -0.9), and a random correlation matrix with a prescribed
spectrum (Bendel-Mickey rotations via ``scipy.stats.random_correlation``).
The ALYZ generator of Section 5 lives in a cited paper and is not reproduced.

Every array is a pure function of its seed.  Seeds are ``BASE_SEED + k`` for
workload k.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 1910056150


def ar_cov(p: int, rho: float) -> np.ndarray:
    j = np.arange(p)
    return rho ** np.abs(j[:, None] - j[None, :]).astype(np.float64)


def random_corr(p: int, rng: np.random.Generator,
                lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """Correlation matrix whose eigenvalues are U[lo, hi] draws rescaled to sum p."""
    from scipy.stats import random_correlation
    eig = rng.uniform(lo, hi, size=p)
    eig = eig * (p / eig.sum())
    c = random_correlation.rvs(eig, random_state=rng)
    c = 0.5 * (c + c.T)
    np.fill_diagonal(c, 1.0)
    return c


def shift_direction(cov: np.ndarray) -> np.ndarray:
    """Smallest-eigenvalue eigenvector v of cov scaled so that v' cov^-1 v = p."""
    p = cov.shape[0]
    w, v = np.linalg.eigh(cov)
    u = v[:, 0]
    if u[np.argmax(np.abs(u))] < 0:
        u = -u
    return u * math.sqrt(p * w[0])


@dataclasses.dataclass
class Dataset:
    X: np.ndarray            # n x p, row-major, float32 or float64
    cov: np.ndarray          # true inlier covariance
    outlier_rows: np.ndarray  # sorted indices of replaced rows
    name: str
    seed: int


def _draw_rows(rng, n, p, chol, out, row0=0, slab=1 << 20):
    """Fill out[row0:row0+n] with N(0, chol chol') rows, drawn in float64 slabs."""
    done = 0
    while done < n:
        k = min(slab, n - done)
        g = rng.standard_normal((k, p))
        out[row0 + done: row0 + done + k] = g @ chol.T
        done += k


def make_dataset(n: int, p: int, cov: np.ndarray, eps: float, kind: str,
                 seed: int, dtype=np.float32, gamma: float = 8.0,
                 scale: float = 5.0, offset: float = 10.0,
                 name: str = "") -> Dataset:
    rng = np.random.Generator(np.random.PCG64(seed))
    chol = np.linalg.cholesky(cov)
    X = np.empty((n, p), dtype=dtype)
    _draw_rows(rng, n, p, chol, X)
    k = int(math.floor(eps * n))
    rows = np.sort(rng.choice(n, size=k, replace=False)) if k > 0 else np.zeros(0, np.int64)
    if k > 0:
        if kind in ("shift", "cluster", "point"):
            mu_c = gamma * shift_direction(cov)
        if kind == "shift":
            O = np.empty((k, p), dtype=np.float64)
            _draw_rows(rng, k, p, chol, O)
            O += mu_c
        elif kind == "cluster":
            O = mu_c + 0.05 * rng.standard_normal((k, p))
        elif kind == "point":
            O = np.broadcast_to(mu_c, (k, p)).copy()
        elif kind == "scatter":
            O = scale * rng.standard_normal((k, p))
        elif kind == "offset":
            O = 0.1 * rng.standard_normal((k, p))
            O[:, 0] += offset
        else:
            raise ValueError(f"unknown contamination kind {kind!r}")
        X[rows] = O.astype(dtype)
    return Dataset(X=X, cov=cov, outlier_rows=rows, name=name, seed=seed)


# ---------------------------------------------------------------------------
# The five workloads.  ``n`` may be shrunk for small-size siblings; every other
# structural property (p, covariance family, contamination type and fraction,
# chunk length where it is fixed) is kept.
# ---------------------------------------------------------------------------

def workload_single_chunk_f64(n: int = 10_000, p: int = 10) -> Dataset:
    """Plain DetMCD on one chunk: AR(0.75), 20% outliers N(10 e1, 0.01 I), float64."""
    return make_dataset(n, p, ar_cov(p, 0.75), 0.20, "offset", BASE_SEED + 0,
                        dtype=np.float64, offset=10.0, name="single_chunk_f64")


def workload_chunked_p20(n: int = 1_000_000, p: int = 20) -> Dataset:
    """One dataset in 64 chunks: AR(0.75), 10% cluster N(8 v, 0.05^2 I), float32."""
    return make_dataset(n, p, ar_cov(p, 0.75), 0.10, "cluster", BASE_SEED + 1,
                        dtype=np.float32, gamma=8.0, name="chunked_p20")


def workload_batched_uneven(n_datasets: int = 512, n_lo: float = 2e3,
                            n_hi: float = 2e5, ps=(5, 10, 20, 40)) -> List[Dataset]:
    """Many independent datasets: n log-uniform, p from ps, eps in {0, .1, .2}, point at 6 v."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 2))
    out = []
    for i in range(n_datasets):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        p = int(rng.choice(ps))
        eps = float(rng.choice([0.0, 0.1, 0.2]))
        seed = int(rng.integers(0, 2**31 - 1))
        out.append(make_dataset(n, p, ar_cov(p, 0.75), eps, "point", seed,
                                dtype=np.float32, gamma=6.0, name=f"batched_{i}"))
    return out


def workload_large_p40(n: int = 10_000_000, p: int = 40) -> Dataset:
    """Large stream-like data: random correlation (eigenvalues U[0.1,10]), 5% N(0, 25 I)."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 3))
    cov = random_corr(p, rng)
    seed = int(rng.integers(0, 2**31 - 1))
    return make_dataset(n, p, cov, 0.05, "scatter", seed, dtype=np.float32,
                        scale=5.0, name="large_p40")


def workload_adjoint_p40(n: int = 200_000, p: int = 40) -> Dataset:
    """Adjoint workload: AR(0.5), 10% shift outliers N(8 v, Sigma), float32."""
    return make_dataset(n, p, ar_cov(p, 0.5), 0.10, "shift", BASE_SEED + 4,
                        dtype=np.float32, gamma=8.0, name="adjoint_p40")


def small_gaussian(n: int, p: int, seed: int, dtype=np.float64,
                   rho: float = 0.5, eps: float = 0.0, kind: str = "shift",
                   gamma: float = 8.0) -> Dataset:
    """Generic small case for unit tests."""
    return make_dataset(n, p, ar_cov(p, rho), eps, kind, BASE_SEED + 100 + seed,
                        dtype=dtype, gamma=gamma, name=f"small_{n}x{p}_{seed}")
