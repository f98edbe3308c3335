"""The fast sorts of long segments give the same fit as the safe sort.

Columns and blocks longer than one LDS segment are sorted by the bucket
sample sort (blocks of the refinement and GSSCM steps) or by global radix
passes with LDS-atomic ranking and a fix-up (standardisation columns); a
handle created with RTDETMCD_SAFE_SORT=1 runs full-width radix passes with
ballot ranking instead.  The sorted keys, and so every output, must be
identical."""
import numpy as np
import pytest

import oracle
import synthdata
from test_gpu_fit import _ALL, check_fit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fit_with_fresh_handle(P, X, **kw):
    """Fit on a handle created under the current environment."""
    from paper_1910_05615_amd import _lib, api
    idx = X.device.index if X.device.index is not None else torch.cuda.current_device()
    saved = api._handles.pop(idx, None)
    try:
        F = P.fit(X, **kw)
        torch.cuda.synchronize()
        api._last_fresh_reruns = P.sort_reruns()
    finally:
        h = api._handles.pop(idx, None)
        if h is not None:
            _lib.load().rtdetmcd_destroy(h)
        if saved is not None:
            api._handles[idx] = saved
    return F


def _data(dtype, n, p, kind):
    """The generator's data; "heavy": 5% of rows scaled by 10^U(0, 6)
    (values over six decades: the extreme buckets crowd into few normalised
    keys); "rounded": the shifted data rounded to integers (many
    repeated values, each a class of its own when sampled)."""
    base = "shift" if kind in ("heavy", "rounded") else kind
    ds = synthdata.small_gaussian(n, p, seed=31, dtype=dtype, rho=0.5, eps=0.1, kind=base,
                                  gamma=8)
    X = ds.X
    if kind == "heavy":
        rng = np.random.default_rng(77)
        rows = rng.choice(n, n // 20, replace=False)
        X = X.copy()
        X[rows] *= (10.0 ** rng.uniform(0, 6, size=(len(rows), 1))).astype(dtype)
    elif kind == "rounded":
        X = np.round(X).astype(dtype)
    return X


@pytest.mark.parametrize("dtype,n,p,q,kind", [(np.float32, 200_000, 20, 4, "shift"),
                                              (np.float64, 90_000, 8, 2, "shift"),
                                              (np.float64, 90_000, 8, 2, "point"),
                                              (np.float32, 120_000, 5, 1, "point"),
                                              (np.float64, 150_000, 6, 1, "heavy"),
                                              (np.float32, 100_000, 10, 2, "rounded")])
def test_atomic_and_ballot_ranking_agree(monkeypatch, dtype, n, p, q, kind):
    # the default handle sorts long blocks of 64-bit keys by buckets (a
    # sample sort: each bucket in LDS) and long columns by radix passes on the
    # high halves with a fix-up of runs of equal high halves; the safe handle
    # runs full-width radix passes with ballot ranking only
    import paper_1910_05615_amd as P
    Xh = _data(dtype, n, p, kind)
    X = torch.from_numpy(Xh).to("cuda:0")
    # blocks of n / q rows: both the standardisation columns and the
    # refinement score columns are longer than one LDS segment
    monkeypatch.delenv("RTDETMCD_SAFE_SORT", raising=False)
    Fa = _fit_with_fresh_handle(P, X, n_chunks=q)
    # the fix-up sufficed: no fit was run again with the full-width sort
    from paper_1910_05615_amd import api
    assert api._last_fresh_reruns == 0
    monkeypatch.setenv("RTDETMCD_SAFE_SORT", "1")
    Fb = _fit_with_fresh_handle(P, X, n_chunks=q)
    for name in _ALL:
        a, b = getattr(Fa, name), getattr(Fb, name)
        assert torch.equal(a, b), name
    # not against the oracle: "rounded" has exact ties of distances; "heavy"
    # makes the univariate MCD's window sums (prefix differences that cancel
    # against the tails' squares, values up to 10^6) ill-conditioned, and the
    # two summation orders pick windows a few places apart
    if n * p <= 2_000_000 and kind not in ("heavy", "rounded"):
        check_fit(Fa, oracle.fit(Xh, n_chunks=q), f"{dtype.__name__} n={n}")


@pytest.mark.parametrize("n,p", [(16_384, 3),    # one LDS segment exactly
                                 (16_385, 3),    # the smallest sample sort: two buckets
                                 (655_360, 2),   # the largest sample sort: 64 buckets
                                 (655_361, 2)])  # beyond it: the global radix passes
def test_sort_paths_at_their_limits(monkeypatch, n, p):
    # single blocks of n rows, so the standardisation columns and the
    # refinement columns are all n keys long
    import paper_1910_05615_amd as P
    ds = synthdata.small_gaussian(n, p, seed=61, dtype=np.float32, rho=0.5, eps=0.1)
    X = torch.from_numpy(ds.X).to("cuda:0")
    monkeypatch.delenv("RTDETMCD_SAFE_SORT", raising=False)
    Fa = _fit_with_fresh_handle(P, X, n_chunks=1)
    from paper_1910_05615_amd import api
    assert api._last_fresh_reruns == 0
    monkeypatch.setenv("RTDETMCD_SAFE_SORT", "1")
    Fb = _fit_with_fresh_handle(P, X, n_chunks=1)
    for name in _ALL:
        assert torch.equal(getattr(Fa, name), getattr(Fb, name)), name
    check_fit(Fa, oracle.fit(ds.X, n_chunks=1), f"n={n}")
