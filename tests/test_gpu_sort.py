"""The two rankings of the global segmented radix sort give the same fit.

Columns and blocks longer than one LDS segment go through the global sort,
whose scatter ranks equal digits with LDS atomics and then checks the order
of the result; a handle created with RTDETMCD_SAFE_SORT=1 ranks with ballots
instead.  The sorted keys, and so every output, must be identical."""
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


@pytest.mark.parametrize("dtype,n,p,q,kind", [(np.float32, 200_000, 20, 4, "shift"),
                                              (np.float64, 90_000, 8, 2, "shift"),
                                              (np.float64, 90_000, 8, 2, "point"),
                                              (np.float32, 120_000, 5, 1, "point")])
def test_atomic_and_ballot_ranking_agree(monkeypatch, dtype, n, p, q, kind):
    # the default handle sorts 64-bit keys on their high halves and fixes the
    # runs of equal high halves in place; identical points make long runs of
    # equal keys (no fix-up needed), continuous values short runs
    import paper_1910_05615_amd as P
    ds = synthdata.small_gaussian(n, p, seed=31, dtype=dtype, rho=0.5, eps=0.1, kind=kind,
                                  gamma=8)
    X = torch.from_numpy(ds.X).to("cuda:0")
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
    if n * p <= 2_000_000:
        check_fit(Fa, oracle.fit(ds.X, n_chunks=q), f"{dtype.__name__} n={n}")
