"""The fit's diagnostics (log det trace of each block's chosen start, the gap
at the h-subset threshold, the margin of the outlier flags) against the
oracle's, and the fit itself unchanged when they are asked for."""
import numpy as np
import pytest

import oracle
import synthdata
from test_gpu_fit import _ALL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _check_diag(F, ref, label):
    g = lambda t: t.cpu().numpy()
    maxs = F.ldtrace.shape[1]
    tr, rtr = g(F.ldtrace), ref.diag["block_logdets"][:, :maxs]
    for l in range(F.q):
        it = int(ref.chunk_iters[l])
        # log det: the method's 1e-6 bar
        np.testing.assert_allclose(tr[l, :it], rtr[l, :it], rtol=0, atol=1e-6, err_msg=label)
        assert np.all(np.isnan(tr[l, it:])), label
    # the gaps are differences of float64 distances of order chi2_p: both
    # sides round the distances differently in the last bits
    np.testing.assert_allclose(g(F.hmargin), ref.diag["block_hgap"], rtol=1e-6, atol=1e-9,
                               err_msg=label)
    np.testing.assert_allclose(g(F.cmargin)[0], ref.diag["cmargin"], rtol=1e-6, atol=1e-9,
                               err_msg=label)


@pytest.mark.parametrize("dtype,n,p,q,mode", [(np.float64, 10_000, 10, 1, "auto"),
                                              (np.float32, 60_000, 8, 4, "auto"),
                                              (np.float64, 20_000, 5, 2, "smw")])
def test_diagnostics_match_oracle(dtype, n, p, q, mode):
    import paper_1910_05615_amd as P
    ds = synthdata.small_gaussian(n, p, seed=41, dtype=dtype, rho=0.5, eps=0.1, gamma=8)
    X = torch.from_numpy(ds.X).to("cuda:0")
    kw = dict(n_chunks=q, cstep_mode=mode)
    F = P.fit(X, diagnostics=True, **kw)
    F0 = P.fit(X, **kw)
    for name in _ALL:   # asking for the diagnostics changes nothing else
        assert torch.equal(getattr(F, name), getattr(F0, name)), name
    ref = oracle.fit(ds.X, n_chunks=q, cstep_mode="smw" if mode == "smw" else "full")
    _check_diag(F, ref, f"{dtype.__name__} n={n} q={q} {mode}")


def test_batched_diagnostics_match_oracle():
    import paper_1910_05615_amd as P
    sets = [synthdata.small_gaussian(n, p, seed=50 + k, dtype=np.float32, eps=0.1)
            for k, (n, p) in enumerate([(9_000, 5), (30_000, 10), (4_000, 3)])]
    Xs = [torch.from_numpy(s.X).to("cuda:0") for s in sets]
    fits, status = P.fit_batched(Xs, diagnostics=True)
    assert status == [0, 0, 0]
    for s, F in zip(sets, fits):
        _check_diag(F, oracle.fit(s.X), f"batched n={s.X.shape[0]}")


def test_plain_launch_diagnostics_equal_batched():
    # the per-block launches keep the same trace, gaps and margin
    import paper_1910_05615_amd as P
    ds = synthdata.small_gaussian(24_000, 6, seed=43, dtype=np.float32, eps=0.1)
    X = torch.from_numpy(ds.X).to("cuda:0")
    Fb = P.fit(X, n_chunks=3, diagnostics=True)
    Fp = P.fit(X, n_chunks=3, diagnostics=True, launch="plain")
    assert torch.equal(Fb.ldtrace.isnan(), Fp.ldtrace.isnan())
    assert torch.equal(torch.nan_to_num(Fb.ldtrace), torch.nan_to_num(Fp.ldtrace))
    assert torch.equal(Fb.hmargin, Fp.hmargin)
    assert torch.equal(Fb.cmargin, Fp.cmargin)
