"""GPU parity of the adjoint (rtdetmcd_backward, RobustMCD): the reweighting
set against the oracle's, the gradient against the oracle's closed form, and
central finite differences through complete GPU refits away from ties."""
import math

import numpy as np
import pytest

import oracle
import synthdata
from test_gpu_fit import check_fit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _P():
    import paper_1910_05615_amd as P
    return P


def _dev():
    return torch.device("cuda:0")


def _cot(n, p, seed, which="all"):
    rng = np.random.default_rng(seed)
    gd = rng.standard_normal(n) if which in ("d", "all") else None
    gm = rng.standard_normal(p) if which in ("mu", "all") else None
    gs = rng.standard_normal((p, p)) if which in ("sigma", "all") else None
    return gd, gm, gs


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(_dev())


def _check_against_closed_form(X, F, gd, gm, gs, tol=1e-9):
    P = _P()
    W = F.rew_mask.cpu().numpy().astype(bool)
    G = P.backward(_t(X), F, _t(gd), _t(gm), _t(gs)).cpu().numpy()
    ref = oracle.adjoint.adjoint(X.astype(np.float64), W, F.c_rew, gd, gm, gs)
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert np.max(np.abs(G - ref)) <= tol * scale


@pytest.mark.parametrize("dtype,n,p,q", [(np.float64, 6000, 5, 2), (np.float32, 40_000, 20, 4)])
def test_reweighting_set_matches_oracle(dtype, n, p, q):
    ds = synthdata.small_gaussian(n, p, seed=21, dtype=dtype, rho=0.5, eps=0.1, kind="shift",
                                  gamma=8)
    ref = oracle.fit(ds.X, n_chunks=q)
    F = _P().fit(_t(ds.X), n_chunks=q)
    assert np.array_equal(F.rew_mask.cpu().numpy(), ref.rew_mask)
    assert int(F.n_w.cpu()[0]) == int(ref.rew_mask.sum()) == ref.n_w


@pytest.mark.parametrize("which", ["d", "mu", "sigma", "all"])
def test_backward_matches_closed_form_f64(which):
    ds = synthdata.small_gaussian(5000, 5, seed=22, dtype=np.float64, rho=0.5, eps=0.1,
                                  kind="shift", gamma=8)
    F = _P().fit(_t(ds.X), n_chunks=2)
    gd, gm, gs = _cot(5000, 5, 3, which)
    _check_against_closed_form(ds.X, F, gd, gm, gs)


def test_backward_matches_closed_form_f32_p20_rew_consistency():
    ds = synthdata.workload_chunked_p20(n=60_000)
    F = _P().fit(_t(ds.X), n_chunks=4, rew_consistency=True)
    assert F.c_rew > 1.0
    gd, gm, gs = _cot(60_000, 20, 4)
    _check_against_closed_form(ds.X, F, gd, gm, gs)


def test_autograd_function_matches_backward():
    P = _P()
    ds = synthdata.small_gaussian(4000, 6, seed=23, dtype=np.float64, rho=0.5, eps=0.1,
                                  kind="point", gamma=6)
    X = _t(ds.X).requires_grad_(True)
    mu, sigma, dist = P.RobustMCD.apply(X, {"n_chunks": 2})
    rng = np.random.default_rng(8)
    a, B, c = _t(rng.standard_normal(6)), _t(rng.standard_normal((6, 6))), _t(rng.standard_normal(4000))
    loss = (a * mu).sum() + (B * sigma).sum() + (c * dist).sum()
    loss.backward()
    F = P.fit(_t(ds.X), n_chunks=2)
    G = P.backward(_t(ds.X), F, c, a, B)
    assert torch.equal(X.grad, G)


def _fd_rows(X, n_chunks, rows, seed, eps_rel=1e-6, tol=1e-6):
    """Central differences of <gd, d> + <gm, mu> + <gs, Sigma> through full GPU
    refits along one random unit direction per row.

    The difference quotient is formed from the elementwise differences of the
    two refits' outputs (d+ - d-, mu+ - mu-, Sigma+ - Sigma-), so the large
    sum itself is never differenced.  Bound: |fd - an| <= tol |an| + floor,
    where the floor is the rounding noise of that quotient: every output
    carries an error of a few sqrt(p) ulps that is uncorrelated between the
    two refits, so the weighted sum of differences has a noise of about
    sqrt(p) u ||gd o d||_2 (plus the mu and Sigma terms), divided by 2 eps;
    the floor is 16 times that.  Returns the worst relative error
    |fd - an| / |an| over the rows whose tol |an| exceeds the floor."""
    P = _P()
    n, p = X.shape
    F = P.fit(_t(X), n_chunks=n_chunks)
    gd, gm, gs = _cot(n, p, seed)
    G = P.backward(_t(X), F, _t(gd), _t(gm), _t(gs)).cpu().numpy()
    W0 = F.rew_mask.cpu().numpy()
    scale = F.scale.cpu().numpy()
    d0, mu0, s0 = F.dist.cpu().numpy(), F.mu.cpu().numpy(), F.sigma.cpu().numpy()
    noise = (np.linalg.norm(gd * d0) + np.linalg.norm(gm * mu0) + np.linalg.norm(gs * s0))
    rng = np.random.default_rng(seed + 1)
    eps = eps_rel * float(np.median(scale))
    floor = 16.0 * math.sqrt(p) * 2.0 ** -53 * noise / (2 * eps)
    worst_rel = 0.0
    for r in rows:
        u = rng.standard_normal(p)
        u /= np.linalg.norm(u)
        outs = []
        for sgn in (1.0, -1.0):
            Xe = X.copy()
            Xe[r] += sgn * eps * u
            Fe = P.fit(_t(Xe), n_chunks=n_chunks)
            assert np.array_equal(Fe.rew_mask.cpu().numpy(), W0), f"W changed at row {r}"
            outs.append((Fe.dist.cpu().numpy(), Fe.mu.cpu().numpy(), Fe.sigma.cpu().numpy()))
        (dp, mp, sp), (dm, mm, sm) = outs
        fd = float(gd @ (dp - dm) + gm @ (mp - mm) + np.sum(gs * (sp - sm))) / (2 * eps)
        an = float(G[r] @ u)
        assert abs(fd - an) <= tol * abs(an) + floor, (r, fd, an, floor)
        if abs(an) * tol > floor:
            worst_rel = max(worst_rel, abs(fd - an) / abs(an))
    print(f"finite differences: worst relative error {worst_rel:.2e} over {len(rows)} rows "
          f"(absolute floor {floor:.1e})")
    return worst_rel


def _rows_away_from_ties(X, n_chunks, k, seed):
    """k rows whose reweighting distance is not within 5% of the cutoff."""
    ref = oracle.fit(X, n_chunks=n_chunks)
    d2 = np.full(X.shape[0], np.inf)
    d2[: len(ref.diag["d2_reweight"])] = ref.diag["d2_reweight"]
    chi2 = ref.diag["chi2"]
    ok = np.nonzero(np.abs(d2 - chi2) > 0.05 * chi2)[0]
    return np.random.default_rng(seed).choice(ok, k, replace=False)


def test_finite_differences_through_gpu_refits_small():
    ds = synthdata.small_gaussian(8000, 5, seed=24, dtype=np.float64, rho=0.5, eps=0.1,
                                  kind="shift", gamma=8)
    rows = _rows_away_from_ties(ds.X, 2, 16, 5)
    _fd_rows(ds.X, 2, rows, 6, eps_rel=1e-5)


def test_adjoint_workload_p40_full_size():
    # 200,000 x 40, one block: float32 forward checked against the closed form,
    # and the float64 check path by central differences on 64 rows
    P = _P()
    ds = synthdata.workload_adjoint_p40()
    F = P.fit(_t(ds.X))
    # the forward fit itself against the oracle's: h-subset, reweighting set,
    # flags, block status and the estimates
    ref = oracle.fit(ds.X)
    check_fit(F, ref, "adjoint workload 200,000 x 40")
    assert np.array_equal(F.rew_mask.cpu().numpy(), ref.rew_mask)
    gd, gm, gs = _cot(ds.X.shape[0], 40, 7)
    _check_against_closed_form(ds.X, F, gd, gm, gs, tol=1e-8)
    X64 = ds.X.astype(np.float64)
    F64 = P.fit(_t(X64))
    # rows whose final squared distance is not within 5% of the cutoff (the
    # reweighting distance differs little; _fd_rows asserts W never changes)
    d = F64.dist.cpu().numpy()
    chi2 = P.chi2_quantile(0.975, 40)
    ok = np.nonzero(np.abs(d * d - chi2) > 0.05 * chi2)[0]
    rows = np.random.default_rng(9).choice(ok, 64, replace=False)
    _fd_rows(X64, 0, rows, 10, eps_rel=1e-4)
