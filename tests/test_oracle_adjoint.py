"""Pins of the oracle's adjoint (Sec. 4 steps 9-10 with the reweighting set
fixed): the hand-derived closed form against central finite differences of
the forward formulas, the forward formulas against the full oracle fit, and
finite differences through complete refits away from ties."""
import numpy as np
import pytest

import oracle
import synthdata

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _functional(X, W, c, gd, gmu, gsig):
    mu, S, d = oracle.adjoint.fixed_set_forward(X, W, c)
    return float(gd @ d + gmu @ mu + np.sum(gsig * S))


def _fd_grad(X, W, c, gd, gmu, gsig, eps):
    G = np.zeros_like(X)
    for i in range(X.shape[0]):
        for j in range(X.shape[1]):
            Xp = X.copy(); Xp[i, j] += eps
            Xm = X.copy(); Xm[i, j] -= eps
            G[i, j] = (_functional(Xp, W, c, gd, gmu, gsig) -
                       _functional(Xm, W, c, gd, gmu, gsig)) / (2 * eps)
    return G


@pytest.mark.parametrize("which", ["d", "mu", "sigma", "all"])
@pytest.mark.parametrize("c", [1.0, 1.17])
def test_closed_form_matches_central_differences(which, c):
    rng = np.random.default_rng(11)
    n, p = 60, 4
    A = rng.standard_normal((p, p))
    X = rng.standard_normal((n, p)) @ A.T + rng.standard_normal(p)
    W = rng.random(n) < 0.8
    gd = rng.standard_normal(n) if which in ("d", "all") else np.zeros(n)
    gmu = rng.standard_normal(p) if which in ("mu", "all") else np.zeros(p)
    gsig = rng.standard_normal((p, p)) if which in ("sigma", "all") else np.zeros((p, p))
    G = oracle.adjoint.adjoint(X, W, c, gd, gmu, gsig)
    Gfd = _fd_grad(X, W, c, gd, gmu, gsig, 1e-6)
    assert np.max(np.abs(G - Gfd)) <= 1e-6 * max(1.0, np.max(np.abs(Gfd)))


def test_asymmetric_sigma_cotangent_uses_symmetric_part():
    # Sigma is symmetric, so only the symmetric part of its cotangent matters
    rng = np.random.default_rng(5)
    X = rng.standard_normal((40, 3))
    W = np.ones(40, bool)
    Gs = rng.standard_normal((3, 3))
    a = oracle.adjoint.adjoint(X, W, 1.0, None, None, Gs)
    b = oracle.adjoint.adjoint(X, W, 1.0, None, None, 0.5 * (Gs + Gs.T))
    assert np.allclose(a, b, rtol=1e-13, atol=1e-13)


def test_rows_outside_w_only_get_the_direct_term():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((50, 3))
    W = np.arange(50) < 40
    gd = np.zeros(50); gd[45] = 1.0          # cotangent on an outside row only
    G = oracle.adjoint.adjoint(X, W, 1.0, gd, None, None)
    mu, S, d = oracle.adjoint.fixed_set_forward(X, W)
    direct = np.linalg.solve(S, X[45] - mu) / d[45]
    assert np.allclose(G[45], direct, rtol=1e-12)
    others = np.delete(np.arange(50), 45)
    assert np.all(G[40:][np.arange(10) != 5] == 0.0)
    assert np.any(G[others] != 0.0)           # mu and Sigma move with the W rows


def test_forward_formulas_reproduce_the_fit():
    ds = synthdata.small_gaussian(3000, 5, seed=3, dtype=np.float64, rho=0.5, eps=0.1,
                                  kind="shift", gamma=8)
    F = oracle.fit(ds.X, n_chunks=2)
    W = F.rew_mask.astype(bool)
    assert int(W.sum()) == F.n_w
    mu, S, d = oracle.adjoint.fixed_set_forward(ds.X, W)
    assert np.allclose(mu, F.mu, rtol=1e-12, atol=1e-13)
    assert np.linalg.norm(S - F.sigma) <= 1e-12 * np.linalg.norm(F.sigma)
    assert np.allclose(d, F.dist, rtol=1e-10)


def test_finite_differences_through_refits():
    # Perturb single rows away from the cutoff and the h-th order statistic:
    # the refit keeps every h-subset and W, and its (mu, Sigma, d) moves as the
    # adjoint says.
    ds = synthdata.small_gaussian(2000, 5, seed=9, dtype=np.float64, rho=0.5, eps=0.1,
                                  kind="shift", gamma=8)
    X = ds.X
    F = oracle.fit(X)
    W = F.rew_mask.astype(bool)
    rng = np.random.default_rng(2)
    gd = rng.standard_normal(X.shape[0])
    gmu = rng.standard_normal(5)
    gsig = rng.standard_normal((5, 5))
    G = oracle.adjoint.adjoint(X, W, 1.0, gd, gmu, gsig)
    chi2 = F.diag["chi2"]
    d2r = np.zeros(X.shape[0]); d2r[: len(F.diag["d2_reweight"])] = F.diag["d2_reweight"]
    safe = np.nonzero(np.abs(d2r - chi2) > 0.05 * chi2)[0]
    rows = rng.choice(safe, 6, replace=False)

    def Fval(Xe):
        Fe = oracle.fit(Xe)
        return Fe, float(gd @ Fe.dist + gmu @ Fe.mu + np.sum(gsig * Fe.sigma))

    eps = 1e-5
    for r in rows:
        u = rng.standard_normal(5); u /= np.linalg.norm(u)
        Xp = X.copy(); Xp[r] += eps * u
        Xm = X.copy(); Xm[r] -= eps * u
        Fp, vp = Fval(Xp)
        Fm, vm = Fval(Xm)
        for Fe in (Fp, Fm):
            assert np.array_equal(Fe.hsubset, F.hsubset)
            assert np.array_equal(Fe.rew_mask, F.rew_mask)
        fd = (vp - vm) / (2 * eps)
        an = float(G[r] @ u)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (r, fd, an)
