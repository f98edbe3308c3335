"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these re-derives a value with the oracle's own formula: each compares
against a closed form, a printed table, a brute-force search, an invariance, or
a textbook routine computed a different way.
"""
import itertools
import math
import os
import statistics

import numpy as np
import pytest

import oracle
import synthdata

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- constants

@pytest.mark.parametrize("q", [0.5, 0.75, 0.9, 0.975, 0.99])
def test_chi2_quantile_p2_closed_form(q):
    # chi2_2 is exponential with mean 2: quantile -2 ln(1-q).
    assert oracle.chi2_quantile(q, 2) == pytest.approx(-2.0 * math.log(1.0 - q), rel=1e-12)


@pytest.mark.parametrize("alpha", [0.5, 0.55, 0.75, 0.9])
def test_consistency_factor_p2_closed_form(alpha):
    # F_{chi2_4}(x) = 1 - e^{-x/2}(1 + x/2), x = -2 ln(1-alpha).
    ref = alpha / (1.0 - (1.0 - alpha) * (1.0 - math.log(1.0 - alpha)))
    assert oracle.consistency_factor(alpha, 2) == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("alpha", [0.5, 0.5001, 0.75, 0.975])
def test_consistency_factor_p1_closed_form(alpha):
    # x = chi2_{1,alpha} = (Phi^-1((1+alpha)/2))^2 ; F_{chi2_3}(x) = erf(sqrt(x/2)) - sqrt(2x/pi) e^{-x/2}
    z = statistics.NormalDist().inv_cdf((1.0 + alpha) / 2.0)
    x = z * z
    F3 = math.erf(math.sqrt(x / 2.0)) - math.sqrt(2.0 * x / math.pi) * math.exp(-x / 2.0)
    assert oracle.consistency_factor(alpha, 1) == pytest.approx(alpha / F3, rel=1e-9)


def test_block_count_rule_table4_panelC():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table4_panelC_blocks.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 10
    cells = 0
    for r in rows:
        n = int(r[0])
        vals = list(map(int, r[1:]))
        for wi, omega in enumerate((2**12, 2**13, 2**14)):
            for pi, p in enumerate((4, 8, 16)):
                assert oracle.n_blocks(n, p, omega) == vals[3 * wi + pi], (n, p, omega)
                cells += 1
    assert cells == 90


def test_subset_size_rule():
    assert oracle.subset_size(10_000, 10, 0.75) == 7500
    assert oracle.subset_size(15_625, 20, 0.75) == 11_718
    assert oracle.subset_size(9_765, 40, 0.75) == 7_323
    # clamped to (m+p+1)/2 from below and m-1 from above
    assert oracle.subset_size(100, 10, 0.3) == 55
    assert oracle.subset_size(100, 10, 1.0) == 99


# ---------------------------------------------------------------- univariate MCD

def _brute_unimcd(x):
    v = np.sort(x)
    n = len(v)
    hh = n // 2 + 1
    best, js = None, None
    for j in range(n - hh + 1):
        w = v[j:j + hh]
        var = float(np.var(w, ddof=1))       # two-pass, independent of prefix sums
        if best is None or var < best - 1e-12 * max(best, 1e-300):
            best, js = var, j
    return js, float(np.mean(v[js:js + hh])), best


@pytest.mark.parametrize("seed", range(6))
def test_unimcd_matches_brute_force_window(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(7, 180))
    x = rng.standard_normal(n)
    x[: n // 5] += rng.uniform(3, 10)          # a contaminated tail
    js, mean, var = _brute_unimcd(x)
    u = oracle.unimcd(x)
    assert u.start == js
    assert u.mu_raw == pytest.approx(mean, rel=1e-12, abs=1e-12)
    hh = n // 2 + 1
    c = oracle.consistency_factor(hh / n, 1)
    assert u.var_raw == pytest.approx(var * c, rel=1e-10)
    # reweighting by brute force
    keep = [xi for xi in x if (xi - u.mu_raw) ** 2 <= oracle.chi2_quantile(0.975, 1) * u.var_raw]
    assert u.n_kept == len(keep)
    assert u.mu == pytest.approx(statistics.fmean(keep), rel=1e-12, abs=1e-12)
    assert u.var == pytest.approx(statistics.variance(keep) * oracle.consistency_factor(0.975, 1),
                                  rel=1e-10)


def test_unimcd_location_scale_equivariance():
    rng = np.random.default_rng(7)
    x = rng.standard_normal(501)
    u = oracle.unimcd(x)
    v = oracle.unimcd(3.0 * x - 2.0)
    assert v.start == u.start
    assert v.mu == pytest.approx(3.0 * u.mu - 2.0, rel=1e-12)
    assert v.var == pytest.approx(9.0 * u.var, rel=1e-12)


def test_unimcd_gaussian_consistency():
    # With the consistency factors, raw and reweighted variances estimate 1 on N(0,1).
    rng = np.random.default_rng(11)
    x = rng.standard_normal(1_000_000)
    u = oracle.unimcd(x)
    assert abs(u.mu) < 0.01
    assert u.var_raw == pytest.approx(1.0, abs=0.02)
    assert u.var == pytest.approx(1.0, abs=0.01)


def test_unimcd_resists_contamination():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(20_000)
    x[:8_000] = 50.0 + rng.standard_normal(8_000)   # 40% far away
    u = oracle.unimcd(x)
    # the far group never enters the reweighted set; the location is unaffected
    assert u.n_kept <= 12_000 and abs(u.mu) < 0.05 and 0.8 < u.var < 1.5


# ---------------------------------------------------------------- wrapping

def test_wrapping_golden_points():
    for line in open(os.path.join(GOLDEN, "wrapping_points.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        z, g, tol = map(float, line.split())
        assert float(oracle.wrap(np.array([z]))[0]) == pytest.approx(g, abs=max(tol, 1e-15))


def test_wrapping_odd_and_bounded():
    z = np.linspace(-6, 6, 2001)
    g = oracle.wrap(z)
    assert np.allclose(g, -oracle.wrap(-z), atol=0)
    assert np.all(np.abs(g) <= 1.5 + 2e-4)
    # continuity at b: 1.541 tanh(0.862 * 2.5) = 1.500147 (printed constants are rounded)
    assert 1.541 * math.tanh(0.862 * 2.5) == pytest.approx(1.500147, abs=1e-6)


def test_wrapping_keeps_about_85_percent():
    # P(|N(0,1)| <= 1.5) = 0.8664 (Sec. 3.2: "about 85% of the values are left unchanged")
    rng = np.random.default_rng(5)
    z = rng.standard_normal(400_000)
    frac = float(np.mean(oracle.wrap(z) == z))
    assert frac == pytest.approx(math.erf(1.5 / math.sqrt(2)), abs=0.003)


# ---------------------------------------------------------------- GSSCM

def test_gsscm_reduces_to_second_moment_when_cutoffs_infinite():
    rng = np.random.default_rng(2)
    Z = rng.standard_normal((500, 4))
    S = oracle.init_gsscm(Z, A=1e300, B=2e300)
    ref = sum(np.outer(z, z) for z in Z) / 500.0
    assert np.allclose(S, ref, rtol=1e-12, atol=1e-14)


def test_gsscm_weight_function():
    r = np.array([0.0, 1.0, 2.0, 2.5, 3.0, 3.5])
    w = oracle.xi_lr(r, 2.0, 3.0)
    assert list(w) == [1.0, 1.0, 1.0, 0.5, 0.0, 0.0]


def test_gsscm_cutoffs_median():
    r = np.array([1.0, 2.0, 4.0, 8.0, 3.0])
    A, B = oracle.gsscm_cutoffs(r)
    assert A == 3.0
    s = sorted(x ** (2 / 3) for x in r)
    med = s[2]
    mad = sorted(abs(x - med) for x in s)[2]
    assert B == pytest.approx((med + mad) ** 1.5, rel=1e-14)
    assert B >= A


def test_wrap_cov_is_classical_cov_of_wrapped():
    rng = np.random.default_rng(4)
    Z = rng.standard_normal((300, 3)) * 2
    W = np.array([[float(oracle.wrap(np.array([v]))[0]) for v in row] for row in Z])
    mu = W.mean(axis=0)
    ref = sum(np.outer(w - mu, w - mu) for w in W) / 299.0
    assert np.allclose(oracle.init_wrap_cov(Z), ref, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- refinement

def test_refinement_consistent_on_clean_gaussian():
    ds = synthdata.small_gaussian(200_000, 4, seed=1, rho=0.6)
    X = ds.X
    loc = np.array([oracle.unimcd(X[:, j]).mu for j in range(4)])
    sc = np.sqrt([oracle.unimcd(X[:, j]).var for j in range(4)])
    Z = (X - loc) / sc
    R = ds.cov          # unit diagonal: the standardised covariance is R
    for S0 in (oracle.init_wrap_cov(Z), oracle.init_gsscm(Z)):
        st = oracle.refine(S0, Z)
        assert st.ok
        assert np.max(np.abs(st.sigma - R)) < 0.03
        assert np.max(np.abs(st.mu)) < 0.02


def test_refinement_signed_permutation_equivariance():
    rng = np.random.default_rng(8)
    Z = rng.standard_normal((3000, 4)) @ np.array(
        [[1, .3, 0, 0], [0, 1, .2, 0], [0, 0, 1, .5], [0, 0, 0, 1.]])
    P = np.eye(4)[[2, 0, 3, 1]] * np.array([1, -1, 1, -1])[:, None]
    a = oracle.refine(oracle.init_gsscm(Z), Z)
    b = oracle.refine(oracle.init_gsscm(Z @ P.T), Z @ P.T)
    assert np.allclose(b.sigma, P @ a.sigma @ P.T, rtol=1e-9, atol=1e-12)
    assert np.allclose(b.mu, P @ a.mu, rtol=1e-9, atol=1e-12)


def test_refinement_drops_ill_conditioned():
    Z = np.random.default_rng(1).standard_normal((200, 3))
    S = np.diag([1.0, 1.0, 1e-4])
    assert not oracle.refine(S, Z).ok


# ---------------------------------------------------------------- distances & C-steps

def test_mahalanobis_matches_textbook_inverse():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((50, 5))
    A = rng.standard_normal((5, 5))
    S = A @ A.T + 5 * np.eye(5)
    mu = rng.standard_normal(5)
    d2 = oracle.mahalanobis2(X, mu, np.linalg.cholesky(S))
    Si = np.linalg.inv(S)
    ref = np.array([(x - mu) @ Si @ (x - mu) for x in X])
    assert np.allclose(d2, ref, rtol=1e-11)
    L = np.linalg.cholesky(S)
    assert 2 * np.sum(np.log(np.diag(L))) == pytest.approx(np.linalg.slogdet(S)[1], rel=1e-12)


def test_select_ties_by_index():
    d2 = np.array([3.0, 1.0, 1.0, 2.0, 1.0, 0.5])
    assert list(oracle.select_h(d2, 2)) == [1, 5]
    assert list(oracle.select_h(d2, 3)) == [1, 2, 5]
    assert list(oracle.select_h(d2, 4)) == [1, 2, 4, 5]


def _contaminated(n, p, seed, eps=0.2):
    return synthdata.small_gaussian(n, p, seed=seed, rho=0.7, eps=eps, kind="shift", gamma=6).X


@pytest.mark.parametrize("seed", range(4))
def test_cstep_monotone_and_fixed_point(seed):
    X = _contaminated(800, 4, seed)
    h = 600
    rng = np.random.default_rng(seed)
    H0 = np.sort(rng.choice(800, h, replace=False))
    mu0, S0 = oracle.subset_stats(X, H0)
    r = oracle.csteps(X, h, mu0, S0)
    assert r.status == oracle.ST_CONVERGED
    # Proposition 1 of FastMCD: det non-increasing between subset covariances
    assert all(b <= a + 1e-12 for a, b in zip(r.logdets, r.logdets[1:]))
    # fixed point: one more C-step reproduces H
    d2 = oracle.mahalanobis2(X, r.mu, np.linalg.cholesky(r.sigma))
    assert np.array_equal(oracle.select_h(d2, h), r.H)
    mu, S = oracle.subset_stats(X, r.H)
    assert np.allclose(mu, r.mu) and np.allclose(S, r.sigma)


def test_cstep_affine_equivariance():
    X = _contaminated(600, 3, 5)
    h = 400
    H0 = np.arange(0, 600, 3)[:h] if 600 // 3 >= h else np.arange(h)
    mu0, S0 = oracle.subset_stats(X, H0)
    A = np.array([[2.0, 0.5, 0.0], [-1.0, 1.0, 0.3], [0.2, 0.0, 3.0]])
    b = np.array([10.0, -5.0, 1.0])
    r1 = oracle.csteps(X, h, mu0, S0)
    r2 = oracle.csteps(X @ A.T + b, h, A @ mu0 + b, A @ S0 @ A.T)
    assert np.array_equal(r1.H, r2.H)
    assert r2.logdet == pytest.approx(r1.logdet + 2 * np.log(abs(np.linalg.det(A))), abs=1e-9)


def test_update_form_equals_full_recompute():
    X = _contaminated(500, 5, 2)
    rng = np.random.default_rng(0)
    H_old = np.sort(rng.choice(500, 300, replace=False))
    H_new = np.sort(np.concatenate([H_old[30:], np.setdiff1d(np.arange(500), H_old)[:30]]))
    mu_o, S_o = oracle.subset_stats(X, H_old)
    mu_u, Lam_u = oracle.update_stats(X, H_old, H_new, mu_o, 299 * S_o)
    mu_f, S_f = oracle.subset_stats(X, H_new)
    assert np.allclose(mu_u, mu_f, rtol=1e-12, atol=1e-13)
    assert np.allclose(Lam_u / 299, S_f, rtol=1e-11, atol=1e-13)


def test_determinant_update_identity():
    # det(Lambda + d u v^T) = (1 + d v^T Lambda^-1 u) det(Lambda)  (Sec. 3.5)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6))
    Lam = A @ A.T + np.eye(6)
    u, v = rng.standard_normal(6), rng.standard_normal(6)
    for d in (1, -1):
        lhs = np.linalg.det(Lam + d * np.outer(u, v))
        assert lhs == pytest.approx((1 + d * v @ np.linalg.solve(Lam, u)) * np.linalg.det(Lam), rel=1e-10)


def _brute_cond1(S):
    # ||S||_1 ||S^-1||_1 from column sums of |S| and of |inverse|, the inverse
    # by Gauss-Jordan elimination written out here (no Cholesky, no LAPACK)
    n = S.shape[0]
    A = np.hstack([S.astype(float), np.eye(n)])
    for c in range(n):
        r = c + int(np.argmax(np.abs(A[c:, c])))
        A[[c, r]] = A[[r, c]]
        A[c] /= A[c, c]
        for k in range(n):
            if k != c:
                A[k] -= A[k, c] * A[c]
    Si = A[:, n:]
    norm1 = lambda M: max(sum(abs(M[i, j]) for i in range(n)) for j in range(n))
    return norm1(S) * norm1(Si)


@pytest.mark.parametrize("seed", [0, 3, 7])
def test_kappa1_is_the_one_norm_condition_number(seed):
    # eq. (choleskymonitor) uses the 1-norm: on a dense SPD matrix whose
    # 2-norm condition is 700 the 1-norm condition exceeds 1000, so a 2-norm
    # (eigenvalue ratio) reading would pass the check and the 1-norm one fails it
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    S = (Q * np.geomspace(1.0, 1.0 / 700.0, 6)) @ Q.T
    S = 0.5 * (S + S.T)
    k1 = _brute_cond1(S)
    assert np.linalg.cond(S, 2) < 1000.0 < k1
    L = np.linalg.cholesky(S)
    assert oracle.kappa1(S, L) == pytest.approx(k1, rel=1e-9)
    # and the C-step refuses a start with that scatter (Sec. 3.4)
    X = _contaminated(400, 6, 2)
    r = oracle.csteps(X, 300, X.mean(0), S)
    assert r.status == oracle.ST_DROP_FIRST
    # the same matrix scaled into the accepted range is taken
    S2 = (Q * np.geomspace(1.0, 1.0 / 20.0, 6)) @ Q.T
    S2 = 0.5 * (S2 + S2.T)
    assert oracle.kappa1(S2, np.linalg.cholesky(S2)) == pytest.approx(_brute_cond1(S2), rel=1e-9)
    assert oracle.csteps(X, 300, X.mean(0), S2).status == oracle.ST_CONVERGED


def _brute_median(v):
    # the middle order statistic, or the mean of the two middle ones, found by
    # counting how many values lie below and above each candidate
    v = [float(x) for x in v]
    n = len(v)
    def kth(k):   # k-th smallest, 0-based
        for x in v:
            below = sum(1 for y in v if y < x)
            equal = sum(1 for y in v if y == x)
            if below <= k < below + equal:
                return x
    return kth(n // 2) if n % 2 else 0.5 * (kth(n // 2 - 1) + kth(n // 2))


@pytest.mark.parametrize("n", [1, 2, 7, 8, 31, 64])
def test_medmad_matches_brute_force(n):
    # median and 1.4826 * median absolute deviation (odd and even counts,
    # with repeated values)
    rng = np.random.default_rng(n)
    x = np.round(rng.standard_normal(n) * 3.0, 1)
    med = _brute_median(x)
    mad = _brute_median([abs(a - med) for a in x])
    got_med, got_scale = oracle.medmad(x)
    assert got_med == med
    assert got_scale == pytest.approx(1.4826 * mad, rel=1e-15)


def test_medmad_consistent_at_the_normal():
    # 1.4826 MAD is consistent for the standard deviation at the normal
    # (1 / Phi^-1(3/4) = 1.482602...), and the median for its centre
    x = np.random.default_rng(12).standard_normal(1_000_000) * 2.5 + 4.0
    med, s = oracle.medmad(x)
    assert abs(med - 4.0) < 0.01
    assert abs(s / 2.5 - 1.0) < 0.005
    # location / scale equivariance
    med2, s2 = oracle.medmad(-3.0 * x + 1.0)
    assert med2 == pytest.approx(-3.0 * med + 1.0, rel=1e-12)
    assert s2 == pytest.approx(3.0 * s, rel=1e-12)


def test_kappa_threshold_stops_cstep():
    X = _contaminated(400, 3, 1)
    mu0 = X.mean(0)
    S0 = np.diag([1.0, 1.0, 1e-5])        # condition 1e5 > 1000
    r = oracle.csteps(X, 300, mu0, S0)
    assert r.status == oracle.ST_DROP_FIRST


# ---------------------------------------------------------------- exact MCD on tiny n

@pytest.mark.parametrize("seed,p", [(0, 1), (1, 2), (2, 2)])
def test_exact_mcd_enumeration(seed, p):
    rng = np.random.default_rng(seed)
    n, h = 12, 8 if p == 2 else 7
    X = rng.standard_normal((n, p))
    X[:3] += 6.0
    best, bestH = math.inf, None
    for H in itertools.combinations(range(n), h):
        H = np.array(H)
        _, S = oracle.subset_stats(X, H)
        ld = float(np.linalg.slogdet(np.atleast_2d(S))[1])
        if ld < best:
            best, bestH = ld, H
    # the global optimum is a C-step fixed point
    mu, S = oracle.subset_stats(X, bestH)
    r = oracle.csteps(X, h, mu, np.atleast_2d(S))
    # (step 1 reproduces H from the start, step 2 confirms it)
    assert np.array_equal(r.H, bestH) and r.iters == 2
    # any C-step fixed point has log-det >= the optimum
    H0 = np.arange(h)
    mu0, S0 = oracle.subset_stats(X, H0)
    r2 = oracle.csteps(X, h, mu0, np.atleast_2d(S0))
    assert r2.logdet >= best - 1e-12


# ---------------------------------------------------------------- aggregation

def test_kl_nonnegative_zero_iff_equal():
    rng = np.random.default_rng(6)
    for _ in range(20):
        A = rng.standard_normal((4, 4)); A = A @ A.T + 0.5 * np.eye(4)
        B = rng.standard_normal((4, 4)); B = B @ B.T + 0.5 * np.eye(4)
        a, b = rng.standard_normal(4), rng.standard_normal(4)
        assert oracle.kl_deviation(a, A, b, B) > 0
        assert oracle.kl_deviation(a, A, a, A) == pytest.approx(0.0, abs=1e-12)


def test_kl_rank_key_orders_like_kl():
    rng = np.random.default_rng(7)
    Amed = np.eye(3) * 1.5
    amed = np.zeros(3)
    fits = []
    for _ in range(12):
        B = rng.standard_normal((3, 3)); B = B @ B.T + 0.3 * np.eye(3)
        fits.append((rng.standard_normal(3), B))
    kl = [oracle.kl_deviation(amed, Amed, b, B) for b, B in fits]
    kp = [oracle.kl_rank_key(amed, Amed, b, B) for b, B in fits]
    assert list(np.argsort(kl)) == list(np.argsort(kp))
    c = -3 - np.linalg.slogdet(Amed)[1]
    assert np.allclose(np.array(kp) + c, kl)


def test_pooling_equals_direct_covariance_of_union():
    rng = np.random.default_rng(1)
    m, p = 40, 3
    blocks = [rng.standard_normal((m, p)) + rng.standard_normal(p) for _ in range(5)]
    mus = [b.mean(0) for b in blocks]
    sig = [np.cov(b, rowvar=False) for b in blocks]
    mu, S = oracle.pool_printed(mus, sig, m)
    U = np.concatenate(blocks)
    assert np.allclose(mu, U.mean(0), rtol=1e-12)
    assert np.allclose(S, np.cov(U, rowvar=False), rtol=1e-11)
    # unequal counts (step 9)
    sizes = [5, 17, 1, 30]
    bl = [rng.standard_normal((k, p)) for k in sizes]
    lams = [(b - b.mean(0)).T @ (b - b.mean(0)) for b in bl]
    mu2, Lam2, n2 = oracle.pool_counts([b.mean(0) for b in bl], lams, sizes)
    U = np.concatenate(bl)
    assert n2 == sum(sizes)
    assert np.allclose(mu2, U.mean(0)) and np.allclose(Lam2 / (n2 - 1), np.cov(U, rowvar=False))


def test_aggregate_single_block_is_identity():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 3)); A = A @ A.T + np.eye(3)
    mu = rng.standard_normal(3)
    m_, S_, keep, _ = oracle.aggregate([mu], [A], 100)
    assert np.allclose(m_, mu) and np.allclose(S_, A) and list(keep) == [0]


def test_aggregate_discards_far_blocks():
    rng = np.random.default_rng(3)
    good = [(0.01 * rng.standard_normal(2), np.eye(2) * (1 + 0.01 * rng.random())) for _ in range(5)]
    bad = [(np.array([20.0, 20.0]), np.eye(2) * 50) for _ in range(3)]
    fits = good + bad
    _, _, keep, _ = oracle.aggregate([f[0] for f in fits], [f[1] for f in fits], 100)
    assert len(keep) == 4 and all(k < 5 for k in keep)


# ---------------------------------------------------------------- full fit

def test_fit_single_chunk_flags_all_planted_outliers():
    ds = synthdata.workload_single_chunk_f64(n=2000, p=5)
    f = oracle.fit(ds.X)
    out = np.zeros(len(ds.X), bool)
    out[ds.outlier_rows] = True
    assert f.outlier[out].all()
    assert 0.005 < f.outlier[~out].mean() < 0.06
    assert f.hsubset.shape == (1, 1500)
    assert not np.isin(ds.outlier_rows, f.hsubset[0]).any()


def test_fit_monomial_equivariance():
    ds = synthdata.small_gaussian(3000, 4, seed=3, rho=0.5, eps=0.15, kind="cluster", gamma=7)
    X = ds.X
    perm = [2, 0, 3, 1]
    s = np.array([2.0, 0.5, 3.0, 1.5])
    b = np.array([1.0, -4.0, 0.0, 7.0])
    Y = X[:, perm] * s + b
    f1 = oracle.fit(X, n_chunks=2)
    f2 = oracle.fit(Y, n_chunks=2)
    assert np.array_equal(f1.hsubset, f2.hsubset)
    assert np.array_equal(f1.outlier, f2.outlier)
    assert np.allclose(f2.mu, f1.mu[perm] * s + b, rtol=1e-9, atol=1e-9)
    assert np.allclose(f2.sigma, f1.sigma[np.ix_(perm, perm)] * np.outer(s, s), rtol=1e-9, atol=1e-12)
    assert np.allclose(f1.dist, f2.dist, rtol=1e-9)


def test_fit_multi_chunk_union_pooling_option():
    ds = synthdata.small_gaussian(8000, 3, seed=4, rho=0.3, eps=0.1, kind="point", gamma=6)
    a = oracle.fit(ds.X, n_chunks=4, pool="printed")
    b = oracle.fit(ds.X, n_chunks=4, pool="union")
    assert np.array_equal(a.hsubset, b.hsubset)
    # both keep the point outliers out of the reweighted fit
    out = np.zeros(len(ds.X), bool)
    out[ds.outlier_rows] = True
    assert a.outlier[out].all() and b.outlier[out].all()


def test_fit_remainder_rows_scored():
    ds = synthdata.small_gaussian(4003, 3, seed=5)
    f = oracle.fit(ds.X, n_chunks=4)
    assert f.m == 1000 and len(f.dist) == 4003
    d2 = oracle.mahalanobis2((ds.X[-3:] - f.loc) / f.scale, f.diag["mu_rew_z"],
                             np.linalg.cholesky(f.diag["sigma_rew_z"]))
    assert np.allclose(f.dist[-3:] ** 2, d2)


def test_refinement_location_translation_equivariance():
    # mu_k(Z + b) = mu_k(Z) + b for a fixed initial scatter (Sec. 3.3 step 4)
    rng = np.random.default_rng(12)
    C = np.array([[1.0, 0.6, 0.1], [0.6, 2.0, -0.4], [0.1, -0.4, 0.7]])
    Z = rng.standard_normal((4000, 3)) @ np.linalg.cholesky(C).T
    S0 = oracle.init_gsscm(Z)
    b = np.array([0.8, -1.5, 0.4])
    a = oracle.refine(S0, Z)
    c = oracle.refine(S0, Z + b)
    assert np.allclose(c.mu, a.mu + b, rtol=0, atol=1e-9)
    assert np.allclose(c.sigma, a.sigma, rtol=1e-9)


def test_refinement_small_case_brute_force():
    # Whole refinement on a tiny block with a brute-force univariate MCD.
    rng = np.random.default_rng(13)
    Z = rng.standard_normal((41, 2)) @ np.array([[1.0, 0.0], [0.7, 0.5]])
    S0 = oracle.init_wrap_cov(Z)

    def brute(x):
        js, mean, var = _brute_unimcd(x)
        n = len(x)
        var_raw = var * oracle.consistency_factor((n // 2 + 1) / n, 1)
        keep = [v for v in x if (v - mean) ** 2 <= oracle.chi2_quantile(0.975, 1) * var_raw]
        return statistics.fmean(keep), statistics.variance(keep) * oracle.consistency_factor(0.975, 1)

    lam, V = np.linalg.eigh(S0)
    V = V[:, ::-1]
    T = Z @ V
    sig2 = np.array([brute(T[:, j])[1] for j in range(2)])
    Sig = V @ np.diag(sig2) @ V.T
    Zt = Z @ (V @ np.diag(sig2 ** -0.5) @ V.T)
    mut = np.array([brute(Zt[:, j])[0] for j in range(2)])
    mu = V @ np.diag(sig2 ** 0.5) @ V.T @ mut
    st = oracle.refine(S0, Z)
    assert np.allclose(st.sigma, Sig, rtol=1e-10) and np.allclose(st.mu, mu, rtol=1e-9, atol=1e-12)


def test_aggregate_keeps_ceil_half_of_odd_count():
    rng = np.random.default_rng(14)
    fits = [(0.01 * rng.standard_normal(2), np.eye(2) * (1 + 0.01 * rng.random())) for _ in range(7)]
    _, _, keep, _ = oracle.aggregate([f[0] for f in fits], [f[1] for f in fits], 50)
    assert len(keep) == 4


def test_fit_reweighting_set_by_textbook_distances():
    ds = synthdata.small_gaussian(3000, 2, seed=6, rho=0.4, eps=0.1, kind="shift", gamma=5)
    f = oracle.fit(ds.X)
    Z = (ds.X - f.loc) / f.scale
    Si = np.linalg.inv(f.diag["sigma_raw_z"])
    D = Z - f.diag["mu_raw_z"]
    d2 = np.einsum("ij,jk,ik->i", D, Si, D)
    W = d2 <= -2.0 * math.log(0.025)          # chi2_{2,0.975} closed form
    assert f.n_w == int(W.sum())
    assert np.allclose(f.diag["mu_rew_z"], Z[W].mean(axis=0), rtol=1e-10)
    Dw = Z[W] - Z[W].mean(axis=0)
    assert np.allclose(f.diag["sigma_rew_z"], Dw.T @ Dw / (W.sum() - 1), rtol=1e-10)
    # flags: final squared distance above the same cutoff
    Si2 = np.linalg.inv(f.diag["sigma_rew_z"])
    D2 = Z - f.diag["mu_rew_z"]
    fl = np.einsum("ij,jk,ik->i", D2, Si2, D2) > -2.0 * math.log(0.025)
    assert np.array_equal(fl.astype(np.uint8), f.outlier)


def test_condition_check_in_standardised_units():
    # The condition monitor of Sec. 3.4 acts on standardised data; raw units pass
    # their column scales so that rescaling a column does not trip it.
    X = _contaminated(500, 2, 3, eps=0.0)
    s = np.array([1.0, 300.0])
    H0 = np.arange(400)
    mu0, S0 = oracle.subset_stats(X, H0)
    Xs = X * s
    r_scaled = oracle.csteps(Xs, 400, mu0 * s, S0 * np.outer(s, s), kappa_scale=s)
    r_plain = oracle.csteps(X, 400, mu0, S0)
    assert r_scaled.status == r_plain.status == oracle.ST_CONVERGED
    assert np.array_equal(r_scaled.H, r_plain.H)
    r_raw = oracle.csteps(Xs, 400, mu0 * s, S0 * np.outer(s, s))
    assert r_raw.status == oracle.ST_DROP_FIRST


def test_random_partition_is_the_fit_of_the_permuted_rows():
    """Sec. 4 partitions the rows at random: fitting X with blocks
    X[perm[l m : (l+1) m]] is fitting X[perm] with contiguous blocks.  The
    global standardisation depends only on the columns' values (up to the
    rounding of its sums, which run in row order), so the two fits make the
    same discrete choices and agree to rounding once rows are mapped back
    through perm."""
    rng = np.random.default_rng(77)
    n, p, q = 1203, 3, 3
    X = rng.standard_normal((n, p)) @ np.array([[1.0, 0.4, 0.0], [0.0, 1.0, 0.3], [0.0, 0.0, 1.0]])
    X[rng.choice(n, 120, replace=False)] += 6.0
    perm = rng.permutation(n)
    fp = oracle.fit(X, n_chunks=q, perm=perm)
    fc = oracle.fit(X[perm], n_chunks=q)
    close = lambda a, b: np.allclose(a, b, rtol=1e-12, atol=1e-14)
    assert close(fp.loc, fc.loc) and close(fp.scale, fc.scale)
    assert close(fp.mu, fc.mu) and close(fp.sigma, fc.sigma)
    assert np.array_equal(fp.chunk_status, fc.chunk_status)
    assert np.array_equal(fp.hsubset, perm[fc.hsubset])
    assert close(fp.dist[perm], fc.dist)
    assert np.array_equal(fp.outlier[perm], fc.outlier)
    assert np.array_equal(fp.rew_mask[perm], fc.rew_mask)
    assert fp.n_w == fc.n_w
    # the identity permutation is the contiguous partition
    fi = oracle.fit(X, n_chunks=q, perm=np.arange(n))
    f0 = oracle.fit(X, n_chunks=q)
    assert np.array_equal(fi.hsubset, f0.hsubset) and np.array_equal(fi.sigma, f0.sigma)


# ---------------------------------------------------------------- explicit-inverse distances (Table 1, I vs ID)

def test_inverse_distances_equal_forward_substitution():
    # Sec. 3.4: ||L^{-1} r||^2 = r^T Sigma^{-1} r; the two are computed by
    # different routines (triangular solve against a general inverse)
    rng = np.random.default_rng(31)
    p = 7
    A = rng.standard_normal((p, p))
    S = A @ A.T + p * np.eye(p)
    X = rng.standard_normal((500, p)) * 3.0
    mu = rng.standard_normal(p)
    d_inv = oracle.mahalanobis2_inverse(X, mu, np.linalg.inv(S))
    d_chol = oracle.mahalanobis2(X, mu, np.linalg.cholesky(S))
    assert np.allclose(d_inv, d_chol, rtol=1e-12, atol=0.0)


def test_inverse_distances_diagonal_closed_form():
    rng = np.random.default_rng(32)
    s = rng.uniform(0.5, 4.0, 5)
    X = rng.standard_normal((100, 5))
    d = oracle.mahalanobis2_inverse(X, np.zeros(5), np.diag(1.0 / s ** 2))
    assert np.allclose(d, np.sum((X / s) ** 2, axis=1), rtol=1e-14)


# ---------------------------------------------------------------- single-swap updates (Sec. 3.5)

def _sscp(X, H):
    mu = X[H].mean(axis=0)
    D = X[H] - mu
    return mu, D.T @ D


def test_smw_swap_matches_recomputation():
    # eq. (woodbury) and eq. (scaleddetUpdate): after one case leaves and one
    # enters, the carried inverse and log determinant equal those of the sscp
    # matrix recomputed from the new subset, and the mean is its mean
    rng = np.random.default_rng(33)
    m, p, h = 200, 4, 150
    X = rng.standard_normal((m, p)) @ rng.standard_normal((p, p))
    H = np.sort(rng.choice(m, h, replace=False))
    out_i = int(H[17])
    in_i = int(np.setdiff1d(np.arange(m), H)[5])
    mu, Lam = _sscp(X, H)
    st = (h, mu, Lam, np.linalg.inv(Lam), float(np.linalg.slogdet(Lam)[1]))
    for i, dlt in ((out_i, -1), (in_i, +1)):
        st = oracle.smw_swap(X[i], dlt, *st)
    hh, mu2, Lam2, Li2, ld2 = st
    H2 = np.sort(np.concatenate([H[H != out_i], [in_i]]))
    mu_r, Lam_r = _sscp(X, H2)
    assert hh == h
    assert np.allclose(mu2, mu_r, rtol=1e-12, atol=1e-13)
    assert np.allclose(Lam2, Lam_r, rtol=1e-11, atol=1e-10)
    assert np.allclose(Li2, np.linalg.inv(Lam_r), rtol=1e-9, atol=1e-13)
    assert ld2 == pytest.approx(np.linalg.slogdet(Lam_r)[1], abs=1e-10)


def test_smw_swap_singular_update_is_refused():
    # p = 1, subset {0, 2}: removing 2 leaves one point, whose sscp is 0:
    # Delta = 1 - (x - mu_new) Lam^{-1} (x - mu_old) = 1 - 2 * 0.5 * 1 = 0
    X = np.array([[0.0], [2.0]])
    Lam = np.array([[2.0]])
    assert oracle.smw_swap(X[1], -1, 2, np.array([1.0]), Lam, np.linalg.inv(Lam),
                           math.log(2.0)) is None


@pytest.mark.parametrize("seed,m,p", [(0, 400, 2), (5, 1000, 3), (10, 3000, 5)])
def test_csteps_smw_mode_follows_full_mode(seed, m, p):
    # the single-swap update is exact: the same subsets, iterations and
    # determinants as full recomputation, with at least one swap step taken
    ds = synthdata.small_gaussian(m, p, seed=seed, rho=0.6, eps=0.1, kind="shift", gamma=3)
    X = ds.X.astype(float)
    h = oracle.subset_size(m, p, 0.75)
    rng = np.random.default_rng(seed)
    mu0, S0 = oracle.subset_stats(X, np.sort(rng.choice(m, h, replace=False)))
    a = oracle.csteps(X, h, mu0, S0)
    b = oracle.csteps(X, h, mu0, S0, mode="smw")
    assert b.smw_steps > 0
    assert (a.status, a.iters) == (b.status, b.iters)
    assert np.array_equal(a.H, b.H)
    assert b.logdet == pytest.approx(a.logdet, abs=1e-10)
    assert np.allclose(b.sigma, a.sigma, rtol=1e-10, atol=1e-12)
    assert np.allclose(a.logdets, b.logdets, atol=1e-10)
    c = oracle.csteps(X, h, mu0, S0, distance="inverse")
    assert np.array_equal(a.H, c.H) and a.iters == c.iters


def test_fit_distance_and_update_switches_leave_the_fit_unchanged():
    # Sec. 5: versions I, ID and IDC agree up to rounding (the paper's
    # "equivalent if numerical precision were perfect")
    ds = synthdata.small_gaussian(6000, 4, seed=12, rho=0.5, eps=0.15, kind="shift", gamma=5)
    a = oracle.fit(ds.X, n_chunks=3)
    b = oracle.fit(ds.X, n_chunks=3, distance="inverse")
    c = oracle.fit(ds.X, n_chunks=3, cstep_mode="smw")
    for f in (b, c):
        assert np.array_equal(a.hsubset, f.hsubset)
        assert np.array_equal(a.outlier, f.outlier)
        assert np.allclose(a.sigma, f.sigma, rtol=1e-10)
    assert sum(r.smw_steps for st in c.diag["starts"] for r in st) > 0


# ---------------------------------------------------------------- warm start (end of Sec. 4)

def test_warm_start_from_a_fixed_point_reproduces_the_fit():
    # a block's converged h-subset is a C-step fixed point: started from that
    # subset's mean and covariance (given in data units), the C-steps select
    # it again at once (two steps: select, then confirm), so the whole fit is
    # reproduced; the data are far from standardised, so the units matter
    ds = synthdata.small_gaussian(3000, 3, seed=4, rho=0.5, eps=0.1, kind="shift", gamma=6)
    X = ds.X * np.array([50.0, 0.01, 3.0]) + np.array([1e3, -2.0, 7.0])
    a = oracle.fit(X)
    assert a.chunk_status[0] == oracle.ST_CONVERGED
    H = a.hsubset[0]
    mu_h = X[H].mean(axis=0)
    S_h = np.cov(X[H], rowvar=False, ddof=1)
    b = oracle.fit(X, warm=(mu_h, S_h))
    assert b.chunk_start[0] == oracle.START_WARM
    assert b.chunk_iters[0] == 2 and b.chunk_status[0] == oracle.ST_CONVERGED
    assert np.array_equal(a.hsubset, b.hsubset)
    assert np.array_equal(a.outlier, b.outlier)
    assert np.allclose(a.sigma, b.sigma, rtol=1e-12)
    assert np.allclose(a.mu, b.mu, rtol=1e-12)


def test_warm_start_on_new_data_lowers_no_determinant():
    # the C-step monotonicity (Prop. 1) holds from a warm start too: each
    # block's determinant sequence from step 2 on does not increase
    old = synthdata.small_gaussian(8000, 4, seed=21, rho=0.6, eps=0.1, kind="shift", gamma=6)
    new = synthdata.small_gaussian(8000, 4, seed=22, rho=0.6, eps=0.1, kind="shift", gamma=6)
    f0 = oracle.fit(old.X, n_chunks=2)
    f1 = oracle.fit(new.X, n_chunks=2, warm=(f0.mu, f0.sigma))
    for st in f1.diag["starts"]:
        assert len(st) == 1
        ld = st[0].logdets
        assert all(b <= a + 1e-9 for a, b in zip(ld[1:], ld[2:]))
    assert np.all(f1.chunk_start == oracle.START_WARM)


# ---------------------------------------------------------------- O12 diagnostics

from oracle import rtdetmcd as R   # noqa: E402

def test_h_gap_hand_case_and_ties():
    # sorted (1, 2, 3, 5): keeping 2 leaves 3 as the smallest left out
    assert R.h_gap(np.array([3.0, 1.0, 2.0, 5.0]), 2) == 1.0
    # a tie across the threshold
    assert R.h_gap(np.array([2.0, 1.0, 2.0, 7.0]), 2) == 0.0
    assert math.isnan(R.h_gap(np.array([1.0, 2.0]), 2))


@pytest.mark.parametrize("seed", range(5))
def test_h_gap_is_the_gap_between_kept_and_left_out(seed):
    # against the selected subset itself: smallest distance outside H minus
    # the largest inside (ties by row index do not change the values)
    rng = np.random.default_rng(seed)
    d2 = np.round(rng.exponential(size=40), 1)   # rounded: ties occur
    for h in (5, 20, 39):
        H = R.select_h(d2, h)
        out = np.setdiff1d(np.arange(40), H)
        assert R.h_gap(d2, h) == d2[out].min() - d2[H].max()


@pytest.mark.parametrize("seed", range(3))
def test_logdet_trace_follows_the_cstep_theorem(seed):
    # Sec. 2.1: a C-step never increases det(Sigma); the trace holds one entry
    # per evaluated step of the chosen start, its last entry that start's
    # final log det (converged blocks), NaN after
    ds = synthdata.small_gaussian(1200, 4, seed=seed, eps=0.1)
    F = R.fit(ds.X, n_chunks=2)
    tr = F.diag["block_logdets"]
    for l in range(F.q):
        it = int(F.chunk_iters[l])
        assert np.all(np.isfinite(tr[l, :it])) and np.all(np.isnan(tr[l, it:]))
        assert np.all(np.diff(tr[l, :it]) <= 1e-12)
        best = F.diag["starts"][l][int(F.chunk_start[l])]
        assert best.logdets == list(tr[l, :it])
        if F.chunk_status[l] == R.ST_CONVERGED:
            assert tr[l, it - 1] == best.logdet


def test_flag_margin_is_the_closest_final_distance_to_the_cutoff():
    ds = synthdata.small_gaussian(1500, 3, seed=4, eps=0.1)
    F = R.fit(ds.X, n_chunks=1)
    chi2 = F.diag["chi2"]
    brute = min(abs(float(d) ** 2 - chi2) for d in F.dist)
    assert math.isclose(F.diag["cmargin"], brute, rel_tol=1e-9, abs_tol=1e-12)
    assert F.diag["cmargin"] <= min(abs(F.diag["d2_final"] - chi2)) + 1e-15
