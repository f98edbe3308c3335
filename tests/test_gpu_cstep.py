"""GPU parity of the C-step core (distances, exact selection, C-step loop)
against the float64 CPU oracle.  Called through the C ABI via the binding."""
import math

import numpy as np
import pytest

import oracle
import synthdata

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _P():
    import paper_1910_05615_amd as P
    return P


def _dev():
    return torch.device("cuda:0")


def _spd(p, rng, cond=20.0):
    A = rng.standard_normal((p, p))
    Q, _ = np.linalg.qr(A)
    ev = np.exp(rng.uniform(0, math.log(cond), p))
    return (Q * ev) @ Q.T


@pytest.mark.parametrize("p", [1, 3, 5, 10, 17, 20, 33, 40, 64])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_distances_match_oracle(p, dtype):
    P = _P()
    rng = np.random.default_rng(p)
    n = 5000 + 17                         # several tiles and a ragged tail
    X = rng.standard_normal((n, p)) * rng.uniform(0.5, 3, p) + rng.uniform(-5, 5, p)
    X = X.astype(np.float32 if dtype == "f32" else np.float64)
    S = _spd(p, rng)
    mu = rng.standard_normal(p)
    L = np.linalg.cholesky(S)
    ref = oracle.mahalanobis2(X.astype(np.float64), mu, L)
    d2 = P.distances(torch.from_numpy(X).to(_dev()), torch.from_numpy(mu), torch.from_numpy(L))
    got = d2.cpu().numpy()
    assert got.shape == (n,)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=0)


def test_distances_strided_rows():
    P = _P()
    rng = np.random.default_rng(1)
    Xf = rng.standard_normal((3001, 24)).astype(np.float32)
    X = Xf[:, :20]                              # row stride 24
    S = _spd(20, rng)
    mu = rng.standard_normal(20)
    ref = oracle.mahalanobis2(X.astype(np.float64), mu, np.linalg.cholesky(S))
    Xt = torch.from_numpy(Xf).to(_dev())[:, :20]
    got = P.distances(Xt, torch.from_numpy(mu), torch.from_numpy(np.linalg.cholesky(S))).cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-11)


@pytest.mark.parametrize("m,h", [(1, 1), (2, 1), (7, 3), (1000, 750), (1024, 1023),
                                 (5000 + 13, 2600), (15625, 11718), (70000, 52500)])
def test_select_bit_exact(m, h):
    P = _P()
    rng = np.random.default_rng(m + h)
    d2 = rng.chisquare(5, m)
    got_idx, got_mask = P.select(torch.from_numpy(d2).to(_dev()), h)
    ref = oracle.select_h(d2, h)
    assert np.array_equal(got_idx.cpu().numpy(), ref)
    mk = np.zeros(m, np.uint8)
    mk[ref] = 1
    assert np.array_equal(got_mask.cpu().numpy(), mk)


@pytest.mark.parametrize("case", ["ties", "all_equal", "zeros", "two_values", "nan", "tiny",
                                  "heavy_tail", "crowded_threshold", "equal_block_at_threshold"])
@pytest.mark.parametrize("m,h", [(4099, 2050), (40_003, 30_001)])   # one chunk / several
def test_select_ties_and_degenerate(case, m, h):
    P = _P()
    rng = np.random.default_rng(3)
    if case == "ties":
        d2 = rng.integers(0, 20, m).astype(np.float64)
    elif case == "all_equal":
        d2 = np.full(m, 3.25)
    elif case == "zeros":
        d2 = np.where(rng.random(m) < 0.6, 0.0, rng.random(m))
    elif case == "two_values":
        d2 = np.where(rng.random(m) < 0.5, 1.0, np.nextafter(1.0, 2.0))
    elif case == "nan":
        d2 = rng.random(m)
        d2[rng.choice(m, 50, replace=False)] = np.nan
    elif case == "heavy_tail":      # keys over many binades
        d2 = np.abs(rng.standard_cauchy(m)) ** 3
    elif case == "crowded_threshold":   # ~400 distinct keys within 1e-12 of the h-th
        d2 = rng.random(m) * 10.0
        near = rng.choice(m, 400, replace=False)
        d2[near] = 5.0 + rng.random(400) * 1e-12
        d2[d2 < 5.0] = d2[d2 < 5.0] * 0.5   # the h-th smallest lands among them
    elif case == "equal_block_at_threshold":   # 300 equal keys across rank h
        d2 = rng.random(m) * 10.0
        d2[rng.choice(m, 300, replace=False)] = float(np.sort(d2)[h])
    else:
        d2 = rng.random(m) * 1e-300
    got_idx, _ = P.select(torch.from_numpy(d2).to(_dev()), h)
    ref = oracle.select_h(np.where(np.isnan(d2), np.inf, d2), h)
    assert np.array_equal(got_idx.cpu().numpy(), ref)


def _start(X, h, seed):
    rng = np.random.default_rng(seed)
    H0 = np.sort(rng.choice(X.shape[0], h, replace=False))
    return oracle.subset_stats(X.astype(np.float64), H0)


@pytest.mark.parametrize("mode", ["full", "update", "auto"])
@pytest.mark.parametrize("launch", ["batched", "plain"])
@pytest.mark.parametrize("p,dtype", [(2, "f64"), (5, "f32"), (10, "f64"), (20, "f32"), (40, "f32")])
def test_cstep_matches_oracle(mode, launch, p, dtype):
    P = _P()
    m = 6000 + 11
    ds = synthdata.small_gaussian(m, p, seed=p, rho=0.6, eps=0.2, kind="shift", gamma=4,
                                  dtype=np.float32 if dtype == "f32" else np.float64)
    X = ds.X
    h = oracle.subset_size(m, p, 0.75)
    mu0, S0 = _start(X, h, p)
    ref = oracle.csteps(X.astype(np.float64), h, mu0, S0)
    r = P.cstep(torch.from_numpy(X).to(_dev()), h, torch.from_numpy(mu0), torch.from_numpy(S0),
                cstep_mode=mode, launch=launch)
    assert r.status == ref.status
    assert r.iters == ref.iters
    assert np.array_equal(r.hsubset.cpu().numpy(), ref.H)
    mu = r.mu.cpu().numpy()
    S = r.sigma.cpu().numpy()
    Si = np.linalg.inv(ref.sigma)
    assert math.sqrt((mu - ref.mu) @ Si @ (mu - ref.mu)) < 1e-9
    assert np.linalg.norm(S - ref.sigma) / np.linalg.norm(ref.sigma) < 1e-10
    assert abs(r.logdet - ref.logdet) < 1e-9


def test_cstep_condition_monitor_in_standardised_units():
    P = _P()
    X = synthdata.small_gaussian(3000, 2, seed=9, rho=0.2).X
    s = np.array([1.0, 300.0])
    Xs = X * s
    h = 2000
    mu0, S0 = _start(X, h, 1)
    ref = oracle.csteps(Xs, h, mu0 * s, S0 * np.outer(s, s), kappa_scale=s)
    r = P.cstep(torch.from_numpy(Xs).to(_dev()), h, torch.from_numpy(mu0 * s),
                torch.from_numpy(S0 * np.outer(s, s)), kappa_scale=torch.from_numpy(s))
    assert r.status == ref.status == oracle.ST_CONVERGED
    assert np.array_equal(r.hsubset.cpu().numpy(), ref.H)
    r2 = P.cstep(torch.from_numpy(Xs).to(_dev()), h, torch.from_numpy(mu0 * s),
                 torch.from_numpy(S0 * np.outer(s, s)))
    assert r2.status == oracle.ST_DROP_FIRST


def test_cstep_max_steps_and_ill_conditioned_start():
    P = _P()
    X = synthdata.small_gaussian(4000, 3, seed=2, rho=0.5, eps=0.2, kind="shift", gamma=3).X
    h = 3000
    mu0, S0 = _start(X, h, 4)
    ref = oracle.csteps(X, h, mu0, S0, max_steps=2)
    r = P.cstep(torch.from_numpy(X).to(_dev()), h, torch.from_numpy(mu0), torch.from_numpy(S0),
                max_csteps=2)
    assert r.status == ref.status and r.iters == ref.iters
    assert np.array_equal(r.hsubset.cpu().numpy(), ref.H)
    bad = np.diag([1.0, 1.0, 1e-6])
    r3 = P.cstep(torch.from_numpy(X).to(_dev()), h, torch.from_numpy(mu0), torch.from_numpy(bad))
    assert r3.status == oracle.ST_DROP_FIRST


@pytest.mark.parametrize("p,dtype", [(4, "f32"), (20, "f32"), (40, "f64"), (7, "f32")])
def test_score_matches_oracle(p, dtype):
    P = _P()
    rng = np.random.default_rng(100 + p)
    n = 10_000 + 33
    X = (rng.standard_normal((n, p)) * 2 + 1).astype(np.float32 if dtype == "f32" else np.float64)
    S = _spd(p, rng)
    mu = rng.standard_normal(p)
    L = np.linalg.cholesky(S)
    Linv = np.linalg.inv(L)
    d2 = oracle.mahalanobis2(X.astype(np.float64), mu, L)
    cut = oracle.chi2_quantile(0.975, p)
    dist, flag = P.score(torch.from_numpy(X).to(_dev()), torch.from_numpy(mu), torch.from_numpy(Linv))
    np.testing.assert_allclose(dist.cpu().numpy(), np.sqrt(d2), rtol=1e-11)
    # flags decided on float64 d2; compare away from the threshold
    far = np.abs(d2 - cut) > 1e-9 * cut
    assert np.array_equal(flag.cpu().numpy()[far], (d2 > cut).astype(np.uint8)[far])


@pytest.mark.parametrize("p,dtype", [(20, "f32"), (10, "f32"), (10, "f64"), (40, "f32"), (16, "f64")])
def test_dense_and_generic_row_paths_agree(p, dtype):
    """Dense, aligned rows take the whole-row vector loads; the same rows one
    element past an aligned base take the per-element path.  Both evaluate
    the same float64 operations in the same order: bitwise equal outputs."""
    P = _P()
    rng = np.random.default_rng(300 + p)
    n = 4096 + 77
    tdt = torch.float32 if dtype == "f32" else torch.float64
    X = (rng.standard_normal((n, p)) * 2 + 1).astype(np.float32 if dtype == "f32" else np.float64)
    S = _spd(p, rng)
    mu = rng.standard_normal(p)
    L = np.linalg.cholesky(S)
    Linv = np.linalg.inv(L)
    Xa = torch.from_numpy(X).to(_dev())
    buf = torch.empty(n * p + 1, dtype=tdt, device=_dev())
    Xu = buf[1:].view(n, p)
    Xu.copy_(Xa)
    assert Xu.data_ptr() % 16 != 0 and Xa.data_ptr() % 16 == 0
    da, fa = P.score(Xa, torch.from_numpy(mu), torch.from_numpy(Linv))
    du, fu = P.score(Xu, torch.from_numpy(mu), torch.from_numpy(Linv))
    assert torch.equal(da, du) and torch.equal(fa, fu)
    ga = P.distances(Xa, torch.from_numpy(mu), torch.from_numpy(L))
    gu = P.distances(Xu, torch.from_numpy(mu), torch.from_numpy(L))
    assert torch.equal(ga, gu)
    ref = oracle.mahalanobis2(X.astype(np.float64), mu, L)
    np.testing.assert_allclose(ga.cpu().numpy(), ref, rtol=1e-11, atol=0)
    np.testing.assert_allclose(da.cpu().numpy(), np.sqrt(ref), rtol=1e-11)


@pytest.mark.parametrize("p,dtype", [(20, "f32"), (1, "f64"), (3, "f32")])
def test_score_and_distances_empty_and_tiny(p, dtype):
    """n = 0 (nothing read or written), a single row, two rows and a ragged
    257; p = 1 and 3 take the per-element row path of their bucket."""
    P = _P()
    rng = np.random.default_rng(500 + p)
    S = _spd(p, rng)
    mu = rng.standard_normal(p)
    L = np.linalg.cholesky(S)
    Linv = np.linalg.inv(L)
    npdt = np.float32 if dtype == "f32" else np.float64
    for n in (0, 1, 2, 257):
        X = (rng.standard_normal((n, p)) * 2).astype(npdt)
        Xt = torch.from_numpy(X).to(_dev())
        d2 = P.distances(Xt, torch.from_numpy(mu), torch.from_numpy(L))
        dist, flag = P.score(Xt, torch.from_numpy(mu), torch.from_numpy(Linv))
        assert d2.shape == (n,) and dist.shape == (n,) and flag.shape == (n,)
        if n:
            ref = oracle.mahalanobis2(X.astype(np.float64), mu, L)
            np.testing.assert_allclose(d2.cpu().numpy(), ref, rtol=1e-11, atol=1e-300)
            np.testing.assert_allclose(dist.cpu().numpy(), np.sqrt(ref), rtol=1e-11)
