"""The batched-uneven and large workloads at full size on the GPU.

512 datasets in one batched fit: every dataset valid, a sample checked
against the oracle, and every dataset checked for the identities that hold at
any size.  10,000,000 x 40 in 1,024 blocks: the standardisation of sampled
columns against the oracle's estimator, each sampled block's h-subset a
C-step fixed point of its own mean and covariance, the reweighted fit equal
to the classical estimates of the kept rows, flags consistent with the
distances of every row (the 640 rows past the last block included), and the
whole fit equal to the oracle's fit of the same data (a stored digest)."""
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


def _check_identities(X, F, c_rew=1.0):
    """Identities of the end of any fit (Sec. 4 steps 8-10)."""
    P = _P()
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    W = F.rew_mask.cpu().numpy().astype(bool)
    assert int(W.sum()) == int(F.n_w.cpu()[0])
    mu = X[W].mean(axis=0)
    S = c_rew * np.cov(X[W], rowvar=False, ddof=1)
    Fm, Fs = F.mu.cpu().numpy(), F.sigma.cpu().numpy()
    assert math.sqrt(float((Fm - mu) @ np.linalg.solve(S, Fm - mu))) < 1e-8
    assert np.linalg.norm(Fs - S) <= 1e-8 * np.linalg.norm(S)
    d = F.dist.cpu().numpy()
    assert np.all(np.isfinite(d))
    chi2 = P.chi2_quantile(0.975, p)
    flag = F.outlier.cpu().numpy().astype(bool)
    differ = flag != (d * d > chi2)
    # d is the square root of the decided d2: only a rounding away from the cutoff
    assert np.all(np.abs(d[differ] ** 2 - chi2) <= 1e-12 * chi2)
    # distances under (mu, Sigma) on a row sample
    rows = np.random.default_rng(0).choice(n, min(n, 4096), replace=False)
    R = X[rows] - Fm
    d2 = np.einsum("ij,ij->i", R, np.linalg.solve(Fs, R.T).T)
    assert np.allclose(d[rows] ** 2, d2, rtol=1e-9, atol=1e-12)


def test_batched_uneven_512_datasets():
    P = _P()
    sets = synthdata.workload_batched_uneven()
    assert len(sets) == 512
    Xs = [torch.from_numpy(s.X).to(_dev()) for s in sets]
    fits, status = P.fit_batched(Xs)
    assert status == [0] * 512
    for s, F in zip(sets, fits):
        assert int((F.block_status < 3).sum().cpu()) >= 1
        _check_identities(s.X, F)
    # oracle parity on a sample spanning every p and the size range
    sizes = np.array([s.X.shape[0] for s in sets])
    pick = []
    for p in (5, 10, 20, 40):
        idx = [i for i, s in enumerate(sets) if s.X.shape[1] == p]
        idx.sort(key=lambda i: sizes[i])
        pick += [idx[0], idx[len(idx) // 2]]
        if p in (5, 40):
            pick.append(idx[-1])   # the longest: p = 5 in 9 blocks, p = 40 in one
    for i in pick:
        check_fit(fits[i], oracle.fit(sets[i].X), sets[i].name)


def test_large_p40_full_size():
    P = _P()
    ds = synthdata.workload_large_p40()
    n, p = ds.X.shape
    X = torch.from_numpy(ds.X).to(_dev())
    F = P.fit(X, n_chunks=1024, cstep_mode="update")
    q, m, h = F.q, F.m, F.h
    assert (q, m, h) == (1024, 9765, 7323)
    bst = F.block_status.cpu().numpy()
    assert np.all(bst < 3)
    # standardisation of sampled columns: the oracle's estimator on 10^7 values
    loc, scale = F.loc.cpu().numpy(), F.scale.cpu().numpy()
    for j in (0, 17, 39):
        u = oracle.unimcd(ds.X[:, j].astype(np.float64))
        assert abs(loc[j] - u.mu) <= 1e-12 * max(1.0, abs(u.mu)) + 1e-13
        assert abs(scale[j] - math.sqrt(u.var)) <= 1e-12 * math.sqrt(u.var)
    # sampled blocks: the h-subset is a C-step fixed point (ties by row index)
    H = F.hsubset.cpu().numpy()
    rng = np.random.default_rng(4)
    checked = 0
    for b in rng.choice(q, 24, replace=False):
        if bst[b] != 0:          # converged blocks only
            continue
        rows = np.arange(b * m, (b + 1) * m)
        Z = (ds.X[rows].astype(np.float64) - loc) / scale
        Hb = H[b] - b * m
        muH = Z[Hb].mean(axis=0)
        SH = np.cov(Z[Hb], rowvar=False, ddof=1)
        L = np.linalg.cholesky(SH)
        d2 = np.sum(np.linalg.solve(L, (Z - muH).T) ** 2, axis=0)
        order = np.lexsort((np.arange(m), d2))
        srt = np.sort(d2)
        if (srt[h] - srt[h - 1]) <= 1e-9 * srt[h]:
            continue             # a near-tie at the h-th distance decides nothing here
        assert np.array_equal(np.sort(order[:h]), Hb), b
        checked += 1
    assert checked >= 12
    _check_identities(ds.X, F)
    # the rows past the last block are scored too
    tail = F.dist.cpu().numpy()[q * m:]
    assert tail.size == n - q * m == 640 and np.all(np.isfinite(tail))
    _check_large_digest(F)


def _check_large_digest(F):
    """The whole fit against the oracle's fit of the same seeded data, stored
    as a digest by tests/golden/make_large_p40_digest.py (oracle only): every
    block's status, start, iterations and h-subset (CRC32 and sum of its
    row indices), standardisation, raw and reweighted fits, the reweighting
    set and the flagged rows exactly, distances on sampled rows."""
    import json
    import os
    import zlib
    path = os.path.join(os.path.dirname(__file__), "golden", "large_p40_oracle_digest.json")
    with open(path) as f:
        g = json.load(f)
    crc = lambda a: int(zlib.crc32(np.ascontiguousarray(a).tobytes()))
    assert (F.q, F.m, F.h) == (g["q"], g["m"], g["h"])
    np.testing.assert_allclose(F.loc.cpu().numpy(), g["loc"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(F.scale.cpu().numpy(), g["scale"], rtol=1e-12)
    assert F.block_status.cpu().numpy().tolist() == g["block_status"]
    assert F.block_start.cpu().numpy().tolist() == g["block_start"]
    assert F.block_iters.cpu().numpy().tolist() == g["block_iters"]
    H = F.hsubset.cpu().numpy().astype(np.int32)
    bad = [b for b in range(F.q) if crc(H[b]) != g["hsubset_crc32"][b] or
           int(H[b].astype(np.int64).sum()) != g["hsubset_sum"][b]]
    assert not bad, f"blocks whose h-subset differs from the oracle's: {bad[:10]}"
    assert int(F.n_w.cpu()[0]) == g["n_w"]
    assert crc(F.rew_mask.cpu().numpy().astype(np.uint8)) == g["rew_mask_crc32"]
    flagged = np.nonzero(F.outlier.cpu().numpy())[0].astype(np.int64)
    assert flagged.size == g["n_flagged"] and crc(flagged) == g["flagged_crc32"]
    for name in ("sigma_raw", "sigma"):
        a, b = getattr(F, name).cpu().numpy(), np.array(g[name])
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-8, name
    for mname, sname in (("mu_raw", "sigma_raw"), ("mu", "sigma")):
        d = getattr(F, mname).cpu().numpy() - np.array(g[mname])
        assert math.sqrt(float(d @ np.linalg.solve(np.array(g[sname]), d))) < 1e-8, mname
    ld = F.logdet.cpu().numpy()
    assert abs(ld[0] - g["logdet_raw"]) < 1e-8 and abs(ld[1] - g["logdet_rew"]) < 1e-8
    rows = np.array(g["dist_rows"])
    np.testing.assert_allclose(F.dist.cpu().numpy()[rows], g["dist_at_rows"], rtol=1e-9)
