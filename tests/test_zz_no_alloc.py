"""GPU check of the allocation-free C-step entry point rtdetmcd_cstep_noalloc:
through the C ABI it gives exactly the outputs of rtdetmcd_cstep on the same
block and start, on two calls in a row (the second on a smaller block, so its
state sits in an array that still holds the first call's), and it refuses
blocks above its stated limit."""
import math

import numpy as np
import pytest

import oracle
import synthdata

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _start(X, h, seed):
    rng = np.random.default_rng(seed)
    H0 = np.sort(rng.choice(X.shape[0], h, replace=False))
    return oracle.subset_stats(X.astype(np.float64), H0)


def _run(P, X, h, mu0, S0, noalloc, **kw):
    dev = torch.device("cuda:0")
    r = P.cstep(torch.from_numpy(X).to(dev), h, torch.from_numpy(mu0), torch.from_numpy(S0),
                noalloc=noalloc, **kw)
    torch.cuda.synchronize()
    return r


def _same(a, b):
    assert a.status == b.status
    assert a.iters == b.iters
    assert torch.equal(a.hsubset, b.hsubset)
    assert torch.equal(a.mu, b.mu)
    assert torch.equal(a.sigma, b.sigma)
    assert a.logdet == b.logdet


@pytest.mark.parametrize("mode", ["full", "update"])
def test_noalloc_cstep_equals_cstep_twice(mode):
    import paper_1910_05615_amd as P
    cases = [(60000, 20, np.float32, 3), (7001, 5, np.float64, 4)]   # second call smaller
    for m, p, dt, seed in cases:
        X = synthdata.small_gaussian(m, p, seed=seed, rho=0.6, eps=0.15, kind="shift", gamma=4,
                                     dtype=dt).X
        h = oracle.subset_size(m, p, 0.75)
        mu0, S0 = _start(X, h, seed)
        print(f"noalloc case m={m} p={p} dtype={np.dtype(dt).name} mode={mode}", flush=True)
        ref = _run(P, X, h, mu0, S0, False, cstep_mode=mode)
        got = _run(P, X, h, mu0, S0, True, cstep_mode=mode)
        _same(got, ref)
        # and the oracle agrees with both (float64 decisions on both sides)
        o = oracle.csteps(X.astype(np.float64), h, mu0, S0)
        assert got.status == o.status and got.iters == o.iters
        assert np.array_equal(got.hsubset.cpu().numpy(), o.H)
        assert np.linalg.norm(got.sigma.cpu().numpy() - o.sigma) / np.linalg.norm(o.sigma) < 1e-10


def test_noalloc_cstep_rejects_blocks_above_the_limit():
    import paper_1910_05615_amd as P
    m, p = 131073, 2
    X = np.zeros((m, p), dtype=np.float32)
    X[:, 0] = np.arange(m, dtype=np.float32)
    X[:, 1] = np.arange(m, dtype=np.float32) % 7
    with pytest.raises(P.RTDetMCDError, match="EINVAL"):
        _run(P, X, m // 2 + 2, np.zeros(p), np.eye(p), True)
