"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-only helpers agree with independent references."""
import os
import re

import numpy as np
import pytest
from scipy import stats

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rtdetmcd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rtdetmcd_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1910_05615_amd import _lib
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.SYMBOLS) == names


@pytest.mark.parametrize("df", [1, 2, 3, 5, 10, 20, 22, 40, 42, 64])
@pytest.mark.parametrize("q", [0.5, 0.5001, 0.75, 0.9, 0.975, 0.99])
def test_chi2_quantile_and_cdf_match_scipy(df, q):
    import paper_1910_05615_amd as P
    x = P.chi2_quantile(q, df)
    assert x == pytest.approx(stats.chi2.ppf(q, df), rel=1e-12)
    assert P.chi2_cdf(x, df) == pytest.approx(q, rel=1e-12)
    for xx in (0.1, 1.0, df * 0.7, df * 1.3, df + 30):
        assert P.chi2_cdf(xx, df) == pytest.approx(stats.chi2.cdf(xx, df), rel=1e-11, abs=1e-300)


@pytest.mark.parametrize("p", [1, 2, 5, 10, 20, 40])
@pytest.mark.parametrize("alpha", [0.5, 0.75, 0.75003, 0.975])
def test_consistency_factor_matches_oracle(p, alpha):
    import paper_1910_05615_amd as P
    assert P.consistency(alpha, p) == pytest.approx(oracle.consistency_factor(alpha, p), rel=1e-11)


def test_plan_rules_match_oracle():
    import paper_1910_05615_amd as P
    for n, p, q in [(1_000_000, 20, 64), (10_000, 10, 1), (10_000_000, 40, 1024),
                    (200_000, 40, 0), (4003, 3, 4), (524288, 4, 0)]:
        qq, m, h = P.plan(n, p, 0, q)
        q_ref = q if q else oracle.n_blocks(n, p)
        assert qq == q_ref and m == n // q_ref and h == oracle.subset_size(m, p, 0.75)
    with pytest.raises(Exception):
        P.plan(10, 8, 0, 0)
    with pytest.raises(Exception):
        P.plan(1000, 65, 0, 0)
