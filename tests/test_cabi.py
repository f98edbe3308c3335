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


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of rtdetmcd_opts, rtdetmcd_out and rtdetmcd_dataset
    have the header's size and field offsets (a C program compiled against
    include/rtdetmcd.h prints them), and the library's defaults hold."""
    import ctypes
    import subprocess
    from paper_1910_05615_amd import _lib
    structs = {"rtdetmcd_opts": _lib.Opts, "rtdetmcd_out": _lib.Out,
               "rtdetmcd_dataset": _lib.DatasetDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rtdetmcd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                             text=True).stdout.splitlines():
        s, f, v = ln.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
    lib = _lib.load()
    o = _lib.Opts()
    lib.rtdetmcd_default_opts(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(_lib.Opts)
    assert (o.tune, o.graph, o.rounds_per_sync, o.distance) == (0, 0, 4, 0)
