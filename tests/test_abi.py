"""CPU checks of the C-ABI library: it loads, exports every symbol declared in
include/fse.h, and its host-side geometry agrees with the oracle's own
derivation of the paper's parameters (no GPU needed)."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fse():
    import paper_1607_04808_amd as F
    return F


def test_library_exports_every_declared_symbol():
    F = _fse()
    lib = F.lib()
    header = open(os.path.join(ROOT, "include", "fse.h")).read()
    names = set(re.findall(r"\b(fse_[a-z_]+)\s*\(", header))
    assert len(names) >= 13
    for name in sorted(names):
        assert hasattr(lib, name), name
    assert set(F.fse.EXPORTS) == names


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("rule", [0, 1])
def test_geometry_matches_oracle(kernel, rule):
    from oracle import se
    F = _fse()
    for xi, rc, M, P, L, lo in ((7.0, 0.63, 48, 16, 2.0, (0, 0, 0)), (60.0, 0.063, 194, 14, 1.0, (0, 0, 0)),
                                (12.0, 0.3, 32, 11, 1.5, (-1.0, 2.0, 0.25))):
        g = F.geometry(kernel, F.make_params(xi, rc, M, P, lo, L, deltaL_rule=rule))
        o = se.geometry(xi, rc, M, P, lo, L, Mt=g.Mt, deltaL_rule=rule)
        assert g.Mt >= se.geometry(xi, rc, M, P, lo, L, deltaL_rule=rule).Mt
        assert g.n_fft == 2 * g.Mt
        for k in ("h", "d", "m", "eta", "alpha", "Lt", "R"):
            assert getattr(g, k) == pytest.approx(getattr(o, k), rel=1e-14), k
        np.testing.assert_allclose(g.x0, o.x0, rtol=0, atol=1e-14)
        assert g.Mg == o.Mg
        assert g.cell >= rc and g.ncell >= 1
        prod = 1
        for r in g.radices:
            assert r in (2, 3, 4, 5, 7, 8)
            prod *= r
        assert prod == g.n_fft


def test_geometry_rejects_bad_parameters():
    F = _fse()
    bad = [dict(xi=-1.0), dict(rc=0.0), dict(M=0), dict(P=1), dict(P=33), dict(L=0.0),
           dict(deltaL_rule=2), dict(Mt=3), dict(Mt=97)]
    base = dict(xi=5.0, rc=0.3, M=20, P=8, box_lo=(0, 0, 0), L=1.0)
    for b in bad:
        kw = dict(base)
        kw.update(b)
        with pytest.raises(F.FseError) as e:
            F.geometry("stokeslet", F.make_params(**kw))
        assert e.value.status == 1
    with pytest.raises(F.FseError):
        F.geometry("stokeslet", F.make_params(xi=5.0, rc=0.3, M=1020, P=8))  # Mt = 1028 > 1024


def test_forced_grid_size_and_padding():
    F = _fse()
    g = F.geometry("rotlet", F.make_params(6.0, 0.5, 20, 8, L=1.0, Mt=35))
    assert g.Mt == 35 and g.radices and math.prod(g.radices) == 70
    assert g.deltaL == pytest.approx(15 * g.h)


def test_no_oracle_in_product_path():
    """The package never imports the oracle (it is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_1607_04808_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dp, f)).read()
                assert "oracle" not in src.replace("oracle_", ""), f
