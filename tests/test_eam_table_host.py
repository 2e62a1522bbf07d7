"""Host-side checks of the tabulated EAM path (no GPU): the library's spline
coefficients and evaluation against the oracle's (scipy's not-a-knot spline
evaluated by the oracle's C code), and the setfl reader."""
import os

import numpy as np
import pytest

from test_oracle_eam_table import sc_tables

P = pytest.importorskip("paper_2603_07321_amd")


def test_library_spline_matches_oracle(orc):
    F, rho, rphi, drho, dr, rc = sc_tables(orc, nr=801, nrho=401)
    T = orc.TabPotential(F, rho, rphi, drho, dr, rc)
    rng = np.random.default_rng(4)
    r = rng.uniform(1.2, rc, 400)
    top = (len(F) - 1) * drho
    # below the first knot (negative densities of some tables) and far past the last
    q = np.concatenate([rng.uniform(0.0, top, 300), [top + 7.5, top * 1e6, 1e12, -0.3 * drho, -2.5 * drho]])
    f1, d1 = P.eam_table_eval(F, rho, rphi, drho, dr, rc, 1, r)
    f2, d2 = P.eam_table_eval(F, rho, rphi, drho, dr, rc, 2, r)
    fF, dF = P.eam_table_eval(F, rho, rphi, drho, dr, rc, 0, q)
    for k, x in enumerate(r):
        V, dV, rh, drh = orc.pair_terms(T.sc, x)
        assert f1[k] == pytest.approx(rh, rel=1e-11, abs=1e-13)
        assert d1[k] == pytest.approx(drh, rel=1e-9, abs=1e-12)
        assert f2[k] / x == pytest.approx(V, rel=1e-11, abs=1e-14)
        assert (d2[k] - f2[k] / x) / x == pytest.approx(dV, rel=1e-9, abs=1e-12)
    for k, x in enumerate(q):
        assert fF[k] == pytest.approx(orc.embed(T.sc, x), rel=1e-12, abs=1e-14)
        assert dF[k] == pytest.approx(orc.embed_deriv(T.sc, x), rel=1e-9, abs=1e-12)


def test_spline_reproduces_cubics_exactly():
    """A not-a-knot spline through samples of one cubic is that cubic."""
    n, h = 30, 0.3
    xs = np.arange(n) * h
    cub = lambda x: 1.0 - 2.0 * x + 0.5 * x ** 2 - 0.03 * x ** 3
    dcub = lambda x: -2.0 + x - 0.09 * x ** 2
    y = cub(xs)
    x = np.linspace(0.0, (n - 1) * h, 97)
    f, df = P.eam_table_eval(y, y, y, h, h, (n - 1) * h, 1, x)
    assert np.allclose(f, cub(x), rtol=0, atol=1e-12)
    assert np.allclose(df, dcub(x), rtol=0, atol=1e-11)


def _write_setfl(path, F, rho, rphi, drho, dr, rc, per_line=5, fortran=False):
    def fmt(v):
        s = f"{v:.16e}"
        return s.replace("e", "D") if fortran else s

    with open(path, "w") as fh:
        fh.write("synthetic table\nSutton-Chen functions on setfl knots\nfor the reader test\n")
        fh.write("1 Al\n")
        fh.write(f"{len(F)} {fmt(drho)} {len(rho)} {fmt(dr)} {fmt(rc)}\n")
        fh.write("13 26.982 4.05 fcc\n")
        for arr in (F, rho, rphi):
            for k in range(0, len(arr), per_line):
                fh.write(" ".join(fmt(v) for v in arr[k:k + per_line]) + "\n")


@pytest.mark.parametrize("per_line,fortran", [(5, False), (3, True), (1, False)])
def test_setfl_round_trip(orc, tmp_path, per_line, fortran):
    F, rho, rphi, drho, dr, rc = sc_tables(orc, nr=301, nrho=201)
    path = os.path.join(tmp_path, "al.setfl")
    _write_setfl(path, F, rho, rphi, drho, dr, rc, per_line, fortran)
    t = P.read_setfl(path)
    assert t["mass"] == 26.982 and t["rc"] == rc and t["dr"] == dr and t["drho"] == drho
    for k, a in (("F", F), ("rho", rho), ("rphi", rphi)):
        assert np.array_equal(t[k], a)


def test_setfl_errors(orc, tmp_path):
    F, rho, rphi, drho, dr, rc = sc_tables(orc, nr=101, nrho=101)
    good = os.path.join(tmp_path, "ok.setfl")
    _write_setfl(good, F, rho, rphi, drho, dr, rc)
    lines = open(good).read().splitlines()
    cases = {
        "missing.setfl": None,
        "two.setfl": lines[:3] + ["2 Al Ni"] + lines[4:],
        "short.setfl": lines[:-3],
        "badnum.setfl": lines[:8] + ["1.0 x2.0 3.0"] + lines[9:],
    }
    for name, content in cases.items():
        path = os.path.join(tmp_path, name)
        if content is not None:
            with open(path, "w") as fh:
                fh.write("\n".join(content) + "\n")
        with pytest.raises(P.PtamdError) as ei:
            P.read_setfl(path)
        assert ei.value.name == "PTAMD_EINVAL", name


def test_table_validation(orc):
    F, rho, rphi, drho, dr, rc = sc_tables(orc, nr=101, nrho=101)
    for bad in (dict(rc=rc + 0.5), dict(rc=-1.0), dict(dr=0.0), dict(F=F[:3]), dict(rho=np.r_[rho[:-1], np.nan])):
        args = dict(F=F, rho=rho, rphi=rphi if "rho" not in bad else np.r_[rphi[:-1], 0.0], drho=drho, dr=dr, rc=rc)
        args.update(bad)
        with pytest.raises(P.PtamdError) as ei:
            P.eam_table_eval(args["F"], args["rho"], args["rphi"], args["drho"], args["dr"], args["rc"], 1, [1.0])
        assert ei.value.name == "PTAMD_EINVAL", bad
