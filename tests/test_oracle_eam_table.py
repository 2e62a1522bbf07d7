"""Pins of the oracle's tabulated EAM path (the setfl form of the potential
of Eq. (pe): F(rhobar), rho(r), r*phi(r) on uniform knots, not-a-knot cubic
splines between them).

  - splines of linear tables are exact: tabulated linear functions come back
    exactly at any argument (this pins the coefficient layout and evaluation);
  - the Sutton-Chen functions tabulated on fine knots reproduce the analytic
    oracle's forces with the O(dr^3) error of spline derivatives (halving dr
    divides it by ~8) and its energy with the O(dr^4) error of values;
  - forces are the exact negative gradient of the tabulated energy (central
    differences, O(delta^2));
  - past the last knot F continues linearly with the end slope.
"""
import numpy as np
import pytest

import synth


def sc_tables(orc, nr=4001, rc=8.1, nrho=4001, rho_max=200.0, r_min=1.0, shift=2):
    """Sutton-Chen functions (with the oracle's shift) on setfl knots; below
    r_min (never reached by neighbours) the functions are held constant."""
    p = orc.sc_params(shift=shift)
    dr = rc / (nr - 1)
    r = np.maximum(np.arange(nr) * dr, r_min)
    V = np.array([orc.pair_terms(p, x)[0] for x in r])
    rho = np.array([orc.pair_terms(p, x)[2] for x in r])
    rphi = r * V
    rho[-1] = 0.0
    rphi[-1] = 0.0  # r = rc: the shifted functions vanish there
    drho = rho_max / (nrho - 1)
    F = np.array([orc.embed(p, x) for x in np.arange(nrho) * drho])
    return F, rho, rphi, drho, dr, rc


def test_linear_tables_are_exact(orc):
    nr, dr, nrho, drho = 50, 0.2, 40, 0.5
    r = np.arange(nr) * dr
    q = np.arange(nrho) * drho
    T = orc.TabPotential(3.0 - 0.25 * q, 2.0 - 0.1 * r, 5.0 - 0.5 * r, drho, dr, rc=(nr - 1) * dr)
    rng = np.random.default_rng(1)
    for x in rng.uniform(0.3, (nr - 1) * dr - 1e-9, 50):
        V, dV, rh, drh = orc.pair_terms(T.sc, x)
        assert rh == pytest.approx(2.0 - 0.1 * x, rel=1e-13)
        assert drh == pytest.approx(-0.1, rel=1e-12)
        assert V == pytest.approx((5.0 - 0.5 * x) / x, rel=1e-13)
        assert dV == pytest.approx(-5.0 / x ** 2, rel=1e-11)
    for x in rng.uniform(0.0, (nrho - 1) * drho, 20):
        assert orc.embed(T.sc, x) == pytest.approx(3.0 - 0.25 * x, rel=1e-13, abs=1e-14)
        assert orc.embed_deriv(T.sc, x) == pytest.approx(-0.25, rel=1e-12)
    # past the last knot: linear continuation with the end slope
    top = (nrho - 1) * drho
    assert orc.embed(T.sc, top + 3.0) == pytest.approx(3.0 - 0.25 * (top + 3.0), rel=1e-12)


@pytest.fixture(scope="module")
def sc_tab(orc):
    return orc.TabPotential(*sc_tables(orc))


def test_tabulated_sutton_chen_matches_analytic(orc, sc_tab):
    """Spline derivatives carry an O(dr^3) interpolation error: halving the
    knot spacing cuts the force error by ~8, and at dr = 2e-3 A it is below
    1e-8 of the rms force (energies: O(dr^4), below 1e-11 relative)."""
    s = synth.cube_state(4, 0.1, 0.0, 3)
    ref = orc.forces(s["x"], s["y"], s["z"], orc.sc_params(), s["group"])
    F = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
    frms = np.sqrt((F ** 2).sum(1).mean())
    errs = []
    for T in (orc.TabPotential(*sc_tables(orc, nr=2001)), sc_tab):
        tab = orc.forces(s["x"], s["y"], s["z"], T.sc, s["group"])
        G = np.stack([tab["fx"], tab["fy"], tab["fz"]], 1)
        errs.append(np.abs(G - F).max() / frms)
        du = abs(tab["U"] - ref["U"]) / abs(ref["U"])
    print(f"\nforce error / F_rms at dr = 4e-3, 2e-3 A: {errs[0]:.2e}, {errs[1]:.2e}; U rel {du:.1e}")
    assert errs[1] <= 1e-8
    assert 5.0 < errs[0] / errs[1] < 11.0
    assert du <= 1e-11
    assert tab["Wzz"] == pytest.approx(ref["Wzz"], rel=1e-8)


def test_tabulated_forces_are_energy_gradients(orc, sc_tab):
    s = synth.cube_state(3, 0.1, 0.0, 9, fix_slabs=False)
    x, y, z = s["x"].copy(), s["y"].copy(), s["z"].copy()
    f = orc.forces(x, y, z, sc_tab.sc)
    d = 1e-5
    for i in (0, 17, 50):
        for arr, comp in ((x, "fx"), (z, "fz")):
            arr[i] += d
            up = orc.forces(x, y, z, sc_tab.sc)["U"]
            arr[i] -= 2 * d
            dn = orc.forces(x, y, z, sc_tab.sc)["U"]
            arr[i] += d
            assert -(up - dn) / (2 * d) == pytest.approx(f[comp][i], rel=1e-6, abs=1e-8)
