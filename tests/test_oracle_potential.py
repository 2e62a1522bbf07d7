"""Pins of the oracle's potential, constants and random numbers against facts
that do not come from the oracle itself: published test vectors, exact values
of powers, SI constants from scipy, finite differences, FCC shell structure
and lattice sums enumerated independently of the oracle's atom loops.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.constants as sc
from scipy import stats

pytestmark = []


def test_constants_against_scipy(orc):
    c = orc.constants()
    u = sc.physical_constants["atomic mass constant"][0]
    # the oracle uses the CODATA 2018 atomic mass constant; scipy may carry a
    # later adjustment (they differ by ~1.4e-9 relative)
    assert c["mvv2e"] == pytest.approx(u * 1e10 / sc.e, rel=1e-8)
    assert c["kb"] == pytest.approx(sc.k / sc.e, rel=1e-12)
    assert c["gpa"] == pytest.approx(sc.e / 1e-30 / 1e9, rel=1e-12)
    assert c["mass"] == pytest.approx(26.9815385, rel=1e-12)


def test_splitmix64_published_vectors(orc):
    # First outputs of Vigna's reference SplitMix64 seeded with 1234567.
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [orc.splitmix64(1234567, k) for k in range(5)] == want


def test_box_muller_normality(orc):
    g = orc.gaussians(42, 200_000)
    assert abs(g.mean()) < 0.01
    assert g.std() == pytest.approx(1.0, abs=0.01)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # the two halves of each Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(g[0::2], g[1::2])[0, 1]) < 0.01
    # counter based: a prefix is the same stream
    assert np.array_equal(orc.gaussians(42, 10), g[:10])


def test_power_law_values(orc):
    # V(a) = eps, rho(a) = 1; at r = a/sqrt(2): (a/r)^n = 2^(n/2).  No shift.
    p = orc.sc_params(shift=0)
    V, dV, rho, drho = orc.pair_terms(p, 4.05)
    assert V == pytest.approx(0.0033147, rel=1e-14)
    assert rho == pytest.approx(1.0, rel=1e-14)
    r = 4.05 / math.sqrt(2.0)
    V, dV, rho, drho = orc.pair_terms(p, r)
    assert V == pytest.approx(0.0033147 * 2 ** 3.5, rel=1e-13)
    assert rho == pytest.approx(8.0, rel=1e-13)
    # beyond or at the cutoff everything vanishes (strict r < rc)
    assert orc.pair_terms(p, 8.1) == (0.0, 0.0, 0.0, 0.0)
    assert orc.pair_terms(p, 9.0) == (0.0, 0.0, 0.0, 0.0)


def test_embedding_values(orc):
    p = orc.sc_params()
    c, eps = 16.399, 0.0033147
    assert orc.embed(p, 1.0) == pytest.approx(-c * eps, rel=1e-14)
    assert orc.embed(p, 4.0) == pytest.approx(-2 * c * eps, rel=1e-14)
    assert orc.embed(p, 0.0) == 0.0
    assert orc.embed_deriv(p, 0.0) == 0.0
    for rho in (0.3, 7.0, 120.0):
        h = 1e-6 * rho
        fd = (orc.embed(p, rho + h) - orc.embed(p, rho - h)) / (2 * h)
        assert orc.embed_deriv(p, rho) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("shift", [0, 1, 2])
def test_pair_derivatives_match_finite_differences(orc, shift):
    p = orc.sc_params(shift=shift)
    for r in np.linspace(2.6, 8.0, 13):
        h = 1e-6
        Vp, _, rp, _ = orc.pair_terms(p, r + h)
        Vm, _, rm, _ = orc.pair_terms(p, r - h)
        V, dV, rho, drho = orc.pair_terms(p, r)
        assert dV == pytest.approx((Vp - Vm) / (2 * h), rel=1e-6, abs=1e-14)
        assert drho == pytest.approx((rp - rm) / (2 * h), rel=1e-6, abs=1e-12)


def test_shift_modes_at_cutoff(orc):
    rc = 8.1
    below = rc * (1 - 1e-9)
    # energy shift: values -> 0 at rc; shifted force: values and slopes -> 0
    V, dV, rho, drho = orc.pair_terms(orc.sc_params(shift=1), below)
    assert abs(V) < 1e-12 and abs(rho) < 1e-9
    assert dV != 0.0
    V, dV, rho, drho = orc.pair_terms(orc.sc_params(shift=2), below)
    assert abs(V) < 1e-15 and abs(rho) < 1e-12
    assert abs(dV) < 1e-12 and abs(drho) < 1e-9
    # the shifted-force density is non-negative below rc (convex rho)
    for r in np.linspace(2.0, rc * 0.999, 50):
        assert orc.pair_terms(orc.sc_params(shift=2), r)[2] >= 0.0


def _fcc_shells(rcut_over_half: float):
    """FCC lattice vectors as integer triples (h,k,l), h+k+l even, in units of
    a/2, grouped by squared length (enumerated here, not by the oracle)."""
    m = int(math.ceil(rcut_over_half))
    shells = {}
    rng = range(-m, m + 1)
    for h in rng:
        for k in rng:
            for l in rng:
                if (h, k, l) == (0, 0, 0) or (h + k + l) % 2:
                    continue
                q = h * h + k * k + l * l
                if q < rcut_over_half ** 2:
                    shells[q] = shells.get(q, 0) + 1
    return dict(sorted(shells.items()))


def test_fcc_shell_counts():
    # textbook FCC coordination shells: 12, 6, 24, 12, 24, 8, 48, 6
    sh = _fcc_shells(4.5)  # up to |v|^2 = 16 in (a/2)^2 units, i.e. r = 2a
    assert list(sh.items())[:8] == [(2, 12), (4, 6), (6, 24), (8, 12), (10, 24), (12, 8), (14, 48), (16, 6)]


def _bulk_energy(orc, p):
    half = p.a / 2
    sh = _fcc_shells(p.rc / half + 1)
    vsum, rsum = 0.0, 0.0
    for q, cnt in sh.items():
        V, _, rho, _ = orc.pair_terms(p, math.sqrt(q) * half)
        vsum += cnt * V
        rsum += cnt * rho
    return 0.5 * vsum + orc.embed(p, rsum)


@pytest.mark.parametrize("shift,rc", [(0, 7.9), (1, 7.9), (2, 7.9), (2, 8.1)])
def test_bulk_atom_energy_equals_shell_sum(orc, shift, rc):
    """An atom at least 2 rc inside a perfect cube has the bulk energy, which
    the shell sum gives independently of the oracle's pair loops.  rc = 8.1 A
    = 2a sits exactly on the 8th shell, where rounding of the coordinates
    decides in or out; that tie only cancels for the shifted-force form, so
    the other forms use a cutoff between shells."""
    p = orc.sc_params(shift=shift, rc=rc)
    nc = 10
    x, y, z, g, pz = orc.fcc_cube(nc, 4.05, False)
    f = orc.forces(x, y, z, p, per_atom_energy=True)
    ctr = (nc - 0.5) * 4.05 / 2 + 0.0
    i = int(np.argmin((x - ctr) ** 2 + (y - ctr) ** 2 + (z - ctr) ** 2))
    assert min(x[i], y[i], z[i], 9 * 4.05 + 2.025 - max(x[i], y[i], z[i])) >= 2 * 8.1 - 1.0
    assert f["e"][i] == pytest.approx(_bulk_energy(orc, p), rel=1e-12)


def test_bulk_energy_known_value(orc):
    # shifted-force bulk energy per atom at the stated parameters; the same
    # value times 10 at eps x 10 (energy is linear in eps)
    p = orc.sc_params()
    e = _bulk_energy(orc, p)
    assert e == pytest.approx(-0.321424942, abs=2e-9)
    assert _bulk_energy(orc, orc.sc_params(eps=0.033147)) == pytest.approx(10 * e, rel=1e-13)


def test_sutton_chen_c_is_the_equilibrium_constant():
    """Sutton and Chen chose c so the infinite perfect lattice is in
    equilibrium at a: c = n S_n / (m sqrt(S_m)), S_k = sum_j (a/r_j)^k.  This
    pins the parameter set (n=7, m=6, c=16.399 at a=4.05) to the functional
    form, independently of the oracle."""
    sh = _fcc_shells(40.0)
    S = {k: sum(cnt * (2.0 / math.sqrt(q)) ** k for q, cnt in sh.items()) for k in (6, 7)}
    # tail beyond |v| = 40 (a/2 units): integral of density 4/a^3 over r>R
    R = 40.0 * 0.5  # in units of a
    for k in (6, 7):
        S[k] += 4.0 * 4 * math.pi * R ** (3 - k) / (k - 3)
    c_eq = 7 * S[7] / (6 * math.sqrt(S[6]))
    assert c_eq == pytest.approx(16.399, abs=2e-3)


def test_table1_golden_parameters():
    here = os.path.dirname(__file__)
    with open(os.path.join(here, "golden", "table1_parameters.json")) as fh:
        t = json.load(fh)
    import synth
    assert synth.A_AL == t["lattice_parameter_A"]
    w = synth.workloads()["cube10_fp64_200"]
    assert w.burst_steps == 200
    assert t["md_timestep_fs"] == 1.0
