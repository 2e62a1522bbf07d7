"""The mixed form's folded step (systems of up to 131,072 atoms), through
the C ABI: its density pass also does the step's kick-drift (lambda, the
sample record, the convergence decision, the atom update) and forms the
pair terms' positions from the force pass's next-position copy.  The FP64
parity tests pin the separate kick-drift path; these run the folded one
against the FP64 oracle at the mixed form's bars, and against itself where
the oracle's FP64 decisions cannot be compared.

Bars (mixed form, as in the parity tests): positions |dr| <= 1e-4 A and
PE per atom 1e-5 eV over bursts of up to 200 steps, other averages
relative 1e-4; mean positions 1e-4 A; a convergence stop is taken at the
first checkpoint where the burst's own recorded series passes the test.
"""
import numpy as np
import pytest

import synth
from oracle import pta as T

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def _orc():
    import oracle
    return oracle


def _state(nc, noise, T0, seed):
    O = _orc()
    s = synth.cube_state(nc, noise, 0.0, seed)
    vx, vy, vz = O.mb_velocities(s["group"], T0, seed)
    s.update(vx=vx, vy=vy, vz=vz)
    return s


def _orc_state(s):
    O = _orc()
    return O.State(s["x"].copy(), s["y"].copy(), s["z"].copy(), s["vx"].copy(), s["vy"].copy(), s["vz"].copy(),
                   s["group"].copy(), s["volume0"], s["area0"])


def _dr(st, os_):
    return max(np.abs(st[k] - getattr(os_, k)).max() for k in ("x", "y", "z"))


@pytest.mark.parametrize("skin,thermostat,n_steps", [(1.0, 1, 150), (0.3, 1, 150), (1.0, 0, 100)])
def test_folded_trajectory_matches_oracle(skin, thermostat, n_steps):
    O = _orc()
    s = _state(5, 0.05, 300.0, 91)
    md = P.md_params(precision=1, lanes_per_atom=4, skin=skin, thermostat=thermostat)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        g.apply_strain_increment(1e-4)
        avg = g.run_fast_md(n_steps)[0]
        st = g.get_state()
        info = g.info()
    os_ = _orc_state(s)
    O.apply_strain(os_, 1e-4)
    ravg, _ = O.run_burst(os_, O.sc_params(), O.md_params(thermostat=thermostat), n_steps)
    dr = _dr(st, os_)
    print(f"\nfolded, skin {skin}, thermostat {thermostat}: |dr| {dr:.2e}, builds {info['list_builds']}, "
          f"dKE {avg['ke'] - ravg['ke']:.2e}, dPE {avg['pe'] - ravg['pe']:.2e}")
    assert info["rollbacks"] == 0
    assert dr <= 1e-4
    assert abs(avg["pe"] - ravg["pe"]) / len(s["x"]) <= 1e-5
    for k in ("ke", "szz"):
        assert avg[k] == pytest.approx(ravg[k], rel=1e-4, abs=1e-6), k
    assert avg["n_samples"] == n_steps


def test_folded_hot_start_short_burst():
    """Velocities drawn at 900 K under a 300 K thermostat: lambda stays
    ~0.3% below 1 and changes by up to ~1e-4 per step.  The density pass's
    neighbour positions take the last lambda for the next one, which leaves
    them within ~1e-6 A of the true ones; over a short burst (no chaotic
    growth yet) the trajectory stays at the mixed form's own rounding level
    (lambda taken as 1 would move the density pass's positions by ~2e-5 A
    on average, |lambda - 1| dt |v|)."""
    O = _orc()
    s = _state(5, 0.05, 900.0, 96)
    md = P.md_params(precision=1, lanes_per_atom=4)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        avg = g.run_fast_md(30)[0]
        st = g.get_state()
        ser = g.get_series(0, 30)
    os_ = _orc_state(s)
    ravg, rser = O.run_burst(os_, O.sc_params(), O.md_params(), 30, series=True)
    dr = _dr(st, os_)
    dlam = np.abs(ser[:, 4] - rser[:, 4]).max()
    print(f"\nfolded, hot start, 30 steps: |dr| {dr:.2e}, lambda {ser[1, 4]:.6f}..{ser[-1, 4]:.6f}, "
          f"|dlambda| {dlam:.1e}, dKE {avg['ke'] - ravg['ke']:.2e}")
    assert dr <= 1e-6
    assert dlam <= 1e-8
    assert avg["ke"] == pytest.approx(ravg["ke"], rel=1e-6)


def test_folded_close_to_the_fp64_path():
    s = _state(6, 0.05, 300.0, 92)
    out = []
    for precision in (0, 1):
        with P.System.from_state(s, T0=300.0, md=P.md_params(precision=precision, lanes_per_atom=4)) as g:
            a = g.run_fast_md(200)[0]
            out.append((a, g.get_state()))
    (a0, s0), (a1, s1) = out
    dr = max(np.abs(s0[k] - s1[k]).max() for k in ("x", "y", "z"))
    print(f"\nmixed (folded) vs FP64 (kick-drift) path, 200 steps: |dr| {dr:.2e}")
    assert dr <= 1e-4
    assert a1["pe"] == pytest.approx(a0["pe"], rel=1e-6)


def test_folded_mean_positions_match_oracle():
    O = _orc()
    s = _state(5, 0.05, 300.0, 93)
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=1, lanes_per_atom=4)) as g:
        g.set_mean_positions(True)
        g.apply_strain_increment(2e-4)
        g.run_fast_md(100)
        mean = g.get_mean_positions()
    os_ = _orc_state(s)
    O.apply_strain(os_, 2e-4)
    _, _, rmean = O.run_burst(os_, O.sc_params(), O.md_params(), 100, mean_positions=True)
    print(f"\nfolded mean positions: max |d| {np.abs(mean - rmean).max():.2e}")
    assert np.abs(mean - rmean).max() <= 1e-4


def test_folded_relaxation_matches_oracle():
    O = _orc()
    s = _state(5, 0.05, 300.0, 94)
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=1, lanes_per_atom=4)) as g:
        avg, nb, ok = g.relax(40, 2, 0.0)
        st = g.get_state()
    os_ = _orc_state(s)
    ravg, rk, rok = O.relax(os_, O.sc_params(), O.md_params(), 40, 2, 0.0)
    assert nb == rk == 2 and not ok[0] and not rok
    assert _dr(st, os_) <= 1e-4
    top = s["group"] == 2
    assert np.array_equal(st["x"][top], s["x"][top]) and not np.array_equal(st["z"][top], s["z"][top])
    for k in ("ke", "szz", "tz"):
        assert avg[0][k] == pytest.approx(ravg[k], rel=1e-4, abs=1e-5), k


def test_folded_convergence_stop_is_self_consistent():
    s = _state(5, 0.05, 300.0, 95)
    lag, n_max = 20, 400
    md = P.md_params(precision=1, lanes_per_atom=4)
    # tolerances that pass at a late checkpoint of a fixed burst's own errors
    with P.System.from_state(s, T0=300.0, md=md) as g:
        g.run_fast_md(n_max)
        ser = g.get_series(0, n_max)
    idx, errs = T.conv_errors(ser[:, [0, 1, 2, 5]], lag)
    e0 = errs[:, 1]
    q = max(j for j in range(1, len(e0)) if e0[j] < e0[:j].min())
    tol = (0.0, 0.5 * (e0[q] + e0[:q].min()), 0.0, 0.0)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        avg, ns = g.run_until_converged(P.conv_params(lag, n_max, tol))
        own = g.get_series(0, max(1, avg[0]["n_samples"]))
        st = g.get_state()
    print(f"\nfolded convergence: N_s {ns[0]} (fixed burst's errors pass from {idx[q]})")
    assert ns[0] > 0 and avg[0]["n_samples"] == ns[0]
    assert T.converged_at(own[:, [0, 1, 2, 5]], lag, tol) == ns[0]
    assert np.all(np.isfinite(st["x"]))


def test_folded_convergence_stop_with_many_blocks():
    """108,000 atoms at 16 lanes per atom, mixed (folded): the density
    launch that records the stopping sample has 6,750 blocks, more than the
    chip holds at once; every block must still take that step's lambda, so
    the stopped state matches a fixed burst of the same length."""
    md = P.md_params(precision=1, lanes_per_atom=16)
    with P.System.cube(30, T0=300.0, seed=1, md=md) as g:
        avg, ns = g.run_until_converged(P.conv_params(10, 100, (1e9, 0, 0, 0)))
        st = g.get_state()
    with P.System.cube(30, T0=300.0, seed=1, md=md) as g:
        ref = g.run_fast_md(20)[0]
        st2 = g.get_state()
    assert ns[0] == 20 and avg[0]["n_samples"] == 20
    for k in ("vx", "vy", "vz"):
        dv = np.abs(st[k] - st2[k]).max() / np.abs(st2[k]).max()
        print(f"\n{k}: {dv:.2e}")
        assert dv <= 1e-5, (k, dv)
    assert np.abs(st["z"] - st2["z"]).max() <= 1e-5
    assert avg[0]["ke"] == pytest.approx(ref["ke"], rel=1e-6)
