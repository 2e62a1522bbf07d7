"""Convergence-terminated bursts and the PTA slow-time driver on the GPU,
through the C ABI, against the FP64 oracle (oracle/pta.py) on the same seeded
inputs.

Bars:
  - N_s (the step at which the running averages pass the test of App. A) is
    an integer decided in FP64 on both sides: equal, for tolerances chosen
    (from the oracle's own error sequence) at least 1e-6 relative away from
    every error value the decision compares;
  - FP64 averages of runs up to a few hundred steps: relative 1e-9 (chaotic
    growth of rounding differences stays far below that at these lengths);
    batch-means standard errors relative 1e-6; final positions 1e-7 A;
  - PTA records: strains bit-exact (the same FP64 increments on both sides),
    R, v_pred, v_d, v relative 1e-8, statuses equal where the oracle's e_v
    and jump errors sit at least 1e-6 relative away from their tolerances;
  - batched replicas that stop at different N_s: each equals its own
    individual run (N_s exactly, averages and frozen state to rounding).
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


def _samples(ser):
    return ser[:, [0, 1, 2, 5]]


def _tolerances(errs, tested):
    """Tolerances from the oracle's own error sequence that make the test
    pass at a late checkpoint q (the last new minimum of the first tested
    function's error), each tolerance halfway between the error values the
    decisions compare, so no decision is near a tie."""
    e0 = errs[:, tested[0]]
    q = 0
    for j in range(1, len(e0)):
        if e0[j] < e0[:j].min():
            q = j
    tol = np.zeros(4)
    tol[tested[0]] = 0.5 * (e0[q] + e0[:q].min()) if q > 0 else 1.5 * e0[0]
    for f in tested[1:]:
        tol[f] = 1.5 * errs[:q + 1, f].max()  # always passes up to q
    return tol, q


# the third case tests T_z with an absolute floor on the error's denominator:
# its running average passes through zero in these short runs; the fourth
# uses a 0.3 A skin, so that the device-side list rebuilds fire often while
# the convergence test runs
@pytest.mark.parametrize("lag,n_max,tested,seed,floor,skin", [(20, 300, (0, 1), 31, 0.0, 1.0),
                                                              (25, 250, (0,), 32, 0.0, 1.0),
                                                              (10, 150, (0, 3), 35, 1.0, 1.0),
                                                              (20, 300, (0, 1), 31, 0.0, 0.3)])
def test_run_until_converged_matches_oracle(lag, n_max, tested, seed, floor, skin):
    O = _orc()
    s = _state(5, 0.05, 300.0, seed)
    fl = (0.0, 0.0, 0.0, floor)
    # the oracle's errors over a full n_max run pick the tolerances
    probe = _orc_state(s)
    _, ser = O.run_burst(probe, O.sc_params(), O.md_params(), n_max, series=True)
    idx, errs = T.conv_errors(_samples(ser), lag, fl)
    tol, q = _tolerances(errs, list(tested))
    assert q > 0 and T.converged_at(_samples(ser), lag, tuple(tol), fl) == idx[q]
    conv = P.conv_params(lag, n_max, tuple(tol), fl)
    os_ = _orc_state(s)
    R, ns_o, rser = T.run_until_converged(os_, O.sc_params(), O.md_params(), lag, n_max, tuple(tol), fl)
    md = P.md_params(precision=0, lanes_per_atom=4, skin=skin)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        avg, ns = g.run_until_converged(conv)
        st = g.get_state()
        gser = g.get_series(0, max(1, avg[0]["n_samples"]))
    a = avg[0]
    print(f"\nlag {lag} n_max {n_max} tested {tested}: N_s oracle {ns_o} gpu {ns[0]}, samples {a['n_samples']}")
    assert ns[0] == ns_o
    assert a["n_samples"] == (ns_o if ns_o else n_max) == len(rser)
    for k in ("ke", "pe", "szz", "tz"):
        ref = R[{"ke": "K", "pe": "U", "szz": "szz", "tz": "tz"}[k]]
        assert a[k] == pytest.approx(ref, rel=1e-9, abs=1e-9), k
    for k in ("ke_se", "pe_se", "szz_se"):
        if np.isnan(R[k]):
            assert np.isnan(a[k])
        else:
            assert a[k] == pytest.approx(R[k], rel=1e-6, abs=1e-12), k
    assert np.allclose(gser[:, :3], rser[:, :3], rtol=1e-9, atol=1e-9)
    dr = max(np.abs(st[k] - getattr(os_, k)).max() for k in ("x", "y", "z"))
    assert dr <= 1e-7


def test_converges_at_first_check_and_stops_at_n_max():
    with P.System.cube(5, md=P.md_params(precision=0)) as g:
        avg, ns = g.run_until_converged(P.conv_params(10, 100, (1e9, 0, 0, 0)))
        assert ns[0] == 20 and avg[0]["n_samples"] == 20
        avg, ns = g.run_until_converged(P.conv_params(10, 95, (1e-30, 0, 0, 0)))
        assert ns[0] == 0 and avg[0]["n_samples"] == 95
        info = g.info()
        # a fixed-length burst afterwards is unaffected by the previous mode
        a = g.run_fast_md(40)[0]
        assert a["n_samples"] == 40 and np.isfinite(a["ke_se"])
    assert info["steps"] >= 115


def test_invalid_convergence_arguments():
    with P.System.cube(4, md=P.md_params(precision=0)) as g:
        for conv in (P.conv_params(0, 100), P.conv_params(10, 15), P.conv_params(10, 100, (0, 0, 0, 0)),
                     P.conv_params(10, 100, (0.05, 0, 0, 0), (-1.0, 0, 0, 0))):
            with pytest.raises(P.PtamdError) as ei:
                g.run_until_converged(conv)
            assert ei.value.name == "PTAMD_EINVAL"


def test_batch_replicas_stop_independently():
    """Replicas of one batch stop at their own N_s: each equals its own
    individual run, and a stopped replica stays frozen while the others run."""
    descs = [P.lattice_desc(4, 100.0, 7), P.lattice_desc(6, 300.0, 8), P.lattice_desc(5, 600.0, 9)]
    md = P.md_params(precision=0, lanes_per_atom=4)
    conv = P.conv_params(20, 400, (0.004, 0, 0, 0))
    singles = []
    for d in descs:
        with P.System(P.create_system(d, P.sc_params(), md)) as s:
            a, n = s.run_until_converged(conv)
            singles.append((a[0], int(n[0]), s.get_state()))
    with P.System.batch(descs, md=md) as b:
        avg, ns = b.run_until_converged(conv)
        st = b.get_state()
    print("\nN_s per replica:", list(ns), "individually:", [x[1] for x in singles])
    off = 0
    for r, (a, n, s1) in enumerate(singles):
        assert ns[r] == n
        for k in ("ke", "pe", "szz", "tz"):
            assert avg[r][k] == pytest.approx(a[k], rel=1e-9, abs=1e-9)
        m = len(s1["x"])
        for k in s1:
            assert np.abs(st[k][off:off + m] - s1[k]).max() <= 1e-8
        off += m


def _pta_tol_ok(rec_o, prm):
    """Status positions whose decision has a margin of 1e-6 (relative)."""
    ok = np.ones(4, bool)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.abs(rec_o.e1 / rec_o.e2 - 1.0)
    for f in range(4):
        for val, tol in ((rec_o.e_v[f], prm.tol_v[f]), (rec_o.e1[f], prm.tol_j[f]), (ratio[f], prm.tol_j[f])):
            if np.isfinite(val) and tol > 0 and abs(val / tol - 1.0) < 1e-6:
                ok[f] = False
    return ok


def test_pta_driver_matches_oracle():
    O = _orc()
    s = _state(5, 0.05, 300.0, 41)
    lag, n_max = 20, 100
    tol_m = (0.01, 0.05, 0.0, 0.0)
    prm_o = T.PTAParams(d_eps_h=2e-3, delta_over_h=0.2, tol_v=(0.01, 0.05, 0.01, 0.01),
                        tol_j=(0.08, 0.01, 0.05, 0.05))
    prm_c = P.pta_params(2e-3, 0.2, P.conv_params(lag, n_max, tol_m), tol_v=prm_o.tol_v, tol_j=prm_o.tol_j)
    os_ = _orc_state(s)
    meas = T.md_measure(os_, O.sc_params(), O.md_params(), lag, n_max, tol_m)
    st_o, rec0_o = T.pta_start(meas, prm_o)
    recs_o = [T.pta_jump(meas, st_o, prm_o) for _ in range(2)]
    md = P.md_params(precision=0, lanes_per_atom=4)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        st_c, rec0_c = g.pta_start(prm_c)
        recs_c = [g.pta_jump(prm_c, st_c)[0] for _ in range(2)]
        strain = g.strain()[0]
    rec0_c = rec0_c[0]
    assert np.array_equal(np.array(rec0_o.strains), rec0_c["strain"])
    assert list(rec0_o.n_steps) == list(rec0_c["n_steps"])
    assert np.allclose(rec0_o.R, rec0_c["R"], rtol=1e-8, atol=1e-9)
    assert np.allclose(rec0_o.v, rec0_c["v"], rtol=1e-8, atol=1e-9)
    assert np.all(rec0_c["status"] == -1)
    for j, (ro, rc) in enumerate(zip(recs_o, recs_c)):
        print(f"\njump {j}: strains {rc['strain']}, N_s {list(rc['n_steps'])}, status {list(rc['status'])}, "
              f"e_v {rc['e_v']}")
        assert np.array_equal(np.array(ro.strains), rc["strain"])
        assert list(ro.n_steps) == list(rc["n_steps"])
        assert np.allclose(ro.R, rc["R"], rtol=1e-8, atol=1e-9)
        for k in ("v_pred", "v_d", "v"):
            assert np.allclose(getattr(ro, k), rc[k], rtol=1e-8, atol=1e-9), k
        ok = _pta_tol_ok(ro, prm_o)
        assert np.array_equal(ro.status[ok], rc["status"][ok])
    assert strain == st_c[0].strain == recs_c[-1]["strain"][2]
    assert st_c[0].n_jumps == 2
