"""Failure paths on the GPU, through the C ABI: each bad state is reported
with its status code by the call that meets it (no hang, no silent result),
and ptamd_set_state brings the system back to normal work afterwards.

  - thermostat at T = 0 (Berendsen's lambda needs T > 0): PTAMD_ESTATE; the
    same gas without the thermostat runs and stays at rest;
  - an atom faster than the neighbour-list bounds allow (more than 0.45 of
    the skin in one step): PTAMD_EESCAPE before any step is taken;
  - an atom leaving the region of 1e4 A around the sample's centre:
    PTAMD_EESCAPE from the kick's check;
  - two atoms at the same place (infinite forces): PTAMD_ENONFINITE.
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def _orc():
    import oracle
    return oracle


def _pair(x1, vx0=0.0, vx1=0.0):
    """Two mobile atoms on the x axis, too far apart to interact."""
    z = np.zeros(2)
    return dict(x=np.array([0.0, x1]), y=z.copy(), z=z.copy(), vx=np.array([vx0, vx1]), vy=z.copy(), vz=z.copy(),
                group=np.zeros(2, np.uint8), volume0=1000.0, area0=0.0)


def _cube(seed):
    O = _orc()
    s = synth.cube_state(4, 0.05, 0.0, seed)
    vx, vy, vz = O.mb_velocities(s["group"], 300.0, seed)
    s.update(vx=vx, vy=vy, vz=vz)
    return s


def _raises(name, fn):
    t0 = time.perf_counter()
    with pytest.raises(P.PtamdError) as ei:
        fn()
    dt = time.perf_counter() - t0
    print(f"\n{name}: {P.last_error()} ({dt:.2f} s)")
    assert ei.value.name == name
    return dt


def test_zero_temperature_with_thermostat_is_a_state_error():
    s = _pair(20.0)
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=0)) as g:
        _raises("PTAMD_ESTATE", lambda: g.run_fast_md(10))
        moving = dict(s, vx=np.array([0.002, -0.002]))
        g.set_state(moving)
        avg = g.run_fast_md(10)[0]
        assert avg["ke"] > 0.0 and np.isfinite(avg["temp"])
    # no thermostat: the gas at rest stays at rest
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=0, thermostat=0)) as g:
        avg = g.run_fast_md(10)[0]
        st = g.get_state()
    assert avg["ke"] == 0.0 and avg["pe"] == 0.0
    assert np.array_equal(st["x"], s["x"])


@pytest.mark.parametrize("precision", [0, 1])
def test_runaway_atom_is_reported_at_once(precision):
    s = _cube(81)
    fast = dict(s, vx=s["vx"].copy())
    i = int(np.flatnonzero(s["group"] == 0)[0])
    fast["vx"][i] = 5.0  # 5 A per 1 fs step
    md = P.md_params(precision=precision, lanes_per_atom=4)
    with P.System.from_state(fast, T0=300.0, md=md) as g:
        assert _raises("PTAMD_EESCAPE", lambda: g.run_fast_md(100)) < 10.0
        # back to the calm state: the burst now matches a fresh system's
        g.set_state(s)
        a = g.run_fast_md(50)[0]
    with P.System.from_state(s, T0=300.0, md=md) as h:
        b = h.run_fast_md(50)[0]
    for k in ("ke", "pe", "szz"):
        assert a[k] == pytest.approx(b[k], rel=1e-9 if precision == 0 else 1e-5), k


def test_atom_leaving_the_region_is_an_escape():
    # the centre sits midway: both atoms start 9995 A from it, the second
    # drifts outward at 0.02 A/fs and crosses 1e4 A after 250 steps
    s = _pair(19990.0, 0.0, 0.02)
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=0, thermostat=0)) as g:
        g.run_fast_md(200)
        st = g.get_state()
        assert st["x"][1] == pytest.approx(19990.0 + 200 * 0.02, abs=1e-9)
        _raises("PTAMD_EESCAPE", lambda: g.run_fast_md(200))
        g.set_state(s)
        g.run_fast_md(100)
        assert g.get_state()["x"][1] == pytest.approx(19992.0, abs=1e-9)


@pytest.mark.parametrize("precision", [0, 1])
def test_coincident_atoms_are_non_finite(precision):
    s = _cube(82)
    mob = np.flatnonzero(s["group"] == 0)
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in s.items()}
    for k in ("x", "y", "z"):
        bad[k][mob[1]] = bad[k][mob[0]]
    md = P.md_params(precision=precision, lanes_per_atom=4)
    with P.System.from_state(bad, T0=300.0, md=md) as g:
        _raises("PTAMD_ENONFINITE", lambda: g.compute_forces())
        _raises("PTAMD_ENONFINITE", lambda: g.run_fast_md(10))
        g.set_state(s)
        f = g.compute_forces()
        assert np.all(np.isfinite(f["fx"])) and np.isfinite(f["U"][0])
        avg = g.run_fast_md(20)[0]
        assert np.isfinite(avg["pe"])


def test_non_finite_input_rejected():
    s = _cube(83)
    for k in ("x", "vz"):
        bad = dict(s)
        bad[k] = s[k].copy()
        bad[k][5] = np.nan
        with pytest.raises(P.PtamdError) as ei:
            P.System.from_state(bad, T0=300.0)
        assert ei.value.name == "PTAMD_EINVAL"
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=0)) as g:
        bad = dict(s, y=s["y"].copy())
        bad["y"][3] = np.inf
        with pytest.raises(P.PtamdError) as ei:
            g.set_state(bad)
        assert ei.value.name == "PTAMD_EINVAL"
        g.run_fast_md(10)
