"""Pins of the oracle's further observables: the per-atom mean positions of
Eq. (mean_pos) and the thermal relaxation of Sec. 2.4.2 (top region free
along z).

  - free flight (no interactions, no thermostat): x(sigma_r) = x0 + r dt v,
    so the mean over r = 1..N is x0 + dt v (N+1)/2;
  - held atoms' mean position is their position (to rounding);
  - with the top region free along z, NVE still conserves K + U with the
    O(dt^2) error of velocity Verlet (K includes the top atoms' z motion);
  - a top atom at rest moves in one step by dt^2 F^int_z / (2m) along z
    (F^int from the single-atom force routine), and not at all along x, y;
  - the reported temperature uses 3 N_mob - 3 + N_top degrees of freedom.
"""
import numpy as np
import pytest

import synth


def _gas_state(orc, n_side, T, seed, top_every=0):
    x, y, z = synth.gas(n_side, 20.0, seed)
    g = np.zeros(len(x), np.uint8)
    if top_every:
        g[::top_every] = 2
    vx, vy, vz = orc.mb_velocities(np.zeros(len(x), np.uint8), T, seed)
    top = g == 2
    vx[top] = 0.0
    vy[top] = 0.0
    return orc.State(x, y, z, vx, vy, vz, g, 1e6, 1e3)


def test_mean_positions_free_flight(orc):
    st = _gas_state(orc, 5, 300.0, 3)
    x0, y0, z0 = st.x.copy(), st.y.copy(), st.z.copy()
    v = np.stack([st.vx, st.vy, st.vz])
    N = 250
    _, _, mean = orc.run_burst(st, orc.sc_params(), orc.md_params(thermostat=0), N, mean_positions=True)
    want = np.stack([x0, y0, z0]) + 1.0 * v * (N + 1) / 2.0
    assert np.abs(mean - want).max() < 1e-11


def test_mean_positions_of_held_atoms(orc):
    s = synth.cube_state(4, 0.05, 0.0, 5)
    vx, vy, vz = orc.mb_velocities(s["group"], 300.0, 5)
    st = orc.State(s["x"], s["y"], s["z"], vx, vy, vz, s["group"], s["volume0"], s["area0"])
    pos0 = np.stack([st.x.copy(), st.y.copy(), st.z.copy()])
    _, _, mean = orc.run_burst(st, orc.sc_params(), orc.md_params(), 30, mean_positions=True)
    held = st.group != 0
    # N additions of the same value, divided by N: equal to rounding
    assert np.allclose(mean[:, held], pos0[:, held], rtol=1e-14, atol=1e-14)
    assert not np.allclose(mean[:, ~held], pos0[:, ~held])


def _slab_state(orc, T=100.0, seed=8):
    s = synth.cube_state(5, 0.05, 0.0, seed)
    vx, vy, vz = orc.mb_velocities(s["group"], T, seed)
    return orc.State(s["x"], s["y"], s["z"], vx, vy, vz, s["group"], s["volume0"], s["area0"])


def test_relaxation_energy_conservation(orc):
    p = orc.sc_params()
    st0 = _slab_state(orc)
    dev = []
    for dt in (1.0, 0.5):
        st = st0.copy()
        n = int(round(150 / dt))
        md = orc.md_params(dt=dt, thermostat=0, top_free_z=1)
        _, ser = orc.run_burst(st, p, md, n, series=True)
        e0 = orc.observables(st0, p)
        E = ser[:, 0] + ser[:, 1]
        dev.append(np.abs(E - (e0["K"] + e0["U"])).max())
        top = st.group == 2
        assert np.array_equal(st.x[top], st0.x[top]) and np.array_equal(st.y[top], st0.y[top])
        assert not np.array_equal(st.z[top], st0.z[top])
        bot = st.group == 1
        assert np.array_equal(st.z[bot], st0.z[bot])
    assert dev[0] / st0.n < 2e-5
    assert 2.5 < dev[0] / dev[1] < 6.0


def test_relaxation_first_step_of_a_top_atom(orc):
    p = orc.sc_params()
    st = _slab_state(orc, T=0.0)
    st.vx[:] = 0.0
    st.vy[:] = 0.0
    st.vz[:] = 0.0
    i = int(np.where(st.group == 2)[0][3])
    f = orc.atom_force(st.x, st.y, st.z, p, i)
    z0, x0 = st.z[i], st.x[i]
    orc.run_burst(st, p, orc.md_params(thermostat=0, top_free_z=1), 1)
    k = orc.constants()
    dz = 0.5 * f[2] / (k["mass"] * k["mvv2e"])  # dt = 1 fs
    # z is ~14 A: the difference carries the rounding of z (ulp ~2e-15)
    assert st.z[i] - z0 == pytest.approx(dz, rel=0, abs=1e-14)
    assert abs(dz) > 1e-8
    assert st.x[i] == x0


def test_relaxation_degrees_of_freedom(orc):
    st = _gas_state(orc, 4, 300.0, 11, top_every=5)
    n_top = int((st.group == 2).sum())
    n_mob = int((st.group == 0).sum())
    _, ser = orc.run_burst(st, orc.sc_params(), orc.md_params(thermostat=0, top_free_z=1), 1, series=True)
    k = orc.constants()
    mv2 = k["mass"] * k["mvv2e"] * (st.vx ** 2 + st.vy ** 2 + st.vz ** 2).sum()
    T = mv2 / ((3 * n_mob - 3 + n_top) * k["kb"])
    assert ser[0, 3] == pytest.approx(T, rel=1e-12)


def test_relax_holds_top_region_afterwards(orc):
    st = _slab_state(orc, T=300.0)
    avg, k, ok = orc.relax(st, orc.sc_params(), orc.md_params(), 20, 2, 0.0)
    top = st.group == 2
    assert k == 2 and not ok
    assert np.all(st.vx[top] == 0) and np.all(st.vy[top] == 0) and np.all(st.vz[top] == 0)
