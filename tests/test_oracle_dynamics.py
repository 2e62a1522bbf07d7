"""Pins of the oracle's time stepping: energy conservation and its second-order
dt scaling (velocity Verlet), time reversibility, the Berendsen closed form in
a non-interacting gas, fixed boundary regions, momentum, strain steps, and the
definition of the burst average (samples r = 1..N_t)."""
import numpy as np
import pytest

import synth


def _state(orc, nc=4, noise=0.05, T=300.0, seed=4, fix=False):
    s = synth.cube_state(nc, noise, 0.0, seed, fix_slabs=fix)
    g = s["group"]
    vx, vy, vz = orc.mb_velocities(g, T, seed)
    return orc.State(s["x"], s["y"], s["z"], vx, vy, vz, g, s["volume0"], s["area0"])


def _total_energy_series(orc, st, p, dt, nsteps):
    md = orc.md_params(dt=dt, thermostat=0)
    _, ser = orc.run_burst(st, p, md, nsteps, series=True)
    return ser[:, 0] + ser[:, 1]


def test_nve_energy_conservation_second_order(orc):
    p = orc.sc_params()
    st0 = _state(orc, T=100.0)
    e0 = orc.observables(st0, p)
    E0 = e0["K"] + e0["U"]
    dev = []
    for dt in (1.0, 0.5):
        st = st0.copy()
        n = int(round(200 / dt))
        E = _total_energy_series(orc, st, p, dt, n)
        dev.append(np.abs(E - E0).max())
    # bounded fluctuation at dt = 1 fs, and the O(dt^2) scaling of Verlet
    assert dev[0] / st0.n < 2e-5
    assert 2.5 < dev[0] / dev[1] < 6.0


def test_time_reversibility(orc):
    p = orc.sc_params()
    st = _state(orc, T=300.0, fix=True)
    x0, y0, z0 = st.x.copy(), st.y.copy(), st.z.copy()
    md = orc.md_params(thermostat=0)
    orc.run_burst(st, p, md, 60)
    st.vx, st.vy, st.vz = -st.vx, -st.vy, -st.vz
    orc.run_burst(st, p, md, 60)
    assert np.abs(st.x - x0).max() < 1e-9
    assert np.abs(st.z - z0).max() < 1e-9


def test_berendsen_closed_form_in_gas(orc):
    """No forces (spacing 20 A, far beyond rc + any drift): lambda^2 T = T + (dt/tau)(T0 - T), so
    T_n - T0 = (1 - dt/tau)^n (T_init - T0) exactly."""
    x, y, z = synth.gas(6, 20.0, 1)
    n = len(x)
    g = np.zeros(n, np.uint8)
    vx, vy, vz = orc.mb_velocities(g, 450.0, 3)
    st = orc.State(x, y, z, vx, vy, vz, g, volume0=1e6)
    md = orc.md_params(T0=300.0, tau=100.0, thermostat=1)
    avg, ser = orc.run_burst(st, orc.sc_params(), md, 300, series=True)
    k = np.arange(1, 301)
    want = 300.0 + (1 - 1.0 / 100.0) ** k * (450.0 - 300.0)
    assert np.allclose(ser[:, 3], want, rtol=1e-11)
    assert np.all(ser[:, 1] == 0.0)


def test_fixed_regions_do_not_move_and_momentum(orc):
    p = orc.sc_params()
    st = _state(orc, nc=5, T=300.0, fix=True)
    fixed = st.group != 0
    x0, z0 = st.x.copy(), st.z.copy()
    orc.run_burst(st, p, orc.md_params(), 50)
    assert np.array_equal(st.x[fixed], x0[fixed]) and np.array_equal(st.z[fixed], z0[fixed])
    assert np.all(st.vx[fixed] == 0.0)
    assert np.abs(st.x[~fixed] - x0[~fixed]).max() > 1e-3
    # free cluster, zero initial momentum: stays zero (NVE and Berendsen)
    for thermo in (0, 1):
        sf = _state(orc, nc=3, T=300.0, fix=False)
        orc.run_burst(sf, p, orc.md_params(thermostat=thermo), 80)
        m = orc.constants()["mass"]
        for v in (sf.vx, sf.vy, sf.vz):
            assert abs(m * v.sum()) < 1e-12


def test_burst_average_definition(orc):
    """The average runs over the post-step samples r = 1..N (Eq. (R_m_t)):
    the first sample equals the observables after one step."""
    p = orc.sc_params()
    st = _state(orc, nc=4, T=300.0, fix=True)
    one = st.copy()
    orc.run_burst(one, p, orc.md_params(thermostat=0), 1)
    obs = orc.observables(one, p)
    avg, ser = orc.run_burst(st.copy(), p, orc.md_params(thermostat=0), 40, series=True)
    assert ser[0, 0] == pytest.approx(obs["K"], rel=1e-12)
    assert ser[0, 1] == pytest.approx(obs["U"], rel=1e-12)
    assert ser[0, 2] == pytest.approx(obs["szz"], rel=1e-9, abs=1e-12)
    assert avg["ke"] == pytest.approx(ser[:, 0].mean(), rel=1e-12)
    assert avg["szz"] == pytest.approx(ser[:, 2].mean(), rel=1e-12, abs=1e-14)
    # 20 blocks of 2 samples
    b = ser[:, 1].reshape(20, 2).mean(1)
    assert avg["pe_se"] == pytest.approx(np.sqrt(((b - b.mean()) ** 2).sum() / (20 * 19)), rel=1e-9)


def test_kinetic_stress_of_ideal_gas(orc):
    """With no forces, sigma_zz = -sum m v_z^2 / V: on average the ideal-gas
    pressure -N k T / V (sign: compression negative)."""
    x, y, z = synth.gas(8, 12.0, 1)
    g = np.zeros(len(x), np.uint8)
    vx, vy, vz = orc.mb_velocities(g, 300.0, 5)
    V = 1e6
    st = orc.State(x, y, z, vx, vy, vz, g, volume0=V)
    obs = orc.observables(st, orc.sc_params())
    c = orc.constants()
    want = -c["mass"] * (vz ** 2).sum() * c["mvv2e"] / V * c["gpa"]
    assert obs["szz"] == pytest.approx(want, rel=1e-12)
    ideal = -len(x) * c["kb"] * 300.0 / V * c["gpa"]
    assert obs["szz"] == pytest.approx(ideal, rel=0.15)


def test_strain_steps(orc):
    st = _state(orc, nc=4)
    z0 = st.z.copy()
    orc.apply_strain(st, 1e-4)
    orc.apply_strain(st, 1e-4)
    assert st.strain == pytest.approx(2e-4, rel=1e-12)
    assert np.allclose(st.z, z0 * (1 + 2e-4), rtol=1e-14, atol=0)
    orc.apply_strain(st, -2e-4)
    assert np.allclose(st.z, z0, rtol=1e-14, atol=1e-14)
    # tension makes the perfect cube's virial stress more tensile
    p = orc.sc_params()
    x, y, z, g, _ = orc.fcc_cube(6, 4.05, True)
    s0 = orc.State(x, y, z, 0 * x, 0 * x, 0 * x, g, 6.0 ** 3 * 4.05 ** 3, (6 * 4.05) ** 2)
    a = orc.observables(s0, p)["szz"]
    orc.apply_strain(s0, 1e-3)
    b = orc.observables(s0, p)["szz"]
    assert b > a > 0
