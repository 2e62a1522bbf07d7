"""Pins of the oracle's forces, virial, lattice, velocities, neighbour sets and
cells: finite differences of the energy, Newton's third law and rotation
invariance, the virial identity and the strain derivative, point symmetries
of the finite FCC cube, brute-force/scipy neighbour sets."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth


def _cluster(nc=3, noise=0.12, seed=5):
    s = synth.cube_state(nc, noise, 0.0, seed, fix_slabs=False)
    return s["x"], s["y"], s["z"]


@pytest.mark.parametrize("shift", [1, 2])
def test_forces_are_minus_energy_gradient(orc, shift):
    p = orc.sc_params(shift=shift)
    x, y, z = _cluster()
    f = orc.forces(x, y, z, p)
    h = 1e-5
    rs = np.random.default_rng(0)
    for i in rs.choice(len(x), 12, replace=False):
        for arr, comp in ((x, "fx"), (y, "fy"), (z, "fz")):
            a0 = arr[i]
            arr[i] = a0 + h
            up = orc.forces(x, y, z, p)["U"]
            arr[i] = a0 - h
            um = orc.forces(x, y, z, p)["U"]
            arr[i] = a0
            fd = -(up - um) / (2 * h)
            assert f[comp][i] == pytest.approx(fd, rel=2e-6, abs=2e-9)


def test_embedding_cross_term_matters(orc):
    """The B'(rho_j) term of Eq. (f_int) is essential: forces without the
    embedding (c = 0) differ from those with it by far more than rounding,
    and both match their own energy gradients (checked above for c != 0)."""
    x, y, z = _cluster()
    f1 = orc.forces(x, y, z, orc.sc_params())
    f0 = orc.forces(x, y, z, orc.sc_params(c=0.0))
    assert np.max(np.abs(f1["fx"] - f0["fx"])) > 1e-3


def test_newton_third_law_and_rotation_invariance(orc):
    p = orc.sc_params()
    x, y, z = _cluster(nc=4, noise=0.2, seed=11)
    f = orc.forces(x, y, z, p)
    F = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    r = np.stack([x, y, z], 1)
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-12 * len(x) * scale
    tq = np.cross(r - r.mean(0), F).sum(0)
    assert np.abs(tq).max() < 1e-11 * len(x) * scale * 20


def test_energy_invariant_under_rigid_motion(orc):
    p = orc.sc_params()
    x, y, z = _cluster()
    u0 = orc.forces(x, y, z, p)["U"]
    th = 0.37
    c, s = np.cos(th), np.sin(th)
    xr, yr = c * x - s * y + 3.3, s * x + c * y - 1.7
    assert orc.forces(xr, yr, z + 0.9, p)["U"] == pytest.approx(u0, rel=1e-12)


def test_virial_identity_and_strain_derivative(orc):
    p = orc.sc_params()
    x, y, z = _cluster(nc=4, noise=0.1, seed=3)
    f = orc.forces(x, y, z, p)
    # pair form equals sum_i z_i F_iz for the full (unconstrained) system
    assert f["Wzz"] == pytest.approx(np.dot(z, f["fz"]), rel=1e-9)
    # W_zz = -dU/d(eps) under z -> z (1 + eps)
    h = 1e-6
    up = orc.forces(x, y, z * (1 + h), p)["U"]
    um = orc.forces(x, y, z * (1 - h), p)["U"]
    assert f["Wzz"] == pytest.approx(-(up - um) / (2 * h), rel=1e-6)


def test_perfect_cube_symmetry(orc):
    p = orc.sc_params()
    nc = 10
    a = 4.05
    x, y, z, g, pz = orc.fcc_cube(nc, a, False)
    f = orc.forces(x, y, z, p)
    F = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    L = (nc - 0.5) * a
    inner = np.minimum.reduce([x, y, z, L - x, L - y, L - z]) >= 2 * 8.1
    assert inner.sum() > 0
    # bulk FCC sites are inversion centres: zero force
    assert np.abs(F[inner]).max() < 1e-12
    # 180-degree rotation about the central z axis maps the set to itself
    key = {(round(a_ / 2.025), round(b_ / 2.025), round(c_ / 2.025)): i for i, (a_, b_, c_) in enumerate(zip(x, y, z))}
    perm = np.array([key[(round((L - a_) / 2.025), round((L - b_) / 2.025), round(c_ / 2.025))]
                     for a_, b_, c_ in zip(x, y, z)])
    Fr = np.stack([-F[:, 0], -F[:, 1], F[:, 2]], 1)
    assert np.abs(F[perm] - Fr).max() < 1e-11
    # x <-> y exchange
    perm2 = np.array([key[(round(b_ / 2.025), round(a_ / 2.025), round(c_ / 2.025))] for a_, b_, c_ in zip(x, y, z)])
    Fs = np.stack([F[:, 1], F[:, 0], F[:, 2]], 1)
    assert np.abs(F[perm2] - Fs).max() < 1e-11
    # the surface does feel a force
    assert np.abs(F).max() > 1e-3


def test_fcc_cube_structure(orc):
    nc = 5
    x, y, z, g, pz = orc.fcc_cube(nc, 4.05, True)
    n = len(x)
    assert n == 4 * nc ** 3
    pts = np.stack([x, y, z], 1)
    t = cKDTree(pts)
    d, _ = t.query(pts, k=13)
    assert np.allclose(d[:, 1], 4.05 / np.sqrt(2), rtol=1e-12)
    # interior atoms have 12 nearest neighbours
    L = (2 * nc - 1) * 2.025
    interior = np.minimum.reduce([x, y, z, L - x, L - y, L - z]) > 3
    assert np.allclose(d[interior, 12], 4.05 / np.sqrt(2), rtol=1e-12)
    assert len(np.unique(np.round(pts / 2.025).astype(int), axis=0)) == n
    # three planes per slab, 2 nc^2 atoms per plane
    assert (g == 1).sum() == 6 * nc ** 2 and (g == 2).sum() == 6 * nc ** 2
    assert set(np.unique(pz[g == 1])) == {0, 1, 2}
    assert set(np.unique(pz[g == 2])) == {2 * nc - 3, 2 * nc - 2, 2 * nc - 1}
    assert np.array_equal(x, synth.fcc_points(nc)[0])


def test_maxwell_boltzmann_init(orc):
    nc = 8
    x, y, z, g, pz = orc.fcc_cube(nc, 4.05, True)
    vx, vy, vz = orc.mb_velocities(g, 300.0, 1)
    mob = g == 0
    c = orc.constants()
    assert np.all(vx[~mob] == 0) and np.all(vz[~mob] == 0)
    for v in (vx, vy, vz):
        assert abs(v[mob].sum()) < 1e-13 * mob.sum()
    mv2 = c["mass"] * (vx[mob] ** 2 + vy[mob] ** 2 + vz[mob] ** 2).sum()
    T = mv2 * c["mvv2e"] / ((3 * mob.sum() - 3) * c["kb"])
    assert T == pytest.approx(300.0, rel=1e-12)
    # components are normal with sigma^2 = kT/m
    sig = np.sqrt(c["kb"] * 300.0 / (c["mass"] * c["mvv2e"]))
    from scipy import stats
    assert stats.kstest(vx[mob] / sig, "norm").pvalue > 1e-3
    v2 = orc.mb_velocities(g, 300.0, 2)[0]
    assert not np.allclose(v2, vx)


def test_neighbor_sets_match_kdtree(orc):
    x, y, z = _cluster(nc=5, noise=0.15, seed=9)
    rl = 9.1
    off, idx = orc.neighbors(x, y, z, rl)
    pts = np.stack([x, y, z], 1)
    ref = cKDTree(pts).query_ball_point(pts, rl)
    for i in range(len(x)):
        mine = idx[off[i]:off[i + 1]].tolist()
        want = sorted(j for j in ref[i] if j != i)
        assert mine == want
    assert off[-1] == sum(len(r) - 1 for r in ref)


def test_cell_rule_covers_all_pairs(orc):
    """With cell edge h >= rlist every pair within rlist sits in adjacent cells,
    also when far atoms are clamped into the edge cells."""
    x, y, z = _cluster(nc=5, noise=0.15, seed=9)
    x = x.copy()
    x[:5] += 300.0  # escaped atoms, clamped into the last column
    rl = 9.1
    h = 9.5
    o = np.array([x.min(), y.min(), z.min()]) - 0.5 * h
    dims = np.array([8, 6, 6], np.int32)
    cx = orc.cell_assign(x, y, z, o, 1.0 / h, dims)
    assert cx.min() >= 0 and np.all(cx.max(0) <= dims - 1)
    off, idx = orc.neighbors(x, y, z, rl)
    for i in range(len(x)):
        for j in idx[off[i]:off[i + 1]]:
            assert np.abs(cx[i] - cx[j]).max() <= 1
    assert np.all(cx[:5, 0] == dims[0] - 1)
