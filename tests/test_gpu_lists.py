"""Forms of the Verlet lists, the order of the bins, and the step, through
the C ABI.

An atom's list is in the 16-bit form (each entry the step in the sorted
order from the same lane's previous entry, the first from the smallest
index in the atom's list) unless its listed indices span 65,535 or more;
then it holds 32-bit indices.  Bins are sorted with the axis of widest
spread slowest, so that a layer of bins holds as few atoms as the sample's
shape allows.  Checked here:
  - a 1,048,576-atom cube (64^3 cells), whose z layers of bins hold ~26,500
    atoms each, puts part of its atoms in the 32-bit form beside others in
    the 16-bit one; forces and neighbour sets against the oracle on sampled
    atoms (forces relative to max(|F|, F_rms): FP64 1e-9; mixed 2e-4, the
    parity tests' bar), and a burst on pruned lists of both forms runs;
  - a film 20 A thick and 518 A wide: its bins are ordered along a wide
    axis, so every atom keeps the 16-bit form; cells (bit-exact) and lists
    against the oracle;
  - lists too long for the staged build's LDS take the direct build.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def _orc():
    import oracle
    return oracle


@pytest.mark.parametrize("precision", [0, 1])
def test_small_systems_use_the_16bit_form(precision):
    with P.System.cube(5, T0=300.0, seed=3, md=P.md_params(precision=precision)) as g:
        g.run_fast_md(50)
        info = g.info()
    assert info["list_index_bits"] == 16
    assert info["folded"] == precision  # mixed form, 500 atoms: folded step


def test_fold_threshold():
    md = P.md_params(precision=1, lanes_per_atom=4)
    with P.System.cube(32, T0=300.0, seed=3, md=md) as g:  # 131,072 atoms
        assert g.info()["folded"] == 1
    with P.System.cube(33, T0=300.0, seed=3, md=md) as g:  # 143,748 atoms
        assert g.info()["folded"] == 0


@pytest.fixture(scope="module")
def film():
    return synth.fcc_slab(128, 128, 5, 0.05, 61)  # 327,680 atoms, 20 A thick


def _sampled_checks(s, f, off, idx, skin, precision, seed):
    O = _orc()
    n = len(s["x"])
    sample = synth.rng(seed).choice(n, size=32, replace=False)
    p = O.sc_params()
    F = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    ref = np.stack([O.atom_force(s["x"], s["y"], s["z"], p, int(i)) for i in sample])
    frms = np.sqrt((ref ** 2).sum(1).mean())
    err = (np.linalg.norm(F[sample] - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), frms)).max()
    print(f"sampled forces: {err:.2e}")
    assert err <= (1e-9 if precision == 0 else 2e-4)
    rl = p.rc + skin
    for i in sample[:12]:
        d2 = (s["x"] - s["x"][i]) ** 2 + (s["y"] - s["y"][i]) ** 2 + (s["z"] - s["z"][i]) ** 2
        want = np.flatnonzero(d2 < rl * rl)
        want = want[want != i]
        assert np.array_equal(idx[off[i]:off[i + 1]], want), i


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [0, 1])
def test_wide_atoms_use_32bit_indices(precision):
    s = synth.cube_state(64, 0.05, 0.0, 61)  # 1,048,576 atoms
    md = P.md_params(precision=precision, lanes_per_atom=4)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        f = g.compute_forces()
        info = g.info()
        off, idx = g.get_neighbors()
        cnt = g.count_pairs()
        a = g.run_fast_md(20)[0]
        cnt2 = g.count_pairs()
    n = len(s["x"])
    print(f"\ncube of {n} atoms, precision {precision}: {cnt['wide_atoms']} with 32-bit lists; after 20 steps "
          f"{cnt2['wide_atoms']}, pruned entries {cnt2['pruned_entries']}")
    assert 0 < cnt["wide_atoms"] < n and 0 < cnt2["wide_atoms"] < n
    _sampled_checks(s, f, off, idx, info["skin"], precision, 62)
    assert np.isfinite(a["pe"]) and a["n_samples"] == 20


@pytest.mark.parametrize("precision", [0, 1])
def test_film_bins_follow_its_wide_axes(film, precision):
    O = _orc()
    s = film
    md = P.md_params(precision=precision, lanes_per_atom=4)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        f = g.compute_forces()
        info = g.info()
        off, idx = g.get_neighbors()
        cnt = g.count_pairs()
        cxyz, origin, inv_h, dims = g.get_cells()
        a = g.run_fast_md(20)[0]
    print(f"\nfilm, precision {precision}: {cnt['wide_atoms']} atoms with 32-bit lists, grid {dims[0]}")
    assert cnt["wide_atoms"] == 0
    rc = O.cell_assign(s["x"], s["y"], s["z"], origin[0], inv_h[0], dims[0])
    assert np.array_equal(cxyz, rc)
    _sampled_checks(s, f, off, idx, info["skin"], precision, 63)
    assert np.isfinite(a["pe"]) and a["n_samples"] == 20


def test_neighbours_of_a_batch():
    """Three replicas: the cell scan restarts at each replica's first atom.
    Every list (16-bit form) matches the oracle's neighbour sets, replica by
    replica."""
    O = _orc()
    descs = [P.lattice_desc(8, 300.0, 21), P.lattice_desc(5, 300.0, 22), P.lattice_desc(7, 300.0, 23)]
    with P.System.batch(descs, md=P.md_params(precision=1, lanes_per_atom=4)) as b:
        b.run_fast_md(30)
        st = b.get_state()
        off, idx = b.get_neighbors()
        info = b.info()
    assert info["list_index_bits"] == 16
    a0 = 0
    for d in descs:
        n = 4 * d.n_cells ** 3
        roff, ridx = O.neighbors(st["x"][a0:a0 + n], st["y"][a0:a0 + n], st["z"][a0:a0 + n], 8.1 + info["skin"])
        assert np.array_equal(off[a0:a0 + n + 1] - off[a0], roff)
        assert np.array_equal(idx[off[a0]:off[a0 + n]], ridx + a0)
        a0 += n


def test_neighbours_over_several_scan_tiles():
    """A loose simple-cubic arrangement (8,000 atoms 6 A apart, 114 A across):
    its grid has ~5,800 bins, so the cell scan spans two 4,096-bin tiles.
    The lists match the oracle's neighbour sets."""
    O = _orc()
    x, y, z = synth.gas(20, 6.0, 31, jitter=0.3)
    n = len(x)
    zero = np.zeros(n)
    s = dict(x=x, y=y, z=z, vx=zero, vy=zero.copy(), vz=zero.copy(), group=np.zeros(n, np.uint8),
             volume0=114.0 ** 3, area0=114.0 ** 2)
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=1, lanes_per_atom=4, thermostat=0)) as g:
        off, idx = g.get_neighbors()
        cxyz, origin, inv_h, dims = g.get_cells()
        info = g.info()
    print(f"\ngrid {dims[0]}: {int(np.prod(dims[0]))} bins")
    assert int(np.prod(dims[0])) > 4096
    roff, ridx = O.neighbors(x, y, z, 8.1 + info["skin"])
    assert np.array_equal(off, roff)
    assert np.array_equal(idx, ridx)


def test_long_lists_take_the_direct_build():
    """A dense simple-cubic arrangement (1.5 A apart, up to ~930 neighbours
    per atom within rc + skin): the lists outgrow what the staged build holds
    in LDS (960 entries; overflow grows the capacity by half until they
    fit), so they are built directly, each kept entry written from the
    candidate loop.  Neighbour sets bit-exact and FP64 forces against the
    oracle."""
    O = _orc()
    x, y, z = synth.gas(14, 1.5, 41, jitter=0.05)  # 2,744 atoms, 20 A across
    n = len(x)
    zero = np.zeros(n)
    s = dict(x=x, y=y, z=z, vx=zero, vy=zero.copy(), vz=zero.copy(), group=np.zeros(n, np.uint8),
             volume0=21.0 ** 3, area0=21.0 ** 2)
    with P.System.from_state(s, T0=300.0, md=P.md_params(precision=0, lanes_per_atom=4, thermostat=0)) as g:
        f = g.compute_forces()
        off, idx = g.get_neighbors()
        info = g.info()
    print(f"\nlist capacity {info['list_capacity']}, entries per atom up to {int(np.diff(off).max())}")
    assert info["list_capacity"] > 960 and info["list_index_bits"] == 16
    roff, ridx = O.neighbors(x, y, z, 8.1 + info["skin"])
    assert np.array_equal(off, roff)
    assert np.array_equal(idx, ridx)
    ref = O.forces(x, y, z, O.sc_params(), s["group"])
    F = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
    G = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    frms = np.sqrt((F ** 2).sum(1).mean())
    err = (np.linalg.norm(G - F, axis=1) / np.maximum(np.linalg.norm(F, axis=1), frms)).max()
    assert err <= 1e-9
