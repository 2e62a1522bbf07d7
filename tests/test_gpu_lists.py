"""Forms of the Verlet lists and of the step, through the C ABI.

Lists start in the 16-bit form (each entry the offset j - i of the
neighbour in the sorted order); every other GPU test of a small system runs
on it.  A system whose offsets outgrow 16 bits switches to 32-bit indices
at the list build that meets one.  Here a film 20 A thick, whose sorted
order puts ~27,000 atoms in each of its three layers of bins (an atom of
the first layer has neighbours up to ~58,000 places on), forces that switch; its forces and
neighbour sets are checked against the oracle on sampled atoms (bars as in
the parity tests: FP64 forces 1e-9 of max(|F|, F_rms), mixed 1e-4).
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
    return synth.fcc_slab(64, 64, 5, 0.05, 61)  # 81,920 atoms, 20 A thick


@pytest.mark.parametrize("precision", [0, 1])
def test_wide_offsets_switch_to_32bit_indices(film, precision):
    O = _orc()
    s = film
    md = P.md_params(precision=precision, lanes_per_atom=4)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        f = g.compute_forces()
        info = g.info()
        off, idx = g.get_neighbors()
        a = g.run_fast_md(20)[0]
        info2 = g.info()
    print(f"\nfilm, precision {precision}: {info['list_index_bits']}-bit lists, "
          f"{info2['rollbacks']} roll-backs, {info2['list_builds']} builds")
    assert info["list_index_bits"] == 32 and info2["list_index_bits"] == 32
    n = len(s["x"])
    sample = synth.rng(62).choice(n, size=48, replace=False)
    p = O.sc_params()
    F = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    ref = np.stack([O.atom_force(s["x"], s["y"], s["z"], p, int(i)) for i in sample])
    frms = np.sqrt((ref ** 2).sum(1).mean())
    err = (np.linalg.norm(F[sample] - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), frms)).max()
    print(f"sampled forces: {err:.2e}")
    assert err <= (1e-9 if precision == 0 else 1e-4)
    rl = p.rc + info["skin"]
    for i in sample[:16]:
        d2 = (s["x"] - s["x"][i]) ** 2 + (s["y"] - s["y"][i]) ** 2 + (s["z"] - s["z"][i]) ** 2
        want = np.flatnonzero(d2 < rl * rl)
        want = want[want != i]
        assert np.array_equal(idx[off[i]:off[i + 1]], want), i
    assert np.isfinite(a["pe"]) and a["n_samples"] == 20
