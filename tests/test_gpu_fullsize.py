"""Full-size checks in the launch configuration the benchmark times.

At the workloads' real sizes the oracle cannot run whole bursts, so:
  - forces of sampled atoms are recomputed one by one by the oracle
    (O(N * nbar) each) from the GPU's state, and compared to the mixed-form
    bar: |dF| <= 2e-4 max(|F|, F_rms), F_rms from the GPU forces;
  - properties that hold at any size: internal forces sum to zero (Newton's
    third law over the whole system);
  - batched replicas against individual runs: mixed batch vs FP64 runs of the
    same replicas, burst averages within three combined block standard errors
    (plus a small absolute floor);
  - the autotuner leaves the state exactly as it found it.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def _orc():
    import oracle
    return oracle


def _sample_atoms(st, group, k, seed):
    """Atoms spread over the cube: interior, surface, both fixed regions."""
    rng = np.random.default_rng(seed)
    n = len(st["x"])
    idx = set(rng.choice(n, k, replace=False).tolist())
    idx.add(int(np.argmin(st["x"])))            # a surface atom
    idx.update(np.where(group == 1)[0][:1].tolist())
    idx.update(np.where(group == 2)[0][-1:].tolist())
    return sorted(idx)


@pytest.mark.parametrize("nc,precision,lanes,steps", [(25, 1, 4, 60), (25, 1, 8, 60), (25, 0, 4, 30)])
def test_cube25_sampled_forces(nc, precision, lanes, steps):
    O = _orc()
    md = P.md_params(precision=precision, lanes_per_atom=lanes)
    with P.System.cube(nc, T0=300.0, seed=1, md=md) as g:
        g.apply_strain_increment(1e-4)
        g.run_fast_md(steps)
        st = g.get_state()
        f = g.compute_forces()
    _, _, _, group, _ = O.fcc_cube(nc, 4.05, True)
    G = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    frms = np.sqrt((G ** 2).sum(1).mean())
    # Newton's third law over the whole (unconstrained) internal force field
    assert np.abs(G.sum(0)).max() < (1e-3 if precision else 1e-9) * frms * np.sqrt(len(G))
    bar = 2e-4 if precision else 1e-5
    worst = 0.0
    for i in _sample_atoms(st, group, 10, 7):
        ref = O.atom_force(st["x"], st["y"], st["z"], O.sc_params(), i)
        err = np.linalg.norm(G[i] - ref) / max(np.linalg.norm(ref), frms)
        worst = max(worst, err)
    print(f"\nN={len(G)} precision={precision} lanes={lanes}: worst sampled force error {worst:.2e}")
    assert worst <= bar


def test_cube50_sampled_forces():
    """500,000-atom cube (the compression workload's size), mixed form."""
    O = _orc()
    md = P.md_params(precision=1, lanes_per_atom=2)
    with P.System.cube(50, T0=300.0, seed=1, md=md) as g:
        g.apply_strain_increment(-1e-4)
        g.run_fast_md(20)
        st = g.get_state()
        f = g.compute_forces()
    _, _, _, group, _ = O.fcc_cube(50, 4.05, True)
    G = np.stack([f["fx"], f["fy"], f["fz"]], 1)
    frms = np.sqrt((G ** 2).sum(1).mean())
    worst = 0.0
    for i in _sample_atoms(st, group, 3, 11):
        ref = O.atom_force(st["x"], st["y"], st["z"], O.sc_params(), i)
        worst = max(worst, np.linalg.norm(G[i] - ref) / max(np.linalg.norm(ref), frms))
    print(f"\nN=500000 mixed: worst sampled force error {worst:.2e}")
    assert worst <= 2e-4


def test_uneven_mixed_batch_against_individual_fp64():
    edges, d_eps = [10, 15, 12], [1e-4, -1e-4, 1e-4]
    descs = [P.lattice_desc(e, 300.0, 100 + k) for k, e in enumerate(edges)]
    with P.System.batch(descs, md=P.md_params(precision=1)) as b:
        b.apply_strain_increments(d_eps)
        avg_b = b.run_fast_md(1000)
    for k, d in enumerate(descs):
        with P.System(P.create_system(d, P.sc_params(), P.md_params(precision=0))) as s:
            s.apply_strain_increment(d_eps[k])
            a = s.run_fast_md(1000)[0]
        for key, se in (("ke", "ke_se"), ("pe", "pe_se"), ("szz", "szz_se")):
            tol = 3.0 * np.hypot(a[se], avg_b[k][se]) + 1e-6 * abs(a[key]) + 1e-9
            print(f"replica {k} {key}: batch {avg_b[k][key]:.6g} fp64 {a[key]:.6g} tol {tol:.2e}")
            assert abs(a[key] - avg_b[k][key]) <= tol


def test_ensemble_temperatures_follow_targets():
    """Replicas at different targets: each burst's mean temperature tracks its
    own T0 (Berendsen), so replica data never mix."""
    temps = [100.0, 250.0, 500.0]
    descs = [P.lattice_desc(8, t, 10 + k) for k, t in enumerate(temps)]
    with P.System.batch(descs, md=P.md_params(precision=1)) as b:
        avg = b.run_fast_md(400)
    for t, a in zip(temps, avg):
        assert abs(a["temp"] - t) < 0.3 * t
    assert avg[0]["temp"] < avg[1]["temp"] < avg[2]["temp"]


def test_autotune_restores_state():
    with P.System.cube(12, md=P.md_params(precision=1)) as g:
        g.run_fast_md(20)
        st0 = g.get_state()
        choice = g.autotune(probe_steps=20, use_cache=False)
        st1 = g.get_state()
        info = g.info()
    assert choice["lanes_per_atom"] in (2, 4, 8, 16) and choice["skin"] in (0.6, 0.8, 1.0, 1.5)
    assert info["lanes_per_atom"] == choice["lanes_per_atom"]
    for k in st0:
        assert np.array_equal(st0[k], st1[k])


def test_convergence_stop_with_more_blocks_than_resident():
    """500,000 atoms: the kick launch has more blocks than the chip holds at
    once, so blocks start after the first block has recorded the stopping
    sample.  Every block must still take that step's lambda: the stopped
    state equals a fixed burst of the same length (FP64, to rounding)."""
    md = P.md_params(precision=0, lanes_per_atom=2)
    with P.System.cube(50, T0=300.0, seed=1, md=md) as g:
        avg, ns = g.run_until_converged(P.conv_params(10, 100, (1e9, 0, 0, 0)))
        st = g.get_state()
    with P.System.cube(50, T0=300.0, seed=1, md=md) as g:
        ref = g.run_fast_md(20)[0]
        st2 = g.get_state()
    assert ns[0] == 20 and avg[0]["n_samples"] == 20
    for k in ("vx", "vy", "vz"):
        dv = np.abs(st[k] - st2[k]).max() / np.abs(st2[k]).max()
        assert dv <= 1e-9, (k, dv)
    assert np.abs(st["z"] - st2["z"]).max() <= 1e-9
    assert avg[0]["ke"] == pytest.approx(ref["ke"], rel=1e-10)
