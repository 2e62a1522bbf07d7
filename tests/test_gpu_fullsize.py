"""Full-size checks of the batched workloads and the autotuner (every-atom
force checks at the benchmark's sizes are in test_gpu_benchmarked.py):
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
    assert choice["lanes_per_atom"] in (2, 4, 8, 16) and choice["skin"] in (1.0, 1.5, 2.0, 2.5)
    assert choice["prune_every"] in (0, 1, 2, 3) and info["prune_every"] == choice["prune_every"]
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
