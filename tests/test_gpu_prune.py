"""Pruned Verlet lists (ptamd_md_params::full_lists = 0, the default).

Every fourth step the density pass walks the full Verlet lists (radius
rc + skin) and keeps, per atom, the entries within rin = rc + 2 (m - 1) dt vs
of it, where vs bounds every atom's speed over the chunk (each kick checks
it); the pair passes in between read those.  Every pair term still tests
r < rc, so the pruned and the full lists give the same results up to the
order of summation, and both match the oracle at the parity bars.  Checked
here:
  - FP64: pruned against full lists and against the oracle over 100 steps
    (|dr| <= 1e-8 A, |dv| <= 1e-10 A/fs) and 400 steps (to rounding), with a
    pruning pass every 4, 8 or 12 steps;
  - mixed, folded step: pruned against full lists (FP32 rounding);
  - the pruned lists hold every pair within rc at the positions where they
    are read: their size lies between the directed pairs within rc and the
    full lists, and their radius between rc and rc + skin;
  - a hot system (900 K) whose chunks use rebuild points every step runs
    on full lists and still matches.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def _orc():
    import oracle
    return oracle


def _state(nc, noise, T, seed):
    O = _orc()
    s = synth.cube_state(nc, noise, 0.0, seed)
    vx, vy, vz = O.mb_velocities(s["group"], T, seed)
    s.update(vx=vx, vy=vy, vz=vz)
    return s


def _run(s, n, precision, full, lanes=4, T0=300.0, prune_every=0):
    md = P.md_params(precision=precision, lanes_per_atom=lanes, full_lists=full, prune_every=prune_every)
    with P.System.from_state(s, T0=T0, md=md) as g:
        avg = g.run_fast_md(n)[0]
        st = g.get_state()
        cnt = g.count_pairs()
        info = g.info()
    return avg, st, cnt, info


@pytest.mark.parametrize("lanes", [2, 4, 16])
def test_fp64_pruned_matches_full_and_oracle(lanes):
    O = _orc()
    s = _state(6, 0.05, 300.0, 51)
    a_p, st_p, cnt, info = _run(s, 100, 0, 0, lanes)
    a_f, st_f, cnt_f, _ = _run(s, 100, 0, 1, lanes)
    os_ = O.State(*(s[k].copy() for k in ("x", "y", "z", "vx", "vy", "vz", "group")), s["volume0"], s["area0"])
    ravg, _ = O.run_burst(os_, O.sc_params(), O.md_params(), 100)
    for st in (st_p, st_f):
        dr = max(np.abs(st[k] - getattr(os_, k)).max() for k in ("x", "y", "z"))
        dv = max(np.abs(st[k] - getattr(os_, k)).max() for k in ("vx", "vy", "vz"))
        assert dr <= 1e-8 and dv <= 1e-10
    for k in ("ke", "pe", "szz", "tz"):
        assert a_p[k] == pytest.approx(ravg[k], rel=1e-9, abs=1e-9), k
        assert a_p[k] == pytest.approx(a_f[k], rel=1e-11, abs=1e-11), k
    rc = 8.1
    print(f"\nlanes {lanes}: pairs {cnt['pairs_in_rc']}, full entries {cnt['list_entries']}, "
          f"pruned {cnt['pruned_entries']} within {cnt['prune_radius']:.4f} A")
    assert rc < cnt["prune_radius"] < rc + info["skin"]
    assert 2 * cnt["pairs_in_rc"] <= cnt["pruned_entries"] < cnt["list_entries"]
    assert cnt_f["pruned_entries"] == 0 and cnt_f["prune_radius"] == 0.0


@pytest.mark.parametrize("prune_every", [2, 3])
def test_fp64_longer_pruning_intervals(prune_every):
    O = _orc()
    s = _state(6, 0.05, 300.0, 55)
    a_p, st_p, cnt, info = _run(s, 100, 0, 0, prune_every=prune_every)
    assert info["prune_every"] == prune_every
    os_ = O.State(*(s[k].copy() for k in ("x", "y", "z", "vx", "vy", "vz", "group")), s["volume0"], s["area0"])
    ravg, _ = O.run_burst(os_, O.sc_params(), O.md_params(), 100)
    dr = max(np.abs(st_p[k] - getattr(os_, k)).max() for k in ("x", "y", "z"))
    dv = max(np.abs(st_p[k] - getattr(os_, k)).max() for k in ("vx", "vy", "vz"))
    print(f"\nprune every {4 * prune_every} steps: radius {cnt['prune_radius']:.4f} A, pruned {cnt['pruned_entries']}, "
          f"|dr| {dr:.2e}")
    assert dr <= 1e-8 and dv <= 1e-10
    for k in ("ke", "pe", "szz", "tz"):
        assert a_p[k] == pytest.approx(ravg[k], rel=1e-9, abs=1e-9), k
    assert 8.1 < cnt["prune_radius"] < 8.1 + info["skin"]


def test_fp64_pruned_long_run_to_rounding():
    s = _state(7, 0.1, 300.0, 52)
    a_p, st_p, _, _ = _run(s, 400, 0, 0)
    a_f, st_f, _, _ = _run(s, 400, 0, 1)
    dr = max(np.abs(st_p[k] - st_f[k]).max() for k in ("x", "y", "z"))
    print(f"\n400 FP64 steps, pruned vs full lists: |dr| {dr:.2e}")
    assert dr <= 1e-9
    for k in ("ke", "pe", "szz"):
        assert a_p[k] == pytest.approx(a_f[k], rel=1e-10, abs=1e-10), k


def test_mixed_folded_pruned_matches_full():
    s = _state(8, 0.05, 300.0, 53)
    a_p, st_p, _, info = _run(s, 200, 1, 0)
    a_f, st_f, _, _ = _run(s, 200, 1, 1)
    assert info["folded"] == 1
    dr = max(np.abs(st_p[k] - st_f[k]).max() for k in ("x", "y", "z"))
    print(f"\n200 mixed steps, pruned vs full lists: |dr| {dr:.2e}")
    assert dr <= 1e-5
    for k in ("ke", "pe"):
        assert a_p[k] == pytest.approx(a_f[k], rel=1e-6), k


def test_hot_system_runs_on_full_lists_where_rebuilds_are_every_step():
    """At 3000 K atoms move fast enough that each step is a rebuild point
    (m = 1): no pruning then.  The result still matches the oracle."""
    O = _orc()
    s = _state(5, 0.05, 3000.0, 54)
    md = P.md_params(precision=0, lanes_per_atom=4, skin=0.6)
    with P.System.from_state(s, T0=3000.0, md=md) as g:
        avg = g.run_fast_md(60)[0]
        st = g.get_state()
        cnt = g.count_pairs()
    os_ = O.State(*(s[k].copy() for k in ("x", "y", "z", "vx", "vy", "vz", "group")), s["volume0"], s["area0"])
    ravg, _ = O.run_burst(os_, O.sc_params(), O.md_params(T0=3000.0), 60)
    dr = max(np.abs(st[k] - getattr(os_, k)).max() for k in ("x", "y", "z"))
    print(f"\n3000 K: prune radius {cnt['prune_radius']}, |dr| {dr:.2e}")
    assert dr <= 1e-8
    for k in ("ke", "pe", "szz"):
        assert avg[k] == pytest.approx(ravg[k], rel=1e-9, abs=1e-9), k


def _run_timed(s, n, precision, prune_every, timed, lanes=4, T0=300.0):
    md = P.md_params(precision=precision, lanes_per_atom=lanes, full_lists=0, prune_every=prune_every)
    with P.System.from_state(s, T0=T0, md=md) as g:
        if timed:
            g.kernel_timing(reset=True)
        avg = g.run_fast_md(n)[0]
        st = g.get_state()
        kt = g.kernel_timing() if timed else None
        info = g.info()
    return avg, st, kt, info


@pytest.mark.parametrize("prune_every,lanes", [(1, 4), (2, 4), (3, 4), (3, 16)])
def test_fp64_timed_chunks_match_the_oracle(prune_every, lanes):
    """With the kernel timing on, each chunk launches its first two steps
    directly (the first prunes) and the rest as a graph whose pruning points
    follow from there (with a pruning pass every 8 or 12 steps the graph's
    first one comes a rebuild point early instead of at its start).  The
    trajectory must meet the FP64 bars against the oracle as without the
    timing."""
    O = _orc()
    s = _state(6, 0.05, 300.0, 57)
    a_t, st_t, kt, info = _run_timed(s, 100, 0, prune_every, True, lanes=lanes)
    a_u, st_u, _, _ = _run_timed(s, 100, 0, prune_every, False, lanes=lanes)
    os_ = O.State(*(s[k].copy() for k in ("x", "y", "z", "vx", "vy", "vz", "group")), s["volume0"], s["area0"])
    ravg, _ = O.run_burst(os_, O.sc_params(), O.md_params(), 100)
    dr = max(np.abs(st_t[k] - getattr(os_, k)).max() for k in ("x", "y", "z"))
    dv = max(np.abs(st_t[k] - getattr(os_, k)).max() for k in ("vx", "vy", "vz"))
    print(f"\ntimed chunks, {lanes} lanes, pruning every {4 * prune_every} steps: {kt['count']} timed steps, |dr| {dr:.2e} "
          f"|dv| {dv:.2e}")
    assert kt["count"] >= 1 and kt["force_event_ms"] > 0.0 and info["rollbacks"] == 0
    assert info["prune_every"] == prune_every and info["lanes_per_atom"] == lanes
    assert dr <= 1e-8 and dv <= 1e-10
    for k in ("ke", "pe", "szz", "tz"):
        assert a_t[k] == pytest.approx(ravg[k], rel=1e-9, abs=1e-9), k
        assert a_t[k] == pytest.approx(a_u[k], rel=1e-11, abs=1e-11), k


@pytest.mark.parametrize("nc", [8, 33])
def test_mixed_timed_chunks_match_untimed(nc):
    """The same in the mixed form: folded (2,048 atoms) and, above 131,072
    atoms (143,748), the three-kernel step the default workload runs; timed
    and untimed runs agree to FP32 rounding."""
    s = _state(nc, 0.05, 300.0, 58)
    a_t, st_t, kt, info = _run_timed(s, 200, 1, 3, True)
    a_u, st_u, _, info_u = _run_timed(s, 200, 1, 3, False)
    dr = max(np.abs(st_t[k] - st_u[k]).max() for k in ("x", "y", "z"))
    print(f"\ncube of {nc} cells, mixed, folded {info['folded']}: {kt['count']} timed steps, "
          f"|dr| timed vs untimed {dr:.2e}")
    assert info["folded"] == (1 if nc == 8 else 0) and info_u["folded"] == info["folded"]
    assert kt["count"] >= 1 and info["rollbacks"] == 0 and info["prune_every"] == 3
    assert dr <= 1e-5
    for k in ("ke", "pe", "szz"):
        assert a_t[k] == pytest.approx(a_u[k], rel=1e-6), k


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_timed_chunks_match_untimed(precision):
    """A batch of three unequal cubes (one launch per kernel for all of them)
    with the kernel timing on, as the batched workloads are timed: each
    replica's averages and state agree with the untimed batch to rounding."""
    descs = [P.lattice_desc(5, 200.0, 3), P.lattice_desc(7, 400.0, 4), P.lattice_desc(4, 300.0, 5)]
    md = P.md_params(precision=precision, lanes_per_atom=4, full_lists=0, prune_every=2)
    out = []
    for timed in (True, False):
        with P.System.batch(descs, md=md) as b:
            if timed:
                b.kernel_timing(reset=True)
            b.apply_strain_increments([1e-4, -1e-4, 0.0])
            avg = b.run_fast_md(150)
            st = b.get_state()
            kt = b.kernel_timing() if timed else None
            info = b.info()
        out.append((avg, st, kt, info))
    (a_t, st_t, kt, info_t), (a_u, st_u, _, info_u) = out
    dr = max(np.abs(st_t[k] - st_u[k]).max() for k in ("x", "y", "z"))
    print(f"\nbatch of 3, precision {precision}: {kt['count']} timed steps, |dr| timed vs untimed {dr:.2e}")
    assert kt["count"] >= 1 and info_t["rollbacks"] == 0 and info_u["rollbacks"] == 0
    rel, dxm = (1e-9, 1e-9) if precision == 0 else (1e-6, 1e-5)
    assert dr <= dxm
    for r in range(3):
        for k in ("ke", "pe", "szz", "tz"):
            assert a_t[r][k] == pytest.approx(a_u[r][k], rel=rel, abs=rel), (r, k)
