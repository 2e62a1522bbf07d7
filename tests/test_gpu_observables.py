"""Mean positions (Eq. (mean_pos)) and thermal relaxation (Sec. 2.4.2) on the
GPU, through the C ABI, against the FP64 oracle on the same seeded inputs.

Bars: FP64 path, runs of up to a few hundred steps: mean positions and final
positions |d| <= 1e-8 A, averages relative 1e-9; mean positions of a
convergence-terminated burst equal those of a fixed burst of N_s steps to
rounding (1e-9 A); held coordinates exactly unchanged.
"""
import numpy as np
import pytest

import synth

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


@pytest.mark.parametrize("n_steps,skin", [(60, 1.0), (200, 0.6)])
def test_mean_positions_match_oracle(n_steps, skin):
    O = _orc()
    s = _state(5, 0.05, 300.0, 51)
    md = P.md_params(precision=0, lanes_per_atom=4, skin=skin)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        g.set_mean_positions(True)
        g.apply_strain_increment(2e-4)
        avg = g.run_fast_md(n_steps)[0]
        mean = g.get_mean_positions()
        info = g.info()
    os_ = _orc_state(s)
    O.apply_strain(os_, 2e-4)
    ravg, _, rmean = O.run_burst(os_, O.sc_params(), O.md_params(), n_steps, mean_positions=True)
    print(f"\n{n_steps} steps, skin {skin}: sorts {info['sorts']}, builds {info['list_builds']}, "
          f"max |d mean| {np.abs(mean - rmean).max():.2e}")
    assert np.abs(mean - rmean).max() <= 1e-8
    for k in ("ke", "pe", "szz"):
        assert avg[k] == pytest.approx(ravg[k], rel=1e-9, abs=1e-9)


def test_mean_positions_batch_and_convergence():
    descs = [P.lattice_desc(4, 200.0, 3), P.lattice_desc(5, 400.0, 4)]
    md = P.md_params(precision=0, lanes_per_atom=4)
    conv = P.conv_params(20, 300, (0.004, 0, 0, 0))
    with P.System.batch(descs, md=md) as b:
        b.set_mean_positions(True)
        avg, ns = b.run_until_converged(conv)
        mean_b = b.get_mean_positions()
    off = 0
    for r, d in enumerate(descs):
        n_s = int(ns[r]) if ns[r] else 300
        with P.System(P.create_system(d, P.sc_params(), md)) as g:
            g.set_mean_positions(True)
            g.run_fast_md(n_s)
            mean = g.get_mean_positions()
        m = mean.shape[1]
        print(f"\nreplica {r}: N_s {ns[r]}, max |d mean| {np.abs(mean - mean_b[:, off:off + m]).max():.2e}")
        assert avg[r]["n_samples"] == n_s
        assert np.abs(mean - mean_b[:, off:off + m]).max() <= 1e-9
        off += m


def test_mean_positions_state_errors():
    with P.System.cube(4, md=P.md_params(precision=0)) as g:
        with pytest.raises(P.PtamdError) as ei:
            g.get_mean_positions()
        assert ei.value.name == "PTAMD_ESTATE"
        g.set_mean_positions(True)
        with pytest.raises(P.PtamdError):
            g.get_mean_positions()  # no burst yet
        g.run_fast_md(10)
        m = g.get_mean_positions()
        assert np.all(np.isfinite(m))
        g.compute_forces()
        with pytest.raises(P.PtamdError):
            g.get_mean_positions()  # the sums were cleared
        g.set_mean_positions(False)
        g.run_fast_md(10)  # bursts run as before without the sums


def test_relaxation_matches_oracle():
    O = _orc()
    s = _state(5, 0.05, 300.0, 61)
    md = P.md_params(precision=0, lanes_per_atom=4)
    with P.System.from_state(s, T0=300.0, md=md) as g:
        avg, nb, ok = g.relax(40, 2, 0.0)
        st = g.get_state()
        after = g.run_fast_md(20)[0]
    os_ = _orc_state(s)
    ravg, rk, rok = O.relax(os_, O.sc_params(), O.md_params(), 40, 2, 0.0)
    assert nb == rk == 2 and not ok[0] and not rok
    for k in ("ke", "pe", "szz", "tz"):
        assert avg[0][k] == pytest.approx(ravg[k], rel=1e-9, abs=1e-9), k
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.abs(st[k] - getattr(os_, k)).max() <= 1e-8, k
    top = s["group"] == 2
    assert np.array_equal(st["x"][top], s["x"][top]) and np.array_equal(st["y"][top], s["y"][top])
    assert not np.array_equal(st["z"][top], s["z"][top])
    assert np.all(st["vz"][top] == 0.0)
    # afterwards the region is held again: a burst leaves it where it is
    r2, _ = O.run_burst(os_, O.sc_params(), O.md_params(), 20)
    assert after["ke"] == pytest.approx(r2["ke"], rel=1e-9)


def test_relaxation_reduces_reaction():
    with P.System.cube(6, md=P.md_params(precision=1)) as g:
        first = g.run_fast_md(200)[0]["tz"]
        st0 = g.get_state()
        avg, nb, ok = g.relax(200, 15, 0.05)
        st1 = g.get_state()
    top = _orc().fcc_cube(6, 4.05, True)[3] == 2
    print(f"\nT_z before {first:.3f} GPa, after {nb} bursts {avg[0]['tz']:.3f} GPa, relaxed {ok[0]}")
    assert abs(avg[0]["tz"]) < abs(first)
    assert not np.array_equal(st0["z"][top], st1["z"][top])
    assert np.array_equal(st0["x"][top], st1["x"][top])
