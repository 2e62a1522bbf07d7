"""The allocation-free strain increment (ptamd_apply_strain_increments_noalloc)
against the allocating one (ptamd_apply_strain_increments), through the C ABI.

Both scale every z of each replica by (1 + eps_k)/(1 + eps_{k-1}) with the
same FP64 factor, so the states they leave are bitwise equal, and so are
the bursts that follow.  Two calls in a row on one GPU, the second with
fewer replicas than the first (the static factor array keeps the first
call's values beyond the second's replicas, which must not matter), and a
batch at the array's 4096-replica limit.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def _check_pair(descs, d_eps, md):
    with P.System.batch(descs, md=md) as a, P.System.batch(descs, md=md) as b:
        a.apply_strain_increments(d_eps)
        b.apply_strain_increments_noalloc(d_eps)
        sa, sb = a.get_state(), b.get_state()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k
        assert np.array_equal(a.strain(), b.strain())
        # a second increment of the other sign, then a burst
        a.apply_strain_increments([-2.0 * e for e in d_eps])
        b.apply_strain_increments_noalloc([-2.0 * e for e in d_eps])
        avg_a = a.run_fast_md(30)
        avg_b = b.run_fast_md(30)
        sa, sb = a.get_state(), b.get_state()
    assert avg_a == avg_b
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_noalloc_matches_allocating_then_smaller_input():
    md = P.md_params(precision=1, lanes_per_atom=4)
    descs5 = [P.lattice_desc(4 + k, 300.0, 10 + k) for k in range(5)]
    _check_pair(descs5, [1e-4, -2e-4, 3e-4, 0.0, -1e-3], md)
    # second call on the same GPU with fewer replicas
    descs2 = [P.lattice_desc(6, 250.0, 30), P.lattice_desc(4, 350.0, 31)]
    _check_pair(descs2, [-5e-4, 2e-4], P.md_params(precision=0, lanes_per_atom=2))


def test_noalloc_single_replica_and_limits():
    with P.System.cube(5, md=P.md_params(precision=0)) as a, P.System.cube(5, md=P.md_params(precision=0)) as b:
        a.apply_strain_increment(1e-4)
        b.apply_strain_increments_noalloc([1e-4])
        assert np.array_equal(a.get_state()["z"], b.get_state()["z"])
        with pytest.raises(P.PtamdError):
            b.apply_strain_increments_noalloc([0.5])  # |d_eps| >= 0.05
        with pytest.raises(ValueError):
            b.apply_strain_increments_noalloc([1e-4, 1e-4])  # one entry per replica


def test_noalloc_at_the_replica_limit():
    """4096 replicas, the array's size and the batch limit (a larger batch
    cannot be created, so the entry point's own size check is a guard)."""
    descs = [P.lattice_desc(4, 300.0, 1 + k) for k in range(4096)]
    d_eps = np.linspace(-1e-3, 1e-3, 4096)
    md = P.md_params(precision=1)
    with P.System.batch(descs, md=md) as a, P.System.batch(descs, md=md) as b:
        a.apply_strain_increments(d_eps)
        b.apply_strain_increments_noalloc(d_eps)
        assert np.array_equal(a.get_state()["z"], b.get_state()["z"])
        assert np.array_equal(a.strain(), b.strain())
    with pytest.raises(P.PtamdError):
        P.System.batch(descs + [P.lattice_desc(4, 300.0, 5000)], md=md)
