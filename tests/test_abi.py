"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/ptamd.h declares, the binding names match,
and argument validation reports PTAMD_EINVAL before any device work."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "ptamd.h")) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"\b(ptamd_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2603_07321_amd as P
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(P._lib, n), n
    # the binding declares the same set
    assert sorted(P.SIGNATURES) == names


def test_binding_has_same_names():
    import paper_2603_07321_amd as P
    for n in _declared():
        short = n[len("ptamd_"):]
        assert callable(getattr(P, short)), short


def test_version_and_error_strings():
    import paper_2603_07321_amd as P
    assert "gfx950" in P.version()
    assert isinstance(P.last_error(), str)


@pytest.mark.parametrize("bad", [
    dict(sc=dict(rc=-1.0)), dict(sc=dict(n=6.5)), dict(sc=dict(shift=3)), dict(sc=dict(rc=20.0)),
    dict(md=dict(dt_fs=0.0)), dict(md=dict(precision=2)), dict(md=dict(skin=0.0)),
    dict(md=dict(lanes_per_atom=3)), dict(md=dict(thermostat=1, tau_fs=0.0)),
    dict(desc=dict(n_cells=3)), dict(desc=dict(lattice_a=-4.0)),
])
def test_invalid_arguments_rejected(bad):
    import paper_2603_07321_amd as P
    sc = P.sc_params(**bad.get("sc", {}))
    md = P.md_params(**bad.get("md", {}))
    d = dict(n_cells=5, T0=300.0, seed=1)
    d.update(bad.get("desc", {}))
    desc = P.LatticeDesc(d["n_cells"], d.get("lattice_a", 4.05), d["T0"], d["seed"], 1)
    with pytest.raises(P.PtamdError) as ei:
        P.create_system(desc, sc, md)
    assert ei.value.name == "PTAMD_EINVAL"


def test_no_device_is_an_error_not_a_fallback():
    import torch
    import paper_2603_07321_amd as P
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.PtamdError) as ei:
        P.System.cube(5)
    assert ei.value.name == "PTAMD_ENODEV"


def test_null_handle_rejected():
    import paper_2603_07321_amd as P
    with pytest.raises(P.PtamdError):
        P.run_fast_md(0, 10) if False else P._check(P._lib.ptamd_run_fast_md(None, 10, None))


def test_too_many_atoms_rejected_before_any_work():
    """Gathers address positions with 32-bit byte offsets: more than 2^27 - 1
    padded atoms in one system is an argument error, reported at once (no
    lattice is built, no device is touched)."""
    import time
    import paper_2603_07321_amd as P
    cases = [[P.lattice_desc(330)], [P.lattice_desc(260), P.lattice_desc(260, seed=2)]]
    for descs in cases:
        t0 = time.perf_counter()
        with pytest.raises(P.PtamdError) as ei:
            P.create_batch(descs, P.sc_params(), P.md_params())
        assert ei.value.name == "PTAMD_EINVAL" and "too many atoms" in P.last_error()
        assert time.perf_counter() - t0 < 1.0
    # the same bound for a caller's state (checked before the arrays are read)
    h = P._SYS()
    st = P._lib.ptamd_create_system_from_state(1 << 27, None, None, None, None, None, None, None, 1.0, 0.0, 0.0,
                                               P.C.byref(P.sc_params()), P.C.byref(P.md_params()), P.C.byref(h))
    assert st == -1 and "too many atoms" in P.last_error() and not h.value


@pytest.mark.parametrize("n", [0, 1])
def test_state_with_fewer_than_two_atoms_rejected(n):
    import numpy as np
    import paper_2603_07321_amd as P
    a = np.zeros(n)
    with pytest.raises(P.PtamdError) as ei:
        P.create_system_from_state(a, a, a, a, a, a, np.zeros(n, np.uint8), 1.0, 0.0, 0.0,
                                   P.sc_params(), P.md_params())
    assert ei.value.name == "PTAMD_EINVAL"
