"""Python binding of libptamd (include/ptamd.h): argument marshalling only.

Every step of the MD burst runs in the library's gfx950 kernels.  There is no
CPU fallback: importing this module raises if ``libptamd.so`` has not been
built (``__graft_entry__.build()``), and every device call raises
``PtamdError`` with the library's status and message when it fails, for
example ``PTAMD_ENODEV`` without a gfx950 GPU.

Module-level functions carry the names of the C entry points without the
``ptamd_`` prefix; :class:`System` wraps a handle for convenience.

In a process that also uses PyTorch on the GPU (to share a stream with
:meth:`System.set_stream`, say), import torch before this package: torch
ships its own copy of the HIP runtime, and when this library's runtime was
loaded first, the library later saw no device (``PTAMD_ENODEV``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PTAMD_LIBRARY may name another build of the library (e.g. a variant built
# for comparison); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("PTAMD_LIBRARY") or os.path.join(_HERE, "libptamd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() (hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)

STATUS = {0: "PTAMD_OK", -1: "PTAMD_EINVAL", -2: "PTAMD_EDEVICE", -3: "PTAMD_ENOMEM", -4: "PTAMD_ENONFINITE",
          -5: "PTAMD_EESCAPE", -6: "PTAMD_EOVERFLOW", -7: "PTAMD_ESTATE", -8: "PTAMD_ENODEV"}

SERIES_COLS = ("K", "U", "szz", "T", "lambda", "tz")


class PtamdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class LatticeDesc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("lattice_a", C.c_double), ("T0", C.c_double), ("seed", C.c_uint64),
                ("fix_slabs", C.c_int32)]


class SCParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("a", C.c_double), ("n", C.c_double), ("m", C.c_double), ("c", C.c_double),
                ("rc", C.c_double), ("shift", C.c_int32)]


class MDParams(C.Structure):
    _fields_ = [("dt_fs", C.c_double), ("tau_fs", C.c_double), ("thermostat", C.c_int32),
                ("precision", C.c_int32), ("skin", C.c_double), ("lanes_per_atom", C.c_int32),
                ("full_lists", C.c_int32), ("prune_every", C.c_int32)]


class Averages(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("szz", C.c_double), ("tz", C.c_double),
                ("ke_se", C.c_double), ("pe_se", C.c_double), ("szz_se", C.c_double), ("temp", C.c_double),
                ("strain", C.c_double), ("n_samples", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ConvParams(C.Structure):
    _fields_ = [("lag", C.c_int64), ("n_max", C.c_int64), ("tol", C.c_double * 4), ("floor", C.c_double * 4)]


class EAMTable(C.Structure):
    _fields_ = [("nrho", C.c_int32), ("drho", C.c_double), ("nr", C.c_int32), ("dr", C.c_double),
                ("rc", C.c_double), ("F", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("rphi", C.POINTER(C.c_double))]


def eam_table(F, rho, rphi, drho: float, dr: float, rc: float):
    """An EAMTable over copies of the arrays; returns (table, arrays kept alive)."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (F, rho, rphi)]
    P_ = C.POINTER(C.c_double)
    t = EAMTable(len(arrs[0]), drho, len(arrs[1]), dr, rc, *[a.ctypes.data_as(P_) for a in arrs])
    if len(arrs[2]) != len(arrs[1]):
        raise ValueError("rho and r*phi need the same number of values")
    return t, arrs


class RelaxParams(C.Structure):
    _fields_ = [("burst_steps", C.c_int64), ("max_bursts", C.c_int64), ("tol_gpa", C.c_double)]


class PTAParams(C.Structure):
    _fields_ = [("d_eps_h", C.c_double), ("delta_over_h", C.c_double), ("conv", ConvParams),
                ("tol_v", C.c_double * 4), ("tol_j", C.c_double * 4)]


class PTAState(C.Structure):
    _fields_ = [("strain", C.c_double), ("R_tmd", C.c_double * 4), ("R_tmh", C.c_double * 4),
                ("R_t", C.c_double * 4), ("R_prev", C.c_double * 4), ("v", C.c_double * 4),
                ("jump_at_t", C.c_int32 * 4), ("n_jumps", C.c_int64)]

    def as_dict(self):
        return _struct_dict(self)


class PTARecord(C.Structure):
    _fields_ = [("strain", C.c_double * 3), ("R", (C.c_double * 4) * 3), ("n_steps", C.c_int64 * 3),
                ("v_pred", C.c_double * 4), ("v_d", C.c_double * 4), ("v", C.c_double * 4),
                ("e_v", C.c_double * 4), ("e1", C.c_double * 4), ("e2", C.c_double * 4),
                ("status", C.c_int32 * 4)]

    def as_dict(self):
        return _struct_dict(self)


def _struct_dict(st) -> dict:
    out = {}
    for k, _ in st._fields_:
        v = getattr(st, k)
        out[k] = np.array([list(r) for r in v]) if k == "R" else (np.array(list(v)) if hasattr(v, "_length_") else v)
    return out


class Info(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("n_replicas", C.c_int32), ("precision", C.c_int32),
                ("lanes_per_atom", C.c_int32), ("list_capacity", C.c_int32), ("list_builds", C.c_int64),
                ("sorts", C.c_int64), ("rollbacks", C.c_int64), ("steps", C.c_int64), ("skin", C.c_double),
                ("bin_margin", C.c_double), ("list_index_bits", C.c_int32), ("folded", C.c_int32),
                ("prune_every", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SYS = C.c_void_p

# (name, argtypes) of every exported entry point, in the order of ptamd.h
SIGNATURES = {
    "ptamd_create_system": [C.POINTER(LatticeDesc), C.POINTER(SCParams), C.POINTER(MDParams), C.POINTER(_SYS)],
    "ptamd_create_system_from_state": [C.c_int64, _P, _P, _P, _P, _P, _P, _P, C.c_double, C.c_double, C.c_double,
                                       C.POINTER(SCParams), C.POINTER(MDParams), C.POINTER(_SYS)],
    "ptamd_create_batch": [C.c_int32, C.POINTER(LatticeDesc), C.POINTER(SCParams), C.POINTER(MDParams),
                           C.POINTER(_SYS)],
    "ptamd_destroy_system": [_SYS],
    "ptamd_apply_strain_increment": [_SYS, C.c_double],
    "ptamd_apply_strain_increments": [_SYS, _P],
    "ptamd_apply_strain_increments_noalloc": [_SYS, _P],
    "ptamd_run_fast_md": [_SYS, C.c_int64, C.POINTER(Averages)],
    "ptamd_run_until_converged": [_SYS, C.POINTER(ConvParams), C.POINTER(Averages), _P],
    "ptamd_set_eam_table": [_SYS, C.POINTER(EAMTable)],
    "ptamd_read_setfl": [C.c_char_p, C.POINTER(EAMTable), _P, _P, _P, _P],
    "ptamd_eam_table_eval": [C.POINTER(EAMTable), C.c_int32, C.c_int64, _P, _P, _P],
    "ptamd_set_mean_positions": [_SYS, C.c_int32],
    "ptamd_get_mean_positions": [_SYS, _P, _P, _P],
    "ptamd_relax": [_SYS, C.POINTER(RelaxParams), C.POINTER(Averages), C.POINTER(C.c_int64), _P],
    "ptamd_pta_start": [_SYS, C.POINTER(PTAParams), C.POINTER(PTAState), C.POINTER(PTARecord)],
    "ptamd_pta_jump": [_SYS, C.POINTER(PTAParams), C.POINTER(PTAState), C.POINTER(PTARecord)],
    "ptamd_pta_update": [C.POINTER(PTAParams), C.POINTER(PTAState), _P, _P, _P, C.POINTER(PTARecord)],
    "ptamd_get_num_atoms": [_SYS, C.POINTER(C.c_int64)],
    "ptamd_get_state": [_SYS, _P, _P, _P, _P, _P, _P],
    "ptamd_set_state": [_SYS, _P, _P, _P, _P, _P, _P],
    "ptamd_get_strain": [_SYS, _P],
    "ptamd_compute_forces": [_SYS, _P, _P, _P, _P, _P],
    "ptamd_get_forces": [_SYS, _P, _P, _P],
    "ptamd_get_neighbors": [_SYS, _P, _P, C.c_int64],
    "ptamd_get_cells": [_SYS, _P, _P, _P, _P],
    "ptamd_get_series": [_SYS, C.c_int32, _P, C.c_int64],
    "ptamd_get_info": [_SYS, C.POINTER(Info)],
    "ptamd_set_stream": [_SYS, C.c_void_p],
    "ptamd_kernel_timing": [_SYS, _D, _D, _D, C.POINTER(C.c_int64), C.c_int32],
    "ptamd_autotune": [_SYS, C.c_int64, C.c_int32, C.POINTER(C.c_int32), _D, C.POINTER(C.c_int32), _D],
    "ptamd_count_pairs": [_SYS, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), _D,
                          C.POINTER(C.c_int64)],
    "ptamd_measure_device": [C.c_int64, C.c_int32, _D, _D, _D],
    "ptamd_last_error": [],
    "ptamd_version": [],
}

for _name, _args in SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_char_p if _name in ("ptamd_last_error", "ptamd_version") else C.c_int


def last_error() -> str:
    return _lib.ptamd_last_error().decode()


def version() -> str:
    return _lib.ptamd_version().decode()


def _check(status: int):
    if status != 0:
        raise PtamdError(status, last_error())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def sc_params(eps=0.0033147, a=4.05, n=7.0, m=6.0, c=16.399, rc=8.1, shift=2) -> SCParams:
    return SCParams(eps, a, n, m, c, rc, shift)


def md_params(dt_fs=1.0, tau_fs=100.0, thermostat=1, precision=0, skin=1.0, lanes_per_atom=0,
              full_lists=0, prune_every=0) -> MDParams:
    return MDParams(dt_fs, tau_fs, thermostat, precision, skin, lanes_per_atom, full_lists, prune_every)


def conv_params(lag=1000, n_max=50000, tol=(0.05, 0.05, 0.0, 0.05), floor=(0.0, 0.0, 0.0, 0.0)) -> ConvParams:
    """Convergence test of the running averages; tolerances and floors in the
    order K, U, sigma_zz, T_z (defaults: Table 1's 5% on K, U and the reaction
    stress, N_max = 50000)."""
    return ConvParams(lag, n_max, (C.c_double * 4)(*tol), (C.c_double * 4)(*floor))


def pta_params(d_eps_h: float, delta_over_h: float = 0.2, conv: Optional[ConvParams] = None,
               tol_v=(0.01, 0.05, 0.01, 0.01), tol_j=(0.08, 0.01, 0.05, 0.05)) -> PTAParams:
    """Slow-time driver parameters; tolerances in the order K, U, sigma_zz, T_z
    (defaults: Table 1, the reaction-stress values also for sigma_zz)."""
    return PTAParams(d_eps_h, delta_over_h, conv if conv is not None else conv_params(),
                     (C.c_double * 4)(*tol_v), (C.c_double * 4)(*tol_j))


def lattice_desc(n_cells: int, T0: float = 300.0, seed: int = 1, lattice_a: float = 4.05,
                 fix_slabs: bool = True) -> LatticeDesc:
    return LatticeDesc(n_cells, lattice_a, T0, seed, int(fix_slabs))


# ---------------------------------------------------------------------------
# module-level functions named after the C entry points
# ---------------------------------------------------------------------------
def create_system(desc: LatticeDesc, sc: SCParams, md: MDParams) -> int:
    h = _SYS()
    _check(_lib.ptamd_create_system(C.byref(desc), C.byref(sc), C.byref(md), C.byref(h)))
    return h.value


def create_system_from_state(x, y, z, vx, vy, vz, group, volume0: float, area0: float, T0: float,
                             sc: SCParams, md: MDParams) -> int:
    arrs = [np.ascontiguousarray(a, np.float64) for a in (x, y, z, vx, vy, vz)]
    g = np.ascontiguousarray(group, np.uint8)
    n = len(arrs[0])
    if any(len(a) != n for a in arrs) or len(g) != n:
        raise ValueError("state arrays differ in length")
    h = _SYS()
    _check(_lib.ptamd_create_system_from_state(n, *[_ptr(a) for a in arrs], _ptr(g), volume0, area0, T0,
                                               C.byref(sc), C.byref(md), C.byref(h)))
    return h.value


def create_batch(descs: Sequence[LatticeDesc], sc: SCParams, md: MDParams) -> int:
    arr = (LatticeDesc * len(descs))(*descs)
    h = _SYS()
    _check(_lib.ptamd_create_batch(len(descs), arr, C.byref(sc), C.byref(md), C.byref(h)))
    return h.value


def destroy_system(sys: int) -> None:
    _check(_lib.ptamd_destroy_system(sys))


def apply_strain_increment(sys: int, d_eps: float) -> None:
    _check(_lib.ptamd_apply_strain_increment(sys, d_eps))


def apply_strain_increments(sys: int, d_eps) -> None:
    d = np.ascontiguousarray(d_eps, np.float64)
    _check(_lib.ptamd_apply_strain_increments(sys, _ptr(d)))


def apply_strain_increments_noalloc(sys: int, d_eps) -> None:
    """ptamd_apply_strain_increments_noalloc: the same increments without any
    allocation inside the library (one entry per replica)."""
    d = np.ascontiguousarray(d_eps, np.float64)
    if d.ndim != 1 or len(d) != get_info(sys)["n_replicas"]:
        raise ValueError("need one strain increment per replica")
    _check(_lib.ptamd_apply_strain_increments_noalloc(sys, _ptr(d)))


def get_info(sys: int) -> dict:
    inf = Info()
    _check(_lib.ptamd_get_info(sys, C.byref(inf)))
    return inf.as_dict()


def run_fast_md(sys: int, n_steps: int) -> list:
    nr = get_info(sys)["n_replicas"]
    out = (Averages * nr)()
    _check(_lib.ptamd_run_fast_md(sys, n_steps, out))
    return [o.as_dict() for o in out]


def run_until_converged(sys: int, conv: ConvParams) -> tuple:
    """Returns (averages per replica, N_s per replica (0: not converged))."""
    nr = get_info(sys)["n_replicas"]
    out = (Averages * nr)()
    n_conv = np.zeros(nr, np.int64)
    _check(_lib.ptamd_run_until_converged(sys, C.byref(conv), out, _ptr(n_conv)))
    return [o.as_dict() for o in out], n_conv


def set_eam_table(sys: int, F, rho, rphi, drho: float, dr: float, rc: float) -> None:
    t, keep = eam_table(F, rho, rphi, drho, dr, rc)
    _check(_lib.ptamd_set_eam_table(sys, C.byref(t)))
    del keep


def read_setfl(path: str) -> dict:
    """Single-element setfl file -> dict(F, rho, rphi, drho, dr, rc, mass)."""
    t = EAMTable()
    mass = C.c_double()
    _check(_lib.ptamd_read_setfl(path.encode(), C.byref(t), None, None, None, C.byref(mass)))
    F, rho, rphi = np.zeros(t.nrho), np.zeros(t.nr), np.zeros(t.nr)
    _check(_lib.ptamd_read_setfl(path.encode(), C.byref(t), _ptr(F), _ptr(rho), _ptr(rphi), C.byref(mass)))
    return dict(F=F, rho=rho, rphi=rphi, drho=t.drho, dr=t.dr, rc=t.rc, mass=mass.value)


def eam_table_eval(F, rho, rphi, drho: float, dr: float, rc: float, which: int, x) -> tuple:
    """The library's spline of table function ``which`` (0 F, 1 rho, 2 r*phi) at x: (f, df)."""
    t, keep = eam_table(F, rho, rphi, drho, dr, rc)
    xa = np.ascontiguousarray(x, np.float64)
    f, df = np.zeros_like(xa), np.zeros_like(xa)
    _check(_lib.ptamd_eam_table_eval(C.byref(t), which, len(xa), _ptr(xa), _ptr(f), _ptr(df)))
    del keep
    return f, df


def set_mean_positions(sys: int, enable: bool = True) -> None:
    _check(_lib.ptamd_set_mean_positions(sys, int(bool(enable))))


def get_mean_positions(sys: int) -> np.ndarray:
    """(3, n) mean positions of Eq. (mean_pos) over the last burst's samples."""
    n = get_num_atoms(sys)
    out = np.zeros((3, n), np.float64)
    _check(_lib.ptamd_get_mean_positions(sys, _ptr(out[0]), _ptr(out[1]), _ptr(out[2])))
    return out


def relax(sys: int, burst_steps: int, max_bursts: int, tol_gpa: float) -> tuple:
    """Thermal relaxation with the top region free along z.  Returns (last
    burst's averages per replica, bursts run, relaxed flags)."""
    nr = get_info(sys)["n_replicas"]
    out = (Averages * nr)()
    nb = C.c_int64()
    flags = np.zeros(nr, np.int32)
    prm = RelaxParams(burst_steps, max_bursts, tol_gpa)
    _check(_lib.ptamd_relax(sys, C.byref(prm), out, C.byref(nb), _ptr(flags)))
    return [o.as_dict() for o in out], nb.value, flags.astype(bool)


def pta_start(sys: int, prm: PTAParams):
    """Returns (ctypes array of PTAState, list of record dicts), one per replica."""
    nr = get_info(sys)["n_replicas"]
    st = (PTAState * nr)()
    rec = (PTARecord * nr)()
    _check(_lib.ptamd_pta_start(sys, C.byref(prm), st, rec))
    return st, [r.as_dict() for r in rec]


def pta_jump(sys: int, prm: PTAParams, states) -> list:
    """Advances ``states`` (from pta_start) in place by one slow jump."""
    nr = get_info(sys)["n_replicas"]
    rec = (PTARecord * nr)()
    _check(_lib.ptamd_pta_jump(sys, C.byref(prm), states, rec))
    return [r.as_dict() for r in rec]


def pta_update(prm: PTAParams, state: PTAState, R, strains, n_steps) -> dict:
    """Host-only arithmetic of one slow step (no device needed); advances ``state``."""
    Ra = np.ascontiguousarray(R, np.float64).reshape(3, 4)
    sa = np.ascontiguousarray(strains, np.float64)
    na = np.ascontiguousarray(n_steps, np.int64)
    rec = PTARecord()
    _check(_lib.ptamd_pta_update(C.byref(prm), C.byref(state), _ptr(Ra), _ptr(sa), _ptr(na), C.byref(rec)))
    return rec.as_dict()


def get_num_atoms(sys: int) -> int:
    n = C.c_int64()
    _check(_lib.ptamd_get_num_atoms(sys, C.byref(n)))
    return n.value


def get_state(sys: int) -> dict:
    n = get_num_atoms(sys)
    arrs = {k: np.zeros(n, np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
    _check(_lib.ptamd_get_state(sys, *[_ptr(arrs[k]) for k in ("x", "y", "z", "vx", "vy", "vz")]))
    return arrs


def set_state(sys: int, x, y, z, vx, vy, vz) -> None:
    arrs = [np.ascontiguousarray(a, np.float64) for a in (x, y, z, vx, vy, vz)]
    _check(_lib.ptamd_set_state(sys, *[_ptr(a) for a in arrs]))


def get_strain(sys: int) -> np.ndarray:
    s = np.zeros(get_info(sys)["n_replicas"], np.float64)
    _check(_lib.ptamd_get_strain(sys, _ptr(s)))
    return s


def compute_forces(sys: int) -> dict:
    n = get_num_atoms(sys)
    nr = get_info(sys)["n_replicas"]
    f = [np.zeros(n, np.float64) for _ in range(3)]
    pe, w = np.zeros(nr), np.zeros(nr)
    _check(_lib.ptamd_compute_forces(sys, *[_ptr(a) for a in f], _ptr(pe), _ptr(w)))
    return {"fx": f[0], "fy": f[1], "fz": f[2], "U": pe, "Wzz": w}


def get_forces(sys: int) -> dict:
    n = get_num_atoms(sys)
    f = [np.zeros(n, np.float64) for _ in range(3)]
    _check(_lib.ptamd_get_forces(sys, *[_ptr(a) for a in f]))
    return {"fx": f[0], "fy": f[1], "fz": f[2]}


def get_neighbors(sys: int):
    n = get_num_atoms(sys)
    off = np.zeros(n + 1, np.int64)
    st = _lib.ptamd_get_neighbors(sys, _ptr(off), None, 0)
    if st not in (0, -6):
        _check(st)
    idx = np.zeros(max(int(off[-1]), 1), np.int32)
    _check(_lib.ptamd_get_neighbors(sys, _ptr(off), _ptr(idx), len(idx)))
    return off, idx[: int(off[-1])]


def get_cells(sys: int):
    n = get_num_atoms(sys)
    nr = get_info(sys)["n_replicas"]
    c = np.zeros(3 * n, np.int32)
    o = np.zeros(3 * nr, np.float64)
    ih = np.zeros(nr, np.float64)
    d = np.zeros(3 * nr, np.int32)
    _check(_lib.ptamd_get_cells(sys, _ptr(c), _ptr(o), _ptr(ih), _ptr(d)))
    return c.reshape(n, 3), o.reshape(nr, 3), ih, d.reshape(nr, 3)


def get_series(sys: int, replica: int, rows: int) -> np.ndarray:
    buf = np.zeros((rows, len(SERIES_COLS)), np.float64)
    _check(_lib.ptamd_get_series(sys, replica, _ptr(buf), rows))
    return buf


def set_stream(sys: int, stream) -> None:
    """stream: a torch.cuda.Stream, a raw hipStream_t address, or None."""
    if stream is None:
        ptr = None
    elif hasattr(stream, "cuda_stream"):
        ptr = C.c_void_p(stream.cuda_stream)
    else:
        ptr = C.c_void_p(int(stream))
    _check(_lib.ptamd_set_stream(sys, ptr))


def kernel_timing(sys: int, reset: bool = False) -> dict:
    """Averages over the timed steps, in ms: the force kernel's span from
    in-kernel device clock stamps, the same launches bracketed by HIP events,
    the density kernel bracketed by HIP events; and the count of timed steps."""
    ms, ev, dev, cnt = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
    _check(_lib.ptamd_kernel_timing(sys, C.byref(ms), C.byref(ev), C.byref(dev), C.byref(cnt), int(reset)))
    return {"force_ms": ms.value, "force_event_ms": ev.value, "density_event_ms": dev.value, "count": cnt.value}


def autotune(sys: int, probe_steps: int = 100, use_cache: bool = True) -> dict:
    l, sk, pe, ms = C.c_int32(), C.c_double(), C.c_int32(), C.c_double()
    _check(_lib.ptamd_autotune(sys, probe_steps, int(use_cache), C.byref(l), C.byref(sk), C.byref(pe), C.byref(ms)))
    return {"lanes_per_atom": l.value, "skin": sk.value, "prune_every": pe.value, "ms_per_step": ms.value}


def measure_device(nbytes: int = 1 << 30, reps: int = 10) -> dict:
    """Achievable copy bandwidth (GB/s) and FP32/FP64 FMA rates (TFLOP/s) of
    the current device (ptamd_measure_device)."""
    cp, f32, f64 = C.c_double(), C.c_double(), C.c_double()
    _check(_lib.ptamd_measure_device(nbytes, reps, C.byref(cp), C.byref(f32), C.byref(f64)))
    return {"copy_GBs": cp.value, "fma32_TFLOPs": f32.value, "fma64_TFLOPs": f64.value}


def count_pairs(sys: int) -> dict:
    """Unique pairs within rc, full-list entries, pruned-list entries, the
    pruned lists' radius (A; 0 when the last chunk ran on full lists) and the
    atoms whose lists hold 32-bit indices."""
    p, e, q, r, w = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double(), C.c_int64()
    _check(_lib.ptamd_count_pairs(sys, C.byref(p), C.byref(e), C.byref(q), C.byref(r), C.byref(w)))
    return {"pairs_in_rc": p.value, "list_entries": e.value, "pruned_entries": q.value, "prune_radius": r.value,
            "wide_atoms": w.value}


# ---------------------------------------------------------------------------
class System:
    """Owning wrapper of a ptamd_system handle."""

    def __init__(self, handle: int):
        self.h = handle

    @classmethod
    def cube(cls, n_cells: int, T0: float = 300.0, seed: int = 1, fix_slabs: bool = True,
             sc: Optional[SCParams] = None, md: Optional[MDParams] = None, lattice_a: float = 4.05) -> "System":
        return cls(create_system(lattice_desc(n_cells, T0, seed, lattice_a, fix_slabs), sc or sc_params(),
                                 md or md_params()))

    @classmethod
    def from_state(cls, st: dict, T0: float = 300.0, sc: Optional[SCParams] = None,
                   md: Optional[MDParams] = None) -> "System":
        return cls(create_system_from_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["group"],
                                            st["volume0"], st.get("area0", 0.0), T0, sc or sc_params(),
                                            md or md_params()))

    @classmethod
    def batch(cls, descs: Sequence[LatticeDesc], sc: Optional[SCParams] = None,
              md: Optional[MDParams] = None) -> "System":
        return cls(create_batch(descs, sc or sc_params(), md or md_params()))

    def close(self):
        if self.h:
            destroy_system(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return get_info(self.h)

    def n_atoms(self):
        return get_num_atoms(self.h)

    def apply_strain_increment(self, d_eps: float):
        apply_strain_increment(self.h, d_eps)

    def apply_strain_increments(self, d_eps):
        apply_strain_increments(self.h, d_eps)

    def apply_strain_increments_noalloc(self, d_eps):
        apply_strain_increments_noalloc(self.h, d_eps)

    def run_fast_md(self, n_steps: int):
        return run_fast_md(self.h, n_steps)

    def run_until_converged(self, conv: Optional[ConvParams] = None):
        return run_until_converged(self.h, conv if conv is not None else conv_params())

    def set_eam_table(self, F, rho, rphi, drho: float, dr: float, rc: float):
        set_eam_table(self.h, F, rho, rphi, drho, dr, rc)

    def set_mean_positions(self, enable: bool = True):
        set_mean_positions(self.h, enable)

    def get_mean_positions(self):
        return get_mean_positions(self.h)

    def relax(self, burst_steps: int, max_bursts: int, tol_gpa: float):
        return relax(self.h, burst_steps, max_bursts, tol_gpa)

    def pta_start(self, prm: PTAParams):
        return pta_start(self.h, prm)

    def pta_jump(self, prm: PTAParams, states):
        return pta_jump(self.h, prm, states)

    def get_state(self):
        return get_state(self.h)

    def set_state(self, st: dict):
        set_state(self.h, st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"])

    def strain(self):
        return get_strain(self.h)

    def compute_forces(self):
        return compute_forces(self.h)

    def get_forces(self):
        return get_forces(self.h)

    def get_neighbors(self):
        return get_neighbors(self.h)

    def get_cells(self):
        return get_cells(self.h)

    def get_series(self, replica: int, rows: int):
        return get_series(self.h, replica, rows)

    def set_stream(self, stream):
        set_stream(self.h, stream)

    def kernel_timing(self, reset: bool = False):
        return kernel_timing(self.h, reset)

    def count_pairs(self):
        return count_pairs(self.h)

    def autotune(self, probe_steps: int = 100, use_cache: bool = True):
        return autotune(self.h, probe_steps, use_cache)
