"""ctypes wrapper of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  The product library never imports it, and it never
imports the product library.  See ``oracle.h`` for what each call computes and
which passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

D = np.float64
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class TAB(C.Structure):
    _fields_ = [("nrho", C.c_int32), ("nr", C.c_int32), ("drho", C.c_double), ("dr", C.c_double),
                ("F", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)), ("rphi", C.POINTER(C.c_double))]


class SC(C.Structure):
    _fields_ = [("eps", C.c_double), ("a", C.c_double), ("n", C.c_double), ("m", C.c_double),
                ("c", C.c_double), ("rc", C.c_double), ("shift", C.c_int32), ("tab", C.POINTER(TAB))]


class MD(C.Structure):
    _fields_ = [("dt", C.c_double), ("tau", C.c_double), ("T0", C.c_double), ("thermostat", C.c_int32),
                ("top_free_z", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.POINTER(C.c_double)) for k in ("x", "y", "z", "vx", "vy", "vz")] + [
        ("group", C.POINTER(C.c_uint8)), ("volume0", C.c_double), ("area0", C.c_double), ("strain", C.c_double)]


class Averages(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("szz", C.c_double), ("tz", C.c_double),
                ("ke_se", C.c_double), ("pe_se", C.c_double), ("szz_se", C.c_double), ("temp", C.c_double),
                ("n_samples", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SER_COLS = ("K", "U", "szz", "T", "lambda", "tz")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = C.CDLL(_LIB)
    L.orc_mass_al.restype = C.c_double
    L.orc_kb.restype = C.c_double
    L.orc_mvv2e.restype = C.c_double
    L.orc_ev_a3_to_gpa.restype = C.c_double
    L.orc_num_threads.restype = C.c_int32
    L.orc_splitmix64.restype = C.c_uint64
    L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.orc_gaussians.argtypes = [C.c_uint64, C.c_int64, _dp]
    L.orc_fcc_count.restype = C.c_int64
    L.orc_fcc_count.argtypes = [C.c_int32]
    L.orc_fcc_cube.argtypes = [C.c_int32, C.c_double, C.c_int32, _dp, _dp, _dp, _u8p, _i32p]
    L.orc_mb_velocities.restype = C.c_int32
    L.orc_mb_velocities.argtypes = [C.c_int64, _u8p, C.c_double, C.c_uint64, _dp, _dp, _dp]
    L.orc_pair_terms.argtypes = [C.POINTER(SC), C.c_double] + [C.POINTER(C.c_double)] * 4
    L.orc_embed.restype = C.c_double
    L.orc_embed.argtypes = [C.POINTER(SC), C.c_double]
    L.orc_embed_deriv.restype = C.c_double
    L.orc_embed_deriv.argtypes = [C.POINTER(SC), C.c_double]
    L.orc_density.argtypes = [C.c_int64, _dp, _dp, _dp, C.POINTER(SC), _dp]
    L.orc_forces.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_void_p, C.POINTER(SC), _dp, _dp, _dp, C.c_void_p,
                             C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.orc_atom_density.restype = C.c_double
    L.orc_atom_density.argtypes = [C.c_int64, _dp, _dp, _dp, C.POINTER(SC), C.c_int64]
    L.orc_atom_force.argtypes = [C.c_int64, _dp, _dp, _dp, C.POINTER(SC), C.c_int64, _dp]
    L.orc_neighbors.restype = C.c_int64
    L.orc_neighbors.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, _i64p, C.c_void_p, C.c_int64]
    L.orc_cell_assign.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double, _i32p, _i32p]
    L.orc_run_burst.restype = C.c_int32
    L.orc_run_burst.argtypes = [C.POINTER(_State), C.POINTER(SC), C.POINTER(MD), C.c_int64,
                                C.POINTER(Averages), C.c_void_p, C.c_void_p]
    L.orc_block_se.argtypes = [_dp, C.c_int64, C.c_int64, C.POINTER(C.c_double)]
    L.orc_apply_strain.argtypes = [C.POINTER(_State), C.c_double]
    L.orc_observables.argtypes = [C.POINTER(_State), C.POINTER(SC)] + [C.POINTER(C.c_double)] * 4
    _lib = L
    return L


def sc_params(eps=0.0033147, a=4.05, n=7.0, m=6.0, c=16.399, rc=8.1, shift=2) -> SC:
    return SC(eps, a, n, m, c, rc, shift)


class TabPotential:
    """Tabulated EAM functions for the oracle: holds the spline coefficients
    and the SC struct (``.sc``) that points at them."""

    def __init__(self, F, rho, rphi, drho: float, dr: float, rc: float):
        from scipy.interpolate import CubicSpline  # not-a-knot cubic spline, a library step

        def coef(y, h):
            y = np.asarray(y, np.float64)
            cs = CubicSpline(np.arange(len(y)) * h, y, bc_type="not-a-knot")
            return np.ascontiguousarray(cs.c.T.reshape(-1))  # per interval: u^3, u^2, u, 1

        self.cF, self.crho, self.crphi = coef(F, drho), coef(rho, dr), coef(rphi, dr)
        P = C.POINTER(C.c_double)
        self.tab = TAB(len(F), len(rho), drho, dr, self.cF.ctypes.data_as(P), self.crho.ctypes.data_as(P),
                       self.crphi.ctypes.data_as(P))
        self.sc = SC(0.0, 1.0, 1.0, 1.0, 0.0, rc, 0, C.pointer(self.tab))


def md_params(dt=1.0, tau=100.0, T0=300.0, thermostat=1, top_free_z=0) -> MD:
    return MD(dt, tau, T0, thermostat, top_free_z)


def constants():
    L = lib()
    return {"mass": L.orc_mass_al(), "kb": L.orc_kb(), "mvv2e": L.orc_mvv2e(), "gpa": L.orc_ev_a3_to_gpa()}


def num_threads() -> int:
    return int(lib().orc_num_threads())


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed, k))


def gaussians(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, D)
    lib().orc_gaussians(seed, count, out)
    return out


def fcc_cube(nc: int, a: float = 4.05, fix_slabs: bool = True):
    L = lib()
    n = int(L.orc_fcc_count(nc))
    x, y, z = (np.zeros(n, D) for _ in range(3))
    g = np.zeros(n, np.uint8)
    pz = np.zeros(n, np.int32)
    L.orc_fcc_cube(nc, a, int(fix_slabs), x, y, z, g, pz)
    return x, y, z, g, pz


def mb_velocities(group: np.ndarray, T0: float, seed: int):
    n = len(group)
    vx, vy, vz = (np.zeros(n, D) for _ in range(3))
    rc = lib().orc_mb_velocities(n, np.ascontiguousarray(group, np.uint8), T0, seed, vx, vy, vz)
    if rc != 0:
        raise ValueError("orc_mb_velocities failed")
    return vx, vy, vz


def pair_terms(p: SC, r: float):
    out = [C.c_double() for _ in range(4)]
    lib().orc_pair_terms(C.byref(p), r, *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def embed(p: SC, rho: float) -> float:
    return lib().orc_embed(C.byref(p), rho)


def embed_deriv(p: SC, rho: float) -> float:
    return lib().orc_embed_deriv(C.byref(p), rho)


def _c(a, dt=D):
    return np.ascontiguousarray(a, dtype=dt)


def density(x, y, z, p: SC) -> np.ndarray:
    x, y, z = _c(x), _c(y), _c(z)
    out = np.zeros(len(x), D)
    lib().orc_density(len(x), x, y, z, C.byref(p), out)
    return out


def forces(x, y, z, p: SC, group=None, per_atom_energy=False):
    """Internal forces before constraints, U, W_zz, R_z (and per-atom energies)."""
    x, y, z = _c(x), _c(y), _c(z)
    n = len(x)
    fx, fy, fz = (np.zeros(n, D) for _ in range(3))
    e = np.zeros(n, D) if per_atom_energy else None
    g = _c(group, np.uint8) if group is not None else None
    U, W, R = C.c_double(), C.c_double(), C.c_double()
    lib().orc_forces(n, x, y, z, g.ctypes.data if g is not None else None, C.byref(p), fx, fy, fz,
                     e.ctypes.data if e is not None else None, C.byref(U), C.byref(W), C.byref(R))
    out = {"fx": fx, "fy": fy, "fz": fz, "U": U.value, "Wzz": W.value, "Rz": R.value}
    if e is not None:
        out["e"] = e
    return out


def atom_density(x, y, z, p: SC, i: int) -> float:
    x, y, z = _c(x), _c(y), _c(z)
    return lib().orc_atom_density(len(x), x, y, z, C.byref(p), i)


def atom_force(x, y, z, p: SC, i: int) -> np.ndarray:
    x, y, z = _c(x), _c(y), _c(z)
    f = np.zeros(3, D)
    lib().orc_atom_force(len(x), x, y, z, C.byref(p), i, f)
    return f


def neighbors(x, y, z, rlist: float):
    """CSR neighbour sets {j != i : r_ij^2 < rlist^2}, ascending j."""
    x, y, z = _c(x), _c(y), _c(z)
    n = len(x)
    off = np.zeros(n + 1, np.int64)
    total = lib().orc_neighbors(n, x, y, z, rlist, off, None, 0)
    idx = np.zeros(max(total, 1), np.int32)
    lib().orc_neighbors(n, x, y, z, rlist, off, idx.ctypes.data, total)
    return off, idx[:total]


def cell_assign(x, y, z, origin, inv_h: float, dims):
    x, y, z = _c(x), _c(y), _c(z)
    out = np.zeros(3 * len(x), np.int32)
    lib().orc_cell_assign(len(x), x, y, z, _c(origin), inv_h, _c(dims, np.int32), out)
    return out.reshape(-1, 3)


@dataclass
class State:
    """An MD state in original atom order (Eq. (state)): positions, velocities, groups."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    group: np.ndarray
    volume0: float
    area0: float = 0.0
    strain: float = 0.0

    def copy(self) -> "State":
        return State(*(np.array(getattr(self, k), copy=True) for k in ("x", "y", "z", "vx", "vy", "vz", "group")),
                     self.volume0, self.area0, self.strain)

    @property
    def n(self) -> int:
        return len(self.x)

    def _cstate(self):
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            setattr(self, k, _c(getattr(self, k)))
        self.group = _c(self.group, np.uint8)
        P = C.POINTER(C.c_double)
        return _State(self.n, *[getattr(self, k).ctypes.data_as(P) for k in ("x", "y", "z", "vx", "vy", "vz")],
                      self.group.ctypes.data_as(C.POINTER(C.c_uint8)), self.volume0, self.area0, self.strain)


def create_cube(nc: int, T0: float, seed: int, a: float = 4.05, fix_slabs: bool = True) -> State:
    """FCC cube + Maxwell-Boltzmann velocities, the oracle's own construction."""
    x, y, z, g, _ = fcc_cube(nc, a, fix_slabs)
    vx, vy, vz = mb_velocities(g, T0, seed)
    return State(x, y, z, vx, vy, vz, g, volume0=float(nc) ** 3 * a ** 3, area0=(nc * a) ** 2)


def run_burst(st: State, p: SC, md: MD, n_steps: int, series: bool = False, mean_positions: bool = False):
    """Advance ``st`` in place by n_steps; returns (averages dict, series array
    or None), plus the per-atom mean positions (3, n) of Eq. (mean_pos) when
    ``mean_positions``."""
    cs = st._cstate()
    avg = Averages()
    ser = np.zeros((n_steps, len(SER_COLS)), D) if series else None
    psum = np.zeros(3 * st.n, D) if mean_positions else None
    rc = lib().orc_run_burst(C.byref(cs), C.byref(p), C.byref(md), n_steps, C.byref(avg),
                             ser.ctypes.data if ser is not None else None,
                             psum.ctypes.data if psum is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle burst failed with status {rc}")
    if mean_positions:
        return avg.as_dict(), ser, psum.reshape(3, st.n) / n_steps
    return avg.as_dict(), ser


def relax(st: State, p: SC, md: MD, burst_steps: int, max_bursts: int, tol_gpa: float):
    """Thermal relaxation of Sec. 2.4.2: bursts with the top region free along
    z until |burst-averaged reaction stress| < tol_gpa (at most max_bursts),
    then the region is held again (v = 0).  Returns (last averages, bursts,
    relaxed)."""
    free = MD(md.dt, md.tau, md.T0, md.thermostat, 1)
    k, ok, avg = 0, False, None
    while not ok and k < max_bursts:
        avg, _ = run_burst(st, p, free, burst_steps)
        k += 1
        ok = abs(avg["tz"]) < tol_gpa
    top = st.group == 2
    st.vx[top] = 0.0
    st.vy[top] = 0.0
    st.vz[top] = 0.0
    return avg, k, ok


def apply_strain(st: State, d_eps: float) -> None:
    cs = st._cstate()
    lib().orc_apply_strain(C.byref(cs), d_eps)
    st.strain = cs.strain


def observables(st: State, p: SC):
    cs = st._cstate()
    out = [C.c_double() for _ in range(4)]
    lib().orc_observables(C.byref(cs), C.byref(p), *[C.byref(o) for o in out])
    return dict(zip(("K", "U", "szz", "tz"), (o.value for o in out)))


def block_se(series) -> float:
    """Standard error of the mean of a 1-D series from 20 batch means
    (the oracle's burst standard error, NaN below 20 samples)."""
    a = np.ascontiguousarray(series, dtype=np.float64)
    out = C.c_double()
    lib().orc_block_se(a, 1, len(a), C.byref(out))
    return out.value
