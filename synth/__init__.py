"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays out input geometry: perturbed
FCC coordinates, Gaussian velocity sets, dilute "gas" arrangements, and the
workload recipes (cube sizes, temperatures, seeds, strain increments).  It
holds none of the method's arithmetic (no potential, force, integrator or
averaging), and imports neither the oracle nor the product library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

A_AL = 4.05  # lattice parameter of Al used throughout the paper's setup (Table 1)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def fcc_points(nc: int, a: float = A_AL):
    """FCC cube of nc^3 cells as integer half-lattice plane indices (px, py, pz)
    and coordinates index * a/2 (cell x fastest, basis atom innermost)."""
    basis = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.int64)
    iz, iy, ix = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    p = (2 * cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    half = 0.5 * a
    xyz = p.astype(np.float64) * half
    return xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), p.astype(np.int32)


def fcc_slab(nx: int, ny: int, nz: int, noise: float, seed: int, a: float = A_AL):
    """Perturbed FCC block of nx x ny x nz cells, every atom mobile, at rest
    (a thin film when nz is small)."""
    basis = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.int64)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    p = (2 * cells[:, None, :] + basis[None, :, :]).reshape(-1, 3).astype(np.float64) * (0.5 * a)
    x, y, z = perturb(p[:, 0], p[:, 1], p[:, 2], noise, seed)
    zero = np.zeros(len(x))
    return dict(x=x, y=y, z=z, vx=zero.copy(), vy=zero.copy(), vz=zero.copy(), group=np.zeros(len(x), np.uint8),
                volume0=nx * ny * nz * a ** 3, area0=nx * ny * a ** 2)


def slab_groups(pz: np.ndarray, nc: int, fix_slabs: bool = True) -> np.ndarray:
    """Tags: 0 mobile, 1 bottom three z planes, 2 top three z planes."""
    g = np.zeros(len(pz), np.uint8)
    if fix_slabs:
        g[pz <= 2] = 1
        g[pz >= 2 * nc - 3] = 2
    return g


def perturb(x, y, z, amp: float, seed: int):
    """Independent uniform displacements in [-amp, amp) per coordinate."""
    r = rng(seed)
    d = r.uniform(-amp, amp, size=(3, len(x)))
    return x + d[0], y + d[1], z + d[2]


def gaussian_velocities(n: int, sigma: float, seed: int, mask=None):
    r = rng(seed)
    v = r.normal(0.0, sigma, size=(3, n))
    if mask is not None:
        v[:, ~mask] = 0.0
    return v[0].copy(), v[1].copy(), v[2].copy()


def gas(n_side: int, spacing: float, seed: int, jitter: float = 0.0):
    """Simple-cubic arrangement with the given spacing (a non-interacting gas
    when spacing exceeds the cutoff plus twice the jitter)."""
    g = np.arange(n_side, dtype=np.float64) * spacing
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = xx.ravel().copy(), yy.ravel().copy(), zz.ravel().copy()
    if jitter > 0:
        x, y, z = perturb(x, y, z, jitter, seed)
    return x, y, z


def cube_state(nc: int, noise: float, v_sigma: float, seed: int, fix_slabs: bool = True, a: float = A_AL):
    """Perturbed FCC cube with Gaussian velocities on the mobile atoms."""
    x, y, z, p = fcc_points(nc, a)
    g = slab_groups(p[:, 2], nc, fix_slabs)
    if noise > 0:
        x, y, z = perturb(x, y, z, noise, seed)
    vx, vy, vz = gaussian_velocities(len(x), v_sigma, seed + 7919, mask=(g == 0))
    return dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, group=g, volume0=float(nc) ** 3 * a ** 3,
                area0=(nc * a) ** 2)


# ---------------------------------------------------------------------------
# Workload recipes (sizes, temperatures, seeds and loads of the benchmark
# configurations).  The potential: Sutton-Chen, eps = 0.0033147 eV, a = 4.05 A,
# n = 7, m = 6, c = 16.399, rc = 8.1 A, shifted force; dt = 1 fs,
# Berendsen tau = 100 fs.
# ---------------------------------------------------------------------------

SC_DEFAULT = dict(eps=0.0033147, a=4.05, n=7.0, m=6.0, c=16.399, rc=8.1, shift=2)


@dataclass
class Workload:
    name: str
    n_cells: list            # cube edge in unit cells, one per replica
    T0: list                 # K, one per replica
    seeds: list
    d_eps: list              # strain increment per replica (0: none)
    increments: int          # load steps, each followed by one burst
    burst_steps: int
    precision: int           # 0 FP64, 1 mixed
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(sum(4 * n ** 3 for n in self.n_cells))


def workloads():
    w = {}
    w["cube10_fp64_200"] = Workload("cube10_fp64_200", [10], [300.0], [1], [0.0], 1, 200, 0,
                                    "4,000-atom cube, plain FP64, one 200-step burst")
    w["cube25_tension_mixed"] = Workload("cube25_tension_mixed", [25], [300.0], [1], [1e-4], 20, 2000, 1,
                                         "62,500-atom cube, 20 x (+1e-4 affine z strain, 2000-step burst), mixed")
    w["cube50_compression_mixed"] = Workload("cube50_compression_mixed", [50], [300.0], [1], [-1e-4], 10, 5000, 1,
                                             "500,000-atom cube, 10 x (-1e-4, 5000-step burst), mixed and FP64")
    temps = [100.0 + 400.0 * r / 63.0 for r in range(64)]
    w["ensemble64_cube15"] = Workload("ensemble64_cube15", [15] * 64, temps, list(range(1, 65)), [0.0] * 64, 1, 1000,
                                      1, "64 replicas of a 13,500-atom cube, 100-500 K, one 1000-step burst")
    r = rng(2026)
    edges = [int(e) for e in r.choice([10, 15, 20, 25, 30], size=16)]
    signs = [float(s) for s in r.choice([-1.0, 1.0], size=16)]
    w["uneven16"] = Workload("uneven16", edges, [300.0] * 16, list(range(101, 117)), [1e-4 * s for s in signs], 1,
                             2000, 1, "16 cubes of edges drawn from {10,15,20,25,30}, +-1e-4 each, 2000 steps")
    return w
