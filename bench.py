#!/usr/bin/env python3
"""Throughput of the PTA fast-MD hot path on one MI355X.

A benchmark step is one load step of the workload: an affine strain increment
along z (skipped where the workload holds the strain fixed) followed by one
averaging burst of velocity-Verlet EAM dynamics with the Berendsen
thermostat and on-device K / U / sigma_zz time averages.  The default
workload is the largest single-GPU one: the 500,000-atom cube (50^3 FCC
cells) in compression, 10 increments of -1e-4 each followed by a 5000-step
burst, mixed precision, with the same seed's FP64 run over the same load
steps beside it; the 62,500-atom cube in tension (20 x (+1e-4, 2000
steps)) is reported as a secondary line.  Other workloads (--workload) are
the 4,000-atom FP64 cube, the 64-replica ensemble and the 16 uneven cubes.

Prints one JSON line: atom-steps/s of the whole job; the roofline of the
dominant pair kernel and of the other, from their average durations
measured inside the timed region (the second step of every burst chunk is
launched directly, its density and force kernels bracketed by HIP events
on the library's stream); the FP64 run; the FP64 CPU oracle timed on a
bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic counts per unique pair within rc (FMA = 2 flops): the force
# term (separation 3, r^2 5, 1/r 1, r 1, powers 5, derivatives and shifts 6,
# pair energy 4, dU/dr 3, pair force 1, both atoms' force updates 12, energy
# 1) is 42 flops (the virial is formed per atom, z_i F_iz, not per pair);
# the density term (separation 3, r^2 5, (a/r)^2 from 1/r 2, its cube 2,
# sqrt 1, shift 3, both atoms' sums 1) is 17.
FLOPS_PER_PAIR = {"force": 42.0, "density": 17.0}
PEAK_TFLOPS = {1: 157.3, 0: 78.6}  # MI355X vector FP32 (mixed form) / FP64
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per atom-step: density pass reads x (24) and writes
# B' (8 FP64 / 4 FP32 rounded into the 128-byte mixed figure); force pass
# reads x (24), B' and v (24), writes v (24) and x (24).
BYTES_PER_ATOM_STEP = {0: 136.0, 1: 128.0}

PKG = os.path.join(ROOT, "paper_2603_07321_amd")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_kernels_traffic.json")
TUNING_FILE = os.path.join(PKG, "tuning.json")
KERNEL_SRC = os.path.join(PKG, "csrc", "kernels.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload: str, precision: int, lanes: int, skin: float, prune_every: int):
    """HBM bytes per launch of each pair kernel from the committed counter
    runs, or None where the kernel source, workload, launch shape, skin or
    pruning interval differs from the profiled one."""
    try:
        with open(TRAFFIC_FILE) as fh:
            recs = json.load(fh)
    except (OSError, ValueError):
        return None
    for t in recs.get("runs", []):
        if (t.get("kernels_hip_sha256_16") == kernel_source_hash() and t.get("workload") == workload
                and t.get("precision") == precision and t.get("lanes_per_atom") == lanes and t.get("skin") == skin
                and t.get("prune_every") == prune_every):
            return t.get("bytes_per_launch")
    return None


def stored_tuning(workload: str, precision: int):
    try:
        with open(TUNING_FILE) as fh:
            return json.load(fh).get(f"{workload}/{precision}")
    except (OSError, ValueError):
        return None


def run_workload(P, wl, precision, steps, warmup, burst, tune, stream, timing=True, lanes=0, skin=1.0,
                 tune_steps=400, eps=None, full_lists=0, prune_every=0):
    """Creates the workload's system, runs warm-up load steps, picks the
    launch configuration (tune: 'stored', 'probe' or 'off') and times
    `steps` load steps."""
    sc = P.sc_params() if eps is None else P.sc_params(eps=eps)
    chosen = None
    if tune == "stored":
        chosen = stored_tuning(wl.name, precision)
        if chosen:
            lanes, skin = chosen["lanes_per_atom"], chosen["skin"]
            full_lists, prune_every = (1, 0) if chosen["prune_every"] == 0 else (0, chosen["prune_every"])
    md = P.md_params(precision=precision, lanes_per_atom=lanes, skin=skin, full_lists=full_lists,
                     prune_every=prune_every)
    descs = [P.lattice_desc(nc, T0, seed) for nc, T0, seed in zip(wl.n_cells, wl.T0, wl.seeds)]
    if len(descs) > 1:
        sysm = P.System.batch(descs, sc=sc, md=md)
    else:
        sysm = P.System.cube(wl.n_cells[0], T0=wl.T0[0], seed=wl.seeds[0], sc=sc, md=md)
    sysm.set_stream(stream)
    strained = any(d != 0.0 for d in wl.d_eps)

    def load_step():
        if strained:
            sysm.apply_strain_increments(wl.d_eps)
        return sysm.run_fast_md(burst)

    # the kernel timing (direct launch of each chunk's first two steps) is on
    # from the start, so that the warm-up instantiates the graphs the timed
    # load steps launch
    if timing:
        sysm.kernel_timing(reset=True)
    for _ in range(warmup):
        load_step()
    # probed on the warmed-up state the timed load steps continue from (the
    # autotuner restores that state exactly, and leaves the graphs of its
    # choice instantiated); not timed
    probe = sysm.autotune(probe_steps=tune_steps, use_cache=False) if tune == "probe" else None
    if timing:
        sysm.kernel_timing(reset=True)
    info0 = sysm.info()
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        last = load_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = sysm.kernel_timing(reset=False) if timing else None
    info1 = sysm.info()
    cnt = sysm.count_pairs()
    return dict(sys=sysm, elapsed=t1 - t0, kt=kt, info0=info0, info1=info1, cnt=cnt, last=last,
                tune={"mode": tune, "stored": chosen, "probe": probe}, n_atoms=sysm.n_atoms())


def roofline_entry(kernel, ms, pairs, precision, traffic):
    flops = FLOPS_PER_PAIR[kernel] * pairs
    achieved = flops / (ms * 1e-3) / 1e12 if ms > 0 else None
    peak = PEAK_TFLOPS[precision]
    return {
        "kernel": kernel,
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": (achieved / peak) if achieved else None,
        "traffic": traffic,
        "kernel_avg_ms": ms,
        "kernel_avg_ms_source": "HIP events on the library's stream around the directly launched second step "
                                "of every burst chunk in the timed region",
        "flops_per_launch": flops,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed load steps (default: the workload's count)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube50_compression_mixed")
    ap.add_argument("--burst", type=int, default=None, help="MD steps per burst (default: the workload's)")
    ap.add_argument("--precision", type=int, default=None, help="1 mixed, 0 FP64 (default: the workload's)")
    ap.add_argument("--tune", choices=("stored", "probe", "off"), default="stored",
                    help="launch configuration: the autotuner's stored choice for this workload (default), a "
                         "fresh autotuner probe, or --lanes/--skin")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--skin", type=float, default=1.0, help="Verlet skin in A with --tune off")
    ap.add_argument("--tune-steps", type=int, default=400)
    ap.add_argument("--eps", type=float, default=None, help="Sutton-Chen eps in eV (default 0.0033147)")
    ap.add_argument("--full-lists", action="store_true", help="pair passes on the full Verlet lists every step")
    ap.add_argument("--prune-every", type=int, default=0,
                    help="with --tune off: a pruning pass every this many rebuild points (1-3; 0 = 1)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run of the same workload")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 load steps (default: as the mixed)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 62,500-atom secondary line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-device-probe", action="store_true",
                    help="skip the achievable copy and FMA rates measured after the timed region")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the timed region, copy this many MiB device-to-device (a known-size kernel "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    rank = int(os.environ.get("RANK", "0"))
    if args.gpus != 1 or world != 1:
        if rank == 0:
            print("bench.py measures one GPU only: the hot path runs on a single MI355X here (how it would "
                  "shard over more GPUs is a design note, not a measured run); use --gpus 1", file=sys.stderr)
        return 2

    import torch  # device memory and streams only

    import paper_2603_07321_amd as P
    import synth

    wls = synth.workloads()
    if args.workload not in wls:
        print(f"unknown workload {args.workload}; choose from {sorted(wls)}", file=sys.stderr)
        return 2
    wl = wls[args.workload]
    precision = wl.precision if args.precision is None else args.precision
    steps = wl.increments if args.steps is None else args.steps
    burst = wl.burst_steps if args.burst is None else args.burst
    stream = torch.cuda.current_stream()

    if args.copy_probe_mb > 0:
        nb = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)  # an elementwise kernel: reads and writes exactly nb * 4 bytes
        torch.cuda.synchronize()
        del src, dst

    fl = 1 if args.full_lists else 0
    r = run_workload(P, wl, precision, steps, args.warmup, burst, args.tune, stream, lanes=args.lanes,
                     skin=args.skin, tune_steps=args.tune_steps, eps=args.eps, full_lists=fl,
                     prune_every=args.prune_every)
    n_atoms = r["n_atoms"]
    value = n_atoms * burst * steps / r["elapsed"]
    lanes = r["info1"]["lanes_per_atom"]
    skin = r["info1"]["skin"]
    pairs = r["cnt"]["pairs_in_rc"]
    prune_every = r["info1"]["prune_every"]
    traffic = measured_traffic(args.workload, precision, lanes, skin, prune_every) or {}
    kt = r["kt"]
    kern = {
        "force": roofline_entry("force", kt["force_event_ms"], pairs, precision, traffic.get("force")),
        "density": roofline_entry("density", kt["density_event_ms"], pairs, precision, traffic.get("density")),
    }
    dom = max(kern, key=lambda k: kern[k]["kernel_avg_ms"])
    other = "density" if dom == "force" else "force"
    roofline = dict(kern[dom])
    roofline["kernel"] = {"force": "k_force", "density": "k_density"}[dom]
    roofline["kernel_launches_timed"] = kt["count"]
    roofline["force_in_kernel_span_ms"] = kt["force_ms"]
    roofline["other_pair_kernel"] = kern[other]
    roofline["unique_pairs_in_rc"] = pairs
    roofline["list_entries"] = r["cnt"]["list_entries"]
    roofline["pruned_list_entries"] = r["cnt"]["pruned_entries"]
    roofline["prune_radius_A"] = r["cnt"]["prune_radius"]
    dev = None if args.no_device_probe else P.measure_device(1 << 30, 10)
    if dev:
        # the dominant kernel against what FMA chains reach here (one FMA per
        # instruction: no packed FP32)
        reach = dev["fma64_TFLOPs"] if precision == 0 else dev["fma32_TFLOPs"]
        roofline["achievable_peak"] = reach
        roofline["frac_of_achievable"] = (roofline["achieved"] / reach) if roofline["achieved"] else None
    eps_note = "" if args.eps is None else f" (eps overridden: {args.eps} eV)"
    out = {
        "metric": "atom-steps/s (EAM force+integrate) and % HBM roofline; FP32-mixed vs FP64",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["elapsed"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-pair/f64-state" if precision == 1 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {wl.notes}; Sutton-Chen EAM (eps 0.0033147 eV, a 4.05 A, n 7, m 6, "
                        f"c 16.399, rc 8.1 A shifted force){eps_note}, velocity Verlet dt 1 fs, Berendsen tau 100 fs; "
                        f"at this eps the 300 K cube melts and thins out over the run",
            "atoms": n_atoms,
            "replicas": len(wl.n_cells),
            "load_steps": steps,
            "burst_steps": burst,
            "precision": "mixed" if precision == 1 else "fp64",
            "lanes_per_atom": lanes,
            "skin_A": skin,
            "prune_every": prune_every,
            "list_index_bits": r["info1"]["list_index_bits"],
            "atoms_with_32bit_lists": r["cnt"]["wide_atoms"],
            "tuning": r["tune"],
        },
        "hbm_frac_algorithmic": BYTES_PER_ATOM_STEP[precision] * value / 1e9 / HBM_PEAK_GBS,
        "roofline": roofline,
        "device_measured": dev,
        "run_stats": {
            "list_builds": r["info1"]["list_builds"] - r["info0"]["list_builds"],
            "sorts": r["info1"]["sorts"] - r["info0"]["sorts"],
            "rollbacks": r["info1"]["rollbacks"] - r["info0"]["rollbacks"],
            "directed_pairs_per_atom_at_end": 2.0 * pairs / n_atoms,
            "last_burst_replica0": r["last"][0] if r["last"] else None,
        },
    }
    r["sys"].close()

    if precision == 1 and not args.no_fp64:
        n64 = steps if args.fp64_steps is None else min(args.fp64_steps, steps)
        f = run_workload(P, wl, 0, n64, args.warmup, burst, args.tune, stream, timing=False,
                         tune_steps=args.tune_steps, eps=args.eps, full_lists=fl)
        v64 = n_atoms * burst * n64 / f["elapsed"]
        out["fp64"] = {"value": v64, "unit": "atom-steps/s", "load_steps": n64, "mixed_over_fp64": value / v64,
                       "lanes_per_atom": f["info1"]["lanes_per_atom"], "skin_A": f["info1"]["skin"],
                       "prune_every": f["info1"]["prune_every"], "tuning": f["tune"],
                       "last_burst_replica0": f["last"][0] if f["last"] else None}
        f["sys"].close()

    if args.workload == "cube50_compression_mixed" and not args.no_secondary:
        w2 = wls["cube25_tension_mixed"]
        s2 = run_workload(P, w2, w2.precision, w2.increments, 1, w2.burst_steps, args.tune, stream, timing=False,
                          tune_steps=args.tune_steps, eps=args.eps, full_lists=fl)
        out["secondary"] = {"workload": w2.name, "atoms": s2["n_atoms"],
                            "value": s2["n_atoms"] * w2.burst_steps * w2.increments / s2["elapsed"],
                            "unit": "atom-steps/s", "lanes_per_atom": s2["info1"]["lanes_per_atom"],
                            "skin_A": s2["info1"]["skin"], "prune_every": s2["info1"]["prune_every"],
                            "tuning": s2["tune"]}
        s2["sys"].close()

    if not args.no_cpu_baseline:
        import oracle as O
        nc = wl.n_cells[0]
        st = O.create_cube(nc, wl.T0[0], wl.seeds[0])
        if wl.d_eps[0] != 0.0:
            O.apply_strain(st, wl.d_eps[0])
        n0 = 4 * nc ** 3
        c0 = time.perf_counter()
        if n0 > 100000:
            # one force evaluation (density and force passes), which is what
            # one step of the oracle's burst costs (the integration is O(N))
            O.forces(st.x, st.y, st.z, O.sc_params(), st.group)
            nsteps, what = 1, "one force evaluation (density and force passes) of the strained cube, the cost of " \
                               "one step of the oracle's burst"
        else:
            nsteps = 3
            O.run_burst(st, O.sc_params(), O.md_params(T0=wl.T0[0]), nsteps)
            what = "one load step with a 3-step burst (burst-start force evaluation included)"
        c1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": n0 * nsteps / (c1 - c0),
            "unit": "atom-steps/s",
            "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"the first replica's cube ({n0} atoms): {what}; FP64, all-pairs loops",
            "seconds": c1 - c0,
        }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
