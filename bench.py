#!/usr/bin/env python3
"""Throughput of the PTA fast-MD hot path on one MI355X.

One benchmark step = one affine strain increment of the 62,500-atom cube
(25^3 FCC cells, Sutton-Chen EAM, +1e-4 along z) followed by one 2000-step
averaging burst (velocity Verlet, Berendsen 100 fs, on-device K/U/sigma_zz
time averages), in the mixed precision form.  The cube's whole job is 20 such
steps; the default run times exactly that.

Prints one JSON line: atom-steps/s of the burst, the roofline of the force
kernel (timed with HIP events on the library's stream inside the timed
region), and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic flop counts per unique pair within rc (FMA = 2 flops): the
# density term (distance, powers, shift, accumulation) and the force term
# (distance, powers, derivatives, shifts, pair force, both atoms' force
# updates, energy, virial)
FLOPS_DENSITY_PER_PAIR = 17.0
FLOPS_FORCE_PER_PAIR = 45.0
PEAK_TFLOPS = {1: 157.3, 0: 78.6}  # vector FP32 (mixed) / FP64, MI355X
HBM_PEAK_GBS = 8000.0
BYTES_PER_ATOM_STEP = {0: 136.0, 1: 128.0}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed load steps (strain increment + burst)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--burst", type=int, default=2000, help="MD steps per burst")
    ap.add_argument("--precision", type=int, default=1, help="1 mixed (default), 0 FP64")
    ap.add_argument("--cells", type=int, default=25)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the timed region, copy this many MiB device-to-device (a known-size kernel "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    rank = int(os.environ.get("RANK", "0"))
    if args.gpus != 1 or world != 1:
        if rank == 0:
            print("bench.py measures one GPU only: the hot path here runs on a single MI355X "
                  "(multi-GPU sharding is a design note, not part of this build); use --gpus 1", file=sys.stderr)
        return 2

    import torch  # device memory and streams only

    import paper_2603_07321_amd as P
    import synth

    wl = synth.workloads()["cube25_tension_mixed"]
    nc = args.cells
    d_eps = wl.d_eps[0]
    md = P.md_params(precision=args.precision, lanes_per_atom=args.lanes)
    sysm = P.System.cube(nc, T0=wl.T0[0], seed=wl.seeds[0], md=md)
    stream = torch.cuda.current_stream()
    sysm.set_stream(stream)
    n_atoms = sysm.n_atoms()
    if args.copy_probe_mb > 0:
        nb = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tune = None
    if not args.no_autotune:
        # warm-up work: probe bursts pick lanes per atom and skin, state restored
        tune = sysm.autotune(probe_steps=args.tune_steps)
    sysm.kernel_timing(reset=True)  # switches on the force-kernel events

    for _ in range(args.warmup):
        sysm.apply_strain_increment(d_eps)
        sysm.run_fast_md(args.burst)
    sysm.kernel_timing(reset=True)
    info0 = sysm.info()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        sysm.apply_strain_increment(d_eps)
        last = sysm.run_fast_md(args.burst)[0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0

    k_ms, k_count = sysm.kernel_timing(reset=False)
    info1 = sysm.info()
    pairs, entries = sysm.count_pairs()  # at the final positions
    atom_steps = n_atoms * args.burst * args.steps
    value = atom_steps / elapsed
    ms_per_step = elapsed / args.steps * 1e3

    flops_launch = FLOPS_FORCE_PER_PAIR * pairs
    achieved = flops_launch / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None
    peak = PEAK_TFLOPS[args.precision]
    roofline = {
        "kernel": "k_force",
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": (achieved / peak) if achieved else None,
        "traffic": None,
        "kernel_avg_ms": k_ms,
        "kernel_launches_timed": k_count,
        "flops_per_launch": flops_launch,
        "unique_pairs_in_rc": pairs,
        "list_entries": entries,
    }
    hbm_algo = BYTES_PER_ATOM_STEP[args.precision] * value / 1e9
    out = {
        "metric": "atom-steps/s (EAM force+integrate) and % HBM roofline; FP32-mixed vs FP64",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-pair/f64-state" if args.precision == 1 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"FCC Al cube {nc}^3 cells ({n_atoms} atoms), Sutton-Chen EAM rc 8.1 A shifted force, "
                        f"{args.steps} x (affine z strain {d_eps:+g}, {args.burst}-step burst, VV dt 1 fs, "
                        f"Berendsen 100 fs, 300 K)",
            "atoms": n_atoms,
            "burst_steps": args.burst,
            "precision": "mixed" if args.precision == 1 else "fp64",
            "lanes_per_atom": info1["lanes_per_atom"],
            "skin_A": info1["skin"],
            "autotune": tune,
        },
        "hbm_frac_algorithmic": hbm_algo / HBM_PEAK_GBS,
        "roofline": roofline,
        "run_stats": {
            "list_builds": info1["list_builds"] - info0["list_builds"],
            "sorts": info1["sorts"] - info0["sorts"],
            "rollbacks": info1["rollbacks"] - info0["rollbacks"],
            "last_burst": last,
        },
    }

    if not args.no_cpu_baseline:
        import oracle as O
        st = O.create_cube(nc, wl.T0[0], wl.seeds[0])
        O.apply_strain(st, d_eps)
        c0 = time.perf_counter()
        O.run_burst(st, O.sc_params(), O.md_params(), args.cpu_steps)
        c1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": n_atoms * args.cpu_steps / (c1 - c0),
            "unit": "atom-steps/s",
            "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"one strain increment + {args.cpu_steps}-step burst of the same {n_atoms}-atom cube "
                      f"(FP64, all-pairs loops, includes the burst-start force evaluation)",
            "seconds": c1 - c0,
        }
    print(json.dumps(out))
    sysm.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
