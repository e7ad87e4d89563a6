#!/usr/bin/env python
"""Benchmark of the ReaxFF force evaluation on one MI355X.

One step = one pass of the whole hot path over one synthetic configuration
already resident in HBM: reaxff_build_lists (cell sort, far/bond/H lists)
followed by reaxff_compute_forces (bond orders, every energy term, forces).
Workload: 1,044,000 atoms (36,000 C5H8N4O12 units) on a jittered simple-cubic
lattice in a periodic 220 A box, parameters drawn from seed 0.

Prints one JSON line: atom-steps/s, the per-kernel roofline fraction of the
dominant kernel (timed with HIP events on its launch stream over the timed
region), a phase breakdown (lists / bonded / nonbonded / backward) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Kernel work models.  nonbonded: FP64 operations per pair evaluation of the
# compiled inner loop (v_fma/v_fmac/v_div_fmas counted as 2, v_add, v_mul,
# v_rcp, v_rsq as 1; compares, conversions and exponent manipulation not
# counted), read from the gfx950 assembly of this library's own build.  Each
# unordered far pair is evaluated from both of its atoms.
WORK = {
    "nonbonded": ("pair_evaluations", 421.0),
}

# Measured HBM bytes per launch of a kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, scaled by the same counters' reading for a 1 GiB device copy),
# recorded in profiles/kernels_petn_1044000.md.  Valid only for the kernel
# version they were taken on; set to None when the kernel changes.
TRAFFIC = {
    "nonbonded": 3.470e9,
}

PHASES = {
    "lists": ("bbox", "cell_hist", "scan", "cell_scatter", "cell_sort", "gather_sorted",
              "list_sweep", "bondtest", "compact", "mirror"),
    "bonded": ("gather_q", "bo_prime", "delta_prime", "bo_corr", "atom_state", "atom_energy",
               "tasks", "angles", "torsions", "hbonds", "hb_acceptors"),
    "nonbonded": ("nonbonded",),
    "backward": ("back_s", "back_corr", "back_dp", "forces"),
}


def cpu_baseline(params, seconds_cap=60.0):
    """The oracle (single-threaded FP64, lists + forces) on a bounded sample of the
    workload: the same generator recipe and density at 32,480 atoms (1,120 units,
    69.2 A periodic box)."""
    import reaxff_synth as rs
    from oracle import Oracle
    s = rs.workload("petn_32480")
    t0 = time.perf_counter()
    o = Oracle(s, params)
    o.forces()
    t = time.perf_counter() - t0
    return {"value": s.n / t, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one oracle force evaluation (lists + energies + forces) on {s.n} atoms "
                      f"of the same recipe (1,120 units, 69.2 A box): {t:.2f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="petn_1044000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-kernel events (value only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by spatial decomposition, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import reaxff_synth as rs
    from paper_1706_07772_amd import ReaxFF
    from paper_1706_07772_amd.binding import load_library

    params = rs.draw_params(0)
    system = rs.workload(args.workload)
    n = system.n
    dev = torch.device("cuda:0")
    pos = torch.tensor(system.pos, dtype=torch.float64, device=dev)
    typ = torch.tensor(system.type, dtype=torch.int32, device=dev)
    q = torch.tensor(system.q, dtype=torch.float64, device=dev)
    box = [float(x) for x in system.box]
    ff = ReaxFF(params)
    forces = torch.empty((n, 3), dtype=torch.float64, device=dev)
    energies = torch.empty(12, dtype=torch.float64, device=dev)

    def step():
        ff.build_lists(pos, typ, box)
        ff.compute_forces(pos, typ, q, box, forces, energies)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({args.warmup} steps, n={n})", file=sys.stderr, flush=True)

    lib = load_library()
    import ctypes
    if not args.no_profile:
        lib.reaxff_profile.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        lib.reaxff_profile(ff._h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    ms_per_step = 1e3 * dt / args.steps
    value = n * args.steps / dt
    print(f"bench: timed {args.steps} steps, {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    counts = ff.interaction_counts()
    kernels = {}
    if not args.no_profile:
        K = 32
        ms = (ctypes.c_double * K)()
        calls = (ctypes.c_int64 * K)()
        names = (ctypes.c_char_p * K)()
        lib.reaxff_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]
        k = lib.reaxff_profile_read(ff._h, K, ms, calls, names)
        lib.reaxff_profile(ff._h, 0)
        for i in range(k):
            if calls[i]:
                kernels[names[i].decode()] = {"ms_total": ms[i], "launches": int(calls[i]),
                                              "ms_avg": ms[i] / calls[i]}
    phases = {}
    for ph, members in PHASES.items():
        phases[ph] = sum(kernels.get(m, {}).get("ms_total", 0.0) for m in members) / args.steps
    zero = kernels.get("zero", {}).get("ms_total", 0.0) / args.steps
    phases["memset"] = zero

    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
        avg_s = kernels[dom]["ms_avg"] * 1e-3
        if dom in WORK:
            unit, per = WORK[dom]
            units = 2 * counts["far_pairs"] if unit == "pair_evaluations" else counts.get(unit)
            if units:
                flops = per * units / (kernels[dom]["launches"] / args.steps)
                achieved = flops / avg_s / 1e12
                roofline = {"kernel": dom, "bound": "alu", "achieved": achieved,
                            "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                            "frac": achieved / PEAK_FP64_VALU_TFLOPS,
                            "traffic": TRAFFIC.get(dom),
                            "units_per_launch": units, "unit_name": unit,
                            "flops_per_unit": per, "avg_ms": kernels[dom]["ms_avg"]}
        if roofline is None:
            roofline = {"kernel": dom, "bound": "alu", "achieved": None,
                        "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s", "frac": None,
                        "traffic": None, "avg_ms": kernels[dom]["ms_avg"]}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(params)

    out = {
        "metric": "ReaxFF atom-steps/s at 1.04M atoms, FP64 plain vs surrogate at stated RMSE",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": n, "box_A": box[0],
                   "path": "plain FP64 ReaxFF: build_lists + compute_forces",
                   "cutoffs_A": {"nonbonded": 10.0, "bond": 5.0, "hbond": 7.5}, "bo_cut": 0.01},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases_ms": phases,
        "counts": counts,
        "kernels_ms_avg": {k: round(v["ms_avg"], 4) for k, v in kernels.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
