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
PEAK_BF16_MFMA_TFLOPS = 2500.0

# Algorithmic work per unit, in FP64 operation equivalents (add/mul = 1,
# fma = 2, exp 20, log 25, pow 60, div/sqrt 10, acos 40): fixed per-unit
# figures of the method's arithmetic, independent of how a kernel is built.
# Each unit is counted once per interaction (an unordered pair, a bond, an
# angle), with the interaction's energy and every force it contributes.
UNIT_FLOPS = {
    "far_candidates": 15.0,     # distance test of one candidate pair of the half stencil
    "far_pairs": 300.0,         # tapered vdW + shielded Coulomb pair, energy and force
    "bond_candidates": 260.0,   # uncorrected bond orders (3 pow + 3 exp) and derivatives
    "bonds": 500.0,             # bond-order correction, bond energy and its adjoint
    "atoms": 300.0,             # lone pair, over- and under-coordination
    "angles": 600.0,            # valence angle, penalty, coalition and adjoints
    "torsions": 500.0,          # torsion and conjugation and adjoints
    "hbonds": 150.0,            # hydrogen-bond triplet
}
# the dominant kernel's unit
WORK = {
    "nonbonded": ("far_pairs", UNIT_FLOPS["far_pairs"]),
}

# Measured HBM bytes per launch of a kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, scaled by the same counters' reading for a 1 GiB device copy),
# recorded in profiles/kernels_petn_1044000.md.  Valid only for the kernel
# version they were taken on; set to None when the kernel changes.
TRAFFIC = {
    "nonbonded": 1.628e9,
}
# the same counters summed over one dispatch of every kernel of a step
# (build_lists + compute_forces at 1,044,000 atoms)
WHOLE_STEP_TRAFFIC = 13.06e9

PHASES = {
    "lists": ("bbox", "cell_hist", "scan", "cell_scatter", "cell_sort", "gather_sorted",
              "list_sweep", "bondtest", "bond_merge", "compact", "mirror"),
    "bonded": ("gather_q", "bo_prime", "delta_prime", "bo_corr", "atom_state", "atom_energy",
               "tasks", "angles", "torsions", "hbonds", "hb_acceptors"),
    "nonbonded": ("nonbonded", "nb_reduce", "nb_energy"),
    "backward": ("back_s", "back_corr", "back_dp", "forces", "energy_fold"),
}


def host_info():
    """Host cores and CPU model of the machine the oracle is timed on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(params, reps=3):
    """The oracle (single-threaded FP64: lists, energies and forces) on a bounded
    sample of the workload: the same generator recipe, density and cutoffs at
    32,480 atoms (1,120 units, 69.2 A periodic box), median of `reps` runs, with
    the calling thread pinned to one core for the duration.  The oracle's work is
    linear in the atom count at fixed density, so its atom-steps/s carries over
    to the 1,044,000-atom workload (an extrapolation, labelled as such)."""
    import statistics

    import reaxff_synth as rs
    from oracle import Oracle
    s = rs.workload("petn_32480")
    info = host_info()
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            o = Oracle(s, params)
            o.forces()
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    t = statistics.median(times)
    return {"value": s.n / t, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "pinned_core": core, "host": info,
            "sample": f"oracle force evaluation (lists + energies + forces, one thread pinned to core "
                      f"{core}) on {s.n} atoms of the same recipe (1,120 units, 69.2 A box), median of "
                      f"{reps}: {t:.2f} s; rate per atom applied to 1,044,000 atoms is an extrapolation "
                      f"(work linear in atoms at fixed density)",
            "seconds": times}


def geometric_counts(system, r_bond=5.0, r_nonb=10.0):
    """Candidate counts the method's list construction must test, from the
    positions alone: unordered pairs within r_bond (bond candidates), and the
    unordered candidate pairs of a half stencil of +-2 cells of r_nonb/2."""
    import numpy as np
    from scipy.spatial import cKDTree
    box = np.asarray(system.box, dtype=np.float64)
    pos = np.mod(system.pos, box)
    n = system.n
    tree = cKDTree(pos, boxsize=box)
    bond_cand = (int(tree.count_neighbors(tree, r_bond)) - n) // 2
    nc = np.floor(box / (0.5 * r_nonb)).astype(int)
    idx = np.floor(pos / box * nc).astype(int) % nc
    m = np.zeros(nc)
    np.add.at(m, (idx[:, 0], idx[:, 1], idx[:, 2]), 1.0)
    S = np.zeros_like(m)
    for a in range(-2, 3):
        for b in range(-2, 3):
            for c in range(-2, 3):
                S += np.roll(m, (a, b, c), axis=(0, 1, 2))
    far_cand = int(((m * S).sum() - n) // 2)
    return {"bond_candidates": bond_cand, "far_candidates": far_cand}


def whole_step_work(counts, n):
    """Sum over the method's units of (FP64 ops per unit) x (units per step)."""
    units = dict(counts)
    units["atoms"] = n
    per = {k: UNIT_FLOPS[k] * units[k] for k in UNIT_FLOPS if k in units}
    return sum(per.values()), per


def read_profile(handle, lib):
    """Per-kernel event times accumulated by a context's profiler (reaxff_profile_read)."""
    import ctypes
    K = 64
    ms = (ctypes.c_double * K)()
    calls = (ctypes.c_int64 * K)()
    names = (ctypes.c_char_p * K)()
    lib.reaxff_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
    k = lib.reaxff_profile_read(handle, K, ms, calls, names)
    return {names[i].decode(): {"ms_total": ms[i], "launches": int(calls[i]), "ms_avg": ms[i] / calls[i]}
            for i in range(k) if calls[i]}


def bench_qeq(ff, n, far_pairs, traj, reps=3, tol=1e-6):
    """Charge equilibration over the lists of the 1,044,000-atom workload, with
    each product (reaxff_set_qeq_product): "auto" (matrix-free over the half far
    list, the default on this grid) and "stored" (H rows built once per call).
    Both systems by preconditioned CG from a zero start to the paper's relative
    residual of 1e-6, per-kernel times from a profiled pass; then along a
    trajectory (below).  The stored rows' product is HBM-bound: algorithmic
    bytes per product = stored entries x 12 B (index + value) + n x 40 B (both
    directions read, the product written, row length and type read).
    traj: (pos, type, q, box, velocities) of the workload."""
    import torch

    import reaxff_synth as rs
    from paper_1706_07772_amd.binding import load_library
    qp = rs.draw_qeq_params(0)
    lib = load_library()
    pos, typ, qq, box, vel = traj
    nnz = 2 * far_pairs

    def measure(mode):
        ff.set_qeq_product(mode)
        ff.build_lists(pos, typ, box)
        q, it, res = ff.qeq(n, qp, tol=tol, guess=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            q, it, res = ff.qeq(n, qp, tol=tol, guess=False, q=q)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        lib.reaxff_profile(ff._h, 1)
        for _ in range(reps):
            ff.qeq(n, qp, tol=tol, guess=False, q=q)
        torch.cuda.synchronize()
        kern = read_profile(ff._h, lib)
        lib.reaxff_profile(ff._h, 0)
        out = {"tol": tol, "iterations": it, "residuals": list(res), "ms_per_qeq": ms,
               "kernels_ms_avg": {k: round(v["ms_avg"], 4) for k, v in kern.items() if k.startswith("qeq")}}
        if "qeq_half" in kern:
            out["product"] = "matrix-free, half far list"
            out["ms_per_product"] = kern["qeq_half"]["ms_avg"] + kern["qeq_hreduce"]["ms_avg"]
        else:
            out["product"] = "stored rows"
            spmv = kern["qeq_spmv"]
            out["ms_per_product"] = spmv["ms_avg"]
            out["stored_entries"] = nnz
            byts = nnz * 12.0 + n * 40.0
            ach = byts / (spmv["ms_avg"] * 1e-3) / 1e9
            out["spmv_roofline"] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                    "frac": ach / PEAK_HBM_GBS, "bytes_per_launch": byts,
                                    "avg_ms": spmv["ms_avg"]}
        # along a trajectory, as an MD run uses it: one velocity-Verlet step
        # (dt 0.1 fs, lists rebuilt at the new positions), then the charges
        # from the extrapolation of the previous solutions
        P = pos.clone()
        V = vel.clone()
        ff.qeq(n, qp, tol=tol, guess=False)   # forget the zero-start solutions above
        its, times = [], []
        for _ in range(8):
            ff.step(P, V, typ, qq, box, 0.1, 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q, it, res = ff.qeq(n, qp, tol=tol, guess=True, q=q)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
            its.append(it)
        out["trajectory"] = {"steps": 8, "dt_fs": 0.1, "iterations": its,
                             "ms_per_qeq": times, "ms_per_qeq_last4": sum(times[-4:]) / 4}
        return out

    try:
        out = {"workload": "petn_1044000 positions of the force benchmark; chi, J from seed 0"}
        out.update(measure("auto"))
        out["stored"] = measure("stored")
    finally:
        ff.set_qeq_product("auto")
        ff.build_lists(pos, typ, box)
    return out


def bench_md(ff, params, steps=100, warmup_steps=5, workload="petn_32480", skin=0.0, every=10):
    """reaxff_step: velocity-Verlet NVE, dt 0.1 fs, on the 32,480-atom box (1,120
    C5H8N4O12 units in a 69.2 A periodic box) or another workload, Maxwell-Boltzmann
    velocities at 300 K; lists built every step, or with skin > 0 kept (Verlet
    skin, rebuilt every `every` steps or when an atom moved more than skin / 2);
    atom-steps/s over `steps` steps in one call."""
    import torch

    import reaxff_synth as rs
    from paper_1706_07772_amd import ReaxFF
    s = rs.workload(workload)
    ff = ReaxFF(params)
    if skin > 0:
        ff.set_skin(skin, every)
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=101)
    dev = torch.device("cuda:0")
    P = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    V = torch.tensor(v0, dtype=torch.float64, device=dev)
    T = torch.tensor(s.type, dtype=torch.int32, device=dev)
    Q = torch.tensor(s.q, dtype=torch.float64, device=dev)
    box = [float(x) for x in s.box]
    ff.step(P.clone(), V.clone(), T, Q, box, 0.1, warmup_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, en = ff.step(P, V, T, Q, box, 0.1, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = en.cpu().numpy()
    etot = e[:, :12].sum(1) + e[:, 12]
    stats = ff.list_stats()
    ff.close()
    lists = ("lists built every step" if skin <= 0 else
             f"Verlet-skin lists: skin {skin} A, rebuilt every {every} steps or on a move beyond skin/2")
    return {"workload": f"{workload}: {s.n} atoms, {s.box[0]} A periodic box, MB 300 K, dt 0.1 fs, {lists}",
            "list_builds_and_refreshes": list(stats),
            "steps": steps, "seconds": dt, "ms_per_step": 1e3 * dt / steps,
            "atom_steps_per_s": s.n * steps / dt,
            "energy_span_kcal": float(etot.max() - etot.min()),
            "kinetic_mean_kcal": float(e[:, 12].mean())}


def bench_batched(ff, steps: int, warmup: int):
    """4,096 non-periodic clusters (sizes uniform in 10-300, seed 3) in one persistent
    graph-replayed launch with the autotuned configuration, against the plain path on the
    same clusters (a) packed 40 A apart in one non-periodic system, (b) one plain
    build_lists + compute_forces call per cluster (timed on the first 256 clusters and
    scaled by atom count)."""
    import numpy as np
    import torch

    import reaxff_synth as rs
    from paper_1706_07772_amd import SCHEDULES, Batch

    dev = torch.device("cuda:0")
    pos, typ, q, off = rs.cluster_batch(4096, seed=3)
    natoms = int(off[-1])
    P = torch.tensor(pos, dtype=torch.float64, device=dev)
    T = torch.tensor(typ, dtype=torch.int32, device=dev)
    Q = torch.tensor(q, dtype=torch.float64, device=dev)
    b = Batch(ff, off)
    t0 = time.perf_counter()
    trials = b.tune(P, T, Q, reps=3)
    tune_s = time.perf_counter() - t0
    cfg = b.config
    print(f"bench: batch tuner {len(trials)} trials in {tune_s:.2f} s, best {cfg}", file=sys.stderr, flush=True)
    f, e = b.compute(P, T, Q)
    for _ in range(warmup):
        b.compute(P, T, Q, f, e)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    for _ in range(steps):
        b.compute(P, T, Q, f, e)
    ev1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / steps
    rc, bad = b.status()
    counts = b.counts().sum(0)
    b.close()

    # (a) the plain path on the packed system
    nc = off.size - 1
    side = int(np.ceil(nc ** (1.0 / 3.0)))
    g = np.stack(np.unravel_index(np.arange(nc), (side, side, side)), axis=1).astype(np.float64)
    sizes = np.diff(off)
    packed = pos + 40.0 * np.repeat(g, sizes, axis=0)
    PP = torch.tensor(packed, dtype=torch.float64, device=dev)
    fp = torch.empty_like(PP)
    ep = torch.empty(12, dtype=torch.float64, device=dev)

    def plain_step():
        ff.build_lists(PP, T, None)
        ff.compute_forces(PP, T, Q, None, fp, ep)

    for _ in range(warmup):
        plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_step()
    torch.cuda.synchronize()
    ms_packed = 1e3 * (time.perf_counter() - t0) / steps

    # (b) one plain call pair per cluster, first 256 clusters
    ns = 256
    subs = [(P[off[c]:off[c + 1]].contiguous(), T[off[c]:off[c + 1]].contiguous(),
             Q[off[c]:off[c + 1]].contiguous()) for c in range(ns)]
    outs = [(torch.empty_like(x), torch.empty(12, dtype=torch.float64, device=dev)) for x, _, _ in subs]
    for (x, t, qq), (fo, eo) in zip(subs, outs):
        ff.build_lists(x, t, None)
        ff.compute_forces(x, t, qq, None, fo, eo)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (x, t, qq), (fo, eo) in zip(subs, outs):
        ff.build_lists(x, t, None)
        ff.compute_forces(x, t, qq, None, fo, eo)
    torch.cuda.synchronize()
    sub_atoms = int(off[ns])
    loop_rate = sub_atoms / (time.perf_counter() - t0)

    rate = natoms / (ms * 1e-3)
    best_ms = min(t for _, t in trials)
    worst_ms = max(t for _, t in trials)
    return {
        "workload": "4,096 clusters, 10-300 atoms (uniform), non-periodic, seed 3",
        "atoms": natoms, "status": rc, "atom_steps_per_s": rate, "ms_per_launch": ms,
        "wall_ms_per_launch": 1e3 * wall / steps,
        "config": {"block": cfg[0], "schedule": SCHEDULES[cfg[1]], "wg_per_cu": cfg[2]},
        "tuner": {"trials": len(trials), "seconds": tune_s, "best_ms": best_ms, "worst_ms": worst_ms},
        "plain_packed": {"ms_per_step": ms_packed, "atom_steps_per_s": natoms / (ms_packed * 1e-3),
                          "speedup_of_batched": ms_packed / ms},
        "plain_loop": {"clusters_timed": ns, "atom_steps_per_s": loop_rate,
                       "speedup_of_batched": rate / loop_rate},
        "counts": {"angles": int(counts[0]), "torsions": int(counts[1]), "hbonds": int(counts[2]),
                   "far_pairs": int(counts[3]), "bonds": int(counts[4])},
        "kernel_stats": "profiles/batch_clusters_4096.md",
    }


def bench_surrogate(ff, params, steps: int, warmup: int, nframes: int = 20000):
    """Learned surrogate: an ensemble of 4 networks trained here by the library's own
    kernels, one Adam step per fresh frame, on `nframes` streamed frames of 1,856 atoms
    (the workload recipe -- stoichiometry, density, jittered lattice -- at 300-3000 K,
    each labelled by the plain GPU path as it arrives); force errors on 3 held-out frames
    against the CPU oracle; throughput at 1,044,000 atoms of the ensemble alone and of
    the gated evaluation (exact plain FP64 forces, through the masked evaluation, where
    the members disagree by more than 0.1 eV/A); the network kernel's share of the
    BF16 matrix-core peak."""
    import ctypes

    import numpy as np
    import torch

    import reaxff_synth as rs
    from oracle import Oracle
    from paper_1706_07772_amd import Surrogate
    from paper_1706_07772_amd import training as T
    from paper_1706_07772_amd.binding import load_library

    sur = Surrogate(ff, 4)
    info = T.train_streamed(sur, ff, T.FrameSource(64, seed=1000), nframes=nframes, lr=2e-3,
                            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    print(f"bench: surrogate trained on {nframes} streamed frames in {info['seconds']:.1f} s",
          file=sys.stderr, flush=True)
    held = T.FrameSource(64, seed=99)
    errs = []
    kcal = T.KCAL_PER_EV
    thr = 0.1 * kcal
    for _ in range(3):
        fr, temp = held.next()
        _, f_ref = Oracle(fr, params).forces()
        pos, typ, q, box = T.to_device(fr)
        ev = sur.evaluate(pos, typ, box)
        fg, mask, _, nf = sur.gated_forces(ff, pos, typ, q, box, thr)
        torch.cuda.synchronize()
        fm = ev["fmean"].cpu().numpy()
        fgn = fg.cpu().numpy()

        def rmse(a):
            return float(np.sqrt(((a - f_ref) ** 2).sum(1).mean())) / kcal

        errs.append({"temp_K": round(temp), "rmse_ensemble_ev": rmse(fm), "rmse_gated_ev": rmse(fgn),
                     "rmse_zero_ev": rmse(np.zeros_like(f_ref)), "fallback_fraction": nf / fr.n})
    # throughput at 1.04M atoms
    big = rs.workload("petn_1044000")
    pos, typ, q, box = T.to_device(big)
    n = big.n
    for _ in range(warmup):
        sur.evaluate(pos, typ, box)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sur.evaluate(pos, typ, box)
    torch.cuda.synchronize()
    ms_sur = 1e3 * (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    nfl = 0
    gsteps = max(1, steps // 2)
    for _ in range(gsteps):
        _, _, _, nfl = sur.gated_forces(ff, pos, typ, q, box, thr)
    torch.cuda.synchronize()
    ms_gated = 1e3 * (time.perf_counter() - t0) / gsteps
    nsub = sur.last_nsub
    # per-kernel times of one evaluation (events on the launch stream), and the
    # network kernel against the BF16 matrix-core peak: per atom and member the
    # forward products (224x128, 128x128, 128) and their transposes for dE/dx
    lib = load_library()
    sctx = lib.reaxff_surrogate_context(sur._h)
    lib.reaxff_profile(sctx, 1)
    for _ in range(steps):
        sur.evaluate(pos, typ, box)
    torch.cuda.synchronize()
    kern = read_profile(ctypes.c_void_p(sctx), lib)
    lib.reaxff_profile(sctx, 0)
    net_flops_atom = 2 * 2 * (224 * 128 + 128 * 128 + 128)
    net = kern.get("sur_net", {})
    mfma = None
    if net:
        fl = net_flops_atom * n * sur.members
        ach = fl / (net["ms_avg"] * 1e-3) / 1e12
        mfma = {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_BF16_MFMA_TFLOPS, "flops_per_atom_member": net_flops_atom,
                "avg_ms": net["ms_avg"]}
    sur.close()
    return {
        "ensemble": "4 members, 224 -> 128 -> 128 -> 1 SiLU per element, BF16 MFMA, FP32 accumulation",
        "training": {"frames_streamed": nframes, "atoms_per_frame": info["atoms_per_frame"],
                     "atom_environments": nframes * info["atoms_per_frame"],
                     "seconds": info["seconds"], "ms_per_frame": info["ms_per_frame"],
                     "final_loss": info["losses"][-1][1]},
        "heldout_vs_oracle": errs,
        "atoms": n,
        "ensemble_ms_per_step": ms_sur, "ensemble_atom_steps_per_s": n / (ms_sur * 1e-3),
        "gated_ms_per_step": ms_gated, "gated_atom_steps_per_s": n / (ms_gated * 1e-3),
        "gated_fallback_fraction": nfl / n, "gated_plain_subsystem_atoms": nsub, "threshold_ev_per_A": 0.1,
        "kernels_ms_avg": {k: round(v["ms_avg"], 4) for k, v in kern.items()},
        "network_mfma_roofline": mfma,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="petn_1044000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the nonbonded and bonded terms in order in the throughput pass too")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-kernel events (value only)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-clusters measurement")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched-clusters measurement (for profiling)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate measurement")
    ap.add_argument("--no-md", action="store_true", help="skip the 32,480-atom MD measurement")
    ap.add_argument("--no-qeq", action="store_true", help="skip the charge-equilibration measurement")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate measurement (for profiling)")
    ap.add_argument("--surrogate-frames", type=int, default=20000,
                    help="streamed training frames of the surrogate (fewer only to profile its kernels)")
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
    if args.batched_only:
        ff = ReaxFF(params)
        out = bench_batched(ff, args.steps, args.warmup)
        print(json.dumps({"batched": out}), flush=True)
        return
    if args.surrogate_only:
        ff = ReaxFF(params)
        out = bench_surrogate(ff, params, args.steps, args.warmup, nframes=args.surrogate_frames)
        print(json.dumps({"surrogate": out}), flush=True)
        return
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

    ff.set_overlap(not args.no_overlap)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({args.warmup} steps, n={n})", file=sys.stderr, flush=True)

    lib = load_library()
    import ctypes
    # throughput pass: the steps as a user runs them (nonbonded term concurrent
    # with the bonded terms unless --no-overlap), no per-kernel events
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
    kernel_pass_ms = None
    if not args.no_profile:
        # kernel pass: the same number of steps with every kernel in order on
        # one stream, each bracketed by HIP events on that stream, so each
        # kernel's time is its own (under overlap a kernel's interval would
        # include the concurrent terms' share of the chip)
        ff.set_overlap(False)
        lib.reaxff_profile.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        lib.reaxff_profile(ff._h, 1)
        torch.cuda.synchronize()
        tk0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        kernel_pass_ms = 1e3 * (time.perf_counter() - tk0) / args.steps
        ff.set_overlap(not args.no_overlap)
        print(f"bench: kernel pass {kernel_pass_ms:.3f} ms/step (terms in order)", file=sys.stderr, flush=True)
        K = 64
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
            units = counts.get(unit)
            if units:
                flops = per * units / (kernels[dom]["launches"] / args.steps)
                achieved = flops / avg_s / 1e12
                roofline = {"kernel": dom, "bound": "alu", "achieved": achieved,
                            "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                            "frac": achieved / PEAK_FP64_VALU_TFLOPS,
                            "traffic": TRAFFIC.get(dom),
                            "units_per_launch": units, "unit_name": unit,
                            "flops_per_unit": per, "avg_ms": kernels[dom]["ms_avg"],
                            "measured": "kernel pass: same steps, terms in order on one stream"}
                # the whole nonbonded term: the pair kernel and, in the half
                # evaluation, the per-atom sum of the cells' partial forces
                extra = [kernels[k]["ms_avg"] for k in ("nb_reduce", "nb_energy") if k in kernels]
                if dom == "nonbonded" and extra:
                    term_ms = kernels[dom]["ms_avg"] + sum(extra)
                    roofline["term_ms"] = term_ms
                    roofline["term_frac"] = flops / (term_ms * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS
        if roofline is None:
            roofline = {"kernel": dom, "bound": "alu", "achieved": None,
                        "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s", "frac": None,
                        "traffic": None, "avg_ms": kernels[dom]["ms_avg"]}

    # whole step against the FP64 vector peak: the method's per-unit work
    # (UNIT_FLOPS) times the units of one step, over the measured step time
    geo = geometric_counts(system)
    work, per_unit = whole_step_work({**counts, **geo}, n)
    whole = {"gflop_eq": work / 1e9, "achieved_tflops": work / (ms_per_step * 1e-3) / 1e12,
             "traffic": WHOLE_STEP_TRAFFIC if args.workload == "petn_1044000" else None,
             "peak": PEAK_FP64_VALU_TFLOPS, "frac": work / (ms_per_step * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS,
             "units": {k: {"count": int(v / UNIT_FLOPS[k]), "flops_per_unit": UNIT_FLOPS[k]}
                       for k, v in per_unit.items()}}

    qeq = None
    if not args.no_qeq:
        print("bench: charge equilibration", file=sys.stderr, flush=True)
        ff.set_overlap(not args.no_overlap)
        step()
        v0 = rs.maxwell_boltzmann(system.type, params.atom["mass"], 300.0, seed=103)
        qeq = bench_qeq(ff, n, counts["far_pairs"],
                        (pos, typ, q, box, torch.tensor(v0, dtype=torch.float64, device=dev)))

    md = None
    if not args.no_md:
        print("bench: MD steps (32,480 atoms; 1,044,000 with skin lists)", file=sys.stderr, flush=True)
        md = {"exact_lists": bench_md(ff, params),
              "skin_lists": bench_md(ff, params, skin=0.5, every=10),
              "skin_lists_1044000": bench_md(ff, params, steps=20, warmup_steps=2, workload="petn_1044000",
                                             skin=0.5, every=10)}

    batched = None
    if not args.no_batched:
        print("bench: batched clusters", file=sys.stderr, flush=True)
        batched = bench_batched(ff, args.steps, args.warmup)

    surrogate = None
    if not args.no_surrogate:
        print("bench: surrogate", file=sys.stderr, flush=True)
        surrogate = bench_surrogate(ff, params, args.steps, args.warmup, nframes=args.surrogate_frames)

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
                   "overlap": not args.no_overlap,
                   "cutoffs_A": {"nonbonded": 10.0, "bond": 5.0, "hbond": 7.5}, "bo_cut": 0.01},
        "roofline": roofline,
        "whole_step_roofline": whole,
        "cpu_baseline": cpu,
        "md": md,
        "qeq": qeq,
        "batched": batched,
        "surrogate": surrogate,
        "phases_ms": phases,
        "kernel_pass_ms_per_step": kernel_pass_ms,
        "counts": counts,
        "kernels_ms_avg": {k: round(v["ms_avg"], 4) for k, v in kernels.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
