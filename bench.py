"""Benchmark of the MD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Headline workload: the Lennard-Jones fcc crystal of 80^3 cells (2,048,000
sites, density 0.8442) with random spherical voids (radius 3-8 sigma)
removing 40 % of the sites, about 1.23 M atoms, cutoff 2.5, skin 0.3,
dt 0.005, T* = 0.72.  One step = one velocity-Verlet step of the whole path
(kick+drift with the rebuild check, binning + neighbour lists whenever the
rule fires, LJ forces, kick), run by the library's native driver md_run.
value = atoms * K / wall time of K steps (inputs resident in HBM; warmup
steps untimed).

Printed: one JSON line with the metric, a roofline object for the dominant
kernel (the LJ force kernel, algorithmic bytes per launch / mean launch time
from HIP events on the launch stream), the FP64 oracle's rate on this host
(cpu_baseline) and the other workloads of the metric (EAM metal, FP64 LJ).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def recorded_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 counter runs
    (profiles/traffic.json), or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[key]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes"]


def _phase_ms(sim):
    out = {}
    for name, a, b in sim.events:
        out.setdefault(name, []).append(a.elapsed_time(b))
    return {k: (float(np.mean(v)), len(v)) for k, v in out.items()}


def run_workload(sim, steps, warmup, torch, phase_steps=20):
    """Warmup, then `steps` timed steps in the native driver (md_run), the
    force kernel bracketed by HIP events on its stream.  A short extra run
    through the per-call API records per-phase event times (untimed)."""
    sim.run(warmup)
    torch.cuda.synchronize()
    b0 = sim.builds
    t0 = time.perf_counter()
    force_ms, force_calls = sim.run(steps, timing=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rebuilds = sim.builds - b0
    sim.events = []
    for _ in range(phase_steps):
        sim.step()
    torch.cuda.synchronize()
    phases = _phase_ms(sim)
    sim.events = None
    return dict(seconds=t1 - t0, phases=phases, rebuilds=rebuilds,
                force_ms=force_ms / max(force_calls, 1), force_calls=force_calls)


def lj_force_bytes(n_atoms, n_entries):
    """Algorithmic bytes of one LJ force launch: each list entry once (4 B),
    each atom's row length (4 B), scaled position (16 B) and force (12 B)
    once."""
    return 4 * n_entries + (4 + 16 + 12) * n_atoms


def eam_force_bytes(n_atoms, n_entries):
    """Both EAM passes: list, row lengths and scaled positions read once per
    pass; rho, F' and the F' word of the scaled coordinates written (12 B);
    forces written (12 B)."""
    return 2 * 4 * n_entries + (2 * 4 + 2 * 16 + 12 + 12) * n_atoms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="all", choices=["all", "lj"])
    ap.add_argument("--cpu-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1611_00075_amd import inputs
    from paper_1611_00075_amd.sim import Simulation

    torch.cuda.set_device(0)
    # ---- headline: LJ with voids ------------------------------------------
    s = inputs.lj_voids()
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005)
    r = run_workload(sim, args.steps, args.warmup, torch)
    n = s.n
    value = n * args.steps / r["seconds"]
    f_ms = r["force_ms"]
    byt = lj_force_bytes(n, sim.n_pairs)
    achieved = byt / (f_ms * 1e-3) / 1e9
    result = {
        "metric": "atom-steps/sec at 1 MI355X (LJ, EAM, MLP vs EAM) + % roofline at stated force err",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "lj_fcc_80^3_voids_40pct",
            "atoms": n, "sites": s.meta["sites"], "voids": s.meta["voids"],
            "rc": 2.5, "skin": 0.3, "dt": 0.005, "T": 0.72,
            "list_entries": sim.n_pairs, "rebuilds": r["rebuilds"],
            "state": "f64 positions/velocities, f32 pair arithmetic and forces",
        },
        "roofline": {
            "bound": "hbm", "kernel": "k_lj32 (md_forces_lj)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("k_lj32_lj_voids_1.23M"),
            "bytes_per_launch": byt, "launch_ms": f_ms,
        },
        "phases_ms_per_call_api": {k: v[0] for k, v in r["phases"].items()},
    }
    del sim
    torch.cuda.empty_cache()

    if args.only == "all":
        extra = {}
        # ---- EAM metal, 4 M atoms ----------------------------------------
        s3 = inputs.eam_cu()
        sim3 = Simulation(s3.L, s3.x, s3.v, potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0,
                          mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        st3 = 200
        r3 = run_workload(sim3, st3, 10, torch)
        f3 = r3["force_ms"]
        b3 = eam_force_bytes(s3.n, sim3.n_pairs)
        extra["eam_cu_fcc_100^3"] = {
            "atoms": s3.n, "steps": st3, "value": s3.n * st3 / r3["seconds"], "unit": "atom-steps/s",
            "ms_per_step": 1e3 * r3["seconds"] / st3, "rebuilds": r3["rebuilds"],
            "forces_ms": f3, "forces_GBs": b3 / (f3 * 1e-3) / 1e9,
            "forces_frac_hbm": b3 / (f3 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "phases_ms_per_call_api": {k: v[0] for k, v in r3["phases"].items()},
        }
        del sim3
        torch.cuda.empty_cache()
        # ---- LJ crystal, 4,000 atoms, FP64 (launch-bound) -------------------
        s1 = inputs.lj_fcc()
        sim1 = Simulation(s1.L, s1.x, s1.v, skin=0.3, dt=0.005, pair_fp64=True)
        r1 = run_workload(sim1, 100, 10, torch)
        extra["lj_fcc_10^3_fp64"] = {
            "atoms": s1.n, "steps": 100, "value": s1.n * 100 / r1["seconds"], "unit": "atom-steps/s",
            "ms_per_step": 1e3 * r1["seconds"] / 100,
        }
        del sim1
        result["extra"] = extra

    if not args.no_cpu_baseline:
        import oracle
        k = args.cpu_steps
        ro = oracle.md_run(s.x.copy(), s.v.copy(), s.L, k, r_list=2.8, skin=0.3, dt=0.005)
        result["cpu_baseline"] = {
            "value": n * k / ro["loop_seconds"], "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle, {k} velocity-Verlet steps of the same {n}-atom void system after its "
                      f"initial list build (step loop timed alone), single thread",
        }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
