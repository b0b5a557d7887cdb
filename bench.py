"""Benchmark of the MD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--reps R] [--no-cpu-baseline]
    python bench.py --counters DIR[,DIR...]     (no GPU: rocprofv3 counter
                                                 CSVs -> profiles/traffic.json)

Headline workload: the Lennard-Jones fcc crystal of 80^3 cells (2,048,000
sites, density 0.8442) with random spherical voids (radius 3-8 sigma)
removing 40 % of the sites, about 1.23 M atoms, cutoff 2.5, skin 0.3,
dt 0.005, T* = 0.72.  One step = one velocity-Verlet step of the whole path
(kick+drift with the rebuild check, binning + neighbour lists whenever the
rule fires, LJ forces, kick), run by the library's native driver md_run.
Each leg is timed R times (default 5, the paper's protocol): W untimed
warmup steps, then R runs of exactly K steps, each bracketed by device
synchronisations; value = atoms * K / wall time, mean over the R runs
(std beside it).  Inputs are resident in HBM before the timed region.

Printed: one JSON line with the metric, a roofline object for the dominant
kernel (the LJ force kernel: algorithmic bytes per launch / mean launch time
from HIP events on the launch stream, against the published 8 TB/s and the
copy rate measured in the same run), the FP64 oracle's rate on this host's
cores (cpu_baseline: one thread and all cores), the measured peaks of this
GPU (vector FMA loops, a matrix-core loop, a device copy) and the other
workloads of the metric (EAM metal, tight-binding, tabulated and two-element
forms, the decomposed force step, the 32 M-atom slab with its own roofline,
FP64 LJ, the learned potential in its BF16 and FP32-activation forms).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# published MI355X peaks (dense): FP32 vector 157.3 TFLOP/s counts packed
# FP32 instructions, which this build does not use (78.6 without them); FP64
# vector 78.6 TFLOP/s; BF16 matrix 2.5 PFLOP/s
FP32_VALU_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2500.0
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


# --------------------------------------------------------------------------
# committed counter figures (profiles/traffic.json)
# --------------------------------------------------------------------------

def _sources_sha(sources):
    h = hashlib.sha256()
    for src in sources:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def recorded(key, field="traffic_bytes"):
    """A figure from the committed rocprofv3 counter runs (HBM bytes per
    launch, VALU instructions per CU per clock, ...), or None when a source
    of the kernel has changed since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC))[key]
        if _sources_sha(rec["sources"]) != rec["sources_sha256"]:
            return None
    except (OSError, KeyError, ValueError):
        return None
    return rec.get(field)


def recorded_traffic(key):
    return recorded(key, "traffic_bytes")


def recorded_pair(k1, k2, field="traffic_bytes"):
    a, b = recorded(k1, field), recorded(k2, field)
    return None if a is None or b is None else a + b


def valu_frac(key):
    """Fraction of the vector ALU's issue cycles a kernel used: VALU issue
    events (SQ_INSTS_VALU less the dual-issued second instructions,
    SQ_ACTIVE_INST_VALU2) over the 4 SIMDs' quad-cycles of the dispatch, so
    at most 1; or None.  The FP32 FMA loop reaches the value recorded for
    k_probe_fma_f32 (about 0.88)."""
    return recorded(key, "valu_issue_frac")


def ta_frac(key):
    """Fraction of the dispatch's cycles the CUs' texture addressers (which
    process every vector-memory address) were busy, or None."""
    return recorded(key, "ta_busy_per_cu_clk")


def mfma_frac(key):
    """Matrix-core busy cycles of a kernel over the same figure for the BF16
    matrix-core loop (which reaches the published BF16 rate), or None."""
    k, p = recorded(key, "mfma_busy_per_cu_clk"), recorded("k_probe_mfma", "mfma_busy_per_cu_clk")
    return None if k is None or not p else k / p


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# timing
# --------------------------------------------------------------------------

def _phase_ms(sim):
    out = {}
    for name, a, b in sim.events:
        out.setdefault(name, []).append(a.elapsed_time(b))
    return {k: (float(np.mean(v)), len(v)) for k, v in out.items()}


def _stats(v):
    v = np.asarray(v, dtype=np.float64)
    return float(v.mean()), float(v.std(ddof=1)) if len(v) > 1 else 0.0


def run_workload(sim, steps, warmup, reps, torch, phase_steps=20):
    """Warmup, then `reps` runs of exactly `steps` steps in the native driver
    (md_run), each bracketed by device synchronisations, the force kernels
    bracketed by HIP events on their stream.  A short extra run through the
    per-call API records per-phase event times (untimed)."""
    sim.run(warmup)
    torch.cuda.synchronize()
    secs, fms, builds = [], [], []
    for _ in range(reps):
        b0 = sim.builds
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        force_ms, force_calls = sim.run(steps, timing=True)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        fms.append(force_ms / max(force_calls, 1))
        builds.append(sim.builds - b0)
    sim.events = []
    for _ in range(phase_steps):
        sim.step()
    torch.cuda.synchronize()
    phases = _phase_ms(sim)
    sim.events = None
    return dict(seconds=secs, force_ms=fms, rebuilds=builds, phases=phases)


def leg_stats(n, steps, r):
    """atom-steps/s, ms per step and force-kernel ms: mean and std over the runs."""
    v, vs = _stats([n * steps / t for t in r["seconds"]])
    m, ms = _stats([1e3 * t / steps for t in r["seconds"]])
    f, fs = _stats(r["force_ms"])
    return {"atoms": n, "steps": steps, "reps": len(r["seconds"]), "value": v, "value_std": vs,
            "unit": "atom-steps/s", "ms_per_step": m, "ms_per_step_std": ms, "forces_ms": f, "forces_ms_std": fs,
            "rebuilds_per_run": r["rebuilds"]}


def lj_force_bytes(n_atoms, n_entries):
    """Algorithmic bytes of one LJ force launch (the LJ row of the method's
    byte count): each list entry once (4 B), each atom's position (24 B of
    FP64 state) read and its force (12 B) written once."""
    return 4 * n_entries + (24 + 12) * n_atoms


def eam_force_bytes(n_atoms, n_entries):
    """Both embedded-atom passes: the list read in each pass (2 x 4 B per
    entry), positions in each pass (2 x 24 B), rho and F' (16 B) and the
    force (12 B) per atom."""
    return 2 * 4 * n_entries + (2 * 24 + 16 + 12) * n_atoms


def roofline_hbm(kernel, byt, ms, copy_gbs, traffic, keys):
    """HBM roofline of one launch (or one pair of passes) with the counter
    fractions of its kernels (profile keys, in launch order)."""
    a = byt / (ms * 1e-3) / 1e9
    one = len(keys) == 1
    valu = [valu_frac(k) for k in keys]
    ta = [ta_frac(k) for k in keys]
    return {"bound": "hbm", "kernel": kernel, "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": a / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": byt, "launch_ms": ms,
            "copy_GBs": copy_gbs, "frac_of_copy": a / copy_gbs if copy_gbs else None,
            "valu_issue_frac": valu[0] if one else valu, "texture_addresser_busy_frac": ta[0] if one else ta}


def mlp_force_flops(n_atoms, n_in, n_entries):
    """Algorithmic FP32 operations of the two MLP force passes (FMA = 2).
    Pass 1 tests every listed pair against the descriptor cutoff (7) and,
    per pair within it, forms the 16 Gaussians from three exponentials (37),
    the cutoff function (16) and the 16 descriptor sums (32).  Pass 2 walks
    the compact list of in-range pairs pass 1 wrote: per pair the distance
    (7), the Gaussians, the cutoff and its derivative (52), the 16
    coefficients and the two weighted sums over them (80) and the force and
    its accumulation (10).  Per atom, pass 1 runs the network forward and
    backward on the matrix cores: 4 x 5,120 multiply-adds = 20,480 BF16
    operations.  Returns (pass-1 VALU, pass-2 VALU, pass-1 matrix)."""
    return (7 * n_entries + 85 * n_in, (7 + 186) * n_in, 20480 * n_atoms)


# --------------------------------------------------------------------------
# measured peaks of this GPU
# --------------------------------------------------------------------------

def copy_bandwidth(torch, gib=2, reps=10):
    """Achievable HBM rate: a device-to-device copy of `gib` GiB (read +
    write counted), timed with HIP events."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def measured_peaks(torch):
    """The library's probe kernels (vector FMA loops in FP32 and FP64, a
    BF16 matrix-core loop) and a device copy, timed with HIP events."""
    from paper_1611_00075_amd import md as M
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    blocks = 256 * 8
    res = {}
    for name, kind, iters, work in (
            ("fp32_fma_TFLOPs", M.MD_PROBE_FMA_F32, 20000, lambda it: blocks * 256 * it * 8 * 2),
            ("fp64_fma_TFLOPs", M.MD_PROBE_FMA_F64, 20000, lambda it: blocks * 256 * it * 8 * 2),
            ("bf16_mfma_TFLOPs", M.MD_PROBE_MFMA_BF16, 2000, lambda it: blocks * 4 * it * 8 * 16384)):
        M.md_probe(kind, iters // 10, blocks, out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        M.md_probe(kind, iters, blocks, out)
        e1.record(st)
        torch.cuda.synchronize()
        res[name] = work(iters) / (e0.elapsed_time(e1) * 1e-3) / 1e12
    res["copy_GBs"] = copy_bandwidth(torch)
    return res


# --------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on this host
# --------------------------------------------------------------------------

def cpu_identity():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, cores


def cpu_baseline(s, steps1, steps_all):
    """The oracle's velocity-Verlet loop on the headline system after its
    initial list build: one thread, then OpenMP over atoms on all of this
    process's cores (at most 16, the host share of one GPU)."""
    import oracle
    model, cores = cpu_identity()
    threads = max(1, min(16, cores))
    t0 = time.perf_counter()
    r1 = oracle.md_run(s.x.copy(), s.v.copy(), s.L, steps1, r_list=2.8, skin=0.3, dt=0.005)
    t1 = time.perf_counter()
    rn = oracle.md_run(s.x.copy(), s.v.copy(), s.L, steps_all, r_list=2.8, skin=0.3, dt=0.005, threads=threads)
    t2 = time.perf_counter()
    n = len(s.x)
    v1 = n * steps1 / r1["loop_seconds"]
    vn = n * steps_all / rn["loop_seconds"]
    return {
        "value": vn, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
        "single_thread_value": v1,
        "sample": f"FP64 oracle (full-list LJ rows, cell-list builds, velocity Verlet with the displacement "
                  f"rule) on the same {n}-atom void system: {steps_all} steps on {threads} OpenMP threads "
                  f"({rn['builds'] - 1} rebuilds) and {steps1} steps on one thread ({r1['builds'] - 1} "
                  f"rebuilds), each after its initial list build; step loops timed alone",
        "cpu_model": model, "nproc": cores, "compiler": oracle.COMPILER_FLAGS,
        "wall_seconds": {"single_thread_run": t1 - t0, "all_core_run": t2 - t1},
    }


# --------------------------------------------------------------------------
# legs
# --------------------------------------------------------------------------

def pairs_within(sim, rc, torch, chunk=131072):
    """Number of list entries closer than rc (a measurement aid: torch
    gathers over the sliced-ELL rows, chunk by chunk)."""
    from paper_1611_00075_amd import md as M
    n, cap = sim.n, sim.row_cap
    rows = sim.idx[: M.ell_size(n, cap)].view(-1, cap // 8, 8, 8).permute(0, 2, 1, 3).reshape(-1, cap)[:n]
    cnt = sim.count[:n]
    L = torch.tensor(sim.L, dtype=torch.float64, device=sim.x.device).view(3, 1, 1)
    total = 0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        r = rows[a:b].long()
        valid = torch.arange(cap, device=r.device)[None, :] < cnt[a:b, None]
        d = sim.x[:, r.clamp_(0, n - 1)] - sim.x[:, a:b, None]
        d -= L * torch.round(d / L)
        total += int(((d * d).sum(0) < rc * rc).logical_and_(valid).sum())
    return total


def mlp_leg(torch, steps, warmup, reps, n_snap, epochs, equil, thermal):
    """Learned potential (Cu surrogate): training data from the GPU's own
    EAM trajectories, training on the GPU, then the 4 M-atom crystal of the
    EAM workload run with MLP forces in the BF16 and the FP32-activation
    forms."""
    from paper_1611_00075_amd import inputs, md as M
    from paper_1611_00075_amd import mlp as P
    from paper_1611_00075_amd.sim import Simulation
    out = {}
    t0 = time.perf_counter()
    temps = P.training_temperatures()
    keep = n_snap - max(1, n_snap // 10)
    snaps = [P.eam_trajectory(float(T), n_snap, seed=3000 + k, keep_from=keep, equil_steps=equil)
             for k, T in enumerate(temps)]
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"MLP: data in {t_data:.1f} s, training")
    Gtr, etr, Gte, ete = P.split(snaps)
    mean, inv = P.normalisation(Gtr)
    sp = P.spec(mean, inv)
    tr = P.Trainer(Gtr, etr, sp, P.init_params(5, e_mean=float(etr.double().mean())), batch=4096, seed=5)
    t1 = time.perf_counter()
    hist = tr.fit(epochs, lr=3e-3, lr_min=3e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    pot = tr.potential
    e_rmse = P.rmse(P.predict(Gte, pot), ete)
    fe, fm = [], []
    for sn in snaps:
        for k in range(0, len(sn.x), 5):
            fe.append(sn.f[k])
            fm.append(P.mlp_forces(pot, sn.L, sn.x[k]))
    fe, fm = np.concatenate(fe), np.concatenate(fm)
    out["training"] = {
        "snapshots": int(sum(s.G.shape[0] for s in snaps)), "atoms_per_snapshot": int(snaps[0].G.shape[1]),
        "temperatures_K": [float(temps[0]), float(temps[-1]), len(temps)],
        "train_rows": int(Gtr.shape[0]), "test_rows": int(Gte.shape[0]), "epochs": epochs, "batch": 4096,
        "steps": tr.step, "data_seconds": t_data, "train_seconds": t_train,
        "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
        "heldout_energy_rmse_eV": e_rmse,
        "heldout_force_rmse_eV_A": float(np.sqrt(np.mean((fm - fe) ** 2))),
        "heldout_force_rms_eam_eV_A": float(np.sqrt(np.mean(fe ** 2))),
    }
    del snaps, Gtr, etr, Gte, ete
    torch.cuda.empty_cache()
    x_th, f_th, T_th = thermal
    s = inputs.eam_cu()
    n = s.n
    for form, fp32 in (("bf16", False), ("fp32_activations", True)):
        spf = P.spec(mean, inv, fp32_activations=fp32)
        log(f"MLP ({form}): 4 M-atom run")
        sim = Simulation(s.L, s.x, s.v, potential="mlp", mlp=spf, mlp_w=pot.w, skin=1.0, dt=1.0,
                         mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        # forces on a thermalised configuration of the EAM run
        f_m = P.mlp_forces(P.Potential(spec=spf, w=pot.w), s.L, x_th) if fp32 else P.mlp_forces(pot, s.L, x_th)
        frmse = float(np.sqrt(np.mean((f_m - f_th) ** 2)))
        frms = float(np.sqrt(np.mean(f_th ** 2)))
        del f_m
        ep0, ek0 = sim.energies()
        r = run_workload(sim, steps, warmup, reps, torch)
        ep1, ek1 = sim.energies()
        res = leg_stats(n, steps, r)
        res.update({
            "force_rmse_vs_eam_eV_A": frmse, "force_rms_eam_eV_A": frms,
            "force_config": f"EAM trajectory of the same crystal after its timed steps, T = {T_th:.0f} K",
            "energy_drift_eV_per_atom": ((ep1 + ek1) - (ep0 + ek0)) / n,
            "drift_steps": warmup + reps * steps + 20,
            "drift_fs": float((warmup + reps * steps + 20) * 1.0),
        })
        if not fp32:
            # pass 2 alone (dE/dG reused), then both passes, timed with HIP events
            st = torch.cuda.current_stream()
            ms = {}
            calls = {
                "both": lambda: M.md_forces_mlp(sim.L, n, sim.xs, sim.row_cap, sim.idx, sim.count, sim.mlp,
                                                sim.mlp_w, sim.dEdG, sim.idx_in, sim.cnt_in, None, sim.f, sim.ev, 0,
                                                sim.ws),
                "pass2": lambda: M.md_forces_mlp(sim.L, n, sim.xs, sim.row_cap, sim.idx_in, sim.cnt_in, sim.mlp,
                                                 None, sim.dEdG, None, None, None, sim.f, sim.ev, M.MD_MLP_REUSE,
                                                 sim.ws),
            }
            G = torch.empty((n, P.N_IN), dtype=torch.float32, device=sim.dev)
            dG, eG = torch.empty_like(G), torch.empty(n, dtype=torch.float32, device=sim.dev)
            M.md_mlp_descriptors(sim.L, n, sim.xs, sim.row_cap, sim.idx, sim.count, sim.mlp, G)
            calls["net"] = lambda: M.md_mlp_eval(n, G, sim.mlp, sim.mlp_w, eG, dG)
            for name in ("both", "pass2", "net"):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                calls[name]()
                a.record(st)
                for _ in range(10):
                    calls[name]()
                b.record(st)
                torch.cuda.synchronize()
                ms[name] = a.elapsed_time(b) / 10
            del G, dG, eG
            entries = sim.n_pairs
            within = pairs_within(sim, float(spf.rc), torch)
            v1, v2, mfma = mlp_force_flops(n, within, entries)
            res.update({"pass1_ms": ms["both"] - ms["pass2"], "pass2_ms": ms["pass2"], "net_ms": ms["net"],
                        "list_entries": entries, "pairs_within_rc": within, "pass1_valu_flops": v1,
                        "pass2_valu_flops": v2, "pass1_mfma_flops": mfma,
                        "phases_ms_per_call_api": {k: v[0] for k, v in r["phases"].items()}})
        out[form] = res
        del sim
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="all", choices=["all", "lj", "mlp", "peaks"])
    ap.add_argument("--mlp-snapshots", type=int, default=1250, help="snapshots per temperature (16 temperatures)")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--mlp-equil", type=int, default=2000, help="equilibration steps per temperature")
    ap.add_argument("--mlp-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=3, help="single-thread oracle steps")
    ap.add_argument("--cpu-all-steps", type=int, default=20, help="all-core oracle steps")
    ap.add_argument("--trace-summary", help="rocprofv3 --kernel-trace output directory: print a per-kernel table")
    ap.add_argument("--nb-candidates", choices=["voids", "cu54"],
                    help="CPU model of the neighbour build's candidate counts on a benchmark system")
    ap.add_argument("--dd-overlap", help="rocprofv3 --kernel-trace output directory of decomposed force "
                                         "evaluations: print the halo/compute overlap")
    ap.add_argument("--counters", default=None,
                    help="comma-separated rocprofv3 --pmc output directories: write profiles/traffic.json")
    args = ap.parse_args()
    if args.counters:
        summarize_counters(args.counters.split(","))
        return
    if args.trace_summary:
        summarize_trace(args.trace_summary)
        return
    if args.dd_overlap:
        summarize_dd_overlap(args.dd_overlap)
        return
    if args.nb_candidates:
        neighbor_candidates(args.nb_candidates)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1611_00075_amd import inputs
    from paper_1611_00075_amd.sim import Simulation

    torch.cuda.set_device(0)
    reps = max(1, args.reps)
    log("measured peaks")
    peaks = measured_peaks(torch)
    copy_gbs = peaks["copy_GBs"]
    if args.only == "peaks":
        print(json.dumps({"measured_peaks": peaks}))
        return
    log("LJ void system: generating")
    # ---- headline: LJ with voids ------------------------------------------
    s = inputs.lj_voids()
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005)
    log(f"LJ void system: {s.n} atoms, running")
    r = run_workload(sim, args.steps, args.warmup, reps, torch)
    n = s.n
    st = leg_stats(n, args.steps, r)
    byt = lj_force_bytes(n, sim.n_pairs)
    result = {
        "metric": "atom-steps/sec at 1 MI355X (LJ, EAM, MLP vs EAM) + % roofline at stated force err",
        "value": st["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": st["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "repetitions": reps,
        "value_std": st["value_std"],
        "ms_per_step_std": st["ms_per_step_std"],
        "config": {
            "workload": "lj_fcc_80^3_voids_40pct",
            "atoms": n, "sites": s.meta["sites"], "voids": s.meta["voids"],
            "rc": 2.5, "skin": 0.3, "dt": 0.005, "T": 0.72,
            "list_entries": sim.n_pairs, "rebuilds_per_run": st["rebuilds_per_run"],
            "state": "f64 positions/velocities, f32 pair arithmetic and forces",
            "force_error_vs_fp64_oracle": "<= 1e-5 normwise and per atom (tests/test_gpu_fullsize.py)",
        },
        "roofline": roofline_hbm("k_lj32 (md_forces_lj)", byt, st["forces_ms"], copy_gbs,
                                 recorded_traffic("k_lj32_lj_voids_1.23M"), ("k_lj32_lj_voids_1.23M",)),
        "forces_ms_std": st["forces_ms_std"],
        "measured_peaks": peaks,
        "phases_ms_per_call_api": {k: v[0] for k, v in r["phases"].items()},
    }
    result["roofline"]["frac_of_measured_copy"] = result["roofline"].pop("frac_of_copy")
    del sim
    torch.cuda.empty_cache()

    extra = {}
    thermal = None
    eam_value = None
    if args.only in ("all", "mlp"):
        # ---- EAM metal, 4 M atoms ----------------------------------------
        log("EAM crystal: generating")
        s3 = inputs.eam_cu()
        sim3 = Simulation(s3.L, s3.x, s3.v, potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0,
                          mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        st3 = 200
        r3 = run_workload(sim3, st3, 10, reps, torch)
        leg = leg_stats(s3.n, st3, r3)
        b3 = eam_force_bytes(s3.n, sim3.n_pairs)
        leg.update({
            "list_entries": sim3.n_pairs, "forces_bytes": b3,
            "roofline": roofline_hbm("k_eam_rho + k_eam_force (md_forces_eam)", b3, leg["forces_ms"], copy_gbs,
                                     recorded_pair("k_eam_rho_cu_4M", "k_eam_force_cu_4M"), ("k_eam_rho_cu_4M", "k_eam_force_cu_4M")),
            "phases_ms_per_call_api": {k: v[0] for k, v in r3["phases"].items()},
        })
        extra["eam_cu_fcc_100^3"] = leg
        eam_value = leg["value"]
        _, ke3 = sim3.energies()
        thermal = (sim3.positions(), sim3.forces().astype(np.float64),
                   2.0 * ke3 / ((3 * s3.n - 3) * inputs.KB_EV))
        del sim3
        torch.cuda.empty_cache()
    if args.only == "all":
        # ---- second-moment tight-binding metal, 4 M atoms -------------------
        log("TB crystal")
        s5 = inputs.eam_cu()
        sim5 = Simulation(s5.L, s5.x, s5.v, potential="tb", tb=inputs.TB_CU, skin=1.0, dt=1.0,
                          mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        r5 = run_workload(sim5, 200, 10, reps, torch)
        leg = leg_stats(s5.n, 200, r5)
        b5 = eam_force_bytes(s5.n, sim5.n_pairs)
        leg.update({
            "list_entries": sim5.n_pairs, "forces_bytes": b5,
            "roofline": roofline_hbm("k_eam_rho<TB32> + k_eam_force<TB32> (md_forces_tb)", b5, leg["forces_ms"],
                                     copy_gbs, recorded_pair("k_tb_rho_cu_4M", "k_tb_force_cu_4M"), ("k_tb_rho_cu_4M", "k_tb_force_cu_4M")),
            "potential": "second-moment tight-binding (exponential psi and Phi, sqrt embedding), "
                         "synthetic Cu-like parameters, rc 5.0 A, list 6.0 A",
        })
        extra["tb_cu_fcc_100^3"] = leg
        del sim5, s5
        torch.cuda.empty_cache()
        # ---- tabulated functions (the FS set sampled at dr = 0.005 A), 4 M atoms
        log("tabulated crystal")
        s7 = inputs.eam_cu()
        tab7 = inputs.fs_table(inputs.FS_CU)
        sim7 = Simulation(s7.L, s7.x, s7.v, potential="tab", tab=tab7, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                          force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        r7 = run_workload(sim7, 200, 10, reps, torch)
        leg = leg_stats(s7.n, 200, r7)
        b7 = eam_force_bytes(s7.n, sim7.n_pairs)
        leg.update({
            "list_entries": sim7.n_pairs, "forces_bytes": b7,
            "roofline": roofline_hbm("k_tab_rho + k_tab_force (md_forces_tab)", b7, leg["forces_ms"], copy_gbs,
                                     recorded_pair("k_tab_rho_cu_4M", "k_tab_force_cu_4M"), ("k_tab_rho_cu_4M", "k_tab_force_cu_4M")),
            "potential": "tabulated psi, Phi, F (cubic Hermite between knots) sampled from the FS set: "
                         f"{len(tab7['psi'])} r knots at 0.005 A, {len(tab7['F'])} rho knots; list 5.4 A",
        })
        extra["tab_cu_fcc_100^3"] = leg
        del sim7, s7
        torch.cuda.empty_cache()
        # ---- domain decomposition on one device (FS, 4 M atoms) --------------
        from paper_1611_00075_amd.dd import DomainSimulation
        for pdd in ((1, 1, 1), (2, 2, 2)):
            name = "dd_fs_cu_100^3_%dx%dx%d" % pdd
            log(name)
            s8 = inputs.eam_cu()
            sim8 = DomainSimulation(s8.L, s8.x, s8.v, p=pdd, potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0,
                                    mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
            st8 = torch.cuda.current_stream()
            sim8.run(10)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st8)
            for _ in range(20):
                sim8.compute_forces()
            e1.record(st8)
            torch.cuda.synchronize()
            f8 = e0.elapsed_time(e1) / 20
            secs, builds = [], []
            for _ in range(reps):
                b0 = sim8.dd.builds
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim8.run(200)
                torch.cuda.synchronize()
                secs.append(time.perf_counter() - t0)
                builds.append(int(sim8.dd.builds - b0))
            leg = leg_stats(s8.n, 200, {"seconds": secs, "force_ms": [f8], "rebuilds": builds})
            leg.update({
                "bricks": list(pdd), "ghosts": int(sim8.dd.n_ghost),
                "note": "forces: local coordinates into the brick frames, halo pack/copy/unpack on a second "
                        "stream beside the inner atoms' passes, outer atoms after; F' of ghosts exchanged "
                        "between the passes; the step loop reads the rebuild flag back every step; forces_ms "
                        "from 20 back-to-back force steps",
            })
            extra[name] = leg
            sim8.close()
            del sim8, s8
            torch.cuda.empty_cache()
        # ---- two elements: random alloy and two layers, 4 M atoms ---------
        for layered in (False, True):
            name = "tbm_cu_au_layers_100^3" if layered else "tbm_cu75au25_alloy_100^3"
            log(name)
            s6 = inputs.cu_au(layered=layered)
            sim6 = Simulation(s6.L, s6.x, s6.v, potential="tbm", tbm=inputs.TB2_PAIRS, types=s6.meta["types"],
                              skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                              force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
            r6 = run_workload(sim6, 200, 10, reps, torch)
            leg = leg_stats(s6.n, 200, r6)
            b6 = eam_force_bytes(s6.n, sim6.n_pairs)
            leg.update({
                "list_entries": sim6.n_pairs, "fraction_element_1": s6.meta["frac_au"], "forces_bytes": b6,
                "roofline": roofline_hbm("k_eam_rho<TBM32> + k_eam_force<TBM32> (md_forces_tbm)", b6,
                                         leg["forces_ms"], copy_gbs,
                                         recorded_pair("k_tbm_rho_cu_au_4M", "k_tbm_force_cu_au_4M"), ("k_tbm_rho_cu_au_4M", "k_tbm_force_cu_au_4M")),
            })
            extra[name] = leg
            del sim6, s6
            torch.cuda.empty_cache()
        # ---- LJ slab with a dense cluster, about 32 M atoms ----------------
        log("LJ slab + cluster: generating")
        s4 = inputs.lj_slab_cluster()
        sim4 = Simulation(s4.L, s4.x, s4.v, skin=0.3, dt=0.005)
        log(f"LJ slab + cluster: {s4.n} atoms, running")
        r4 = run_workload(sim4, 100, 10, reps, torch, phase_steps=5)
        leg = leg_stats(s4.n, 100, r4)
        b4 = lj_force_bytes(s4.n, sim4.n_pairs)
        leg.update({
            "list_entries": sim4.n_pairs, "slab_atoms": s4.meta["slab_atoms"],
            "cluster_atoms": s4.meta["cluster_atoms"],
            "roofline": roofline_hbm("k_lj32 (md_forces_lj)", b4, leg["forces_ms"], copy_gbs,
                                     recorded_traffic("k_lj32_lj_slab_32M"), ("k_lj32_lj_slab_32M",)),
            "phases_ms_per_call_api": {k: v[0] for k, v in r4["phases"].items()},
        })
        extra["lj_slab_cluster_32M"] = leg
        del sim4, s4
        torch.cuda.empty_cache()
        # ---- LJ crystal, 4,000 atoms, FP64 (launch-bound) -------------------
        log("LJ crystal FP64")
        s1 = inputs.lj_fcc()
        sim1 = Simulation(s1.L, s1.x, s1.v, skin=0.3, dt=0.005, pair_fp64=True)
        r1 = run_workload(sim1, 100, 10, reps, torch)
        extra["lj_fcc_10^3_fp64"] = leg_stats(s1.n, 100, r1)
        del sim1
    if args.only in ("all", "mlp"):
        # ---- learned potential: train on the GPU, run the 4 M-atom crystal --
        log("MLP: EAM training data")
        m = mlp_leg(torch, args.mlp_steps, 10, reps, args.mlp_snapshots, args.mlp_epochs, args.mlp_equil,
                    thermal)
        bf = m["bf16"]
        bf["vs_eam"] = bf["value"] / eam_value if eam_value else None
        m["fp32_activations"]["vs_eam"] = m["fp32_activations"]["value"] / eam_value if eam_value else None
        # the longest of the three kernels: the pair-force pass
        t_ms, fl = bf["pass2_ms"], bf["pass2_valu_flops"]
        bf["roofline"] = {
            "bound": "alu", "kernel": "k_mlp_force (pass 2)",
            "achieved": fl / (t_ms * 1e-3) / 1e12, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": fl / (t_ms * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS,
            "frac_of_measured_fma_loop": fl / (t_ms * 1e-3) / 1e12 / peaks["fp32_fma_TFLOPs"],
            "traffic": recorded_traffic("k_mlp_force_cu_4M"),
            "valu_issue_frac": valu_frac("k_mlp_force_cu_4M"),
            "texture_addresser_busy_frac": ta_frac("k_mlp_force_cu_4M"),
            "net_mfma_frac_of_mfma_loop": mfma_frac("k_mlp_net_cu_4M"),
            "launch_ms": t_ms,
        }
        extra["mlp_cu_fcc_100^3"] = m
    if extra:
        result["extra"] = extra

    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(s, args.cpu_steps, args.cpu_all_steps)
    print(json.dumps(result))


# --------------------------------------------------------------------------
# counters -> profiles/traffic.json
# --------------------------------------------------------------------------

FORCES_SRC = ["paper_1611_00075_amd/csrc/md_forces.hip", "paper_1611_00075_amd/csrc/md_pair.h",
              "paper_1611_00075_amd/csrc/md_common.h"]
TAB_SRC = ["paper_1611_00075_amd/csrc/md_tab.hip", "paper_1611_00075_amd/csrc/md_pair.h",
           "paper_1611_00075_amd/csrc/md_common.h"]
MLP_SRC = ["paper_1611_00075_amd/csrc/md_mlp.hip", "paper_1611_00075_amd/csrc/md_pair.h",
           "paper_1611_00075_amd/csrc/md_common.h"]
CELLS_SRC = ["paper_1611_00075_amd/csrc/md_cells.hip", "paper_1611_00075_amd/csrc/md_pair.h",
             "paper_1611_00075_amd/csrc/md_common.h"]
PROBE_SRC = ["paper_1611_00075_amd/csrc/md_probe.hip", "paper_1611_00075_amd/csrc/md_common.h"]

# key: (sources, kernel-name pattern, grid size)  -- grid sizes of the
# benchmark's systems: 1,228,798 (voids), 4,000,000 (Cu), 31,860,227 (slab)
# atoms; 103,823 / 287,496 / 216,000 / 3,375,000 cells
COUNTER_KERNELS = {
    "k_lj32_lj_voids_1.23M": (FORCES_SRC, r"k_lj32<8, \d+, true, false, true>", 9830400),
    "k_lj32_lj_slab_32M": (FORCES_SRC, r"k_lj32<8, \d+, true, false, true>", 254882048),
    "k_eam_rho_cu_4M": (FORCES_SRC, r"k_eam_rho<md::FS32,", 32000000),
    "k_eam_force_cu_4M": (FORCES_SRC, r"k_eam_force<md::FS32,", 32000000),
    "k_tb_rho_cu_4M": (FORCES_SRC, r"k_eam_rho<md::TB32,", 32000000),
    "k_tb_force_cu_4M": (FORCES_SRC, r"k_eam_force<md::TB32,", 32000000),
    "k_tbm_rho_cu_au_4M": (FORCES_SRC, r"k_eam_rho<md::TBM32<", 32000000),
    "k_tbm_force_cu_au_4M": (FORCES_SRC, r"k_eam_force<md::TBM32<", 32000000),
    "k_tab_rho_cu_4M": (TAB_SRC, r"k_tab_rho<", None),
    "k_tab_force_cu_4M": (TAB_SRC, r"k_tab_force<", None),
    "k_mlp_desc_cu_4M": (MLP_SRC, r"k_mlp_desc\(", 32000000),
    "k_mlp_net_cu_4M": (MLP_SRC, r"k_mlp_net<1>", 524288),
    "k_mlp_force_cu_4M": (MLP_SRC, r"k_mlp_force<2, false, true>", 32000000),
    "k_neighbors_lj_voids_1.23M": (CELLS_SRC, r"k_neighbors\(", 103823 * 64),
    "k_neighbors_cu_5.4A_4M": (CELLS_SRC, r"k_neighbors\(", 287496 * 64),
    "k_neighbors_lj_slab_32M": (CELLS_SRC, r"k_neighbors\(", 3375000 * 64),
    "k_probe_fma_f32": (PROBE_SRC, r"k_probe_fma<float>", None),
    "k_probe_fma_f64": (PROBE_SRC, r"k_probe_fma<double>", None),
    "k_probe_mfma": (PROBE_SRC, r"k_probe_mfma\(", None),
}


def _read_counters(dirs):
    """{(kernel name, grid): {counter: [value per dispatch]}} from rocprofv3
    counter-collection CSVs (each counter summed over its instances)."""
    import csv
    import glob
    out = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*_counter_collection.csv"), recursive=True):
            per = {}
            for row in csv.DictReader(open(f)):
                k = (row["Dispatch_Id"], row["Kernel_Name"], int(row["Grid_Size"]), row["Counter_Name"])
                per[k] = per.get(k, 0.0) + float(row["Counter_Value"])
            for (disp, name, grid, ctr), v in per.items():
                out.setdefault((name, grid), {}).setdefault(ctr, []).append(v)
    return out


def summarize_trace(d):
    """Per (kernel, grid) table of a rocprofv3 --kernel-trace output
    directory: launches, mean and median duration, and the mean over the
    full launches (those above a quarter of the median; the force kernels'
    skipped speculative launches fall below it)."""
    import csv
    import glob
    rows = {}
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            rows.setdefault((r["Kernel_Name"], g), []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    print("kernel\tgrid\tlaunches\tmean_us\tmedian_us\tfull_launches\tfull_mean_us\ttotal_ms")
    for (name, g), v in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        v = np.asarray(v)
        full = v[v >= 0.25 * np.median(v)]
        print(f"{name[:120]}\t{g}\t{len(v)}\t{v.mean():.2f}\t{np.median(v):.2f}\t{len(full)}\t"
              f"{full.mean():.2f}\t{v.sum() / 1e3:.3f}")


def summarize_dd_overlap(d):
    """Halo exchange against compute per force evaluation of a decomposed
    system, from a rocprofv3 --kernel-trace of repeated
    DomainSimulation.compute_forces calls: for each evaluation (it starts
    with k_dd_scale_local) the span, the inner and outer launches of the two
    passes (the inner one has the larger grid), and the position and F'
    halos from the start of their pack to the end of their unpack, with
    whether each ends inside the inner launch it overlaps.  Prints means,
    minima and maxima over the evaluations after the first two."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            m = re.search(r"(k_\w+?)(<[^()]*>)?\(", r["Kernel_Name"])   # the kernel's own name
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), m.group(1) if m else r["Kernel_Name"],
                         int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])))
    rows.sort()
    evals = []
    for t0, t1, name, grid in rows:
        if name == "k_dd_scale_local":
            evals.append({"t0": t0, "k": []})
        if evals:
            evals[-1]["k"].append((t0, t1, name, grid))
    res = []
    for e in evals:
        ks = e["k"]

        def pick(kernel):
            return [k for k in ks if k[2] == kernel]

        rho = sorted(pick("k_eam_rho")[:2], key=lambda k: -k[3])
        frc = sorted(pick("k_eam_force")[:2], key=lambda k: -k[3])
        pk, up, pkw, upw = pick("k_dd_pack"), pick("k_dd_unpack"), pick("k_dd_pack_w"), pick("k_dd_unpack_w")
        if len(rho) < 2 or len(frc) < 2 or not (pk and up and pkw and upw):
            continue
        end = max(k[1] for k in ks if "k_eam" in k[2] or "k_dd" in k[2])
        us = 1e-3
        res.append({"span_us": (end - e["t0"]) * us,
                    "rho_inner_us": (rho[0][1] - rho[0][0]) * us, "rho_outer_us": (rho[1][1] - rho[1][0]) * us,
                    "force_inner_us": (frc[0][1] - frc[0][0]) * us, "force_outer_us": (frc[1][1] - frc[1][0]) * us,
                    "position_halo_us": (up[0][1] - pk[0][0]) * us,
                    "position_halo_inside": float(up[0][1] <= rho[0][1]),
                    "fprime_halo_us": (upw[0][1] - pkw[0][0]) * us,
                    "fprime_halo_inside": float(upw[0][1] <= frc[0][1])})
    tail = res[2:]
    print(f"evaluations: {len(res)} of {len(evals)}; statistics over the {len(tail)} after the first two")
    for k in (tail[0] if tail else {}):
        v = np.array([r[k] for r in tail])
        print(f"{k}\tmean {v.mean():.2f}\tmin {v.min():.2f}\tmax {v.max():.2f}")


def neighbor_candidates(which, samples=3000, seed=0):
    """CPU model of the neighbour build's candidate selection on a system's
    initial configuration: for a sample of occupied cells (edge >= r_list,
    27-cell stencil), the candidates each home atom's wave streams (all atoms
    of the stencil), those within r_list of the bounding box of the cell's
    home atoms (kept and tested exactly, in 64-candidate chunks), and the
    home atom's list entries.  Prints one JSON line."""
    from paper_1611_00075_amd import inputs
    s, rl = (inputs.lj_voids(), 2.8) if which == "voids" else (inputs.eam_cu(), 5.4)
    L = float(s.L[0])
    x = np.mod(s.x, L)
    nc = int(np.floor(L / rl))
    c = np.minimum((x * (nc / L)).astype(np.int64), nc - 1)
    lin = c[:, 0] + nc * (c[:, 1] + nc * c[:, 2])
    order = np.argsort(lin, kind="stable")
    xs, ls = x[order], lin[order]
    start = np.concatenate([[0], np.cumsum(np.bincount(ls, minlength=nc ** 3))])
    occupied = np.nonzero(np.diff(start))[0]
    cells = np.random.default_rng(seed).choice(occupied, min(samples, len(occupied)), replace=False)
    homes = streamed = kept = chunks = hits = 0
    for cl in cells:
        cz, rem = divmod(int(cl), nc * nc)
        cy, cx = divmod(rem, nc)
        h = xs[start[cl]:start[cl + 1]]
        cand = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    k = np.array([cx + dx, cy + dy, cz + dz])
                    img, k = np.floor_divide(k, nc), np.mod(k, nc)
                    q = k[0] + nc * (k[1] + nc * k[2])
                    cand.append(xs[start[q]:start[q + 1]] + img * L)
        cand = np.concatenate(cand)
        lo, hi = h.min(0), h.max(0)
        d = np.maximum(np.maximum(lo - cand, cand - hi), 0.0)
        kc = cand[(d * d).sum(1) < rl * rl]
        r2 = ((h[:, None, :] - kc[None, :, :]) ** 2).sum(2)
        homes += len(h)
        streamed += len(cand) * len(h)
        kept += len(kc) * len(h)
        chunks += -(-len(kc) // 64) * len(h)
        hits += int((r2 < rl * rl).sum()) - len(h)        # less each home itself
    print(json.dumps({"system": which, "r_list": rl, "cells_sampled": int(len(cells)), "home_atoms": homes,
                      "streamed_per_home": streamed / homes, "kept_per_home": kept / homes,
                      "chunks_per_home": chunks / homes, "entries_per_home": hits / homes,
                      "tested_per_entry": 64.0 * chunks / hits, "streamed_per_entry": streamed / hits}))


def summarize_counters(dirs):
    """profiles/traffic.json from rocprofv3 --pmc runs of bench.py: HBM bytes
    per launch (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for
    the benchmark's 2 GiB device copies), issued VALU instructions and
    matrix-core busy cycles per CU per clock (GRBM_GUI_ACTIVE summed over the
    8 XCDs, so divided by 8 for the dispatch's cycles; 256 CUs), the fraction
    of VALU issue quad-cycles used (dual-issued pairs counted once), and the
    texture addressers' busy fraction.  Each directory is one pass; launches
    the device skipped (speculative evaluations) are dropped: their counts
    are far below the kernel's median."""
    passes = [_read_counters([d]) for d in dirs]
    # copy calibration: the largest copy kernel moves 2 GiB each way
    cal = {"FETCH_SIZE": None, "WRITE_SIZE": None}
    for data in passes:
        for (name, grid), ctrs in data.items():
            if "copyBuffer" in name or "copy_kernel" in name:
                for c in cal:
                    if c in ctrs:
                        v = max(ctrs[c])
                        if cal[c] is None or v > cal[c]:
                            cal[c] = v
    scale = {c: (2 * (1 << 30) / 1024.0) / v if v else None for c, v in cal.items()}

    def kept(vals):
        vals = np.asarray(vals)
        med = np.median(vals)
        return vals[vals >= 0.25 * med] if med > 0 else vals

    out = {}
    for data in passes:
        for key, (sources, pat, grid) in COUNTER_KERNELS.items():
            rx = re.compile(pat)
            hits = [(name, g, ctrs) for (name, g), ctrs in data.items()
                    if rx.search(name) and (grid is None or g == grid)]
            if not hits:
                continue
            name, g, ctrs = max(hits, key=lambda h: max(len(v) for v in h[2].values()))
            rec = out.setdefault(key, {"kernel": name[:160], "grid_size": g, "sources": sources,
                                       "sources_sha256": _sources_sha(sources)})
            if "FETCH_SIZE" in ctrs and scale["FETCH_SIZE"]:
                f = kept(ctrs["FETCH_SIZE"])
                rec.update(fetch_kib=float(f.mean()), fetch_scale=scale["FETCH_SIZE"], launches=int(len(f)))
            if "WRITE_SIZE" in ctrs and scale["WRITE_SIZE"]:
                w = kept(ctrs["WRITE_SIZE"])
                rec.update(write_kib=float(w.mean()), write_scale=scale["WRITE_SIZE"])
            if "GRBM_GUI_ACTIVE" not in ctrs:
                continue
            gui = np.asarray(ctrs["GRBM_GUI_ACTIVE"])
            keep = gui >= 0.25 * np.median(gui)
            cyc = gui[keep].mean() / 8.0
            rec["cycles_per_xcd"] = float(cyc)

            def mean(ctr):
                for c in (ctr, ctr + "_sum"):
                    if c in ctrs and len(ctrs[c]) == len(gui):
                        return float(np.asarray(ctrs[c])[keep].mean())
                return None

            for ctr, field in (("SQ_INSTS_VALU", "valu_inst_per_cu_clk"),
                               ("SQ_VALU_MFMA_BUSY_CYCLES", "mfma_busy_per_cu_clk"),
                               ("TA_TA_BUSY", "ta_busy_per_cu_clk")):
                v = mean(ctr)
                if v is not None:
                    rec[field] = v / (cyc * 256.0)
                    rec[ctr.lower()] = v
            # issue events: a dual issue puts two VALU instructions in one
            # quad-cycle of a SIMD; 256 CUs x 4 SIMDs x cycles / 4 quad-cycles
            ins, dual = mean("SQ_INSTS_VALU"), mean("SQ_ACTIVE_INST_VALU2")
            if ins is not None and dual is not None:
                rec["valu_dual_issued"] = dual
                rec["valu_issue_frac"] = (ins - dual) / (cyc * 256.0)
            for ctr in ("TA_BUFFER_READ_WAVEFRONTS", "TCP_TOTAL_CACHE_ACCESSES", "TCP_TCC_READ_REQ"):
                v = mean(ctr)
                if v is not None:
                    rec[ctr.lower()] = v
    for rec in out.values():
        if "fetch_kib" in rec and "write_kib" in rec:
            rec["traffic_bytes"] = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] +
                                             rec["write_kib"] * rec["write_scale"])
    old = {}
    try:
        old = json.load(open(TRAFFIC))
    except (OSError, ValueError):
        pass
    for k, v in out.items():
        if old.get(k, {}).get("sources_sha256") == v["sources_sha256"]:
            old[k].update(v)      # further counters of the same sources
        else:
            old[k] = v            # new sources: nothing of the old record holds
    json.dump(old, open(TRAFFIC, "w"), indent=1)
    print(json.dumps({"calibration": cal, "scale": scale, "kernels": sorted(out)}))


if __name__ == "__main__":
    main()
