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
from HIP events on the launch stream, against the published 8 TB/s and
against a device-to-device copy measured in the same run), the FP64
oracle's rate on this host (cpu_baseline) and the other workloads of the
metric (EAM metal, the 32 M-atom slab, FP64 LJ, the learned potential).
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
# FP32 vector peak without packed instructions: 256 CUs x 64 lanes x 2 (FMA)
# x 2.4 GHz (the packed form, which doubles it, is not used on this platform)
FP32_VALU_PEAK_TFLOPS = 78.6


def recorded(key, field="traffic_bytes"):
    """A figure from the committed rocprofv3 counter runs
    (profiles/traffic.json: HBM bytes per launch, VALU busy percent, ...),
    or None when a source of the kernel has changed since the counters
    were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[key]
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec.get(field)


def recorded_traffic(key):
    """HBM bytes per launch from the committed counter runs, or None."""
    return recorded(key, "traffic_bytes")


def recorded_pair(k1, k2):
    """Recorded traffic of a two-pass force evaluation (both passes), or None."""
    a, b = recorded_traffic(k1), recorded_traffic(k2)
    return None if a is None or b is None else a + b


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


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


def mlp_leg(torch, steps, warmup, n_snap, epochs, equil, thermal):
    """Learned potential (Cu surrogate): training data from the GPU's own
    EAM trajectories, training on the GPU, then the 4 M-atom crystal of the
    EAM workload run with MLP forces."""
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
    # the 4 M-atom crystal with MLP forces
    log(f"MLP: trained in {t_train:.1f} s; 4 M-atom run")
    s = inputs.eam_cu()
    sim = Simulation(s.L, s.x, s.v, potential="mlp", mlp=sp, mlp_w=pot.w, skin=1.0, dt=1.0,
                     mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    # forces on a thermalised configuration of the EAM run
    x_th, f_th, T_th = thermal
    f_m = P.mlp_forces(pot, s.L, x_th)
    frmse = float(np.sqrt(np.mean((f_m - f_th) ** 2)))
    frms = float(np.sqrt(np.mean(f_th ** 2)))
    del f_m
    ep0, ek0 = sim.energies()
    r = run_workload(sim, steps, warmup, torch)
    ep1, ek1 = sim.energies()
    # pass 2 alone (dE/dG reused), then both passes, timed with HIP events
    n = s.n
    st = torch.cuda.current_stream()
    ms = {}
    # pass 2 alone walks the compact list pass 1 left, as in a full evaluation
    calls = {
        "both": lambda: M.md_forces_mlp(sim.L, n, sim.xs, sim.row_cap, sim.idx, sim.count, sim.mlp, sim.mlp_w,
                                        sim.dEdG, sim.idx_in, sim.cnt_in, None, sim.f, sim.ev, 0, sim.ws),
        "pass2": lambda: M.md_forces_mlp(sim.L, n, sim.xs, sim.row_cap, sim.idx_in, sim.cnt_in, sim.mlp, None,
                                         sim.dEdG, None, None, None, sim.f, sim.ev, M.MD_MLP_REUSE, sim.ws),
    }
    # the network kernel alone, on descriptors of the same configuration
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
    entries = sim.n_pairs
    within = pairs_within(sim, float(sp.rc), torch)
    v1, v2, mfma = mlp_force_flops(n, within, entries)
    out.update({
        "atoms": n, "steps": steps, "value": n * steps / r["seconds"], "unit": "atom-steps/s",
        "ms_per_step": 1e3 * r["seconds"] / steps, "rebuilds": r["rebuilds"], "forces_ms": r["force_ms"],
        "pass1_ms": ms["both"] - ms["pass2"], "pass2_ms": ms["pass2"], "net_ms": ms["net"],
        "list_entries": entries,
        "force_rmse_vs_eam_eV_A": frmse, "force_rms_eam_eV_A": frms,
        "force_config": f"EAM trajectory of the same crystal after its timed steps, T = {T_th:.0f} K",
        "energy_drift_eV_per_atom": ((ep1 + ek1) - (ep0 + ek0)) / n,
        "pairs_within_rc": within, "pass1_valu_flops": v1, "pass2_valu_flops": v2, "pass1_mfma_flops": mfma,
        "phases_ms_per_call_api": {k: v[0] for k, v in r["phases"].items()},
    })
    return out, sim


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


def copy_bandwidth(torch, gib=2, reps=10):
    """Achievable HBM rate on this GPU: a device-to-device copy of `gib` GiB
    (read + write counted), timed with HIP events -- the measured peak the
    kernels' rates are also compared with."""
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="all", choices=["all", "lj", "mlp"])
    ap.add_argument("--mlp-snapshots", type=int, default=1250, help="snapshots per temperature (16 temperatures)")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--mlp-equil", type=int, default=2000, help="equilibration steps per temperature")
    ap.add_argument("--mlp-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1611_00075_amd import inputs
    from paper_1611_00075_amd.sim import Simulation

    torch.cuda.set_device(0)
    log("LJ void system: generating")
    # ---- headline: LJ with voids ------------------------------------------
    s = inputs.lj_voids()
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005)
    log(f"LJ void system: {s.n} atoms, running")
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
            "valu_inst_per_cu_clk": recorded("k_lj32_lj_voids_1.23M", "valu_inst_per_cu_clk"),
            "bytes_per_launch": byt, "launch_ms": f_ms,
        },
        "phases_ms_per_call_api": {k: v[0] for k, v in r["phases"].items()},
    }
    del sim
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth(torch)
    result["roofline"]["copy_GBs"] = copy_gbs
    result["roofline"]["frac_of_copy"] = achieved / copy_gbs

    extra = {}
    thermal = None
    if args.only in ("all", "mlp"):
        # ---- EAM metal, 4 M atoms ----------------------------------------
        log("EAM crystal: generating")
        s3 = inputs.eam_cu()
        sim3 = Simulation(s3.L, s3.x, s3.v, potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0,
                          mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        if args.only == "mlp":
            sim3.run(100)
        if args.only == "all":
            st3 = 200
            r3 = run_workload(sim3, st3, 10, torch)
            f3 = r3["force_ms"]
            b3 = eam_force_bytes(s3.n, sim3.n_pairs)
            extra["eam_cu_fcc_100^3"] = {
                "atoms": s3.n, "steps": st3, "value": s3.n * st3 / r3["seconds"], "unit": "atom-steps/s",
                "ms_per_step": 1e3 * r3["seconds"] / st3, "rebuilds": r3["rebuilds"],
                "forces_ms": f3, "forces_GBs": b3 / (f3 * 1e-3) / 1e9,
                "forces_frac_hbm": b3 / (f3 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "forces_frac_copy": b3 / (f3 * 1e-3) / 1e9 / copy_gbs,
                "forces_traffic_bytes": recorded_pair("k_eam_rho_cu_4M", "k_eam_force_cu_4M"),
                "valu_inst_per_cu_clk": [recorded("k_eam_rho_cu_4M", "valu_inst_per_cu_clk"),
                                         recorded("k_eam_force_cu_4M", "valu_inst_per_cu_clk")],
                "forces_bytes": b3,
                "phases_ms_per_call_api": {k: v[0] for k, v in r3["phases"].items()},
            }
        _, ke3 = sim3.energies()
        thermal = (sim3.positions(), sim3.forces().astype(np.float64),
                   2.0 * ke3 / ((3 * s3.n - 3) * inputs.KB_EV))
        del sim3
        torch.cuda.empty_cache()
    if args.only == "all":
        # ---- second-moment tight-binding metal, 4 M atoms -------------------
        log("TB crystal: generating")
        s5 = inputs.eam_cu()
        sim5 = Simulation(s5.L, s5.x, s5.v, potential="tb", tb=inputs.TB_CU, skin=1.0, dt=1.0,
                          mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        log("TB crystal: running")
        r5 = run_workload(sim5, 200, 10, torch)
        f5 = r5["force_ms"]
        b5 = eam_force_bytes(s5.n, sim5.n_pairs)
        extra["tb_cu_fcc_100^3"] = {
            "atoms": s5.n, "steps": 200, "value": s5.n * 200 / r5["seconds"], "unit": "atom-steps/s",
            "ms_per_step": 1e3 * r5["seconds"] / 200, "rebuilds": r5["rebuilds"], "list_entries": sim5.n_pairs,
            "forces_ms": f5, "forces_GBs": b5 / (f5 * 1e-3) / 1e9,
            "forces_frac_hbm": b5 / (f5 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "forces_frac_copy": b5 / (f5 * 1e-3) / 1e9 / copy_gbs,
            "forces_traffic_bytes": recorded_pair("k_tb_rho_cu_4M", "k_tb_force_cu_4M"), "forces_bytes": b5,
            "potential": "second-moment tight-binding (exponential psi and Phi, sqrt embedding), "
                         "synthetic Cu-like parameters, rc 5.0 A, list 6.0 A",
            "phases_ms_per_call_api": {k: v[0] for k, v in r5["phases"].items()},
        }
        del sim5, s5
        torch.cuda.empty_cache()
        # ---- tabulated functions (the FS set sampled at dr = 0.005 A), 4 M atoms
        log("tabulated crystal: generating")
        s7 = inputs.eam_cu()
        tab7 = inputs.fs_table(inputs.FS_CU)
        sim7 = Simulation(s7.L, s7.x, s7.v, potential="tab", tab=tab7, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                          force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        log("tabulated crystal: running")
        r7 = run_workload(sim7, 200, 10, torch)
        f7 = r7["force_ms"]
        b7 = eam_force_bytes(s7.n, sim7.n_pairs)
        extra["tab_cu_fcc_100^3"] = {
            "atoms": s7.n, "steps": 200, "value": s7.n * 200 / r7["seconds"], "unit": "atom-steps/s",
            "ms_per_step": 1e3 * r7["seconds"] / 200, "rebuilds": r7["rebuilds"], "list_entries": sim7.n_pairs,
            "forces_ms": f7, "forces_GBs": b7 / (f7 * 1e-3) / 1e9,
            "forces_frac_hbm": b7 / (f7 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "forces_frac_copy": b7 / (f7 * 1e-3) / 1e9 / copy_gbs,
            "forces_traffic_bytes": recorded_pair("k_tab_rho_cu_4M", "k_tab_force_cu_4M"), "forces_bytes": b7,
            "potential": "tabulated psi, Phi, F (cubic Hermite between knots) sampled from the FS set: "
                         f"{len(tab7['psi'])} r knots at 0.005 A, {len(tab7['F'])} rho knots; list 5.4 A",
            "phases_ms_per_call_api": {k: v[0] for k, v in r7["phases"].items()},
        }
        del sim7, s7
        torch.cuda.empty_cache()
        # ---- domain decomposition on one device (FS, 4 M atoms) --------------
        from paper_1611_00075_amd.dd import DomainSimulation
        for pdd in ((1, 1, 1), (2, 2, 2)):
            name = "dd_fs_cu_100^3_%dx%dx%d" % pdd
            log(f"{name}: generating")
            s8 = inputs.eam_cu()
            sim8 = DomainSimulation(s8.L, s8.x, s8.v, p=pdd, potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0,
                                    mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
            log(f"{name}: running")
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
            b0 = sim8.dd.builds
            t0 = time.perf_counter()
            sim8.run(200)
            torch.cuda.synchronize()
            sec8 = time.perf_counter() - t0
            extra[name] = {
                "atoms": s8.n, "steps": 200, "value": s8.n * 200 / sec8, "unit": "atom-steps/s",
                "ms_per_step": 1e3 * sec8 / 200, "rebuilds": int(sim8.dd.builds - b0), "bricks": list(pdd),
                "ghosts": int(sim8.dd.n_ghost), "forces_ms": f8,
                "note": "forces: local coordinates into the brick frames, halo pack/copy/unpack on a second stream "
                        "beside the inner atoms' passes, outer atoms after; F' of ghosts exchanged between the "
                        "passes; the step loop reads the rebuild flag back every step",
            }
            sim8.close()
            del sim8, s8
            torch.cuda.empty_cache()
        # ---- two elements: random alloy and two layers, 4 M atoms ---------
        for layered in (False, True):
            name = "tbm_cu_au_layers_100^3" if layered else "tbm_cu75au25_alloy_100^3"
            log(f"{name}: generating")
            s6 = inputs.cu_au(layered=layered)
            sim6 = Simulation(s6.L, s6.x, s6.v, potential="tbm", tbm=inputs.TB2_PAIRS, types=s6.meta["types"],
                              skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                              force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
            log(f"{name}: running")
            r6 = run_workload(sim6, 200, 10, torch)
            f6 = r6["force_ms"]
            b6 = eam_force_bytes(s6.n, sim6.n_pairs)
            extra[name] = {
                "atoms": s6.n, "steps": 200, "value": s6.n * 200 / r6["seconds"], "unit": "atom-steps/s",
                "ms_per_step": 1e3 * r6["seconds"] / 200, "rebuilds": r6["rebuilds"],
                "list_entries": sim6.n_pairs, "fraction_element_1": s6.meta["frac_au"],
                "forces_ms": f6, "forces_GBs": b6 / (f6 * 1e-3) / 1e9,
                "forces_frac_hbm": b6 / (f6 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "forces_frac_copy": b6 / (f6 * 1e-3) / 1e9 / copy_gbs,
                "forces_traffic_bytes": recorded_pair("k_tbm_rho_cu_au_4M", "k_tbm_force_cu_au_4M"),
                "forces_bytes": b6,
                "phases_ms_per_call_api": {k: v[0] for k, v in r6["phases"].items()},
            }
            del sim6, s6
            torch.cuda.empty_cache()
        # ---- LJ slab with a dense cluster, about 32 M atoms ----------------
        log("LJ slab + cluster: generating")
        s4 = inputs.lj_slab_cluster()
        sim4 = Simulation(s4.L, s4.x, s4.v, skin=0.3, dt=0.005)
        log(f"LJ slab + cluster: {s4.n} atoms, running")
        r4 = run_workload(sim4, 100, 10, torch, phase_steps=5)
        b4 = lj_force_bytes(s4.n, sim4.n_pairs)
        extra["lj_slab_cluster_32M"] = {
            "atoms": s4.n, "steps": 100, "value": s4.n * 100 / r4["seconds"], "unit": "atom-steps/s",
            "ms_per_step": 1e3 * r4["seconds"] / 100, "rebuilds": r4["rebuilds"], "list_entries": sim4.n_pairs,
            "forces_ms": r4["force_ms"], "forces_GBs": b4 / (r4["force_ms"] * 1e-3) / 1e9,
            "forces_frac_hbm": b4 / (r4["force_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "forces_frac_copy": b4 / (r4["force_ms"] * 1e-3) / 1e9 / copy_gbs,
            "slab_atoms": s4.meta["slab_atoms"], "cluster_atoms": s4.meta["cluster_atoms"],
        }
        del sim4, s4
        torch.cuda.empty_cache()
        # ---- LJ crystal, 4,000 atoms, FP64 (launch-bound) -------------------
        log("LJ crystal FP64")
        s1 = inputs.lj_fcc()
        sim1 = Simulation(s1.L, s1.x, s1.v, skin=0.3, dt=0.005, pair_fp64=True)
        r1 = run_workload(sim1, 100, 10, torch)
        extra["lj_fcc_10^3_fp64"] = {
            "atoms": s1.n, "steps": 100, "value": s1.n * 100 / r1["seconds"], "unit": "atom-steps/s",
            "ms_per_step": 1e3 * r1["seconds"] / 100,
        }
        del sim1
    if args.only in ("all", "mlp"):
        # ---- learned potential: train on the GPU, run the 4 M-atom crystal --
        log("MLP: EAM training data")
        m, simm = mlp_leg(torch, args.mlp_steps, 10, args.mlp_snapshots, args.mlp_epochs, args.mlp_equil,
                          thermal)
        del simm
        eam = extra.get("eam_cu_fcc_100^3")
        m["vs_eam"] = m["value"] / eam["value"] if eam else None
        # the longest of the three kernels: the pair-force pass
        t_ms, fl = m["pass2_ms"], m["pass2_valu_flops"]
        m["roofline"] = {
            "bound": "alu", "kernel": "k_mlp_force (pass 2)",
            "achieved": fl / (t_ms * 1e-3) / 1e12, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": fl / (t_ms * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS,
            "traffic": recorded_traffic("k_mlp_force_cu_4M"),
            "valu_inst_per_cu_clk": recorded("k_mlp_force_cu_4M", "valu_inst_per_cu_clk"),
            "net_mfma_util_pct": recorded("k_mlp_net_cu_4M", "mfma_util_pct"),
            "launch_ms": t_ms,
        }
        extra["mlp_cu_fcc_100^3"] = m
    if extra:
        result["extra"] = extra

    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
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
