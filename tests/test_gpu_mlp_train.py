"""Training of the learned potential on the GPU from EAM trajectories made
by the FP64 oracle, and what the network gains over the method without it.

Data: 16 temperatures 300-1200 K, one 256-atom Cu trajectory each
(equilibration with velocity rescaling, then 40 NVE snapshots 20 fs apart),
labels = the oracle's per-atom EAM energies and forces.  The last quarter of
every trajectory is held out as a whole block.

The method without the network is ridge regression of the per-atom energy
on the same normalised descriptors (closed form, FP64).  The test reports
held-out per-atom energy and force errors of both against the EAM labels
and requires the trained network to beat the linear model on both; an
untrained network is the floor.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_00075_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

CU = inputs.FS_CU
TEMPS = np.linspace(300.0, 1200.0, 16)
N_SNAP = 40


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_00075_amd import md
    md.lib()
    return md


@pytest.fixture(scope="module")
def data(M, orc):
    from oracle import mlp as om
    starts = []
    for k, T in enumerate(TEMPS):
        s = inputs.eam_cu(ncell=4, T=float(T), seed=2000 + k)
        starts.append((s.x, s.v, s.L))
    runs = om.training_set(starts, TEMPS, CU, n_samples=N_SNAP, threads=8, sample_every=20,
                           equil_steps=1000, rescale_every=100)
    L = starts[0][2]
    rows = {"train": [], "test": []}
    for r in runs:
        for k in range(N_SNAP):
            pos = r["pos"][k]
            off, idx = orc.neighbors_brute(pos, L, 6.0)
            G = om.descriptors(pos, L, off, idx, om.Spec())
            part = "test" if k >= 3 * N_SNAP // 4 else "train"
            rows[part].append(dict(pos=pos, off=off, idx=idx, G=G, e=r["e_atom"][k], f=r["forces"][k]))
    return dict(L=L, **rows)


def _stack(snaps, key):
    return np.concatenate([s[key] for s in snaps])


@pytest.fixture(scope="module")
def trained(M, data):
    from paper_1611_00075_amd import mlp as P
    Gtr = torch.tensor(_stack(data["train"], "G").astype(np.float32), device="cuda")
    etr = torch.tensor(_stack(data["train"], "e").astype(np.float32), device="cuda")
    mean, inv = P.normalisation(Gtr)
    sp = P.spec(mean, inv)
    master = P.init_params(7, e_mean=float(etr.double().mean()))
    tr = P.Trainer(Gtr, etr, sp, master, batch=4096, seed=7)
    untrained = P.Potential(sp, tr.w.clone())
    hist = tr.fit(600, lr=1e-2, lr_min=1e-4)
    return dict(pot=tr.potential, untrained=untrained, hist=hist, mean=mean, inv=inv)


def test_training_reduces_loss(trained):
    h = trained["hist"]
    print("epoch losses:", ", ".join(f"{v:.3e}" for v in h[::10]), f"... {h[-1]:.3e}")
    assert h[-1] < 0.05 * h[0]
    assert np.isfinite(h).all()


def test_network_beats_linear_model(M, orc, data, trained):
    from oracle import mlp as om
    from paper_1611_00075_amd import mlp as P
    mean, inv = trained["mean"], trained["inv"]
    Xtr = (_stack(data["train"], "G") - mean) * inv
    u, b = om.ridge_fit(Xtr, _stack(data["train"], "e"), lam=1e-6)
    Gte = _stack(data["test"], "G")
    ete = _stack(data["test"], "e")
    ridge_e = ((Gte - mean) * inv) @ u + b
    Gd = torch.tensor(Gte.astype(np.float32), device="cuda")
    mlp_e = P.predict(Gd, trained["pot"]).cpu().numpy().astype(np.float64)
    raw_e = P.predict(Gd, trained["untrained"]).cpu().numpy().astype(np.float64)
    rm = lambda a: float(np.sqrt(np.mean((a - ete) ** 2)))  # noqa: E731
    e_mlp, e_ridge, e_raw = rm(mlp_e), rm(ridge_e), rm(raw_e)
    # forces on the held-out snapshots: MLP on the GPU; the linear model's
    # forces through the oracle (dE_i/dG_i = u * inv_std for every atom)
    L = data["L"]
    fe, fm, fr = [], [], []
    sp = om.Spec(mean=mean, inv_std=inv)
    dE = np.tile(u * inv, (256, 1))
    for s in data["test"][::4]:
        fe.append(s["f"])
        fm.append(P.mlp_forces(trained["pot"], L, s["pos"]))
        fr.append(om.forces(s["pos"], L, s["off"], s["idx"], sp, dE)[0])
    fe, fm, fr = map(np.concatenate, (fe, fm, fr))
    f_mlp = float(np.sqrt(np.mean((fm - fe) ** 2)))
    f_ridge = float(np.sqrt(np.mean((fr - fe) ** 2)))
    f_scale = float(np.sqrt(np.mean(fe ** 2)))
    print(f"held-out per-atom energy RMSE (eV): MLP {e_mlp:.2e}, ridge {e_ridge:.2e}, untrained {e_raw:.2e}")
    print(f"held-out force RMSE (eV/A): MLP {f_mlp:.3f}, ridge {f_ridge:.3f}, EAM force RMS {f_scale:.3f}")
    assert e_raw > e_ridge
    assert e_mlp < 0.5 * e_ridge
    assert f_mlp < f_ridge


def test_md_run_with_trained_network_conserves_energy(M, trained):
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.eam_cu(ncell=5, T=600.0, seed=2100)
    sim = Simulation(s.L, s.x, s.v, potential="mlp", mlp=trained["pot"].spec, mlp_w=trained["pot"].w, skin=1.0,
                     dt=1.0, mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    e = []
    for _ in range(10):
        ep, ek = sim.energies()
        e.append(ep + ek)
        sim.run(100)
    ep, ek = sim.energies()
    e.append(ep + ek)
    e = np.array(e) / s.n
    T = 2 * ek / ((3 * s.n - 3) * inputs.KB_EV)
    print(f"MLP NVE 1 ps: E/N spread {np.ptp(e):.2e} eV, drift {e[-1] - e[0]:.2e} eV, T {T:.0f} K")
    assert np.isfinite(e).all()
    assert np.ptp(e) < 2e-3
