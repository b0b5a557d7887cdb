"""GPU parity of the two-element tight-binding potential (md_forces_tbm,
md_set_elements, md_run with MD_POT_TBM) against the FP64 oracle, on a
random Cu75Au25-like alloy and on two element layers.  Bars as for one
element: densities and site energies to FP32 accuracy, forces 1e-5
normwise and per atom within 1e-5 of its sum of pair-force magnitudes; the energy trace of an NVE run follows the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_00075_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
PAIRS = inputs.TB2_PAIRS
R_LIST = 5.7 + 1.0
A_ALLOY = 0.75 * inputs.CU_A0 + 0.25 * inputs.AU_A0


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_00075_amd import md
    md.lib()
    return md


def _system(orc, ncell, jit, seed, layered):
    s = inputs.jitter(inputs.eam_cu(ncell=ncell), jit, seed=seed)
    x = orc.wrap(s.x * (A_ALLOY / inputs.CU_A0), s.L * (A_ALLOY / inputs.CU_A0))
    L = s.L * (A_ALLOY / inputs.CU_A0)
    if layered:
        t = (x[:, 2] >= 0.5 * L[2]).astype(np.int32)
    else:
        t = (np.random.default_rng(seed).random(len(x)) < 0.25).astype(np.int32)
    return x, L, t


# per-kind smooth cutoffs (a separate device path from the shared cutoff)
PAIRS_CUTS = (dict(inputs.TB2_CU, rs=4.6, rc=5.1), dict(inputs.TB2_CUAU, rs=5.0, rc=5.5),
              dict(inputs.TB2_AU, rs=5.2, rc=5.7))


def _gpu_tbm(M, x, L, t, pairs=PAIRS):
    from test_gpu_parity import _gpu_lists
    n = len(x)
    rows, st = _gpu_lists(M, x, L, R_LIST)
    p = st["perm"].cpu().numpy()[:n]
    xsc = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    M.md_scale_positions(L, n, st["x"], xsc)
    M.md_set_elements(n, torch.tensor(t[p], dtype=torch.int32, device="cuda"), xsc)
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    rho = torch.zeros(n, dtype=torch.float32, device="cuda")
    fp = torch.zeros(n, dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    ea = torch.zeros(n, dtype=torch.float32, device="cuda")
    M.md_forces_tbm(L, n, xsc, st["cap"], st["idx"], st["cnt"], pairs, rho, fp, f, ev, M.MD_ENERGY, st["ws"],
                    e_atom=ea)
    out = dict(ev=ev.cpu().numpy(), w=xsc[:, 3].cpu().numpy().astype(np.uint32))
    for k, v in (("rho", rho), ("fprime", fp), ("e_atom", ea)):
        a = np.empty(n)
        a[p] = v.cpu().numpy()[:n]
        out[k] = a
    fg = np.empty((n, 3))
    fg[p] = f.cpu().numpy().T[:n]
    out["f"] = fg
    out["t_sorted"] = t[p]
    return out


@pytest.mark.parametrize("layered,seed,pairs", [(False, 61, PAIRS), (True, 62, PAIRS), (False, 64, PAIRS_CUTS)],
                         ids=["alloy", "layers", "alloy-own-cutoffs"])
def test_forces_tbm_vs_oracle(M, orc, layered, seed, pairs):
    x, L, t = _system(orc, 6, 0.1, seed, layered)
    g = _gpu_tbm(M, x, L, t, pairs)
    oc, ic = orc.neighbors_cells(x, L, R_LIST)
    r = orc.forces_tbm(x, L, oc, ic, t, pairs)
    assert np.abs(g["rho"] - r["rho"]).max() / r["rho"].max() < 1e-5
    assert np.abs(g["e_atom"] - r["e_atom"]).max() < 2e-6 * np.abs(r["e_atom"]).max()
    import force_scale as FSC
    FSC.check_form(orc, "tbm", g["f"], x, L, oc, ic, r, pairs, types=t,
                   what=f"TBM {'layers' if layered else 'alloy'}")
    assert g["ev"][0] == pytest.approx(r["ev"][0], rel=1e-6)
    for c in range(2, 5):
        assert g["ev"][c] == pytest.approx(r["ev"][c], rel=1e-5)
    # the element word after the passes: F' with its lowest bit replaced by the element
    assert np.array_equal(g["w"] & 1, g["t_sorted"].astype(np.uint32))


def _oracle_nve(orc, x, v, L, t, steps, every, dt=1.0, mass=None):
    k = 1.0 / inputs.AMU_A2_FS2_IN_EV
    m = mass[:, None]
    x, v = x.copy(), v.copy()

    def force(x):
        w = orc.wrap(x, L)
        oc, ic = orc.neighbors_cells(w, L, R_LIST)
        r = orc.forces_tbm(w, L, oc, ic, t, PAIRS)
        return r["f"], r["ev"][0]

    f, ep = force(x)
    out = []
    for step in range(steps + 1):
        if step % every == 0:
            out.append((ep + 0.5 * (m * v ** 2).sum() / k) / len(x))
        if step == steps:
            break
        v += 0.5 * dt * f * k / m
        x += dt * v
        f, ep = force(x)
        v += 0.5 * dt * f * k / m
    return np.array(out)


def test_md_run_tbm_follows_the_oracle_energy_trace(M, orc):
    """Equal masses for both elements (the driver's mass is one scalar):
    the NVE energy every 40 fs follows the oracle's velocity Verlet, and the
    elements stay with their atoms through the rebuilds."""
    from paper_1611_00075_amd.sim import Simulation
    x, L, t = _system(orc, 5, 0.05, 63, False)
    v = inputs.eam_cu(ncell=5, T=600.0, seed=63).v
    sim = Simulation(L, x, v, potential="tbm", tbm=PAIRS, types=t, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                     force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    e = []
    for _ in range(5):
        ep, ek = sim.energies()
        e.append(ep + ek)
        sim.run(40)
    ep, ek = sim.energies()
    e.append(ep + ek)
    e = np.array(e) / len(x)
    eo = _oracle_nve(orc, x, v, L, t, 200, 40, mass=np.full(len(x), inputs.CU_MASS_AMU))
    print(f"TBM NVE 200 fs: |GPU - oracle| max {np.abs(e - eo).max():.2e} eV/atom, builds {sim.builds}")
    assert np.abs(e - eo).max() < 1e-5
    assert sim.builds >= 1
    assert np.array_equal(sim.by_id(sim.types).astype(np.int32), t)
