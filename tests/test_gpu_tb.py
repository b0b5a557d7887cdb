"""GPU parity of the second-moment tight-binding potential (md_forces_tb,
md_run with MD_POT_TB) against the FP64 oracle.  Bars as for the
Finnis-Sinclair form: densities and site energies to FP32 accuracy, forces
within 1e-5 normwise and per atom within 1e-5 of its sum of pair-force
magnitudes (tests/force_scale.py)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_00075_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
TB = inputs.TB_CU
R_LIST = TB["rc"] + 1.0


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_00075_amd import md
    md.lib()
    return md


def _gpu_tb(M, x, L, r_list=R_LIST):
    from test_gpu_parity import _gpu_lists
    n = len(x)
    rows, st = _gpu_lists(M, x, L, r_list)
    xsc = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    M.md_scale_positions(L, n, st["x"], xsc)
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    rho = torch.zeros(n, dtype=torch.float32, device="cuda")
    fp = torch.zeros(n, dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    ea = torch.zeros(n, dtype=torch.float32, device="cuda")
    M.md_forces_tb(L, n, xsc, st["cap"], st["idx"], st["cnt"], TB, rho, fp, f, ev, M.MD_ENERGY, st["ws"], e_atom=ea)
    p = st["perm"].cpu().numpy()[:n]
    out = dict(ev=ev.cpu().numpy())
    for k, t in (("rho", rho), ("fprime", fp), ("e_atom", ea)):
        a = np.empty(n)
        a[p] = t.cpu().numpy()[:n]
        out[k] = a
    fg = np.empty((n, 3))
    fg[p] = f.cpu().numpy().T[:n]
    out["f"] = fg
    return out


@pytest.mark.parametrize("ncell,jit,seed", [(6, 0.1, 41), (5, 0.2, 42)])
def test_forces_tb_vs_oracle(M, orc, ncell, jit, seed):
    s = inputs.jitter(inputs.eam_cu(ncell=ncell), jit, seed=seed)
    x = orc.wrap(s.x, s.L)
    g = _gpu_tb(M, x, s.L)
    oc, ic = orc.neighbors_cells(x, s.L, R_LIST)
    r = orc.forces_tb(x, s.L, oc, ic, TB)
    assert np.abs(g["rho"] - r["rho"]).max() / r["rho"].max() < 1e-5
    assert np.abs(g["fprime"] - r["fprime"]).max() / np.abs(r["fprime"]).max() < 1e-5
    assert np.abs(g["e_atom"] - r["e_atom"]).max() < 2e-6 * np.abs(r["e_atom"]).max()
    import force_scale as FSC
    FSC.check_form(orc, "tb", g["f"], x, s.L, oc, ic, r, TB, what="TB")
    assert g["ev"][0] == pytest.approx(r["ev"][0], rel=1e-6)
    assert g["ev"][1] == pytest.approx(r["ev"][1], rel=1e-6)
    for c in range(2, 5):
        assert g["ev"][c] == pytest.approx(r["ev"][c], rel=1e-5)


def test_tb_perfect_lattice(M, orc):
    """On the perfect crystal the GPU gives the cohesive energy the
    parameters were solved for, and forces of FP32 rounding size."""
    x = inputs.fcc_sites(6, 6, 6, inputs.CU_A0)
    L = np.full(3, 6 * inputs.CU_A0)
    x = orc.wrap(x, L)
    g = _gpu_tb(M, x, L)
    assert g["ev"][0] / len(x) == pytest.approx(-3.54, rel=1e-6)
    assert np.abs(g["f"]).max() < 1e-4


def test_tb_rejects_bad_parameters(M):
    import ctypes as C
    bad = dict(TB, rs=TB["rc"])
    x = inputs.fcc_sites(3, 3, 3, inputs.CU_A0)
    n = len(x)
    xs = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    idx = torch.zeros(M.ell_size(n, 8), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    f = torch.zeros(3 * n, dtype=torch.float32, device="cuda")
    ws = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MDError) as e:
        M.md_forces_tb(np.full(3, 3 * inputs.CU_A0), n, xs, 8, idx, cnt, bad, v, v, f, None, 0, ws)
    assert e.value.code == M.MD_ERR_ARG
    assert C.sizeof(M.System) > C.sizeof(M.TB)


def _oracle_nve(orc, x, v, L, steps, every, dt=1.0):
    """Total energy per atom every `every` velocity-Verlet steps with the
    oracle's FP64 forces (lists rebuilt every step)."""
    m, k = inputs.CU_MASS_AMU, 1.0 / inputs.AMU_A2_FS2_IN_EV
    x, v = x.copy(), v.copy()

    def force(x):
        w = orc.wrap(x, L)
        oc, ic = orc.neighbors_cells(w, L, R_LIST)
        r = orc.forces_tb(w, L, oc, ic, TB)
        return r["f"], r["ev"][0]

    f, ep = force(x)
    out = []
    for step in range(steps + 1):
        if step % every == 0:
            out.append((ep + 0.5 * m * (v ** 2).sum() / k) / len(x))
        if step == steps:
            break
        v += 0.5 * dt * f * k / m
        x += dt * v
        f, ep = force(x)
        v += 0.5 * dt * f * k / m
    return np.array(out)


def test_md_run_tb_follows_the_oracle_energy_trace(M, orc):
    """NVE through the native driver (rebuilds included): the total energy
    every 40 fs follows the FP64 oracle's velocity-Verlet trace (whose own
    Verlet fluctuation is ~2e-5 eV per atom) to FP32 accuracy."""
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.eam_cu(ncell=6, T=600.0, seed=43)
    sim = Simulation(s.L, s.x, s.v, potential="tb", tb=TB, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                     force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    e = []
    for _ in range(5):
        ep, ek = sim.energies()
        e.append(ep + ek)
        sim.run(40)
    ep, ek = sim.energies()
    e.append(ep + ek)
    e = np.array(e) / s.n
    eo = _oracle_nve(orc, s.x, s.v, s.L, 200, 40)
    print(f"TB NVE 200 fs: GPU E/N {e}, |GPU - oracle| max {np.abs(e - eo).max():.2e} eV, builds {sim.builds}")
    assert np.abs(e - eo).max() < 1e-5
    assert sim.builds >= 1
