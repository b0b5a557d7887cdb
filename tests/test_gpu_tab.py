"""GPU parity of the tabulated embedded-atom form (md_tab_pack,
md_forces_tab, md_run with MD_POT_TAB) against the FP64 oracle on the same
knot arrays.  Tables: the Finnis-Sinclair Cu-like functions sampled at
dr = 0.005 A (the benchmark's table), a coarse table with perturbed slopes
(not a sampled polynomial anywhere), and a short F table that the crystal's
densities run past (tangent continuation).  Bars as for the analytic
forms: densities and site energies to FP32 accuracy, forces 1e-5 normwise
and per atom within 1e-5 of its sum of pair-force magnitudes, energy and virial 1e-6 / 1e-5 relative."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_00075_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
FS = inputs.FS_CU


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_00075_amd import md
    md.lib()
    return md


def _perturbed(seed=81):
    tab = inputs.fs_table(FS, dr=0.05, drho=0.5)
    rng = np.random.default_rng(seed)
    for k in ("dpsi", "dphi", "dF"):
        tab[k] = tab[k] * (1 + 0.05 * rng.normal(size=len(tab[k])))
    return tab


TABLES = {
    "fs-fine": lambda: inputs.fs_table(FS),
    "perturbed-coarse": _perturbed,
    "short-F": lambda: inputs.fs_table(FS, drho=0.25, rho_max=30.0),
}


def _system(orc, cells, jit, seed):
    nx, ny, nz = cells
    x = inputs.fcc_sites(nx, ny, nz, inputs.CU_A0)
    L = np.array([nx, ny, nz], dtype=np.float64) * inputs.CU_A0
    x = x + np.random.default_rng(seed).normal(0.0, jit, size=x.shape)
    return orc.wrap(x, L), L


def _gpu_tab(M, x, L, tab, r_list):
    from test_gpu_parity import _gpu_lists
    n = len(x)
    rows, st = _gpu_lists(M, x, L, r_list)
    p = st["perm"].cpu().numpy()[:n]
    table = torch.empty(M.md_tab_bytes(tab), dtype=torch.uint8, device="cuda")
    M.md_tab_pack(tab, table)
    xsc = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    M.md_scale_positions(L, n, st["x"], xsc)
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    rho = torch.zeros(n, dtype=torch.float32, device="cuda")
    fp = torch.zeros(n, dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    ea = torch.zeros(n, dtype=torch.float32, device="cuda")
    M.md_forces_tab(L, n, xsc, st["cap"], st["idx"], st["cnt"], tab, table, rho, fp, f, ev, M.MD_ENERGY, st["ws"],
                    e_atom=ea)
    out = dict(ev=ev.cpu().numpy())
    for k, v in (("rho", rho), ("fprime", fp), ("e_atom", ea)):
        a = np.empty(n)
        a[p] = v.cpu().numpy()[:n]
        out[k] = a
    fg = np.empty((n, 3))
    fg[p] = f.cpu().numpy().T[:n]
    out["f"] = fg
    return out


@pytest.mark.parametrize("table", list(TABLES))
@pytest.mark.parametrize("cells,seed", [((6, 6, 6), 82), ((5, 6, 7), 83)], ids=["cubic-864", "box-5x6x7"])
def test_forces_tab_vs_oracle(M, orc, table, cells, seed):
    tab = TABLES[table]()
    x, L = _system(orc, cells, 0.1, seed)
    rc = (len(tab["psi"]) - 1) * tab["dr"]
    g = _gpu_tab(M, x, L, tab, rc + 1.0)
    oc, ic = orc.neighbors_cells(x, L, rc + 1.0)
    r = orc.forces_tab(x, L, oc, ic, tab)
    assert np.abs(g["rho"] - r["rho"]).max() < 1e-5 * r["rho"].max()
    assert np.abs(g["fprime"] - r["fprime"]).max() < 1e-5 * np.abs(r["fprime"]).max()
    assert np.abs(g["e_atom"] - r["e_atom"]).max() < 2e-6 * np.abs(r["e_atom"]).max()
    import force_scale as FSC
    FSC.check_form(orc, "tab", g["f"], x, L, oc, ic, r, tab, what=f"TAB {table} {cells}")
    assert g["ev"][0] == pytest.approx(r["ev"][0], rel=1e-6)
    assert g["ev"][1] == pytest.approx(r["ev"][1], rel=1e-6)
    for c in range(2, 5):
        assert g["ev"][c] == pytest.approx(r["ev"][c], rel=1e-5)
    if table == "short-F":
        assert r["rho"].max() > 30.0        # the tangent continuation was exercised


def test_tabulated_fs_tracks_the_analytic_fs_kernels(M, orc):
    """The same crystal through md_forces_eam (analytic) and md_forces_tab
    (fine table): both FP32, within the FP32 error of each."""
    x, L = _system(orc, (6, 6, 6), 0.1, 84)
    tab = inputs.fs_table(FS)
    g = _gpu_tab(M, x, L, tab, 5.4)
    oc, ic = orc.neighbors_cells(x, L, 5.4)
    a = orc.forces_eam(x, L, oc, ic, FS)
    err = np.linalg.norm(g["f"] - a["f"]) / np.linalg.norm(a["f"])
    assert err < 1e-5, err


def test_empty_system_and_argument_checks(M):
    tab = inputs.fs_table(FS)
    table = torch.empty(M.md_tab_bytes(tab), dtype=torch.uint8, device="cuda")
    M.md_tab_pack(tab, table)
    L = np.full(3, 30.0)
    xs = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    z32 = torch.zeros(8, dtype=torch.int32, device="cuda")
    g = M.md_grid_init(L, 5.4, 1)
    ws = torch.empty(M.md_workspace_bytes(g, 0), dtype=torch.uint8, device="cuda")
    M.md_workspace_init(g, 0, ws)
    ev = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    f = torch.zeros(3, dtype=torch.float32, device="cuda")
    r = torch.zeros(1, dtype=torch.float32, device="cuda")
    M.md_forces_tab(L, 0, xs, 8, z32, z32, tab, table, r, r, f, ev, M.MD_ENERGY, ws)
    torch.cuda.synchronize()
    assert np.all(ev.cpu().numpy() == 0.0)
    bad = dict(tab)
    bad["phi"] = tab["phi"].copy()
    bad["phi"][3] = np.nan
    with pytest.raises(M.MDError):
        M.md_tab_pack(bad, table)
    big = dict(tab, psi=np.zeros(2002), dpsi=np.zeros(2002), phi=np.zeros(2002), dphi=np.zeros(2002))
    assert M.md_tab_bytes(big) == 0


def _oracle_nve(orc, x, v, L, tab, r_list, steps, every, dt=1.0):
    k = 1.0 / inputs.AMU_A2_FS2_IN_EV
    m = inputs.CU_MASS_AMU
    x, v = x.copy(), v.copy()

    def force(x):
        w = orc.wrap(x, L)
        oc, ic = orc.neighbors_cells(w, L, r_list)
        r = orc.forces_tab(w, L, oc, ic, tab)
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


def test_md_run_tab_follows_the_oracle_energy_trace(M, orc):
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.eam_cu(ncell=5, T=600.0, seed=85)
    tab = inputs.fs_table(FS)
    sim = Simulation(s.L, s.x, s.v, potential="tab", tab=tab, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                     force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    e = []
    for _ in range(5):
        ep, ek = sim.energies()
        e.append(ep + ek)
        sim.run(40)
    ep, ek = sim.energies()
    e.append(ep + ek)
    e = np.array(e) / s.n
    eo = _oracle_nve(orc, s.x, s.v, s.L, tab, 5.4, 200, 40)
    print(f"TAB NVE 200 fs: |GPU - oracle| max {np.abs(e - eo).max():.2e} eV/atom, builds {sim.builds}")
    assert np.abs(e - eo).max() < 1e-5
    assert sim.builds >= 1
