"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: bit-exact wrapped positions, cell assignments and neighbour sets;
FP32 forces within 1e-5 normwise (the tolerance the method is specified
to) and per atom within 1e-5 of the sum of pair-force magnitudes, except
for atoms with a pair within 1e-5 of the cutoff, where the FP32 and FP64
cutoff tests may legitimately disagree (both results are checked);
FP64 forces within 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_00075_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_00075_amd import md
    md.lib()
    return md


def _dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _bin(M, x, L, r_list, reach=1):
    n = len(x)
    g = M.md_grid_init(L, r_list, reach)
    ws = torch.empty(M.md_workspace_bytes(g, n), dtype=torch.uint8, device="cuda")
    M.md_workspace_init(g, n, ws)
    xd = _dev(x.T, torch.float64)
    cell = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    perm = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    cs = torch.empty(g.n_cells + 1, dtype=torch.int32, device="cuda")
    M.md_bin_cells(g, n, xd, cell, perm, cs, ws)
    torch.cuda.synchronize()
    return g, ws, xd, cell, perm, cs


CASES = [
    # (name, L, r_list, n, seed, reach)
    ("gas_nc3", (10.0, 10.0, 10.0), 2.8, 700, 1, 1),
    ("gas_nc2_mixed", (6.0, 7.0, 11.0), 2.9, 300, 2, 1),
    ("gas_reach2", (12.0, 9.0, 10.0), 2.5, 900, 3, 2),
    ("gas_tiny_nc2", (3.0, 3.0, 3.0), 1.45, 37, 4, 1),
    ("gas_ragged", (17.3, 11.1, 13.7), 2.8, 3001, 5, 1),
    # about 130 atoms per cell: several home batches and candidate tiles per cell
    ("gas_dense", (16.0, 16.0, 16.0), 3.9, 8000, 6, 1),
]


@pytest.mark.parametrize("name,L,r_list,n,seed,reach", CASES)
def test_bin_cells_bit_exact(M, orc, name, L, r_list, n, seed, reach):
    L = np.array(L)
    x = inputs.random_gas(n, L, seed) + np.random.default_rng(seed).integers(-2, 3, (n, 3)) * L
    g, ws, xd, cell, perm, cs = _bin(M, x, L, r_list, reach)
    # wrap: bitwise equal to the oracle
    w_or = orc.wrap(x, L)
    w_gpu = xd.cpu().numpy().T
    assert np.array_equal(w_gpu.view(np.uint64), w_or.view(np.uint64))
    # cell coordinates per atom: bitwise equal
    nc = np.array(g.nc[:])
    c_or = orc.cell_coords(w_or, L, nc)
    ranks = M.md_grid_cell_ranks(g)
    lin = np.empty(g.n_cells, np.int64)
    lin[ranks] = np.arange(g.n_cells)
    l = lin[cell.cpu().numpy()[:n]]
    c_gpu = np.stack([l % nc[0], (l // nc[0]) % nc[1], l // (nc[0] * nc[1])], 1)
    assert np.array_equal(c_gpu, c_or)
    # stable counting sort: perm sorted by rank, ties in input order
    p = perm.cpu().numpy()[:n]
    assert np.array_equal(np.sort(p), np.arange(n))
    r_or = ranks[c_or[:, 0] + nc[0] * (c_or[:, 1] + nc[1] * c_or[:, 2])]
    assert np.array_equal(p, np.lexsort((np.arange(n), r_or)))
    counts = np.bincount(r_or, minlength=g.n_cells)
    assert np.array_equal(cs.cpu().numpy(), np.concatenate([[0], np.cumsum(counts)]))


def _gpu_lists(M, x, L, r_list, reach=1, row_cap=8):
    """Bin, sort and build lists on the GPU; rows mapped back to input ids.
    Starts with a small row capacity to exercise the capacity protocol."""
    n = len(x)
    g, ws, xd, cell, perm, cs = _bin(M, x, L, r_list, reach)
    xs = torch.empty_like(xd)
    M.md_permute(n, 3, perm, xd, xs, 8)
    cnt = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    mx = torch.zeros(1, dtype=torch.int32, device="cuda")
    idx = torch.empty(max(M.ell_size(n, row_cap), 1), dtype=torch.int32, device="cuda")
    rc, longest = M.md_build_neighbors(g, n, xs, cs, row_cap, idx, cnt, mx, ws)
    if longest > row_cap:
        assert rc == M.MD_ERR_CAPACITY
        row_cap = (longest + 7) // 8 * 8
        idx = torch.empty(max(M.ell_size(n, row_cap), 1), dtype=torch.int32, device="cuda")
        rc, longest2 = M.md_build_neighbors(g, n, xs, cs, row_cap, idx, cnt, mx, ws)
        assert rc == M.MD_OK and longest2 == longest
    assert int(mx[0]) == longest
    p = perm.cpu().numpy()[:n]
    r = M.ell_rows(n, row_cap, idx, cnt)
    rows = [None] * n
    for k in range(n):
        rows[p[k]] = np.sort(p[r[k]])
    need = int(cnt[:n].sum()) if n else 0
    return rows, dict(g=g, ws=ws, x=xs, perm=perm, cap=row_cap, idx=idx, cnt=cnt, need=need)


@pytest.mark.parametrize("name,L,r_list,n,seed,reach", CASES)
def test_neighbor_sets_bit_exact(M, orc, name, L, r_list, n, seed, reach):
    L = np.array(L)
    x = orc.wrap(inputs.random_gas(n, L, seed), L)
    rows, _ = _gpu_lists(M, x, L, r_list, reach)
    ob, ib = orc.neighbors_brute(x, L, r_list)
    for i in range(n):
        assert np.array_equal(rows[i], ib[ob[i]:ob[i + 1]]), f"row {i}"


def test_neighbor_sets_fcc_lattice(M, orc):
    s = inputs.jitter(inputs.lj_fcc(ncell=8), 0.05, seed=9)
    x = orc.wrap(s.x, s.L)
    rows, st = _gpu_lists(M, x, s.L, 2.8)
    oc, ic = orc.neighbors_cells(x, s.L, 2.8)
    assert st["need"] == len(ic)
    for i in range(len(x)):
        assert np.array_equal(rows[i], ic[oc[i]:oc[i + 1]])


def test_empty_and_single_atom(M):
    L = np.array([10.0, 10.0, 10.0])
    for n in (0, 1):
        x = np.full((n, 3), 1.5)
        g, ws, xd, cell, perm, cs = _bin(M, x, L, 2.8)
        assert int(cs[-1]) == n
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        mx = torch.zeros(1, dtype=torch.int32, device="cuda")
        idx = torch.empty(64, dtype=torch.int32, device="cuda")
        rc, longest = M.md_build_neighbors(g, n, xd, cs, 8, idx, cnt, mx, ws)
        assert rc == M.MD_OK and longest == 0


def test_abi_rejects_bad_arguments(M):
    with pytest.raises(M.MDError) as e:
        M.md_grid_init([5.0, 5.0, 5.0], 2.6)          # r_list >= L/2
    assert e.value.code == M.MD_ERR_BOX
    with pytest.raises(M.MDError):
        M.md_grid_init([5.0, 5.0, 5.0], 1.0, reach=3)
    # row capacity past the largest the list layout addresses
    g, ws, xd, cell, perm, cs = _bin(M, np.zeros((0, 3)), np.array([10.0, 10.0, 10.0]), 2.8)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    mx = torch.zeros(1, dtype=torch.int32, device="cuda")
    idx = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(M.MDError) as e:
        M.md_build_neighbors(g, 0, xd, cs, M.MD_MAX_ROW_CAP + 8, idx, cnt, mx, ws)
    assert e.value.code == M.MD_ERR_ARG


# ---------------------------------------------------------------------------
# forces
# ---------------------------------------------------------------------------

def _lj_setup(M, x, L, r_list=2.8):
    n = len(x)
    rows, st = _gpu_lists(M, x, L, r_list)
    xsc = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    M.md_scale_positions(L, n, st["x"], xsc)
    return st, xsc


def _check_forces(f_gpu, f_ref, fabs_sum, near_cut, contrib, tol=1e-5):
    """Normwise and per-atom checks; atoms in `near_cut` may differ by the
    contribution of their near-cutoff pairs (`contrib`)."""
    err = np.linalg.norm(f_gpu - f_ref) / np.linalg.norm(f_ref)
    assert err <= tol, err
    d = np.linalg.norm(f_gpu - f_ref, axis=1)
    ok = d <= tol * fabs_sum + 1e-12
    for i in np.nonzero(~ok)[0]:
        assert i in near_cut, (i, d[i], fabs_sum[i])
        alt = np.linalg.norm(f_gpu[i] - (f_ref[i] + contrib[i]))
        assert alt <= tol * fabs_sum[i] + 1e-12
    return err


def _pair_sums_lj(x, L, off, idx, rc):
    """Per-atom sum of |f_ij| and near-cutoff bookkeeping (host numpy)."""
    n = len(x)
    fabs = np.zeros(n)
    near = set()
    contrib = np.zeros((n, 3))
    for i in range(n):
        js = idx[off[i]:off[i + 1]]
        d = x[i] - x[js]
        d -= L * np.round(d / L)
        r2 = np.sum(d * d, 1)
        m = r2 < rc * rc
        s6 = 1.0 / r2 ** 3
        fs = 24 * s6 * (2 * s6 - 1) / r2
        fabs[i] = np.sum(np.abs(fs[m]) * np.sqrt(r2[m]))
        amb = np.abs(np.sqrt(r2) - rc) < 1e-5 * rc
        if amb.any():
            near.add(i)
            sgn = np.where(m[amb], -1.0, 1.0)      # a flip removes or adds the pair
            contrib[i] = np.sum((sgn * fs[amb])[:, None] * d[amb], 0)
    return fabs, near, contrib


@pytest.mark.parametrize("ncell,jit,seed", [(6, 0.06, 1), (9, 0.08, 2)])
def test_forces_lj_fp32_vs_oracle(M, orc, ncell, jit, seed):
    s = inputs.jitter(inputs.lj_fcc(ncell=ncell), jit, seed=seed)
    x = orc.wrap(s.x, s.L)
    n = len(x)
    st, xsc = _lj_setup(M, x, s.L)
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.md_forces_lj(s.L, n, st["x"], xsc, st["cap"], st["idx"], st["cnt"], (1.0, 1.0, 2.5), f, ev, M.MD_ENERGY,
                   st["ws"])
    p = st["perm"].cpu().numpy()[:n]
    fg = np.empty((n, 3))
    fg[p] = f.cpu().numpy().T.astype(np.float64)
    oc, ic = orc.neighbors_cells(x, s.L, 2.8)
    fo, evo = orc.forces_lj(x, s.L, oc, ic, rc=2.5)
    fabs, near, contrib = _pair_sums_lj(x, s.L, oc, ic, 2.5)
    err = _check_forces(fg, fo, fabs, near, contrib)
    print(f"LJ FP32 force error (normwise) {err:.3e}")
    evg = ev.cpu().numpy()
    assert evg[0] == pytest.approx(evo[0], rel=2e-6)
    assert evg[1] == pytest.approx(evo[1], rel=2e-6)
    for c in range(2, 5):
        assert evg[c] == pytest.approx(evo[c], rel=2e-6)
    scale = abs(evo[2])
    assert np.abs(evg[5:] - evo[5:]).max() < 2e-6 * scale


def test_forces_lj_fp64_vs_oracle(M, orc):
    s = inputs.jitter(inputs.lj_fcc(ncell=7), 0.07, seed=3)
    x = orc.wrap(s.x, s.L)
    n = len(x)
    st, _ = _lj_setup(M, x, s.L)
    f = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.md_forces_lj(s.L, n, st["x"], None, st["cap"], st["idx"], st["cnt"], (1.0, 1.0, 2.5), f, ev,
                   M.MD_ENERGY | M.MD_PAIR_FP64, st["ws"])
    p = st["perm"].cpu().numpy()[:n]
    fg = np.empty((n, 3))
    fg[p] = f.cpu().numpy().T
    oc, ic = orc.neighbors_cells(x, s.L, 2.8)
    fo, evo = orc.forces_lj(x, s.L, oc, ic, rc=2.5)
    assert np.linalg.norm(fg - fo) / np.linalg.norm(fo) < 1e-12
    assert np.allclose(ev.cpu().numpy(), evo, rtol=1e-12, atol=1e-9)


def test_forces_lj_deterministic(M, orc):
    s = inputs.jitter(inputs.lj_fcc(ncell=6), 0.05, seed=8)
    x = orc.wrap(s.x, s.L)
    n = len(x)
    st, xsc = _lj_setup(M, x, s.L)
    out = []
    for _ in range(2):
        f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
        ev = torch.zeros(8, dtype=torch.float64, device="cuda")
        M.md_forces_lj(s.L, n, st["x"], xsc, st["cap"], st["idx"], st["cnt"], (1.0, 1.0, 2.5), f, ev,
                       M.MD_ENERGY, st["ws"])
        out.append((f.cpu().numpy(), ev.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_forces_eam_vs_oracle(M, orc):
    s = inputs.jitter(inputs.eam_cu(ncell=6), 0.1, seed=4)
    x = orc.wrap(s.x, s.L)
    n = len(x)
    r_list = 5.4
    rows, st = _gpu_lists(M, x, s.L, r_list)
    xsc = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    M.md_scale_positions(s.L, n, st["x"], xsc)
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    rho = torch.zeros(n, dtype=torch.float32, device="cuda")
    fp = torch.zeros(n, dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    ea = torch.zeros(n, dtype=torch.float32, device="cuda")
    M.md_forces_eam(s.L, n, xsc, st["cap"], st["idx"], st["cnt"], inputs.FS_CU, rho, fp, f, ev, M.MD_ENERGY,
                    st["ws"], e_atom=ea)
    p = st["perm"].cpu().numpy()[:n]
    eg = np.empty(n)
    eg[p] = ea.cpu().numpy()
    fg = np.empty((n, 3))
    fg[p] = f.cpu().numpy().T
    rg = np.empty(n)
    rg[p] = rho.cpu().numpy()
    oc, ic = orc.neighbors_cells(x, s.L, r_list)
    r = orc.forces_eam(x, s.L, oc, ic, inputs.FS_CU)
    assert np.abs(rg - r["rho"]).max() / r["rho"].max() < 1e-5
    # site energies F(rho_i) + 1/2 sum_j V(r_ij): FP32 values of ~3.5 eV
    assert np.abs(eg - r["e_atom"]).max() < 2e-6 * np.abs(r["e_atom"]).max()
    import force_scale as FSC
    FSC.check_form(orc, "fs", fg, x, s.L, oc, ic, r, inputs.FS_CU, what="EAM")
    evg = ev.cpu().numpy()
    assert evg[0] == pytest.approx(r["ev"][0], rel=1e-6)
    assert evg[1] == pytest.approx(r["ev"][1], rel=1e-6)
    for c in range(2, 5):
        assert evg[c] == pytest.approx(r["ev"][c], rel=1e-5)


# ---------------------------------------------------------------------------
# dynamics
# ---------------------------------------------------------------------------

def test_vv_trajectory_fp64_within_oracle_envelope(M, orc):
    """10^3-cell LJ crystal (4,000 atoms), 100 NVE steps, FP64 pair path:
    the GPU trajectory stays within 10x the oracle's own sensitivity to the
    order of summation (natural vs reversed neighbour order)."""
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.lj_fcc(ncell=10)
    steps = 100
    a = orc.md_run(s.x.copy(), s.v.copy(), s.L, steps, r_list=2.8, skin=0.3, dt=0.005)
    b = orc.md_run(s.x.copy(), s.v.copy(), s.L, steps, r_list=2.8, skin=0.3, dt=0.005, reverse_order=True)
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005, pair_fp64=True)
    e0 = sim.energies()
    for _ in range(steps):
        sim.step()
    xg = sim.positions()

    def dev(p, q):
        d = p - q
        d -= s.L * np.round(d / s.L)
        return np.abs(d).max()

    env = max(dev(a["x"], b["x"]), 1e-13)
    assert dev(xg, a["x"]) <= 10 * env, (dev(xg, a["x"]), env)
    assert sim.builds == a["builds"]
    ep, ek = sim.energies()
    assert ep + ek == pytest.approx(a["epot"][-1] + a["ekin"][-1], rel=1e-10)
    assert e0[0] + e0[1] == pytest.approx(a["epot"][0] + a["ekin"][0], rel=1e-11)


def test_vv_fp32_energy_conservation(M, orc):
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.lj_fcc(ncell=10)
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005)
    e = [sum(sim.energies())]
    for k in range(100):
        sim.step()
        if k % 10 == 9:
            e.append(sum(sim.energies()))
    a = orc.md_run(s.x.copy(), s.v.copy(), s.L, 100, r_list=2.8, skin=0.3, dt=0.005)
    eo = a["epot"] + a["ekin"]
    # same energy trace as the oracle to FP32 accuracy
    assert np.abs(np.array(e) - eo[::10]).max() / s.n < 1e-4
    # FP32 forces cancel only to rounding: total momentum stays small
    assert np.abs(sim.velocities().sum(0)).max() < 1e-3


def test_md_run_matches_per_call_path(M, orc):
    """The native driver (fused kicks) and the per-call API take the same
    trajectory up to rounding, with the same list rebuilds."""
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.lj_fcc(ncell=8)
    a = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005, pair_fp64=True)
    b = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005, pair_fp64=True)
    for _ in range(60):
        a.step()
    b.run(25)
    b.run(35)
    assert a.builds == b.builds and b.step_count == 60
    d = a.positions() - b.positions()
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-10
    assert np.abs(a.velocities() - b.velocities()).max() < 1e-9


def test_md_run_fp64_trajectory_within_oracle_envelope(M, orc):
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.lj_fcc(ncell=10)
    steps = 100
    a = orc.md_run(s.x.copy(), s.v.copy(), s.L, steps, r_list=2.8, skin=0.3, dt=0.005)
    b = orc.md_run(s.x.copy(), s.v.copy(), s.L, steps, r_list=2.8, skin=0.3, dt=0.005, reverse_order=True)
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005, pair_fp64=True)
    sim.run(steps)

    def dev(p, q):
        d = p - q
        d -= s.L * np.round(d / s.L)
        return np.abs(d).max()

    env = max(dev(a["x"], b["x"]), 1e-13)
    assert dev(sim.positions(), a["x"]) <= 10 * env, (dev(sim.positions(), a["x"]), env)
    assert sim.builds == a["builds"]


def test_md_run_capacity_protocol_resumes(M):
    """A row capacity far too small: md_run stops with MD_ERR_CAPACITY in the
    middle of a step, the caller grows the list and the run resumes to the
    same state as an unconstrained run."""
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.jitter(inputs.lj_fcc(ncell=8), 0.02, seed=5)
    ref = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005, pair_fp64=True)
    ref.run(40)
    sim = Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005, pair_fp64=True)
    sim.row_cap = 8                      # force the protocol at the next rebuild
    sim.idx = torch.empty(M.ell_size(sim.n, 8), dtype=torch.int32, device="cuda")
    sim._sys.need_build = 1
    sim.run(40)
    assert sim.row_cap >= sim.longest or sim.row_cap > 8
    d = sim.positions() - ref.positions()
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-10


def test_md_run_eam_energy_conservation(M, orc):
    """EAM (FP32 pair path) through the driver: the energy trace follows the
    FP64 oracle's to FP32 accuracy."""
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.eam_cu(ncell=6, T=600.0)
    kw = dict(potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
              force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    sim = Simulation(s.L, s.x, s.v, **kw)
    e = []
    for k in range(5):
        ep, ek = sim.energies()
        e.append(ep + ek)
        sim.run(20)
    ep, ek = sim.energies()
    e.append(ep + ek)
    a = orc.md_run(s.x.copy(), s.v.copy(), s.L, 100, potential="eam", fs=inputs.FS_CU, r_list=5.4, skin=1.0,
                   dt=1.0, mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    eo = a["epot"] + a["ekin"] * inputs.AMU_A2_FS2_IN_EV
    assert np.abs(np.array(e) - eo[::20]).max() / s.n < 2e-5
