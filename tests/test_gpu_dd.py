"""GPU tests of the domain decomposition on one device (md_dd_rebuild,
md_dd_forces, md_dd_run): forces and energies against the FP64 oracle for
LJ and FS with several brick layouts (cubic and non-cubic brick frames),
the ghost sets against an independent count of periodic images in each
brick's halo shell, every ghost slot against its source position, inner
atoms free of ghost neighbours, buffer growth, determinism, and NVE energy
traces against the oracle's velocity Verlet."""
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


def _lj(orc, seed=91):
    s = inputs.jitter(inputs.lj_fcc(ncell=14), 0.05, seed=seed)
    return orc.wrap(s.x, s.L), s.v, s.L


def _cu(orc, seed=92):
    s = inputs.jitter(inputs.eam_cu(ncell=12), 0.08, seed=seed)
    return orc.wrap(s.x, s.L), s.v, s.L


def _dd(x, v, L, p, potential, **kw):
    from paper_1611_00075_amd.dd import DomainSimulation
    if potential == "lj":
        return DomainSimulation(L, x, v, p=p, potential="lj", skin=0.3, dt=0.005, **kw)
    return DomainSimulation(L, x, v, p=p, potential="eam", fs=FS, skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                            force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV, **kw)


LAYOUTS = [(1, 1, 1), (2, 2, 2), (2, 1, 2)]


@pytest.mark.parametrize("p", LAYOUTS, ids=["1x1x1", "2x2x2", "2x1x2"])
def test_lj_forces_vs_oracle(M, orc, p):
    x, v, L = _lj(orc)
    sim = _dd(x, v, L, p, "lj")
    sim.compute_forces(energy=True)
    ev = sim.ev.cpu().numpy()
    fg = sim.forces().astype(np.float64)
    off, idx = orc.neighbors_cells(x, L, 2.8)
    fo, evo = orc.forces_lj(x, L, off, idx)
    err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    print(f"DD LJ {p}: force error (normwise) {err:.2e}, ghosts {sim.dd.n_ghost}")
    assert err < 1e-5
    assert ev[0] == pytest.approx(evo[0], rel=1e-6)
    assert ev[1] == pytest.approx(evo[1], rel=1e-6)
    for c in range(2, 5):
        assert ev[c] == pytest.approx(evo[c], rel=1e-5)
    sim.close()


@pytest.mark.parametrize("p", LAYOUTS, ids=["1x1x1", "2x2x2", "2x1x2"])
def test_fs_forces_vs_oracle(M, orc, p):
    x, v, L = _cu(orc)
    sim = _dd(x, v, L, p, "eam")
    sim.compute_forces(energy=True)
    ev = sim.ev.cpu().numpy()
    fg = sim.forces().astype(np.float64)
    off, idx = orc.neighbors_cells(x, L, 5.4)
    r = orc.forces_eam(x, L, off, idx, FS)
    err = np.linalg.norm(fg - r["f"]) / np.linalg.norm(r["f"])
    print(f"DD FS {p}: force error (normwise) {err:.2e}, ghosts {sim.dd.n_ghost}")
    assert err < 1e-5
    rho = sim.by_id(sim.rho.cpu().numpy())
    assert np.abs(rho - r["rho"]).max() < 1e-5 * r["rho"].max()
    assert ev[0] == pytest.approx(r["ev"][0], rel=1e-6)
    assert ev[1] == pytest.approx(r["ev"][1], rel=1e-6)
    for c in range(2, 5):
        assert ev[c] == pytest.approx(r["ev"][c], rel=1e-5)
    sim.close()


def _brick_geometry(sim):
    dd = sim.dd
    p = np.array(dd.p[:])
    B = sim.L / p
    c = np.array(dd.c[:])
    return p, B, c


@pytest.mark.parametrize("p,system", [((2, 2, 2), "lj"), ((2, 1, 2), "lj"), ((1, 1, 1), "eam")])
def test_ghosts_are_the_images_in_each_halo_shell(M, orc, p, system):
    x, v, L = _lj(orc) if system == "lj" else _cu(orc)
    sim = _dd(x, v, L, p, system)
    dd = sim.dd
    pv, B, c = _brick_geometry(sim)
    xb = sim.x.cpu().numpy().T           # wrapped at the build, grouped by brick
    G = dd.n_ghost
    gh = sim.gh.cpu().numpy()[:, :G]
    src, slot, code = gh[0], gh[1], gh[2]
    xs = sim.xs.cpu().numpy().view(np.uint32)
    kv = 4294967296.0 / np.array(dd.vbox.L[:])
    shifts = np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij")).reshape(3, -1).T * L
    for t in range(dd.n_bricks):
        tc = np.array([t % pv[0], (t // pv[0]) % pv[1], t // (pv[0] * pv[1])])
        o = tc * B
        # independent count: images of all atoms in the shell around brick t
        want = 0
        for sh in shifts:
            y = xb + sh
            in_shell = np.all((y >= o - c) & (y < o + B + c), axis=1)
            in_brick = np.all((y >= o) & (y < o + B), axis=1)
            want += int(np.count_nonzero(in_shell & ~in_brick))
        g0, g1 = dd.ghost_start[t], dd.ghost_start[t + 1]
        assert g1 - g0 == want, (t, g1 - g0, want)
        # each entry: one image of its source in the shell (a source can
        # have two, through different periodic shifts), placed in the slot
        # at its frame position; no (source, image) pair twice
        ks = np.arange(g0, g1)
        assert np.all(code[ks] // 27 == t)
        ys = xb[src[ks]][:, None, :] + shifts[None, :, :]
        ok = np.all((ys >= o - c) & (ys < o + B + c), axis=2) & ~np.all((ys >= o) & (ys < o + B), axis=2)
        frame = xs[slot[ks], :3].astype(np.float64) / kv
        y_gpu = frame + o - c
        near = np.abs(ys - y_gpu[:, None, :]).max(axis=2) < 1e-6 * L.max()
        hit = ok & near
        assert np.all(hit.sum(1) == 1)
        pairs = src[ks].astype(np.int64) * 27 + hit.argmax(1)
        assert len(np.unique(pairs)) == len(ks)
        s0, s1 = dd.slot0[t], dd.slot0[t + 1]
        nt = dd.brick_start[t + 1] - dd.brick_start[t]
        assert np.all((slot[ks] >= s0 + nt) & (slot[ks] < s0 + nt + (g1 - g0)))
    # every slot of every brick's ghost range is filled once
    assert len(np.unique(slot)) == G
    sim.close()


def test_inner_atoms_list_no_ghosts(M, orc):
    x, v, L = _cu(orc)
    sim = _dd(x, v, L, (2, 2, 2), "eam")
    dd = sim.dd
    cap = sim.row_cap
    total_inner = 0
    for t in range(dd.n_bricks):
        nt = dd.brick_start[t + 1] - dd.brick_start[t]
        m = nt + dd.ghost_start[t + 1] - dd.ghost_start[t]
        s0 = dd.slot0[t]
        rows = M.ell_rows(m, cap, sim.idx[s0 * cap:], sim.count[s0:])
        ni = dd.n_inner[t]
        total_inner += ni
        assert 0 < ni < nt
        for i in range(ni):
            assert np.all(rows[i] < nt)
        # outer atoms do see ghosts (the split is not empty on the other side)
        assert any(np.any(rows[i] >= nt) for i in range(ni, nt))
    assert total_inner > 0
    sim.close()


def test_buffers_grow_and_results_stay(M, orc):
    x, v, L = _lj(orc, seed=93)
    a = _dd(x, v, L, (2, 2, 2), "lj")
    b = _dd(x, v, L, (2, 2, 2), "lj", ghost_slack=0.01, row_cap=8)
    assert b.ghost_cap >= b.dd.n_ghost and b.row_cap >= 40
    fa, fb = a.forces(), b.forces()
    assert np.array_equal(fa, fb)
    # repeated evaluation and one stream instead of two: the same bits
    b.compute_forces()
    fb2 = b.forces()
    from paper_1611_00075_amd import md as M2
    M2.md_dd_forces(b.dd, None, 0, comm=None)
    assert np.array_equal(fb, fb2) and np.array_equal(fb, b.forces())
    a.close()
    b.close()


def test_lj_run_follows_the_oracle_energy_trace(M, orc):
    s = inputs.lj_fcc(ncell=14)
    sim = _dd(s.x, s.v, s.L, (2, 2, 2), "lj")
    e = [sum(sim.energies())]
    for _ in range(5):
        sim.run(20)
        e.append(sum(sim.energies()))
    a = orc.md_run(s.x.copy(), s.v.copy(), s.L, 100, r_list=2.8, skin=0.3, dt=0.005)
    eo = a["epot"] + a["ekin"]
    d = np.abs(np.array(e) - eo[::20]).max() / s.n
    print(f"DD LJ NVE 100 steps: |GPU - oracle| max {d:.2e} per atom, builds {sim.dd.builds} vs {a['builds']}")
    assert d < 1e-4
    assert sim.dd.builds >= 2
    sim.close()


def test_fs_run_follows_the_oracle_energy_trace(M, orc):
    s = inputs.eam_cu(ncell=12, T=600.0, seed=94)
    sim = _dd(s.x, s.v, s.L, (2, 2, 2), "eam")
    e = [sum(sim.energies())]
    for _ in range(5):
        sim.run(20)
        e.append(sum(sim.energies()))
    a = orc.md_run(s.x.copy(), s.v.copy(), s.L, 100, potential="eam", fs=FS, r_list=5.4, skin=1.0, dt=1.0,
                   mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    eo = a["epot"] + a["ekin"] * inputs.AMU_A2_FS2_IN_EV
    d = np.abs(np.array(e) - eo[::20]).max() / s.n
    print(f"DD FS NVE 100 fs: |GPU - oracle| max {d:.2e} eV/atom, builds {sim.dd.builds} vs {a['builds']}")
    assert d < 2e-5
    assert sim.dd.builds >= 2
    sim.close()
