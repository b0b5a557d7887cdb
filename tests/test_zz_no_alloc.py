"""The allocation-free entry point md_forces_lj_noalloc against
md_forces_lj: the same kernels on the same inputs, so forces, energy and
virial must agree bit for bit, on two calls in a row (the second with a
smaller system, so the library's array holds the first call's rows), for
the FP32 and FP64 pair paths, with and without the energy sums."""
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


def _system(ncell, seed):
    from paper_1611_00075_amd.sim import Simulation
    s = inputs.jitter(inputs.lj_fcc(ncell=ncell), 0.06, seed=seed)
    return Simulation(s.L, s.x, s.v, skin=0.3, dt=0.005)


@pytest.mark.parametrize("flags", ["energy", "energy+fp64", "forces"])
def test_noalloc_matches_workspace_entry_point(M, flags):
    fl = {"energy": M.MD_ENERGY, "energy+fp64": M.MD_ENERGY | M.MD_PAIR_FP64, "forces": 0}[flags]
    fdt = torch.float64 if fl & M.MD_PAIR_FP64 else torch.float32
    for ncell, seed in ((24, 1), (9, 2)):           # 55,296 atoms, then 2,916
        sim = _system(ncell, seed)
        n = sim.n
        out = []
        for fn in ("ws", "noalloc"):
            f = torch.full((3, n), float("nan"), dtype=fdt, device="cuda")
            ev = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
            if fn == "ws":
                M.md_forces_lj(sim.L, n, sim.x, sim.xs, sim.row_cap, sim.idx, sim.count, sim.lj, f, ev, fl, sim.ws)
            else:
                M.md_forces_lj_noalloc(sim.L, n, sim.x, sim.xs, sim.row_cap, sim.idx, sim.count, sim.lj, f, ev, fl)
            torch.cuda.synchronize()
            out.append((f.cpu().numpy(), ev.cpu().numpy()))
        assert np.array_equal(out[0][0], out[1][0]), (flags, n)
        if fl & M.MD_ENERGY:
            assert np.array_equal(out[0][1], out[1][1]), (flags, n)
            assert np.all(np.isfinite(out[1][1]))
        print(f"noalloc {flags}: {n} atoms, forces and ev bit-identical to md_forces_lj")


def test_noalloc_rejects_energy_beyond_its_array(M):
    """With MD_ENERGY, more atoms than the array's rows cover is an
    argument error, detected on the host before anything is queued."""
    n = M.MD_NOALLOC_MAX_ATOMS + 1
    L = [600.0, 600.0, 600.0]
    x = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    xs = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    idx = torch.zeros(M.ell_size(n, 8), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MDError) as e:
        M.md_forces_lj_noalloc(L, n, x, xs, 8, idx, cnt, (1.0, 1.0, 2.5), f, ev, M.MD_ENERGY)
    assert e.value.code == M.MD_ERR_ARG
