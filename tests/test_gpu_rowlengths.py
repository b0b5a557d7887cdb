"""GPU parity of the pair kernels on rows of every length: lattices whose
density falls from the full lattice's to zero across the box, so the rows
hold from 0 to ~110 entries and every lane of a slice meets each case of
the row walk (no full batch, one or two full batches, a tail of 1 to U - 1
entries, no tail).  LJ (with and without the energy sums), Finnis-Sinclair,
tight-binding, tabulated and two-element forms against the FP64 oracle."""
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


def _counts_cover(cnt, hi):
    """Row lengths from 0-3 to at least `hi`, with most values in between."""
    c = np.asarray(cnt)
    assert c.min() <= 3 and c.max() >= hi, (c.min(), c.max())
    assert len(np.unique(c)) >= 0.6 * hi


def _by_id(st, t, n, ncomp=1):
    p = st["perm"].cpu().numpy()[:n]
    a = t.cpu().numpy()
    if ncomp == 1:
        out = np.empty(n)
        out[p] = a[:n]
    else:
        out = np.empty((n, ncomp))
        out[p] = a.T[:n]
    return out


@pytest.mark.parametrize("energy", [False, True], ids=["forces", "energy"])
def test_lj_rows_of_every_length(M, orc, energy):
    from test_gpu_parity import _check_forces, _lj_setup, _pair_sums_lj
    x, L = inputs.graded(14, inputs.fcc_lattice_constant(1.2), 0.03, seed=71)
    x = orc.wrap(x, L)
    n = len(x)
    st, xsc = _lj_setup(M, x, L)
    _counts_cover(st["cnt"].cpu().numpy()[:n], 95)
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.md_forces_lj(L, n, st["x"], xsc, st["cap"], st["idx"], st["cnt"], (1.0, 1.0, 2.5), f, ev,
                   M.MD_ENERGY if energy else 0, st["ws"])
    fg = _by_id(st, f, n, 3)
    oc, ic = orc.neighbors_cells(x, L, 2.8)
    fo, evo = orc.forces_lj(x, L, oc, ic, rc=2.5)
    fabs, near, contrib = _pair_sums_lj(x, L, oc, ic, 2.5)
    err = _check_forces(fg, fo, fabs, near, contrib)
    print(f"graded LJ ({n} atoms): force error (normwise) {err:.3e}")
    if energy:
        evg = ev.cpu().numpy()
        assert evg[0] == pytest.approx(evo[0], rel=2e-6)
        assert evg[1] == pytest.approx(evo[1], rel=2e-6)


def _cu_graded(M, orc, r_list, seed):
    from test_gpu_parity import _gpu_lists
    x, L = inputs.graded(14, 3.35, 0.05, seed=seed)
    x = orc.wrap(x, L)
    n = len(x)
    rows, st = _gpu_lists(M, x, L, r_list)
    xsc = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    M.md_scale_positions(L, n, st["x"], xsc)
    return x, L, n, st, xsc


def _eam_outputs(n):
    z = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    return z(3, n), z(n), z(n), torch.zeros(8, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("form", ["fs", "tb", "tab", "tbm"])
def test_eam_forms_rows_of_every_length(M, orc, form):
    r_list = {"tb": 6.0, "tbm": 6.7}.get(form, 5.4)
    x, L, n, st, xsc = _cu_graded(M, orc, r_list, seed=72)
    _counts_cover(st["cnt"].cpu().numpy()[:n], {"tb": 80, "tbm": 95}.get(form, 60))
    f, rho, fp, ev = _eam_outputs(n)
    oc, ic = orc.neighbors_cells(x, L, r_list)
    if form == "fs":
        M.md_forces_eam(L, n, xsc, st["cap"], st["idx"], st["cnt"], inputs.FS_CU, rho, fp, f, ev, 0, st["ws"])
        r = orc.forces_eam(x, L, oc, ic, inputs.FS_CU)
    elif form == "tb":
        M.md_forces_tb(L, n, xsc, st["cap"], st["idx"], st["cnt"], inputs.TB_CU, rho, fp, f, ev, 0, st["ws"])
        r = orc.forces_tb(x, L, oc, ic, inputs.TB_CU)
    elif form == "tbm":
        # a random alloy, 25 % of element 1
        t = (inputs.rng_for(73, "elements").uniform(size=n) < 0.25).astype(np.int32)
        p = st["perm"].cpu().numpy()[:n]
        M.md_set_elements(n, torch.tensor(t[p], dtype=torch.int32, device="cuda"), xsc)
        M.md_forces_tbm(L, n, xsc, st["cap"], st["idx"], st["cnt"], inputs.TB2_PAIRS, rho, fp, f, ev, 0, st["ws"])
        r = orc.forces_tbm(x, L, oc, ic, t, inputs.TB2_PAIRS)
    else:
        tab = inputs.fs_table(inputs.FS_CU)
        table = torch.empty(M.md_tab_bytes(tab), dtype=torch.uint8, device="cuda")
        M.md_tab_pack(tab, table)
        M.md_forces_tab(L, n, xsc, st["cap"], st["idx"], st["cnt"], tab, table, rho, fp, f, ev, 0, st["ws"])
        r = orc.forces_tab(x, L, oc, ic, tab)
    rg = _by_id(st, rho, n)
    fg = _by_id(st, f, n, 3)
    assert np.abs(rg - r["rho"]).max() <= 1e-5 * r["rho"].max()
    import force_scale as FSC
    prm = {"fs": inputs.FS_CU, "tb": inputs.TB_CU, "tbm": inputs.TB2_PAIRS}.get(form)
    FSC.check_form(orc, form, fg, x, L, oc, ic, r, prm if form != "tab" else tab,
                   types=t if form == "tbm" else None, what=f"graded {form} ({n} atoms)")
