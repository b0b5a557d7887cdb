"""The per-atom error scales of the parity tests (tests/force_scale.py)
are pair decompositions of the oracle's forces: summing each pair's signed
term over a row must give the oracle's force on that atom, so a scale with a
dropped term, a wrong derivative or a wrong pair kind fails here."""
import numpy as np
import pytest

import force_scale as FSC
from paper_1611_00075_amd import inputs


def _resum(x, L, off, idx, s):
    I, J, R, r = FSC.pair_table(x, L, off, idx)
    vec = -(s / r)[:, None] * R
    return np.stack([np.bincount(I, weights=vec[:, k], minlength=len(x)) for k in range(3)], 1)


def _cu(orc, ncell=4, jit=0.15, seed=3, scale=1.0):
    s = inputs.jitter(inputs.eam_cu(ncell=ncell), jit, seed=seed)
    return orc.wrap(s.x * scale, s.L * scale), s.L * scale


def test_lj_pair_terms_resum_to_oracle(orc):
    s = inputs.jitter(inputs.lj_fcc(ncell=5), 0.08, seed=2)
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_brute(x, s.L, 2.8)
    fo, _ = orc.forces_lj(x, s.L, off, idx)
    I, J, R, r = FSC.pair_table(x, s.L, off, idx)
    mag, sg, _ = FSC.lj_terms(I, J, r)
    assert np.allclose(_resum(x, s.L, off, idx, sg), fo, rtol=0, atol=1e-10 * np.abs(fo).max())
    assert np.all(mag >= np.abs(sg))


def test_fs_pair_terms_resum_to_oracle(orc):
    x, L = _cu(orc)
    off, idx = orc.neighbors_brute(x, L, 5.4)
    r_o = orc.forces_eam(x, L, off, idx, inputs.FS_CU)
    I, J, R, r = FSC.pair_table(x, L, off, idx)
    mag, sg, cuts = FSC.fs_terms(r_o["fprime"], I, J, r, inputs.FS_CU)
    assert np.allclose(_resum(x, L, off, idx, sg), r_o["f"], rtol=0, atol=1e-10 * np.abs(r_o["f"]).max())
    assert cuts == (4.4, 3.25)


def test_tb_pair_terms_resum_to_oracle(orc):
    x, L = _cu(orc, seed=4)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    r_o = orc.forces_tb(x, L, off, idx, inputs.TB_CU)
    I, J, R, r = FSC.pair_table(x, L, off, idx)
    _, sg, _ = FSC.tb_terms(r_o["fprime"], I, J, r, inputs.TB_CU)
    assert np.allclose(_resum(x, L, off, idx, sg), r_o["f"], rtol=0, atol=1e-10 * np.abs(r_o["f"]).max())


def test_tbm_pair_terms_resum_to_oracle(orc):
    a = 0.75 * inputs.CU_A0 + 0.25 * inputs.AU_A0
    x, L = _cu(orc, seed=5, scale=a / inputs.CU_A0)
    t = (np.random.default_rng(5).random(len(x)) < 0.25).astype(np.int32)
    off, idx = orc.neighbors_brute(x, L, 6.7)
    r_o = orc.forces_tbm(x, L, off, idx, t, inputs.TB2_PAIRS)
    I, J, R, r = FSC.pair_table(x, L, off, idx)
    _, sg, _ = FSC.tbm_terms(r_o["fprime"], I, J, r, t, inputs.TB2_PAIRS)
    assert np.allclose(_resum(x, L, off, idx, sg), r_o["f"], rtol=0, atol=1e-10 * np.abs(r_o["f"]).max())


def test_tab_pair_terms_resum_to_oracle(orc):
    x, L = _cu(orc, ncell=3, seed=6)
    tab = inputs.fs_table(inputs.FS_CU, dr=0.05)
    rc = (len(tab["psi"]) - 1) * tab["dr"]
    off, idx = orc.neighbors_brute(x, L, rc + 1.0)
    r_o = orc.forces_tab(x, L, off, idx, tab)
    I, J, R, r = FSC.pair_table(x, L, off, idx)
    _, sg, _ = FSC.tab_terms(orc, r_o["fprime"], I, J, r, tab)
    assert np.allclose(_resum(x, L, off, idx, sg), r_o["f"], rtol=0, atol=1e-10 * np.abs(r_o["f"]).max())


def test_check_per_atom_catches_a_dropped_pair(orc):
    """A force missing one pair's term fails the per-atom bound although it
    can pass the normwise one."""
    x, L = _cu(orc, seed=7)
    off, idx = orc.neighbors_brute(x, L, 5.4)
    r_o = orc.forces_eam(x, L, off, idx, inputs.FS_CU)
    I, J, R, r = FSC.pair_table(x, L, off, idx)
    mag, sg, cuts = FSC.fs_terms(r_o["fprime"], I, J, r, inputs.FS_CU)
    p = int(np.argmax(np.abs(sg) * (np.abs(r - 4.4) > 0.1) * (np.abs(r - 3.25) > 0.1)))
    bad = r_o["f"].copy()
    bad[I[p]] -= -(sg[p] / r[p]) * R[p]
    err, ratio = FSC.check_per_atom(r_o["f"], r_o["f"], I, R, r, mag, sg, cuts)
    assert err == 0.0 and ratio == 0.0
    with pytest.raises(AssertionError):
        FSC.check_per_atom(bad, r_o["f"], I, R, r, mag, sg, cuts, tol=1e-2)


def test_check_form_on_a_subset_of_atoms(orc):
    x, L = _cu(orc, seed=8)
    off, idx = orc.neighbors_brute(x, L, 5.4)
    r_o = orc.forces_eam(x, L, off, idx, inputs.FS_CU)
    atoms = np.arange(3, len(x), 7)
    err, ratio = FSC.check_form(orc, "fs", r_o["f"][atoms], x, L, off, idx, r_o, inputs.FS_CU, atoms=atoms)
    assert err == 0.0 and ratio == 0.0
    bad = r_o["f"][atoms].copy()
    bad[5] *= 1.01
    with pytest.raises(AssertionError):
        FSC.check_form(orc, "fs", bad, x, L, off, idx, r_o, inputs.FS_CU, atoms=atoms, tol=1e-3)
