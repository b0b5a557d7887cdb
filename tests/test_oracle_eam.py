"""Pins for the oracle's embedded-atom (Finnis-Sinclair) evaluation.

The Cu-like coefficients were fitted to four measured properties of copper
(cohesive energy 3.54 eV, lattice constant 3.615 A, bulk modulus 138 GPa,
vacancy formation energy 1.28 eV).  Recovering all four through the oracle
pins both the coefficients and the oracle's energy (a dropped factor 1/2 on
the pair term, a wrong embedding sign or a missed shell breaks at least one).
Forces are pinned to finite differences of the energy."""
import math

import numpy as np
import pytest

from paper_1611_00075_amd import inputs

FS = inputs.FS_CU
EV_PER_A3_IN_GPA = 160.21766208


def _lattice(orc, a, ncell=4, drop=None):
    x = inputs.fcc_sites(ncell, ncell, ncell, a)
    if drop is not None:
        x = np.delete(x, drop, axis=0)
    L = np.full(3, ncell * a)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_cells(x, L, 5.4)
    return x, L, orc.forces_eam(x, L, off, idx, FS)


def test_eam_perfect_lattice_closed_form(orc):
    a = inputs.CU_A0
    x, L, r = _lattice(orc, a)
    r1, r2, r3 = a / math.sqrt(2), a, a * math.sqrt(1.5)
    assert r2 < FS["d"] < r3 and r1 < FS["c"] < r2
    rho = 12 * (r1 - FS["d"]) ** 2 + 6 * (r2 - FS["d"]) ** 2
    assert np.allclose(r["rho"], rho, rtol=1e-13)
    V1 = (r1 - FS["c"]) ** 2 * (FS["c0"] + FS["c1"] * r1 + FS["c2"] * r1 ** 2)
    e = -FS["A"] * math.sqrt(rho) + 6 * V1
    n = len(x)
    assert r["ev"][0] / n == pytest.approx(e, rel=1e-13)
    assert r["ev"][1] / n == pytest.approx(-FS["A"] * math.sqrt(rho), rel=1e-13)
    assert np.allclose(r["e_atom"], e, rtol=1e-12)
    assert np.allclose(r["fprime"], -FS["A"] / (2 * math.sqrt(rho)), rtol=1e-13)
    assert np.abs(r["f"]).max() < 1e-12


def test_eam_reproduces_fitted_copper_properties(orc):
    a0 = inputs.CU_A0

    def e_atom(a):
        x, L, r = _lattice(orc, a)
        return r["ev"][0] / len(x)

    e0 = e_atom(a0)
    assert e0 == pytest.approx(-3.54, abs=1e-6)                  # cohesive energy
    h = 1e-4
    ep, em = e_atom(a0 + h), e_atom(a0 - h)
    assert abs((ep - em) / (2 * h)) < 1e-6                       # zero pressure at a0
    d2 = (ep - 2 * e0 + em) / h ** 2
    B = 4.0 * d2 / (9.0 * a0) * EV_PER_A3_IN_GPA
    assert B == pytest.approx(138.0, rel=1e-4)                   # bulk modulus
    x, L, rv = _lattice(orc, a0, drop=0)
    evac = rv["ev"][0] - len(x) * e0
    assert evac == pytest.approx(1.28, abs=1e-6)                 # vacancy energy
    # fcc is preferred over bcc at the same density scan
    best_bcc = min(_bcc_energy(orc, ab) for ab in np.linspace(2.75, 3.05, 31))
    assert best_bcc > e0


def _bcc_energy(orc, a, ncell=5):
    base = np.array([[0.0, 0, 0], [0.5, 0.5, 0.5]])
    g = np.stack(np.meshgrid(*[np.arange(ncell)] * 3, indexing="ij"), -1).reshape(-1, 1, 3)
    x = ((g + base[None]) * a).reshape(-1, 3)
    L = np.full(3, ncell * a)
    off, idx = orc.neighbors_cells(x, L, 5.4)
    return orc.forces_eam(x, L, off, idx, FS)["ev"][0] / len(x)


def _energy(orc, x, L):
    off, idx = orc.neighbors_brute(x, L, 5.4)
    return orc.forces_eam(x, L, off, idx, FS)


def test_eam_forces_are_minus_energy_gradient(orc):
    s = inputs.jitter(inputs.eam_cu(ncell=3), 0.08, seed=21)
    x = orc.wrap(s.x, s.L)
    r = _energy(orc, x, s.L)
    h = 1e-6
    rng = np.random.default_rng(3)
    for i in rng.choice(len(x), 6, replace=False):
        for a in range(3):
            xp = x.copy(); xp[i, a] += h
            xm = x.copy(); xm[i, a] -= h
            fd = -(_energy(orc, xp, s.L)["ev"][0] - _energy(orc, xm, s.L)["ev"][0]) / (2 * h)
            assert r["f"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    assert r["e_atom"].sum() == pytest.approx(r["ev"][0], rel=1e-12)
    assert np.abs(r["f"].sum(axis=0)).max() < 1e-11


def test_eam_virial_is_minus_strain_derivative(orc):
    s = inputs.jitter(inputs.eam_cu(ncell=3), 0.05, seed=22)
    x = orc.wrap(s.x, s.L)
    r = _energy(orc, x, s.L)
    h = 1e-6
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        ep = _energy(orc, x * sc, s.L * sc)["ev"][0]
        sc[a] = 1 - h
        em = _energy(orc, x * sc, s.L * sc)["ev"][0]
        assert r["ev"][2 + a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6)


def test_eam_isolated_atom_and_dimer(orc):
    L = np.full(3, 30.0)
    # isolated atom: rho = 0 gives F = F' = 0 and no force
    r = _energy(orc, np.array([[1.0, 2.0, 3.0]]), L)
    assert r["ev"][0] == 0.0 and r["fprime"][0] == 0.0
    # dimer at separation s: E = 2 F(psi(s)) + V(s)
    s = 2.9
    x = np.array([[5.0, 5.0, 5.0], [5.0 + s, 5.0, 5.0]])
    r = _energy(orc, x, L)
    psi = (s - FS["d"]) ** 2
    V = (s - FS["c"]) ** 2 * (FS["c0"] + FS["c1"] * s + FS["c2"] * s * s)
    assert r["ev"][0] == pytest.approx(2 * (-FS["A"] * math.sqrt(psi)) + V, rel=1e-14)
    assert r["f"][0, 0] == pytest.approx(-r["f"][1, 0], rel=1e-15)
