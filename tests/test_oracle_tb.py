"""Pins for the oracle's second-moment tight-binding potential (exponential
density and pair functions, square-root embedding: the functional form the
paper gives for its copper potential, Eqs. (1)-(2) and Sec. 3.1).

The parameter set is synthetic (the published one is not available here):
p = 10 and q = 2.5 chosen, r0 the nearest-neighbour distance at a = 3.615 A,
cutoff smoothed between the third and fourth neighbour shells, and A, xi
fixed by the cohesive energy 3.54 eV and zero pressure at a = 3.615 A.  The
tests re-derive A and xi from those two conditions in closed form (lattice
shells of the fcc crystal), compare the oracle's lattice energies, densities,
pressure and bulk modulus with the closed form, and pin forces and virial to
finite differences of the oracle's own energy."""
import math

import numpy as np
import pytest

from paper_1611_00075_amd import inputs

TB = inputs.TB_CU
EV_PER_A3_IN_GPA = 160.21766208


def _shells(a):
    """(count, distance) of the fcc shells inside the smooth-cutoff start."""
    from lattice_util import fcc_shell_counts
    counts = fcc_shell_counts(5)
    out = [(n, a * math.sqrt(k / 2.0)) for k, n in enumerate(counts, start=1)]
    return [(n, r) for n, r in out if r < TB["rs"]]


def _closed_form(a):
    """(rho, E/N) of the perfect crystal from the lattice shells."""
    sh = _shells(a)
    rho = sum(n * TB["xi"] ** 2 * math.exp(-2 * TB["q"] * (r / TB["r0"] - 1)) for n, r in sh)
    pair = sum(n * TB["A"] * math.exp(-TB["p"] * (r / TB["r0"] - 1)) for n, r in sh)
    return rho, -math.sqrt(rho) + pair


def _lattice(orc, a, ncell=4):
    x = inputs.fcc_sites(ncell, ncell, ncell, a)
    L = np.full(3, ncell * a)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_cells(x, L, 6.0)
    return x, L, orc.forces_tb(x, L, off, idx, TB)


def test_parameters_solve_the_two_fitting_conditions():
    a0 = inputs.CU_A0
    assert TB["r0"] == pytest.approx(a0 / math.sqrt(2), rel=1e-10)
    sh = _shells(a0)
    assert [n for n, _ in sh] == [12, 6, 24]                 # shells 1-3 inside rs, shell 4 beyond rc
    assert a0 * math.sqrt(2) > TB["rc"]
    # E = -xi sqrt(B) + A R with B, R and their a-derivatives from the shells
    f = [r / a0 for _, r in sh]
    n = [m for m, _ in sh]
    e2q = [math.exp(-2 * TB["q"] * (fk * a0 / TB["r0"] - 1)) for fk in f]
    ep = [math.exp(-TB["p"] * (fk * a0 / TB["r0"] - 1)) for fk in f]
    B = sum(m * e for m, e in zip(n, e2q))
    dB = sum(m * e * (-2 * TB["q"] * fk / TB["r0"]) for m, e, fk in zip(n, e2q, f))
    R = sum(m * e for m, e in zip(n, ep))
    dR = sum(m * e * (-TB["p"] * fk / TB["r0"]) for m, e, fk in zip(n, ep, f))
    # -xi sqrt(B) + A R = -3.54 and -xi dB / (2 sqrt B) + A dR = 0
    M = np.array([[-math.sqrt(B), R], [-dB / (2 * math.sqrt(B)), dR]])
    xi, A = np.linalg.solve(M, [-3.54, 0.0])
    assert xi == pytest.approx(TB["xi"], rel=1e-9)
    assert A == pytest.approx(TB["A"], rel=1e-9)


def test_perfect_lattice_closed_form(orc):
    a = inputs.CU_A0
    x, L, r = _lattice(orc, a)
    rho, e = _closed_form(a)
    n = len(x)
    assert np.allclose(r["rho"], rho, rtol=1e-13)
    assert r["ev"][0] / n == pytest.approx(e, rel=1e-13)
    assert r["ev"][1] / n == pytest.approx(-math.sqrt(rho), rel=1e-13)
    assert np.allclose(r["e_atom"], e, rtol=1e-12)
    assert np.allclose(r["fprime"], -1 / (2 * math.sqrt(rho)), rtol=1e-13)
    assert np.abs(r["f"]).max() < 1e-12
    assert e == pytest.approx(-3.54, abs=1e-9)


def test_pressure_and_bulk_modulus_match_the_closed_form(orc):
    a0 = inputs.CU_A0
    h = 1e-3    # the same step for the oracle and the closed form; rounding stays far below

    def e_oracle(a):
        x, L, r = _lattice(orc, a)
        return r["ev"][0] / len(x)

    hp = 1e-5
    assert abs((e_oracle(a0 + hp) - e_oracle(a0 - hp)) / (2 * hp)) < 1e-6   # zero pressure at a0
    e0, ep, em = e_oracle(a0), e_oracle(a0 + h), e_oracle(a0 - h)
    B_or = 4.0 * (ep - 2 * e0 + em) / h ** 2 / (9.0 * a0) * EV_PER_A3_IN_GPA
    c = [_closed_form(a)[1] for a in (a0 - h, a0, a0 + h)]
    B_cf = 4.0 * (c[2] - 2 * c[1] + c[0]) / h ** 2 / (9.0 * a0) * EV_PER_A3_IN_GPA
    assert B_or == pytest.approx(B_cf, rel=1e-6)
    assert B_or == pytest.approx(139.19, abs=0.01)             # derived from the parameters
    # the static virial of a uniformly compressed crystal is minus the strain derivative
    x, L, r = _lattice(orc, 0.98 * a0)
    e_plus = _lattice(orc, 0.98 * a0 * (1 + 1e-6))[2]["ev"][0]
    e_minus = _lattice(orc, 0.98 * a0 * (1 - 1e-6))[2]["ev"][0]
    assert sum(r["ev"][2:5]) == pytest.approx(-(e_plus - e_minus) / 2e-6, rel=1e-6)


def _energy(orc, x, L):
    off, idx = orc.neighbors_brute(x, L, 6.0)
    return orc.forces_tb(x, L, off, idx, TB)


def test_forces_are_minus_energy_gradient(orc):
    s = inputs.jitter(inputs.eam_cu(ncell=3), 0.12, seed=31)
    x = orc.wrap(s.x, s.L)
    r = _energy(orc, x, s.L)
    # some pairs sit in the smooth-cutoff region
    off, idx = orc.neighbors_brute(x, s.L, 6.0)
    d = x[np.repeat(np.arange(len(x)), np.diff(off))] - x[idx]
    d -= s.L * np.round(d / s.L)
    rr = np.sqrt((d * d).sum(1))
    assert ((rr > TB["rs"]) & (rr < TB["rc"])).sum() > 100
    h = 1e-6
    rng = np.random.default_rng(5)
    for i in rng.choice(len(x), 6, replace=False):
        for a in range(3):
            xp = x.copy(); xp[i, a] += h
            xm = x.copy(); xm[i, a] -= h
            fd = -(_energy(orc, xp, s.L)["ev"][0] - _energy(orc, xm, s.L)["ev"][0]) / (2 * h)
            assert r["f"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    assert r["e_atom"].sum() == pytest.approx(r["ev"][0], rel=1e-12)
    assert np.abs(r["f"].sum(axis=0)).max() < 1e-11


def test_virial_is_minus_strain_derivative(orc):
    s = inputs.jitter(inputs.eam_cu(ncell=3), 0.05, seed=32)
    x = orc.wrap(s.x, s.L)
    r = _energy(orc, x, s.L)
    h = 1e-6
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        ep = _energy(orc, x * sc, s.L * sc)["ev"][0]
        sc[a] = 1 - h
        em = _energy(orc, x * sc, s.L * sc)["ev"][0]
        assert r["ev"][2 + a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6)


def test_dimer_energy_is_continuous_and_vanishes_at_the_cutoff(orc):
    L = np.full(3, 30.0)

    def dimer(s):
        x = np.array([[5.0, 5.0, 5.0], [5.0 + s, 5.0, 5.0]])
        return _energy(orc, x, L)

    # isolated atom: rho = 0 gives F = F' = 0
    r1 = _energy(orc, np.array([[1.0, 2.0, 3.0]]), L)
    assert r1["ev"][0] == 0.0 and r1["fprime"][0] == 0.0
    # across the start of the smooth cutoff: value and slope continuous
    eps = 1e-7
    e_in, e_out = dimer(TB["rs"] - eps)["ev"][0], dimer(TB["rs"] + eps)["ev"][0]
    assert abs(e_in - e_out) < 1e-6
    f_in, f_out = dimer(TB["rs"] - eps)["f"][0, 0], dimer(TB["rs"] + eps)["f"][0, 0]
    assert abs(f_in - f_out) < 1e-5
    # approaching rc: energy and force go to zero (the force of an isolated
    # dimer only as the square root of the distance to rc, through the
    # square-root embedding); beyond rc nothing interacts
    fs_ = [abs(dimer(TB["rc"] - dlt)["f"][0, 0]) for dlt in (1e-3, 1e-5, 1e-7)]
    assert fs_[0] > fs_[1] > fs_[2] and fs_[2] < 1e-3
    assert fs_[1] / fs_[0] == pytest.approx(0.1, rel=0.05)
    assert abs(dimer(TB["rc"] - 1e-3)["ev"][0]) < 1e-4
    far = dimer(TB["rc"] + 1e-3)
    assert far["ev"][0] == 0.0 and np.all(far["f"] == 0.0)
    # Newton's third law on the dimer
    mid = dimer(4.7)
    assert mid["f"][0, 0] == pytest.approx(-mid["f"][1, 0], rel=1e-14)
