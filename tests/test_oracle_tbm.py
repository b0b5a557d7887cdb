"""Pins for the oracle's two-element tight-binding potential (the same
second-moment form with the parameters of each pair's kind, Sec. 3.1's
Cu-Au systems; synthetic Cu-like and Au-like parameter sets).

Each element's A and xi are re-derived from its cohesive energy and zero
pressure on its own perfect lattice; the two-element evaluation must reduce
to the one-element oracle when all pair kinds share one parameter set and
must be symmetric under exchanging the elements together with their
parameters; the mixed pair kind is checked on a dimer against the
one-element oracle run with the mixed parameters; forces and virial are
pinned to finite differences of the energy."""
import math

import numpy as np
import pytest

from paper_1611_00075_amd import inputs

PAIRS = inputs.TB2_PAIRS
R_LIST = 6.7


def _solve(tb, a0, ecoh):
    from lattice_util import fcc_shell_counts
    counts = fcc_shell_counts(5)
    sh = [(n, a0 * math.sqrt(k / 2.0)) for k, n in enumerate(counts, start=1)]
    sh = [(n, r) for n, r in sh if r < tb["rs"]]
    e2q = [n * math.exp(-2 * tb["q"] * (r / tb["r0"] - 1)) for n, r in sh]
    ep = [n * math.exp(-tb["p"] * (r / tb["r0"] - 1)) for n, r in sh]
    B, R = sum(e2q), sum(ep)
    dB = sum(e * (-2 * tb["q"] * r / a0 / tb["r0"]) for e, (_, r) in zip(e2q, sh))
    dR = sum(e * (-tb["p"] * r / a0 / tb["r0"]) for e, (_, r) in zip(ep, sh))
    M = np.array([[-math.sqrt(B), R], [-dB / (2 * math.sqrt(B)), dR]])
    return np.linalg.solve(M, [-ecoh, 0.0]), [n for n, _ in sh]


@pytest.mark.parametrize("el,a0,ecoh,shells", [(0, inputs.CU_A0, 3.54, [12, 6, 24, 12]),
                                               (1, inputs.AU_A0, 3.81, [12, 6, 24])])
def test_each_element_solves_its_fitting_conditions(orc, el, a0, ecoh, shells):
    tb = PAIRS[2 * el]
    assert tb["r0"] == pytest.approx(a0 / math.sqrt(2), rel=1e-10)
    (xi, A), used = _solve(tb, a0, ecoh)
    assert used == shells
    assert xi == pytest.approx(tb["xi"], rel=1e-9) and A == pytest.approx(tb["A"], rel=1e-9)
    x = inputs.fcc_sites(4, 4, 4, a0)
    L = np.full(3, 4 * a0)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_cells(x, L, R_LIST)
    r = orc.forces_tbm(x, L, off, idx, np.full(len(x), el), PAIRS)
    assert r["ev"][0] / len(x) == pytest.approx(-ecoh, abs=1e-8)
    assert np.abs(r["f"]).max() < 1e-12


def _alloy(orc, ncell=3, jit=0.1, seed=51, frac=0.25):
    a = 0.75 * inputs.CU_A0 + 0.25 * inputs.AU_A0
    s = inputs.jitter(inputs.eam_cu(ncell=ncell), jit, seed=seed)
    x = s.x * (a / inputs.CU_A0)
    L = s.L * (a / inputs.CU_A0)
    x = orc.wrap(x, L)
    t = (np.random.default_rng(seed).random(len(x)) < frac).astype(np.int32)
    return x, L, t


def _tbm(orc, x, L, t, pairs=PAIRS):
    off, idx = orc.neighbors_brute(x, L, R_LIST)
    return orc.forces_tbm(x, L, off, idx, t, pairs)


def test_one_parameter_set_reduces_to_the_one_element_oracle(orc):
    x, L, t = _alloy(orc)
    same = (inputs.TB2_CU,) * 3
    r = _tbm(orc, x, L, t, same)
    off, idx = orc.neighbors_brute(x, L, R_LIST)
    r1 = orc.forces_tb(x, L, off, idx, inputs.TB2_CU)
    assert np.array_equal(r["f"], r1["f"]) and np.array_equal(r["ev"], r1["ev"])
    assert np.array_equal(r["rho"], r1["rho"])


def test_exchanging_the_elements_with_their_parameters(orc):
    x, L, t = _alloy(orc)
    r = _tbm(orc, x, L, t)
    rs = _tbm(orc, x, L, 1 - t, PAIRS[::-1])
    assert np.allclose(r["f"], rs["f"], rtol=1e-13, atol=1e-13)
    assert r["ev"][0] == pytest.approx(rs["ev"][0], rel=1e-13)
    # and the alloy differs from either pure element
    r0 = _tbm(orc, x, L, np.zeros_like(t))
    assert abs(r0["ev"][0] - r["ev"][0]) > 0.1


def test_mixed_pair_uses_the_mixed_parameters(orc):
    Lb = np.full(3, 30.0)
    for s in (2.7, 4.0, 5.4):
        x = np.array([[5.0, 5.0, 5.0], [5.0 + s, 5.0, 5.0]])
        off, idx = orc.neighbors_brute(x, Lb, R_LIST)
        for ti, tj, tb in ((0, 0, inputs.TB2_CU), (0, 1, inputs.TB2_CUAU), (1, 1, inputs.TB2_AU)):
            r = orc.forces_tbm(x, Lb, off, idx, np.array([ti, tj]), PAIRS)
            r1 = orc.forces_tb(x, Lb, off, idx, tb)
            assert r["ev"][0] == pytest.approx(r1["ev"][0], rel=1e-14)
            assert np.allclose(r["f"], r1["f"], rtol=1e-14, atol=0)


def test_forces_and_virial_are_energy_derivatives(orc):
    x, L, t = _alloy(orc, jit=0.15, seed=52)
    r = _tbm(orc, x, L, t)
    h = 1e-5    # the total energy is ~370 eV: a smaller step drowns in its rounding
    rng = np.random.default_rng(7)
    for i in rng.choice(len(x), 6, replace=False):
        for a in range(3):
            xp = x.copy(); xp[i, a] += h
            xm = x.copy(); xm[i, a] -= h
            fd = -(_tbm(orc, xp, L, t)["ev"][0] - _tbm(orc, xm, L, t)["ev"][0]) / (2 * h)
            assert r["f"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        ep = _tbm(orc, x * sc, L * sc, t)["ev"][0]
        sc[a] = 1 - h
        em = _tbm(orc, x * sc, L * sc, t)["ev"][0]
        assert r["ev"][2 + a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6)
    assert r["e_atom"].sum() == pytest.approx(r["ev"][0], rel=1e-12)
    assert np.abs(r["f"].sum(axis=0)).max() < 1e-11
