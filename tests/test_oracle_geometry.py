"""Pins for the oracle's periodic geometry, cells and neighbour sets.

The neighbour set is pinned to its O(N^2) definition and to an independent
numpy computation; the cell assignment to exact rational arithmetic."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1611_00075_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_fcc_generator_counts_match_paper():
    # Sec. 3.1: Cu105 holds 4,630,500 atoms in 105^3 fcc cells.
    g = json.load(open(os.path.join(GOLD, "paper_counts.json")))
    n = g["Cu105"]["cells"]
    assert n ** 3 * len(inputs.FCC_BASIS) == g["Cu105"]["atoms"]
    # the generator itself, on a small instance: 4 sites per cell, all distinct
    x = inputs.fcc_sites(3, 4, 5, 1.0)
    assert x.shape == (3 * 4 * 5 * 4, 3)
    assert len(np.unique(np.round(x * 2).astype(int), axis=0)) == len(x)
    # the configuration sizes of the workloads
    assert inputs.fcc_sites(10, 10, 10, 1.0).shape[0] == 4000


def test_maxwell_boltzmann_exact_temperature_zero_momentum():
    s = inputs.eam_cu(ncell=4, T=600.0)
    assert abs(inputs.temperature(s.v, s.mass, s.kB, s.e_unit) - 600.0) < 1e-9
    assert np.abs(s.v.sum(axis=0)).max() < 1e-12
    s = inputs.lj_fcc(ncell=4)
    assert abs(inputs.temperature(s.v, s.mass, s.kB, s.e_unit) - 0.72) < 1e-12


def test_wrap_range_and_congruence(orc):
    L = np.array([3.0, 5.5, 7.25])
    rng = np.random.default_rng(0)
    x = rng.uniform(-30, 30, size=(5000, 3))
    x[:3] = [[3.0, 5.5, 7.25], [-1e-300, -5.5, 0.0], [-3.0, 11.0, -7.25]]
    w = orc.wrap(x, L)
    assert np.all(w >= 0.0) and np.all(w < L)
    k = (x - w) / L
    assert np.abs(k - np.round(k)).max() < 1e-9
    # exact multiples of L land on 0
    assert w[0].tolist() == [0.0, 0.0, 0.0]
    assert w[2].tolist() == [0.0, 0.0, 0.0]
    # a value just below zero wraps to the top of the box or to 0, never to L
    assert 0.0 <= w[1, 0] < L[0]


def test_cell_coords_against_exact_rationals(orc):
    L = np.array([10.0, 13.7, 9.1])
    nc = np.array([4, 5, 3])
    rng = np.random.default_rng(1)
    w = rng.uniform(0, 1, size=(3000, 3)) * L
    c = orc.cell_coords(w, L, nc)
    for a in range(3):
        for i in range(len(w)):
            ex = Fraction(w[i, a]) * nc[a] / Fraction(L[a])
            exact = min(math.floor(ex), nc[a] - 1)
            if exact != c[i, a]:
                # only allowed within rounding distance of a cell boundary
                assert abs(float(ex) - round(float(ex))) < 1e-12
    assert c.min() >= 0 and np.all(c.max(axis=0) <= nc - 1)


def _numpy_neighbors(x, L, r_list):
    """Independent all-pairs set with numpy rounding-based minimum image."""
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.round(d / L)
    r2 = np.sum(d * d, axis=-1)
    np.fill_diagonal(r2, np.inf)
    return r2 < r_list * r_list, r2


@pytest.mark.parametrize("L,r_list,n", [
    ((10.0, 10.0, 10.0), 2.8, 500),    # n_c = 3
    ((6.0, 7.0, 11.0), 2.9, 300),      # n_c = 2, 2, 3 (duplicated stencil)
    ((5.0, 5.0, 5.0), 2.4, 200),       # n_c = 2 everywhere
    ((4.0, 9.0, 4.5), 1.9, 150),       # n_c = 2, 4, 2
    ((3.0, 3.0, 3.0), 1.45, 80),       # n_c = 2 at almost L/2
    ((12.0, 12.0, 12.0), 2.5, 900),    # n_c = 4
])
def test_neighbors_brute_vs_cells_vs_numpy(orc, L, r_list, n):
    L = np.array(L)
    x = inputs.random_gas(n, L, seed=n)
    x = orc.wrap(x, L)
    ob, ib = orc.neighbors_brute(x, L, r_list)
    oc, ic = orc.neighbors_cells(x, L, r_list)
    assert np.array_equal(ob, oc) and np.array_equal(ib, ic)
    mask, r2 = _numpy_neighbors(x, L, r_list)
    near = np.abs(r2 - r_list * r_list) < 1e-9
    for i in range(n):
        row = set(ib[ob[i]:ob[i + 1]].tolist())
        ref = set(np.nonzero(mask[i])[0].tolist())
        amb = set(np.nonzero(near[i])[0].tolist())
        assert (row ^ ref) <= amb
    # symmetry j in N(i) <=> i in N(j)
    pairs = {(i, int(j)) for i in range(n) for j in ib[ob[i]:ob[i + 1]]}
    assert all((j, i) in pairs for (i, j) in pairs)


def test_neighbors_single_cell_and_empty(orc):
    L = np.array([2.5, 2.5, 2.5])
    x = orc.wrap(inputs.random_gas(40, L, seed=3), L)
    ob, ib = orc.neighbors_brute(x, L, 1.2)
    oc, ic = orc.neighbors_cells(x, L, 1.2)     # n_c = 2
    assert np.array_equal(ib, ic)
    oc, ic = orc.neighbors_cells(np.zeros((0, 3)), L, 1.2)
    assert oc.tolist() == [0] and len(ic) == 0
    # one atom: no neighbours
    oc, ic = orc.neighbors_cells(np.array([[1.0, 1.0, 1.0]]), L, 1.2)
    assert oc.tolist() == [0, 0]


def test_neighbors_fcc_shell_counts(orc):
    """On the perfect fcc lattice the list holds whole shells: with
    r_list = 2.8 sigma at rho* = 0.8442 the shells k = 1..5 (12+6+24+12+24)
    lie inside and shell 6 (8 at sqrt(6) a_nn = 2.909) outside."""
    s = inputs.lj_fcc(ncell=6)
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_cells(x, s.L, 2.8)
    counts = np.diff(off)
    from lattice_util import fcc_shell_counts
    m = fcc_shell_counts(6)
    assert m[:5] == [12, 6, 24, 12, 24] and m[5] == 8
    assert np.all(counts == sum(m[:5]))


def test_neighbors_invariant_under_translation_and_permutation(orc):
    L = np.array([9.0, 9.0, 9.0])
    x = orc.wrap(inputs.random_gas(400, L, seed=7), L)
    off, idx = orc.neighbors_cells(x, L, 2.2)
    sets = [set(idx[off[i]:off[i + 1]].tolist()) for i in range(len(x))]
    perm = np.random.default_rng(2).permutation(len(x))
    inv = np.argsort(perm)
    # translate by a lattice-compatible shift of exactly 1/4 box (exact in FP)
    y = orc.wrap(x[perm] + L / 4, L)
    o2, i2 = orc.neighbors_cells(y, L, 2.2)
    amb = 0
    for k in range(len(x)):
        got = {int(perm[j]) for j in i2[o2[k]:o2[k + 1]]}
        if got != sets[perm[k]]:
            amb += 1
    # translation changes rounding of the minimum-image; allow only boundary ties
    assert amb <= 2
    del inv
