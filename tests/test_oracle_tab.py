"""Pins for the oracle's tabulated embedded-atom form (functions given at
knots by value and slope, cubic Hermite interpolation in between; the paper
names piecewise-defined functions for its iron potential in Sec. 3.1 and
equates an interpolation table with such a definition in Sec. 5).

What fixes the oracle here, independently of its own code:
- a cubic polynomial is its own Hermite interpolant, so a table sampled from
  any cubic must give that cubic and its derivative everywhere (a dropped or
  mis-signed basis term, or a wrong interval, fails);
- a piecewise cubic with its breakpoints on knots (the form of the iron
  potential's pair function: a sum of a_m (r_m - r)^3 over r < r_m) is
  reproduced exactly across many intervals;
- the textbook error bounds of cubic Hermite interpolation, h^4/384
  max|f''''| for values and (sqrt 3/216) h^3 max|f''''| for slopes: the
  Finnis-Sinclair functions tabulated at dr = 0.005 A give the analytic
  oracle's energies and forces to that accuracy;
- a dimer with a linear embedding table has E = -2 psi(r) + Phi(r);
- forces and virial are derivatives of the oracle's own energy."""
import numpy as np
import pytest

from paper_1611_00075_amd import inputs

FS = inputs.FS_CU


def _table_from(f, df, h, m):
    u = np.arange(m) * h
    return f(u), df(u)


def test_a_cubic_is_its_own_interpolant(orc):
    rng = np.random.default_rng(5)
    c = rng.normal(size=4)
    p = np.polynomial.Polynomial(c)
    h, m = 0.37, 12
    f, df = _table_from(p, p.deriv(), h, m)
    u = np.concatenate([rng.uniform(0.0, (m - 1) * h, 200), np.arange(m) * h])
    val, slope = orc.tab_eval(f, df, h, u)
    assert np.allclose(val, p(u), rtol=0, atol=1e-12 * np.abs(p(u)).max())
    assert np.allclose(slope, p.deriv()(u), rtol=0, atol=1e-12 * np.abs(p.deriv()(u)).max())


def test_piecewise_cubic_with_breakpoints_on_knots(orc):
    # f(r) = sum_m a_m (r_m - r)^3 [r < r_m]: cubic between breakpoints
    h = 0.05
    rm = np.array([2.4, 2.65, 3.0, 3.45, 4.1, 4.6])
    am = np.array([-3.1, 5.2, -1.7, 0.9, -0.35, 0.12])
    f = lambda r: sum(a * np.where(r < b, (b - r) ** 3, 0.0) for a, b in zip(am, rm))
    df = lambda r: sum(-3.0 * a * np.where(r < b, (b - r) ** 2, 0.0) for a, b in zip(am, rm))
    m = int(round(4.6 / h)) + 1
    tf, tdf = _table_from(f, df, h, m)
    r = np.random.default_rng(6).uniform(1.5, 4.6, 500)
    val, slope = orc.tab_eval(tf, tdf, h, r)
    assert np.abs(val - f(r)).max() < 1e-12 * np.abs(f(r)).max()
    assert np.abs(slope - df(r)).max() < 1e-11 * np.abs(df(r)).max()


def test_embedding_continues_along_the_end_tangents(orc):
    h, m = 0.5, 9
    f = np.sin(np.arange(m) * h)
    df = np.cos(np.arange(m) * h)
    umax = (m - 1) * h
    for u in (-0.7, -0.01, umax + 0.01, umax + 2.3):
        v, s = orc.tab_eval(f, df, h, [u])
        k = 0 if u < 0 else m - 1
        assert v[0] == pytest.approx(f[k] + df[k] * (u - k * h), abs=1e-14)
        assert s[0] == pytest.approx(df[k], abs=1e-15)


def test_hermite_error_bound_on_a_smooth_function(orc):
    # |f - p| <= h^4/384 max|f''''| for cubic Hermite interpolation
    h, m = 0.1, 31
    u = np.arange(m) * h
    v, _ = orc.tab_eval(np.exp(-u), -np.exp(-u), h, np.linspace(0, (m - 1) * h, 777))
    err = np.abs(v - np.exp(-np.linspace(0, (m - 1) * h, 777))).max()
    assert err <= h ** 4 / 384 * 1.0 * (1 + 1e-9)
    assert err > 0.2 * h ** 4 / 384 * np.exp(-h)   # the bound is attained to a modest factor


def test_dimer_energy_with_linear_embedding(orc):
    tab = inputs.fs_table()
    rho = np.arange(len(tab["F"])) * tab["drho"]
    tab = dict(tab, F=-rho, dF=-np.ones_like(rho))       # F(rho) = -rho exactly
    L = np.full(3, 30.0)
    rc = (len(tab["psi"]) - 1) * tab["dr"]
    for r in (2.3, 2.5561910140, 3.249, 3.3, 4.2, rc - 1e-9, rc + 1e-9, 5.0):
        x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
        off, idx = orc.neighbors_brute(x, L, 6.0)
        o = orc.forces_tab(x, L, off, idx, tab)
        psi, dpsi = orc.tab_eval(tab["psi"], tab["dpsi"], tab["dr"], [r])
        phi, dphi = orc.tab_eval(tab["phi"], tab["dphi"], tab["dr"], [r])
        inside = r < rc
        e = (-2.0 * psi[0] + phi[0]) if inside else 0.0
        assert o["ev"][0] == pytest.approx(e, abs=1e-13)
        assert o["rho"][0] == pytest.approx(psi[0] if inside else 0.0, abs=1e-14)
        # force on atom 0 along +x: -dU/dx0 = dU/dr
        fx = (-2.0 * dpsi[0] + dphi[0]) if inside else 0.0
        assert o["f"][0, 0] == pytest.approx(fx, abs=1e-12)
        assert o["f"][1, 0] == pytest.approx(-fx, abs=1e-12)


def _cu(orc, seed, ncell=5, jit=0.08):
    s = inputs.jitter(inputs.eam_cu(ncell=ncell), jit, seed=seed)
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_cells(x, s.L, 5.4)
    return x, s.L, off, idx


def test_tabulated_fs_matches_the_analytic_oracle(orc):
    x, L, off, idx = _cu(orc, 71)
    a = orc.forces_eam(x, L, off, idx, FS)
    t = orc.forces_tab(x, L, off, idx, inputs.fs_table(FS))
    n = len(x)
    # psi is quadratic (exact); V is quartic: |V - p| <= h^4/384 * 24 c2 per
    # pair; F(rho) = -A sqrt(rho) near rho ~ 40 is far smoother still
    h = 0.005
    bound_pair = h ** 4 / 384 * 24 * FS["c2"]
    assert np.abs(t["rho"] - a["rho"]).max() < 1e-12 * a["rho"].max()
    assert abs(t["ev"][0] - a["ev"][0]) < n * 20 * bound_pair + 1e-10 * abs(a["ev"][0])
    # slope error of cubic Hermite interpolation (Birkhoff and Priver):
    # |f' - p'| <= (sqrt 3 / 216) h^3 max|f''''| per pair within c; at most
    # 20 such pairs per atom here
    bound_slope = np.sqrt(3.0) / 216 * h ** 3 * 24 * FS["c2"]
    err = np.abs(t["f"] - a["f"]).max()
    assert err < 20 * bound_slope
    assert err > 1e-3 * bound_slope          # not exact: V is quartic
    # virial: sum over pairs within c of r * (slope error), ~10 such pairs per atom
    assert np.abs(t["ev"][2:] - a["ev"][2:]).max() < n * 10 * FS["c"] * bound_slope
    assert np.abs(t["e_atom"] - a["e_atom"]).max() < 1e-9


def test_forces_and_virial_are_energy_derivatives(orc):
    x, L, off, idx = _cu(orc, 72, ncell=4, jit=0.12)
    # a table that is not a sampled polynomial anywhere: slopes perturbed
    tab = inputs.fs_table(FS, dr=0.05, drho=0.5)
    rng = np.random.default_rng(73)
    tab["dpsi"] = tab["dpsi"] * (1 + 0.05 * rng.normal(size=len(tab["dpsi"])))
    tab["dphi"] = tab["dphi"] * (1 + 0.05 * rng.normal(size=len(tab["dphi"])))
    tab["dF"] = tab["dF"] * (1 + 0.05 * rng.normal(size=len(tab["dF"])))
    o = orc.forces_tab(x, L, off, idx, tab)
    hstep = 1e-5
    for i, c in [(0, 0), (7, 1), (33, 2), (101, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, c] += hstep
        xm[i, c] -= hstep
        ep = orc.forces_tab(xp, L, off, idx, tab)["ev"][0]
        em = orc.forces_tab(xm, L, off, idx, tab)["ev"][0]
        assert o["f"][i, c] == pytest.approx(-(ep - em) / (2 * hstep), abs=2e-6)
    # virial W_xx = -dE/d(eps_xx) under a uniform strain of x
    eps = 1e-6
    Lp, Lm = L.copy(), L.copy()
    Lp[0] *= 1 + eps
    Lm[0] *= 1 - eps
    xp, xm = x.copy(), x.copy()
    xp[:, 0] *= 1 + eps
    xm[:, 0] *= 1 - eps
    ep = orc.forces_tab(xp, Lp, off, idx, tab)["ev"][0]
    em = orc.forces_tab(xm, Lm, off, idx, tab)["ev"][0]
    assert o["ev"][2] == pytest.approx(-(ep - em) / (2 * eps), rel=1e-5)
