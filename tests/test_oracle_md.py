"""Pins for the oracle's velocity-Verlet dynamics and list-rebuild rule:
energy conservation, time reversibility, momentum conservation, exact free
flight, and independence of the trajectory from the skin (the rebuild rule
of Sec. 3.3 must never let a pair inside the cutoff go missing)."""
import numpy as np
import pytest

from paper_1611_00075_amd import inputs


def _run(orc, s, steps, **kw):
    p = dict(r_list=2.8, skin=0.3, dt=0.005)
    p.update(kw)
    return orc.md_run(s.x.copy(), s.v.copy(), s.L, steps, **p)


def test_lj_nve_energy_conservation(orc):
    """Velocity Verlet is second order: the energy error over a fixed time
    shrinks fourfold when dt is halved."""
    s = inputs.lj_fcc(ncell=5)
    errs = []
    for k, dt in enumerate((0.005, 0.0025)):
        r = _run(orc, s, 100 * 2 ** k, dt=dt)
        e = r["epot"] + r["ekin"]
        errs.append(np.abs(e - e[0]).max() / s.n)
        assert r["builds"] > 1            # the rule fired during the run
        # kinetic energy moved into the potential (equipartition in a crystal)
        assert r["ekin"][-1] < r["ekin"][0]
    assert errs[0] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_lj_time_reversibility(orc):
    s = inputs.lj_fcc(ncell=4)
    x0 = orc.wrap(s.x, s.L)
    r = _run(orc, s, 60)
    back = orc.md_run(r["x"], -r["v"], s.L, 60, r_list=2.8, skin=0.3, dt=0.005)
    d = back["x"] - x0
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(back["v"] + s.v).max() < 1e-9


def test_lj_momentum_conserved(orc):
    s = inputs.lj_fcc(ncell=4)
    r = _run(orc, s, 50)
    assert np.abs(r["v"].sum(axis=0)).max() < 1e-11


def test_trajectory_independent_of_skin(orc):
    """A run that rebuilds every step (tiny skin) and one that rebuilds
    rarely (large skin) visit the same pairs inside rc: identical forces up
    to summation order."""
    s = inputs.lj_fcc(ncell=5)
    a = _run(orc, s, 40, r_list=2.5 + 1e-9, skin=1e-9)
    b = _run(orc, s, 40, r_list=2.8, skin=0.3)
    c = _run(orc, s, 40, r_list=3.4, skin=0.9)
    assert a["builds"] == 41
    assert c["builds"] < b["builds"] < a["builds"]
    for r in (b, c):
        d = r["x"] - a["x"]
        d -= s.L * np.round(d / s.L)
        assert np.abs(d).max() < 1e-10


def test_free_flight_is_exact(orc):
    L = np.full(3, 40.0)
    x = np.array([[1.0, 1.0, 1.0], [20.0, 20.0, 20.0], [5.0, 30.0, 12.0]])
    v = np.array([[0.25, -0.5, 0.125], [0.0, 0.5, -0.25], [-0.125, 0.0, 0.5]])
    r = orc.md_run(x, v, L, 16, r_list=2.8, skin=0.3, dt=0.0625)
    assert np.array_equal(r["v"], v)
    ref = orc.wrap(x + 16 * 0.0625 * v, L)
    d = r["x"] - ref
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-13
    assert np.all(r["epot"] == 0.0)


def test_rebuild_count_matches_displacement_rule(orc):
    """Free flight at speed u: the list is rebuilt exactly when the drift
    since the last build exceeds skin/2."""
    L = np.full(3, 40.0)
    x = np.array([[1.0, 1.0, 1.0]])
    v = np.array([[0.25, 0.0, 0.0]])
    # each step moves 0.25 * 0.25 = 0.0625; skin/2 = 0.15 -> rebuild every 3rd step
    r = orc.md_run(x, v, L, 30, r_list=2.8, skin=0.3, dt=0.25)
    assert r["builds"] == 1 + 30 // 3


def test_eam_nve_energy_conservation(orc):
    s = inputs.eam_cu(ncell=4, T=600.0)
    errs = []
    for k, dt in enumerate((1.0, 0.5)):
        r = orc.md_run(s.x.copy(), s.v.copy(), s.L, 100 * 2 ** k, potential="eam",
                       fs=inputs.FS_CU, r_list=5.4, skin=1.0, dt=dt,
                       mass=inputs.CU_MASS_AMU,
                       force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
        ekin = r["ekin"] * inputs.AMU_A2_FS2_IN_EV     # amu A^2/fs^2 -> eV
        e = r["epot"] + ekin
        errs.append(np.abs(e - e[0]).max() / s.n)
        assert ekin[0] / s.n == pytest.approx(
            1.5 * inputs.KB_EV * 600.0 * (s.n - 1) / s.n, rel=1e-12)
    assert errs[0] < 5e-5
    assert 3.0 < errs[0] / errs[1] < 5.0
