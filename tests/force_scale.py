"""Per-atom force bounds for the parity tests (test helper, not a test).

The FP32 pair kernels are held to 1e-5 of each atom's sum of pair-force
magnitudes, sum_j |f_ij|, besides the normwise 1e-5: a per-atom relative
error is unbounded where F_i -> 0 by cancellation, while the rounding error
of a sum scales with its terms.  For the embedded-atom forms the pair force
on i from j is -[(F'_i + F'_j) psi'(r) + Phi'(r)] (r_i - r_j)/r (the third
step of Sec. 3.1 after Eqs. (1)-(2)); its magnitude is taken term by term,
|(F'_i + F'_j) psi'(r)| + |Phi'(r)|, the scale of the FP32 rounding of the
pair's two terms.  The functional forms below only set that error scale;
every expected value comes from the oracle.

Pairs closer to a cutoff than 1e-5 of it may be decided differently by the
FP32 test on the GPU and the FP64 test of the oracle; an atom with such a
pair may instead match the oracle's force with that pair's term added or
removed.
"""
import numpy as np

AMBIG = 1e-5


def pair_table(x, L, off, idx):
    """Every listed pair (i, j): arrays I, J, R = minimum-image r_i - r_j
    (n_pairs, 3) and r."""
    n = len(x)
    cnt = np.diff(off)
    I = np.repeat(np.arange(n), cnt)
    J = np.asarray(idx[: off[-1]], np.int64)
    R = x[I] - x[J]
    R -= L * np.round(R / L)
    return I, J, R, np.sqrt(np.sum(R * R, 1))


def check_per_atom(fg, fo, I, R, r, mag, s, cutoffs, tol=1e-5, what=""):
    """Normwise and per-atom bounds.  mag[p]: the pair's force magnitude
    (term by term), s[p]: its signed scalar (force on I[p] is -s R / r),
    both zero for pairs beyond every cutoff; cutoffs: the radii where a
    pair's term switches on or off.  Returns (normwise error, largest
    per-atom ratio |dF_i| / sum_j |f_ij|)."""
    n = len(fg)
    err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    assert err <= tol, (what, err)
    fabs = np.bincount(I, weights=mag, minlength=n)
    d = np.linalg.norm(fg - fo, axis=1)
    ok = d <= tol * fabs + 1e-12
    amb = np.zeros(len(r), bool)
    for c in cutoffs:
        amb |= np.abs(r - c) < AMBIG * c
    if not ok.all():
        vec = -(s / np.where(r > 0, r, 1.0))[:, None] * R
        contrib = np.zeros((n, 3))
        for k in range(3):
            contrib[:, k] = np.bincount(I[amb], weights=vec[amb, k], minlength=n)
        near = np.bincount(I[amb], minlength=n) > 0
        for i in np.nonzero(~ok)[0]:
            assert near[i], (what, i, d[i], fabs[i])
            alt = min(np.linalg.norm(fg[i] - (fo[i] + contrib[i])), np.linalg.norm(fg[i] - (fo[i] - contrib[i])))
            assert alt <= tol * fabs[i] + 1e-12, (what, i, alt, fabs[i])
    ratio = float(np.max(np.where(fabs > 0, d / np.where(fabs > 0, fabs, 1.0), 0.0))) if n else 0.0
    return err, ratio


def _embed_terms(fp, I, J, dpsi, dphi):
    emb = (fp[I] + fp[J]) * dpsi
    return np.abs(emb) + np.abs(dphi), emb + dphi


def fs_terms(fp, I, J, r, fs):
    """Finnis-Sinclair: psi = (r - d)^2 (r < d), V = (r - c)^2 (c0 + c1 r + c2 r^2) (r < c)."""
    d, c = fs["d"], fs["c"]
    dpsi = np.where(r < d, 2.0 * (r - d), 0.0)
    poly = fs["c0"] + fs["c1"] * r + fs["c2"] * r * r
    dv = 2.0 * (r - c) * poly + (r - c) ** 2 * (fs["c1"] + 2.0 * fs["c2"] * r)
    dphi = np.where(r < c, dv, 0.0)
    mag, s = _embed_terms(fp, I, J, dpsi, dphi)
    return mag, s, (d, c)


def _smooth(r, rs, rc):
    x = np.clip((r - rs) / (rc - rs), 0.0, 1.0)
    S = 1.0 - x ** 3 * (10.0 - 15.0 * x + 6.0 * x * x)
    dS = -30.0 * x * x * (1.0 - x) ** 2 / (rc - rs)
    return np.where(r < rc, S, 0.0), np.where(r < rc, dS, 0.0)


def _tb_derivs(r, t):
    S, dS = _smooth(r, t["rs"], t["rc"])
    ep = t["xi"] ** 2 * np.exp(-2.0 * t["q"] * (r / t["r0"] - 1.0))
    eP = 2.0 * t["A"] * np.exp(-t["p"] * (r / t["r0"] - 1.0))
    return ep * (-2.0 * t["q"] / t["r0"] * S + dS), eP * (-t["p"] / t["r0"] * S + dS)


def tb_terms(fp, I, J, r, tb):
    """Second-moment tight-binding: psi = xi^2 exp(-2q(r/r0 - 1)) S,
    Phi = 2A exp(-p(r/r0 - 1)) S."""
    dpsi, dphi = _tb_derivs(r, tb)
    mag, s = _embed_terms(fp, I, J, dpsi, dphi)
    return mag, s, (tb["rc"],)


def tbm_terms(fp, I, J, r, types, pairs):
    """Two elements: the parameters of the pair's kind t_i + t_j."""
    kind = np.asarray(types)[I] + np.asarray(types)[J]
    dpsi, dphi = np.zeros(len(r)), np.zeros(len(r))
    for k in range(3):
        m = kind == k
        dpsi[m], dphi[m] = _tb_derivs(r[m], pairs[k])
    mag, s = _embed_terms(fp, I, J, dpsi, dphi)
    return mag, s, tuple(sorted({float(p["rc"]) for p in pairs}))


def tab_terms(orc, fp, I, J, r, tab):
    """Tabulated psi, Phi: slopes of the oracle's own interpolant."""
    rc = (len(tab["psi"]) - 1) * tab["dr"]
    inside = r < rc
    dpsi, dphi = np.zeros(len(r)), np.zeros(len(r))
    if inside.any():
        dpsi[inside] = orc.tab_eval(tab["psi"], tab["dpsi"], tab["dr"], r[inside])[1]
        dphi[inside] = orc.tab_eval(tab["phi"], tab["dphi"], tab["dr"], r[inside])[1]
    mag, s = _embed_terms(fp, I, J, dpsi, dphi)
    return mag, s, (rc,)


def lj_terms(I, J, r, rc=2.5, eps=1.0, sigma=1.0):
    """Lennard-Jones, truncated at rc: force on i is 24 eps s6 (2 s6 - 1) / r^2 (r_i - r_j)."""
    s6 = (sigma * sigma / (r * r)) ** 3
    fs = np.where(r < rc, 24.0 * eps * s6 * (2.0 * s6 - 1.0) / (r * r), 0.0)
    return np.abs(fs) * r, -fs * r, (rc,)


def check_form(orc, form, fg, x, L, off, idx, ref, params, types=None, what="", tol=1e-5, atoms=None):
    """check_per_atom for an embedded-atom form ("fs", "tb", "tbm", "tab")
    or "lj" (ref: the oracle's output dict, or its force array for LJ).
    With `atoms` (indices into x), fg holds the forces of those atoms only
    and only they are checked.  Prints and returns (normwise error, largest
    per-atom ratio)."""
    I, J, R, r = pair_table(x, L, off, idx)
    if form == "lj":
        mag, s, cuts = lj_terms(I, J, r, **(params or {}))
        fo = ref
    else:
        fp = ref["fprime"]
        fo = ref["f"]
        if form == "fs":
            mag, s, cuts = fs_terms(fp, I, J, r, params)
        elif form == "tb":
            mag, s, cuts = tb_terms(fp, I, J, r, params)
        elif form == "tbm":
            mag, s, cuts = tbm_terms(fp, I, J, r, types, params)
        else:
            mag, s, cuts = tab_terms(orc, fp, I, J, r, params)
    if atoms is not None:
        atoms = np.asarray(atoms)
        pos = np.full(len(x), -1)
        pos[atoms] = np.arange(len(atoms))
        keep = pos[I] >= 0
        I, R, r, mag, s = pos[I[keep]], R[keep], r[keep], mag[keep], s[keep]
        fo = fo[atoms]
    err, ratio = check_per_atom(fg, fo, I, R, r, mag, s, cuts, tol=tol, what=what)
    print(f"{what}: FP32 force error normwise {err:.2e}, per atom <= {ratio:.2e} of sum_j |f_ij|")
    return err, ratio
