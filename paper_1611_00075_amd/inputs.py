"""Seeded synthetic inputs for the molecular-dynamics hot path.

This module only *draws* inputs: lattice sites, voids, clusters and
Maxwell-Boltzmann velocities.  It holds none of the method's arithmetic
(no binning, neighbour search, forces or integration), so both the FP64
oracle and the GPU library may be fed from it.

Every generator is deterministic in its seed.  Random numbers come from
numpy's PCG64 generator, one independent stream per (seed, purpose) pair.

The workloads stand in for the paper's benchmark geometries (Sec. 3.1:
the bulk fcc crystal Cu105, the porous sintered copper, the phononic crystal
with vacuum), which are not available: homogeneous fcc, fcc riddled with
spherical voids, and a slab with a vacuum gap holding a denser cluster.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# eV per (amu * Angstrom^2 / fs^2): converts m v^2 into eV in metal units
AMU_A2_FS2_IN_EV = 103.6427
# Boltzmann constant in eV/K
KB_EV = 8.617333262e-5
# copper
CU_MASS_AMU = 63.546
CU_A0 = 3.615

# Cu-like Finnis-Sinclair parameters for psi(r) = (r-d)^2, F = -A sqrt(rho),
# V(r) = (r-c)^2 (c0 + c1 r + c2 r^2).  They are the solution of four
# conditions on the perfect fcc lattice at a = 3.615 A (cohesive energy
# 3.54 eV, zero pressure, bulk modulus 138 GPa, unrelaxed vacancy formation
# energy 1.28 eV); the CPU tests re-derive each condition.
FS_CU = dict(A=0.6904081156, d=4.4, c=3.25,
             c0=12.35488532, c1=-9.40961636, c2=1.84672514)

# Second-moment tight-binding (exponential) potential of the same form as the
# paper's copper potential, with a synthetic parameter set: p and q chosen,
# r0 = the nearest-neighbour distance at a = 3.615 A, smooth cutoff between
# the third (4.43 A) and fourth (5.11 A) neighbour shells, and A, xi solved
# from the cohesive energy 3.54 eV and zero pressure at a = 3.615 A.
TB_CU = dict(A=0.1044093115, xi=1.3137843239, p=10.0, q=2.5, r0=2.5561910140, rs=4.5, rc=5.0)

# Two elements of the same form (a Cu-like 0 and an Au-like 1; synthetic):
# a common smooth cutoff 5.2-5.7 A (Cu shells 1-4 inside, Au shells 1-3),
# A and xi of each element solved from its cohesive energy (3.54 eV at
# a = 3.615 A; 3.81 eV at a = 4.078 A) and zero pressure; the mixed pair by
# geometric means of A and xi and arithmetic means of p, q and r0.
TB2_CU = dict(A=0.1051590565, xi=1.3123219176, p=10.0, q=2.5, r0=2.5561910140, rs=5.2, rc=5.7)
TB2_AU = dict(A=0.1313829015, xi=1.5090414023, p=10.5, q=3.0, r0=2.8835814537, rs=5.2, rc=5.7)
TB2_CUAU = dict(A=float(np.sqrt(TB2_CU["A"] * TB2_AU["A"])), xi=float(np.sqrt(TB2_CU["xi"] * TB2_AU["xi"])),
                p=0.5 * (TB2_CU["p"] + TB2_AU["p"]), q=0.5 * (TB2_CU["q"] + TB2_AU["q"]),
                r0=0.5 * (TB2_CU["r0"] + TB2_AU["r0"]), rs=5.2, rc=5.7)
TB2_PAIRS = (TB2_CU, TB2_CUAU, TB2_AU)
AU_A0 = 4.078

FCC_BASIS = np.array([[0.0, 0.0, 0.0],
                      [0.5, 0.5, 0.0],
                      [0.5, 0.0, 0.5],
                      [0.0, 0.5, 0.5]])


@dataclasses.dataclass
class System:
    """A periodic orthorhombic system: FP64 positions and velocities (n, 3)."""
    name: str
    L: np.ndarray            # (3,) box edge lengths
    x: np.ndarray            # (n, 3) float64
    v: np.ndarray            # (n, 3) float64
    mass: float
    kB: float                # Boltzmann constant in the system's energy unit
    e_unit: float            # m v^2 -> energy factor (1 reduced, 103.6427 metal)
    meta: dict

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def rng_for(seed: int, purpose: str) -> np.random.Generator:
    """Independent PCG64 stream for a (seed, purpose) pair."""
    key = [int(seed)] + [ord(c) for c in purpose]
    return np.random.default_rng(np.random.SeedSequence(key))


def fcc_sites(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    """fcc sites in id order: id = 4*((ix*ny + iy)*nz + iz) + b."""
    out = np.empty((nx, ny, nz, 4, 3))
    for b in range(4):
        out[:, :, :, b, 0] = (np.arange(nx)[:, None, None] + FCC_BASIS[b, 0]) * a
        out[:, :, :, b, 1] = (np.arange(ny)[None, :, None] + FCC_BASIS[b, 1]) * a
        out[:, :, :, b, 2] = (np.arange(nz)[None, None, :] + FCC_BASIS[b, 2]) * a
    return out.reshape(-1, 3)


def fcc_lattice_constant(density: float) -> float:
    return (4.0 / density) ** (1.0 / 3.0)


def maxwell_boltzmann(n: int, T: float, mass: float, kB: float, e_unit: float,
                      rng: np.random.Generator) -> np.ndarray:
    """Gaussian velocities with zero total momentum, rescaled so that
    2 KE / ((3n-3) kB) equals T exactly (KE = 1/2 m v^2 * e_unit)."""
    v = rng.standard_normal((n, 3))
    v -= v.mean(axis=0, keepdims=True)
    if n < 2 or T <= 0.0:
        return np.zeros((n, 3))
    ke = 0.5 * mass * e_unit * float(np.sum(v * v))
    target = 0.5 * (3 * n - 3) * kB * T
    v *= math.sqrt(target / ke)
    return v


def temperature(v: np.ndarray, mass: float, kB: float, e_unit: float) -> float:
    n = v.shape[0]
    ke = 0.5 * mass * e_unit * float(np.sum(v * v))
    return 2.0 * ke / ((3 * n - 3) * kB)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def lj_fcc(ncell: int = 10, density: float = 0.8442, T: float = 0.72,
           seed: int = 1001) -> System:
    """Lennard-Jones fcc crystal in reduced units (10^3 cells = 4,000 atoms)."""
    a = fcc_lattice_constant(density)
    x = fcc_sites(ncell, ncell, ncell, a)
    L = np.full(3, ncell * a)
    v = maxwell_boltzmann(len(x), T, 1.0, 1.0, 1.0, rng_for(seed, "velocity"))
    return System("lj_fcc", L, x, v, 1.0, 1.0, 1.0,
                  dict(a=a, density=density, T=T, seed=seed, ncell=ncell))


def lj_voids(ncell: int = 80, density: float = 0.8442, T: float = 0.72,
             remove_frac: float = 0.40, rmin: float = 3.0, rmax: float = 8.0,
             seed: int = 1002) -> System:
    """fcc Lennard-Jones crystal riddled with random spherical voids.

    Void centres are uniform in the box, radii uniform in [rmin, rmax];
    a site is removed when its periodic distance to a centre is strictly
    below the radius.  Voids are added until at least `remove_frac` of the
    sites are gone (80^3 cells: 2,048,000 sites, about 1.23 M atoms left)."""
    a = fcc_lattice_constant(density)
    n = ncell
    L = n * a
    keep = np.ones((n, n, n, 4), dtype=bool)
    rng = rng_for(seed, "voids")
    target = int(math.ceil(remove_frac * keep.size))
    removed = 0
    nvoid = 0
    while removed < target:
        c = rng.uniform(0.0, L, size=3)
        R = rng.uniform(rmin, rmax)
        lo = np.floor((c - R) / a).astype(int) - 1
        hi = np.floor((c + R) / a).astype(int) + 1
        rng_ax = [np.arange(lo[k], hi[k] + 1) for k in range(3)]
        I, J, K = np.meshgrid(*rng_ax, indexing="ij")
        cells = np.stack([I, J, K], -1).reshape(-1, 1, 3)
        pos = (cells + FCC_BASIS[None]) * a          # unwrapped image positions
        d = pos - c
        r2 = np.sum(d * d, axis=-1)
        hit = r2 < R * R
        ci = np.mod(cells.reshape(-1, 3), n)
        hi_idx = np.nonzero(hit)
        cc = ci[hi_idx[0]]
        bb = hi_idx[1]
        before = keep[cc[:, 0], cc[:, 1], cc[:, 2], bb]
        removed += int(np.count_nonzero(before))
        keep[cc[:, 0], cc[:, 1], cc[:, 2], bb] = False
        nvoid += 1
    x = fcc_sites(n, n, n, a)[keep.reshape(-1)]
    v = maxwell_boltzmann(len(x), T, 1.0, 1.0, 1.0, rng_for(seed, "velocity"))
    return System("lj_voids", np.full(3, L), x, v, 1.0, 1.0, 1.0,
                  dict(a=a, density=density, T=T, seed=seed, ncell=n,
                       sites=keep.size, voids=nvoid))


def lj_slab_cluster(nxy: int = 251, nz_slab: int = 125, density: float = 0.8442,
                    cluster_density: float = 1.05, cluster_atoms: int = 2_000_000,
                    T: float = 0.72, seed: int = 1004) -> System:
    """fcc slab filling the lower half of a cubic periodic box (vacuum above)
    with a denser spherical fcc cluster at the slab centre.

    The box edge is nxy fcc cells of the slab lattice in every direction;
    slab sites within R + 0.5 of the centre are removed and the sphere of
    radius R is re-filled with fcc at `cluster_density`, R chosen so that the
    sphere holds about `cluster_atoms` atoms (defaults: about 32 M atoms)."""
    a = fcc_lattice_constant(density)
    L = nxy * a
    slab = fcc_sites(nxy, nxy, nz_slab, a)
    centre = np.array([0.5 * L, 0.5 * L, 0.5 * nz_slab * a])
    R = (3.0 * cluster_atoms / (4.0 * math.pi * cluster_density)) ** (1.0 / 3.0)
    keep = np.ones(len(slab), dtype=bool)
    step = 1 << 22
    for k in range(0, len(slab), step):
        d = slab[k:k + step] - centre
        keep[k:k + step] = np.einsum("ij,ij->i", d, d) >= (R + 0.5) ** 2
    slab = slab[keep]
    del keep
    a2 = fcc_lattice_constant(cluster_density)
    m = int(math.ceil(R / a2)) + 1
    cl = fcc_sites(2 * m, 2 * m, 2 * m, a2) - m * a2 + centre
    dc = cl - centre
    cl = cl[np.sum(dc * dc, axis=1) < R * R]
    x = np.concatenate([slab, cl])
    v = maxwell_boltzmann(len(x), T, 1.0, 1.0, 1.0, rng_for(seed, "velocity"))
    return System("lj_slab_cluster", np.full(3, L), x, v, 1.0, 1.0, 1.0,
                  dict(a=a, density=density, cluster_density=cluster_density,
                       R=R, T=T, seed=seed, slab_atoms=len(slab),
                       cluster_atoms=len(cl)))


def eam_cu(ncell: int = 100, a: float = CU_A0, T: float = 600.0,
           seed: int = 1003) -> System:
    """fcc Cu-like metal in eV, Angstrom, amu, fs (100^3 cells = 4 M atoms)."""
    x = fcc_sites(ncell, ncell, ncell, a)
    v = maxwell_boltzmann(len(x), T, CU_MASS_AMU, KB_EV, AMU_A2_FS2_IN_EV,
                          rng_for(seed, "velocity"))
    return System("eam_cu", np.full(3, ncell * a), x, v, CU_MASS_AMU, KB_EV,
                  AMU_A2_FS2_IN_EV, dict(a=a, T=T, seed=seed, ncell=ncell))


def cu_au(ncell: int = 100, layered: bool = False, frac_au: float = 0.25, T: float = 600.0,
          seed: int = 1006) -> System:
    """Two-element fcc metal on one lattice (a by Vegard's rule for 25 % of
    element 1): a random alloy with fraction frac_au of element 1 (the
    paper's Alloy system), or two layers, element 0 below z = L/2 and
    element 1 above (its Layer system).  meta["types"] holds the element of
    each atom.  One mass (Cu's) for both elements."""
    a = (1.0 - 0.25) * CU_A0 + 0.25 * AU_A0
    x = fcc_sites(ncell, ncell, ncell, a)
    L = np.full(3, ncell * a)
    if layered:
        t = (x[:, 2] >= 0.5 * L[2]).astype(np.int32)
    else:
        t = (rng_for(seed, "elements").random(len(x)) < frac_au).astype(np.int32)
    v = maxwell_boltzmann(len(x), T, CU_MASS_AMU, KB_EV, AMU_A2_FS2_IN_EV, rng_for(seed, "velocity"))
    return System("cu_au_layers" if layered else "cu_au_alloy", L, x, v, CU_MASS_AMU, KB_EV, AMU_A2_FS2_IN_EV,
                  dict(a=a, T=T, seed=seed, ncell=ncell, types=t, frac_au=float(t.mean())))


def fs_table(fs: dict = FS_CU, dr: float = 0.005, drho: float = 0.05, rho_max: float = 100.0) -> dict:
    """Input tables of the tabulated embedded-atom form sampled from a
    Finnis-Sinclair parameter set (its functions psi = (r - d)^2 below d,
    V = (r - c)^2 (c0 + c1 r + c2 r^2) below c, F = -A sqrt(rho)): values and
    slopes at r_k = k dr up to d (dr must divide d and c) and at
    rho_k = k drho up to rho_max.  At rho = 0, where F has no finite slope,
    the slope given is that of the chord to the next knot."""
    d, c = fs["d"], fs["c"]
    nr = int(round(d / dr)) + 1
    if abs((nr - 1) * dr - d) > 1e-9 or abs(round(c / dr) * dr - c) > 1e-9:
        raise ValueError("dr must divide both cutoffs")
    r = np.arange(nr) * dr
    psi = np.where(r < d, (r - d) ** 2, 0.0)
    dpsi = np.where(r < d, 2.0 * (r - d), 0.0)
    q = fs["c0"] + fs["c1"] * r + fs["c2"] * r * r
    dq = fs["c1"] + 2.0 * fs["c2"] * r
    phi = np.where(r < c, (r - c) ** 2 * q, 0.0)
    dphi = np.where(r < c, 2.0 * (r - c) * q + (r - c) ** 2 * dq, 0.0)
    nrho = int(round(rho_max / drho)) + 1
    rho = np.arange(nrho) * drho
    F = -fs["A"] * np.sqrt(rho)
    dF = np.empty(nrho)
    dF[1:] = -0.5 * fs["A"] / np.sqrt(rho[1:])
    dF[0] = (F[1] - F[0]) / drho
    return dict(dr=dr, drho=drho, psi=psi, dpsi=dpsi, phi=phi, dphi=dphi, F=F, dF=dF)


def jitter(sys: System, sigma: float, seed: int) -> System:
    """Copy of `sys` with Gaussian position noise of width sigma (a stand-in
    for a thermalised snapshot in per-call parity tests)."""
    rng = rng_for(seed, "jitter")
    x = sys.x + rng.normal(0.0, sigma, size=sys.x.shape)
    return dataclasses.replace(sys, x=x, meta=dict(sys.meta, jitter=sigma))


def graded(ncell: int, a: float, jit: float, seed: int, n_gas: int = 60, gas_sep: float = 2.0) -> tuple:
    """fcc sites (ncell^3 cells of edge a) with site i kept with probability
    2 |1 - 2 x_i / L| - 1 (clipped to [0, 1]) along the first axis, then
    Gaussian noise of width jit: the local density falls from the lattice's
    at the (periodic) box face to zero over a quarter of the box; the empty
    middle half holds n_gas random atoms (x in [0.3 L, 0.7 L], no two closer
    than gas_sep).  The neighbour counts thus take every value from 0 to the
    full lattice's.  Returns (positions, box)."""
    x = fcc_sites(ncell, ncell, ncell, a)
    L = np.full(3, ncell * a)
    rng = rng_for(seed, "graded")
    keep = rng.uniform(0.0, 1.0, size=len(x)) < 2.0 * np.abs(1.0 - 2.0 * x[:, 0] / L[0]) - 1.0
    x = x[keep] + rng.normal(0.0, jit, size=(int(keep.sum()), 3))
    gas = []
    while len(gas) < n_gas:
        p = rng.uniform(0.0, 1.0, size=3) * L
        p[0] = L[0] * (0.3 + 0.4 * p[0] / L[0])
        d = np.array(gas) - p if gas else np.zeros((0, 3))
        d -= L * np.round(d / L)
        if not len(gas) or float(np.min(np.sum(d * d, axis=1))) >= gas_sep * gas_sep:
            gas.append(p)
    return np.concatenate([x, np.array(gas).reshape(-1, 3)]), L


def random_gas(n: int, L, seed: int, min_dist: float = 0.0) -> np.ndarray:
    """n uniform random points in a box (optionally rejecting points closer
    than min_dist to an earlier point, by periodic distance)."""
    rng = rng_for(seed, "gas")
    L = np.asarray(L, dtype=np.float64)
    if min_dist <= 0.0:
        return rng.uniform(0.0, 1.0, size=(n, 3)) * L
    pts = []
    while len(pts) < n:
        p = rng.uniform(0.0, 1.0, size=3) * L
        ok = True
        for q in pts:
            d = p - q
            d -= L * np.round(d / L)
            if float(np.dot(d, d)) < min_dist * min_dist:
                ok = False
                break
        if ok:
            pts.append(p)
    return np.array(pts)
