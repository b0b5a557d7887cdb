"""ctypes view of the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["oracle.c", "mlp.c"]


COMPILER_FLAGS = "gcc -O2 -std=gnu11 -fPIC -shared -ffp-contract=off -fopenmp -lm"


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, s) for s in _SOURCES
                if os.path.exists(os.path.join(_HERE, s))]
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fopenmp", *srcs, "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


class LJParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double)]


class FSParams(C.Structure):
    _fields_ = [("A", C.c_double), ("d", C.c_double), ("c", C.c_double),
                ("c0", C.c_double), ("c1", C.c_double), ("c2", C.c_double)]


class MDParams(C.Structure):
    _fields_ = [("potential", C.c_int32), ("lj", LJParams), ("fs", FSParams),
                ("r_list", C.c_double), ("skin", C.c_double), ("dt", C.c_double),
                ("mass", C.c_double), ("force_to_accel", C.c_double),
                ("reverse_order", C.c_int32), ("threads", C.c_int32)]


POT_LJ, POT_EAM = 0, 1


def _declare(L):
    L.or_wrap.argtypes = [C.c_int64, _dp, _dp, _dp, _dp]
    L.or_cell_coords.argtypes = [C.c_int64, _dp, _i32p, _dp, _dp, _dp, _i32p, _i32p, _i32p]
    L.or_minimg.argtypes = [C.c_double, C.c_double, C.c_double]
    L.or_minimg.restype = C.c_double
    for f in (L.or_neighbors_brute, L.or_neighbors_cells):
        f.argtypes = [C.c_int64, _dp, C.c_double, _dp, _dp, _dp, _i64p, _i32p, C.c_int64]
        f.restype = C.c_int64
    L.or_forces_lj.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                               C.POINTER(LJParams), _dp, _dp, _dp, _dp]
    L.or_neighbors_cells_omp.argtypes = [C.c_int64, _dp, C.c_double, _dp, _dp, _dp, _i64p, _i32p, C.c_int64,
                                         C.c_int32]
    L.or_neighbors_cells_omp.restype = C.c_int64
    L.or_forces_lj_omp.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                   C.POINTER(LJParams), _dp, _dp, _dp, _dp, C.c_int32]
    L.or_forces_eam.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                C.POINTER(FSParams), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_forces_tb.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                               C.POINTER(TBParams), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_forces_tbm.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i32p, _i64p, _i32p,
                                C.POINTER(TBParams), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_forces_tab.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                C.POINTER(TabParams), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_tab_eval.argtypes = [C.c_int32, C.c_double, _dp, _dp, C.c_double, _dp, _dp]
    L.or_md_run.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                            C.POINTER(MDParams), C.c_int64, _dp, _dp, _dp]
    L.or_md_run.restype = C.c_int64
    if hasattr(L, "or_mlp_descriptors"):
        _declare_mlp(L)


def _p(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def _soa(x):
    x = np.asarray(x, dtype=np.float64)
    return [np.ascontiguousarray(x[:, k]) for k in range(3)]


def _box(L):
    return np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))


# --------------------------------------------------------------------------
def wrap(x, L):
    """Positions (n,3) wrapped into [0, L)."""
    xs = _soa(x)
    Lb = _box(L)
    lib().or_wrap(len(xs[0]), _p(Lb), *[_p(c) for c in xs])
    return np.stack(xs, axis=1)


def cell_coords(x, L, nc):
    xs = _soa(x)
    n = len(xs[0])
    out = [np.empty(n, np.int32) for _ in range(3)]
    ncv = np.ascontiguousarray(np.asarray(nc, dtype=np.int32).reshape(3))
    lib().or_cell_coords(n, _p(_box(L)), _p(ncv, _i32p), *[_p(c) for c in xs],
                         *[_p(c, _i32p) for c in out])
    return np.stack(out, axis=1)


def minimg(a, b, L):
    return lib().or_minimg(float(a), float(b), float(L))


def _neighbors(fn, x, L, r_list):
    xs = _soa(x)
    n = len(xs[0])
    off = np.zeros(n + 1, np.int64)
    cap = 0
    idx = np.zeros(1, np.int32)
    total = fn(n, _p(_box(L)), float(r_list), *[_p(c) for c in xs], _p(off, _i64p),
               _p(idx, _i32p), cap)
    idx = np.zeros(max(total, 1), np.int32)
    fn(n, _p(_box(L)), float(r_list), *[_p(c) for c in xs], _p(off, _i64p),
       _p(idx, _i32p), total)
    return off, idx[:total]


def neighbors_brute(x, L, r_list):
    """CSR full list {j != i : r^2 < r_list^2}, rows ascending (O(N^2))."""
    return _neighbors(lib().or_neighbors_brute, x, L, r_list)


def neighbors_cells_omp(x, L, r_list, threads=2):
    """neighbors_cells with the rows shared among OpenMP threads (timing aid)."""
    return _neighbors(lambda *a: lib().or_neighbors_cells_omp(*a, int(threads)), x, L, r_list)


def neighbors_cells(x, L, r_list):
    """The same set through a 27-cell list; positions must be wrapped."""
    return _neighbors(lib().or_neighbors_cells, x, L, r_list)


def forces_lj(x, L, off, idx, eps=1.0, sigma=1.0, rc=2.5):
    """FP64 LJ forces (n,3) and ev[8] = E, E_shift, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    ev = np.zeros(8)
    prm = LJParams(eps, sigma, rc)
    lib().or_forces_lj(n, _p(_box(L)), *[_p(c) for c in xs],
                       _p(np.ascontiguousarray(off, np.int64), _i64p),
                       _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(prm),
                       *[_p(c) for c in f], _p(ev))
    return np.stack(f, axis=1), ev


def forces_lj_omp(x, L, off, idx, eps=1.0, sigma=1.0, rc=2.5, threads=2):
    """forces_lj with the rows shared among OpenMP threads (timing aid)."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    ev = np.zeros(8)
    prm = LJParams(eps, sigma, rc)
    lib().or_forces_lj_omp(n, _p(_box(L)), *[_p(c) for c in xs],
                           _p(np.ascontiguousarray(off, np.int64), _i64p),
                           _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(prm),
                           *[_p(c) for c in f], _p(ev), int(threads))
    return np.stack(f, axis=1), ev


def forces_eam(x, L, off, idx, fs: dict):
    """FP64 Finnis-Sinclair EAM: dict with rho, fprime, f (n,3), e_atom, ev[8]
    (E_total, E_embed, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz)."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    rho, fp, ea, ev = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(8)
    prm = FSParams(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"])
    lib().or_forces_eam(n, _p(_box(L)), *[_p(c) for c in xs],
                        _p(np.ascontiguousarray(off, np.int64), _i64p),
                        _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(prm),
                        _p(rho), _p(fp), *[_p(c) for c in f], _p(ea), _p(ev))
    return dict(rho=rho, fprime=fp, f=np.stack(f, axis=1), e_atom=ea, ev=ev)


class TBParams(C.Structure):
    _fields_ = [("A", C.c_double), ("xi", C.c_double), ("p", C.c_double), ("q", C.c_double),
                ("r0", C.c_double), ("rs", C.c_double), ("rc", C.c_double)]


def forces_tb(x, L, off, idx, tb: dict):
    """FP64 second-moment tight-binding potential: dict as forces_eam."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    rho, fp, ea, ev = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(8)
    prm = TBParams(*[float(tb[k]) for k in ("A", "xi", "p", "q", "r0", "rs", "rc")])
    lib().or_forces_tb(n, _p(_box(L)), *[_p(c) for c in xs],
                       _p(np.ascontiguousarray(off, np.int64), _i64p),
                       _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(prm),
                       _p(rho), _p(fp), *[_p(c) for c in f], _p(ea), _p(ev))
    return dict(rho=rho, fprime=fp, f=np.stack(f, axis=1), e_atom=ea, ev=ev)


def forces_tbm(x, L, off, idx, types, pairs):
    """FP64 two-element tight-binding potential; `pairs` = three parameter
    dicts for the element pairs 0-0, 0-1, 1-1.  Output as forces_eam."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    rho, fp, ea, ev = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(8)
    prm = (TBParams * 3)(*[TBParams(*[float(t[k]) for k in ("A", "xi", "p", "q", "r0", "rs", "rc")])
                           for t in pairs])
    lib().or_forces_tbm(n, _p(_box(L)), *[_p(c) for c in xs], _p(np.ascontiguousarray(types, np.int32), _i32p),
                        _p(np.ascontiguousarray(off, np.int64), _i64p),
                        _p(np.ascontiguousarray(idx, np.int32), _i32p), prm,
                        _p(rho), _p(fp), *[_p(c) for c in f], _p(ea), _p(ev))
    return dict(rho=rho, fprime=fp, f=np.stack(f, axis=1), e_atom=ea, ev=ev)


class TabParams(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nrho", C.c_int32), ("dr", C.c_double), ("drho", C.c_double),
                ("psi", _dp), ("dpsi", _dp), ("phi", _dp), ("dphi", _dp), ("F", _dp), ("dF", _dp)]


def _tab_struct(tab):
    arrs = {k: np.ascontiguousarray(tab[k], dtype=np.float64) for k in ("psi", "dpsi", "phi", "dphi", "F", "dF")}
    nr, nrho = len(arrs["psi"]), len(arrs["F"])
    assert all(len(arrs[k]) == nr for k in ("dpsi", "phi", "dphi")) and len(arrs["dF"]) == nrho
    prm = TabParams(nr, nrho, float(tab["dr"]), float(tab["drho"]), *[_p(arrs[k]) for k in
                                                                       ("psi", "dpsi", "phi", "dphi", "F", "dF")])
    return prm, arrs


def tab_eval(f, df, h, u):
    """One tabulated function (values f, slopes df at knots k h) at the
    points u: (values, slopes) of its cubic Hermite interpolant."""
    f = np.ascontiguousarray(f, np.float64)
    df = np.ascontiguousarray(df, np.float64)
    u = np.atleast_1d(np.asarray(u, np.float64))
    val, slope = np.zeros(len(u)), np.zeros(len(u))
    v, s = C.c_double(), C.c_double()
    for k, uk in enumerate(u):
        lib().or_tab_eval(len(f), float(h), _p(f), _p(df), float(uk), C.byref(v), C.byref(s))
        val[k], slope[k] = v.value, s.value
    return val, slope


def forces_tab(x, L, off, idx, tab):
    """FP64 tabulated embedded-atom potential.  `tab`: dict with dr, drho and
    the knot arrays psi, dpsi, phi, dphi (r_k = k dr) and F, dF
    (rho_k = k drho).  Output as forces_eam."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    rho, fp, ea, ev = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(8)
    prm, keep = _tab_struct(tab)
    lib().or_forces_tab(n, _p(_box(L)), *[_p(c) for c in xs],
                        _p(np.ascontiguousarray(off, np.int64), _i64p),
                        _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(prm),
                        _p(rho), _p(fp), *[_p(c) for c in f], _p(ea), _p(ev))
    del keep
    return dict(rho=rho, fprime=fp, f=np.stack(f, axis=1), e_atom=ea, ev=ev)


def md_run(x, v, L, steps, *, potential="lj", lj=(1.0, 1.0, 2.5), fs=None,
           r_list, skin, dt, mass=1.0, force_to_accel=1.0, reverse_order=False, threads=1):
    """Velocity-Verlet run.  Returns dict(x, v, epot[steps+1], ekin[steps+1],
    builds, loop_seconds).  threads > 1: LJ forces and the per-atom loops on
    that many OpenMP threads (for timing)."""
    xs = _soa(x)
    vs = _soa(v)
    n = len(xs[0])
    prm = MDParams()
    prm.potential = POT_LJ if potential == "lj" else POT_EAM
    prm.lj = LJParams(*lj)
    if fs is not None:
        prm.fs = FSParams(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"])
    prm.r_list, prm.skin, prm.dt = r_list, skin, dt
    prm.mass, prm.force_to_accel = mass, force_to_accel
    prm.reverse_order = 1 if reverse_order else 0
    prm.threads = int(threads)
    ep = np.zeros(steps + 1)
    ek = np.zeros(steps + 1)
    secs = np.zeros(1)
    builds = lib().or_md_run(n, _p(_box(L)), *[_p(c) for c in xs], *[_p(c) for c in vs],
                             C.byref(prm), int(steps), _p(ep), _p(ek), _p(secs))
    if builds < 0:
        raise MemoryError("oracle md_run failed to allocate")
    return dict(x=np.stack(xs, 1), v=np.stack(vs, 1), epot=ep, ekin=ek, builds=builds,
                loop_seconds=float(secs[0]))


def _declare_mlp(L):  # filled in by the MLP part of the oracle
    from . import mlp as _m
    _m.declare(L)
