"""ctypes view of the FP64 oracle of the learned descriptor-MLP potential.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  The model,
the parameter layout and the BF16 rounding points are stated in mlp.h.
"""
from __future__ import annotations

import ctypes as C
from concurrent.futures import ThreadPoolExecutor
import dataclasses

import numpy as np

from . import FSParams, MDParams, POT_EAM, _box, _dp, _i32p, _i64p, _p, _soa, lib

N_IN = 16
N_HID = 64
N_PARAM = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_HID + 1  # 5,313


class MLPSpec(C.Structure):
    _fields_ = [("rc", C.c_double), ("mu0", C.c_double), ("dmu", C.c_double),
                ("width", C.c_double), ("mean", C.c_double * N_IN),
                ("inv_std", C.c_double * N_IN)]


def declare(L):
    L.or_bf16_round.argtypes = [C.c_double]
    L.or_bf16_round.restype = C.c_double
    L.or_mlp_descriptors.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                     C.POINTER(MLPSpec), _dp]
    L.or_mlp_energy.argtypes = [C.c_int64, _dp, C.POINTER(MLPSpec), _dp, C.c_int32, _dp, _dp]
    L.or_mlp_forces.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                C.POINTER(MLPSpec), _dp, _dp, _dp, _dp, _dp]
    L.or_mlp_loss_grad.argtypes = [C.c_int64, _dp, _dp, C.POINTER(MLPSpec), _dp,
                                   C.c_int32, _dp]
    L.or_mlp_loss_grad.restype = C.c_double
    L.or_eam_samples.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                 C.POINTER(MDParams), C.c_double, C.c_double, C.c_double,
                                 C.c_int64, C.c_int64, C.c_int64, C.c_int64, _dp, _dp, _dp]
    L.or_eam_samples.restype = C.c_int64


@dataclasses.dataclass
class Spec:
    """Descriptor geometry and input normalisation."""
    rc: float = 5.0
    mu0: float = 2.0
    dmu: float = 0.2
    width: float = 0.2
    mean: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(N_IN))
    inv_std: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(N_IN))

    def c(self) -> MLPSpec:
        s = MLPSpec(self.rc, self.mu0, self.dmu, self.width)
        s.mean[:] = [float(v) for v in np.asarray(self.mean, np.float64)]
        s.inv_std[:] = [float(v) for v in np.asarray(self.inv_std, np.float64)]
        return s


def unpack(params):
    """Parameter vector -> dict of W1 (64,16), b1, W2 (64,64), b2, w3, b3."""
    p = np.asarray(params, np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)),
                        ("b2", (N_HID,)), ("w3", (N_HID,)), ("b3", ())):
        size = int(np.prod(shape)) if shape else 1
        out[name] = p[o:o + size].reshape(shape) if shape else float(p[o])
        o += size
    assert o == N_PARAM
    return out


def bf16_round(v: float) -> float:
    return lib().or_bf16_round(float(v))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def descriptors(x, L, off, idx, spec: Spec):
    """Raw descriptors G (n, 16) from a full neighbour list."""
    xs = _soa(x)
    n = len(xs[0])
    G = np.zeros((n, N_IN))
    sp = spec.c()
    lib().or_mlp_descriptors(n, _p(_box(L)), *[_p(c) for c in xs],
                             _p(np.ascontiguousarray(off, np.int64), _i64p),
                             _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(sp), _p(G))
    return G


def energy(G, spec: Spec, params, bf16: bool = False, grad: bool = True):
    """Per-atom energies (n,) and dE_i/dG_i (n, 16) (None if grad is False)."""
    G = _c64(G)
    n = G.shape[0]
    e = np.zeros(n)
    d = np.zeros((n, N_IN)) if grad else None
    sp = spec.c()
    lib().or_mlp_energy(n, _p(G), C.byref(sp), _p(_c64(params)), 1 if bf16 else 0, _p(e), _p(d))
    return e, d


def forces(x, L, off, idx, spec: Spec, dEdG):
    """Forces (n, 3) and virial [xx, yy, zz, xy, xz, yz]."""
    xs = _soa(x)
    n = len(xs[0])
    f = [np.zeros(n) for _ in range(3)]
    w6 = np.zeros(6)
    sp = spec.c()
    lib().or_mlp_forces(n, _p(_box(L)), *[_p(c) for c in xs],
                        _p(np.ascontiguousarray(off, np.int64), _i64p),
                        _p(np.ascontiguousarray(idx, np.int32), _i32p), C.byref(sp),
                        _p(_c64(dEdG)), *[_p(c) for c in f], _p(w6))
    return np.stack(f, axis=1), w6


def loss_grad(G, target, spec: Spec, params, bf16: bool = False, grad: bool = True):
    """Mean squared per-atom energy error and its parameter gradient."""
    G = _c64(G)
    g = np.zeros(N_PARAM) if grad else None
    sp = spec.c()
    loss = lib().or_mlp_loss_grad(G.shape[0], _p(G), _p(_c64(target)), C.byref(sp),
                                  _p(_c64(params)), 1 if bf16 else 0, _p(g))
    return loss, g


def potential_energy(x, L, off, idx, spec: Spec, params, bf16: bool = False):
    """E = sum_i E_i for positions x (the function the forces differentiate)."""
    e, _ = energy(descriptors(x, L, off, idx, spec), spec, params, bf16, grad=False)
    return float(np.sum(e))


def adam(params, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) in FP64; step counts from 1.
    Returns new (params, m1, m2)."""
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mh = m1 / (1.0 - beta1 ** step)
    vh = m2 / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2


def ridge_fit(X, y, lam=1e-8):
    """Closed-form ridge regression y ~ X u + b (bias unpenalised).
    Returns (u, b)."""
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    xm = X.mean(axis=0)
    ym = y.mean()
    Xc = X - xm
    A = Xc.T @ Xc + lam * X.shape[0] * np.eye(X.shape[1])
    u = np.linalg.solve(A, Xc.T @ (y - ym))
    return u, float(ym - xm @ u)


def eam_samples(x, v, L, fs: dict, T, *, n_samples, sample_every=20, equil_steps=2000,
                rescale_every=100, r_list=5.4, skin=1.0, dt=1.0, mass=63.546,
                kB=8.617333262e-5, e_unit=103.6427):
    """One Finnis-Sinclair trajectory at temperature T (K): equilibration with
    velocity rescaling, then n_samples NVE snapshots.  Returns dict(pos
    (s, n, 3), e_atom (s, n), forces (s, n, 3), builds)."""
    xs = _soa(x)
    vs = _soa(v)
    n = len(xs[0])
    prm = MDParams()
    prm.potential = POT_EAM
    prm.fs = FSParams(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"])
    prm.r_list, prm.skin, prm.dt = r_list, skin, dt
    prm.mass, prm.force_to_accel = mass, 1.0 / e_unit
    pos = np.zeros((n_samples, n, 3))
    ea = np.zeros((n_samples, n))
    fo = np.zeros((n_samples, n, 3))
    b = lib().or_eam_samples(n, _p(_box(L)), *[_p(c) for c in xs], *[_p(c) for c in vs],
                             C.byref(prm), float(T), kB, e_unit, int(equil_steps),
                             int(rescale_every), int(n_samples), int(sample_every),
                             _p(pos), _p(ea), _p(fo))
    if b < 0:
        raise MemoryError("oracle eam_samples failed")
    return dict(pos=pos, e_atom=ea, forces=fo, builds=int(b))


def training_set(starts, temps, fs: dict, n_samples, threads=8, **kw):
    """Trajectories for each (x, v, L) start and temperature, run in parallel
    threads (the C calls release the interpreter lock).  Returns a list of
    eam_samples dicts in the order of temps."""
    def one(k):
        x, v, L = starts[k]
        return eam_samples(x, v, L, fs, temps[k], n_samples=n_samples, **kw)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(len(temps))))
