"""Pins for the oracle of the learned descriptor-MLP potential.

What fixes each part, independently of the oracle's own code:
  - bfloat16 rounding: torch's CPU float32 -> bfloat16 conversion (round to
    nearest even);
  - the pair basis: closed forms on a dimer at special distances
    (cos(3 pi / 5) = (1 - sqrt 5) / 4, exp(-n^2 / 2) off-centre);
  - the neighbour sum: fcc shell counts (12, 6, 24 within 5 A at 3.615 A);
  - the network, its input gradient and its weight gradient, with and
    without the BF16 rounding points: the same network built from torch
    operations and differentiated by torch's autograd;
  - forces and virial: central finite differences of the FP64 energy in
    the positions and in a uniaxial strain; zero net force;
  - Adam: the bias-corrected first step, lr * g / (|g| + eps);
  - ridge regression: numpy's least-squares solver as lambda -> 0;
  - training trajectories: per-atom energies re-derived from the returned
    snapshots by the EAM oracle, and the sampled temperature.
"""
import math

import numpy as np
import pytest
import torch

from paper_1611_00075_amd import inputs

CU = inputs.FS_CU


@pytest.fixture(scope="module")
def mlp(orc):
    from oracle import mlp as m
    return m


def _rand_params(mlp, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.N_PARAM)
    o = 0
    for rows, cols in ((64, 16), (64, 1), (64, 64), (64, 1), (1, 64), (1, 1)):
        k = rows * cols
        fan = cols if cols > 1 else 1
        p[o:o + k] = rng.standard_normal(k) * scale / math.sqrt(fan) * (0.3 if cols == 1 else 1.0)
        o += k
    return p


def _snapshot(seed=3, ncell=4, sigma=0.12):
    s = inputs.eam_cu(ncell=ncell, T=600.0, seed=seed)
    s = inputs.jitter(s, sigma, seed)
    return s


# ---------------------------------------------------------------- rounding
def test_bf16_round_matches_torch(mlp):
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.standard_normal(400) * 10.0 ** rng.integers(-30, 30, 400),
        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -(1.0 + 2 ** -8), 0.0, -0.0,
         1e-40, -3e-39, 3.3e38, 1.0 + 2 ** -8 + 2 ** -20],
    ])
    want = torch.tensor(vals, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64)
    got = np.array([mlp.bf16_round(v) for v in vals])
    assert np.array_equal(got, want.numpy())


# ---------------------------------------------------------------- descriptors
def _dimer(mlp, r):
    L = np.full(3, 30.0)
    x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    off = np.array([0, 1, 2], np.int64)
    idx = np.array([1, 0], np.int32)
    return mlp.descriptors(x, L, off, idx, mlp.Spec())


def test_descriptor_dimer_closed_forms(mlp):
    k = np.arange(16)
    # r = 3.0 = mu_5: fc = (1 + cos(3 pi / 5)) / 2 = (5 - sqrt 5) / 8
    G = _dimer(mlp, 3.0)
    want = np.exp(-0.5 * (k - 5.0) ** 2) * (5.0 - math.sqrt(5.0)) / 8.0
    assert np.allclose(G[0], want, rtol=1e-13, atol=1e-300)
    assert np.array_equal(G[0], G[1])
    # r = 2.5 = rc / 2: fc = 1/2, centres sit 2.5 widths away from k = 0
    G = _dimer(mlp, 2.5)
    assert np.allclose(G[0], 0.5 * np.exp(-0.5 * (k - 2.5) ** 2), rtol=1e-13, atol=1e-300)
    # strict cutoff
    assert np.all(_dimer(mlp, 5.0) == 0.0)
    assert np.all(_dimer(mlp, 4.999999) > 0.0)


def test_descriptor_fcc_shells(mlp, orc):
    a = inputs.CU_A0
    x = inputs.fcc_sites(4, 4, 4, a)
    L = np.full(3, 4 * a)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G = mlp.descriptors(x, L, off, idx, mlp.Spec())
    # shells within 5 A: 12 at a/sqrt2, 6 at a, 24 at a sqrt(3/2) (a sqrt2 = 5.11 A is out)
    one = lambda r: _dimer(mlp, r)[0]  # noqa: E731
    want = 12 * one(a / math.sqrt(2)) + 6 * one(a) + 24 * one(a * math.sqrt(1.5))
    assert np.allclose(G, want[None, :], rtol=1e-12)


# ---------------------------------------------------------------- network vs torch
class _Round(torch.autograd.Function):
    """Forward: round to bfloat16; backward: identity."""
    @staticmethod
    def forward(ctx, t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


class _GradRound(torch.autograd.Function):
    """Forward: identity; backward: round the incoming gradient to bfloat16."""
    @staticmethod
    def forward(ctx, t):
        return t.clone()

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _torch_energy(mlp, G, spec, params, bf16):
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in mlp.unpack(params).items()}
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    r = _Round.apply if bf16 else (lambda t: t)
    gr = _GradRound.apply if bf16 else (lambda t: t)
    x = r((Gt - torch.tensor(spec.mean)) * torch.tensor(spec.inv_std))
    a1 = gr(x @ P["W1"].T) + P["b1"]
    h1 = r(torch.nn.functional.silu(a1))
    a2 = gr(h1 @ P["W2"].T) + P["b2"]
    E = torch.nn.functional.silu(a2) @ P["w3"] + P["b3"]
    return E, Gt, P


def _spec_for(mlp, G):
    return mlp.Spec(mean=G.mean(axis=0), inv_std=1.0 / G.std(axis=0))


@pytest.mark.parametrize("bf16", [False, True])
def test_network_and_input_gradient_match_torch(mlp, orc, bf16):
    s = _snapshot()
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_cells(x, s.L, 6.0)
    G = mlp.descriptors(x, s.L, off, idx, mlp.Spec())
    spec = _spec_for(mlp, G)
    params = _rand_params(mlp, 11)
    if bf16:
        params = np.array([mlp.bf16_round(v) for v in params])
    e, dEdG = mlp.energy(G, spec, params, bf16=bf16)
    Et, Gt, _ = _torch_energy(mlp, G, spec, params, bf16)
    Et.sum().backward()
    assert np.allclose(e, Et.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(dEdG, Gt.grad.numpy(), rtol=1e-9, atol=1e-12)
    if bf16:  # the rounding points are real: the FP64 network differs
        e64, _ = mlp.energy(G, spec, params, bf16=False)
        assert np.max(np.abs(e64 - e)) > 1e-5


@pytest.mark.parametrize("bf16", [False, True])
def test_weight_gradient_matches_torch(mlp, orc, bf16):
    s = _snapshot(seed=4)
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_cells(x, s.L, 6.0)
    G = mlp.descriptors(x, s.L, off, idx, mlp.Spec())
    spec = _spec_for(mlp, G)
    params = _rand_params(mlp, 12)
    rng = np.random.default_rng(5)
    target = rng.normal(-3.5, 0.05, len(G))
    loss, g = mlp.loss_grad(G, target, spec, params, bf16=bf16)
    Et, _, P = _torch_energy(mlp, G, spec, params, bf16)
    lt = torch.mean((Et - torch.tensor(target)) ** 2)
    lt.backward()
    gt = np.concatenate([P[k].grad.reshape(-1).numpy() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    assert np.allclose(g, gt, rtol=1e-8, atol=1e-14 * np.max(np.abs(gt)))


def test_weight_gradient_finite_differences(mlp, orc):
    s = _snapshot(seed=6)
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_cells(x, s.L, 6.0)
    G = mlp.descriptors(x, s.L, off, idx, mlp.Spec())
    spec = _spec_for(mlp, G)
    params = _rand_params(mlp, 13)
    target = np.random.default_rng(7).normal(-3.5, 0.05, len(G))
    _, g = mlp.loss_grad(G, target, spec, params)
    h = 1e-6
    for k in [0, 17, 1023, 1024 + 5, 1088 + 4095, 5184 + 3, 5248 + 63, 5312]:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss_grad(G, target, spec, pp, grad=False)[0]
              - mlp.loss_grad(G, target, spec, pm, grad=False)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------- forces
def test_forces_finite_differences_and_virial(mlp, orc):
    s = _snapshot(seed=8)
    x = orc.wrap(s.x, s.L)
    off, idx = orc.neighbors_cells(x, s.L, 6.0)
    G = mlp.descriptors(x, s.L, off, idx, mlp.Spec())
    spec = _spec_for(mlp, G)
    params = _rand_params(mlp, 14)
    _, dEdG = mlp.energy(G, spec, params)
    f, w6 = mlp.forces(x, s.L, off, idx, spec, dEdG)
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * np.abs(f).max() * len(f)
    h = 1e-5
    rng = np.random.default_rng(9)
    fmax = np.abs(f).max()
    for i in rng.choice(len(x), 6, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(mlp.potential_energy(xp, s.L, off, idx, spec, params)
                   - mlp.potential_energy(xm, s.L, off, idx, spec, params)) / (2 * h)
            assert fd == pytest.approx(f[i, a], abs=1e-7 * fmax)
    # uniaxial strain: W_aa = -dE/d(eps_aa)
    eps = 1e-6
    for a in range(3):
        sc = np.ones(3)
        sc[a] = 1 + eps
        ep = mlp.potential_energy(x * sc, s.L * sc, off, idx, spec, params)
        sc[a] = 1 - eps
        em = mlp.potential_energy(x * sc, s.L * sc, off, idx, spec, params)
        assert -(ep - em) / (2 * eps) == pytest.approx(w6[a], rel=1e-6, abs=1e-7 * abs(w6[:3]).max())


# ---------------------------------------------------------------- optimiser / baseline
def test_adam_first_step_closed_form(mlp):
    g = np.array([1e-3, -2.0, 5e-9, 0.0])
    p = np.ones(4)
    new, m1, m2 = mlp.adam(p, g, np.zeros(4), np.zeros(4), step=1, lr=1e-2, eps=1e-8)
    assert np.allclose(new, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_ridge_matches_least_squares(mlp):
    rng = np.random.default_rng(10)
    X = rng.standard_normal((500, 16))
    y = X @ rng.standard_normal(16) + 0.3 + 0.01 * rng.standard_normal(500)
    u, b = mlp.ridge_fit(X, y, lam=0.0)
    A = np.concatenate([X, np.ones((500, 1))], axis=1)
    sol = np.linalg.lstsq(A, y, rcond=None)[0]
    assert np.allclose(u, sol[:16], rtol=1e-10, atol=1e-12)
    assert b == pytest.approx(sol[16], rel=1e-10)


# ---------------------------------------------------------------- training data
def test_eam_samples_labels_and_temperature(mlp, orc):
    s = inputs.eam_cu(ncell=4, T=900.0, seed=21)
    r = mlp.eam_samples(s.x, s.v, s.L, CU, 900.0, n_samples=8, equil_steps=300,
                        sample_every=20)
    assert r["pos"].shape == (8, 256, 3)
    for k in (0, 7):
        off, idx = orc.neighbors_brute(r["pos"][k], s.L, 5.4)
        e = orc.forces_eam(r["pos"][k], s.L, off, idx, CU)
        assert np.array_equal(e["e_atom"], r["e_atom"][k])
        assert np.array_equal(e["f"], r["forces"][k])
    # equilibrated at 900 K: the potential energy per atom rises above the
    # lattice value by about (3/2) kB T (harmonic equipartition)
    rise = r["e_atom"].mean() - (-3.54)
    assert 0.5 * 1.5 * inputs.KB_EV * 900 < rise < 1.5 * 1.5 * inputs.KB_EV * 900
    # snapshots differ (the trajectory moves between samples)
    assert np.abs(r["pos"][1] - r["pos"][0]).max() > 1e-3
