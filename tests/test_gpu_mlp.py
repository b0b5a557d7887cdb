"""GPU parity of the learned descriptor-MLP potential (descriptors, network,
forces, training) against the FP64 oracle, through the C ABI.

Bars:
  - descriptors: FP32 sums of the 16 Gaussians, per atom within 1e-5 of the
    atom's largest component;
  - network, gradient and forces: the GPU rounds to bfloat16 where the
    oracle's BF16 mode does, so the two differ only by FP32 vs FP64
    arithmetic and by the rare rounding decisions that FP32 and FP64 values
    take differently.  Inputs are chosen so that the descriptor rounding is
    exact (FP32 descriptors given to both, mean 0 and power-of-two scales).
    At least 99% of atoms agree to 2e-5 (relative to the size of the
    quantity) and no atom differs by more than the whole BF16 rounding
    effect (the oracle's BF16 result minus its FP64 result);
  - forces from given dE/dG (pass 2 alone): 1e-5 normwise, as the pair
    kernels;
  - full forces (both passes, descriptors computed on each side): the GPU
    is closer to the BF16 oracle than half the BF16 rounding effect.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_00075_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

CU = inputs.FS_CU


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_00075_amd import md
    md.lib()
    return md


@pytest.fixture(scope="module")
def om(orc):
    from oracle import mlp
    return mlp


def _params(om, seed, scale=1.0):
    """Random parameters rounded to bfloat16: (float64 values, int16 bits)."""
    from paper_1611_00075_amd import mlp as P
    rng = np.random.default_rng(seed)
    p = np.zeros(om.N_PARAM)
    o = 0
    for name, shape in P.SHAPES:
        k = int(np.prod(shape)) if shape else 1
        fan = shape[1] if len(shape) == 2 else 1
        std = scale / np.sqrt(fan) if len(shape) == 2 else 0.3 * scale
        p[o:o + k] = rng.standard_normal(k) * std
        o += k
    bits = P.bf16_bits(p)
    return P.bf16_values(bits), bits


def _system(seed, ncell=6, drop=0, sigma=0.12):
    s = inputs.jitter(inputs.eam_cu(ncell=ncell, T=600.0, seed=seed), sigma, seed)
    x = s.x
    if drop:
        x = np.delete(x, np.random.default_rng(seed).choice(len(x), drop, replace=False), axis=0)
    return x, s.L


def _mlp_sim(M, x, L, spec, w):
    from paper_1611_00075_amd.sim import Simulation
    return Simulation(L, x, np.zeros_like(x), potential="mlp", mlp=spec, mlp_w=w, skin=1.0, dt=1.0,
                      mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)


def _agree(gpu, ref, scale, full_effect, tight=2e-5, frac=0.99):
    """Most rows within tight * scale; every row within the BF16 effect."""
    d = np.abs(gpu - ref)
    d = d.reshape(len(d), -1).max(axis=1)
    s = np.asarray(scale).reshape(-1)
    ok = d <= tight * s
    assert ok.mean() >= frac, (ok.mean(), d.max())
    fe = np.abs(full_effect).reshape(len(d), -1).max(axis=1)
    assert np.all(d <= np.maximum(fe, tight * s)), (d.max(), fe.max())


def _spec_exact(M, P, k=-2):
    """Descriptor normalisation whose FP32 arithmetic is exact: mean 0,
    inv_std a power of two."""
    return P.spec(np.zeros(16), np.full(16, 2.0 ** k))


# ------------------------------------------------------------------ descriptors
@pytest.mark.parametrize("ncell,drop,seed", [(6, 0, 1), (5, 7, 2), (4, 0, 3)])
def test_descriptors_vs_oracle(M, orc, om, ncell, drop, seed):
    from paper_1611_00075_amd import mlp as P
    x, L = _system(seed, ncell, drop)
    x = orc.wrap(x, L)
    _, bits = _params(om, 1)
    sim = _mlp_sim(M, x, L, P.spec(), bits.cuda())
    Gs = sim.descriptors(P.spec()).cpu().numpy()
    ids = sim.ids.cpu().numpy()
    G = np.empty_like(Gs, dtype=np.float64)
    G[ids] = Gs
    off, idx = orc.neighbors_brute(x, L, 6.0)
    Go = om.descriptors(x, L, off, idx, om.Spec())
    err = np.abs(G - Go).max(axis=1) / np.abs(Go).max(axis=1)
    print(f"descriptor error max {err.max():.2e} mean {err.mean():.2e}")
    assert err.max() < 1e-5


def test_descriptors_perfect_lattice_uniform(M, om):
    from paper_1611_00075_amd import mlp as P
    s = inputs.eam_cu(ncell=5)
    _, bits = _params(om, 1)
    sim = _mlp_sim(M, s.x, s.L, P.spec(), bits.cuda())
    G = sim.descriptors(P.spec()).cpu().numpy().astype(np.float64)
    # every site sees the same shells
    assert np.abs(G - G[0]).max() <= 1e-5 * np.abs(G[0]).max()


# ------------------------------------------------------------------ network
@pytest.mark.parametrize("n", [1000, 16, 1, 0])
def test_network_vs_oracle(M, orc, om, n):
    from paper_1611_00075_amd import mlp as P
    x, L = _system(5, 7)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G32 = om.descriptors(x, L, off, idx, om.Spec())[:n].astype(np.float32)
    sp = _spec_exact(M, P)
    osp = om.Spec(mean=np.zeros(16), inv_std=np.full(16, 0.25))
    p, bits = _params(om, 7)
    Gd = torch.tensor(G32, device="cuda").reshape(-1, 16) if n else torch.zeros((1, 16), device="cuda")
    e = torch.full((max(n, 1),), np.nan, dtype=torch.float32, device="cuda")
    d = torch.zeros((max(n, 1), 16), dtype=torch.float32, device="cuda")
    M.md_mlp_eval(n, Gd, sp, bits.cuda(), e, d)
    if n == 0:
        assert torch.isnan(e).all()
        return
    eg, dg = e.cpu().numpy().astype(np.float64), d.cpu().numpy().astype(np.float64)
    eo, do = om.energy(G32.astype(np.float64), osp, p, bf16=True)
    e64, d64 = om.energy(G32.astype(np.float64), osp, p, bf16=False)
    _agree(eg, eo, 1.0 + np.abs(eo), eo - e64)
    _agree(dg, do, np.abs(do).max(axis=1) + 1e-3, do - d64)


# ------------------------------------------------------------------ forces
def test_forces_from_given_dEdG_vs_oracle(M, orc, om):
    """Pass 2 alone (MD_MLP_REUSE): both sides take the same dE/dG."""
    from paper_1611_00075_amd import mlp as P
    x, L = _system(8, 6, drop=3)
    x = orc.wrap(x, L)
    n = len(x)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G = om.descriptors(x, L, off, idx, om.Spec())
    osp = om.Spec(mean=G.mean(0), inv_std=1.0 / G.std(0))
    p, bits = _params(om, 9)
    _, dEdG = om.energy(G, osp, p, bf16=True)
    dEdG = dEdG.astype(np.float32).astype(np.float64)
    fo, wo = om.forces(x, L, off, idx, osp, dEdG)
    sim = _mlp_sim(M, x, L, P.spec(osp.mean, osp.inv_std), bits.cuda())
    ids = sim.ids.cpu().numpy()
    sim.dEdG[:n] = torch.tensor(dEdG[ids].astype(np.float32), device="cuda")
    ev = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.md_forces_mlp(L, n, sim.xs, sim.row_cap, sim.idx, sim.count, sim.mlp, None, sim.dEdG, None, None, None, sim.f,
                    ev, M.MD_MLP_REUSE | M.MD_ENERGY, sim.ws)
    fg = sim.forces()
    err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    print(f"MLP pass-2 force error (normwise) {err:.3e}")
    assert err < 1e-5
    assert np.abs(fg - fo).max() < 1e-4 * np.sqrt(np.mean(fo * fo))
    w = ev.cpu().numpy()[2:]
    assert np.allclose(w[:3], wo[:3], rtol=1e-5)
    assert np.allclose(w[3:], wo[3:], atol=1e-5 * np.abs(wo[:3]).max())
    assert ev[0].item() == 0.0


def test_forces_full_vs_oracle(M, orc, om):
    from paper_1611_00075_amd import mlp as P
    x, L = _system(10, 6, drop=5, sigma=0.15)
    x = orc.wrap(x, L)
    n = len(x)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G = om.descriptors(x, L, off, idx, om.Spec())
    mean = G.mean(0).astype(np.float32).astype(np.float64)
    inv = (1.0 / G.std(0)).astype(np.float32).astype(np.float64)
    osp = om.Spec(mean=mean, inv_std=inv)
    p, bits = _params(om, 11)
    eo, do = om.energy(G, osp, p, bf16=True)
    e64, d64 = om.energy(G, osp, p, bf16=False)
    fo, wo = om.forces(x, L, off, idx, osp, do)
    f64, _ = om.forces(x, L, off, idx, osp, d64)
    sim = _mlp_sim(M, x, L, P.spec(mean, inv), bits.cuda())
    sim.compute_forces(energy=True, site=True)
    fg = sim.forces()
    eg = sim.by_id(sim.e_atom).astype(np.float64)
    effect = np.linalg.norm(fo - f64)
    err = np.linalg.norm(fg - fo)
    print(f"MLP forces: |gpu - bf16 oracle| {err / np.linalg.norm(fo):.2e}, "
          f"|gpu - fp64 oracle| {np.linalg.norm(fg - f64) / np.linalg.norm(f64):.2e}, "
          f"BF16 effect {effect / np.linalg.norm(fo):.2e} (normwise)")
    assert err < 0.5 * effect
    assert np.linalg.norm(eg - eo) < 0.5 * np.linalg.norm(eo - e64)
    ev = sim.ev.cpu().numpy()
    assert ev[0] == pytest.approx(float(np.sum(eg.astype(np.float32).astype(np.float64))), rel=1e-6)
    assert abs(ev[0] - eo.sum()) < 0.5 * abs(eo.sum() - e64.sum()) + 1e-4 * n


def test_compact_list_holds_the_pairs_within_rc(M, orc, om):
    """Pass 1's compact rows are exactly the neighbours closer than rc (as
    sets, in input ids); pass 2 on the compact list equals pass 2 on the
    full list bit for bit."""
    from paper_1611_00075_amd import mlp as P
    x, L = _system(21, 5, drop=2, sigma=0.2)
    x = orc.wrap(x, L)
    n = len(x)
    _, bits = _params(om, 22)
    sim = _mlp_sim(M, x, L, P.spec(), bits.cuda())
    sim.compute_forces()
    ids = sim.ids.cpu().numpy()
    rows = M.ell_rows(n, sim.row_cap, sim.idx_in, sim.cnt_in)
    off, idx = orc.neighbors_brute(x, L, 5.0)
    for k in range(n):
        got = np.sort(ids[rows[k]])
        want = idx[off[ids[k]]:off[ids[k] + 1]]
        assert np.array_equal(got, want), k
    f_full = torch.zeros_like(sim.f)
    f_comp = torch.zeros_like(sim.f)
    for f, li, lc in ((f_full, sim.idx, sim.count), (f_comp, sim.idx_in, sim.cnt_in)):
        M.md_forces_mlp(L, n, sim.xs, sim.row_cap, li, lc, sim.mlp, None, sim.dEdG, None, None, None, f, sim.ev,
                        M.MD_MLP_REUSE, sim.ws)
    assert torch.equal(f_comp[:, :n], sim.f[:, :n])
    assert torch.allclose(f_full[:, :n], f_comp[:, :n], rtol=1e-5, atol=1e-6)


def test_forces_deterministic_and_md_run_path(M, orc, om):
    from paper_1611_00075_amd import mlp as P
    x, L = _system(12, 5)
    p, bits = _params(om, 13, scale=0.5)
    out = []
    for _ in range(2):
        sim = _mlp_sim(M, x, L, P.spec(), bits.cuda())
        sim.compute_forces(energy=True)
        out.append((sim.forces(), sim.ev.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


# ------------------------------------------------------------------ training
@pytest.mark.parametrize("batch,use_sel", [(1000, True), (4096, False), (37, True)])
def test_gradient_vs_oracle(M, orc, om, batch, use_sel):
    from paper_1611_00075_amd import mlp as P
    x, L = _system(14, 11)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G32 = om.descriptors(x, L, off, idx, om.Spec()).astype(np.float32)
    rng = np.random.default_rng(15)
    target = (-3.5 + 0.05 * rng.standard_normal(len(G32))).astype(np.float32)
    sel = rng.permutation(len(G32))[:batch].astype(np.int32) if use_sel else np.arange(batch, dtype=np.int32)
    sp = _spec_exact(M, P)
    osp = om.Spec(mean=np.zeros(16), inv_std=np.full(16, 0.25))
    p, bits = _params(om, 16)
    tws = torch.empty(M.md_mlp_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
    grad = torch.zeros(om.N_PARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    M.md_mlp_grad(batch, torch.tensor(sel, device="cuda") if use_sel else None, torch.tensor(G32, device="cuda"),
                  torch.tensor(target, device="cuda"), sp, bits.cuda(), grad, loss, tws)
    g = grad.cpu().numpy().astype(np.float64)
    lo, go = om.loss_grad(G32[sel].astype(np.float64), target[sel].astype(np.float64), osp, p, bf16=True)
    assert loss.item() == pytest.approx(lo, rel=1e-5)
    o = 0
    from paper_1611_00075_amd.mlp import SHAPES
    for name, shape in SHAPES:
        k = int(np.prod(shape)) if shape else 1
        a, b = g[o:o + k], go[o:o + k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(f"grad {name}: rel err {rel:.2e}")
        assert rel < 1e-5, name
        o += k


def test_adam_steps_vs_oracle(M, orc, om):
    from paper_1611_00075_amd import mlp as P
    x, L = _system(17, 6)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G32 = om.descriptors(x, L, off, idx, om.Spec()).astype(np.float32)
    n = len(G32)
    target = (-3.5 + 0.05 * np.random.default_rng(18).standard_normal(n)).astype(np.float32)
    sp = _spec_exact(M, P)
    osp = om.Spec(mean=np.zeros(16), inv_std=np.full(16, 0.25))
    p, bits = _params(om, 19)
    master = torch.tensor(p.astype(np.float32), device="cuda")
    m1 = torch.zeros_like(master)
    m2 = torch.zeros_like(master)
    w = bits.cuda()
    tws = torch.empty(M.md_mlp_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    Gd, td = torch.tensor(G32, device="cuda"), torch.tensor(target, device="cuda")
    lr = 1e-3
    po, a1, a2 = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for step in (1, 2):
        before = master.cpu().numpy().astype(np.float64)
        M.md_mlp_train_step(n, None, Gd, td, sp, M.Adam(lr, 0.9, 0.999, 1e-8, step), master, m1, m2, w, None, tws)
        _, go = om.loss_grad(G32.astype(np.float64), target.astype(np.float64), osp,
                             P.bf16_values(P.bf16_bits(po)), bf16=True)
        po_new, a1, a2 = om.adam(po, go, a1, a2, step, lr)
        dg = master.cpu().numpy().astype(np.float64) - before
        do = po_new - po
        stable = np.abs(go) > 1e-2 * np.abs(go).max()
        assert np.abs(dg - do)[stable].max() < 2e-2 * lr, step
        po = master.cpu().numpy().astype(np.float64)   # continue both from the GPU state
        assert np.array_equal(w.cpu().numpy(), P.bf16_bits(master.cpu().numpy()).numpy())


def test_moments_match_numpy(M):
    from paper_1611_00075_amd import mlp as P
    rng = np.random.default_rng(20)
    G = (rng.standard_normal((100_003, 16)) * np.arange(1, 17) + 5.0).astype(np.float32)
    mean, inv = P.normalisation(torch.tensor(G, device="cuda"))
    assert np.allclose(mean, G.astype(np.float64).mean(0), rtol=1e-12)
    assert np.allclose(1.0 / inv, G.astype(np.float64).std(0), rtol=1e-9)


def test_training_abi_rejects_bad_arguments(M):
    from paper_1611_00075_amd import mlp as P
    sp = P.spec()
    bad = P.spec()
    bad.width = 0.0
    G = torch.zeros((64, 16), device="cuda")
    e = torch.zeros(64, device="cuda")
    w = torch.zeros(om_n := M.MD_MLP_NPARAM, dtype=torch.int16, device="cuda")
    with pytest.raises(M.MDError):
        M.md_mlp_eval(64, G, bad, w, e)
    tws = torch.empty(16, dtype=torch.uint8, device="cuda")
    g = torch.zeros(om_n, dtype=torch.float32, device="cuda")
    with pytest.raises(M.MDError) as ex:
        M.md_mlp_grad(64, None, G, e, sp, w, g, None, tws)
    assert ex.value.code == M.MD_ERR_WORKSPACE


# ------------------------------------------------------------------ FP32-activation form
def test_network_fp32_activations_vs_oracle(M, orc, om):
    """The FP32-activation form (each activation split exactly into three
    bfloat16 terms on the matrix cores) against the oracle's FP64 network
    with the same bfloat16 parameters: every atom within FP32 rounding, far
    inside the BF16 rounding effect."""
    from paper_1611_00075_amd import mlp as P
    x, L = _system(5, 7)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G32 = om.descriptors(x, L, off, idx, om.Spec()).astype(np.float32)
    n = len(G32)
    sp = P.spec(np.zeros(16), np.full(16, 0.25), fp32_activations=True)
    osp = om.Spec(mean=np.zeros(16), inv_std=np.full(16, 0.25))
    p, bits = _params(om, 7)
    e = torch.zeros(n, dtype=torch.float32, device="cuda")
    d = torch.zeros((n, 16), dtype=torch.float32, device="cuda")
    M.md_mlp_eval(n, torch.tensor(G32, device="cuda"), sp, bits.cuda(), e, d)
    eg, dg = e.cpu().numpy().astype(np.float64), d.cpu().numpy().astype(np.float64)
    e64, d64 = om.energy(G32.astype(np.float64), osp, p, bf16=False)
    e16, d16 = om.energy(G32.astype(np.float64), osp, p, bf16=True)
    de = np.abs(eg - e64) / (1.0 + np.abs(e64))
    dd = np.abs(dg - d64).max(axis=1) / (np.abs(d64).max(axis=1) + 1e-3)
    print(f"FP32-activation network: energy <= {de.max():.2e}, dE/dG <= {dd.max():.2e} "
          f"(BF16 effect {np.abs(e16 - e64).max():.2e}, {np.abs(d16 - d64).max():.2e})")
    assert de.max() < 2e-6 and dd.max() < 2e-5
    assert np.abs(eg - e64).max() < 0.02 * np.abs(e16 - e64).max()


def test_forces_fp32_activations_vs_oracle(M, orc, om):
    """Full forces of the FP32-activation form against the oracle's FP64
    forces (FP64 network, same bfloat16 parameters): FP32 accuracy, a small
    fraction of the BF16 effect."""
    from paper_1611_00075_amd import mlp as P
    x, L = _system(10, 6, drop=5, sigma=0.15)
    x = orc.wrap(x, L)
    off, idx = orc.neighbors_brute(x, L, 6.0)
    G = om.descriptors(x, L, off, idx, om.Spec())
    mean = G.mean(0).astype(np.float32).astype(np.float64)
    inv = (1.0 / G.std(0)).astype(np.float32).astype(np.float64)
    osp = om.Spec(mean=mean, inv_std=inv)
    p, bits = _params(om, 11)
    _, d16 = om.energy(G, osp, p, bf16=True)
    e64, d64 = om.energy(G, osp, p, bf16=False)
    f16, _ = om.forces(x, L, off, idx, osp, d16)
    f64, _ = om.forces(x, L, off, idx, osp, d64)
    sim = _mlp_sim(M, x, L, P.spec(mean, inv, fp32_activations=True), bits.cuda())
    sim.compute_forces(energy=True, site=True)
    fg = sim.forces()
    eg = sim.by_id(sim.e_atom).astype(np.float64)
    err = np.linalg.norm(fg - f64) / np.linalg.norm(f64)
    effect = np.linalg.norm(f16 - f64) / np.linalg.norm(f64)
    print(f"MLP FP32-activation forces: |gpu - fp64 oracle| {err:.2e} normwise (BF16 effect {effect:.2e})")
    assert err < 2e-5 and err < 0.05 * effect
    assert np.abs(eg - e64).max() < 1e-5 * (1.0 + np.abs(e64).max())


def _oracle_mlp_nve(orc, om, x, v, L, spec, p, steps, every, dt=1.0):
    """Total energy per atom every `every` velocity-Verlet steps with the
    oracle's FP64 network and forces (lists rebuilt every step)."""
    m, k = inputs.CU_MASS_AMU, 1.0 / inputs.AMU_A2_FS2_IN_EV
    x, v = x.copy(), v.copy()

    def force(x):
        w = orc.wrap(x, L)
        off, idx = orc.neighbors_brute(w, L, 6.0)
        G = om.descriptors(w, L, off, idx, om.Spec())
        e, d = om.energy(G, spec, p, bf16=False)
        f, _ = om.forces(w, L, off, idx, spec, d)
        return f, e.sum()

    f, ep = force(x)
    out = []
    for step in range(steps + 1):
        if step % every == 0:
            out.append((ep + 0.5 * m * (v ** 2).sum() / k) / len(x))
        if step == steps:
            break
        v += 0.5 * dt * f * k / m
        x += dt * v
        f, ep = force(x)
        v += 0.5 * dt * f * k / m
    return np.array(out)


def test_md_run_fp32_activations_follows_the_oracle_energy_trace(M, orc, om):
    """NVE through the native driver with the FP32-activation form (rebuilds
    included): the total energy every 40 fs of a 200 fs run follows the
    trajectory of the oracle's FP64 network with the same bfloat16
    parameters, within 1e-6 eV per atom (measured 8e-8; the oracle's own
    Verlet fluctuation is 1e-5)."""
    from paper_1611_00075_amd import mlp as P
    s = inputs.eam_cu(ncell=4, T=600.0, seed=47)
    x = orc.wrap(s.x, s.L)
    # normalisation from thermally displaced copies of the lattice, as a
    # training set would give it
    xj = orc.wrap(inputs.jitter(s, 0.1, 48).x, s.L)
    off, idx = orc.neighbors_brute(xj, s.L, 6.0)
    G = om.descriptors(xj, s.L, off, idx, om.Spec())
    mean = G.mean(0).astype(np.float32).astype(np.float64)
    inv = (1.0 / G.std(0)).astype(np.float32).astype(np.float64)
    p, bits = _params(om, 13, scale=0.3)
    from paper_1611_00075_amd.sim import Simulation
    sim = Simulation(s.L, x, s.v, potential="mlp", mlp=P.spec(mean, inv, fp32_activations=True),
                     mlp_w=bits.cuda(), skin=1.0, dt=1.0, mass=inputs.CU_MASS_AMU,
                     force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    e = []
    for _ in range(5):
        ep, ek = sim.energies()
        e.append(ep + ek)
        sim.run(40)
    ep, ek = sim.energies()
    e.append(ep + ek)
    e = np.array(e) / s.n
    eo = _oracle_mlp_nve(orc, om, x, s.v, s.L, om.Spec(mean=mean, inv_std=inv), p, 200, 40)
    print(f"MLP FP32-activation NVE 200 fs: GPU E/N {e}, |GPU - oracle| max {np.abs(e - eo).max():.2e} eV, "
          f"oracle drift {eo.max() - eo.min():.2e} eV, builds {sim.builds}")
    assert np.abs(e - eo).max() < 1e-6
    assert sim.builds >= 1
