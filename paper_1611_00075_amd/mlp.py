"""The learned descriptor-MLP potential: training on the GPU and the EAM
trajectories it learns from.

Every numeric step runs in libmd's kernels -- descriptors
(md_mlp_descriptors), site energies of the embedded-atom model
(md_forces_eam), trajectories (md_run), input moments (md_mlp_moments),
gradient and Adam step (md_mlp_train_step), inference (md_mlp_eval,
md_forces_mlp).  This module holds what surrounds them: parameter
initialisation, the data layout, epoch shuffles and the learning-rate
schedule.

Training reading (the configuration leaves it open): per-atom energy
mean-squared error, Adam with cosine-decayed learning rate, batches of 4,096
atom environments, FP32 master weights with a bfloat16 copy for the
network.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import inputs
from . import md as M
from .sim import Simulation

N_IN, N_HID, N_PARAM = M.MD_MLP_IN, M.MD_MLP_HID, M.MD_MLP_NPARAM
SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("w3", (N_HID,)), ("b3", ()))

# descriptor geometry of the Cu surrogate: 16 Gaussians centred 2.0 ... 5.0 A,
# width 0.2 A, cosine cutoff 5.0 A
RC, MU0, DMU, WIDTH = 5.0, 2.0, 0.2, 0.2


def bf16_bits(a) -> torch.Tensor:
    """bfloat16 bit patterns (int16, CPU) of float values, round to nearest
    even (torch's conversion)."""
    t = torch.as_tensor(np.asarray(a, np.float32))
    return t.to(torch.bfloat16).view(torch.int16)


def bf16_values(bits) -> np.ndarray:
    """float64 values of bfloat16 bit patterns."""
    b = torch.as_tensor(bits).cpu().to(torch.int16)
    return b.view(torch.bfloat16).to(torch.float64).numpy()


def init_params(seed: int, e_mean: float = 0.0, w3_scale: float = 0.01) -> np.ndarray:
    """FP32 parameter vector: weights N(0, 1/fan_in), zero biases, a small
    last layer and b3 at the mean target energy."""
    rng = inputs.rng_for(seed, "mlp-init")
    p = np.zeros(N_PARAM, np.float32)
    o = 0
    for name, shape in SHAPES:
        k = int(np.prod(shape)) if shape else 1
        if name in ("W1", "W2"):
            p[o:o + k] = rng.standard_normal(k) / math.sqrt(shape[1])
        elif name == "w3":
            p[o:o + k] = rng.standard_normal(k) * w3_scale
        elif name == "b3":
            p[o] = e_mean
        o += k
    return p


def spec(mean=None, inv_std=None, fp32_activations=False) -> M.MLP:
    """Descriptor geometry and normalisation; fp32_activations selects the
    network's FP32-activation form (otherwise BF16 activations)."""
    return M.mlp_spec(RC, MU0, DMU, WIDTH, mean, inv_std,
                      M.MD_MLP_ACT_FP32 if fp32_activations else M.MD_MLP_ACT_BF16)


def normalisation(G: torch.Tensor, tws=None):
    """(mean, inv_std) of the descriptor rows G (N, 16) from md_mlp_moments."""
    n = G.shape[0]
    tws = tws if tws is not None else torch.empty(M.md_mlp_workspace_bytes(0), dtype=torch.uint8, device=G.device)
    mom = torch.empty(2 * N_IN, dtype=torch.float64, device=G.device)
    M.md_mlp_moments(n, G, mom, tws)
    m = mom.cpu().numpy()
    std = m[N_IN:]
    return m[:N_IN], np.where(std > 0, 1.0 / np.maximum(std, 1e-30), 1.0)


@dataclasses.dataclass
class Potential:
    """A trained network: descriptor geometry + normalisation and the
    bfloat16 parameters on the device."""
    spec: M.MLP
    w: torch.Tensor            # int16 [N_PARAM]

    def params(self) -> np.ndarray:
        return bf16_values(self.w)


def predict(G: torch.Tensor, pot: Potential, dEdG: bool = False):
    """Per-atom energies (and dE/dG) of descriptor rows G (N, 16)."""
    n = G.shape[0]
    e = torch.empty(n, dtype=torch.float32, device=G.device)
    d = torch.empty((n, N_IN), dtype=torch.float32, device=G.device) if dEdG else None
    M.md_mlp_eval(n, G, pot.spec, pot.w, e, d)
    return (e, d) if dEdG else e


class Trainer:
    """Adam on the per-atom energy loss over descriptor rows G (N, 16) and
    targets (N,), both device float32."""

    def __init__(self, G: torch.Tensor, target: torch.Tensor, sp: M.MLP, master: np.ndarray, *,
                 batch: int = 4096, seed: int = 0):
        self.G, self.t = G.contiguous(), target.contiguous()
        self.n = int(G.shape[0])
        self.spec = sp
        self.batch = int(min(batch, self.n))
        d = G.device
        self.master = torch.tensor(np.asarray(master, np.float32), device=d)
        self.m1 = torch.zeros(N_PARAM, dtype=torch.float32, device=d)
        self.m2 = torch.zeros(N_PARAM, dtype=torch.float32, device=d)
        self.w = bf16_bits(master).to(d)
        self.tws = torch.empty(M.md_mlp_workspace_bytes(self.batch), dtype=torch.uint8, device=d)
        self.rng = inputs.rng_for(seed, "mlp-batches")
        self.step = 0
        self.history = []

    @property
    def potential(self) -> Potential:
        return Potential(self.spec, self.w)

    def steps_per_epoch(self) -> int:
        return (self.n + self.batch - 1) // self.batch

    def fit(self, epochs: int, lr: float = 1e-3, lr_min: float = 1e-5, beta1: float = 0.9,
            beta2: float = 0.999, eps: float = 1e-8):
        """Runs `epochs` passes over the data in shuffled batches, the learning
        rate decaying from lr to lr_min on a cosine.  Returns the mean batch
        loss of each epoch."""
        spe = self.steps_per_epoch()
        total = epochs * spe
        out = []
        adam = M.Adam(0.0, beta1, beta2, eps, 0)
        for _ in range(epochs):
            perm = torch.tensor(self.rng.permutation(self.n).astype(np.int32), device=self.G.device)
            losses = torch.zeros(spe, dtype=torch.float64, device=self.G.device)
            for b in range(spe):
                k = self.step
                adam.lr = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * min(k, total) / total))
                adam.step = k + 1
                lo = b * self.batch
                nb = min(self.batch, self.n - lo)
                M.md_mlp_train_step(nb, perm[lo:lo + nb], self.G, self.t, self.spec, adam, self.master,
                                    self.m1, self.m2, self.w, losses[b:b + 1], self.tws)
                self.step += 1
            out.append(float(losses.mean()))
        self.history += out
        return out


def rmse(pred: torch.Tensor, ref: torch.Tensor) -> float:
    d = (pred.double() - ref.double()).reshape(-1)
    return float(torch.sqrt(torch.mean(d * d)))


# ---------------------------------------------------------------------------
# training data from the embedded-atom model (the method's own trajectories)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Snapshots:
    """Snapshots of one trajectory, each in its own sorted atom order:
    G (S, n, 16) raw descriptors, e (S, n) site energies (device float32);
    optionally x (S, n, 3) positions and f (S, n, 3) EAM forces (host)."""
    T: float
    L: np.ndarray
    G: torch.Tensor
    e: torch.Tensor
    x: np.ndarray | None = None
    f: np.ndarray | None = None


def eam_simulation(system: inputs.System) -> Simulation:
    return Simulation(system.L, system.x, system.v, potential="eam", fs=inputs.FS_CU, skin=1.0, dt=1.0,
                      mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)


def equilibrate(sim: Simulation, T: float, steps: int, rescale_every: int):
    """Velocity-Verlet steps with the velocities rescaled to temperature T
    (K) after every `rescale_every` steps."""
    n = sim.n
    done = 0
    while done < steps:
        k = min(rescale_every, steps - done)
        sim.run(k)
        _, ke = sim.energies()
        Tn = 2.0 * ke / ((3 * n - 3) * inputs.KB_EV)
        if Tn > 0:
            sim.v.mul_(math.sqrt(T / Tn))
        done += k


def eam_trajectory(T: float, n_snap: int, *, seed: int, sample_every: int = 20, equil_steps: int = 2000,
                   rescale_every: int = 100, ncell: int = 4, keep_from: int | None = None) -> Snapshots:
    """One Cu trajectory at temperature T on the GPU: equilibration with
    velocity rescaling, then n_snap NVE snapshots every `sample_every` fs with
    their descriptors and site energies; positions and EAM forces of the
    snapshots from index keep_from on are copied to the host."""
    s = inputs.eam_cu(ncell=ncell, T=T, seed=seed)
    sim = eam_simulation(s)
    equilibrate(sim, T, equil_steps, rescale_every)
    n = sim.n
    sp = spec()
    d = sim.dev
    G = torch.empty((n_snap, n, N_IN), dtype=torch.float32, device=d)
    E = torch.empty((n_snap, n), dtype=torch.float32, device=d)
    xs, fs = [], []
    for k in range(n_snap):
        sim.run(sample_every)
        sim.descriptors(sp, out=G[k])
        sim.compute_forces(site=True)
        E[k].copy_(sim.e_atom[:n])
        if keep_from is not None and k >= keep_from:
            xs.append(sim.x[:, :n].T.cpu().numpy())
            fs.append(sim.f[:, :n].T.double().cpu().numpy())
    return Snapshots(T, s.L.copy(), G, E, np.stack(xs) if xs else None, np.stack(fs) if fs else None)


def training_temperatures(k: int = 16, lo: float = 300.0, hi: float = 1200.0) -> np.ndarray:
    return np.linspace(lo, hi, k)


def split(snaps: list[Snapshots], blocks: int = 10, held: int = 9):
    """Whole blocks of consecutive snapshots held out: every trajectory is cut
    into `blocks` blocks and block `held` goes to the test set.  Returns
    (G_train, e_train, G_test, e_test) flattened to atom rows."""
    tr_g, tr_e, te_g, te_e = [], [], [], []
    for s in snaps:
        S = s.G.shape[0]
        edges = np.linspace(0, S, blocks + 1).astype(int)
        for b in range(blocks):
            a, z = edges[b], edges[b + 1]
            (te_g if b == held else tr_g).append(s.G[a:z].reshape(-1, N_IN))
            (te_e if b == held else tr_e).append(s.e[a:z].reshape(-1))
    return torch.cat(tr_g), torch.cat(tr_e), torch.cat(te_g), torch.cat(te_e)


def mlp_forces(pot: Potential, L, x, skin: float = 1.0) -> np.ndarray:
    """MLP forces (n, 3) of positions x (n, 3) in their given order."""
    n = len(x)
    sim = Simulation(L, x, np.zeros_like(x), potential="mlp", mlp=pot.spec, mlp_w=pot.w, skin=skin, dt=1.0,
                     mass=inputs.CU_MASS_AMU, force_to_accel=1.0 / inputs.AMU_A2_FS2_IN_EV)
    assert sim.n == n
    return sim.forces().astype(np.float64)
