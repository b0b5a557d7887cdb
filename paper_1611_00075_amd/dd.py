"""Domain-decomposed system on one GPU (bricks with ghost layers, the halo
exchange and the inner/outer split of the force step): owns the device
buffers of an md_dd_t and grows them when md_dd_rebuild reports a capacity
shortfall.  Argument marshalling only; every step runs in libmd.so."""
from __future__ import annotations

import numpy as np
import torch

from . import md as M


class DomainSimulation:
    """potential "lj" (lj = (eps, sigma, rc)) or "eam" (Finnis-Sinclair
    dict); p = bricks per axis.  Positions and velocities FP64, forces FP32,
    grouped by brick after every build (`ids` maps to input order)."""

    def __init__(self, L, x, v, *, p=(2, 2, 2), potential="lj", lj=(1.0, 1.0, 2.5), fs=None, skin=0.3, dt=0.005,
                 mass=1.0, force_to_accel=1.0, row_cap=64, ghost_slack=1.3, compensate=True, device="cuda"):
        self.L = np.asarray(L, dtype=np.float64).reshape(3)
        x = np.asarray(x, dtype=np.float64)
        self.n = n = int(x.shape[0])
        self.potential = potential
        if potential == "lj":
            rc = float(lj[2])
        elif potential == "eam":
            rc = max(fs["d"], fs["c"])
        else:
            raise ValueError("the decomposed path runs the LJ and FS forms")
        self.skin, self.dt = float(skin), float(dt)
        self.accel = float(force_to_accel) / float(mass)
        self.mass = float(mass)
        self.r_list = rc + self.skin
        d = self.dev = torch.device(device)
        dd = self.dd = M.md_dd_init(self.L, p, self.r_list)
        dd.potential = M.MD_POT_LJ if potential == "lj" else M.MD_POT_EAM
        dd.flags = 0 if compensate else M.MD_NO_COMPENSATE
        dd.lj = M.LJ(*[float(a) for a in lj])
        if fs is not None:
            dd.fs = M.FS(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"])
        dd.n = n
        self.x = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float64, device=d)
        self.v = torch.tensor(np.ascontiguousarray(np.asarray(v, np.float64).T), dtype=torch.float64, device=d)
        self.xref = torch.empty_like(self.x)
        self.ids = torch.arange(n, dtype=torch.int32, device=d)
        self._x2, self._v2, self._ids2 = torch.empty_like(self.x), torch.empty_like(self.v), torch.empty_like(self.ids)
        self.f = torch.zeros((3, n), dtype=torch.float32, device=d)
        self.rho = torch.zeros(n, dtype=torch.float32, device=d)
        self.fprime = torch.zeros(n, dtype=torch.float32, device=d)
        self.status = torch.zeros(2, dtype=torch.int32, device=d)
        self.ev = torch.zeros(8, dtype=torch.float64, device=d)
        # expected ghosts: the halo shell of every brick
        B = self.L / np.asarray(p)
        c = np.array(dd.c[:])
        frac = np.prod(B + 2 * c) / np.prod(B) - 1.0
        self.row_cap = (int(row_cap) + 7) // 8 * 8
        self.ghost_cap = int(n * frac * ghost_slack) + 4096
        self.slot_cap = n + self.ghost_cap + 8 * dd.n_bricks
        self.comm = torch.cuda.Stream(device=d)
        self._alloc()
        self.rebuild()
        self.compute_forces()

    # ------------------------------------------------------------------
    def _alloc(self):
        d, dd = self.dev, self.dd
        dd.row_cap, dd.slot_cap, dd.ghost_cap = self.row_cap, self.slot_cap, self.ghost_cap
        gc = max(self.ghost_cap, 1)
        self.xs = torch.zeros((self.slot_cap, 4), dtype=torch.int32, device=d)
        self.count = torch.zeros(self.slot_cap, dtype=torch.int32, device=d)
        self.idx = torch.empty(self.slot_cap * self.row_cap, dtype=torch.int32, device=d)
        self.gh = torch.zeros((4, gc), dtype=torch.int32, device=d)
        self.send = torch.empty(3 * gc, dtype=torch.float64, device=d)
        self.recv = torch.empty(3 * gc, dtype=torch.float64, device=d)
        self.send_w = torch.empty(gc, dtype=torch.int32, device=d)
        self.recv_w = torch.empty(gc, dtype=torch.int32, device=d)
        self.vws = torch.empty(M.md_workspace_bytes(dd.vgrid, self.slot_cap), dtype=torch.uint8, device=d)
        self._bind()
        self.dws = torch.empty(M.md_dd_scratch_bytes(dd), dtype=torch.uint8, device=d)
        self._bind()
        M.md_dd_workspace_init(dd)

    def _bind(self):
        dd = self.dd
        p = lambda t: t.data_ptr() if t is not None else None
        dd.x, dd.v, dd.xref, dd.ids = p(self.x), p(self.v), p(self.xref), p(self.ids)
        dd.x2, dd.v2, dd.ids2 = p(self._x2), p(self._v2), p(self._ids2)
        dd.f, dd.rho, dd.fprime, dd.status = p(self.f), p(self.rho), p(self.fprime), p(self.status)
        dd.xs, dd.count, dd.idx = p(self.xs), p(self.count), p(self.idx)
        dd.gh_src, dd.gh_slot, dd.gh_code, dd.gh_src_slot = (p(self.gh[0]), p(self.gh[1]), p(self.gh[2]),
                                                             p(self.gh[3]))
        dd.send, dd.recv, dd.send_w, dd.recv_w = p(self.send), p(self.recv), p(self.send_w), p(self.recv_w)
        dd.vws, dd.vws_bytes = p(self.vws), self.vws.numel()
        dws = getattr(self, "dws", None)
        dd.dws, dd.dws_bytes = (p(dws), dws.numel()) if dws is not None else (None, 0)

    def rebuild(self):
        """Regroup by brick, select ghosts, sort and build lists (grows the
        buffers when they are too small)."""
        for _ in range(8):
            rc = M.md_dd_rebuild(self.dd)
            if rc == M.MD_OK:
                return
            dd = self.dd
            grow = False
            if dd.ghost_needed > self.ghost_cap:
                self.ghost_cap = int(dd.ghost_needed * 1.2) + 1024
                self.slot_cap = max(self.slot_cap, self.n + self.ghost_cap + 8 * dd.n_bricks)
                grow = True
            if dd.slot_needed > self.slot_cap:
                self.slot_cap = int(dd.slot_needed * 1.1) + 1024
                grow = True
            if dd.row_cap_needed > self.row_cap:
                self.row_cap = (int(dd.row_cap_needed * 1.2) + 7) // 8 * 8
                grow = True
            dd.ghost_needed = dd.slot_needed = dd.row_cap_needed = 0
            if not grow:
                raise M.MDError(rc, "md_dd_rebuild")
            self._alloc()
        raise RuntimeError("md_dd_rebuild: capacities did not converge")

    def compute_forces(self, energy: bool = False):
        M.md_dd_forces(self.dd, self.ev if energy else None, M.MD_ENERGY if energy else 0, comm=self.comm)

    def run(self, steps: int):
        """`steps` velocity-Verlet steps in the native loop (rebuilds when
        some atom moved more than skin/2; buffers grown on demand)."""
        left = int(steps)
        while left > 0:
            before = self.dd.steps
            rc = M.md_dd_run(self.dd, left, self.dt, self.accel, self.skin, comm=self.comm)
            left -= self.dd.steps - before
            if rc == M.MD_ERR_CAPACITY:
                self.rebuild()            # grows the buffers; the pending step then goes on
                if self.dd.phase == 2:
                    self.dd.phase = 1

    # ------------------------------------------------------------------
    def energies(self):
        """(potential, kinetic) energy (host sync)."""
        self.compute_forces(energy=True)
        ev = self.ev.cpu().numpy()
        ke = 0.5 * self.mass * float((self.v.double() ** 2).sum()) / (self.accel * self.mass)
        return (ev[1] if self.potential == "lj" else ev[0]), ke

    def by_id(self, a):
        ids = self.ids.cpu().numpy()
        out = np.empty_like(a)
        out[ids] = a
        return out

    def positions(self):
        return self.by_id(self.x.cpu().numpy().T)

    def forces(self):
        return self.by_id(self.f.cpu().numpy().T)

    def bricks(self):
        """Per brick: (atoms, inner atoms, ghosts, first slot)."""
        dd = self.dd
        return [(dd.brick_start[t + 1] - dd.brick_start[t], dd.n_inner[t], dd.ghost_start[t + 1] - dd.ghost_start[t],
                 dd.slot0[t]) for t in range(dd.n_bricks)]

    def close(self):
        M.md_dd_release(self.dd)
