"""Velocity-Verlet driver over the C ABI: owns the device buffers of one
system and sequences the library calls of a step (Sec. 3.3 of the paper):

    half kick + drift (+ rebuild check)  -> md_integrate(MD_KICK_DRIFT)
    if some atom moved > skin/2:            md_bin_cells, md_permute,
                                            md_scale_positions,
                                            md_build_neighbors
    forces                               -> md_forces_lj | md_forces_eam
                                            | md_forces_mlp
    half kick (+ kinetic energy)         -> md_integrate(MD_KICK)

All arithmetic runs in the HIP kernels; this module only allocates torch
device tensors and reads back the 8-byte status words and scalar energies.
"""
from __future__ import annotations

import numpy as np
import torch

from . import md as M


class Simulation:
    """One periodic system on one GPU.

    potential: "lj" (params eps, sigma, rc), "eam" (Finnis-Sinclair dict),
    "tb" (second-moment tight-binding dict: A, xi, p, q, r0, rs, rc), "tbm"
    (two elements: `tbm` = three such dicts for the pair kinds 0-0, 0-1, 1-1,
    `types` = the element 0/1 of each input atom), "tab" (tabulated
    embedded-atom functions: dict with dr, drho and the knot arrays psi,
    dpsi, phi, dphi, F, dF) or
    "mlp" (descriptor geometry and normalisation `mlp`, an md.MLP, and the
    MD_MLP_NPARAM bfloat16 parameters `mlp_w`, an int16 device tensor).
    Positions and velocities are FP64; forces FP32 (FP64 with pair_fp64).
    Atoms are kept in cell (Morton) order; `ids` maps back to input order.
    """

    def __init__(self, L, x, v, *, potential="lj", lj=(1.0, 1.0, 2.5), fs=None, tb=None, tbm=None, types=None,
                 tab=None, mlp=None, mlp_w=None,
                 skin=0.3, dt=0.005, mass=1.0, force_to_accel=1.0, reach=1, pair_fp64=False,
                 compensate=True, device="cuda", row_cap=None, list_slack=1.2):
        self.L = np.asarray(L, dtype=np.float64).reshape(3)
        x = np.asarray(x, dtype=np.float64)
        self.n = n = int(x.shape[0])
        self.potential = potential
        self.lj = tuple(float(a) for a in lj)
        self.fs = fs
        self.tb = tb
        self.tbm = tbm
        self.tab = tab
        self.tab_table = None
        self.mlp, self.mlp_w = mlp, mlp_w
        if potential == "lj":
            rc = self.lj[2]
        elif potential == "eam":
            rc = max(fs["d"], fs["c"])
        elif potential == "tb":
            rc = float(tb["rc"])
        elif potential == "tbm":
            if tbm is None or types is None:
                raise ValueError("potential 'tbm' needs tbm and types")
            rc = max(float(t["rc"]) for t in tbm)
        elif potential == "tab":
            if tab is None:
                raise ValueError("potential 'tab' needs tab")
            rc = (len(tab["psi"]) - 1) * float(tab["dr"])
        elif potential == "mlp":
            if mlp is None or mlp_w is None:
                raise ValueError("potential 'mlp' needs mlp and mlp_w")
            rc = float(mlp.rc)
        else:
            raise ValueError(f"unknown potential {potential!r}")
        self.rc = rc
        self.skin = float(skin)
        self.r_list = rc + self.skin
        self.dt, self.mass, self.k = float(dt), float(mass), float(force_to_accel)
        self.accel = self.k / self.mass
        self.half_skin_sq = 0.25 * self.skin * self.skin
        self.flags = M.MD_PAIR_FP64 if pair_fp64 else 0
        if not compensate:
            self.flags |= M.MD_NO_COMPENSATE
        if potential != "lj" and pair_fp64:
            raise ValueError("the embedded-atom and MLP paths are FP32 only")
        self.dev = torch.device(device)
        self.list_slack = float(list_slack)
        d = self.dev
        self.grid = M.md_grid_init(self.L, self.r_list, reach)
        self.x = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float64, device=d)
        self.v = torch.tensor(np.ascontiguousarray(np.asarray(v, np.float64).T), dtype=torch.float64, device=d)
        self._x2 = torch.empty_like(self.x)
        self._v2 = torch.empty_like(self.v)
        self.xref = torch.empty_like(self.x)
        self.ids = torch.arange(n, dtype=torch.int32, device=d)
        self._ids2 = torch.empty_like(self.ids)
        self.types = self._types2 = None
        if potential == "tbm":
            self.types = torch.tensor(np.asarray(types, np.int32).reshape(-1), dtype=torch.int32, device=d)
            if self.types.numel() != n:
                raise ValueError("types needs one element per atom")
            self._types2 = torch.empty_like(self.types)
        if potential == "tab":
            self.tab_table = torch.empty(M.md_tab_bytes(tab), dtype=torch.uint8, device=d)
            M.md_tab_pack(tab, self.tab_table)
        self.xs = torch.zeros((max(n, 1), 4), dtype=torch.int32, device=d)
        fdt = torch.float64 if pair_fp64 else torch.float32
        self.f = torch.zeros((3, max(n, 1)), dtype=fdt, device=d)
        self.rho = torch.zeros(max(n, 1), dtype=torch.float32, device=d)
        self.fprime = torch.zeros(max(n, 1), dtype=torch.float32, device=d)
        self.e_atom = torch.zeros(max(n, 1), dtype=torch.float32, device=d)
        self.dEdG = (torch.zeros((max(n, 1), M.MD_MLP_IN), dtype=torch.float32, device=d)
                     if potential == "mlp" else None)
        self.cell = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.cell_start = torch.empty(self.grid.n_cells + 1, dtype=torch.int32, device=d)
        self.count = torch.zeros(max(n, 1), dtype=torch.int32, device=d)
        self.max_count = torch.zeros(1, dtype=torch.int32, device=d)
        # row capacity: the expected neighbour count of a dense region plus slack
        self.row_cap = (int(row_cap) + 7) // 8 * 8 if row_cap else 64
        self.idx_in = self.cnt_in = None
        self._alloc_lists()
        self.ws = torch.empty(M.md_workspace_bytes(self.grid, n), dtype=torch.uint8, device=d)
        M.md_workspace_init(self.grid, n, self.ws)
        self.status = torch.zeros(2, dtype=torch.int32, device=d)
        self.ev = torch.zeros(8, dtype=torch.float64, device=d)
        self.ke = torch.zeros(1, dtype=torch.float64, device=d)
        self.longest = 0
        self.builds = 0
        self.step_count = 0
        self._status_host = torch.zeros(2, dtype=torch.int32).pin_memory()
        self._flag_host = torch.zeros(4, dtype=torch.int32).pin_memory()   # md_run's polled word
        self._sys = M.System()
        self._sys.need_build = 0
        self._sys.phase = 0
        # optional per-phase timing: a list that step() appends
        # (phase, start_event, end_event) to, events recorded on the stream
        self.events = None
        self.rebuild()
        self.compute_forces(energy=False)

    def _alloc_lists(self):
        """List buffers for the current row capacity (and, for the learned
        potential, the compact-list scratch of the same size)."""
        size = max(M.ell_size(self.n, self.row_cap), 1)
        self.idx = torch.empty(size, dtype=torch.int32, device=self.dev)
        if self.potential == "mlp":
            self.idx_in = torch.empty(size, dtype=torch.int32, device=self.dev)
            self.cnt_in = torch.zeros(max(self.n, 1), dtype=torch.int32, device=self.dev)

    # ------------------------------------------------------------------
    def rebuild(self):
        """Wrap, bin and sort the atoms, then build the full lists."""
        n = self.n
        M.md_bin_cells(self.grid, n, self.x, self.cell, self.perm, self.cell_start, self.ws)
        if n > 0:
            M.md_permute(n, 3, self.perm, self.x, self._x2, 8)
            M.md_permute(n, 3, self.perm, self.v, self._v2, 8)
            M.md_permute(n, 1, self.perm, self.ids, self._ids2, 4)
            self.x, self._x2 = self._x2, self.x
            self.v, self._v2 = self._v2, self.v
            self.ids, self._ids2 = self._ids2, self.ids
            if self.types is not None:
                M.md_permute(n, 1, self.perm, self.types, self._types2, 4)
                self.types, self._types2 = self._types2, self.types
        self.xref.copy_(self.x)
        if not (self.flags & M.MD_PAIR_FP64):
            M.md_scale_positions(self.L, n, self.x, self.xs)
            if self.types is not None:
                M.md_set_elements(n, self.types, self.xs)
        rc, longest = M.md_build_neighbors(self.grid, n, self.x, self.cell_start, self.row_cap, self.idx,
                                           self.count, self.max_count, self.ws)
        if rc == M.MD_ERR_CAPACITY:
            self.row_cap = (int(longest * self.list_slack) + 4 + 7) // 8 * 8
            self._alloc_lists()
            rc, longest = M.md_build_neighbors(self.grid, n, self.x, self.cell_start, self.row_cap, self.idx,
                                               self.count, self.max_count, self.ws)
        self.longest = longest
        self.builds += 1

    @property
    def n_pairs(self) -> int:
        """Number of list entries (host sync)."""
        return int(self.count[: self.n].sum()) if self.n else 0

    def compute_forces(self, energy: bool = False, site: bool = False):
        """Forces of the current positions; with energy, ev as well; with
        site (EAM, MLP), the per-atom energies in e_atom."""
        fl = self.flags | (M.MD_ENERGY if energy or site else 0)
        ea = self.e_atom if site else None
        if self.potential == "lj":
            M.md_forces_lj(self.L, self.n, self.x, self.xs, self.row_cap, self.idx, self.count, self.lj, self.f,
                           self.ev, fl, self.ws)
        elif self.potential == "eam":
            M.md_forces_eam(self.L, self.n, self.xs, self.row_cap, self.idx, self.count, self.fs, self.rho,
                            self.fprime, self.f, self.ev, fl, self.ws, e_atom=ea)
        elif self.potential == "tb":
            M.md_forces_tb(self.L, self.n, self.xs, self.row_cap, self.idx, self.count, self.tb, self.rho,
                           self.fprime, self.f, self.ev, fl, self.ws, e_atom=ea)
        elif self.potential == "tbm":
            M.md_forces_tbm(self.L, self.n, self.xs, self.row_cap, self.idx, self.count, self.tbm, self.rho,
                            self.fprime, self.f, self.ev, fl, self.ws, e_atom=ea)
        elif self.potential == "tab":
            M.md_forces_tab(self.L, self.n, self.xs, self.row_cap, self.idx, self.count, self.tab, self.tab_table,
                            self.rho, self.fprime, self.f, self.ev, fl, self.ws, e_atom=ea)
        else:
            M.md_forces_mlp(self.L, self.n, self.xs, self.row_cap, self.idx, self.count, self.mlp, self.mlp_w,
                            self.dEdG, self.idx_in, self.cnt_in, ea, self.f, self.ev, fl, self.ws)

    def descriptors(self, spec, out=None):
        """Raw MLP descriptors (n, 16) of the current positions in the
        sorted atom order (the list cutoff must be >= spec.rc)."""
        if spec.rc > self.r_list:
            raise ValueError("descriptor cutoff exceeds the list cutoff")
        G = out if out is not None else torch.empty((self.n, M.MD_MLP_IN), dtype=torch.float32,
                                                    device=self.dev)
        M.md_mlp_descriptors(self.L, self.n, self.xs, self.row_cap, self.idx, self.count, spec, G)
        return G

    def _mark(self, name):
        if self.events is None:
            return None
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return (name, e)

    def _done(self, m):
        if m is not None:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.events.append((m[0], m[1], e))

    def step(self, energy: bool = False, kinetic: bool = False) -> bool:
        """One velocity-Verlet step; returns True when the lists were rebuilt."""
        self.step_count += 1
        tag = self.step_count
        xs = None if self.flags & M.MD_PAIR_FP64 else self.xs
        m = self._mark("kick_drift")
        M.md_integrate(M.MD_KICK_DRIFT, self.L, self.n, self.x, self.v, self.f, self.dt, self.accel,
                       self.mass, self.xref, self.half_skin_sq, self.status, tag, xs, None,
                       (self.flags & M.MD_PAIR_FP64) | (M.MD_XS_ELEMENT if self.types is not None else 0),
                       self.ws)
        self._done(m)
        self._status_host.copy_(self.status)          # synchronises with the stream
        st = self._status_host.tolist()
        if st[1]:
            raise M.MDError(M.MD_ERR_NONFINITE, "md_integrate")
        rebuilt = st[0] == tag
        if rebuilt:
            m = self._mark("rebuild")
            self.rebuild()
            self._done(m)
        m = self._mark("forces")
        self.compute_forces(energy)
        self._done(m)
        m = self._mark("kick")
        M.md_integrate(M.MD_KICK, self.L, self.n, self.x, self.v, self.f, self.dt, self.accel, self.mass,
                       None, 0.0, None, 0, None, self.ke if kinetic else None, self.flags & M.MD_PAIR_FP64,
                       self.ws)
        self._done(m)
        return rebuilt

    # ------------------------------------------------------------------
    def _system(self) -> "M.System":
        """md_system_t view of the current buffers (pointers refreshed)."""
        S = self._sys
        S.box = M.box(self.L)
        S.grid = self.grid
        S.lj = M.LJ(*self.lj)
        if self.fs is not None:
            S.fs = M.FS(self.fs["A"], self.fs["d"], self.fs["c"], self.fs["c0"], self.fs["c1"], self.fs["c2"])
        S.dt, S.accel, S.half_skin_sq = self.dt, self.accel, self.half_skin_sq
        S.n = self.n
        S.step, S.builds = self.step_count, self.builds
        ptr = lambda t: t.data_ptr() if t is not None else None
        S.x, S.v, S.xref, S.scratch = ptr(self.x), ptr(self.v), ptr(self.xref), ptr(self._x2)
        S.ids, S.ids_scratch = ptr(self.ids), ptr(self._ids2)
        S.xs, S.f, S.rho, S.fprime = ptr(self.xs), ptr(self.f), ptr(self.rho), ptr(self.fprime)
        S.cell, S.perm, S.cell_start = ptr(self.cell), ptr(self.perm), ptr(self.cell_start)
        S.idx, S.count, S.max_count = ptr(self.idx), ptr(self.count), ptr(self.max_count)
        S.status, S.host_status = ptr(self.status), ptr(self._flag_host)
        S.ws, S.ws_bytes = ptr(self.ws), self.ws.numel()
        S.row_cap = self.row_cap
        if self.tb is not None:
            S.tb = M.tb_params(self.tb)
        if self.tbm is not None:
            S.tbm = M.tbm_params(self.tbm)
            S.types, S.types_scratch = ptr(self.types), ptr(self._types2)
        if self.tab is not None:
            S.tab, S.tab_table = M.tab_params(self.tab), ptr(self.tab_table)
        S.potential = {"lj": M.MD_POT_LJ, "eam": M.MD_POT_EAM, "mlp": M.MD_POT_MLP,
                       "tb": M.MD_POT_TB, "tbm": M.MD_POT_TBM, "tab": M.MD_POT_TAB}[self.potential]
        if self.potential == "mlp":
            S.mlp, S.mlp_w, S.dEdG = self.mlp, ptr(self.mlp_w), ptr(self.dEdG)
            S.idx_in, S.cnt_in = ptr(self.idx_in), ptr(self.cnt_in)
        S.flags = self.flags
        return S

    def run(self, steps: int, timing: bool = False):
        """`steps` velocity-Verlet steps in the native driver (md_run).  With
        timing, returns (summed force-kernel ms, force evaluations)."""
        S = self._system()
        S.timing = 1 if timing else 0
        S.force_ms, S.force_calls = 0.0, 0
        target = S.step + int(steps)
        while S.step < target:
            rc = M.md_run(S, target - S.step)
            if rc == M.MD_ERR_CAPACITY:
                self.row_cap = (int(S.row_cap_needed * self.list_slack) + 4 + 7) // 8 * 8
                self._alloc_lists()
                S.idx, S.row_cap = self.idx.data_ptr(), self.row_cap
                if self.potential == "mlp":
                    S.idx_in, S.cnt_in = self.idx_in.data_ptr(), self.cnt_in.data_ptr()
                S.need_build = 1
        self.step_count, self.builds = S.step, S.builds
        return S.force_ms, S.force_calls

    def energies(self):
        """(potential, kinetic) of the current state, FP64, both in the
        potential's energy unit (the kinetic energy 1/2 m v^2 divided by
        force_to_accel); potential is E_shift for LJ and E_total for EAM and
        MLP (forces are recomputed)."""
        self.compute_forces(energy=True)
        M.md_integrate(M.MD_KICK, self.L, self.n, self.x, self.v, self.f, 0.0, self.accel, self.mass,
                       None, 0.0, None, 0, None, self.ke, self.flags & M.MD_PAIR_FP64, self.ws)
        ev = self.ev.cpu().numpy()
        ke = float(self.ke.cpu()[0]) / self.k
        return (ev[1] if self.potential == "lj" else ev[0]), ke

    def by_id(self, t, ncomp=3):
        """Host copy of a per-atom (ncomp, n) tensor in input order, (n, ncomp)."""
        ids = self.ids.long()
        out = torch.empty_like(t[:, : self.n] if t.dim() == 2 else t[: self.n])
        if t.dim() == 2:
            out[:, ids] = t[:, : self.n]
            return out.cpu().numpy().T.copy()
        out[ids] = t[: self.n]
        return out.cpu().numpy()

    def positions(self):
        return self.by_id(self.x)

    def velocities(self):
        return self.by_id(self.v)

    def forces(self):
        return self.by_id(self.f)

    def neighbor_sets(self):
        """Neighbour rows mapped to input ids: list of sorted arrays."""
        r = M.ell_rows(self.n, self.row_cap, self.idx, self.count)
        ids = self.ids.cpu().numpy()
        rows = [None] * self.n
        for k in range(self.n):
            rows[ids[k]] = np.sort(ids[r[k]])
        return rows
