"""ctypes binding of libmd.so: the entry points of include/md.h under the
same names.  Argument marshalling only -- every step of the path runs in the
HIP kernels.  Device buffers are torch tensors on the current GPU; kernels
run on torch's current stream.

Raises RuntimeError when libmd.so has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd.so")

MD_OK, MD_ERR_ARG, MD_ERR_BOX, MD_ERR_CAPACITY = 0, -1, -2, -3
MD_ERR_NONFINITE, MD_ERR_HIP, MD_ERR_WORKSPACE = -4, -5, -6
MD_NOALLOC_MAX_ATOMS = 1 << 22
MD_PROBE_FMA_F32, MD_PROBE_FMA_F64, MD_PROBE_MFMA_BF16 = 0, 1, 2
MD_MLP_ACT_BF16, MD_MLP_ACT_FP32 = 0, 1
MD_ENERGY, MD_PAIR_FP64, MD_NO_COMPENSATE, MD_MLP_REUSE, MD_XS_ELEMENT = 0x1, 0x2, 0x4, 0x8, 0x10
MD_KICK_DRIFT, MD_KICK = 1, 2
MD_SLICE = 8
MD_MAX_ROW_CAP = 1 << 24
MD_MAX_ATOMS_FP32 = (1 << 28) - 1


class Box(C.Structure):
    _fields_ = [("L", C.c_double * 3)]


class Grid(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("r_list", C.c_double), ("inv_cell", C.c_double * 3),
                ("nc", C.c_int32 * 3), ("reach", C.c_int32), ("n_cells", C.c_int64)]


class LJ(C.Structure):
    _fields_ = [("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double)]


class FS(C.Structure):
    _fields_ = [("A", C.c_double), ("d", C.c_double), ("c", C.c_double),
                ("c0", C.c_double), ("c1", C.c_double), ("c2", C.c_double)]


class TB(C.Structure):
    """md_tb_t: second-moment tight-binding parameters."""
    _fields_ = [("A", C.c_double), ("xi", C.c_double), ("p", C.c_double), ("q", C.c_double),
                ("r0", C.c_double), ("rs", C.c_double), ("rc", C.c_double)]


def tb_params(tb: dict) -> TB:
    return TB(*[float(tb[k]) for k in ("A", "xi", "p", "q", "r0", "rs", "rc")])


class TBM(C.Structure):
    """md_tbm_t: tight-binding parameters of the pair kinds 0-0, 0-1, 1-1."""
    _fields_ = [("pair", TB * 3)]


class TAB(C.Structure):
    """md_tab_t: knot counts and spacings of a tabulated embedded-atom form."""
    _fields_ = [("nr", C.c_int32), ("nrho", C.c_int32), ("dr", C.c_double), ("drho", C.c_double)]


def tab_params(tab: dict) -> TAB:
    return TAB(len(tab["psi"]), len(tab["F"]), float(tab["dr"]), float(tab["drho"]))


def tbm_params(pairs) -> TBM:
    m = TBM()
    for k in range(3):
        m.pair[k] = tb_params(pairs[k])
    return m


MD_MLP_IN, MD_MLP_HID, MD_MLP_NPARAM = 16, 64, 5313


class MLP(C.Structure):
    """md_mlp_t: descriptor geometry and input normalisation."""
    _fields_ = [("rc", C.c_double), ("mu0", C.c_double), ("dmu", C.c_double), ("width", C.c_double),
                ("mean", C.c_float * MD_MLP_IN), ("inv_std", C.c_float * MD_MLP_IN),
                ("activations", C.c_int32), ("reserved", C.c_int32)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("step", C.c_int64)]


def mlp_spec(rc=5.0, mu0=2.0, dmu=0.2, width=0.2, mean=None, inv_std=None, activations=MD_MLP_ACT_BF16) -> MLP:
    m = MLP(float(rc), float(mu0), float(dmu), float(width))
    m.mean[:] = [float(v) for v in (np.zeros(MD_MLP_IN) if mean is None else mean)]
    m.inv_std[:] = [float(v) for v in (np.ones(MD_MLP_IN) if inv_std is None else inv_std)]
    m.activations = int(activations)
    return m


class System(C.Structure):
    """md_system_t of include/md.h."""
    _fields_ = [("box", Box), ("grid", Grid), ("lj", LJ), ("fs", FS),
                ("dt", C.c_double), ("accel", C.c_double), ("half_skin_sq", C.c_double),
                ("n", C.c_int64), ("step", C.c_int64), ("builds", C.c_int64),
                ("x", C.c_void_p), ("v", C.c_void_p), ("xref", C.c_void_p), ("scratch", C.c_void_p),
                ("ids", C.c_void_p), ("ids_scratch", C.c_void_p), ("xs", C.c_void_p), ("f", C.c_void_p),
                ("rho", C.c_void_p), ("fprime", C.c_void_p), ("cell", C.c_void_p), ("perm", C.c_void_p),
                ("cell_start", C.c_void_p), ("idx", C.c_void_p), ("count", C.c_void_p),
                ("max_count", C.c_void_p), ("status", C.c_void_p), ("host_status", C.c_void_p),
                ("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("row_cap", C.c_int32),
                ("row_cap_needed", C.c_int32), ("potential", C.c_int32), ("flags", C.c_int32),
                ("need_build", C.c_int32), ("phase", C.c_int32), ("timing", C.c_int32), ("pad_", C.c_int32),
                ("force_ms", C.c_double), ("force_calls", C.c_int64),
                ("mlp", MLP), ("mlp_w", C.c_void_p), ("dEdG", C.c_void_p), ("idx_in", C.c_void_p),
                ("cnt_in", C.c_void_p), ("tb", TB), ("tbm", TBM), ("types", C.c_void_p),
                ("types_scratch", C.c_void_p), ("tab", TAB), ("tab_table", C.c_void_p)]


MD_DD_MAX_BRICKS = 64


class DD(C.Structure):
    """md_dd_t: a domain decomposition on one device (include/md.h)."""
    _vp = C.c_void_p
    _fields_ = [("box", Box), ("p", C.c_int32 * 3), ("n_bricks", C.c_int32), ("k", C.c_int32 * 3),
                ("c", C.c_double * 3), ("vbox", Box), ("vgrid", Grid), ("inner_cells", C.c_int64),
                ("potential", C.c_int32), ("flags", C.c_int32), ("lj", LJ), ("fs", FS), ("n", C.c_int64),
                ("x", _vp), ("v", _vp), ("xref", _vp), ("ids", _vp), ("x2", _vp), ("v2", _vp), ("ids2", _vp),
                ("f", _vp), ("rho", _vp), ("fprime", _vp), ("row_cap", C.c_int32), ("slot_cap", C.c_int64),
                ("xs", _vp), ("count", _vp), ("idx", _vp), ("ghost_cap", C.c_int64), ("gh_src", _vp),
                ("gh_slot", _vp), ("gh_code", _vp), ("gh_src_slot", _vp), ("send", _vp), ("recv", _vp),
                ("send_w", _vp), ("recv_w", _vp), ("vws", _vp), ("vws_bytes", C.c_size_t), ("dws", _vp),
                ("dws_bytes", C.c_size_t), ("status", _vp), ("n_ghost", C.c_int64),
                ("brick_start", C.c_int64 * (MD_DD_MAX_BRICKS + 1)), ("slot0", C.c_int64 * (MD_DD_MAX_BRICKS + 1)),
                ("ghost_start", C.c_int64 * (MD_DD_MAX_BRICKS + 1)), ("n_inner", C.c_int64 * MD_DD_MAX_BRICKS),
                ("ghost_needed", C.c_int64), ("slot_needed", C.c_int64), ("row_cap_needed", C.c_int32),
                ("phase", C.c_int32), ("builds", C.c_int64), ("steps", C.c_int64), ("events", _vp * 4)]


MD_POT_LJ, MD_POT_EAM, MD_POT_MLP, MD_POT_TB, MD_POT_TBM, MD_POT_TAB = 0, 1, 2, 3, 4, 5
MD_TAB_MAX_KNOTS = 2001


class MDError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {error_string(code)} ({code})")


_lib = None
_vp = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing "
                               "(run python -m paper_1611_00075_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.md_error_string.argtypes = [C.c_int]
        L.md_error_string.restype = C.c_char_p
        L.md_grid_init.argtypes = [C.POINTER(Box), C.c_double, C.c_int32, C.POINTER(Grid)]
        L.md_grid_cell_ranks.argtypes = [C.POINTER(Grid), _vp]
        L.md_workspace_bytes.argtypes = [C.POINTER(Grid), C.c_int64]
        L.md_workspace_bytes.restype = C.c_size_t
        L.md_workspace_init.argtypes = [C.POINTER(Grid), C.c_int64, _vp, C.c_size_t, _vp]
        L.md_bin_cells.argtypes = [C.POINTER(Grid), C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]
        L.md_permute.argtypes = [C.c_int64, C.c_int32, _vp, _vp, _vp, C.c_int32, _vp]
        L.md_scale_positions.argtypes = [C.POINTER(Box), C.c_int64, _vp, _vp, _vp]
        L.md_build_neighbors.argtypes = [C.POINTER(Grid), C.c_int64, _vp, _vp, C.c_int32, _vp, _vp, _vp,
                                         C.POINTER(C.c_int32), _vp, C.c_size_t, _vp]
        L.md_forces_lj.argtypes = [C.POINTER(Box), C.c_int64, _vp, _vp, C.c_int32, _vp, _vp, C.POINTER(LJ),
                                   _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.md_probe.argtypes = [C.c_int32, C.c_int64, C.c_int32, _vp, _vp]
        L.md_forces_lj_noalloc.argtypes = [C.POINTER(Box), C.c_int64, _vp, _vp, C.c_int32, _vp, _vp,
                                           C.POINTER(LJ), _vp, _vp, C.c_int32, _vp]
        L.md_forces_eam.argtypes = [C.POINTER(Box), C.c_int64, _vp, C.c_int32, _vp, _vp, C.POINTER(FS), _vp,
                                    _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.md_forces_tb.argtypes = [C.POINTER(Box), C.c_int64, _vp, C.c_int32, _vp, _vp, C.POINTER(TB), _vp,
                                   _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.md_forces_tbm.argtypes = [C.POINTER(Box), C.c_int64, _vp, C.c_int32, _vp, _vp, C.POINTER(TBM), _vp,
                                    _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.md_set_elements.argtypes = [C.c_int64, _vp, _vp, _vp]
        L.md_dd_init.argtypes = [C.POINTER(DD), C.POINTER(Box), _vp, C.c_double]
        L.md_dd_scratch_bytes.argtypes = [C.POINTER(DD)]
        L.md_dd_scratch_bytes.restype = C.c_size_t
        L.md_dd_workspace_init.argtypes = [C.POINTER(DD), _vp]
        L.md_dd_rebuild.argtypes = [C.POINTER(DD), _vp]
        L.md_dd_forces.argtypes = [C.POINTER(DD), _vp, C.c_int32, _vp, _vp]
        L.md_dd_run.argtypes = [C.POINTER(DD), C.c_int64, C.c_double, C.c_double, C.c_double, _vp, _vp]
        L.md_dd_release.argtypes = [C.POINTER(DD)]
        L.md_tab_bytes.argtypes = [C.POINTER(TAB)]
        L.md_tab_bytes.restype = C.c_int64
        L.md_tab_pack.argtypes = [C.POINTER(TAB), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.md_forces_tab.argtypes = [C.POINTER(Box), C.c_int64, _vp, C.c_int32, _vp, _vp, C.POINTER(TAB), _vp,
                                    _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.md_mlp_descriptors.argtypes = [C.POINTER(Box), C.c_int64, _vp, C.c_int32, _vp, _vp, C.POINTER(MLP),
                                         _vp, _vp]
        L.md_mlp_eval.argtypes = [C.c_int64, _vp, C.POINTER(MLP), _vp, _vp, _vp, _vp]
        L.md_forces_mlp.argtypes = [C.POINTER(Box), C.c_int64, _vp, C.c_int32, _vp, _vp, C.POINTER(MLP), _vp,
                                    _vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]
        L.md_mlp_workspace_bytes.argtypes = [C.c_int64]
        L.md_mlp_workspace_bytes.restype = C.c_size_t
        L.md_mlp_moments.argtypes = [C.c_int64, _vp, _vp, _vp, C.c_size_t, _vp]
        L.md_mlp_grad.argtypes = [C.c_int64, _vp, _vp, _vp, C.POINTER(MLP), _vp, _vp, _vp, _vp, C.c_size_t,
                                  _vp]
        L.md_mlp_train_step.argtypes = [C.c_int64, _vp, _vp, _vp, C.POINTER(MLP), C.POINTER(Adam), _vp, _vp,
                                        _vp, _vp, _vp, _vp, C.c_size_t, _vp]
        L.md_integrate.argtypes = [C.c_int32, C.POINTER(Box), C.c_int64, _vp, _vp, _vp, C.c_double,
                                   C.c_double, C.c_double, _vp, C.c_double, _vp, C.c_int32, _vp, _vp,
                                   C.c_int32, _vp, C.c_size_t, _vp]
        L.md_run.argtypes = [C.POINTER(System), C.c_int64, _vp]
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().md_error_string(int(code)).decode()


def _check(rc: int, where: str, allow=()):
    if rc != MD_OK and rc not in allow:
        raise MDError(rc, where)
    return rc


def _ptr(t, dtype=None, numel=None, name="buffer"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def box(L) -> Box:
    b = Box()
    for a in range(3):
        b.L[a] = float(L[a])
    return b


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------

def md_grid_init(L, r_list: float, reach: int = 1) -> Grid:
    g = Grid()
    _check(lib().md_grid_init(C.byref(box(L)), float(r_list), int(reach), C.byref(g)), "md_grid_init")
    return g


def md_grid_cell_ranks(grid: Grid) -> np.ndarray:
    r = np.empty(grid.n_cells, np.int32)
    _check(lib().md_grid_cell_ranks(C.byref(grid), r.ctypes.data_as(C.c_void_p)), "md_grid_cell_ranks")
    return r


def md_workspace_bytes(grid: Grid, n: int) -> int:
    b = lib().md_workspace_bytes(C.byref(grid), int(n))
    if b == 0:
        raise MDError(MD_ERR_ARG, "md_workspace_bytes")
    return int(b)


def md_workspace_init(grid: Grid, n: int, ws, stream=None):
    _check(lib().md_workspace_init(C.byref(grid), int(n), _ptr(ws, name="ws"), ws.numel(),
                                   _stream(stream)), "md_workspace_init")


def md_bin_cells(grid: Grid, n: int, x, cell, perm, cell_start, ws, stream=None):
    import torch
    _check(lib().md_bin_cells(C.byref(grid), int(n), _ptr(x, torch.float64, 3 * n, "x"),
                              _ptr(cell, torch.int32, n, "cell"), _ptr(perm, torch.int32, n, "perm"),
                              _ptr(cell_start, torch.int32, grid.n_cells + 1, "cell_start"),
                              _ptr(ws, name="ws"), ws.numel(), _stream(stream)), "md_bin_cells")


def md_permute(n: int, ncomp: int, perm, src, dst, elem_bytes: int, stream=None):
    import torch
    need = ncomp * n * elem_bytes
    for t, nm in ((src, "src"), (dst, "dst")):
        if t.numel() * t.element_size() < need:
            raise ValueError(f"{nm} holds fewer than {need} bytes")
    _check(lib().md_permute(int(n), int(ncomp), _ptr(perm, torch.int32, n, "perm"),
                            _ptr(src, name="src"), _ptr(dst, name="dst"), int(elem_bytes),
                            _stream(stream)), "md_permute")


def md_scale_positions(L, n: int, x, xs, stream=None):
    import torch
    _check(lib().md_scale_positions(C.byref(box(L)), int(n), _ptr(x, torch.float64, 3 * n, "x"),
                                    _ptr(xs, torch.int32, 4 * n, "xs"), _stream(stream)),
           "md_scale_positions")


def ell_size(n: int, row_cap: int) -> int:
    """int32 entries of a sliced-ELL index array for n atoms."""
    return ((n + MD_SLICE - 1) // MD_SLICE) * MD_SLICE * row_cap


def md_build_neighbors(grid: Grid, n: int, x, cell_start, row_cap: int, idx, count, max_count, ws,
                       sync: bool = True, stream=None) -> tuple[int, int]:
    """Returns (status, longest row): status MD_OK or MD_ERR_CAPACITY.
    With sync=False the call does not wait; (MD_OK, -1) is returned and the
    longest row is left in max_count (device)."""
    import torch
    needed = C.c_int32(-1)
    rc = lib().md_build_neighbors(C.byref(grid), int(n), _ptr(x, torch.float64, 3 * n, "x"),
                                  _ptr(cell_start, torch.int32, grid.n_cells + 1, "cell_start"), int(row_cap),
                                  _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                                  _ptr(count, torch.int32, n, "count"), _ptr(max_count, torch.int32, 1, "max_count"),
                                  C.byref(needed) if sync else None, _ptr(ws, name="ws"), ws.numel(), _stream(stream))
    _check(rc, "md_build_neighbors", allow=(MD_ERR_CAPACITY,))
    return rc, int(needed.value)


def md_forces_lj(L, n: int, x, xs, row_cap: int, idx, count, lj: tuple, f, ev, flags: int, ws, stream=None):
    import torch
    fdt = torch.float64 if flags & MD_PAIR_FP64 else torch.float32
    p = LJ(*[float(v) for v in lj])
    _check(lib().md_forces_lj(C.byref(box(L)), int(n), _ptr(x, torch.float64, 3 * n, "x"),
                              _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                              _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"), _ptr(count, torch.int32, n, "count"),
                              C.byref(p), _ptr(f, fdt, 3 * n, "f"), _ptr(ev, torch.float64, 8, "ev"), int(flags),
                              _ptr(ws, name="ws"), ws.numel(), _stream(stream)), "md_forces_lj")


def md_probe(kind: int, iters: int, blocks: int, out, stream=None):
    """Launch one peak-measurement kernel (see md.h)."""
    _check(lib().md_probe(int(kind), int(iters), int(blocks), _ptr(out, name="out"), _stream(stream)), "md_probe")


def md_forces_lj_noalloc(L, n: int, x, xs, row_cap: int, idx, count, lj: tuple, f, ev, flags: int,
                         stream=None):
    """md_forces_lj without a workspace (the library's own per-GPU array)."""
    import torch
    fdt = torch.float64 if flags & MD_PAIR_FP64 else torch.float32
    p = LJ(*[float(v) for v in lj])
    _check(lib().md_forces_lj_noalloc(C.byref(box(L)), int(n), _ptr(x, torch.float64, 3 * n, "x"),
                                      _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                                      _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                                      _ptr(count, torch.int32, n, "count"), C.byref(p), _ptr(f, fdt, 3 * n, "f"),
                                      _ptr(ev, torch.float64, 8, "ev"), int(flags), _stream(stream)),
           "md_forces_lj_noalloc")


def md_forces_eam(L, n: int, xs, row_cap: int, idx, count, fs: dict, rho, fprime, f, ev, flags: int, ws,
                  stream=None, e_atom=None):
    import torch
    p = FS(fs["A"], fs["d"], fs["c"], fs["c0"], fs["c1"], fs["c2"])
    _check(lib().md_forces_eam(C.byref(box(L)), int(n), _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                               _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                               _ptr(count, torch.int32, n, "count"), C.byref(p), _ptr(rho, torch.float32, n, "rho"),
                               _ptr(fprime, torch.float32, n, "fprime"), _ptr(f, torch.float32, 3 * n, "f"),
                               _ptr(e_atom, torch.float32, n, "e_atom"),
                               _ptr(ev, torch.float64, 8, "ev"), int(flags), _ptr(ws, name="ws"), ws.numel(),
                               _stream(stream)), "md_forces_eam")


def md_forces_tb(L, n: int, xs, row_cap: int, idx, count, tb: dict, rho, fprime, f, ev, flags: int, ws,
                 stream=None, e_atom=None):
    import torch
    p = tb_params(tb)
    _check(lib().md_forces_tb(C.byref(box(L)), int(n), _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                              _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                              _ptr(count, torch.int32, n, "count"), C.byref(p), _ptr(rho, torch.float32, n, "rho"),
                              _ptr(fprime, torch.float32, n, "fprime"), _ptr(f, torch.float32, 3 * n, "f"),
                              _ptr(e_atom, torch.float32, n, "e_atom"),
                              _ptr(ev, torch.float64, 8, "ev"), int(flags), _ptr(ws, name="ws"), ws.numel(),
                              _stream(stream)), "md_forces_tb")


def md_forces_tbm(L, n: int, xs, row_cap: int, idx, count, pairs, rho, fprime, f, ev, flags: int, ws,
                  stream=None, e_atom=None):
    import torch
    p = tbm_params(pairs)
    _check(lib().md_forces_tbm(C.byref(box(L)), int(n), _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                               _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                               _ptr(count, torch.int32, n, "count"), C.byref(p), _ptr(rho, torch.float32, n, "rho"),
                               _ptr(fprime, torch.float32, n, "fprime"), _ptr(f, torch.float32, 3 * n, "f"),
                               _ptr(e_atom, torch.float32, n, "e_atom"),
                               _ptr(ev, torch.float64, 8, "ev"), int(flags), _ptr(ws, name="ws"), ws.numel(),
                               _stream(stream)), "md_forces_tbm")


def md_set_elements(n: int, types, xs, stream=None):
    import torch
    _check(lib().md_set_elements(int(n), _ptr(types, torch.int32, n, "types"), _ptr(xs, torch.int32, 4 * n, "xs"),
                                 _stream(stream)), "md_set_elements")


def md_dd_init(L, p, r_list: float) -> DD:
    """Geometry of a decomposition of box L into p bricks (host only)."""
    dd = DD()
    pv = (C.c_int32 * 3)(*[int(a) for a in p])
    _check(lib().md_dd_init(C.byref(dd), C.byref(box(L)), C.cast(pv, C.c_void_p), float(r_list)), "md_dd_init")
    return dd


def md_dd_scratch_bytes(dd: DD) -> int:
    return int(lib().md_dd_scratch_bytes(C.byref(dd)))


def md_dd_workspace_init(dd: DD, stream=None):
    _check(lib().md_dd_workspace_init(C.byref(dd), _stream(stream)), "md_dd_workspace_init")


def md_dd_rebuild(dd: DD, stream=None) -> int:
    """MD_OK, or MD_ERR_CAPACITY with dd.ghost_needed / slot_needed /
    row_cap_needed set."""
    return _check(lib().md_dd_rebuild(C.byref(dd), _stream(stream)), "md_dd_rebuild", allow=(MD_ERR_CAPACITY,))


def md_dd_forces(dd: DD, ev=None, flags: int = 0, stream=None, comm=None):
    import torch
    _check(lib().md_dd_forces(C.byref(dd), _ptr(ev, torch.float64, 8, "ev"), int(flags), _stream(stream),
                              _stream(comm) if comm is not None else None), "md_dd_forces")


def md_dd_run(dd: DD, steps: int, dt: float, accel: float, skin: float, stream=None, comm=None) -> int:
    return _check(lib().md_dd_run(C.byref(dd), int(steps), float(dt), float(accel), float(skin), _stream(stream),
                                  _stream(comm) if comm is not None else None), "md_dd_run",
                  allow=(MD_ERR_CAPACITY,))


def md_dd_release(dd: DD):
    _check(lib().md_dd_release(C.byref(dd)), "md_dd_release")


def md_tab_bytes(tab: dict) -> int:
    return int(lib().md_tab_bytes(C.byref(tab_params(tab))))


def md_tab_pack(tab: dict, table, stream=None):
    """Fill the device table (uint8 tensor of md_tab_bytes bytes) from the
    host knot arrays of `tab` (dict with dr, drho, psi, dpsi, phi, dphi, F,
    dF)."""
    import numpy as np
    import torch
    t = tab_params(tab)
    arrs = [np.ascontiguousarray(tab[k], dtype=np.float64) for k in ("psi", "dpsi", "phi", "dphi", "F", "dF")]
    if any(len(a) != t.nr for a in arrs[:4]) or any(len(a) != t.nrho for a in arrs[4:]):
        raise ValueError("knot arrays of unequal length")
    _check(lib().md_tab_pack(C.byref(t), *[a.ctypes.data_as(_vp) for a in arrs],
                             _ptr(table, torch.uint8, md_tab_bytes(tab), "table"), _stream(stream)), "md_tab_pack")


def md_forces_tab(L, n: int, xs, row_cap: int, idx, count, tab: dict, table, rho, fprime, f, ev, flags: int, ws,
                  stream=None, e_atom=None):
    import torch
    t = tab_params(tab)
    _check(lib().md_forces_tab(C.byref(box(L)), int(n), _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                               _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                               _ptr(count, torch.int32, n, "count"), C.byref(t),
                               _ptr(table, torch.uint8, md_tab_bytes(tab), "table"),
                               _ptr(rho, torch.float32, n, "rho"), _ptr(fprime, torch.float32, n, "fprime"),
                               _ptr(f, torch.float32, 3 * n, "f"), _ptr(e_atom, torch.float32, n, "e_atom"),
                               _ptr(ev, torch.float64, 8, "ev"), int(flags), _ptr(ws, name="ws"), ws.numel(),
                               _stream(stream)), "md_forces_tab")


def md_mlp_descriptors(L, n: int, xs, row_cap: int, idx, count, mlp: MLP, G, stream=None):
    import torch
    _check(lib().md_mlp_descriptors(C.byref(box(L)), int(n), _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                                    _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                                    _ptr(count, torch.int32, n, "count"), C.byref(mlp),
                                    _ptr(G, torch.float32, MD_MLP_IN * n, "G"), _stream(stream)),
           "md_mlp_descriptors")


def md_mlp_eval(n: int, G, mlp: MLP, w, e_atom, dEdG=None, stream=None):
    import torch
    _check(lib().md_mlp_eval(int(n), _ptr(G, torch.float32, MD_MLP_IN * n, "G"), C.byref(mlp),
                             _ptr(w, torch.int16, MD_MLP_NPARAM, "w"), _ptr(e_atom, torch.float32, n, "e_atom"),
                             _ptr(dEdG, torch.float32, MD_MLP_IN * n, "dEdG"), _stream(stream)), "md_mlp_eval")


MD_MLP_MAX_ROW = 256


def md_forces_mlp(L, n: int, xs, row_cap: int, idx, count, mlp: MLP, w, dEdG, idx_in, cnt_in, e_atom, f, ev,
                  flags: int, ws, stream=None):
    import torch
    _check(lib().md_forces_mlp(C.byref(box(L)), int(n), _ptr(xs, torch.int32, 4 * n, "xs"), int(row_cap),
                               _ptr(idx, torch.int32, ell_size(n, row_cap), "idx"),
                               _ptr(count, torch.int32, n, "count"), C.byref(mlp),
                               _ptr(w, torch.int16, MD_MLP_NPARAM, "w"),
                               _ptr(dEdG, torch.float32, MD_MLP_IN * n, "dEdG"),
                               _ptr(idx_in, torch.int32, ell_size(n, row_cap), "idx_in"),
                               _ptr(cnt_in, torch.int32, n, "cnt_in"),
                               _ptr(e_atom, torch.float32, n, "e_atom"), _ptr(f, torch.float32, 3 * n, "f"),
                               _ptr(ev, torch.float64, 8, "ev"), int(flags), _ptr(ws, name="ws"), ws.numel(),
                               _stream(stream)), "md_forces_mlp")


def md_mlp_workspace_bytes(batch: int) -> int:
    b = lib().md_mlp_workspace_bytes(int(batch))
    if b == 0:
        raise MDError(MD_ERR_ARG, "md_mlp_workspace_bytes")
    return int(b)


def md_mlp_moments(n: int, G, moments, tws, stream=None):
    import torch
    _check(lib().md_mlp_moments(int(n), _ptr(G, torch.float32, MD_MLP_IN * n, "G"),
                                _ptr(moments, torch.float64, 2 * MD_MLP_IN, "moments"), _ptr(tws, name="tws"),
                                tws.numel(), _stream(stream)), "md_mlp_moments")


def _batch_rows(batch: int, sel, G, target):
    """Rows of G / target a batch reads: sel[:batch] (whose entries must
    index rows of both) or rows 0..batch-1."""
    rows = min(G.numel() // MD_MLP_IN, target.numel())
    if sel is None and rows < batch:
        raise ValueError(f"batch of {batch} rows, G/target hold {rows}")
    if sel is not None and sel.numel() < batch:
        raise ValueError(f"sel holds {sel.numel()} of {batch} entries")


def md_mlp_grad(batch: int, sel, G, target, mlp: MLP, w, grad, loss, tws, stream=None):
    import torch
    _batch_rows(batch, sel, G, target)
    _check(lib().md_mlp_grad(int(batch), _ptr(sel, torch.int32, batch, "sel"), _ptr(G, torch.float32, None, "G"),
                             _ptr(target, torch.float32, None, "target"), C.byref(mlp),
                             _ptr(w, torch.int16, MD_MLP_NPARAM, "w"),
                             _ptr(grad, torch.float32, MD_MLP_NPARAM, "grad"),
                             _ptr(loss, torch.float64, 1, "loss"), _ptr(tws, name="tws"), tws.numel(),
                             _stream(stream)), "md_mlp_grad")


def md_mlp_train_step(batch: int, sel, G, target, mlp: MLP, adam: Adam, master, m1, m2, w, loss, tws,
                      stream=None):
    import torch
    _batch_rows(batch, sel, G, target)
    _check(lib().md_mlp_train_step(int(batch), _ptr(sel, torch.int32, batch, "sel"),
                                   _ptr(G, torch.float32, None, "G"), _ptr(target, torch.float32, None, "target"),
                                   C.byref(mlp), C.byref(adam),
                                   _ptr(master, torch.float32, MD_MLP_NPARAM, "master"),
                                   _ptr(m1, torch.float32, MD_MLP_NPARAM, "m1"),
                                   _ptr(m2, torch.float32, MD_MLP_NPARAM, "m2"),
                                   _ptr(w, torch.int16, MD_MLP_NPARAM, "w"), _ptr(loss, torch.float64, 1, "loss"),
                                   _ptr(tws, name="tws"), tws.numel(), _stream(stream)), "md_mlp_train_step")


def ell_rows(n: int, row_cap: int, idx, count):
    """Host view of a sliced-ELL list: list of int arrays (sorted-index rows)."""
    cnt = count[:n].cpu().numpy()
    ix = idx[: ell_size(n, row_cap)].cpu().numpy().reshape(-1, row_cap // MD_SLICE, MD_SLICE, MD_SLICE)
    return [ix[i // MD_SLICE, :, i % MD_SLICE, :].reshape(-1)[: cnt[i]] for i in range(n)]


def md_integrate(phase: int, L, n: int, x, v, f, dt: float, accel: float, mass: float, xref,
                 half_skin_sq: float, status, tag: int, xs, ke, flags: int, ws, stream=None):
    import torch
    fdt = torch.float64 if flags & MD_PAIR_FP64 else torch.float32
    _check(lib().md_integrate(int(phase), C.byref(box(L)), int(n), _ptr(x, torch.float64, 3 * n, "x"),
                              _ptr(v, torch.float64, 3 * n, "v"), _ptr(f, fdt, 3 * n, "f"), float(dt),
                              float(accel), float(mass), _ptr(xref, torch.float64, 3 * n, "xref"),
                              float(half_skin_sq), _ptr(status, torch.int32, 2, "status"), int(tag),
                              _ptr(xs, torch.int32, 4 * n, "xs"), _ptr(ke, torch.float64, 1, "ke"), int(flags),
                              _ptr(ws, name="ws"), ws.numel(), _stream(stream)), "md_integrate")


def md_run(sys: System, steps: int, stream=None) -> int:
    """Returns MD_OK or MD_ERR_CAPACITY (sys.row_cap_needed set); raises on
    other errors."""
    rc = lib().md_run(C.byref(sys), int(steps), _stream(stream))
    return _check(rc, "md_run", allow=(MD_ERR_CAPACITY,))
