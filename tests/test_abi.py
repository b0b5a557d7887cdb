"""The C-ABI library loads on a CPU-only host and exports every entry point
that include/md.h declares; the host-only entry points work without a GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")
LIB = os.path.join(ROOT, "paper_1611_00075_amd", "libmd.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1611_00075_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = _declared()
    for n in ("md_bin_cells", "md_build_neighbors", "md_forces_lj", "md_forces_eam", "md_integrate"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (md_[a-z0-9_]+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(lib, n)


def test_host_only_entry_points(lib):
    from paper_1611_00075_amd import md
    g = md.md_grid_init([20.0, 14.0, 9.0], 2.8, 1)
    assert list(g.nc) == [7, 5, 3] and g.n_cells == 105
    assert g.inv_cell[0] == 7 / 20.0
    g2 = md.md_grid_init([20.0, 14.0, 9.0], 2.8, 2)
    assert list(g2.nc) == [14, 10, 6]
    with pytest.raises(md.MDError):
        md.md_grid_init([5.0, 5.0, 5.0], 2.5)
    assert md.md_workspace_bytes(g, 1000) > 0
    assert "neighbour" in md.error_string(md.MD_ERR_CAPACITY)


def test_tab_bytes_host_only(lib):
    from paper_1611_00075_amd import inputs, md
    tab = inputs.fs_table(inputs.FS_CU)
    nr, nrho = len(tab["psi"]), len(tab["F"])
    assert md.md_tab_bytes(tab) == 32 * (nr - 1) + 16 * (nrho - 1)
    assert md.md_tab_bytes(dict(tab, psi=np.zeros(md.MD_TAB_MAX_KNOTS + 1))) == 0
    assert md.md_tab_bytes(dict(tab, psi=np.zeros(1))) == 0
    assert md.md_tab_bytes(dict(tab, dr=0.0)) == 0
    assert md.md_tab_bytes(dict(tab, drho=float("nan"))) == 0


def _morton(x, y, z):
    c = 0
    for b in range(21):
        c |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return c


@pytest.mark.parametrize("L", [(20.0, 14.0, 9.0), (30.0, 30.0, 30.0), (200.0, 9.0, 9.0)])
def test_morton_ranks(lib, L):
    from paper_1611_00075_amd import md
    g = md.md_grid_init(L, 2.8, 1)
    r = md.md_grid_cell_ranks(g)
    nc = list(g.nc)
    lin = np.arange(g.n_cells)
    cx, cy, cz = lin % nc[0], (lin // nc[0]) % nc[1], lin // (nc[0] * nc[1])
    codes = np.array([_morton(int(a), int(b), int(c)) for a, b, c in zip(cx, cy, cz)])
    assert np.array_equal(np.argsort(codes, kind="stable"), np.argsort(r))
    assert np.array_equal(np.sort(r), lin)


def test_product_path_fails_loudly_without_library(monkeypatch):
    from paper_1611_00075_amd import md
    monkeypatch.setattr(md, "_lib", None)
    monkeypatch.setattr(md, "LIB_PATH", "/nonexistent/libmd.so")
    with pytest.raises(RuntimeError, match="not built"):
        md.lib()


def test_size_limits_rejected_before_any_device_work(lib):
    """Atom counts past the FP32 paths' 32-bit position range and row
    capacities past MD_MAX_ROW_CAP are argument errors, returned before any
    pointer is used (NULL buffers here; no GPU needed)."""
    from paper_1611_00075_amd import md
    vp = C.c_void_p
    box = md.Box((C.c_double * 3)(20.0, 20.0, 20.0))
    big = md.MD_MAX_ATOMS_FP32 + 1
    lib.md_forces_lj.argtypes = [C.POINTER(md.Box), C.c_int64, vp, vp, C.c_int32, vp, vp, C.POINTER(md.LJ),
                                 vp, vp, C.c_int32, vp, C.c_size_t, vp]
    lj = md.LJ(1.0, 1.0, 2.5)
    assert lib.md_forces_lj(C.byref(box), big, None, None, 64, None, None, C.byref(lj), None, None, 0,
                            None, 0, None) == md.MD_ERR_ARG
    lib.md_forces_eam.argtypes = [C.POINTER(md.Box), C.c_int64, vp, C.c_int32, vp, vp, C.POINTER(md.FS), vp,
                                  vp, vp, vp, vp, C.c_int32, vp, C.c_size_t, vp]
    fs = md.FS(1.0, 4.0, 4.0, 1.0, 0.0, 0.0)
    assert lib.md_forces_eam(C.byref(box), big, None, 64, None, None, C.byref(fs), None, None, None, None, None, 0,
                             None, 0, None) == md.MD_ERR_ARG
    assert lib.md_forces_eam(C.byref(box), 10, None, md.MD_MAX_ROW_CAP + 8, None, None, C.byref(fs), None, None,
                             None, None, None, 0, None, 0, None) == md.MD_ERR_ARG
    g = md.md_grid_init([20.0, 20.0, 20.0], 2.8, 1)
    lib.md_build_neighbors.argtypes = [C.POINTER(md.Grid), C.c_int64, vp, vp, C.c_int32, vp, vp, vp,
                                       C.POINTER(C.c_int32), vp, C.c_size_t, vp]
    assert lib.md_build_neighbors(C.byref(g), 0, None, vp(8), md.MD_MAX_ROW_CAP + 8, None, None, vp(8), None,
                                  None, 0, None) == md.MD_ERR_ARG


def test_probe_and_noalloc_reject_bad_arguments(lib):
    """The measurement probe and the allocation-free LJ entry point check
    their arguments before any device work (NULL buffers; no GPU needed)."""
    from paper_1611_00075_amd import md
    vp = C.c_void_p
    lib.md_probe.argtypes = [C.c_int32, C.c_int64, C.c_int32, vp, vp]
    out = vp(8)
    assert lib.md_probe(99, 1, 1, out, None) == md.MD_ERR_ARG            # unknown kind
    assert lib.md_probe(md.MD_PROBE_FMA_F32, 0, 1, out, None) == md.MD_ERR_ARG
    assert lib.md_probe(md.MD_PROBE_FMA_F32, 1, 0, out, None) == md.MD_ERR_ARG
    assert lib.md_probe(md.MD_PROBE_MFMA_BF16, 1, 1, None, None) == md.MD_ERR_ARG
    box = md.Box((C.c_double * 3)(20.0, 20.0, 20.0))
    lj = md.LJ(1.0, 1.0, 2.5)
    lib.md_forces_lj_noalloc.argtypes = [C.POINTER(md.Box), C.c_int64, vp, vp, C.c_int32, vp, vp,
                                         C.POINTER(md.LJ), vp, vp, C.c_int32, vp]
    big = md.MD_MAX_ATOMS_FP32 + 1
    assert lib.md_forces_lj_noalloc(C.byref(box), big, None, None, 64, None, None, C.byref(lj), None, None, 0,
                                    None) == md.MD_ERR_ARG
    assert lib.md_forces_lj_noalloc(C.byref(box), 10, None, None, 64, None, None, C.byref(lj), None, None, 0,
                                    None) == md.MD_ERR_ARG                # NULL buffers
