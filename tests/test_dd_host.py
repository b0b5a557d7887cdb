"""Host-side geometry of the domain decomposition (md_dd_init,
md_dd_scratch_bytes): no GPU needed."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def M():
    import os
    from paper_1611_00075_amd import md
    if not os.path.exists(md.LIB_PATH):
        from paper_1611_00075_amd import build
        build.build()
    return md


@pytest.mark.parametrize("L,p,r_list", [((23.5, 23.5, 23.5), (2, 2, 2), 2.8), ((43.38, 43.38, 43.38), (1, 1, 1), 5.4),
                                        ((60.0, 40.0, 30.0), (3, 2, 1), 2.8)])
def test_geometry(M, L, p, r_list):
    dd = M.md_dd_init(L, p, r_list)
    assert dd.n_bricks == int(np.prod(p))
    for a in range(3):
        B = L[a] / p[a]
        k = math.floor(B / (r_list * (1 + 1e-6)))
        assert dd.k[a] == k and k >= 3
        assert dd.c[a] == pytest.approx(B / k, rel=1e-15)
        assert dd.c[a] >= r_list
        # frame: halo cell, k brick cells, halo cell, empty gap cell
        assert dd.vbox.L[a] == pytest.approx((k + 3) * dd.c[a], rel=1e-15)
        assert dd.vgrid.nc[a] == k + 3
        assert dd.vgrid.inv_cell[a] == pytest.approx((k + 3) / dd.vbox.L[a], rel=1e-15)
    assert dd.vgrid.n_cells == int(np.prod([k + 3 for k in dd.k]))
    assert dd.inner_cells == int(np.prod([k - 2 for k in dd.k]))


def test_rejects_bricks_thinner_than_three_cells(M):
    with pytest.raises(M.MDError):
        M.md_dd_init((16.8, 16.8, 16.8), (2, 2, 2), 2.8)      # brick 8.4 < 3 * 2.8 (with the margin)
    with pytest.raises(M.MDError):
        M.md_dd_init((200.0, 200.0, 200.0), (5, 5, 3), 2.8)   # 75 bricks > 64


def test_scratch_grows_with_capacities(M):
    dd = M.md_dd_init((43.38,) * 3, (2, 2, 2), 5.4)
    dd.n, dd.ghost_cap, dd.slot_cap = 1000, 1000, 3000
    a = M.md_dd_scratch_bytes(dd)
    dd.n, dd.ghost_cap, dd.slot_cap = 100000, 50000, 160000
    b = M.md_dd_scratch_bytes(dd)
    assert 0 < a < b
