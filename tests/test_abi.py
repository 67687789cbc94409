"""C-ABI contract checks that need no GPU: the library loads, exports every
function declared in include/cdg2.h, and rejects invalid configurations before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_1403_1157_amd import cdg2 as B
from paper_1403_1157_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(cdg2_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = declared_functions()
    assert "cdg2_apply_operator" in names and "cdg2_rk_step" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_exposes_the_c_names():
    for n in declared_functions():
        assert hasattr(B, n), n


def test_struct_layout_matches_header():
    # 26 doubles of coefficients; config = 6 ints + pad to 8 + 2 doubles + coeffs
    assert ctypes.sizeof(B.cdg2_coeffs) == 26 * 8
    assert B.cdg2_config.coeffs.offset == ctypes.sizeof(ctypes.c_int) * 8 + 16
    # flux selection after the coefficients: 2 ints + 1 double
    assert B.cdg2_config.diff_flux.offset == B.cdg2_config.coeffs.offset + 26 * 8
    assert B.cdg2_config.flux_eta.offset == B.cdg2_config.diff_flux.offset + 8
    assert ctypes.sizeof(B.cdg2_config) == B.cdg2_config.flux_eta.offset + 8
    # implicit controls: 3 ints + pad + 2 doubles; statistics: 4 ints + 1 double
    assert ctypes.sizeof(B.cdg2_implicit_opts) == 32
    assert B.cdg2_implicit_opts.newton_rtol.offset == 16
    assert ctypes.sizeof(B.cdg2_implicit_stats) == 24
    assert B.cdg2_implicit_stats.max_residual.offset == 16


@pytest.mark.parametrize("field,value", [
    ("dim", 4), ("dim", 1), ("order", 0), ("order", 5), ("n0", 1), ("wall_axis", 3),
    ("wall_axis", -2), ("precision", 7), ("llf_mode", 3), ("g1", (0.8, 0.2)),
    ("nan", None), ("neg_diff", None), ("order3d", 4), ("flux", 5), ("flux", -1), ("eta", -1.0),
    ("eta", float("inf"))])
def test_invalid_config_rejected(field, value):
    c = inputs.base_coeffs()
    dim, order = 2, 2
    if field == "order3d":
        dim, order = 3, 4
    cfg = B.make_config(dim, (8, 8, 8), order, c)
    if field == "dim":
        cfg.dim = value
    elif field == "order":
        cfg.order = value
    elif field == "n0":
        cfg.n[0] = value
    elif field == "wall_axis":
        cfg.wall_axis = value
    elif field == "precision":
        cfg.precision = value
    elif field == "llf_mode":
        cfg.llf_mode = value
    elif field == "g1":
        cfg.gamma1_in[:] = list(value)
    elif field == "flux":
        cfg.diff_flux = value
    elif field == "eta":
        cfg.flux_eta = value
    elif field == "nan":
        cfg.coeffs.k = float("nan")
    elif field == "neg_diff":
        cfg.coeffs.mu[1] = -1.0
    with pytest.raises(B.CDG2Error) as ei:
        B.cdg2_create(cfg)
    assert ei.value.code == B.CDG2_EINVAL
    assert len(B.lib().cdg2_last_error()) > 0


def test_null_arguments_rejected():
    L = B.lib()
    assert L.cdg2_create(None, None) == B.CDG2_EINVAL
    assert L.cdg2_apply_operator(None, None, None) == B.CDG2_EINVAL
    assert L.cdg2_rk_step(None, None, 0.1, 1) == B.CDG2_EINVAL
    assert L.cdg2_rk_step_noalloc(None, None, 0.1, 1) == B.CDG2_EINVAL
    assert L.cdg2_rk_step_adjoint(None, None, None, None, 0.1, None) == B.CDG2_EINVAL
    assert L.cdg2_rk_adjoint_segment(None, None, 1, 0.1, None, None) == B.CDG2_EINVAL
    assert L.cdg2_dirk_step(None, None, 0.1, None, None) == B.CDG2_EINVAL
    assert L.cdg2_batch_autotune(None, None) == B.CDG2_EINVAL
    assert L.cdg2_batch_set_graph(None, 1) == B.CDG2_EINVAL
    assert L.cdg2_batch_rk(None, None, None, None, 1) == B.CDG2_EINVAL
    assert L.cdg2_batch_create(None, 0, 0, None) == B.CDG2_EINVAL
    assert L.cdg2_destroy(None) == B.CDG2_OK
    assert L.cdg2_num_dofs(None) == 0


def test_triangle_mesh_rejected_before_any_device_call():
    """Invalid triangle meshes and orders fail in the host checks (no GPU needed)."""
    import numpy as np
    from paper_1403_1157_amd import inputs
    xy, nbr, nbe = inputs.kuhn_mesh(3, 2)
    c = inputs.base_coeffs()
    L = B.lib()
    assert L.cdg2_tri_create(1, 1, None, None, None, None, 0.0, 1.0, None) == B.CDG2_EINVAL
    for order in (0, 4):
        with pytest.raises(B.CDG2Error) as ei:
            B.cdg2_tri_create(order, xy, nbr, nbe, c)
        assert ei.value.code == B.CDG2_EINVAL
    bad = nbr.copy()
    bad[0, 1] = (bad[0, 1] + 1) % len(xy)                # not reciprocal
    with pytest.raises(B.CDG2Error) as ei:
        B.cdg2_tri_create(1, xy, bad, nbe, c)
    assert ei.value.code == B.CDG2_EINVAL and "reciprocal" in str(ei.value)
    code = nbr.copy()
    code[np.where(nbr == -1)] = -5                        # unknown boundary code
    with pytest.raises(B.CDG2Error):
        B.cdg2_tri_create(1, xy, code, nbe, c)
    cw = xy.copy()
    cw[0] = cw[0][::-1]                                   # clockwise element
    with pytest.raises(B.CDG2Error) as ei:
        B.cdg2_tri_create(1, cw, nbr, nbe, c)
    assert "counter-clockwise" in str(ei.value)
    assert L.cdg2_tri_destroy(None) == B.CDG2_OK
    assert L.cdg2_tri_num_dofs(None) == 0
    assert L.cdg2_tri_apply_operator(None, None, None) == B.CDG2_EINVAL
    assert L.cdg2_tri_rk_step(None, None, 0.1, 1) == B.CDG2_EINVAL


def test_tetrahedral_mesh_rejected_before_any_device_call():
    """Invalid tetrahedral meshes and orders fail in the host checks."""
    import numpy as np
    from paper_1403_1157_amd import inputs
    xyz, vid, nbr, nbe = inputs.kuhn_tet_mesh(3, 3, 1)
    c = inputs.base_coeffs()
    L = B.lib()
    assert L.cdg2_tet_create(1, 1, None, None, None, None, None, 0.0, 1.0, None) == B.CDG2_EINVAL
    for order in (0, 4):
        with pytest.raises(B.CDG2Error) as ei:
            B.cdg2_tet_create(order, xyz, vid, nbr, nbe, c)
        assert ei.value.code == B.CDG2_EINVAL
    bad = nbr.copy()
    bad[0, 0] = (bad[0, 0] + 1) % len(xyz)                 # not reciprocal
    with pytest.raises(B.CDG2Error) as ei:
        B.cdg2_tet_create(1, xyz, vid, bad, nbe, c)
    assert "reciprocal" in str(ei.value)
    vbad = vid.copy()
    e, f = np.argwhere(nbr >= 0)[0]
    vbad[e, (f + 1) % 4] = vid.max() + 7                 # a face vertex its neighbour lacks
    with pytest.raises(B.CDG2Error) as ei:
        B.cdg2_tet_create(1, xyz, vbad, nbr, nbe, c)
    assert ei.value.code == B.CDG2_EINVAL
    neg = xyz.copy()
    neg[0, [1, 2]] = neg[0, [2, 1]]                      # negatively oriented element
    with pytest.raises(B.CDG2Error) as ei:
        B.cdg2_tet_create(1, neg, vid, nbr, nbe, c)
    assert "oriented" in str(ei.value)
    assert L.cdg2_tet_destroy(None) == B.CDG2_OK
    assert L.cdg2_tet_num_dofs(None) == 0
    assert L.cdg2_tet_apply_operator(None, None, None) == B.CDG2_EINVAL
    assert L.cdg2_tet_rk_step(None, None, 0.1, 1) == B.CDG2_EINVAL
