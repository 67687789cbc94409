"""GPU parity of the triangle-mesh operator (C ABI cdg2_tri_*) against the
float64 oracle on the same seeded meshes and states: relative 1e-12 element by
element against the species scale and in the per-species 2-norm."""
import pytest
import torch

from oracle.tri_oracle import TriMesh, TriOracle
from paper_1403_1157_amd import inputs
from parity_util import TOL, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def strong():
    c = inputs.base_coeffs()
    c.update(chi0_11=0.05, chi0_13=0.03, chi0_21=0.04, chi0_22=0.02)
    return c


def case(nx, ny, k, jitter, key, coeffs, g1=(0.0, 1.0), amp=0.02):
    from paper_1403_1157_amd.cdg2 import TriOperator
    xy, nbr, nbe = inputs.kuhn_mesh(nx, ny, jitter, key)
    o = TriOracle(TriMesh(xy, nbr, nbe), k, coeffs, gamma1_in=g1)
    op = TriOperator(k, xy, nbr, nbe, coeffs, gamma1_in=g1)
    U = torch.from_numpy(inputs.tri_modes(len(xy), k, key=key, amp=amp))
    return o, op, U


@pytest.mark.parametrize("nx,ny,k,jitter,g1", [
    (3, 1, 2, 0.0, (0.0, 1.0)),         # smallest mesh: 6 triangles, every one on a wall
    (3, 2, 1, 0.0, (0.0, 1.0)),         # 12 elements: one partial workgroup
    (5, 3, 2, 0.25, (0.2, 0.7)),        # 30 elements, jittered, Gamma1,in sub-interval
    (7, 5, 1, 0.3, (0.0, 1.0)),         # 70 elements: several workgroups, ragged tail
    (8, 6, 2, 0.2, (0.3, 0.6)),
    (3, 1, 3, 0.0, (0.0, 1.0)),         # P3 on the smallest mesh
    (7, 5, 3, 0.3, (0.2, 0.7)),         # P3: several workgroups, ragged tail, Gamma1,in
])
def test_tri_apply_parity(nx, ny, k, jitter, g1):
    o, op, U = case(nx, ny, k, jitter, (nx, ny, k), strong(), g1)
    print(f"[tri] apply {nx}x{ny} k{k} jitter {jitter}", flush=True)
    f = op.apply(U.to(DEV).contiguous())
    op.sync()
    assert_close(f, o.apply(U), TOL["fp64"], f"tri apply {nx}x{ny} k{k}")


@pytest.mark.parametrize("k", [1, 2, 3])
def test_tri_rk_steps_parity(k):
    o, op, U = case(6, 5, k, 0.2, (11, k), strong(), (0.25, 0.75))
    dt = 2e-4
    print(f"[tri] rk k{k}", flush=True)
    Ud = U.to(DEV).contiguous()
    op.rk_step(Ud, dt, 10)
    op.sync()
    assert_close(Ud, o.rk_step(U, dt, 10), TOL["fp64"], f"tri rk k{k}")


@pytest.mark.parametrize("k", [1, 2, 3])
def test_tri_large_mesh_apply_parity(k):
    """64 x 64 squares (8192 triangles), jittered: every output against the oracle."""
    o, op, U = case(64, 64, k, 0.2, (12, k), strong())
    print(f"[tri] large k{k}", flush=True)
    f = op.apply(U.to(DEV).contiguous())
    op.sync()
    assert_close(f, o.apply(U), TOL["fp64"], f"tri large k{k}")


def test_tri_constant_state_and_conservation():
    """Device-side invariants: a constant state under pure diffusion gives zero;
    the element means are conserved (sum |K| f_0 = 0) with zero-flux walls."""
    c = inputs.base_coeffs()
    for key in list(c):
        if key.startswith(("chi0", "d1", "d2", "gamma", "alpha", "f1", "beta", "sigma")) or key == "k":
            c[key] = 0.0
    o, op, U = case(6, 4, 2, 0.3, (13,), c, amp=0.1)
    Ud = U.to(DEV).contiguous()
    f = op.apply(Ud).cpu()
    op.sync()
    tot = (f[:, :, 0] * o.area[None, :]).sum(1)
    assert tot.abs().max() < 1e-13
    Uc = torch.zeros_like(Ud)
    Uc[:, :, 0] = 0.5
    fc = op.apply(Uc)
    op.sync()
    assert fc.abs().max() < 1e-12
