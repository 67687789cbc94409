"""GPU parity: the HIP library (through its C ABI) against the float64 oracle on
the same seeded inputs.  Bar: relative 1e-12 in FP64, 1e-5 in FP32, both
element by element against the species scale and in the per-species 2-norm."""
import math

import pytest
import torch

from parity_util import TOL, assert_close, make_case, oracle_for
from paper_1403_1157_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu_op(cfg, precision="fp64"):
    from paper_1403_1157_amd.cdg2 import Operator
    return Operator(cfg.dim, cfg.n, cfg.order, cfg.coeffs, precision=precision,
                    wall_axis=cfg.wall_axis, llf_mode=cfg.llf_mode, gamma1_in=cfg.gamma1_in)


def strong():
    c = inputs.base_coeffs()
    c.update(chi0_11=0.05, chi0_13=0.03, chi0_21=0.04, chi0_22=0.02)
    return c


def to_dev(U, precision="fp64"):
    dt = torch.float32 if precision == "fp32" else torch.float64
    return U.to(DEV, dt).contiguous()


APPLY_CASES = [
    # dim, n, p, coeff set, wall axis, llf mode, gamma1_in
    (2, (16, 16), 1, "base", None, "all", (0, 1)),          # 2D plain method, 16x16 Q1
    (2, (12, 10), 2, "strong", None, "all", (0, 1)),
    (2, (7, 9), 3, "strong", None, "all", (0.3, 0.8)),      # ragged grid, LDL inflow sub-interval
    (2, (10, 6), 4, "strong", None, "cells", (0, 1)),
    (2, (5, 5), 2, "strong", -1, "all", (0, 1)),            # fully periodic
    (2, (6, 5), 2, "strong", 0, "all", (0.2, 0.7)),         # wall along x
    (2, (2, 2), 1, "strong", None, "all", (0, 1)),          # smallest grid
    (3, (5, 4, 3), 1, "strong", None, "all", (0, 1)),
    (3, (6, 5, 4), 2, "strong", None, "all", (0.25, 0.5)),
    (3, (4, 3, 5), 3, "strong", None, "cells", (0, 1)),
    (3, (3, 4, 2), 2, "strong", 1, "all", (0, 1)),
    (3, (4, 3, 11), 2, "strong", None, "all", (0, 1)),      # two z-slabs of the processing order, ragged
    # the face point passes split their leftover points into own and neighbour
    # halves (2D p <= 2, 3D p = 2): inflow walls and ragged workgroups among them
    (2, (9, 7), 1, "strong", 0, "all", (0.2, 0.7)),
    (3, (7, 5, 3), 2, "strong", 0, "all", (0.1, 0.6)),
]


@pytest.mark.parametrize("case", APPLY_CASES, ids=lambda c: f"d{c[0]}n{'x'.join(map(str, c[1]))}p{c[2]}{c[3]}w{c[4]}{c[5]}")
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_operator_parity(case, precision):
    dim, n, p, cs, wall, mode, g1 = case
    coeffs = inputs.base_coeffs() if cs == "base" else strong()
    U, cfg = make_case(dim, n, p, key=(0,), coeffs=coeffs, wall_axis=wall, llf_mode=mode, gamma1_in=g1)
    if precision == "fp32":
        U = U.float().double()          # both sides see the same (rounded) input
    print(f"[parity] apply {case} {precision}", flush=True)
    f_ref = oracle_for(cfg).apply(U)
    op = gpu_op(cfg, precision)
    Ud = to_dev(U, precision)
    f = op.apply(Ud)
    op.sync()
    assert_close(f, f_ref, TOL[precision], f"apply {case} {precision}")


def test_cfg0_apply_and_ten_rk_steps():
    """16x16 Q1, base coefficients, CFL dt, one apply then 10 SSP-RK3 steps."""
    U, cfg = make_case(2, (16, 16), 1, key=(0,))
    o = oracle_for(cfg)
    dt = o.max_dt(U, 0.9)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    assert_close(op.apply(Ud), o.apply(U), TOL["fp64"], "cfg0 apply")
    Uo = o.rk_step(U, dt, 10)
    op.rk_step(Ud, dt, 10)
    op.sync()
    assert_close(Ud, Uo, TOL["fp64"], "cfg0 10 RK steps")


@pytest.mark.parametrize("dim,n,p,steps", [(2, (24, 20), 2, 20), (2, (10, 12), 4, 10), (3, (8, 8, 6), 2, 5),
                                            (3, (6, 5, 19), 2, 10),   # three z-slabs, the last ragged
                                            (3, (5, 4, 12), 1, 10), (3, (4, 3, 10), 3, 10)])
def test_rk_steps_parity(dim, n, p, steps):
    U, cfg = make_case(dim, n, p, key=(1,), coeffs=strong())
    o = oracle_for(cfg)
    dt = o.max_dt(U, 0.9)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    print(f"[parity] rk d{dim} {n} p{p} steps {steps} dt {dt:.3e}", flush=True)
    op.rk_step(Ud, dt, steps)
    op.sync()
    assert_close(Ud, o.rk_step(U, dt, steps), TOL["fp64"], "rk")


def test_rk_fp32():
    U, cfg = make_case(2, (16, 16), 2, key=(1,), coeffs=strong())
    U = U.float().double()
    o = oracle_for(cfg)
    dt = o.max_dt(U, 0.9)
    op = gpu_op(cfg, "fp32")
    Ud = to_dev(U, "fp32")
    op.rk_step(Ud, dt, 10)
    op.sync()
    assert_close(Ud, o.rk_step(U, dt, 10), TOL["fp32"], "rk fp32")


def test_rk_fp32_3d():
    """FP32 SSP-RK3 steps on a 3D Q2 grid (the nodal stage kernel in single precision)."""
    U, cfg = make_case(3, (6, 5, 7), 2, key=(1,), coeffs=strong())
    U = U.float().double()
    o = oracle_for(cfg)
    dt = o.max_dt(U, 0.9)
    op = gpu_op(cfg, "fp32")
    Ud = to_dev(U, "fp32")
    op.rk_step(Ud, dt, 5)
    op.sync()
    assert_close(Ud, o.rk_step(U, dt, 5), TOL["fp32"], "rk fp32 3d")


@pytest.mark.parametrize("dim,n,p", [(2, (256, 256), 2), (2, (256, 256), 4), (3, (64, 64, 64), 2)])
def test_full_size_apply_parity(dim, n, p):
    """Full-size workloads (256^2 Q2/Q4, 64^3 Q2) in the benchmark's launch
    configuration, compared on every output."""
    U, cfg = make_case(dim, n, p, key=(1 if dim == 2 else 2,))
    print(f"[parity] full-size d{dim} {n} p{p}", flush=True)
    f_ref = oracle_for(cfg).apply(U)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    f = op.apply(Ud)
    op.sync()
    assert_close(f, f_ref, TOL["fp64"], f"full-size d{dim} p{p}")


def test_full_size_q4_apply_against_extended_precision():
    """At 256^2 Q4 the float64 noise floor reaches the 1e-12 bar (the oracle itself
    is ~1e-12 from an extended-precision evaluation of the same operator).  There
    the GPU result is also compared with the extended-precision value: it must be
    as close to it as the float64 oracle is (within a factor 2, plus 1e-13)."""
    import numpy as np
    from ld_operator import LDOperator
    from parity_util import rel_errors
    U, cfg = make_case(2, (256, 256), 4, key=(1,))
    print("[parity] 256^2 Q4 against the extended-precision evaluation", flush=True)
    truth = LDOperator(2, (256, 256), 4, cfg.coeffs).apply(U.numpy())
    truth64 = torch.from_numpy(truth.astype(np.float64))
    f_or = oracle_for(cfg).apply(U)
    op = gpu_op(cfg)
    f = op.apply(to_dev(U))
    op.sync()

    def rel(g):
        a = np.asarray(g.detach().cpu(), dtype=np.longdouble).reshape(6, -1)
        t = truth.reshape(6, -1)
        d = abs(a - t)
        return float((d.max(1) / abs(t).max(1)).max()), float((np.sqrt((d * d).sum(1)) / np.sqrt((t * t).sum(1))).max())

    e_gpu, e_or = rel(f), rel(f_or)
    print(f"[parity] 256^2 Q4: GPU {e_gpu[0]:.2e}/{e_gpu[1]:.2e}, float64 oracle {e_or[0]:.2e}/{e_or[1]:.2e} "
          f"from the extended-precision value (element-wise/norm); GPU vs oracle "
          f"{rel_errors(f, f_or)[0]:.2e}/{rel_errors(f, f_or)[1]:.2e}", flush=True)
    assert rel_errors(truth64, f_or)[0] < 2e-12
    for k in range(2):
        assert e_gpu[k] <= 2 * e_or[k] + 1e-13, (e_gpu, e_or)


def test_full_size_rk_step_3d_q2_64():
    """One SSP-RK3 step of the 64^3 Q2 workload (the three fused stage launches the
    benchmark times: eight z-slabs, the u0 combination, stage 3 in place) against
    the oracle's step, on every output."""
    U, cfg = make_case(3, (64, 64, 64), 2, key=(2,))
    o = oracle_for(cfg)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    dt = op.max_dt(Ud, 0.9)
    print(f"[parity] full-size 3D Q2 64^3 one RK step dt {dt:.3e}", flush=True)
    op.rk_step(Ud, dt, 1)
    op.sync()
    assert_close(Ud, o.rk_step(U, dt, 1), TOL["fp64"], "64^3 Q2 RK step")


def test_full_size_rk_steps_2d_q2_256():
    """Ten SSP-RK3 steps of the 256^2 Q2 workload against the oracle."""
    U, cfg = make_case(2, (256, 256), 2, key=(1,))
    o = oracle_for(cfg)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    dt = op.max_dt(Ud, 0.9)
    print(f"[parity] full-size 2D Q2 256^2 ten RK steps dt {dt:.3e}", flush=True)
    op.rk_step(Ud, dt, 10)
    op.sync()
    assert_close(Ud, o.rk_step(U, dt, 10), TOL["fp64"], "256^2 Q2 10 RK steps")


def test_set_coeffs_is_ordered_on_the_current_stream():
    """set_coeffs binds the caller's current stream before the parameter upload:
    an apply on another stream right after it sees the new coefficients."""
    U, cfg = make_case(2, (12, 10), 2, key=(3,), coeffs=strong())
    op = gpu_op(cfg)
    Ud = to_dev(U)
    c2 = strong()
    c2.update(mu1=0.03, chi0_11=0.07, alpha1=1.3)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        op.apply(Ud)
    with torch.cuda.stream(s2):
        op.set_coeffs(c2)
        f = op.apply(Ud)
        op.sync()
    cfg.coeffs = c2
    assert_close(f, oracle_for(cfg).apply(U), TOL["fp64"], "apply after set_coeffs on another stream")


@pytest.mark.parametrize("dim,n,p", [(2, (16, 16), 1), (2, (20, 12), 3), (3, (6, 5, 4), 2)])
def test_max_dt_parity(dim, n, p):
    U, cfg = make_case(dim, n, p, key=(0,), coeffs=strong())
    o = oracle_for(cfg)
    op = gpu_op(cfg)
    rho_o = o.spectral_constant()
    assert abs(op.rho_hat - rho_o) <= 1e-9 * rho_o
    dt_g = op.max_dt(to_dev(U), 0.9)
    dt_o = o.max_dt(U, 0.9, rho_hat=op.rho_hat)
    assert abs(dt_g - dt_o) <= 1e-12 * dt_o


def test_nonfinite_is_reported():
    from paper_1403_1157_amd.cdg2 import CDG2_ENONFINITE, CDG2Error
    U, cfg = make_case(2, (8, 8), 2)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    Ud[0, 3, 0] = float("nan")
    op.rk_step(Ud, 1e-4, 1)
    with pytest.raises(CDG2Error) as ei:
        op.sync()
    assert ei.value.code == CDG2_ENONFINITE
    op.sync()   # flags were cleared


def test_domain_error_is_reported():
    from paper_1403_1157_amd.cdg2 import CDG2_EDOMAIN, CDG2Error
    U, cfg = make_case(2, (8, 8), 1)
    op = gpu_op(cfg)
    Ud = to_dev(U)
    Ud[3] = 0.0
    Ud[3, :, 0] = -2.0          # c1 = -2 makes c1 + chi^th negative
    out = op.apply(Ud)
    with pytest.raises(CDG2Error) as ei:
        op.sync()
    assert ei.value.code == CDG2_EDOMAIN


def test_apply_is_deterministic():
    U, cfg = make_case(3, (8, 8, 8), 2, key=(2,))
    op = gpu_op(cfg)
    Ud = to_dev(U)
    a = op.apply(Ud).clone()
    b = op.apply(Ud)
    op.sync()
    assert torch.equal(a, b)


def test_3d_state_buffers_must_be_16_byte_aligned():
    """3D launches load whole cells in 16-byte chunks: an 8-byte-aligned view is
    rejected before any launch, an aligned one runs."""
    from paper_1403_1157_amd.cdg2 import CDG2_EINVAL, CDG2Error
    U, cfg = make_case(3, (3, 2, 2), 1, key=(1,))
    op = gpu_op(cfg)
    n = U.numel()
    buf = torch.zeros(n + 2, dtype=torch.float64, device=DEV)
    bad = buf[1:1 + n].view(U.shape)
    bad.copy_(U.to(DEV))
    with pytest.raises(CDG2Error) as ei:
        op.apply(bad)
    assert ei.value.code == CDG2_EINVAL
    with pytest.raises(CDG2Error) as ei:
        op.rk_step(bad, 1e-4, 1)
    assert ei.value.code == CDG2_EINVAL
    good = buf[2:2 + n].view(U.shape)
    good.copy_(U.to(DEV))
    out = op.apply(good)
    op.sync()
    assert torch.isfinite(out).all()
