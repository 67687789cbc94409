"""Pins of the oracle's implicit DIRK integrator (Section 3.2: DIRK of order 2-4
solved by Newton) against the mathematics: the Runge-Kutta order conditions and
L-stability of the tableaux, the convergence order on a reaction ODE with a
closed-form solution, the damping of stiff diffusion at huge time steps, and the
agreement with the explicit SSP-RK3 scheme as dt -> 0."""
import math

import numpy as np
import pytest
import torch

from oracle.cdg2_oracle import Config, Oracle, diffusion_only_coeffs, sdirk_tableau
from paper_1403_1157_amd import inputs

DT = torch.float64


@pytest.mark.parametrize("order", [2, 3, 4])
def test_sdirk_tableaux_order_conditions_and_l_stability(order):
    A, b, c = sdirk_tableau(order)
    A = np.array(A)
    b = np.array(b)
    c = np.array(c)
    s = len(b)
    # singly diagonally implicit, stiffly accurate, consistent row sums
    assert np.allclose(np.triu(A, 1), 0)
    assert np.allclose(np.diag(A), A[0, 0])
    assert np.allclose(b, A[-1])
    assert np.allclose(A.sum(1), c, atol=1e-15)
    # Butcher order conditions (trees up to the stated order)
    Ac = A @ c
    conds = [(b.sum(), 1.0)]
    if order >= 2:
        conds += [(b @ c, 1 / 2)]
    if order >= 3:
        conds += [(b @ c ** 2, 1 / 3), (b @ Ac, 1 / 6)]
    if order >= 4:
        conds += [(b @ c ** 3, 1 / 4), (b @ (c * Ac), 1 / 8), (b @ (A @ c ** 2), 1 / 12),
                  (b @ (A @ Ac), 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 2e-15, (got, want)
    # one condition of the next order fails (the order is not higher)
    nxt = {2: (b @ c ** 2, 1 / 3), 3: (b @ c ** 3, 1 / 4), 4: (b @ c ** 4, 1 / 5)}[order]
    assert abs(nxt[0] - nxt[1]) > 1e-6
    # L-stability: R(z) = 1 + z b^T (I - z A)^{-1} 1 -> 1 - b^T A^{-1} 1 = 0
    assert abs(1.0 - b @ np.linalg.solve(A, np.ones(s))) < 1e-13
    # A-stability sample: |R(iy)| <= 1 on the imaginary axis
    for y in np.linspace(-50, 50, 101):
        z = 1j * y
        R = 1 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))
        assert abs(R) <= 1 + 1e-12


def _uniform(o, vals):
    U = torch.zeros(6, o.E, o.nm, dtype=DT)
    U[:, :, 0] = torch.tensor(vals, dtype=DT)[:, None]
    return U


@pytest.mark.parametrize("order,steps", [(2, (4, 8)), (3, (4, 8)), (4, (2, 4))])
def test_dirk_uniform_state_reaction_ode_order(order, steps):
    """Spatially uniform state: the operator reduces to the linear reaction ODE
    of n1, n2, n3, c1, c2, c3 (alpha = 0), solved in closed form."""
    c = inputs.base_coeffs()
    c.update(alpha1=0.0, alpha2=0.0, c1_star=5.0, c1_sstar=5.0, sigma=0.0)
    o = Oracle(Config(dim=2, n=(2, 2), order=1, coeffs=c))
    v0 = [0.4, 0.5, 0.3, 0.6, 0.45, 0.35]
    d1, d2, gm, f1, k = c["d1"], c["d2"], c["gamma"], c["f1"], c["k"]
    n10, n20, n30, c10, c20, c30 = v0
    T = 1.0

    def exact(t):
        e1, e2, ek = math.exp(-d1 * t), math.exp(-d2 * t), math.exp(-k * t)
        n3 = n30 + (d1 - gm) * n10 * (1 - e1) / d1 + d2 * n20 * (1 - e2) / d2
        I3 = (n30 * t + (d1 - gm) * n10 / d1 * (t - (1 - e1) / d1)
              + d2 * n20 / d2 * (t - (1 - e2) / d2))
        return [n10 * e1, n20 * e2, n3, c10 + f1 * I3, c20 * ek, c30 + c20 * (1 - ek)]

    errs = []
    for nst in steps:
        U = _uniform(o, v0)
        for _ in range(nst):
            U, _ = o.dirk_step(U, T / nst, order)
        assert float(U[:, :, 1:].abs().max()) < 1e-14
        errs.append(max(abs(float(U[s, 0, 0]) - exact(T)[s]) for s in range(6)))
    eoc = math.log2(errs[0] / errs[1])
    assert abs(eoc - order) < 0.35, (errs, eoc)


def test_dirk_damps_stiff_diffusion_at_huge_steps():
    """Pure diffusion, dt far beyond any explicit limit: an L-stable scheme leaves
    only the conserved cell-average mean of each species."""
    cfg = Config(dim=2, n=(4, 4), order=1, wall_axis=-1, coeffs=diffusion_only_coeffs(1.0))
    o = Oracle(cfg)
    g = torch.Generator().manual_seed(3)
    U = 0.1 * torch.randn(6, o.E, o.nm, generator=g, dtype=DT)
    U[:, :, 0] += 0.5
    mean = U[:, :, 0].mean(1)
    for order in (2, 3, 4):
        # at this dt the rounding of dt f(X) (cancellation inside L_h) sits far
        # above 1e-13 of the stage terms: a looser Newton tolerance
        V, _ = o.dirk_step(U, 1e6, order, tol=1e-6)
        # conserved up to the Newton tolerance (1e-6 of the stage terms)
        assert torch.allclose(V[:, :, 0].mean(1), mean, rtol=0, atol=1e-7)
        dev = (V - 0).clone()
        dev[:, :, 0] -= mean[:, None]
        assert float(dev.abs().max()) < 1e-5 * float((U - U.mean()).abs().max())


def test_dirk_agrees_with_ssp_rk3_as_dt_vanishes():
    """Both integrate the same ODE: DIRK2 (local error dt^3) and SSP-RK3 (dt^4)
    differ by O(dt^3) over one step."""
    c = inputs.base_coeffs()
    c.update(chi0_11=0.05, chi0_13=0.03, chi0_21=0.04, chi0_22=0.02)
    o = Oracle(Config(dim=2, n=(3, 3), order=1, coeffs=c))
    U = torch.from_numpy(inputs.initial_modes(2, (3, 3), 1, (5,)))
    dt0 = o.max_dt(U, 0.5) / 16      # asymptotic range: dt |lambda_max| << 1
    d = []
    for dt in (dt0, dt0 / 2):
        V, _ = o.dirk_step(U, dt, 2)
        d.append(float((V - o.rk_step(U, dt)).abs().max()))
    assert 6.0 < d[0] / d[1] < 10.0, d
