"""Pins of the triangle-mesh oracle (CDG2 on P_k triangles) against what the
mathematics fixes: the basis, constants, conservation, symmetry and sign of the
diffusion form, the inflow integrals and the L2 convergence order on an exact
heat solution."""
import math

import numpy as np
import pytest
import torch

from oracle.tri_oracle import TriBasis, TriMesh, TriOracle, duffy_rule
from paper_1403_1157_amd import inputs


def mesh(nx, ny, jitter=0.0, key=(7,)):
    return TriMesh(*inputs.kuhn_mesh(nx, ny, jitter, key))


def diffusion(a=0.05):
    c = inputs.base_coeffs()
    for k in list(c):
        if k.startswith(("chi0", "d1", "d2", "gamma", "alpha", "f1", "k", "beta", "sigma")) or k == "k":
            c[k] = 0.0
    for k in ("mu1", "mu2", "mu3", "nu1", "nu2", "nu3"):
        c[k] = a
    return c


@pytest.mark.parametrize("k", [1, 2])
def test_basis_orthonormal_and_mean_mode(k):
    b = TriBasis(k)
    p, w = duffy_rule(k + 4)
    V = b.values(p)
    M = (V * (2.0 * w)[:, None]).T @ V
    assert np.abs(M - np.eye(b.nb)).max() < 1e-13
    assert np.abs(V[:, 0] - 1.0).max() < 1e-14
    # gradients against finite differences of the values
    x = np.array([[0.21, 0.33]])
    e = 1e-6
    g = b.grads(x)[0]
    fd = np.stack([(b.values(x + [[e, 0]]) - b.values(x - [[e, 0]]))[0] / (2 * e),
                   (b.values(x + [[0, e]]) - b.values(x - [[0, e]]))[0] / (2 * e)], axis=-1)
    assert np.abs(g - fd).max() < 1e-7


def test_kuhn_mesh_tables():
    xy, nbr, nbe = inputs.kuhn_mesh(4, 3, 0.2)
    E = xy.shape[0]
    assert E == 24
    for e in range(E):
        for j in range(3):
            f = nbr[e, j]
            if f >= 0:
                assert nbr[f, nbe[e, j]] == e and nbe[f, nbe[e, j]] == j
    assert (nbr == -1).sum() == 4 and (nbr == -2).sum() == 4
    m = TriMesh(xy, nbr, nbe)
    assert abs(m.area.sum() - 1.0) < 1e-14
    # every edge: its neighbour's edge joins the same two points (up to the x period)
    for e in range(E):
        for j in range(3):
            f = nbr[e, j]
            if f >= 0:
                k = nbe[e, j]
                a, b = xy[e, j], xy[e, (j + 1) % 3]
                c, d = xy[f, k], xy[f, (k + 1) % 3]
                sh = np.round(a[0] - d[0])                 # periodic image offset
                assert np.allclose(a, d + [sh, 0]) and np.allclose(b, c + [sh, 0])
    with pytest.raises(AssertionError):
        inputs.kuhn_mesh(2, 3)


@pytest.mark.parametrize("k", [1, 2])
def test_constant_state_has_no_flux(k):
    """A constant state: every diffusive, chemotactic and penalty term vanishes
    (zero gradients, zero jumps); with the inflow switched off what is left is
    the reaction source S(U) in mode 0."""
    m = mesh(3, 3, 0.25)
    c = inputs.base_coeffs()
    c.update(beta1=0.0, beta2=0.0, sigma=0.0)
    o = TriOracle(m, k, c)
    U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
    val = torch.tensor([0.4, 0.3, 0.5, 0.6, 0.2, 0.35], dtype=torch.float64)
    U[:, :, 0] = val[:, None]
    f = o.apply(U)
    th = o.th
    n1, n2, n3, c1, c2, c3 = val
    S = torch.stack([-th[14] * n1, -th[15] * n2, th[14] * n1 + th[15] * n2 - th[16] * n1,
                     -th[17] * n1 * c1 - th[18] * n2 * c1 + th[19] * n3, -th[20] * c2, th[20] * c2])
    assert torch.allclose(f[:, :, 0], S[:, None].expand(6, m.E), rtol=0, atol=1e-13)
    assert f[:, :, 1:].abs().max() < 1e-13


@pytest.mark.parametrize("k", [1, 2])
def test_diffusion_form_symmetric_negative_semidefinite(k):
    """The CDG2 diffusion form is symmetric and coercive: <phi_i, L_h phi_j>
    (one species, pure diffusion, zero-flux walls) is a symmetric negative
    semidefinite matrix whose kernel is the constants."""
    m = mesh(3, 2, 0.3)
    o = TriOracle(m, k, diffusion(0.7))
    n = m.E * o.nb
    A = np.zeros((n, n))
    for col in range(n):
        U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
        U[0].view(-1)[col] = 1.0
        A[:, col] = o.residual(U)[0].reshape(-1).numpy()
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-12 * scale
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < 1e-12 * scale
    assert (ev > -1e-10 * scale).sum() == 1          # only the constants


@pytest.mark.parametrize("k", [1, 2])
def test_conservation_of_means_under_zero_flux(k):
    m = mesh(4, 3, 0.2)
    o = TriOracle(m, k, diffusion(0.3))
    U = torch.from_numpy(inputs.tri_modes(m.E, k, key=(9,), amp=0.1))
    f = o.apply(U)
    tot = (f[:, :, 0] * o.area[None, :]).sum(1)
    assert tot.abs().max() < 1e-13


def test_inflow_integrals():
    """Only the inflow fluxes: the total n1 production is mu1 beta1 |Gamma1|, the
    n2 production mu2 beta2 |Gamma2|, the c2 production nu2 sigma |Gamma1,in|."""
    m = mesh(5, 2)
    c = diffusion(0.0)
    c.update(beta1=0.7, beta2=0.4, sigma=0.9, mu1=0.5, mu2=0.25, nu2=0.3, c1_star=0.0, c1_sstar=0.0)
    o = TriOracle(m, 1, c, gamma1_in=(0.2, 0.6))
    U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
    U[:, :, 0] = 0.5
    f = o.apply(U)
    tot = (f[:, :, 0] * o.area[None, :]).sum(1)
    assert abs(float(tot[0]) - 0.5 * 0.7) < 1e-14
    assert abs(float(tot[1]) - 0.25 * 0.4) < 1e-14
    assert abs(float(tot[4]) - 0.3 * 0.9 * 0.4) < 1e-14
    # the Gamma1,in mask is a step at the edge points: with the 2-point rule on edges of
    # length 0.2, [0.2, 0.6] covers exactly two edges


@pytest.mark.parametrize("k,rate", [(1, 1.8), (2, 2.5)])
def test_l2_convergence_on_heat_solution(k, rate):
    """u = 0.5 + 0.2 exp(-5 pi^2 a t) cos(2 pi x) cos(pi y) solves u_t = a lap u
    with zero normal derivative on the walls and periodicity in x; the L2 error
    after SSP-RK3 to T falls at about the order k + 1 under mesh refinement (4 -> 8
    cells per side, still pre-asymptotic: measured rates 2.0 and 2.7)."""
    a, T = 0.05, 0.02

    def exact(t):
        def f(x, y):
            u = 0.5 + 0.2 * math.exp(-5 * math.pi ** 2 * a * t) * np.cos(2 * np.pi * x) * np.cos(np.pi * y)
            return np.broadcast_to(u, (6,) + u.shape)
        return f

    errs = []
    for n in (4, 8):
        m = mesh(n, n, 0.15)
        o = TriOracle(m, k, diffusion(a))
        U = o.project(exact(0.0))
        h = 1.0 / n
        steps = int(math.ceil(T / (0.01 * h * h / (a * (k + 1) ** 4))))
        U = o.rk_step(U, T / steps, steps)
        errs.append(o.l2_error(U, exact(T)))
    assert errs[0] / errs[1] > 2 ** rate, errs
