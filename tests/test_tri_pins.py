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


@pytest.mark.parametrize("k", [1, 2, 3])
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


@pytest.mark.parametrize("k", [1, 2, 3])
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


@pytest.mark.parametrize("k", [1, 2, 3])
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


@pytest.mark.parametrize("k", [1, 2, 3])
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


@pytest.mark.parametrize("k,Ns,rate", [(1, (8, 16), 1.9), (2, (8, 16), 2.8), (3, (4, 8), 3.7)])
def test_l2_convergence_on_heat_solution(k, Ns, rate):
    """u = 0.5 + 0.2 exp(-5 pi^2 a t) cos(2 pi x) cos(pi y) solves u_t = a lap u
    with zero normal derivative on the walls and periodicity in x; the L2 error
    after SSP-RK3 to T falls at the order k + 1 under mesh refinement (measured
    rates 1.98, 2.97, 4.00 for k = 1, 2, 3)."""
    a, T = 0.05, 0.02

    def exact(t):
        def f(x, y):
            u = 0.5 + 0.2 * math.exp(-5 * math.pi ** 2 * a * t) * np.cos(2 * np.pi * x) * np.cos(np.pi * y)
            return np.broadcast_to(u, (6,) + u.shape)
        return f

    errs = []
    for n in Ns:
        m = mesh(n, n, 0.15)
        o = TriOracle(m, k, diffusion(a))
        U = o.project(exact(0.0))
        h = 1.0 / n
        steps = int(math.ceil(T / (0.08 * h * h / (a * (k + 1) ** 4))))
        U = o.rk_step(U, T / steps, steps)
        errs.append(o.l2_error(U, exact(T)))
    assert errs[0] / errs[1] > 2 ** rate, errs


def _gauss01(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def _tri_rule(q):
    """Collapsed Gauss rule on the reference triangle, written here: exact for
    total degree 2q - 2."""
    x, w = _gauss01(q)
    pts = [(x[i], x[j] * (1.0 - x[i])) for i in range(q) for j in range(q)]
    wts = [w[i] * w[j] * (1.0 - x[i]) for i in range(q) for j in range(q)]
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_diffusion_energy_equals_the_cdg2_form_with_the_k_minus_lifting(k):
    """The oracle's pure-diffusion quadratic form -<U, R(U)> (one species,
    diffusivity a, zero-flux walls) equals the CDG2 bilinear form assembled here
    independently:
      B(u, u) = sum_K int_K a |grad u|^2 - 2 sum_e int_e a {grad u}.n^- (u^- - u^+)
                + 4 chi_e sum_e int_{K^-} a |r_e|^2,
    chi_e = 3/2, where r_e in [P_k(K^-)]^2 is the lifting of the edge's jump on
    K^- (the smaller triangle, ties to the lower index) defined by
      int_{K^-} r_e . tau = -1/2 int_e (u^- - u^+) n^- . tau   for all tau,
    solved in a physical monomial basis of K^- with a mass matrix from a
    higher-order rule.  Doubling or halving 2 chi_e changes the lifting term by
    far more than the tolerance."""
    a = 0.7
    m = mesh(3, 3, 0.3)
    c = diffusion(a)
    o = TriOracle(m, k, c)
    rng = np.random.default_rng(21 + k)
    U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
    U[0] = torch.from_numpy(rng.standard_normal((m.E, o.nb)))
    form_oracle = -float((U[0] * o.residual(U)[0]).sum())

    basis = TriBasis(k)
    xy, nbr, nbe = m.xy, m.nbr, m.nbe
    E = m.E
    J = [np.column_stack([xy[e, 1] - xy[e, 0], xy[e, 2] - xy[e, 0]]) for e in range(E)]
    area = np.array([0.5 * abs(np.linalg.det(J[e])) for e in range(E)])
    coef = U[0].numpy()

    def u_and_grad(e, X):
        """u and its physical gradient at physical points X [n, 2] of element e."""
        ref = np.linalg.solve(J[e], (X - xy[e, 0]).T).T
        val = basis.values(ref) @ coef[e]
        g = np.einsum("njb,j->nb", basis.grads(ref), coef[e]) @ np.linalg.inv(J[e])
        return val, g

    # volume: sum_K int a |grad u|^2 with a rule exact beyond the integrand's degree
    rp, rw = _tri_rule(k + 3)
    vol = 0.0
    for e in range(E):
        X = xy[e, 0] + rp @ J[e].T
        _, g = u_and_grad(e, X)
        vol += a * 2.0 * area[e] * np.sum(rw * np.sum(g * g, axis=1))
    # monomials of degree <= k in physical coordinates centred on a triangle
    pw = [(d - b, b) for d in range(k + 1) for b in range(d + 1)]

    def mono(X, x0):
        Y = X - x0
        return np.stack([Y[:, 0] ** i * Y[:, 1] ** j for i, j in pw], axis=1)

    sx, sw = _gauss01(k + 3)
    face, lift = 0.0, 0.0
    for e in range(E):
        for j in range(3):
            f = nbr[e, j]
            if f < 0 or (f, nbe[e, j]) < (e, j):
                continue                                   # boundary edge, or done from the other side
            v0, v1 = xy[e, j], xy[e, (j + 1) % 3]
            L = np.hypot(*(v1 - v0))
            n_e = np.array([v1[1] - v0[1], -(v1[0] - v0[0])]) / L   # outward from e
            Xe = v0 + sx[:, None] * (v1 - v0)
            fj = nbe[e, j]
            w0, w1 = xy[f, (fj + 1) % 3], xy[f, fj]          # the same points, neighbour's image
            Xf = w0 + sx[:, None] * (w1 - w0)
            ue, ge = u_and_grad(e, Xe)
            uf, gf = u_and_grad(f, Xf)
            e_minus = area[e] < area[f] or (area[e] == area[f] and e < f)
            km, nm_, Xm = (e, n_e, Xe) if e_minus else (f, -n_e, Xf)
            jump = (ue - uf) if e_minus else (uf - ue)     # u^- - u^+
            avg_n = 0.5 * ((ge + gf) @ nm_)
            face += -2.0 * a * L * np.sum(sw * avg_n * jump)
            # lifting on K^-: mass matrix of the monomials, right-hand sides per component
            x0 = xy[km].mean(axis=0)
            Xq = xy[km, 0] + rp @ J[km].T
            Vq = mono(Xq, x0)
            Mk = (Vq * (rw * 2.0 * area[km])[:, None]).T @ Vq
            Ve = mono(Xm, x0)
            r2 = 0.0
            for comp in range(2):
                rhs = -0.5 * L * (Ve * (sw * jump * nm_[comp])[:, None]).sum(axis=0)
                rc = np.linalg.solve(Mk, rhs)
                r2 += rc @ Mk @ rc
            lift += 4.0 * 1.5 * a * r2
    form_here = vol + face + lift
    assert abs(form_oracle - form_here) <= 1e-11 * abs(form_here), (form_oracle, form_here)
    # the lifting term is a visible part of the form: a factor 2 on 2 chi_e would fail
    assert abs(lift) > 1e-3 * abs(form_here)
