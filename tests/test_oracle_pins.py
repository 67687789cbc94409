"""Pins of the float64 oracle against what the paper and the mathematics fix.

Each test ties the oracle to something other than itself: closed forms, exact
solutions, invariants, symmetry properties, spectral definitions or numbers
printed in the paper.  None of them needs a GPU.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle.cdg2_oracle import (C1, C2, C3, N1, N2, N3, Config, Oracle, basis1d,
                                coeff_vector, diffusion_only_coeffs, gauss_legendre01)
from paper_1403_1157_amd import inputs

DT = torch.float64
HERE = os.path.dirname(os.path.abspath(__file__))


def rand_state(o, seed=0, lo=0.3, hi=0.7, modes=0.05):
    g = torch.Generator().manual_seed(seed)
    U = modes * (2 * torch.rand(6, o.E, o.nm, generator=g, dtype=DT) - 1)
    U[:, :, 0] = lo + (hi - lo) * torch.rand(6, o.E, generator=g, dtype=DT)
    return U


def strong_coeffs():
    """Base table with chemotaxis made large enough to matter in the tests."""
    c = inputs.base_coeffs()
    c.update(chi0_11=0.05, chi0_13=0.03, chi0_21=0.04, chi0_22=0.02)
    return c


# --------------------------------------------------------------------------
# Tables: Gauss rules and Legendre end values (closed forms).
# --------------------------------------------------------------------------

def test_gauss_rules_closed_forms():
    x, w = gauss_legendre01(2)
    s = math.sqrt(3) / 6
    assert np.allclose(x.numpy(), [0.5 - s, 0.5 + s], atol=1e-16, rtol=0)
    assert np.allclose(w.numpy(), [0.5, 0.5], atol=1e-16, rtol=0)
    x, w = gauss_legendre01(3)
    s = math.sqrt(15) / 10
    assert np.allclose(x.numpy(), [0.5 - s, 0.5, 0.5 + s], atol=2e-16, rtol=0)
    assert np.allclose(w.numpy(), [5 / 18, 4 / 9, 5 / 18], atol=2e-16, rtol=0)
    # q points integrate monomials up to degree 2q-1 exactly
    for q in range(1, 8):
        x, w = gauss_legendre01(q)
        for k in range(2 * q):
            assert abs(float((w * x ** k).sum()) - 1.0 / (k + 1)) < 1e-15


def test_legendre_basis_end_values_and_orthonormality():
    p = 6
    ends = torch.tensor([0.0, 1.0], dtype=DT)
    v, d = basis1d(p, ends)
    for i in range(p + 1):
        r = math.sqrt(2 * i + 1)
        assert abs(float(v[1, i]) - r) < 1e-13
        assert abs(float(v[0, i]) - (-1) ** i * r) < 1e-13
        assert abs(float(d[1, i]) - r * i * (i + 1)) < 1e-11
        assert abs(float(d[0, i]) - (-1) ** (i + 1) * r * i * (i + 1)) < 1e-11
    x, w = gauss_legendre01(p + 1)
    B, _ = basis1d(p, x)
    G = torch.einsum("q,qi,qj->ij", w, B, B)
    assert torch.allclose(G, torch.eye(p + 1, dtype=DT), atol=1e-14, rtol=0)


def test_eoc_definition_reproduces_table1():
    """EOC = log2(e_{l-1} / e_l) reproduces the paper's printed EOC column from its
    printed L2 errors (Table 1), up to the 3-digit rounding of those errors."""
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_eoc.txt"))
    for col in (1, 3, 5):
        err, eoc = rows[:, col], rows[:, col + 1]
        for lvl in range(1, rows.shape[0]):
            assert abs(math.log2(err[lvl - 1] / err[lvl]) - eoc[lvl]) < 1e-2


# --------------------------------------------------------------------------
# Diffusion part: symmetric positive semi-definite, constants in the kernel.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,p,wall", [
    (2, (3, 3), 1, -2), (2, (4, 3), 2, -2), (2, (3, 3), 2, -1), (3, (2, 2, 2), 1, -2),
    (2, (2, 3), 3, -2)])
def test_diffusion_matrix_spsd(dim, n, p, wall):
    o = Oracle(Config(dim=dim, n=n, order=p, wall_axis=wall, coeffs=diffusion_only_coeffs(1.0)))
    K = o.assemble()
    nrm = K.abs().max()
    assert float((K - K.T).abs().max()) <= 1e-13 * float(nrm)
    ev = torch.linalg.eigvalsh(0.5 * (K + K.T))
    assert float(ev.min()) >= -1e-12 * float(nrm)
    # null space = per-species constants (dimension 6)
    assert int((ev.abs() < 1e-10 * float(nrm)).sum()) == 6
    ones = torch.zeros(6, o.E, o.nm, dtype=DT)
    ones[:, :, 0] = 1.0
    assert float((K @ ones.reshape(-1)).abs().max()) < 1e-12 * float(nrm)


# --------------------------------------------------------------------------
# CDG2 lifting: the general mass-solve lifting equals the closed form
# r_e . n^- = -(p+1)^2 / (2 h) (u^- - u^+) on Cartesian Q_p cells.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 4), (3, 2), (3, 3)])
def test_lifting_closed_form(dim, p):
    n = (3, 4, 5)[:dim]
    o = Oracle(Config(dim=dim, n=n, order=p, coeffs=inputs.base_coeffs()))
    g = torch.Generator().manual_seed(p)
    for ax in range(dim):
        nf = (p + 1) ** (dim - 1)
        jump = torch.randn(6, 7, nf, generator=g, dtype=DT)
        r = o.lift_trace(jump, ax)
        closed = -(p + 1) ** 2 / (2.0 * o.h[ax]) * jump
        assert float((r - closed).abs().max()) <= 1e-12 * float(closed.abs().max())


# --------------------------------------------------------------------------
# Conservation and exact balance laws.
# --------------------------------------------------------------------------

def _integrals(o, f):
    return (o.vol * f[:, :, 0]).sum(dim=1)       # int over Omega of each species rate


@pytest.mark.parametrize("dim,n,p,mode", [(2, (5, 4), 2, "all"), (3, (3, 3, 3), 1, "all"),
                                          (2, (4, 4), 3, "cells")])
def test_conservation_without_sources(dim, n, p, mode):
    c = strong_coeffs()
    for k in ("d1", "d2", "gamma", "alpha1", "alpha2", "f1", "k", "beta1", "beta2", "sigma"):
        c[k] = 0.0
    o = Oracle(Config(dim=dim, n=n, order=p, llf_mode=mode, coeffs=c))
    U = rand_state(o, seed=3)
    f = o.apply(U)
    scale = float(f.abs().max()) * o.vol * o.E
    assert float(_integrals(o, f).abs().max()) < 1e-13 * scale


def test_balance_laws_with_reactions():
    c = strong_coeffs()
    c["c1_star"] = c["c1_sstar"] = 5.0       # inflow switched off
    c["sigma"] = 0.0
    o = Oracle(Config(dim=2, n=(5, 6), order=2, coeffs=c))
    U = rand_state(o, seed=5)
    f = o.apply(U)
    I = _integrals(o, f)
    un = (o.vol * U[:, :, 0]).sum(dim=1)
    scale = float(f.abs().max()) * o.vol * o.E
    # c2 + c3 is conserved (k c2 moves mass from c2 to c3)
    assert abs(float(I[C2] + I[C3])) < 1e-13 * scale
    # d/dt int (n1 + n2 + n3) = -gamma int n1
    assert abs(float(I[N1] + I[N2] + I[N3] + c["gamma"] * un[N1])) < 1e-13 * scale


def test_boundary_inflow_rates():
    """Uniform state: every flux term vanishes except the inflow, so the species
    integrals change at the rates fixed by eqs. (7)-(9)."""
    c = inputs.base_coeffs()
    o = Oracle(Config(dim=2, n=(8, 4), order=2, gamma1_in=(0.25, 0.75), coeffs=c))
    for c1val, on in ((0.6, True), (0.3, False)):
        vals = torch.tensor([0.4, 0.5, 0.3, c1val, 0.45, 0.35], dtype=DT)
        U = torch.zeros(6, o.E, o.nm, dtype=DT)
        U[:, :, 0] = vals[:, None]
        I = _integrals(o, o.apply(U))
        n1, n2, n3, c1, c2, c3 = [float(v) for v in vals]
        H1 = 1.0 if c1 > c["c1_star"] else 0.0
        H2 = 1.0 if c1 > c["c1_sstar"] else 0.0
        assert (H1 == 1.0) == on
        exp_n1 = c["mu1"] * c["beta1"] * H1 - c["d1"] * n1
        exp_n2 = c["mu2"] * c["beta2"] * H2 - c["d2"] * n2
        exp_c2 = c["nu2"] * c["sigma"] * 0.5 - c["k"] * c2
        assert abs(float(I[N1]) - exp_n1) < 1e-14
        assert abs(float(I[N2]) - exp_n2) < 1e-14
        assert abs(float(I[C2]) - exp_c2) < 1e-14


# --------------------------------------------------------------------------
# Spatially uniform states: the operator reduces to the reaction ODE; SSP-RK3
# must reach the closed-form solutions with third-order accuracy.
# --------------------------------------------------------------------------

def _uniform(o, vals):
    U = torch.zeros(6, o.E, o.nm, dtype=DT)
    U[:, :, 0] = torch.tensor(vals, dtype=DT)[:, None]
    return U


def test_uniform_state_linear_reactions_exact_solution():
    c = inputs.base_coeffs()
    c.update(alpha1=0.0, alpha2=0.0, c1_star=5.0, c1_sstar=5.0, sigma=0.0)
    # small diffusivities keep the large reaction time step inside the SSP-RK3
    # stability region for the (zero) higher modes
    c.update(mu1=1e-4, mu2=1e-4, mu3=1e-4, nu1=1e-4, nu2=1e-4, nu3=1e-4)
    o = Oracle(Config(dim=2, n=(3, 3), order=1, coeffs=c))
    v0 = [0.4, 0.5, 0.3, 0.6, 0.45, 0.35]
    d1, d2, gm, f1, k = c["d1"], c["d2"], c["gamma"], c["f1"], c["k"]
    n10, n20, n30, c10, c20, c30 = v0
    T = 0.5

    def exact(t):
        e1, e2, ek = math.exp(-d1 * t), math.exp(-d2 * t), math.exp(-k * t)
        n3 = n30 + (d1 - gm) * n10 * (1 - e1) / d1 + d2 * n20 * (1 - e2) / d2
        I3 = (n30 * t + (d1 - gm) * n10 / d1 * (t - (1 - e1) / d1)
              + d2 * n20 / d2 * (t - (1 - e2) / d2))
        return [n10 * e1, n20 * e2, n3, c10 + f1 * I3, c20 * ek, c30 + c20 * (1 - ek)]

    errs = []
    for nst in (10, 20):
        U = o.rk_step(_uniform(o, v0), T / nst, nst)
        assert float(U[:, :, 1:].abs().max()) < 1e-15
        errs.append(max(abs(float(U[s, 0, 0]) - exact(T)[s]) for s in range(6)))
    assert errs[1] < 1e-5
    assert 2.7 < math.log2(errs[0] / errs[1]) < 3.3


def test_uniform_state_neutralisation_exact_solution():
    """c1' = -(alpha1 n1 + alpha2 n2) c1 with n1, n2 frozen (d1 = d2 = gamma = 0)."""
    c = inputs.base_coeffs()
    c.update(d1=0.0, d2=0.0, gamma=0.0, f1=0.0, c1_star=5.0, c1_sstar=5.0, sigma=0.0)
    o = Oracle(Config(dim=3, n=(2, 2, 2), order=1, coeffs=c))
    v0 = [0.4, 0.5, 0.3, 0.6, 0.45, 0.35]
    rate = c["alpha1"] * v0[0] + c["alpha2"] * v0[1]
    T = 0.8
    errs = []
    for nst in (8, 16):
        U = o.rk_step(_uniform(o, v0), T / nst, nst)
        errs.append(abs(float(U[C1, 0, 0]) - v0[3] * math.exp(-rate * T)))
    assert 2.7 < math.log2(errs[0] / errs[1]) < 3.3


# --------------------------------------------------------------------------
# Accuracy: exact heat solution and a manufactured solution of the full model.
# --------------------------------------------------------------------------

def _eoc_run(cfg_fn, exact, forcing_t, p, Ns, T, a_max, chi_e_rho):
    errs = []
    for N in Ns:
        o = Oracle(cfg_fn(N))
        U = o.project(exact(0.0))
        rho = o.d * chi_e_rho * a_max * N * N
        nst = int(math.ceil(T / (0.5 * 2.51 / rho)))
        U = o.rk_step(U, T / nst, nst, forcing_t=forcing_t)
        errs.append(o.l2_error(U, exact(T)))
    return errs


RHO_HAT_2D = {1: 84.0, 2: 362.06, 3: 1058.74}


@pytest.mark.parametrize("p,Ns", [(1, (8, 16)), (2, (8, 16)), (3, (6, 12))])
def test_heat_equation_eoc(p, Ns):
    """chi = 0, no reactions, no inflow: u = 0.5 + A e^{-a pi^2 (4kx^2 + ky^2) t}
    cos(2 pi kx x) cos(pi ky y) solves every species' heat equation; the L2 error
    (quadrature of order 2p+4) must converge with order p+1."""
    a, A = 0.05, 0.2
    lam = a * math.pi ** 2 * (4 + 1)

    def exact(t):
        def f(x):
            v = 0.5 + A * math.exp(-lam * t) * torch.cos(2 * math.pi * x[..., 0]) * torch.cos(math.pi * x[..., 1])
            return torch.stack([v] * 6)
        return f

    errs = _eoc_run(lambda N: Config(dim=2, n=(N, N), order=p, coeffs=diffusion_only_coeffs(a)),
                    exact, None, p, Ns, 0.02, a, RHO_HAT_2D[p])
    eoc = float(torch.log2(errs[0] / errs[1]).min())
    assert abs(eoc - (p + 1)) < 0.2, eoc


def _mms(coeffs):
    """Manufactured solution u_s = 0.5 + 0.2 e^{-t} cos(2 pi x + ph_s) cos(pi k_s y)
    (zero normal derivative on both walls) and the forcing that makes it exact,
    g = du/dt + div(F(u) - A grad u) - S(u), with derivatives from autograd."""
    th = coeff_vector(coeffs)
    ph = [0.3, 1.1, 2.0, 0.7, 2.9, 1.6]
    ky = [1, 1, 1, 1, 1, 1]

    def ufun(x, t):
        return torch.stack([0.5 + 0.2 * math.exp(-t) * torch.cos(2 * math.pi * x[..., 0] + ph[s])
                            * torch.cos(math.pi * ky[s] * x[..., 1]) for s in range(6)])

    def exact(t):
        return lambda x: ufun(x, t)

    def forcing_t(t):
        def g(x):
            x = x.detach().clone().requires_grad_(True)
            u = ufun(x, t)
            grads = [torch.autograd.grad(u[s].sum(), x, create_graph=True)[0] for s in range(6)]
            gu = torch.stack(grads)                                     # [6, ..., 2]
            n1, n2, c1, c3 = u[N1], u[N2], u[C1], u[C3]
            w1 = (th[6] / (c1 + th[10]))[..., None] * gu[C1] + (th[7] / (c3 + th[11]))[..., None] * gu[C3]
            w2 = (th[8] / (c1 + th[12]))[..., None] * gu[C1] - (th[9] / (n1 + th[13]))[..., None] * gu[N1]
            flux = -th[0:6].reshape(6, *([1] * (gu.dim() - 1))) * gu
            flux = flux + torch.stack([n1[..., None] * w1, n2[..., None] * w2] + [torch.zeros_like(w1)] * 4)
            div = []
            for s in range(6):
                dv = 0.0
                for b in range(2):
                    dv = dv + torch.autograd.grad(flux[s][..., b].sum(), x, retain_graph=True)[0][..., b]
                div.append(dv)
            div = torch.stack(div)
            dudt = -(u - 0.5)
            # reaction terms of eqs. (1)-(6)
            d1, d2, gm, a1, a2, f1, k = [float(th[i]) for i in range(14, 21)]
            S = torch.stack([-d1 * n1, -d2 * n2, d1 * n1 + d2 * n2 - gm * n1,
                             -a1 * n1 * c1 - a2 * n2 * c1 + f1 * u[N3], -k * u[C2], k * u[C2]])
            return (dudt + div - S).detach()
        return g

    return exact, forcing_t


@pytest.mark.parametrize("p,Ns,T,tol_all,min_chem", [
    (1, (8, 16), 0.01, 0.25, 1.75), (2, (8, 16), 0.004, 0.45, 2.0), (3, (6, 12), 0.002, 0.3, 3.7)])
def test_manufactured_solution_eoc(p, Ns, T, tol_all, min_chem):
    """Full nonlinear model with a manufactured solution.  The four species without
    a chemotactic flux converge with order p+1.  The two cell species carry the
    chemotactic flux, whose face value uses the element-broken gradients of both
    sides; their rate is only bounded below by p (observed: ~p+1 for odd p,
    ~p+0.3 for p = 2 on these grids, rising under refinement)."""
    c = strong_coeffs()
    c.update(c1_star=5.0, c1_sstar=5.0, sigma=0.0)
    exact, forcing_t = _mms(c)
    errs = _eoc_run(lambda N: Config(dim=2, n=(N, N), order=p, coeffs=c),
                    exact, forcing_t, p, Ns, T, 0.05, RHO_HAT_2D[p])
    eoc = torch.log2(errs[0] / errs[1])
    others = eoc[[N3, C1, C2, C3]]
    assert float((others - (p + 1)).abs().max()) < tol_all, eoc
    assert float(eoc[[N1, N2]].min()) > min_chem, eoc


def test_chemotaxis_sign_by_manufactured_solution():
    """Flipping the sign of the chemotactic flux must break the manufactured
    solution: the error then stays O(1) instead of converging."""
    c = strong_coeffs()
    c.update(c1_star=5.0, c1_sstar=5.0, sigma=0.0)
    exact, forcing_t = _mms(c)
    bad = dict(c)
    for k in ("chi0_11", "chi0_13", "chi0_21", "chi0_22"):
        bad[k] = -c[k]

    def run(coeffs, N):
        o = Oracle(Config(dim=2, n=(N, N), order=2, coeffs=coeffs))
        U = o.project(exact(0.0))
        nst = 20
        U = o.rk_step(U, 0.02 / nst, nst, forcing_t=forcing_t)
        dev = U - o.project(exact(0.02))
        return (o.vol * (dev ** 2).sum(dim=(1, 2))).sqrt()      # Parseval, per species

    good, wrong = run(c, 8), run(bad, 8)
    assert float(wrong[N1]) > 10 * float(good[N1])
    assert float(wrong[N2]) > 10 * float(good[N2])


# --------------------------------------------------------------------------
# LLF dissipation speed = spectral radius of d(F.n)/dU.
# --------------------------------------------------------------------------

def test_llf_speed_is_spectral_radius():
    c = strong_coeffs()
    o = Oracle(Config(dim=2, n=(2, 2), order=1, coeffs=c))
    th = coeff_vector(c)
    g = torch.Generator().manual_seed(11)
    for _ in range(20):
        u0 = 0.2 + 0.6 * torch.rand(6, generator=g, dtype=DT)
        gr = torch.randn(6, 2, generator=g, dtype=DT)
        nvec = torch.tensor([1.0, 0.0], dtype=DT)

        def Fn(u):
            w1, w2 = o.velocities(u, gr, th)
            return torch.stack([u[N1] * (w1 @ nvec), u[N2] * (w2 @ nvec)] + [u[0] * 0] * 4)

        J = torch.autograd.functional.jacobian(Fn, u0)
        rho = float(torch.linalg.eigvals(J).abs().max())
        w1, w2 = o.velocities(u0, gr, th)
        lam = max(abs(float(w1[0])), abs(float(w2[0])))
        assert abs(rho - lam) < 1e-14 * max(1.0, lam)


# --------------------------------------------------------------------------
# Indexing and symmetry: periodic shifts commute with f; mirror symmetry.
# --------------------------------------------------------------------------

def test_periodic_shift_commutes():
    o = Oracle(Config(dim=3, n=(4, 3, 3), order=2, coeffs=strong_coeffs()))
    U = rand_state(o, seed=8)
    f = o.apply(U)
    for ax in (0, 1):
        dim = o.gdim(ax, 1)
        Us = o.flat(torch.roll(o.grid(U), 1, dims=dim))
        fs = o.flat(torch.roll(o.grid(f), 1, dims=dim))
        assert float((o.apply(Us) - fs).abs().max()) < 1e-14 * float(f.abs().max())


def _mirror(o, X, ax):
    """Reflect the field x_ax -> 1 - x_ax: cells reversed, mode i_ax gets (-1)^i."""
    G = torch.flip(o.grid(X), dims=[o.gdim(ax, 1)])
    q = o.p + 1
    sign = torch.tensor([(-1) ** ((m // q ** ax) % q) for m in range(o.nm)], dtype=DT)
    return o.flat(G) * sign


@pytest.mark.parametrize("ax", [0, 1])
def test_mirror_equivariance(ax):
    c = strong_coeffs()
    if ax == 1:           # reflecting the wall axis swaps Gamma1 and Gamma2
        c.update(beta1=0.0, beta2=0.0, sigma=0.0)
    o = Oracle(Config(dim=2, n=(5, 4), order=3, coeffs=c))
    U = rand_state(o, seed=9)
    lhs = o.apply(_mirror(o, U, ax))
    rhs = _mirror(o, o.apply(U), ax)
    assert float((lhs - rhs).abs().max()) < 1e-13 * float(rhs.abs().max())


# --------------------------------------------------------------------------
# Discrete adjoint: autograd vector-Jacobian products agree with central
# finite differences of the oracle.
# --------------------------------------------------------------------------

def test_oracle_vjp_matches_finite_differences():
    c = strong_coeffs()
    o = Oracle(Config(dim=2, n=(3, 3), order=2, coeffs=c))
    U = rand_state(o, seed=12)
    g = torch.Generator().manual_seed(13)
    w = torch.randn(6, o.E, o.nm, generator=g, dtype=DT)
    v = torch.randn(6, o.E, o.nm, generator=g, dtype=DT)
    th = coeff_vector(c).clone().requires_grad_(True)
    X = U.clone().requires_grad_(True)
    val = (o.apply(X, th) * w).sum()
    gU, gth = torch.autograd.grad(val, (X, th))
    eps = 1e-6
    fd = ((o.apply(U + eps * v, th.detach()) - o.apply(U - eps * v, th.detach())) * w).sum() / (2 * eps)
    assert abs(float(fd) - float((gU * v).sum())) < 1e-7 * abs(float(fd))
    for j in (0, 6, 10, 14, 17, 20):
        e = torch.zeros_like(th.detach())
        e[j] = eps * max(1.0, abs(float(th[j])))
        fdj = ((o.apply(U, th.detach() + e) - o.apply(U, th.detach() - e)) * w).sum() / (2 * float(e[j]))
        assert abs(float(fdj) - float(gth[j])) < 1e-6 * max(1.0, abs(float(fdj)))


def test_input_fields_positive_and_in_range():
    for dim, n, p in ((2, (16, 16), 1), (3, (6, 5, 4), 2)):
        U = inputs.initial_modes(dim, n, p, (0,))
        o = Oracle(Config(dim=dim, n=n, order=p, coeffs=inputs.base_coeffs()))
        u = torch.einsum("sem,qm->seq", torch.from_numpy(U), o.Phi)
        assert float(u.min()) > 0.05 and float(u.max()) < 0.95
