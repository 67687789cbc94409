"""Pins of the tetrahedral-mesh oracle (CDG2 on P_k tetrahedra) against what the
mathematics fixes: the reference basis, the symmetric face rules, the mesh
tables, constants, conservation, the symmetric semidefinite diffusion form with
the K^- lifting assembled independently, the inflow integrals and the L2
convergence order on an exact heat solution."""
import math
from itertools import permutations

import numpy as np
import pytest
import torch

from oracle.tet_oracle import (FACE_VERTS, TetBasis, TetMesh, TetOracle, collapsed_tet_rule,
                               symmetric_face_rule, symmetric_tet_rule, tet_rule_degree,
                               tet_volume_rule)
from paper_1403_1157_amd import inputs


def mesh(nx, ny, nz, jitter=0.0, key=(17,)):
    return TetMesh(*inputs.kuhn_tet_mesh(nx, ny, nz, jitter, key))


def diffusion(a=0.05):
    c = inputs.base_coeffs()
    for k in list(c):
        if k.startswith(("chi0", "d1", "d2", "gamma", "alpha", "f1", "beta", "sigma")) or k == "k":
            c[k] = 0.0
    for k in ("mu1", "mu2", "mu3", "nu1", "nu2", "nu3"):
        c[k] = a
    return c


def _gauss01(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def _stroud_rule(q):
    """Conical product rule on the reference tetrahedron, written here with
    Gauss-Jacobi-free weights: nested Gauss rules on [0,1] with the Jacobian
    (1-u)^2 (1-v) folded into the weights; q points per direction."""
    x, w = _gauss01(q)
    P, W = [], []
    for i in range(q):
        for j in range(q):
            for l in range(q):
                P.append((x[i], x[j] * (1 - x[i]), x[l] * (1 - x[i]) * (1 - x[j])))
                W.append(w[i] * w[j] * w[l] * (1 - x[i]) ** 2 * (1 - x[j]))
    return np.array(P), np.array(W)


def _tet_monomial_mean(a, b, c):
    """Mean of xi^a eta^b zeta^c over the reference tetrahedron (Dirichlet
    integral: 6 a! b! c! / (a + b + c + 3)!)."""
    f = math.factorial
    return 6.0 * f(a) * f(b) * f(c) / f(a + b + c + 3)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_basis_orthonormal_and_mean_mode(k):
    b = TetBasis(k)
    assert b.nb == (k + 1) * (k + 2) * (k + 3) // 6
    p, w = _stroud_rule(k + 4)
    # the test rule itself integrates monomials exactly
    for a, bb, c in [(0, 0, 0), (2, 1, 0), (1, 1, 1), (0, 0, 4), (3, 2, 1)]:
        got = 6.0 * np.sum(w * p[:, 0] ** a * p[:, 1] ** bb * p[:, 2] ** c)
        assert abs(got - _tet_monomial_mean(a, bb, c)) < 1e-15
    V = b.values(p)
    M = (V * (6.0 * w)[:, None]).T @ V
    assert np.abs(M - np.eye(b.nb)).max() < 1e-13
    assert np.abs(V[:, 0] - 1.0).max() < 1e-14
    x = np.array([[0.21, 0.13, 0.33]])
    e = 1e-6
    g = b.grads(x)[0]
    fd = np.stack([(b.values(x + e * np.eye(3)[i]) - b.values(x - e * np.eye(3)[i]))[0] / (2 * e)
                   for i in range(3)], axis=-1)
    assert np.abs(g - fd).max() < 1e-7


@pytest.mark.parametrize("k", [1, 2, 3])
def test_volume_rule_symmetric_exact_positive(k):
    """The operator's volume rule: exact for every monomial of degree <= 2k (k = 2:
    5, which makes the 14-point rule unique) in the barycentric coordinates (mean
    6 a! b! c! d! / (a + b + c + d + 3)!), mapped onto itself by every permutation
    of the vertices, positive weights, points inside; 4, 14, 24 points.  In
    reference coordinates it integrates the monomials of the reference
    tetrahedron exactly too."""
    P, W = symmetric_tet_rule(k)
    assert len(W) == {1: 4, 2: 14, 3: 24}[k]
    assert tet_rule_degree(k) == {1: 2, 2: 5, 3: 6}[k]
    assert (W > 0).all() and (P > 0).all() and abs(W.sum() - 1.0) < 1e-15
    f = math.factorial
    for d in range(tet_rule_degree(k) + 1):
        for a in range(d + 1):
            for b in range(d - a + 1):
                for c in range(d - a - b + 1):
                    e = d - a - b - c
                    got = np.sum(W * P[:, 0] ** a * P[:, 1] ** b * P[:, 2] ** c * P[:, 3] ** e)
                    assert abs(got - 6.0 * f(a) * f(b) * f(c) * f(e) / f(d + 3)) < 1e-15
    for perm in permutations(range(4)):
        Q = P[:, list(perm)]
        for q, wq in zip(Q, W):
            i = np.argmin(np.abs(P - q).sum(axis=1))
            assert np.abs(P[i] - q).max() < 1e-15 and abs(W[i] - wq) < 1e-16
    p, w = tet_volume_rule(k)
    for d in range(tet_rule_degree(k) + 1):
        for a in range(d + 1):
            for b in range(d - a + 1):
                c = d - a - b
                got = 6.0 * np.sum(w * p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** c)
                assert abs(got - _tet_monomial_mean(a, b, c)) < 1e-14, (a, b, c)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_face_rule_symmetric_exact_positive(k):
    """Exact for every monomial of degree <= 2k in the barycentric coordinates
    (mean 2 a! b! c! / (a + b + c + 2)!), mapped onto itself by every permutation
    of the vertices, positive weights, points inside the triangle."""
    P, W = symmetric_face_rule(k)
    assert len(W) == {1: 3, 2: 6, 3: 12}[k]
    assert (W > 0).all() and (P > 0).all() and abs(W.sum() - 1.0) < 1e-15
    f = math.factorial
    for d in range(2 * k + 1):
        for a in range(d + 1):
            for b in range(d - a + 1):
                c = d - a - b
                got = np.sum(W * P[:, 0] ** a * P[:, 1] ** b * P[:, 2] ** c)
                assert abs(got - 2.0 * f(a) * f(b) * f(c) / f(a + b + c + 2)) < 1e-15
    for perm in permutations(range(3)):
        Q = P[:, list(perm)]
        for q, wq in zip(Q, W):
            i = np.argmin(np.abs(P - q).sum(axis=1))
            assert np.abs(P[i] - q).max() < 1e-15 and W[i] == wq


def test_kuhn_tet_mesh_tables():
    xyz, vid, nbr, nbe = inputs.kuhn_tet_mesh(3, 4, 2, 0.2)
    E = len(xyz)
    assert E == 6 * 3 * 4 * 2
    for e in range(E):
        for f in range(4):
            g = nbr[e, f]
            if g >= 0:
                assert nbr[g, nbe[e, f]] == e and nbe[g, nbe[e, f]] == f
                # the same three vertices, and the same points up to a periodic shift
                mine = {int(vid[e, v]): xyz[e, v] for v in FACE_VERTS[f]}
                theirs = {int(vid[g, v]): xyz[g, v] for v in FACE_VERTS[nbe[e, f]]}
                assert set(mine) == set(theirs)
                shifts = [mine[i] - theirs[i] for i in mine]
                for s in shifts:
                    assert np.abs(s - shifts[0]).max() < 1e-14
                    assert np.abs(s[:2] - np.round(s[:2])).max() < 1e-14 and abs(s[2]) < 1e-14
    assert (nbr == -1).sum() == 2 * 3 * 4 and (nbr == -2).sum() == 2 * 3 * 4
    m = TetMesh(xyz, vid, nbr, nbe)
    assert abs(m.vol.sum() - 1.0) < 1e-14
    # Gamma1 faces lie on z = 0 with outward normal -e_z, Gamma2 on z = 1
    for code, z, nz in ((-1, 0.0, -1.0), (-2, 1.0, 1.0)):
        e, f = np.where(nbr == code)
        for ee, ff in zip(e, f):
            assert np.abs(xyz[ee, list(FACE_VERTS[ff]), 2] - z).max() < 1e-15
            assert abs(m.n[ee, ff, 2] - nz) < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3])
def test_constant_state_has_no_flux(k):
    """A constant state: every flux term vanishes (no inflow: beta = sigma = 0),
    leaving S(U) in mode 0 only."""
    m = mesh(3, 3, 2, 0.25)
    c = inputs.base_coeffs()
    c.update(beta1=0.0, beta2=0.0, sigma=0.0)
    o = TetOracle(m, k, c)
    vals = [0.6, 0.4, 0.3, 0.5, 0.2, 0.45]
    U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
    for s, v in enumerate(vals):
        U[s, :, 0] = v
    f = o.apply(U)
    n1, n2, n3, c1, c2, c3 = vals
    S = [-c["d1"] * n1, -c["d2"] * n2, c["d1"] * n1 + c["d2"] * n2 - c["gamma"] * n1,
         -c["alpha1"] * n1 * c1 - c["alpha2"] * n2 * c1 + c["f1"] * n3, -c["k"] * c2, c["k"] * c2]
    assert f[:, :, 1:].abs().max() < 1e-12
    for s in range(6):
        assert (f[s, :, 0] - S[s]).abs().max() < 1e-13


@pytest.mark.parametrize("k", [1, 2])
def test_diffusion_form_symmetric_negative_semidefinite(k):
    m = mesh(3, 3, 1, 0.3)
    o = TetOracle(m, k, diffusion(0.7))
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
    m = mesh(3, 3, 2, 0.2)
    o = TetOracle(m, k, diffusion(0.3))
    U = torch.from_numpy(inputs.tet_modes(m.E, k, key=(19,), amp=0.1))
    f = o.apply(U)
    tot = (f[:, :, 0] * o.vol[None, :]).sum(1)
    assert tot.abs().max() < 1e-13


def test_inflow_integrals():
    """Only the inflow fluxes: total n1 production mu1 beta1 |Gamma1|, n2
    production mu2 beta2 |Gamma2|, c2 production nu2 sigma |Gamma1,in|; with the
    face rule's points on a 3x3 grid of cube faces and Gamma1,in = [0, 1/3 + eps]
    exactly one column of cubes' faces counts, |Gamma1,in| = 1/3."""
    m = mesh(3, 3, 1)
    c = diffusion(0.0)
    c.update(beta1=0.7, beta2=0.4, sigma=0.9, mu1=0.5, mu2=0.25, nu2=0.3, c1_star=0.0, c1_sstar=0.0)
    o = TetOracle(m, 1, c, gamma1_in=(0.0, 1.0 / 3.0 + 1e-12))
    U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
    U[:, :, 0] = 0.5
    f = o.apply(U)
    tot = (f[:, :, 0] * o.vol[None, :]).sum(1)
    assert abs(float(tot[0]) - 0.5 * 0.7) < 1e-14
    assert abs(float(tot[1]) - 0.25 * 0.4) < 1e-14
    assert abs(float(tot[4]) - 0.3 * 0.9 / 3.0) < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3])
def test_diffusion_energy_equals_the_cdg2_form_with_the_k_minus_lifting(k):
    """-<U, R(U)> (one species, pure diffusion) equals the CDG2 form assembled
    here independently, sum_K int a |grad u|^2 - 2 sum_e int_e a {grad u}.n^- [u]
    + 4 chi_e sum_e int_{K^-} a |r_e|^2 with chi_e = 2 and the lifting of each
    face's jump solved on K^- in a physical monomial basis (mass matrix from a
    higher-order rule, face integrals with a Gauss product rule on the face)."""
    a = 0.7
    m = mesh(3, 3, 1, 0.3)
    o = TetOracle(m, k, diffusion(a))
    rng = np.random.default_rng(40 + k)
    U = torch.zeros(6, m.E, o.nb, dtype=torch.float64)
    U[0] = torch.from_numpy(rng.standard_normal((m.E, o.nb)))
    form_oracle = -float((U[0] * o.residual(U)[0]).sum())
    basis = TetBasis(k)
    xyz, vid, nbr, nbe = m.xyz, m.vid, m.nbr, m.nbe
    J = [np.column_stack([xyz[e, i] - xyz[e, 0] for i in (1, 2, 3)]) for e in range(m.E)]
    vol = np.array([abs(np.linalg.det(Je)) / 6.0 for Je in J])
    coef = U[0].numpy()

    def u_and_grad(e, X):
        ref = np.linalg.solve(J[e], (X - xyz[e, 0]).T).T
        val = basis.values(ref) @ coef[e]
        g = np.einsum("njb,j->nb", basis.grads(ref), coef[e]) @ np.linalg.inv(J[e])
        return val, g

    rp, rw = _stroud_rule(k + 3)
    vterm = 0.0
    for e in range(m.E):
        X = xyz[e, 0] + rp @ J[e].T
        _, g = u_and_grad(e, X)
        vterm += a * 6.0 * vol[e] * np.sum(rw * np.sum(g * g, axis=1))
    pw = [(d - b - c, b, c) for d in range(k + 1) for c in range(d + 1) for b in range(d - c + 1)]

    def mono(X, x0):
        Y = X - x0
        return np.stack([Y[:, 0] ** i * Y[:, 1] ** j * Y[:, 2] ** l for i, j, l in pw], axis=1)

    # Gauss product rule on the triangle (collapsed), barycentric points
    gx, gw = _gauss01(k + 3)
    tb, tw = [], []
    for i in range(len(gx)):
        for j in range(len(gx)):
            l2, l3 = gx[i], gx[j] * (1 - gx[i])
            tb.append((1 - l2 - l3, l2, l3))
            tw.append(2.0 * gw[i] * gw[j] * (1 - gx[i]))
    tb, tw = np.array(tb), np.array(tw)
    face, lift = 0.0, 0.0
    for e in range(m.E):
        for f in range(4):
            g = nbr[e, f]
            if g < 0 or (g, nbe[e, f]) < (e, f):
                continue
            vs = FACE_VERTS[f]
            A, B, C = (xyz[e, v] for v in vs)
            cr = np.cross(B - A, C - A)
            area = 0.5 * np.linalg.norm(cr)
            n_e = cr / (2 * area)
            if np.dot(n_e, A - xyz[e, f]) < 0:
                n_e = -n_e
            Xe = tb @ np.array([A, B, C])
            gvs = FACE_VERTS[nbe[e, f]]
            pos = {int(vid[g, v]): xyz[g, v] for v in gvs}
            Xg = tb @ np.array([pos[int(vid[e, v])] for v in vs])
            ue, ge = u_and_grad(e, Xe)
            ug, gg = u_and_grad(g, Xg)
            e_minus = vol[e] < vol[g] or (vol[e] == vol[g] and e < g)
            km, nm_, Xm = (e, n_e, Xe) if e_minus else (g, -n_e, Xg)
            jump = (ue - ug) if e_minus else (ug - ue)
            avg_n = 0.5 * ((ge + gg) @ nm_)
            face += -2.0 * a * area * np.sum(tw * avg_n * jump)
            x0 = xyz[km].mean(axis=0)
            Xq = xyz[km, 0] + rp @ J[km].T
            Vq = mono(Xq, x0)
            Mk = (Vq * (rw * 6.0 * vol[km])[:, None]).T @ Vq
            Vf = mono(Xm, x0)
            r2 = 0.0
            for comp in range(3):
                rhs = -0.5 * area * (Vf * (tw * jump * nm_[comp])[:, None]).sum(axis=0)
                rc = np.linalg.solve(Mk, rhs)
                r2 += rc @ Mk @ rc
            lift += 4.0 * 2.0 * a * r2
    form_here = vterm + face + lift
    assert abs(form_oracle - form_here) <= 1e-11 * abs(form_here), (form_oracle, form_here)
    assert abs(lift) > 1e-3 * abs(form_here)


@pytest.mark.parametrize("k,Ns,rate", [(1, (4, 8), 1.7), (2, (3, 6), 2.5)])
def test_l2_convergence_on_heat_solution(k, Ns, rate):
    """u = 0.5 + 0.2 exp(-a pi^2 (4 + 4 + 1) t) cos(2 pi x) cos(2 pi y) cos(pi z)
    solves u_t = a lap u, periodic in x, y, zero normal derivative on the walls;
    the L2 error after SSP-RK3 to T falls at about the order k + 1 (measured
    rates, still pre-asymptotic on these coarse meshes: 1.78 for P1 from 4 to 8
    cubes per side, 2.61 for P2 from 3 to 6; 2.72 for P2 from 4 to 8 and 3.59
    for P3 from 3 to 6 are too slow for this suite)."""
    a, T = 0.05, 0.005
    lam = a * math.pi ** 2 * 9

    def exact(t):
        def f(x, y, z):
            u = 0.5 + 0.2 * math.exp(-lam * t) * np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y) * np.cos(np.pi * z)
            return np.broadcast_to(u, (6,) + u.shape)
        return f

    errs = []
    for n in Ns:
        m = mesh(n, n, n, 0.1)
        o = TetOracle(m, k, diffusion(a))
        U = o.project(exact(0.0))
        h = 1.0 / n
        steps = int(math.ceil(T / (0.05 * h * h / (a * (k + 1) ** 4))))
        U = o.rk_step(U, T / steps, steps)
        errs.append(o.l2_error(U, exact(T)))
    assert errs[0] / errs[1] > 2 ** rate, errs
