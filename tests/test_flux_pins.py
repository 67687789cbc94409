"""Pins of the oracle's comparison diffusion fluxes (BR2, interior penalty,
Baumann-Oden, compact DG) against the mathematics.  On uniform Cartesian cells the lifting
of a face jump has the same trace on both neighbours, so BR2 with eta = N and
the interior penalty with eta = d reproduce CDG2; Baumann-Oden drops the
stabilisation and flips the symmetry term, which makes its quadratic form the
broken energy sum_K int a |grad u|^2; compact DG (switch on K^-) has the quadratic
form of the lifted gradient, sum_K int a |grad u + sum_e r~_e|^2 over the faces
whose K^- is K."""
import dataclasses
import math

import pytest
import torch

from oracle.cdg2_oracle import Config, Oracle, diffusion_only_coeffs
from paper_1403_1157_amd import inputs

DT = torch.float64


def rand_state(o, seed=0):
    g = torch.Generator().manual_seed(seed)
    U = 0.05 * (2 * torch.rand(6, o.E, o.nm, generator=g, dtype=DT) - 1)
    U[:, :, 0] = 0.3 + 0.4 * torch.rand(6, o.E, generator=g, dtype=DT)
    return U


def strong():
    c = inputs.base_coeffs()
    c.update(chi0_11=0.05, chi0_13=0.03, chi0_21=0.04, chi0_22=0.02)
    return c


@pytest.mark.parametrize("dim,n,p", [(2, (4, 3), 1), (2, (3, 4), 3), (3, (3, 2, 3), 2)])
def test_br2_and_ip_reduce_to_cdg2_on_uniform_cells(dim, n, p):
    cfg = Config(dim=dim, n=n, order=p, coeffs=strong())
    U = rand_state(Oracle(cfg), dim + p)
    ref = Oracle(cfg).apply(U)
    scale = float(ref.abs().max())
    br2 = Oracle(dataclasses.replace(cfg, diff_flux="br2", flux_eta=2 * dim)).apply(U)
    ip = Oracle(dataclasses.replace(cfg, diff_flux="ip", flux_eta=dim)).apply(U)
    assert float((br2 - ref).abs().max()) < 1e-13 * scale
    assert float((ip - ref).abs().max()) < 1e-13 * scale
    # a different penalty changes the operator
    ip2 = Oracle(dataclasses.replace(cfg, diff_flux="ip", flux_eta=2 * dim)).apply(U)
    assert float((ip2 - ref).abs().max()) > 1e-3 * scale


def _matrix(cfg):
    o = Oracle(cfg)
    return o, o.assemble()     # matrix of -R around 0 (the diffusion form)


def test_interior_penalty_form_is_symmetric_psd_with_constant_null_space():
    cfg = Config(dim=2, n=(3, 3), order=2, wall_axis=-1, coeffs=diffusion_only_coeffs(1.0),
                 diff_flux="ip", flux_eta=4.0)
    o, A = _matrix(cfg)
    assert torch.allclose(A, A.T, atol=1e-10 * float(A.abs().max()))
    ev = torch.linalg.eigvalsh(0.5 * (A + A.T))
    tol = 1e-10 * float(ev.abs().max())
    assert float(ev.min()) > -tol
    assert int((ev.abs() < tol).sum()) == 6          # one constant per species


def test_baumann_oden_form_is_the_broken_energy():
    """u^T A u = sum_K int a |grad u|^2 for every u (the face terms cancel)."""
    a = 0.7
    cfg = Config(dim=2, n=(3, 4), order=2, wall_axis=-1, coeffs=diffusion_only_coeffs(a),
                 diff_flux="bo")
    o, A = _matrix(cfg)
    assert float((A - A.T).abs().max()) > 1e-3 * float(A.abs().max())   # not symmetric
    for seed in range(3):
        u = rand_state(o, seed)
        quad = float(u.reshape(-1) @ (A @ u.reshape(-1)))
        g = torch.einsum("sem,qmg->seqg", u, o.dPhi)
        energy = float(a * torch.einsum("q,seqg->", o.wq, g * g))
        assert abs(quad - energy) < 1e-11 * energy


def test_compact_dg_form_is_the_energy_of_the_lifted_gradient():
    """CDG (one-sided on K^-, lifting of the whole jump onto K^-): for every u,
    u^T A u = sum_K int_K a |grad u + sum_{e: K = K^-_e} r~_e|^2 with
    int_K r~_e . tau = -int_e (u^- - u^+) n^- . tau (here: r~_e = n^- rho,
    rho = -(1/|K|) sum_m phi_m int_e (u^- - u^+) phi_m for the orthonormal modes).
    Liftings of different axes are orthogonal, so the form is semidefinite; a
    wrong side, weight or lifting factor breaks the identity."""
    a = 0.6
    for dim, n, p in [(2, (3, 4), 2), (3, (3, 3, 2), 1)]:
        cfg = Config(dim=dim, n=n, order=p, wall_axis=-1, coeffs=diffusion_only_coeffs(a), diff_flux="cdg")
        o, A = _matrix(cfg)
        assert float((A - A.T).abs().max()) < 1e-11 * float(A.abs().max())
        for seed in range(2):
            u = rand_state(o, seed)
            quad = float(u.reshape(-1) @ (A @ u.reshape(-1)))
            g = torch.einsum("sem,qmg->seqg", u, o.dPhi)               # grad u at the volume points
            UG = o.grid(u)
            lifted = g.clone()
            for ax in range(dim):
                F = o.faces[ax]
                Up = torch.roll(UG, shifts=-1, dims=o.gdim(ax, 1))     # the K^+ neighbour
                jump = torch.einsum("s...m,tm->s...t", UG, F["PhiHi"]) - torch.einsum("s...m,tm->s...t", Up, F["PhiLo"])
                rho = -torch.einsum("t,s...t,tm->s...m", F["wf"], jump, F["PhiHi"]) / o.vol
                lifted[..., ax] = lifted[..., ax] + torch.einsum("sem,qm->seq", o.flat(rho), o.Phi)
            energy = float(a * torch.einsum("q,seqg->", o.wq, lifted * lifted))
            assert abs(quad - energy) < 1e-11 * energy, (quad, energy)


@pytest.mark.parametrize("flux,eta,p,rho_mult", [("ip", 4.0, 1, 2.0), ("ip", 4.0, 2, 2.0), ("bo", 0.0, 1, 1.0),
                                                 ("cdg", 0.0, 1, 1.0), ("cdg", 0.0, 2, 1.0)])
def test_comparison_fluxes_heat_equation_eoc(flux, eta, p, rho_mult):
    """The exact heat solution of the CDG2 pin: IP and CDG converge with order
    p+1, Baumann-Oden with odd p = 1 with order 2."""
    a, A0 = 0.05, 0.2
    lam = a * math.pi ** 2 * (4 + 1)
    rho_hat = {1: 84.0, 2: 362.06}[p] * rho_mult

    def exact(t):
        def f(x):
            v = 0.5 + A0 * math.exp(-lam * t) * torch.cos(2 * math.pi * x[..., 0]) * torch.cos(math.pi * x[..., 1])
            return torch.stack([v] * 6)
        return f

    errs = []
    T = 0.02
    for N in (8, 16):
        o = Oracle(Config(dim=2, n=(N, N), order=p, coeffs=diffusion_only_coeffs(a), diff_flux=flux,
                          flux_eta=eta))
        U = o.project(exact(0.0))
        rho = o.d * rho_hat * a * N * N
        nst = int(math.ceil(T / (0.4 * 2.51 / rho)))
        U = o.rk_step(U, T / nst, nst)
        errs.append(o.l2_error(U, exact(T)))
    eoc = float(torch.log2(errs[0] / errs[1]).min())
    assert abs(eoc - (p + 1)) < 0.25, eoc


def test_heat_solution_inputs_are_the_projection_of_the_exact_solution():
    """The benchmark's heat-solution modes (numpy, inputs module) against the
    oracle's L2 projection of the same function."""
    a, t = 0.05, 0.013
    n, p = (6, 5), 2
    U = torch.from_numpy(inputs.heat_modes(n, p, t, a))
    o = Oracle(Config(dim=2, n=n, order=p, coeffs=diffusion_only_coeffs(a)))

    def f(x):
        v = 0.5 + 0.2 * math.exp(-5 * math.pi ** 2 * a * t) * torch.cos(2 * math.pi * x[..., 0]) \
            * torch.cos(math.pi * x[..., 1])
        return torch.stack([v] * 6)

    assert float((U - o.project(f)).abs().max()) < 1e-14
    assert inputs.diffusion_only_coeffs(a) == diffusion_only_coeffs(a)
