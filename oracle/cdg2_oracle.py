"""Plain float64 CPU oracle of the CDG2 operator for the six-species plaque model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only the test-suite, the graft smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code, tables or constants with the HIP library.

What it computes (Girke, Kloefkorn, Ohlberger, "Efficient parallel simulation of
atherosclerotic plaque formation using higher order DG schemes"):

* the model of Section 2, eqs. (1)-(6), written in the vector form
  dU/dt = -div(F(U) - A grad U) + S(U) given at the end of Section 2;
* the discrete operator <phi, L_h(U)> = <phi, K_h(U)> + <phi, I_h(U)> of
  Section 3.1 (element integrals, surface integrals with averages and jumps,
  local Lax-Friedrichs convective flux, CDG2 diffusion flux with the lifting
  r_e formed on K^-_e and lift factor chi_e = N/2);
* f(U) = M^{-1} L_h(U) of Section 3.2;
* explicit SSP-RK3 (Shu-Osher form) used as the time integrator;
* the implicit DIRK integrator of Section 3.2 (SDIRK of order 2, 3, 4), each
  stage solved by Newton's method with the exact (autograd) Jacobian;
* a CFL time step.

Everything is evaluated by DIRECT quadrature sums (u(x_q) = sum_m U_m phi_m(x_q),
no sum-factorisation).  The lifting is computed the general way: assemble the mass
matrix of K^- by quadrature, Cholesky-solve, evaluate the trace.  The element mass
matrix is likewise assembled and solved, not assumed diagonal.  All arithmetic is
torch float64 on the CPU and differentiable, so torch.autograd gives the exact
discrete adjoint (vector-Jacobian products) of every function here.

Readings where the paper is silent or garbled:
  * grid: uniform Cartesian cells on [0,1]^d, tensor Legendre Q_p basis
    phi_i(xi) = sqrt(2i+1) P_i(2 xi - 1) per direction (orthonormal on [0,1]);
  * p+1 Gauss-Legendre points per direction for volume and face integrals;
  * K^-_e is the low-coordinate neighbour (uniform grid: the "smaller volume"
    rule of Section 3.1 is a tie everywhere);
  * chi_e = N/2 with N = 2d faces per cell (2 for quads, 3 for hexes);
  * the c1 row of S uses alpha2 n2 c1 (eq. (4)), not alpha2 n2 c2;
  * gamma := F is a constant (diseased state), f1 a constant;
  * the second chemotaxis term of the n2 equation has its own constants chi22;
  * inflow boundary conditions (eqs. (7)-(9)) are read as inflow fluxes
    mu1 beta1 H(c1-c1*), mu2 beta2 H(c1-c1**), nu2 sigma into the domain, with
    H(x) = 1 for x > 0 else 0, evaluated pointwise on the interior trace;
  * boundary faces carry only that Neumann flux (no lifting / average / LLF);
  * the LLF dissipation speed is the spectral radius of d(F.n)/dU, i.e.
    max(|w1.n|, |w2.n|) over both sides, applied to all six rows ("all") or only
    to the two cell rows ("cells");
  * F^:[[phi]] is read as (F^ n^-)(phi^- - phi^+);
  * the comparison fluxes of Section 4 (named there without their constants):
    BR2 eta {A r_e}, interior penalty eta A (p+1)^2/h [[U]], Baumann-Oden (no
    stabilisation, symmetry term of the opposite sign), and CDG read as the
    compact DG of Peraire and Persson with its switch on K^-: one-sided flux
    A (grad U^- + r~).n^- with the lifting r~ of the whole jump onto K^- and the
    symmetry term on K^- only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

DT = torch.float64
NSPEC = 6
N1, N2, N3, C1, C2, C3 = range(6)

# Coefficient vector order (26 entries; the first 21 are the differentiable
# diffusion / chemotaxis / reaction coefficients of Section 2).
COEFF_NAMES = [
    "mu1", "mu2", "mu3", "nu1", "nu2", "nu3",
    "chi0_11", "chi0_13", "chi0_21", "chi0_22",
    "chith_11", "chith_13", "chith_21", "chith_22",
    "d1", "d2", "gamma", "alpha1", "alpha2", "f1", "k",
    "beta1", "beta2", "sigma", "c1_star", "c1_sstar",
]
NCOEFF = len(COEFF_NAMES)
NDIFF = 21


@dataclass
class Config:
    dim: int = 2
    n: tuple = (16, 16)
    order: int = 1
    wall_axis: int = -2          # -2: default (last axis); -1: fully periodic
    gamma1_in: tuple = (0.0, 1.0)
    llf_mode: str = "all"        # "all" | "cells"
    coeffs: dict = field(default_factory=dict)
    diff_flux: str = "cdg2"      # "cdg2" | "br2" | "ip" | "bo" | "cdg" (diffusion flux, Section 3.1)
    flux_eta: float = 0.0        # penalty of br2 / ip; 0: default (br2: N = 2d, ip: 2d)

    def resolved_wall(self) -> int:
        return self.dim - 1 if self.wall_axis == -2 else self.wall_axis


# ---------------------------------------------------------------------------
# 1D tables (own implementation from the mathematics).
# ---------------------------------------------------------------------------

def legendre(n: int, x: torch.Tensor):
    """Legendre P_0..P_n and derivatives at x by the three-term (Bonnet) recurrence."""
    P = [torch.ones_like(x), x.clone()]
    for k in range(1, n):
        P.append(((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1))
    P = P[: n + 1]
    dP = [torch.zeros_like(x)]
    for k in range(1, n + 1):
        # P_k' = k (x P_k - P_{k-1}) / (x^2 - 1) is singular at the ends; use the
        # derivative recurrence P_k' = P_{k-2}' + (2k-1) P_{k-1} instead.
        prev2 = dP[k - 2] if k >= 2 else torch.zeros_like(x)
        dP.append(prev2 + (2 * k - 1) * P[k - 1])
    return P, dP


def gauss_legendre01(q: int):
    """q-point Gauss-Legendre rule mapped to [0,1]: Newton iteration on P_q started
    from the Chebyshev-like guess cos(pi (4j-1)/(4q+2))."""
    xs = []
    for j in range(1, q + 1):
        x = torch.tensor(math.cos(math.pi * (4 * j - 1) / (4 * q + 2)), dtype=DT)
        for _ in range(100):
            P, dP = legendre(q, x)
            dx = P[q] / dP[q]
            x = x - dx
            if abs(float(dx)) < 1e-17:
                break
        xs.append(float(x))
    x = torch.tensor(sorted(xs), dtype=DT)
    _, dP = legendre(q, x)
    w = 2.0 / ((1.0 - x * x) * dP[q] ** 2)
    return 0.5 * (x + 1.0), 0.5 * w


def basis1d(p: int, xi: torch.Tensor):
    """Orthonormal Legendre basis on [0,1]: phi_i(xi) = sqrt(2i+1) P_i(2xi-1),
    returned as [len(xi), p+1] values and d/dxi derivatives."""
    P, dP = legendre(p, 2.0 * xi - 1.0)
    val = torch.stack([math.sqrt(2 * i + 1) * P[i] for i in range(p + 1)], dim=-1)
    der = torch.stack([math.sqrt(2 * i + 1) * 2.0 * dP[i] for i in range(p + 1)], dim=-1)
    return val, der


def mode_multi_index(p: int, dim: int):
    """Mode m = i + (p+1) (j + (p+1) k): x index fastest."""
    q = p + 1
    out = []
    for m in range(q ** dim):
        idx, r = [], m
        for _ in range(dim):
            idx.append(r % q)
            r //= q
        out.append(idx)
    return out


def eval_basis(p: int, dim: int, xi: torch.Tensor, h):
    """All (p+1)^dim tensor basis functions and their physical gradients at the
    reference points xi [N, dim] of a cell with side lengths h."""
    modes = mode_multi_index(p, dim)
    vals, ders = [], []
    for a in range(dim):
        v, d = basis1d(p, xi[:, a])
        vals.append(v)
        ders.append(d)
    N = xi.shape[0]
    Phi = torch.ones(N, len(modes), dtype=DT)
    for m, idx in enumerate(modes):
        for a in range(dim):
            Phi[:, m] = Phi[:, m] * vals[a][:, idx[a]]
    dPhi = torch.ones(N, len(modes), dim, dtype=DT)
    for m, idx in enumerate(modes):
        for g in range(dim):
            for a in range(dim):
                f = ders[a][:, idx[a]] / h[a] if a == g else vals[a][:, idx[a]]
                dPhi[:, m, g] = dPhi[:, m, g] * f
    return Phi, dPhi


def tensor_points(x1: torch.Tensor, w1: torch.Tensor, dim: int):
    """Tensor rule on [0,1]^dim, x index fastest."""
    q = x1.shape[0]
    pts, wts = [], []
    for n in range(q ** dim):
        idx, r = [], n
        for _ in range(dim):
            idx.append(r % q)
            r //= q
        pts.append([float(x1[i]) for i in idx])
        wts.append(math.prod(float(w1[i]) for i in idx))
    return torch.tensor(pts, dtype=DT), torch.tensor(wts, dtype=DT)


# ---------------------------------------------------------------------------
# The operator.
# ---------------------------------------------------------------------------

def coeff_vector(c) -> torch.Tensor:
    if isinstance(c, torch.Tensor):
        return c
    return torch.tensor([float(c[k]) for k in COEFF_NAMES], dtype=DT)


class Oracle:
    """Direct-sum oracle on a uniform Cartesian grid of [0,1]^dim."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        d, p = cfg.dim, cfg.order
        assert d in (2, 3) and 1 <= p
        self.d, self.p, self.q = d, p, p + 1
        self.n = tuple(int(v) for v in cfg.n)[:d]
        self.h = [1.0 / v for v in self.n]
        self.E = math.prod(self.n)
        self.nm = (p + 1) ** d
        self.wall = cfg.resolved_wall()
        self.chi_e = float(d)             # N/2 with N = 2d faces per cell
        assert cfg.diff_flux in ("cdg2", "br2", "ip", "bo", "cdg")
        self.flux_eta = float(cfg.flux_eta) if cfg.flux_eta > 0 else float(2 * d)
        self.vol = math.prod(self.h)
        x1, w1 = gauss_legendre01(self.q)
        self.x1, self.w1 = x1, w1
        # Volume quadrature (p+1 points per direction).
        xq, wq = tensor_points(x1, w1, d)
        self.wq = wq * self.vol
        self.Phi, self.dPhi = eval_basis(p, d, xq, self.h)
        # Element mass matrix assembled by quadrature.
        self.M = torch.einsum("q,qm,qn->mn", self.wq, self.Phi, self.Phi)
        self.Mchol = torch.linalg.cholesky(self.M)
        # Face tables per axis: tangential points, weights, traces on both sides.
        self.faces = []
        for a in range(d):
            tang = [b for b in range(d) if b != a]
            xt, wt = tensor_points(x1, w1, d - 1)
            area = math.prod(self.h[b] for b in tang)
            hi = torch.zeros(xt.shape[0], d, dtype=DT)
            lo = torch.zeros(xt.shape[0], d, dtype=DT)
            for j, b in enumerate(tang):
                hi[:, b] = xt[:, j]
                lo[:, b] = xt[:, j]
            hi[:, a] = 1.0
            lo[:, a] = 0.0
            PhiHi, dPhiHi = eval_basis(p, d, hi, self.h)
            PhiLo, dPhiLo = eval_basis(p, d, lo, self.h)
            self.faces.append(dict(tang=tang, xt=xt, wf=wt * area, PhiHi=PhiHi,
                                   dPhiHi=dPhiHi, PhiLo=PhiLo, dPhiLo=dPhiLo))

    # -- grid helpers -------------------------------------------------------
    def grid(self, X: torch.Tensor) -> torch.Tensor:
        """[..., E, k] -> [..., n_{d-1}, ..., n_0, k] (x fastest)."""
        lead = X.shape[:-2]
        return X.reshape(*lead, *reversed(self.n), X.shape[-1])

    def flat(self, G: torch.Tensor) -> torch.Tensor:
        lead = G.shape[: -(self.d + 1)]
        return G.reshape(*lead, self.E, G.shape[-1])

    def gdim(self, a: int, lead: int) -> int:
        """Tensor dim of grid axis a (x = axis 0 is the last grid dim)."""
        return lead + (self.d - 1 - a)

    def cell_coords(self):
        """Lower-left corner of each cell, [E, d]."""
        idx = torch.arange(self.E)
        out = torch.zeros(self.E, self.d, dtype=DT)
        r = idx.clone()
        for a in range(self.d):
            out[:, a] = (r % self.n[a]).to(DT) * self.h[a]
            r = r // self.n[a]
        return out

    # -- pointwise physics (Section 2) ---------------------------------------
    @staticmethod
    def chi(x, y, a, b):
        """Tactic sensitivity chi(x, y, a, b) = a x / (y + b)."""
        return a * x / (y + b)

    def velocities(self, u, g, th):
        """Chemotactic velocities: F_n1 = n1 w1, F_n2 = n2 w2 (vector form of eqs.
        (1)-(2)); u [6, ...], g [6, ..., d] (gradient components)."""
        chi11 = th[6] / (u[C1] + th[10])
        chi13 = th[7] / (u[C3] + th[11])
        chi21 = th[8] / (u[C1] + th[12])
        chi22 = th[9] / (u[N1] + th[13])
        w1 = chi11[..., None] * g[C1] + chi13[..., None] * g[C3]
        w2 = chi21[..., None] * g[C1] - chi22[..., None] * g[N1]
        return w1, w2

    def source(self, u, th):
        """S(U) of Section 2 with the c1 row of eq. (4)."""
        n1, n2, n3, c1, c2, c3 = u
        d1, d2, gam, al1, al2, f1, k = th[14], th[15], th[16], th[17], th[18], th[19], th[20]
        return torch.stack([
            -d1 * n1,
            -d2 * n2,
            d1 * n1 + d2 * n2 - gam * n1,
            -al1 * n1 * c1 - al2 * n2 * c1 + f1 * n3,
            -k * c2,
            k * c2,
        ])

    def diffusivities(self, th):
        return th[0:6]

    # -- L_h ------------------------------------------------------------------
    def residual(self, U: torch.Tensor, theta=None, forcing=None) -> torch.Tensor:
        """<phi_j, L_h(U)> for every basis function: [6, E, nm].

        ``forcing`` (tests only) is an optional callable x[..., d] -> [6, ...]
        added to S, for manufactured solutions."""
        cfg, d = self.cfg, self.d
        th = coeff_vector(cfg.coeffs if theta is None else theta)
        a = self.diffusivities(th)
        # ---- element integrals K_h (Section 3.1) ----
        u = torch.einsum("sem,qm->seq", U, self.Phi)                 # [6,E,Q]
        g = torch.einsum("sem,qmg->seqg", U, self.dPhi)              # [6,E,Q,d]
        w1, w2 = self.velocities(u, g, th)
        Fc = torch.stack([u[N1][..., None] * w1, u[N2][..., None] * w2]
                         + [torch.zeros_like(w1)] * 4)
        flux = Fc - a[:, None, None, None] * g                       # F - A grad U
        S = self.source(u, th)
        if forcing is not None:
            xq = self.cell_coords()[:, None, :] + self._xq_ref()[None, :, :] * torch.tensor(self.h, dtype=DT)
            S = S + forcing(xq)
        R = torch.einsum("q,seqg,qmg->sem", self.wq, flux, self.dPhi) \
            + torch.einsum("q,seq,qm->sem", self.wq, S, self.Phi)
        # ---- surface integrals I_h ----
        RG = self.grid(R)
        UG = self.grid(U)
        for ax in range(d):
            RG = RG + self._faces_axis(UG, th, a, ax)
        R = self.flat(RG)
        return R

    def _xq_ref(self):
        xq, _ = tensor_points(self.x1, self.w1, self.d)
        return xq

    def _faces_axis(self, UG, th, a, ax):
        """Contributions of all faces normal to axis ``ax`` to the residual."""
        d, F = self.d, self.faces[ax]
        dim = self.gdim(ax, 1)
        periodic = ax != self.wall
        Um = UG
        Up = torch.roll(UG, shifts=-1, dims=dim)                     # cell i+1
        # traces at the face points of the face between cell i (K-) and i+1 (K+)
        um = torch.einsum("s...m,tm->s...t", Um, F["PhiHi"])
        up = torch.einsum("s...m,tm->s...t", Up, F["PhiLo"])
        gm = torch.einsum("s...m,tmg->s...tg", Um, F["dPhiHi"])
        gp = torch.einsum("s...m,tmg->s...tg", Up, F["dPhiLo"])
        # n^- = +e_ax: normal components
        dnm = gm[..., ax]
        dnp = gp[..., ax]
        # jump u^- - u^+, formed basis function by basis function: the constant mode
        # (phi_0 = 1 on both sides) cancels exactly, so the O(1) cell means do not
        # leave their rounding in the small jump (same value in exact arithmetic).
        jump = (Um[..., 0] - Up[..., 0]).unsqueeze(-1) \
            + torch.einsum("s...m,tm->s...t", Um[..., 1:], F["PhiHi"][:, 1:]) \
            - torch.einsum("s...m,tm->s...t", Up[..., 1:], F["PhiLo"][:, 1:])
        # LLF (Section 3.1): F^ n = 1/2 (F^- + F^+).n + 1/2 lam (u^- - u^+)
        w1m, w2m = self.velocities(um, gm, th)
        w1p, w2p = self.velocities(up, gp, th)
        w1m, w2m, w1p, w2p = w1m[..., ax], w2m[..., ax], w1p[..., ax], w2p[..., ax]
        lam = torch.maximum(torch.maximum(w1m.abs(), w2m.abs()),
                            torch.maximum(w1p.abs(), w2p.abs()))
        Fn = torch.stack([0.5 * (um[N1] * w1m + up[N1] * w1p),
                          0.5 * (um[N2] * w2m + up[N2] * w2p)]
                         + [torch.zeros_like(w1m)] * 4)
        if self.cfg.llf_mode == "all":
            Fhat = Fn + 0.5 * lam[None] * jump
        else:
            diss = torch.cat([0.5 * lam[None] * jump[:2], torch.zeros_like(jump[2:])])
            Fhat = Fn + diss
        # consistency average {A grad U}.n^- (CDG: one-sided, the K^- value)
        ab = a.reshape(6, *([1] * (jump.dim() - 1)))
        flux = self.cfg.diff_flux
        avg = ab * dnm if flux == "cdg" else 0.5 * ab * (dnm + dnp)
        # diffusion stabilisation (the comparison fluxes of Section 4 share the
        # consistency term; they differ in the stabilisation and the symmetry term)
        if flux == "cdg2":
            # CDG2: lifting on K^- (general route: mass solve on K^-)
            Ahat = 2.0 * self.chi_e * ab * self.lift_trace(jump, ax)
        elif flux == "br2":
            # BR2: eta times the average of the liftings on K^- and K^+
            rbar = 0.5 * (self.lift_trace(jump, ax) + self.lift_trace_plus(jump, ax))
            Ahat = self.flux_eta * ab * rbar
        elif flux == "ip":
            # interior penalty: eta a (p+1)^2 / h [[U]]
            Ahat = -self.flux_eta * ab * (self.p + 1) ** 2 / self.h[ax] * jump
        elif flux == "cdg":
            # compact DG with the switch on K^-: the lifting of the whole jump onto
            # K^- only, int_{K^-} r~ . tau = -int_e [[V]] . tau (twice the half-jump
            # lifting of lift_trace), and no average
            Ahat = 2.0 * ab * self.lift_trace(jump, ax)
        else:
            # Baumann-Oden: no stabilisation, symmetry term with the opposite sign
            Ahat = torch.zeros_like(jump)
        gflux = avg - Fhat + Ahat                                    # multiplies (phi^- - phi^+)
        sym = 0.5 * ab * jump                                        # multiplies dn phi (both sides)
        if flux == "bo":
            sym = -sym
        sym_m, sym_p = sym, sym
        if flux == "cdg":
            # one-sided symmetry term: on K^- only, with the whole jump
            sym_m, sym_p = 2.0 * sym, torch.zeros_like(sym)
        wf = F["wf"]
        # test functions on K- (trace at xi_ax = 1) and on K+ (xi_ax = 0)
        Rm = torch.einsum("t,s...t,tm->s...m", wf, gflux, F["PhiHi"]) \
            + torch.einsum("t,s...t,tm->s...m", wf, sym_m, F["dPhiHi"][..., ax])
        Rp = -torch.einsum("t,s...t,tm->s...m", wf, gflux, F["PhiLo"]) \
            + torch.einsum("t,s...t,tm->s...m", wf, sym_p, F["dPhiLo"][..., ax])
        if not periodic:
            # the face after the last cell along the wall axis does not exist
            n = self.n[ax]
            mask = torch.ones(n, dtype=DT)
            mask[n - 1] = 0.0
            shape = [1] * Rm.dim()
            shape[dim] = n
            mask = mask.reshape(shape)
            Rm = Rm * mask
            Rp = Rp * mask
        out = Rm + torch.roll(Rp, shifts=1, dims=dim)
        if not periodic:
            out = out + self._boundary(UG, th, ax)
        return out

    def lift_trace(self, jump: torch.Tensor, ax: int) -> torch.Tensor:
        """Normal component of the lifting r_e([[V]]) restricted to K^-, evaluated at
        the face points.  Definition (Section 3.1): for all tau in V_h^d,
        int_Omega r_e : tau = - int_e [[V]] : {tau}.  Restricted to K^- and the
        n-component: M_{K-} rho = -1/2 n^-_ax int_e (u^- - u^+) phi^{K-}."""
        F = self.faces[ax]
        b = -0.5 * torch.einsum("t,s...t,tm->s...m", F["wf"], jump, F["PhiHi"])
        shp = b.shape
        rho = torch.cholesky_solve(b.reshape(-1, self.nm).T, self.Mchol).T.reshape(shp)
        return torch.einsum("s...m,tm->s...t", rho, F["PhiHi"])

    def lift_trace_plus(self, jump: torch.Tensor, ax: int) -> torch.Tensor:
        """n^- component of the lifting r_e([[V]]) restricted to K^+, at the face
        points: M_{K+} rho = -1/2 n^-_ax int_e (u^- - u^+) phi^{K+}."""
        F = self.faces[ax]
        b = -0.5 * torch.einsum("t,s...t,tm->s...m", F["wf"], jump, F["PhiLo"])
        shp = b.shape
        rho = torch.cholesky_solve(b.reshape(-1, self.nm).T, self.Mchol).T.reshape(shp)
        return torch.einsum("s...m,tm->s...t", rho, F["PhiLo"])

    def _boundary(self, UG, th, ax):
        """Inflow boundary fluxes of eqs. (7)-(9) on Gamma1 (low end of the wall
        axis) and Gamma2 (high end)."""
        F = self.faces[ax]
        dim = self.gdim(ax, 1)
        n = self.n[ax]
        wf = F["wf"]
        # Gamma1: low face of the cells with index 0 along ax, interior trace at xi = 0
        U0 = UG.narrow(dim, 0, 1)
        c1m = torch.einsum("...m,tm->...t", U0[C1], F["PhiLo"])
        H1 = (c1m - th[24] > 0).to(DT)
        z = torch.zeros_like(H1)
        q1 = torch.stack([th[0] * th[21] * H1, z, z, z,
                          th[4] * th[23] * self._gamma1_in_mask(c1m.shape, ax), z])
        contrib0 = torch.einsum("t,s...t,tm->s...m", wf, q1, F["PhiLo"])
        # Gamma2: high face of the cells with index n-1, interior trace at xi = 1
        UN = UG.narrow(dim, n - 1, 1)
        c1p = torch.einsum("...m,tm->...t", UN[C1], F["PhiHi"])
        H2 = (c1p - th[25] > 0).to(DT)
        z = torch.zeros_like(H2)
        q2 = torch.stack([z, th[1] * th[22] * H2, z, z, z, z])
        contribN = torch.einsum("t,s...t,tm->s...m", wf, q2, F["PhiHi"])
        if n == 1:
            return contrib0 + contribN
        parts = [contrib0]
        if n > 2:
            parts.append(torch.zeros_like(UG.narrow(dim, 1, n - 2)))
        parts.append(contribN)
        return torch.cat(parts, dim=dim)

    def _gamma1_in_mask(self, shape, ax):
        """1 where the first tangential coordinate of a Gamma1 face point lies in
        Gamma_{1,in} = [g0, g1], else 0; ``shape`` = grid dims + [face points]."""
        F = self.faces[ax]
        g0, g1 = self.cfg.gamma1_in
        tang0 = F["tang"][0]
        dimt = self.gdim(tang0, 0)
        ncell = self.n[tang0]
        xt = F["xt"][:, 0]                          # reference coordinate along tang0
        x = (torch.arange(ncell, dtype=DT)[:, None] + xt[None, :]) * self.h[tang0]
        m = ((x >= g0) & (x <= g1)).to(DT)         # [ncell, T]
        view = [1] * len(shape)
        view[dimt] = ncell
        view[-1] = xt.shape[0]
        return m.reshape(view).expand(*shape)

    def apply(self, U: torch.Tensor, theta=None, forcing=None) -> torch.Tensor:
        """f(U) = M^{-1} L_h(U) (Section 3.2), [6, E, nm]."""
        R = self.residual(U, theta, forcing)
        shp = R.shape
        f = torch.cholesky_solve(R.reshape(-1, self.nm).T, self.Mchol).T
        return f.reshape(shp)

    # -- time stepping ---------------------------------------------------------
    def rk_step(self, U, dt, nsteps=1, theta=None, forcing_t=None, t0=0.0):
        """Explicit SSP-RK3 (Shu-Osher):
        U1 = U + dt f(U); U2 = 3/4 U + 1/4 (U1 + dt f(U1));
        U^{n+1} = 1/3 U + 2/3 (U2 + dt f(U2)).
        ``forcing_t`` (tests only): callable t -> forcing callable."""
        t = t0
        for _ in range(nsteps):
            fr = (lambda tt: None) if forcing_t is None else forcing_t
            U1 = U + dt * self.apply(U, theta, fr(t))
            U2 = 0.75 * U + 0.25 * (U1 + dt * self.apply(U1, theta, fr(t + dt)))
            U = U / 3.0 + (2.0 / 3.0) * (U2 + dt * self.apply(U2, theta, fr(t + 0.5 * dt)))
            t += dt
        return U

    # -- implicit DIRK (Section 3.2: DIRK of order 2-4 solved by Newton) --------
    def dirk_step(self, U, dt, order, tol=1e-13, maxit=60, theta=None):
        """One step of the L-stable, stiffly accurate SDIRK scheme of the given
        order (sdirk_tableau): for each stage i the stage value X_i solves
            X_i - dt a_ii f(X_i) = U^n + dt sum_{j<i} a_ij f(X_j),
        then U^{n+1} = U^n + dt sum_i b_i K_i with K_i = (X_i - rhs_i) / (dt a_ii)
        (= f(X_i) once the stage equation holds).  Each stage equation
        G(X) = X - dt a_ii f(X) - rhs = 0 is solved to
        ||G|| <= tol (||X|| + dt a_ii ||f(X)||) (2-norms over all modes: relative
        to the size of its terms) by Newton's method with the exact Jacobian of
        f (autograd), kept fixed within a stage and recomputed if the iteration
        stalls.  Returns (U^{n+1}, total Newton iterations)."""
        A, b, _ = sdirk_tableau(order)
        shape = U.shape
        n = U.numel()
        eye = torch.eye(n, dtype=DT)

        def jac(X):
            J = torch.autograd.functional.jacobian(
                lambda y: self.apply(y.reshape(shape), theta).reshape(-1), X.reshape(-1), vectorize=True)
            return J.reshape(n, n)

        K = []
        iters = 0
        for i in range(len(b)):
            rhs = U.clone()
            for j in range(i):
                rhs = rhs + dt * A[i][j] * K[j]
            g = A[i][i]
            X = rhs.clone()
            lu = None
            prev = None
            for _ in range(maxit):
                F = self.apply(X, theta)
                G = X - dt * g * F - rhs
                r = float(G.norm())
                if r <= tol * (float(X.norm()) + dt * g * float(F.norm())):
                    break
                if lu is None or (prev is not None and r > 0.5 * prev):
                    lu = torch.linalg.lu_factor(eye - dt * g * jac(X))
                prev = r
                d = torch.linalg.lu_solve(*lu, -G.reshape(-1, 1)).reshape(shape)
                X = X + d
                iters += 1
            else:
                raise RuntimeError("oracle DIRK stage did not converge")
            # stage derivative from the solved stage equation: equal to f(X_i) at
            # convergence, and free of dt-amplified rounding when dt is large
            K.append((X - rhs) / (dt * g))
        out = U.clone()
        for i in range(len(b)):
            out = out + dt * b[i] * K[i]
        return out, iters

    # -- CFL time step ----------------------------------------------------------
    def spectral_constant(self, ncell: int = 4) -> float:
        """rho_hat: spectral radius of M^{-1} K for the pure diffusion operator
        (a = 1) on a fully periodic ncell^d grid, times h^2 / d.  Computed
        matrix-free with a library Lanczos eigen-solver (scipy eigsh) on the
        oracle operator."""
        import numpy as np
        from scipy.sparse.linalg import LinearOperator, eigsh
        cfg = Config(dim=self.d, n=(ncell,) * self.d, order=self.p, wall_axis=-1,
                     coeffs=diffusion_only_coeffs(1.0))
        o = Oracle(cfg)
        shp = (NSPEC, o.E, o.nm)
        n = NSPEC * o.E * o.nm

        def mv(x):
            X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).reshape(shp)
            return (-o.apply(X)).reshape(-1).numpy()

        op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
        ev = eigsh(op, k=1, which="LA", tol=0, return_eigenvectors=False,
                   v0=np.random.default_rng(0).standard_normal(n))
        return float(ev[0]) * (1.0 / ncell) ** 2 / self.d

    def max_dt(self, U, cfl=0.9, rho_hat=None):
        """dt = cfl / (rho_hat a_max sum_a h_a^-2 / 2.51 + (2p+1) lam_max sum_a h_a^-1
        + r_max / 2.51); lam_max = max |w_i| components, r_max = d1 + d2 + |gamma|
        + k + alpha1 max n1 + alpha2 max n2 over the volume quadrature points."""
        th = coeff_vector(self.cfg.coeffs)
        if rho_hat is None:
            rho_hat = self.spectral_constant()
        u = torch.einsum("sem,qm->seq", U, self.Phi)
        g = torch.einsum("sem,qmg->seqg", U, self.dPhi)
        w1, w2 = self.velocities(u, g, th)
        lam = float(torch.maximum(w1.abs().max(), w2.abs().max()))
        amax = float(th[0:6].abs().max())
        rmax = float(th[14] + th[15] + th[16].abs() + th[20]
                     + th[17] * u[N1].max().clamp(min=0) + th[18] * u[N2].max().clamp(min=0))
        inv = (rho_hat * amax * sum(1.0 / hh ** 2 for hh in self.h) / 2.51
               + (2 * self.p + 1) * lam * sum(1.0 / hh for hh in self.h)
               + rmax / 2.51)
        return cfl / inv

    # -- assembly helpers -------------------------------------------------------
    def assemble(self, U0=None, theta=None) -> torch.Tensor:
        """Matrix of -R (the residual) with respect to U around U0 (zero by default),
        by applying the residual to unit vectors through autograd's Jacobian.
        Only for tiny grids."""
        n = NSPEC * self.E * self.nm
        if U0 is None:
            U0 = torch.zeros(NSPEC, self.E, self.nm, dtype=DT)
        J = torch.autograd.functional.jacobian(
            lambda x: self.residual(x.reshape(U0.shape), theta).reshape(-1), U0.reshape(-1))
        return -J.reshape(n, n)

    # -- projection / errors (tests) ------------------------------------------
    def project(self, func, extra=2):
        """L2 projection of func(x[..., d]) -> [6, ...] onto V_h, with
        p+1+extra Gauss points per direction: M^{-1} int func phi."""
        xg, wg = gauss_legendre01(self.q + extra)
        xq, wq = tensor_points(xg, wg, self.d)
        Phi, _ = eval_basis(self.p, self.d, xq, self.h)
        x = self.cell_coords()[:, None, :] + xq[None] * torch.tensor(self.h, dtype=DT)
        vals = func(x)                                          # [6, E, Q]
        b = torch.einsum("q,seq,qm->sem", wq * self.vol, vals, Phi)
        shp = b.shape
        return torch.cholesky_solve(b.reshape(-1, self.nm).T, self.Mchol).T.reshape(shp)

    def l2_error(self, U, func, species=None):
        """||u_h - func||_{L2(Omega)} per species, with a Gauss rule of order
        >= 2p+4 (p+3 points per direction)."""
        xg, wg = gauss_legendre01(self.p + 3)
        xq, wq = tensor_points(xg, wg, self.d)
        Phi, _ = eval_basis(self.p, self.d, xq, self.h)
        x = self.cell_coords()[:, None, :] + xq[None] * torch.tensor(self.h, dtype=DT)
        uh = torch.einsum("sem,qm->seq", U, Phi)
        ex = func(x)
        err = torch.einsum("q,seq->s", wq * self.vol, (uh - ex) ** 2).sqrt()
        return err if species is None else err[species]


def sdirk_tableau(order: int):
    """Butcher tableau (A, b, c) of an L-stable, stiffly accurate (b = last row
    of A) singly diagonally implicit Runge-Kutta scheme of the given order, for
    the DIRK integrator of Section 3.2 (the paper names only the orders):
      order 2: Alexander's two-stage scheme, gamma = 1 - 1/sqrt(2);
      order 3: Alexander's three-stage scheme, gamma the root in (1/6, 1/2) of
               x^3 - 3x^2 + 3x/2 - 1/6, c = (gamma, (1+gamma)/2, 1);
      order 4: the five-stage scheme of Hairer and Wanner with gamma = 1/4.
    Floats (float64); the order conditions are checked in the pins."""
    if order == 2:
        g = 1.0 - 1.0 / math.sqrt(2.0)
        A = [[g, 0.0], [1.0 - g, g]]
        c = [g, 1.0]
    elif order == 3:
        g = 0.4358665215
        for _ in range(50):     # Newton on the cubic
            g -= (g ** 3 - 3 * g ** 2 + 1.5 * g - 1.0 / 6.0) / (3 * g ** 2 - 6 * g + 1.5)
        b1 = -(6 * g * g - 16 * g + 1) / 4.0
        b2 = (6 * g * g - 20 * g + 5) / 4.0
        A = [[g, 0.0, 0.0], [(1 - g) / 2.0, g, 0.0], [b1, b2, g]]
        c = [g, (1 + g) / 2.0, 1.0]
    elif order == 4:
        A = [[1 / 4, 0, 0, 0, 0],
             [1 / 2, 1 / 4, 0, 0, 0],
             [17 / 50, -1 / 25, 1 / 4, 0, 0],
             [371 / 1360, -137 / 2720, 15 / 544, 1 / 4, 0],
             [25 / 24, -49 / 48, 125 / 16, -85 / 12, 1 / 4]]
        c = [1 / 4, 3 / 4, 11 / 20, 1 / 2, 1.0]
    else:
        raise ValueError("SDIRK order must be 2, 3 or 4")
    return A, list(A[-1]), c


def diffusion_only_coeffs(a=1.0) -> dict:
    c = {k: 0.0 for k in COEFF_NAMES}
    for k in ("mu1", "mu2", "mu3", "nu1", "nu2", "nu3"):
        c[k] = a
    for k in ("chith_11", "chith_13", "chith_21", "chith_22"):
        c[k] = 1.0
    c["c1_star"] = 10.0
    c["c1_sstar"] = 10.0
    return c
