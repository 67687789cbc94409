"""Float64 CPU oracle of the CDG2 operator on unstructured triangle meshes (P_k).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU baseline; the library never calls it, and it shares no code with the HIP
path.

What it computes (Section 3.1 on simplices, the element type the paper uses):
the residual <phi_j, L_h(U)> of the six-species model of Section 2 with

  * V_h = P_k on each triangle K (full polynomial space, k = 1, 2, 3), basis
    phi_j = phi^_j o F_K^{-1} with phi^_j orthonormal on the reference
    triangle T^ = {xi, eta >= 0, xi + eta <= 1} for the mean (1/|T^|) int_T^,
    built by Gram-Schmidt from the monomials xi^a eta^b ordered by total degree,
    then by the power of eta (1, xi, eta, xi^2, xi eta, eta^2, xi^3, ...),
    evaluated about the centroid; so
    phi_0 = 1 (mode 0 is the cell mean) and M_K = |K| I;
  * volume integrals with the collapsed (Duffy) Gauss rule of k + 1 points per
    direction: (xi, eta) = (u, v (1 - u)), weight w_u w_v (1 - u), exact for
    total degree 2k (the mass matrix);
  * edge integrals with the (k + 1)-point Gauss rule;
  * interior edges: consistency {a grad u}.n, symmetry 1/2 a (u_o - u_n) d_n phi,
    LLF flux of the chemotactic fluxes (lambda = max over both sides of
    |w1.n|, |w2.n|, applied to all six species), and the CDG2 flux
    A^ = 2 chi_e a r_e|_{K^-} with the lifting r_e of the jump formed on K^- only:
    int_{K^-} r_e . tau = -1/2 int_e (u^- - u^+) n^- . tau for all tau in
    [P_k(K^-)]^2; chi_e = 3/2 (half the number of faces of a triangle); K^- is
    the smaller of the two triangles, ties broken by the lower element index;
  * boundary edges: the inflow fluxes of eqs. (7)-(9) on Gamma1 (y = 0) and
    Gamma2 (y = 1), nothing else (zero diffusive flux);
  * f = M^{-1} R = R / |K|; SSP-RK3 (Shu-Osher) for time steps.

Parity: the pins in tests/test_tri_pins.py fix it against closed forms,
invariants (constants, conservation, symmetry and semidefiniteness of the
diffusion form) and the L2 convergence order on an exact heat solution.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle.cdg2_oracle import C1, C2, C3, DT, N1, N2, N3, NSPEC, Oracle, coeff_vector

CHI_E = 1.5


def gauss01(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def monomial_powers(k: int):
    """(a, b) of xi^a eta^b, by total degree, then by the power of eta."""
    return [(d - b, b) for d in range(k + 1) for b in range(d + 1)]


def duffy_rule(q: int):
    """Collapsed Gauss rule on the reference triangle: points [n, 2], weights [n]
    (sum 1/2)."""
    u, wu = gauss01(q)
    v, wv = gauss01(q)
    pts, wts = [], []
    for i in range(q):
        for j in range(q):
            pts.append((u[i], v[j] * (1.0 - u[i])))
            wts.append(wu[i] * wv[j] * (1.0 - u[i]))
    return np.array(pts), np.array(wts)


class TriBasis:
    """Orthonormal basis of P_k on the reference triangle (for the mean)."""

    def __init__(self, k: int):
        self.k = k
        self.pw = monomial_powers(k)
        nb = len(self.pw)
        pts, wts = duffy_rule(k + 3)                   # exact for degree 2k + 4
        V = self._mono(pts)                            # [n, nb]
        G = (V * (2.0 * wts)[:, None]).T @ V           # mean inner products
        C = np.zeros((nb, nb))
        for j in range(nb):                            # Gram-Schmidt, monomial order
            c = np.zeros(nb)
            c[j] = 1.0
            for i in range(j):
                c = c - (C[i] @ G @ c) * C[i]
            c = c / math.sqrt(c @ G @ c)
            C[j] = c
        self.C = C                                     # phi_j = sum_m C[j, m] mono_m
        self.nb = nb

    # The monomials are taken about the centroid (1/3, 1/3): each one differs from
    # the plain xi^a eta^b by monomials earlier in the order, so every prefix spans
    # the same space and Gram-Schmidt gives the same basis; evaluated about the
    # centroid the expansion cancels far less (plain monomials leave the P3 basis
    # orthonormal only to ~1e-12).
    CENTRE = 1.0 / 3.0

    def _mono(self, pts):
        xi, eta = pts[:, 0] - self.CENTRE, pts[:, 1] - self.CENTRE
        return np.stack([xi ** a * eta ** b for a, b in self.pw], axis=1)

    def _mono_grad(self, pts):
        xi, eta = pts[:, 0] - self.CENTRE, pts[:, 1] - self.CENTRE
        gx = [a * xi ** max(a - 1, 0) * eta ** b if a > 0 else 0.0 * xi for a, b in self.pw]
        gy = [b * xi ** a * eta ** max(b - 1, 0) if b > 0 else 0.0 * xi for a, b in self.pw]
        return np.stack(gx, axis=1), np.stack(gy, axis=1)

    def values(self, pts):
        return self._mono(pts) @ self.C.T              # [n, nb]

    def grads(self, pts):
        gx, gy = self._mono_grad(pts)
        return np.stack([gx @ self.C.T, gy @ self.C.T], axis=-1)   # [n, nb, 2]


def edge_ref_points(edge: int, s: np.ndarray) -> np.ndarray:
    """Reference points of local edge `edge` (from vertex edge to vertex edge+1)
    at parameters s."""
    V = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    a, b = V[edge], V[(edge + 1) % 3]
    return a[None, :] + s[:, None] * (b - a)[None, :]


class TriMesh:
    """Geometry of a conforming triangle mesh given as per-element vertex
    coordinates xy [E, 3, 2] (counter-clockwise, periodic images unwrapped) and
    the neighbour tables nbr [E, 3] (element across edge j = (v_j, v_j+1), or -1
    on Gamma1, -2 on Gamma2) and nbe [E, 3] (the neighbour's local edge)."""

    def __init__(self, xy, nbr, nbe):
        self.xy = np.asarray(xy, dtype=np.float64)
        self.nbr = np.asarray(nbr, dtype=np.int64)
        self.nbe = np.asarray(nbe, dtype=np.int64)
        E = self.xy.shape[0]
        self.E = E
        x0 = self.xy[:, 0]
        J = np.stack([self.xy[:, 1] - x0, self.xy[:, 2] - x0], axis=2)   # [E, 2, 2] columns
        det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
        assert (det > 0).all(), "elements must be counter-clockwise"
        self.J = J
        self.area = 0.5 * det
        self.JinvT = np.linalg.inv(J).transpose(0, 2, 1)               # grad = J^-T grad^
        # edges: length and outward unit normal
        L = np.zeros((E, 3))
        nrm = np.zeros((E, 3, 2))
        for j in range(3):
            t = self.xy[:, (j + 1) % 3] - self.xy[:, j]
            L[:, j] = np.hypot(t[:, 0], t[:, 1])
            nrm[:, j, 0] = t[:, 1] / L[:, j]
            nrm[:, j, 1] = -t[:, 0] / L[:, j]
        self.L, self.n = L, nrm
        # K^-: the smaller triangle of an interior edge, ties to the lower index
        minus = np.zeros((E, 3), dtype=bool)
        for j in range(3):
            nb = self.nbr[:, j]
            inner = nb >= 0
            an = np.where(inner, self.area[np.maximum(nb, 0)], np.inf)
            e = np.arange(E)
            minus[:, j] = inner & ((self.area < an) | ((self.area == an) & (e < nb)))
        self.minus = minus


class TriOracle:
    """Direct evaluation of the operator above, vectorised over elements."""

    def __init__(self, mesh: TriMesh, order: int, coeffs, gamma1_in=(0.0, 1.0)):
        self.mesh = mesh
        self.k = order
        self.th = coeff_vector(coeffs)
        self.gamma1_in = gamma1_in
        self.basis = TriBasis(order)
        nb = self.basis.nb
        self.nb = nb
        q = order + 1
        pts, wts = duffy_rule(q)
        self.Bv = torch.tensor(self.basis.values(pts), dtype=DT)          # [Q, nb]
        self.Bg = torch.tensor(self.basis.grads(pts), dtype=DT)           # [Q, nb, 2]
        self.wv = torch.tensor(2.0 * wts, dtype=DT)                        # mean weights (sum 1)
        s, ws = gauss01(q)
        self.s, self.ws = s, torch.tensor(ws, dtype=DT)
        # edge tables for each local edge, points in the edge's own direction
        self.Be = torch.tensor(np.stack([self.basis.values(edge_ref_points(j, s)) for j in range(3)]), dtype=DT)
        self.Bge = torch.tensor(np.stack([self.basis.grads(edge_ref_points(j, s)) for j in range(3)]), dtype=DT)
        self.JinvT = torch.tensor(mesh.JinvT, dtype=DT)
        self.area = torch.tensor(mesh.area, dtype=DT)
        self.L = torch.tensor(mesh.L, dtype=DT)
        self.nrm = torch.tensor(mesh.n, dtype=DT)

    # physical gradients of the basis of every element at reference points g [P, nb, 2]
    def _phys_grad(self, g, elems=None):
        Jt = self.JinvT if elems is None else self.JinvT[elems]
        return torch.einsum("eab,pjb->epja", Jt, g)                        # [E, P, nb, 2]

    def residual(self, U: torch.Tensor) -> torch.Tensor:
        U = U.to(DT)
        m, th = self.mesh, self.th
        E = m.E
        mu = th[0:6]
        R = torch.zeros_like(U)
        # ---- volume ----
        u = torch.einsum("qj,sej->seq", self.Bv, U)                       # [6, E, Q]
        G = self._phys_grad(self.Bg)                                       # [E, Q, nb, 2]
        g = torch.einsum("eqja,sej->seqa", G, U)                          # [6, E, Q, 2]
        w1, w2 = Oracle.velocities(None, u, g, th)
        flux = -mu[:, None, None, None] * g
        flux[N1] = flux[N1] + u[N1][..., None] * w1
        flux[N2] = flux[N2] + u[N2][..., None] * w2
        S = Oracle.source(None, u, th)                                     # [6, E, Q]
        wK = self.wv[None, :] * self.area[:, None]                         # [E, Q]
        R += torch.einsum("eq,seqa,eqja->sej", wK, flux, G)
        R += torch.einsum("eq,seq,qj->sej", wK, S, self.Bv)
        # ---- edges ----
        ne = len(self.s)
        for j in range(3):
            nbr = torch.tensor(m.nbr[:, j])
            nbe = torch.tensor(m.nbe[:, j])
            inner = nbr >= 0
            nn = self.nrm[:, j]                                            # [E, 2] outward
            Lw = self.L[:, j][:, None] * self.ws[None, :]                  # [E, P] edge weights
            Bo = self.Be[j]                                                # [P, nb] own
            Go = self._phys_grad(self.Bge[j])                              # [E, P, nb, 2]
            uo = torch.einsum("pj,sej->sep", Bo, U)
            go = torch.einsum("epja,sej->sepa", Go, U)
            dno = torch.einsum("sepa,ea->sep", go, nn)
            dphi = torch.einsum("epja,ea->epj", Go, nn)                    # d_n phi_j at own points
            # boundary edges: inflow fluxes, test functions phi_j
            bd1 = (m.nbr[:, j] == -1)
            bd2 = (m.nbr[:, j] == -2)
            if bd1.any() or bd2.any():
                c1 = uo[C1]
                xpts = (torch.tensor(m.xy[:, j, 0])[:, None] +
                        torch.tensor(self.s)[None, :] * torch.tensor(m.xy[:, (j + 1) % 3, 0] - m.xy[:, j, 0])[:, None])
                g0, g1 = self.gamma1_in
                inside = ((xpts >= g0) & (xpts <= g1)).to(DT)
                q = torch.zeros_like(uo)
                b1 = torch.tensor(bd1, dtype=DT)[:, None]
                b2 = torch.tensor(bd2, dtype=DT)[:, None]
                q[N1] = b1 * th[0] * th[21] * (c1 - th[24] > 0).to(DT)
                q[C2] = b1 * th[4] * th[23] * inside
                q[N2] = b2 * th[1] * th[22] * (c1 - th[25] > 0).to(DT)
                R += torch.einsum("ep,sep,pj->sej", Lw, q, Bo)
            if not inner.any():
                continue
            # neighbour traces at the same physical points (its edge runs the other way)
            nbc = torch.clamp(nbr, min=0)
            rev = torch.arange(ne - 1, -1, -1)
            Bn = self.Be[nbe][:, rev]                                      # [E, P, nb]
            Gn = torch.einsum("eab,epjb->epja", self.JinvT[nbc], self.Bge[nbe][:, rev])
            Un = U[:, nbc]                                                 # [6, E, nb]
            un = torch.einsum("epj,sej->sep", Bn, Un)
            gn = torch.einsum("epja,sej->sepa", Gn, Un)
            dnn = torch.einsum("sepa,ea->sep", gn, nn)
            # LLF
            uo_all, un_all = uo, un
            w1o, w2o = Oracle.velocities(None, uo_all, go, th)
            w1n, w2n = Oracle.velocities(None, un_all, gn, th)
            lam = torch.stack([torch.einsum("epa,ea->ep", w, nn).abs() for w in (w1o, w2o, w1n, w2n)]).amax(0)
            Fno = torch.zeros_like(uo)
            Fnn = torch.zeros_like(uo)
            Fno[N1] = uo[N1] * torch.einsum("epa,ea->ep", w1o, nn)
            Fno[N2] = uo[N2] * torch.einsum("epa,ea->ep", w2o, nn)
            Fnn[N1] = un[N1] * torch.einsum("epa,ea->ep", w1n, nn)
            Fnn[N2] = un[N2] * torch.einsum("epa,ea->ep", w2n, nn)
            jump = uo - un                                                 # u_o - u_n
            # CDG2: A^.n_o = -(chi a / |K^-|) (n^- . n_o) sum_j phi_j^-(x) int_e (u^- - u^+) phi_j^-
            minus = torch.tensor(m.minus[:, j])
            Bm = torch.where(minus[:, None, None], Bo[None].expand(E, -1, -1), Bn)   # K^- basis at the points
            am = torch.where(minus, self.area, self.area[nbc])
            sgn = torch.where(minus, 1.0, -1.0).to(DT)                     # n^- . n_o
            gm = jump * sgn[None, :, None]                                 # u^- - u^+
            proj = torch.einsum("ep,sep,epj->sej", Lw, gm, Bm)             # int_e g phi_j^-
            rtr = torch.einsum("epj,sej->sep", Bm, proj)                   # sum_j phi_j^-(x) (...)
            An = -(CHI_E * mu[:, None, None] / am[None, :, None]) * sgn[None, :, None] * rtr
            gv = 0.5 * mu[:, None, None] * (dno + dnn) + An - 0.5 * (Fno + Fnn) - 0.5 * lam[None] * jump
            hv = 0.5 * mu[:, None, None] * jump
            fi = inner.to(DT)[None, :, None]
            R += torch.einsum("ep,sep,pj->sej", Lw, gv * fi, Bo)
            R += torch.einsum("ep,sep,epj->sej", Lw, hv * fi, dphi)
        return R

    def apply(self, U: torch.Tensor) -> torch.Tensor:
        return self.residual(U) / self.area[None, :, None]

    def rk_step(self, U: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        U = U.to(DT).clone()
        for _ in range(nsteps):
            U1 = U + dt * self.apply(U)
            U2 = 0.75 * U + 0.25 * (U1 + dt * self.apply(U1))
            U = U / 3.0 + (2.0 / 3.0) * (U2 + dt * self.apply(U2))
        return U

    # -- helpers for the pins ---------------------------------------------------------
    def project(self, func, extra: int = 3) -> torch.Tensor:
        """L2 projection of func(x, y) -> [6, ...] onto P_k (exact rule of higher
        degree)."""
        pts, wts = duffy_rule(self.k + 1 + extra)
        B = torch.tensor(self.basis.values(pts), dtype=DT)
        xy = self.mesh.xy
        X = (xy[:, 0][:, None, :] + pts[None, :, 0:1] * (xy[:, 1] - xy[:, 0])[:, None, :]
             + pts[None, :, 1:2] * (xy[:, 2] - xy[:, 0])[:, None, :])     # [E, n, 2]
        f = torch.as_tensor(np.array(func(X[..., 0], X[..., 1])), dtype=DT)   # [6, E, n]
        return torch.einsum("n,sen,nj->sej", torch.tensor(2.0 * wts, dtype=DT), f, B)

    def l2_error(self, U, func, species=0, extra: int = 3) -> float:
        pts, wts = duffy_rule(self.k + 1 + extra)
        B = torch.tensor(self.basis.values(pts), dtype=DT)
        xy = self.mesh.xy
        X = (xy[:, 0][:, None, :] + pts[None, :, 0:1] * (xy[:, 1] - xy[:, 0])[:, None, :]
             + pts[None, :, 1:2] * (xy[:, 2] - xy[:, 0])[:, None, :])
        f = torch.as_tensor(np.array(func(X[..., 0], X[..., 1])), dtype=DT)[species]
        uh = torch.einsum("nj,ej->en", B, U[species].to(DT))
        w = torch.tensor(2.0 * wts, dtype=DT)[None, :] * self.area[:, None]
        return float(torch.sqrt((w * (uh - f) ** 2).sum()))
