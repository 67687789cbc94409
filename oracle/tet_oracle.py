"""Float64 CPU oracle of the CDG2 operator on unstructured tetrahedral meshes (P_k).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU baseline; the library never calls it, and it shares no code with the HIP
path.

What it computes (Section 3.1 on tetrahedra, the element of the paper's 3D runs):
the residual <phi_j, L_h(U)> of the six-species model of Section 2 with

  * V_h = P_k on each tetrahedron K (full polynomial space, k = 1, 2, 3), basis
    phi_j = phi^_j o F_K^{-1} with phi^_j orthonormal on the reference
    tetrahedron T^ = {xi, eta, zeta >= 0, xi + eta + zeta <= 1} for the mean,
    by Gram-Schmidt of the monomials xi^a eta^b zeta^c ordered by total degree,
    then by the power of zeta, then of eta (1, xi, eta, zeta, xi^2, xi eta,
    eta^2, xi zeta, eta zeta, zeta^2, ...), taken about the centroid (every
    prefix spans the same space as the plain monomials; far less cancellation);
    so phi_0 = 1 (mode 0 is the element mean) and M_K = |K| I;
  * volume integrals with a fully symmetric rule on the tetrahedron exact for
    degree 2k (the mass matrix): k = 1: 4 points, degree 2; k = 2: 14 points,
    degree 5 (at degree 4 that layout is a one-parameter family of rules;
    degree 5 leaves one); k = 3: 24 points, degree 6; orbits of the vertex
    permutations with positive weights, their parameters solving the moment
    equations (Newton, here);
  * face integrals with a fully symmetric rule on the triangle, exact for
    degree 2k (k = 1: 3 points, degree 2; k = 2: 6 points, degree 4; k = 3:
    12 points, degree 6), so that both elements of a face use the same physical
    points whatever the orientation of their local faces; the orbit parameters
    solve the moment equations (Newton, here);
  * interior faces: consistency {a grad u}.n, symmetry 1/2 a (u_o - u_n) d_n phi,
    LLF flux of the chemotactic fluxes (lambda = max over both sides of
    |w1.n|, |w2.n|, applied to all six species) and the CDG2 flux
    A^ = 2 chi_e a r_e|_{K^-}, the lifting of the jump formed on K^- only:
    int_{K^-} r_e . tau = -1/2 int_e (u^- - u^+) n^- . tau for tau in
    [P_k(K^-)]^3, chi_e = 2 (half the number of faces of a tetrahedron); K^- is
    the smaller tetrahedron, ties to the lower element index;
  * boundary faces: the inflow fluxes of eqs. (7)-(9) on the faces coded Gamma1
    and Gamma2 (Gamma1,in: the Gamma1 points with x in [g0, g1]), nothing else;
  * f = M^{-1} R = R / |K|; SSP-RK3 (Shu-Osher) for time steps.

Local face f of a tetrahedron is the face opposite local vertex f, with the other
three vertices in increasing local order.  The neighbour's trace is evaluated at
the same physical points, found from the shared vertex ids (barycentric
coordinates carried over) and the neighbour's own affine map.
"""
from __future__ import annotations

import math
from itertools import permutations

import numpy as np
import torch

from oracle.cdg2_oracle import C1, C2, C3, DT, N1, N2, N3, NSPEC, Oracle, coeff_vector

CHI_E = 2.0
FACE_VERTS = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))


def gauss01(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def monomial_powers3(k: int):
    """(a, b, c) of xi^a eta^b zeta^c: total degree, then power of zeta, then eta."""
    return [(d - b - c, b, c) for d in range(k + 1) for c in range(d + 1) for b in range(d - c + 1)]


def collapsed_tet_rule(k: int):
    """Points [n, 3] and weights [n] (sum 1/6) on the reference tetrahedron."""
    u, wu = gauss01(k + 2)
    v, wv = gauss01(k + 1)
    w, ww = gauss01(k + 1)
    pts, wts = [], []
    for i in range(len(u)):
        for j in range(len(v)):
            for l in range(len(w)):
                pts.append((u[i], v[j] * (1 - u[i]), w[l] * (1 - u[i]) * (1 - v[j])))
                wts.append(wu[i] * wv[j] * ww[l] * (1 - u[i]) ** 2 * (1 - v[j]))
    return np.array(pts), np.array(wts)


def _tet_mean(a, b, c, d):
    """Mean of l0^a l1^b l2^c l3^d over a tetrahedron (barycentric coordinates)."""
    f = math.factorial
    return 6.0 * f(a) * f(b) * f(c) * f(d) / f(a + b + c + d + 3)


def symmetric_tet_rule(k: int):
    """Fully symmetric rule on the tetrahedron exact for degree 2k (k = 2: 5), as
    barycentric points [n, 4] and weights [n] for the mean (sum 1).  Orbits of the
    vertex permutations: (a, a, a, 1 - 3a) with 4 points, (b, b, 1/2 - b, 1/2 - b)
    with 6, (b, b, c, 1 - 2b - c) with 12.  k = 1: one 4-orbit; k = 2: two 4-orbits
    and a 6-orbit; k = 3: three 4-orbits and a 12-orbit.  The orbit parameters and
    all but the last weight solve the moment equations of every monomial up to
    that degree (least-squares Newton from rough starting values).  For k = 2 the
    14-point layout has one parameter more than the symmetric moment equations of
    degree 4 fix, a one-parameter family of rules; degree 5 leaves the one rule of
    that layout.  The solution must be isolated (Jacobian of full column rank), so
    that any solver of the same equations finds the same rule."""
    if k == 1:
        layout, x = [("s31", 1)], [0.14]
    elif k == 2:
        layout, x = [("s31", 1), ("s31", 1), ("s22", 1)], [0.093, 0.073, 0.311, 0.113, 0.045]
    elif k == 3:
        layout, x = ([("s31", 1), ("s31", 1), ("s31", 1), ("s211", 2)],
                     [0.215, 0.24, 0.041, 0.06, 0.322, 0.33, 0.064, 0.27])
    else:
        raise ValueError("volume rules for k = 1, 2, 3")

    def orbit(kind, q):
        if kind == "s31":
            base = (q[0], q[0], q[0], 1 - 3 * q[0])
        elif kind == "s22":
            base = (q[0], q[0], 0.5 - q[0], 0.5 - q[0])
        else:
            base = (q[0], q[0], q[1], 1 - 2 * q[0] - q[1])
        return sorted(set(permutations(base)))

    def expand(y):
        groups, i, used = [], 0, 0.0
        for o, (kind, npar) in enumerate(layout):
            pts = orbit(kind, y[i:i + npar])
            i += npar
            if o < len(layout) - 1:
                w = y[i]
                i += 1
                used += len(pts) * w
            else:
                w = None
            groups.append((pts, w))
        pts, _ = groups[-1]
        groups[-1] = (pts, (1.0 - used) / len(pts))
        P = np.array([p for pts, w in groups for p in pts], dtype=np.float64)
        W = np.array([w for pts, w in groups for p in pts], dtype=np.float64)
        return P, W

    deg = tet_rule_degree(k)
    mons = [(a, b, c, d - a - b - c) for d in range(deg + 1) for a in range(d + 1)
            for b in range(d - a + 1) for c in range(d - a - b + 1)]

    def resid(y):
        P, W = expand(y)
        return np.array([np.sum(W * P[:, 0] ** a * P[:, 1] ** b * P[:, 2] ** c * P[:, 3] ** d) - _tet_mean(a, b, c, d)
                         for a, b, c, d in mons])

    def jac(y):
        Jm = np.zeros((len(mons), len(y)))
        for i in range(len(y)):
            e = np.zeros(len(y))
            e[i] = 1e-7
            Jm[:, i] = (resid(y + e) - resid(y - e)) / 2e-7
        return Jm

    x = np.array(x, dtype=np.float64)
    for _ in range(100):
        r = resid(x)
        if np.abs(r).max() < 1e-15:
            break
        x = x - np.linalg.lstsq(jac(x), r, rcond=None)[0]
    P, W = expand(x)
    assert np.abs(resid(x)).max() < 1e-14, "volume rule did not converge"
    sv = np.linalg.svd(jac(x), compute_uv=False)
    assert sv[-1] > 1e-6 * sv[0], "volume rule is not an isolated solution"
    return P, W


def tet_rule_degree(k: int) -> int:
    """Polynomial degree of the volume rule of order k: 2k, but 5 for k = 2."""
    return 5 if k == 2 else 2 * k


def tet_volume_rule(k: int):
    """The operator's volume rule: reference points [n, 3] (xi, eta, zeta) =
    barycentric coordinates of vertices 1, 2, 3, and weights [n] (sum 1/6)."""
    P, W = symmetric_tet_rule(k)
    return P[:, 1:4].copy(), W / 6.0


def _tri_mean(a, b, c):
    """Mean of l1^a l2^b l3^c over a triangle (barycentric coordinates)."""
    return 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)


def symmetric_face_rule(k: int):
    """Fully symmetric rule on the triangle exact for degree 2k, as barycentric
    points [n, 3] and weights [n] for the mean (sum 1).  Orbits: (a, a, 1 - 2a)
    with 3 points, (b, c, 1 - b - c) with 6.  The free parameters solve the
    moment equations for every monomial up to degree 2k (least squares Newton;
    the system is consistent)."""
    if k == 1:
        layout, guess = ["s21"], [1.0 / 6.0]
    elif k == 2:
        layout, guess = ["s21", "s21"], [0.4459, 0.2234, 0.0916]
    elif k == 3:
        layout, guess = ["s21", "s21", "s111"], [0.2493, 0.1168, 0.0631, 0.0508, 0.0531, 0.3104]
    else:
        raise ValueError("face rules for k = 1, 2, 3")

    def expand(x):
        """Parameter vector -> (points, weights); the last weight closes sum 1."""
        pts, wts, i = [], [], 0
        ws = []
        for o in layout:
            if o == "s21":
                a = x[i]
                i += 1
                orb = {(a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a)}
            else:
                b, c = x[i], x[i + 1]
                i += 2
                orb = set(permutations((b, c, 1 - b - c)))
            orb = sorted(orb)
            if len(ws) < len(layout) - 1:
                wgt = x[i]
                i += 1
            else:
                wgt = None
            ws.append((orb, wgt))
        used = sum(len(orb) * w for orb, w in ws if w is not None)
        last = ws[-1]
        ws[-1] = (last[0], (1.0 - used) / len(last[0]))
        for orb, w in ws:
            for p in orb:
                pts.append(p)
                wts.append(w)
        return np.array(pts, dtype=np.float64), np.array(wts, dtype=np.float64)

    # parameter order per orbit: s21 -> a (then its weight unless last),
    # s111 -> b, c (then weight unless last)
    if k == 1:
        x = np.array(guess)
    elif k == 2:
        x = np.array([guess[0], guess[1], guess[2]])
    else:
        x = np.array([guess[0], guess[1], guess[2], guess[3], guess[4], guess[5]])
    mons = [(a, b, d - a - b) for d in range(2 * k + 1) for a in range(d + 1) for b in range(d - a + 1)]

    def resid(x):
        P, W = expand(x)
        return np.array([np.sum(W * P[:, 0] ** a * P[:, 1] ** b * P[:, 2] ** c) - _tri_mean(a, b, c)
                         for a, b, c in mons])

    for _ in range(60):
        r = resid(x)
        if np.abs(r).max() < 1e-15:
            break
        Jm = np.zeros((len(r), len(x)))
        for i in range(len(x)):
            e = np.zeros(len(x))
            e[i] = 1e-7
            Jm[:, i] = (resid(x + e) - resid(x - e)) / 2e-7
        x = x - np.linalg.lstsq(Jm, r, rcond=None)[0]
    P, W = expand(x)
    assert np.abs(resid(x)).max() < 1e-14, "face rule did not converge"
    return P, W


class TetBasis:
    """Orthonormal basis of P_k on the reference tetrahedron (for the mean)."""

    CENTRE = 0.25

    def __init__(self, k: int):
        self.k = k
        self.pw = monomial_powers3(k)
        nb = len(self.pw)
        pts, wts = collapsed_tet_rule(k + 2)            # exact for degree 2k + 4
        V = self._mono(pts)
        G = (V * (6.0 * wts)[:, None]).T @ V            # mean inner products
        C = np.zeros((nb, nb))
        for j in range(nb):
            c = np.zeros(nb)
            c[j] = 1.0
            for i in range(j):
                c = c - (C[i] @ G @ c) * C[i]
            C[j] = c / math.sqrt(c @ G @ c)
        self.C = C
        self.nb = nb

    def _mono(self, pts):
        x, y, z = (pts[:, i] - self.CENTRE for i in range(3))
        return np.stack([x ** a * y ** b * z ** c for a, b, c in self.pw], axis=1)

    def _mono_grad(self, pts):
        x, y, z = (pts[:, i] - self.CENTRE for i in range(3))
        gx = [a * x ** max(a - 1, 0) * y ** b * z ** c if a else 0 * x for a, b, c in self.pw]
        gy = [b * x ** a * y ** max(b - 1, 0) * z ** c if b else 0 * x for a, b, c in self.pw]
        gz = [c * x ** a * y ** b * z ** max(c - 1, 0) if c else 0 * x for a, b, c in self.pw]
        return np.stack(gx, 1), np.stack(gy, 1), np.stack(gz, 1)

    def values(self, pts):
        return self._mono(pts) @ self.C.T

    def grads(self, pts):
        gx, gy, gz = self._mono_grad(pts)
        return np.stack([gx @ self.C.T, gy @ self.C.T, gz @ self.C.T], axis=-1)   # [n, nb, 3]


REF_VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


class TetMesh:
    """Conforming tetrahedral mesh: per-element vertex coordinates xyz [E, 4, 3]
    (positively oriented, periodic images unwrapped), vertex ids vid [E, 4] (the
    same id for the same mesh vertex, across periodic images), neighbour tables
    nbr [E, 4] (element across local face f, -1 Gamma1, -2 Gamma2) and nbe [E, 4]
    (the neighbour's local face)."""

    def __init__(self, xyz, vid, nbr, nbe):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.vid = np.asarray(vid, dtype=np.int64)
        self.nbr = np.asarray(nbr, dtype=np.int64)
        self.nbe = np.asarray(nbe, dtype=np.int64)
        E = self.xyz.shape[0]
        self.E = E
        J = np.stack([self.xyz[:, i] - self.xyz[:, 0] for i in (1, 2, 3)], axis=2)   # columns
        det = np.linalg.det(J)
        assert (det > 0).all(), "elements must be positively oriented"
        self.J = J
        self.vol = det / 6.0
        self.Jinv = np.linalg.inv(J)
        self.JinvT = self.Jinv.transpose(0, 2, 1)
        area = np.zeros((E, 4))
        nrm = np.zeros((E, 4, 3))
        for f, (a, b, c) in enumerate(FACE_VERTS):
            A, B, Cc = self.xyz[:, a], self.xyz[:, b], self.xyz[:, c]
            cr = np.cross(B - A, Cc - A)
            ar = 0.5 * np.linalg.norm(cr, axis=1)
            n = cr / (2.0 * ar[:, None])
            # outward: away from the opposite vertex
            away = np.sign(np.einsum("ei,ei->e", n, A - self.xyz[:, f]))
            area[:, f] = ar
            nrm[:, f] = n * away[:, None]
        self.area, self.n = area, nrm
        minus = np.zeros((E, 4), dtype=bool)
        for f in range(4):
            nb = self.nbr[:, f]
            inner = nb >= 0
            vn = np.where(inner, self.vol[np.maximum(nb, 0)], np.inf)
            e = np.arange(E)
            minus[:, f] = inner & ((self.vol < vn) | ((self.vol == vn) & (e < nb)))
        self.minus = minus


class TetOracle:
    """Direct evaluation of the operator above (vectorised over elements)."""

    def __init__(self, mesh: TetMesh, order: int, coeffs, gamma1_in=(0.0, 1.0)):
        self.mesh = mesh
        self.k = order
        self.th = coeff_vector(coeffs)
        self.gamma1_in = gamma1_in
        self.basis = TetBasis(order)
        self.nb = self.basis.nb
        pts, wts = tet_volume_rule(order)
        self.Bv = torch.tensor(self.basis.values(pts), dtype=DT)
        self.Bg = torch.tensor(self.basis.grads(pts), dtype=DT)
        self.wv = torch.tensor(6.0 * wts, dtype=DT)                      # mean weights
        self.fbary, fw = symmetric_face_rule(order)
        self.fw = torch.tensor(fw, dtype=DT)                              # mean weights over a face
        E = mesh.E
        # face points: physical, and each element's own reference coordinates
        P = len(fw)
        self.fx = np.zeros((E, 4, P, 3))
        self.fref = np.zeros((4, P, 3))
        for f, vs in enumerate(FACE_VERTS):
            self.fref[f] = self.fbary @ REF_VERTS[list(vs)]
            self.fx[:, f] = np.einsum("pi,eij->epj", self.fbary, mesh.xyz[:, list(vs)])
        self.Bf = torch.tensor(np.stack([self.basis.values(self.fref[f]) for f in range(4)]), dtype=DT)
        self.Bgf = torch.tensor(np.stack([self.basis.grads(self.fref[f]) for f in range(4)]), dtype=DT)
        # the neighbour's reference coordinates of this element's face points:
        # carry the barycentric coordinates over by vertex id
        self.nref = np.zeros((E, 4, P, 3))
        for e in range(E):
            for f, vs in enumerate(FACE_VERTS):
                g = mesh.nbr[e, f]
                if g < 0:
                    continue
                gf = mesh.nbe[e, f]
                gvs = FACE_VERTS[gf]
                ids = [mesh.vid[e, v] for v in vs]
                gpos = np.array([mesh.xyz[g, gvs[[mesh.vid[g, w] for w in gvs].index(i)]] for i in ids])
                X = self.fbary @ gpos                                     # [P, 3] in g's image
                self.nref[e, f] = (X - mesh.xyz[g, 0]) @ mesh.Jinv[g].T
        # the neighbour's basis and reference gradients at those points, per face
        self.Bn, self.Gn_ref = [], []
        for f in range(4):
            nr = self.nref[:, f].reshape(-1, 3)
            self.Bn.append(torch.tensor(self.basis.values(nr).reshape(E, P, self.nb), dtype=DT))
            self.Gn_ref.append(torch.tensor(self.basis.grads(nr).reshape(E, P, self.nb, 3), dtype=DT))
        self.vol = torch.tensor(mesh.vol, dtype=DT)
        self.area = torch.tensor(mesh.area, dtype=DT)
        self.nrm = torch.tensor(mesh.n, dtype=DT)
        self.JinvT = torch.tensor(mesh.JinvT, dtype=DT)

    def residual(self, U: torch.Tensor) -> torch.Tensor:
        U = U.to(DT)
        m, th = self.mesh, self.th
        E = m.E
        mu = th[0:6]
        R = torch.zeros_like(U)
        # ---- volume ----
        u = torch.einsum("qj,sej->seq", self.Bv, U)
        G = torch.einsum("eab,qjb->eqja", self.JinvT, self.Bg)              # physical gradients
        g = torch.einsum("eqja,sej->seqa", G, U)
        w1, w2 = Oracle.velocities(None, u, g, th)
        flux = -mu[:, None, None, None] * g
        flux[N1] = flux[N1] + u[N1][..., None] * w1
        flux[N2] = flux[N2] + u[N2][..., None] * w2
        S = Oracle.source(None, u, th)
        wK = self.wv[None, :] * self.vol[:, None]
        R += torch.einsum("eq,seqa,eqja->sej", wK, flux, G)
        R += torch.einsum("eq,seq,qj->sej", wK, S, self.Bv)
        # ---- faces ----
        for f in range(4):
            nbr = torch.tensor(m.nbr[:, f])
            inner = nbr >= 0
            nn = self.nrm[:, f]
            Aw = self.area[:, f][:, None] * self.fw[None, :]                 # [E, P]
            Bo = self.Bf[f]
            Go = torch.einsum("eab,pjb->epja", self.JinvT, self.Bgf[f])
            uo = torch.einsum("pj,sej->sep", Bo, U)
            go = torch.einsum("epja,sej->sepa", Go, U)
            dno = torch.einsum("sepa,ea->sep", go, nn)
            dphi = torch.einsum("epja,ea->epj", Go, nn)
            bd1 = m.nbr[:, f] == -1
            bd2 = m.nbr[:, f] == -2
            if bd1.any() or bd2.any():
                c1 = uo[C1]
                xpts = torch.tensor(self.fx[:, f, :, 0])
                g0, g1 = self.gamma1_in
                inside = ((xpts >= g0) & (xpts <= g1)).to(DT)
                q = torch.zeros_like(uo)
                b1 = torch.tensor(bd1, dtype=DT)[:, None]
                b2 = torch.tensor(bd2, dtype=DT)[:, None]
                q[N1] = b1 * th[0] * th[21] * (c1 - th[24] > 0).to(DT)
                q[C2] = b1 * th[4] * th[23] * inside
                q[N2] = b2 * th[1] * th[22] * (c1 - th[25] > 0).to(DT)
                R += torch.einsum("ep,sep,pj->sej", Aw, q, Bo)
            if not inner.any():
                continue
            nbc = torch.clamp(nbr, min=0)
            Bn = self.Bn[f]
            Gn = torch.einsum("eab,epjb->epja", self.JinvT[nbc], self.Gn_ref[f])
            Un = U[:, nbc]
            un = torch.einsum("epj,sej->sep", Bn, Un)
            gn = torch.einsum("epja,sej->sepa", Gn, Un)
            dnn = torch.einsum("sepa,ea->sep", gn, nn)
            w1o, w2o = Oracle.velocities(None, uo, go, th)
            w1n, w2n = Oracle.velocities(None, un, gn, th)
            lam = torch.stack([torch.einsum("epa,ea->ep", w, nn).abs() for w in (w1o, w2o, w1n, w2n)]).amax(0)
            Fno = torch.zeros_like(uo)
            Fnn = torch.zeros_like(uo)
            Fno[N1] = uo[N1] * torch.einsum("epa,ea->ep", w1o, nn)
            Fno[N2] = uo[N2] * torch.einsum("epa,ea->ep", w2o, nn)
            Fnn[N1] = un[N1] * torch.einsum("epa,ea->ep", w1n, nn)
            Fnn[N2] = un[N2] * torch.einsum("epa,ea->ep", w2n, nn)
            jump = uo - un
            # CDG2: A^.n_o = -(chi a / |K^-|) (n^- . n_o) sum_j phi_j^-(x) int_e (u^- - u^+) phi_j^-
            minus = torch.tensor(m.minus[:, f])
            Bm = torch.where(minus[:, None, None], Bo[None].expand(E, -1, -1), Bn)
            vm = torch.where(minus, self.vol, self.vol[nbc])
            sgn = torch.where(minus, 1.0, -1.0).to(DT)
            gm = jump * sgn[None, :, None]
            proj = torch.einsum("ep,sep,epj->sej", Aw, gm, Bm)
            rtr = torch.einsum("epj,sej->sep", Bm, proj)
            An = -(CHI_E * mu[:, None, None] / vm[None, :, None]) * sgn[None, :, None] * rtr
            gv = 0.5 * mu[:, None, None] * (dno + dnn) + An - 0.5 * (Fno + Fnn) - 0.5 * lam[None] * jump
            hv = 0.5 * mu[:, None, None] * jump
            fi = inner.to(DT)[None, :, None]
            R += torch.einsum("ep,sep,pj->sej", Aw, gv * fi, Bo)
            R += torch.einsum("ep,sep,epj->sej", Aw, hv * fi, dphi)
        return R

    def apply(self, U: torch.Tensor) -> torch.Tensor:
        return self.residual(U) / self.vol[None, :, None]

    def rk_step(self, U: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        U = U.to(DT).clone()
        for _ in range(nsteps):
            U1 = U + dt * self.apply(U)
            U2 = 0.75 * U + 0.25 * (U1 + dt * self.apply(U1))
            U = U / 3.0 + (2.0 / 3.0) * (U2 + dt * self.apply(U2))
        return U

    # -- helpers for the pins ---------------------------------------------------------
    def _phys(self, pts):
        xyz = self.mesh.xyz
        return xyz[:, 0][:, None, :] + np.einsum("pi,eji->epj", pts, self.mesh.J)

    def project(self, func, extra: int = 2) -> torch.Tensor:
        """L2 projection of func(x, y, z) -> [6, ...] onto P_k."""
        pts, wts = collapsed_tet_rule(self.k + extra)
        B = torch.tensor(self.basis.values(pts), dtype=DT)
        X = self._phys(pts)
        f = torch.as_tensor(np.array(func(X[..., 0], X[..., 1], X[..., 2])), dtype=DT)
        return torch.einsum("n,sen,nj->sej", torch.tensor(6.0 * wts, dtype=DT), f, B)

    def l2_error(self, U, func, species=0, extra: int = 2) -> float:
        pts, wts = collapsed_tet_rule(self.k + extra)
        B = torch.tensor(self.basis.values(pts), dtype=DT)
        X = self._phys(pts)
        f = torch.as_tensor(np.array(func(X[..., 0], X[..., 1], X[..., 2])), dtype=DT)[species]
        uh = torch.einsum("nj,ej->en", B, U[species].to(DT))
        w = torch.tensor(6.0 * wts, dtype=DT)[None, :] * self.vol[:, None]
        return float(torch.sqrt((w * (uh - f) ** 2).sum()))
