"""Extended-precision evaluation of f = M^-1 L_h(U) on uniform Cartesian grids,
for pinning the float64 oracle's rounding (the noise floor of the parity bar).

TEST INFRASTRUCTURE.  Written separately from oracle/cdg2_oracle.py (numpy,
generic in the floating-point type: np.longdouble is the x87 80-bit format here,
64-bit significand).  It evaluates the same discrete operator of Section 3.1 on
the same readings (tensor Legendre Q_p, p+1 Gauss points per direction, LLF,
inflow conditions of eqs. (7)-(9)); the CDG2 lifting enters through its exact
trace on Cartesian cells, -(p+1)^2 / (2h) (u^- - u^+) (the equality with the
general lifting is pinned separately), so Â.n^- = -chi_e a (p+1)^2 / h (u^- - u^+).
The face jump is formed either mode by mode (the constant modes cancel
exactly) or as the plain difference of the two traces (``jump="plain"``)."""
import numpy as np


def gauss01(q, dt):
    """q-point Gauss-Legendre rule on [0, 1] in the type dt (Newton on P_q)."""
    one = dt(1)
    xs = []
    for j in range(1, q + 1):
        x = dt(np.cos(np.pi * (4 * j - 1) / (4 * q + 2)))
        for _ in range(60):
            p0, p1 = one, x
            for k in range(1, q):
                p0, p1 = p1, (dt(2 * k + 1) * x * p1 - dt(k) * p0) / dt(k + 1)
            dp = dt(q) * (x * p1 - p0) / (x * x - one)
            step = p1 / dp
            x = x - step
            if abs(step) < dt(1e-30):
                break
        xs.append(x)
    x = np.array(sorted(xs), dtype=dt)
    p0, p1 = np.ones_like(x), x.copy()
    for k in range(1, q):
        p0, p1 = p1, (dt(2 * k + 1) * x * p1 - dt(k) * p0) / dt(k + 1)
    dp = dt(q) * (x * p1 - p0) / (x * x - one)
    w = dt(2) / ((one - x * x) * dp * dp)
    return (x + one) / dt(2), w / dt(2)


def legendre01(p, xi, dt):
    """sqrt(2i+1) P_i(2 xi - 1) and d/dxi for i = 0..p: arrays [len(xi), p+1]."""
    t = dt(2) * np.asarray(xi, dtype=dt) - dt(1)
    P = [np.ones_like(t), t.copy()]
    D = [np.zeros_like(t), np.ones_like(t)]
    for k in range(1, p):
        P.append((dt(2 * k + 1) * t * P[k] - dt(k) * P[k - 1]) / dt(k + 1))
        D.append(D[k - 1] + dt(2 * k + 1) * P[k])
    sc = [np.sqrt(dt(2 * i + 1)) for i in range(p + 1)]
    val = np.stack([sc[i] * P[i] for i in range(p + 1)], axis=-1)
    der = np.stack([dt(2) * sc[i] * D[i] for i in range(p + 1)], axis=-1)
    return val, der


def _tensor(tabs, d):
    """Tensor product of per-axis tables [npt_a, p+1] -> [prod npt, (p+1)^d],
    x index fastest in both points and modes."""
    out = tabs[0]
    for a in range(1, d):
        out = np.einsum("PM,qm->qPmM", out, tabs[a]).reshape(out.shape[0] * tabs[a].shape[0], -1)
    return out


class LDOperator:
    def __init__(self, dim, n, p, coeffs, dt=np.longdouble, wall_axis=None, chi_e=None):
        self.d, self.n, self.p, self.dt = dim, tuple(n), p, dt
        self.wall = dim - 1 if wall_axis is None else wall_axis
        names = ["mu1", "mu2", "mu3", "nu1", "nu2", "nu3", "chi0_11", "chi0_13", "chi0_21", "chi0_22",
                 "chith_11", "chith_13", "chith_21", "chith_22", "d1", "d2", "gamma", "alpha1", "alpha2",
                 "f1", "k", "beta1", "beta2", "sigma", "c1_star", "c1_sstar"]
        self.c = {k: dt(coeffs[k]) for k in names}
        self.a = np.array([self.c[k] for k in names[:6]], dtype=dt)
        self.h = [dt(1) / dt(v) for v in self.n]
        self.chi = dt(dim) if chi_e is None else dt(chi_e)
        q = p + 1
        x, w = gauss01(q, dt)
        self.x1, self.w1 = x, w
        V, Dv = legendre01(p, x, dt)
        E0, dE0 = legendre01(p, np.array([0.0]), dt)
        E1, dE1 = legendre01(p, np.array([1.0]), dt)
        self.V, self.Dv, self.ends = V, Dv, {0: (E0, dE0), 1: (E1, dE1)}
        self.vol = np.prod(np.array(self.h, dtype=dt))
        # volume tables: values and physical gradients of all modes at all points
        self.Phi = _tensor([V] * dim, dim)
        self.dPhi = np.stack([_tensor([Dv / self.h[a] if b == a else V for b in range(dim)], dim)
                              for a in range(dim)], axis=-1)
        self.wq = _tensor([w[:, None]] * dim, dim)[:, 0] * self.vol

    def _face_tabs(self, ax, side):
        """Values and normal derivatives of all modes at the face points of the face
        xi_ax = side, and the face weights (x index fastest over the other axes)."""
        d, dt = self.d, self.dt
        E, dE = self.ends[side]
        val = _tensor([E if b == ax else self.V for b in range(d)], d)
        dn = _tensor([dE / self.h[ax] if b == ax else self.V for b in range(d)], d)
        area = np.prod(np.array([self.h[b] for b in range(d) if b != ax], dtype=dt))
        wt = _tensor([self.w1[:, None]] * (d - 1), d - 1)[:, 0] if d > 1 else np.ones(1, dtype=dt)
        return val, dn, wt * area

    def velocities(self, u, g):
        """Chemotactic velocities w1, w2 from values u[s] and gradients g[s] (any
        trailing shape; g[s] may carry a leading axis of components)."""
        c = self.c
        k11 = c["chi0_11"] / (u[3] + c["chith_11"])
        k13 = c["chi0_13"] / (u[5] + c["chith_13"])
        k21 = c["chi0_21"] / (u[3] + c["chith_21"])
        k22 = c["chi0_22"] / (u[0] + c["chith_22"])
        return k11 * g[3] + k13 * g[5], k21 * g[3] - k22 * g[0]

    def apply(self, U, jump="modes"):
        """U: [6, E, (p+1)^d] (any float type, converted) -> f [6, E, (p+1)^d]."""
        d, dt, c, a = self.d, self.dt, self.c, self.a
        U = np.asarray(U).astype(dt)
        gshape = (6,) + tuple(reversed(self.n)) + (U.shape[-1],)
        # volume
        u = np.einsum("sem,qm->seq", U, self.Phi)
        g = np.einsum("sem,qma->aseq", U, self.dPhi)
        w1, w2 = self.velocities(u, g.swapaxes(0, 1))      # [d, E, Q]
        flux = -a[None, :, None, None] * g                  # [d, 6, E, Q]
        flux[:, 0] += u[0][None] * w1
        flux[:, 1] += u[1][None] * w2
        n1, n2, n3, c1, c2, c3 = u
        S = np.stack([-c["d1"] * n1, -c["d2"] * n2, c["d1"] * n1 + c["d2"] * n2 - c["gamma"] * n1,
                      -c["alpha1"] * n1 * c1 - c["alpha2"] * n2 * c1 + c["f1"] * n3, -c["k"] * c2, c["k"] * c2])
        R = np.einsum("q,aseq,qma->sem", self.wq, flux, self.dPhi) + np.einsum("q,seq,qm->sem", self.wq, S, self.Phi)
        R = R.reshape(gshape)
        UG = U.reshape(gshape)
        for ax in range(d):
            gd = 1 + (d - 1 - ax)                            # grid dim of axis ax
            vh, dh, wf = self._face_tabs(ax, 1)
            vl, dl, _ = self._face_tabs(ax, 0)
            Up = np.roll(UG, -1, axis=gd)
            um = np.einsum("s...m,tm->s...t", UG, vh)
            up = np.einsum("s...m,tm->s...t", Up, vl)
            if jump == "modes":
                jm = (UG[..., :1] - Up[..., :1]) + np.einsum("s...m,tm->s...t", UG[..., 1:], vh[:, 1:]) \
                    - np.einsum("s...m,tm->s...t", Up[..., 1:], vl[:, 1:])
            else:
                jm = um - up
            dm = np.einsum("s...m,tm->s...t", UG, dh)
            dp = np.einsum("s...m,tm->s...t", Up, dl)
            w1m, w2m = self.velocities(um, dm)
            w1p, w2p = self.velocities(up, dp)
            lam = np.maximum(np.maximum(abs(w1m), abs(w2m)), np.maximum(abs(w1p), abs(w2p)))
            Fh = np.zeros_like(um)
            Fh[0] = (um[0] * w1m + up[0] * w1p) / dt(2)
            Fh[1] = (um[1] * w2m + up[1] * w2p) / dt(2)
            Fh = Fh + lam[None] * jm / dt(2)
            ab = a.reshape((6,) + (1,) * (jm.ndim - 1))
            avg = ab * (dm + dp) / dt(2)
            Ahat = -self.chi * ab * dt((self.p + 1) ** 2) / self.h[ax] * jm
            gfl = avg - Fh + Ahat
            sym = ab * jm / dt(2)
            Rm = np.einsum("t,s...t,tm->s...m", wf, gfl, vh) + np.einsum("t,s...t,tm->s...m", wf, sym, dh)
            Rp = -np.einsum("t,s...t,tm->s...m", wf, gfl, vl) + np.einsum("t,s...t,tm->s...m", wf, sym, dl)
            if ax == self.wall:
                N = self.n[ax]
                keep = np.ones(N, dtype=dt)
                keep[N - 1] = 0
                shp = [1] * Rm.ndim
                shp[gd] = N
                Rm = Rm * keep.reshape(shp)
                Rp = Rp * keep.reshape(shp)
                # inflow fluxes on Gamma1 (low end) and Gamma2 (high end)
                lo = np.take(UG, [0], axis=gd)
                hi = np.take(UG, [N - 1], axis=gd)
                c1lo = np.einsum("...m,tm->...t", lo[3], vl)
                c1hi = np.einsum("...m,tm->...t", hi[3], vh)
                q1 = np.zeros((6,) + c1lo.shape, dtype=dt)
                q1[0] = c["mu1"] * c["beta1"] * (c1lo - c["c1_star"] > 0)
                q1[4] = c["nu2"] * c["sigma"]                # Gamma1,in = all of Gamma1
                q2 = np.zeros((6,) + c1hi.shape, dtype=dt)
                q2[1] = c["mu2"] * c["beta2"] * (c1hi - c["c1_sstar"] > 0)
                bl = np.einsum("t,s...t,tm->s...m", wf, q1, vl)
                bh = np.einsum("t,s...t,tm->s...m", wf, q2, vh)
                edge = np.zeros_like(R)
                idx = [slice(None)] * R.ndim
                idx[gd] = slice(0, 1)
                edge[tuple(idx)] += bl
                idx[gd] = slice(N - 1, N)
                edge[tuple(idx)] += bh
                R = R + edge
            R = R + Rm + np.roll(Rp, 1, axis=gd)
        return (R / self.vol).reshape(U.shape)
