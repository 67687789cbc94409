"""Seeded synthetic workloads for the CDG2 plaque operator.

This module only draws random numbers and prepares input arrays: initial fields,
coefficient sets and batched instance lists.  It contains none of the operator's
arithmetic and is shared, as plain data, by the tests, the benchmark and the
smoke check.

Initial data (Section 2 asks for given initial fields n_i^0, c_i^0; Section 3.2
takes U(0) as the L2 projection of U_0 onto V_h):

    u_s(x) = 0.5 + sum_{j=1..4} a_sj * prod_{b periodic} cos(2 pi k_b x_b + phi_b)
                                      * cos(pi k_w x_w)

with integer wave numbers k in {0..3} (not all zero), phases phi ~ U[0, 2 pi),
amplitudes a ~ U[0, 0.2] rescaled so that sum_j a_sj <= 0.4, hence
u_s in [0.1, 0.9] (positive).  The wall factor cos(pi k_w x_w) has zero normal
derivative on both walls.  Each term is a product of 1D factors, so its
projection onto the tensor Legendre basis is the product of 1D projections,
computed with numpy's Gauss-Legendre rule (p+3 points per direction).

The paper gives the coefficients only as symbols, so a nondimensional base table
is chosen here (fields stay in about [0.1, 0.9], chemotaxis is a small fraction
of the diffusive flux, diffusion limits the explicit time step).
"""
from __future__ import annotations

import math

import numpy as np

COEFF_NAMES = [
    "mu1", "mu2", "mu3", "nu1", "nu2", "nu3",
    "chi0_11", "chi0_13", "chi0_21", "chi0_22",
    "chith_11", "chith_13", "chith_21", "chith_22",
    "d1", "d2", "gamma", "alpha1", "alpha2", "f1", "k",
    "beta1", "beta2", "sigma", "c1_star", "c1_sstar",
]

BASE = dict(mu1=1e-2, mu2=5e-3, mu3=1e-3, nu1=5e-2, nu2=2e-2, nu3=2e-2,
            chi0_11=2e-3, chi0_13=1e-3, chi0_21=1e-3, chi0_22=1e-3,
            chith_11=0.5, chith_13=0.5, chith_21=0.5, chith_22=0.5,
            d1=0.5, d2=0.2, gamma=-0.3, alpha1=1.0, alpha2=0.5, f1=0.4, k=0.8,
            beta1=0.5, beta2=0.2, sigma=0.3, c1_star=0.45, c1_sstar=0.55)

SEED_ROOT = 1403


def base_coeffs() -> dict:
    return dict(BASE)


def rng_for(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, *key])))


def _basis_1d(p: int, xi: np.ndarray) -> np.ndarray:
    """sqrt(2i+1) P_i(2 xi - 1) via numpy's Legendre evaluator, [len(xi), p+1]."""
    t = 2.0 * xi - 1.0
    out = np.empty((xi.size, p + 1))
    for i in range(p + 1):
        c = np.zeros(i + 1)
        c[i] = 1.0
        out[:, i] = math.sqrt(2 * i + 1) * np.polynomial.legendre.legval(t, c)
    return out


def _project_1d(fn, n: int, p: int) -> np.ndarray:
    """1D L2-projection coefficients of fn on n cells of [0,1]: [n, p+1]."""
    xg, wg = np.polynomial.legendre.leggauss(p + 3)
    xi = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    B = _basis_1d(p, xi)                                   # [Qg, p+1]
    x = (np.arange(n)[:, None] + xi[None, :]) / n          # [n, Qg]
    return np.einsum("q,nq,qm->nm", w, fn(x), B)


def field_params(dim: int, wall_axis: int, key: tuple):
    """Random Fourier description of the six initial fields."""
    rng = rng_for(*key)
    out = []
    for _s in range(6):
        terms = []
        for _j in range(4):
            while True:
                k = rng.integers(0, 4, size=dim)
                if k.any():
                    break
            phase = rng.uniform(0.0, 2.0 * math.pi, size=dim)
            amp = rng.uniform(0.0, 0.2)
            terms.append([k, phase, amp])
        tot = sum(t[2] for t in terms)
        if tot > 0.4:
            for t in terms:
                t[2] *= 0.4 / tot
        out.append(terms)
    return out


def initial_modes(dim: int, n, p: int, key: tuple, wall_axis: int | None = None) -> np.ndarray:
    """Modal coefficients U[6, E, (p+1)^dim] (float64) of the projected initial fields.
    Element e = ix + nx (iy + ny iz); mode m = i + (p+1) (j + (p+1) k)."""
    n = tuple(int(v) for v in n)[:dim]
    wall = dim - 1 if wall_axis is None else wall_axis
    q = p + 1
    E = int(np.prod(n))
    U = np.zeros((6, E, q ** dim))
    U[:, :, 0] = 0.5
    params = field_params(dim, wall, key)
    for s in range(6):
        acc = np.zeros((*reversed(n), *([q] * dim)))
        for k, phase, amp in params[s]:
            facs = []
            for b in range(dim):
                if b == wall:
                    kb = int(k[b])
                    fn = (lambda x, kb=kb: np.cos(math.pi * kb * x))
                else:
                    kb, ph = int(k[b]), float(phase[b])
                    fn = (lambda x, kb=kb, ph=ph: np.cos(2.0 * math.pi * kb * x + ph))
                facs.append(_project_1d(fn, n[b], p))          # [n_b, q]
            if dim == 2:
                term = np.einsum("ya,xb->yxab", facs[1], facs[0])
            else:
                term = np.einsum("zc,yb,xa->zyxcba", facs[2], facs[1], facs[0])
            acc += amp * term
        U[s] += acc.reshape(E, q ** dim)
    return U


def coeff_array(c: dict) -> np.ndarray:
    return np.array([float(c[k]) for k in COEFF_NAMES])


def sample_coeffs(key: tuple) -> dict:
    """Each coefficient scaled by a log-uniform factor in [0.5, 1.5] (signs kept)."""
    rng = rng_for(*key)
    out = {}
    for name in COEFF_NAMES:
        out[name] = BASE[name] * math.exp(rng.uniform(math.log(0.5), math.log(1.5)))
    return out


def batch_instances(count: int = 256, key: tuple = (3,)):
    """Batched workload: grid side N ~ U{32,48,64,96,128}, order p ~ U{1,2,3},
    coefficients by sample_coeffs; instance i uses seed (1403, 3, i)."""
    rng = rng_for(*key)
    sides = [32, 48, 64, 96, 128]
    out = []
    for i in range(count):
        N = int(sides[rng.integers(0, len(sides))])
        p = int(rng.integers(1, 4))
        out.append(dict(n=(N, N), order=p, coeffs=sample_coeffs((*key, i, 1)), key=(*key, i)))
    return out


def adjoint_coeffs() -> dict:
    """Base table with the Heaviside thresholds moved outside the field range so that
    the inflow switches stay fixed and the loss is differentiable."""
    c = base_coeffs()
    c["c1_star"] = 0.05
    c["c1_sstar"] = 0.95
    return c


def adjoint_target_coeffs(key: tuple = (4,)) -> dict:
    """Target coefficients: each of the 21 differentiable coefficients times
    (1 + 0.1 xi_j) with xi_j = +-1 drawn from the seed."""
    rng = rng_for(*key, 7)
    c = adjoint_coeffs()
    for name in COEFF_NAMES[:21]:
        c[name] = c[name] * (1.0 + 0.1 * (1.0 if rng.integers(0, 2) else -1.0))
    return c


def diffusion_only_coeffs(a: float = 0.05) -> dict:
    """Pure diffusion with the same motility a for every species: no chemotaxis,
    no reactions, inflow switches off (thresholds above any field value)."""
    c = {k: 0.0 for k in BASE}
    for k in ("mu1", "mu2", "mu3", "nu1", "nu2", "nu3"):
        c[k] = a
    for k in ("chith_11", "chith_13", "chith_21", "chith_22"):
        c[k] = 1.0
    c["c1_star"] = 10.0
    c["c1_sstar"] = 10.0
    return c


def heat_modes(n, p: int, t: float, a: float, amp: float = 0.2) -> np.ndarray:
    """Projection onto Q_p of u = 0.5 + amp exp(-5 pi^2 a t) cos(2 pi x) cos(pi y)
    (every species; solves u_t = a Laplace u, periodic in x, zero flux at y = 0, 1)
    on an n[0] x n[1] grid: U[6, E, (p+1)^2]."""
    nx, ny = int(n[0]), int(n[1])
    q = p + 1
    fx = _project_1d(lambda x: np.cos(2.0 * math.pi * x), nx, p)
    fy = _project_1d(lambda y: np.cos(math.pi * y), ny, p)
    term = np.einsum("ya,xb->yxab", fy, fx).reshape(nx * ny, q * q)
    U = np.zeros((6, nx * ny, q * q))
    U[:, :, 0] = 0.5
    U += amp * math.exp(-5.0 * math.pi ** 2 * a * t) * term[None]
    return U


def reduced_3d_coeffs(base: dict | None = None) -> dict:
    """The three-species model of the paper's 3D experiment (immune cells n1,
    debris n3, chemoattractant c1, eq. (02)) as a coefficient set of the
    six-species model: run with n2 = c2 = c3 = 0 (they stay zero: no sources,
    no inflow of LDL (sigma = 0) or of smooth muscle cells (beta2 = 0)), n1
    without its death term and the debris source (d1 - F) n1 kept, i.e.
    d1 := 0 and gamma := gamma - d1.  The immune-cell inflow on Gamma1 stays."""
    c = dict(base_coeffs() if base is None else base)
    c["gamma"] = c["gamma"] - c["d1"]
    c["d1"] = 0.0
    c["sigma"] = 0.0
    c["beta2"] = 0.0
    return c


def reduced_3d_modes(n, p: int, key: tuple = (6,)) -> np.ndarray:
    """Initial data of the 3D experiment: the seeded n1 and c1 fields, a local
    bump of debris n3 (the inflammation trigger: no LDL inflow in 3D), and
    n2 = c2 = c3 = 0.  The bump is exp(-|x - x0|^2 / (2 s^2)) projected per axis
    (separable), amplitude 0.5, s = 0.08, x0 = (0.5, 0.5, 0.15)."""
    U = initial_modes(3, n, p, key)
    U[1] = 0.0                                  # n2
    U[4] = 0.0                                  # c2
    U[5] = 0.0                                  # c3
    q = p + 1
    facs = []
    for b, x0 in enumerate((0.5, 0.5, 0.15)):
        facs.append(_project_1d(lambda x, x0=x0: np.exp(-((x - x0) ** 2) / (2 * 0.08 ** 2)), int(n[b]), p))
    bump = np.einsum("zc,yb,xa->zyxcba", facs[2], facs[1], facs[0]).reshape(-1, q ** 3)
    U[2] = 0.0
    U[2, :, 0] = 0.05
    U[2] += 0.5 * bump
    return U


def kuhn_mesh(nx: int, ny: int, jitter: float = 0.0, key: tuple = (7,)):
    """Triangle mesh of [0,1]^2: each of nx x ny squares split along its rising
    diagonal, periodic in x, walls y = 0 (Gamma1) and y = 1 (Gamma2).  Optional
    seeded jitter moves every vertex (x, and y off the walls) by up to `jitter`
    cell widths, which makes the mesh non-uniform (unequal triangles).

    Returns xy [E, 3, 2] (vertex coordinates per element, counter-clockwise,
    periodic images unwrapped), nbr [E, 3] (element across edge j, from vertex j
    to vertex j+1, or -1 on Gamma1, -2 on Gamma2) and nbe [E, 3] (that edge's
    index in the neighbour)."""
    # with fewer than 3 squares across, two different edges would join the same
    # pair of (periodic) vertices and the edge matching below would pair them
    assert nx >= 3 and ny >= 1, "kuhn_mesh needs nx >= 3 and ny >= 1"
    hx, hy = 1.0 / nx, 1.0 / ny
    rng = rng_for(*key)
    dx = rng.uniform(-jitter, jitter, size=(nx, ny + 1)) * hx
    dy = rng.uniform(-jitter, jitter, size=(nx, ny + 1)) * hy
    dy[:, 0] = 0.0
    dy[:, ny] = 0.0

    def vert(i, j):
        ii = i % nx
        return (i * hx + dx[ii, j], j * hy + dy[ii, j]), ii + nx * j

    xy, vid = [], []
    for j in range(ny):
        for i in range(nx):
            (a, va), (b, vb), (c, vc), (d, vd) = vert(i, j), vert(i + 1, j), vert(i + 1, j + 1), vert(i, j + 1)
            xy.append([a, b, c])
            vid.append([va, vb, vc])
            xy.append([a, c, d])
            vid.append([va, vc, vd])
    xy = np.array(xy, dtype=np.float64)
    E = len(vid)
    nbr = np.full((E, 3), -9, dtype=np.int32)
    nbe = np.full((E, 3), -1, dtype=np.int32)
    owner = {}
    for e in range(E):
        for k in range(3):
            a, b = vid[e][k], vid[e][(k + 1) % 3]
            key2 = (min(a, b), max(a, b))
            if key2 in owner:
                f, kk = owner.pop(key2)
                nbr[e, k], nbe[e, k] = f, kk
                nbr[f, kk], nbe[f, kk] = e, k
            else:
                owner[key2] = (e, k)
    for (a, b), (e, k) in owner.items():
        nbr[e, k] = -1 if a < nx and b < nx else -2
    assert (nbr != -9).all()
    return xy, nbr, nbe


def tri_modes(E: int, k: int, key: tuple = (8,), amp: float = 0.02) -> np.ndarray:
    """Random modal coefficients U[6, E, (k+1)(k+2)/2] of a positive field on a
    triangle mesh: cell means in [0.3, 0.7], the other modes within +-amp."""
    rng = rng_for(*key)
    nb = (k + 1) * (k + 2) // 2
    U = rng.uniform(-amp, amp, size=(6, E, nb))
    U[:, :, 0] = rng.uniform(0.3, 0.7, size=(6, E))
    return U


def kuhn_tet_mesh(nx: int, ny: int, nz: int, jitter: float = 0.0, key: tuple = (17,)):
    """Tetrahedral mesh of [0,1]^3: each of nx x ny x nz cubes split into the six
    tetrahedra of its Kuhn (Freudenthal) subdivision along the main diagonal,
    periodic in x and y, walls z = 0 (Gamma1) and z = 1 (Gamma2).  Optional seeded
    jitter moves every vertex by up to `jitter` cell widths (z only off the walls),
    which makes the tetrahedra unequal.

    Returns xyz [E, 4, 3] (vertex coordinates per element, positively oriented,
    periodic images unwrapped), vid [E, 4] (periodic vertex ids), nbr [E, 4]
    (element across the face opposite local vertex f, or -1 on Gamma1, -2 on
    Gamma2) and nbe [E, 4] (that face's index in the neighbour)."""
    # with fewer than 3 cubes across a periodic axis two different faces would
    # join the same (periodic) vertices and the face matching would pair them
    assert nx >= 3 and ny >= 3 and nz >= 1, "kuhn_tet_mesh needs nx, ny >= 3"
    h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    rng = rng_for(*key)
    d = rng.uniform(-jitter, jitter, size=(3, nx, ny, nz + 1)) * np.array(h)[:, None, None, None]
    d[2, :, :, 0] = 0.0
    d[2, :, :, nz] = 0.0

    def vert(i, j, l):
        ii, jj = i % nx, j % ny
        p = (i * h[0] + d[0, ii, jj, l], j * h[1] + d[1, ii, jj, l], l * h[2] + d[2, ii, jj, l])
        return p, ii + nx * (jj + ny * l)

    paths = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    xyz, vid = [], []
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                for path in paths:
                    c = [0, 0, 0]
                    pts, ids = [], []
                    for step in (None,) + path:
                        if step is not None:
                            c[step] += 1
                        p, v = vert(i + c[0], j + c[1], l + c[2])
                        pts.append(p)
                        ids.append(v)
                    P = np.array(pts)
                    if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)) < 0:
                        pts[1], pts[2] = pts[2], pts[1]
                        ids[1], ids[2] = ids[2], ids[1]
                    xyz.append(pts)
                    vid.append(ids)
    xyz = np.array(xyz, dtype=np.float64)
    vid = np.array(vid, dtype=np.int32)
    E = len(vid)
    faces = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
    nbr = np.full((E, 4), -9, dtype=np.int32)
    nbe = np.full((E, 4), -1, dtype=np.int32)
    owner = {}
    for e in range(E):
        for f, vs in enumerate(faces):
            k2 = tuple(sorted(int(vid[e, v]) for v in vs))
            if k2 in owner:
                g, gf = owner.pop(k2)
                nbr[e, f], nbe[e, f] = g, gf
                nbr[g, gf], nbe[g, gf] = e, f
            else:
                owner[k2] = (e, f)
    layer = nx * ny
    for k2, (e, f) in owner.items():
        nbr[e, f] = -1 if max(k2) < layer else -2
    assert (nbr != -9).all()
    return xyz, vid, nbr, nbe


def tet_modes(E: int, k: int, key: tuple = (18,), amp: float = 0.02) -> np.ndarray:
    """Random modal coefficients U[6, E, (k+1)(k+2)(k+3)/6] of a positive field on
    a tetrahedral mesh: element means in [0.3, 0.7], the other modes within +-amp."""
    rng = rng_for(*key)
    nb = (k + 1) * (k + 2) * (k + 3) // 6
    U = rng.uniform(-amp, amp, size=(6, E, nb))
    U[:, :, 0] = rng.uniform(0.3, 0.7, size=(6, E))
    return U
