"""Pins of the oracle's CFL time step (the spectral constant rho_hat and
Oracle.max_dt) against what the mathematics fixes, independently of the oracle's
own matrices:

* on uniform Cartesian cells the CDG2 lifting has the closed-form trace
  -(p+1)^2 / (2h) [[u]] (pinned in test_oracle_pins), so along one axis the
  diffusion operator is the textbook symmetric interior penalty method with
  penalty chi_e (p+1)^2 / h.  Its Fourier symbol, written here in a monomial
  basis with exact integrals, gives the spectral radius per axis;
* on a uniform grid the d-dimensional operator is the Kronecker sum of the
  1D operators, so its spectral radius is d times the 1D one;
* SSP-RK3 is stable on the negative real axis down to -2.5127: the step of
  max_dt (cfl = 0.9) keeps a pure-diffusion run non-increasing in the L2 norm,
  while cfl = 1.05 puts the top eigenvalue outside the stability interval."""
import math

import numpy as np
import pytest
import torch

from oracle.cdg2_oracle import NSPEC, Config, Oracle, diffusion_only_coeffs
from paper_1403_1157_amd import inputs

# The spectral constants to the digits printed for the CFL reading (quads with
# chi_e = 2 for p = 1..4, hexes with chi_e = 3 for p = 1..3).
PRINTED = {(2, 1): 84.00, (2, 2): 362.06, (2, 3): 1058.74, (2, 4): 2470.93,
           (3, 1): 132.00, (3, 2): 578.04, (3, 3): 1698.46}


def sipg_1d_top_eigenvalue(p, chi, thetas):
    """Largest eigenvalue of M^-1 A(theta) over the given wavenumbers, for the
    1D periodic SIPG form with h = a = 1 and penalty eta = chi (p+1)^2:
      B(u, v) = sum_K int u'v' - sum_e ({u'}[v] + {v'}[u]) + eta sum_e [u][v],
    [u] = u_k(1) - u_{k+1}(0), {u'} = (u_k'(1) + u_{k+1}'(0)) / 2, with the
    Bloch ansatz u_{k+1} = e^{i theta} u_k, in the monomial basis x^i on [0, 1]
    (mass 1/(i+j+1), stiffness ij/(i+j-1))."""
    n = p + 1
    M = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])
    S = np.array([[i * j / (i + j - 1) if i and j else 0.0 for j in range(n)] for i in range(n)])
    one = np.ones(n)                                   # x^i at 1
    zero = np.eye(n)[0]                                # x^i at 0
    done = np.arange(n, dtype=float)                   # (x^i)' at 1
    dzero = np.eye(n)[1] if n > 1 else np.zeros(n)     # (x^i)' at 0
    eta = chi * (p + 1) ** 2
    Li = np.linalg.inv(np.linalg.cholesky(M))
    top = -np.inf
    for th in thetas:
        z = np.exp(1j * th)
        J = one - z * zero
        Dv = 0.5 * (done + z * dzero)
        A = S - np.outer(J.conj(), Dv) - np.outer(Dv.conj(), J) + eta * np.outer(J.conj(), J)
        top = max(top, np.linalg.eigvalsh(Li @ A @ Li.T.conj()).max())
    return top


@pytest.mark.parametrize("dim,p", sorted(PRINTED))
def test_spectral_constant_is_the_1d_sipg_spectral_radius(dim, p):
    o = Oracle(Config(dim=dim, n=(4,) * dim, order=p, coeffs=inputs.base_coeffs()))
    rho = o.spectral_constant()                        # on a periodic 4^d grid, a = 1
    chi = float(dim)                                   # chi_e = N/2
    on_grid = sipg_1d_top_eigenvalue(p, chi, [2 * math.pi * k / 4 for k in range(4)])
    sup = sipg_1d_top_eigenvalue(p, chi, np.linspace(0.0, 2 * math.pi, 721))
    assert abs(rho - on_grid) <= 1e-10 * on_grid, (rho, on_grid)
    # the 4-cell grid already holds the maximising wavenumber: the constant is
    # the supremum over all grids
    assert abs(sup - on_grid) <= 1e-10 * on_grid
    assert round(rho, 2) == PRINTED[(dim, p)]


@pytest.mark.parametrize("p", [1, 2])
def test_spectral_radius_is_a_kronecker_sum(p):
    """On the fully periodic 4x4 grid the top eigenvalue of -M^-1 K is twice the
    top eigenvalue on the invariant subspace of states constant in y (only the
    modes with j = 0, the same in every cell of a column along y)."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    o = Oracle(Config(dim=2, n=(4, 4), order=p, wall_axis=-1, coeffs=diffusion_only_coeffs(1.0)))
    shp = (NSPEC, o.E, o.nm)
    n = NSPEC * o.E * o.nm
    ymask = torch.zeros(o.nm, dtype=torch.float64)
    ymask[: p + 1] = 1.0                               # m = i + (p+1) j with j = 0

    def y_constant(X):
        # orthogonal projector: drop the y modes, average the cells of each column
        X = (X * ymask).reshape(NSPEC, 4, 4, o.nm)     # [s, iy, ix, m]
        return X.mean(dim=1, keepdim=True).expand(-1, 4, -1, -1).reshape(shp)

    def top(project):
        def mv(x):
            X = project(torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).reshape(shp))
            return project(-o.apply(X)).reshape(-1).numpy()
        op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
        v0 = project(torch.from_numpy(np.random.default_rng(1).standard_normal(n)).reshape(shp))
        return float(eigsh(op, k=1, which="LA", tol=0, v0=v0.reshape(-1).numpy(), return_eigenvectors=False)[0])

    full, along_x = top(lambda X: X), top(y_constant)
    assert abs(full - 2.0 * along_x) <= 1e-9 * full, (full, along_x)
    h = 0.25
    assert abs(along_x * h * h - sipg_1d_top_eigenvalue(p, 2.0, [0, math.pi / 2, math.pi, 1.5 * math.pi])) \
        <= 1e-9 * along_x * h * h


@pytest.mark.parametrize("dim,n,p", [(2, (6, 4), 2), (3, (3, 3, 4), 1)])
def test_max_dt_on_a_uniform_state(dim, n, p):
    """A spatially uniform state has no chemotactic velocity (lambda = 0), so
    dt = cfl / (rho_hat a_max sum_a h_a^-2 / 2.51 + r_max / 2.51) with
    r_max = d1 + d2 + |gamma| + k + alpha1 n1 + alpha2 n2."""
    c = inputs.base_coeffs()
    o = Oracle(Config(dim=dim, n=n, order=p, coeffs=c))
    vals = [0.7, 0.4, 0.3, 0.6, 0.2, 0.5]
    U = torch.zeros(NSPEC, o.E, o.nm, dtype=torch.float64)
    for s, v in enumerate(vals):
        U[s, :, 0] = v
    rho = sipg_1d_top_eigenvalue(p, float(dim), [0, math.pi / 2, math.pi, 1.5 * math.pi])
    amax = max(c[k] for k in ("mu1", "mu2", "mu3", "nu1", "nu2", "nu3"))
    rmax = c["d1"] + c["d2"] + abs(c["gamma"]) + c["k"] + c["alpha1"] * vals[0] + c["alpha2"] * vals[1]
    sih2 = sum(v * v for v in n)
    want = 0.9 / (rho * amax * sih2 / 2.51 + rmax / 2.51)
    got = o.max_dt(U, 0.9)
    assert abs(got - want) <= 1e-12 * want, (got, want)


def test_max_dt_is_the_ssp_rk3_stability_limit():
    """Pure diffusion on a fully periodic grid: at the max_dt step (cfl 0.9) the
    L2 norm (M = |K| I) never grows over 80 SSP-RK3 steps; at cfl 1.05 the top
    eigenvalue leaves the stability interval and a random state blows up."""
    o = Oracle(Config(dim=2, n=(4, 4), order=2, wall_axis=-1, coeffs=diffusion_only_coeffs(0.3)))
    g = torch.Generator().manual_seed(3)
    U0 = torch.rand(NSPEC, o.E, o.nm, generator=g, dtype=torch.float64) - 0.5
    dt = o.max_dt(U0, 0.9)
    U = U0.clone()
    prev = float(U.norm())
    for _ in range(80):
        U = o.rk_step(U, dt, 1)
        now = float(U.norm())
        assert now <= prev * (1 + 1e-12)
        prev = now
    U = o.rk_step(U0.clone(), dt * 1.05 / 0.9, 80)
    assert float(U.norm()) > 1e3 * float(U0.norm())
